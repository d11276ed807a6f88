"""The allocation-free Dyson step (gwsym_dyson_G_noalloc) through the C-ABI against the regular
gwsym_dyson_G (eq. dyson) on the same inputs: two calls in a row on one GPU, the second on a
smaller workload (the shared scratch array keeps the first call's contents), each compared with
the regular call to the FP64 bar, and a workload beyond the array refused with ESHAPE."""
import numpy as np
import pytest
import torch

from tests.gpu_common import DeviceRun, oracle_run, say
from tests.helpers import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _one(name):
    run = DeviceRun(name, 2)
    ref = oracle_run(name)
    c = run.ctx
    # inputs: the oracle's self-energy after one iteration and its chemical potential
    r = ref["iters"][0]
    S = torch.zeros(c.g_size, dtype=torch.complex128, device=run.dev)
    c.to_block(1, torch.as_tensor(np.ascontiguousarray(r["Sigma"][run.ibz]), device=run.dev), S)
    run.mu.fill_(float(r["mu"]))
    G_reg = torch.zeros_like(S)
    G_new = torch.full_like(S, float("nan"))
    c.dyson_G(run.F, S, run.mu, G_reg)
    c.dyson_G_noalloc(run.F, S, run.mu, G_new)
    c.check()
    torch.cuda.synchronize()
    e = rel(G_new.cpu().numpy(), G_reg.cpu().numpy())
    eo = rel(run.full(1, G_new), r["G"])
    say(f"[no-alloc dyson] {name}: vs regular call {e:.1e}, vs oracle {eo:.1e}")
    assert e < 1e-10
    assert eo < 1e-10
    return run


def test_noalloc_dyson_two_calls_second_smaller():
    big = _one("cfg0")               # 8 k, 9 orbitals, 81 frequencies
    small = _one("small_diamond")    # smaller frequency workspaces than the first call
    assert small.ctx.g_size * small.ctx.nw < big.ctx.g_size * big.ctx.nw


def test_noalloc_dyson_rejects_oversized_workload():
    from paper_2405_09494_amd.gwsym import GwsymError
    from tests.helpers import make_context
    from gwinputs import workload
    wl = workload("cfg4")      # 6x6x6 diamond: frequency workspaces of about 160 MB
    c = make_context(wl)
    c.device_init()
    z = lambda n: torch.zeros(n, dtype=torch.complex128, device="cuda:0")
    F, S, G = z(c.f_size), z(c.g_size), z(c.g_size)
    mu = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(GwsymError, match="ESHAPE"):
        c.dyson_G_noalloc(F, S, mu, G)
    c.close()
