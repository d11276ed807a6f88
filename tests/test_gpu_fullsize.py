"""Parity at the full benchmark size (cfg1: simple cubic 4x4x4 mesh, nao 26, naux 150,
ntau 64) in the launch configuration the benchmark times (block mode, default tau chunk and
half-tau mirror), on outputs the oracle computes one at a time: one P0^q(tau_j) over every
k (eq. P0) and one Sigma^k(tau_j) over every q (eq. sigma).  The Sigma check feeds a seeded,
symmetric stand-in for P at one tau (zero elsewhere), so every oracle input comes from the
generator.  Bars: 1e-10 relative in FP64, 1e-6 with FP32 or three-piece bfloat16 contractions."""
import os

import numpy as np
import pytest
import torch

import oracle
from gwinputs import Inputs, add_k, workload
from tests.gpu_common import say
from tests.helpers import make_context, rel, sub_table

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cfg1():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = workload("cfg1")
    dev = torch.device("cuda:0")
    say("[full size] generating cfg1 inputs")
    inp = Inputs(wl, device=dev)
    F = inp.fock()
    ctx = make_context(wl)
    ibz = ctx.table("ibz")
    nk, nib = wl.nk, len(ibz)
    add, sub = add_k(wl.n), sub_table(wl.n)
    q, j = int(ibz[3]), 5            # a P0 output: irreducible q, tau index j
    k, js = int(ibz[2]), 41          # a Sigma output: irreducible k, tau index js
    pairs = [(int(ibz[i]), kp) for i in range(nib) for kp in range(nk)]
    pairs += [(kk, int(add[kk, q])) for kk in range(nk)]
    pairs += [(k, int(sub[k, qq])) for qq in range(nk)]
    pairs += [(kp, k) for kp in range(nk)] + [(kp, kp) for kp in range(nk)]
    V = inp.three_index(pairs)
    Vibz = V[: nib * nk].reshape(nib, nk, *V.shape[1:]).contiguous()
    Vq = V[nib * nk: nib * nk + nk].cpu().numpy()
    Vk = V[nib * nk + nk: nib * nk + 2 * nk].cpu().numpy()
    Vcol = V[nib * nk + 2 * nk: nib * nk + 3 * nk].cpu().numpy()     # V^{k',k}
    Vdiag = V[nib * nk + 3 * nk:].cpu().numpy()                      # V^{k',k'}
    Vrow = Vibz[2].cpu().numpy()                                     # V^{k,k'}, k = ibz[2]
    del V
    X = inp.aux_matrices(1)[:, 0]    # [nk, naux, naux], symmetric Hermitian stand-in for P(tau_js)
    tau = oracle.tau_grid(wl.beta, wl.ntau)
    G0 = oracle.g0_closed_form(F.cpu().numpy(), 0.0, wl.beta, tau)
    say("[full size] oracle outputs")
    ref_p0 = oracle.polarization_unit(G0, Vq, add, q, j, wl.spin)
    ref_s = oracle.self_energy_unit(G0, Vk, X.cpu().numpy(), sub, k, js)
    # F = H0 + J + K of eq. sigma_hf at k from the free G0
    ref_f = (F[k].cpu().numpy() + oracle.hartree_unit(G0, Vdiag, k, wl.spin)
             + oracle.exchange_unit(G0, Vrow, Vcol))
    return dict(wl=wl, dev=dev, F=F, Vibz=Vibz, X=X, ibz=ibz, q=q, j=j, k=k, js=js, ref_p0=ref_p0, ref_s=ref_s,
                ref_f=ref_f)


def run(d, precision):
    wl, dev = d["wl"], d["dev"]
    ctx = make_context(wl, precision=precision)
    ctx.device_init()
    ctx.load_V(d["Vibz"])
    # the launch plans the benchmark uses (stored ones, else timed here)
    ctx.autotune(cache=os.path.join(ROOT, "paper_2405_09494_amd", "plans.json"), update=False)
    z = lambda n: torch.zeros(n, dtype=torch.complex128, device=dev)
    Fb, G, P0, Pb, S = z(ctx.f_size), z(ctx.g_size), z(ctx.p_size), z(ctx.p_size), z(ctx.g_size)
    ctx.to_block(0, d["F"][torch.as_tensor(d["ibz"], device=dev)].contiguous(), Fb)
    ctx.g0(Fb, 0.0, G)
    ctx.polarization(G, P0)
    nk, nt, na, no = wl.nk, wl.ntau, wl.naux, wl.nao
    full = torch.zeros(nk * nt * na * na, dtype=torch.complex128, device=dev)
    ctx.from_block(2, P0, full)
    torch.cuda.synchronize()
    p0 = full.view(nk, nt, na, na)[d["q"], d["j"]].cpu().numpy()
    del full
    # the stand-in P is placed at tau_js and at beta - tau_js (P(tau) = P(beta - tau), the
    # bosonic symmetry with time reversal that the half-tau mode relies on), zero elsewhere
    Pin = torch.zeros((len(d["ibz"]), nt, na, na), dtype=torch.complex128, device=dev)
    Pin[:, d["js"]] = d["X"][torch.as_tensor(d["ibz"], device=dev)]
    Pin[:, nt - 1 - d["js"]] = d["X"][torch.as_tensor(d["ibz"], device=dev)]
    ctx.to_block(2, Pin, Pb)
    ctx.self_energy(G, Pb, S)
    sfull = torch.zeros(nk * nt * no * no, dtype=torch.complex128, device=dev)
    ctx.from_block(1, S, sfull)
    torch.cuda.synchronize()
    s = sfull.view(nk, nt, no, no)[d["k"], d["js"]].cpu().numpy()
    return p0, s


def test_cfg1_sampled_fp64(cfg1):
    say("[full size] fp64")
    p0, s = run(cfg1, 0)
    e0, es = rel(p0, cfg1["ref_p0"]), rel(s, cfg1["ref_s"])
    say(f"  P0 {e0:.2e} Sigma {es:.2e}")
    assert e0 < 1e-10 and es < 1e-10


def test_cfg1_sampled_fp32(cfg1):
    say("[full size] fp32 contractions")
    p0, s = run(cfg1, 1)
    e0, es = rel(p0, cfg1["ref_p0"]), rel(s, cfg1["ref_s"])
    say(f"  P0 {e0:.2e} Sigma {es:.2e}")
    assert e0 < 1e-6 and es < 1e-6


def test_cfg1_sampled_bf16x6(cfg1):
    say("[full size] bf16 x6 contractions")
    p0, s = run(cfg1, 2)
    e0, es = rel(p0, cfg1["ref_p0"]), rel(s, cfg1["ref_s"])
    say(f"  P0 {e0:.2e} Sigma {es:.2e}")
    assert e0 < 1e-6 and es < 1e-6


def test_cfg1_static_self_energy_fp64(cfg1):
    """F = H0 + J + K (eq. sigma_hf) at one irreducible k from the free G0, at full size."""
    say("[full size] F = H0 + J + K")
    d = cfg1
    wl, dev = d["wl"], d["dev"]
    ctx = make_context(wl)
    ctx.device_init()
    ctx.load_V(d["Vibz"])
    z = lambda n: torch.zeros(n, dtype=torch.complex128, device=dev)
    Fb, G, F1 = z(ctx.f_size), z(ctx.g_size), z(ctx.f_size)
    ctx.to_block(0, d["F"][torch.as_tensor(d["ibz"], device=dev)].contiguous(), Fb)
    ctx.g0(Fb, 0.0, G)
    ctx.fock(Fb, G, F1)
    no = wl.nao
    full = torch.zeros(wl.nk * no * no, dtype=torch.complex128, device=dev)
    ctx.from_block(0, F1, full)
    torch.cuda.synchronize()
    f = full.view(wl.nk, no, no)[d["k"]].cpu().numpy()
    e = rel(f, d["ref_f"])
    say(f"  F {e:.2e}")
    assert e < 1e-10
