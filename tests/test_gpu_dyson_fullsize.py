"""Parity of the two Dyson steps at the block sizes of the 6^3 workloads (cfg2: rocksalt,
nao 52, naux 250, ntau 100; cfg4: diamond Fd-3m, nao 52, naux 300, ntau 128), through the
C-ABI, against the oracle:

  * gwsym_screened_interaction (eq. P02P: tau -> i Omega, [I - P0]^{-1} P0 per auxiliary
    block, back to tau) at two irreducible q: Gamma and the point with the largest auxiliary
    block (300 at cfg4, the inverse that works in global memory);
  * gwsym_find_mu and gwsym_dyson_G (eq. dyson with the electron count of Sec. 4.1 fixed).

The inputs are seeded symmetric stand-ins from the generator, never library outputs:
P0(tau) = -c [f(tau) X^2 + g(tau) X^4], with X a group-averaged Hermitian auxiliary matrix and
f, g > 0 mirror-symmetric in tau (so P0 is negative semidefinite and time-reversal symmetric),
and Sigma(tau) = f(tau) Y_1 + g(tau) Y_2 with group-averaged Hermitian orbital matrices.
The library's block outputs are compared with the diagonal blocks of U^H X_oracle U at that
point (the off-block part of the oracle's result must vanish).  The chemical potential is
checked by the oracle's electron count at the library's mu (the oracle's own 64-step bisection
over all 216 k would take minutes) and G by the oracle's Dyson equation at that mu.

Bar: both sides evaluate the same tau <-> i omega transforms in FP64 with their own summation
order, and a rounding difference in the frequency data reaches tau amplified by the norm of the
inverse transform while the data themselves are bounded through the forward one: the relative
difference is about eps ||T||_2 ||B||_2 times the growth of the sums and of the per-frequency
solve.  On the Chebyshev grid ||T|| ||B|| grows with beta and ntau (8.0e3 for the bosonic
transforms at beta 200, ntau 100; 7.7e4 at beta 400, ntau 128), so the bar is
max(1e-10, 1000 eps ||T|| ||B||) of the transform the quantity passes through (the factor 1000
covers the sqrt(ntau) growth of the sums and the conditioning of I - P0 and of the Dyson
matrix; measured at cfg2: 1.9e-10 = 105 eps ||T|| ||B||)."""
import numpy as np
import pytest
import torch

import oracle
from gwinputs import Inputs, workload
from tests.gpu_common import say
from tests.helpers import make_context

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

EPS = np.finfo(np.float64).eps


def bar(wl, boson):
    T, B, _ = oracle.transform_matrices(wl.beta, wl.ntau, wl.nw, boson)
    return max(1e-10, 1000 * EPS * np.linalg.norm(T, 2) * np.linalg.norm(B, 2))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _shapes(wl):
    tau = oracle.tau_grid(wl.beta, wl.ntau)
    f = np.exp(-8.0 * tau / wl.beta) + np.exp(-8.0 * (wl.beta - tau) / wl.beta)
    g = 0.5 + 0.25 * np.cos(2 * np.pi * tau / wl.beta)
    return f, g


def _blocks_err(M_lib_packed, off, sizes, M_ref, U):
    R = U.conj().T @ M_ref @ U
    mask = np.ones(R.shape, bool)
    err, o, p = 0.0, 0, off
    for s in sizes:
        err = max(err, np.abs(M_lib_packed[p:p + s * s].reshape(s, s) - R[o:o + s, o:o + s]).max())
        mask[o:o + s, o:o + s] = False
        o += s
        p += s * s
    offb = np.abs(R[mask]).max() if mask.any() else 0.0
    return err, offb


@pytest.mark.parametrize("name", ["cfg2", "cfg4"])
def test_screened_interaction_fullsize(name):
    wl = workload(name)
    dev = torch.device("cuda:0")
    say(f"[{name}] stand-in P0 (group-averaged X)")
    inp = Inputs(wl)
    X = inp.aux_matrices(1, scale=1.0)[:, 0].numpy()       # [nk, naux, naux]
    X2 = X @ X
    X4 = X2 @ X2
    c2 = 1.0 / (wl.beta * np.abs(np.linalg.eigvalsh(X2)).max())
    c4 = 0.2 / (wl.beta * np.abs(np.linalg.eigvalsh(X4)).max())
    f, g = _shapes(wl)
    tol = bar(wl, True)
    say(f"[{name}] bar {tol:.1e}")
    ctx = make_context(wl)
    ctx.device_init()
    ibz = ctx.table("ibz")
    bx = ctx.blocks(aux=True)
    big = int(np.argmax([max(b) for b in bx]))
    qs = sorted({0, big})
    say(f"[{name}] irreducible q {qs}, largest auxiliary block {max(bx[big])}")
    P0 = np.zeros(ctx.p_size, complex)
    full = torch.zeros((len(ibz), wl.ntau, wl.naux, wl.naux), dtype=torch.complex128, device=dev)
    for i, q in enumerate(ibz):
        Xq2, Xq4 = torch.as_tensor(X2[q], device=dev), torch.as_tensor(X4[q], device=dev)
        for j in range(wl.ntau):
            full[i, j] = -(c2 * f[j]) * Xq2 - (c4 * g[j]) * Xq4
    P0d = torch.as_tensor(P0, device=dev)
    ctx.to_block(2, full, P0d)
    del full
    Pd = torch.zeros_like(P0d)
    ctx.screened_interaction(P0d, Pd)
    ctx.check()
    Pl = Pd.cpu().numpy()
    Ux = ctx.table("U_aux").reshape(wl.nk, wl.naux, wl.naux)
    for i in qs:
        q = int(ibz[i])
        P0q = np.stack([-(c2 * f[j]) * X2[q] - (c4 * g[j]) * X4[q] for j in range(wl.ntau)])[None]
        say(f"[{name}] oracle screened interaction at q = {q}")
        Pref = oracle.screened(P0q, wl.beta, wl.nw)[0][0]
        scale = np.abs(Pref).max()
        packed = sum(m * m for m in bx[i])
        worst, offw = 0.0, 0.0
        for j in range(0, wl.ntau, 7):
            e, ob = _blocks_err(Pl, int(ctx.p_off[i]) + j * packed, bx[i], Pref[j], Ux[q])
            worst, offw = max(worst, e), max(offw, ob)
        say(f"  q {q}: P {worst / scale:.2e} (off-block {offw / scale:.1e})")
        assert offw < 1e-11 * scale
        assert worst < tol * scale
    ctx.close()


@pytest.mark.parametrize("name", ["cfg4"])
def test_find_mu_and_dyson_fullsize(name):
    wl = workload(name)
    dev = torch.device("cuda:0")
    inp = Inputs(wl)
    F = inp.fock().numpy()
    Y = inp.orb_matrices(2, scale=0.02).numpy()            # [nk, 2, nao, nao]
    f, g = _shapes(wl)
    Sig = f[None, :, None, None] * Y[:, None, 0] + g[None, :, None, None] * Y[:, None, 1]   # [nk, ntau, ...]
    n_target = oracle.free_count(F, 0.0, wl.beta, wl.spin)
    tol = bar(wl, False)
    say(f"[{name}] bar {tol:.1e}")
    ctx = make_context(wl)
    ctx.device_init()
    ibz = ctx.table("ibz")
    it = torch.as_tensor(ibz, device=dev)
    z = lambda n: torch.zeros(n, dtype=torch.complex128, device=dev)
    Fb, Sb, Gb = z(ctx.f_size), z(ctx.g_size), z(ctx.g_size)
    ctx.to_block(0, torch.as_tensor(F, device=dev)[it].contiguous(), Fb)
    ctx.to_block(1, torch.as_tensor(Sig, device=dev)[it].contiguous(), Sb)
    mu = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.find_mu(Fb, Sb, n_target, mu)
    ctx.dyson_G(Fb, Sb, mu, Gb)
    ctx.check()
    m = float(mu.item())
    say(f"[{name}] library mu {m:.15f}, N_target {n_target:.12f}")
    say(f"[{name}] oracle Dyson equation over all k at that mu")
    G, _, _ = oracle.dyson(F, Sig, m, wl.beta, wl.nw)
    N = oracle.particle_number(G, wl.spin)
    say(f"  N(mu) - N_target = {N - n_target:.2e}")
    assert abs(N - n_target) < tol * n_target
    # mu is the root: the count is below the target just under it and above just over it
    for d, sign in ((-1e-6, -1), (1e-6, 1)):
        Gd, _, _ = oracle.dyson(F, Sig, m + d, wl.beta, wl.nw)
        assert sign * (oracle.particle_number(Gd, wl.spin) - n_target) > 0
    Gl = Gb.cpu().numpy()
    bo = ctx.blocks()
    Uo = ctx.table("U_ao").reshape(wl.nk, wl.nao, wl.nao)
    worst, offw, scale = 0.0, 0.0, np.abs(G).max()
    for i, k in enumerate(ibz):
        packed = sum(s * s for s in bo[i])
        for j in range(0, wl.ntau, 9):
            e, ob = _blocks_err(Gl, int(ctx.g_off[i]) + j * packed, bo[i], G[k, j], Uo[k])
            worst, offw = max(worst, e), max(offw, ob)
    say(f"  G {worst / scale:.2e} (off-block {offw / scale:.1e})")
    assert offw < 1e-11 * scale
    assert worst < tol * scale
    ctx.close()
