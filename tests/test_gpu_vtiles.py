"""Sec. 4.3: the tiles of V that the contractions skip.  In the symmetry-adapted bases a
(auxiliary block s, orbital block r, orbital block r') tile of V^{k1,k2} can vanish by symmetry;
the library flags such tiles at load time and the P0 and Sigma orbital GEMMs leave them out.

The flags are index work, so they are compared exactly with flags computed here in numpy from
the generator's V and the basis tables (U^k, block sizes) of the host symmetry code: a tile is
kept when its squared Frobenius norm exceeds 1e-26 times that of its pair.  The contractions that
skip the tiles are held to the oracle by the parity tests, which run on these workloads."""
import numpy as np
import pytest
import torch

from gwinputs import add_k
from tests.gpu_common import DeviceRun, inputs, say
from tests.helpers import sub_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(int)


def _tile_flags(T, sx, sa, sb):
    """T[s, a, b] in the block bases; flags per (s block, a block, b block), row-major"""
    ox, oa, ob = _offsets(sx), _offsets(sa), _offsets(sb)
    A = np.abs(T) ** 2
    n = np.array([[[A[ox[s]:ox[s + 1], oa[r]:oa[r + 1], ob[t]:ob[t + 1]].sum() for t in range(len(sb))]
                   for r in range(len(sa))] for s in range(len(sx))])
    return (n > 1e-26 * A.sum()).astype(np.int64).ravel()


@pytest.mark.parametrize("name", ["small_diamond", "small_hbn", "small_sc4"])
def test_vtile_flags(name):
    say(f"[vtiles] {name}")
    run = DeviceRun(name, 2)
    wl, inp, F, V = inputs(name)
    c = run.ctx
    nk, no, na = wl.nk, wl.nao, wl.naux
    ibz, rep = c.table("ibz"), c.table("rep")
    Uo = c.table("U_ao").reshape(nk, no, no)
    Ux = c.table("U_aux").reshape(nk, na, na)
    bo, bx = c.blocks(), c.blocks(aux=True)
    add, sub = add_k(wl.n), sub_table(wl.n)
    got = {"s": c.table("vtile_flags_s"), "p": c.table("vtile_flags_p")}
    off = {"s": c.table("vtile_off_s"), "p": c.table("vtile_off_p")}
    total = {"s": [0, 0], "p": [0, 0]}
    for i, k0 in enumerate(ibz):
        for k in range(nk):
            p = i * nk + k
            # self-energy copy: V^{k0,k'} with Q at k0 - k' (coefficients U^q, unconjugated)
            q = int(sub[k0, k])
            X = Uo[k0].conj().T[None] @ V[k0, k] @ Uo[k][None]
            T = np.einsum("Qs,Qab->sab", Ux[q], X)
            want = _tile_flags(T, bx[rep[q]], bo[i], bo[rep[k]])
            have = got["s"][off["s"][p]:off["s"][p + 1]]
            assert np.array_equal(have, want), (name, "self-energy copy", i, k)
            total["s"][0] += want.size
            total["s"][1] += int(want.sum())
            # polarization copy: V^{k,k+q0} with Q at q0 (coefficients conj U^{q0})
            kq = int(add[k, k0])
            X = Uo[k].conj().T[None] @ V[k, kq] @ Uo[kq][None]
            T = np.einsum("Qs,Qab->sab", Ux[k0].conj(), X)
            want = _tile_flags(T, bx[i], bo[rep[k]], bo[rep[kq]])
            have = got["p"][off["p"][p]:off["p"][p + 1]]
            assert np.array_equal(have, want), (name, "polarization copy", i, k)
            total["p"][0] += want.size
            total["p"][1] += int(want.sum())
    st = c.table("vtile_stats")
    assert list(st[:4]) == [total["s"][0], total["s"][1], total["p"][0], total["p"][1]]
    say(f"  kept tiles {total['s'][1]}/{total['s'][0]} (self-energy), {total['p'][1]}/{total['p'][0]} "
        f"(polarization); GEMM MACs kept P0 {st[5] / st[4]:.3f}, Sigma orbital {st[7] / st[6]:.3f}")
    # these crystals have symmetry-forbidden tiles, and skipping them lowers the GEMM work; where
    # it saves more than 30 % of a stage's multiply-adds, that stage's launches skip them
    assert total["s"][1] < total["s"][0] and total["p"][1] < total["p"][0]
    assert st[5] < st[4] and st[7] < st[6]
    say(f"  launches skipping tiles: P0 {int(st[8])}/{int(st[10])}, Sigma orbital {int(st[9])}/{int(st[11])}")
    if st[5] < 0.7 * st[4]:
        assert st[8] > 0
    if st[7] < 0.7 * st[6]:
        assert st[9] > 0
