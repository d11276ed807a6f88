"""Shared steps of the parity tests at the full sizes of the two 6^3 workloads: cfg2 (rocksalt Fm-3m, nao 52, naux 250,
ntau 100) and cfg4 (diamond Fd-3m, non-symmorphic, nao 52, naux 300, ntau 128).  One P0^q(tau_j)
over every k (eq. P0) and one Sigma^k(tau_j) over every q (eq. sigma) are computed by the
oracle one at a time and compared with the library's block-packed outputs at the same point,
in the library's block basis: the oracle output X is rotated to U^H X U with the host U table
of that point, its off-block part must vanish (the symmetry the block form relies on) and its
diagonal blocks must match.  (A full-zone readout of P0 would take 40 GB at cfg4.)  The
Sigma check feeds a seeded symmetric stand-in for P at one tau and its mirror (zero
elsewhere).  Inputs are drawn once on the GPU and copied to the host for the oracle.  Bars:
1e-10 relative in FP64, 1e-6 with FP32 or three-piece bfloat16 contractions."""
import numpy as np
import pytest
import torch

import oracle
from gwinputs import Inputs, add_k, workload
from tests.gpu_common import say
from tests.helpers import make_context, sub_table


def blocks_of(M, sizes):
    """diagonal blocks of M and the largest off-block entry"""
    out, o = [], 0
    mask = np.ones(M.shape, bool)
    for s in sizes:
        out.append(M[o:o + s, o:o + s])
        mask[o:o + s, o:o + s] = False
        o += s
    return out, (np.abs(M[mask]).max() if mask.any() else 0.0)


def packed(buf, off, sizes):
    out, o = [], off
    for s in sizes:
        out.append(buf[o:o + s * s].reshape(s, s))
        o += s * s
    return out


def setup(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = workload(name)
    dev = torch.device("cuda:0")
    say(f"[{name}] inputs on the GPU (pair-keyed draws)")
    inp = Inputs(wl, device=dev)
    F = inp.fock()
    ctx = make_context(wl)
    say(f"[{name}] symmetry basis built")
    ibz = ctx.table("ibz")
    nk, nib = wl.nk, len(ibz)
    add, sub = add_k(wl.n), sub_table(wl.n)
    iq, j = min(3, nib - 1), wl.ntau // 3      # P0 output: irreducible q, tau index j
    ik, js = min(2, nib - 1), (2 * wl.ntau) // 3   # Sigma output: irreducible k, tau index js
    q, k = int(ibz[iq]), int(ibz[ik])
    Vq = inp.three_index([(kk, int(add[kk, q])) for kk in range(nk)]).cpu().numpy()
    Vk = inp.three_index([(k, int(sub[k, qq])) for qq in range(nk)]).cpu().numpy()
    Vibz = torch.empty((nib, nk, wl.naux, wl.nao, wl.nao), dtype=torch.complex128, device=dev)
    for i in range(nib):
        Vibz[i] = inp.three_index([(int(ibz[i]), kp) for kp in range(nk)])
        say(f"[{name}] V row {i + 1} of {nib}")
    say(f"[{name}] stand-in P")
    X = inp.aux_matrices(1)[:, 0]    # [nk, naux, naux], symmetric Hermitian stand-in for P(tau_js)
    torch.cuda.empty_cache()
    Fh = F.cpu().numpy()
    tau = oracle.tau_grid(wl.beta, wl.ntau)
    say(f"[{name}] oracle G0")
    G0 = oracle.g0_closed_form(Fh, 0.0, wl.beta, tau)
    say(f"[{name}] oracle P0 output")
    ref_p0 = oracle.polarization_unit(G0, Vq, add, q, j, wl.spin)
    say(f"[{name}] oracle Sigma output")
    ref_s = oracle.self_energy_unit(G0, Vk, X.cpu().numpy(), sub, k, js)
    del G0, Vq, Vk
    Ux = ctx.table("U_aux").reshape(nk, wl.naux, wl.naux)[q]
    Uo = ctx.table("U_ao").reshape(nk, wl.nao, wl.nao)[k]
    ctx.close()
    return dict(wl=wl, dev=dev, F=F, Vibz=Vibz, X=X, ibz=ibz, iq=iq, j=j, ik=ik, js=js, ref_p0=ref_p0,
                ref_s=ref_s, Ux=Ux, Uo=Uo)


def run(d, precision):
    wl, dev = d["wl"], d["dev"]
    say(f"[{wl.name}] library, precision {precision}")
    ctx = make_context(wl, precision=precision)
    say(f"[{wl.name}] device tables and plans")
    ctx.device_init()
    ctx.load_V(d["Vibz"])
    torch.cuda.synchronize()
    say(f"[{wl.name}] V loaded")
    z = lambda n: torch.zeros(n, dtype=torch.complex128, device=dev)
    Fb, G, P0, Pb, S = z(ctx.f_size), z(ctx.g_size), z(ctx.p_size), z(ctx.p_size), z(ctx.g_size)
    ibz_t = torch.as_tensor(d["ibz"], device=dev)
    ctx.to_block(0, d["F"][ibz_t].contiguous(), Fb)
    ctx.g0(Fb, 0.0, G)
    ctx.polarization(G, P0)
    torch.cuda.synchronize()
    say(f"[{wl.name}] polarization done")
    nt = wl.ntau
    Pin = torch.zeros((len(d["ibz"]), nt, wl.naux, wl.naux), dtype=torch.complex128, device=dev)
    Pin[:, d["js"]] = d["X"][ibz_t]
    Pin[:, nt - 1 - d["js"]] = d["X"][ibz_t]
    ctx.to_block(2, Pin, Pb)
    del Pin
    ctx.self_energy(G, Pb, S)
    torch.cuda.synchronize()
    say(f"[{wl.name}] self-energy done")
    bx, bo = ctx.blocks(aux=True)[d["iq"]], ctx.blocks()[d["ik"]]
    p0 = packed(P0.cpu().numpy(), int(ctx.p_off[d["iq"]]) + d["j"] * sum(s * s for s in bx), bx)
    s = packed(S.cpu().numpy(), int(ctx.g_off[d["ik"]]) + d["js"] * sum(s * s for s in bo), bo)
    ctx.close()
    torch.cuda.empty_cache()
    return p0, s, bx, bo


def compare(d, p0, s, bx, bo, tol):
    Bp, offp = blocks_of(d["Ux"].conj().T @ d["ref_p0"] @ d["Ux"], bx)
    Bs, offs = blocks_of(d["Uo"].conj().T @ d["ref_s"] @ d["Uo"], bo)
    sp, ss = np.abs(d["ref_p0"]).max(), np.abs(d["ref_s"]).max()
    e0 = max(np.abs(a - b).max() for a, b in zip(p0, Bp)) / sp
    es = max(np.abs(a - b).max() for a, b in zip(s, Bs)) / ss
    say(f"  off-block P0 {offp / sp:.1e} Sigma {offs / ss:.1e}; P0 {e0:.2e} Sigma {es:.2e}")
    assert offp < 1e-11 * sp and offs < 1e-11 * ss
    assert e0 < tol and es < tol


