"""Shared test helpers: contexts for named workloads and oracle inputs."""
import numpy as np

from gwinputs import Inputs, workload, crystal, add_k, minus_k


def crystal_arrays(cr):
    rot = np.array([W for W, _ in cr.ops])
    trans = np.array([w for _, w in cr.ops])
    return cr.lattice, cr.positions, rot, trans


def make_context(wl, mode=None, precision=0, half_tau=True, tau_chunk=0, build=True, identity_only=False, sched=0,
                 ir=None, blocks=None):
    """identity_only: give the library the trivial group (every block is the whole matrix,
    every mesh point is irreducible) although the inputs have the crystal's symmetry.
    blocks: the library's default (partner-function blocks) unless given."""
    from paper_2405_09494_amd import gwsym
    if mode is None:
        mode = gwsym.MODE_BLOCK
    if blocks is None:
        blocks = gwsym.BLOCKS_PARTNER
    nt, nw = (0, 0) if ir else (wl.ntau, wl.nw)
    ctx = gwsym.Context(wl.beta, nt, nw, wl.spin, mode, precision, half_tau, tau_chunk, sched, ir=ir, blocks=blocks)
    if build:
        cr = crystal(wl.crystal)
        lat, pos, rot, trans = crystal_arrays(cr)
        if identity_only:
            rot, trans = rot[:1], trans[:1]
        ctx.build_symmetry_basis(lat, pos, rot, trans, wl.n, wl.ao, wl.aux)
    return ctx


def sub_table(n):
    add, mk = add_k(n), minus_k(n)
    nk = n ** 3
    return np.array([[add[k, mk[q]] for q in range(nk)] for k in range(nk)])


def rel(a, b):
    """max-norm error relative to the largest reference entry"""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
