"""GPU-side helpers for the parity tests: run the library's iteration for a workload and
read every quantity back as full matrices over the full Brillouin zone, and run the
oracle on the same seeded inputs."""
import functools
import sys
import time

import numpy as np
import torch

import oracle
from gwinputs import Inputs, workload, add_k
from tests.helpers import make_context, sub_table


from tests.progress import say  # noqa: F401  (re-exported for the test modules)


@functools.lru_cache(maxsize=None)
def inputs(name):
    wl = workload(name)
    inp = Inputs(wl)
    F = inp.fock().numpy()
    V = inp.three_index_full().numpy()
    return wl, inp, F, V


@functools.lru_cache(maxsize=None)
def oracle_run(name, iterations=1, ir=None):
    """ir: None (the workload's Chebyshev grid) or (wmax, eps) of an IR grid built by the oracle"""
    wl, inp, F, V = inputs(name)
    grid = oracle.ir_grid(wl.beta, ir[0], ir[1]) if ir else None
    tau = grid["tau"] if grid else oracle.tau_grid(wl.beta, wl.ntau)
    nw = len(grid["nf"]) if grid else wl.nw
    G = oracle.g0_closed_form(F, 0.0, wl.beta, tau)
    add, sub = add_k(wl.n), sub_table(wl.n)
    nt = None if wl.mu_fixed else oracle.free_count(F, 0.0, wl.beta, wl.spin)
    out = dict(G0=G, n_target=nt, iters=[])
    mu = 0.0
    for _ in range(iterations):
        r = oracle.gw_iteration(F, V, G, mu, wl.beta, nw, wl.spin, add, sub, n_target=nt, grid=grid)
        out["iters"].append(r)
        G, mu = r["G"], r["mu"]
    return out


class DeviceRun:
    """Device buffers and calls of one workload in one mode."""

    def __init__(self, name, mode, half_tau=True, tau_chunk=0, precision=0, identity_only=False, sched=0, ir=None):
        wl, inp, F, V = inputs(name)
        self.wl = wl
        self.ctx = make_context(wl, mode=mode, half_tau=half_tau, tau_chunk=tau_chunk, precision=precision,
                                identity_only=identity_only, sched=sched, ir=ir)
        c = self.ctx
        dev = torch.device("cuda:0")
        self.dev = dev
        c.device_init()
        ibz = c.table("ibz")
        self.ibz = ibz
        Vi = torch.as_tensor(np.ascontiguousarray(V[ibz]), device=dev)
        c.load_V(Vi)
        Ff = torch.as_tensor(np.ascontiguousarray(F[ibz]), device=dev)
        self.F = torch.zeros(c.f_size, dtype=torch.complex128, device=dev)
        c.to_block(0, Ff, self.F)
        z = lambda n: torch.zeros(n, dtype=torch.complex128, device=dev)
        self.G, self.P0, self.P, self.S = z(c.g_size), z(c.p_size), z(c.p_size), z(c.g_size)
        self.mu = torch.zeros(1, dtype=torch.float64, device=dev)
        self.nfree = torch.zeros(1, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()

    def full(self, kind, blk):
        c = self.ctx
        nb = c.naux if kind == 2 else c.nao
        nt = 1 if kind == 0 else c.ntau
        out = torch.zeros(c.nk * nt * nb * nb, dtype=torch.complex128, device=self.dev)
        c.from_block(kind, blk, out)
        torch.cuda.synchronize()
        return out.cpu().numpy().reshape(c.nk, nt, nb, nb) if kind else out.cpu().numpy().reshape(c.nk, nb, nb)

    def g0(self, mu=0.0):
        self.ctx.g0(self.F, mu, self.G, self.nfree)

    def iteration(self, n_target=None):
        c = self.ctx
        c.polarization(self.G, self.P0)
        c.screened_interaction(self.P0, self.P)
        c.self_energy(self.G, self.P, self.S)
        if n_target is not None:
            c.find_mu(self.F, self.S, n_target, self.mu)
        c.dyson_G(self.F, self.S, self.mu, self.G)
