#!/usr/bin/env python3
"""Seconds per symmetry-adapted GW iteration on one MI355X.

A step is one GW iteration of the hot path: P0 contraction, screened interaction
(tau -> i Omega, per-block Dyson, back), Sigma contraction, chemical-potential bisection
and the Dyson equation for G, in the irreducible wedge and partner-function blocks (FP64).  The
default workload is the largest single-GPU one: diamond Fd-3m on a 6x6x6 mesh, nao 52,
naux 300, ntau 128 ("cfg4").  Inputs are seeded synthetic tensors of the workload's shapes,
resident in HBM before the timed region; each timed iteration is one replay of a HIP graph.

    python bench.py [--steps K] [--warmup W] [--workload cfg4] [--legs fp32,bf16x6,full,unbatched]
                    [--no-cpu]

--legs adds comparison runs that are not part of the headline: the same block path with
reduced-precision contractions, the full-matrix form without symmetry (all-pair V, so cfg0 and
cfg1 only), and the unbatched per-block schedule.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s/GW iteration + contraction TFLOP/s, block-grouped vs full FP64, at ≤1e-6 rel Σ err"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
RIDGE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)   # flop per byte where the two bounds meet


PLANS_FILE = os.path.join(ROOT, "paper_2405_09494_amd", "plans.json")
CRYSTAL_NAMES = {"sc": "simple cubic Pm-3m", "rocksalt": "rocksalt Fm-3m (two atoms)",
                 "diamond": "diamond Fd-3m (two atoms, non-symmorphic)"}


def source_digest():
    """sha256 over the kernel and launch-plan sources, the default launch plan and the stored
    launch plans: measured counters apply only to the code and plans they were taken from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("csrc/kernels.hip", "csrc/bdiag.hip", "csrc/pipeline.hip", "csrc/capi.cpp", "plans.json"):
        path = os.path.join(ROOT, "paper_2405_09494_amd", f)
        if os.path.exists(path):
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, cls):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of the workload, or None when there is none or it was taken from other
    kernel sources."""
    try:
        text = open(os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")).read()
    except OSError:
        return None
    digest = None
    for line in text.splitlines():
        if line.startswith("source-sha256:"):
            digest = line.split(":", 1)[1].strip()
    if digest != source_digest():
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == cls:
            try:
                return float(cells[-1])
            except ValueError:
                return None
    return None


CONTRACTIONS = {"polarization (eq. P0)": ("p0_contraction", "two_sided_block_multiply"),
                "self-energy (eq. sigma)": ("sigma_aux_contraction", "row_block_multiply", "sigma_orb_contraction")}


_T0 = time.perf_counter()


def log(*a):
    print(f"[{time.perf_counter() - _T0:7.1f} s]", *a, file=sys.stderr, flush=True)


def make_ctx(wl, mode, half_tau=True, tau_chunk=0, precision=0, sched=0):
    from gwinputs import crystal
    from paper_2405_09494_amd import gwsym
    cr = crystal(wl.crystal)
    rot = np.array([W for W, _ in cr.ops])
    trans = np.array([w for _, w in cr.ops])
    ctx = gwsym.Context(wl.beta, wl.ntau, wl.nw, wl.spin, mode, precision, half_tau, tau_chunk, sched)
    ctx.build_symmetry_basis(cr.lattice, cr.positions, rot, trans, wl.n, wl.ao, wl.aux)
    return ctx


class Path:
    """Device state of one mode: F, G, P0, P, Sigma, mu, and the iteration."""

    def __init__(self, ctx, F_all, V_src, torch, dev, graph=False):
        """V_src: V over every pair [Nk, Nk, ...], or a function of the irreducible indices
        that returns V for those rows."""
        self.ctx, self.torch = ctx, torch
        self.graph = torch.cuda.Stream() if graph else None
        ctx.device_init()
        log("[bench] device state initialised")
        ibz = torch.as_tensor(ctx.table("ibz"), device=dev)
        V = V_src(ibz) if callable(V_src) else V_src[ibz].contiguous()
        torch.cuda.synchronize()
        log("[bench] irreducible rows of V ready")
        ctx.load_V(V)
        del V
        torch.cuda.synchronize()
        log("[bench] V in block form (both device copies)")
        z = lambda n: torch.zeros(n, dtype=torch.complex128, device=dev)
        self.F, self.G, self.P0, self.P, self.S = z(ctx.f_size), z(ctx.g_size), z(ctx.p_size), z(ctx.p_size), z(ctx.g_size)
        ctx.to_block(0, F_all[ibz].contiguous(), self.F)
        self.mu = torch.zeros(1, dtype=torch.float64, device=dev)
        self.nfree = torch.zeros(1, dtype=torch.float64, device=dev)
        ctx.g0(self.F, 0.0, self.G, self.nfree)
        torch.cuda.synchronize()
        self.n_target = float(self.nfree.item())
        self.G0 = self.G.clone()

    def step(self, eager=False, restart=True):
        """One GW iteration.  restart: from G0 (every timed step is the same iteration: repeated
        undamped iterations on the synthetic inputs do not settle, and at the diamond 6^3
        workload the chemical potential leaves its bracket within 25 of them); the cost of an
        iteration does not depend on the values.  restart=False continues from the current G."""
        c = self.ctx
        if restart:
            self.G.copy_(self.G0)
        if self.graph is not None and not eager:
            # the whole iteration replayed from one captured HIP graph on a side stream
            self.torch.cuda.current_stream().synchronize()
            c.iteration(self.F, self.G, self.P0, self.P, self.S, self.mu, self.n_target, use_graph=True,
                        stream=self.graph)
            self.graph.synchronize()
            return
        c.polarization(self.G, self.P0)
        c.screened_interaction(self.P0, self.P)
        c.self_energy(self.G, self.P, self.S)
        c.find_mu(self.F, self.S, self.n_target, self.mu)
        c.dyson_G(self.F, self.S, self.mu, self.G)

    def full(self, kind, blk):
        c, torch = self.ctx, self.torch
        nb = c.naux if kind == 2 else c.nao
        out = torch.zeros(c.nk * c.ntau * nb * nb, dtype=torch.complex128, device=blk.device)
        c.from_block(kind, blk, out)
        return out


def iteration_errors(ref, red, n, torch):
    """[P0 rel, Sigma rel, occupation abs] after each of n iterations run by both paths from the
    same G0 (mu from the electron count in both)."""
    nk_, nt_, no_ = ref.ctx.nk, ref.ctx.ntau, ref.ctx.nao
    occ = lambda g: -torch.diagonal(g.view(nk_, nt_, no_, no_)[:, -1], dim1=-2, dim2=-1).real
    for pth in (ref, red):
        pth.ctx.g0(pth.F, 0.0, pth.G, pth.nfree)
    hist = []
    for _ in range(n):
        for pth in (ref, red):
            pth.step(eager=True, restart=False)
        torch.cuda.synchronize()
        a, b = red.full(2, red.P0), ref.full(2, ref.P0)
        e0 = float((a - b).abs().max() / b.abs().max())
        del a, b
        a, b = red.full(1, red.S), ref.full(1, ref.S)
        es = float((a - b).abs().max() / b.abs().max())
        a, b = red.full(1, red.G), ref.full(1, ref.G)
        eo = float((occ(a) - occ(b)).abs().max())
        hist.append((e0, es, eo))
    return hist


def time_steps(path, steps, warmup, torch):
    """Seconds per step over `steps` timed steps after `warmup` untimed ones.  Each step ends
    with its stream synchronised, so a progress line per finished step (stderr, microseconds)
    keeps a long run visibly alive without adding device work."""
    for w in range(warmup):
        path.step()
        torch.cuda.synchronize()
        log(f"[bench] warm-up step {w + 1} of {warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        path.step()
        if path.graph is None:
            torch.cuda.synchronize()
        log(f"[bench] step {k + 1} of {steps} done ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1)


def profile_step(path, torch):
    path.ctx.profile(True)
    path.step(eager=True)   # per-launch events need the launches themselves, not a graph replay
    torch.cuda.synchronize()
    prof = path.ctx.profile_read()
    path.ctx.profile(False)
    return prof


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(wl, F_all, vpairs, ibz_rep_q, torch):
    """The FP64 oracle (full matrices, no symmetry) on the host, timed on a bounded sample of
    one iteration at the workload's shapes and scaled to a full iteration (Nk x ntau outputs of
    each contraction, Nk screened-interaction momenta, 65 Dyson solves for the bisection):
    with every BLAS thread, up to 32 P0 outputs (one q, every k) and 32 Sigma outputs (one k,
    every q) within about 6 s each, the screened interaction of 4 momenta (1 at the 6^3 sizes)
    and one Dyson solve over every k (8 of the k at the 6^3 sizes, scaled); and with one BLAS
    thread, one output of each contraction where that takes seconds."""
    import oracle
    from gwinputs import add_k, minus_k
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    nk, nt = wl.nk, wl.ntau
    ns = min(32, nt)
    add = add_k(wl.n)
    mk = minus_k(wl.n)
    sub = np.array([[add[k, mk[q]] for q in range(nk)] for k in range(nk)])
    F = F_all.cpu().numpy()
    tau = oracle.tau_grid(wl.beta, nt)
    G = oracle.g0_closed_form(F, 0.0, wl.beta, tau)
    q = k = ibz_rep_q
    Vq = vpairs([(kk, int(add[kk, q])) for kk in range(nk)]).cpu().numpy()
    Vk = vpairs([(k, int(sub[k, qq])) for qq in range(nk)]).cpu().numpy()
    rng = np.random.default_rng(0)
    Ph = rng.standard_normal((nk, wl.naux, wl.naux)) * 1e-3
    Ph = Ph + Ph.transpose(0, 2, 1)

    def contractions(nmax, limit):
        t, n_p0 = time.perf_counter(), 0
        while n_p0 < nmax and (n_p0 == 0 or time.perf_counter() - t < limit):
            oracle.polarization_unit(G, Vq, add, q, n_p0, wl.spin)
            n_p0 += 1
        t_p0 = (time.perf_counter() - t) / n_p0
        t, n_s = time.perf_counter(), 0
        while n_s < nmax and (n_s == 0 or time.perf_counter() - t < limit):
            oracle.self_energy_unit(G, Vk, Ph, sub, k, n_s)
            n_s += 1
        return t_p0, n_p0, (time.perf_counter() - t) / n_s, n_s

    t_p0, n_p0, t_s, n_s = contractions(ns, 6.0)
    # the screened interaction per momentum and the Dyson solve per k scale linearly: a few of
    # each at the 6^3 sizes (one momentum takes seconds there, one Dyson solve over all k minutes)
    nq = 1 if wl.pairwise else min(4, nk)
    X = rng.standard_normal((nq, nt, wl.naux, wl.naux)) * 1e-3
    X = X + X.transpose(0, 1, 3, 2)
    t = time.perf_counter()
    oracle.screened(X.astype(complex), wl.beta, wl.nw)
    t_scr = (time.perf_counter() - t) / nq
    nkd = min(8, nk) if wl.pairwise else nk
    S0 = np.zeros((nkd, nt, wl.nao, wl.nao), complex)
    t = time.perf_counter()
    oracle.dyson(F[:nkd], S0, 0.0, wl.beta, wl.nw)
    t_dys = (time.perf_counter() - t) * nk / nkd
    total = (t_p0 + t_s) * nk * nt + t_scr * nk + 65 * t_dys
    sample = (f"measured: {n_p0} P0 outputs (q={q}, all {nk} k) at {t_p0:.3f} s each, {n_s} Sigma outputs (k={k}, "
              f"all {nk} q) at {t_s:.3f} s each, screened interaction for {nq} momenta at {t_scr:.2f} s each, "
              f"Dyson solve for {nkd} of the {nk} k (scaled to all k: {t_dys:.2f} s); scaled to {nk * nt} outputs "
              f"of each contraction, {nk} momenta and 65 Dyson solves over all k")
    # one BLAS thread: one output of each contraction (the bulk of the work), where that stays
    # within about 15 s (at the 6^3 sizes one output alone would take a minute or more)
    if (t_p0 + t_s) * cores <= 15.0:
        with threadpool_limits(limits=1):
            t1_p0, _, t1_s, _ = contractions(1, 0.0)
        single = {"value": (t1_p0 + t1_s) * nk * nt, "unit": "s/iteration (contractions only)", "cores": 1,
                  "sample": f"one BLAS thread: one P0 output ({t1_p0:.2f} s) and one Sigma output ({t1_s:.2f} s), "
                            f"scaled to {nk * nt} outputs of each"}
    else:
        single = {"value": None, "unit": "s/iteration (contractions only)", "cores": 1,
                  "sample": f"not measured: one output of each contraction took {t_p0 + t_s:.1f} s on {cores} "
                            f"threads"}
    return {"value": total, "unit": "s/iteration", "cores": int(cores), "kind": "oracle", "sample": sample,
            "extrapolated": True, "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "single_thread": single}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg4")
    ap.add_argument("--tau-chunk", type=int, default=0)
    ap.add_argument("--legs", default=None,
                    help="comma-separated comparison runs: fp32, bf16x6, bf16x3 (reduced-precision contractions), "
                         "full (no symmetry, all-pair V: cfg0/cfg1 only), full_sample (the full-matrix form of a "
                         "6^3 workload timed on a 2^3 mesh of the same crystal and bases, scaled to Nk^2 pairs), "
                         "unbatched (per-block launches), none; default: full_sample on the 6^3 workloads, none otherwise")
    ap.add_argument("--graph", type=int, default=1, help="1 (default): replay each iteration from a captured HIP graph; 0: eager launches")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1 (default): each block path takes its launch plan from --plans, or times candidate "
                         "plans (gwsym_autotune) when the file has none for this workload and device (small "
                         "workloads only); 0: default plan")
    ap.add_argument("--plans", default=PLANS_FILE, help="JSON file of autotuned launch plans")
    ap.add_argument("--no-exchange", action="store_true", help="skip timing the exchange term (profiling runs)")
    ap.add_argument("--error-iterations", type=int, default=10,
                    help="iterations over which the reduced-precision legs are compared with the FP64 path")
    ap.add_argument("--update-plans", action="store_true", help="add newly autotuned plans to --plans")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="before the timed steps, copy a buffer of this many MiB once (a plain copy kernel "
                         "of known traffic, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding over several GPUs is "
              "designed (pairs split by flops, one all-reduce of P0 and Sigma per iteration) but not "
              "implemented", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in (args.legs or "").split(",") if x and x != "none"]
    for x in legs:
        if x not in ("fp32", "bf16x6", "bf16x3", "full", "full_sample", "unbatched"):
            ap.error(f"unknown leg {x!r}")

    import torch
    from gwinputs import Inputs, workload
    from paper_2405_09494_amd import gwsym

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = workload(args.workload)
    if "full" in legs and wl.pairwise:
        ap.error("the full-matrix leg needs V over every pair, which the 6^3 workloads cannot hold (full_sample)")
    if args.legs is None and wl.pairwise:
        legs = ["full_sample"]
    log(f"[bench] workload {wl.name}: {wl.crystal} n={wl.n} nao={wl.nao} naux={wl.naux} ntau={wl.ntau} beta={wl.beta}")
    t = time.perf_counter()
    inp = Inputs(wl, device=dev)
    F_all = inp.fock()
    if wl.pairwise:
        # 6^3 meshes: only the irreducible rows of V are drawn (V over every pair would not fit)
        V_all, rows = None, {}

        def V_src(ibz):
            key = tuple(ibz.tolist())
            if key not in rows:
                rows.clear()
                V = torch.empty((len(key), wl.nk, wl.naux, wl.nao, wl.nao), dtype=torch.complex128, device=dev)
                for i, k0 in enumerate(key):
                    V[i] = inp.three_index([(k0, kp) for kp in range(wl.nk)])
                    log(f"[bench] V row {i + 1} of {len(key)}")
                rows[key] = V
                torch.cuda.empty_cache()
            return rows[key]
    else:
        V_all = inp.three_index_full()
        V_src = V_all
    torch.cuda.synchronize()
    log(f"[bench] inputs generated in {time.perf_counter() - t:.1f} s")

    if args.copy_calib_mb > 0:
        n = args.copy_calib_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calib_mb} MiB done")
        del a, b

    def plan_for(path):
        if not args.autotune:
            return path.ctx.get_tuning(), "default"
        tuning = path.ctx.autotune(cache=args.plans, update=args.update_plans, time_missing=not wl.pairwise)
        return tuning, getattr(path.ctx, "plan_source", "default")

    # ---- block-grouped, irreducible wedge, FP64 (the headline) ----
    t = time.perf_counter()
    ctx_blk = make_ctx(wl, gwsym.MODE_BLOCK, tau_chunk=args.tau_chunk)
    log("[bench] symmetry-adapted basis built")
    blk = Path(ctx_blk, F_all, V_src, torch, dev,
               graph=bool(args.graph))
    log(f"[bench] block path set up in {time.perf_counter() - t:.1f} s; N_target={blk.n_target:.6f}")
    t = time.perf_counter()
    tuning, plan_source = plan_for(blk)
    log(f"[bench] launch plan, {plan_source} ({time.perf_counter() - t:.1f} s): {tuning}")
    s_blk = time_steps(blk, args.steps, args.warmup, torch)
    blk.ctx.check()
    log(f"[bench] block: {s_blk:.4f} s/iteration")
    prof = profile_step(blk, torch)
    p0_macs, s_macs = blk.ctx.flop_counts()
    log("[bench] profile: " + ", ".join(f"{k} {v[0]:.1f} ms/{v[1]}" for k, v in prof.items()))

    # per contraction: every kernel class it launches, block-executed flops, one call per iteration
    def contraction(name, classes):
        ms = sum(prof[k][0] for k in classes)
        flops = 8.0 * sum(prof[k][2] for k in classes)
        traffic = [measured_traffic(wl.name, k) for k in classes]
        launches = {k: prof[k][1] for k in classes}
        achieved = flops / (ms * 1e-3) / 1e12
        return {"kernel": name, "kernels": list(classes), "bound": "mfma", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": (sum(traffic) if all(x is not None for x in traffic) else None),
                "per_call_flops": flops, "per_call_ms": ms, "launches_per_call": launches}

    contr = {name: contraction(name, cl) for name, cl in CONTRACTIONS.items()}
    dom = max(contr, key=lambda k: contr[k]["per_call_ms"])
    for name, r in contr.items():
        log(f"[bench] {name}: {r['per_call_ms']:.1f} ms, {r['achieved']:.1f} TF/s = {r['frac']:.3f} of FP64 MFMA peak")
    flops_iter = sum(r["per_call_flops"] for r in contr.values())
    contr_ms = sum(r["per_call_ms"] for r in contr.values())

    # per kernel class (for the profiles): bound chosen by the algorithmic intensity
    def class_roofline(name):
        ms, nl, macs, nbytes = prof[name]
        flops = 8.0 * macs
        avg_s = ms / nl * 1e-3
        entry = {"avg_launch_ms": ms / nl, "launches": nl, "per_launch_flops": flops / nl,
                 "per_launch_bytes": nbytes / nl}
        if nbytes > 0 and flops / nbytes < RIDGE:
            entry.update({"bound": "hbm", "achieved": nbytes / nl / avg_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"})
        else:
            entry.update({"bound": "mfma", "achieved": flops / nl / avg_s / 1e12, "peak": PEAK_FP64_TFLOPS,
                          "unit": "TFLOP/s"})
        entry["frac"] = entry["achieved"] / entry["peak"]
        entry["traffic"] = measured_traffic(wl.name, name)
        return entry

    kernels = {k: class_roofline(k) for cl in CONTRACTIONS.values() for k in cl if prof[k][1] > 0}

    # tiles of V that symmetry makes zero (Sec. 4.3) and the GEMM work skipped with them
    vt = blk.ctx.table("vtile_stats")
    vtiles = {"self_energy_copy_tiles_kept": [int(vt[1]), int(vt[0])],
              "polarization_copy_tiles_kept": [int(vt[3]), int(vt[2])],
              "p0_gemm_flops_all_tiles": 8.0 * vt[4], "p0_gemm_flops_kept_tiles": 8.0 * vt[5],
              "sigma_orbital_gemm_flops_all_tiles": 8.0 * vt[6], "sigma_orbital_gemm_flops_kept_tiles": 8.0 * vt[7],
              "p0_gemm_launches_skipping_tiles": [int(vt[8]), int(vt[10])],
              "sigma_orbital_gemm_launches_skipping_tiles": [int(vt[9]), int(vt[11])]}
    log(f"[bench] V tiles kept: self-energy copy {int(vt[1])}/{int(vt[0])}, polarization copy "
        f"{int(vt[3])}/{int(vt[2])}; GEMM flops on kept tiles / all: P0 {vt[5] / max(vt[4], 1):.4f}, "
        f"Sigma orbital {vt[7] / max(vt[6], 1):.4f}; launches skipping tiles: P0 {int(vt[8])}/{int(vt[10])}, "
        f"Sigma orbital {int(vt[9])}/{int(vt[11])}")

    # static self-energy (eq. sigma_hf) from the current G, once each: K, J and F = H0 + J + K
    exchange_ms = hartree_ms = fock_ms = None
    if not args.no_exchange:
        Kx = torch.zeros(blk.ctx.f_size, dtype=torch.complex128, device=dev)

        def once(call):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            call()
            ev0.record()
            call()
            ev1.record()
            torch.cuda.synchronize()
            return ev0.elapsed_time(ev1)

        exchange_ms = once(lambda: blk.ctx.exchange(blk.G, Kx))
        hartree_ms = once(lambda: blk.ctx.hartree(blk.G, Kx))
        fock_ms = once(lambda: blk.ctx.fock(blk.F, blk.G, Kx))
        log(f"[bench] Sigma_HF: exchange {exchange_ms:.2f} ms, Hartree {hartree_ms:.3f} ms, "
            f"F = H0 + J + K {fock_ms:.2f} ms")
        del Kx

    out = {"metric": METRIC, "value": s_blk, "unit": "s/iteration", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * s_blk, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{wl.name}: {CRYSTAL_NAMES[wl.crystal]}, Gamma-centred {wl.n}^3 k mesh "
                                  f"(Nk={wl.nk}, {blk.ctx.nibz} irreducible), nao={wl.nao}, naux={wl.naux}, "
                                  f"ntau={wl.ntau}, nw={wl.nw}, beta={wl.beta}",
                      "mode": "irreducible wedge + partner-function blocks, grouped contractions", "precision": "fp64"},
           "contraction_tflops": flops_iter / (contr_ms * 1e-3) / 1e12 if contr_ms > 0 else None,
           "algorithmic_flops_per_iteration": flops_iter,
           "contractions": contr,
           "profile_ms": {k: v[0] for k, v in prof.items()},
           "exchange_ms": exchange_ms, "hartree_ms": hartree_ms, "fock_ms": fock_ms,
           "launch_plan": tuning, "launch_plan_source": plan_source,
           "kernels": kernels, "v_tiles": vtiles,
           "roofline": contr[dom]}

    # ---- comparison legs (not part of the headline) ----
    if "full" in legs:
        full = Path(make_ctx(wl, gwsym.MODE_FULL, tau_chunk=args.tau_chunk), F_all, V_all, torch, dev)
        blk.ctx.g0(blk.F, 0.0, blk.G, blk.nfree)   # one iteration from the same G0 in both forms
        full.step()
        blk.step()
        torch.cuda.synchronize()
        a, b = full.full(1, full.S), blk.full(1, blk.S)
        err = float((a - b).abs().max() / b.abs().max())
        s_full = time_steps(full, 1, 0, torch)
        fp0, fs = full.ctx.flop_counts()
        out["full_fp64"] = {"s_per_iteration": s_full, "speedup_block_vs_full": s_full / s_blk,
                            "algorithmic_flops_per_iteration": 8.0 * (fp0 + fs), "sigma_rel_err_block_vs_full": err}
        log(f"[bench] full: {s_full:.3f} s/iteration, Sigma block vs full {err:.2e}")
        del full
    if "full_sample" in legs:
        # V over every pair of a 6^3 mesh does not fit (606 GB at cfg4): the full-matrix FP64 form
        # runs on the 2^3 mesh of the same crystal, bases, grid and temperature (64 pairs), and its
        # contraction time is scaled by the pair count, (Nk / 8)^2, the rest by Nk / 8
        import dataclasses
        wls = dataclasses.replace(wl, name=wl.name + "_2x2x2", n=2, pairwise=False)
        inp_s = Inputs(wls, device=dev)
        fpath = Path(make_ctx(wls, gwsym.MODE_FULL, tau_chunk=args.tau_chunk), inp_s.fock(),
                     inp_s.three_index_full(), torch, dev)
        s_sample = time_steps(fpath, 1, 1, torch)
        prof_f = profile_step(fpath, torch)
        cls_c = {c for v in CONTRACTIONS.values() for c in v}
        c_ms = sum(v[0] for k, v in prof_f.items() if k in cls_c)
        r_ms = sum(v[0] for k, v in prof_f.items() if k not in cls_c)
        fk = wl.nk / wls.nk
        s_est = (c_ms * fk * fk + r_ms * fk) / 1e3
        out["full_fp64_sample"] = {
            "s_per_iteration_extrapolated": s_est, "speedup_block_vs_full_extrapolated": s_est / s_blk,
            "sample": f"full-matrix FP64 iteration on the 2x2x2 mesh ({wls.nk ** 2} pairs) of the same crystal, "
                      f"bases, tau grid and beta: {s_sample:.3f} s measured, contractions {c_ms:.0f} ms scaled by "
                      f"(Nk/8)^2 = {fk * fk:.0f}, the rest {r_ms:.0f} ms by Nk/8 = {fk:.0f}",
            "profile_ms": {k: v[0] for k, v in prof_f.items()}}
        log(f"[bench] full-matrix form, 2x2x2 sample {s_sample:.3f} s -> {s_est:.0f} s/iteration at Nk = {wl.nk} "
            f"(block form {s_est / s_blk:.0f}x faster)")
        del fpath, inp_s
        torch.cuda.empty_cache()
    if "unbatched" in legs:
        ub = Path(make_ctx(wl, gwsym.MODE_BLOCK, tau_chunk=args.tau_chunk, sched=gwsym.SCHED_UNBATCHED), F_all,
                  V_src, torch, dev)
        s_ub = time_steps(ub, 1, 1, torch)
        out["unbatched_fp64"] = {"s_per_iteration": s_ub, "speedup_grouped_vs_unbatched": s_ub / s_blk,
                                 "schedule": "one launch per pair (block multiplies) and per (pair, block) (GEMMs), "
                                             "in order, eager"}
        log(f"[bench] unbatched: {s_ub:.3f} s/iteration")
        del ub
        torch.cuda.empty_cache()
    reduced = [(k, p) for k, p in (("fp32", gwsym.FP32), ("bf16x6", gwsym.BF16X6), ("bf16x3", gwsym.BF16X3))
               if k in legs]
    ibz_blk = blk.ctx.table("ibz")
    if wl.pairwise and reduced:
        # the 6^3 workloads hold one path at a time: free the FP64 path's device state now
        blk.ctx.close()
        del blk
        torch.cuda.empty_cache()
        blk = None
    for key, prec in reduced:
        red = Path(make_ctx(wl, gwsym.MODE_BLOCK, tau_chunk=args.tau_chunk, precision=prec), F_all, V_src,
                   torch, dev, graph=bool(args.graph))
        red_tuning, _ = plan_for(red)
        s_red = time_steps(red, args.steps, args.warmup, torch)
        entry = {"s_per_iteration": s_red, "speedup_vs_fp64_block": s_blk / s_red, "launch_plan": red_tuning}
        if blk is not None and args.error_iterations > 0:
            # errors against the FP64 block path over several iterations from the same G0 (the
            # FP64 path is held to the oracle at 1e-10 per iteration by the parity tests)
            hist = iteration_errors(blk, red, args.error_iterations, torch)
            entry["errors_over_iterations"] = {
                "iterations": args.error_iterations, "reference": "FP64 block path, same G0",
                "p0_rel_max": max(h[0] for h in hist), "sigma_rel_max": max(h[1] for h in hist),
                "occupation_abs_max": max(h[2] for h in hist),
                "per_iteration": [[float(f"{x:.3e}") for x in h] for h in hist]}
        prof_red = profile_step(red, torch)
        entry["profile_ms"] = {k: v[0] for k, v in prof_red.items()}
        out[key + "_contractions"] = entry
        log(f"[bench] {key}: {s_red:.4f} s/iteration; profile " + ", ".join(f"{k} {v[0]:.1f} ms"
                                                                            for k, v in prof_red.items()))
        red.ctx.close()
        del red
        torch.cuda.empty_cache()

    if not args.no_cpu:
        vpairs = (lambda pr: inp.three_index(pr)) if wl.pairwise else (lambda pr: V_all[tuple(zip(*pr))])
        out["cpu_baseline"] = cpu_baseline(wl, F_all, vpairs, int(ibz_blk[1]), torch)
        log(f"[bench] cpu oracle (extrapolated): {out['cpu_baseline']['value']:.1f} s/iteration on "
            f"{out['cpu_baseline']['cores']} threads ({out['cpu_baseline']['cpu_model']})")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
