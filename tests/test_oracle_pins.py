"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
closed forms, brute-force index sums on tiny inputs, exact identities of the
imaginary-time formalism, the group relation, and the irreducible-wedge counts
printed in the paper's Table 2.  A test at the end plants plausible mistakes in
copies of the oracle's contractions and checks that these pins catch them."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from gwinputs import (Inputs, workload, add_k, minus_k, kmap, crystal, cubic_point_group,
                      in_td, mesh_points, mesh_index)

HERE = os.path.dirname(os.path.abspath(__file__))


def _herm(X):
    return 0.5 * (X + np.conj(np.swapaxes(X, -1, -2)))


def _sub_table(n):
    add, mk = add_k(n), minus_k(n)
    nk = n ** 3
    return np.array([[add[k, mk[q]] for q in range(nk)] for k in range(nk)])


# ----------------------------------------------------------------------------- P1

def test_g0_closed_form_identities():
    rng = np.random.default_rng(1)
    nk, nao, beta = 3, 5, 40.0
    A = rng.standard_normal((nk, nao, nao)) + 1j * rng.standard_normal((nk, nao, nao))
    F = _herm(A)
    tau = oracle.tau_grid(beta, 20)
    G = oracle.g0_closed_form(F, 0.3, beta, tau)
    I = np.eye(nao)
    assert np.abs(G - np.conj(np.swapaxes(G, -1, -2))).max() < 1e-15
    # G(0+) + G(beta-) = -I
    assert np.abs(G[:, 0] + G[:, -1] + I).max() < 1e-14
    # gamma = -G(beta) has the Fermi occupations as eigenvalues
    occ = np.linalg.eigvalsh(-G[:, -1])
    e = np.linalg.eigvalsh(F - 0.3 * I)
    f = 1.0 / (1.0 + np.exp(beta * e))
    assert np.abs(np.sort(occ, axis=-1) - np.sort(f, axis=-1)).max() < 1e-14
    assert occ.min() > -1e-14 and occ.max() < 1 + 1e-14


def test_g0_matches_matrix_exponential_route():
    rng = np.random.default_rng(2)
    nao, beta, mu = 4, 5.0, -0.1
    A = rng.standard_normal((1, nao, nao)) + 1j * rng.standard_normal((1, nao, nao))
    F = 0.5 * _herm(A)
    tau = oracle.tau_grid(beta, 9)
    G = oracle.g0_closed_form(F, mu, beta, tau)[0]
    H = F[0] - mu * np.eye(nao)
    Z = np.linalg.inv(np.eye(nao) + sla.expm(-beta * H))
    for j, t in enumerate(tau):
        ref = -sla.expm(-t * H) @ Z
        assert np.abs(G[j] - ref).max() < 1e-13


# ----------------------------------------------------------------------------- P2

def _tiny_inputs(seed=3, n=3, nao=2, naux=3, nt=4):
    rng = np.random.default_rng(seed)
    nk = n ** 3
    V = (rng.standard_normal((nk, nk, naux, nao, nao))
         + 1j * rng.standard_normal((nk, nk, naux, nao, nao)))
    V = 0.5 * (V + np.conj(np.swapaxes(V.transpose(1, 0, 2, 3, 4), -1, -2)))  # V^{k2,k1} = V^{k1,k2 H}
    G = _herm(rng.standard_normal((nk, nt, nao, nao)) + 1j * rng.standard_normal((nk, nt, nao, nao)))
    P = _herm(rng.standard_normal((nk, nt, naux, naux)) + 1j * rng.standard_normal((nk, nt, naux, naux)))
    return V, G, P


def test_bruteforce_polarization():
    n, s = 3, 2.0
    V, G, _ = _tiny_inputs()
    nk, nt, nao, _ = G.shape
    naux = V.shape[2]
    add = add_k(n)
    ref = np.zeros((nk, nt, naux, naux), complex)
    for q in range(nk):
        for j in range(nt):
            for Q in range(naux):
                for Qp in range(naux):
                    acc = 0j
                    for k in range(nk):
                        kq = add[k, q]
                        for a in range(nao):
                            for b in range(nao):
                                for c in range(nao):
                                    for d in range(nao):
                                        acc += (V[k, kq, Q, d, a] * G[k, nt - 1 - j, c, d]
                                                * G[kq, j, a, b] * V[kq, k, Qp, b, c])
                    ref[q, j, Q, Qp] = -s / nk * acc
    got = oracle.polarization(G, V, add, s)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_bruteforce_self_energy():
    n = 3
    V, G, P = _tiny_inputs(seed=4)
    nk, nt, nao, _ = G.shape
    naux = V.shape[2]
    sub = _sub_table(n)
    ref = np.zeros((nk, nt, nao, nao), complex)
    for k in range(nk):
        for j in range(nt):
            for i in range(nao):
                for jj in range(nao):
                    acc = 0j
                    for q in range(nk):
                        kmq = sub[k, q]
                        for a in range(nao):
                            for b in range(nao):
                                for Q in range(naux):
                                    for Qp in range(naux):
                                        acc += (G[kmq, j, a, b] * V[k, kmq, Q, i, a]
                                                * P[q, j, Q, Qp] * V[kmq, k, Qp, b, jj])
                    ref[k, j, i, jj] = -acc / nk
    got = oracle.self_energy(G, V, P, sub)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


# ----------------------------------------------------------------------------- P3

def _two_level(eps1, eps2, v, beta, s, nt):
    F = np.diag([eps1, eps2]).astype(complex)[None]
    V = np.zeros((1, 1, 1, 2, 2), complex)
    V[0, 0, 0, 0, 1] = v
    V[0, 0, 0, 1, 0] = np.conj(v)
    tau = oracle.tau_grid(beta, nt)
    G = oracle.g0_closed_form(F, 0.0, beta, tau)
    P0 = oracle.polarization(G, V, np.zeros((1, 1), int), s)[0, :, 0, 0]
    f1, f2 = 1 / (1 + np.exp(beta * eps1)), 1 / (1 + np.exp(beta * eps2))
    dlt = eps2 - eps1
    ref = -s * abs(v) ** 2 * (f1 * (1 - f2) * np.exp(-dlt * tau) + f2 * (1 - f1) * np.exp(dlt * tau))
    return tau, P0, ref, f1, f2, dlt


def test_two_level_polarization_closed_form():
    beta, s, v = 10.0, 2.0, 0.7 - 0.2j
    tau, P0, ref, f1, f2, dlt = _two_level(-0.3, 0.5, v, beta, s, 40)
    assert np.abs(P0 - ref).max() < 1e-14
    assert np.abs(P0 - P0[::-1]).max() < 1e-14          # tau -> beta - tau
    Tb, _, _ = oracle.transform_matrices(beta, 40, 81, boson=True)
    P0w = Tb @ P0
    Om = oracle.matsubara(beta, 81, boson=True)
    refw = -2 * s * abs(v) ** 2 * (f1 - f2) * dlt / (Om ** 2 + dlt ** 2)
    assert np.abs(P0w - refw).max() < 1e-10
    assert (P0w.real <= 1e-12).all()


# ----------------------------------------------------------------------------- P12, P13

def test_transform_exact_on_polynomials():
    beta, nt, nw = 2.0, 12, 25
    tau = oracle.tau_grid(beta, nt)
    for boson in (False, True):
        Tf, _, _ = oracle.transform_matrices(beta, nt, nw, boson)
        nu = oracle.matsubara(beta, nw, boson)
        for m in range(0, 6):
            got = Tf @ tau ** m
            ref = np.empty(nw, complex)
            for i, w in enumerate(nu):
                if w == 0:
                    ref[i] = beta ** (m + 1) / (m + 1)
                    continue
                I = (np.exp(1j * w * beta) - 1) / (1j * w)
                for p in range(1, m + 1):
                    I = beta ** p * np.exp(1j * w * beta) / (1j * w) - p / (1j * w) * I
                ref[i] = I
            assert np.abs(got - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("boson", [False, True])
def test_transform_round_trip(boson):
    beta, nt = 100.0, 40
    nw = 2 * nt + 1
    rng = np.random.default_rng(5)
    X = _herm(rng.standard_normal((nt, 3, 3)) + 1j * rng.standard_normal((nt, 3, 3)))
    Tf, Bf, rows = oracle.transform_matrices(beta, nt, nw, boson)
    back = oracle.to_tau(oracle.to_freq(X, Tf), Bf, rows)
    assert np.abs(back - X).max() < 1e-11


def test_dyson_free_limit_matches_closed_form_and_analytic_frequency():
    rng = np.random.default_rng(6)
    nao, beta, mu, nt = 4, 10.0, 0.2, 40
    nw = 2 * nt + 1
    F = 0.5 * _herm(rng.standard_normal((2, nao, nao)) + 1j * rng.standard_normal((2, nao, nao)))
    tau = oracle.tau_grid(beta, nt)
    G0 = oracle.g0_closed_form(F, mu, beta, tau)
    Tf, _, _ = oracle.transform_matrices(beta, nt, nw, boson=False)
    w = oracle.matsubara(beta, nw, boson=False)
    Gw_ref = np.linalg.inv((1j * w[:, None, None] + mu) * np.eye(nao) - F[:, None])
    assert np.abs(oracle.to_freq(G0, Tf) - Gw_ref).max() < 1e-8
    G, Gw, _ = oracle.dyson(F, np.zeros((2, nt, nao, nao), complex), mu, beta, nw)
    assert np.abs(Gw - Gw_ref).max() < 1e-15
    assert np.abs(G - G0).max() < 1e-8


# ----------------------------------------------------------------------------- P4-P6, P14, P15 on a workload

@pytest.fixture(scope="module")
def diamond_run():
    wl = workload("small_diamond")
    inp = Inputs(wl)
    F = inp.fock().numpy()
    V = inp.three_index_full().numpy()
    tau = oracle.tau_grid(wl.beta, wl.ntau)
    G0 = oracle.g0_closed_form(F, 0.0, wl.beta, tau)
    add, sub = add_k(wl.n), _sub_table(wl.n)
    nt = oracle.free_count(F, 0.0, wl.beta, wl.spin)
    r = oracle.gw_iteration(F, V, G0, 0.0, wl.beta, wl.nw, wl.spin, add, sub, n_target=nt)
    return dict(wl=wl, inp=inp, F=F, V=V, G0=G0, r=r, n_target=nt)


def test_hermiticity(diamond_run):
    r = diamond_run["r"]
    for key in ("P0", "P", "Sigma", "G"):
        X = r[key]
        assert np.abs(X - np.conj(np.swapaxes(X, -1, -2))).max() < 1e-13 * np.abs(X).max(), key


def test_bosonic_mirror_with_time_reversal(diamond_run):
    r = diamond_run["r"]
    for key in ("P0", "P"):
        X = r[key]
        assert np.abs(X - X[:, ::-1]).max() < 1e-12 * np.abs(X).max(), key


def test_bosonic_mirror_without_time_reversal():
    # P^q(beta - tau) = P^{-q}(tau)^T holds for any Hermitian-paired input
    n, s = 3, 2.0
    V, G, _ = _tiny_inputs(seed=8, nao=3, naux=4, nt=6)
    add, mk = add_k(n), minus_k(n)
    P0 = oracle.polarization(G, V, add, s)
    assert np.abs(P0[:, ::-1] - np.swapaxes(P0[mk], -1, -2)).max() < 1e-13 * np.abs(P0).max()


def test_group_relation(diamond_run):
    inp, r = diamond_run["inp"], diamond_run["r"]
    for a in range(inp.h):
        for k in range(inp.nk):
            ak = inp.kmap[a, k]
            O = inp.ao.matrix(a, k)
            Ob = inp.aux.matrix(a, k)
            for key, M in (("Sigma", O), ("G", O), ("P", Ob), ("P0", Ob)):
                X = r[key]
                rot = M[None] @ X[k] @ M.conj().T[None]
                assert np.abs(rot - X[ak]).max() < 1e-12 * np.abs(X).max(), (key, a, k)


def test_screened_invariants(diamond_run):
    r = diamond_run["r"]
    P0w, Pw = r["P0w"], r["Pw"]
    assert np.abs(P0w - np.conj(np.swapaxes(P0w, -1, -2))).max() < 1e-12
    ev0 = np.linalg.eigvalsh(_herm(P0w))
    assert ev0.max() < 1e-12
    evP = np.linalg.eigvalsh(_herm(Pw))
    assert evP.min() > -1.0 and evP.max() < 1e-12


def test_particle_number_and_mu(diamond_run):
    wl, F = diamond_run["wl"], diamond_run["F"]
    nt = wl.ntau
    Z = np.zeros((wl.nk, nt, wl.nao, wl.nao), complex)
    Ns = []
    for mu in (-0.5, -0.1, 0.0, 0.1, 0.5):
        G, _, _ = oracle.dyson(F, Z, mu, wl.beta, wl.nw)
        Ns.append(oracle.particle_number(G, wl.spin))
    assert all(b > a for a, b in zip(Ns, Ns[1:]))
    mu = oracle.find_mu(F, Z, Ns[2], wl.beta, wl.nw, wl.spin)
    assert abs(mu) < 1e-12
    r = diamond_run["r"]
    assert abs(oracle.particle_number(r["G"], wl.spin) - diamond_run["n_target"]) < 1e-10


# ----------------------------------------------------------------------------- N_e (free count)

def test_free_count_one_level_closed_form():
    # one level at energy e: the count is s f(e - mu), f(x) = 1/(1 + e^{beta x}); a level far
    # below mu holds s electrons, one far above none, one at mu half of s, and
    # beta (e - mu) = ln 3 gives f = 1/4 (Sec. 4.1: N_e counts the occupied states with spin)
    s, beta = 2.0, 50.0
    F = np.array([[[0.7]]], complex)
    assert abs(oracle.free_count(F, 0.7, beta, s) - 1.0) < 1e-15
    assert abs(oracle.free_count(F, 0.7 + 5.0, beta, s) - s) < 1e-15
    assert oracle.free_count(F, 0.7 - 5.0, beta, s) < 1e-100
    mu = 0.7 - np.log(3.0) / beta
    assert abs(oracle.free_count(F, mu, beta, s) - s * 0.25) < 1e-15
    # two k points, two levels each: the mean over k of the summed occupations
    F2 = np.array([np.diag([-0.2, 0.4]), np.diag([0.1, 0.3])], complex)
    f = lambda x: 1.0 / (1.0 + np.exp(beta * x))
    want = s * (f(-0.2) + f(0.4) + f(0.1) + f(0.3)) / 2
    assert abs(oracle.free_count(F2, 0.0, beta, s) - want) < 1e-15


def test_free_count_equals_particle_number_of_closed_form_g0():
    # the count is the trace of gamma = -G0(beta) of the closed form, whose occupations are
    # pinned to the Fermi function above and whose Dyson limit is pinned to (i w + mu - F)^{-1}
    rng = np.random.default_rng(31)
    nk, nao, beta, s = 4, 6, 30.0, 2.0
    A = rng.standard_normal((nk, nao, nao)) + 1j * rng.standard_normal((nk, nao, nao))
    F = 0.4 * _herm(A)
    tau = oracle.tau_grid(beta, 12)
    for mu in (-0.7, 0.0, 0.25):
        G0 = oracle.g0_closed_form(F, mu, beta, tau)
        assert abs(oracle.free_count(F, mu, beta, s) - oracle.particle_number(G0, s)) < 1e-12
    # and a flipped Fermi function (occupying the states above mu) is far off
    e = np.linalg.eigvalsh(F) + 0.7
    flipped = s * (1.0 / (1.0 + np.exp(-beta * e))).sum() / nk
    assert abs(flipped - oracle.free_count(F, -0.7, beta, s)) > 1.0


def test_planted_free_count_mistakes_are_caught():
    # flipped occupations (1 - f) and a dropped spin factor each break the one-level values
    F = np.array([[[0.7]]], complex)
    for old, new in [("1.0 / (1 + np.exp(-beta * np.abs(e))))", "np.exp(-beta * np.abs(e)) / (1 + np.exp(-beta * np.abs(e))))"),
                     ("return spin * f.sum()", "return f.sum()")]:
        bad = _mutant(oracle.free_count, old, new)
        assert abs(bad(F, 0.7 + 5.0, 50.0, 2.0) - 2.0) > 0.5


# ----------------------------------------------------------------------------- Table 2 counts

def _ibz_count(ops_frac, n):
    pts = mesh_points(n)
    seen = np.zeros(len(pts), bool)
    count = 0
    for k in range(len(pts)):
        if seen[k]:
            continue
        count += 1
        for W in ops_frac:
            WiT = np.rint(np.linalg.inv(W).T).astype(np.int64)
            seen[mesh_index(WiT @ pts[k], n)] = True
    return count


def test_table2_irreducible_counts():
    gold = json.load(open(os.path.join(HERE, "golden", "table2_nik.json")))
    oh = cubic_point_group()
    A = crystal("rocksalt").lattice
    Ai = np.linalg.inv(A)
    frac = {"Oh": [np.rint(Ai @ R @ A).astype(np.int64) for R in oh],
            "Td": [np.rint(Ai @ R @ A).astype(np.int64) for R in oh if in_td(R)],
            "D6h": [W for W, _ in crystal("hbn").ops]}
    for g, d in gold["groups"].items():
        for nkk, cnt in d["nik"].items():
            assert _ibz_count(frac[d["point_group"]], int(nkk)) == cnt, (g, nkk)


def test_workload_star_sizes():
    cr = crystal("sc")
    km = kmap(cr, 4)
    sizes = sorted(len(set(km[:, k])) for k in range(64) if k == min(km[:, k]))
    assert sizes == [1, 1, 3, 3, 6, 6, 8, 12, 12, 12]
    cr = crystal("rocksalt")
    km = kmap(cr, 6)
    sizes = sorted(len(set(km[:, k])) for k in range(216) if k == min(km[:, k]))
    assert sizes == [1, 3, 4, 6, 6, 8, 8, 12, 12, 12, 24, 24, 24, 24, 24, 24]


# ----------------------------------------------------------------------------- planted mistakes

def _mutant(func, old, new):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(func))
    assert old in src
    src = src.replace(old, new)
    ns = dict(func.__globals__)
    exec(compile(src, "<mutant>", "exec"), ns)
    return ns[func.__name__]


MUTATIONS = [
    (oracle.polarization, "Grev = G[:, ::-1]", "Grev = G"),
    (oracle.polarization, "return -(spin / nk) * P0", "return (spin / nk) * P0"),
    (oracle.polarization, "AH = np.conj(np.swapaxes(A, -1, -2))", "AH = np.swapaxes(A, -1, -2)"),
    (oracle.polarization, "kq = add[k, q]", "kq = add[q, q]"),
    (oracle.self_energy, "Y = np.swapaxes(P[q], -1, -2) @", "Y = P[q] @"),
    (oracle.self_energy, "kmq = sub[k, q]", "kmq = sub[q, k]"),
    (oracle.self_energy, "Af = np.conj(", "Af = ("),
]


@pytest.mark.parametrize("func,old,new", MUTATIONS)
def test_planted_mistakes_are_caught(func, old, new):
    bad = _mutant(func, old, new)
    n, s = 3, 2.0
    V, G, P = _tiny_inputs(seed=11, nao=3, naux=4, nt=6)
    if func is oracle.polarization:
        good = oracle.polarization(G, V, add_k(n), s)
        got = bad(G, V, add_k(n), s)
    else:
        good = oracle.self_energy(G, V, P, _sub_table(n))
        got = bad(G, V, P, _sub_table(n))
    # the brute-force pins above compare `good` with the printed index sums;
    # a planted mistake must move the result far outside their tolerance
    assert np.abs(got - good).max() > 1e-6 * np.abs(good).max()


def test_single_output_units_match_full_contractions():
    # the one-output forms used for sampled checks and CPU timing equal the full ones
    n, s = 3, 2.0
    V, G, P = _tiny_inputs(seed=12, nao=3, naux=4, nt=6)
    add, sub = add_k(n), _sub_table(n)
    P0 = oracle.polarization(G, V, add, s)
    S = oracle.self_energy(G, V, P, sub)
    nk = n ** 3
    for q, j in [(0, 0), (5, 2), (13, 5)]:
        Vq = np.stack([V[k, add[k, q]] for k in range(nk)])
        assert np.abs(oracle.polarization_unit(G, Vq, add, q, j, s) - P0[q, j]).max() < 1e-13
    for k, j in [(0, 1), (7, 3)]:
        Vk = np.stack([V[k, sub[k, q]] for q in range(nk)])
        assert np.abs(oracle.self_energy_unit(G, Vk, P[:, j], sub, k, j) - S[k, j]).max() < 1e-13


# ----------------------------------------------------------------------------- exchange (eq. sigma_hf, K)

def test_bruteforce_exchange():
    """K^k_ij = -(1/Nk) sum_{k'} sum_{ab} sum_Q V^{kk'}_{ia}(Q) gamma^{k'}_{ab} V^{k'k}_{bj}(Q),
    gamma = G(0^-) = -G(beta), written out index by index on a tiny mesh."""
    V, G, _ = _tiny_inputs(seed=7)
    nk, nt, nao, _ = G.shape
    naux = V.shape[2]
    ref = np.zeros((nk, nao, nao), complex)
    for k in range(nk):
        for i in range(nao):
            for j in range(nao):
                acc = 0j
                for kp in range(nk):
                    for a in range(nao):
                        for b in range(nao):
                            for Q in range(naux):
                                acc += V[k, kp, Q, i, a] * (-G[kp, nt - 1, a, b]) * V[kp, k, Q, b, j]
                ref[k, i, j] = -acc / nk
    got = oracle.exchange(G, V)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_exchange_one_orbital_pair_closed_form():
    """One k point, one auxiliary function, V = [[0, v], [v*, 0]], F = diag(e1, e2): gamma is
    diag(f1, f2) with f = 1/(1 + exp(beta e)), so K = -V gamma V = -diag(|v|^2 f2, |v|^2 f1)."""
    e1, e2, v, beta = -0.4, 0.7, 0.3 - 0.2j, 10.0
    F = np.diag([e1, e2]).astype(complex)[None]
    V = np.zeros((1, 1, 1, 2, 2), complex)
    V[0, 0, 0, 0, 1] = v
    V[0, 0, 0, 1, 0] = np.conj(v)
    G = oracle.g0_closed_form(F, 0.0, beta, oracle.tau_grid(beta, 8))
    f1, f2 = 1 / (1 + np.exp(beta * e1)), 1 / (1 + np.exp(beta * e2))
    K = oracle.exchange(G, V)[0]
    assert np.abs(K - np.diag([-abs(v) ** 2 * f2, -abs(v) ** 2 * f1])).max() < 1e-15


def test_exchange_hermitian_negative_semidefinite_and_symmetric(diamond_run):
    """With Hermitian pairing of V and 0 <= gamma <= 1, K = -sum (V gamma^1/2)(V gamma^1/2)^H is
    Hermitian and negative semidefinite; it obeys the group relation like Sigma."""
    inp, V = diamond_run["inp"], diamond_run["V"]
    K = oracle.exchange(diamond_run["G0"], V)
    scale = np.abs(K).max()
    assert np.abs(K - np.conj(np.swapaxes(K, -1, -2))).max() < 1e-14 * scale
    assert np.linalg.eigvalsh(K).max() < 1e-13 * scale
    for a in range(inp.h):
        for k in range(inp.nk):
            O = inp.ao.matrix(a, k)
            assert np.abs(O @ K[k] @ O.conj().T - K[inp.kmap[a, k]]).max() < 1e-12 * scale



# ----------------------------------------------------------------------------- Hartree (eq. sigma_hf, J)

def test_bruteforce_hartree():
    """J^k_ij = (s/Nk) sum_{k'} sum_{ab} sum_Q V^{kk}_{ij}(Q) gamma^{k'}_{ab} V^{k'k'}_{ba}(Q),
    gamma = -G(beta), written out index by index on a tiny mesh."""
    V, G, _ = _tiny_inputs(seed=11)
    s = 2.0
    nk, nt, nao, _ = G.shape
    naux = V.shape[2]
    ref = np.zeros((nk, nao, nao), complex)
    for k in range(nk):
        for i in range(nao):
            for j in range(nao):
                acc = 0j
                for kp in range(nk):
                    for a in range(nao):
                        for b in range(nao):
                            for Q in range(naux):
                                acc += V[k, k, Q, i, j] * (-G[kp, nt - 1, a, b]) * V[kp, kp, Q, b, a]
                ref[k, i, j] = s * acc / nk
    got = oracle.hartree(G, V, s)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_hartree_one_orbital_pair_closed_form():
    """One k point, one auxiliary function, V = [[v1, w], [w*, v2]], F = diag(e1, e2): gamma is
    diag(f1, f2), the density on the auxiliary function is v1 f1 + v2 f2 (the off-diagonal w
    does not contribute), and J = s (v1 f1 + v2 f2) V."""
    e1, e2, v1, v2, w, beta, s = -0.4, 0.7, 0.9, 0.35, 0.3 - 0.2j, 10.0, 2.0
    F = np.diag([e1, e2]).astype(complex)[None]
    V = np.zeros((1, 1, 1, 2, 2), complex)
    V[0, 0, 0] = [[v1, w], [np.conj(w), v2]]
    G = oracle.g0_closed_form(F, 0.0, beta, oracle.tau_grid(beta, 8))
    f1, f2 = 1 / (1 + np.exp(beta * e1)), 1 / (1 + np.exp(beta * e2))
    J = oracle.hartree(G, V, s)[0]
    assert np.abs(J - s * (v1 * f1 + v2 * f2) * V[0, 0, 0]).max() < 1e-15


def test_hartree_hermitian_positive_energy_and_symmetric(diamond_run):
    """With Hermitian V^{kk}(Q) and gamma, the density on each auxiliary function is real, J is
    Hermitian and the Hartree energy sum_k Tr[gamma^k J^k] = (s/Nk) sum_Q rho(Q)^2 is real and
    positive; J obeys the group relation like Sigma.  A Gamma-only reading of the sum over k'
    (dropping the other momenta) changes J."""
    inp, V, G0, wl = diamond_run["inp"], diamond_run["V"], diamond_run["G0"], diamond_run["wl"]
    J = oracle.hartree(G0, V, wl.spin)
    scale = np.abs(J).max()
    assert scale > 0
    assert np.abs(J - np.conj(np.swapaxes(J, -1, -2))).max() < 1e-14 * scale
    E = sum(np.trace(-G0[k, -1] @ J[k]) for k in range(inp.nk))
    assert abs(E.imag) < 1e-13 * abs(E) and E.real > 0
    for a in range(inp.h):
        for k in range(inp.nk):
            O = inp.ao.matrix(a, k)
            assert np.abs(O @ J[k] @ O.conj().T - J[inp.kmap[a, k]]).max() < 1e-12 * scale
    G1 = np.zeros_like(G0)
    G1[0] = G0[0] * inp.nk
    assert np.abs(oracle.hartree(G1, V, wl.spin) - J).max() > 1e-6 * scale


def test_static_units_match_whole_zone(diamond_run):
    """The one-k forms of K and J used by the full-size check equal the whole-zone forms."""
    inp, V, G0, wl = diamond_run["inp"], diamond_run["V"], diamond_run["G0"], diamond_run["wl"]
    K, J = oracle.exchange(G0, V), oracle.hartree(G0, V, wl.spin)
    nk = inp.nk
    Vdiag = np.stack([V[kp, kp] for kp in range(nk)])
    for k in (0, 3, nk - 1):
        Kk = oracle.exchange_unit(G0, V[k], V[:, k])
        Jk = oracle.hartree_unit(G0, Vdiag, k, wl.spin)
        assert np.abs(Kk - K[k]).max() < 1e-14 * np.abs(K).max()
        assert np.abs(Jk - J[k]).max() < 1e-14 * np.abs(J).max()


# ----------------------------------------------------------------------------- IR sampling grids (Sec. 5.1)

IR_CASES = [(30.0, 5.0, 1e-6), (100.0, 4.0, 1e-8)]


@pytest.mark.parametrize("beta,wmax,eps", IR_CASES)
def test_ir_basis_properties(beta, wmax, eps):
    g = oracle.ir_grid(beta, wmax, eps)
    b = g["basis"]
    L = b["L"]
    # orthonormal on [-1, 1] (a finer rule than the one that built them), singular values falling
    xf, wf = np.polynomial.legendre.leggauss(48)
    u = np.concatenate([oracle.ir_eval(b, 0.5 * (q - p) * xf + 0.5 * (q + p)) * np.sqrt(0.5 * (q - p) * wf)[:, None]
                        for p, q in zip(b["xb"][:-1], b["xb"][1:])])
    assert np.abs(u.T @ u - np.eye(L + 1)).max() < 1e-10
    assert (np.diff(b["s"]) < 0).all() and b["s"][L - 1] > eps * b["s"][0] >= b["s"][L]
    # the logistic kernel is centrosymmetric: u_l(-x) = (-1)^l u_l(x) for the well-resolved l
    x = np.linspace(-1, 1, 101)
    par = oracle.ir_eval(b, -x)[:, :10] - oracle.ir_eval(b, x)[:, :10] * (-1.0) ** np.arange(10)
    assert np.abs(par).max() < 1e-8
    # tau grid: 0, the L zeros of u_L, beta; mirror symmetric
    tau = g["tau"]
    assert len(tau) == L + 2 and tau[0] == 0.0 and tau[-1] == beta
    assert np.abs(tau + tau[::-1] - beta).max() < 1e-12 * beta
    assert (np.diff(tau) > 0).all()
    # (u_L is determined to about the double-precision rounding over s_L / s_0, so are its zeros)
    assert np.abs(oracle.ir_eval(b, 2 * tau[1:-1] / beta - 1)[:, L]).max() < 1e-6 * np.abs(oracle.ir_eval(b, x)[:, L]).max()
    # the frequency fits are determined: 2 nw rows (bosons: 2 nw - 1) for L unknowns
    assert len(g["nf"]) == len(g["nb"]) and 2 * len(g["nb"]) - 1 >= L
    assert 0 in g["nb"] and (np.diff(g["nf"]) > 0).all() and (np.diff(g["nb"]) > 0).all()


@pytest.mark.parametrize("beta,wmax,eps", IR_CASES)
def test_ir_transforms_against_closed_forms(beta, wmax, eps):
    g = oracle.ir_grid(beta, wmax, eps)
    tau = g["tau"]
    Tf, Bf, rf = oracle.ir_transform_matrices(g, False)
    Tb, Bb, rb = oracle.ir_transform_matrices(g, True)
    # free fermion levels inside the cutoff: G0(tau) -> the analytic 1/(i w_n - e), to the basis accuracy
    levels = np.array([-0.9 * wmax, -0.3, 0.05, 1.7, 0.8 * wmax])
    G = -oracle.fermi_factor_parts(levels, tau, beta)                       # [tau, level]
    w = (2 * g["nf"] + 1) * np.pi / beta
    ref = 1.0 / (1j * w[:, None] - levels[None, :])
    assert np.abs(Tf @ G - ref).max() < 50 * eps * np.abs(ref).max()
    back = Bf @ np.concatenate([Tf @ G, (Tf @ G)[rf].conj()])
    assert np.abs(back - G).max() < 50 * eps
    # the two-level polarization of the Chebyshev pin: tau form -> -2 s |v|^2 (f1 - f2) D / (W^2 + D^2)
    e1, e2, s, v = -0.3, 0.5, 2.0, 0.7
    f1, f2 = 1 / (1 + np.exp(beta * e1)), 1 / (1 + np.exp(beta * e2))
    h1, h2 = 1 / (1 + np.exp(-beta * e1)), 1 / (1 + np.exp(-beta * e2))     # 1 - f without cancellation
    dl = e2 - e1
    P0 = -s * v ** 2 * (f1 * h2 * np.exp(-dl * tau) + f2 * h1 * np.exp(dl * tau))
    Om = 2 * g["nb"] * np.pi / beta
    refb = -2 * s * v ** 2 * (f1 - f2) * dl / (Om ** 2 + dl ** 2)
    assert np.abs(Tb @ P0 - refb).max() < 50 * eps * np.abs(refb).max()


def test_ir_round_trip_is_exact_on_the_basis():
    g = oracle.ir_grid(30.0, 5.0, 1e-6)
    b, beta, L = g["basis"], 30.0, g["basis"]["L"]
    rng = np.random.default_rng(41)
    x = rng.standard_normal(L)
    for boson in (False, True):
        n = g["nb"] if boson else g["nf"]
        nu = (2 * n + (0 if boson else 1)) * np.pi / beta
        Ut = np.sqrt(2 / beta) * oracle.ir_eval(b, 2 * g["tau"] / beta - 1)[:, :L]
        Fm = oracle.ir_fourier(b, beta, nu)[:, :L]
        T, B, rows = oracle.ir_transform_matrices(g, boson)
        Xt = Ut @ x
        assert np.abs(T @ Xt - Fm @ x).max() < 1e-11 * np.abs(Fm @ x).max()
        Xw = T @ Xt
        # real X(tau) is its own Hermitian conjugate: the conjugate rows are conj(X(i nu))
        assert np.abs(B @ np.concatenate([Xw, Xw[rows].conj()]) - Xt).max() < 1e-11 * np.abs(Xt).max()


def test_ir_fourier_against_quadrature():
    # the Legendre-Bessel panel formula against brute-force quadrature of u_l e^{i nu tau}
    g = oracle.ir_grid(20.0, 3.0, 1e-6)
    b, beta = g["basis"], 20.0
    nu = np.array([np.pi / beta, 7 * np.pi / beta, 40 * np.pi / beta])
    xq, wq = np.polynomial.legendre.leggauss(400)
    ref = np.zeros((3, b["L"] + 1), complex)
    for p, q in zip(b["xb"][:-1], b["xb"][1:]):
        x = 0.5 * (q - p) * xq + 0.5 * (q + p)
        w = 0.5 * (q - p) * wq * beta / 2 * np.sqrt(2 / beta)
        ref += (np.exp(1j * np.outer(nu, beta * (x + 1) / 2)) * w) @ oracle.ir_eval(b, x)
    assert np.abs(oracle.ir_fourier(b, beta, nu) - ref).max() < 1e-12
