"""Plain FP64 CPU oracle for one finite-temperature GW iteration.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with the
GPU library and never takes an input produced by it.

Everything here works with full matrices over the full Brillouin zone and uses
no symmetry at all.  Arrays (complex128, numpy):

  F[k, i, j]                 Fock / one-body matrix H0 + Sigma_HF (held fixed)
  V[k1, k2, Q, i, j]         density-fitted three-index tensor V^{k1,k2}_{ij}(Q)
  G[k, t, i, j]              Green's function G^k(tau_t)
  P0[q, t, Q, Q'], P[q, t, Q, Q']
  S[k, t, i, j]              dynamic self-energy Sigma~^k(tau_t)

k, q are linear indices of a Gamma-centred n^3 mesh (index (m0 n + m1) n + m2);
sums and differences of momenta are reduced on the mesh.

Readings of the paper used here (each also listed in the design notes):
  * P0 carries an overall minus sign with G^k(beta - tau) in place of G^k(-tau)
    (Sec. 4.1, eq. for P0; the fermionic antiperiodicity G(-tau) = -G(beta-tau)
    turns the printed form into a positive-semidefinite P0, which would make
    I - P0 singular), and an explicit spin factor s.
  * tau grid: Chebyshev-Gauss-Lobatto nodes; Matsubara transforms through the
    degree-(ntau-1) interpolating polynomial; the inverse transform is the
    least-squares inverse over n >= 0 and the conjugate rows n < 0.
  * nw = 2 ntau + 1 frequencies stored for n >= 0.
  * IR grids (Sec. 5.1): tau = 0, the zeros of the first dropped singular function of the
    logistic kernel and beta; Matsubara indices where its transform changes sign, both
    statistics filled to one length (ir_grid).
  * S^k = identity (orthonormal synthetic basis).
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# grids and transforms (Sec. 4.1: G(i w_n) = int_0^beta G(tau) e^{i w_n tau};
# eq. P02P: bosonic frequencies Omega_n = 2 n pi / beta)


def tau_grid(beta: float, ntau: int) -> np.ndarray:
    """Chebyshev-Gauss-Lobatto nodes on [0, beta]; tau_0 = 0, tau_{ntau-1} = beta,
    and tau_{ntau-1-j} = beta - tau_j."""
    j = np.arange(ntau)
    return 0.5 * beta * (1.0 - np.cos(np.pi * j / (ntau - 1)))


def matsubara(beta: float, nw: int, boson: bool) -> np.ndarray:
    n = np.arange(nw)
    return (2 * n + (0 if boson else 1)) * np.pi / beta


def _cheb_vander(x: np.ndarray, deg: int) -> np.ndarray:
    return np.polynomial.chebyshev.chebvander(x, deg)


def fourier_of_chebyshev(beta: float, ntau: int, nu: np.ndarray) -> np.ndarray:
    """Fmat[n, l] = int_0^beta T_l(2 tau / beta - 1) exp(i nu_n tau) d tau, by
    Gauss-Legendre quadrature with enough nodes to be exact to rounding."""
    nq = int(2 * (ntau + nu.max() * beta / 2)) + 100
    xq, wq = np.polynomial.legendre.leggauss(nq)
    tq = 0.5 * beta * (xq + 1.0)
    Tq = _cheb_vander(xq, ntau - 1)
    return (np.exp(1j * np.outer(nu, tq)) * (0.5 * beta * wq)) @ Tq


def transform_matrices(beta: float, ntau: int, nw: int, boson: bool):
    """Returns (Tfwd, Binv, rows).

    Tfwd[n, j]: X(i nu_n) = sum_j Tfwd[n, j] X(tau_j) for the polynomial through
    the samples (n = 0 ... nw-1).
    Binv[j, r]: the least-squares inverse of the stacked system
    [X(i nu_n), n = 0..nw-1 ; X(-i nu_n) = X(i nu_n)^H, n in rows] -> X(tau_j);
    for bosons the n = 0 row is not repeated in the conjugate half.
    """
    tau = tau_grid(beta, ntau)
    x = 2.0 * tau / beta - 1.0
    Vm = _cheb_vander(x, ntau - 1)                      # Vm[j, l] = T_l(x_j)
    nu = matsubara(beta, nw, boson)
    Fm = fourier_of_chebyshev(beta, ntau, nu)           # Fm[n, l]
    Tfwd = np.linalg.solve(Vm.T, Fm.T).T                 # Fm @ inv(Vm)
    conj_rows = np.arange(1, nw) if boson else np.arange(nw)
    S = np.vstack([Fm, Fm[conj_rows].conj()])
    Binv = Vm @ np.linalg.pinv(S)
    return Tfwd, Binv, conj_rows


def to_freq(X: np.ndarray, Tfwd: np.ndarray) -> np.ndarray:
    """X[..., t, a, b] -> X[..., n, a, b]."""
    return np.einsum("nt,...tab->...nab", Tfwd, X)


def to_tau(Xw: np.ndarray, Binv: np.ndarray, conj_rows: np.ndarray) -> np.ndarray:
    """Applies the least-squares inverse to the stacked data [X(i nu_n); X(i nu_n)^H]."""
    nw = Xw.shape[-3]
    stacked = np.concatenate([Xw, np.conj(np.swapaxes(Xw[..., conj_rows, :, :], -1, -2))],
                             axis=-3)
    return np.einsum("tr,...rab->...tab", Binv, stacked)


# ----------------------------------------------------------------------------
# sparse sampling on the intermediate-representation basis (Sec. 5.1: the tau and Matsubara
# grids of the paper's calculations).  The basis is the singular value expansion of the
# logistic kernel K(x, y) = exp(-L y (x + 1)/2) / (1 + exp(-L y)) on x = 2 tau/beta - 1 and
# y = omega / wmax in [-1, 1], L = beta wmax: the same tau functions serve fermions and bosons.
# Discretised by composite Gauss-Legendre rules (panels halving towards x = +-1 and y = 0 down
# to 1/L), the singular vectors of sqrt(w_x) K sqrt(w_y) give u_l at the nodes, continued
# inside each panel by the Legendre series through its nodes.


def _ir_panels(lam):
    k = int(np.ceil(np.log2(lam))) + 2
    xb = sorted({-1.0, 0.0, 1.0} | {s * (1.0 - 2.0 ** -j) for j in range(1, k) for s in (1, -1)})
    yb = sorted({-1.0, 0.0, 1.0} | {s * 2.0 ** -j for j in range(1, k) for s in (1, -1)})
    return np.array(xb), np.array(yb)


def _gauss_panels(breaks, order):
    xg, wg = np.polynomial.legendre.leggauss(order)
    h = 0.5 * np.diff(breaks)
    m = 0.5 * (breaks[1:] + breaks[:-1])
    return (m[:, None] + h[:, None] * xg[None]).ravel(), (h[:, None] * wg[None]).ravel()


def logistic_kernel(lam, x, y):
    """exp(-lam y (x + 1)/2) / (1 + exp(-lam y)), in the form that never overflows"""
    x, y = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float))
    ay = np.abs(y)
    e = np.where(y >= 0, -lam * y * (x + 1) / 2, lam * y * (1 - x) / 2)
    return np.exp(e) / (1.0 + np.exp(-lam * ay))


def ir_basis(lam, eps, order=16):
    """Singular functions u_0..u_L (L = number of s_l / s_0 > eps) as per-panel Legendre
    coefficients: dict(lam, L, s, xb, coef[panel, degree, l], order)."""
    xb, yb = _ir_panels(lam)
    x, wx = _gauss_panels(xb, order)
    y, wy = _gauss_panels(yb, order)
    A = np.sqrt(wx)[:, None] * logistic_kernel(lam, x[:, None], y[None, :]) * np.sqrt(wy)[None, :]
    U, S, _ = np.linalg.svd(A)
    L = int(np.sum(S / S[0] > eps))
    u = U[:, :L + 1] / np.sqrt(wx)[:, None]
    # fix the sign of each function: positive at x = 1 (u_l(1) != 0 for this kernel)
    xg, wg = np.polynomial.legendre.leggauss(order)
    Pn = np.polynomial.legendre.legvander(xg, order - 1)                  # [node, degree]
    norm = (2 * np.arange(order) + 1) / 2
    coef = np.stack([norm[:, None] * (Pn * wg[:, None]).T @ u[p * order:(p + 1) * order]
                     for p in range(len(xb) - 1)])                        # [panel, degree, l]
    sign = np.sign(coef[-1].sum(axis=0))                                  # u_l(1) = sum_n c_n P_n(1)
    return dict(lam=lam, L=L, s=S[:L + 1], xb=xb, coef=coef * sign[None, None, :], order=order)


def ir_eval(b, x):
    """u_l(x) for the basis b, [len(x), L + 1]"""
    x = np.atleast_1d(np.asarray(x, float))
    p = np.clip(np.searchsorted(b["xb"], x, side="right") - 1, 0, len(b["xb"]) - 2)
    a, c = b["xb"][p], b["xb"][p + 1]
    V = np.polynomial.legendre.legvander((2 * x - a - c) / (c - a), b["order"] - 1)
    return np.einsum("qn,qnl->ql", V, b["coef"][p])


def ir_fourier(b, beta, nu):
    """hat u_l(i nu) = int_0^beta sqrt(2/beta) u_l(2 tau/beta - 1) exp(i nu tau) d tau, panel by
    panel from the Legendre series: int_{-1}^{1} P_n(t) exp(i a t) dt = 2 i^n j_n(a)."""
    from scipy.special import spherical_jn
    nu = np.asarray(nu, float)
    out = np.zeros((len(nu), b["L"] + 1), complex)
    for p in range(len(b["xb"]) - 1):
        h, m = 0.5 * (b["xb"][p + 1] - b["xb"][p]), 0.5 * (b["xb"][p + 1] + b["xb"][p])
        a = nu * beta * h / 2
        J = np.stack([2.0 * (1j ** n) * spherical_jn(n, a) for n in range(b["order"])], axis=1)
        out += (np.exp(1j * nu * beta * (m + 1) / 2) * h)[:, None] * (J @ b["coef"][p])
    return out * np.sqrt(beta / 2)


def _roots(b, l):
    """the zeros of u_l on (-1, 1): sign changes on a fine grid refined by bisection"""
    x = np.concatenate([np.linspace(b["xb"][p], b["xb"][p + 1], 64, endpoint=False)
                        for p in range(len(b["xb"]) - 1)] + [[1.0]])
    f = ir_eval(b, x)[:, l]
    out = []
    for i in np.nonzero(np.sign(f[:-1]) * np.sign(f[1:]) < 0)[0]:
        lo, hi, flo = x[i], x[i + 1], f[i]
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            fm = ir_eval(b, [mid])[0, l]
            if np.sign(fm) == np.sign(flo):
                lo, flo = mid, fm
            else:
                hi = mid
        out.append(0.5 * (lo + hi))
    return np.array(out)


def _matsubara_sign_changes(b, beta, boson, nmax):
    """Matsubara indices n >= 0 at which hat u_L changes sign (its nonzero part: real for
    fermions of one parity, imaginary for the other), the bosonic n = 0 always included"""
    n = np.arange(nmax)
    nu = (2 * n + (0 if boson else 1)) * np.pi / beta
    uh = ir_fourier(b, beta, nu)[:, b["L"]]
    part = uh.real if np.abs(uh.real).max() > np.abs(uh.imag).max() else uh.imag
    idx = [int(i) for i in np.nonzero(np.sign(part[:-1]) * np.sign(part[1:]) < 0)[0]]
    if boson and 0 not in idx:
        idx = [0] + idx
    return np.array(idx)


def ir_grid(beta, wmax, eps, nmax=None):
    """Sampling points of the IR basis: tau = 0, the zeros of u_L mapped to tau (symmetric about
    beta/2) and beta; Matsubara indices n >= 0 where hat u_L changes sign, for fermions and for
    bosons, the shorter list extended by the next indices so both hold nw entries.  Returns
    dict(basis, tau, nf, nb)."""
    b = ir_basis(beta * wmax, eps)
    r = _roots(b, b["L"])
    r = 0.5 * (r - r[::-1])                                   # exact mirror symmetry
    tau = np.concatenate([[0.0], beta * (r + 1) / 2, [beta]])
    nmax = nmax or int(4 * beta * wmax / np.pi) + 64
    nf = _matsubara_sign_changes(b, beta, False, nmax)
    nb = _matsubara_sign_changes(b, beta, True, nmax)
    nw = max(len(nf), len(nb), (b["L"] + 2) // 2)      # the bosonic stacked system needs 2 nw - 1 >= L

    def pad(a):
        # fill the widest gap: the integer geometric mean of the pair with the largest ratio
        a = [int(v) for v in a]
        while len(a) < nw:
            i = max(range(len(a) - 1), key=lambda i: (a[i + 1] + 1) / (a[i] + 1))
            m = int(round(np.sqrt((a[i] + 1) * (a[i + 1] + 1)))) - 1
            if m <= a[i] or m >= a[i + 1]:
                m = a[-1] + 1
                a.append(m)
            else:
                a.insert(i + 1, m)
        return np.array(a, dtype=int)

    return dict(basis=b, tau=tau, nf=pad(nf), nb=pad(nb), beta=beta)


def ir_transform_matrices(grid, boson):
    """The IR counterpart of transform_matrices: X(i nu_n) = sum_j Tfwd[n, j] X(tau_j) through
    the least-squares fit of the tau samples with u_0..u_{L-1}, and Binv from the stacked system
    [X(i nu_n); X(i nu_n)^H] of the sampled frequencies and their negatives (bosonic n = 0
    once).  Returns (Tfwd, Binv, conj_rows)."""
    b, beta = grid["basis"], grid["beta"]
    L = b["L"]
    n = grid["nb"] if boson else grid["nf"]
    nu = (2 * n + (0 if boson else 1)) * np.pi / beta
    Ut = np.sqrt(2 / beta) * ir_eval(b, 2 * grid["tau"] / beta - 1)[:, :L]    # [tau, l]
    Fm = ir_fourier(b, beta, nu)[:, :L]                                       # [n, l]
    Tfwd = Fm @ np.linalg.pinv(Ut)
    conj_rows = np.nonzero(n != 0)[0] if boson else np.arange(len(n))
    S = np.vstack([Fm, Fm[conj_rows].conj()])
    return Tfwd, Ut @ np.linalg.pinv(S), conj_rows


# ----------------------------------------------------------------------------
# free Green's function (closed form from the eigen-decomposition of F; Sec. 4.1 definition of G)


def fermi_factor_parts(eps: np.ndarray, tau: np.ndarray, beta: float) -> np.ndarray:
    """g[..., t, i] = exp(-eps tau) / (1 + exp(-beta eps)), evaluated without overflow
    (for eps < 0 the equal form exp(eps (beta - tau)) / (1 + exp(beta eps)) is used)."""
    e = eps[..., None, :]
    t = tau[:, None]
    ep = np.maximum(e, 0.0)
    en = np.minimum(e, 0.0)
    a = np.exp(-ep * t) / (1.0 + np.exp(-beta * ep))
    b = np.exp(en * (beta - t)) / (1.0 + np.exp(beta * en))
    return np.where(e >= 0, a, b)


def g0_closed_form(F: np.ndarray, mu: float, beta: float, tau: np.ndarray) -> np.ndarray:
    """G0^k(tau) = -U diag(exp(-e tau)/(1 + exp(-beta e))) U^H with F^k - mu = U diag(e) U^H."""
    nao = F.shape[-1]
    e, U = np.linalg.eigh(F - mu * np.eye(nao))
    g = fermi_factor_parts(e, tau, beta)                 # [k, t, i]
    return -np.einsum("kai,kti,kbi->ktab", U, g, U.conj())


def free_count(F: np.ndarray, mu: float, beta: float, spin: float) -> float:
    """(s / Nk) sum_k sum_i 1/(1 + exp(beta (e_i - mu))), the free electron count (Sec. 4.1, N_e)."""
    e = np.linalg.eigvalsh(F) - mu
    f = np.where(e >= 0, np.exp(-beta * np.abs(e)) / (1 + np.exp(-beta * np.abs(e))),
                 1.0 / (1 + np.exp(-beta * np.abs(e))))
    return spin * f.sum() / F.shape[0]


# ----------------------------------------------------------------------------
# contractions (eq. P0 and eq. sigma of Sec. 4.1)


def polarization(G: np.ndarray, V: np.ndarray, add: np.ndarray, spin: float) -> np.ndarray:
    """P0^q_{QQ'}(tau_j) = -(s/Nk) sum_k Tr[V^{k,k+q}(Q) G^{k+q}(tau_j) V^{k+q,k}(Q') G^k(beta - tau_j)]
    with V^{k+q,k}(Q') = V^{k,k+q}(Q')^H and G^k(beta - tau_j) = G^k(tau_{ntau-1-j})."""
    nk, nt, nao, _ = G.shape
    naux = V.shape[2]
    P0 = np.zeros((nk, nt, naux, naux), dtype=complex)
    Grev = G[:, ::-1]
    for q in range(nk):
        for k in range(nk):
            kq = add[k, q]
            A = V[k, kq]                                         # [Q, a, b]
            AH = np.conj(np.swapaxes(A, -1, -2))                 # V^{k+q,k}(Q') = A(Q')^H
            X1 = A[None] @ G[kq][:, None]                        # [t, Q, a, b] = A(Q) G^{k+q}
            X2 = AH[None] @ Grev[k][:, None]                     # [t, Q', b, a] = A(Q')^H G^k(b-t)
            # Tr[X1(Q) X2(Q')] = sum_{ab} X1[Q,a,b] X2[Q',b,a]
            X2t = np.swapaxes(X2, -1, -2).reshape(nt, naux, nao * nao)
            P0[q] += X1.reshape(nt, naux, nao * nao) @ np.swapaxes(X2t, -1, -2)
    return -(spin / nk) * P0


def self_energy(G: np.ndarray, V: np.ndarray, P: np.ndarray, sub: np.ndarray) -> np.ndarray:
    """Sigma~^k_{ij}(tau) = -(1/Nk) sum_q sum_{ab} sum_{QQ'} G^{k-q}_{ab}(tau) V^{k,k-q}_{ia}(Q)
    P^q_{QQ'}(tau) V^{k-q,k}_{bj}(Q'), V^{k-q,k}(Q') = V^{k,k-q}(Q')^H.
    sub[k, q] is the index of k - q."""
    nk, nt, nao, _ = G.shape
    naux = V.shape[2]
    S = np.zeros((nk, nt, nao, nao), dtype=complex)
    for k in range(nk):
        for q in range(nk):
            kmq = sub[k, q]
            A = V[k, kmq]                                        # [Q, i, a]
            X1 = A[None] @ G[kmq][:, None]                       # [t, Q, i, b]
            Y = np.swapaxes(P[q], -1, -2) @ X1.reshape(nt, naux, nao * nao)   # sum_Q P[Q,Q'] X1[Q]
            Y = Y.reshape(nt, naux, nao, nao)                    # [t, Q', i, b]
            # sum_{Q', b} Y[Q', i, b] conj(A[Q', j, b])
            Yf = np.swapaxes(Y, 1, 2).reshape(nt, nao, naux * nao)
            Af = np.conj(np.swapaxes(A, 0, 1).reshape(nao, naux * nao))
            S[k] += Yf @ Af.T
    return -(1.0 / nk) * S


def polarization_unit(G: np.ndarray, Vq: np.ndarray, add: np.ndarray, q: int, j: int, spin: float) -> np.ndarray:
    """One output of eq. P0: P0^q_{QQ'}(tau_j), with Vq[k] = V^{k,k+q} for every k."""
    nk, nt, nao, _ = G.shape
    naux = Vq.shape[1]
    acc = np.zeros((naux, naux), dtype=complex)
    for k in range(nk):
        A = Vq[k]
        X1 = (A @ G[add[k, q], j]).reshape(naux, nao * nao)
        X2 = np.conj(np.swapaxes(A, -1, -2)) @ G[k, nt - 1 - j]
        acc += X1 @ np.swapaxes(X2, -1, -2).reshape(naux, nao * nao).T
    return -(spin / nk) * acc


def self_energy_unit(G: np.ndarray, Vk: np.ndarray, P: np.ndarray, sub: np.ndarray, k: int, j: int) -> np.ndarray:
    """One output of eq. sigma: Sigma~^k(tau_j), with Vk[q] = V^{k,k-q} and P[q] = P^q(tau_j)."""
    nk, nt, nao, _ = G.shape
    naux = Vk.shape[1]
    acc = np.zeros((nao, nao), dtype=complex)
    for q in range(nk):
        A = Vk[q]
        X1 = A @ G[sub[k, q], j]
        Y = (P[q].T @ X1.reshape(naux, nao * nao)).reshape(naux, nao, nao)
        acc += np.swapaxes(Y, 0, 1).reshape(nao, naux * nao) @ np.conj(np.swapaxes(A, 0, 1).reshape(nao, naux * nao)).T
    return -(1.0 / nk) * acc


def exchange(G: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Exchange part of the static self-energy (eq. sigma_hf, K term) with the density matrix
    gamma^k = G^k(0^-) = -G^k(beta):
    K^k = -(1/Nk) sum_{k'} sum_Q V^{k,k'}(Q) gamma^{k'} V^{k',k}(Q).  Spin-diagonal: no spin
    factor."""
    nk = G.shape[0]
    gamma = -G[:, -1]
    K = np.zeros((nk,) + G.shape[2:], dtype=complex)
    for k in range(nk):
        for kp in range(nk):
            K[k] += np.einsum("Qia,ab,Qbj->ij", V[k, kp], gamma[kp], V[kp, k], optimize=True)
    return -K / nk


def hartree(G: np.ndarray, V: np.ndarray, spin: float) -> np.ndarray:
    """Hartree part of the static self-energy (eq. sigma_hf, J term) with the density matrix
    gamma^k = G^k(0^-) = -G^k(beta): the density on the auxiliary functions,
    rho(Q) = sum_{k'} sum_{ab} gamma^{k'}_{ab} V^{k'k'}_{ba}(Q), then
    J^k_ij = (s/Nk) sum_Q V^{kk}_ij(Q) rho(Q).  The sum over the spin index sigma_1 of the
    equation gives the spin factor s (gamma is the density matrix of one spin)."""
    nk = G.shape[0]
    gamma = -G[:, -1]
    rho = np.zeros(V.shape[2], dtype=complex)
    for kp in range(nk):
        rho += np.einsum("ab,Qba->Q", gamma[kp], V[kp, kp])
    J = np.zeros((nk,) + G.shape[2:], dtype=complex)
    for k in range(nk):
        J[k] = np.einsum("Q,Qij->ij", rho, V[k, k])
    return (spin / nk) * J


def exchange_unit(G: np.ndarray, Vrow: np.ndarray, Vcol: np.ndarray) -> np.ndarray:
    """K^k of eq. sigma_hf at one k, from Vrow[k'] = V^{k,k'} and Vcol[k'] = V^{k',k} for every
    k' (the full-size check cannot hold V over all pairs)."""
    nk = G.shape[0]
    gamma = -G[:, -1]
    acc = np.zeros(G.shape[2:], dtype=complex)
    for kp in range(nk):
        acc += np.einsum("Qia,ab,Qbj->ij", Vrow[kp], gamma[kp], Vcol[kp], optimize=True)
    return -acc / nk


def hartree_unit(G: np.ndarray, Vdiag: np.ndarray, k: int, spin: float) -> np.ndarray:
    """J^k of eq. sigma_hf at one k, from the diagonal pairs Vdiag[k'] = V^{k',k'}."""
    nk = G.shape[0]
    gamma = -G[:, -1]
    rho = np.zeros(Vdiag.shape[1], dtype=complex)
    for kp in range(nk):
        rho += np.einsum("ab,Qba->Q", gamma[kp], Vdiag[kp])
    return (spin / nk) * np.einsum("Q,Qij->ij", rho, Vdiag[k])


# ----------------------------------------------------------------------------
# screened interaction (eq. P02P) and Dyson equation (eq. dyson)


def _transforms(beta, nt, nw, boson, grid):
    """the Chebyshev transforms, or those of an IR grid (ir_grid)"""
    if grid is not None:
        return ir_transform_matrices(grid, boson)
    return transform_matrices(beta, nt, nw, boson)


def _fermion_freqs(beta, nw, grid):
    if grid is not None:
        return (2 * grid["nf"] + 1) * np.pi / beta
    return matsubara(beta, nw, boson=False)


def screened(P0: np.ndarray, beta: float, nw: int, grid=None):
    """P(i Omega_n) = [I - P0(i Omega_n)]^{-1} P0(i Omega_n), then back to tau.
    Returns (P(tau), P0(i Omega), P(i Omega)).  grid: None (Chebyshev) or an IR grid."""
    nk, nt, naux, _ = P0.shape
    Tb, Bb, rows = _transforms(beta, nt, nw, True, grid)
    P0w = to_freq(P0, Tb)
    I = np.eye(naux)
    Pw = np.linalg.solve(I - P0w, P0w)
    return to_tau(Pw, Bb, rows), P0w, Pw


def dyson(F: np.ndarray, Sigma: np.ndarray, mu: float, beta: float, nw: int, grid=None):
    """G(i w_n) = [(i w_n + mu) I - F - Sigma~(i w_n)]^{-1} (S = I), then back to tau.
    Returns (G(tau), G(i w), Sigma~(i w)).  grid: None (Chebyshev) or an IR grid."""
    nk, nt, nao, _ = Sigma.shape
    Tf, Bf, rows = _transforms(beta, nt, nw, False, grid)
    Sw = to_freq(Sigma, Tf)
    w = _fermion_freqs(beta, nw, grid)
    I = np.eye(nao)
    A = (1j * w[:, None, None] + mu) * I[None] - F[:, None] - Sw
    Gw = np.linalg.inv(A)
    return to_tau(Gw, Bf, rows), Gw, Sw


def particle_number(G: np.ndarray, spin: float) -> float:
    """N_e = (s/Nk) sum_k Tr[gamma^k], gamma^k = G^k(tau = 0^-) = -G^k(beta) (S = I)."""
    nk = G.shape[0]
    return float(np.real(spin / nk * np.trace(-G[:, -1], axis1=-2, axis2=-1).sum()))


def find_mu(F, Sigma, n_target, beta, nw, spin, steps=64, grid=None):
    """Bisection on the strictly increasing N(mu) over [min eps - 20, max eps + 20]."""
    e = np.linalg.eigvalsh(F)
    lo, hi = e.min() - 20.0, e.max() + 20.0
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        G, _, _ = dyson(F, Sigma, mid, beta, nw, grid)
        if particle_number(G, spin) < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# ----------------------------------------------------------------------------
# one iteration (Alg. 2 order: P0 -> P -> Sigma -> Dyson)


def gw_iteration(F, V, G, mu, beta, nw, spin, add, sub, n_target=None, mu_steps=64, grid=None):
    """One GW iteration from G.  With n_target None, mu stays fixed.  grid: None (Chebyshev
    tau grid of G's length) or an IR grid (ir_grid) whose tau points G is sampled on."""
    P0 = polarization(G, V, add, spin)
    P, P0w, Pw = screened(P0, beta, nw, grid)
    Sigma = self_energy(G, V, P, sub)
    if n_target is not None:
        mu = find_mu(F, Sigma, n_target, beta, nw, spin, mu_steps, grid)
    Gn, Gw, Sw = dyson(F, Sigma, mu, beta, nw, grid)
    return dict(P0=P0, P=P, P0w=P0w, Pw=Pw, Sigma=Sigma, Sigmaw=Sw, G=Gn, Gw=Gw, mu=mu)
