"""Crystal descriptions, space-group operation tables, Gamma-centred meshes and
the named workloads.

This module only describes inputs: lattices, atom positions, the space-group
operations {alpha | v(alpha)} (Sec. 3.1 of the paper), basis-shell lists and
the integer k-mesh.  It performs no step of the GW method.

Conventions (shared by every consumer as an input format):

* ``lattice`` is a 3x3 array whose *columns* are the primitive vectors a_i in
  units of the cubic constant a.  A point r has fractional coordinates f with
  r = lattice @ f.
* An operation is a pair (W, w): W is the 3x3 integer rotation acting on
  fractional coordinates and w the fractional translation, so the operation maps
  f -> W f + w.  Its Cartesian rotation is R = lattice @ W @ inv(lattice).
* k points are stored as integer triples m on a Gamma-centred n x n x n mesh;
  k has fractional reciprocal coordinates m / n (units of the reciprocal basis
  b_i, b_i . a_j = 2 pi delta_ij).  The linear index of m is
  (m0 * n + m1) * n + m2.
* A shell list is a list of (atom, l).  Basis functions are numbered shell by
  shell in list order and, within a shell, by m = -l ... l (real harmonics).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


def cubic_point_group() -> list[np.ndarray]:
    """The 48 signed 3x3 permutation matrices (the holohedry O_h), identity first.

    Order: permutations of (0, 1, 2) in itertools order, then sign triples in
    product order over (+1, -1).  R[i, perm[i]] = sign[i].
    """
    ops = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for i in range(3):
                R[i, perm[i]] = signs[i]
            ops.append(R)
    return ops


def in_td(R: np.ndarray) -> bool:
    """True when the cubic operation R belongs to T_d: it maps the tetrahedron
    (1,1,1), (1,-1,-1), (-1,1,-1), (-1,-1,1) onto itself, i.e. the product of
    its three signs is +1."""
    return int(round(np.prod(R[np.nonzero(R)]))) == 1


FCC = 0.5 * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]]).T  # columns


@dataclass
class Crystal:
    name: str
    lattice: np.ndarray                      # 3x3, columns a_i
    positions: np.ndarray                    # natom x 3, fractional
    species: list[int]
    ops: list[tuple[np.ndarray, np.ndarray]]  # (W int 3x3, w fractional 3)
    symmorphic: bool = True

    @property
    def natom(self) -> int:
        return len(self.positions)

    def cart_rot(self, a: int) -> np.ndarray:
        W = self.ops[a][0].astype(float)
        A = self.lattice
        return A @ W @ np.linalg.inv(A)


def _ops_from_cart(lattice, cart_ops, trans_frac):
    A = lattice
    Ai = np.linalg.inv(A)
    out = []
    for R, t in zip(cart_ops, trans_frac):
        W = Ai @ R @ A
        Wi = np.rint(W).astype(np.int64)
        assert np.allclose(W, Wi, atol=1e-12)
        out.append((Wi, np.asarray(t, dtype=float)))
    return out


HEX_C = 2.664   # c/a of hexagonal boron nitride


def hexagonal_lattice(c: float = HEX_C) -> np.ndarray:
    """Columns a1 = (1, 0, 0), a2 = (-1/2, sqrt(3)/2, 0), a3 = (0, 0, c), in units of a."""
    return np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3.0) / 2.0, 0.0], [0.0, 0.0, c]]).T


def close_group(gens):
    """All products of the generators (W, w) acting on fractional coordinates, translations
    reduced to [0, 1); identity first, then in order of discovery."""
    def key(W, w):
        return tuple(W.ravel()), tuple(np.round(np.mod(w, 1.0), 9) % 1.0)
    ops = [(np.eye(3, dtype=np.int64), np.zeros(3))]
    seen = {key(*ops[0])}
    frontier = list(ops)
    while frontier:
        new = []
        for W1, w1 in frontier:
            for W2, w2 in gens:
                W = W1 @ W2
                w = np.mod(W1 @ w2 + w1, 1.0)
                w[np.isclose(w, 1.0)] = 0.0
                k = key(W, w)
                if k not in seen:
                    seen.add(k)
                    ops.append((W, w))
                    new.append((W, w))
        frontier = new
    return ops


def p63mmc_ops():
    """The 24 operations of P6_3/mmc (No. 194) in the hexagonal setting, from the screw axis
    6_3 = (x - y, x, z + 1/2), the inversion and the two-fold axis (y, x, -z)."""
    g6 = (np.array([[1, -1, 0], [1, 0, 0], [0, 0, 1]], dtype=np.int64), np.array([0.0, 0.0, 0.5]))
    inv = (-np.eye(3, dtype=np.int64), np.zeros(3))
    c2 = (np.array([[0, 1, 0], [1, 0, 0], [0, 0, -1]], dtype=np.int64), np.zeros(3))
    return close_group([g6, inv, c2])


def crystal(name: str) -> Crystal:
    """Named crystals: 'sc' (Pm-3m, one atom), 'rocksalt' (Fm-3m, atoms at 0
    and (1/2,1/2,1/2)a), 'diamond' (Fd-3m origin choice 1, atoms at 0 and
    (1/4,1/4,1/4)a; the 24 operations outside T_d carry v = (1/4,1/4,1/4)a), and 'hbn'
    (P6_3/mmc, No. 194, hexagonal boron nitride: B at (1/3, 2/3, 1/4) and (2/3, 1/3, 3/4), N at
    (1/3, 2/3, 3/4) and (2/3, 1/3, 1/4); half of the operations carry v = (0, 0, 1/2))."""
    oh = cubic_point_group()
    if name == "sc":
        A = np.eye(3)
        ops = _ops_from_cart(A, oh, [np.zeros(3)] * 48)
        return Crystal("sc", A, np.zeros((1, 3)), [0], ops, True)
    if name == "rocksalt":
        ops = _ops_from_cart(FCC, oh, [np.zeros(3)] * 48)
        pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
        return Crystal("rocksalt", FCC.copy(), pos, [0, 1], ops, True)
    if name == "diamond":
        tr = [np.zeros(3) if in_td(R) else np.full(3, 0.25) for R in oh]
        ops = _ops_from_cart(FCC, oh, tr)
        pos = np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25]])
        return Crystal("diamond", FCC.copy(), pos, [0, 0], ops, False)
    if name == "hbn":
        pos = np.array([[1 / 3, 2 / 3, 0.25], [2 / 3, 1 / 3, 0.75], [1 / 3, 2 / 3, 0.75], [2 / 3, 1 / 3, 0.25]])
        return Crystal("hbn", hexagonal_lattice(), pos, [0, 0, 1, 1], p63mmc_ops(), False)
    raise ValueError(f"unknown crystal {name!r}")


# ----------------------------------------------------------------------------
# k mesh

def mesh_points(n: int) -> np.ndarray:
    """All integer triples of the Gamma-centred n^3 mesh, in linear-index order."""
    g = np.arange(n)
    return np.array(list(itertools.product(g, g, g)), dtype=np.int64)


def mesh_index(m: np.ndarray, n: int) -> np.ndarray:
    m = np.mod(m, n)
    return (m[..., 0] * n + m[..., 1]) * n + m[..., 2]


def kmap(cr: Crystal, n: int) -> np.ndarray:
    """kmap[a, k] = index of alpha_a k on the mesh.  In fractional reciprocal
    coordinates the rotation acts as W^{-T}."""
    pts = mesh_points(n)
    out = np.empty((len(cr.ops), len(pts)), dtype=np.int64)
    for a, (W, _) in enumerate(cr.ops):
        WiT = np.rint(np.linalg.inv(W).T).astype(np.int64)
        out[a] = mesh_index(pts @ WiT.T, n)
    return out


def minus_k(n: int) -> np.ndarray:
    return mesh_index(-mesh_points(n), n)


def add_k(n: int) -> np.ndarray:
    """add[k1, k2] = index of k1 + k2."""
    p = mesh_points(n)
    return mesh_index(p[:, None, :] + p[None, :, :], n)


# ----------------------------------------------------------------------------
# shells

S, P, D, F_, G_ = 0, 1, 2, 3, 4


def shells_on_atoms(per_atom: list[int], natom: int) -> list[tuple[int, int]]:
    return [(x, l) for x in range(natom) for l in per_atom]


def nbf(shells) -> int:
    return sum(2 * l + 1 for _, l in shells)


@dataclass
class Workload:
    """One named workload: crystal, mesh, shells, grid and iteration settings."""
    name: str
    crystal: str
    n: int
    ao: list
    aux: list
    ntau: int
    beta: float
    seed: int
    mu_fixed: bool = False          # True: mu stays 0; False: N_e held fixed
    pairwise: bool = False          # raw V drawn per (k1, k2) pair (large meshes)
    iterations: int = 1
    spin: float = 2.0
    extra: dict = field(default_factory=dict)

    @property
    def nao(self):
        return nbf(self.ao)

    @property
    def naux(self):
        return nbf(self.aux)

    @property
    def nk(self):
        return self.n ** 3

    @property
    def nw(self):
        return 2 * self.ntau + 1


BASE_SEED = 240509494

_AO26 = [S, S, S, P, P, D, D, F_]
_AUX25 = [S, P, D, F_, G_]


def workload(name: str) -> Workload:
    """The named workloads.  'cfg0'...'cfg4' are the five configurations of the
    benchmark specification; the 'small_*' ones are reduced versions (same
    crystals, fewer k points, shells and tau points) sized so that the oracle
    finishes in seconds."""
    if name == "cfg0":
        return Workload(name, "sc", 2, shells_on_atoms([S, P, D], 1),
                        shells_on_atoms([S, S, P, P, D, F_, F_, G_], 1),
                        40, 100.0, BASE_SEED + 0, mu_fixed=True, iterations=1)
    if name == "cfg1":
        return Workload(name, "sc", 4, shells_on_atoms(_AO26, 1),
                        shells_on_atoms(_AUX25 * 6, 1), 64, 100.0, BASE_SEED + 1,
                        iterations=10)
    if name == "cfg2":
        return Workload(name, "rocksalt", 6, shells_on_atoms(_AO26, 2),
                        shells_on_atoms(_AUX25 * 5, 2), 100, 200.0, BASE_SEED + 2,
                        iterations=10, pairwise=True)
    if name == "cfg4":
        return Workload(name, "diamond", 6, shells_on_atoms(_AO26, 2),
                        shells_on_atoms(_AUX25 * 6, 2), 128, 400.0, BASE_SEED + 4,
                        iterations=10, pairwise=True)
    # reduced workloads for parity tests
    if name == "small_sc2":        # cfg0 crystal, more aux functions: several tiles + tail
        return Workload(name, "sc", 2, shells_on_atoms([S, P, D], 1),
                        shells_on_atoms(_AUX25 * 3, 1), 16, 20.0, BASE_SEED + 10)
    if name == "small_sc4":        # cfg1 crystal and mesh, small basis
        return Workload(name, "sc", 4, shells_on_atoms([S, P, D], 1),
                        shells_on_atoms([S, S, P, P, D, F_, F_, G_], 1), 12, 20.0,
                        BASE_SEED + 11, iterations=2)
    if name == "small_rocksalt":
        return Workload(name, "rocksalt", 2, shells_on_atoms([S, P, D], 2),
                        shells_on_atoms([S, P, D, F_], 2), 16, 30.0, BASE_SEED + 12)
    if name == "small_diamond":
        return Workload(name, "diamond", 2, shells_on_atoms([S, P, D], 2),
                        shells_on_atoms([S, P, D, F_], 2), 16, 30.0, BASE_SEED + 13)
    if name == "small_diamond4":
        return Workload(name, "diamond", 4, shells_on_atoms([S, P], 2),
                        shells_on_atoms([S, P, D], 2), 8, 20.0, BASE_SEED + 14)
    if name == "gamma_sc":         # a single k point (Gamma only)
        return Workload(name, "sc", 1, shells_on_atoms([S, P, D], 1),
                        shells_on_atoms(_AUX25 * 2, 1), 16, 20.0, BASE_SEED + 17)
    if name == "wide_rocksalt":    # cfg2 orbital basis (nao 52 > 32), small mesh and aux basis
        return Workload(name, "rocksalt", 2, shells_on_atoms(_AO26, 2),
                        shells_on_atoms([S, P, D, F_], 2), 16, 30.0, BASE_SEED + 15)
    if name == "wide_diamond":     # cfg4 orbital basis, non-symmorphic
        return Workload(name, "diamond", 2, shells_on_atoms(_AO26, 2),
                        shells_on_atoms([S, P, D, F_], 2), 16, 30.0, BASE_SEED + 16)
    if name == "small_hbn":        # hexagonal P6_3/mmc (non-symmorphic screw axis), 2x2x2 mesh
        return Workload(name, "hbn", 2, shells_on_atoms([S, P], 4),
                        shells_on_atoms([S, P, D], 4), 12, 25.0, BASE_SEED + 19)
    if name == "small_hbn3":       # the 3x3x3 mesh holds the K points (1/3, 1/3, 0) and (1/3, 1/3, 1/3)
        return Workload(name, "hbn", 3, shells_on_atoms([S, P], 4),
                        shells_on_atoms([S, P], 4), 10, 20.0, BASE_SEED + 20)
    if name == "pair_diamond":     # small_diamond with the pair-keyed V draws of the 6^3 meshes
        return Workload(name, "diamond", 2, shells_on_atoms([S, P, D], 2),
                        shells_on_atoms([S, P, D, F_], 2), 16, 30.0, BASE_SEED + 18, pairwise=True)
    raise ValueError(f"unknown workload {name!r}")
