"""Real spherical harmonics, their rotation matrices and the Bloch-orbital
representation used to group-average the synthetic inputs.

This is input preparation: the synthetic Fock matrices and three-index tensors
are projected onto the space-group-symmetric subspace with these matrices, as
the workload specification asks ("symmetrised by group averaging with Wigner
rotation matrices").  The library under test builds its own representation
matrices from the same crystal description; nothing here is shared with it.

Real-harmonic convention (part of the input format):
  Y_{l,0}  = N_l0 P_l(z)
  Y_{l,m}  = sqrt(2) N_lm P_l^m(z) cos(m phi)    (m > 0)
  Y_{l,-m} = sqrt(2) N_lm P_l^m(z) sin(m phi)    (m > 0)
  N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),  P_l^m without the Condon-Shortley
  phase, functions ordered m = -l ... l.
"""
from __future__ import annotations

import math

import numpy as np

from .crystals import Crystal, mesh_points


def real_harmonics(l: int, pts: np.ndarray) -> np.ndarray:
    """Values of the 2l+1 real harmonics at unit vectors pts (N x 3)."""
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    out = np.zeros((len(pts), 2 * l + 1))
    w = (x + 1j * y)
    for m in range(0, l + 1):
        # Q_j^m(z) = P_j^m(z) / (1 - z^2)^{m/2}, by upward recursion in j
        qmm = float(np.prod(np.arange(1, 2 * m, 2))) if m > 0 else 1.0
        q_prev, q = None, np.full_like(z, qmm)
        for j in range(m + 1, l + 1):
            if q_prev is None:
                q_new = z * (2 * m + 1) * q
            else:
                q_new = ((2 * j - 1) * z * q - (j + m - 1) * q_prev) / (j - m)
            q_prev, q = q, q_new
        norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                         * math.factorial(l - m) / math.factorial(l + m))
        wm = w ** m
        if m == 0:
            out[:, l] = norm * q
        else:
            out[:, l + m] = math.sqrt(2) * norm * q * wm.real
            out[:, l - m] = math.sqrt(2) * norm * q * wm.imag
    return out


_PTS = None


def _sample_points():
    global _PTS
    if _PTS is None:
        rng = np.random.Generator(np.random.Philox(key=7))
        p = rng.standard_normal((64, 3))
        _PTS = p / np.linalg.norm(p, axis=1, keepdims=True)
    return _PTS


def wigner_real(l: int, R: np.ndarray) -> np.ndarray:
    """D^l(R) with Y_m(R^{-1} r) = sum_m' Y_m'(r) D[m', m] (proper or improper R)."""
    pts = _sample_points()
    A = real_harmonics(l, pts)
    B = real_harmonics(l, pts @ np.linalg.inv(R).T)
    D, *_ = np.linalg.lstsq(A, B, rcond=None)
    return D


class BasisRep:
    """Action of the space group on Bloch orbitals built from a shell list."""

    def __init__(self, cr: Crystal, shells, n: int):
        self.cr, self.shells, self.n = cr, list(shells), n
        self.offsets = np.cumsum([0] + [2 * l + 1 for _, l in shells])[:-1]
        self.size = int(sum(2 * l + 1 for _, l in shells))
        # local shell index of each shell on its atom
        count = {}
        self.local = []
        for x, l in shells:
            self.local.append(count.get(x, 0))
            count[x] = count.get(x, 0) + 1
        self.lookup = {(x, t): s for s, (x, t) in enumerate(zip([x for x, _ in shells], self.local))}
        self.perm, self.shift = self._atom_maps()
        self.D = [{l: wigner_real(l, cr.cart_rot(a)) for l in sorted({l for _, l in shells})}
                  for a in range(len(cr.ops))]
        self.pts = mesh_points(n)

    def _atom_maps(self):
        cr = self.cr
        perm = np.zeros((len(cr.ops), cr.natom), dtype=np.int64)
        shift = np.zeros((len(cr.ops), cr.natom, 3), dtype=np.int64)
        for a, (W, w) in enumerate(cr.ops):
            for x in range(cr.natom):
                img = W @ cr.positions[x] + w
                for y in range(cr.natom):
                    d = img - cr.positions[y]
                    if np.allclose(d, np.rint(d), atol=1e-9):
                        perm[a, x], shift[a, x] = y, np.rint(d).astype(np.int64)
                        break
                else:
                    raise ValueError("operation does not map the crystal onto itself")
        return perm, shift

    def template(self, a: int) -> np.ndarray:
        """O^k(alpha_a) without its k-dependent phases: the Wigner blocks at the permuted
        shell positions."""
        O = np.zeros((self.size, self.size), dtype=complex)
        for s, (x, l) in enumerate(self.shells):
            sp = self.lookup[(self.perm[a, x], self.local[s])]
            o, op = self.offsets[s], self.offsets[sp]
            O[op:op + 2 * l + 1, o:o + 2 * l + 1] = self.D[a][l]
        return O

    def column_phases(self, a: int) -> np.ndarray:
        """[Nk, size]: the phase every column of O^k(alpha_a) carries (that of its shell), so
        that O^k(alpha_a) = template(a) * column_phases(a)[k][None, :]."""
        W = self.cr.ops[a][0]
        kt = (self.pts @ np.rint(np.linalg.inv(W)).astype(np.int64)) % self.n     # rows: W^{-T} k
        shell_of_col = np.repeat(np.arange(len(self.shells)), [2 * l + 1 for _, l in self.shells])
        sh = self.shift[a][[x for x, _ in self.shells]]                            # [shells, 3]
        ph = np.exp(-2j * np.pi * (kt @ sh.T) / self.n)                           # [Nk, shells]
        return ph[:, shell_of_col]

    def matrix(self, a: int, k: int) -> np.ndarray:
        """O^k(alpha_a): columns are the images of the Bloch orbitals at k,
        expanded in the Bloch orbitals at alpha k (reduced to the mesh)."""
        W = self.cr.ops[a][0]
        kt = (np.rint(np.linalg.inv(W).T).astype(np.int64) @ self.pts[k]) % self.n
        O = np.zeros((self.size, self.size), dtype=complex)
        for s, (x, l) in enumerate(self.shells):
            xp = self.perm[a, x]
            sp = self.lookup[(xp, self.local[s])]
            phase = np.exp(-2j * np.pi * np.dot(kt, self.shift[a, x]) / self.n)
            o, op = self.offsets[s], self.offsets[sp]
            O[op:op + 2 * l + 1, o:o + 2 * l + 1] = phase * self.D[a][l]
        return O
