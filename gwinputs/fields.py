"""Seeded synthetic inputs: Fock matrices F^k, three-index tensors V^{k1,k2}(Q)
and symmetric auxiliary-basis test matrices.

Recipe (one reading of the workload specification, stated once here):

* raw F^k = (A + A^H)/2, A_ij = (x + i y)/sqrt(2), x, y ~ N(0,1);
* raw V^{k1,k2}_{ij}(Q) = (x + i y)/sqrt(2) / (1 + Q/8), Q counted from 0;
* every raw draw comes from a Philox counter-based generator keyed by
  (seed, tensor id, first momentum index), so any row can be regenerated alone;
  workloads marked ``pairwise`` (the 6^3 meshes, whose Nk^2 raw pairs would take
  hundreds of GB) key the raw V by (seed, tensor id, k1, k2) instead and draw it from a
  counter-based generator evaluated in bulk on the generating device: the uniform
  numbers are the SplitMix64 finaliser of key + counter x 0x9E3779B97F4A7C15, turned into
  normal pairs by the Box-Muller transform (the same numbers on any device, up to the
  last bits of log, cos and sin), and only the pairs an output needs are drawn;
* the raw tensors are projected onto the subspace fixed by three commuting
  projections: space-group averaging (with the orbital representation of
  ``rep.BasisRep``; for V the auxiliary index rotates with the auxiliary
  representation at q = k2 - k1), Hermitian pairing V^{k2,k1}(Q) = V^{k1,k2}(Q)^H,
  and time reversal X^{-k} = X^{k*};
* F is finally rescaled, F <- a F + b I, so that its eigenvalues over all k span
  exactly [-2, 3] Ha.

Arrays are torch tensors (complex128) on the requested device; the group
averaging of V runs on the GPU when one is used, which keeps the
4096-pair workload to seconds.
"""
from __future__ import annotations

import numpy as np
import torch

from .crystals import Workload, crystal, kmap, minus_k, mesh_points, mesh_index
from .rep import BasisRep

TENSOR_F, TENSOR_V, TENSOR_AUXMAT, TENSOR_ORBMAT = 1, 2, 3, 4


def _philox(seed: int, tensor: int, a: int, b: int = 0) -> np.random.Generator:
    key = (seed << 64) | (tensor << 48) | (a << 24) | b
    return np.random.Generator(np.random.Philox(key=key))


def _pair_seed(seed: int, tensor: int, a: int, b: int) -> int:
    """63-bit generator seed of one (tensor, k1, k2) stream: the SplitMix64 finaliser of the
    packed key."""
    m = (1 << 64) - 1
    x = ((seed & 0xFFFFFFFF) << 32 | (tensor & 0xFF) << 24 | (a & 0xFFF) << 12 | (b & 0xFFF)) & m
    x = (x + 0x9E3779B97F4A7C15) & m
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & m
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & m
    x ^= x >> 31
    return x & ((1 << 63) - 1)


def _signed64(x: int) -> int:
    return x - (1 << 64) if x >= (1 << 63) else x


_GOLDEN = _signed64(0x9E3779B97F4A7C15)
_MIX1 = _signed64(0xBF58476D1CE4E5B9)
_MIX2 = _signed64(0x94D049BB133111EB)


def _srl(x: torch.Tensor, s: int) -> torch.Tensor:
    """logical right shift of int64 (torch shifts arithmetically)"""
    return (x >> s) & ((1 << (64 - s)) - 1)


def _mix64(x: torch.Tensor) -> torch.Tensor:
    """SplitMix64 finaliser on int64 tensors (wrapping arithmetic)."""
    x = x ^ _srl(x, 30)
    x = x * _MIX1
    x = x ^ _srl(x, 27)
    x = x * _MIX2
    return x ^ _srl(x, 31)


def _counter_normals(keys: torch.Tensor, n: int) -> torch.Tensor:
    """Standard normal pairs [len(keys), n, 2]: element e of stream `key` takes the uniforms of
    counters 2e + 1 and 2e + 2, u = (top 53 bits + 1) / 2^53 in (0, 1], through Box-Muller."""
    c = torch.arange(1, 2 * n + 1, dtype=torch.int64, device=keys.device)
    x = _mix64(keys[:, None] + c[None, :] * _GOLDEN)
    u = ((_srl(x, 11) + 1).to(torch.float64) * (2.0 ** -53)).view(len(keys), n, 2)
    r = torch.sqrt(-2.0 * torch.log(u[..., 0]))
    t = (2.0 * np.pi) * u[..., 1]
    return torch.stack((r * torch.cos(t), r * torch.sin(t)), dim=-1)


def _cnormal(rng, shape):
    z = rng.standard_normal(shape + (2,))
    return (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)


class Inputs:
    """Holds the workload, its crystal and the two orbital representations."""

    def __init__(self, wl: Workload, device="cpu"):
        self.wl = wl
        self.cr = crystal(wl.crystal)
        self.n = wl.n
        self.nk = wl.nk
        self.device = torch.device(device)
        self.ao = BasisRep(self.cr, wl.ao, wl.n)
        self.aux = BasisRep(self.cr, wl.aux, wl.n)
        self.kmap = kmap(self.cr, wl.n)                 # [op, k] -> alpha k
        self.inv_kmap = np.argsort(self.kmap, axis=1)   # [op, k] -> alpha^{-1} k
        self.mk = minus_k(wl.n)
        pts = mesh_points(wl.n)
        self.sub = mesh_index(pts[None, :, :] - pts[:, None, :], wl.n)  # sub[k1,k2] = k2-k1
        self.h = len(self.cr.ops)

    def _t(self, x):
        return torch.as_tensor(x, dtype=torch.complex128, device=self.device)

    # -- two-index quantities -------------------------------------------------
    def _sym_two_index(self, rep: BasisRep, raw: np.ndarray) -> np.ndarray:
        """Time reversal, then group averaging, of a [Nk, ..., n, n] array."""
        X = 0.5 * (raw + raw[self.mk].conj())
        out = np.zeros_like(X)
        for a in range(self.h):
            for k in range(self.nk):
                p = self.inv_kmap[a, k]
                O = rep.matrix(a, p)
                out[k] += O @ X[p] @ O.conj().T
        return out / self.h

    def fock(self) -> torch.Tensor:
        wl = self.wl
        raw = np.stack([_cnormal(_philox(wl.seed, TENSOR_F, k), (wl.nao, wl.nao))
                        for k in range(self.nk)])
        raw = 0.5 * (raw + raw.conj().transpose(0, 2, 1))
        F = self._sym_two_index(self.ao, raw)
        F = 0.5 * (F + F.conj().transpose(0, 2, 1))
        ev = np.linalg.eigvalsh(F)
        lo, hi = ev.min(), ev.max()
        a = 5.0 / (hi - lo)
        F = a * F + (-2.0 - a * lo) * np.eye(wl.nao)[None]
        return self._t(F)

    def aux_matrices(self, ntau: int, scale: float = 0.05, qs=None) -> torch.Tensor:
        """Symmetric Hermitian auxiliary-basis matrices X^q(tau_j), [Nk, ntau, naux, naux];
        used as a stand-in screened interaction for contraction-only tests."""
        wl = self.wl
        raw = np.stack([np.stack([_cnormal(_philox(wl.seed, TENSOR_AUXMAT, q, j), (wl.naux, wl.naux))
                                  for j in range(ntau)]) for q in range(self.nk)])
        raw = 0.5 * (raw + raw.conj().swapaxes(-1, -2))
        X = self._sym_two_index(self.aux, raw)
        X = scale * 0.5 * (X + X.conj().swapaxes(-1, -2))
        if qs is not None:
            X = X[list(qs)]
        return self._t(X)

    def orb_matrices(self, nmat: int, scale: float = 0.01) -> torch.Tensor:
        """Symmetric Hermitian orbital-basis matrices Y^k_j, [Nk, nmat, nao, nao] (time reversal
        and group averaging as for F); the orbital twin of aux_matrices, used to assemble
        stand-in self-energies for Dyson-only tests."""
        wl = self.wl
        raw = np.stack([np.stack([_cnormal(_philox(wl.seed, TENSOR_ORBMAT, k, j), (wl.nao, wl.nao))
                                  for j in range(nmat)]) for k in range(self.nk)])
        raw = 0.5 * (raw + raw.conj().swapaxes(-1, -2))
        Y = self._sym_two_index(self.ao, raw)
        return self._t(scale * 0.5 * (Y + Y.conj().swapaxes(-1, -2)))

    # -- three-index tensor ---------------------------------------------------
    def _raw_V(self) -> torch.Tensor:
        wl = self.wl
        scale = 1.0 / (1.0 + np.arange(wl.naux) / 8.0)
        rows = []
        for k1 in range(self.nk):
            r = _cnormal(_philox(wl.seed, TENSOR_V, k1), (self.nk, wl.naux, wl.nao, wl.nao))
            r *= scale[None, :, None, None]
            rows.append(torch.as_tensor(r, dtype=torch.complex128).to(self.device))
        return torch.stack(rows)

    def _paired_V(self) -> torch.Tensor:
        """Hermitian pairing and time reversal of the raw tensor, all pairs."""
        raw = self._raw_V()
        mk = torch.as_tensor(self.mk, device=self.device)
        W = raw.clone()
        W += raw.transpose(0, 1).conj().transpose(-1, -2)          # V^{k2,k1}(Q)^H
        W += raw[mk][:, mk].conj()                                   # V^{-k1,-k2}(Q)^*
        W += raw.transpose(0, 1)[mk][:, mk].transpose(-1, -2)        # V^{-k2,-k1}(Q)^T
        del raw
        return W * 0.25

    def _raw_pairs(self, p1, p2) -> torch.Tensor:
        """Raw V^{p1,p2}(Q) of pairwise workloads, each pair from its own keyed counter stream."""
        wl = self.wl
        n = wl.naux * wl.nao * wl.nao
        keys = torch.as_tensor([_signed64(_pair_seed(wl.seed, TENSOR_V, int(a), int(b))) for a, b in zip(p1, p2)],
                               dtype=torch.int64, device=self.device)
        out = torch.empty((len(p1), wl.naux, wl.nao, wl.nao), dtype=torch.complex128, device=self.device)
        for c0 in range(0, len(p1), 32):     # bounded temporaries
            z = _counter_normals(keys[c0:c0 + 32], n)       # [pairs, n, 2]
            out[c0:c0 + 32] = torch.view_as_complex(z).view(-1, wl.naux, wl.nao, wl.nao)
        scale = torch.as_tensor(1.0 / (1.0 + np.arange(wl.naux) / 8.0) / np.sqrt(2.0), device=self.device)
        out *= scale[None, :, None, None]
        return out

    def _paired_pairs(self, p1, p2) -> torch.Tensor:
        """Hermitian pairing and time reversal of the raw pairs (p1, p2), as _paired_V does for
        the whole mesh: (V^{k1,k2} + V^{k2,k1 H} + V^{-k1,-k2 *} + V^{-k2,-k1 T}) / 4."""
        m1, m2 = self.mk[p1], self.mk[p2]
        W = self._raw_pairs(p1, p2)
        W += self._raw_pairs(p2, p1).conj().transpose(-1, -2)
        W += self._raw_pairs(m1, m2).conj()
        W += self._raw_pairs(m2, m1).transpose(-1, -2)
        return W * 0.25

    def three_index(self, pairs, chunk: int = 256) -> torch.Tensor:
        """Symmetric V^{k1,k2} for the given list of (k1, k2): [len(pairs), naux, nao, nao]."""
        pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        wl = self.wl
        if wl.pairwise:
            if len(pairs) > 1 and (pairs[:, 0] == pairs[0, 0]).all():
                return self._three_index_row(int(pairs[0, 0]), pairs[:, 1])
            return self._three_index_pairwise(pairs, max(1, min(chunk, 64)))
        W = self._paired_V()
        out = torch.zeros((len(pairs), wl.naux, wl.nao, wl.nao), dtype=torch.complex128,
                          device=self.device)
        for a in range(self.h):
            Oao = self._t(np.stack([self.ao.matrix(a, k) for k in range(self.nk)]))
            Oaux = self._t(np.stack([self.aux.matrix(a, q) for q in range(self.nk)]))
            for c0 in range(0, len(pairs), chunk):
                pc = pairs[c0:c0 + chunk]
                p1 = self.inv_kmap[a, pc[:, 0]]
                p2 = self.inv_kmap[a, pc[:, 1]]
                q0 = self.sub[p1, p2]
                Wsel = W[torch.as_tensor(p1, device=self.device), torch.as_tensor(p2, device=self.device)]
                L = Oao[torch.as_tensor(p1, device=self.device)]
                R = Oao[torch.as_tensor(p2, device=self.device)]
                T = L[:, None] @ Wsel @ R.conj().transpose(-1, -2)[:, None]
                X = Oaux[torch.as_tensor(q0, device=self.device)]
                T = (X @ T.reshape(len(pc), wl.naux, wl.nao * wl.nao)).reshape(T.shape)
                out[c0:c0 + chunk] += T
        del W
        return out / self.h

    def _omats(self, rep: BasisRep, a: int) -> torch.Tensor:
        """O^k(alpha_a) for every k of the mesh, [Nk, size, size], formed on the device."""
        return self._t(rep.template(a))[None] * self._t(rep.column_phases(a))[:, None, :]

    def _three_index_pairwise(self, pairs, chunk: int) -> torch.Tensor:
        wl = self.wl
        dev = self.device
        out = torch.zeros((len(pairs), wl.naux, wl.nao, wl.nao), dtype=torch.complex128, device=dev)
        for a in range(self.h):
            Oao = self._omats(self.ao, a)
            Oaux = self._omats(self.aux, a)
            for c0 in range(0, len(pairs), chunk):
                pc = pairs[c0:c0 + chunk]
                p1 = self.inv_kmap[a, pc[:, 0]]
                p2 = self.inv_kmap[a, pc[:, 1]]
                q0 = self.sub[p1, p2]
                Wsel = self._paired_pairs(p1, p2)
                L = Oao[torch.as_tensor(p1, device=dev)]
                R = Oao[torch.as_tensor(p2, device=dev)].conj().transpose(-1, -2).contiguous()
                T = L[:, None] @ Wsel @ R[:, None]
                X = Oaux[torch.as_tensor(q0, device=dev)]
                T = (X @ T.reshape(len(pc), wl.naux, wl.nao * wl.nao)).reshape(T.shape)
                out[c0:c0 + chunk] += T
        return out / self.h

    def _paired_rows(self, p1: int):
        """Paired V^{x,p2} for every p2 of the mesh and x in {p1, -p1}, as _paired_pairs makes
        them, from the raw rows V^{x,.} and columns V^{.,x} drawn once: each pairing reads the
        raw sets of x and of -x."""
        m1 = int(self.mk[p1])
        xs = [p1] if m1 == p1 else [p1, m1]
        all_k = np.arange(self.nk)
        row = {x: self._raw_pairs(np.full(self.nk, x), all_k) for x in xs}
        col = {x: self._raw_pairs(all_k, np.full(self.nk, x)) for x in xs}
        mk = torch.as_tensor(self.mk, device=self.device)
        out = {}
        for x in xs:
            mx = int(self.mk[x])
            W = row[x].clone()
            W += col[x].conj().transpose(-1, -2)
            W += row[mx][mk].conj()
            W += col[mx][mk].transpose(-1, -2)
            out[x] = W * 0.25
        return out

    def _three_index_row(self, k1: int, k2s) -> torch.Tensor:
        """The same projection for pairs (k1, k2) with one k1: every operation alpha reads the raw
        row p1 = alpha^{-1} k1, so each distinct p1 (the star of k1) is paired once and reused,
        together with -p1 when that is in the star too.  Per operation the orbital factors and
        the auxiliary rotation run as large GEMMs: R^{p2} over the stacked rows (Q, a) of each
        pair, the auxiliary template over Q (its column phases scale the rows first), and L over
        the stacked columns (pair, Q, b)."""
        wl = self.wl
        dev = self.device
        k2s = np.asarray(k2s, dtype=np.int64)
        npair, na, no = len(k2s), wl.naux, wl.nao
        out = torch.zeros((npair, na, no, no), dtype=torch.complex128, device=dev)
        by_p1 = {}
        for a in range(self.h):
            by_p1.setdefault(int(self.inv_kmap[a, k1]), []).append(a)
        done = set()
        for p1 in by_p1:
            if p1 in done:
                continue
            W = self._paired_rows(p1)
            for x, Wx in W.items():
                if x not in by_p1:
                    continue
                done.add(x)
                for a in by_p1[x]:
                    p2 = torch.as_tensor(self.inv_kmap[a, k2s], device=dev)
                    q0 = torch.as_tensor(self.sub[x, self.inv_kmap[a, k2s]], device=dev)
                    Oao = self._omats(self.ao, a)
                    L = Oao[x]
                    R = Oao[p2].conj().transpose(-1, -2)
                    T = Wx[p2].reshape(npair, na * no, no) @ R                       # V R
                    ph = self._t(self.aux.column_phases(a))[q0]                     # [pair, Q]
                    T = (T.reshape(npair, na, no * no) * ph[:, :, None]).reshape(npair, na, no * no)
                    T = self._t(self.aux.template(a)) @ T                            # O_aux V R
                    T = T.reshape(npair * na, no, no).transpose(1, 2).reshape(-1, no) @ L.transpose(0, 1)
                    out += T.reshape(npair, na, no, no).transpose(-1, -2)            # L (.) per matrix
            del W
        return out / self.h

    def three_index_full(self) -> torch.Tensor:
        """V^{k1,k2} for every pair of the mesh: [Nk, Nk, naux, nao, nao]."""
        nk = self.nk
        pairs = [(a, b) for a in range(nk) for b in range(nk)]
        V = self.three_index(pairs)
        return V.reshape(nk, nk, *V.shape[1:])
