"""ctypes binding of libgwsym (include/gwsym.h).

Argument marshalling only: every numerical step runs in the library.  Device buffers are
torch CUDA tensors (complex128) or raw integer addresses; the stream is the current torch
stream unless one is given.  A missing library raises at import time.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgwsym.so")

if not os.path.exists(_LIB_PATH):
    raise ImportError(f"libgwsym.so not built at {_LIB_PATH}; run python -m paper_2405_09494_amd.build")
lib = C.CDLL(_LIB_PATH)

MODE_FULL, MODE_ROTATE, MODE_BLOCK = 0, 1, 2
FP64, FP32, BF16X6, BF16X3 = 0, 1, 2, 3
SCHED_GROUPED, SCHED_UNBATCHED = 0, 1
GRID_CHEBYSHEV, GRID_IR = 0, 1
BLOCKS_ISOTYPIC, BLOCKS_PARTNER = 0, 1
KIND_F, KIND_G, KIND_P = 0, 1, 2

STATUS = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ENOMEM", -4: "EHIP", -5: "ESINGULAR", -6: "ENOCONV",
          -7: "ESTATE"}


class Params(C.Structure):
    _fields_ = [("beta", C.c_double), ("ntau", C.c_int), ("nw", C.c_int), ("spin", C.c_double),
                ("mode", C.c_int), ("precision", C.c_int), ("half_tau", C.c_int), ("tau_chunk", C.c_int),
                ("sched", C.c_int), ("grid", C.c_int), ("ir_wmax", C.c_double), ("ir_eps", C.c_double),
                ("blocks", C.c_int)]


class Crystal(C.Structure):
    _fields_ = [("lattice", C.c_double * 9), ("natom", C.c_int), ("positions", C.POINTER(C.c_double)),
                ("nop", C.c_int), ("rot", C.POINTER(C.c_int)), ("trans", C.POINTER(C.c_double)),
                ("kmesh", C.c_int), ("nshell_ao", C.c_int), ("ao_atom", C.POINTER(C.c_int)),
                ("ao_l", C.POINTER(C.c_int)), ("nshell_aux", C.c_int), ("aux_atom", C.POINTER(C.c_int)),
                ("aux_l", C.POINTER(C.c_int))]


class Tuning(C.Structure):
    _fields_ = [("tau_chunk", C.c_int), ("wg_target", C.c_int * 3), ("cols", C.c_int * 3),
                ("xcd_order", C.c_int * 3), ("kdepth", C.c_int * 3), ("prefetch", C.c_int * 3)]
    _LISTS = ("wg_target", "cols", "xcd_order", "kdepth", "prefetch")
    _DEFAULTS = {"prefetch": [2, 2, 2]}   # fields a plan stored before they existed

    def to_dict(self):
        d = {"tau_chunk": int(self.tau_chunk)}
        d.update({f: list(getattr(self, f)) for f in self._LISTS})
        return d

    @classmethod
    def from_dict(cls, d):
        t = cls()
        t.tau_chunk = int(d["tau_chunk"])
        for f in cls._LISTS:
            getattr(t, f)[:] = [int(x) for x in d.get(f, cls._DEFAULTS.get(f))]
        return t


_vp = C.c_void_p
lib.gwsym_create.argtypes = [C.POINTER(Params), C.POINTER(_vp)]
lib.gwsym_destroy.argtypes = [_vp]
lib.gwsym_destroy.restype = None
lib.gwsym_last_error.argtypes = [_vp]
lib.gwsym_last_error.restype = C.c_char_p
lib.gwsym_build_symmetry_basis.argtypes = [_vp, C.POINTER(Crystal)]
lib.gwsym_table_size.argtypes = [_vp, C.c_char_p]
lib.gwsym_table_size.restype = C.c_int64
lib.gwsym_get.argtypes = [_vp, C.c_char_p, _vp, C.c_int64]
lib.gwsym_device_init.argtypes = [_vp, _vp]
lib.gwsym_load_V.argtypes = [_vp, _vp, _vp]
lib.gwsym_to_block.argtypes = [_vp, C.c_int, _vp, _vp, _vp]
lib.gwsym_from_block.argtypes = [_vp, C.c_int, _vp, _vp, _vp]
lib.gwsym_g0.argtypes = [_vp, _vp, C.c_double, _vp, _vp, _vp]
lib.gwsym_polarization.argtypes = [_vp, _vp, _vp, _vp]
lib.gwsym_screened_interaction.argtypes = [_vp, _vp, _vp, _vp]
lib.gwsym_self_energy.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.gwsym_find_mu.argtypes = [_vp, _vp, _vp, C.c_double, _vp, _vp]
lib.gwsym_dyson_G.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
lib.gwsym_dyson_G_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
lib.gwsym_iteration.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_double, C.c_int, _vp]
lib.gwsym_exchange.argtypes = [_vp, _vp, _vp, _vp]
lib.gwsym_hartree.argtypes = [_vp, _vp, _vp, _vp]
lib.gwsym_fock.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.gwsym_scf_iteration.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_double, C.c_int, _vp]
lib.gwsym_autotune.argtypes = [_vp, _vp, C.POINTER(Tuning)]
lib.gwsym_get_tuning.argtypes = [_vp, C.POINTER(Tuning)]
lib.gwsym_set_tuning.argtypes = [_vp, C.POINTER(Tuning), _vp]
lib.gwsym_flop_counts.argtypes = [_vp, C.POINTER(C.c_double)]
lib.gwsym_check.argtypes = [_vp, _vp]
lib.gwsym_profile.argtypes = [_vp, C.c_int]
lib.gwsym_profile_read.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]

EXPORTED = ["gwsym_create", "gwsym_destroy", "gwsym_last_error", "gwsym_build_symmetry_basis",
            "gwsym_table_size", "gwsym_get", "gwsym_device_init", "gwsym_load_V", "gwsym_to_block",
            "gwsym_from_block", "gwsym_g0", "gwsym_polarization", "gwsym_screened_interaction",
            "gwsym_self_energy", "gwsym_find_mu", "gwsym_dyson_G", "gwsym_iteration", "gwsym_exchange",
            "gwsym_hartree", "gwsym_fock", "gwsym_scf_iteration", "gwsym_autotune", "gwsym_get_tuning",
            "gwsym_set_tuning", "gwsym_flop_counts", "gwsym_profile", "gwsym_profile_read", "gwsym_check", "gwsym_dyson_G_noalloc"]

PROFILE_CLASSES = ["p0_contraction", "sigma_aux_contraction", "sigma_orb_contraction", "row_block_multiply",
                   "two_sided_block_multiply", "transforms", "inverses", "other"]


class GwsymError(RuntimeError):
    pass


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


class Context:
    """One symmetry-adapted GW problem: crystal, mesh, bases, grids, device state."""

    def __init__(self, beta, ntau, nw, spin=2.0, mode=MODE_BLOCK, precision=FP64, half_tau=True, tau_chunk=0,
                 sched=SCHED_GROUPED, ir=None, blocks=BLOCKS_PARTNER):
        """ir: None for the Chebyshev grid of ntau points and nw frequencies, or (wmax, eps) for
        the sparse-sampling IR grid (ntau and nw are then chosen by the library).  blocks:
        BLOCKS_PARTNER (partner-function blocks) or BLOCKS_ISOTYPIC (one block per irrep)."""
        grid, wmax, eps = (GRID_IR, float(ir[0]), float(ir[1])) if ir else (GRID_CHEBYSHEV, 0.0, 0.0)
        self.params = Params(beta, ntau, nw, spin, mode, precision, int(half_tau), tau_chunk, sched, grid, wmax,
                             eps, blocks)
        h = _vp()
        self._check(lib.gwsym_create(C.byref(self.params), C.byref(h)), None)
        self.h = h
        self._keep = []

    def _check(self, st, h="self"):
        if st != 0:
            msg = lib.gwsym_last_error(self.h if h == "self" else None).decode()
            raise GwsymError(f"{STATUS.get(st, st)}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            lib.gwsym_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- host ------------------------------------------------------------------
    def build_symmetry_basis(self, lattice, positions, rot, trans, kmesh, ao_shells, aux_shells):
        lattice = np.ascontiguousarray(lattice, dtype=np.float64).reshape(9)
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1)
        rot = np.ascontiguousarray(rot, dtype=np.int32).reshape(-1)
        trans = np.ascontiguousarray(trans, dtype=np.float64).reshape(-1)
        ao = np.ascontiguousarray(ao_shells, dtype=np.int32).reshape(-1, 2)
        aux = np.ascontiguousarray(aux_shells, dtype=np.int32).reshape(-1, 2)
        ao_atom, ao_l = np.ascontiguousarray(ao[:, 0]), np.ascontiguousarray(ao[:, 1])
        aux_atom, aux_l = np.ascontiguousarray(aux[:, 0]), np.ascontiguousarray(aux[:, 1])
        self._keep = [pos, rot, trans, ao_atom, ao_l, aux_atom, aux_l]
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        cr = Crystal((C.c_double * 9)(*lattice), len(pos) // 3, pos.ctypes.data_as(dp), len(rot) // 9,
                     rot.ctypes.data_as(ip), trans.ctypes.data_as(dp), int(kmesh), len(ao),
                     ao_atom.ctypes.data_as(ip), ao_l.ctypes.data_as(ip), len(aux), aux_atom.ctypes.data_as(ip),
                     aux_l.ctypes.data_as(ip))
        self._check(lib.gwsym_build_symmetry_basis(self.h, C.byref(cr)))
        d = self.table("dims")
        self.nk, self.nibz, self.nao, self.naux, self.ntau, self.nw, self.nop, self.mode = map(int, d)
        self.g_off = self.table("g_off")
        self.p_off = self.table("p_off")
        self.f_off = self.table("f_off")
        return self

    _COMPLEX = {"U_ao", "U_aux", "O_ao", "O_aux", "Tf", "Tb", "Bf", "Bb"}
    _REAL = {"tau", "vtile_stats"}

    def table(self, name):
        nb = lib.gwsym_table_size(self.h, name.encode())
        if nb < 0:
            self._check(int(nb))
        if name in self._COMPLEX:
            out = np.empty(nb // 16, dtype=np.complex128)
        elif name in self._REAL:
            out = np.empty(nb // 8, dtype=np.float64)
        else:
            out = np.empty(nb // 8, dtype=np.int64)
        self._check(lib.gwsym_get(self.h, name.encode(), out.ctypes.data, nb))
        return out

    def blocks(self, aux=False):
        n = self.naux if aux else self.nao
        t = self.table("aux_blocks" if aux else "ao_blocks").reshape(self.nibz, 1 + n)
        return [list(map(int, row[1:1 + row[0]])) for row in t]

    def leads(self, aux=False):
        """per irreducible point and block: the block whose values it repeats (itself if none)"""
        n = self.naux if aux else self.nao
        t = self.table("aux_lead" if aux else "ao_lead").reshape(self.nibz, n)
        return [list(map(int, row[row >= 0])) for row in t]

    # sizes of the packed layouts (complex elements)
    @property
    def g_size(self):
        return int(self.g_off[-1])

    @property
    def p_size(self):
        return int(self.p_off[-1])

    @property
    def f_size(self):
        return int(self.f_off[-1])

    # -- device ------------------------------------------------------------------
    def device_init(self, stream=None):
        self._check(lib.gwsym_device_init(self.h, _stream(stream)))
        return self

    def load_V(self, V_ibz, stream=None):
        self._check(lib.gwsym_load_V(self.h, _ptr(V_ibz), _stream(stream)))

    def to_block(self, kind, full, blk, stream=None):
        self._check(lib.gwsym_to_block(self.h, kind, _ptr(full), _ptr(blk), _stream(stream)))

    def from_block(self, kind, blk, full, stream=None):
        self._check(lib.gwsym_from_block(self.h, kind, _ptr(blk), _ptr(full), _stream(stream)))

    def g0(self, F_blk, mu, G_blk, n_free=None, stream=None):
        self._check(lib.gwsym_g0(self.h, _ptr(F_blk), float(mu), _ptr(G_blk), _ptr(n_free), _stream(stream)))

    def polarization(self, G_blk, P0_blk, stream=None):
        self._check(lib.gwsym_polarization(self.h, _ptr(G_blk), _ptr(P0_blk), _stream(stream)))

    def screened_interaction(self, P0_blk, P_blk, stream=None):
        self._check(lib.gwsym_screened_interaction(self.h, _ptr(P0_blk), _ptr(P_blk), _stream(stream)))

    def self_energy(self, G_blk, P_blk, S_blk, stream=None):
        self._check(lib.gwsym_self_energy(self.h, _ptr(G_blk), _ptr(P_blk), _ptr(S_blk), _stream(stream)))

    def find_mu(self, F_blk, S_blk, n_target, mu, stream=None):
        self._check(lib.gwsym_find_mu(self.h, _ptr(F_blk), _ptr(S_blk), float(n_target), _ptr(mu), _stream(stream)))

    def dyson_G(self, F_blk, S_blk, mu, G_blk, stream=None):
        self._check(lib.gwsym_dyson_G(self.h, _ptr(F_blk), _ptr(S_blk), _ptr(mu), _ptr(G_blk), _stream(stream)))

    def dyson_G_noalloc(self, F_blk, S_blk, mu, G_blk, stream=None):
        self._check(lib.gwsym_dyson_G_noalloc(self.h, _ptr(F_blk), _ptr(S_blk), _ptr(mu), _ptr(G_blk),
                                              _stream(stream)))

    def exchange(self, G_blk, K_blk, stream=None):
        self._check(lib.gwsym_exchange(self.h, _ptr(G_blk), _ptr(K_blk), _stream(stream)))

    def hartree(self, G_blk, J_blk, stream=None):
        self._check(lib.gwsym_hartree(self.h, _ptr(G_blk), _ptr(J_blk), _stream(stream)))

    def fock(self, H0_blk, G_blk, F_blk, stream=None):
        self._check(lib.gwsym_fock(self.h, _ptr(H0_blk), _ptr(G_blk), _ptr(F_blk), _stream(stream)))

    def scf_iteration(self, H0_blk, F_blk, G_blk, P0_blk, P_blk, S_blk, mu, n_target=0.0, use_graph=False,
                      stream=None):
        self._check(lib.gwsym_scf_iteration(self.h, _ptr(H0_blk), _ptr(F_blk), _ptr(G_blk), _ptr(P0_blk),
                                            _ptr(P_blk), _ptr(S_blk), _ptr(mu), float(n_target or 0.0),
                                            int(bool(use_graph)), _stream(stream)))

    def iteration(self, F_blk, G_blk, P0_blk, P_blk, S_blk, mu, n_target=0.0, use_graph=False, stream=None):
        self._check(lib.gwsym_iteration(self.h, _ptr(F_blk), _ptr(G_blk), _ptr(P0_blk), _ptr(P_blk), _ptr(S_blk),
                                        _ptr(mu), float(n_target or 0.0), int(bool(use_graph)), _stream(stream)))

    def check(self, stream=None):
        """Waits for the queued work and raises GwsymError for a flagged singular inverse
        (ESINGULAR) or an unbracketed chemical potential (ENOCONV); clears the flags."""
        self._check(lib.gwsym_check(self.h, _stream(stream)))

    # -- launch plan ----------------------------------------------------------------
    def plan_key(self):
        """Hash of what a contraction plan depends on: parameters, sizes and block structure."""
        import hashlib
        h = hashlib.sha256()
        p = self.params
        h.update(repr((p.beta, p.ntau, p.nw, p.mode, p.precision, p.half_tau)
                      + ((p.sched,) if p.sched else ())
                      + ((p.grid, p.ir_wmax, p.ir_eps) if p.grid else ())
                      + (("isotypic",) if p.blocks == BLOCKS_ISOTYPIC else ())).encode())
        for name in ("dims", "ibz", "rep", "ao_blocks", "aux_blocks"):
            h.update(self.table(name).tobytes())
        return h.hexdigest()

    @staticmethod
    def device_key():
        """Architecture and compute-unit count of device 0, e.g. gfx950-256cu."""
        import torch
        p = torch.cuda.get_device_properties(0)
        return f"{p.gcnArchName.split(':')[0]}-{p.multi_processor_count}cu"

    def autotune(self, stream=None, cache=None, update=True, time_missing=True):
        """Time candidate contraction plans and keep the fastest (gwsym_autotune); returns the
        plan as a dict.  cache: optional JSON file of plans keyed by plan_key() and
        device_key(); a plan found there is applied without timing, and (update=True) a newly
        timed one is added to it.  time_missing=False keeps the current plan when the cache has
        none.  self.plan_source tells which happened ("stored", "timed" or "default")."""
        import json
        key, known = None, {}
        self.plan_source = "timed"
        if cache is not None:
            key = self.plan_key() + ":" + self.device_key()
            try:
                with open(cache) as f:
                    known = json.load(f)
            except (OSError, ValueError):
                known = {}
            if key in known:
                self.set_tuning(known[key], stream)
                self.plan_source = "stored"
                return self.get_tuning()
        if not time_missing:
            self.plan_source = "default"
            return self.get_tuning()
        t = Tuning()
        self._check(lib.gwsym_autotune(self.h, _stream(stream), C.byref(t)))
        plan = t.to_dict()
        if cache is not None and update:
            known[key] = plan
            with open(cache, "w") as f:
                json.dump(known, f, indent=1, sort_keys=True)
        return plan

    def get_tuning(self):
        t = Tuning()
        self._check(lib.gwsym_get_tuning(self.h, C.byref(t)))
        return t.to_dict()

    def set_tuning(self, plan, stream=None):
        t = Tuning.from_dict(plan)
        self._check(lib.gwsym_set_tuning(self.h, C.byref(t), _stream(stream)))

    def profile(self, enable=True):
        self._check(lib.gwsym_profile(self.h, int(enable)))

    def profile_read(self):
        """{class: (ms, launches, complex MACs, algorithmic bytes)} since the previous read."""
        ms = (C.c_double * 8)()
        n = (C.c_int64 * 8)()
        macs = (C.c_double * 8)()
        nbytes = (C.c_double * 8)()
        self._check(lib.gwsym_profile_read(self.h, ms, n, macs, nbytes))
        return {name: (ms[i], n[i], macs[i], nbytes[i]) for i, name in enumerate(PROFILE_CLASSES)}

    def flop_counts(self):
        out = (C.c_double * 2)()
        self._check(lib.gwsym_flop_counts(self.h, out))
        return float(out[0]), float(out[1])
