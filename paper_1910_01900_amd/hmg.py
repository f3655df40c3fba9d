"""Thin ctypes binding of libhmg.so (include/hmg.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch provides device memory
(workspaces and vectors) and the current HIP stream.  Importing this module
does not touch the GPU; loading the library fails loudly if it is not built.
"""
import ctypes as C
import os
import re
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hmg.h")

DG, FE = 0, 1
F64, F32 = 0, 1
STATUS = {0: "HMG_OK", 1: "HMG_NOT_CONVERGED", -1: "HMG_ERR_INVALID", -2: "HMG_ERR_UNSUPPORTED",
          -3: "HMG_ERR_HIP", -4: "HMG_ERR_BREAKDOWN", -5: "HMG_ERR_NONFINITE", -6: "HMG_ERR_WORKSPACE"}


class HmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("nel", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("degree", C.c_int32), ("deformed", C.c_int32), ("deform_amp", C.c_double),
                ("deform_waves", C.c_int32), ("bc", C.c_uint8 * 6), ("ip_factor", C.c_double),
                ("tau_scale", C.POINTER(C.c_double)), ("mapping_degree", C.c_int32)]


class LevelInfo(C.Structure):
    _fields_ = [("space", C.c_int32), ("degree", C.c_int32), ("nel", C.c_int32 * 3),
                ("prec", C.c_int32), ("n_dofs", C.c_int64), ("lmax", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("r0", C.c_double), ("rn", C.c_double),
                ("rho", C.c_double), ("n10", C.c_double)]


_lib = None
_P = C.c_void_p


def lib():
    """Load libhmg.so once (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhmg.so is not built: run `python -m paper_1910_01900_amd.build`")
        # One HIP runtime per process: torch's copy of libamdhip64.so.7 is
        # loaded first, and the library's DT_NEEDED entry resolves to it by
        # SONAME (two runtimes in one process do not share the device).
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        sig = {
            "hmg_last_error": (C.c_char_p, []),
            "hmg_version": (C.c_int, []),
            "hmg_level_create": (C.c_int, [C.POINTER(MeshDesc), C.c_int, C.c_int, C.POINTER(_P)]),
            "hmg_level_query": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
            "hmg_level_bind": (C.c_int, [_P, _P, C.c_size_t, _P]),
            "hmg_level_destroy": (None, [_P]),
            "hmg_operator_apply": (C.c_int, [_P, _P, _P, _P]),
            "hmg_operator_apply_noalloc": (C.c_int, [_P, _P, _P, _P]),
            "hmg_residual": (C.c_int, [_P, _P, _P, _P, _P]),
            "hmg_operator_apply_batched": (C.c_int, [_P, C.c_int, _P, _P, C.c_int64, _P]),
            "hmg_residual_batched": (C.c_int, [_P, C.c_int, _P, _P, _P, C.c_int64, _P]),
            "hmg_diagonal": (C.c_int, [_P, _P, _P]),
            "hmg_level_diagonal_host": (C.c_int, [_P, C.POINTER(C.c_double)]),
            "hmg_estimate_lambda_max": (C.c_int, [_P, C.c_int, C.c_uint64, C.POINTER(C.c_double), _P]),
            "hmg_chebyshev_smooth": (C.c_int, [_P, _P, _P, C.c_int, C.c_double, C.c_double, C.c_double,
                                               C.c_int, _P]),
            "hmg_transfer_create": (C.c_int, [_P, _P, C.c_char, C.POINTER(_P)]),
            "hmg_transfer_query": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
            "hmg_transfer_bind": (C.c_int, [_P, _P, C.c_size_t]),
            "hmg_transfer_destroy": (None, [_P]),
            "hmg_prolongate_add": (C.c_int, [_P, _P, _P, _P]),
            "hmg_restrict": (C.c_int, [_P, _P, _P, _P]),
            "hmg_hierarchy_create": (C.c_int, [C.POINTER(MeshDesc), C.c_char_p, C.c_int, C.c_int, C.c_int,
                                               C.c_int, C.c_uint64, C.POINTER(_P)]),
            "hmg_hierarchy_query": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
            "hmg_hierarchy_bind": (C.c_int, [_P, _P, C.c_size_t, _P]),
            "hmg_hierarchy_destroy": (None, [_P]),
            "hmg_hierarchy_levels": (C.c_int, [_P, C.POINTER(C.c_int)]),
            "hmg_hierarchy_level_info": (C.c_int, [_P, C.c_int, C.POINTER(LevelInfo)]),
            "hmg_hierarchy_set_lmax": (C.c_int, [_P, C.c_int, C.c_double]),
            "hmg_vcycle": (C.c_int, [_P, _P, _P, _P]),
            "hmg_hierarchy_set_graph": (C.c_int, [_P, C.c_int]),
            "hmg_pcg_solve": (C.c_int, [_P, _P, _P, C.c_double, C.c_double, C.c_int,
                                        C.POINTER(SolveStats), _P]),
            "hmg_rhs_sine": (C.c_int, [_P, C.c_double, _P, _P]),
            "hmg_hierarchy_set_max_rhs": (C.c_int, [_P, C.c_int]),
            "hmg_vcycle_batched": (C.c_int, [_P, C.c_int, _P, _P, C.c_int64, _P]),
            "hmg_pcg_solve_batched": (C.c_int, [_P, C.c_int, _P, _P, C.c_int64, C.c_double, C.c_double, C.c_int,
                                                C.POINTER(SolveStats), _P]),
            "hmg_net_create": (C.c_int, [C.c_int, C.c_int, C.c_uint64, C.POINTER(_P)]),
            "hmg_net_query": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
            "hmg_net_bind": (C.c_int, [_P, _P, C.c_size_t, _P]),
            "hmg_net_destroy": (None, [_P]),
            "hmg_net_get_params": (C.c_int, [_P, _P, _P]),
            "hmg_net_set_params": (C.c_int, [_P, _P, _P]),
            "hmg_net_forward": (C.c_int, [_P, _P, _P, C.c_int, _P]),
            "hmg_net_gradient": (C.c_int, [_P, _P, _P, C.c_int, _P, _P, _P]),
            "hmg_net_train_step": (C.c_int, [_P, _P, _P, C.c_int, C.c_double, _P, _P]),
            "hmg_hierarchy_set_coarse": (C.c_int, [_P, C.c_int, _P, C.c_double]),
            "hmg_hierarchy_set_flexible": (C.c_int, [_P, C.c_int]),
            "hmg_hierarchy_set_coarse_cg": (C.c_int, [_P, C.c_double, C.c_int]),
            "hmg_hierarchy_coarse_info": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int),
                                                    C.POINTER(C.c_int), C.POINTER(C.c_int),
                                                    C.POINTER(C.c_double)]),
            "hmg_hierarchy_capture": (C.c_int, [_P, _P, C.c_int]),
            "hmg_hierarchy_captured": (C.c_int, [_P, C.POINTER(C.c_int)]),
            "hmg_hierarchy_coarse_solve_batch": (C.c_int, [_P, _P, _P, C.c_int, _P]),
            "hmg_hierarchy_learned_data": (C.c_int, [_P, C.c_int, _P, _P, C.c_int, _P, _P, _P]),
            "hmg_hierarchy_coarse_stats": (C.c_int, [_P, C.POINTER(C.c_int), _P]),
            "hmg_batch_create": (C.c_int, [C.POINTER(_P), C.c_int, C.c_int, C.POINTER(_P)]),
            "hmg_batch_query": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
            "hmg_batch_layout": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
            "hmg_batch_bind": (C.c_int, [_P, _P, C.c_size_t, _P]),
            "hmg_batch_destroy": (None, [_P]),
            "hmg_batch_set_schedule": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int]),
            "hmg_batch_autotune": (C.c_int, [_P, _P, _P, C.c_int, _P, C.POINTER(C.c_double)]),
            "hmg_batch_schedule": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "hmg_batch_unit_info": (C.c_int, [_P, C.c_int] + [C.POINTER(C.c_int)] * 6 +
                                    [C.POINTER(C.c_uint), C.POINTER(C.c_double)]),
            "hmg_batch_apply": (C.c_int, [_P, _P, _P, _P]),
            "hmg_batch_residual": (C.c_int, [_P, _P, _P, _P, _P]),
            "hmg_batch_set_chebyshev": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int, C.c_double,
                                                  C.c_double, _P]),
            "hmg_batch_chebyshev_smooth": (C.c_int, [_P, _P, _P, _P, _P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols():
    """Function names declared in include/hmg.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hmg_[a-z0-9_]+)\s*\(", txt)))


def check(code, allow=(0,)):
    if code in allow:
        return code
    if code > 0:
        return code
    raise HmgError(code, lib().hmg_last_error().decode())


@dataclass
class Mesh:
    """Structured box mesh (hmg_mesh_desc)."""
    nel: tuple
    degree: int
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    deformed: bool = False
    amp: float = 0.0
    waves: int = 1
    bc: tuple = (0, 0, 0, 0, 0, 0)
    ip: float = 1.0
    tau_scale: np.ndarray = field(default=None)
    mapping: int = 3  # 3: cubic interpolant of the deformation (Sec. 5.3); 0: exact

    def desc(self):
        d = MeshDesc()
        for i in range(3):
            d.nel[i] = int(self.nel[i])
            d.lo[i] = float(self.lo[i])
            d.hi[i] = float(self.hi[i])
        d.degree = int(self.degree)
        d.deformed = 1 if self.deformed else 0
        d.deform_amp = float(self.amp)
        d.deform_waves = int(self.waves)
        for i in range(6):
            d.bc[i] = int(self.bc[i])
        d.ip_factor = float(self.ip)
        if self.tau_scale is not None:
            self._ts = np.ascontiguousarray(self.tau_scale, dtype=np.float64)
            d.tau_scale = self._ts.ctypes.data_as(C.POINTER(C.c_double))
        else:
            d.tau_scale = None
        d.mapping_degree = int(self.mapping)
        return d

    @property
    def n_el(self):
        return int(np.prod(self.nel))


def _torch():
    import torch
    return torch


def stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return C.c_void_p(t.data_ptr())


def vec(t, dtype, n, name="vector"):
    """ptr(t) after checking that t holds at least n values of dtype: the
    kernels read and write n values of the handle's precision and trust the
    pointer, so a shorter or differently typed tensor is refused here,
    before any launch."""
    if t.dtype != dtype:
        raise ValueError("%s: expected %s, got %s" % (name, dtype, t.dtype))
    if t.numel() < n:
        raise ValueError("%s: %d values, need at least %d" % (name, t.numel(), n))
    return ptr(t)


def rows(t, dtype, width, name="vectors"):
    """ptr(t) for a 2-D tensor of rows of at least `width` values of dtype,
    contiguous within each row (row stride = t.stride(0))."""
    if t.dim() != 2:
        raise ValueError("%s: expected a 2-D tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s: expected %s, got %s" % (name, dtype, t.dtype))
    if t.shape[1] < width or t.stride(1) != 1 or t.stride(0) < width:
        raise ValueError("%s: rows of %d contiguous values needed" % (name, width))
    if not t.is_cuda:
        raise ValueError("%s: expected a CUDA tensor" % name)
    return C.c_void_p(t.data_ptr())


def _dtype(prec):
    torch = _torch()
    return torch.float64 if prec == F64 else torch.float32


def _workspace(nbytes):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


class Level:
    """A bound level (hmg_level): create on the host, bind to a torch workspace."""

    def __init__(self, mesh, space=DG, prec=F64):
        self.mesh, self.space, self.prec = mesh, space, prec
        self._h = C.c_void_p()
        desc = mesh.desc()
        check(lib().hmg_level_create(C.byref(desc), space, prec, C.byref(self._h)))
        n, ws = C.c_int64(), C.c_size_t()
        check(lib().hmg_level_query(self._h, C.byref(n), C.byref(ws)))
        self.n_dofs = n.value
        self.ws_bytes = ws.value
        self.ws = _workspace(ws.value)
        check(lib().hmg_level_bind(self._h, ptr(self.ws), ws.value, stream()))
        self.dtype = _dtype(prec)

    def vector(self, values=None):
        torch = _torch()
        if values is None:
            return torch.zeros(self.n_dofs, dtype=self.dtype, device="cuda")
        return torch.as_tensor(np.asarray(values), dtype=self.dtype).to("cuda").contiguous()

    def apply(self, u, v=None):
        v = self.vector() if v is None else v
        n, dt = self.n_dofs, self.dtype
        check(lib().hmg_operator_apply(self._h, vec(u, dt, n, "u"), vec(v, dt, n, "v"), stream()))
        return v

    def apply_noalloc(self, u, v):
        """v = A u through hmg_operator_apply_noalloc (no allocation; the FE
        element-local results in the library's static device buffer)."""
        n, dt = self.n_dofs, self.dtype
        check(lib().hmg_operator_apply_noalloc(self._h, vec(u, dt, n, "u"), vec(v, dt, n, "v"), stream()))
        return v

    def residual(self, b, u, r=None):
        r = self.vector() if r is None else r
        n, dt = self.n_dofs, self.dtype
        check(lib().hmg_residual(self._h, vec(b, dt, n, "b"), vec(u, dt, n, "u"), vec(r, dt, n, "r"), stream()))
        return r

    def vectors(self, nrhs):
        """nrhs zero vectors as rows of one [nrhs, ld] tensor, ld padded to 256 bytes."""
        torch = _torch()
        per = 256 // (8 if self.prec == F64 else 4)
        ld = (self.n_dofs + per - 1) // per * per
        return torch.zeros(nrhs, ld, dtype=self.dtype, device="cuda")

    def apply_batched(self, u, v=None):
        """v[r, :n] = A u[r, :n] for every row of the 2-D tensors u, v."""
        v = self.vectors(u.shape[0]) if v is None else v
        if u.stride(0) != v.stride(0) or u.shape[0] != v.shape[0]:
            raise ValueError("u and v need the same rows and row stride")
        n, dt = self.n_dofs, self.dtype
        check(lib().hmg_operator_apply_batched(self._h, u.shape[0], rows(u, dt, n, "u"), rows(v, dt, n, "v"),
                                               u.stride(0), stream()))
        return v

    def residual_batched(self, b, u, r=None):
        r = self.vectors(u.shape[0]) if r is None else r
        if not (b.stride(0) == u.stride(0) == r.stride(0)) or not (b.shape[0] == u.shape[0] == r.shape[0]):
            raise ValueError("b, u and r need the same rows and row stride")
        n, dt = self.n_dofs, self.dtype
        check(lib().hmg_residual_batched(self._h, u.shape[0], rows(b, dt, n, "b"), rows(u, dt, n, "u"),
                                         rows(r, dt, n, "r"), u.stride(0), stream()))
        return r

    def diagonal(self):
        d = self.vector()
        check(lib().hmg_diagonal(self._h, vec(d, self.dtype, self.n_dofs, "d"), stream()))
        return d

    def lambda_max(self, iters=20, seed=1):
        out = C.c_double()
        check(lib().hmg_estimate_lambda_max(self._h, iters, seed, C.byref(out), stream()))
        return out.value

    def chebyshev(self, b, x, degree, lmax, lo=0.06, hi=1.2, x_is_zero=False):
        n, dt = self.n_dofs, self.dtype
        check(lib().hmg_chebyshev_smooth(self._h, vec(b, dt, n, "b"), vec(x, dt, n, "x"), degree, lmax, lo, hi,
                                         1 if x_is_zero else 0, stream()))
        return x

    def rhs_sine(self, freq):
        b = self.vector()
        check(lib().hmg_rhs_sine(self._h, freq, ptr(b), stream()))
        return b

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.hmg_level_destroy(self._h)
            self._h = C.c_void_p()


class Transfer:
    def __init__(self, fine, coarse, kind):
        self.fine, self.coarse = fine, coarse
        self._h = C.c_void_p()
        check(lib().hmg_transfer_create(fine._h, coarse._h, kind.encode(), C.byref(self._h)))
        ws = C.c_size_t()
        check(lib().hmg_transfer_query(self._h, C.byref(ws)))
        self.ws = _workspace(ws.value)
        check(lib().hmg_transfer_bind(self._h, ptr(self.ws), ws.value))

    def prolongate_add(self, c, f):
        F, Cl = self.fine, self.coarse
        check(lib().hmg_prolongate_add(self._h, vec(c, Cl.dtype, Cl.n_dofs, "coarse"),
                                       vec(f, F.dtype, F.n_dofs, "fine"), stream()))
        return f

    def restrict(self, f, c=None):
        c = self.coarse.vector() if c is None else c
        F, Cl = self.fine, self.coarse
        check(lib().hmg_restrict(self._h, vec(f, F.dtype, F.n_dofs, "fine"),
                                 vec(c, Cl.dtype, Cl.n_dofs, "coarse"), stream()))
        return c

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.hmg_transfer_destroy(self._h)
            self._h = C.c_void_p()


class Batch:
    """Many DG levels (bound Level objects), nrhs vectors each (hmg_batch).

    Vectors are packed: one 1-D tensor of `total` values; vector r of mesh i
    is view(v, i, r) (offset[i] + r * ld[i], n_dofs[i] values).
    """

    def __init__(self, levels, nrhs=1, bind=True):
        self.levels, self.nrhs = list(levels), nrhs
        self._h = C.c_void_p()
        arr = (_P * len(self.levels))(*[L._h for L in self.levels])
        check(lib().hmg_batch_create(arr, len(self.levels), nrhs, C.byref(self._h)))
        n, ws = C.c_int64(), C.c_size_t()
        check(lib().hmg_batch_query(self._h, C.byref(n), C.byref(ws)))
        self.total, self.ws_bytes = n.value, ws.value
        self.offset, self.ld = [], []
        for i in range(len(self.levels)):
            o, l = C.c_int64(), C.c_int64()
            check(lib().hmg_batch_layout(self._h, i, C.byref(o), C.byref(l)))
            self.offset.append(o.value)
            self.ld.append(l.value)
        self.dtype = self.levels[0].dtype
        if bind:
            self.ws = _workspace(ws.value)
            check(lib().hmg_batch_bind(self._h, ptr(self.ws), ws.value, stream()))

    def vector(self):
        return _torch().zeros(self.total, dtype=self.dtype, device="cuda")

    def view(self, v, i, r):
        o = self.offset[i] + r * self.ld[i]
        return v[o:o + self.levels[i].n_dofs]

    def set_schedule(self, single=False, persistent=False, chunks_per_tile=1, blocks_per_cu=1):
        check(lib().hmg_batch_set_schedule(self._h, int(single), int(persistent), chunks_per_tile,
                                           blocks_per_cu))

    def autotune(self, u, v, reps=5):
        ms = C.c_double()
        check(lib().hmg_batch_autotune(self._h, vec(u, self.dtype, self.total, "u"), vec(v, self.dtype, self.total, "v"),
                                       reps, stream(), C.byref(ms)))
        return ms.value

    def schedule(self):
        single, units = C.c_int(), C.c_int()
        check(lib().hmg_batch_schedule(self._h, C.byref(single), C.byref(units)))
        out = []
        for u in range(units.value):
            v = [C.c_int() for _ in range(6)]
            g, ms = C.c_uint(), C.c_double()
            check(lib().hmg_batch_unit_info(self._h, u, *[C.byref(x) for x in v], C.byref(g), C.byref(ms)))
            out.append({"n": v[0].value, "curved": v[1].value, "meshes": v[2].value,
                        "persistent": v[3].value, "chunks_per_tile": v[4].value,
                        "blocks_per_cu": v[5].value, "grid": g.value, "ms": ms.value})
        return {"single": bool(single.value), "units": out}

    def apply(self, u, v=None):
        v = self.vector() if v is None else v
        n, dt = self.total, self.dtype
        check(lib().hmg_batch_apply(self._h, vec(u, dt, n, "u"), vec(v, dt, n, "v"), stream()))
        return v

    def residual(self, b, u, r=None):
        r = self.vector() if r is None else r
        n, dt = self.total, self.dtype
        check(lib().hmg_batch_residual(self._h, vec(b, dt, n, "b"), vec(u, dt, n, "u"), vec(r, dt, n, "r"), stream()))
        return r

    def set_chebyshev(self, lmax, degree, lo=0.06, hi=1.2):
        arr = (C.c_double * len(lmax))(*[float(x) for x in lmax])
        check(lib().hmg_batch_set_chebyshev(self._h, arr, degree, lo, hi, stream()))

    def chebyshev(self, b, x, tmp=None):
        tmp = self.vector() if tmp is None else tmp
        n, dt = self.total, self.dtype
        check(lib().hmg_batch_chebyshev_smooth(self._h, vec(b, dt, n, "b"), vec(x, dt, n, "x"), vec(tmp, dt, n, "tmp"),
                                               stream()))
        return x

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.hmg_batch_destroy(self._h)
            self._h = C.c_void_p()


COARSE_EXACT, COARSE_SMOOTH, COARSE_LEARNED, COARSE_CG = 0, 1, 2, 3


class Net:
    """Learned coarse-grid correction network (hmg_net): U-Net on a grid^3 grid."""

    def __init__(self, grid=16, max_batch=64, seed=1):
        self.grid, self.max_batch = grid, max_batch
        self._h = C.c_void_p()
        check(lib().hmg_net_create(grid, max_batch, seed, C.byref(self._h)))
        n, ws = C.c_int64(), C.c_size_t()
        check(lib().hmg_net_query(self._h, C.byref(n), C.byref(ws)))
        self.n_params, self.ws_bytes = n.value, ws.value
        self.ws = _workspace(ws.value)
        check(lib().hmg_net_bind(self._h, ptr(self.ws), ws.value, stream()))
        torch = _torch()
        self._loss = torch.zeros(32, dtype=torch.float64, device="cuda")

    def _check_batch(self, inp, target=None):
        """Batch size of inp [B, G, G, G, 2] (and target [B, G, G, G]), FP32."""
        torch, G = _torch(), self.grid
        if inp.dtype != torch.float32 or tuple(inp.shape[1:]) != (G, G, G, 2):
            raise ValueError("input: expected float32 [batch, %d, %d, %d, 2]" % (G, G, G))
        B = inp.shape[0]
        if not 1 <= B <= self.max_batch:
            raise ValueError("batch %d outside 1..%d" % (B, self.max_batch))
        if target is not None and (target.dtype != torch.float32 or tuple(target.shape) != (B, G, G, G)):
            raise ValueError("target: expected float32 [%d, %d, %d, %d]" % (B, G, G, G))
        return B

    def params(self):
        t = _torch().empty(self.n_params, dtype=_torch().float32, device="cuda")
        check(lib().hmg_net_get_params(self._h, ptr(t), stream()))
        return t

    def set_params(self, t):
        check(lib().hmg_net_set_params(self._h, vec(t.contiguous(), _torch().float32, self.n_params, "params"),
                                       stream()))

    def forward(self, inp):
        B = self._check_batch(inp)
        out = _torch().empty((B,) + tuple(inp.shape[1:-1]), dtype=_torch().float32, device="cuda")
        check(lib().hmg_net_forward(self._h, ptr(inp), ptr(out), B, stream()))
        return out

    def gradient(self, inp, target):
        B = self._check_batch(inp, target)
        g = _torch().empty(self.n_params, dtype=_torch().float32, device="cuda")
        check(lib().hmg_net_gradient(self._h, ptr(inp), ptr(target), B, ptr(g), ptr(self._loss),
                                     stream()))
        return float(self._loss[0]), g

    def train_step(self, inp, target, lr):
        """One Adam step; returns the loss as a device scalar (no sync)."""
        B = self._check_batch(inp, target)
        check(lib().hmg_net_train_step(self._h, ptr(inp), ptr(target), B, lr, ptr(self._loss),
                                       stream()))
        return self._loss[0]

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.hmg_net_destroy(self._h)
            self._h = C.c_void_p()


class Hierarchy:
    """Hybrid multigrid hierarchy + FP64 PCG (hmg_hierarchy)."""

    def __init__(self, mesh, strategy="cph", pseq=1, h_min=4, smoother_degree=5, mg_prec=F64,
                 lmax_seed=1, graph=False, max_rhs=1):
        self.mesh = mesh
        self._h = C.c_void_p()
        desc = mesh.desc()
        check(lib().hmg_hierarchy_create(C.byref(desc), strategy.encode(), pseq, h_min, smoother_degree,
                                         mg_prec, lmax_seed, C.byref(self._h)))
        self.max_rhs = max_rhs
        if max_rhs != 1:
            check(lib().hmg_hierarchy_set_max_rhs(self._h, max_rhs))
        n, ws = C.c_int64(), C.c_size_t()
        check(lib().hmg_hierarchy_query(self._h, C.byref(n), C.byref(ws)))
        self.n_dofs, self.ws_bytes = n.value, ws.value
        self.ws = _workspace(ws.value)
        check(lib().hmg_hierarchy_bind(self._h, ptr(self.ws), ws.value, stream()))
        self.set_graph(graph)

    def set_graph(self, enable):
        """Replay PCG iterations / V-cycles from recorded HIP graphs (hmg_hierarchy_set_graph)."""
        check(lib().hmg_hierarchy_set_graph(self._h, 1 if enable else 0))

    def levels(self):
        n = C.c_int()
        check(lib().hmg_hierarchy_levels(self._h, C.byref(n)))
        out = []
        for l in range(n.value):
            info = LevelInfo()
            check(lib().hmg_hierarchy_level_info(self._h, l, C.byref(info)))
            out.append({"space": "DG" if info.space == DG else "FE", "degree": info.degree,
                        "nel": tuple(info.nel), "prec": info.prec, "n_dofs": info.n_dofs,
                        "lmax": info.lmax})
        return out

    def set_lmax(self, l, lmax):
        check(lib().hmg_hierarchy_set_lmax(self._h, l, lmax))

    def set_coarse(self, mode, net=None, accept=0.5):
        """Coarsest-level solve: COARSE_EXACT, COARSE_SMOOTH or COARSE_LEARNED (with net)."""
        self._net = net
        check(lib().hmg_hierarchy_set_coarse(self._h, mode, net._h if net is not None else None, accept))

    def set_coarse_cg(self, rtol=1e-3, maxit=50):
        """Tolerance and iteration cap of the iterative (Jacobi-PCG) coarse solve."""
        check(lib().hmg_hierarchy_set_coarse_cg(self._h, rtol, maxit))

    def set_flexible(self, enable):
        check(lib().hmg_hierarchy_set_flexible(self._h, 1 if enable else 0))

    def coarse_info(self):
        n, mx, my, mz, sc = C.c_int64(), C.c_int(), C.c_int(), C.c_int(), C.c_double()
        check(lib().hmg_hierarchy_coarse_info(self._h, C.byref(n), C.byref(mx), C.byref(my), C.byref(mz),
                                              C.byref(sc)))
        return {"n": n.value, "nodes": (mx.value, my.value, mz.value), "scale": sc.value}

    def capture(self, buf):
        """Copy the coarse right-hand side of following V-cycles into rows of buf [cap, n] (FP64)."""
        self._cap = buf
        if buf is not None:
            rows(buf, _torch().float64, self.coarse_info()["n"], "capture buffer")
            if buf.stride(0) != self.coarse_info()["n"]:
                raise ValueError("capture buffer: rows of exactly n values")
        check(lib().hmg_hierarchy_capture(self._h, ptr(buf) if buf is not None else None,
                                          0 if buf is None else buf.shape[0]))

    def captured(self):
        c = C.c_int()
        check(lib().hmg_hierarchy_captured(self._h, C.byref(c)))
        return c.value

    def coarse_solve_batch(self, R):
        self._coarse_rows(R, "R")
        E = _torch().empty_like(R)
        check(lib().hmg_hierarchy_coarse_solve_batch(self._h, ptr(R), ptr(E), R.shape[0], stream()))
        return E

    def learned_data(self, grid, R, E=None):
        """Network inputs [count, grid, grid, grid, 2] (and targets) of coarse vectors R (and E)."""
        torch = _torch()
        self._coarse_rows(R, "R")
        if E is not None:
            self._coarse_rows(E, "E")
            if E.shape[0] != R.shape[0]:
                raise ValueError("R and E need the same number of rows")
        cnt = R.shape[0]
        inp = torch.empty((cnt, grid, grid, grid, 2), dtype=torch.float32, device="cuda")
        tgt = torch.empty((cnt, grid, grid, grid), dtype=torch.float32, device="cuda") if E is not None else None
        for a in range(0, cnt, 1024):
            b = min(cnt, a + 1024)
            check(lib().hmg_hierarchy_learned_data(self._h, grid, ptr(R[a:b]), ptr(E[a:b]) if E is not None else None,
                                                   b - a, ptr(inp[a:b]), ptr(tgt[a:b]) if tgt is not None else None,
                                                   stream()))
        return inp, tgt

    def _coarse_rows(self, t, name):
        """t: [count, n] FP64 coarse vectors, rows of exactly n values."""
        n = self.coarse_info()["n"]
        if t.dim() != 2 or t.dtype != _torch().float64 or t.shape[1] != n or not t.is_contiguous():
            raise ValueError("%s: expected a contiguous float64 [count, %d] tensor" % (name, n))

    def coarse_stats(self):
        f = C.c_int()
        check(lib().hmg_hierarchy_coarse_stats(self._h, C.byref(f), stream()))
        return f.value

    def vcycle(self, b, x=None):
        torch = _torch()
        x = torch.zeros_like(b) if x is None else x
        n, dt = self.n_dofs, torch.float64
        check(lib().hmg_vcycle(self._h, vec(b, dt, n, "b"), vec(x, dt, n, "x"), stream()))
        return x

    def solve(self, b, x=None, rtol=1e-10, atol=0.0, maxit=200, allow_not_converged=False):
        torch = _torch()
        x = torch.zeros_like(b) if x is None else x
        st = SolveStats()
        n, dt = self.n_dofs, torch.float64
        code = lib().hmg_pcg_solve(self._h, vec(b, dt, n, "b"), vec(x, dt, n, "x"), rtol, atol, maxit, C.byref(st),
                                   stream())
        check(code, allow=(0, 1) if allow_not_converged else (0,))
        return x, {"iters": st.iters, "r0": st.r0, "rn": st.rn, "rho": st.rho, "n10": st.n10,
                   "status": STATUS.get(code, code)}

    def vectors(self, nrhs):
        """nrhs zero FP64 vectors as rows of one [nrhs, ld] tensor, ld padded to 256 bytes."""
        torch = _torch()
        ld = (self.n_dofs + 31) // 32 * 32
        return torch.zeros(nrhs, ld, dtype=torch.float64, device="cuda")

    def vcycle_batched(self, B, X=None):
        """X[q] = M^{-1} B[q] for every row (2-D tensors of FP64 rows)."""
        X = self.vectors(B.shape[0]) if X is None else X
        if B.shape[0] != X.shape[0] or B.stride(0) != X.stride(0):
            raise ValueError("B and X need the same rows and row stride")
        n, dt = self.n_dofs, _torch().float64
        check(lib().hmg_vcycle_batched(self._h, B.shape[0], rows(B, dt, n, "B"), rows(X, dt, n, "X"), B.stride(0),
                                       stream()))
        return X

    def solve_batched(self, B, X=None, rtol=1e-10, atol=0.0, maxit=200, allow_not_converged=False):
        """PCG on every row of B at once (hmg_pcg_solve_batched); X holds the
        start vectors (zeros if None).  Returns X and a list of stats."""
        X = self.vectors(B.shape[0]) if X is None else X
        if B.shape[0] != X.shape[0] or B.stride(0) != X.stride(0):
            raise ValueError("B and X need the same rows and row stride")
        nrhs = B.shape[0]
        st = (SolveStats * nrhs)()
        n, dt = self.n_dofs, _torch().float64
        code = lib().hmg_pcg_solve_batched(self._h, nrhs, rows(B, dt, n, "B"), rows(X, dt, n, "X"), B.stride(0),
                                           rtol, atol, maxit, st, stream())
        check(code, allow=(0, 1) if allow_not_converged else (0,))
        return X, [{"iters": s.iters, "r0": s.r0, "rn": s.rn, "rho": s.rho, "n10": s.n10,
                    "status": STATUS.get(code, code)} for s in st]

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.hmg_hierarchy_destroy(self._h)
            self._h = C.c_void_p()
