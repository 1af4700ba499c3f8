"""ctypes binding of libnair_hip.so (argument marshalling only).

Every step of the setup and solve runs in the library's HIP kernels; this
module passes torch device tensors' pointers and the current stream through
the C ABI declared in include/nair.h, and fails loudly if the library is
missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnair_hip.so")

STATUS = {0: "OK", 1: "EINVAL", 2: "ESINGULAR", 3: "ENOCONV", 4: "ENUMERIC", 5: "ENOMEM",
          6: "EDEVICE", 7: "ECOARSEN"}

EXPORTED = ["nair_default_params", "nair_setup", "nair_solve", "nair_solve_T", "nair_vcycle",
            "nair_vcycle_T", "nair_history", "nair_info", "nair_get_level", "nair_last_error",
            "nair_destroy", "nair_pool_trim", "nair_timer_select", "nair_timer_read", "nair_grad_vals",
            "nair_setup_batch", "nair_solve_batch", "nair_batch_history", "nair_get_systems",
            "nair_autotune", "nair_solve_noalloc"]

TUNE_KINDS = ("relax", "relax_T", "residual_T", "restrict", "interp_T", "residual")

KERNELS = {"relax": 0, "residual": 1, "restrict": 2, "interp": 3, "spgemm_numeric": 4,
           "spgemm_symbolic": 5, "block_inverse": 6, "galerkin": 7, "dense": 8, "block_product": 9}


class NairError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str = ""):
        self.code = code
        self.status = STATUS.get(code, str(code))
        super().__init__(f"{where}: {self.status}" + (f" ({msg})" if msg else ""))


class _Params(C.Structure):
    _fields_ = [("degree", C.c_int32), ("theta", C.c_double), ("phi", C.c_double),
                ("drop", C.c_double), ("relax", C.c_int32), ("max_levels", C.c_int32),
                ("max_coarse_dofs", C.c_int32), ("seed", C.c_uint64),
                ("cf_override_host", C.c_void_p), ("precision", C.c_int32), ("tuning", C.c_void_p),
                ("form", C.c_int32), ("cycle", C.c_int32), ("gmres", C.c_int32), ("faces", C.c_int32),
                ("sweep_copy", C.c_int32), ("matrix_cores", C.c_int32), ("allocator", C.c_void_p)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


def _torch_allocator(device):
    """nair_allocator callbacks on torch's caching allocator (device memory for
    the library's buffers; torch counts it in memory_allocated).  The returned
    objects must outlive the handle."""
    import torch
    dev = torch.device(device).index or 0

    def alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except Exception:
            return None   # (the library reports NAIR_ENOMEM)

    def free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = _Allocator()
    keep = (_ALLOC_FN(alloc), _FREE_FN(free))
    a.alloc, a.free, a.ctx = keep[0], keep[1], None
    return a, keep


class _Result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("rho_avg", C.c_double), ("rho_last5", C.c_double)]


class _LevelView(C.Structure):
    _fields_ = [("nb", C.c_int32), ("bs", C.c_int32), ("nnzb", C.c_int32), ("coarsest", C.c_int32),
                ("rowptr", C.c_void_p), ("colidx", C.c_void_p), ("vals", C.c_void_p),
                ("dinv", C.c_void_p), ("bnorm", C.c_void_p), ("mask", C.c_void_p),
                ("lam", C.c_void_p), ("cf", C.c_void_p), ("cidx", C.c_void_p),
                ("pmap", C.c_void_p), ("dround", C.c_void_p), ("nc", C.c_int32),
                ("pmis_rounds", C.c_int32), ("z_nnzb", C.c_int32), ("z_rowptr", C.c_void_p),
                ("z_colidx", C.c_void_p), ("z_vals", C.c_void_p), ("dense_n", C.c_int32),
                ("dense_inv", C.c_void_p), ("face_rmax", C.c_int32), ("face_cmax", C.c_int32),
                ("face_meta", C.c_void_p), ("face_vals", C.c_void_p), ("face_dvals", C.c_void_p),
                ("margin", C.c_int32 * 4), ("sweep_nnzb", C.c_int32)]


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or python paper_1704_05001_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.nair_default_params.argtypes = [C.POINTER(_Params)]
        L.nair_default_params.restype = C.c_int
        L.nair_setup.argtypes = [i32, i32, vp, vp, vp, C.POINTER(_Params), vp, C.POINTER(vp)]
        L.nair_setup.restype = C.c_int
        for f in (L.nair_solve, L.nair_solve_T):
            f.argtypes = [vp, vp, vp, dbl, i32, C.POINTER(_Result), vp]
            f.restype = C.c_int
        for f in (L.nair_vcycle, L.nair_vcycle_T):
            f.argtypes = [vp, vp, vp, vp]
            f.restype = C.c_int
        L.nair_history.argtypes = [vp, vp, i32, C.POINTER(i32)]
        L.nair_history.restype = C.c_int
        L.nair_info.argtypes = [vp, C.POINTER(i32), vp, vp, C.POINTER(dbl), C.POINTER(dbl)]
        L.nair_info.restype = C.c_int
        L.nair_get_level.argtypes = [vp, i32, C.POINTER(_LevelView)]
        L.nair_get_level.restype = C.c_int
        L.nair_last_error.argtypes = [vp]
        L.nair_last_error.restype = C.c_char_p
        L.nair_destroy.argtypes = [vp]
        L.nair_destroy.restype = None
        L.nair_pool_trim.argtypes = []
        L.nair_pool_trim.restype = C.c_int
        L.nair_timer_select.argtypes = [i32, i32]
        L.nair_timer_select.restype = C.c_int
        L.nair_timer_read.argtypes = [C.POINTER(C.c_int64), C.POINTER(dbl)]
        L.nair_timer_read.restype = C.c_int
        L.nair_grad_vals.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
        L.nair_grad_vals.restype = C.c_int
        L.nair_setup_batch.argtypes = [i32, vp, i32, vp, vp, vp, C.POINTER(_Params), vp, C.POINTER(vp)]
        L.nair_setup_batch.restype = C.c_int
        L.nair_solve_batch.argtypes = [vp, i32, vp, vp, dbl, i32, i32, vp, vp]
        L.nair_solve_batch.restype = C.c_int
        L.nair_batch_history.argtypes = [vp, i32, vp, i32, C.POINTER(i32)]
        L.nair_batch_history.restype = C.c_int
        L.nair_get_systems.argtypes = [vp, i32, i32, C.POINTER(i32), vp, vp, vp]
        L.nair_get_systems.restype = C.c_int
        L.nair_autotune.argtypes = [vp, i32, vp, vp]
        L.nair_autotune.restype = C.c_int
        L.nair_solve_noalloc.argtypes = [vp, vp, vp, dbl, i32, C.POINTER(_Result), vp]
        L.nair_solve_noalloc.restype = C.c_int
        _lib = L
    return _lib


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check_vector(t, n: int, name: str, device, out: bool = False):
    """Raise ValueError unless t is a contiguous float64 tensor of n entries on
    `device` (the library reads or writes exactly n doubles through its pointer)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must hold {n} entries (nb * bs), got {t.numel()}")
    if t.device != torch.device(device):
        raise ValueError(f"{name} is on {t.device}, the hierarchy on {device}")
    if out and t.requires_grad:
        raise ValueError(f"{name} is written by the library and must not require grad")


def _check_pattern(rowptr, colidx, vals, bs: int):
    """Raise ValueError unless rowptr/colidx are contiguous int32 and vals a
    contiguous float64 [nnzb, bs, bs] tensor on one device, with colidx and
    vals sized by rowptr[-1] (one 4-byte device read)."""
    import torch
    for t, dt, name in ((rowptr, torch.int32, "rowptr"), (colidx, torch.int32, "colidx"),
                        (vals, torch.float64, "vals")):
        if not isinstance(t, torch.Tensor) or t.dtype != dt or not t.is_contiguous():
            raise ValueError("rowptr/colidx must be contiguous int32 and vals float64 tensors "
                             f"({name} is not)")
    if not rowptr.is_cuda or colidx.device != rowptr.device or vals.device != rowptr.device:
        raise ValueError("rowptr, colidx and vals must be on the same HIP device")
    if rowptr.numel() < 1:
        raise ValueError("rowptr must hold nb + 1 >= 1 entries")
    _check_block_sizes(int(rowptr[-1].item()), colidx.numel(), vals.numel(), bs)


def _check_block_sizes(nnzb: int, ncolidx: int, nvals: int, bs: int):
    """colidx must hold nnzb = rowptr[-1] entries and vals nnzb * bs * bs."""
    if int(bs) < 1:
        raise ValueError("bs >= 1 required")
    if ncolidx != nnzb:
        raise ValueError(f"colidx holds {ncolidx} entries, rowptr[-1] = {nnzb}")
    if nvals != nnzb * int(bs) * int(bs):
        raise ValueError(f"vals holds {nvals} entries, nnzb * bs * bs = {nnzb * int(bs) * int(bs)}")


def _dcopy(ptr: int, dtype, count: int, device):
    """Copy `count` elements at device pointer `ptr` into a new torch tensor."""
    import torch
    out = torch.empty(int(count), dtype=dtype, device=device)
    if count > 0 and ptr:
        nbytes = int(count) * out.element_size()
        _hip().hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(ptr), C.c_size_t(nbytes), 3)
    return out


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = C.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip_lib.hipMemcpy.restype = C.c_int
    return _hip_lib


@dataclass
class Params:
    degree: int = 1
    theta: float = 0.75
    phi: float = 0.025
    drop: float = 1e-3
    relax: int = 0
    max_levels: int = 30
    max_coarse_dofs: int = 128
    seed: int = 0
    cf_override: Optional[np.ndarray] = None
    precision: str = "fp64"      # "fp64" or "fp32" (FP32-stored hierarchy, FP64 refinement)
    tuning: Optional[np.ndarray] = None   # [levels, 6] lane groups from Hierarchy.autotune
    form: str = "block"          # "block" or "scalar" (scalar nAIR of D^{-1} A, D the block diagonal)
    cycle: str = "V"             # "V" or "F"
    gmres: int = 0               # 0: stationary iteration; m > 0: GMRES(m) preconditioned by the cycle
    faces: bool = True           # compact copy of the finest operator's face blocks for the cycle
    sweep_copy: str = "auto"     # F rows in F order for the sweeps: "auto" (large levels), "off", "all"
    matrix_cores: bool = True    # setup block products of 9x9/16x16/25x25 blocks on the FP64 matrix cores
    allocator: str = "pool"      # device memory: "pool" (the library's caching pool) or "torch" (torch's caching allocator)


@dataclass
class Result:
    status: str
    iters: int
    converged: bool
    relres: float
    rho_avg: float
    rho_last5: float


class Hierarchy:
    """nAIR hierarchy on the GPU.  rowptr/colidx (int32) and vals (float64,
    [nnzb, bs, bs]) are torch tensors on the current HIP device.  With
    `sys_nb` (block rows per system) the matrix holds independent systems one
    after another and one batched hierarchy is built for all of them."""

    def __init__(self, rowptr, colidx, vals, bs: int, params: Params | None = None, stream=None,
                 sys_nb=None):
        import torch
        params = params or Params()
        if params.allocator not in ("pool", "torch"):
            raise ValueError("allocator must be 'pool' or 'torch'")
        _check_pattern(rowptr, colidx, vals, bs)
        L = lib()
        self.nb = rowptr.numel() - 1
        self.bs = int(bs)
        self.device = rowptr.device
        self.params = params
        p = _Params()
        L.nair_default_params(C.byref(p))
        p.degree, p.theta, p.phi, p.drop = params.degree, params.theta, params.phi, params.drop
        p.relax, p.max_levels, p.max_coarse_dofs = params.relax, params.max_levels, params.max_coarse_dofs
        p.seed = params.seed
        if params.precision not in ("fp64", "fp32"):
            raise ValueError("precision must be 'fp64' or 'fp32'")
        p.precision = 1 if params.precision == "fp32" else 0
        if params.form not in ("block", "scalar"):
            raise ValueError("form must be 'block' or 'scalar'")
        p.form = 1 if params.form == "scalar" else 0
        if params.cycle not in ("V", "F"):
            raise ValueError("cycle must be 'V' or 'F'")
        p.cycle = 1 if params.cycle == "F" else 0
        p.gmres = int(params.gmres)
        p.faces = 1 if params.faces else 0
        if params.sweep_copy not in ("auto", "off", "all"):
            raise ValueError("sweep_copy must be 'auto', 'off' or 'all'")
        p.sweep_copy = {"auto": -1, "off": 0, "all": 1}[params.sweep_copy]
        p.matrix_cores = 1 if params.matrix_cores else 0
        self._alloc_keep = None   # the callbacks stay alive as long as the handle
        if params.allocator == "torch":
            alloc, keep = _torch_allocator(self.device)
            self._alloc_keep = (alloc, keep)
            p.allocator = C.addressof(alloc)
        cf = None
        if params.cf_override is not None:
            cf = np.ascontiguousarray(params.cf_override, dtype=np.int8)
            p.cf_override_host = cf.ctypes.data
        tune = None
        if params.tuning is not None:
            t = np.asarray(params.tuning, dtype=np.int8)
            tune = np.zeros((64, len(TUNE_KINDS)), dtype=np.int8)
            tune[:t.shape[0]] = t
            p.tuning = tune.ctypes.data
        h = C.c_void_p()
        if sys_nb is None:
            self.nsys = 1
            self.sys_nb = np.array([self.nb], dtype=np.int32)
            st = L.nair_setup(self.nb, self.bs, C.c_void_p(rowptr.data_ptr()), C.c_void_p(colidx.data_ptr()),
                              C.c_void_p(vals.data_ptr()), C.byref(p), _stream_ptr(stream), C.byref(h))
            where = "nair_setup"
        else:
            self.sys_nb = np.ascontiguousarray(sys_nb, dtype=np.int32)
            self.nsys = int(self.sys_nb.size)
            if int(self.sys_nb.sum()) != self.nb:
                raise ValueError("sys_nb must add up to the number of block rows")
            st = L.nair_setup_batch(self.nsys, self.sys_nb.ctypes.data_as(C.c_void_p), self.bs,
                                    C.c_void_p(rowptr.data_ptr()), C.c_void_p(colidx.data_ptr()),
                                    C.c_void_p(vals.data_ptr()), C.byref(p), _stream_ptr(stream), C.byref(h))
            where = "nair_setup_batch"
        if st != 0:
            raise NairError(st, where, L.nair_last_error(None).decode())
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().nair_destroy(h)   # (returns its buffers to the allocator, whose callbacks are still held)
        self._h = None
        self._alloc_keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self):
        return self.nb * self.bs

    def _err(self):
        return lib().nair_last_error(self._h).decode()

    def _solve(self, fn, name, b, x, rtol, max_iter, stream, raise_on):
        import torch
        _check_vector(b, self.n, "right-hand side", self.device)
        if x is None:
            x = torch.empty_like(b)
        _check_vector(x, self.n, "solution", self.device, out=True)
        if x.data_ptr() == b.data_ptr():
            raise ValueError("the solution must not share memory with the right-hand side")
        res = _Result()
        st = fn(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(rtol), int(max_iter),
                C.byref(res), _stream_ptr(stream))
        status = STATUS.get(st, str(st))
        if st != 0 and status in raise_on:
            raise NairError(st, name, self._err())
        return x, Result(status, res.iters, bool(res.converged), res.relres, res.rho_avg, res.rho_last5)

    def solve(self, b, x=None, rtol=1e-10, max_iter=200, stream=None,
              raise_on=("EINVAL", "EDEVICE", "ENOMEM")):
        """x = A^{-1} b by nAIR cycles (the stationary iteration, or GMRES(m)
        preconditioned by the cycle when Params.gmres = m > 0).  Returns (x, Result)."""
        return self._solve(lambda *a: lib().nair_solve(*a), "nair_solve", b, x, rtol, max_iter, stream, raise_on)

    def solve_noalloc(self, b, x, rtol=1e-10, max_iter=200, stream=None,
                      raise_on=("EINVAL", "EDEVICE", "ENOMEM")):
        """nair_solve_noalloc: the solve with no allocation in the library (its
        buffers in the library's static device scratch array); the caller passes x.
        Returns (x, Result)."""
        if x is None:
            raise ValueError("solve_noalloc writes into a solution vector the caller passes")
        return self._solve(lambda *a: lib().nair_solve_noalloc(*a), "nair_solve_noalloc", b, x, rtol, max_iter,
                           stream, raise_on)

    def solve_T(self, g, y=None, rtol=1e-10, max_iter=200, stream=None,
                raise_on=("EINVAL", "EDEVICE", "ENOMEM")):
        """y = A^{-T} g by transposed nAIR cycles (GMRES(m) with Params.gmres = m).
        Returns (y, Result)."""
        return self._solve(lambda *a: lib().nair_solve_T(*a), "nair_solve_T", g, y, rtol, max_iter, stream,
                           raise_on)

    def solve_batch(self, b, x=None, rtol=1e-10, max_iter=200, trans=False, graph=True, stream=None,
                    raise_on=("EINVAL", "EDEVICE", "ENOMEM")):
        """Every system to its own relative residual (A x = b, or A^T x = b with
        trans), one graph-captured iteration replayed.  Returns (x, [Result per system])."""
        import torch
        _check_vector(b, self.n, "right-hand side", self.device)
        if x is None:
            x = torch.empty_like(b)
        _check_vector(x, self.n, "solution", self.device, out=True)
        if x.data_ptr() == b.data_ptr():
            raise ValueError("the solution must not share memory with the right-hand side")
        res = (_Result * self.nsys)()
        st = lib().nair_solve_batch(self._h, 1 if trans else 0, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                    float(rtol), int(max_iter), 1 if graph else 0, C.cast(res, C.c_void_p),
                                    _stream_ptr(stream))
        status = STATUS.get(st, str(st))
        if st != 0 and status in raise_on:
            raise NairError(st, "nair_solve_batch", self._err())
        out = []
        for r in res:
            if r.converged:
                s_k = "OK"
            elif r.iters == 0 or not np.isfinite(r.relres):   # non-finite ||b|| or residual
                s_k = "ENUMERIC"
            else:
                s_k = "ENOCONV"
            out.append(Result(s_k, r.iters, bool(r.converged), r.relres, r.rho_avg, r.rho_last5))
        return x, out

    def autotune(self, reps: int = 20, stream=None) -> np.ndarray:
        """Time the lane-group choices of every cycle kernel on every level and
        keep the fastest; returns the [levels, 6] table (0 = default) for
        Params(tuning=...) of later hierarchies of the same structure."""
        table = np.zeros((64, len(TUNE_KINDS)), dtype=np.int8)
        st = lib().nair_autotune(self._h, int(reps), table.ctypes.data_as(C.c_void_p), _stream_ptr(stream))
        if st != 0:
            raise NairError(st, "nair_autotune", self._err())
        return table[:self.num_levels].copy()

    def batch_history(self, sys: int):
        n = C.c_int32()
        st = lib().nair_batch_history(self._h, int(sys), None, 0, C.byref(n))
        if st != 0:
            raise NairError(st, "nair_batch_history", self._err())
        buf = np.zeros(max(1, n.value))
        lib().nair_batch_history(self._h, int(sys), buf.ctypes.data_as(C.c_void_p), n.value, C.byref(n))
        return buf[:n.value].copy()

    def systems(self, l: int) -> dict:
        """Block offsets (seg), modes (0 none left, 1 coarsened, 2 direct) and
        dense-inverse offsets (-1 unless direct) of the systems on level l."""
        ns = self.nsys
        seg = np.zeros(ns + 1, dtype=np.int32)
        mode = np.zeros(ns, dtype=np.int8)
        off = np.zeros(ns, dtype=np.int64)
        n = C.c_int32()
        st = lib().nair_get_systems(self._h, int(l), ns, C.byref(n), seg.ctypes.data_as(C.c_void_p),
                                    mode.ctypes.data_as(C.c_void_p), off.ctypes.data_as(C.c_void_p))
        if st != 0:
            raise NairError(st, "nair_get_systems", self._err())
        return dict(seg=seg, mode=mode, dense_off=off)

    def vcycle(self, r, stream=None):
        import torch
        _check_vector(r, self.n, "residual", self.device)
        e = torch.empty_like(r)
        st = lib().nair_vcycle(self._h, C.c_void_p(r.data_ptr()), C.c_void_p(e.data_ptr()), _stream_ptr(stream))
        if st != 0:
            raise NairError(st, "nair_vcycle", self._err())
        return e

    def vcycle_T(self, g, stream=None):
        import torch
        _check_vector(g, self.n, "right-hand side", self.device)
        y = torch.empty_like(g)
        st = lib().nair_vcycle_T(self._h, C.c_void_p(g.data_ptr()), C.c_void_p(y.data_ptr()), _stream_ptr(stream))
        if st != 0:
            raise NairError(st, "nair_vcycle_T", self._err())
        return y

    def history(self):
        n = C.c_int32()
        lib().nair_history(self._h, None, 0, C.byref(n))
        buf = np.zeros(max(1, n.value))
        lib().nair_history(self._h, buf.ctypes.data_as(C.c_void_p), n.value, C.byref(n))
        return buf[:n.value].copy()

    def info(self):
        lv = C.c_int32()
        nbl = np.zeros(64, dtype=np.int32)
        nnz = np.zeros(64, dtype=np.int64)
        oc, cc = C.c_double(), C.c_double()
        st = lib().nair_info(self._h, C.byref(lv), nbl.ctypes.data_as(C.c_void_p), nnz.ctypes.data_as(C.c_void_p),
                             C.byref(oc), C.byref(cc))
        if st != 0:
            raise NairError(st, "nair_info", self._err())
        L = lv.value
        return dict(levels=L, nb=nbl[:L].tolist(), nnzb=nnz[:L].tolist(), oc=oc.value, cc=cc.value)

    @property
    def num_levels(self):
        return self.info()["levels"]

    def level(self, l: int, fields=None) -> dict:
        """Copies of level l's device arrays (torch tensors on the device);
        `fields` (names) restricts which arrays are copied."""
        import torch
        v = _LevelView()
        st = lib().nair_get_level(self._h, l, C.byref(v))
        if st != 0:
            raise NairError(st, "nair_get_level", self._err())
        torch.cuda.synchronize(self.device)
        dev = self.device
        nb, bs, nnzb = v.nb, v.bs, v.nnzb
        bb = bs * bs
        want = (lambda k: True) if fields is None else (lambda k: k in fields)
        out = dict(nb=nb, bs=bs, nnzb=nnzb, coarsest=bool(v.coarsest), nc=v.nc, pmis_rounds=v.pmis_rounds,
                   face_rmax=v.face_rmax, face_cmax=v.face_cmax, margin=tuple(int(m) for m in v.margin),
                   sweep_nnzb=v.sweep_nnzb)
        spec = [("rowptr", v.rowptr, torch.int32, nb + 1, None),
                ("colidx", v.colidx, torch.int32, nnzb, None),
                ("vals", v.vals, torch.float64, nnzb * bb, (nnzb, bs, bs))]
        if v.dinv:
            spec += [("dinv", v.dinv, torch.float64, nb * bb, (nb, bs, bs)),
                     ("bnorm", v.bnorm, torch.float64, nnzb, None),
                     ("mask", v.mask, torch.uint8, nnzb, None),
                     ("lam", v.lam, torch.int32, nb, None),
                     ("cf", v.cf, torch.int8, nb, None),
                     ("cidx", v.cidx, torch.int32, nb, None),
                     ("dround", v.dround, torch.int32, nb, None)]
        if v.pmap:
            spec += [("pmap", v.pmap, torch.int32, nb, None),
                     ("z_rowptr", v.z_rowptr, torch.int32, v.nc + 1, None),
                     ("z_colidx", v.z_colidx, torch.int32, v.z_nnzb, None),
                     ("z_vals", v.z_vals, torch.float64, v.z_nnzb * bb, (v.z_nnzb, bs, bs))]
        if v.dense_inv and v.dense_n > 0:
            n = v.dense_n
            spec += [("dense_inv", v.dense_inv, torch.float64, n * n, (n, n))]
        elif v.dense_inv:   # several systems solved directly on this level: packed inverses
            sy = self.systems(l)
            d = [(int(o), int(sy["seg"][k + 1] - sy["seg"][k]) * bs) for k, o in enumerate(sy["dense_off"]) if o >= 0]
            total = max(o + m * m for o, m in d)
            spec += [("dense_inv", v.dense_inv, torch.float64, total, None)]
        if v.face_meta:   # meta as int64 bit patterns: rows in bits 0..31, columns in 32..63
            rc = v.face_rmax * v.face_cmax
            spec += [("face_meta", v.face_meta, torch.int64, nnzb, None),
                     ("face_vals", v.face_vals, torch.float64, nnzb * max(rc, 1),
                      (nnzb, v.face_rmax, v.face_cmax) if rc > 0 else None),
                     ("face_dvals", v.face_dvals, torch.float64, nb * bb, (nb, bs, bs))]
        for name, ptr, dt, cnt, shape in spec:
            if want(name):
                t = _dcopy(ptr, dt, cnt, dev)
                out[name] = t.view(*shape) if shape else t
        torch.cuda.synchronize(self.device)
        return out


# NAIR_NOALLOC_SCRATCH_BYTES: the per-device scratch array of nair_solve_noalloc
NOALLOC_SCRATCH_BYTES = 4 * 1024 * 1024


def pool_trim():
    st = lib().nair_pool_trim()
    if st != 0:
        raise NairError(st, "nair_pool_trim")


def timer_select(kernel, level=-1):
    """Time every later launch of `kernel` (name or id; None = off) on `level` (-1 = all)."""
    kid = -1 if kernel is None else (KERNELS[kernel] if isinstance(kernel, str) else int(kernel))
    st = lib().nair_timer_select(kid, level)
    if st != 0:
        raise NairError(st, "nair_timer_select")


def timer_read():
    """(number of timed launches, total milliseconds) since the last read."""
    n = C.c_int64()
    ms = C.c_double()
    st = lib().nair_timer_read(C.byref(n), C.byref(ms))
    if st != 0:
        raise NairError(st, "nair_timer_read")
    return n.value, ms.value


def grad_vals(rowptr, colidx, ybar, x, bs: int, stream=None):
    """-ybar_I x_J^T on the block pattern (device tensors), as [nnzb, bs, bs]."""
    import torch
    for t, name in ((rowptr, "rowptr"), (colidx, "colidx")):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous int32 tensor")
    nb = rowptr.numel() - 1
    if nb < 0 or int(bs) < 1:
        raise ValueError("bs >= 1 and rowptr of nb + 1 >= 1 entries required")
    _check_vector(ybar, nb * int(bs), "ybar", rowptr.device)
    _check_vector(x, nb * int(bs), "x", rowptr.device)
    nnzb = colidx.numel()
    if colidx.device != rowptr.device or int(rowptr[-1].item()) != nnzb:
        raise ValueError("colidx must be on rowptr's device and hold rowptr[-1] entries")
    out = torch.empty((nnzb, bs, bs), dtype=torch.float64, device=x.device)
    st = lib().nair_grad_vals(nb, bs, C.c_void_p(rowptr.data_ptr()), C.c_void_p(colidx.data_ptr()),
                              C.c_void_p(ybar.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                              _stream_ptr(stream))
    if st != 0:
        raise NairError(st, "nair_grad_vals", lib().nair_last_error(None).decode())
    return out
