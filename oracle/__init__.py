"""ctypes binding of the plain CPU oracle (test infrastructure).

THIS IS TEST INFRASTRUCTURE.  Only `tests/`, the smoke check and the bench's
CPU-baseline leg may import it; the product path never does.  It shares no
code with the HIP library and imports nothing from the package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nair_oracle.c")
_LIB = os.path.join(_HERE, "libnair_oracle.so")

STATUS = {0: "OK", 1: "EINVAL", 2: "ESINGULAR", 3: "ENOCONV", 4: "ENUMERIC", 5: "ENOMEM",
          7: "ECOARSEN"}


def build_oracle(out: str = _LIB) -> str:
    """Compile the oracle with gcc (one thread, no implicit fma contraction)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class _Params(C.Structure):
    _fields_ = [("degree", C.c_int32), ("theta", C.c_double), ("phi", C.c_double),
                ("drop", C.c_double), ("relax", C.c_int32), ("max_levels", C.c_int32),
                ("max_coarse_dofs", C.c_int32), ("seed", C.c_uint64),
                ("cf_override", C.c_void_p), ("form", C.c_int32), ("cycle", C.c_int32),
                ("gmres", C.c_int32)]


class _LevelView(C.Structure):
    _fields_ = [("nb", C.c_int32), ("bs", C.c_int32), ("nnzb", C.c_int32), ("coarsest", C.c_int32),
                ("rowptr", C.c_void_p), ("colidx", C.c_void_p), ("vals", C.c_void_p),
                ("dinv", C.c_void_p), ("bnorm", C.c_void_p), ("mask", C.c_void_p),
                ("lam", C.c_void_p), ("cf", C.c_void_p), ("cidx", C.c_void_p),
                ("pmap", C.c_void_p), ("nc", C.c_int32), ("pmis_rounds", C.c_int32),
                ("dround", C.c_void_p), ("z_nnzb", C.c_int32), ("z_rowptr", C.c_void_p), ("z_colidx", C.c_void_p),
                ("z_vals", C.c_void_p), ("dense_n", C.c_int32), ("dense_lu", C.c_void_p),
                ("dense_piv", C.c_void_p), ("margin", C.c_int64 * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle()
        L = C.CDLL(_LIB)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.ora_default_params.argtypes = [C.POINTER(_Params)]
        L.ora_setup.argtypes = [i32, i32, vp, vp, vp, C.POINTER(_Params), C.POINTER(vp)]
        L.ora_setup.restype = C.c_int
        for f in (L.ora_solve, L.ora_solve_T):
            f.argtypes = [vp, vp, vp, dbl, i32, vp, C.POINTER(i32), C.POINTER(dbl)]
            f.restype = C.c_int
        for f in (L.ora_vcycle, L.ora_vcycle_T):
            f.argtypes = [vp, vp, vp]
            f.restype = C.c_int
        L.ora_num_levels.argtypes = [vp]
        L.ora_num_levels.restype = i32
        L.ora_level.argtypes = [vp, i32, C.POINTER(_LevelView)]
        L.ora_level.restype = C.c_int
        L.ora_complexity.argtypes = [vp, C.POINTER(dbl), C.POINTER(dbl)]
        L.ora_block_inverse.argtypes = [i32, vp, vp]
        L.ora_block_inverse.restype = C.c_int
        L.ora_splitmix64.argtypes = [C.c_uint64]
        L.ora_splitmix64.restype = C.c_uint64
        L.ora_free.argtypes = [vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _view(addr, dtype, n):
    if not addr or n == 0:
        return np.zeros(0, dtype=dtype)
    buf = (C.c_byte * (int(n) * np.dtype(dtype).itemsize)).from_address(addr)
    return np.frombuffer(buf, dtype=dtype).copy()


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS.get(code, code)}")
        self.code = code
        self.status = STATUS.get(code, str(code))


@dataclass
class Params:
    degree: int = 1
    theta: float = 0.75
    phi: float = 0.025
    drop: float = 1e-3
    relax: int = 0            # 0 = F, 1 = FC
    max_levels: int = 30
    max_coarse_dofs: int = 128
    seed: int = 0
    cf_override: Optional[np.ndarray] = None
    form: int = 0             # 0 = block nAIR, 1 = scalar nAIR after block-diagonal scaling
    cycle: int = 0            # 0 = V-cycle, 1 = F-cycle
    gmres: int = 0            # 0 = stationary iteration, m > 0 = GMRES(m) preconditioned by the cycle


@dataclass
class Level:
    nb: int
    bs: int
    coarsest: bool
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray
    dinv: Optional[np.ndarray] = None
    bnorm: Optional[np.ndarray] = None
    mask: Optional[np.ndarray] = None
    lam: Optional[np.ndarray] = None
    cf: Optional[np.ndarray] = None
    cidx: Optional[np.ndarray] = None
    pmap: Optional[np.ndarray] = None
    nc: int = 0
    pmis_rounds: int = 0
    dround: Optional[np.ndarray] = None
    z_rowptr: Optional[np.ndarray] = None
    z_colidx: Optional[np.ndarray] = None
    z_vals: Optional[np.ndarray] = None
    dense_lu: Optional[np.ndarray] = None
    dense_piv: Optional[np.ndarray] = None
    # decision-margin audit: comparisons within 1e-12 relative (theta strength,
    # phi strength, one-point choice, drop test of the next coarse operator)
    margin: tuple = (0, 0, 0, 0)


class Hierarchy:
    """Oracle nAIR hierarchy for a block-CSR matrix (host numpy arrays)."""

    def __init__(self, nb, bs, rowptr, colidx, vals, params: Params | None = None):
        params = params or Params()
        L = lib()
        self._rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        self._colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        self._vals = np.ascontiguousarray(vals, dtype=np.float64)
        self.nb, self.bs, self.params = int(nb), int(bs), params
        p = _Params()
        L.ora_default_params(C.byref(p))
        p.degree, p.theta, p.phi, p.drop = params.degree, params.theta, params.phi, params.drop
        p.relax, p.max_levels, p.max_coarse_dofs = params.relax, params.max_levels, params.max_coarse_dofs
        p.seed = params.seed
        p.form = params.form
        p.cycle = params.cycle
        p.gmres = params.gmres
        self._cf = None
        if params.cf_override is not None:
            self._cf = np.ascontiguousarray(params.cf_override, dtype=np.int8)
            p.cf_override = self._cf.ctypes.data
        h = C.c_void_p()
        st = L.ora_setup(self.nb, self.bs, _ptr(self._rowptr), _ptr(self._colidx), _ptr(self._vals),
                         C.byref(p), C.byref(h))
        if st != 0:
            raise OracleError(st, "ora_setup")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().ora_free(h)
            self._h = None

    @property
    def n(self):
        return self.nb * self.bs

    @property
    def num_levels(self) -> int:
        return int(lib().ora_num_levels(self._h))

    def level(self, l: int) -> Level:
        v = _LevelView()
        st = lib().ora_level(self._h, l, C.byref(v))
        if st != 0:
            raise OracleError(st, "ora_level")
        nb, bs, nnzb = v.nb, v.bs, v.nnzb
        bb = bs * bs
        lv = Level(nb=nb, bs=bs, coarsest=bool(v.coarsest),
                   rowptr=_view(v.rowptr, np.int32, nb + 1), colidx=_view(v.colidx, np.int32, nnzb),
                   vals=_view(v.vals, np.float64, nnzb * bb).reshape(nnzb, bs, bs))
        if v.dinv:
            lv.dinv = _view(v.dinv, np.float64, nb * bb).reshape(nb, bs, bs)
            lv.bnorm = _view(v.bnorm, np.float64, nnzb)
            lv.mask = _view(v.mask, np.uint8, nnzb)
            lv.lam = _view(v.lam, np.int32, nb)
            lv.cf = _view(v.cf, np.int8, nb)
            lv.cidx = _view(v.cidx, np.int32, nb)
            lv.dround = _view(v.dround, np.int32, nb)
        if v.pmap:
            lv.pmap = _view(v.pmap, np.int32, nb)
            lv.nc = v.nc
            lv.pmis_rounds = v.pmis_rounds
            lv.z_rowptr = _view(v.z_rowptr, np.int32, v.nc + 1)
            lv.z_colidx = _view(v.z_colidx, np.int32, v.z_nnzb)
            lv.z_vals = _view(v.z_vals, np.float64, v.z_nnzb * bb).reshape(v.z_nnzb, bs, bs)
        lv.margin = tuple(int(m) for m in v.margin)
        if v.dense_lu:
            n = v.dense_n
            lv.dense_lu = _view(v.dense_lu, np.float64, n * n).reshape(n, n)
            lv.dense_piv = _view(v.dense_piv, np.int32, n)
        return lv

    def levels(self):
        return [self.level(l) for l in range(self.num_levels)]

    def _solve(self, fn, b, rtol, max_iter):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        hist = np.zeros(max(1, max_iter))
        it = C.c_int32()
        rel = C.c_double()
        st = fn(self._h, _ptr(b), _ptr(x), rtol, max_iter, _ptr(hist), C.byref(it), C.byref(rel))
        return x, hist[:it.value].copy(), STATUS.get(st, str(st))

    def solve(self, b, rtol=1e-10, max_iter=100):
        """Returns (x, relative-residual history, status string)."""
        return self._solve(lib().ora_solve, b, rtol, max_iter)

    def solve_T(self, g, rtol=1e-10, max_iter=100):
        return self._solve(lib().ora_solve_T, g, rtol, max_iter)

    def vcycle(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        e = np.zeros_like(r)
        lib().ora_vcycle(self._h, _ptr(r), _ptr(e))
        return e

    def vcycle_T(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        y = np.zeros_like(g)
        lib().ora_vcycle_T(self._h, _ptr(g), _ptr(y))
        return y

    def complexity(self):
        oc, cc = C.c_double(), C.c_double()
        lib().ora_complexity(self._h, C.byref(oc), C.byref(cc))
        return oc.value, cc.value


def block_inverse(M: np.ndarray) -> np.ndarray:
    """Inverse of one square block by the oracle's LU recipe."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    out = np.zeros_like(M)
    st = lib().ora_block_inverse(M.shape[0], _ptr(M), _ptr(out))
    if st != 0:
        raise OracleError(st, "ora_block_inverse")
    return out


def splitmix64(x: int) -> int:
    return int(lib().ora_splitmix64(x))


def bsr_to_dense(nb, bs, rowptr, colidx, vals, ncols=None):
    ncols = nb if ncols is None else ncols
    D = np.zeros((nb * bs, ncols * bs))
    for I in range(nb):
        for t in range(rowptr[I], rowptr[I + 1]):
            J = colidx[t]
            D[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = vals[t]
    return D


def rho_stats(hist):
    """Average and last-5 convergence factors of a relative-residual history."""
    hist = np.asarray(hist)
    K = len(hist)
    if K == 0:
        return float("nan"), float("nan")
    avg = hist[-1] ** (1.0 / K)
    last5 = (hist[-1] / hist[-6]) ** 0.2 if K > 5 else avg
    return float(avg), float(last5)


def wpd(cc: float, rho: float) -> float:
    """Work units per digit of accuracy, -CC / log10(rho) (section 6)."""
    return -cc / np.log10(rho)


def adjoint_gradients(H: "Hierarchy", rowptr, colidx, b, xbar, rtol=1e-12, max_iter=200):
    """Gradients of a loss L(x) of the solution x = A^{-1} b by the adjoint method.

    Given xbar = dL/dx, the oracle solves A x = b and the adjoint system
    A^T ybar = xbar (its transposed cycle, section 5), then dL/db = ybar and,
    because dx = -A^{-1} (dA) x, dL/dA_IJ = -ybar_I x_J^T for every stored block
    (I, J) of A.  Returns (x, ybar, grad_vals [nnzb, bs, bs]).
    """
    bs = H.bs
    x, h, st = H.solve(b, rtol, max_iter)
    if st != "OK":
        raise OracleError(3, "adjoint_gradients: forward solve")
    ybar, hT, stT = H.solve_T(xbar, rtol, max_iter)
    if stT != "OK":
        raise OracleError(3, "adjoint_gradients: adjoint solve")
    nb = len(rowptr) - 1
    g = np.zeros((int(rowptr[nb]), bs, bs))
    for I in range(nb):
        for t in range(rowptr[I], rowptr[I + 1]):
            J = colidx[t]
            g[t] = -np.outer(ybar[I * bs:(I + 1) * bs], x[J * bs:(J + 1) * bs])
    return x, ybar, g
