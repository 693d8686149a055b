"""ctypes binding of libhfmm.so (include/hfmm.h) with the same entry-point names.

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the method runs in the library's kernels.
There is no fallback: if the library is missing or no GPU is present the
calls raise.

Complex arrays cross the boundary column-major (n x nrhs); the helpers here
accept torch tensors of shape (n,) or (n, nrhs) and transpose as needed.
"""

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfmm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hfmm.h")

HFMM_OK = 0
HFMM_NOT_CONVERGED = 1
HFMM_ERR_ARG = -1
FP64 = 0
FP32 = 1

_STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_HIP", -3: "ERR_OOM", -4: "ERR_STATE",
           -5: "ERR_INTERNAL", -6: "ERR_NUMERIC"}


class HFMMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("rel_res_true", ctypes.c_double), ("rel_res_est", ctypes.c_double),
                ("ms_precond", ctypes.c_double), ("ms_krylov", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_setup", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_vp, _i32, _i64, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "hfmm_last_error": ([], ctypes.c_char_p),
    "hfmm_version": ([], _i32),
    "hfmm_build_tree": ([_vp, _i64, _f64, _f64, _f64, _i32, _vp, ctypes.POINTER(_vp)], _i32),
    "hfmm_tree_info": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                        ctypes.POINTER(_i32)], _i32),
    "hfmm_tree_export": ([_vp, _vp, _vp, _vp], _i32),
    "hfmm_tree_destroy": ([_vp], _i32),
    "hfmm_tree_set_options": ([_vp, _i32, _i32], _i32),
    "hfmm_fmm_apply_dipole": ([_vp, _f64, _i32, _i32, _vp, _vp, _vp, _i32, _vp], _i32),
    "hfmm_tune_cache_save": ([ctypes.c_char_p], _i32),
    "hfmm_tune_cache_load": ([ctypes.c_char_p, ctypes.POINTER(_i32)], _i32),
    "hfmm_tune_cache_size": ([], _i32),
    "hfmm_tune_cache_clear": ([], _i32),
    "hfmm_solver_set_k2_blocks": ([_vp, _vp, _i32, _vp], _i32),
    "hfmm_k2_gradient": ([_i32, _vp, _vp, _i32, _vp, _vp], _i32),
    "hfmm_dirichlet_apply": ([_vp, _vp, _vp, _vp, _i32, _vp], _i32),
    "hfmm_solver_boundary_nodes": ([_vp, _vp, _vp], _i32),
    "hfmm_bicgstab_solve": ([_vp, _vp, _vp, _i32, _f64, ctypes.POINTER(SolveInfo), _vp], _i32),
    "hfmm_fmm_apply": ([_vp, _f64, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
    "hfmm_fmm_apply_noalloc": ([_vp, _f64, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
    "hfmm_fmm_noalloc_capacity": ([], _i64),
    "hfmm_fmm_apply_timed": ([_vp, _f64, _i32, _i32, _vp, _vp, _i32, ctypes.POINTER(ctypes.c_float), _vp], _i32),
    "hfmm_fmm_plan_info": ([_vp, _f64, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                            ctypes.POINTER(_i64)], _i32),
    "hfmm_fd_helmholtz_matvec": ([_i32, _f64, _vp, _f64, _vp, _vp, _i32, _vp], _i32),
    "hfmm_solver_create": ([_i32, _f64, _vp, _f64, _f64, _i32, _i32, _i32, _i32, _vp, ctypes.POINTER(_vp)], _i32),
    "hfmm_solver_set_k2": ([_vp, _vp, _f64, _vp], _i32),
    "hfmm_matched_wavenumber": ([_f64, _f64, ctypes.POINTER(_f64)], _i32),
    "hfmm_precond_apply": ([_vp, _vp, _vp, _i32, _vp], _i32),
    "hfmm_fgmres_solve": ([_vp, _vp, _vp, _i32, _i32, _f64, _i32, ctypes.POINTER(SolveInfo), _vp], _i32),
    "hfmm_fgmres_solve_batched": ([ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i32, _i32,
                                   _f64, _i32, ctypes.POINTER(SolveInfo), _vp], _i32),
    "hfmm_tree_set_m2l_input_rounding": ([_vp, _i32], _i32),
    "hfmm_solver_set_m2l_input_rounding": ([_vp, _i32], _i32),
    "hfmm_solver_info": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_f64), ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
                         _i32),
    "hfmm_solver_destroy": ([_vp], _i32),
    "hfmm3_build_tree": ([_vp, _i64, _f64, _f64, _f64, _f64, _i32, _vp, ctypes.POINTER(_vp)], _i32),
    "hfmm3_tree_info": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                         ctypes.POINTER(_i32)], _i32),
    "hfmm3_tree_destroy": ([_vp], _i32),
    "hfmm3_fmm_apply": ([_vp, _f64, _i32, _i32, _vp, _vp, _vp], _i32),
    "hfmm3_fmm_apply_timed": ([_vp, _f64, _i32, _i32, _vp, _vp, ctypes.POINTER(ctypes.c_float), _vp], _i32),
    "hfmm3_fmm_orders": ([_vp, _f64, _i32, ctypes.POINTER(_i32)], _i32),
    "hfmm3_fd_matvec": ([_i32, _f64, _vp, _vp, _vp], _i32),
    "hfmm3_solver_create": ([_i32, _f64, _i32, _i32, _i32, _vp, ctypes.POINTER(_vp)], _i32),
    "hfmm3_precond_apply": ([_vp, _vp, _vp, _vp], _i32),
    "hfmm3_fgmres_solve": ([_vp, _vp, _vp, _i32, _i32, _f64, ctypes.POINTER(SolveInfo), _vp], _i32),
    "hfmm3_solver_info": ([_vp, ctypes.POINTER(_f64), ctypes.POINTER(_i32), ctypes.POINTER(_f64)], _i32),
    "hfmm3_solver_destroy": ([_vp], _i32),
}


def lib():
    """Load libhfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def header_functions():
    """Entry-point names declared in include/hfmm.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hfmm3?_[a-z0-9_]+)\s*\(", text)))


def _check(status, allow_not_converged=False):
    if status == HFMM_OK or (allow_not_converged and status == HFMM_NOT_CONVERGED):
        return status
    raise HFMMError(status, lib().hfmm_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require_cuda(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")


def _colmajor(x, dtype, name):
    """(n,) or (n, nrhs) tensor -> contiguous (nrhs, n) tensor (column-major n x nrhs)."""
    _require_cuda(x, dtype, name)
    if x.dim() == 1:
        return x.contiguous().view(1, -1), True
    return x.t().contiguous(), False


def _from_colmajor(y, squeeze):
    return y.view(-1) if squeeze else y.t()


# ---------------------------------------------------------------------- tree
class Tree:
    """Uniform quad-tree over points xy (n, 2) float64 on the device."""

    def __init__(self, xy, x0=0.0, y0=0.0, side=1.0, leaf_size=64, stream=None):
        _require_cuda(xy, torch.float64, "xy")
        xy = xy.contiguous()
        h = ctypes.c_void_p()
        _check(lib().hfmm_build_tree(_ptr(xy), xy.shape[0], x0, y0, side, leaf_size, _stream(stream),
                                     ctypes.byref(h)))
        self.handle = h
        self.n = xy.shape[0]
        self.device = xy.device

    def info(self):
        L, n, nl, mx = _i32(), _i64(), _i64(), _i32()
        _check(lib().hfmm_tree_info(self.handle, ctypes.byref(L), ctypes.byref(n), ctypes.byref(nl), ctypes.byref(mx)))
        return {"levels": L.value, "n_points": n.value, "n_leaves": nl.value, "max_leaf_count": mx.value}

    def set_options(self, m2l_valu=False, autotune=True):
        """Options of the plans made from now on (cached plans are dropped)."""
        _check(lib().hfmm_tree_set_options(self.handle, int(m2l_valu), int(autotune)))

    def set_m2l_input_rounding(self, mode="none"):
        """Accuracy experiment: M2L operands rounded to "fp16" or "bf16" ("none": off)."""
        _check(lib().hfmm_tree_set_m2l_input_rounding(self.handle, ROUNDING[mode]))

    def export(self, stream=None):
        inf = self.info()
        perm = torch.empty(self.n, dtype=torch.int32, device=self.device)
        off = torch.empty(inf["n_leaves"] + 1, dtype=torch.int32, device=self.device)
        _check(lib().hfmm_tree_export(self.handle, _ptr(perm), _ptr(off), _stream(stream)))
        return perm, off

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.hfmm_tree_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def hfmm_build_tree(xy, x0=0.0, y0=0.0, side=1.0, leaf_size=64, stream=None):
    return Tree(xy, x0, y0, side, leaf_size, stream)


def hfmm_fmm_apply(tree, k, p, q, prec=FP64, stream=None):
    """phi = sum_{j != i} q_j (i/4) H0(k |x_i - x_j|); q is (n,) or (n, nrhs) complex."""
    dtype = torch.complex128 if prec == FP64 else torch.complex64
    qc, squeeze = _colmajor(q, dtype, "q")
    if qc.shape[1] != tree.n:
        raise ValueError("q has the wrong number of points")
    phi = torch.empty_like(qc)
    _check(lib().hfmm_fmm_apply(tree.handle, float(k), int(p), int(prec), _ptr(qc), _ptr(phi), qc.shape[0],
                                _stream(stream)))
    return _from_colmajor(phi, squeeze)


def hfmm_fmm_apply_dipole(tree, k, p, q, normals, prec=FP64, stream=None):
    """phi_i = sum_{j: r_ij > 0} q_j dG/dn_j(x_i, x_j) (double layer); normals (n, 2) float64 unit vectors."""
    dtype = torch.complex128 if prec == FP64 else torch.complex64
    qc, squeeze = _colmajor(q, dtype, "q")
    if qc.shape[1] != tree.n:
        raise ValueError("q has the wrong number of points")
    _require_cuda(normals, torch.float64, "normals")
    if tuple(normals.shape) != (tree.n, 2):
        raise ValueError("normals must be (n, 2)")
    nrm = normals.contiguous()
    phi = torch.empty_like(qc)
    _check(lib().hfmm_fmm_apply_dipole(tree.handle, float(k), int(p), int(prec), _ptr(qc), _ptr(nrm), _ptr(phi),
                                       qc.shape[0], _stream(stream)))
    return _from_colmajor(phi, squeeze)


def hfmm_tune_cache_save(path):
    _check(lib().hfmm_tune_cache_save(os.fsencode(path)))


def hfmm_tune_cache_load(path):
    n = _i32()
    _check(lib().hfmm_tune_cache_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def hfmm_tune_cache_size():
    return lib().hfmm_tune_cache_size()


def hfmm_tune_cache_clear():
    _check(lib().hfmm_tune_cache_clear())


def hfmm_k2_gradient(n, u, mu, nb, stream=None):
    """Block sums of Re(conj(mu) u) over nb x nb blocks (nb = n: per node); u, mu (n*n,) complex128."""
    _require_cuda(u, torch.complex128, "u")
    _require_cuda(mu, torch.complex128, "mu")
    if u.numel() != n * n or mu.numel() != n * n:
        raise ValueError("u and mu must have n*n entries")
    uc, mc = u.contiguous(), mu.contiguous()
    grad = torch.empty(nb * nb, dtype=torch.float64, device=u.device)
    _check(lib().hfmm_k2_gradient(int(n), _ptr(uc), _ptr(mc), int(nb), _ptr(grad), _stream(stream)))
    return grad.view(nb, nb)


def hfmm_fmm_apply_noalloc(tree, k, p, q, prec=FP64, phi=None, stream=None):
    """hfmm_fmm_apply with no device allocation in the library (its fixed work
    array); the plan of (k, p, prec) must exist.  phi (column-major layout as
    returned by a previous call, or None) receives the result."""
    dtype = torch.complex128 if prec == FP64 else torch.complex64
    qc, squeeze = _colmajor(q, dtype, "q")
    if qc.shape[1] != tree.n:
        raise ValueError("q has the wrong number of points")
    out = torch.empty_like(qc) if phi is None else phi
    _check(lib().hfmm_fmm_apply_noalloc(tree.handle, float(k), int(p), int(prec), _ptr(qc), _ptr(out), qc.shape[0],
                                        _stream(stream)))
    return _from_colmajor(out, squeeze)


def hfmm_fmm_noalloc_capacity():
    return lib().hfmm_fmm_noalloc_capacity()


# modes of the M2L input-rounding experiment
ROUNDING = {"none": 0, "fp16": 1, "bf16": 2}

# stage names of hfmm_fmm_apply_timed (the order of its ms_stages); on a tree
# of depth >= 2 "far_chain" (M2M + M2L + L2L + L2P) runs on the tree's second
# stream beside "p2p", "combine" adds the two (and waits for the chain), and
# "m2m", "m2l", "l2l_l2p" are the chain's parts
STAGES = ("gather", "p2m", "far_chain", "combine", "p2p", "scatter", "m2m", "m2l", "l2l_l2p")


def hfmm_fmm_apply_timed(tree, k, p, q, prec=FP64, stream=None):
    """The FMM apply with per-stage device times; returns (phi, {stage: ms})."""
    dtype = torch.complex128 if prec == FP64 else torch.complex64
    qc, squeeze = _colmajor(q, dtype, "q")
    phi = torch.empty_like(qc)
    ms = (ctypes.c_float * len(STAGES))()
    _check(lib().hfmm_fmm_apply_timed(tree.handle, float(k), int(p), int(prec), _ptr(qc), _ptr(phi), qc.shape[0], ms,
                                      _stream(stream)))
    return _from_colmajor(phi, squeeze), dict(zip(STAGES, list(ms)))


def hfmm_fmm_plan_info(tree, k, p, prec=FP64):
    L = tree.info()["levels"]
    orders = (_i32 * (L + 1))()
    deg, g, pairs = _i32(), _i32(), _i64()
    _check(lib().hfmm_fmm_plan_info(tree.handle, float(k), int(p), int(prec), orders, ctypes.byref(deg),
                                    ctypes.byref(g), ctypes.byref(pairs)))
    return {"orders": list(orders), "near_deg": deg.value, "lanes_per_target": g.value, "pairs": pairs.value}


# ---------------------------------------------------------------------- 3-D
STAGES3 = ("upward", "m2l", "l2l", "p2p", "l2p", "total")


class Tree3:
    """Uniform oct-tree over points xyz (n, 3) float64 on the device."""

    def __init__(self, xyz, x0=0.0, y0=0.0, z0=0.0, side=1.0, leaf_size=64, stream=None):
        _require_cuda(xyz, torch.float64, "xyz")
        xyz = xyz.contiguous()
        h = ctypes.c_void_p()
        _check(lib().hfmm3_build_tree(_ptr(xyz), xyz.shape[0], x0, y0, z0, side, leaf_size, _stream(stream),
                                      ctypes.byref(h)))
        self.handle = h
        self.n = xyz.shape[0]
        self.device = xyz.device

    def info(self):
        L, n, nl, mx = _i32(), _i64(), _i64(), _i32()
        _check(lib().hfmm3_tree_info(self.handle, ctypes.byref(L), ctypes.byref(n), ctypes.byref(nl),
                                     ctypes.byref(mx)))
        return {"levels": L.value, "n_points": n.value, "n_leaves": nl.value, "max_leaf_count": mx.value}

    def orders(self, k, p):
        L = self.info()["levels"]
        o = (_i32 * (L + 1))()
        _check(lib().hfmm3_fmm_orders(self.handle, float(k), int(p), o))
        return list(o)

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.hfmm3_tree_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def hfmm3_build_tree(xyz, x0=0.0, y0=0.0, z0=0.0, side=1.0, leaf_size=64, stream=None):
    return Tree3(xyz, x0, y0, z0, side, leaf_size, stream)


def _q3(tree, q, prec):
    dtype = torch.complex128 if prec == FP64 else torch.complex64
    _require_cuda(q, dtype, "q")
    if q.dim() != 1 or q.shape[0] != tree.n:
        raise ValueError("q must be a vector with one charge per point")
    return q.contiguous()


def hfmm3_fmm_apply(tree, k, p, q, prec=FP64, stream=None):
    """phi_i = sum_{j != i} q_j exp(i k r_ij) / (4 pi r_ij) by the oct-tree FMM."""
    qc = _q3(tree, q, prec)
    phi = torch.empty_like(qc)
    _check(lib().hfmm3_fmm_apply(tree.handle, float(k), int(p), int(prec), _ptr(qc), _ptr(phi), _stream(stream)))
    return phi


def hfmm3_fmm_apply_timed(tree, k, p, q, prec=FP64, stream=None):
    """The 3-D apply with per-stage device times; returns (phi, {stage: ms})."""
    qc = _q3(tree, q, prec)
    phi = torch.empty_like(qc)
    ms = (ctypes.c_float * len(STAGES3))()
    _check(lib().hfmm3_fmm_apply_timed(tree.handle, float(k), int(p), int(prec), _ptr(qc), _ptr(phi), ms,
                                       _stream(stream)))
    return phi, dict(zip(STAGES3, list(ms)))


def hfmm3_fd_matvec(n, k2, x, stream=None):
    """y = (-Laplace_h - k^2) x on the n^3 interior nodes of the unit cube (complex128)."""
    _require_cuda(x, torch.complex128, "x")
    if x.dim() != 1 or x.shape[0] != n ** 3:
        raise ValueError("x must hold n^3 values")
    x = x.contiguous()
    y = torch.empty_like(x)
    _check(lib().hfmm3_fd_matvec(int(n), float(k2), _ptr(x), _ptr(y), _stream(stream)))
    return y


class Solver3:
    """The 3-D model problem with the oct-tree FMM volume-potential preconditioner."""

    def __init__(self, n, k, p=6, leaf_size=64, prec=FP64, stream=None):
        h = ctypes.c_void_p()
        _check(lib().hfmm3_solver_create(int(n), float(k), int(p), int(leaf_size), int(prec), _stream(stream),
                                         ctypes.byref(h)))
        self.handle = h
        self.n = n
        self.N = n ** 3

    def _vec(self, v, name):
        _require_cuda(v, torch.complex128, name)
        if v.dim() != 1 or v.shape[0] != self.N:
            raise ValueError(f"{name} must hold n^3 values")
        return v.contiguous()

    def precond_apply(self, r, stream=None):
        r = self._vec(r, "r")
        z = torch.empty_like(r)
        _check(lib().hfmm3_precond_apply(self.handle, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def solve(self, b, x0=None, restart=50, maxit=2000, rtol=1e-6, stream=None, strict=False):
        b = self._vec(b, "b")
        x = torch.zeros_like(b) if x0 is None else self._vec(x0, "x0").clone()
        info = SolveInfo()
        st = lib().hfmm3_fgmres_solve(self.handle, _ptr(b), _ptr(x), int(restart), int(maxit), float(rtol),
                                      ctypes.byref(info), _stream(stream))
        _check(st, allow_not_converged=not strict)
        return x, info.as_dict()

    def info(self):
        c = (_f64 * 2)()
        L, ms = _i32(), _f64()
        _check(lib().hfmm3_solver_info(self.handle, c, ctypes.byref(L), ctypes.byref(ms)))
        return {"self_term": complex(c[0], c[1]), "levels": L.value, "ms_setup": ms.value}

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.hfmm3_solver_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def hfmm_fd_helmholtz_matvec(n, h, x, k2=None, k2_const=0.0, stream=None):
    """y = A x for the 5-point operator; x is (n*n,) or (n*n, nrhs) complex128."""
    xc, squeeze = _colmajor(x, torch.complex128, "x")
    if xc.shape[1] != n * n:
        raise ValueError("x has the wrong length")
    if k2 is not None:
        _require_cuda(k2, torch.float64, "k2")
        k2 = k2.contiguous()
    y = torch.empty_like(xc)
    _check(lib().hfmm_fd_helmholtz_matvec(n, h, _ptr(k2), float(k2_const), _ptr(xc), _ptr(y), xc.shape[0],
                                          _stream(stream)))
    return _from_colmajor(y, squeeze)


# ---------------------------------------------------------------------- solver
class Solver:
    """FMM-BEM preconditioned FGMRES for the n x n FD Helmholtz system (h = 1/(n+1))."""

    def __init__(self, n, k0, k2=None, k2_const=None, p=6, leaf_size=32, prec=FP64, nrhs=1, device="cuda",
                 stream=None):
        self.n, self.nrhs, self.prec, self.k0, self.p = n, nrhs, prec, k0, p
        self.h = 1.0 / (n + 1)
        self.device = torch.device(device)
        if k2 is not None:
            _require_cuda(k2, torch.float64, "k2")
            k2 = k2.contiguous()
        kc = float(k0 * k0 if k2_const is None else k2_const)
        hdl = ctypes.c_void_p()
        _check(lib().hfmm_solver_create(n, self.h, _ptr(k2), kc, float(k0), int(p), int(leaf_size), int(prec),
                                        int(nrhs), _stream(stream), ctypes.byref(hdl)))
        self.handle = hdl

    def set_k2(self, k2=None, k2_const=0.0, stream=None):
        if k2 is not None:
            _require_cuda(k2, torch.float64, "k2")
            k2 = k2.contiguous()
        _check(lib().hfmm_solver_set_k2(self.handle, _ptr(k2), float(k2_const), _stream(stream)))

    def set_k2_blocks(self, kb, stream=None):
        """k^2 constant on square blocks: kb (nb, nb) float64, block rows follow y."""
        _require_cuda(kb, torch.float64, "kb")
        kb = kb.contiguous()
        _check(lib().hfmm_solver_set_k2_blocks(self.handle, _ptr(kb), int(kb.shape[0]), _stream(stream)))

    def boundary_nodes(self, stream=None):
        """(4(n+1), 2) element midpoints in the library's boundary order."""
        xy = torch.empty((4 * (self.n + 1), 2), dtype=torch.float64, device=self.device)
        _check(lib().hfmm_solver_boundary_nodes(self.handle, _ptr(xy), _stream(stream)))
        return xy

    def dirichlet_apply(self, f, g, stream=None):
        """Boundary-element solution with source f (n*n) and Dirichlet data g (4(n+1)) at the midpoints."""
        fc, squeeze = _colmajor(f, torch.complex128, "f")
        gc, _ = _colmajor(g, torch.complex128, "g")
        if fc.shape[1] != self.n * self.n or gc.shape[1] != 4 * (self.n + 1) or gc.shape[0] != fc.shape[0]:
            raise ValueError("f must have n*n rows and g 4(n+1) rows, with the same columns")
        u = torch.empty_like(fc)
        _check(lib().hfmm_dirichlet_apply(self.handle, _ptr(fc), _ptr(gc), _ptr(u), fc.shape[0], _stream(stream)))
        return _from_colmajor(u, squeeze)

    def bicgstab(self, b, x0=None, maxit=5000, rtol=1e-6, stream=None, strict=False):
        bc, squeeze = _colmajor(b, torch.complex128, "b")
        x = torch.zeros_like(bc) if x0 is None else _colmajor(x0, torch.complex128, "x0")[0].clone()
        info = SolveInfo()
        st = lib().hfmm_bicgstab_solve(self.handle, _ptr(bc), _ptr(x), int(maxit), float(rtol), ctypes.byref(info),
                                       _stream(stream))
        _check(st, allow_not_converged=not strict)
        return _from_colmajor(x, squeeze), info.as_dict()

    def precond_apply(self, r, stream=None):
        rc, squeeze = _colmajor(r, torch.complex128, "r")
        z = torch.empty_like(rc)
        _check(lib().hfmm_precond_apply(self.handle, _ptr(rc), _ptr(z), rc.shape[0], _stream(stream)))
        return _from_colmajor(z, squeeze)

    def solve(self, b, x0=None, restart=30, maxit=5000, rtol=1e-6, transpose=False, stream=None, strict=False):
        bc, squeeze = _colmajor(b, torch.complex128, "b")
        x = torch.zeros_like(bc) if x0 is None else _colmajor(x0, torch.complex128, "x0")[0].clone()
        info = SolveInfo()
        st = lib().hfmm_fgmres_solve(self.handle, _ptr(bc), _ptr(x), int(restart), int(maxit), float(rtol),
                                     1 if transpose else 0, ctypes.byref(info), _stream(stream))
        _check(st, allow_not_converged=not strict)
        return _from_colmajor(x, squeeze), info.as_dict()

    def info(self):
        ng, cond, L, leaf = _i32(), _f64(), _i32(), _i32()
        _check(lib().hfmm_solver_info(self.handle, ctypes.byref(ng), ctypes.byref(cond), ctypes.byref(L),
                                      ctypes.byref(leaf)))
        return {"n_gamma": ng.value, "cond_S": cond.value, "levels": L.value, "leaf_size": leaf.value}

    def set_m2l_input_rounding(self, mode="none"):
        """Accuracy experiment: M2L operands rounded to "fp16" or "bf16" ("none": off)."""
        _check(lib().hfmm_solver_set_m2l_input_rounding(self.handle, ROUNDING[mode]))

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.hfmm_solver_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def hfmm_solver_create(n, k0, **kw):
    return Solver(n, k0, **kw)


def hfmm_fgmres_solve(solver, b, **kw):
    return solver.solve(b, **kw)


def hfmm_precond_apply(solver, r, **kw):
    return solver.precond_apply(r, **kw)


def hfmm_matched_wavenumber(k, h):
    """Preconditioner wavenumber matched to the 5-point stencil's dispersion."""
    out = _f64()
    _check(lib().hfmm_matched_wavenumber(float(k), float(h), ctypes.byref(out)))
    return out.value


def hfmm_fgmres_solve_batched(solvers, bs, restart=50, maxit=5000, rtol=1e-6, use_graph=True, stream=None):
    """Solve every (solvers[i], bs[i]) together; returns (list of x, list of info dicts)."""
    m = len(solvers)
    cols = [_colmajor(b, torch.complex128, "b") for b in bs]
    xs = [torch.zeros_like(c) for c, _ in cols]
    hs = (ctypes.c_void_p * m)(*[s.handle.value for s in solvers])
    bp = (ctypes.c_void_p * m)(*[c.data_ptr() for c, _ in cols])
    xp = (ctypes.c_void_p * m)(*[x.data_ptr() for x in xs])
    infos = (SolveInfo * m)()
    st = lib().hfmm_fgmres_solve_batched(hs, m, bp, xp, int(restart), int(maxit), float(rtol), 1 if use_graph else 0,
                                         infos, _stream(stream))
    _check(st, allow_not_converged=True)
    return [_from_colmajor(x, sq) for x, (_, sq) in zip(xs, cols)], [i.as_dict() for i in infos]


def hfmm_last_error():
    return lib().hfmm_last_error().decode()


def hfmm_version():
    return lib().hfmm_version()
