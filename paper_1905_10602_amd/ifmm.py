"""ctypes binding of the C ABI in include/ifmm.h (argument marshalling only).

Host arrays are numpy; device arrays are torch tensors on the GPU (PyTorch is
used for device memory and streams only).  Every entry point maps to one C
call; no step of the method runs in Python.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATUS = {0: "IFMM_OK", -1: "IFMM_EINVAL", -2: "IFMM_ENOMEM", -3: "IFMM_EDEVICE", -4: "IFMM_ESINGULAR",
          -5: "IFMM_ENONFINITE", -6: "IFMM_ESTATE", -7: "IFMM_ENOCONV"}


RANK_FEATURES = 14


class IfmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Options(C.Structure):
    _fields_ = [("leaf_max", C.c_int32), ("cheb_order", C.c_int32), ("precision", C.c_int32),
                ("top_tau", C.c_int32), ("rank_model", C.c_char_p), ("tune_cache", C.c_char_p),
                ("max_device_bytes", C.c_int64), ("deterministic", C.c_int32), ("bottom_level", C.c_int32),
                ("rank_cap", C.c_int32), ("colouring", C.c_int32), ("stream", C.c_void_p)]


def library_path() -> str:
    return os.path.join(_HERE, "libifmm.so")


def load_library():
    """Loads libifmm.so from the package directory (raises if it is not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() or paper_1905_10602_amd/build.py")
    lib = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "ifmm_default_options": (None, [C.POINTER(Options)]),
        "ifmm_build": (I32, [P, I64, P, P, D, I32, D, I32, C.POINTER(Options), C.POINTER(P)]),
        "ifmm_factor": (I32, [P]),
        "ifmm_solve": (I32, [P, P, P, I32, I64, I32]),
        "ifmm_solve_noalloc": (I32, [P, P, P, I32, I64]),
        "ifmm_solve_noalloc_max_bytes": (I64, []),
        "ifmm_stats": (I32, [P, C.c_char_p, I64]),
        "ifmm_tree_depth": (I32, [P, C.POINTER(I32)]),
        "ifmm_tree_perm": (I32, [P, P]),
        "ifmm_tree_level": (I32, [P, I32, C.POINTER(I32), P, P, P, C.POINTER(I32)]),
        "ifmm_tree_lists": (I32, [P, I32, I32, P, P]),
        "ifmm_ranks": (I32, [P, I32, P]),
        "ifmm_last_error": (C.c_char_p, []),
        "ifmm_destroy": (None, [P]),
        "ifmm_rank_model_params": (I64, [I32]),
        "ifmm_rank_model_eval": (I32, [P, I32, P, I64, P]),
        "ifmm_rank_model_grad": (I32, [P, I32, P, P, I64, C.c_float, C.POINTER(D), P]),
        "ifmm_rank_model_train": (I32, [P, P, I64, I32, I32, C.c_float, C.c_float, P, P]),
        "ifmm_set_rank_model": (I32, [P, P, I32]),
        "ifmm_record_ranks": (I32, [P, I32]),
        "ifmm_rank_records": (I32, [P, P, P, I64, C.POINTER(I64)]),
        "ifmm_factor_batch": (I32, [P, I32, I32, C.POINTER(I32)]),
        "ifmm_solve_batch": (I32, [P, I32, P, P, I32, P, I32, I32, C.POINTER(I32)]),
        "fmm_build": (I32, [P, I64, P, P, D, I32, I32, P, C.POINTER(P)]),
        "fmm_matvec": (I32, [P, P, P, I32]),
        "fmm_gmres": (I32, [P, P, P, D, I32, I32, P, I32, C.POINTER(I32), C.POINTER(D)]),
        "fmm_stats": (I32, [P, C.c_char_p, I64]),
        "fmm_destroy": (None, [P]),
        "fmbem_gmres": (I32, [P, P, P, I64, P, P, I32, D, I32, I32, P, C.POINTER(I32), C.POINTER(D)]),
        "bd_build": (I32, [P, I64, P, P, D, I32, I32, P, C.POINTER(P)]),
        "bd_apply": (I32, [P, P, P, I32]),
        "fmm_gmres_bd": (I32, [P, P, P, D, I32, I32, P, I32, C.POINTER(I32), C.POINTER(D)]),
        "bd_stats": (I32, [P, C.c_char_p, I64]),
        "bd_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def _check(code):
    if code != 0:
        msg = load_library().ifmm_last_error().decode(errors="replace")
        raise IfmmError(code, msg)


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


class IFMM:
    """Handle of one factorisation (ifmm_build / ifmm_factor / ifmm_solve)."""

    def __init__(self, points, eps, sigma, diag=None, weights=None, leaf_max=64, cheb_order=4, rank_cap=0,
                 max_device_bytes=0, stream=None, precision="fp64", top_tau=2, bottom_level=0, rank_model=None,
                 tune_cache=None, colouring="stride"):
        lib = load_library()
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2 or pts.shape[1] != 3:
            raise ValueError("points must be (N, 3)")
        self.N = pts.shape[0]
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        dvec, dsc = None, 0.0
        if diag is None:
            raise ValueError("diag (scalar or array) is required")
        if np.isscalar(diag):
            dsc = float(diag)
        else:
            dvec = np.ascontiguousarray(diag, dtype=np.float64)
        opt = Options()
        lib.ifmm_default_options(C.byref(opt))
        opt.leaf_max = leaf_max
        opt.cheb_order = cheb_order
        opt.rank_cap = rank_cap
        opt.precision = {"fp64": 0, "mixed": 1}[precision]
        opt.max_device_bytes = max_device_bytes
        opt.top_tau = top_tau
        opt.bottom_level = bottom_level
        opt.colouring = {"stride": 0, "lookback": 1}[colouring]
        opt.rank_model = None if rank_model is None else os.fsencode(rank_model)
        opt.tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
        opt.stream = None if stream is None else C.c_void_p(stream)
        h = C.c_void_p()
        _check(lib.ifmm_build(_ptr(pts), self.N, _ptr(w), _ptr(dvec), dsc, 0, float(eps), int(sigma),
                              C.byref(opt), C.byref(h)))
        self._h = h
        self.eps = eps
        self.sigma = sigma

    def close(self):
        if getattr(self, "_h", None):
            load_library().ifmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- method
    def factor(self):
        _check(load_library().ifmm_factor(self._h))
        return self

    def solve(self, b):
        """b: numpy (N,) / (N, k) on the host, or a torch tensor on the GPU
        (column-major (N, k) is taken as b.T contiguous (k, N))."""
        lib = load_library()
        if hasattr(b, "is_cuda") and b.is_cuda:
            import torch
            vec = b.dim() == 1
            B = b.reshape(-1, 1) if vec else b
            k = B.shape[1]
            Bc = B.t().contiguous()  # (k, N) row-major == (N, k) column-major
            X = torch.empty_like(Bc)
            _check(lib.ifmm_solve(self._h, _ptr(Bc), _ptr(X), k, self.N, 1))
            out = X.t()
            return out[:, 0] if vec else out
        B = np.asarray(b, dtype=np.float64)
        vec = B.ndim == 1
        Bf = np.asfortranarray(B.reshape(self.N, -1))
        X = np.empty_like(Bf, order="F")
        _check(lib.ifmm_solve(self._h, _ptr(Bf), _ptr(X), Bf.shape[1], self.N, 0))
        return X[:, 0] if vec else X

    def stats(self):
        buf = C.create_string_buffer(1 << 16)
        _check(load_library().ifmm_stats(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    # -- structure queries
    def depth(self):
        d = C.c_int32()
        _check(load_library().ifmm_tree_depth(self._h, C.byref(d)))
        return d.value

    def perm(self):
        p = np.empty(self.N, dtype=np.int64)
        _check(load_library().ifmm_tree_perm(self._h, _ptr(p)))
        return p

    def level(self, lvl):
        lib = load_library()
        nn = C.c_int32()
        _check(lib.ifmm_tree_level(self._h, lvl, C.byref(nn), None, None, None, None))
        n = nn.value
        coords = np.empty((n, 3), dtype=np.int32)
        parent = np.empty(n, dtype=np.int32)
        colour = np.empty(n, dtype=np.int32)
        nc = C.c_int32()
        _check(lib.ifmm_tree_level(self._h, lvl, C.byref(nn), _ptr(coords), _ptr(parent), _ptr(colour),
                                   C.byref(nc)))
        return {"coords": coords, "parent": parent, "colour": colour, "ncolour": nc.value}

    def lists(self, lvl, which):
        lib = load_library()
        n = self.level(lvl)["coords"].shape[0]
        ptr = np.empty(n + 1, dtype=np.int32)
        _check(lib.ifmm_tree_lists(self._h, lvl, which, _ptr(ptr), None))
        idx = np.empty(int(ptr[-1]), dtype=np.int32)
        _check(lib.ifmm_tree_lists(self._h, lvl, which, _ptr(ptr), _ptr(idx)))
        return ptr, idx

    # -- learned recompression rank
    def set_rank_model(self, theta):
        """theta: flat float32 parameters (None clears the model)."""
        lib = load_library()
        if theta is None:
            _check(lib.ifmm_set_rank_model(self._h, None, RANK_FEATURES))
            return self
        th = np.ascontiguousarray(theta, dtype=np.float32)
        _check(lib.ifmm_set_rank_model(self._h, _ptr(th), RANK_FEATURES))
        return self

    def record_ranks(self, on=True):
        _check(load_library().ifmm_record_ranks(self._h, 1 if on else 0))
        return self

    def rank_records(self):
        lib = load_library()
        cnt = C.c_int64()
        _check(lib.ifmm_rank_records(self._h, None, None, 0, C.byref(cnt)))
        X = np.zeros((cnt.value, RANK_FEATURES), dtype=np.float32)
        t = np.zeros(cnt.value, dtype=np.float32)
        _check(lib.ifmm_rank_records(self._h, _ptr(X), _ptr(t), cnt.value, C.byref(cnt)))
        return X, t

    def ranks(self, lvl):
        n = self.level(lvl)["coords"].shape[0]
        r = np.empty(n, dtype=np.int32)
        _check(load_library().ifmm_ranks(self._h, lvl, _ptr(r)))
        return r


def _is_dev(a):
    return hasattr(a, "is_cuda") and a.is_cuda


class FMM:
    """Handle of the Chebyshev FMM product y = A~ x (fmm_build / fmm_matvec / fmm_gmres)."""

    def __init__(self, points, diag, weights=None, cheb_order=5, leaf_max=64, stream=None):
        lib = load_library()
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2 or pts.shape[1] != 3:
            raise ValueError("points must be (N, 3)")
        self.N = pts.shape[0]
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        dvec, dsc = (None, float(diag)) if np.isscalar(diag) else (np.ascontiguousarray(diag, dtype=np.float64), 0.0)
        h = C.c_void_p()
        _check(lib.fmm_build(_ptr(pts), self.N, _ptr(w), _ptr(dvec), dsc, int(cheb_order), int(leaf_max),
                             None if stream is None else C.c_void_p(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().fmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec(self, x):
        """x: numpy (N,) on the host or a contiguous torch (N,) float64 tensor on the GPU."""
        lib = load_library()
        if _is_dev(x):
            import torch
            y = torch.empty_like(x)
            _check(lib.fmm_matvec(self._h, _ptr(x.contiguous()), _ptr(y), 1))
            return y
        xv = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(xv)
        _check(lib.fmm_matvec(self._h, _ptr(xv), _ptr(y), 0))
        return y

    def gmres(self, b, precond=None, tol=1e-8, restart=50, maxit=1000, allow_noconv=False):
        """Returns (x, iterations, relative residual).  precond: a factored IFMM, a BD or None."""
        lib = load_library()
        it, rr = C.c_int32(), C.c_double()
        ph = None if precond is None else precond._h
        fn = lib.fmm_gmres_bd if isinstance(precond, BD) else lib.fmm_gmres
        if _is_dev(b):
            import torch
            bc = b.contiguous()
            x = torch.empty_like(bc)
            code = fn(self._h, _ptr(bc), ph, float(tol), int(restart), int(maxit), _ptr(x), 1, C.byref(it), C.byref(rr))
        else:
            bc = np.ascontiguousarray(b, dtype=np.float64)
            x = np.empty_like(bc)
            code = fn(self._h, _ptr(bc), ph, float(tol), int(restart), int(maxit), _ptr(x), 0, C.byref(it), C.byref(rr))
        if not (allow_noconv and code == -7):
            _check(code)
        return x, it.value, rr.value

    def stats(self):
        buf = C.create_string_buffer(4096)
        _check(load_library().fmm_stats(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())


class BD:
    """Handle of the block-diagonal preconditioner (bd_build / bd_apply)."""

    def __init__(self, points, diag, weights=None, level=0, leaf_max=64, stream=None):
        lib = load_library()
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2 or pts.shape[1] != 3:
            raise ValueError("points must be (N, 3)")
        self.N = pts.shape[0]
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        dvec, dsc = (None, float(diag)) if np.isscalar(diag) else (np.ascontiguousarray(diag, dtype=np.float64), 0.0)
        h = C.c_void_p()
        _check(lib.bd_build(_ptr(pts), self.N, _ptr(w), _ptr(dvec), dsc, int(level), int(leaf_max),
                            None if stream is None else C.c_void_p(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().bd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, r):
        lib = load_library()
        if _is_dev(r):
            import torch
            z = torch.empty_like(r)
            _check(lib.bd_apply(self._h, _ptr(r.contiguous()), _ptr(z), 1))
            return z
        rv = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(rv)
        _check(lib.bd_apply(self._h, _ptr(rv), _ptr(z), 0))
        return z

    def stats(self):
        buf = C.create_string_buffer(1024)
        _check(load_library().bd_stats(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())


def fmbem_gmres(centroids, areas, self_terms, f, precond=None, fmm_cheb_order=5, tol=1e-8, restart=50, maxit=1000):
    """The one-call FMBEM driver (host arrays).  Returns (sol, iterations, relres)."""
    lib = load_library()
    c = np.ascontiguousarray(centroids, dtype=np.float64)
    a = np.ascontiguousarray(areas, dtype=np.float64)
    st = np.ascontiguousarray(self_terms, dtype=np.float64)
    fv = np.ascontiguousarray(f, dtype=np.float64)
    sol = np.empty_like(fv)
    it, rr = C.c_int32(), C.c_double()
    _check(lib.fmbem_gmres(_ptr(c), _ptr(a), _ptr(st), c.shape[0], _ptr(fv), None if precond is None else precond._h,
                           int(fmm_cheb_order), float(tol), int(restart), int(maxit), _ptr(sol), C.byref(it),
                           C.byref(rr)))
    return sol, it.value, rr.value


# -- the rank network (device forward / gradient / training)
def rank_model_params(nfeat=RANK_FEATURES):
    return int(load_library().ifmm_rank_model_params(nfeat))


def rank_model_eval(theta, X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    th = np.ascontiguousarray(theta, dtype=np.float32)
    y = np.zeros(X.shape[0], dtype=np.float32)
    _check(load_library().ifmm_rank_model_eval(_ptr(th), X.shape[1], _ptr(X), X.shape[0], _ptr(y)))
    return y


def rank_model_grad(theta, X, t, tau):
    X = np.ascontiguousarray(X, dtype=np.float32)
    tt = np.ascontiguousarray(t, dtype=np.float32)
    th = np.ascontiguousarray(theta, dtype=np.float32)
    g = np.zeros_like(th)
    L = C.c_double()
    _check(load_library().ifmm_rank_model_grad(_ptr(th), X.shape[1], _ptr(X), _ptr(tt), X.shape[0], float(tau),
                                               C.byref(L), _ptr(g)))
    return L.value, g


def rank_model_train(X, t, theta, steps, lr=1e-3, tau=0.9):
    """Returns (trained theta, loss history)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    tt = np.ascontiguousarray(t, dtype=np.float32)
    th = np.array(theta, dtype=np.float32, copy=True)
    hist = np.zeros(max(int(steps), 1))
    _check(load_library().ifmm_rank_model_train(_ptr(X), _ptr(tt), X.shape[0], X.shape[1], int(steps), float(lr),
                                                float(tau), _ptr(th), _ptr(hist)))
    return th, hist[:int(steps)]


def factor_batch(handles, threads=0):
    """ifmm_factor_batch over IFMM handles; returns the handles."""
    lib = load_library()
    arr = (C.c_void_p * len(handles))(*[h._h.value for h in handles])
    failed = C.c_int32(-1)
    _check(lib.ifmm_factor_batch(C.cast(arr, C.c_void_p), len(handles), int(threads), C.byref(failed)))
    return handles


def solve_batch(handles, rhs, threads=0):
    """ifmm_solve_batch: rhs is a list of host (N_g, k) arrays (same k); returns the solutions."""
    lib = load_library()
    G = len(handles)
    Bs = [np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(h.N, -1)) for h, b in zip(handles, rhs)]
    k = Bs[0].shape[1]
    Xs = [np.empty_like(b, order="F") for b in Bs]
    hp = (C.c_void_p * G)(*[h._h.value for h in handles])
    rp = (C.c_void_p * G)(*[b.ctypes.data for b in Bs])
    xp = (C.c_void_p * G)(*[x.ctypes.data for x in Xs])
    ld = (C.c_int64 * G)(*[h.N for h in handles])
    failed = C.c_int32(-1)
    _check(lib.ifmm_solve_batch(C.cast(hp, C.c_void_p), G, C.cast(rp, C.c_void_p), C.cast(xp, C.c_void_p), k,
                                C.cast(ld, C.c_void_p), 0, int(threads), C.byref(failed)))
    return Xs
