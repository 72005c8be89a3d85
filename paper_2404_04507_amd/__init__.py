"""Python binding of libiwfpm (the IWFPM Hamiltonian apply and eigensolver for gfx950).

Argument marshalling only: every step of the method runs in the HIP library.
Vectors are torch complex128 tensors on the plan's GPU, shaped (nvec, N)
(each vector contiguous, i.e. the library's N x nvec column-major block) or (N,).
torch supplies device memory and the stream; nothing here computes.

The library is loaded on first use; if it has not been built the binding
raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

__all__ = ["Plan", "Learned", "IwfpmError", "load_library", "library_path", "EXPORTED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

EXPORTED = ["iwfpm_default_opts", "iwfpm_status_string", "iwfpm_plan", "iwfpm_destroy", "iwfpm_dof",
            "iwfpm_grid_shape", "iwfpm_indices", "iwfpm_kinetic", "iwfpm_norm_bound", "iwfpm_apply",
            "iwfpm_apply_prec", "iwfpm_default_eigs_opts", "iwfpm_eigs", "iwfpm_profile",
            "iwfpm_profile_read", "iwfpm_dense_geneig", "iwfpm_dense_svqb", "iwfpm_dense_heev_lowest",
            "iwfpm_tune", "iwfpm_schedule",
            "iwfpm_batch_create", "iwfpm_batch_apply", "iwfpm_batch_destroy", "iwfpm_eigs_batched",
            "iwfpm_conv", "iwfpm_default_learned_opts", "iwfpm_default_train_opts", "iwfpm_learned_create",
            "iwfpm_learned_destroy", "iwfpm_learned_nparams", "iwfpm_learned_get", "iwfpm_learned_set",
            "iwfpm_learned_attach", "iwfpm_learned_shells", "iwfpm_learned_forward", "iwfpm_learned_grad",
            "iwfpm_learned_step", "iwfpm_learned_train", "iwfpm_eigenfunction", "iwfpm_apply_noalloc",
            "iwfpm_noalloc_scratch_bytes"]

_VOID_FUNCS = ("iwfpm_default_opts", "iwfpm_status_string", "iwfpm_default_eigs_opts",
               "iwfpm_default_learned_opts", "iwfpm_default_train_opts")
LEARNED_FEATURES = 8
LEARNED_HIDDEN = 256

PREC = {"fp64": 0, "fp32": 1}
WINDOW = {"exact": 0, "rounded": 1, "pm": 2}
ORDER = {"grid": 0, "window": 1}
SCHED = {"auto": 0, "fused": 1, "threepass": 2}
PRECOND = {"none": 0, "plain": 1, "learned": 2}
ARITH = {"auto": 0, "complex": 1, "real": 2}


class IwfpmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib().iwfpm_status_string(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("window_variant", ctypes.c_int), ("order", ctypes.c_int),
                ("device", ctypes.c_int), ("schedule", ctypes.c_int), ("split", ctypes.c_int),
                ("tile", ctypes.c_int)]


class _EigsOpts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int), ("block", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("precond", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("polish", ctypes.c_int), ("arith", ctypes.c_int)]


class _LearnedOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("shells", ctypes.c_int), ("seed", ctypes.c_uint64)]


class _TrainOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("lr", ctypes.c_double), ("nev", ctypes.c_int), ("block", ctypes.c_int),
                ("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("snapshots", ctypes.c_int),
                ("stride", ctypes.c_int), ("seed", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("matvecs", ctypes.c_int64), ("converged", ctypes.c_int),
                ("restarts", ctypes.c_int), ("fallback", ctypes.c_int), ("polished", ctypes.c_int),
                ("t_total", ctypes.c_double), ("t_apply", ctypes.c_double)]


def library_path() -> str:
    return os.environ.get("IWFPM_LIBRARY") or os.path.join(_HERE, "libiwfpm.so")


def load_library():
    """Load libiwfpm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2404_04507_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    lib.iwfpm_default_opts.argtypes = [ctypes.POINTER(_Opts)]
    lib.iwfpm_default_opts.restype = None
    lib.iwfpm_status_string.argtypes = [ctypes.c_int]
    lib.iwfpm_status_string.restype = ctypes.c_char_p
    lib.iwfpm_plan.argtypes = [ctypes.c_int, ctypes.c_int, dp, ip, ip, ctypes.c_int, ip, dp,
                               ctypes.POINTER(_Opts), ctypes.POINTER(vp)]
    lib.iwfpm_destroy.argtypes = [vp]
    lib.iwfpm_dof.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.iwfpm_grid_shape.argtypes = [vp, ip]
    lib.iwfpm_indices.argtypes = [vp, ip]
    lib.iwfpm_kinetic.argtypes = [vp, dp]
    lib.iwfpm_norm_bound.argtypes = [vp, dp]
    lib.iwfpm_apply.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.iwfpm_apply_prec.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    lib.iwfpm_apply_noalloc.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.iwfpm_noalloc_scratch_bytes.argtypes = []
    lib.iwfpm_noalloc_scratch_bytes.restype = ctypes.c_int64
    lib.iwfpm_profile.argtypes = [vp, ctypes.c_int]
    lib.iwfpm_profile_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.iwfpm_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    lib.iwfpm_batch_apply.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int), vp]
    lib.iwfpm_batch_destroy.argtypes = [vp]
    lib.iwfpm_eigs_batched.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(_EigsOpts), dp, dp,
                                       ctypes.POINTER(_Stats), vp]
    lib.iwfpm_tune.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, dp]
    lib.iwfpm_schedule.argtypes = [vp, ctypes.c_int, ip]
    lib.iwfpm_dense_geneig.argtypes = [ctypes.c_int, dp, dp, dp, dp]
    lib.iwfpm_dense_svqb.argtypes = [ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_int)]
    lib.iwfpm_dense_heev_lowest.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
    lib.iwfpm_default_eigs_opts.argtypes = [ctypes.POINTER(_EigsOpts)]
    lib.iwfpm_default_eigs_opts.restype = None
    lib.iwfpm_eigs.argtypes = [vp, ctypes.POINTER(_EigsOpts), vp, dp, vp, dp, ctypes.POINTER(_Stats), vp]
    lib.iwfpm_conv.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    lib.iwfpm_eigenfunction.argtypes = [vp, vp, dp, dp, ip, vp, vp]
    fp = ctypes.POINTER(ctypes.c_float)
    lib.iwfpm_default_learned_opts.argtypes = [ctypes.POINTER(_LearnedOpts)]
    lib.iwfpm_default_learned_opts.restype = None
    lib.iwfpm_default_train_opts.argtypes = [ctypes.POINTER(_TrainOpts)]
    lib.iwfpm_default_train_opts.restype = None
    lib.iwfpm_learned_create.argtypes = [ctypes.POINTER(_LearnedOpts), ctypes.POINTER(vp)]
    lib.iwfpm_learned_destroy.argtypes = [vp]
    lib.iwfpm_learned_nparams.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.iwfpm_learned_get.argtypes = [vp, fp]
    lib.iwfpm_learned_set.argtypes = [vp, fp]
    lib.iwfpm_learned_attach.argtypes = [vp, vp]
    lib.iwfpm_learned_shells.argtypes = [vp, ip, fp]
    lib.iwfpm_learned_forward.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.iwfpm_learned_grad.argtypes = [vp, vp, ctypes.c_int, dp, dp, fp, vp]
    lib.iwfpm_learned_step.argtypes = [vp, vp, ctypes.c_int, dp, ctypes.c_double, dp, vp]
    lib.iwfpm_learned_train.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(_TrainOpts), dp, vp]
    for name in EXPORTED:
        if name not in _VOID_FUNCS:
            getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


def _lib():
    return load_library()


def _check(status: int, where: str):
    if status != 0:
        raise IwfpmError(status, where)


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def dense_geneig(A, B=None):
    """The library's host Rayleigh-Ritz solver: A c = w B c (Hermitian, B PD)."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    a = _f64(np.asfortranarray(A).reshape(-1, order="F").view(np.float64))
    b = None if B is None else _f64(np.asfortranarray(np.asarray(B, dtype=np.complex128)).reshape(-1, order="F").view(np.float64))
    w = np.zeros(n)
    C = np.zeros(2 * n * n)
    st = _lib().iwfpm_dense_geneig(n, _ptr(a, ctypes.c_double), None if b is None else _ptr(b, ctypes.c_double),
                                   _ptr(w, ctypes.c_double), _ptr(C, ctypes.c_double))
    _check(st, "iwfpm_dense_geneig")
    return w, C.view(np.complex128).reshape(n, n, order="F")


def dense_heev_lowest(A, nv):
    """The Rayleigh-Ritz step's eigensolver: all eigenvalues, eigenvectors of the nv lowest."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    a = _f64(np.asfortranarray(A).reshape(-1, order="F").view(np.float64))
    w = np.zeros(n)
    V = np.zeros(2 * n * max(nv, 1))
    _check(_lib().iwfpm_dense_heev_lowest(n, int(nv), _ptr(a, ctypes.c_double), _ptr(w, ctypes.c_double),
                                          _ptr(V, ctypes.c_double)), "iwfpm_dense_heev_lowest")
    return w, V.view(np.complex128)[:n * nv].reshape(n, nv, order="F")


def dense_svqb(G):
    G = np.asarray(G, dtype=np.complex128)
    k = G.shape[0]
    g = _f64(np.asfortranarray(G).reshape(-1, order="F").view(np.float64))
    T = np.zeros(2 * k * k)
    r = ctypes.c_int()
    _check(_lib().iwfpm_dense_svqb(k, _ptr(g, ctypes.c_double), _ptr(T, ctypes.c_double), ctypes.byref(r)),
           "iwfpm_dense_svqb")
    return T.view(np.complex128)[:k * r.value].reshape(k, r.value, order="F")


class Batch:
    """A ragged batch of plans applied by one persistent launch per pass (iwfpm_batch_*)."""

    def __init__(self, plans, precision="fp32", graph=True):
        lib = _lib()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib.iwfpm_batch_create(len(self.plans), arr, PREC[precision], int(bool(graph)), ctypes.byref(h)),
               "iwfpm_batch_create")
        self._h = h

    def apply(self, psis, outs, stream=None):
        n = len(self.plans)
        nv = (ctypes.c_int * n)()
        ps = (ctypes.c_void_p * n)()
        hs = (ctypes.c_void_p * n)()
        for i, (plan, x, y) in enumerate(zip(self.plans, psis, outs)):
            if x is None or x.numel() == 0:
                nv[i] = 0
                continue
            nv[i] = plan._check_block(x)
            plan._check_block(y)
            ps[i] = x.data_ptr()
            hs[i] = y.data_ptr()
        _check(_lib().iwfpm_batch_apply(self._h, ps, hs, nv, _stream_handle(stream)), "iwfpm_batch_apply")
        return outs

    def close(self):
        if getattr(self, "_h", None):
            _lib().iwfpm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eigs_batched(plans, nev, tol=1e-8, maxit=500, block=0, precond="plain", seed=2404045070, polish=True,
                 stream=None, allow_noconv=False, arith="auto"):
    """Lowest nev eigenpairs of every plan, solved in lock step (iwfpm_eigs_batched)."""
    lib = _lib()
    B = len(plans)
    o = _EigsOpts()
    lib.iwfpm_default_eigs_opts(ctypes.byref(o))
    o.nev, o.block, o.tol, o.maxit = int(nev), int(block), float(tol), int(maxit)
    o.precond, o.seed, o.polish = PRECOND[precond], int(seed), int(bool(polish))
    o.arith = ARITH[arith]
    evals = np.zeros((B, nev))
    eta = np.zeros((B, nev))
    stats = (_Stats * B)()
    arr = (ctypes.c_void_p * B)(*[p._h.value for p in plans])
    st = lib.iwfpm_eigs_batched(B, arr, ctypes.byref(o), _ptr(evals, ctypes.c_double), _ptr(eta, ctypes.c_double),
                                stats, _stream_handle(stream))
    if st != 0 and not (allow_noconv and st == -8):
        raise IwfpmError(st, "iwfpm_eigs_batched")
    return evals, eta, [{"iterations": s.iterations, "matvecs": s.matvecs, "converged": s.converged,
                         "polished": s.polished, "fallback": s.fallback, "t_total": s.t_total} for s in stats], st


@dataclass
class EigsResult:
    evals: np.ndarray
    evecs: object          # torch tensor (nev, N) complex128 or None
    eta: np.ndarray
    iterations: int
    matvecs: int
    converged: int
    restarts: int
    fallback: int
    polished: int
    t_total: float
    t_apply: float
    status: int


class Learned:
    """The learned preconditioner's network (wraps iwfpm_learned_t)."""

    def __init__(self, shells=1024, seed=2404045070, device=0):
        lib = _lib()
        o = _LearnedOpts()
        lib.iwfpm_default_learned_opts(ctypes.byref(o))
        o.device, o.shells, o.seed = int(device), int(shells), int(seed)
        h = ctypes.c_void_p()
        _check(lib.iwfpm_learned_create(ctypes.byref(o), ctypes.byref(h)), "iwfpm_learned_create")
        self._h = h
        self.shells = int(shells)
        self.device = int(device)
        n = ctypes.c_int64()
        _check(lib.iwfpm_learned_nparams(h, ctypes.byref(n)), "iwfpm_learned_nparams")
        self.nparams = int(n.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib().iwfpm_learned_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def get(self) -> np.ndarray:
        out = np.zeros(self.nparams, dtype=np.float32)
        _check(_lib().iwfpm_learned_get(self._h, _ptr(out, ctypes.c_float)), "iwfpm_learned_get")
        return out

    def set(self, params):
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        if a.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {a.size}")
        _check(_lib().iwfpm_learned_set(self._h, _ptr(a, ctypes.c_float)), "iwfpm_learned_set")

    def layout(self) -> list:
        """[(name, offset, shape)] of the parameter vector."""
        dims = [LEARNED_FEATURES, LEARNED_HIDDEN, LEARNED_HIDDEN, LEARNED_HIDDEN, 2]
        out, off = [], 0
        for l in range(4):
            out.append((f"W{l + 1}", off, (dims[l], dims[l + 1])))
            off += dims[l] * dims[l + 1]
            out.append((f"b{l + 1}", off, (dims[l + 1],)))
            off += dims[l + 1]
        out.append(("beta", off, (2,)))
        return out

    def save(self, path: str):
        np.savez(path, params=self.get(), shells=np.int64(self.shells))

    def load(self, path: str):
        with np.load(path, allow_pickle=False) as z:
            if int(z["shells"]) != self.shells:
                raise ValueError("shell count of the saved network differs")
            self.set(z["params"])

    def train(self, plans, steps=3000, lr=1e-3, nev=8, block=0, tol=1e-8, maxit=1000, snapshots=24, stride=4,
              seed=2404045070, stream=None) -> np.ndarray:
        """Train on data from plain solves of `plans` (iwfpm_learned_train); returns the loss per step."""
        lib = _lib()
        o = _TrainOpts()
        lib.iwfpm_default_train_opts(ctypes.byref(o))
        o.steps, o.lr, o.nev, o.block, o.tol = int(steps), float(lr), int(nev), int(block), float(tol)
        o.maxit, o.snapshots, o.stride, o.seed = int(maxit), int(snapshots), int(stride), int(seed)
        arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
        loss = np.zeros(max(1, steps))
        _check(lib.iwfpm_learned_train(self._h, len(plans), arr, ctypes.byref(o), _ptr(loss, ctypes.c_double),
                                       _stream_handle(stream)), "iwfpm_learned_train")
        for p in plans:
            p._net = self
        return loss[:steps]


class Plan:
    """An IWFPM plan (wraps iwfpm_plan_t).

    P: d x n (kinetic 1/2 |2 pi P k|^2), K: d ints, L: n-d ints,
    modes: n_modes x n ints, vhat: n_modes complex.
    """

    def __init__(self, P, K, L, modes, vhat, *, precision="fp64", window="exact", order="grid",
                 device=0, schedule="auto", split=0, tile=0):
        lib = _lib()
        P = _f64(np.atleast_2d(P))
        d, n = P.shape
        K = _i32(np.atleast_1d(K))
        L = _i32(np.atleast_1d(L))
        modes = _i32(np.asarray(modes).reshape(-1, n))
        vh = np.asarray(vhat, dtype=np.complex128).reshape(-1)
        vri = _f64(np.stack([vh.real, vh.imag], axis=1).reshape(-1)) if vh.size else _f64(np.zeros(2))
        opts = _Opts()
        lib.iwfpm_default_opts(ctypes.byref(opts))
        opts.precision = PREC[precision]
        opts.window_variant = WINDOW[window]
        opts.order = ORDER[order]
        opts.device = int(device)
        opts.schedule = SCHED[schedule]
        opts.split = int(split)
        opts.tile = int(tile)
        h = ctypes.c_void_p()
        st = lib.iwfpm_plan(d, n, _ptr(P, ctypes.c_double), _ptr(K, ctypes.c_int32), _ptr(L, ctypes.c_int32),
                            modes.shape[0], _ptr(modes, ctypes.c_int32), _ptr(vri, ctypes.c_double),
                            ctypes.byref(opts), ctypes.byref(h))
        _check(st, "iwfpm_plan")
        self._h = h
        self.d, self.n = d, n
        self.device = int(device)
        self.precision = precision
        N = ctypes.c_int64()
        _check(lib.iwfpm_dof(h, ctypes.byref(N)), "iwfpm_dof")
        self.N = int(N.value)
        ext = np.zeros(n, dtype=np.int32)
        _check(lib.iwfpm_grid_shape(h, _ptr(ext, ctypes.c_int32)), "iwfpm_grid_shape")
        self.ext = tuple(int(x) for x in ext)

    @classmethod
    def from_problem(cls, prob, **kw):
        return cls(prob.P, prob.K, prob.L, prob.modes, prob.vhat, **kw)

    def close(self):
        if getattr(self, "_h", None):
            _lib().iwfpm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- host queries --------------------------------------------------------
    def indices(self) -> np.ndarray:
        out = np.zeros((self.N, self.n), dtype=np.int32)
        _check(_lib().iwfpm_indices(self._h, _ptr(out, ctypes.c_int32)), "iwfpm_indices")
        return out

    def kinetic(self) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.float64)
        _check(_lib().iwfpm_kinetic(self._h, _ptr(out, ctypes.c_double)), "iwfpm_kinetic")
        return out

    def norm_bound(self) -> float:
        out = ctypes.c_double()
        _check(_lib().iwfpm_norm_bound(self._h, ctypes.byref(out)), "iwfpm_norm_bound")
        return out.value

    # -- device --------------------------------------------------------------
    def _check_block(self, x):
        import torch
        if not isinstance(x, torch.Tensor) or x.dtype != torch.complex128 or not x.is_cuda:
            raise TypeError("vectors must be complex128 CUDA tensors")
        if x.shape[-1] != self.N or not x.is_contiguous():
            raise ValueError(f"vectors must be contiguous with last dimension N={self.N}")
        return 1 if x.dim() == 1 else int(np.prod(x.shape[:-1]))

    def apply(self, psi, out=None, precision=None, stream=None):
        """H psi; psi (nvec, N) or (N,) complex128 on the plan's GPU."""
        import torch
        nvec = self._check_block(psi)
        if out is None:
            out = torch.empty_like(psi)
        else:
            self._check_block(out)
        prec = PREC[precision] if precision is not None else PREC[self.precision]
        st = _lib().iwfpm_apply_prec(self._h, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     nvec, prec, _stream_handle(stream))
        _check(st, "iwfpm_apply")
        return out

    def apply_noalloc(self, psi, out, stream=None):
        """H psi through iwfpm_apply_noalloc (the library's static scratch, no
        device allocation); `out` must be given."""
        nvec = self._check_block(psi)
        self._check_block(out)
        st = _lib().iwfpm_apply_noalloc(self._h, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        nvec, _stream_handle(stream))
        _check(st, "iwfpm_apply_noalloc")
        return out

    def eigenfunction(self, u, origin, step, npts, out=None, stream=None):
        """u(xi) = sum_k U_k exp(i 2 pi (P k) . xi) on the tensor grid
        xi_j = origin[j] + step[j] * i_j (iwfpm_eigenfunction); u: (N,)
        complex128 on the plan's GPU; returns a complex128 tensor of shape npts."""
        import torch
        if u.dim() != 1 or u.dtype != torch.complex128 or u.numel() != self.N or not u.is_cuda:
            raise ValueError(f"u must be a CUDA complex128 vector of length {self.N}")
        u = u.contiguous()
        npts = [int(x) for x in npts]
        if not (len(origin) == len(step) == len(npts) == self.d):
            raise ValueError(f"origin, step and npts need {self.d} entries")
        if out is None:
            out = torch.empty(npts, dtype=torch.complex128, device=u.device)
        elif tuple(out.shape) != tuple(npts) or out.dtype != torch.complex128 or not out.is_contiguous():
            raise ValueError("out must be a contiguous complex128 tensor of shape npts")
        o = (ctypes.c_double * self.d)(*[float(x) for x in origin])
        h = (ctypes.c_double * self.d)(*[float(x) for x in step])
        n = (ctypes.c_int32 * self.d)(*npts)
        _check(_lib().iwfpm_eigenfunction(self._h, ctypes.c_void_p(u.data_ptr()), o, h, n,
                                          ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
               "iwfpm_eigenfunction")
        return out

    def conv(self, psi, out=None, precision=None, stream=None):
        """The potential block alone, F V F^{-1} psi (iwfpm_conv)."""
        import torch
        nvec = self._check_block(psi)
        if out is None:
            out = torch.empty_like(psi)
        else:
            self._check_block(out)
        prec = PREC[precision] if precision is not None else PREC[self.precision]
        st = _lib().iwfpm_conv(self._h, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               nvec, prec, _stream_handle(stream))
        _check(st, "iwfpm_conv")
        return out

    # -- learned preconditioner ----------------------------------------------
    def attach(self, net):
        """Attach a Learned network (None detaches)."""
        _check(_lib().iwfpm_learned_attach(self._h, net._h if net is not None else None), "iwfpm_learned_attach")
        self._net = net

    def learned_shells(self, shells: int):
        """(shell index per vector entry, S x features) of the attached network."""
        sh = np.zeros(self.N, dtype=np.int32)
        ft = np.zeros((shells, LEARNED_FEATURES), dtype=np.float32)
        _check(_lib().iwfpm_learned_shells(self._h, _ptr(sh, ctypes.c_int32), _ptr(ft, ctypes.c_float)),
               "iwfpm_learned_shells")
        return sh, ft

    def learned_forward(self, r, out=None, stream=None):
        import torch
        nvec = self._check_block(r)
        if out is None:
            out = torch.empty_like(r)
        _check(_lib().iwfpm_learned_forward(self._h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            nvec, _stream_handle(stream)), "iwfpm_learned_forward")
        return out

    def learned_grad(self, x, lam, want_grad=True, stream=None):
        """(loss, gradient over the parameter vector or None) of the attached
        network on the iterate block x with exact eigenvalues lam."""
        nvec = self._check_block(x)
        lam = _f64(lam)
        loss = ctypes.c_double()
        g = np.zeros(self._net.nparams, dtype=np.float32) if want_grad else None
        _check(_lib().iwfpm_learned_grad(self._h, ctypes.c_void_p(x.data_ptr()), nvec, _ptr(lam, ctypes.c_double),
                                         ctypes.byref(loss), _ptr(g, ctypes.c_float) if g is not None else None,
                                         _stream_handle(stream)), "iwfpm_learned_grad")
        return loss.value, g

    def learned_step(self, x, lam, lr=2e-3, stream=None) -> float:
        nvec = self._check_block(x)
        lam = _f64(lam)
        loss = ctypes.c_double()
        _check(_lib().iwfpm_learned_step(self._h, ctypes.c_void_p(x.data_ptr()), nvec, _ptr(lam, ctypes.c_double),
                                         float(lr), ctypes.byref(loss), _stream_handle(stream)),
               "iwfpm_learned_step")
        return loss.value

    def tune(self, nvec=16, precision=None, stream=None) -> float:
        """Autotune the apply schedule on the device; returns the best microseconds per apply."""
        best = ctypes.c_double()
        prec = -1 if precision is None else PREC[precision]
        _check(_lib().iwfpm_tune(self._h, int(nvec), prec, _stream_handle(stream), ctypes.byref(best)), "iwfpm_tune")
        return best.value

    def schedule(self, precision=None) -> dict:
        out = np.zeros(5, dtype=np.int32)
        prec = -1 if precision is None else PREC[precision]
        _check(_lib().iwfpm_schedule(self._h, prec, _ptr(out, ctypes.c_int32)), "iwfpm_schedule")
        return {"fused": bool(out[0]), "split": int(out[1]), "tile": int(out[2]), "slabs_per_wg": int(out[3]),
                "threads": int(out[4])}

    def profile(self, enable: bool):
        _check(_lib().iwfpm_profile(self._h, int(bool(enable))), "iwfpm_profile")

    def profile_read(self) -> dict:
        ms = np.zeros(4)
        la = np.zeros(4, dtype=np.int64)
        pt = np.zeros(4, dtype=np.int64)
        _check(_lib().iwfpm_profile_read(self._h, _ptr(ms, ctypes.c_double), _ptr(la, ctypes.c_int64),
                                         _ptr(pt, ctypes.c_int64)), "iwfpm_profile_read")
        names = ["fused", "pass1", "pass2", "pass3"]
        return {n: {"ms": float(ms[i]), "launches": int(la[i]), "points": int(pt[i])} for i, n in enumerate(names)}

    def eigs(self, nev, tol=1e-8, maxit=500, block=0, precond="plain", x0=None, seed=2404045070,
             polish=True, want_vectors=True, stream=None, allow_noconv=False, arith="auto") -> EigsResult:
        import torch
        lib = _lib()
        o = _EigsOpts()
        lib.iwfpm_default_eigs_opts(ctypes.byref(o))
        o.nev, o.block, o.tol, o.maxit = int(nev), int(block), float(tol), int(maxit)
        o.precond, o.seed, o.polish = PRECOND[precond], int(seed), int(bool(polish))
        o.arith = ARITH[arith]
        evals = np.zeros(nev)
        eta = np.zeros(nev)
        vecs = None
        if want_vectors:
            vecs = torch.empty((nev, self.N), dtype=torch.complex128, device=f"cuda:{self.device}")
        x0p = ctypes.c_void_p(x0.data_ptr()) if x0 is not None else ctypes.c_void_p()
        if x0 is not None:
            self._check_block(x0)
        stats = _Stats()
        st = lib.iwfpm_eigs(self._h, ctypes.byref(o), x0p, _ptr(evals, ctypes.c_double),
                            ctypes.c_void_p(vecs.data_ptr()) if vecs is not None else ctypes.c_void_p(),
                            _ptr(eta, ctypes.c_double), ctypes.byref(stats), _stream_handle(stream))
        if st != 0 and not (allow_noconv and st == -8):
            raise IwfpmError(st, "iwfpm_eigs")
        return EigsResult(evals, vecs, eta, stats.iterations, stats.matvecs, stats.converged, stats.restarts,
                          stats.fallback, stats.polished, stats.t_total, stats.t_apply, st)
