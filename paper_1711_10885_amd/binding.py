"""ctypes binding of libdgmf (the C ABI of include/dg.h).

Argument marshalling only: every step of the operator and the solvers runs in
the HIP library.  torch supplies device memory and streams.  If the library is
not built, ``load()`` raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgmf.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_ENOTCONV, DG_ENAN, DG_EIO = 0, -1, -2, -3, -4, -5, -6
DG_WITH_BLOCK_JACOBI = 2
DG_PERIODIC_X, DG_PERIODIC_Y, DG_PERIODIC_Z = 4, 8, 16
DG_B_PRODUCT = 32
DG_KAPPA_POLY = 64
DG_AFFINE = 128
DG_MULTILINEAR = 256
DG_KERNEL_AUTO, DG_KERNEL_REFERENCE = 0, 1
DG_GMRES64, DG_GMRES_IR, DG_FGMRES = 0, 1, 2
DG_PREC_NONE, DG_PREC_BLOCK_JACOBI, DG_PREC_LEARNED = 0, 1, 2
DG_ORTH_CGS1, DG_ORTH_CGS2 = 0, 1

_STATUS = {DG_EINVAL: "DG_EINVAL", DG_ENOMEM: "DG_ENOMEM", DG_EHIP: "DG_EHIP",
           DG_ENOTCONV: "DG_ENOTCONV", DG_ENAN: "DG_ENAN", DG_EIO: "DG_EIO"}

# every symbol include/dg.h declares
EXPORTS = ["dg_setup", "dg_apply", "dg_apply_f32", "dg_load_vector", "dg_project_gaussian", "dg_set_kernel", "dg_solve", "dg_precond_apply",
           "dg_learned_train", "dg_learned_nparams", "dg_learned_set_params", "dg_learned_get_params",
           "dg_learned_save", "dg_learned_load",
           "dg_mlp_forward", "dg_mlp_grad", "dg_mlp_step", "dg_heun", "dg_heun_noalloc", "dg_ndof", "dg_degree", "dg_bj_nblocks",
           "dg_last_error", "dg_destroy"]


class DGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [
        ("ncell", ctypes.c_int32 * 3),
        ("nodes", ctypes.POINTER(ctypes.c_double) * 3),
        ("k", ctypes.c_int32),
        ("K", ctypes.c_double * 9),
        ("kappa", ctypes.POINTER(ctypes.c_double)),
        ("b_const", ctypes.c_double * 3),
        ("b_sin", ctypes.c_double * 3),
        ("b_axis", ctypes.c_int32 * 3),
        ("c", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("flags", ctypes.c_int32),
        ("b_amp", ctypes.c_double * 3),
        ("b_freq", ctypes.c_double * 9),
        ("b_phase", ctypes.c_double * 9),
        ("kappa_poly", ctypes.c_double * 9),
        ("quad_extra", ctypes.c_int32),
        ("affine", ctypes.c_double * 9),
        ("vertices", ctypes.POINTER(ctypes.c_double)),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precond", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("orth", ctypes.c_int32), ("inner_tol", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer", ctypes.c_int32), ("applies", ctypes.c_int32),
                ("applies_f32", ctypes.c_int32), ("fallback_used", ctypes.c_int32),
                ("fallback_step", ctypes.c_int32), ("fallback_cycle", ctypes.c_int32),
                ("fallback_resid", ctypes.c_double), ("rel_resid", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LearnOpts(ctypes.Structure):
    _fields_ = [("npairs", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("epochs", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("max_steps", ctypes.c_int32)]


class LearnStats(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("steps", ctypes.c_int32), ("train_loss", ctypes.c_double),
                ("val_loss", ctypes.c_double), ("val_loss_initial", ctypes.c_double),
                ("seconds", ctypes.c_double), ("seconds_data", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Open libdgmf.so.  Raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() "
                           "(the HIP library is the only compute path)")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    H = ctypes.c_void_p
    lib.dg_setup.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(H)]
    lib.dg_setup.restype = ctypes.c_int
    lib.dg_apply.argtypes = [H, vp, vp, vp]
    lib.dg_apply.restype = ctypes.c_int
    lib.dg_load_vector.argtypes = [H, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int32), vp, vp]
    lib.dg_load_vector.restype = ctypes.c_int
    lib.dg_project_gaussian.argtypes = [H, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp, vp]
    lib.dg_project_gaussian.restype = ctypes.c_int
    lib.dg_heun.argtypes = [H, vp, vp, ctypes.c_double, ctypes.c_int32, vp]
    lib.dg_heun.restype = ctypes.c_int
    lib.dg_heun_noalloc.argtypes = [H, vp, vp, ctypes.c_double, ctypes.c_int32, vp]
    lib.dg_heun_noalloc.restype = ctypes.c_int
    lib.dg_apply_f32.argtypes = [H, vp, vp, vp]
    lib.dg_apply_f32.restype = ctypes.c_int
    lib.dg_set_kernel.argtypes = [H, ctypes.c_int32]
    lib.dg_set_kernel.restype = ctypes.c_int
    lib.dg_solve.argtypes = [H, vp, vp, ctypes.c_double, ctypes.POINTER(SolveOpts),
                             ctypes.POINTER(SolveStats), vp]
    lib.dg_solve.restype = ctypes.c_int
    lib.dg_precond_apply.argtypes = [H, ctypes.c_int32, vp, vp, vp]
    lib.dg_precond_apply.restype = ctypes.c_int
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.dg_learned_train.argtypes = [H, ctypes.POINTER(LearnOpts), ctypes.POINTER(LearnStats), vp]
    lib.dg_learned_train.restype = ctypes.c_int
    lib.dg_learned_nparams.argtypes = [H]
    lib.dg_learned_nparams.restype = ctypes.c_int64
    lib.dg_learned_set_params.argtypes = [H, fp, ctypes.c_int64]
    lib.dg_learned_set_params.restype = ctypes.c_int
    lib.dg_learned_get_params.argtypes = [H, fp, ctypes.c_int64]
    lib.dg_learned_save.argtypes = [H, ctypes.c_char_p]
    lib.dg_learned_save.restype = ctypes.c_int
    lib.dg_learned_load.argtypes = [H, ctypes.c_char_p]
    lib.dg_learned_load.restype = ctypes.c_int
    lib.dg_learned_get_params.restype = ctypes.c_int
    lib.dg_mlp_forward.argtypes = [H, vp, ctypes.c_int32, vp, vp]
    lib.dg_mlp_forward.restype = ctypes.c_int
    lib.dg_mlp_grad.argtypes = [H, vp, vp, ctypes.c_int32, fp, ctypes.c_int64, dp, vp]
    lib.dg_mlp_grad.restype = ctypes.c_int
    lib.dg_mlp_step.argtypes = [H, vp, vp, ctypes.c_int32, ctypes.c_float, dp, vp]
    lib.dg_mlp_step.restype = ctypes.c_int
    lib.dg_ndof.argtypes = [H]
    lib.dg_ndof.restype = ctypes.c_int64
    lib.dg_degree.argtypes = [H]
    lib.dg_degree.restype = ctypes.c_int32
    lib.dg_bj_nblocks.argtypes = [H]
    lib.dg_bj_nblocks.restype = ctypes.c_int64
    lib.dg_last_error.argtypes = []
    lib.dg_last_error.restype = ctypes.c_char_p
    lib.dg_destroy.argtypes = [H]
    lib.dg_destroy.restype = None
    _lib = lib
    return lib


def _check(rc: int):
    if rc != DG_OK:
        raise DGError(rc, load().dg_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_vec(t, n, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} entries")


def _check_rows(t, ncols, name, B=None):
    """Rows for the network entry points: a contiguous float32 tensor of
    shape (B, ncols), B a positive multiple of 64 (and equal to B if given);
    _check_on_gpu then checks the device.  Both run before any pointer
    reaches the library, whose kernels read B x ncols floats from it."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.dim() != 2 or t.shape[1] != ncols:
        raise ValueError(f"{name} must have shape (B, {ncols})")
    rows = int(t.shape[0])
    if rows < 64 or rows % 64:
        raise ValueError(f"{name}: B = {rows} rows, must be a positive multiple of 64")
    if B is not None and rows != B:
        raise ValueError(f"{name} must have {B} rows")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return rows


def _check_on_gpu(*named):
    for t, name in named:
        if t.device.type != "cuda":
            raise ValueError(f"{name} must live on the GPU")


class DG:
    """Handle on one problem (mesh, degree, coefficients) on the current GPU."""

    def __init__(self, prob, flags: int = 0):
        lib = load()
        import torch
        torch.cuda.current_device()  # make sure the device context exists
        self._keep = [np.ascontiguousarray(prob.nodes[a], dtype=np.float64) for a in range(3)]
        kap = None if prob.kappa is None else np.ascontiguousarray(prob.kappa, dtype=np.float64).ravel()
        self._keep.append(kap)
        s = _Problem()
        for a in range(3):
            s.ncell[a] = int(prob.ncell[a])
            s.nodes[a] = _dptr(self._keep[a])
            s.b_const[a] = float(prob.b_const[a])
            s.b_sin[a] = float(prob.b_sin[a])
            s.b_axis[a] = int(prob.b_axis[a])
        s.k = int(prob.k)
        K = np.asarray(prob.K, dtype=np.float64).reshape(9)
        for i in range(9):
            s.K[i] = float(K[i])
        s.kappa = _dptr(kap) if kap is not None else ctypes.POINTER(ctypes.c_double)()
        s.c = float(prob.c)
        s.sigma = float(prob.sigma)
        per = getattr(prob, "periodic", (False, False, False))
        s.flags = int(flags) | sum(DG_PERIODIC_X << a for a in range(3) if per[a])
        amp = getattr(prob, "b_amp", None)
        if amp is not None:
            s.flags |= DG_B_PRODUCT
            for r in range(3):
                s.b_amp[r] = float(amp[r])
            for t in range(9):
                s.b_freq[t] = float(prob.b_freq[t])
                s.b_phase[t] = float(prob.b_phase[t])
        s.quad_extra = int(getattr(prob, "quad_extra", 0))
        aff = getattr(prob, "affine", None)
        if aff is not None:
            s.flags |= DG_AFFINE
            for i, v in enumerate(np.asarray(aff, dtype=np.float64).ravel()):
                s.affine[i] = float(v)
        kpoly = getattr(prob, "kappa_poly", None)
        if kpoly is not None:
            s.flags |= DG_KAPPA_POLY
            for t in range(9):
                s.kappa_poly[t] = float(kpoly[t])
        verts = getattr(prob, "vertices", None)
        if verts is not None:
            V = np.ascontiguousarray(verts, dtype=np.float64).ravel()
            if V.size != 3 * int(np.prod([prob.ncell[a] + 1 for a in range(3)])):
                raise ValueError("vertices must hold (N1+1)(N2+1)(N3+1) points")
            self._keep.append(V)
            s.flags |= DG_MULTILINEAR
            s.vertices = _dptr(V)
        h = ctypes.c_void_p()
        _check(lib.dg_setup(ctypes.byref(s), ctypes.byref(h)))
        self._h = h
        self.prob = prob
        self.ndof = int(lib.dg_ndof(h))
        self.k = int(lib.dg_degree(h))

    def close(self):
        if getattr(self, "_h", None):
            load().dg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_kernel(self, variant: int):
        _check(load().dg_set_kernel(self._h, int(variant)))

    def apply(self, x, y=None, stream=None):
        """y := A x on the GPU (float64, cell-block layout of include/dg.h)."""
        import torch
        _check_vec(x, self.ndof, torch.float64, "x")
        if y is None:
            y = torch.empty_like(x)
        _check_vec(y, self.ndof, torch.float64, "y")
        _check(load().dg_apply(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                               _stream_ptr(stream)))
        return y

    def load_vector(self, terms, f=None, stream=None):
        """Load vector of a separable source: terms = [(alpha, (kind1, kind2,
        kind3)), ...], kind 0 = 1, 1 = sin(pi .), 2 = cos(pi .)."""
        import torch
        alpha = np.ascontiguousarray([t[0] for t in terms], dtype=np.float64)
        kinds = np.ascontiguousarray([t[1] for t in terms], dtype=np.int32).reshape(-1)
        if f is None:
            f = torch.empty(self.ndof, dtype=torch.float64, device="cuda")
        _check_vec(f, self.ndof, torch.float64, "f")
        _check(load().dg_load_vector(self._h, int(alpha.size), alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     kinds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     ctypes.c_void_p(f.data_ptr()), _stream_ptr(stream)))
        return f

    def project_gaussian(self, amp: float, width: float, center, u=None, stream=None):
        """L2 projection of amp exp(-width |x - center|^2) onto the DG space."""
        import torch
        c = np.ascontiguousarray(center, dtype=np.float64).reshape(3)
        if u is None:
            u = torch.empty(self.ndof, dtype=torch.float64, device="cuda")
        _check_vec(u, self.ndof, torch.float64, "u")
        _check(load().dg_project_gaussian(self._h, float(amp), float(width), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          ctypes.c_void_p(u.data_ptr()), _stream_ptr(stream)))
        return u

    def apply_f32(self, x, y=None, stream=None):
        """y := A x with FP32 vectors (mixed-precision operator)."""
        import torch
        _check_vec(x, self.ndof, torch.float32, "x")
        if y is None:
            y = torch.empty_like(x)
        _check_vec(y, self.ndof, torch.float32, "y")
        _check(load().dg_apply_f32(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   _stream_ptr(stream)))
        return y

    def heun(self, u, dt: float, nsteps: int, f=None, stream=None):
        """Advance u (float64 device tensor, in place) by nsteps Heun steps of
        M du/dt + A u = f (f = 0 if None); returns u."""
        import torch
        _check_vec(u, self.ndof, torch.float64, "u")
        fp = ctypes.c_void_p()
        if f is not None:
            _check_vec(f, self.ndof, torch.float64, "f")
            fp = ctypes.c_void_p(f.data_ptr())
        _check(load().dg_heun(self._h, ctypes.c_void_p(u.data_ptr()), fp, float(dt), int(nsteps),
                              _stream_ptr(stream)))
        return u

    def heun_noalloc(self, u, dt: float, nsteps: int, f=None, stream=None):
        """heun() through dg_heun_noalloc: the stage workspace is the library's
        fixed per-device array, nothing is allocated."""
        import torch
        _check_vec(u, self.ndof, torch.float64, "u")
        fp = ctypes.c_void_p()
        if f is not None:
            _check_vec(f, self.ndof, torch.float64, "f")
            fp = ctypes.c_void_p(f.data_ptr())
        _check(load().dg_heun_noalloc(self._h, ctypes.c_void_p(u.data_ptr()), fp, float(dt), int(nsteps),
                                      _stream_ptr(stream)))
        return u

    def bj_nblocks(self) -> int:
        """Inverse cell blocks stored by block Jacobi (ncells, or fewer when shared)."""
        return int(load().dg_bj_nblocks(self._h))

    def precond_apply(self, r, z=None, precond: int = DG_PREC_BLOCK_JACOBI, stream=None):
        """z := M^{-1} r for the handle's preconditioner (float64 device tensors)."""
        import torch
        _check_vec(r, self.ndof, torch.float64, "r")
        if z is None:
            z = torch.empty_like(r)
        _check_vec(z, self.ndof, torch.float64, "z")
        _check(load().dg_precond_apply(self._h, int(precond), ctypes.c_void_p(r.data_ptr()),
                                       ctypes.c_void_p(z.data_ptr()), _stream_ptr(stream)))
        return z

    def solve(self, f, u=None, tol: float = 1e-8, method: int = DG_GMRES64,
              precond: int = DG_PREC_NONE, restart: int = 30, maxit: int = 20000,
              inner_tol: float = 1e-4, orth: int = 0, stream=None, check: bool = True):
        """Solve A u = f (float64 device tensors); u is the initial guess (zero
        if None).  Returns (u, stats dict, status).  With check=True a status
        other than DG_OK raises DGError."""
        import torch
        _check_vec(f, self.ndof, torch.float64, "f")
        if u is None:
            u = torch.zeros_like(f)
        _check_vec(u, self.ndof, torch.float64, "u")
        o = SolveOpts(int(method), int(precond), int(restart), int(maxit), int(orth), float(inner_tol))
        st = SolveStats()
        rc = load().dg_solve(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                             float(tol), ctypes.byref(o), ctypes.byref(st), _stream_ptr(stream))
        if check:
            _check(rc)
        return u, st.as_dict(), rc

    # ---- learned preconditioner -------------------------------------------
    def learned_nparams(self) -> int:
        return int(load().dg_learned_nparams(self._h))

    def learned_train(self, npairs=100000, nrhs=8, epochs=20, batch=1024, lr=1e-3, seed=6, max_steps=0,
                      stream=None):
        """Train the cell-patch network on the GPU; returns the stats dict."""
        o = LearnOpts(int(npairs), int(nrhs), int(epochs), int(batch), float(lr), int(seed), int(max_steps))
        st = LearnStats()
        _check(load().dg_learned_train(self._h, ctypes.byref(o), ctypes.byref(st), _stream_ptr(stream)))
        return st.as_dict()

    def learned_set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(load().dg_learned_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            int(p.size)))

    def learned_get_params(self) -> np.ndarray:
        n = self.learned_nparams()
        p = np.empty(n, dtype=np.float32)
        _check(load().dg_learned_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n))
        return p

    def learned_save(self, path: str):
        """Checkpoint of the network, its Adam moments and step count."""
        _check(load().dg_learned_save(self._h, os.fsencode(path)))

    def learned_load(self, path: str):
        """Restore a checkpoint written by learned_save (same degree)."""
        _check(load().dg_learned_load(self._h, os.fsencode(path)))

    def mlp_forward(self, X, stream=None):
        """Network outputs for rows X (float32 device tensor, B x in)."""
        import torch
        B = _check_rows(X, 7 * self.k_nb(), "X")
        _check_on_gpu((X, "X"))
        Y = torch.empty((B, self.k_nb()), dtype=torch.float32, device=X.device)
        _check(load().dg_mlp_forward(self._h, ctypes.c_void_p(X.data_ptr()), int(B),
                                     ctypes.c_void_p(Y.data_ptr()), _stream_ptr(stream)))
        return Y

    def mlp_grad(self, X, T, stream=None):
        """(loss, gradient in the public parameter layout) for rows X, targets T."""
        B = _check_rows(X, 7 * self.k_nb(), "X")
        _check_rows(T, self.k_nb(), "T", B)
        _check_on_gpu((X, "X"), (T, "T"))
        n = self.learned_nparams()
        g = np.empty(n, dtype=np.float32)
        loss = ctypes.c_double()
        _check(load().dg_mlp_grad(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                  B, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n,
                                  ctypes.byref(loss), _stream_ptr(stream)))
        return loss.value, g

    def mlp_step(self, X, T, lr=1e-3, stream=None):
        B = _check_rows(X, 7 * self.k_nb(), "X")
        _check_rows(T, self.k_nb(), "T", B)
        _check_on_gpu((X, "X"), (T, "T"))
        loss = ctypes.c_double()
        _check(load().dg_mlp_step(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                  B, float(lr), ctypes.byref(loss), _stream_ptr(stream)))
        return loss.value

    def k_nb(self) -> int:
        return (self.k + 1) ** 3
