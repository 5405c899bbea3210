"""CPU oracle for the weighted SIPG convection-diffusion-reaction operator of
Muething, Piatkowski & Bastian, "High-performance Implementation of
Matrix-free High-order Discontinuous Galerkin Methods" (arXiv 1711.10885).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the HIP path; both sides receive the same plain arrays from the
seeded input generators.

Contents
--------
* ``apply`` / ``apply_rows`` -- y = A x of eq. (blf), Sec. 2.2, by the plain
  quadrature definition (C, ``dg_oracle.c``), Algorithm 1 of Sec. 3.6 order.
* ``rhs`` / ``l2err`` -- load vector (f, phi_j) of the right-hand-side
  functional (Sec. 2.2, g = 0) and the L2 error of a coefficient vector.
* ``project_gaussian`` -- L2 projection of a Gaussian (the initial
  concentration of the transport example, Sec. 5.4).
* ``gauss`` / ``basis`` -- the 1D Gauss rule and orthonormal Legendre basis
  (Sec. 3.1; the L2-orthogonal Legendre basis of Sec. 2.2, normalised).
* ``assemble`` -- the sparse matrix of the operator by probing ``apply`` with
  coloured unit vectors (the DG coupling is face-local, Sec. 2.2).
* ``block_diagonal`` -- the per-cell diagonal blocks A_TT of the same operator.
* ``cell_volumes`` / ``heun`` / ``heun_step_rows`` -- explicit Heun time
  stepping of M du/dt + A u = f (Sec. 2.2, Sec. 5.4) with the diagonal mass
  matrix of the orthonormal basis; the last evaluates one step on listed
  cells only (for checks on meshes too large to step whole).
* ``gmres`` -- restarted, right-preconditioned GMRES in float64 (numpy).

Meshes: tensor grids of per-axis nodes (optionally one global affine image),
or, with ``prob.vertices``, logically structured meshes of trilinear cells
through the given vertices (multilinear geometry, Sec. 4 and Problem C of
Sec. 5.1), where every geometric quantity is evaluated at each quadrature
point.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libdg_oracle.so")

VOLUME, INTERIOR, BOUNDARY = 1, 2, 4
ALL_TERMS = VOLUME | INTERIOR | BOUNDARY


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no intrinsics)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-D_GNU_SOURCE",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


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
        ("periodic", ctypes.c_int32 * 3),
        ("b_product", ctypes.c_int32),
        ("b_amp", ctypes.c_double * 3),
        ("b_freq", ctypes.c_double * 9),
        ("b_phase", ctypes.c_double * 9),
        ("kappa_poly_on", ctypes.c_int32),
        ("kappa_poly", ctypes.c_double * 9),
        ("quad_extra", ctypes.c_int32),
        ("affine_on", ctypes.c_int32),
        ("affine", ctypes.c_double * 9),
        ("multilinear_on", ctypes.c_int32),
        ("vertices", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_apply.argtypes = [P, dp, dp, ctypes.c_int, ctypes.c_int]
        lib.oracle_apply_rows.argtypes = [P, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                          dp, ctypes.c_int, ctypes.c_int]
        lib.oracle_rhs.argtypes = [P, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int32), dp,
                                   ctypes.c_int]
        lib.oracle_project_gaussian.argtypes = [P, ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int]
        lib.oracle_l2err2.argtypes = [P, dp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_l2err2.restype = ctypes.c_double
        lib.oracle_gauss.argtypes = [ctypes.c_int, dp, dp]
        lib.oracle_basis.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        lib.oracle_ndof.argtypes = [P]
        lib.oracle_ndof.restype = ctypes.c_int64
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Marshalled:
    """Keeps the numpy arrays referenced by a _Problem alive."""

    def __init__(self, prob):
        self.nodes = [np.ascontiguousarray(prob.nodes[a], dtype=np.float64) for a in range(3)]
        self.kappa = (None if prob.kappa is None
                      else np.ascontiguousarray(prob.kappa, dtype=np.float64).ravel())
        s = _Problem()
        for a in range(3):
            s.ncell[a] = int(prob.ncell[a])
            s.nodes[a] = _dptr(self.nodes[a])
            s.b_const[a] = float(prob.b_const[a])
            s.b_sin[a] = float(prob.b_sin[a])
            s.b_axis[a] = int(prob.b_axis[a])
        s.k = int(prob.k)
        K = np.asarray(prob.K, dtype=np.float64).reshape(9)
        for i in range(9):
            s.K[i] = float(K[i])
        s.kappa = _dptr(self.kappa) if self.kappa is not None else ctypes.POINTER(ctypes.c_double)()
        s.c = float(prob.c)
        s.sigma = float(prob.sigma)
        per = getattr(prob, "periodic", (False, False, False))
        for a in range(3):
            s.periodic[a] = 1 if per[a] else 0
        amp = getattr(prob, "b_amp", None)
        s.b_product = 0 if amp is None else 1
        if amp is not None:
            for r in range(3):
                s.b_amp[r] = float(amp[r])
            for t in range(9):
                s.b_freq[t] = float(prob.b_freq[t])
                s.b_phase[t] = float(prob.b_phase[t])
        kpoly = getattr(prob, "kappa_poly", None)
        s.kappa_poly_on = 0 if kpoly is None else 1
        if kpoly is not None:
            for t in range(9):
                s.kappa_poly[t] = float(kpoly[t])
        s.quad_extra = int(getattr(prob, "quad_extra", 0))
        A = getattr(prob, "affine", None)
        s.affine_on = 0 if A is None else 1
        if A is not None:
            for i, v in enumerate(np.asarray(A, dtype=np.float64).ravel()):
                s.affine[i] = float(v)
        V = getattr(prob, "vertices", None)
        s.multilinear_on = 0 if V is None else 1
        self.vertices = None if V is None else np.ascontiguousarray(V, dtype=np.float64).ravel()
        if V is not None:
            if self.vertices.size != 3 * np.prod([prob.ncell[a] + 1 for a in range(3)]):
                raise ValueError("vertices must hold (N1+1)(N2+1)(N3+1) points")
            s.vertices = _dptr(self.vertices)
        self.struct = s


def default_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def ndof(prob) -> int:
    n = prob.k + 1
    return int(prob.ncell[0] * prob.ncell[1] * prob.ncell[2] * n ** 3)


def apply(prob, x: np.ndarray, terms: int = ALL_TERMS, nthreads: int | None = None) -> np.ndarray:
    """y = A x (eq. (blf) with tensor Gauss quadrature, Algorithm 1)."""
    lib = _load()
    m = _Marshalled(prob)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.size != ndof(prob):
        raise ValueError("x has wrong size")
    y = np.empty_like(x)
    rc = lib.oracle_apply(ctypes.byref(m.struct), _dptr(x), _dptr(y), int(terms),
                          int(nthreads or default_threads()))
    if rc != 0:
        raise ValueError("oracle_apply rejected the problem")
    return y


def apply_rows(prob, x: np.ndarray, cells, terms: int = ALL_TERMS,
               nthreads: int | None = None) -> np.ndarray:
    """Rows of A x for the listed cells; shape (len(cells), n^3)."""
    lib = _load()
    m = _Marshalled(prob)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.size != ndof(prob):
        raise ValueError("x has wrong size")
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    nb = (prob.k + 1) ** 3
    y = np.empty((cells.size, nb), dtype=np.float64)
    rc = lib.oracle_apply_rows(ctypes.byref(m.struct), _dptr(x),
                               cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               int(cells.size), _dptr(y), int(terms),
                               int(nthreads or default_threads()))
    if rc != 0:
        raise ValueError("oracle_apply_rows rejected its arguments")
    return y


def _terms(terms):
    alpha = np.ascontiguousarray([t[0] for t in terms], dtype=np.float64)
    kinds = np.ascontiguousarray([t[1] for t in terms], dtype=np.int32).reshape(-1, 3)
    return alpha, kinds


def rhs(prob, source_terms, nthreads: int | None = None) -> np.ndarray:
    """Load vector f_{T,j} = (f, phi_j)_T for f = sum alpha * g1(x) g2(y) g3(z)."""
    lib = _load()
    m = _Marshalled(prob)
    alpha, kinds = _terms(source_terms)
    f = np.empty(ndof(prob), dtype=np.float64)
    rc = lib.oracle_rhs(ctypes.byref(m.struct), int(alpha.size), _dptr(alpha),
                        kinds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(f),
                        int(nthreads or default_threads()))
    if rc != 0:
        raise ValueError("oracle_rhs rejected the problem")
    return f


def project_gaussian(prob, amp: float, width: float, center, nthreads: int | None = None) -> np.ndarray:
    """L2 projection of amp exp(-width |x - center|^2) onto the DG space
    (coefficients (g, phi_j)_T / |T| by the operator's Gauss rule)."""
    lib = _load()
    m = _Marshalled(prob)
    c = np.ascontiguousarray(center, dtype=np.float64).reshape(3)
    u = np.empty(ndof(prob), dtype=np.float64)
    rc = lib.oracle_project_gaussian(ctypes.byref(m.struct), float(amp), float(width), _dptr(c), _dptr(u),
                                     int(nthreads or default_threads()))
    if rc != 0:
        raise ValueError("oracle_project_gaussian rejected the problem")
    return u


def l2err(prob, x: np.ndarray, exact_terms) -> float:
    lib = _load()
    m = _Marshalled(prob)
    alpha, kinds = _terms(exact_terms)
    x = np.ascontiguousarray(x, dtype=np.float64)
    e2 = lib.oracle_l2err2(ctypes.byref(m.struct), _dptr(x), int(alpha.size), _dptr(alpha),
                           kinds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), )
    return float(np.sqrt(e2))


def gauss(m: int):
    lib = _load()
    xi = np.empty(m)
    w = np.empty(m)
    if lib.oracle_gauss(int(m), _dptr(xi), _dptr(w)) != 0:
        raise ValueError("bad m")
    return xi, w


def basis(k: int, t: float):
    lib = _load()
    v = np.empty(k + 1)
    d = np.empty(k + 1)
    lib.oracle_basis(int(k), float(t), _dptr(v), _dptr(d))
    return v, d


def _cell_colours(prob):
    """Colour of each cell, per axis i_a mod C_a with C_a = 3 (or, on a
    periodic axis whose length is not a multiple of 3, C_a = ncell[a]): cells
    of one colour are at least three cells apart along every axis, also
    across a periodic boundary, so probing one colour at a time separates
    the columns of every face-coupled pair."""
    per = getattr(prob, "periodic", (False, False, False))
    C = [prob.ncell[a] if per[a] and prob.ncell[a] % 3 else 3 for a in range(3)]
    N1, N2, N3 = prob.ncell
    i1, i2, i3 = np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3), indexing="ij")
    col = (i1 % C[0]) + C[0] * ((i2 % C[1]) + C[1] * (i3 % C[2]))
    return col.transpose(2, 1, 0).ravel(), C[0] * C[1] * C[2]  # cell id order: axis 1 fastest


def assemble(prob, terms: int = ALL_TERMS, nthreads: int | None = None):
    """Sparse matrix of the operator, column by column from ``apply``.

    Column (T, j) of A is supported on T and its face neighbours (across a
    periodic boundary too).  All cells of one colour are probed with e_j at
    once; the rows of each probed cell's neighbourhood are then attributed to
    it unambiguously (each distinct neighbour once)."""
    import scipy.sparse as sp

    nb = (prob.k + 1) ** 3
    N1, N2, N3 = prob.ncell
    Nv = np.array([N1, N2, N3])
    per = np.array(getattr(prob, "periodic", (False, False, False)), dtype=bool)
    ncells = N1 * N2 * N3
    col, ncol = _cell_colours(prob)
    cid = np.arange(ncells)
    ci = np.stack([cid % N1, (cid // N1) % N2, cid // (N1 * N2)], axis=1)
    # distinct cells of each cell's neighbourhood (itself and its face neighbours)
    offs = ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))
    hood = []
    for c in range(ncells):
        cells = set()
        for d in offs:
            q = ci[c] + np.array(d)
            q = np.where(per, q % Nv, q)
            if np.all((q >= 0) & (q < Nv)):
                cells.add(int(q[0] + N1 * (q[1] + N2 * q[2])))
        hood.append(sorted(cells))
    rows_all, cols_all, vals_all = [], [], []
    for colour in range(ncol):
        probed = np.nonzero(col == colour)[0]
        if probed.size == 0:
            continue
        for j in range(nb):
            x = np.zeros(ncells * nb)
            x[probed * nb + j] = 1.0
            y = apply(prob, x, terms, nthreads).reshape(ncells, nb)
            src = np.concatenate([np.full(len(hood[c]), c) for c in probed])
            dst = np.concatenate([np.array(hood[c], dtype=np.int64) for c in probed])
            blk = y[dst]  # (len, nb)
            r = (dst[:, None] * nb + np.arange(nb)[None, :]).ravel()
            c = np.repeat(src * nb + j, nb)
            v = blk.ravel()
            nz = v != 0.0
            rows_all.append(r[nz])
            cols_all.append(c[nz])
            vals_all.append(v[nz])
    n = ncells * nb
    return sp.csr_matrix((np.concatenate(vals_all), (np.concatenate(rows_all),
                                                     np.concatenate(cols_all))), shape=(n, n))


def cell_volumes(prob) -> np.ndarray:
    """|T| per cell (cell order: axis 1 fastest); |det A| times the tensor-grid
    volume on an affine mesh x = A xi."""
    h = [np.diff(np.asarray(prob.nodes[a], dtype=np.float64)) for a in range(3)]
    vol = np.einsum("k,j,i->kji", h[2], h[1], h[0]).ravel()
    A = getattr(prob, "affine", None)
    return vol if A is None else vol * abs(np.linalg.det(np.asarray(A, dtype=np.float64)))


def heun(prob, u0: np.ndarray, dt: float, nsteps: int, f: np.ndarray | None = None,
         nthreads: int | None = None) -> np.ndarray:
    """Explicit two-stage strong-stability-preserving Runge-Kutta (Heun) for
    the semi-discrete system M du/dt + A u = f of Sec. 2.2 (eq.
    (ODE_system)), the time stepping of the paper's transport example
    (Sec. 5.4).  The orthonormal basis gives M = |T| I on cell T:
        k1 = M^{-1} (f - A u),  u1 = u + dt k1,
        k2 = M^{-1} (f - A u1), u  <- u + dt (k1 + k2) / 2."""
    nb = (prob.k + 1) ** 3
    minv = np.repeat(1.0 / cell_volumes(prob), nb)
    rhs = 0.0 if f is None else np.asarray(f, dtype=np.float64)
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        k1 = minv * (rhs - apply(prob, u, ALL_TERMS, nthreads))
        u1 = u + dt * k1
        k2 = minv * (rhs - apply(prob, u1, ALL_TERMS, nthreads))
        u = u + 0.5 * dt * (k1 + k2)
    return u


def face_neighbours(prob, cell: int) -> list:
    """Cells sharing a face with ``cell`` (periodic axes wrap; a cell that
    would be its own neighbour, one cell along a periodic axis, is left out)."""
    n = [int(v) for v in prob.ncell]
    i = [cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])]
    per = tuple(getattr(prob, "periodic", (False, False, False)))
    out = set()
    for a in range(3):
        for d in (-1, 1):
            j = list(i)
            j[a] += d
            if not 0 <= j[a] < n[a]:
                if not per[a]:
                    continue
                j[a] %= n[a]
            c = j[0] + n[0] * (j[1] + n[1] * j[2])
            if c != cell:
                out.add(c)
    return sorted(out)


def heun_step_rows(prob, u: np.ndarray, dt: float, cells, f: np.ndarray | None = None,
                   nthreads: int | None = None) -> np.ndarray:
    """One step of ``heun`` evaluated on the listed cells only; shape
    (len(cells), n^3).  A u1 on a cell reads u1 on that cell and its face
    neighbours (the operator couples face neighbours only, Sec. 2.2), and u1
    there needs A u on the same cells, so the step is exact from rows of A
    on the listed cells and their neighbours."""
    nb = (prob.k + 1) ** 3
    vol = cell_volumes(prob)
    cells = [int(c) for c in cells]
    near = sorted(set(cells).union(*[face_neighbours(prob, c) for c in cells]))
    u = np.asarray(u, dtype=np.float64)
    rows = lambda v, c: (0.0 if v is None else v[c * nb:(c + 1) * nb])
    Au = apply_rows(prob, u, near, ALL_TERMS, nthreads)
    u1 = np.zeros_like(u)
    k1 = {}
    for r, c in enumerate(near):
        k1[c] = (rows(f, c) - Au[r]) / vol[c]
        u1[c * nb:(c + 1) * nb] = u[c * nb:(c + 1) * nb] + dt * k1[c]
    Au1 = apply_rows(prob, u1, cells, ALL_TERMS, nthreads)
    out = np.empty((len(cells), nb))
    for r, c in enumerate(cells):
        k2 = (rows(f, c) - Au1[r]) / vol[c]
        out[r] = u[c * nb:(c + 1) * nb] + 0.5 * dt * (k1[c] + k2)
    return out


def block_diagonal(prob, nthreads: int | None = None) -> np.ndarray:
    """Diagonal blocks A_TT (ncells, n^3, n^3): a_h(phi_j, phi_i) for i, j in T.

    Face neighbours differ in exactly one index by one, so the two parity
    classes of i1+i2+i3 never touch: probing one class at a time with e_j
    leaves, in the rows of a probed cell, exactly column j of its block.
    (With a periodic axis of odd length the classes are per-axis colours.)"""
    nb = (prob.k + 1) ** 3
    N1, N2, N3 = prob.ncell
    ncells = N1 * N2 * N3
    cid = np.arange(ncells)
    idx = [cid % N1, (cid // N1) % N2, cid // (N1 * N2)]
    per = getattr(prob, "periodic", (False, False, False))
    odd = [per[a] and prob.ncell[a] > 1 and prob.ncell[a] % 2 == 1 for a in range(3)]
    if any(odd):
        # a periodic axis of odd length joins the first and last cells, which
        # share a parity: colour each axis by parity, the last cell apart
        col = [np.where((idx[a] == prob.ncell[a] - 1) & odd[a], 2, idx[a] % 2) for a in range(3)]
        par = col[0] + 3 * col[1] + 9 * col[2]
    else:
        par = (idx[0] + idx[1] + idx[2]) % 2
    B = np.zeros((ncells, nb, nb))
    for p in np.unique(par):
        probed = np.nonzero(par == p)[0]
        for j in range(nb):
            x = np.zeros(ncells * nb)
            x[probed * nb + j] = 1.0
            y = apply(prob, x, ALL_TERMS, nthreads).reshape(ncells, nb)
            B[probed, :, j] = y[probed]
    return B


def gmres(matvec, b: np.ndarray, x0=None, tol: float = 1e-8, restart: int = 30,
          maxit: int = 10000, precond=None):
    """Restarted GMRES(restart) with right preconditioning, float64.

    Arnoldi with modified Gram-Schmidt and Givens rotations (Saad, Iterative
    Methods for Sparse Linear Systems, Alg. 6.9/9.5).  Stops when the true
    residual ||b - A x|| / ||b|| <= tol, checked at every restart.
    Returns (x, iterations, relative residual)."""
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    it = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or it >= maxit:
            return x, it, beta / bnorm
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j_done = 0
        for j in range(restart):
            z = M(V[j])
            Z.append(z)
            w = matvec(z)
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            if abs(g[j + 1]) / bnorm <= tol or it >= maxit or hn == 0.0:
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        for i in range(j_done):
            x = x + y[i] * Z[i]
