"""Seeded synthetic inputs for the DG operator workloads.

This module only generates inputs (meshes, coefficients, vectors, manufactured
sources).  It contains none of the discretisation's arithmetic, imports
nothing from the HIP library or the oracle, and is the one module both of them
are fed from.  Every random array is drawn with ``numpy.random.default_rng``
(PCG64) from a fixed seed.

Workloads (sizes from the benchmark configuration, coefficients as read from
the paper's model problem, Sec. 2.1, and Problem A of Sec. 5.1):

* ``poisson_k2_8``   K = I, b = 0, c = 0, k = 2, 8^3 uniform cubes, penalty
  sigma = 3k(k+1) (gamma = sigma/h), x ~ U[-1, 1] seed 1 (13,824 DOF).
* ``cdr_k7_32``      k = 7, 32^3 tensor cuboids with per-axis spacings drawn
  U[0.5h, 1.5h] (seed 2) and rescaled to [0,1]; K = Q diag(1, 0.1, 0.01) Q^T,
  Q = Rz(pi/6) Ry(pi/4) Rx(pi/3); b = (sin pi y, sin pi z, sin pi x); c = 1;
  sigma = 2k(k+2); x ~ U[-1, 1] seed 3 (16,777,216 DOF).
* ``cdr_sweep(k)``   uniform N^3 cubes with N = round((2e7)^(1/3)/(k+1)),
  coefficients as ``cdr_k7_32``, x seed 300+k.
* ``mixed_k5_48``    k = 5, 48^3, K = I, b = (1, .5, .25), c = 0.1,
  sigma = 2k(k+2); source of the manufactured u = sin(pi x) sin(pi y) sin(pi z).
* ``learned_k3_64``  k = 3, 64^3, kappa_T = exp(g(center_T)), g a seeded smooth
  random field (random Fourier features, M = 128, length scale 0.1, seed 5),
  b = (1, .5, .25), c = 0.1, sigma = 2k(k+2), f = 1.
* ``transport_k5_64`` the transport example of Sec. 5.4 at one GPU's size:
  k = 5, 64^3 uniform cubes of the periodic box (-pi, pi)^3, K = 5e-6 I,
  c = 0, f = 0, the Taylor-Green flow field of that section (eq. (2)) in
  product form, sigma = 2k(k+2); initial concentration exp(-2 |x - x0|^2),
  x0 = (1/2, 0, 0), taken at the cell centres as the cell-constant mode.
* ``transport_paper_k5_64`` the same with the paper's rule q = 2p + 4 for the
  trigonometric flow field; the initial state is the L2 projection of the
  Gaussian (computed by the library and, for checks, by the oracle).
* ``problem_c(k)``, ``problem_b_cells(k)`` multilinear (trilinear) cells:
  a smoothly curved vertex grid of the unit cube with the rule q = 3p + 4,
  and a grid sheared layer by layer (affine cells with different
  Jacobians) with q = 2p + 4, about 4M DOF.

Problem fields beyond the model problem: ``periodic`` (per axis), the product-form
flow field ``b_amp``/``b_freq``/``b_phase``, the diffusion factor ``kappa_poly``
(per-axis quadratics), ``quad_extra`` (2: the rule q = 2p + 4) and ``affine``
(the mesh as the image x = A xi of the tensor grid).  ``random_problem`` draws
small problems of every kind for the tests; ``random_kappa_poly`` draws the
diffusion factor.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np


@dataclass
class Problem:
    ncell: tuple
    nodes: tuple  # three float64 arrays of length ncell[a]+1
    k: int
    K: np.ndarray  # (3,3) SPD
    kappa: np.ndarray | None = None  # per cell, axis-1 fastest
    b_const: tuple = (0.0, 0.0, 0.0)
    b_sin: tuple = (0.0, 0.0, 0.0)
    b_axis: tuple = (0, 1, 2)
    c: float = 0.0
    sigma: float = 1.0
    periodic: tuple = (False, False, False)  # per axis
    # product-form flow field b_r = b_amp[r] prod_j sin(b_freq[3r+j] x_j + b_phase[3r+j])
    # (factor 1 where b_freq is 0); replaces b_const/b_sin/b_axis when b_amp is set
    b_amp: tuple | None = None
    b_freq: tuple = (0.0,) * 9
    b_phase: tuple = (0.0,) * 9
    # polynomial diffusion factor: D(x) = kappa_T kp(x) K with
    # kp(x) = prod_j (c[3j] + c[3j+1] x_j + c[3j+2] x_j^2), c = kappa_poly (None: kp = 1)
    kappa_poly: tuple | None = None
    # Gauss points per direction m = k + 1 + quad_extra (2: the raised rule q = 2p + 4)
    quad_extra: int = 0
    # affine geometry: the mesh is x = A xi of the tensor grid xi of the nodes (None: A = I)
    affine: np.ndarray | None = None
    # multilinear geometry: vertex coordinates, shape (N3+1, N2+1, N1+1, 3) (axis 1 fastest);
    # cell (i1,i2,i3) is the trilinear image of [0,1]^3 through its eight vertices (None: the
    # tensor grid of the nodes)
    vertices: np.ndarray | None = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def ncells(self) -> int:
        return int(self.ncell[0] * self.ncell[1] * self.ncell[2])

    @property
    def ndof(self) -> int:
        return self.ncells * (self.k + 1) ** 3

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def uniform_nodes(N: int) -> np.ndarray:
    return np.linspace(0.0, 1.0, N + 1)


def random_nodes(N: int, rng, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """Spacings U[lo*h, hi*h], rescaled so the axis spans [0, 1]."""
    s = rng.uniform(lo, hi, N)
    nodes = np.concatenate([[0.0], np.cumsum(s)])
    nodes /= nodes[-1]
    nodes[-1] = 1.0
    return nodes


def _rot(axis: int, ang: float) -> np.ndarray:
    c, s = math.cos(ang), math.sin(ang)
    R = np.eye(3)
    i, j = [(1, 2), (0, 2), (0, 1)][axis]
    R[i, i] = c
    R[j, j] = c
    R[i, j] = -s if axis != 1 else s
    R[j, i] = s if axis != 1 else -s
    return R


def anisotropic_K(eigs=(1.0, 0.1, 0.01)) -> np.ndarray:
    """K = Q diag(eigs) Q^T with Q = Rz(pi/6) Ry(pi/4) Rx(pi/3): a full tensor."""
    Q = _rot(2, math.pi / 6) @ _rot(1, math.pi / 4) @ _rot(0, math.pi / 3)
    K = Q @ np.diag(eigs) @ Q.T
    return 0.5 * (K + K.T)


def random_spd(rng, lo: float = 0.2, hi: float = 2.0) -> np.ndarray:
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    K = Q @ np.diag(rng.uniform(lo, hi, 3)) @ Q.T
    return 0.5 * (K + K.T)


SINE_CYCLIC = dict(b_const=(0.0, 0.0, 0.0), b_sin=(1.0, 1.0, 1.0), b_axis=(1, 2, 0))

# Taylor-Green field of Sec. 5.4, eq. (2), as b_r = amp_r prod_j sin(freq x_j + phase):
#   b_1 = cos(x_1) sin(-x_2) sin(-x_3), b_2 = 1/2 sin(x_1) cos(-x_2) sin(-x_3),
#   b_3 = 1/2 sin(x_1) sin(-x_2) cos(-x_3)   (cos s = sin(s + pi/2))
TAYLOR_GREEN = dict(b_amp=(1.0, 0.5, 0.5),
                    b_freq=(1.0, -1.0, -1.0, 1.0, -1.0, -1.0, 1.0, -1.0, -1.0),
                    b_phase=(math.pi / 2, 0.0, 0.0, 0.0, math.pi / 2, 0.0, 0.0, 0.0, math.pi / 2))
TRANSPORT_DT_H = 0.01  # dt / h: rho(M^-1 A) h stays below 83 at k = 5, so dt rho < 0.83


def paper_sigma(k: int) -> float:
    """alpha * p (p + d - 1) with alpha = 2, d = 3 (penalty of Sec. 2.2)."""
    return 2.0 * k * (k + 2)


def poisson_k2_8() -> Problem:
    k, N = 2, 8
    return Problem(ncell=(N, N, N), nodes=(uniform_nodes(N),) * 3, k=k, K=np.eye(3),
                   sigma=3.0 * k * (k + 1), name="poisson_k2_8", meta={"x_seed": 1})


def cdr_k7_32(N: int = 32, k: int = 7) -> Problem:
    rng = np.random.default_rng(2)
    nodes = tuple(random_nodes(N, rng) for _ in range(3))
    return Problem(ncell=(N, N, N), nodes=nodes, k=k, K=anisotropic_K(), c=1.0,
                   sigma=paper_sigma(k), name=f"cdr_k{k}_{N}", meta={"x_seed": 3},
                   **SINE_CYCLIC)


def sweep_N(k: int) -> int:
    return int(round((2e7) ** (1.0 / 3.0) / (k + 1)))


def cdr_sweep(k: int) -> Problem:
    N = sweep_N(k)
    return Problem(ncell=(N, N, N), nodes=(uniform_nodes(N),) * 3, k=k, K=anisotropic_K(),
                   c=1.0, sigma=paper_sigma(k), name=f"cdr_sweep_k{k}_{N}",
                   meta={"x_seed": 300 + k}, **SINE_CYCLIC)


B_CONST = dict(b_const=(1.0, 0.5, 0.25), b_sin=(0.0, 0.0, 0.0), b_axis=(0, 1, 2))


def mixed_k5_48(N: int = 48, k: int = 5) -> Problem:
    return Problem(ncell=(N, N, N), nodes=(uniform_nodes(N),) * 3, k=k, K=np.eye(3), c=0.1,
                   sigma=paper_sigma(k), name=f"mixed_k{k}_{N}", **B_CONST)


def smooth_field(centers: np.ndarray, seed: int = 5, M: int = 128, ell: float = 0.1):
    """g(x) = sqrt(2/M) sum_j cos(w_j . x + phi_j), w_j ~ N(0, ell^-2 I),
    phi_j ~ U[0, 2 pi): a stationary Gaussian random field of unit variance."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((M, 3)) / ell
    ph = rng.uniform(0.0, 2.0 * math.pi, M)
    return math.sqrt(2.0 / M) * np.cos(centers @ w.T + ph[None, :]).sum(axis=1)


def cell_centers(nodes) -> np.ndarray:
    c = [0.5 * (nd[1:] + nd[:-1]) for nd in nodes]
    C3, C2, C1 = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    return np.stack([C1.ravel(), C2.ravel(), C3.ravel()], axis=1)  # axis-1 fastest


def learned_k3_64(N: int = 64, k: int = 3, log_sigma: float = 1.0) -> Problem:
    nodes = (uniform_nodes(N),) * 3
    kappa = np.exp(log_sigma * smooth_field(cell_centers(nodes)))
    return Problem(ncell=(N, N, N), nodes=nodes, k=k, K=np.eye(3), kappa=kappa, c=0.1,
                   sigma=paper_sigma(k), name=f"learned_k{k}_{N}", **B_CONST)


def random_problem(seed: int, ncell=(3, 2, 2), k: int = 2, b: str = "sine",
                   kappa: bool = True, c: float | None = None, periodic=(False, False, False)) -> Problem:
    """Small random problem: nonuniform tensor grid on [0,1]^3, random SPD K,
    random per-cell kappa, b constant or sine-cyclic, random c; optional
    periodic axes (b takes the same value at both ends of every axis)."""
    rng = np.random.default_rng(seed)
    nodes = tuple(random_nodes(ncell[a], rng) for a in range(3))
    K = random_spd(rng)
    kap = rng.uniform(0.3, 3.0, int(np.prod(ncell))) if kappa else None
    if b == "sine":
        bk = dict(b_const=tuple(rng.uniform(-0.5, 0.5, 3)), b_sin=tuple(rng.uniform(0.5, 2, 3)),
                  b_axis=(1, 2, 0))
    elif b == "product":  # random product-form field: every factor a sine of its coordinate
        bk = dict(b_amp=tuple(rng.uniform(-1.5, 1.5, 3)),
                  b_freq=tuple(rng.choice([-2.0, -1.0, 1.0, 3.0], 9) * math.pi),
                  b_phase=tuple(rng.uniform(0.0, 2.0 * math.pi, 9)))
    elif b == "product_sparse":  # some factors constant (frequency 0)
        fr = rng.choice([-2.0, -1.0, 1.0, 3.0], 9) * math.pi * (rng.uniform(0, 1, 9) < 0.5)
        bk = dict(b_amp=tuple(rng.uniform(-1.5, 1.5, 3)), b_freq=tuple(fr),
                  b_phase=tuple(rng.uniform(0.0, 2.0 * math.pi, 9)))
    elif b == "const":
        bk = dict(b_const=tuple(rng.uniform(-2, 2, 3)), b_sin=(0.0, 0.0, 0.0), b_axis=(0, 1, 2))
    else:
        bk = dict(b_const=(0.0, 0.0, 0.0), b_sin=(0.0, 0.0, 0.0), b_axis=(0, 1, 2))
    cc = float(rng.uniform(0.1, 2.0)) if c is None else float(c)
    return Problem(ncell=tuple(ncell), nodes=nodes, k=k, K=K, kappa=kap, c=cc,
                   sigma=paper_sigma(k), periodic=tuple(bool(v) for v in periodic), name=f"random_{seed}", **bk)


def random_kappa_poly(rng) -> tuple:
    """Per-axis quadratics c0 + c1 s + c2 s^2 positive on [0, 1] (c0 in [0.5, 1.5],
    |c1| <= 0.4, c2 in [0, 0.8]): a smooth diffusion factor varying by up to 3x."""
    c = []
    for _ in range(3):
        c += [float(rng.uniform(0.5, 1.5)), float(rng.uniform(-0.4, 0.4)), float(rng.uniform(0.0, 0.8))]
    return tuple(c)


def random_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


def workload_vector(prob: Problem) -> np.ndarray:
    return random_vector(prob.ndof, int(prob.meta.get("x_seed", 0)))


# ---------------------------------------------------------------------------
# Manufactured solution u = sin(pi x) sin(pi y) sin(pi z) for
# -div(K grad u) + div(b u) + c u = f with constant K, constant b, constant c
# (strong form of the model problem, Sec. 2.1).  Functions are lists of
# separable terms (alpha, (kind1, kind2, kind3)), kind 0 = 1, 1 = sin(pi .),
# 2 = cos(pi .).
# ---------------------------------------------------------------------------
SIN, COS, ONE = 1, 2, 0


def transport_k5_64(N: int = 64, k: int = 5) -> Problem:
    """The Taylor-Green transport problem of Sec. 5.4 on one GPU's share:
    periodic box (-pi, pi)^3, K = 5e-6 I, c = 0, f = 0.  meta["dt"] keeps
    dt rho(M^{-1} A) below 1, inside the real-axis stability interval
    [-2, 0] of Heun's method."""
    nodes = tuple(np.linspace(-math.pi, math.pi, N + 1) for _ in range(3))
    return Problem(ncell=(N, N, N), nodes=nodes, k=k, K=5e-6 * np.eye(3), c=0.0,
                   sigma=paper_sigma(k), periodic=(True, True, True), name=f"transport_k{k}_{N}",
                   meta={"dt": TRANSPORT_DT_H * (2.0 * math.pi / N)}, **TAYLOR_GREEN)


def transport_paper_k5_64(N: int = 64, k: int = 5) -> Problem:
    """The transport problem with the paper's quadrature for its
    trigonometric flow field, q = 2p + 4 (k + 3 points per direction, Sec.
    5.4); its initial state is the L2 projection of the Gaussian
    (``TRANSPORT_GAUSSIAN``), which the library computes."""
    p = transport_k5_64(N, k)
    return p.with_(quad_extra=2, name=f"transport_paper_k{k}_{N}")


# the initial concentration of Sec. 5.4: amp exp(-width |x - center|^2)
TRANSPORT_GAUSSIAN = dict(amp=1.0, width=2.0, center=(0.5, 0.0, 0.0))


def transport_initial(prob: Problem, x0=(0.5, 0.0, 0.0)) -> np.ndarray:
    """Coefficient vector of the initial concentration exp(-2 |x - x0|^2) of
    Sec. 5.4: its value at each cell centre as the cell's constant mode (the
    first coefficient of every cell block), the other coefficients zero."""
    nb = (prob.k + 1) ** 3
    c = cell_centers(prob.nodes)
    u = np.zeros(prob.ndof)
    u[::nb] = np.exp(-2.0 * ((c - np.asarray(x0)) ** 2).sum(axis=1))
    return u


def manufactured_u():
    return [(1.0, (SIN, SIN, SIN))]


def manufactured_source(K, b, c):
    """f = -sum_rs K_rs d_r d_s u + b . grad u + c u for u = prod sin(pi x_a).

    d_r d_r u = -pi^2 u;  d_r d_s u (r != s) = pi^2 cos cos sin (in r, s);
    d_r u = pi cos(pi x_r) prod_{a != r} sin(pi x_a)."""
    K = np.asarray(K, dtype=np.float64)
    terms = []
    pi2 = math.pi ** 2
    diag = sum(K[r, r] for r in range(3))
    terms.append((pi2 * diag + c, (SIN, SIN, SIN)))
    for r in range(3):
        for s in range(3):
            if r != s and K[r, s] != 0.0:
                kinds = [SIN, SIN, SIN]
                kinds[r] = COS
                kinds[s] = COS
                terms.append((-pi2 * K[r, s], tuple(kinds)))
    for r in range(3):
        if b[r] != 0.0:
            kinds = [SIN, SIN, SIN]
            kinds[r] = COS
            terms.append((math.pi * b[r], tuple(kinds)))
    return terms


def constant_source(value: float = 1.0):
    return [(float(value), (ONE, ONE, ONE))]


# ---------------------------------------------------------------------------
# Vertex meshes: logically structured grids of (N1+1)(N2+1)(N3+1) vertices,
# array shape (N3+1, N2+1, N1+1, 3) (axis 1 fastest); every cell is the
# trilinear image of the reference cube through its eight vertices
# (multilinear geometry, Sec. 4 and Problem C of Sec. 5.1).
# ---------------------------------------------------------------------------
def tensor_vertices(nodes) -> np.ndarray:
    """The vertices of the tensor grid of the per-axis nodes."""
    X = np.stack(np.meshgrid(nodes[0], nodes[1], nodes[2], indexing="ij"), axis=-1)
    return np.ascontiguousarray(X.transpose(2, 1, 0, 3))


def affine_vertices(nodes, A) -> np.ndarray:
    """The vertices x = A xi of the tensor grid xi of the nodes."""
    return np.ascontiguousarray(tensor_vertices(nodes) @ np.asarray(A, dtype=np.float64).T)


def curved_vertices(ncell, eps: float = 0.04, jitter: float = 0.0, seed: int = 0) -> np.ndarray:
    """Uniform vertex grid of [0,1]^3 moved by the smooth field
        d_a(xi) = eps sin(pi xi_a) sin(pi (xi_{a+1} + 2 xi_{a+2}) + a)
    (indices mod 3) plus, with jitter > 0, independent uniform offsets of up to
    jitter times the cell size per coordinate.  Offsets normal to the boundary
    are zero on boundary vertices, so every boundary face stays in its plane of
    the cube; cells are general (non-affine) hexahedra."""
    N1, N2, N3 = ncell
    X = tensor_vertices((uniform_nodes(N1), uniform_nodes(N2), uniform_nodes(N3)))
    xi = X.copy()
    for a in range(3):
        X[..., a] += eps * np.sin(math.pi * xi[..., a]) * np.sin(
            math.pi * (xi[..., (a + 1) % 3] + 2.0 * xi[..., (a + 2) % 3]) + a)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        h = np.array([1.0 / N1, 1.0 / N2, 1.0 / N3])
        off = rng.uniform(-1.0, 1.0, X.shape) * jitter * h
        for a in range(3):
            on_bnd = (xi[..., a] == 0.0) | (xi[..., a] == 1.0)
            off[..., a][on_bnd] = 0.0
        X += off
    return np.ascontiguousarray(X)


def sheared_vertices(nodes, seed: int = 0, amount: float = 0.3) -> np.ndarray:
    """x = xi + s(xi_3) e_1 + r(xi_1) e_2 with s and r piecewise linear between
    the nodes (random values of up to `amount` times the local spacing at each
    node): every cell is a parallelepiped, and its Jacobian changes from one
    layer of cells to the next (affine cells, Problem B of Sec. 5.1)."""
    rng = np.random.default_rng(seed)
    X = tensor_vertices(nodes)
    h3 = np.diff(nodes[2]).min()
    h1 = np.diff(nodes[0]).min()
    s = rng.uniform(-amount, amount, len(nodes[2])) * h3
    r = rng.uniform(-amount, amount, len(nodes[0])) * h1
    X[..., 0] += s[:, None, None]
    X[..., 1] += r[None, None, :]
    return np.ascontiguousarray(X)


def vertex_problem(vertices, k: int, quad_extra: int = 0, K=None, kappa=None, b: str = "sine",
                   c: float = 1.0, kappa_poly=None, name: str = "vertex") -> Problem:
    """A problem on a vertex mesh with the coefficient forms of the other
    workloads (b: 'sine' = (sin pi y, sin pi z, sin pi x), 'const' =
    (1, .5, .25), 'zero')."""
    V = np.asarray(vertices, dtype=np.float64)
    ncell = (V.shape[2] - 1, V.shape[1] - 1, V.shape[0] - 1)
    nodes = tuple(uniform_nodes(ncell[a]) for a in range(3))
    bk = SINE_CYCLIC if b == "sine" else B_CONST if b == "const" else dict(
        b_const=(0.0, 0.0, 0.0), b_sin=(0.0, 0.0, 0.0), b_axis=(0, 1, 2))
    return Problem(ncell=ncell, nodes=nodes, k=k, K=np.eye(3) if K is None else np.asarray(K), kappa=kappa,
                   c=c, sigma=paper_sigma(k), quad_extra=quad_extra, kappa_poly=kappa_poly, vertices=V,
                   name=name, **bk)


def problem_c_quad_extra(k: int) -> int:
    """Extra Gauss points of the rule q = 3p + 4 (Problem C, Sec. 5.1): the
    Gauss rule exact to degree 3k + 4 has ceil((3k + 5) / 2) points."""
    return (3 * k + 5 + 1) // 2 - (k + 1)


def geometry_N(k: int, target_dof: float = 4e6) -> int:
    """Cells per axis of the multilinear-geometry workloads: about 4M DOF."""
    return max(2, int(round(target_dof ** (1.0 / 3.0) / (k + 1))))


def problem_c(k: int, N: int | None = None) -> Problem:
    """Problem C of Sec. 5.1 at one GPU's size: multilinear cells (the uniform
    N^3 vertex grid of the unit cube moved by the smooth field of
    ``curved_vertices``, eps = 0.04), the rotated K of the k = 7 workload
    times a diffusion factor polynomial in the coordinates (seed 7),
    b = (sin pi y, sin pi z, sin pi x), c = 1, sigma = 2k(k+2), the rule
    q = 3p + 4; x ~ U[-1, 1] seed 500+k."""
    N = N or geometry_N(k)
    V = curved_vertices((N, N, N), eps=0.04)
    p = vertex_problem(V, k, quad_extra=problem_c_quad_extra(k), K=anisotropic_K(), b="sine", c=1.0,
                       kappa_poly=random_kappa_poly(np.random.default_rng(7)), name=f"problem_c_k{k}_{N}")
    p.meta["x_seed"] = 500 + k
    return p


def problem_b_cells(k: int, N: int | None = None) -> Problem:
    """Problem B of Sec. 5.1 with affine cells whose Jacobians differ: the
    uniform N^3 grid sheared layer by layer (``sheared_vertices``, seed 8),
    coefficients as ``problem_c``, the rule q = 2p + 4; x seed 600+k."""
    N = N or geometry_N(k)
    V = sheared_vertices((uniform_nodes(N),) * 3, seed=8)
    p = vertex_problem(V, k, quad_extra=2, K=anisotropic_K(), b="sine", c=1.0,
                       kappa_poly=random_kappa_poly(np.random.default_rng(7)), name=f"problem_b_cells_k{k}_{N}")
    p.meta["x_seed"] = 600 + k
    return p
