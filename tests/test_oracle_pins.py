"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test pins the oracle to something other than itself: closed forms, a
library routine, an independent brute-force assembly, or an identity that the
weighted SIPG form of eq. (blf) (Sec. 2.2) satisfies exactly under the tensor
Gauss rule.  A plausible slip in the oracle (a dropped term, a wrong sign, a
wrong weight or index, a transposed operand) breaks at least one of them.
"""
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as L

import oracle
from paper_1711_10885_amd import workloads as W
from tests.ref_assemble import assemble_dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# 1D rule and basis (Sec. 3.1; Legendre basis of Sec. 2.2)
# --------------------------------------------------------------------------
def test_gauss_closed_forms():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "gauss_legendre_01.txt"))
            if l.strip() and not l.startswith("#")]
    for m, i, x, w in rows:
        xi, wi = oracle.gauss(int(m))
        assert abs(xi[int(i)] - float(x)) < 1e-15
        assert abs(wi[int(i)] - float(w)) < 1e-15


@pytest.mark.parametrize("m", range(1, 12))
def test_gauss_exactness_and_library(m):
    xi, w = oracle.gauss(m)
    for e in range(2 * m):  # exact for degree <= 2m-1
        assert abs(np.dot(w, xi ** e) - 1.0 / (e + 1)) < 2e-15 * (e + 1)
    # degree 2m: the error is the closed form (m!)^4 / ((2m+1) ((2m)!)^2)
    err = 1.0 / (2 * m + 1) - np.dot(w, xi ** (2 * m))
    E = math.factorial(m) ** 4 / ((2 * m + 1) * math.factorial(2 * m) ** 2)
    assert abs(err - E) <= 1e-15 + 1e-9 * E
    xr, wr = L.leggauss(m)
    assert np.allclose(xi, 0.5 * (xr + 1), rtol=0, atol=1e-15)
    assert np.allclose(w, 0.5 * wr, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", range(1, 11))
def test_basis_orthonormal_and_endpoints(k):
    xi, w = oracle.gauss(k + 1)
    V = np.array([oracle.basis(k, t)[0] for t in xi])
    # degree <= 2k, exact under the (k+1)-point rule: orthonormal on [0,1]
    assert np.allclose(V.T @ np.diag(w) @ V, np.eye(k + 1), atol=1e-13)
    v0, d0 = oracle.basis(k, 0.0)
    v1, d1 = oracle.basis(k, 1.0)
    for j in range(k + 1):
        s = math.sqrt(2 * j + 1)
        assert abs(v1[j] - s) < 1e-13 * s
        assert abs(v0[j] - (-1) ** j * s) < 1e-13 * s
        assert abs(d1[j] - j * (j + 1) * s) < 1e-12 * max(1, j * (j + 1) * s)
        assert abs(d0[j] - (-1) ** (j + 1) * j * (j + 1) * s) < 1e-12 * max(1, j * (j + 1) * s)
    # against numpy's Legendre series at interior points
    for t in (0.1, 0.37, 0.5, 0.93):
        v, d = oracle.basis(k, t)
        for j in range(k + 1):
            c = np.zeros(j + 1)
            c[j] = math.sqrt(2 * j + 1)
            assert abs(v[j] - L.legval(2 * t - 1, c)) < 1e-13 * max(1, abs(v[j]))
            assert abs(d[j] - 2 * L.legval(2 * t - 1, L.legder(c))) < 1e-12 * max(1, abs(d[j]))


# --------------------------------------------------------------------------
# Whole operator: brute force on tiny inputs
# --------------------------------------------------------------------------
BRUTE_CASES = [
    dict(seed=11, ncell=(1, 1, 1), k=1, b="sine"),
    dict(seed=12, ncell=(2, 2, 2), k=1, b="const"),
    dict(seed=13, ncell=(3, 2, 2), k=2, b="sine"),
    dict(seed=14, ncell=(2, 2, 2), k=2, b="zero"),
    dict(seed=15, ncell=(2, 1, 2), k=3, b="const"),
    dict(seed=16, ncell=(1, 2, 1), k=3, b="sine"),
]


@pytest.mark.parametrize("case", BRUTE_CASES, ids=lambda c: f"s{c['seed']}k{c['k']}{c['b']}")
def test_oracle_equals_bruteforce_assembly(case):
    p = W.random_problem(case["seed"], ncell=case["ncell"], k=case["k"], b=case["b"])
    A = assemble_dense(p)
    x = W.random_vector(p.ndof, case["seed"] + 100)
    y = oracle.apply(p, x)
    ref = A @ x
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    # the probing assembly of the oracle reproduces the same matrix
    As = oracle.assemble(p).toarray()
    assert np.abs(As - A).max() <= 1e-13 * np.abs(A).max()


def test_apply_rows_equals_apply():
    p = W.random_problem(21, ncell=(3, 3, 2), k=2, b="sine")
    x = W.random_vector(p.ndof, 5)
    y = oracle.apply(p, x).reshape(p.ncells, -1)
    cells = np.array([0, 4, 7, 17, 9])
    yr = oracle.apply_rows(p, x, cells)
    assert np.abs(yr - y[cells]).max() <= 1e-13 * np.abs(y).max()
    for terms in (oracle.VOLUME, oracle.INTERIOR, oracle.BOUNDARY):
        yt = oracle.apply(p, x, terms).reshape(p.ncells, -1)
        yrt = oracle.apply_rows(p, x, cells, terms)
        assert np.abs(yrt - yt[cells]).max() <= 1e-13 * np.abs(y).max()


# --------------------------------------------------------------------------
# Identities of the bilinear form
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,k", [(31, 1), (32, 2), (33, 3)])
def test_symmetry_pure_diffusion(seed, k):
    """b = 0: consistency and symmetry terms of eq. (blf) are a transposed
    pair, so A = A^T (also with per-cell kappa, full K and reaction)."""
    p = W.random_problem(seed, ncell=(3, 2, 2), k=k, b="zero")
    A = oracle.assemble(p).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    x = W.random_vector(p.ndof, 1)
    z = W.random_vector(p.ndof, 2)
    assert abs(x @ oracle.apply(p, z) - z @ oracle.apply(p, x)) <= 1e-12 * np.abs(A).max() * p.ndof
    # coercivity of the symmetric form for this penalty
    assert np.linalg.eigvalsh(A).min() > 0


def test_symmetry_breaks_with_convection():
    p = W.random_problem(34, ncell=(2, 2, 2), k=2, b="const")
    A = oracle.assemble(p).toarray()
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()


def test_reaction_is_scaled_mass():
    """A(c0) - A(0) = c0 diag(|T|): orthonormal basis, degree-2k rule exact."""
    p = W.random_problem(41, ncell=(3, 2, 2), k=2, b="sine", c=0.0)
    c0 = 1.7
    x = W.random_vector(p.ndof, 3)
    y0 = oracle.apply(p, x)
    d = oracle.apply(p.with_(c=c0), x) - y0
    vol = np.array([np.diff(p.nodes[0])[i1] * np.diff(p.nodes[1])[i2] * np.diff(p.nodes[2])[i3]
                    for i3 in range(p.ncell[2]) for i2 in range(p.ncell[1])
                    for i1 in range(p.ncell[0])])
    expect = c0 * np.repeat(vol, (p.k + 1) ** 3) * x
    # the difference cancels the diffusion/penalty part: rounding scales with |A x|
    assert np.abs(d - expect).max() <= 1e-14 * np.abs(y0).max()


def _faces(p):
    """Yield (a, cell_minus or None, cell_plus or None, h_minus, h_plus, area)."""
    N = p.ncell
    h = [np.diff(p.nodes[a]) for a in range(3)]
    for i3 in range(N[2]):
        for i2 in range(N[1]):
            for i1 in range(N[0]):
                i = (i1, i2, i3)
                c = i1 + N[0] * (i2 + N[1] * i3)
                for a in range(3):
                    t = [b for b in range(3) if b != a]
                    area = h[t[0]][i[t[0]]] * h[t[1]][i[t[1]]]
                    if i[a] == 0:
                        yield a, None, c, None, h[a][i[a]], area, i
                    ip = list(i)
                    ip[a] += 1
                    if ip[a] < N[a]:
                        cp = ip[0] + N[0] * (ip[1] + N[1] * ip[2])
                        yield a, c, cp, h[a][i[a]], h[a][ip[a]], area, i
                    else:
                        yield a, c, None, h[a][i[a]], None, area, i


@pytest.mark.parametrize("seed", [51, 52])
def test_penalty_energy_piecewise_constants(seed):
    """x piecewise constant (mode 0 only), b = 0, c = 0: grad u = 0 so only
    the penalty term survives: x^T A x = sum_F gamma_F |F| [[u]]^2 with
    gamma_F = sigma <d-,d+>/min(h_a-,h_a+) inside, sigma d/h_a on the boundary."""
    p = W.random_problem(seed, ncell=(3, 3, 2), k=2, b="zero", c=0.0)
    nb = (p.k + 1) ** 3
    u0 = W.random_vector(p.ncells, seed)
    x = np.zeros(p.ndof)
    x[::nb] = u0  # theta_0 = 1, so u = x_{T,0} on T
    kap = p.kappa
    expect = 0.0
    for a, cm, cp, hm, hp, area, _ in _faces(p):
        if cm is not None and cp is not None:
            dm, dp = kap[cm] * p.K[a, a], kap[cp] * p.K[a, a]
            g = p.sigma * (2 * dm * dp / (dm + dp)) / min(hm, hp)
            expect += g * area * (u0[cm] - u0[cp]) ** 2
        else:
            c = cm if cm is not None else cp
            hh = hm if cm is not None else hp
            g = p.sigma * kap[c] * p.K[a, a] / hh
            expect += g * area * u0[c] ** 2
    got = x @ oracle.apply(p, x)
    assert abs(got - expect) <= 1e-12 * abs(expect)


def _face_values(p, x, a, c, e, h_all, kind):
    """u of cell c on its face x_a = e at the tangential Gauss nodes, by
    numpy Legendre series (independent of the oracle's basis code)."""
    k = p.k
    n = k + 1
    xi, _ = L.leggauss(k + 1)
    xi = 0.5 * (xi + 1)

    def tab(t):
        return np.array([[L.legval(2 * tt - 1, np.eye(n)[j] * math.sqrt(2 * j + 1))
                          for j in range(n)] for tt in np.atleast_1d(t)])
    T = [tab(xi), tab(xi), tab(xi)]
    T[a] = tab([float(e)])
    X = x[c * n ** 3:(c + 1) * n ** 3].reshape(n, n, n)  # [j3, j2, j1]
    u = np.einsum("kji,ai,bj,ck->cba", X, T[0], T[1], T[2])
    return u.squeeze(axis=2 - a)  # drop the normal axis: [t_slow, t_fast]


@pytest.mark.parametrize("b", ["const", "sine"])
def test_upwind_energy_identity(b):
    """For divergence-free b with b_a independent of x_a:
    x^T (A(b) - A(0)) x = 1/2 sum_F sum_q W |b.nu| [[u]]^2  (boundary [[u]] = u).
    Integration by parts along x_a is exact under the (k+1)-point rule and the
    face rule reuses the tangential nodes, so this holds to rounding."""
    p = W.random_problem(61, ncell=(3, 2, 2), k=2, b=b)
    p0 = p.with_(b_const=(0, 0, 0), b_sin=(0, 0, 0))
    x = W.random_vector(p.ndof, 7)
    got = x @ (oracle.apply(p, x) - oracle.apply(p0, x))
    xi, wq = L.leggauss(p.k + 1)
    xi, wq = 0.5 * (xi + 1), 0.5 * wq
    expect = 0.0
    for a, cm, cp, hm, hp, area, i in _faces(p):
        t = [bb for bb in range(3) if bb != a]
        c = cm if cm is not None else cp
        o = [p.nodes[d][i[d]] for d in range(3)]
        hh = [p.nodes[d][i[d] + 1] - p.nodes[d][i[d]] for d in range(3)]
        xa = p.nodes[a][i[a] + 1] if cm is not None else p.nodes[a][i[a]]
        # points ordered [t1 slow, t0 fast]
        P0 = o[t[0]] + hh[t[0]] * xi
        P1 = o[t[1]] + hh[t[1]] * xi
        G1, G0 = np.meshgrid(P1, P0, indexing="ij")
        X = np.zeros(G0.shape + (3,))
        X[..., a] = xa
        X[..., t[0]] = G0
        X[..., t[1]] = G1
        bnu = p.b_const[a] + p.b_sin[a] * np.sin(np.pi * X[..., p.b_axis[a]])
        Wf = np.outer(wq, wq) * area
        um = _face_values(p, x, a, cm, 1, None, None) if cm is not None else 0.0
        up = _face_values(p, x, a, cp, 0, None, None) if cp is not None else 0.0
        J = um - up
        expect += 0.5 * np.sum(Wf * np.abs(bnu) * J ** 2)
    assert abs(got - expect) <= 1e-11 * abs(expect)


def test_patch_constant():
    """u = 1 everywhere: for a cell without boundary face y_{T,0} = c |T| and
    y_{T,j} = 0 otherwise, for any K, per-cell kappa and the sine-cyclic b
    (div b = 0)."""
    p = W.random_problem(71, ncell=(3, 3, 3), k=3, b="sine")
    nb = (p.k + 1) ** 3
    x = np.zeros(p.ndof)
    x[::nb] = 1.0
    y = oracle.apply(p, x).reshape(p.ncells, nb)
    c = 1 + 3 * (1 + 3 * 1)  # the only interior cell
    vol = np.prod([p.nodes[a][2] - p.nodes[a][1] for a in range(3)])
    assert abs(y[c, 0] - p.c * vol) <= 1e-13 * max(1.0, p.c * vol) * 10
    assert np.abs(y[c, 1:]).max() <= 1e-12


@pytest.mark.parametrize("k", [1, 3])
def test_patch_linear(k):
    """u = alpha + beta . x, constant coefficients: consistency of the DG form
    gives y_{T,j} = sum_q W (b . grad u + c u) phi_j for interior cells."""
    p = W.random_problem(72, ncell=(3, 3, 3), k=k, b="const", kappa=False)
    n = k + 1
    nb = n ** 3
    alpha, beta = 0.3, np.array([1.2, -0.7, 0.4])
    x = np.zeros((p.ncells, nb))
    N = p.ncell
    for i3 in range(N[2]):
        for i2 in range(N[1]):
            for i1 in range(N[0]):
                i = (i1, i2, i3)
                c = i1 + N[0] * (i2 + N[1] * i3)
                o = np.array([p.nodes[a][i[a]] for a in range(3)])
                h = np.array([p.nodes[a][i[a] + 1] - p.nodes[a][i[a]] for a in range(3)])
                # x_a = o_a + h_a/2 + h_a/(2 sqrt 3) theta_1(t_a)
                x[c, 0] = alpha + beta @ (o + h / 2)
                for a, jj in enumerate((1, n, n * n)):
                    x[c, jj] = beta[a] * h[a] / (2 * math.sqrt(3))
    y = oracle.apply(p, x.ravel()).reshape(p.ncells, nb)
    c = 1 + 3 * (1 + 3 * 1)
    i = (1, 1, 1)
    o = np.array([p.nodes[a][i[a]] for a in range(3)])
    h = np.array([p.nodes[a][i[a] + 1] - p.nodes[a][i[a]] for a in range(3)])
    xi, wq = L.leggauss(n)
    xi, wq = 0.5 * (xi + 1), 0.5 * wq
    Vt = np.array([[L.legval(2 * t - 1, np.eye(n)[j] * math.sqrt(2 * j + 1)) for j in range(n)]
                   for t in xi])
    expect = np.zeros(nb)
    bvec = np.array(p.b_const)
    for q3 in range(n):
        for q2 in range(n):
            for q1 in range(n):
                X = o + h * np.array([xi[q1], xi[q2], xi[q3]])
                Wq = wq[q1] * wq[q2] * wq[q3] * np.prod(h)
                val = bvec @ beta + p.c * (alpha + beta @ X)
                phi = np.einsum("k,j,i->kji", Vt[q3], Vt[q2], Vt[q1]).ravel()
                expect += Wq * val * phi
    assert np.abs(y[c] - expect).max() <= 1e-11 * np.abs(expect).max()


# --------------------------------------------------------------------------
# Manufactured solution: textbook SIPG convergence O(h^{k+1}) in L2
# --------------------------------------------------------------------------
def _solve_manufactured(N, k):
    import scipy.sparse.linalg as spla
    base = W.mixed_k5_48(N=N, k=k)
    A = oracle.assemble(base)
    f = oracle.rhs(base, W.manufactured_source(base.K, base.b_const, base.c))
    u = spla.spsolve(A.tocsc(), f)
    return oracle.l2err(base, u, W.manufactured_u()), A, f, u


@pytest.mark.parametrize("k,Ns", [(1, (4, 8)), (2, (2, 4, 8)), (3, (2, 4))])
def test_manufactured_convergence_order(k, Ns):
    errs = [_solve_manufactured(N, k)[0] for N in Ns]
    orders = [math.log(errs[i] / errs[i + 1], 2) for i in range(len(errs) - 1)]
    assert abs(orders[-1] - (k + 1)) <= 0.3, (errs, orders)


def test_oracle_gmres_matches_direct_solve():
    _, A, f, u_direct = _solve_manufactured(4, 1)
    u, it, rel = oracle.gmres(lambda v: A @ v, f, tol=1e-10, restart=30, maxit=5000)
    assert rel <= 1e-10
    assert np.linalg.norm(u - u_direct) <= 1e-7 * np.linalg.norm(u_direct)


def test_block_diagonal_matches_assembly():
    p = W.random_problem(81, ncell=(2, 3, 2), k=1, b="sine")
    A = oracle.assemble(p).toarray()
    B = oracle.block_diagonal(p)
    nb = (p.k + 1) ** 3
    for c in range(p.ncells):
        s = slice(c * nb, (c + 1) * nb)
        assert np.abs(B[c] - A[s, s]).max() <= 1e-14 * np.abs(A).max()


# --------------------------------------------------------------------------
# Absolute scale of the L2 error (the measure |T| and the orthonormal basis)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 3])
def test_l2err_of_zero_against_the_sine_product(k):
    """u_h = 0 against u = sin(pi x) sin(pi y) sin(pi z) on the box
    [0,1] x [0,2] x [0,3]: ||u||^2 = (1/2)(2/2)(3/2) = 3/4 in closed form.  On
    uniform cells the composite Gauss sum of cos(2 pi x) over whole periods
    vanishes, so the quadrature is exact to rounding; a wrong cell measure,
    weight or axis length changes the value."""
    base = W.mixed_k5_48(N=2, k=k)
    nodes = (W.uniform_nodes(3), 2.0 * W.uniform_nodes(4), 3.0 * W.uniform_nodes(6))
    p = base.with_(ncell=(3, 4, 6), nodes=nodes)
    e = oracle.l2err(p, np.zeros(p.ndof), W.manufactured_u())
    assert abs(e * e - 0.75) <= 1e-13, e * e


@pytest.mark.parametrize("k", [1, 2, 4])
def test_l2err_of_a_coefficient_vector_is_its_weighted_norm(k):
    """With the orthonormal basis, ||u_h - c||^2 for the constant c = 1 and
    u_h = 1 + d (d any coefficient vector) is sum_T |T| sum_j d_{T,j}^2
    exactly (the (k+3)-point rule integrates the degree-2k products exactly):
    pins the cell measure on a non-uniform mesh."""
    p = W.random_problem(90 + k, ncell=(3, 2, 4), k=k, b="const")
    nb = (k + 1) ** 3
    d = W.random_vector(p.ndof, 95 + k)
    x = d.copy()
    x[::nb] += 1.0  # the constant 1 is theta_0^3 = 1 in the constant mode
    vol = np.array([(p.nodes[0][i + 1] - p.nodes[0][i]) * (p.nodes[1][j + 1] - p.nodes[1][j])
                    * (p.nodes[2][l + 1] - p.nodes[2][l])
                    for l in range(p.ncell[2]) for j in range(p.ncell[1]) for i in range(p.ncell[0])])
    expect = float((vol * (d.reshape(p.ncells, nb) ** 2).sum(axis=1)).sum())
    e = oracle.l2err(p, x, [(1.0, (0, 0, 0))])
    assert abs(e * e - expect) <= 1e-13 * expect, (e * e, expect)
