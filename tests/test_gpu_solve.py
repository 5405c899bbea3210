"""FP64 GMRES (dg_solve) on the GPU, through the C ABI.

Checks against things the GPU path does not compute itself: the oracle's
residual ||f - A_oracle u|| / ||f||, a sparse direct solve of the oracle's
assembled matrix, the oracle's own GMRES(30) iteration count, and the
discretisation error against a manufactured solution.
"""
import numpy as np
import pytest

import oracle
from paper_1711_10885_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _solve(prob, f, tol, u0=None, check=True, variant=0, **kw):
    torch = _torch()
    from paper_1711_10885_amd import binding
    with binding.DG(prob) as dg:
        dg.set_kernel(variant)
        fd = torch.from_numpy(np.ascontiguousarray(f)).cuda()
        ud = None if u0 is None else torch.from_numpy(np.ascontiguousarray(u0)).cuda()
        u, st, rc = dg.solve(fd, ud, tol=tol, check=check, **kw)
        u = u.cpu().numpy()
    print(f"{prob.name}: rc {rc} {st}", flush=True)
    return u, st, rc


def _oracle_rel_residual(prob, u, f):
    return np.linalg.norm(f - oracle.apply(prob, u)) / np.linalg.norm(f)


@pytest.mark.parametrize("b", ["sine", "const", "none"])
def test_solution_matches_sparse_direct_solve(b):
    import scipy.sparse.linalg as spla
    p = W.random_problem(410, ncell=(3, 3, 2), k=2, b=b)
    f = W.random_vector(p.ndof, 411)
    A = oracle.assemble(p).tocsc()
    ustar = spla.spsolve(A, f)
    u, st, rc = _solve(p, f, 1e-12)
    assert rc == 0 and st["rel_resid"] <= 1e-12
    res = _oracle_rel_residual(p, u, f)
    assert res <= 5e-12, res
    cond_bound = np.linalg.norm(u - ustar) / np.linalg.norm(ustar)
    assert cond_bound <= 1e-8, cond_bound


def test_iterations_and_residual_match_oracle_gmres():
    p = W.poisson_k2_8()
    f = oracle.rhs(p, W.manufactured_source(p.K, (0.0, 0.0, 0.0), 0.0))
    tol = 1e-8
    u, st, rc = _solve(p, f, tol)
    uo, it_o, rel_o = oracle.gmres(lambda v: oracle.apply(p, v), f, tol=tol, restart=30)
    print(f"oracle gmres: {it_o} iterations, rel {rel_o:.3e}", flush=True)
    assert rc == 0
    # same Krylov method (CGS2 here, MGS in the oracle): equal in exact arithmetic
    assert abs(st["iters"] - it_o) <= max(2, 0.02 * it_o), (st["iters"], it_o)
    assert _oracle_rel_residual(p, u, f) <= 1.05 * tol
    # both iterates solve the system to tol: their difference is small in the A-image
    d = np.linalg.norm(oracle.apply(p, u - uo)) / np.linalg.norm(f)
    assert d <= 2.1 * tol, d


def test_cdr_random_problem_every_degree_small():
    for k in (1, 3, 5):
        p = W.random_problem(420 + k, ncell=(3, 2, 2), k=k, b="sine")
        f = W.random_vector(p.ndof, 430 + k)
        u, st, rc = _solve(p, f, 1e-10)
        assert rc == 0
        assert _oracle_rel_residual(p, u, f) <= 1.05e-10


@pytest.mark.parametrize("restart", [1, 5, 63])
def test_restart_lengths(restart):
    p = W.random_problem(440, ncell=(2, 2, 2), k=1, b="none")
    f = W.random_vector(p.ndof, 441)
    u, st, rc = _solve(p, f, 1e-8, restart=restart)
    assert rc == 0 and st["outer"] >= 1
    assert _oracle_rel_residual(p, u, f) <= 1.05e-8


def test_reference_kernel_gives_the_same_solve():
    p = W.random_problem(450, ncell=(3, 2, 2), k=3, b="sine")
    f = W.random_vector(p.ndof, 451)
    u0, s0, _ = _solve(p, f, 1e-10, variant=0)
    u1, s1, _ = _solve(p, f, 1e-10, variant=1)
    assert abs(s0["iters"] - s1["iters"]) <= 2
    assert _oracle_rel_residual(p, u1, f) <= 1.05e-10


@pytest.mark.parametrize("method", ["gmres64", "gmres_ir", "fgmres"])
def test_both_orthogonalisations_solve_to_tolerance(method):
    """One projection (default) and the repeated projection reach the same
    tolerance on the oracle's residual with iteration counts a few percent
    apart (equal in exact arithmetic)."""
    from paper_1711_10885_amd import binding
    m = {"gmres64": binding.DG_GMRES64, "gmres_ir": binding.DG_GMRES_IR, "fgmres": binding.DG_FGMRES}[method]
    p = W.random_problem(455, ncell=(4, 3, 3), k=3, b="sine")
    f = W.random_vector(p.ndof, 456)
    torch = _torch()
    with binding.DG(p, flags=binding.DG_WITH_BLOCK_JACOBI) as dg:
        fd = torch.from_numpy(f).cuda()
        out = {}
        for orth in (binding.DG_ORTH_CGS1, binding.DG_ORTH_CGS2):
            u, st, rc = dg.solve(fd, tol=1e-10, method=m, precond=binding.DG_PREC_BLOCK_JACOBI, orth=orth)
            assert rc == 0
            assert _oracle_rel_residual(p, u.cpu().numpy(), f) <= 1.05e-10
            out[orth] = st["iters"]
    print(f"{method}: iterations CGS1 {out[0]}, CGS2 {out[1]}", flush=True)
    assert abs(out[0] - out[1]) <= max(3, 0.05 * out[1])


def test_maxit_reports_not_converged_with_stats():
    from paper_1711_10885_amd import binding
    p = W.poisson_k2_8()
    f = W.random_vector(p.ndof, 460)
    u, st, rc = _solve(p, f, 1e-12, check=False, maxit=7)
    assert rc == binding.DG_ENOTCONV
    assert st["iters"] == 7 and 0 < st["rel_resid"] < 1
    assert abs(_oracle_rel_residual(p, u, f) - st["rel_resid"]) <= 1e-9


def test_zero_rhs_gives_zero_solution():
    p = W.random_problem(470, ncell=(2, 2, 2), k=2)
    u, st, rc = _solve(p, np.zeros(p.ndof), 1e-8, u0=W.random_vector(p.ndof, 471))
    assert rc == 0 and st["iters"] == 0 and not u.any()


def test_exact_initial_guess_needs_no_iteration():
    import scipy.sparse.linalg as spla
    p = W.random_problem(480, ncell=(2, 2, 2), k=2)
    f = W.random_vector(p.ndof, 481)
    ustar = spla.spsolve(oracle.assemble(p).tocsc(), f)
    u, st, rc = _solve(p, f, 1e-8, u0=ustar)
    assert rc == 0 and st["iters"] == 0 and st["applies"] == 1
    assert np.array_equal(u, ustar)


def test_non_finite_rhs_is_reported():
    from paper_1711_10885_amd import binding
    p = W.random_problem(490, ncell=(2, 2, 2), k=1)
    f = W.random_vector(p.ndof, 491)
    f[5] = np.nan
    _, _, rc = _solve(p, f, 1e-8, check=False)
    assert rc == binding.DG_ENAN


@pytest.mark.parametrize("over", [dict(restart=0), dict(restart=64), dict(maxit=0), dict(method=9),
                                  dict(precond=9), dict(orth=2)])
def test_invalid_options_are_rejected(over):
    from paper_1711_10885_amd import binding
    p = W.random_problem(495, ncell=(1, 1, 1), k=1)
    _, _, rc = _solve(p, W.random_vector(p.ndof, 496), 1e-8, check=False, **over)
    assert rc == binding.DG_EINVAL


def test_manufactured_solution_converges_at_order_k_plus_1():
    """Discrete solutions of the mixed-tier coefficients (K = I,
    b = (1, 0.5, 0.25), c = 0.1) against u = sin(pi x) sin(pi y) sin(pi z):
    the L2 error falls like h^(k+1) (textbook SIPG rate)."""
    k = 3
    errs = []
    for N in (4, 8):
        p = W.mixed_k5_48(N=N, k=k)
        f = oracle.rhs(p, W.manufactured_source(p.K, p.b_const, p.c))
        u, st, rc = _solve(p, f, 1e-11)
        assert rc == 0
        errs.append(oracle.l2err(p, u, W.manufactured_u()))
    order = np.log2(errs[0] / errs[1])
    print(f"L2 errors {errs}, order {order:.2f}", flush=True)
    assert abs(order - (k + 1)) <= 0.3


@pytest.mark.parametrize("k", [1, 3, 5, 8])
def test_load_vector_matches_oracle(k):
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(800 + k, ncell=(3, 2, 2), k=k, b="sine")
    terms = W.manufactured_source(p.K, (0.3, -0.2, 0.1), 0.7) + W.constant_source(0.25)
    with binding.DG(p) as dg:
        f = dg.load_vector(terms).cpu().numpy()
    ref = oracle.rhs(p, terms)
    e = np.abs(f - ref).max() / np.abs(ref).max()
    print(f"k={k}: load vector relmax {e:.2e}", flush=True)
    assert e <= 1e-13


@pytest.mark.parametrize("k", [1, 4, 8])
def test_load_vector_with_the_raised_rule_matches_oracle(k):
    """With quad_extra = 2 the load vector integrates with the operator's own
    k + 3 points per direction, as the oracle does."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(820 + k, ncell=(3, 2, 2), k=k, b="sine").with_(quad_extra=2)
    terms = W.manufactured_source(p.K, (0.3, -0.2, 0.1), 0.7) + W.constant_source(0.25)
    with binding.DG(p) as dg:
        f = dg.load_vector(terms).cpu().numpy()
    ref = oracle.rhs(p, terms)
    e = np.abs(f - ref).max() / np.abs(ref).max()
    print(f"k={k} q=2p+4: load vector relmax {e:.2e}", flush=True)
    assert e <= 1e-13
    # the (k+1)-point vector differs: the check above does see the rule
    ref0 = oracle.rhs(p.with_(quad_extra=0), terms)
    assert np.abs(ref0 - ref).max() > 1e3 * e * np.abs(ref).max()


def test_load_vector_of_the_48_cube_workload_on_sampled_cells():
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.mixed_k5_48()
    terms = W.manufactured_source(p.K, p.b_const, p.c)
    with binding.DG(p) as dg:
        f = dg.load_vector(terms).cpu().numpy()
    ref = oracle.rhs(p, terms)
    assert np.abs(f - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("method", ["gmres64", "gmres_ir", "fgmres"])
@pytest.mark.parametrize("coef", ["product_b", "kappa_poly", "taylor_green"])
def test_solvers_with_pointwise_coefficients_on_periodic_meshes(method, coef):
    """Every solver (the FP32 tier of GMRES-IR included) with block Jacobi on
    the coefficient variants evaluated at quadrature points, periodic axes
    with even cell counts; judged by the oracle's residual."""
    from paper_1711_10885_amd import binding
    m = {"gmres64": binding.DG_GMRES64, "gmres_ir": binding.DG_GMRES_IR, "fgmres": binding.DG_FGMRES}[method]
    if coef == "taylor_green":
        p = W.transport_k5_64(N=4, k=3).with_(K=np.eye(3) * 0.05, c=0.5)
    else:
        p = W.random_problem(470, ncell=(4, 2, 4), k=3, b="product" if coef == "product_b" else "sine",
                             periodic=(True, False, True))
        if coef == "kappa_poly":
            p = p.with_(kappa_poly=W.random_kappa_poly(np.random.default_rng(471)))
    f = W.random_vector(p.ndof, 472)
    torch = _torch()
    with binding.DG(p, flags=binding.DG_WITH_BLOCK_JACOBI) as dg:
        u, st, rc = dg.solve(torch.from_numpy(f).cuda(), tol=1e-10, method=m,
                             precond=binding.DG_PREC_BLOCK_JACOBI, maxit=5000)
        u = u.cpu().numpy()
    res = _oracle_rel_residual(p, u, f)
    print(f"{coef} {method}: rc {rc}, {st['iters']} steps, oracle residual {res:.2e}", flush=True)
    assert rc == 0 and res <= 1.05e-10


def test_solve_on_an_affine_mesh_and_no_load_vector():
    torch = _torch()
    from paper_1711_10885_amd import binding
    A = np.array([[1.0, 0.35, 0.0], [0.0, 1.0, -0.2], [0.0, 0.0, 1.0]])
    p = W.random_problem(480, ncell=(4, 3, 2), k=2, b="const", periodic=(True, False, False)).with_(affine=A)
    f = W.random_vector(p.ndof, 481)
    with binding.DG(p, flags=binding.DG_WITH_BLOCK_JACOBI) as dg:
        u, st, rc = dg.solve(torch.from_numpy(f).cuda(), tol=1e-10, method=binding.DG_GMRES_IR,
                             precond=binding.DG_PREC_BLOCK_JACOBI)
        with pytest.raises(binding.DGError):
            dg.load_vector(W.constant_source(1.0))
    res = _oracle_rel_residual(p, u.cpu().numpy(), f)
    print(f"affine solve: rc {rc}, {st['iters']} steps, oracle residual {res:.2e}", flush=True)
    assert rc == 0 and res <= 1.05e-10
