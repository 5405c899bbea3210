"""GPU parity of the FP64 apply against the CPU oracle, through the C ABI.

Bar: relative error <= 1e-12 in both the 2-norm and the max-norm
(||y - y_o|| <= 1e-12 ||y_o||, max|y - y_o| <= 1e-12 max|y_o|).
Both kernel variants are checked on the same seeded inputs.
"""
import numpy as np
import pytest

import oracle
from paper_1711_10885_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
VARIANTS = [0, 1]  # DG_KERNEL_AUTO, DG_KERNEL_REFERENCE


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _gpu_apply(prob, x, variant, repeat=1):
    torch = _torch()
    from paper_1711_10885_amd import binding
    with binding.DG(prob) as dg:
        dg.set_kernel(variant)
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        outs = [dg.apply(xd).cpu().numpy() for _ in range(repeat)]
    torch.cuda.synchronize()
    return outs if repeat > 1 else outs[0]


def _check(y, ref, what):
    e2 = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    emax = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"{what}: rel2 {e2:.2e} relmax {emax:.2e}", flush=True)
    assert e2 <= TOL and emax <= TOL, (what, e2, emax)


@pytest.mark.parametrize("variant", VARIANTS)
def test_poisson_k2_8_full(variant):
    p = W.poisson_k2_8()
    x = W.workload_vector(p)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"poisson_k2_8 v{variant}")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", range(1, 11))
def test_random_small_every_degree(variant, k):
    ncell = (4, 3, 2) if k <= 5 else (3, 2, 2)
    p = W.random_problem(100 + k, ncell=ncell, k=k, b="sine" if k % 2 else "const")
    x = W.random_vector(p.ndof, 200 + k)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"random k={k} {ncell} v{variant}")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("ncell", [(1, 1, 1), (5, 1, 1), (1, 4, 1), (1, 1, 3), (2, 3, 5)])
def test_degenerate_meshes(variant, ncell):
    p = W.random_problem(300, ncell=ncell, k=3, b="sine")
    x = W.random_vector(p.ndof, 301)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"mesh {ncell} v{variant}")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("terms", ["b_axis_self", "no_kappa_zero_b", "diag_K"])
def test_coefficient_kinds(variant, terms):
    p = W.random_problem(400, ncell=(3, 3, 2), k=4, b="sine")
    if terms == "b_axis_self":  # b_a depends on x_a itself (node tables on faces)
        p = p.with_(b_axis=(0, 1, 2))
    elif terms == "no_kappa_zero_b":
        p = p.with_(kappa=None, b_const=(0, 0, 0), b_sin=(0, 0, 0))
    else:
        p = p.with_(K=np.diag([2.0, 0.5, 1.5]))
    x = W.random_vector(p.ndof, 401)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"{terms} v{variant}")


def test_deterministic_and_variants_agree():
    p = W.random_problem(500, ncell=(4, 4, 4), k=5, b="sine")
    x = W.random_vector(p.ndof, 501)
    a1, a2 = _gpu_apply(p, x, 0, repeat=2)
    assert np.array_equal(a1, a2)
    r = _gpu_apply(p, x, 1)
    assert np.abs(a1 - r).max() <= 1e-13 * np.abs(r).max()


def test_aliasing_rejected():
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.poisson_k2_8()
    with binding.DG(p) as dg:
        x = torch.zeros(dg.ndof, dtype=torch.float64, device="cuda")
        with pytest.raises(binding.DGError, match="overlap"):
            dg.apply(x, x)


PERIODIC = [(True, False, False), (False, True, False), (False, False, True), (True, True, True)]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", range(1, 11))
def test_periodic_axes_every_degree(variant, k):
    """Periodic axes (first and last cells are face neighbours): odd, even and
    single-cell periodic axes across the degrees, both kernels."""
    ncell = [(3, 2, 4), (1, 3, 2), (4, 1, 3)][k % 3] if k <= 6 else [(3, 2, 2), (2, 1, 3)][k % 2]
    per = PERIODIC[k % 4]
    p = W.random_problem(700 + k, ncell=ncell, k=k, b="sine" if k % 2 else "const", periodic=per)
    x = W.random_vector(p.ndof, 710 + k)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"periodic {per} k={k} {ncell} v{variant}")


@pytest.mark.parametrize("k", [2, 5, 7])
def test_periodic_fp32_operator_matches_fp64(k):
    """FP32 operator on a fully periodic mesh against the FP64 oracle, with the
    error bar of the FP32 tier (traces and contractions rounded to FP32)."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(720 + k, ncell=(3, 2, 3), k=k, b="sine", periodic=(True, True, True))
    x = W.random_vector(p.ndof, 730 + k)
    ref = oracle.apply(p, x)
    with binding.DG(p) as dg:
        y = dg.apply_f32(torch.from_numpy(x).float().cuda()).double().cpu().numpy()
    e = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"periodic fp32 k={k}: relmax {e:.2e}", flush=True)
    assert e <= 30 * (k + 1) * 2.0 ** -24


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", range(1, 11))
def test_product_b_every_degree(variant, k):
    """Product-form flow field b_r = amp_r prod_j sin(w_rj x_j + phi_rj) (every
    factor non-constant, or some factors constant), with Dirichlet and
    periodic axes, both kernels."""
    ncell = (3, 3, 2) if k <= 5 else (3, 2, 2)
    per = PERIODIC[k % 4]
    p = W.random_problem(1500 + k, ncell=ncell, k=k, b="product" if k % 2 else "product_sparse", periodic=per)
    x = W.random_vector(p.ndof, 1510 + k)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"product b {per} k={k} {ncell} v{variant}")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", [3, 5])
def test_taylor_green_box(variant, k):
    """The transport problem's operator (Taylor-Green b on the periodic box
    (-pi, pi)^3) on a 4^3 mesh."""
    p = W.transport_k5_64(N=4, k=k)
    x = W.transport_initial(p) + 0.1 * W.random_vector(p.ndof, 1520 + k)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"taylor-green 4^3 k={k} v{variant}")


@pytest.mark.parametrize("k", [2, 5, 7])
def test_product_b_fp32_operator_matches_fp64(k):
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(1530 + k, ncell=(3, 2, 3), k=k, b="product", periodic=(True, False, True))
    x = W.random_vector(p.ndof, 1540 + k)
    ref = oracle.apply(p, x)
    with binding.DG(p) as dg:
        y = dg.apply_f32(torch.from_numpy(x).float().cuda()).double().cpu().numpy()
    e = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"product b fp32 k={k}: relmax {e:.2e}", flush=True)
    assert e <= 30 * (k + 1) * 2.0 ** -24


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", range(1, 11))
def test_kappa_polynomial_every_degree(variant, k):
    """Diffusion polynomial in the coordinates, D(x) = kappa_T kp(x) K,
    evaluated at the quadrature points, with sum-form or product-form b,
    Dirichlet and periodic axes, both kernels."""
    ncell = (3, 3, 2) if k <= 5 else (3, 2, 2)
    per = PERIODIC[(k + 1) % 4]
    p = W.random_problem(1700 + k, ncell=ncell, k=k, b="sine" if k % 2 else "product", periodic=per)
    p = p.with_(kappa_poly=W.random_kappa_poly(np.random.default_rng(1710 + k)))
    x = W.random_vector(p.ndof, 1720 + k)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"kappa poly {per} k={k} {ncell} v{variant}")


@pytest.mark.parametrize("k", [2, 5, 7])
def test_kappa_polynomial_fp32_operator_matches_fp64(k):
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(1730 + k, ncell=(3, 2, 3), k=k, b="const", periodic=(False, True, False))
    p = p.with_(kappa_poly=W.random_kappa_poly(np.random.default_rng(1740 + k)))
    x = W.random_vector(p.ndof, 1750 + k)
    ref = oracle.apply(p, x)
    with binding.DG(p) as dg:
        y = dg.apply_f32(torch.from_numpy(x).float().cuda()).double().cpu().numpy()
    e = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"kappa poly fp32 k={k}: relmax {e:.2e}", flush=True)
    assert e <= 30 * (k + 1) * 2.0 ** -24


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", range(1, 9))
def test_raised_quadrature_every_degree(variant, k):
    """The rule q = 2p + 4 (k + 3 Gauss points per direction, Problem B of
    Sec. 5.1) with the polynomial diffusion factor, product- or sum-form b
    and periodic axes; both kernel selections run the rectangular
    reference-layout kernel."""
    p = W.random_problem(1900 + k, ncell=(3, 2, 2), k=k, b="product" if k % 2 else "sine",
                         periodic=PERIODIC[k % 4])
    p = p.with_(quad_extra=2, kappa_poly=W.random_kappa_poly(np.random.default_rng(1910 + k)))
    x = W.random_vector(p.ndof, 1920 + k)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"q=2p+4 k={k} v{variant}")


def test_raised_quadrature_with_cellwise_coefficients():
    p = W.random_problem(1930, ncell=(4, 3, 2), k=3, b="const").with_(quad_extra=2)
    x = W.random_vector(p.ndof, 1931)
    _check(_gpu_apply(p, x, 0), oracle.apply(p, x), "q=2p+4 cellwise")


@pytest.mark.parametrize("k", [1, 4, 7])
def test_raised_quadrature_fp32_operator_and_gmres_ir(k):
    """The raised rule runs the FP32 tier too (the degree-(k+2) FP32 kernel on
    padded vectors): the FP32 operator against the FP64 oracle with the FP32
    error bar, and GMRES-IR to 1e-10 on the oracle's residual."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(1940 + k, ncell=(2, 2, 2), k=k, b="product", periodic=(True, False, False))
    p = p.with_(quad_extra=2, kappa_poly=W.random_kappa_poly(np.random.default_rng(1950 + k)))
    x = W.random_vector(p.ndof, 1960 + k)
    ref = oracle.apply(p, x)
    with binding.DG(p, flags=binding.DG_WITH_BLOCK_JACOBI) as dg:
        y = dg.apply_f32(torch.from_numpy(x).float().cuda()).double().cpu().numpy()
        f = torch.from_numpy(W.random_vector(p.ndof, 1970 + k)).cuda()
        u, st, rc = dg.solve(f, tol=1e-10, method=binding.DG_GMRES_IR, precond=binding.DG_PREC_BLOCK_JACOBI)
        u, f = u.cpu().numpy(), f.cpu().numpy()
    e = np.abs(y - ref).max() / np.abs(ref).max()
    res = np.linalg.norm(f - oracle.apply(p, u)) / np.linalg.norm(f)
    print(f"q=2p+4 fp32 k={k}: relmax {e:.2e}; GMRES-IR rc {rc}, {st['iters']} steps, residual {res:.2e}", flush=True)
    assert e <= 30 * (k + 3) * 2.0 ** -24
    assert rc == 0 and res <= 1.05e-10


AFFINE = np.array([[1.2, 0.3, -0.1], [0.1, 0.8, 0.25], [-0.2, 0.15, 1.1]])


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", [1, 2, 4, 7, 10])
def test_affine_geometry(variant, k):
    """The mesh as the image x = A xi of a tensor grid (affine cells): the GPU
    runs the tensor-grid kernels with coefficients transformed at setup, the
    oracle the physical geometry (normals, measures, |F|/|T|)."""
    ncell = (3, 2, 2) if k <= 7 else (2, 2, 2)
    p = W.random_problem(2100 + k, ncell=ncell, k=k, b="const", periodic=PERIODIC[k % 4]).with_(affine=AFFINE)
    x = W.random_vector(p.ndof, 2110 + k)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"affine k={k} v{variant}")


def test_affine_geometry_with_the_raised_rule():
    p = W.random_problem(2120, ncell=(3, 2, 2), k=3, b="const", periodic=(True, False, False))
    p = p.with_(affine=AFFINE, quad_extra=2)
    x = W.random_vector(p.ndof, 2121)
    _check(_gpu_apply(p, x, 0), oracle.apply(p, x), "affine q=2p+4")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("case", ["raised_one_cell_axis", "raised_single_cell", "affine_one_cell_axis",
                                  "product_single_cell"])
def test_new_paths_on_degenerate_meshes(variant, case):
    """Axes of one cell (periodic: the cell is its own face neighbour) and a
    single cell, through the raised rule, affine geometry and product b."""
    if case == "raised_one_cell_axis":
        p = W.random_problem(2200, ncell=(1, 3, 2), k=3, b="product", periodic=(True, True, False))
        p = p.with_(quad_extra=2, kappa_poly=W.random_kappa_poly(np.random.default_rng(2201)))
    elif case == "raised_single_cell":
        p = W.random_problem(2202, ncell=(1, 1, 1), k=5, b="sine").with_(quad_extra=2)
    elif case == "affine_one_cell_axis":
        p = W.random_problem(2203, ncell=(3, 1, 2), k=4, b="const", periodic=(False, True, True)).with_(affine=AFFINE)
    else:
        p = W.random_problem(2204, ncell=(1, 1, 1), k=6, b="product", periodic=(True, True, True))
    x = W.random_vector(p.ndof, 2210)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"{case} v{variant}")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", [2, 5])
def test_problem_b_affine_polynomial_raised(variant, k):
    """Problem B's three features together: affine cells, the diffusion factor
    polynomial in the grid coordinates, and the rule q = 2p + 4."""
    p = W.random_problem(2300 + k, ncell=(3, 2, 2), k=k, b="const", periodic=(False, True, False))
    p = p.with_(affine=AFFINE, quad_extra=2, kappa_poly=W.random_kappa_poly(np.random.default_rng(2310 + k)))
    x = W.random_vector(p.ndof, 2320 + k)
    _check(_gpu_apply(p, x, variant), oracle.apply(p, x), f"problem B k={k} v{variant}")
