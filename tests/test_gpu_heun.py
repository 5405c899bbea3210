"""GPU parity of explicit Heun time stepping (dg_heun) against the oracle,
through the C ABI.

dg_heun runs each stage as one launch of the operator kernel that writes the
stage value in place of A x (the fused variant) or as the reference operator
followed by an elementwise pass; both are checked.  Bar: the change of u over
the run, u_n - u_0, agrees with the oracle's to 1e-12 relative (2-norm and
max-norm), and u_n itself to 1e-12; at the transport workload's full size
(64^3, k = 5) one step is compared on sampled cells the oracle steps one by
one.  Time steps keep dt rho(M^{-1} A) below 1 (explicit stability), so the
runs stay in the regime the method is used in.
"""
import numpy as np
import pytest

import oracle
from paper_1711_10885_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
VARIANTS = [0, 1]  # DG_KERNEL_AUTO (fused stages), DG_KERNEL_REFERENCE


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _mild(p, scale=1e-3):
    return p.with_(K=np.asarray(p.K) * scale)


def _dt(p):
    """Half the inverse of a power-iteration estimate of rho(M^{-1} A)."""
    nb = (p.k + 1) ** 3
    minv = np.repeat(1.0 / oracle.cell_volumes(p), nb)
    v = W.random_vector(p.ndof, 7)
    rho = 0.0
    for _ in range(30):
        w = minv * oracle.apply(p, v)
        rho = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    return 0.5 / (1.2 * rho)


def _gpu_heun(p, u0, dt, n, variant=0, f=None, calls=1):
    torch = _torch()
    from paper_1711_10885_amd import binding
    with binding.DG(p) as dg:
        dg.set_kernel(variant)
        u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
        fd = None if f is None else torch.from_numpy(np.ascontiguousarray(f)).cuda()
        for _ in range(calls):
            dg.heun(u, dt, n, f=fd)
        out = u.cpu().numpy()
    torch.cuda.synchronize()
    return out


def _check(u, ref, u0, what):
    d, dr = u - u0, ref - u0
    e2 = np.linalg.norm(d - dr) / np.linalg.norm(dr)
    emax = np.abs(d - dr).max() / np.abs(dr).max()
    eu = np.abs(u - ref).max() / np.abs(ref).max()
    print(f"{what}: increment rel2 {e2:.2e} relmax {emax:.2e}, u relmax {eu:.2e}", flush=True)
    assert e2 <= TOL and emax <= TOL and eu <= TOL, (what, e2, emax, eu)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("k", [1, 2, 4, 5, 7])
@pytest.mark.parametrize("per", [(True, True, True), (False, False, False), (True, False, True)])
def test_heun_matches_oracle(variant, k, per):
    ncell = (4, 3, 2) if k <= 4 else (3, 2, 2)
    p = _mild(W.random_problem(1000 + k, ncell=ncell, k=k, b="sine", periodic=per))
    u0 = W.random_vector(p.ndof, 1100 + k)
    dt, n = _dt(p), 4
    ref = oracle.heun(p, u0, dt, n)
    _check(_gpu_heun(p, u0, dt, n, variant), ref, u0, f"heun k={k} per={per} v{variant} dt={dt:.3g}")


@pytest.mark.parametrize("variant", VARIANTS)
def test_heun_with_source_and_diffusion(variant):
    """Full-strength diffusion (K of order one, kappa per cell) and a load
    vector f; dt from the stiff spectrum."""
    p = W.random_problem(1200, ncell=(3, 3, 2), k=3, b="const", periodic=(False, True, False))
    u0 = W.random_vector(p.ndof, 1201)
    f = W.random_vector(p.ndof, 1202)
    dt, n = _dt(p), 3
    _check(_gpu_heun(p, u0, dt, n, variant, f=f), oracle.heun(p, u0, dt, n, f=f), u0, f"source v{variant}")


def test_repeated_calls_continue_the_run():
    """Two calls of 3 steps equal one of 6 (the workspace is reused)."""
    p = _mild(W.random_problem(1250, ncell=(3, 2, 2), k=4, periodic=(True, True, True)))
    u0 = W.random_vector(p.ndof, 1251)
    dt = _dt(p)
    a = _gpu_heun(p, u0, dt, 3, calls=2)
    b = _gpu_heun(p, u0, dt, 6)
    assert np.array_equal(a, b)
    _check(a, oracle.heun(p, u0, dt, 6), u0, "2 x 3 steps")


def test_zero_steps_leave_u_unchanged():
    p = W.random_problem(1260, ncell=(2, 2, 2), k=2)
    u0 = W.random_vector(p.ndof, 1261)
    assert np.array_equal(_gpu_heun(p, u0, 1e-3, 0), u0)


def test_mass_is_conserved_on_a_periodic_mesh():
    """c = 0, f = 0, no boundary faces: sum_T |T| u_T0 is invariant."""
    p = _mild(W.random_problem(1270, ncell=(4, 4, 3), k=3, b="sine", c=0.0, periodic=(True, True, True)))
    nb = (p.k + 1) ** 3
    u0 = W.random_vector(p.ndof, 1271)
    vol = oracle.cell_volumes(p)
    u = _gpu_heun(p, u0, _dt(p), 50)
    m0, m1 = (vol * u0[::nb]).sum(), (vol * u[::nb]).sum()
    print(f"mass {m0:.15e} -> {m1:.15e}", flush=True)
    assert abs(m1 - m0) <= 1e-13 * (vol * np.abs(u0[::nb])).sum()
    assert np.abs(u - u0).max() > 1e-3  # the field did move


def test_constant_field_decays_by_the_stability_function():
    c = 0.8
    p = _mild(W.random_problem(1280, ncell=(3, 2, 2), k=5, b="sine", c=c, periodic=(True, True, True)))
    nb = (p.k + 1) ** 3
    u0 = np.zeros(p.ndof)
    u0[::nb] = 1.0
    dt, n = _dt(p), 10
    z = -c * dt
    u = _gpu_heun(p, u0, dt, n)
    assert np.abs(u - (1.0 + z + 0.5 * z * z) ** n * u0).max() <= 1e-13


def test_transport_full_size_sampled_cells():
    """One step at the bench's transport workload (Taylor-Green b, 64^3, k = 5,
    56.6M DOF), in the bench's launch configuration, against the oracle
    stepping sampled cells (corners and faces of the periodic box, where the
    wrap is taken, and interior cells)."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.transport_k5_64()
    nb = (p.k + 1) ** 3
    N = p.ncell[0]
    u0 = W.random_vector(p.ndof, 1290)
    dt = p.meta["dt"]
    with binding.DG(p) as dg:
        u = torch.from_numpy(u0).cuda()
        dg.heun(u, dt, 1)
        got = u.cpu().numpy().reshape(-1, nb)
        del u
    torch.cuda.synchronize()
    rng = np.random.default_rng(1291)
    cells = [0, N - 1, N * N - 1, N * N * N - 1, N * N * (N - 1), N // 2 + N * (N // 2) + N * N * (N // 2)]
    cells += [int(c) for c in rng.choice(p.ncells, 18, replace=False)]
    ref = oracle.heun_step_rows(p, u0, dt, cells)
    base = u0.reshape(-1, nb)[cells]
    d, dr = got[cells] - base, ref - base
    e = np.abs(d - dr).max() / np.abs(dr).max()
    print(f"transport 64^3 k=5 sampled {len(cells)} cells: increment relmax {e:.2e}", flush=True)
    assert e <= TOL
    assert np.abs(got[cells] - ref).max() <= TOL * np.abs(ref).max()


@pytest.mark.parametrize("variant", VARIANTS)
def test_heun_taylor_green(variant):
    """The transport problem (Taylor-Green b, periodic box (-pi, pi)^3,
    K = 5e-6 I) on a 4^3 mesh at k = 3 from its Gaussian initial field, with
    the workload's own time step rule."""
    p = W.transport_k5_64(N=4, k=3)
    u0 = W.transport_initial(p)
    dt, n = p.meta["dt"], 6
    _check(_gpu_heun(p, u0, dt, n, variant), oracle.heun(p, u0, dt, n), u0, f"taylor-green v{variant}")


def test_taylor_green_mass_is_conserved():
    p = W.transport_k5_64(N=6, k=4)
    nb = (p.k + 1) ** 3
    u0 = W.transport_initial(p)
    u = _gpu_heun(p, u0, p.meta["dt"], 100)
    m0, m1 = u0[::nb].sum(), u[::nb].sum()  # uniform cells: |T| is a common factor
    print(f"taylor-green mass {m0:.15e} -> {m1:.15e}", flush=True)
    assert abs(m1 - m0) <= 1e-13 * np.abs(u0[::nb]).sum()
    assert np.abs(u - u0).max() > 1e-3


@pytest.mark.parametrize("k,qe,N", [(2, 0, 5), (3, 2, 4), (5, 2, 3)])
def test_gaussian_projection_matches_oracle(k, qe, N):
    """dg_project_gaussian (the L2 projection of the initial concentration of
    Sec. 5.4) on the periodic box against the oracle's projection."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.transport_k5_64(N=N, k=k).with_(quad_extra=qe)
    G = W.TRANSPORT_GAUSSIAN
    ref = oracle.project_gaussian(p, G["amp"], G["width"], G["center"])
    with binding.DG(p) as dg:
        u = dg.project_gaussian(G["amp"], G["width"], G["center"]).cpu().numpy()
    e = np.abs(u - ref).max() / np.abs(ref).max()
    print(f"projection k={k} quad_extra={qe}: relmax {e:.2e}", flush=True)
    assert e <= TOL


def test_taylor_green_with_the_paper_rule_from_the_projected_gaussian():
    """The transport example as the paper runs it (Sec. 5.4): the rule
    q = 2p + 4 for the trigonometric flow field and the L2-projected Gaussian
    start; 6 Heun steps on a 4^3 mesh at k = 3 against the oracle started
    from its own projection."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.transport_paper_k5_64(N=4, k=3)
    G = W.TRANSPORT_GAUSSIAN
    u0_ref = oracle.project_gaussian(p, G["amp"], G["width"], G["center"])
    dt, n = p.meta["dt"], 6
    with binding.DG(p) as dg:
        u = dg.project_gaussian(G["amp"], G["width"], G["center"])
        u0 = u.cpu().numpy()
        dg.heun(u, dt, n)
        got = u.cpu().numpy()
    assert np.abs(u0 - u0_ref).max() <= TOL * np.abs(u0_ref).max()
    _check(got, oracle.heun(p, u0_ref, dt, n), u0_ref, "taylor-green q=2p+4, projected start")


@pytest.mark.parametrize("variant", VARIANTS)
def test_heun_with_a_kappa_polynomial(variant):
    p = _mild(W.random_problem(1320, ncell=(3, 2, 2), k=4, b="product", periodic=(True, True, False)))
    p = p.with_(kappa_poly=W.random_kappa_poly(np.random.default_rng(1321)))
    u0 = W.random_vector(p.ndof, 1322)
    dt, n = _dt(p), 4
    _check(_gpu_heun(p, u0, dt, n, variant), oracle.heun(p, u0, dt, n), u0, f"kappa poly heun v{variant}")


def test_heun_with_raised_quadrature():
    p = _mild(W.random_problem(1330, ncell=(3, 2, 2), k=3, b="product", periodic=(True, True, True)))
    p = p.with_(quad_extra=2, kappa_poly=W.random_kappa_poly(np.random.default_rng(1331)))
    u0 = W.random_vector(p.ndof, 1332)
    dt, n = _dt(p), 3
    _check(_gpu_heun(p, u0, dt, n), oracle.heun(p, u0, dt, n), u0, "q=2p+4 heun")


@pytest.mark.parametrize("variant", VARIANTS)
def test_heun_on_an_affine_mesh(variant):
    """The stage update divides by the physical cell volume |det A| |T_xi|."""
    A = np.array([[1.2, 0.3, -0.1], [0.1, 0.8, 0.25], [-0.2, 0.15, 1.1]])
    p = _mild(W.random_problem(1340, ncell=(3, 2, 2), k=3, b="const", c=0.3, periodic=(True, True, False)))
    p = p.with_(affine=A)
    u0 = W.random_vector(p.ndof, 1341)
    dt, n = _dt(p), 4
    _check(_gpu_heun(p, u0, dt, n, variant), oracle.heun(p, u0, dt, n), u0, f"affine heun v{variant}")


@pytest.mark.parametrize("case", ["dt0", "dtnan", "dtneg", "nsteps", "overlap"])
def test_invalid_arguments(case):
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(1300, ncell=(2, 2, 2), k=2)
    with binding.DG(p) as dg:
        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        args = dict(dt0=(0.0, 1, None), dtnan=(float("nan"), 1, None), dtneg=(-1e-3, 1, None),
                    nsteps=(1e-3, -1, None), overlap=(1e-3, 1, u))[case]
        with pytest.raises(binding.DGError) as ei:
            dg.heun(u, args[0], args[1], f=args[2])
        assert ei.value.status == binding.DG_EINVAL
