"""GPU parity of the multilinear-geometry operator (every cell the trilinear
image of the reference cube through its eight vertices; Sec. 4, Problem C
of Sec. 5.1) against the oracle, through the C ABI.

Bar: relative error <= 1e-12 in the 2-norm and in the max-norm (the kernel
evaluates the same quadrature sums by sum factorization, an exact
re-bracketing, with the geometry per point).  Cases: every degree k = 1..7
with the three rules the path takes (k+1, k+3 and the rule q = 3p + 4 of
Problem C), curved and jittered meshes with one, several and many cells,
every b form, per-cell kappa and the polynomial diffusion factor; parallel-
epiped cells with different Jacobians (Problem B's affine cells); tensor
and affine vertex meshes against the tuned kernels; the paths the handle
rejects.
"""
import numpy as np
import pytest

import oracle
from paper_1711_10885_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _gpu_apply(p, x):
    torch = _torch()
    from paper_1711_10885_amd import binding
    with binding.DG(p) as dg:
        y = dg.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    return y


def _check(y, ref, what):
    e2 = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    emax = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"{what}: rel2 {e2:.2e} relmax {emax:.2e}", flush=True)
    assert e2 <= TOL and emax <= TOL, (what, e2, emax)


def _curved(seed, ncell, k, b, qe, kpoly=True, jitter=0.2):
    p = W.random_problem(seed, ncell=ncell, k=k, b=b)
    V = W.curved_vertices(ncell, eps=0.05, jitter=jitter, seed=seed)
    kp = W.random_kappa_poly(np.random.default_rng(seed)) if kpoly else None
    return p.with_(vertices=V, quad_extra=qe, kappa_poly=kp)


def _rules(k):
    return sorted({0, 2, W.problem_c_quad_extra(k)})


@pytest.mark.parametrize("k", range(1, 8))
@pytest.mark.parametrize("rule", [0, 1, 2])
def test_curved_mesh_every_degree_and_rule(k, rule):
    rules = _rules(k)
    if rule >= len(rules):
        pytest.skip("k = 1: the raised rule and the rule q = 3p + 4 coincide")
    qe = rules[rule]
    p = _curved(4000 + 10 * k + rule, (3, 2, 2), k, "sine", qe)
    x = W.random_vector(p.ndof, 4100 + k)
    print(f"curved k={k} quad_extra={qe}", flush=True)
    _check(_gpu_apply(p, x), oracle.apply(p, x), f"curved 3x2x2 k={k} m={k + 1 + qe}")


@pytest.mark.parametrize("k,b,kpoly,ncell", [
    (2, "product", True, (1, 1, 1)),
    (3, "const", False, (4, 3, 3)),
    (3, "zero", True, (2, 3, 1)),
    (5, "product", False, (2, 2, 3)),
    (7, "const", True, (1, 2, 1)),
])
def test_curved_mesh_coefficient_forms(k, b, kpoly, ncell):
    qe = W.problem_c_quad_extra(k)
    p = _curved(4200 + k, ncell, k, b, qe, kpoly)
    x = W.random_vector(p.ndof, 4300 + k)
    print(f"curved {ncell} k={k} b={b} kp={kpoly}", flush=True)
    _check(_gpu_apply(p, x), oracle.apply(p, x), f"curved {ncell} k={k} b={b}")


@pytest.mark.parametrize("k,qe", [(2, 0), (4, 2), (3, 3)])
def test_parallelepiped_cells_with_different_jacobians(k, qe):
    """Affine cells (Problem B): every cell a parallelepiped, the Jacobian
    changing from one layer of cells to the next."""
    p = W.random_problem(4400 + k, ncell=(3, 3, 2), k=k, b="sine")
    p = p.with_(vertices=W.sheared_vertices(p.nodes, seed=4400 + k), quad_extra=qe,
                kappa_poly=W.random_kappa_poly(np.random.default_rng(4401)))
    x = W.random_vector(p.ndof, 4402 + k)
    _check(_gpu_apply(p, x), oracle.apply(p, x), f"sheared k={k} quad_extra={qe}")


@pytest.mark.parametrize("k,qe", [(3, 0), (5, 2)])
def test_tensor_and_affine_vertices_match_the_tuned_kernels(k, qe):
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(4500 + k, ncell=(3, 2, 2), k=k, b="const").with_(quad_extra=qe)
    x = W.random_vector(p.ndof, 4501)
    A = np.array([[1.1, 0.2, -0.1], [0.05, 0.9, 0.2], [-0.15, 0.1, 1.05]])
    for q, v in ((p, W.tensor_vertices(p.nodes)), (p.with_(affine=A), W.affine_vertices(p.nodes, A))):
        with binding.DG(q) as dg:
            yt = dg.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        yv = _gpu_apply(p.with_(vertices=v), x)
        _check(yv, yt, f"vertex mesh against the tuned kernel k={k} affine={q.affine is not None}")


def test_many_cells_whole_vector():
    """A curved mesh of 6 x 5 x 4 cells (several workgroups per XCD) at k = 3
    with the rule q = 3p + 4, every entry."""
    p = _curved(4600, (6, 5, 4), 3, "sine", W.problem_c_quad_extra(3), jitter=0.1)
    x = W.random_vector(p.ndof, 4601)
    _check(_gpu_apply(p, x), oracle.apply(p, x), "curved 6x5x4 k=3")


def test_gmres_on_a_curved_mesh_judged_by_the_oracle():
    """dg_solve (FP64 GMRES, no preconditioner) on a curved mesh; the oracle's
    residual of the returned iterate."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.vertex_problem(W.curved_vertices((3, 3, 3), eps=0.04), 2, b="const", c=0.1)
    f = W.random_vector(p.ndof, 4700)
    with binding.DG(p) as dg:
        u, st, rc = dg.solve(torch.from_numpy(f).cuda(), tol=1e-9, maxit=5000)
        u = u.cpu().numpy()
    res = np.linalg.norm(f - oracle.apply(p, u)) / np.linalg.norm(f)
    print(f"GMRES on the curved mesh: {st['iters']} steps, oracle residual {res:.3e}", flush=True)
    assert rc == 0 and res <= 1.05e-9


def test_multilinear_handles_reject_the_tensor_only_paths():
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.vertex_problem(W.curved_vertices((2, 2, 2), eps=0.04), 2)
    with binding.DG(p) as dg:
        x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        for call in (lambda: dg.apply_f32(x.float()), lambda: dg.heun(x, 1e-3, 1),
                     lambda: dg.heun_noalloc(x, 1e-3, 1), lambda: dg.load_vector(W.constant_source()),
                     lambda: dg.solve(x + 1.0, method=binding.DG_GMRES_IR)):
            with pytest.raises(binding.DGError) as e:
                call()
            assert e.value.status == binding.DG_EINVAL
