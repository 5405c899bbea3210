"""Whole-vector parity at the full benchmark sizes, through the C ABI.

Every entry of y = A x from the GPU is compared with the CPU oracle's full
apply (all host threads) on the same seeded input, in the launch
configuration the benchmark times: the k = 7 32^3 workload (both kernel
selections), every degree of the sweep (about 2e7 DOF each), and the
operators of the two solve workloads; for the multilinear workloads (about
4e6 DOF each) and the raised-rule, Problem B, polynomial-diffusion and
affine workloads the rows of 256 cells per workload.  Bar: relative error <= 1e-12 in the
2-norm and in the max-norm.  Sum factorization is an exact re-bracketing of
the quadrature sums (Sec. 3.5), so the two differ by rounding only.

The mixed-precision solve of the 48^3 k = 5 workload is judged by the
oracle's own FP64 residual of the returned iterate, with the oracle's load
vector as the right-hand side.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1711_10885_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
_ORACLE = {}


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _oracle_apply(key, p, x):
    """The oracle's full y = A x, kept for the tests of this module that share
    the input (the k = 7 workload is checked for both kernel selections)."""
    if key not in _ORACLE:
        t0 = time.perf_counter()
        _ORACLE.clear()
        _ORACLE[key] = oracle.apply(p, x)
        print(f"oracle apply {key}: {p.ndof} DOF in {time.perf_counter() - t0:.1f} s on "
              f"{oracle.default_threads()} threads", flush=True)
    return _ORACLE[key]


def _gpu_apply(p, x, variant=0):
    torch = _torch()
    from paper_1711_10885_amd import binding
    with binding.DG(p) as dg:
        dg.set_kernel(variant)
        y = dg.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    return y


def _check(y, ref, what):
    e2 = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    emax = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"{what}: {y.size} entries, rel2 {e2:.2e} relmax {emax:.2e}", flush=True)
    assert e2 <= TOL and emax <= TOL, (what, e2, emax)


@pytest.mark.parametrize("variant", [0, 1])
def test_cdr_k7_32_whole_vector(variant):
    p = W.cdr_k7_32()
    x = W.workload_vector(p)
    print(f"cdr_k7_32 variant {variant}", flush=True)
    _check(_gpu_apply(p, x, variant), _oracle_apply("cdr_k7_32", p, x), f"cdr_k7_32 v{variant}")


@pytest.mark.parametrize("k", range(1, 11))
def test_degree_sweep_whole_vector(k):
    p = W.cdr_sweep(k)
    x = W.workload_vector(p)
    print(f"sweep k={k} {p.ncell}", flush=True)
    _check(_gpu_apply(p, x), _oracle_apply(f"sweep_k{k}", p, x), f"sweep k={k} {p.ncell}")


@pytest.mark.parametrize("name", ["mixed_k5_48", "learned_k3_64"])
def test_solver_workload_operators_whole_vector(name):
    p = getattr(W, name)()
    x = W.random_vector(p.ndof, 60)
    print(f"{name}", flush=True)
    _check(_gpu_apply(p, x), _oracle_apply(name, p, x), name)


def test_fp32_operator_k7_32_whole_vector():
    """The FP32 tier's operator on the k = 7 workload against the FP64 oracle
    on the same FP32-representable input, every entry, with the FP32 bar of
    the tier (2^-24 per rounding, about 3 (k+1) roundings on the longest
    contraction chain, amplification below 10)."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.cdr_k7_32()
    x32 = W.workload_vector(p).astype(np.float32)
    with binding.DG(p) as dg:
        y32 = dg.apply_f32(torch.from_numpy(x32).cuda()).double().cpu().numpy()
    ref = oracle.apply(p, x32.astype(np.float64))
    bar = 30 * (p.k + 1) * 2.0 ** -24
    e2 = np.linalg.norm(y32 - ref) / np.linalg.norm(ref)
    emax = np.abs(y32 - ref).max() / np.abs(ref).max()
    print(f"cdr_k7_32 FP32: rel2 {e2:.2e} relmax {emax:.2e} (bar {bar:.2e})", flush=True)
    assert e2 <= bar and emax <= bar


def test_mixed_k5_48_gmres_ir_oracle_residual():
    """GMRES-IR (FP32 inner GMRES(30), block Jacobi, FP64 refinement) on the
    full 48^3 k = 5 workload to 1e-8, with the right-hand side the benchmark
    solves (the library's load vector of the manufactured source); the oracle
    recomputes the FP64 residual of the returned iterate against its own load
    vector of the same source (the two load vectors differ by rounding)."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.mixed_k5_48()
    src = W.manufactured_source(p.K, p.b_const, p.c)
    t0 = time.perf_counter()
    f = oracle.rhs(p, src)
    print(f"oracle load vector: {time.perf_counter() - t0:.1f} s", flush=True)
    with binding.DG(p, flags=binding.DG_WITH_BLOCK_JACOBI) as dg:
        fd = dg.load_vector(src)
        diff = np.abs(fd.cpu().numpy() - f).max() / np.abs(f).max()
        print(f"library load vector against the oracle's: relmax {diff:.2e}", flush=True)
        assert diff <= 1e-13
        u, st, rc = dg.solve(fd, tol=1e-8, method=binding.DG_GMRES_IR, precond=binding.DG_PREC_BLOCK_JACOBI,
                             maxit=40000, check=False)
        u = u.cpu().numpy()
    print(f"GMRES-IR: rc {rc}, {st['iters']} inner steps, {st['outer']} refinements, "
          f"library residual {st['rel_resid']:.3e}", flush=True)
    res = np.linalg.norm(f - oracle.apply(p, u)) / np.linalg.norm(f)
    print(f"oracle residual of the GMRES-IR iterate: {res:.3e}", flush=True)
    assert rc == 0 and res <= 1.05e-8


@pytest.mark.parametrize("name", [f"problem_c_k{k}" for k in range(1, 8)] +
                         [f"problem_b_cells_k{k}" for k in (1, 3, 5, 7)])
def test_multilinear_workloads_sampled_cells(name):
    """The multilinear workloads the benchmark times (Problem C with the rule
    q = 3p + 4, and Problem B's sheared affine cells; about 4M DOF each) at
    their full sizes and launch configuration: the rows of the eight corner
    cells and of 248 random cells against the oracle's rows."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    k = int(name.rsplit("_k", 1)[1])
    p = W.problem_c(k) if name.startswith("problem_c") else W.problem_b_cells(k)
    x = W.workload_vector(p)
    with binding.DG(p) as dg:
        y = dg.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    n0, n1, n2 = p.ncell
    corners = [i0 + n0 * (i1 + n1 * i2) for i0 in (0, n0 - 1) for i1 in (0, n1 - 1) for i2 in (0, n2 - 1)]
    rng = np.random.default_rng(9000 + k)
    cells = np.unique(np.concatenate([corners, rng.choice(n0 * n1 * n2, 248, replace=False)]))
    ref = oracle.apply_rows(p, x, cells)
    nb = (k + 1) ** 3
    got = y.reshape(-1, nb)[cells]
    _check(got.ravel(), ref.ravel(), f"{name} ({p.ndof} DOF), {cells.size} cells")


@pytest.mark.parametrize("name", [f"raised_sweep_k{k}" for k in range(1, 9)] +
                         [f"problem_b_k{k}" for k in (3, 5, 7)] +
                         [f"kpoly_sweep_k{k}" for k in (1, 2, 5, 7, 10)] + ["affine_k7_32"])
def test_coefficient_and_rule_workloads_sampled_cells(name):
    """The benchmark's raised-rule (q = 2p + 4), Problem B, polynomial-
    diffusion and affine workloads (about 2e7 DOF each, built as bench.py
    builds them) at their full sizes: the rows of the eight corner cells and
    of 248 random cells against the oracle's rows."""
    import bench
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = bench.make_workload(name)
    x = W.workload_vector(p)
    with binding.DG(p) as dg:
        y = dg.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    n0, n1, n2 = p.ncell
    corners = [i0 + n0 * (i1 + n1 * i2) for i0 in (0, n0 - 1) for i1 in (0, n1 - 1) for i2 in (0, n2 - 1)]
    rng = np.random.default_rng(9100 + p.k)
    cells = np.unique(np.concatenate([corners, rng.choice(n0 * n1 * n2, 248, replace=False)]))
    ref = oracle.apply_rows(p, x, cells)
    got = y.reshape(-1, (p.k + 1) ** 3)[cells]
    _check(got.ravel(), ref.ravel(), f"{name} ({p.ndof} DOF), {cells.size} cells")
