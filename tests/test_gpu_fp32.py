"""FP32 operator (dg_apply_f32) and GMRES-IR (dg_solve, DG_GMRES_IR) on the GPU.

The FP32 operator is compared with the FP64 oracle applied to the same
(FP32-representable) input, so the difference is the FP32 arithmetic alone.
The bound: 2^-24 per rounding, about 3 (k+1) roundings along the longest
chain of 1D contractions (forward and transposed sweeps in three
directions, even-odd split) and an amplification of the entries by
|V^T| |W| |V| against |V^T W V| that stays below 10 for these bases,
i.e. 2^-24 * 30 (k+1) relative to max|A x|; the measured errors are printed.
GMRES-IR is judged by the oracle's FP64 residual.
"""
import numpy as np
import pytest

import oracle
from paper_1711_10885_amd import workloads as W

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _apply32(prob, x32):
    torch = _torch()
    from paper_1711_10885_amd import binding
    with binding.DG(prob) as dg:
        y = dg.apply_f32(torch.from_numpy(x32).cuda()).cpu().numpy()
    return y


def _check32(y32, ref, k, what):
    bar = 30 * (k + 1) * U32
    emax = np.abs(y32 - ref).max() / np.abs(ref).max()
    e2 = np.linalg.norm(y32 - ref) / np.linalg.norm(ref)
    print(f"{what}: FP32 rel2 {e2:.2e} relmax {emax:.2e} (bar {bar:.2e})", flush=True)
    assert emax <= bar and e2 <= bar, (what, e2, emax)


@pytest.mark.parametrize("k", range(1, 11))
def test_fp32_operator_every_degree(k):
    ncell = (4, 3, 2) if k <= 5 else (3, 2, 2)
    p = W.random_problem(600 + k, ncell=ncell, k=k, b="sine" if k % 2 else "const")
    x32 = W.random_vector(p.ndof, 610 + k).astype(np.float32)
    _check32(_apply32(p, x32), oracle.apply(p, x32.astype(np.float64)), k, f"random k={k}")


@pytest.mark.parametrize("ncell", [(1, 1, 1), (5, 1, 1), (1, 1, 3)])
def test_fp32_operator_degenerate_meshes(ncell):
    p = W.random_problem(620, ncell=ncell, k=3)
    x32 = W.random_vector(p.ndof, 621).astype(np.float32)
    _check32(_apply32(p, x32), oracle.apply(p, x32.astype(np.float64)), 3, f"mesh {ncell}")


def test_fp32_operator_on_the_k7_32_workload_against_fp64():
    """Full 32^3 k = 7 workload: FP32 operator against the FP64 GPU operator
    (itself checked against the oracle to 1e-12) on the same input, plus
    sampled cells against the oracle directly."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.cdr_k7_32()
    x32 = W.workload_vector(p).astype(np.float32)
    with binding.DG(p) as dg:
        xd = torch.from_numpy(x32).cuda()
        y32 = dg.apply_f32(xd).cpu().numpy()
        y64 = dg.apply(xd.double()).cpu().numpy()
    _check32(y32, y64, 7, "cdr_k7_32 vs FP64 GPU")
    cells = np.array([0, 777, p.ncells // 2, p.ncells - 1])
    ref = oracle.apply_rows(p, x32.astype(np.float64), cells)
    got = y32.reshape(p.ncells, -1)[cells]
    assert np.abs(got - ref).max() <= 30 * 8 * U32 * np.abs(y64).max()


def test_fp32_operator_is_deterministic():
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(630, ncell=(4, 4, 4), k=4)
    x = torch.from_numpy(W.random_vector(p.ndof, 631).astype(np.float32)).cuda()
    with binding.DG(p) as dg:
        a = dg.apply_f32(x).cpu().numpy()
        b = dg.apply_f32(x).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precond", [0, 1])
def test_gmres_ir_reaches_fp64_tolerance(precond):
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(640 + precond, ncell=(4, 3, 3), k=3, b="sine")
    f = W.random_vector(p.ndof, 650)
    flags = binding.DG_WITH_BLOCK_JACOBI if precond else 0
    with binding.DG(p, flags=flags) as dg:
        fd = torch.from_numpy(f).cuda()
        u, st, rc = dg.solve(fd, tol=1e-11, method=binding.DG_GMRES_IR, precond=precond)
        _, st64, _ = dg.solve(fd, tol=1e-11, precond=precond)
        u = u.cpu().numpy()
    print(f"IR {st}\nFP64 {st64}", flush=True)
    assert rc == 0 and st["rel_resid"] <= 1e-11
    res = np.linalg.norm(f - oracle.apply(p, u)) / np.linalg.norm(f)
    assert res <= 1.05e-11, res
    assert st["applies"] == st["outer"]  # one FP64 residual per refinement step (zero guess)
    assert st["applies_f32"] >= st["iters"] >= st["outer"]


def test_gmres_ir_manufactured_solution():
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.mixed_k5_48(N=6, k=3)
    f = oracle.rhs(p, W.manufactured_source(p.K, p.b_const, p.c))
    with binding.DG(p) as dg:
        u, st, rc = dg.solve(torch.from_numpy(f).cuda(), tol=1e-9, method=binding.DG_GMRES_IR)
        u = u.cpu().numpy()
    assert rc == 0
    res = np.linalg.norm(f - oracle.apply(p, u)) / np.linalg.norm(f)
    assert res <= 1.05e-9
    # the discretisation error dominates: IR solution as good as an exact solve
    import scipy.sparse.linalg as spla
    ustar = spla.spsolve(oracle.assemble(p).tocsc(), f)
    e_ir = oracle.l2err(p, u, W.manufactured_u())
    e_ex = oracle.l2err(p, ustar, W.manufactured_u())
    assert abs(e_ir - e_ex) <= 1e-6 * e_ex


def test_gmres_ir_rejects_bad_inner_tolerance():
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(660, ncell=(1, 1, 1), k=1)
    with binding.DG(p) as dg:
        f = torch.ones(p.ndof, dtype=torch.float64, device="cuda")
        _, _, rc = dg.solve(f, method=binding.DG_GMRES_IR, inner_tol=1.5, check=False)
    assert rc == binding.DG_EINVAL
