"""Pins of the oracle's pointwise diffusion coefficient D(x) = kappa_T kp(x) K,
kp(x) = prod_j (c0 + c1 x_j + c2 x_j^2) (coefficients polynomial in the
coordinates, Problems B and C of Sec. 5.1), CPU only.

* equality with the independent numpy brute-force assembly (D, d = nu^T D nu,
  the weights and gamma_F evaluated at every quadrature point) on small meshes
  with Dirichlet and periodic axes, per-cell kappa and full K;
* a constant factor (c1 = c2 = 0) equals multiplying kappa by its value;
* with b = 0 the operator is symmetric and positive definite (the SIPG form
  with pointwise coefficients).
"""
import numpy as np
import pytest

import oracle
from paper_1711_10885_amd import workloads as W
from tests.ref_assemble import assemble_dense


def _with_kp(p, seed):
    return p.with_(kappa_poly=W.random_kappa_poly(np.random.default_rng(seed)))


@pytest.mark.parametrize("b,per,k,ncell", [
    ("sine", (False, False, False), 1, (3, 2, 2)),
    ("const", (True, False, True), 2, (2, 3, 2)),
    ("product", (True, True, True), 1, (3, 2, 2)),
    ("sine", (False, True, False), 2, (2, 2, 3)),
])
def test_assemble_matches_brute_force(b, per, k, ncell):
    p = _with_kp(W.random_problem(1600 + k, ncell=ncell, k=k, b=b, periodic=per), 1610 + k)
    A = oracle.assemble(p).toarray()
    ref = assemble_dense(p)
    err = np.abs(A - ref).max() / np.abs(ref).max()
    print(f"kappa_poly {b} per={per} k={k}: max rel {err:.2e}")
    assert err <= 1e-13
    # the factor does change the operator
    A0 = oracle.assemble(p.with_(kappa_poly=None)).toarray()
    assert np.abs(A - A0).max() > 1e-3 * np.abs(A0).max()


def test_a_constant_factor_scales_kappa():
    p = W.random_problem(1620, ncell=(3, 3, 2), k=3, b="sine")
    c = (1.5, 0.0, 0.0, 0.8, 0.0, 0.0, 1.25, 0.0, 0.0)
    q = p.with_(kappa_poly=c)
    s = p.with_(kappa=np.asarray(p.kappa) * (1.5 * 0.8 * 1.25))
    x = W.random_vector(p.ndof, 1621)
    y1, y2 = oracle.apply(q, x), oracle.apply(s, x)
    assert np.abs(y1 - y2).max() <= 1e-13 * np.abs(y2).max()


@pytest.mark.parametrize("per", [(False, False, False), (True, True, False)])
def test_symmetric_positive_definite_without_convection(per):
    p = _with_kp(W.random_problem(1630, ncell=(2, 3, 2), k=2, b="none", periodic=per), 1631)
    A = oracle.assemble(p).toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > 0.0
