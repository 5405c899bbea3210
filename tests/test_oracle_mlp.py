"""Pins of the network oracle (CPU): finite differences for the chain rule,
an independent bfloat16 converter for the rounding, Adam's first step, and
the patch layout on a hand-checked mesh."""
import numpy as np
import pytest

from oracle import mlp


def _rand_params(k, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mlp.nparams(k)) * scale


def test_bf16_matches_torch_converter():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-20, 20, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8)]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x32.astype(np.float64)), ref)


def test_bf16_ties_to_even():
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0                 # tie, 1.0 is even
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6   # tie, rounds up to even
    assert mlp.bf16(1.0 + 2 ** -7) == 1.0 + 2 ** -7       # representable


def test_sizes_and_layout_roundtrip():
    k = 1
    p = _rand_params(k, 1)
    assert p.size == 256 * 56 + 256 + 256 * 256 + 256 + 8 * 256 + 8
    assert np.array_equal(mlp.pack(mlp.unpack(p, k)), p)


@pytest.mark.parametrize("k", [1, 2])
def test_gradient_matches_central_differences(k):
    """Unrounded float64 network: every parameter block against central
    differences of the loss (O(h^2) truncation, h = 1e-6)."""
    rng = np.random.default_rng(10 + k)
    nin, nout = mlp.sizes(k)
    X = rng.standard_normal((8, nin))
    T = rng.standard_normal((8, nout))
    p = _rand_params(k, 20 + k, scale=0.2)
    _, g = mlp.backward(p, X, T, k, rounded=False)
    sizes = [256 * nin, 256, 256 * 256, 256, nout * 256, nout]
    offs = np.cumsum([0] + sizes)
    h = 1e-6
    for b in range(6):
        for idx in rng.integers(offs[b], offs[b + 1], 6):
            q = p.copy()
            q[idx] += h
            lp = mlp.loss(q, X, T, k, rounded=False)
            q[idx] -= 2 * h
            lm = mlp.loss(q, X, T, k, rounded=False)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])) + 1e-9, (b, idx, fd, g[idx])


def test_rounded_gradient_is_close_to_exact_gradient():
    """bfloat16 rounding perturbs the gradient by about 2^-8 relative."""
    k = 1
    rng = np.random.default_rng(30)
    nin, nout = mlp.sizes(k)
    X = rng.standard_normal((64, nin))
    T = rng.standard_normal((64, nout))
    p = _rand_params(k, 31)
    _, g0 = mlp.backward(p, X, T, k, rounded=False)
    _, g1 = mlp.backward(p, X, T, k, rounded=True)
    assert np.linalg.norm(g1 - g0) <= 0.05 * np.linalg.norm(g0)


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(40)
    p = rng.standard_normal(1000)
    g = rng.standard_normal(1000)
    p1, m, v = mlp.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3)
    # m_hat = g, v_hat = g^2 after bias correction: step = lr g / (|g| + eps)
    assert np.allclose(p - p1, 1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a second identical gradient keeps the same step
    p2, _, _ = mlp.adam(p1, g, m, v, 2, lr=1e-3)
    assert np.allclose(p1 - p2, p - p1, rtol=1e-9)


def test_patch_layout_on_a_2x2x1_mesh():
    k = 0  # one value per cell keeps the layout readable
    ncell = (2, 2, 1)
    r = np.array([1.0, 2.0, 3.0, 4.0])  # cells (0,0), (1,0), (0,1), (1,1)
    P, s = mlp.patches(r, ncell, k, [0, 3])
    # order T, -x, +x, -y, +y, -z, +z
    assert np.array_equal(P[0], [1.0, 0.0, 2.0, 0.0, 3.0, 0.0, 0.0])
    assert np.array_equal(P[1], [4.0, 3.0, 0.0, 2.0, 0.0, 0.0, 0.0])
    assert np.allclose(s, [np.sqrt(14.0), np.sqrt(29.0)])


def test_precondition_with_zero_last_layer_is_block_jacobi():
    k = 1
    ncell = (2, 1, 1)
    nb = 8
    rng = np.random.default_rng(50)
    p = _rand_params(k, 51)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, k)
    p = mlp.pack([W1, b1, W2, b2, np.zeros_like(W3), np.zeros_like(b3)])
    blocks = rng.standard_normal((2, nb, nb)) + 5 * np.eye(nb)
    r = rng.standard_normal(2 * nb)
    z = mlp.precondition(p, r, ncell, k, blocks)
    ref = np.concatenate([np.linalg.solve(blocks[c], r[c * nb:(c + 1) * nb]) for c in range(2)])
    assert np.allclose(z, ref, rtol=1e-13, atol=0)


def test_precondition_is_odd_in_the_residual():
    k = 1
    ncell = (2, 2, 1)
    nb = 8
    rng = np.random.default_rng(60)
    p = _rand_params(k, 61, scale=0.3)
    blocks = rng.standard_normal((4, nb, nb)) + 5 * np.eye(nb)
    r = rng.standard_normal(4 * nb)
    z1 = mlp.precondition(p, r, ncell, k, blocks)
    z2 = mlp.precondition(p, -r, ncell, k, blocks)
    z3 = mlp.precondition(p, 2.5 * r, ncell, k, blocks)
    assert np.allclose(z2, -z1, rtol=1e-13, atol=0)
    assert np.allclose(z3, 2.5 * z1, rtol=1e-13, atol=0)   # homogeneous of degree one
