"""CPU oracle for the learned cell-patch preconditioner (float64, numpy).

TEST INFRASTRUCTURE ONLY (imported by ``tests/``), sharing no code with the
HIP path.  The network and the optimiser are not in the paper (which stops at
the operator, Sec. 1); this module restates their textbook definitions:

* ``bf16`` -- round to the nearest bfloat16 (8 significant bits, ties to
  even), the storage format of weights and activations on the GPU.
* ``forward`` / ``backward`` -- the MLP  h1 = relu(W1 x + b1),
  h2 = relu(W2 h1 + b2), y = W3 h2 + b3  and the gradient of the loss
  L = mean over B x out of (y - t)^2, by the chain rule, in float64.  With
  ``rounded=True`` the values the GPU stores in bfloat16 (x, the weights,
  h1, h2, dL/dy, dL/dh2, dL/dh1) are rounded at the same points, so that
  the remaining differences are the order of FP32 accumulation.
* ``adam`` -- one Adam step (Kingma & Ba, 2015, Algorithm 1).
* ``patches`` / ``precondition`` -- the patch of a cell (cell and six face
  neighbours, zero outside the domain) of q = BJ r (q_T = A_TT^{-1} r_T),
  its norm s_T, and z_T = q_T + s_T (N(p_T / s_T) - N(-p_T / s_T)) / 2
  (the odd part of the network, so that z(-r) = -z(r)).

Public parameter layout: W1 [H x in] | b1 [H] | W2 [H x H] | b2 [H] |
W3 [out x H] | b3 [out], row-major.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 256


def bf16(x) -> np.ndarray:
    """Nearest bfloat16 value (ties to even) of each entry, as float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    r = np.ldexp(np.round(np.ldexp(m, 8)), e - 8)  # 8 significant bits, half to even
    return np.where(np.isfinite(x), r, x)


def sizes(k: int):
    nb = (k + 1) ** 3
    return 7 * nb, nb


def unpack(params: np.ndarray, k: int, hidden: int = HIDDEN):
    nin, nout = sizes(k)
    p = np.asarray(params, dtype=np.float64)
    o = 0
    out = []
    for shape in ((hidden, nin), (hidden,), (hidden, hidden), (hidden,), (nout, hidden), (nout,)):
        n = int(np.prod(shape))
        out.append(p[o:o + n].reshape(shape))
        o += n
    assert o == p.size, "parameter count does not match the layout"
    return out


def pack(blocks) -> np.ndarray:
    return np.concatenate([np.asarray(b, dtype=np.float64).ravel() for b in blocks])


def nparams(k: int, hidden: int = HIDDEN) -> int:
    nin, nout = sizes(k)
    return hidden * nin + hidden + hidden * hidden + hidden + nout * hidden + nout


def _r(a, rounded):
    return bf16(a) if rounded else np.asarray(a, dtype=np.float64)


def forward(params, X, k: int, rounded: bool = True):
    """Network outputs y (B x out) and the intermediate values."""
    W1, b1, W2, b2, W3, b3 = unpack(params, k)
    W1, W2, W3 = _r(W1, rounded), _r(W2, rounded), _r(W3, rounded)
    x = _r(X, rounded)
    h1 = _r(np.maximum(x @ W1.T + b1, 0.0), rounded)
    h2 = _r(np.maximum(h1 @ W2.T + b2, 0.0), rounded)
    y = h2 @ W3.T + b3
    return y, (x, h1, h2, W1, W2, W3)


def loss(params, X, T, k: int, rounded: bool = True) -> float:
    y, _ = forward(params, X, k, rounded)
    return float(np.mean((y - T) ** 2))


def backward(params, X, T, k: int, rounded: bool = True):
    """(loss, gradient in the public layout)."""
    y, (x, h1, h2, W1, W2, W3) = forward(params, X, k, rounded)
    B, nout = y.shape
    L = float(np.mean((y - T) ** 2))
    dy = _r(2.0 * (y - T) / (B * nout), rounded)
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dh2 = _r((dy @ W3) * (h2 > 0), rounded)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = _r((dh2 @ W2) * (h1 > 0), rounded)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(axis=0)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step at step number t (1-based); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def neighbours(ncell, c: int):
    """Cell c and its face neighbours in the order T, -x, +x, -y, +y, -z, +z
    (None outside the domain); cell index c = i1 + N1 (i2 + N2 i3)."""
    N1, N2, N3 = ncell
    i = [c % N1, (c // N1) % N2, c // (N1 * N2)]
    out = [c]
    for a in range(3):
        for step in (-1, +1):
            j = list(i)
            j[a] += step
            if 0 <= j[a] < (N1, N2, N3)[a]:
                out.append(j[0] + N1 * (j[1] + N2 * j[2]))
            else:
                out.append(None)
    return out


def patches(r: np.ndarray, ncell, k: int, cells):
    """Rows p_T (len(cells) x 7 nb) and norms s_T."""
    nb = (k + 1) ** 3
    R = np.asarray(r, dtype=np.float64).reshape(-1, nb)
    P = np.zeros((len(cells), 7 * nb))
    for row, c in enumerate(cells):
        for q, cn in enumerate(neighbours(ncell, int(c))):
            if cn is not None:
                P[row, q * nb:(q + 1) * nb] = R[cn]
    return P, np.linalg.norm(P, axis=1)


def precondition(params, r: np.ndarray, ncell, k: int, blocks: np.ndarray, rounded: bool = True):
    """z = q_T + s_T (N(p_T / s_T) - N(-p_T / s_T)) / 2 for every cell,
    q_T = A_TT^{-1} r_T (blocks: A_TT), p_T the patch of q."""
    nb = (k + 1) ** 3
    ncells = int(np.prod(ncell))
    q = np.linalg.solve(blocks, np.asarray(r, dtype=np.float64).reshape(ncells, nb)[:, :, None])[:, :, 0]
    P, s = patches(q.ravel(), ncell, k, range(ncells))
    safe = np.where(s > 0, s, 1.0)
    yp, _ = forward(params, P / safe[:, None], k, rounded)
    ym, _ = forward(params, -P / safe[:, None], k, rounded)
    corr = np.where(s[:, None] > 0, s[:, None] * 0.5 * (yp - ym), 0.0)
    return (q + corr).ravel()
