"""The compile-time 1D tables of the fused kernels (gl_tables.inc).

Pins: the committed header is exactly what its generator writes, and its
entries match numpy's Gauss-Legendre rule and Legendre series (library
routines) and the closed-form endpoint values theta_j(1) = sqrt(2j+1),
theta_j'(1) = j(j+1) sqrt(2j+1)."""
import importlib.util
import math
import os
import re

import numpy as np
from numpy.polynomial import legendre as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1711_10885_amd", "csrc")


def _tables():
    s = open(os.path.join(CSRC, "gl_tables.inc")).read()
    out = {}
    for m in re.finditer(r"struct GLTab<(\d+)> \{\s*static constexpr double v\[(\d+)\] = \{(.*?)\};", s, re.S):
        vals = [float.fromhex(x.strip()) for x in m.group(3).split(",")]
        assert len(vals) == int(m.group(2))
        out[int(m.group(1))] = np.array(vals)
    return out


def test_header_is_generator_output(tmp_path):
    spec = importlib.util.spec_from_file_location("gen", os.path.join(CSRC, "gen_gl_tables.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    for n in (2, 5, 8, 11, 12, 13):
        want = [float(v) for v in gen.table(n)]
        assert np.array_equal(np.array(want), _tables()[n])


def test_entries_match_library_and_closed_forms():
    T = _tables()
    assert sorted(T) == list(range(2, 14))
    for n, v in T.items():
        H = (n + 1) // 2
        x, w = L.leggauss(n)
        xi, w = 0.5 * (x + 1), 0.5 * w
        Vr = v[:H * n].reshape(H, n)
        Dr = v[H * n:2 * H * n].reshape(H, n)
        e1 = v[2 * H * n:2 * H * n + n]
        f1 = v[2 * H * n + n:2 * H * n + 2 * n]
        wh = v[2 * H * n + 2 * n:2 * H * n + 2 * n + H]
        g = v[2 * H * n + 2 * n + H:]
        assert g.size == n
        # modal derivative: D = V G with G_kj = g_k g_j for k < j, j - k odd
        G = np.array([[g[k] * g[j] if (k < j and (j - k) % 2) else 0.0 for j in range(n)]
                      for k in range(n)])
        assert np.allclose(Vr @ G, Dr, rtol=0, atol=1e-12 * max(1, n * n))
        assert np.allclose(wh, w[:H], rtol=0, atol=1e-15)  # numpy: a few ulps
        for j in range(n):
            c = np.zeros(j + 1)
            c[j] = math.sqrt(2 * j + 1)
            assert np.allclose(Vr[:, j], L.legval(2 * xi[:H] - 1, c), rtol=0, atol=1e-13)
            assert np.allclose(Dr[:, j], 2 * L.legval(2 * xi[:H] - 1, L.legder(c)), rtol=0,
                               atol=1e-12 * max(1, j * j))
            assert abs(e1[j] - math.sqrt(2 * j + 1)) <= 1e-15 * math.sqrt(2 * j + 1)
            assert abs(f1[j] - j * (j + 1) * math.sqrt(2 * j + 1)) <= 1e-14 * max(1, j * j)
