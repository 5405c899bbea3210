"""The C-ABI library: loads, exports every symbol include/dg.h declares, and
rejects invalid problems before touching the GPU (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1711_10885_amd import binding, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1711_10885_amd import build
        build.build()
    return binding.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name


def _struct(prob, **over):
    s = binding._Problem()
    keep = [np.ascontiguousarray(prob.nodes[a], dtype=np.float64) for a in range(3)]
    for a in range(3):
        s.ncell[a] = prob.ncell[a]
        s.nodes[a] = keep[a].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.b_axis[a] = prob.b_axis[a]
    s.k = prob.k
    for i, v in enumerate(np.asarray(prob.K).ravel()):
        s.K[i] = v
    s.c = prob.c
    s.sigma = prob.sigma
    for key, val in over.items():
        if key == "K":
            for i, v in enumerate(np.asarray(val).ravel()):
                s.K[i] = v
        elif key == "b_axis0":
            s.b_axis[0] = val
        else:
            setattr(s, key, val)
    return s, keep


@pytest.mark.parametrize("over,msg", [
    (dict(k=0), "k must be"),
    (dict(k=11), "k must be"),
    (dict(sigma=0.0), "sigma"),
    (dict(K=np.diag([1.0, -1.0, 1.0])), "positive definite"),
    (dict(K=np.array([[1, 0.5, 0], [0, 1, 0], [0, 0, 1.0]])), "symmetric"),
    (dict(b_axis0=3), "b_axis"),
    (dict(c=float("nan")), "c must be finite"),
    (dict(flags=512), "unknown flag"),
    (dict(quad_extra=1), "quad_extra"),
    (dict(k=9, quad_extra=2), "raised quadrature supports"),
    (dict(k=8, flags=2), "block Jacobi supports"),
])
def test_setup_rejects_invalid_problems(over, msg):
    lib = _lib()
    s, keep = _struct(workloads.poisson_k2_8(), **over)
    h = ctypes.c_void_p()
    rc = lib.dg_setup(ctypes.byref(s), ctypes.byref(h))
    assert rc == binding.DG_EINVAL
    assert msg in lib.dg_last_error().decode()
    assert not h.value


def test_block_jacobi_rejects_an_odd_periodic_axis():
    """Two-colour probing needs the first and last cells of a periodic axis
    to differ in parity: an odd periodic axis (> 1 cell) is rejected before
    any device work."""
    lib = _lib()
    s, keep = _struct(workloads.random_problem(60, ncell=(3, 2, 2), k=1), flags=2 | 4)
    h = ctypes.c_void_p()
    assert lib.dg_setup(ctypes.byref(s), ctypes.byref(h)) == binding.DG_EINVAL
    assert "even number of cells" in lib.dg_last_error().decode()
    assert not h.value


def test_setup_rejects_a_non_finite_product_field():
    lib = _lib()
    s, keep = _struct(workloads.poisson_k2_8(), flags=binding.DG_B_PRODUCT)
    s.b_amp[0] = 1.0
    s.b_freq[4] = float("inf")
    h = ctypes.c_void_p()
    assert lib.dg_setup(ctypes.byref(s), ctypes.byref(h)) == binding.DG_EINVAL
    assert "product-form b" in lib.dg_last_error().decode()
    assert not h.value


@pytest.mark.parametrize("coef,msg", [((0.5, 0.0, -1.0), "positive on the mesh"), ((1.0, float("nan"), 0.0), "finite")])
def test_setup_rejects_a_bad_kappa_polynomial(coef, msg):
    """kp_2(s) = 0.5 - s^2 vanishes inside [0, 1]; a NaN coefficient is not finite."""
    lib = _lib()
    s, keep = _struct(workloads.poisson_k2_8(), flags=binding.DG_KAPPA_POLY)
    for t, v in enumerate((1.0, 0.0, 0.0, 1.0, 0.0, 0.0) + coef):
        s.kappa_poly[t] = v
    h = ctypes.c_void_p()
    assert lib.dg_setup(ctypes.byref(s), ctypes.byref(h)) == binding.DG_EINVAL
    assert msg in lib.dg_last_error().decode()
    assert not h.value


@pytest.mark.parametrize("case", ["singular", "nan", "sine_b"])
def test_setup_rejects_invalid_affine_problems(case):
    lib = _lib()
    p = workloads.random_problem(70, ncell=(2, 2, 2), k=1, b="sine" if case == "sine_b" else "const")
    flags = binding.DG_AFFINE | (binding.DG_KAPPA_POLY if case == "kpoly" else 0)
    s, keep = _struct(p, flags=flags)
    A = {"singular": [1, 2, 0, 2, 4, 0, 0, 0, 1], "nan": [1, 0, 0, 0, float("nan"), 0, 0, 0, 1]}.get(
        case, [1, 0.3, 0, 0, 1, 0, 0, 0, 1])
    for i, v in enumerate(A):
        s.affine[i] = v
    if case == "kpoly":
        for t, v in enumerate((1.0, 0, 0, 1.0, 0, 0, 1.0, 0, 0)):
            s.kappa_poly[t] = v
    if case == "sine_b":
        s.b_sin[0] = 1.0
    h = ctypes.c_void_p()
    assert lib.dg_setup(ctypes.byref(s), ctypes.byref(h)) == binding.DG_EINVAL
    msg = {"singular": "invertible", "nan": "finite"}.get(case, "constant b")
    assert msg in lib.dg_last_error().decode()
    assert not h.value


def test_setup_rejects_non_increasing_nodes():
    lib = _lib()
    p = workloads.poisson_k2_8()
    bad = p.with_(nodes=(p.nodes[0], np.concatenate([[0.0, 0.5, 0.4], p.nodes[1][3:]]), p.nodes[2]))
    s, keep = _struct(bad)
    h = ctypes.c_void_p()
    assert lib.dg_setup(ctypes.byref(s), ctypes.byref(h)) == binding.DG_EINVAL
    assert "increasing" in lib.dg_last_error().decode()


def test_null_arguments():
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.dg_setup(None, ctypes.byref(h)) == binding.DG_EINVAL
    assert lib.dg_apply(None, None, None, None) == binding.DG_EINVAL
    assert lib.dg_ndof(None) == -1
    assert lib.dg_heun(None, None, None, 1e-3, 1, None) == binding.DG_EINVAL
    assert "handle" in lib.dg_last_error().decode()
    lib.dg_destroy(None)


@pytest.mark.parametrize("cname,pystruct", [("dg_problem", "_Problem"), ("dg_solve_opts", "SolveOpts"),
                                            ("dg_solve_stats", "SolveStats"), ("dg_learn_opts", "LearnOpts"),
                                            ("dg_learn_stats", "LearnStats")])
def test_binding_structs_match_the_header_layout(cname, pystruct, tmp_path):
    """Size and field offsets of every struct, as the C compiler lays it out
    from include/dg.h, against the ctypes mirror in the binding."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    st = getattr(binding, pystruct)
    names = [f for f, _ in st._fields_]
    body = "".join(f'  printf("%zu\\n", offsetof({cname}, {f}));\n' for f in names)
    src = tmp_path / "layout.c"
    src.write_text(f'#include <stddef.h>\n#include <stdio.h>\n#include "dg.h"\nint main(void) {{\n'
                   f'  printf("%zu\\n", sizeof({cname}));\n{body}  return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(st), (cname, out[0], ctypes.sizeof(st))
    assert out[1:] == [getattr(st, f).offset for f in names], cname


def _unbound_handle(k=3):
    """A DG object without a library handle: the network entry points must
    reject bad rows before any pointer reaches the library."""
    dg = binding.DG.__new__(binding.DG)
    dg._h = None
    dg.k = k
    return dg


@pytest.mark.parametrize("method", ["mlp_forward", "mlp_grad", "mlp_step"])
@pytest.mark.parametrize("case,exc", [("numpy", TypeError), ("float64", TypeError), ("narrow", ValueError),
                                      ("rows_not_64", ValueError), ("strided", ValueError),
                                      ("cpu", ValueError), ("T_rows", ValueError), ("T_cols", ValueError)])
def test_network_rows_are_validated_before_the_library(method, case, exc):
    import torch
    dg = _unbound_handle(3)
    nin, nout = 7 * 64, 64
    X = torch.zeros((128, nin), dtype=torch.float32)
    T = torch.zeros((128, nout), dtype=torch.float32)
    if case == "numpy":
        X = X.numpy()
    elif case == "float64":
        X = X.double()
    elif case == "narrow":
        X = X[:, : nin - 1].contiguous()
    elif case == "rows_not_64":
        X, T = X[:100].contiguous(), T[:100].contiguous()
    elif case == "strided":
        X = torch.zeros((128, 2 * nin), dtype=torch.float32)[:, ::2]
    elif case == "T_rows":
        T = T[:64].contiguous()
    elif case == "T_cols":
        T = torch.zeros((128, nout + 1), dtype=torch.float32)
    if method == "mlp_forward" and case.startswith("T_"):
        pytest.skip("mlp_forward takes no targets")
    with pytest.raises(exc):
        if method == "mlp_forward":
            dg.mlp_forward(X)
        elif method == "mlp_grad":
            dg.mlp_grad(X, T)
        else:
            dg.mlp_step(X, T)


@pytest.mark.parametrize("case,msg", [
    ("periodic", "excludes"), ("block_jacobi", "excludes"), ("affine", "excludes"), ("k8", "k <= 7"),
    ("quad_extra", "quad_extra must be 0, 2"), ("inverted", "determinant must be positive"),
    ("no_vertices", "needs vertices"), ("nan", "vertices must be finite"), ("kpoly", "positive on the mesh"),
])
def test_setup_rejects_invalid_multilinear_problems(case, msg):
    """Vertex meshes are validated before any device work: exclusive flags,
    degree and rule, cell orientation (det J > 0 at the corners and centre),
    finite vertices, the diffusion factor on the vertices' bounding box."""
    lib = _lib()
    k = 8 if case == "k8" else 2
    p = workloads.random_problem(80, ncell=(2, 2, 2), k=k, b="const")
    V = workloads.curved_vertices((2, 2, 2), eps=0.03)
    if case == "inverted":
        V = V.copy()
        V[1, 1, 1] = V[2, 2, 2] + 0.3  # interior vertex pushed past the far corner
    if case == "nan":
        V = V.copy()
        V[0, 0, 1, 2] = float("nan")
    flags = binding.DG_MULTILINEAR | {"periodic": binding.DG_PERIODIC_Y, "block_jacobi": binding.DG_WITH_BLOCK_JACOBI,
                                      "affine": binding.DG_AFFINE, "kpoly": binding.DG_KAPPA_POLY}.get(case, 0)
    s, keep = _struct(p, flags=flags, quad_extra=1 if case == "quad_extra" else 0)
    Vf = np.ascontiguousarray(V, dtype=np.float64).ravel()
    if case != "no_vertices":
        s.vertices = Vf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if case == "kpoly":  # kp_0(s) = 0.25 - s^2 vanishes inside [0, 1]
        for t, v in enumerate((0.25, 0.0, -1.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0)):
            s.kappa_poly[t] = v
    h = ctypes.c_void_p()
    assert lib.dg_setup(ctypes.byref(s), ctypes.byref(h)) == binding.DG_EINVAL
    assert msg in lib.dg_last_error().decode(), lib.dg_last_error().decode()
    assert not h.value
