"""dg_heun_noalloc, the Heun entry point that allocates nothing, against
dg_heun through the C ABI.

Both run the same kernels in the same order; the non-allocating one takes
its stage workspace from the library's fixed per-device array instead of the
handle's.  Two calls in a row on different handles, the second with a
smaller input, so the second reads an array that still holds the first
call's data.  Bar: the states after the steps agree to 1e-12 relative
(2-norm and max-norm); the two are expected to be identical.
"""
import numpy as np
import pytest

from paper_1711_10885_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _problem(seed, ncell, k, periodic=(True, True, False), **kw):
    p = W.random_problem(seed, ncell=ncell, k=k, b="sine", periodic=periodic)
    return p.with_(K=np.asarray(p.K) * 1e-3, **kw)


def _pair(p, u0, dt, nsteps, variant=0, f=None):
    """(dg_heun result, dg_heun_noalloc result) from the same start."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    with binding.DG(p) as dg:
        dg.set_kernel(variant)
        fd = None if f is None else torch.from_numpy(f).cuda()
        ua = torch.from_numpy(u0.copy()).cuda()
        dg.heun(ua, dt, nsteps, f=fd)
        ub = torch.from_numpy(u0.copy()).cuda()
        dg.heun_noalloc(ub, dt, nsteps, f=fd)
        torch.cuda.synchronize()
        return ua.cpu().numpy(), ub.cpu().numpy()


def _check(a, b, what):
    e2 = np.linalg.norm(a - b) / np.linalg.norm(a)
    emax = np.abs(a - b).max() / np.abs(a).max()
    print(f"{what}: rel2 {e2:.2e} relmax {emax:.2e} identical {np.array_equal(a, b)}", flush=True)
    assert e2 <= TOL and emax <= TOL, (what, e2, emax)


@pytest.mark.parametrize("variant", [0, 1])
def test_noalloc_matches_heun_two_calls_second_smaller(variant):
    big = _problem(21, (6, 5, 4), 3)
    small = _problem(22, (3, 2, 2), 2)
    for p, seed in ((big, 5), (small, 6)):
        u0 = W.random_vector(p.ndof, seed)
        f = W.random_vector(p.ndof, seed + 100)
        print(f"variant {variant} ncell {p.ncell} k {p.k} ndof {p.ndof}", flush=True)
        a, b = _pair(p, u0, 2e-3, 4, variant, f)
        _check(a, b, f"variant {variant} ndof {p.ndof}")


def test_noalloc_raised_rule_two_calls_second_smaller():
    big = _problem(23, (4, 4, 3), 3, quad_extra=2)
    small = _problem(24, (2, 2, 2), 1, quad_extra=2)
    for p, seed in ((big, 7), (small, 8)):
        u0 = W.random_vector(p.ndof, seed)
        print(f"raised rule ncell {p.ncell} k {p.k} ndof {p.ndof}", flush=True)
        a, b = _pair(p, u0, 2e-3, 3)
        _check(a, b, f"raised rule ndof {p.ndof}")


def test_noalloc_rejects_sizes_beyond_the_static_array():
    """8 DOF per cell at k = 1: 128 x 128 x 65 cells need 8,519,680 doubles on
    the fused path, above the 64 MiB array; the call fails before any launch."""
    torch = _torch()
    from paper_1711_10885_amd import binding
    p = W.random_problem(25, ncell=(128, 128, 65), k=1, b="sine", kappa=False)
    with binding.DG(p) as dg:
        u = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        with pytest.raises(binding.DGError) as e:
            dg.heun_noalloc(u, 1e-3, 1)
        assert "static limit" in str(e.value)
        assert e.value.status == binding.DG_EINVAL
