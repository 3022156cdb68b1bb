"""The allocation-free PCG solve (amg_solve_noalloc, for callers that cannot
allocate device memory) against amg_solve on the same handles, through the
C ABI: identical kernels in the same order, so x, the iteration count and
the true residual must be identical bit for bit.  Two calls in a row on one
GPU, the second on a smaller system (the static workspace keeps the first
call's contents), then the limits."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2606_09001_amd import _lib
from paper_2606_09001_amd import matrices as M
from paper_2606_09001_amd.solver import AmgHierarchy

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _call(fn, H, b, tol):
    x = torch.full_like(b, float("nan"))
    info = _lib.amg_info()
    s = torch.cuda.current_stream().cuda_stream
    if fn == "noalloc":
        st = _lib.load().amg_solve_noalloc(H.handle, b.data_ptr(), x.data_ptr(), float(tol), C.byref(info), s)
    else:
        st = _lib.load().amg_solve(H.handle, b.data_ptr(), x.data_ptr(), float(tol), 1, C.byref(info), s)
    torch.cuda.synchronize()
    return st, x.cpu().numpy(), info.to_dict()


def _same(H, b, tol):
    st0, x0, i0 = _call("solve", H, b, tol)
    st1, x1, i1 = _call("noalloc", H, b, tol)
    assert st0 == st1 == _lib.AMG_OK, (st0, st1)
    assert i0["iters"] == i1["iters"] and i0["restarts"] == i1["restarts"], (i0, i1)
    assert np.array_equal(x0.view(np.int64), x1.view(np.int64))
    assert i0["rel_resid"] == i1["rel_resid"] <= tol
    return i1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_solve_twice_second_smaller(prec):
    # first call: 3D lognormal diffusion 48^3 (110,592 unknowns)
    N1 = 48
    rp, ci, v = M.diffusion(np.exp(M.grf(N1, 3, seed=2)))
    print(f"[case] noalloc {prec} diffusion {N1}^3 n={len(rp) - 1}", flush=True)
    H1 = AmgHierarchy(_dev(rp), _dev(ci), _dev(v), vcycle_prec=prec)
    b1 = _dev(M.rhs_normal(len(rp) - 1, 100))
    i1 = _same(H1, b1, 1e-8)
    assert i1["iters"] > 5
    # second call: a smaller system, 2D Poisson 40^2 with V(2,2) and the L1 smoother
    rp2, ci2, v2 = M.poisson(40, 2)
    print(f"[case] noalloc {prec} poisson 40^2 n={len(rp2) - 1}", flush=True)
    H2 = AmgHierarchy(_dev(rp2), _dev(ci2), _dev(v2), vcycle_prec=prec, nu_pre=2, nu_post=2, smoother="l1",
                      max_coarse=32)
    b2 = _dev(M.rhs_normal(len(rp2) - 1, 0))
    _same(H2, b2, 1e-10)
    # the first handle again, after the smaller call
    _same(H1, b1, 1e-8)
    # zero right-hand side: x = 0 in 0 iterations on both entry points
    z = torch.zeros_like(b2)
    st, x, info = _call("noalloc", H2, z, 1e-8)
    assert st == _lib.AMG_OK and info["iters"] == 0 and not x.any()
    H1.close()
    H2.close()


def test_noalloc_limits():
    # BiCGSTAB handles and widths other than one column are not served
    rp, ci, v = M.poisson(16, 2)
    Hb = AmgHierarchy(_dev(rp), _dev(ci), _dev(v), solver="bicgstab")
    b = _dev(M.rhs_normal(len(rp) - 1, 1))
    st, _, _ = _call("noalloc", Hb, b, 1e-8)
    assert st == _lib.AMG_ERR_INVALID_ARG
    Hb.close()
    # one row beyond the workspace: refused before any launch
    N = 129
    rp, ci, v = M.poisson(N, 3)
    assert len(rp) - 1 > _lib.AMG_NOALLOC_MAX_N
    print(f"[case] noalloc limit n={len(rp) - 1}", flush=True)
    H = AmgHierarchy(_dev(rp), _dev(ci), _dev(v))
    b = _dev(M.rhs_normal(len(rp) - 1, 1))
    st, x, _ = _call("noalloc", H, b, 1e-8)
    assert st == _lib.AMG_ERR_SCRATCH_LIMIT
    assert np.isnan(x).all()          # nothing was written
    assert _lib.status_string(st) == "AMG_ERR_SCRATCH_LIMIT"
    H.close()
