"""The one-workgroup PCG solve of small hierarchies (amg_params.fused_small)
against the FP64 oracle and against the per-kernel path on the same handle's
hierarchy: the 32^2 Poisson workload (b seed 0, tol 1e-10), small 2D/3D
diffusion systems and systems whose coarsest levels hold 12, 25 and 63 rows;
converged counts within one of the oracle's, true residuals, fixed-count
iterate parity at 1e-9, the flexible recurrence, the iteration limit, a zero
right-hand side and bitwise reproducibility."""
import numpy as np
import pytest

from paper_2606_09001_amd import matrices as M
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _systems():
    yield "poisson2d_32", M.poisson(32, 2), 0, 1e-10, {}
    yield "diffusion2d_24", M.diffusion(np.exp(M.grf(24, 2, seed=7))), 3, 1e-10, {}
    yield "diffusion3d_10", M.diffusion(np.exp(M.grf(10, 3, seed=8))), 4, 1e-9, {}
    # tiny coarsest levels: 12 (padded 16, waves without columns), 25 and 63
    yield "poisson2d_8", M.poisson(8, 2), 5, 1e-10, {"max_coarse": 16}
    yield "poisson3d_6", M.poisson(6, 3), 6, 1e-10, {"max_coarse": 30}
    yield "poisson2d_20", M.poisson(20, 2), 7, 1e-10, {}


@pytest.mark.parametrize("case", list(_systems()), ids=lambda c: c[0])
def test_single_workgroup_vs_oracle(case):
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    name, (rp, ci, v), seed, tol, kw = case
    n = len(rp) - 1
    b = M.rhs_normal(n, seed)
    print(f"[case] single workgroup {name} n={n}", flush=True)
    H = AmgHierarchy(dev(rp), dev(ci), dev(v), **kw)
    st = H.stats()
    assert st["single_workgroup"] == 1 and st["num_levels"] == 2
    O = oracle.OracleHierarchy(rp, ci, v, **kw)
    x, info = H.solve(dev(b), tol)
    xo, io = O.pcg(b, tol=tol)
    rr = oracle.rel_residual(rp, ci, v, b, host(x))
    assert info["status"] == 0 and rr <= tol and abs(info["rel_resid"] - rr) <= 1e-6 * rr
    assert abs(info["iters"] - io["iters"]) <= 1, (info["iters"], io["iters"])
    # the per-kernel path on the same hierarchy (cache hit), same tolerance
    Hk = AmgHierarchy(dev(rp), dev(ci), dev(v), fused_small=0, **kw)
    xk, ik = Hk.solve(dev(b), tol)
    assert ik["cache_event"] == 1 and abs(ik["iters"] - info["iters"]) <= 1
    # iterate parity at fixed counts (tol = 0 runs exactly maxiter iterations)
    for k in (1, 5, io["iters"]):
        Hf = AmgHierarchy(dev(rp), dev(ci), dev(v), maxiter=k, **kw)
        xf, fi = Hf.solve(dev(b), 0.0)
        xof, _ = O.pcg(b, tol=0.0, maxiter=k)
        err = np.linalg.norm(host(xf) - xof) / np.linalg.norm(xof)
        assert fi["iters"] == k and fi["status"] == 1 and err <= 1e-9, (k, err)
    # bitwise reproducible
    x2, _ = H.solve(dev(b), tol)
    assert np.array_equal(host(x).view(np.int64), host(x2).view(np.int64))


def test_single_workgroup_flexible_limits_and_zero():
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    rp, ci, v = M.poisson(32, 2)
    n = len(rp) - 1
    b = M.rhs_normal(n, 0)
    O = oracle.OracleHierarchy(rp, ci, v)
    # flexible (Polak-Ribiere) beta: the same iterates as the oracle's flexible PCG
    Hf = AmgHierarchy(dev(rp), dev(ci), dev(v), flexible=1, maxiter=9)
    xf, fi = Hf.solve(dev(b), 0.0)
    xo, _ = O.pcg(b, tol=0.0, maxiter=9, flexible=True)
    assert fi["iters"] == 9 and np.linalg.norm(host(xf) - xo) <= 1e-9 * np.linalg.norm(xo)
    # iteration limit: not converged, x is the last iterate
    Hl = AmgHierarchy(dev(rp), dev(ci), dev(v), maxiter=3)
    xl, li = Hl.solve(dev(b), 1e-12)
    xo3, _ = O.pcg(b, tol=0.0, maxiter=3)
    assert li["status"] == 1 and li["iters"] == 3
    assert np.linalg.norm(host(xl) - xo3) <= 1e-9 * np.linalg.norm(xo3)
    # zero right-hand side: x = 0 in 0 iterations
    z, zi = Hl.solve(dev(np.zeros(n)), 1e-8)
    assert zi["status"] == 0 and zi["iters"] == 0 and not host(z).any()
    # maxiter = 0
    H0 = AmgHierarchy(dev(rp), dev(ci), dev(v), maxiter=0)
    x0, i0 = H0.solve(dev(b), 1e-8)
    assert i0["iters"] == 0 and i0["status"] == 1 and not host(x0).any()


def test_single_workgroup_not_taken_when_ineligible():
    from paper_2606_09001_amd.solver import AmgHierarchy
    # three levels (64^2) and the FP32 cycle fall back to the per-kernel path
    rp, ci, v = M.poisson(64, 2)
    assert AmgHierarchy(dev(rp), dev(ci), dev(v)).stats()["single_workgroup"] == 0
    rp, ci, v = M.poisson(32, 2)
    assert AmgHierarchy(dev(rp), dev(ci), dev(v), vcycle_prec="fp32").stats()["single_workgroup"] == 0
