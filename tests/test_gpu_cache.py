"""Setup-cache semantics on the GPU (Section 2.1, "C++/CUDA backend": a hit
with new values repeats the numeric setup): in-place refresh when only the
cache holds a hierarchy, copy on write when another caller's handle still
holds it, a refresh that fails part-way is never handed out again, and with
a strength threshold a refresh equals a fresh setup of the new values."""
import numpy as np
import pytest

from paper_2606_09001_amd import matrices as M
from gpu_util import dev, host, assert_hierarchy_bitexact

pytestmark = pytest.mark.gpu


def _values(N, seeds):
    rp, ci, _ = M.diffusion(np.ones((N, N)))
    return rp, ci, [M.diffusion(np.exp(M.grf(N, 2, seed=s)))[2] for s in seeds]


def test_refresh_in_place_and_copy_on_write():
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy, make_preconditioner
    N = 40
    rp, ci, (v1, v2) = _values(N, (11, 12))
    kw = dict(max_coarse=16)
    O1 = oracle.OracleHierarchy(rp, ci, v1, **kw)
    O2 = oracle.OracleHierarchy(rp, ci, v2, **kw)
    r = M.rhs_normal(N * N, 3)
    H1 = AmgHierarchy(dev(rp), dev(ci), dev(v1), **kw)
    pre1 = make_preconditioner(dev(rp), dev(ci), dev(v1), **kw)     # a hit: shares H1's hierarchy
    z_before = host(pre1(dev(r)))
    # H1 and the preconditioner hold v1's hierarchy: v2 gets a new one (cold)
    H2 = AmgHierarchy(dev(rp), dev(ci), dev(v2), **kw)
    _, i2 = H2.solve(dev(r), 1e-8)
    assert i2["cache_event"] == 0
    assert_hierarchy_bitexact(H2, O2)
    assert_hierarchy_bitexact(H1, O1)
    assert np.array_equal(host(pre1(dev(r))), z_before)
    del pre1
    H1.close()
    H2.close()
    # only the cache holds v2's hierarchy: v1 refreshes it in place
    H3 = AmgHierarchy(dev(rp), dev(ci), dev(v1), **kw)
    _, i3 = H3.solve(dev(r), 1e-8)
    assert i3["cache_event"] == 2
    assert_hierarchy_bitexact(H3, O1)
    # amg_update_values on a shared hierarchy: the caller gets its own
    H4 = AmgHierarchy(dev(rp), dev(ci), dev(v1), **kw)                # hit on H3's hierarchy
    H3.update_values(dev(v2))
    assert_hierarchy_bitexact(H3, O2)
    assert_hierarchy_bitexact(H4, O1)
    x4, _ = H4.solve(dev(r), 1e-10)
    xo, _ = O1.pcg(r, tol=1e-10)
    assert np.linalg.norm(host(x4) - xo) <= 1e-7 * np.linalg.norm(xo)
    # H4 now alone (with the cache): in place
    H4.update_values(dev(v2))
    assert_hierarchy_bitexact(H4, O2)


@pytest.mark.parametrize("bad", ["indefinite", "zero_diagonal"])
def test_failed_refresh_is_never_handed_out(bad):
    import oracle
    from paper_2606_09001_amd import _lib
    from paper_2606_09001_amd.solver import AmgHierarchy
    N = 32
    rp, ci, (v,) = _values(N, (21,))
    kw = dict(max_coarse=16)
    if bad == "indefinite":
        vb = -v                       # refresh reaches the coarse Cholesky and breaks down there
        st = _lib.AMG_ERR_BREAKDOWN
    else:
        vb = v.copy()
        i = N * N // 2 + N // 2
        k = rp[i] + int(np.searchsorted(ci[rp[i]:rp[i + 1]], i))
        assert ci[k] == i
        vb[k] = 0.0                   # a zero diagonal: level 0's numerics fail
        st = _lib.AMG_ERR_ZERO_DIAG
    b = M.rhs_normal(N * N, 4)
    O = oracle.OracleHierarchy(rp, ci, v, **kw)
    xo, io = O.pcg(b, tol=1e-10)
    H = AmgHierarchy(dev(rp), dev(ci), dev(v), **kw)
    H.close()
    print(f"[case] failed refresh ({bad}) through amg_setup", flush=True)
    for _ in range(2):           # the second attempt must fail the same way, not hit the cache
        with pytest.raises(_lib.AmgError) as e:
            AmgHierarchy(dev(rp), dev(ci), dev(vb), **kw)
        assert e.value.status == st
    Hg = AmgHierarchy(dev(rp), dev(ci), dev(v), **kw)
    x, info = Hg.solve(dev(b), 1e-10)
    assert info["cache_event"] == 0 and info["status"] == 0
    assert np.linalg.norm(host(x) - xo) <= 1e-7 * np.linalg.norm(xo)
    print(f"[case] failed refresh ({bad}) through amg_update_values", flush=True)
    with pytest.raises(_lib.AmgError) as e:
        Hg.update_values(dev(vb))
    assert e.value.status == st
    for call in (lambda: Hg.solve(dev(b), 1e-10), lambda: Hg.apply_vcycle(dev(b)),
                 lambda: Hg.solve_adjoint(dev(b), 1e-10)):
        with pytest.raises(_lib.AmgError) as e:
            call()
        assert e.value.status == st
    Hg.update_values(dev(v))
    assert_hierarchy_bitexact(Hg, O)
    x, info = Hg.solve(dev(b), 1e-10)
    assert info["status"] == 0 and abs(info["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(host(x) - xo) <= 1e-7 * np.linalg.norm(xo)


def test_theta_refresh_equals_fresh_setup():
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    N = 48
    rp, ci, (v1, v2) = _values(N, (31, 32))
    kw = dict(max_coarse=16, theta=0.25)
    O1 = oracle.OracleHierarchy(rp, ci, v1, **kw)
    O2 = oracle.OracleHierarchy(rp, ci, v2, **kw)
    assert not np.array_equal(O1.level(0)["agg"], O2.level(0)["agg"])
    H = AmgHierarchy(dev(rp), dev(ci), dev(v1), **kw)
    assert_hierarchy_bitexact(H, O1)
    H.close()
    H2 = AmgHierarchy(dev(rp), dev(ci), dev(v2), **kw)       # refresh of the cached hierarchy
    b = M.rhs_normal(N * N, 5)
    x, info = H2.solve(dev(b), 1e-10)
    assert info["cache_event"] == 2
    assert_hierarchy_bitexact(H2, O2)
    xo, io = O2.pcg(b, tol=1e-10)
    assert info["status"] == 0 and abs(info["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(host(x) - xo) <= 1e-7 * np.linalg.norm(xo)
    H2.update_values(dev(v1))
    assert_hierarchy_bitexact(H2, O1)
