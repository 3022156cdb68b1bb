"""Batched solves on the GPU vs the FP64 oracle solving each column alone.

Many right-hand sides of one matrix (row-major [n][k]) and many systems
sharing one pattern (values [nnz][S]); every column is an independent CG, so
per column: iteration count within one of the oracle's, true residual within
the tolerance, and at equal iteration counts the iterate within 1e-9.
Per-system hierarchies are bit-exact with the oracle run on that system.
"""
import numpy as np
import pytest
import torch

from paper_2606_09001_amd import matrices as M
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _oracle(rp, ci, v, **kw):
    import oracle
    return oracle.OracleHierarchy(rp, ci, v, **kw)


@pytest.mark.parametrize("k", [2, 5, 32])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_rhs(k, prec):
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    rp, ci, v = M.diffusion(np.exp(M.grf(20, 3, seed=3)))
    n = len(rp) - 1
    B = M.rhs_normal(n, 11, nrhs=k)
    print(f"[case] multi-rhs n={n} k={k} prec={prec}", flush=True)
    H = AmgHierarchy(dev(rp), dev(ci), dev(v), vcycle_prec=prec)
    X, info = H.solve(dev(B), 1e-9)
    cols = H.columns(k)
    O = _oracle(rp, ci, v)
    Xh = host(X)
    for c in range(k):
        xo, io = O.pcg(B[:, c].copy(), tol=1e-9)
        rr = oracle.rel_residual(rp, ci, v, B[:, c].copy(), Xh[:, c].copy())
        assert cols["status"][c] == 0 and rr <= 1e-9, (c, rr)
        assert abs(cols["rel_resid"][c] - rr) <= 1e-6 * rr + 1e-15
        if prec == "fp64":
            assert abs(cols["iters"][c] - io["iters"]) <= 1, (c, cols["iters"][c], io["iters"])
    assert info["iters"] == max(cols["iters"])
    if prec == "fp64":
        # iterate parity at a fixed iteration count for every column
        kk = 7
        Hk = AmgHierarchy(dev(rp), dev(ci), dev(v), maxiter=kk)
        Xk, _ = Hk.solve(dev(B), 0.0)
        Xkh = host(Xk)
        for c in range(k):
            xo, io = O.pcg(B[:, c].copy(), tol=0.0, maxiter=kk)
            assert np.linalg.norm(Xkh[:, c] - xo) <= 1e-9 * np.linalg.norm(xo)


def test_multi_rhs_matches_single_solves_bitwise_deterministic():
    from paper_2606_09001_amd.solver import AmgHierarchy
    rp, ci, v = M.poisson(30, 2)
    n = len(rp) - 1
    B = M.rhs_normal(n, 4, nrhs=8)
    H = AmgHierarchy(dev(rp), dev(ci), dev(v), max_coarse=32)
    X1, _ = H.solve(dev(B), 1e-10)
    X2, _ = H.solve(dev(B), 1e-10)
    assert torch.equal(X1, X2)
    # zero column and a finished column do not disturb the others
    B0 = B.copy()
    B0[:, 3] = 0.0
    X3, _ = H.solve(dev(B0), 1e-10)
    cols = H.columns(8)
    assert cols["iters"][3] == 0 and not host(X3)[:, 3].any()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_system(prec):
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    N, S = 16, 4
    vals = []
    for s in range(S):
        rp, ci, v = M.diffusion(np.exp(M.grf(N, 3, seed=1000 + s)))
        vals.append(v)
    V = np.ascontiguousarray(np.stack(vals, axis=1))   # [nnz][S]
    n = len(rp) - 1
    B = np.ascontiguousarray(np.stack([M.rhs_normal(n, 2000 + s) for s in range(S)], axis=1))
    print(f"[case] multi-system n={n} S={S} prec={prec}", flush=True)
    H = AmgHierarchy(dev(rp), dev(ci), dev(V), vcycle_prec=prec, max_coarse=32)
    st = H.stats()
    X, info = H.solve(dev(B), 1e-9)
    cols = H.columns(S)
    Xh = host(X)
    for s in range(S):
        O = _oracle(rp, ci, vals[s], max_coarse=32)
        assert O.num_levels == st["num_levels"]
        # hierarchy of system s is bit-exact with the oracle's
        for l in range(O.num_levels):
            o = O.level(l)
            coarsest = l == O.num_levels - 1
            names = ["A_v", "dinv"] + ([] if coarsest else ["P_v", "R_v"])
            for name in names:
                g = host(H.export(l, name)).reshape(-1, S)[:, s]
                assert np.array_equal(g.view(np.int64), o[name].view(np.int64)), (s, l, name)
            for name in ["A_rp", "A_ci"] + ([] if coarsest else ["agg", "P_rp", "P_ci", "R_rp", "R_ci"]):
                assert np.array_equal(host(H.export(l, name)), o[name]), (s, l, name)
        b = B[:, s].copy()
        rr = oracle.rel_residual(rp, ci, vals[s], b, Xh[:, s].copy())
        xo, io = O.pcg(b, tol=1e-9)
        assert cols["status"][s] == 0 and rr <= 1e-9
        if prec == "fp64":
            assert abs(cols["iters"][s] - io["iters"]) <= 1
    if prec == "fp64":
        # iterate parity at a fixed iteration count, every system against the
        # oracle run on that system alone
        kk = 9
        Hk = AmgHierarchy(dev(rp), dev(ci), dev(V), max_coarse=32, maxiter=kk)
        Xk, ik = Hk.solve(dev(B), 0.0)
        Xkh = host(Xk)
        assert ik["iters"] == kk
        for s in range(S):
            O = _oracle(rp, ci, vals[s], max_coarse=32)
            xo, _ = O.pcg(B[:, s].copy(), tol=0.0, maxiter=kk)
            err = np.linalg.norm(Xkh[:, s] - xo) / np.linalg.norm(xo)
            print(f"[iterate parity] system {s} k={kk} err={err:.2e}", flush=True)
            assert err <= 1e-9, (s, err)


def test_batched_pattern_grads():
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    rp, ci, v = M.poisson(12, 3)
    n = len(rp) - 1
    rng = np.random.default_rng(3)
    lam, x = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    H = AmgHierarchy(dev(rp), dev(ci), dev(v), max_coarse=32)
    g = host(H.pattern_grad(dev(lam), dev(x)))
    ref = np.zeros(len(ci))
    for c in range(3):        # same summation order: columns ascending
        ref = ref + oracle.pattern_grad(rp, ci, lam[:, c].copy(), x[:, c].copy())
    assert np.array_equal(g, ref)
    V = np.ascontiguousarray(np.stack([v, 2.0 * v], axis=1))
    H2 = AmgHierarchy(dev(rp), dev(ci), dev(V), max_coarse=32)
    g2 = host(H2.pattern_grad(dev(lam[:, :2].copy()), dev(x[:, :2].copy())))
    for s in range(2):
        assert np.array_equal(g2[:, s], oracle.pattern_grad(rp, ci, lam[:, s].copy(), x[:, s].copy()))


def test_multi_system_refresh_and_adjoint():
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    N, S = 12, 3
    vals = [M.diffusion(np.exp(M.grf(N, 3, seed=50 + s)))[2] for s in range(S)]
    rp, ci, _ = M.poisson(N, 3)
    V = np.ascontiguousarray(np.stack(vals, axis=1))
    H = AmgHierarchy(dev(rp), dev(ci), dev(V), max_coarse=16)
    V2 = np.ascontiguousarray(V[:, ::-1])
    H.update_values(dev(V2))
    n = len(rp) - 1
    G = np.ascontiguousarray(np.stack([M.rhs_normal(n, 60 + s) for s in range(S)], axis=1))
    L, _ = H.solve_adjoint(dev(G), 1e-10)
    Lh = host(L)
    for s in range(S):
        O = _oracle(rp, ci, V2[:, s].copy(), max_coarse=16)
        lo, _ = O.solve_adjoint(G[:, s].copy(), tol=1e-10)
        assert np.linalg.norm(Lh[:, s] - lo) <= 1e-7 * np.linalg.norm(lo)
        o = O.level(0)
        assert np.array_equal(host(H.export(0, "P_v")).reshape(-1, S)[:, s], o["P_v"])


@pytest.mark.parametrize("k,prec", [(6, "fp64"), (12, "fp32"), (3, "fp32")])
def test_multi_rhs_widths_with_idle_lanes(k, prec):
    """Widths whose lane groups hold idle lanes (6 FP64 columns: three lanes of
    two columns in a group of four; 12 FP32: three of four columns each; 3:
    one column per lane): each column against the oracle."""
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    rp, ci, v = M.diffusion(np.exp(M.grf(14, 3, seed=21)))
    n = len(rp) - 1
    B = M.rhs_normal(n, 31, nrhs=k)
    print(f"[case] multi-rhs widths n={n} k={k} prec={prec}", flush=True)
    O = _oracle(rp, ci, v, max_coarse=32)
    if prec == "fp64":
        kk = 6
        H = AmgHierarchy(dev(rp), dev(ci), dev(v), max_coarse=32, maxiter=kk)
        X, info = H.solve(dev(B), 0.0)
        Xh = host(X)
        assert info["iters"] == kk
        for c in range(k):
            xo, _ = O.pcg(B[:, c].copy(), tol=0.0, maxiter=kk)
            assert np.linalg.norm(Xh[:, c] - xo) <= 1e-9 * np.linalg.norm(xo), c
    else:
        H = AmgHierarchy(dev(rp), dev(ci), dev(v), max_coarse=32, vcycle_prec=prec)
        X, info = H.solve(dev(B), 1e-9)
        Xh = host(X)
        cols = H.columns(k)
        for c in range(k):
            rr = oracle.rel_residual(rp, ci, v, B[:, c].copy(), Xh[:, c].copy())
            assert cols["status"][c] == 0 and rr <= 1e-9, (c, rr)


def test_multi_rhs_unaligned_caller_buffers():
    """b and x 8 bytes off a 16-byte boundary (views into larger buffers): the
    sweeps that read the caller's arrays take one column per lane; the
    solution equals the aligned solve's."""
    from paper_2606_09001_amd.solver import AmgHierarchy
    rp, ci, v = M.poisson(20, 3)
    n, k = len(rp) - 1, 8
    B = M.rhs_normal(n, 41, nrhs=k)
    H = AmgHierarchy(dev(rp), dev(ci), dev(v))
    X0, i0 = H.solve(dev(B), 1e-10)
    bbuf = torch.zeros(n * k + 1, dtype=torch.float64, device="cuda")
    xbuf = torch.zeros(n * k + 1, dtype=torch.float64, device="cuda")
    bmis = bbuf[1:].view(n, k)
    xmis = xbuf[1:].view(n, k)
    bmis.copy_(dev(B))
    assert bmis.data_ptr() % 16 == 8 and xmis.data_ptr() % 16 == 8
    X1, i1 = H.solve(bmis, 1e-10, out=xmis)
    assert X1.data_ptr() == xmis.data_ptr()
    assert i1["iters"] == i0["iters"] and i1["status"] == 0
    assert np.allclose(host(X1), host(X0), rtol=0, atol=1e-12 * np.abs(host(X0)).max())
    assert xbuf[0].item() == 0.0          # nothing written before the view
    with pytest.raises(ValueError):
        H.solve(dev(B), 1e-10, out=torch.empty((n, k + 1), dtype=torch.float64, device="cuda")[:, :k])
