"""Pins of the oracle's nonsymmetric path (CPU).

Coarse LU: same pivots as LAPACK's getrf (partial pivoting, first largest
entry) and the same factors to rounding.  BiCGSTAB: same iterates as SciPy's
BiCGSTAB driven by the same preconditioner (none, or the oracle's V-cycle);
solutions against LAPACK; status paths.  Setup on a nonsymmetric A:
prolongator and Galerkin product against their dense definitions (with A,
not A^T), strength graph = union of the off-diagonal patterns of A and A^T.
Adjoint (Eq. (1)/(2)) of a nonsymmetric A: explicit transpose against SciPy,
lambda against a dense transposed solve, gradient against central finite
differences.
"""
import numpy as np
import pytest
import scipy.linalg as sla_dense
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from paper_2606_09001_amd import matrices as M


def _A(rp, ci, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


def _cd(N, d, wind=None):
    if wind is None:
        wind = (40.0, 20.0, 10.0)[:d]
    return M.convection_diffusion(N, d, wind)


def test_convection_diffusion_generator():
    # upwind M-matrix: nonsymmetric values, symmetric pattern, weak diagonal
    # dominance, and w = 0 reduces to the Poisson stencil
    rp, ci, v = _cd(12, 2)
    A = _A(rp, ci, v).toarray()
    assert np.abs(A - A.T).max() > 0.1
    assert np.array_equal(A != 0, (A != 0).T)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0)
    assert np.all(np.diag(A) + off.sum(axis=1) >= -1e-14)
    rp0, ci0, v0 = M.convection_diffusion(12, 2, (0.0, 0.0))
    rpp, cip, vp = M.poisson(12, 2)
    assert np.array_equal(rp0, rpp) and np.array_equal(ci0, cip) and np.array_equal(v0, vp)
    # first-order upwind: row of an interior node with w = (5, -3), h = 1/13
    h = 1.0 / 13
    rp, ci, v = M.convection_diffusion(12, 2, (5.0, -3.0))
    A = _A(rp, ci, v).toarray()
    i = 5 + 12 * 6
    assert A[i, i] == pytest.approx(4 + h * 8)
    assert A[i, i - 1] == pytest.approx(-1 - 5 * h) and A[i, i + 1] == -1.0
    assert A[i, i + 12] == pytest.approx(-1 - 3 * h) and A[i, i - 12] == -1.0


@pytest.mark.parametrize("N,kw", [(12, dict(max_coarse=500)), (16, dict(max_coarse=40))])
def test_coarse_lu_matches_lapack(oracle_mod, N, kw):
    rp, ci, v = M.convection_diffusion(N, 2, M.recirculating_wind(N, 2, 150.0))
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, **kw)
    lc = H.level(H.num_levels - 1)
    Ac = _A(lc["A_rp"], lc["A_ci"], lc["A_v"]).toarray()
    lu, piv = sla_dense.lu_factor(Ac)
    mine = H.coarse_factor()
    assert np.array_equal(H.coarse_pivots(), piv)
    assert np.max(np.abs(mine - lu)) <= 1e-13 * np.abs(lu).max()
    # the factorization reproduces the coarse matrix
    n = Ac.shape[0]
    Lm = np.tril(mine, -1) + np.eye(n)
    Um = np.triu(mine)
    PA = Ac.copy()
    for k, p in enumerate(H.coarse_pivots()):
        PA[[k, p]] = PA[[p, k]]
    assert np.max(np.abs(Lm @ Um - PA)) <= 1e-13 * np.abs(Ac).max()
    # a symmetric hierarchy reports no pivots
    Hs = oracle_mod.OracleHierarchy(*M.poisson(8, 2))
    assert Hs.coarse_pivots() is None


def test_coarse_lu_pivot_ties_take_the_first_row(oracle_mod):
    # |column 0| ties in every row: LAPACK (and the oracle) keep the first
    Ad = np.array([[1.0, 2.0, 0.0, 0.0], [-1.0, 1.0, 1.0, 0.0], [1.0, 0.0, 3.0, 1.0], [-1.0, 0.0, 1.0, 2.0]])
    S = sp.csr_matrix(Ad)
    S.sort_indices()
    H = oracle_mod.OracleHierarchy(S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data, symmetric=False,
                                   max_coarse=10)
    lu, piv = sla_dense.lu_factor(Ad)
    assert np.array_equal(H.coarse_pivots(), piv) and piv[0] == 0
    assert np.max(np.abs(H.coarse_factor() - lu)) <= 1e-15 * np.abs(lu).max()


def test_single_level_nonsymmetric_is_direct_solve(oracle_mod):
    rp, ci, v = _cd(10, 2)
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, max_coarse=1000)
    assert H.num_levels == 1
    b = M.rhs_normal(100, 4)
    A = _A(rp, ci, v).toarray()
    xr = np.linalg.solve(A, b)
    assert np.max(np.abs(H.vcycle(b) - xr)) <= 1e-13 * np.abs(xr).max()
    x, info = H.bicgstab(b, tol=1e-12)
    assert info["status"] == 0 and info["iters"] == 1
    assert np.max(np.abs(x - xr)) <= 1e-12 * np.abs(xr).max()


def test_setup_on_nonsymmetric_matrix_uses_a_not_its_transpose(oracle_mod):
    # P = (I - omega_P D^-1 A) T and A_c = R A P with R = P^T, dense
    rp, ci, v = M.convection_diffusion(14, 2, M.recirculating_wind(14, 2, 300.0))
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, max_coarse=20)
    assert H.num_levels >= 3
    for l in range(H.num_levels - 1):
        o = H.level(l)
        A = _A(o["A_rp"], o["A_ci"], o["A_v"]).toarray()
        n, nagg = o["n"], o["nagg"]
        T = np.zeros((n, nagg))
        T[np.arange(n), o["agg"]] = 1.0
        P = (np.eye(n) - o["omegaP"] * np.diag(1.0 / np.diag(A)) @ A) @ T
        Pg = sp.csr_matrix((o["P_v"], o["P_ci"], o["P_rp"]), shape=(n, nagg)).toarray()
        assert np.max(np.abs(Pg - P)) <= 1e-14 * np.abs(P).max()
        Rg = sp.csr_matrix((o["R_v"], o["R_ci"], o["R_rp"]), shape=(nagg, n)).toarray()
        assert np.array_equal(Rg, Pg.T)
        nxt = H.level(l + 1)
        Ac = _A(nxt["A_rp"], nxt["A_ci"], nxt["A_v"]).toarray()
        ref = P.T @ A @ P
        assert np.max(np.abs(Ac - ref)) <= 1e-12 * np.abs(ref).max()
        assert np.abs(Ac - Ac.T).max() > 1e-6 * np.abs(Ac).max()  # the nonsymmetry survives


def test_strength_graph_of_structurally_nonsymmetric_matrix(oracle_mod):
    rp, ci, v = M.drop_entries(*_cd(12, 2), frac=0.4, seed=3)
    A = _A(rp, ci, v).toarray()
    assert not np.array_equal(A != 0, (A != 0).T)
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, max_coarse=10)
    o = H.level(0)
    G = sp.csr_matrix((np.ones(len(o["G_ci"])), o["G_ci"], o["G_rp"]), shape=A.shape).toarray() != 0
    S = (A != 0) | (A != 0).T
    np.fill_diagonal(S, False)
    assert np.array_equal(G, S)


def test_transpose_matches_scipy(oracle_mod):
    rp, ci, v = M.drop_entries(*_cd(9, 3), frac=0.3, seed=5)
    rpT, ciT, vT = oracle_mod.transpose(rp, ci, v)
    T = _A(rp, ci, v).T.tocsr()
    T.sort_indices()
    assert np.array_equal(rpT, T.indptr) and np.array_equal(ciT, T.indices) and np.array_equal(vT, T.data)


def _scipy_bicgstab_iterates(A, b, Minv, kmax):
    out = []
    for k in range(1, kmax + 1):
        x, _ = sla.bicgstab(A, b, rtol=0.0, atol=0.0, maxiter=k, M=Minv)
        out.append(x)
    return out


@pytest.mark.parametrize("precondition", [True, False])
def test_bicgstab_iterates_match_scipy(oracle_mod, precondition):
    N = 20
    rp, ci, v = M.convection_diffusion(N, 2, M.recirculating_wind(N, 2, 120.0))
    A = _A(rp, ci, v)
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, max_coarse=16)
    assert H.num_levels >= 2
    b = M.rhs_normal(N * N, 5)
    Minv = sla.LinearOperator(A.shape, matvec=lambda r: H.vcycle(np.asarray(r).ravel())) if precondition else None
    ref = _scipy_bicgstab_iterates(A, b, Minv, 6)
    for k, xr in enumerate(ref, start=1):
        x, info = H.bicgstab(b, tol=0.0, maxiter=k, precondition=precondition)
        assert info["iters"] == k and info["status"] == 1
        assert np.linalg.norm(x - xr) <= 1e-11 * np.linalg.norm(xr), k


def test_unpreconditioned_bicgstab_count_poisson_32_ones(oracle_mod):
    # Section 3.1's example system (32x32 Poisson, b = 1, tol 1e-6), no
    # preconditioner: the iteration count equals SciPy's BiCGSTAB count
    # (same stopping rule on the recursive residual).
    rp, ci, v = M.poisson(32, 2)
    A = _A(rp, ci, v)
    b = M.rhs_ones(1024)
    count = [0]
    sla.bicgstab(A, b, rtol=1e-6, atol=0.0, maxiter=1000, callback=lambda xk: count.__setitem__(0, count[0] + 1))
    H = oracle_mod.OracleHierarchy(rp, ci, v)
    _, info = H.bicgstab(b, tol=1e-6, precondition=False)
    assert info["status"] == 0 and abs(info["iters"] - count[0]) <= 1
    _, info_amg = H.bicgstab(b, tol=1e-6)
    assert info_amg["status"] == 0 and info_amg["iters"] <= count[0] // 3


@pytest.mark.parametrize("N,d,wind", [(32, 2, None), (12, 3, None), (24, 2, "recirc")])
def test_bicgstab_vs_dense_solve(oracle_mod, N, d, wind):
    w = M.recirculating_wind(N, d, 400.0) if wind == "recirc" else None
    rp, ci, v = _cd(N, d, w)
    A = _A(rp, ci, v).toarray()
    b = M.rhs_normal(N ** d, 2)
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, max_coarse=32)
    tol = 1e-10
    x, info = H.bicgstab(b, tol=tol)
    assert info["status"] == 0 and info["rel_resid"] <= tol
    xr = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xr) <= np.linalg.cond(A) * tol * np.linalg.norm(xr)
    _, info0 = H.bicgstab(b, tol=tol, precondition=False)
    assert info["iters"] < info0["iters"]


def test_bicgstab_status_paths(oracle_mod):
    rp, ci, v = _cd(10, 2)
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, max_coarse=16)
    x, info = H.bicgstab(np.zeros(100), tol=1e-8)
    assert info["status"] == 0 and info["iters"] == 0 and not x.any()
    b = M.rhs_normal(100, 1)
    x, info = H.bicgstab(b, tol=1e-14, maxiter=2)
    assert info["status"] == 1 and info["iters"] == 2
    bad = b.copy()
    bad[3] = np.nan
    _, info = H.bicgstab(bad, tol=1e-8)
    assert info["status"] == -4
    # recursive-residual stop followed by the true-residual check
    x, info = H.bicgstab(b, tol=1e-12)
    assert info["status"] == 0 and info["rel_resid"] <= 1e-12


def test_nonsymmetric_setup_rejects_zero_diagonal_and_singular_coarse(oracle_mod):
    # a stored zero diagonal is rejected before any setup
    rp = np.array([0, 2, 5, 7], np.int32)
    ci = np.array([0, 1, 0, 1, 2, 1, 2], np.int32)
    vals = np.array([2.0, -1.0, -2.0, 0.0, -2.0, -1.0, 2.0])
    with pytest.raises(Exception) as e:
        oracle_mod.OracleHierarchy(rp, ci, vals, symmetric=False, max_coarse=10)
    assert getattr(e.value, "status", None) == -2
    # nonzero diagonal, singular matrix [[1, 2], [0.5, 1]]: the LU meets a zero pivot
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    with pytest.raises(Exception) as e:
        oracle_mod.OracleHierarchy(rp, ci, np.array([1.0, 2.0, 0.5, 1.0]), symmetric=False, max_coarse=10)
    assert getattr(e.value, "status", None) == -4


def _loss_and_grad(oracle_mod, rp, ci, v, b, u_obs, tol):
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, max_coarse=16)
    x, _ = H.bicgstab(b, tol=tol)
    gx = x - u_obs
    lam, ainfo = H.solve_adjoint(gx, tol=tol)
    assert ainfo["status"] == 0
    return 0.5 * np.dot(gx, gx), x, lam, H.pattern_grad(lam, x)


def test_nonsymmetric_adjoint_vs_dense_and_fd(oracle_mod):
    N = 8
    rp, ci, v = M.drop_entries(*M.convection_diffusion(N, 2, M.recirculating_wind(N, 2, 100.0)), frac=0.2, seed=9)
    n = N * N
    b = np.ones(n)
    u_obs = M.rhs_normal(n, 3) * 0.01
    L0, x, lam, gval = _loss_and_grad(oracle_mod, rp, ci, v, b, u_obs, 1e-13)
    A = _A(rp, ci, v).toarray()
    xr = np.linalg.solve(A, b)
    lam_r = np.linalg.solve(A.T, xr - u_obs)
    lam_wrong = np.linalg.solve(A, xr - u_obs)  # what a missing transpose would give
    assert np.max(np.abs(lam - lam_r)) <= 1e-10 * np.abs(lam_r).max()
    assert np.max(np.abs(lam_wrong - lam_r)) > 1e-3 * np.abs(lam_r).max()
    for seed in (7, 8):
        dv = np.random.default_rng(seed).standard_normal(len(v))
        eps = 1e-4
        Lp = _loss_and_grad(oracle_mod, rp, ci, v + eps * dv, b, u_obs, 1e-13)[0]
        Lm = _loss_and_grad(oracle_mod, rp, ci, v - eps * dv, b, u_obs, 1e-13)[0]
        fd = (Lp - Lm) / (2 * eps)
        an = np.dot(gval, dv)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12)


def test_transpose_hierarchy_refresh(oracle_mod):
    # value refresh of a nonsymmetric hierarchy also refreshes its transpose's
    rp, ci, v = _cd(12, 2)
    H = oracle_mod.OracleHierarchy(rp, ci, v, symmetric=False, max_coarse=16)
    g = M.rhs_normal(144, 8)
    H.solve_adjoint(g, tol=1e-12)
    v2 = v * (1.0 + 0.1 * np.random.default_rng(2).random(len(v)))
    H.update_values(v2)
    lam, info = H.solve_adjoint(g, tol=1e-12)
    A2 = _A(rp, ci, v2).toarray()
    lam_r = np.linalg.solve(A2.T, g)
    assert info["status"] == 0
    assert np.max(np.abs(lam - lam_r)) <= 1e-9 * np.abs(lam_r).max()
    F = oracle_mod.OracleHierarchy(*oracle_mod.transpose(rp, ci, v2), symmetric=False, max_coarse=16)
    lam_f, _ = F.bicgstab(g, tol=1e-12)
    assert np.array_equal(lam, lam_f)
