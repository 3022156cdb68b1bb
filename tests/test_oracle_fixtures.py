"""Pins of the input generators against closed forms (CPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2606_09001_amd import matrices as M


def _A(rp, ci, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


@pytest.mark.parametrize("N,d", [(1, 2), (2, 2), (7, 2), (32, 2), (1, 3), (3, 3), (6, 3)])
def test_nnz_formula(N, d):
    rp, ci, v = M.poisson(N, d)
    assert len(ci) == M.expected_nnz(N, d) == rp[-1]


@pytest.mark.parametrize("N,d", [(8, 2), (12, 2), (5, 3), (7, 3)])
def test_poisson_spectrum_closed_form(N, d):
    # eig(A) = sum over axes of 4 sin^2(j_a pi h / 2), j_a = 1..N (Dirichlet Laplacian).
    rp, ci, v = M.poisson(N, d)
    A = _A(rp, ci, v).toarray()
    h = 1.0 / (N + 1)
    lam1 = 4.0 * np.sin(np.arange(1, N + 1) * np.pi * h / 2) ** 2
    grids = np.meshgrid(*([lam1] * d), indexing="ij")
    expected = np.sort(sum(grids).ravel())
    got = np.linalg.eigvalsh(A)
    assert np.max(np.abs(got - expected)) < 1e-12


@pytest.mark.parametrize("N,d", [(8, 2), (5, 3)])
def test_columns_sorted_symmetric(N, d):
    rp, ci, v = M.poisson(N, d)
    for i in range(len(rp) - 1):
        seg = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0)
    A = _A(rp, ci, v)
    assert (A - A.T).nnz == 0


@pytest.mark.parametrize("d", [2, 3])
def test_diffusion_unit_k_is_poisson_bitexact(d):
    N = 6
    k = np.ones((N,) * d)
    a = M.diffusion(k)
    b = M.poisson(N, d)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("d", [2, 3])
def test_diffusion_symmetric_exactly_and_dominant(d):
    N = 7
    k = np.exp(M.grf(N, d, seed=3))
    rp, ci, v = M.diffusion(k)
    A = _A(rp, ci, v)
    assert abs(A - A.T).max() == 0.0
    # row sums: zero for interior rows, positive with a boundary face
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.all(rs > -1e-12)


def test_diffusion_manual_entry():
    # 2x2 grid, k = [[1,2],[3,4]] ([j, i]): node 0 (i=0,j=0) couples to node 1 (x) and node 2 (y).
    k = np.array([[1.0, 2.0], [3.0, 4.0]])
    rp, ci, v = M.diffusion(k)
    A = _A(rp, ci, v).toarray()
    kf01 = 2 * 1 * 2 / 3
    kf02 = 2 * 1 * 3 / 4
    assert A[0, 1] == pytest.approx(-kf01, rel=1e-15)
    assert A[0, 2] == pytest.approx(-kf02, rel=1e-15)
    # two boundary faces of node 0 contribute k_0 = 1 each
    assert A[0, 0] == pytest.approx(kf01 + kf02 + 2.0, rel=1e-15)


def test_diffusion_torch_matches_numpy():
    import torch
    k = np.exp(M.grf(9, 2, seed=5))
    rp, ci, v = M.diffusion(k)
    vt = M.diffusion_values_torch(torch.from_numpy(k)).numpy()
    assert np.array_equal(vt, v)


def test_tridiagonal():
    rp, ci, v = M.tridiagonal(5, 4.0)
    A = _A(rp, ci, v).toarray()
    ref = 4.0 * np.eye(5) - np.eye(5, k=1) - np.eye(5, k=-1)
    assert np.array_equal(A, ref)


def test_manufactured_sin_is_exact_eigenvector_2d():
    # u_ij = sin(pi x_i) sin(pi y_j) satisfies A u = 8 sin^2(pi h / 2) u exactly (up to rounding).
    N = 32
    rp, ci, v = M.poisson(N, 2)
    x, y = M.grid_coords(N, 2)
    u = np.sin(np.pi * x) * np.sin(np.pi * y)
    h = 1.0 / (N + 1)
    lam = 8.0 * np.sin(np.pi * h / 2) ** 2
    Au = _A(rp, ci, v) @ u
    assert np.max(np.abs(Au - lam * u)) < 1e-14


def test_grf_statistics():
    # Circulant embedding with numpy FFT normalisation: Var u ~ sigma^2 = 1,
    # correlation at lag ell = 0.1 ~ exp(-1/2).  Loose statistical pins.
    N = 96
    vals, corr = [], []
    h = 1.0 / (N + 1)
    lag = int(round(0.1 / h))
    for seed in range(6):
        u = M.grf(N, 2, seed=seed)
        vals.append(u.var())
        corr.append(np.mean(u[:, :-lag] * u[:, lag:]))
    assert abs(np.mean(vals) - 1.0) < 0.25
    expected = np.exp(-((lag * h) ** 2) / (2 * 0.1 ** 2))
    assert abs(np.mean(corr) - expected) < 0.2
