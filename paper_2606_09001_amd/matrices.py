"""Seeded synthetic PDE systems in CSR form (the library's test-problem module).

This module builds the inputs the solver is exercised on; it contains none of
the solver's arithmetic (no aggregation, smoothing, Krylov or adjoint step), so
both the HIP path and the CPU oracle can take their inputs from here.

Conventions (shared by every generator):
  * Unknowns are the interior nodes of the unit square / cube, h = 1/(N+1),
    numbered lexicographically with x fastest: idx = i + N*j (+ N*N*k).
    Fields are numpy arrays indexed [k, j, i] (3D) or [j, i] (2D) in C order,
    so ``field.ravel()`` is in unknown order.
  * Dirichlet boundary nodes are eliminated with zero boundary data.
  * The Poisson stencil is unscaled (diagonal 2d, neighbours -1); a
    right-hand side absorbs h^2.  Relative tolerances are scale-free.
  * CSR: int32 row_ptr[n+1], int32 col[nnz] ascending within each row,
    float64 val[nnz].

The paper's example module offers Poisson and tridiagonal test matrices and a
ones right-hand side (Section 3.1, 3.2); diffusion with harmonic-mean face
coefficients on a log-normal field is the variable-coefficient workload.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "stencil_offsets", "poisson", "diffusion", "diffusion_face_coeffs",
    "diffusion_values_torch", "tridiagonal", "grf", "rhs_normal", "rhs_ones",
    "expected_nnz", "grid_coords", "csr_to_dense", "convection_diffusion", "recirculating_wind",
    "drop_entries",
]


def expected_nnz(N: int, d: int) -> int:
    """nnz of the (2d+1)-point stencil on an N^d interior grid."""
    return (2 * d + 1) * N ** d - 2 * d * N ** (d - 1)


def stencil_offsets(N: int, d: int):
    """Column offsets of the stencil in ascending order, with their axis/sign.

    Returns a list of (offset, axis, sign); axis 0 is x (fastest).
    The diagonal appears as (0, -1, 0).
    """
    offs = []
    for a in reversed(range(d)):          # -N^2, -N, -1
        offs.append((-(N ** a), a, -1))
    offs.append((0, -1, 0))
    for a in range(d):                     # +1, +N, +N^2
        offs.append((N ** a, a, +1))
    return offs


def _grid_index_arrays(N: int, d: int):
    """Per-unknown grid coordinate along each axis (axis 0 = x fastest)."""
    n = N ** d
    idx = np.arange(n, dtype=np.int64)
    return [(idx // (N ** a)) % N for a in range(d)]


def grid_coords(N: int, d: int):
    """Physical coordinates x_a = (i_a+1) h of every unknown, axis 0 = x."""
    h = 1.0 / (N + 1)
    return [(c + 1) * h for c in _grid_index_arrays(N, d)]


def _pack_stencil(N: int, d: int, vals_by_offset):
    """Pack per-offset value arrays (n,) into CSR, dropping missing neighbours."""
    n = N ** d
    coords = _grid_index_arrays(N, d)
    offs = stencil_offsets(N, d)
    S = len(offs)
    present = np.ones((n, S), dtype=bool)
    for s, (off, a, sgn) in enumerate(offs):
        if sgn < 0:
            present[:, s] = coords[a] > 0
        elif sgn > 0:
            present[:, s] = coords[a] < N - 1
    cols = np.arange(n, dtype=np.int64)[:, None] + np.array([o for o, _, _ in offs], dtype=np.int64)[None, :]
    vals = np.stack(vals_by_offset, axis=1)
    counts = present.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[present].astype(np.int32)
    val = np.ascontiguousarray(vals[present], dtype=np.float64)
    return row_ptr.astype(np.int32), col, val


def poisson(N: int, d: int):
    """(2d+1)-point Laplacian, Dirichlet, unscaled: diag 2d, off-diagonals -1."""
    n = N ** d
    vals = []
    for off, a, sgn in stencil_offsets(N, d):
        vals.append(np.full(n, float(2 * d) if sgn == 0 else -1.0))
    return _pack_stencil(N, d, vals)


def convection_diffusion(N: int, d: int, wind):
    """-Laplace(u) + w . grad(u) with first-order upwind differences, scaled
    like ``poisson`` (by h^2): a nonsymmetric M-matrix with a symmetric
    pattern.  Row i, axis a, w = w_a(x_i):
        diagonal          2d + h sum_a |w_a|
        neighbour -e_a    -1 - h max(w_a, 0)
        neighbour +e_a    -1 - h max(-w_a, 0)
    ``wind`` holds d entries (axis 0 = x), each a constant or an array of
    the n unknowns' values; the cell Peclet number is h |w_a| / 2.
    """
    n = N ** d
    h = 1.0 / (N + 1)
    w = [np.broadcast_to(np.asarray(wa, dtype=np.float64), (n,)) for wa in wind]
    assert len(w) == d
    vals = []
    for off, a, sgn in stencil_offsets(N, d):
        if sgn == 0:
            dg = np.full(n, float(2 * d))
            for wa in w:
                dg = dg + h * np.abs(wa)
            vals.append(dg)
        elif sgn < 0:
            vals.append(-1.0 - h * np.maximum(w[a], 0.0))
        else:
            vals.append(-1.0 - h * np.maximum(-w[a], 0.0))
    return _pack_stencil(N, d, vals)


def recirculating_wind(N: int, d: int, speed: float):
    """Rotating flow w = speed (sin(pi x) cos(pi y), -cos(pi x) sin(pi y), 0)."""
    c = grid_coords(N, d)
    x, y = c[0], c[1]
    w = [speed * np.sin(np.pi * x) * np.cos(np.pi * y), -speed * np.cos(np.pi * x) * np.sin(np.pi * y)]
    w += [np.zeros_like(x)] * (d - 2)
    return w


def drop_entries(row_ptr, col, val, frac: float, seed: int):
    """Structurally nonsymmetric variant: removes a seeded random fraction of
    the strictly upper off-diagonal entries (numpy default_rng(seed)); the
    diagonal and the lower part are kept, so diagonal dominance is kept."""
    row_ptr = np.asarray(row_ptr)
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    rng = np.random.default_rng(seed)
    drop = (np.asarray(col) > rows) & (rng.random(len(col)) < frac)
    keep = ~drop
    counts = np.bincount(rows[keep], minlength=n)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return rp.astype(np.int32), np.asarray(col)[keep].astype(np.int32), np.ascontiguousarray(np.asarray(val)[keep])


def diffusion_face_coeffs(k: np.ndarray):
    """Face coefficients of -div(k grad u) with harmonic-mean faces.

    Returns, per axis a, (kf_interior[a], kb_lo[a], kb_hi[a]) where
    kf_interior[a] has the field's shape with the last index along axis a
    dropped (face between node and its +e_a neighbour), and the boundary face
    coefficient equals the node's own k.
    Interior face: k_f = ((2*k_p)*k_q)/(k_p+k_q)  (symmetric in p, q exactly).
    """
    d = k.ndim
    out = []
    for a in range(d):
        ax = d - 1 - a                      # numpy axis of grid axis a
        kp = np.take(k, np.arange(k.shape[ax] - 1), axis=ax)
        kq = np.take(k, np.arange(1, k.shape[ax]), axis=ax)
        kf = ((2.0 * kp) * kq) / (kp + kq)
        out.append(kf)
    return out


def diffusion(k: np.ndarray):
    """7/5-point FV/FD diffusion -div(k grad u) = f, Dirichlet, harmonic faces.

    A_pq = -k_f for interior faces, A_pp = sum of the node's face coefficients,
    where a boundary face contributes k_f = k_p.  With k == 1 this is exactly
    ``poisson``.
    """
    k = np.asarray(k, dtype=np.float64)
    d = k.ndim
    N = k.shape[0]
    assert all(s == N for s in k.shape), "cubic grids only"
    n = N ** d
    kfs = diffusion_face_coeffs(k)
    kflat = k.ravel()
    # coefficient of the face on the - and + side of every node, per axis
    lo = []
    hi = []
    for a in range(d):
        ax = d - 1 - a
        kf = kfs[a]
        pad_lo = np.concatenate([np.take(k, [0], axis=ax), kf], axis=ax)          # boundary face = k_p
        pad_hi = np.concatenate([kf, np.take(k, [k.shape[ax] - 1], axis=ax)], axis=ax)
        lo.append(pad_lo.ravel())
        hi.append(pad_hi.ravel())
    diag = np.zeros(n)
    for a in range(d):                     # fixed summation order: axis x lo, hi, y lo, hi, ...
        diag = diag + lo[a]
        diag = diag + hi[a]
    vals = []
    for off, a, sgn in stencil_offsets(N, d):
        if sgn == 0:
            vals.append(diag)
        elif sgn < 0:
            vals.append(-lo[a])
        else:
            vals.append(-hi[a])
    del kflat
    return _pack_stencil(N, d, vals)


def diffusion_values_torch(k):
    """Differentiable (torch) assembly of ``diffusion(k)`` values.

    Same pattern, same arithmetic as ``diffusion``; ``k`` is a torch tensor of
    shape (N,)*d on any device.  Used to chain pattern gradients dL/dA_ij to a
    coefficient field through autograd.
    """
    import torch
    d = k.dim()
    N = k.shape[0]
    lo, hi = [], []
    for a in range(d):
        ax = d - 1 - a
        kp = k.narrow(ax, 0, N - 1)
        kq = k.narrow(ax, 1, N - 1)
        kf = ((2.0 * kp) * kq) / (kp + kq)
        lo.append(torch.cat([k.narrow(ax, 0, 1), kf], dim=ax).reshape(-1))
        hi.append(torch.cat([kf, k.narrow(ax, N - 1, 1)], dim=ax).reshape(-1))
    diag = torch.zeros(N ** d, dtype=k.dtype, device=k.device)
    for a in range(d):
        diag = diag + lo[a]
        diag = diag + hi[a]
    cols = []
    for off, a, sgn in stencil_offsets(N, d):
        if sgn == 0:
            cols.append(diag)
        elif sgn < 0:
            cols.append(-lo[a])
        else:
            cols.append(-hi[a])
    vals = torch.stack(cols, dim=1)
    mask = _stencil_mask_torch(N, d, k.device)
    return vals[mask]


_MASK_CACHE = {}


def _stencil_mask_torch(N, d, device):
    import torch
    key = (N, d, str(device))
    if key not in _MASK_CACHE:
        n = N ** d
        coords = _grid_index_arrays(N, d)
        offs = stencil_offsets(N, d)
        present = np.ones((n, len(offs)), dtype=bool)
        for s, (off, a, sgn) in enumerate(offs):
            if sgn < 0:
                present[:, s] = coords[a] > 0
            elif sgn > 0:
                present[:, s] = coords[a] < N - 1
        _MASK_CACHE[key] = torch.from_numpy(present).to(device)
    return _MASK_CACHE[key]


def tridiagonal(n: int, diagonal_value: float, off_value: float = -1.0):
    """Toeplitz tridiag(off, diagonal_value, off) of size n (Section 3.2)."""
    counts = np.full(n, 3, dtype=np.int64)
    counts[0] = counts[-1] = 2
    if n == 1:
        counts[0] = 1
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.empty(row_ptr[-1], dtype=np.int32)
    val = np.empty(row_ptr[-1], dtype=np.float64)
    for i in range(n):
        s = row_ptr[i]
        c = [j for j in (i - 1, i, i + 1) if 0 <= j < n]
        col[s:s + len(c)] = c
        val[s:s + len(c)] = [diagonal_value if j == i else off_value for j in c]
    return row_ptr.astype(np.int32), col, val


def grf(N: int, d: int, seed: int, sigma: float = 1.0, ell: float = 0.1):
    """Stationary Gaussian random field on the N^d interior grid.

    Circulant embedding on a periodic grid of M = 2N points per axis with the
    grid's spacing h = 1/(N+1); squared-exponential covariance
    C(r) = sigma^2 exp(-r^2 / (2 ell^2)) on minimal-image distances; negative
    eigenvalues clipped to 0; white noise from numpy's default_rng(seed).
    With numpy's FFT normalisation the field has variance sigma^2.
    Returns an array of shape (N,)*d indexed [k, j, i].
    """
    import scipy.fft as sfft
    h = 1.0 / (N + 1)
    M = 2 * N
    m = np.arange(M)
    dist1 = h * np.minimum(m, M - m)
    r2 = np.zeros((M,) * d)
    for ax in range(d):
        shp = [1] * d
        shp[ax] = M
        r2 = r2 + (dist1.reshape(shp)) ** 2
    c = sigma ** 2 * np.exp(-r2 / (2.0 * ell ** 2))
    lam = np.real(sfft.fftn(c, workers=-1))
    lam = np.clip(lam, 0.0, None)
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((M,) * d)
    u = np.real(sfft.ifftn(np.sqrt(lam) * sfft.fftn(xi, workers=-1), workers=-1))
    sl = tuple(slice(0, N) for _ in range(d))
    return np.ascontiguousarray(u[sl])


def rhs_normal(n: int, seed: int, nrhs: int | None = None):
    """b ~ N(0,1) from numpy default_rng(seed); shape (n,) or row-major (n, nrhs)."""
    rng = np.random.default_rng(seed)
    if nrhs is None:
        return rng.standard_normal(n)
    return rng.standard_normal((n, nrhs))


def rhs_ones(n: int):
    """All-ones right-hand side (the paper's example RHS, Section 3.1)."""
    return np.ones(n, dtype=np.float64)


def csr_to_dense(row_ptr, col, val, n=None):
    n = len(row_ptr) - 1 if n is None else n
    A = np.zeros((len(row_ptr) - 1, n))
    for i in range(len(row_ptr) - 1):
        A[i, col[row_ptr[i]:row_ptr[i + 1]]] = val[row_ptr[i]:row_ptr[i + 1]]
    return A
