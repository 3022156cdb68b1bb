"""Pins of the oracle's matrix-free assembly (graph-colored probing, CPU).

Coloring: a structurally orthogonal column partition (no two columns of a
color share a row), checked by brute force on grids, random symmetric and
nonsymmetric patterns; at least as many colors as the longest row; the greedy
(Grundy) property for the decreasing-key order (every column of color c has,
for each smaller color, a conflicting column of that color earlier in the
order), which also bounds the count by the largest conflict degree plus one.
Assembly: the values gathered from SciPy's products Y = A V equal A's values
bit for bit; the scatter is the assembly's adjoint (dot-product test).
Section 3.3's matrix-free inverse problem gives the explicit problem's
trajectory.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2606_09001_amd import matrices as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_pattern(n, density, seed, symmetric):
    rng = np.random.default_rng(seed)
    S = sp.random(n, n, density=density, random_state=rng, format="csr")
    S.data[:] = rng.standard_normal(S.nnz)
    if symmetric:
        S = S + S.T
    S = S + sp.eye(n) * 10.0
    S = S.tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)


def _conflicts(rp, ci):
    """Boolean conflict matrix: columns j, j' share a row (brute force, dense)."""
    n = len(rp) - 1
    P = np.zeros((n, n), dtype=bool)
    for i in range(n):
        P[i, ci[rp[i]:rp[i + 1]]] = True
    C = (P.T.astype(np.int64) @ P.astype(np.int64)) > 0
    np.fill_diagonal(C, False)
    return C


PATTERNS = {
    "tridiag_40": lambda: M.tridiagonal(40, 3.0),
    "poisson2d_12": lambda: M.poisson(12, 2),
    "poisson3d_7": lambda: M.poisson(7, 3),
    "random_sym_80": lambda: _random_pattern(80, 0.04, 1, True),
    "random_nonsym_90": lambda: _random_pattern(90, 0.03, 2, False),
    "dropped_cd_10": lambda: M.drop_entries(*M.convection_diffusion(10, 2, (20.0, 5.0)), frac=0.3, seed=3),
}


@pytest.mark.parametrize("name", list(PATTERNS))
def test_coloring_is_structurally_orthogonal_and_greedy(oracle_mod, name):
    rp, ci, _ = PATTERNS[name]()
    n = len(rp) - 1
    color, nc = oracle_mod.color_columns(rp, ci)
    assert color.min() == 0 and color.max() == nc - 1
    # no row holds two columns of one color
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        assert len(set(color[cols].tolist())) == len(cols), i
    # lower bound: the longest row; upper bound: largest conflict degree + 1
    C = _conflicts(rp, ci)
    assert nc >= np.diff(rp).max()
    assert nc <= C.sum(axis=1).max() + 1
    # Grundy property in decreasing key order
    keys = [oracle_mod.node_key(j) for j in range(n)]
    order = sorted(range(n), key=lambda j: -keys[j])
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    for j in range(n):
        earlier = np.nonzero(C[j] & (rank < rank[j]))[0]
        have = set(color[earlier].tolist())
        assert all(c in have for c in range(color[j])), j
        assert not np.any(C[j] & (color == color[j]))


def test_coloring_special_cases(oracle_mod):
    # diagonal matrix: one color; one dense row: n colors
    n = 9
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    c, nc = oracle_mod.color_columns(rp, ci)
    assert nc == 1 and not c.any()
    rp = np.concatenate([[0, n], n + np.arange(1, n, dtype=np.int32)]).astype(np.int32)
    ci = np.concatenate([np.arange(n), np.arange(1, n)]).astype(np.int32)
    c, nc = oracle_mod.color_columns(rp, ci)
    assert nc == n and sorted(c.tolist()) == list(range(n))


@pytest.mark.parametrize("name", list(PATTERNS))
def test_assembly_from_probes_is_exact(oracle_mod, name):
    rp, ci, v = PATTERNS[name]()
    n = len(rp) - 1
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    color, nc = oracle_mod.color_columns(rp, ci)
    V = oracle_mod.probe_vectors(color, nc)
    assert V.shape == (nc, n) and np.array_equal(V.sum(axis=0), np.ones(n))
    Y = (A @ V.T).T                       # one operator application per color
    val = oracle_mod.probe_assemble(rp, ci, color, Y)
    assert np.array_equal(val.view(np.int64), v.view(np.int64))
    # the scatter is the assembly's adjoint: <S(dval), Y> = <dval, G(Y)>
    rng = np.random.default_rng(4)
    dval = rng.standard_normal(len(ci))
    Yr = rng.standard_normal((nc, n))
    dY = oracle_mod.probe_scatter(rp, ci, color, nc, dval)
    lhs = np.sum(dY * Yr)
    rhs = np.dot(dval, oracle_mod.probe_assemble(rp, ci, color, Yr))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def _tridiag_operator(d):
    """tridiag(-1, d, -1) with Dirichlet ends as a callable (the operator of
    Section 3.3): y_i = d x_i - x_{i-1} - x_{i+1}, with x_{-1} = x_n = 0."""
    def matvec(x):
        xp = np.concatenate(([0.0], x, [0.0]))
        return d * x - xp[:-2] - xp[2:]
    return matvec


def test_section_3_3_matrix_free_inverse_problem(oracle_mod):
    """Section 3.3: the inverse problem of Section 3.2 with the operator given
    as a callable; the pattern and coloring are computed once, the values are
    assembled from probes at every step.  The trajectory equals the explicit
    matrix's (identical values, so identical solves)."""
    with open(os.path.join(GOLDEN, "tridiag_inverse_problem.json")) as f:
        gold = json.load(f)
    n, d_true, lr, tol = gold["n"], gold["true_diag"], gold["lr"], gold["grad_tol"]
    b = np.ones(n)
    rp, ci, vt = M.tridiagonal(n, d_true)
    color, nc = oracle_mod.color_columns(rp, ci)
    V = oracle_mod.probe_vectors(color, nc)
    x_target, _ = oracle_mod.OracleHierarchy(rp, ci, vt).pcg(b, tol=1e-14)
    diag_mask = np.repeat(np.arange(n), np.diff(rp)) == ci

    def step_values(d, matrix_free):
        if matrix_free:
            op = _tridiag_operator(d)
            Y = np.stack([op(V[c]) for c in range(nc)])
            v = oracle_mod.probe_assemble(rp, ci, color, Y)
        else:
            v = M.tridiagonal(n, d)[2]
        H = oracle_mod.OracleHierarchy(rp, ci, v)
        x, _ = H.pcg(b, tol=1e-14)
        lam, _ = H.solve_adjoint(2.0 * (x - x_target), tol=1e-14)
        gval = H.pattern_grad(lam, x)
        return v, np.sum(gval[diag_mask])

    traj = {}
    for mf in (False, True):
        d = gold["init_diag"]
        ds = []
        for step in range(gold["max_iters"]):
            v, g = step_values(d, mf)
            d -= lr * g
            ds.append(d)
            if abs(g) < tol:
                break
        traj[mf] = ds
    assert traj[True] == traj[False]
    assert abs(traj[True][-1] - d_true) < 1e-3 and len(traj[True]) < gold["max_iters"]
