"""Matrix-free assembly on the GPU (graph-colored probing), against the oracle.

Bars: colors bit-exact (the Jones-Plassmann rounds reproduce the oracle's
greedy coloring), probe vectors, assembled values and scatter bit-exact;
an operator given as a torch stencil callable assembles to the explicit
matrix's values bit for bit, so its solves equal the explicit solves; the
Section 3.3 matrix-free inverse problem follows the explicit one.
"""
import ctypes as C
import json
import os

import numpy as np
import pytest
import torch

from paper_2606_09001_amd import matrices as M
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_nonsym(n, density, seed):
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    S = sp.random(n, n, density=density, random_state=rng, format="csr")
    S.data[:] = rng.standard_normal(S.nnz)
    S = (S + sp.eye(n) * 10.0).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)


PATTERNS = {
    "tridiag_1000": lambda: M.tridiagonal(1000, 2.5),
    "poisson3d_24": lambda: M.poisson(24, 3),
    "cd2d_64_dropped": lambda: M.drop_entries(*M.convection_diffusion(64, 2, (30.0, -10.0)), frac=0.2, seed=4),
    "random_nonsym_3000": lambda: _random_nonsym(3000, 0.002, 5),
    "diffusion2d_75": lambda: M.diffusion(np.exp(M.grf(75, 2, seed=3))),
}


def _stencil_operator(rp, ci, v):
    """The matrix as a torch callable built from its per-offset coefficient
    vectors (y_i = sum_off c_off[i] x[i + off]); what a user's stencil code
    computes, without the CSR arrays."""
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    offs = ci.astype(np.int64) - rows
    coef = {}
    for off in np.unique(offs):
        c = np.zeros(n)
        sel = offs == off
        c[rows[sel]] = v[sel]
        coef[int(off)] = (dev(c), dev(np.clip(np.arange(n) + off, 0, n - 1)))

    def matvec(x):
        y = torch.zeros_like(x)
        for off in sorted(coef):
            c, idx = coef[off]
            y = y + c * x[idx]
        return y
    return matvec


@pytest.mark.parametrize("name", list(PATTERNS))
def test_coloring_and_assembly_match_oracle(name):
    import oracle
    from paper_2606_09001_amd.solver import MatrixFreeOperator
    rp, ci, v = PATTERNS[name]()
    n = len(rp) - 1
    print(f"[case] {name} n={n} nnz={len(ci)}", flush=True)
    op = MatrixFreeOperator(dev(rp), dev(ci), _stencil_operator(rp, ci, v))
    co, nco = oracle.color_columns(rp, ci)
    assert op.ncolors == nco
    assert np.array_equal(host(op.color), co)
    assert np.array_equal(host(op.probes), oracle.probe_vectors(co, nco))
    val = op.assemble()
    assert np.array_equal(host(val).view(np.int64), v.view(np.int64))
    # scatter (the assembly's adjoint) against the oracle's
    dval = M.rhs_normal(len(ci), 7)
    Y = torch.zeros(op.ncolors, n, dtype=torch.float64, device="cuda", requires_grad=True)
    from paper_2606_09001_amd.solver import _ProbeAssemble
    _ProbeAssemble.apply(Y, op).backward(dev(dval))
    assert np.array_equal(host(Y.grad), oracle.probe_scatter(rp, ci, co, nco, dval))


def test_matrix_free_solve_equals_explicit():
    from paper_2606_09001_amd.solver import AmgHierarchy, MatrixFreeOperator
    rp, ci, v = M.convection_diffusion(32, 3, M.recirculating_wind(32, 3, 200.0))
    n = len(rp) - 1
    b = dev(M.rhs_normal(n, 8))
    op = MatrixFreeOperator(dev(rp), dev(ci), _stencil_operator(rp, ci, v))
    kw = dict(symmetric=False, solver="bicgstab")
    xe, ie = AmgHierarchy(dev(rp), dev(ci), dev(v), **kw).solve(b, 1e-10)
    xm = op.solve(b, 1e-10, **kw)
    assert ie["status"] == 0 and torch.equal(xe, xm)


def test_probe_entry_points_reject_bad_colors():
    from paper_2606_09001_amd import _lib
    rp, ci, v = M.tridiagonal(50, 3.0)
    color = dev(np.full(50, 7, np.int32))        # outside [0, 3)
    Y = torch.zeros(3 * 50, dtype=torch.float64, device="cuda")
    val = torch.zeros(len(ci), dtype=torch.float64, device="cuda")
    L = _lib.load()
    s = torch.cuda.current_stream().cuda_stream
    st = L.amg_probe_assemble(50, len(ci), dev(rp).data_ptr(), dev(ci).data_ptr(), color.data_ptr(), 3,
                              Y.data_ptr(), val.data_ptr(), s)
    assert st == _lib.AMG_ERR_INVALID_ARG and not val.any()
    st = L.amg_probe_vectors(50, color.data_ptr(), 3, Y.data_ptr(), s)
    assert st == _lib.AMG_ERR_INVALID_ARG
    nc = C.c_int32(0)
    bad_ci = dev(np.where(ci == 0, 60, ci).astype(np.int32))   # column out of range
    st = L.amg_color_columns(50, len(ci), dev(rp).data_ptr(), bad_ci.data_ptr(), color.data_ptr(), C.byref(nc), s)
    assert st == _lib.AMG_ERR_INVALID_ARG


def _tridiag_operator(d):
    """tridiag(-1, d, -1) with Dirichlet ends as a callable (the operator of
    Section 3.3; d a torch scalar): y_i = d x_i - x_{i-1} - x_{i+1}, with
    x_{-1} = x_n = 0."""
    def matvec(x):
        xp = torch.nn.functional.pad(x, (1, 1))
        return d * x - xp[:-2] - xp[2:]
    return matvec


def test_section_3_3_matrix_free_inverse_problem_gpu():
    """Section 3.3: d = 10 -> 4 with the operator as a callable, gradients
    through the solve, the assembly's adjoint and the operator; the explicit
    Section 3.2 formulation on the GPU takes the same steps."""
    from paper_2606_09001_amd.solver import MatrixFreeOperator, amg_solve
    with open(os.path.join(GOLDEN, "tridiag_inverse_problem.json")) as f:
        gold = json.load(f)
    n, d_true, lr, tol = gold["n"], gold["true_diag"], gold["lr"], gold["grad_tol"]
    rp, ci, vt = M.tridiagonal(n, d_true)
    d_rp, d_ci = dev(rp), dev(ci)
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x_target = amg_solve(d_rp, d_ci, dev(vt), b, 1e-14).detach()
    diag = dev(np.repeat(np.arange(n), np.diff(rp)) == ci)
    base = MatrixFreeOperator(d_rp, d_ci)
    assert base.ncolors <= 4
    traj = {}
    for mf in (False, True):
        d = torch.tensor(gold["init_diag"], dtype=torch.float64, device="cuda")
        ds = []
        for step in range(gold["max_iters"]):
            dd = d.clone().requires_grad_(True)
            if mf:
                val = base.with_operator(_tridiag_operator(dd)).assemble()
            else:
                val = torch.where(diag, dd, torch.tensor(-1.0, dtype=torch.float64, device="cuda"))
            x = amg_solve(d_rp, d_ci, val, b, 1e-14)
            loss = torch.sum((x - x_target) ** 2)
            loss.backward()
            g = dd.grad.item()
            d = d - lr * g
            ds.append(d.item())
            if abs(g) < tol:
                break
        traj[mf] = ds
    assert len(traj[True]) == len(traj[False]) < gold["max_iters"]
    assert np.max(np.abs(np.array(traj[True]) - np.array(traj[False]))) <= 1e-10
    assert abs(traj[True][-1] - d_true) < 1e-3
