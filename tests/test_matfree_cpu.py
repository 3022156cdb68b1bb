"""Matrix-free helpers that run without a GPU: one-hot pattern detection
(the fallback for operators whose pattern is not known) on torch CPU
tensors, against the pattern of the explicit matrix."""
import numpy as np
import torch

from paper_2606_09001_amd import matrices as M


def _operator(rp, ci, v):
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    A = torch.sparse_coo_tensor(np.stack([rows, ci]), v, (n, n)).coalesce()
    return lambda x: torch.sparse.mm(A, x.reshape(-1, 1)).reshape(-1)


def test_detect_pattern_cpu():
    from paper_2606_09001_amd.solver import detect_pattern
    for rp, ci, v in (M.tridiagonal(20, 3.0), M.drop_entries(*M.convection_diffusion(7, 2, (9.0, 2.0)), frac=0.4,
                                                             seed=1)):
        drp, dci = detect_pattern(_operator(rp, ci, v), len(rp) - 1, device="cpu")
        assert np.array_equal(drp.numpy(), rp) and np.array_equal(dci.numpy(), ci)


def test_detect_pattern_adds_missing_diagonal():
    from paper_2606_09001_amd.solver import detect_pattern
    # operator with a zero diagonal entry in row 2: the pattern still stores it
    rp, ci, v = M.tridiagonal(6, 2.0)
    v = v.copy()
    v[np.nonzero((np.repeat(np.arange(6), np.diff(rp)) == ci) & (ci == 2))[0]] = 0.0
    drp, dci = detect_pattern(_operator(rp, ci, v), 6, device="cpu")
    assert np.array_equal(drp.numpy(), rp) and np.array_equal(dci.numpy(), ci)
