"""The V-cycle exported as an operator (make_preconditioner) driving a
Krylov loop written in plain torch on the caller's side: the loop converges
like the library's own PCG (iteration counts within one, true residual from
the oracle's SpMV)."""
import numpy as np
import pytest
import torch

from paper_2606_09001_amd import matrices as M
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def test_make_preconditioner_in_a_torch_pcg_loop():
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy, make_preconditioner
    rp, ci, v = M.diffusion(np.exp(M.grf(64, 2, seed=5)))
    n = len(rp) - 1
    b = dev(M.rhs_normal(n, 11))
    A = torch.sparse_csr_tensor(dev(rp.astype(np.int64)), dev(ci.astype(np.int64)), dev(v), (n, n))
    Minv = make_preconditioner(dev(rp), dev(ci), dev(v))
    tol = 1e-10
    x = torch.zeros_like(b)
    r = b.clone()
    z = Minv(r)
    p = z.clone()
    rz = torch.dot(r, z)
    bn = torch.linalg.norm(b)
    iters = 0
    while iters < 500:
        q = A @ p
        alpha = rz / torch.dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        iters += 1
        if torch.linalg.norm(r) <= tol * bn:
            break
        z = Minv(r)
        rzn = torch.dot(r, z)
        p = z + (rzn / rz) * p
        rz = rzn
    _, info = AmgHierarchy(dev(rp), dev(ci), dev(v)).solve(b, tol)
    assert abs(iters - info["iters"]) <= 1, (iters, info["iters"])
    assert oracle.rel_residual(rp, ci, v, host(b), host(x)) <= 2 * tol
