"""Torch-facing API over the C ABI: hierarchy handles, solve, and autograd.

Section 2.1 ("Python API" / "JAX integration"): a single solve entry point
returning (x, info), with a reverse-mode rule that solves the adjoint system
A^T lambda = dL/dx (Eq. (1)) on the cached hierarchy and returns
dL/dA = -lambda x^T on the stored pattern and dL/db = lambda (Eq. (2)).
Torch only supplies device memory and the stream; every arithmetic step runs
in libamg355.so.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from . import _lib

__all__ = ["AmgHierarchy", "solve", "amg_solve", "AmgSolve", "make_params", "finalize", "cache_size",
           "set_cache_capacity", "make_preconditioner", "MatrixFreeOperator"]

_PARAM_KEYS = ("vcycle_prec", "transfer_bf16", "theta", "max_coarse", "max_levels", "smoother", "omega", "nu_pre",
               "nu_post", "maxiter", "flexible", "symmetric", "check_every", "use_graphs", "autotune",
               "precondition", "solver", "fused_small")


def make_params(**kw) -> _lib.amg_params:
    """amg_params with the library defaults, overridden by keyword (Section 2.2:
    users set only the parameters they change).  Accepts 'pcg'/'bicgstab' for
    solver, 'fp64'/'fp32' for vcycle_prec and 'jacobi'/'l1' for smoother."""
    L = _lib.load()
    p = _lib.amg_params()
    L.amg_params_default(C.byref(p))
    for k, v in kw.items():
        if k not in _PARAM_KEYS:
            raise TypeError(f"unknown AMG parameter {k!r}")
        if k == "vcycle_prec" and isinstance(v, str):
            v = {"fp64": _lib.AMG_PREC_FP64, "fp32": _lib.AMG_PREC_FP32, "mixed": _lib.AMG_PREC_FP32}[v]
        if k == "smoother" and isinstance(v, str):
            v = {"jacobi": _lib.AMG_SMOOTHER_JACOBI, "l1": _lib.AMG_SMOOTHER_L1}[v]
        if k == "solver" and isinstance(v, str):
            v = {"pcg": _lib.AMG_SOLVER_PCG, "cg": _lib.AMG_SOLVER_PCG,
                 "bicgstab": _lib.AMG_SOLVER_BICGSTAB, "pbicgstab": _lib.AMG_SOLVER_BICGSTAB}[v.lower()]
        if k == "symmetric":
            v = int(bool(v))
        setattr(p, k, v)
    return p


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev_i32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.int32:
        t = t.to(torch.int32)
    return t.contiguous()


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:          # automatic promotion (Section 2.2)
        t = t.to(torch.float64)
    return t.contiguous()


class AmgHierarchy:
    """Handle on a cached smoothed-aggregation hierarchy of a CSR matrix.

    Construction calls amg_setup: a cold setup, a cache hit, or an in-place
    value refresh when the same pattern arrives with new values.  A 2-D `val`
    of shape (nnz, S) sets up S systems sharing the pattern (one column of a
    batched solve per system).
    """

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, **params):
        self._L = _lib.load()
        self.row_ptr = _dev_i32(row_ptr, "row_ptr")
        self.col = _dev_i32(col, "col")
        val = _dev_f64(val, "val")
        self.n = self.row_ptr.numel() - 1
        self.nnz = self.col.numel()
        self.n_systems = 1 if val.dim() == 1 else val.shape[1]
        if val.shape[0] != self.nnz:
            raise ValueError("val and col must have the same length")
        self.params = make_params(**params)
        h = C.c_void_p()
        st = self._L.amg_setup(C.byref(self.params), self.n, self.nnz, self.row_ptr.data_ptr(),
                               self.col.data_ptr(), val.data_ptr(), self.n_systems, _stream(), C.byref(h))
        _lib.check(st, "amg_setup")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.amg_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_values(self, val: torch.Tensor):
        val = _dev_f64(val, "val")
        _lib.check(self._L.amg_update_values(self._h, val.data_ptr(), _stream()), "amg_update_values")

    def _solve(self, fn, b: torch.Tensor, tol: float, out: Optional[torch.Tensor]):
        b = _dev_f64(b, "b")
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        if b.shape[0] != self.n:
            raise ValueError(f"rhs has {b.shape[0]} rows, matrix has {self.n}")
        if out is None:
            x = torch.empty_like(b)
        else:
            if (not out.is_cuda or out.dtype != torch.float64 or out.shape != b.shape
                    or not out.is_contiguous()):
                raise ValueError("out must be a contiguous float64 device tensor shaped like b")
            x = out
        info = _lib.amg_info()
        st = fn(self._h, b.data_ptr(), x.data_ptr(), float(tol), nrhs, C.byref(info), _stream())
        _lib.check(st, fn.__name__, allow=(_lib.AMG_OK, _lib.AMG_NOT_CONVERGED))
        d = info.to_dict()
        d["converged"] = st == _lib.AMG_OK
        return x, d

    def solve(self, b: torch.Tensor, tol: float = 1e-8, out: Optional[torch.Tensor] = None):
        """x with A x = b (x0 = 0); returns (x, info)."""
        return self._solve(self._L.amg_solve, b, tol, out)

    def solve_adjoint(self, g: torch.Tensor, tol: float = 1e-8, out: Optional[torch.Tensor] = None):
        """lambda with A^T lambda = g (Eq. (1)); returns (lambda, info)."""
        return self._solve(self._L.amg_solve_adjoint, g, tol, out)

    def pattern_grad(self, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        """dL/dA on the stored pattern: -(lambda_i x_j) per entry (Eq. (2)).

        Batched (n, k) inputs: (nnz, S) per system, or for k right-hand sides
        of one matrix the sum over the columns."""
        lam = _dev_f64(lam, "lambda")
        x = _dev_f64(x, "x")
        if lam.dim() == 1:
            g = torch.empty(self.nnz, dtype=torch.float64, device=lam.device)
            _lib.check(self._L.amg_pattern_grad(self._h, lam.data_ptr(), x.data_ptr(), g.data_ptr(), _stream()),
                       "amg_pattern_grad")
            return g
        k = lam.shape[1]
        g = torch.empty((self.nnz, k) if self.n_systems > 1 else (self.nnz,), dtype=torch.float64,
                        device=lam.device)
        _lib.check(self._L.amg_pattern_grad_batched(self._h, lam.data_ptr(), x.data_ptr(), k, g.data_ptr(),
                                                    _stream()), "amg_pattern_grad_batched")
        return g

    def columns(self, k: int) -> dict:
        """Per-column iterations, true relative residuals and statuses of the
        last batched solve of width k."""
        it = (C.c_int * k)()
        rr = (C.c_double * k)()
        st = (C.c_int * k)()
        _lib.check(self._L.amg_solve_columns(self._h, k, it, rr, st), "amg_solve_columns")
        return dict(iters=list(it), rel_resid=list(rr), status=list(st))

    def apply_vcycle(self, r: torch.Tensor) -> torch.Tensor:
        """z = M^-1 r, one V-cycle (the preconditioner as an operator)."""
        r = _dev_f64(r, "r")
        z = torch.empty_like(r)
        _lib.check(self._L.amg_apply_vcycle(self._h, r.data_ptr(), z.data_ptr(), _stream()), "amg_apply_vcycle")
        return z

    def instrument(self, kernel: str | None, level: int = 0):
        """Time every launch of `kernel` at `level` inside later solves (HIP events)."""
        kid = -1 if kernel is None else _lib.KERNELS[kernel]
        _lib.check(self._L.amg_instrument(self._h, kid, level), "amg_instrument")

    def instrument_read(self) -> dict:
        n = C.c_int(0)
        tot, mn, mx = C.c_double(0), C.c_double(0), C.c_double(0)
        _lib.check(self._L.amg_instrument_read(self._h, C.byref(n), C.byref(tot), C.byref(mn), C.byref(mx)),
                   "amg_instrument_read")
        return dict(launches=n.value, total_ms=tot.value, min_ms=mn.value, max_ms=mx.value,
                    avg_ms=tot.value / n.value if n.value else 0.0)

    def kernel_bytes(self, kernel: str | None, level: int = 0, flexible: bool = False) -> float:
        """Algorithmic bytes of one launch (kernel None: one PCG iteration)."""
        kid = -1 if kernel is None else _lib.KERNELS[kernel]
        b = C.c_double(0)
        _lib.check(self._L.amg_kernel_bytes(self._h, kid, level, int(flexible), C.byref(b)), "amg_kernel_bytes")
        return b.value

    def kernel_bytes_batched(self, kernel: str | None, level: int = 0, flexible: bool = False,
                             width: int | None = None) -> float:
        """Algorithmic bytes of one launch of a batched sweep with `width`
        columns (default: the number of systems); kernel None: one batched
        PCG iteration with every column active."""
        kid = -1 if kernel is None else _lib.KERNELS[kernel]
        w = self.n_systems if width is None else int(width)
        b = C.c_double(0)
        _lib.check(self._L.amg_kernel_bytes_batched(self._h, kid, level, int(flexible), w, C.byref(b)),
                   "amg_kernel_bytes_batched")
        return b.value

    def stats(self) -> dict:
        s = _lib.amg_hier_stats()
        _lib.check(self._L.amg_hierarchy_stats(self._h, C.byref(s)), "amg_hierarchy_stats")
        return s.to_dict()

    def export(self, level: int, field: str) -> torch.Tensor:
        """Copy of one level array (aggregates, A, P, R, strength graph, coarse factor...)."""
        fid = _lib.FIELDS[field]
        count = C.c_int64(0)
        eb = C.c_int(0)
        _lib.check(self._L.amg_field_info(self._h, level, fid, C.byref(count), C.byref(eb)), "amg_field_info")
        dtype = {(4, False): torch.int32, (8, False): torch.float64, (2, False): torch.int16}[(eb.value, False)]
        if field in ("A_v32", "sw32", "coarse_inv32"):
            dtype = torch.float32
        t = torch.empty(max(count.value, 1), dtype=dtype, device="cuda")
        _lib.check(self._L.amg_export_field(self._h, level, fid, t.data_ptr(), t.numel() * t.element_size(),
                                            _stream()), "amg_export_field")
        return t[:count.value]


def solve(A, b: torch.Tensor, tol: float = 1e-8, **params):
    """Solve A x = b; A is (row_ptr, col, val) or a torch sparse CSR tensor.
    Returns (x, info) (Section 3.1)."""
    row_ptr, col, val = _unpack(A)
    h = AmgHierarchy(row_ptr, col, val, **params)
    try:
        return h.solve(b, tol)
    finally:
        h.close()


def _unpack(A):
    if isinstance(A, torch.Tensor) and A.layout == torch.sparse_csr:
        return A.crow_indices(), A.col_indices(), A.values()
    return A


class AmgSolve(torch.autograd.Function):
    """x = A^-1 b with A = CSR(row_ptr, col, val), differentiable in val and b.

    Backward (Eq. (1)-(2)): A^T lambda = dL/dx on the cached hierarchy
    (A symmetric: A's own hierarchy, no transpose formed; symmetric=False:
    the hierarchy of the explicit transpose, formed once); grad_val =
    -(lambda_i x_j) on the stored entries; grad_b = lambda.
    """

    @staticmethod
    def forward(ctx, row_ptr, col, val, b, tol, params):
        kw = dict(params)
        h = AmgHierarchy(row_ptr, col, val, **kw)
        try:
            x, info = h.solve(b, tol)
        finally:
            h.close()
        ctx.save_for_backward(row_ptr, col, val, x)
        ctx.tol = tol
        ctx.params = kw
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        row_ptr, col, val, x = ctx.saved_tensors
        # a cache hit: same pattern and values as the forward solve
        h = AmgHierarchy(row_ptr, col, val.detach(), **ctx.params)
        try:
            lam, _ = h.solve_adjoint(gx.contiguous(), ctx.tol)
            gval = h.pattern_grad(lam, x) if ctx.needs_input_grad[2] else None
        finally:
            h.close()
        gb = lam if ctx.needs_input_grad[3] else None
        return None, None, gval, gb, None, None


def amg_solve(row_ptr, col, val, b, tol: float = 1e-8, **params):
    """Differentiable solve (autograd through val and b)."""
    return AmgSolve.apply(row_ptr, col, val, b, tol, tuple(sorted(params.items())))


class _ProbeAssemble(torch.autograd.Function):
    """CSR values gathered from the probe products Y ([ncolors][n]); the
    backward is the assembly's adjoint (scatter), so gradients reach the
    operator's parameters through the caller's own autograd graph."""

    @staticmethod
    def forward(ctx, Y, op):
        L = _lib.load()
        Y = _dev_f64(Y, "Y")
        val = torch.empty(op.nnz, dtype=torch.float64, device=Y.device)
        _lib.check(L.amg_probe_assemble(op.n, op.nnz, op.row_ptr.data_ptr(), op.col.data_ptr(),
                                        op.color.data_ptr(), op.ncolors, Y.data_ptr(), val.data_ptr(), _stream()),
                   "amg_probe_assemble")
        ctx.op = op
        return val

    @staticmethod
    def backward(ctx, dval):
        op = ctx.op
        L = _lib.load()
        dval = _dev_f64(dval, "dval")
        dY = torch.empty(op.ncolors, op.n, dtype=torch.float64, device=dval.device)
        _lib.check(L.amg_probe_scatter(op.n, op.nnz, op.row_ptr.data_ptr(), op.col.data_ptr(), op.color.data_ptr(),
                                       op.ncolors, dval.data_ptr(), dY.data_ptr(), _stream()), "amg_probe_scatter")
        return dY, None


class MatrixFreeOperator:
    """A linear operator given as a callable x -> A x (torch, on the device)
    together with its CSR sparsity pattern, materialized by graph-colored
    probing (Section 2.1, "Matrix-free operator support").

    The column coloring and the probe vectors are computed once per pattern
    (the paper's cache_coloring / with_cache); ``assemble(matvec)`` applies
    the operator once per color and gathers the values, differentiably.  Use
    ``solve`` / ``amg_solve_op`` to solve with the assembled matrix."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, matvec=None):
        L = _lib.load()
        self.row_ptr = _dev_i32(row_ptr, "row_ptr")
        self.col = _dev_i32(col, "col")
        self.n = self.row_ptr.numel() - 1
        self.nnz = self.col.numel()
        self.matvec = matvec
        self.color = torch.empty(self.n, dtype=torch.int32, device=self.row_ptr.device)
        nc = C.c_int32(0)
        _lib.check(L.amg_color_columns(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                                       self.color.data_ptr(), C.byref(nc), _stream()), "amg_color_columns")
        self.ncolors = nc.value
        self.probes = torch.empty(self.ncolors, self.n, dtype=torch.float64, device=self.row_ptr.device)
        _lib.check(L.amg_probe_vectors(self.n, self.color.data_ptr(), self.ncolors, self.probes.data_ptr(),
                                       _stream()), "amg_probe_vectors")

    def with_operator(self, matvec) -> "MatrixFreeOperator":
        """The same pattern and coloring for another operator (e.g. new parameters)."""
        op = object.__new__(MatrixFreeOperator)
        op.__dict__.update(self.__dict__)
        op.matvec = matvec
        return op

    def assemble(self, matvec=None) -> torch.Tensor:
        """CSR values of the operator: one application per color."""
        f = matvec if matvec is not None else self.matvec
        if f is None:
            raise ValueError("no operator to assemble")
        Y = torch.stack([f(self.probes[c]) for c in range(self.ncolors)])
        return _ProbeAssemble.apply(Y, self)

    def csr(self, matvec=None):
        return self.row_ptr, self.col, self.assemble(matvec)

    def solve(self, b: torch.Tensor, tol: float = 1e-8, **params):
        """Differentiable solve A x = b with the assembled operator."""
        return amg_solve(self.row_ptr, self.col, self.assemble(), b, tol, **params)


def make_preconditioner(row_ptr, col, val, **params):
    """The V-cycle as a callable r -> M^-1 r for other Krylov solvers (Section 2.2)."""
    h = AmgHierarchy(row_ptr, col, val, **params)
    return h.apply_vcycle


def finalize():
    """Empty the setup cache (Section 3.4)."""
    _lib.check(_lib.load().amg_finalize(), "amg_finalize")


def cache_size() -> int:
    return _lib.load().amg_cache_size()


def set_cache_capacity(n: int):
    _lib.check(_lib.load().amg_set_cache_capacity(n), "amg_set_cache_capacity")
