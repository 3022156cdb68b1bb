"""ctypes shim over liboracle.so, plus the explicit diffusion chain rule.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg of the
benchmark).  Everything here is FP64 and runs on the host.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["OracleHierarchy", "spmv", "pattern_grad", "rel_residual", "node_key", "validate", "transpose",
           "color_columns", "probe_vectors", "probe_assemble", "probe_scatter",
           "diffusion_theta_grad", "OR_OK", "OR_NOT_CONVERGED", "OR_ERR_INVALID_ARG", "OR_ERR_ZERO_DIAG",
           "OR_ERR_PATTERN_MISMATCH", "OR_ERR_BREAKDOWN", "OR_ERR_COARSE_TOO_LARGE", "load",
           "set_threads", "get_threads", "host_cores", "OracleError"]

OR_OK = 0
OR_NOT_CONVERGED = 1
OR_ERR_INVALID_ARG = -1
OR_ERR_ZERO_DIAG = -2
OR_ERR_PATTERN_MISMATCH = -3
OR_ERR_BREAKDOWN = -4
OR_ERR_COARSE_TOO_LARGE = -7

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def load():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    L = C.CDLL(path)
    L.or_setup.restype = C.c_void_p
    L.or_setup.argtypes = [C.c_int, _ip, _ip, _dp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                           C.c_int, C.c_int, C.POINTER(C.c_int)]
    L.or_update_values.restype = C.c_int
    L.or_update_values.argtypes = [C.c_void_p, _dp]
    L.or_destroy.argtypes = [C.c_void_p]
    L.or_num_levels.restype = C.c_int
    L.or_num_levels.argtypes = [C.c_void_p]
    L.or_level_sizes.restype = C.c_int
    L.or_level_sizes.argtypes = [C.c_void_p, C.c_int, np.ctypeslib.ndpointer(dtype=np.int64)]
    L.or_export_level.restype = C.c_int
    L.or_export_level.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 14
    L.or_export_sw.restype = C.c_int
    L.or_export_sw.argtypes = [C.c_void_p, C.c_int, _dp]
    L.or_coarse_factor.restype = C.c_int
    L.or_coarse_factor.argtypes = [C.c_void_p, _dp]
    L.or_coarse_pivots.restype = C.c_int
    L.or_coarse_pivots.argtypes = [C.c_void_p, _ip]
    L.or_bicgstab.restype = C.c_int
    L.or_bicgstab.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int),
                              C.POINTER(C.c_double), C.c_void_p]
    L.or_transpose.argtypes = [C.c_int, _ip, _ip, _dp, _ip, _ip, _dp]
    L.or_vcycle.restype = C.c_int
    L.or_vcycle.argtypes = [C.c_void_p, _dp, _dp]
    L.or_pcg.restype = C.c_int
    L.or_pcg.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int),
                         C.POINTER(C.c_double), C.c_void_p, C.c_void_p]
    L.or_solve_adjoint.restype = C.c_int
    L.or_solve_adjoint.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int),
                                   C.POINTER(C.c_double)]
    L.or_pattern_grad.argtypes = [C.c_int, _ip, _ip, _dp, _dp, _dp]
    L.or_spmv.argtypes = [C.c_int, _ip, _ip, _dp, _dp, _dp]
    L.or_rel_residual.restype = C.c_double
    L.or_rel_residual.argtypes = [C.c_int, _ip, _ip, _dp, _dp, _dp]
    L.or_color_columns.restype = C.c_int
    L.or_color_columns.argtypes = [C.c_int, _ip, _ip, _ip]
    L.or_probe_assemble.argtypes = [C.c_int, _ip, _ip, _ip, _dp, _dp]
    L.or_probe_scatter.argtypes = [C.c_int, _ip, _ip, _ip, C.c_int, _dp, _dp]
    L.or_node_key.restype = C.c_uint64
    L.or_node_key.argtypes = [C.c_int]
    L.or_validate.restype = C.c_int
    L.or_validate.argtypes = [C.c_int, _ip, _ip]
    L.or_set_threads.argtypes = [C.c_int]
    L.or_get_threads.restype = C.c_int
    _LIB = L
    return L


def set_threads(k: int):
    """Threads of the oracle's solve loops (default 1).  Results do not depend
    on it: rows and fixed dot-product blocks are shared out, never split."""
    load().or_set_threads(int(k))


def get_threads() -> int:
    return load().or_get_threads()


def host_cores() -> int:
    """Cores this process may run on (its affinity mask, capped at 16, the
    CPU share of one GPU on the box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"oracle {where} failed with status {status}")
        self.status = status


class OracleHierarchy:
    """FP64 SA-AMG hierarchy built on the host by the oracle.

    symmetric=False: the coarsest level gets an LU factorization with partial
    pivoting instead of Cholesky, and the adjoint is solved on the hierarchy
    of the explicit transpose (built on first use with the same parameters).
    """

    def __init__(self, row_ptr, col, val, theta=0.0, max_coarse=256, max_levels=20, smoother="jacobi",
                 omega=2.0 / 3.0, nu_pre=1, nu_post=1, symmetric=True):
        L = load()
        self.rp, self.ci, self.v = _i32(row_ptr), _i32(col), _f64(val)
        self.n = len(self.rp) - 1
        self.symmetric = bool(symmetric)
        self._kw = dict(theta=theta, max_coarse=max_coarse, max_levels=max_levels, smoother=smoother, omega=omega,
                        nu_pre=nu_pre, nu_post=nu_post)
        self._adj = None
        st = C.c_int(0)
        sm = {"jacobi": 0, "l1": 1}[smoother]
        h = L.or_setup(self.n, self.rp, self.ci, self.v, float(theta), int(max_coarse), int(max_levels), sm,
                       float(omega), int(nu_pre), int(nu_post), int(self.symmetric), C.byref(st))
        if not h:
            raise OracleError(st.value, "setup")
        self._h = h
        self._L = L

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.or_destroy(h)
            self._h = None

    # -- structure
    @property
    def num_levels(self):
        return self._L.or_num_levels(self._h)

    def level_sizes(self, l):
        out = np.zeros(5, dtype=np.int64)
        st = self._L.or_level_sizes(self._h, l, out)
        if st:
            raise OracleError(st, "level_sizes")
        return dict(n=int(out[0]), nnz=int(out[1]), nnzP=int(out[2]), nagg=int(out[3]), nnzG=int(out[4]))

    def level(self, l):
        """All arrays of level l as numpy (P/R/agg empty on the coarsest level;
        sw = smoother weights)."""
        s = self.level_sizes(l)
        n, nnz, nnzP, nagg, nnzG = s["n"], s["nnz"], s["nnzP"], s["nagg"], s["nnzG"]
        coarsest = (l == self.num_levels - 1)
        out = dict(
            A_rp=np.zeros(n + 1, np.int32), A_ci=np.zeros(nnz, np.int32), A_v=np.zeros(nnz),
            dinv=np.zeros(n),
        )
        if not coarsest:
            out.update(agg=np.zeros(n, np.int32), P_rp=np.zeros(n + 1, np.int32), P_ci=np.zeros(nnzP, np.int32),
                       P_v=np.zeros(nnzP), R_rp=np.zeros(nagg + 1, np.int32), R_ci=np.zeros(nnzP, np.int32),
                       R_v=np.zeros(nnzP), G_rp=np.zeros(n + 1, np.int32), G_ci=np.zeros(nnzG, np.int32))
        scal = np.zeros(2)
        g = out.get
        st = self._L.or_export_level(self._h, l, _ptr(g("agg")), _ptr(g("A_rp")), _ptr(g("A_ci")), _ptr(g("A_v")),
                                     _ptr(g("dinv")), _ptr(g("P_rp")), _ptr(g("P_ci")), _ptr(g("P_v")),
                                     _ptr(g("R_rp")), _ptr(g("R_ci")), _ptr(g("R_v")), _ptr(g("G_rp")),
                                     _ptr(g("G_ci")), _ptr(scal))
        if st:
            raise OracleError(st, "export_level")
        out["sw"] = np.zeros(n)
        st = self._L.or_export_sw(self._h, l, out["sw"])
        if st:
            raise OracleError(st, "export_sw")
        out["rho"], out["omegaP"] = float(scal[0]), float(scal[1])
        out["n"], out["nagg"] = n, nagg
        return out

    def coarse_factor(self):
        """Cholesky factor (lower) or, for symmetric=False, the packed LU
        factor (unit-lower multipliers below the diagonal, U on and above)."""
        n = self.level_sizes(self.num_levels - 1)["n"]
        Lf = np.zeros(n * n)
        self._L.or_coarse_factor(self._h, Lf)
        return Lf.reshape(n, n)

    def coarse_pivots(self):
        """LU pivot rows (row exchanged with row k at step k); None for Cholesky."""
        n = self.level_sizes(self.num_levels - 1)["n"]
        piv = np.zeros(n, np.int32)
        return piv if self._L.or_coarse_pivots(self._h, piv) else None

    # -- numerics
    def update_values(self, val):
        self.v = _f64(val)
        st = self._L.or_update_values(self._h, self.v)
        if st:
            raise OracleError(st, "update_values")
        if self._adj is not None:
            self._adj.update_values(transpose(self.rp, self.ci, self.v)[2])

    def vcycle(self, b):
        b = _f64(b)
        x = np.zeros(self.n)
        self._L.or_vcycle(self._h, b, x)
        return x

    def pcg(self, b, tol=1e-8, maxiter=1000, flexible=False, precondition=True, history=False,
            variable_preconditioner=False):
        """Returns (x, info) with info = dict(iters, rel_resid, status).

        history=True adds the recursive residual per iteration and the cosine
        between each new direction and A times the previous one.
        variable_preconditioner=True scales the V-cycle output by a positive
        diagonal that changes every iteration (test hook).
        """
        b = _f64(b)
        x = np.zeros(self.n)
        it = C.c_int(0)
        rr = C.c_double(0.0)
        hist = np.zeros(max(maxiter, 1)) if history else None
        conj = np.zeros(max(maxiter, 1)) if history else None
        mode = 2 if variable_preconditioner else int(bool(precondition))
        st = self._L.or_pcg(self._h, b, x, float(tol), int(maxiter), int(bool(flexible)), mode,
                            C.byref(it), C.byref(rr), _ptr(hist), _ptr(conj))
        info = dict(iters=it.value, rel_resid=rr.value, status=st)
        if history:
            info["history"] = hist[:it.value].copy()
            info["conj"] = conj[:max(it.value - 1, 0)].copy()
        return x, info

    def bicgstab(self, b, tol=1e-8, maxiter=1000, precondition=True, history=False):
        """Right-preconditioned BiCGSTAB from x0 = 0; returns (x, info) like pcg."""
        b = _f64(b)
        x = np.zeros(self.n)
        it = C.c_int(0)
        rr = C.c_double(0.0)
        hist = np.zeros(max(maxiter, 1)) if history else None
        st = self._L.or_bicgstab(self._h, b, x, float(tol), int(maxiter), int(bool(precondition)), C.byref(it),
                                 C.byref(rr), _ptr(hist))
        info = dict(iters=it.value, rel_resid=rr.value, status=st)
        if history:
            info["history"] = hist[:it.value].copy()
        return x, info

    def transpose_hierarchy(self):
        """Hierarchy of A^T with the same parameters (nonsymmetric adjoint)."""
        if self._adj is None:
            rpT, ciT, vT = transpose(self.rp, self.ci, self.v)
            self._adj = OracleHierarchy(rpT, ciT, vT, symmetric=False, **self._kw)
        return self._adj

    def solve_adjoint(self, g, tol=1e-8, maxiter=1000, flexible=False, solver="pcg"):
        """A^T lambda = g (Eq. (1)).  Symmetric A: A's own hierarchy; otherwise
        the hierarchy of the explicit transpose.  solver: "pcg" or "bicgstab"
        (a nonsymmetric A always takes BiCGSTAB)."""
        if not self.symmetric:
            return self.transpose_hierarchy().bicgstab(g, tol=tol, maxiter=maxiter)
        if solver == "bicgstab":
            return self.bicgstab(g, tol=tol, maxiter=maxiter)
        g = _f64(g)
        lam = np.zeros(self.n)
        it = C.c_int(0)
        rr = C.c_double(0.0)
        st = self._L.or_solve_adjoint(self._h, g, lam, float(tol), int(maxiter), int(bool(flexible)), C.byref(it),
                                      C.byref(rr))
        return lam, dict(iters=it.value, rel_resid=rr.value, status=st)

    def pattern_grad(self, lam, x):
        return pattern_grad(self.rp, self.ci, lam, x)


def spmv(rp, ci, v, x):
    rp, ci, v, x = _i32(rp), _i32(ci), _f64(v), _f64(x)
    y = np.zeros(len(rp) - 1)
    load().or_spmv(len(rp) - 1, rp, ci, v, x, y)
    return y


def pattern_grad(rp, ci, lam, x):
    """grad_val[k] = -(lambda[row k] * x[col k]) (Eq. (2) on the stored pattern)."""
    rp, ci, lam, x = _i32(rp), _i32(ci), _f64(lam), _f64(x)
    g = np.zeros(len(ci))
    load().or_pattern_grad(len(rp) - 1, rp, ci, lam, x, g)
    return g


def transpose(rp, ci, v):
    """Explicit CSR transpose (row_ptr, col, val) of a square CSR matrix."""
    rp, ci, v = _i32(rp), _i32(ci), _f64(v)
    n = len(rp) - 1
    rpT = np.zeros(n + 1, np.int32)
    ciT = np.zeros(len(ci), np.int32)
    vT = np.zeros(len(ci))
    load().or_transpose(n, rp, ci, v, rpT, ciT, vT)
    return rpT, ciT, vT


def rel_residual(rp, ci, v, b, x):
    rp, ci, v, b, x = _i32(rp), _i32(ci), _f64(v), _f64(b), _f64(x)
    return float(load().or_rel_residual(len(rp) - 1, rp, ci, v, b, x))


def color_columns(rp, ci):
    """(color[n], ncolors): greedy column coloring in decreasing key order
    (no two columns of one color share a row)."""
    rp, ci = _i32(rp), _i32(ci)
    n = len(rp) - 1
    color = np.zeros(n, np.int32)
    nc = load().or_color_columns(n, rp, ci, color)
    return color, int(nc)


def probe_vectors(color, ncolors):
    """V[c][j] = 1 if column j has color c (the probe vectors, [ncolors][n])."""
    color = np.asarray(color)
    V = np.zeros((ncolors, len(color)))
    V[color, np.arange(len(color))] = 1.0
    return V


def probe_assemble(rp, ci, color, Y):
    """CSR values from the probe products Y = A V^T ([ncolors][n])."""
    rp, ci, color = _i32(rp), _i32(ci), _i32(color)
    Y = _f64(Y)
    val = np.zeros(len(ci))
    load().or_probe_assemble(len(rp) - 1, rp, ci, color, Y.ravel(), val)
    return val


def probe_scatter(rp, ci, color, ncolors, dval):
    """Adjoint of probe_assemble: dY ([ncolors][n])."""
    rp, ci, color, dval = _i32(rp), _i32(ci), _i32(color), _f64(dval)
    n = len(rp) - 1
    dY = np.zeros(ncolors * n)
    load().or_probe_scatter(n, rp, ci, color, int(ncolors), dval, dY)
    return dY.reshape(ncolors, n)


def node_key(i: int) -> int:
    return int(load().or_node_key(int(i)))


def validate(rp, ci):
    return int(load().or_validate(len(rp) - 1, _i32(rp), _i32(ci)))


def diffusion_theta_grad(k: np.ndarray, rp, ci, grad_val) -> np.ndarray:
    """dL/dtheta for k = exp(theta) through the harmonic-face diffusion assembly.

    Written out explicitly (no autograd): for an interior face (p, q) with
    k_f = 2 k_p k_q / (k_p + k_q), the face touches A_pp, A_qq (+k_f) and
    A_pq, A_qp (-k_f), so dL/dk_f = g_pp + g_qq - g_pq - g_qp and
    dk_f/dk_p = 2 k_q^2 / (k_p + k_q)^2.  A boundary face of p has k_f = k_p
    and touches A_pp only.  Finally dk/dtheta = k.  Pattern gradients
    g = grad_val come from Eq. (2).
    """
    k = np.asarray(k, dtype=np.float64)
    d = k.ndim
    N = k.shape[0]
    n = N ** d
    kflat = k.ravel()
    rp = np.asarray(rp)
    ci = np.asarray(ci)
    g = np.asarray(grad_val)
    rows = np.repeat(np.arange(n), np.diff(rp))

    def entry(p, q):
        # position of (p, q) in the CSR arrays (vectorised over p, q)
        lo = rp[p]
        hi = rp[p + 1]
        out = np.empty(len(p), dtype=np.int64)
        for t in range(len(p)):
            seg = ci[lo[t]:hi[t]]
            out[t] = lo[t] + np.searchsorted(seg, q[t])
        return out

    # diagonal positions
    diag_pos = np.empty(n, dtype=np.int64)
    for i in range(n):
        seg = ci[rp[i]:rp[i + 1]]
        diag_pos[i] = rp[i] + np.searchsorted(seg, i)
    gdiag = g[diag_pos]
    dk = np.zeros(n)
    idx = np.arange(n)
    coords = [(idx // (N ** a)) % N for a in range(d)]
    for a in range(d):
        stride = N ** a
        # interior faces between p and q = p + e_a
        p = idx[coords[a] < N - 1]
        q = p + stride
        kp, kq = kflat[p], kflat[q]
        gpq = g[entry(p, q)]
        gqp = g[entry(q, p)]
        dLdkf = gdiag[p] + gdiag[q] - gpq - gqp
        s = kp + kq
        np.add.at(dk, p, dLdkf * (2.0 * kq * kq) / (s * s))
        np.add.at(dk, q, dLdkf * (2.0 * kp * kp) / (s * s))
        # boundary faces: low side (coord 0) and high side (coord N-1)
        for bnd in (idx[coords[a] == 0], idx[coords[a] == N - 1]):
            np.add.at(dk, bnd, gdiag[bnd])
    del rows
    return (dk * kflat).reshape(k.shape)
