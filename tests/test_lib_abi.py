"""The C-ABI library loads and exports every symbol include/amg355.h declares;
host-side argument validation (CPU only, no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amg355.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amg_[a-z_0-9]+)\s*\(", text)))


def test_header_lists_the_boundary():
    names = _declared()
    for must in ("amg_setup", "amg_solve", "amg_solve_adjoint", "amg_update_values", "amg_pattern_grad",
                 "amg_destroy", "amg_finalize"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2606_09001_amd import _lib
    L = _lib.load()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == _declared()


def test_params_default_and_status_strings():
    from paper_2606_09001_amd import _lib
    L = _lib.load()
    p = _lib.amg_params()
    L.amg_params_default(C.byref(p))
    assert p.vcycle_prec == _lib.AMG_PREC_FP64 and p.max_coarse == 256 and p.max_levels == 20
    assert p.omega == pytest.approx(2.0 / 3.0) and p.nu_pre == 1 and p.nu_post == 1
    assert p.theta == 0.0 and p.symmetric == 1 and p.flexible == -1 and p.precondition == 1
    assert p.solver == _lib.AMG_SOLVER_PCG
    for st, name in [(0, "AMG_OK"), (1, "AMG_NOT_CONVERGED"), (-1, "AMG_ERR_INVALID_ARG"),
                     (-4, "AMG_ERR_BREAKDOWN"), (-7, "AMG_ERR_COARSE_TOO_LARGE")]:
        assert _lib.status_string(st) == name


def test_setup_rejects_bad_arguments_before_touching_a_device():
    from paper_2606_09001_amd import _lib
    L = _lib.load()
    h = C.c_void_p()
    p = _lib.amg_params()
    L.amg_params_default(C.byref(p))
    assert L.amg_setup(C.byref(p), 0, 0, 1, 1, 1, 1, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    assert L.amg_setup(C.byref(p), 4, 4, None, 1, 1, 1, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 0, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 65, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    p.theta = 0.1   # several systems need the pattern-only aggregation
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 2, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    p.theta = 0.0
    p.nu_pre = 2    # and V(1,1)
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 2, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    p.nu_pre = 1
    p.symmetric = 0  # CG needs A = A^T: a nonsymmetric A takes BiCGSTAB
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 1, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    p.symmetric = 2
    p.solver = _lib.AMG_SOLVER_BICGSTAB
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 1, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    p.symmetric = 0  # BiCGSTAB: one system only
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 2, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    p.solver = 2
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 1, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    p.solver = _lib.AMG_SOLVER_PCG
    p.symmetric = 1
    p.precondition = 2
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 1, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    p.precondition = 1
    p.max_levels = 99
    assert L.amg_setup(C.byref(p), 4, 4, 1, 1, 1, 1, None, C.byref(h)) == _lib.AMG_ERR_INVALID_ARG
    assert L.amg_solve(None, 1, 1, 1e-8, 1, None, None) == _lib.AMG_ERR_INVALID_ARG
    assert L.amg_destroy(None) == _lib.AMG_ERR_INVALID_ARG
    assert not h.value


def test_make_params_overrides():
    from paper_2606_09001_amd.solver import make_params
    p = make_params(vcycle_prec="fp32", smoother="l1", omega=0.5, max_coarse=64)
    assert p.vcycle_prec == 1 and p.smoother == 1 and p.omega == 0.5 and p.max_coarse == 64
    p = make_params(solver="bicgstab", symmetric=False)
    assert p.solver == 1 and p.symmetric == 0
    with pytest.raises(TypeError):
        make_params(bogus=1)


def test_matrix_free_entry_points_reject_bad_arguments_before_touching_a_device():
    from paper_2606_09001_amd import _lib
    L = _lib.load()
    nc = C.c_int32(0)
    E = _lib.AMG_ERR_INVALID_ARG
    assert L.amg_color_columns(0, 0, 1, 1, 1, C.byref(nc), None) == E          # n <= 0
    assert L.amg_color_columns(4, 3, 1, 1, 1, C.byref(nc), None) == E          # nnz < n
    assert L.amg_color_columns(4, 4, None, 1, 1, C.byref(nc), None) == E       # null row_ptr
    assert L.amg_color_columns(4, 4, 1, 1, 1, None, None) == E                 # null ncolors
    assert L.amg_probe_vectors(4, 1, 0, 1, None) == E                          # ncolors <= 0
    assert L.amg_probe_vectors(4, None, 2, 1, None) == E
    assert L.amg_probe_assemble(4, 4, 1, 1, 1, 0, 1, 1, None) == E             # ncolors <= 0
    assert L.amg_probe_assemble(4, 4, 1, 1, 1, 2, None, 1, None) == E          # null Y
    assert L.amg_probe_scatter(4, 4, 1, 1, 1, 2, 1, None, None) == E           # null dY
    assert L.amg_probe_scatter(-1, 4, 1, 1, 1, 2, 1, 1, None) == E
    assert L.amg_solve_adjoint(None, 1, 1, 1e-8, 1, None, None) == E


def test_convert_bf16_rejects_bad_arguments_before_touching_a_device():
    from paper_2606_09001_amd import _lib
    L = _lib.load()
    assert L.amg_convert_bf16(1, 1, -1, None) == _lib.AMG_ERR_INVALID_ARG
    assert L.amg_convert_bf16(None, 1, 4, None) == _lib.AMG_ERR_INVALID_ARG
    assert L.amg_convert_bf16(1, None, 4, None) == _lib.AMG_ERR_INVALID_ARG
    assert L.amg_convert_bf16(None, None, 0, None) == _lib.AMG_OK      # nothing to convert
