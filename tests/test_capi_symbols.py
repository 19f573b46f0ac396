"""The C-ABI library loads on the CPU host and exports every function that
include/hyperpower.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyperpower.h")
LIB = os.path.join(ROOT, "paper_2311_06926_amd", "libhyperpower.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(hp_\w+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hp_setup", "hp_apply_K", "hp_apply_P0", "hp_apply_hyperpower", "hp_solve"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_the_header():
    from paper_2311_06926_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_functions())
    lib = _lib.load()
    opts = _lib.hp_opts()
    lib.hp_default_opts(ctypes.byref(opts))
    assert opts.c_pen == 0.0 and opts.order == 2 and opts.max_rhs == 1
    assert opts.autotune == 1 and opts.op_kchunk == 0 and opts.op_order == -1 and opts.fd_plan == -1
    assert opts.op_slabs == 0 and opts.schur_level == 0
    assert opts.schur_pcg_iters == 20 and opts.schur_pcg_tol == 1e-2 and opts.op_fused == -1
    assert opts.op_staged == -1 and opts.use_graph == 0 and opts.poll_lag == 1
    assert opts.forward == 0 and opts.use_x0 == 0 and opts.spectrum_gate == 0
    assert opts.p0_scale == 1.0 and opts.breakdown_tol == 0.0 and opts.op_dma == -1
    assert opts.op_pres_wide == -1
    assert lib.hp_status_string(-6) == b"not converged within maxit"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_setup_rejects_bad_arguments_without_touching_the_gpu():
    from paper_2311_06926_amd import _lib
    lib = _lib.load()
    ctx = ctypes.c_void_p()
    # invalid degree / elements / viscosity are rejected before any HIP call
    assert lib.hp_setup(8, 1, 1.0, None, None, ctypes.byref(ctx)) == -1
    assert lib.hp_setup(0, 2, 1.0, None, None, ctypes.byref(ctx)) == -1
    assert lib.hp_setup(8, 2, -1.0, None, None, ctypes.byref(ctx)) == -1
    assert lib.hp_setup(8, 2, 1.0, None, None, None) == -1
    assert lib.hp_apply_K(None, None, None, 1) == -1
    assert lib.hp_get_tuning(None, 1, ctypes.byref(_lib.hp_tuning())) == -1
    d, lo, hi = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    assert lib.hp_spectrum(None, 0, 2, 0, 0, 10, None, None, None, ctypes.byref(d),
                           ctypes.byref(lo), ctypes.byref(hi)) == -1
    # out-of-range launch-shape options are rejected before any HIP call
    for field, bad in (("op_kchunk", -1), ("op_order", 2), ("fd_plan", 10), ("fd_plan", -2),
                       ("op_slabs", -1), ("schur_level", -1), ("schur_level", 7),
                       ("schur_variant", 0), ("schur_variant", 4), ("schur_pcg_iters", 0),
                       ("schur_pcg_tol", -1.0), ("op_fused", -2), ("op_fused", 2),
                       ("op_staged", -2), ("op_staged", 2), ("use_graph", -1), ("use_graph", 2),
                       ("poll_lag", 0), ("poll_lag", 4), ("forward", -1), ("forward", 2),
                       ("use_x0", 2), ("use_x0", -1), ("spectrum_gate", -1),
                       ("p0_scale", -0.5), ("p0_scale", float("nan")),
                       ("breakdown_tol", -1.0), ("op_dma", -2), ("op_dma", 2),
                       ("op_pres_wide", -2), ("op_pres_wide", 2)):
        opts = _lib.hp_opts()
        lib.hp_default_opts(ctypes.byref(opts))
        setattr(opts, field, bad)
        assert lib.hp_setup(8, 2, 1.0, ctypes.byref(opts), None, ctypes.byref(ctx)) == -1, field
