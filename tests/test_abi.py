"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and rejects bad descriptors before touching the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gp.h")
LIB = os.path.join(ROOT, "paper_2003_03590_amd", "libgp_mi355x.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^GP_API [^()]*?\b(gp_\w+)\(", txt, flags=re.M)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def test_header_declares_the_boundary():
    names = declared()
    for must in ("gp_plan", "gp_init_phase", "gp_step_n", "gp_energies", "gp_spectra", "gp_adjoint_step_n"):
        assert must in names


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


@needs_lib
def test_binding_signatures_cover_header():
    from paper_2003_03590_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared()


@needs_lib
def test_host_side_validation_without_gpu():
    import paper_2003_03590_amd as gp
    from paper_2003_03590_amd import _lib
    lib = gp.lib()
    h = C.c_void_p()
    bad = [((5, 8, 8), 0), ((0, 8, 8), 0), ((8, 8, 2048), 0), ((8, 8, 8), 7)]
    want = [_lib.GP_ERR_UNSUPPORTED, _lib.GP_ERR_ARG, _lib.GP_ERR_UNSUPPORTED, _lib.GP_ERR_UNSUPPORTED]
    for (n, prec), w in zip(bad, want):
        d = _lib.gp_desc((C.c_int32 * 3)(*n), 1.0, 1.0, 1e-3, prec, 0)
        assert lib.gp_plan(C.byref(d), None, C.byref(h)) == w
        assert h.value is None
        assert lib.gp_last_error().decode()
    d = _lib.gp_desc((C.c_int32 * 3)(8, 8, 8), float("nan"), 1.0, 1e-3, 0, 0)
    assert lib.gp_plan(C.byref(d), None, C.byref(h)) == _lib.GP_ERR_ARG
    assert lib.gp_plan(None, None, C.byref(h)) == _lib.GP_ERR_ARG
    assert lib.gp_step_n(None, None, 1) == _lib.GP_ERR_ARG
    assert lib.gp_plan_destroy(None) == _lib.GP_ERR_ARG


@needs_lib
def test_every_supported_length_has_a_schedule():
    import paper_2003_03590_amd as gp
    lib = gp.lib()
    for n in (2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024):
        for prec in (0, 1):
            assert lib.gp_variant_count(n, prec) >= 1, (n, prec)


@needs_lib
def test_new_entry_points_reject_null_plans_without_gpu():
    """Every entry point validates its arguments on the host before any GPU work:
    a null plan is GP_ERR_ARG with a message, for the imaginary-time, velocity
    statistics and helicity calls as for the rest."""
    import paper_2003_03590_amd as gp
    from paper_2003_03590_amd import _lib
    lib = gp.lib()
    d = C.c_double()
    two = (C.c_double * 2)()
    rep = _lib.gp_argle_report()
    calls = [
        lambda: lib.gp_argle_step(None, None, None, 0.01, 1, None),
        lambda: lib.gp_argle_energy(None, None, None, None, C.byref(d)),
        lambda: lib.gp_argle_run(None, None, None, 0.01, 10, 5, 0.0, None, C.byref(rep)),
        lambda: lib.gp_structure_fn_velocity(None, None, None, 2, two, None),
        lambda: lib.gp_mach(None, None, None, two),
        lambda: lib.gp_helicity(None, None, None, two, None, 0),
    ]
    for f in calls:
        assert f() == _lib.GP_ERR_ARG
        assert lib.gp_last_error().decode()
    assert lib.gp_helicity_work_bytes(None) == 0
    assert lib.gp_schedule_name(None, 4) == b""


@needs_lib
def test_allocation_fault_is_nomem_without_gpu(monkeypatch):
    """GP_FAULT_INJECT=alloc: plan creation stops at its first device allocation
    (before any HIP call) with GP_ERR_NOMEM and a message, and hands back no plan."""
    import paper_2003_03590_amd as gp
    from paper_2003_03590_amd import _lib
    lib = gp.lib()
    monkeypatch.setenv("GP_FAULT_INJECT", "alloc")
    h = C.c_void_p()
    for prec in (0, 1):
        d = _lib.gp_desc((C.c_int32 * 3)(16, 12, 8), 1.0, 1.0, 1e-3, prec, 0)
        assert lib.gp_plan(C.byref(d), None, C.byref(h)) == _lib.GP_ERR_NOMEM
        assert h.value is None
        assert "injected" in lib.gp_last_error().decode()
