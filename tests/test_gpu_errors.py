"""The error model of the C ABI on the GPU, with every failure forced from the
host (no kernel faults, traps or hangs): non-finite diagnostics, allocation
failure, and a HIP error that leaves the plan unusable."""
import ctypes as C
import math

import numpy as np
import pytest

import gp_inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _lib():
    import paper_2003_03590_amd as gp
    from paper_2003_03590_amd import _lib as L
    return gp, L, gp.lib()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_nonfinite_field_reports_nonfinite_with_values_written(prec):
    gp, L, lib = _lib()
    plan = gp.Plan(16, 0.5, 2.0, 1e-3, prec)
    a = I.random_field(16, seed=3)
    a[5, 6, 7] = complex(float("nan"), 0.0)
    psi = torch.from_numpy(a).to(DEV).to(plan.dtype).contiguous()
    e = L.gp_energy(*([-1.0] * 7))
    st = lib.gp_energies(plan._h, C.c_void_p(psi.data_ptr()), C.c_void_p(plan.work().data_ptr()), C.byref(e))
    assert st == L.GP_ERR_NONFINITE
    assert "not finite" in lib.gp_last_error().decode()
    assert math.isnan(e.mass)                       # written, not left at the sentinel
    spec = np.full(4 * plan.nshell, -1.0)
    e2 = L.gp_energy(*([-1.0] * 7))
    st = lib.gp_spectra(plan._h, C.c_void_p(psi.data_ptr()), C.c_void_p(plan.work().data_ptr()),
                        spec.ctypes.data_as(C.POINTER(C.c_double)), plan.nshell, C.byref(e2))
    assert st == L.GP_ERR_NONFINITE
    assert not np.all(np.isfinite(spec)) and not np.any(spec == -1.0)
    # a non-finite result does not break the plan: a finite field diagnoses normally
    good = torch.from_numpy(I.random_field(16, seed=4)).to(DEV).to(plan.dtype).contiguous()
    assert math.isfinite(plan.energies(good)["energy"])
    plan.close()


def test_allocation_failure_is_nomem_and_recoverable(monkeypatch):
    gp, L, lib = _lib()
    monkeypatch.setenv("GP_FAULT_INJECT", "alloc")
    for prec in ("c128", "c64"):
        with pytest.raises(gp.GPError) as ei:
            gp.Plan(32, 0.5, 2.0, 1e-3, prec)
        assert ei.value.status == L.GP_ERR_NOMEM
    with pytest.raises(gp.GPError) as ei:
        gp.BatchPlan([dict(n=16, alpha=0.3, beta=2.0, dt=0.01), dict(n=24, alpha=0.3, beta=2.0, dt=0.01)], "c64")
    assert ei.value.status == L.GP_ERR_NOMEM
    monkeypatch.delenv("GP_FAULT_INJECT")
    plan = gp.Plan(32, 0.5, 2.0, 1e-3, "c128")     # the library is still usable
    psi = torch.from_numpy(I.random_field(32, seed=5)).to(DEV).contiguous()
    plan.step_n(psi, 2)
    assert math.isfinite(plan.energies(psi)["mass"])
    plan.close()


def test_hip_error_breaks_the_plan(monkeypatch):
    """A HIP error reported by a launch check (forced from the host) returns
    GP_ERR_HIP and leaves the plan unusable: every later call on it returns
    GP_ERR_STATE; other plans are unaffected and the broken plan is destroyed
    cleanly."""
    gp, L, lib = _lib()
    plan = gp.Plan(16, 0.5, 2.0, 1e-3, "c128")
    other = gp.Plan(16, 0.5, 2.0, 1e-3, "c128")
    psi = torch.from_numpy(I.random_field(16, seed=6)).to(DEV).contiguous()
    monkeypatch.setenv("GP_FAULT_INJECT", "launch")
    with pytest.raises(gp.GPError) as ei:
        plan.step_n(psi, 1)
    assert ei.value.status == L.GP_ERR_HIP
    monkeypatch.delenv("GP_FAULT_INJECT")
    for call in (lambda: plan.step_n(psi, 1), lambda: plan.energies(psi), lambda: plan.substep_linear(psi, 0, 0.1)):
        with pytest.raises(gp.GPError) as ei:
            call()
        assert ei.value.status == L.GP_ERR_STATE
        assert "unusable" in lib.gp_last_error().decode()
    x = torch.from_numpy(I.random_field(16, seed=7)).to(DEV).contiguous()
    other.step_n(x, 3)
    assert math.isfinite(other.energies(x)["energy"])
    plan.close()
    other.close()


def test_single_grid_calls_reject_a_batch_plan():
    """A batch plan carries no tables of its own: every single-grid entry point
    returns GP_ERR_STATE for it without launching anything."""
    gp, L, lib = _lib()
    bp = gp.BatchPlan([dict(n=16, alpha=0.3, beta=2.0, dt=0.01), dict(n=24, alpha=0.3, beta=2.0, dt=0.01)], "c128")
    h = bp._h
    x = torch.zeros((16, 16, 16), dtype=torch.complex128, device=DEV)
    p = C.c_void_p(x.data_ptr())
    th = torch.zeros((16, 16, 16), dtype=torch.float64, device=DEV)
    work = torch.zeros(1 << 20, dtype=torch.uint8, device=DEV)
    w = C.c_void_p(work.data_ptr())
    e = L.gp_energy()
    J = C.c_double()
    spec = (C.c_double * 4096)()
    pairs = (C.c_double * 6)(0.5, 1.0, 1.0, 1.0, 1.0, 0)
    calls = {
        "gp_init_phase": lambda: lib.gp_init_phase(h, C.c_void_p(th.data_ptr()), p),
        "gp_init_rvr": lambda: lib.gp_init_rvr(h, pairs, 1, 0.2, p),
        "gp_substep_linear": lambda: lib.gp_substep_linear(h, p, 0, 0.01),
        "gp_substep_nonlinear": lambda: lib.gp_substep_nonlinear(h, p, 0.01),
        "gp_step_n": lambda: lib.gp_step_n(h, p, 1),
        "gp_step_literal_n": lambda: lib.gp_step_literal_n(h, p, 1),
        "gp_fft3": lambda: lib.gp_fft3(h, p, p, -1),
        "gp_energies": lambda: lib.gp_energies(h, p, w, C.byref(e)),
        "gp_spectra": lambda: lib.gp_spectra(h, p, w, spec, 8, C.byref(e)),
        "gp_structure_fn": lambda: lib.gp_structure_fn(h, p, w, 2, spec),
        "gp_loss_ekin_i_shells": lambda: lib.gp_loss_ekin_i_shells(h, p, w, 1, 3, C.byref(J), p),
        "gp_adjoint_step_n": lambda: lib.gp_adjoint_step_n(h, p, p, 1, w),
        "gp_phase_grad": lambda: lib.gp_phase_grad(h, p, p, C.c_void_p(th.data_ptr())),
    }
    for name, f in calls.items():
        assert f() == L.GP_ERR_STATE, name
        assert "batch plan" in lib.gp_last_error().decode(), name
    torch.cuda.synchronize()
    bp.close()
