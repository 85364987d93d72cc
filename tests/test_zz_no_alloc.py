"""The entry point that allocates nothing (gp_energies_static) against
gp_energies, through the C ABI: two calls in a row, the second on a smaller
grid, each equal to gp_energies on the same field; device allocations by the
library are made to fail during the calls (GP_FAULT_INJECT=alloc), so a call
that allocated would return GP_ERR_NOMEM; grids beyond the static workspace and
batch plans are rejected before any GPU work."""
import ctypes as C

import numpy as np
import pytest

import gp_inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
FIELDS = ("mass", "energy", "e_kin", "e_kin_i", "e_kin_c", "e_q", "e_int")


def test_static_workspace_energies_equal_gp_energies(monkeypatch):
    import paper_2003_03590_amd as gp
    from paper_2003_03590_amd import _lib as L
    lib = gp.lib()
    cases = [((96, 96, 96), "c128", 0.0694, 28.8), ((24, 16, 12), "c64", 0.3, 4.0)]   # the second is smaller
    for k, (shape, prec, alpha, beta) in enumerate(cases):
        plan = gp.Plan(shape, alpha, beta, 1e-3, prec)
        a = I.random_field((shape[2], shape[1], shape[0]), seed=40 + k)
        psi = torch.from_numpy(a).to(DEV).to(plan.dtype).contiguous()
        plan.step_n(psi, 3)
        ref = plan.energies(psi)                       # the existing entry point, caller workspace
        torch.cuda.synchronize()
        monkeypatch.setenv("GP_FAULT_INJECT", "alloc")
        e = L.gp_energy()
        st = lib.gp_energies_static(plan._h, C.c_void_p(psi.data_ptr()), C.byref(e))
        monkeypatch.delenv("GP_FAULT_INJECT")
        assert st == L.GP_OK, lib.gp_last_error().decode()
        got = e.as_dict()
        for f in FIELDS:
            # same kernels, same fixed-order reductions: equal values
            assert got[f] == ref[f], (shape, prec, f, got[f], ref[f])
        plan.close()


def test_static_workspace_rejects_large_grids_and_batch_plans():
    import paper_2003_03590_amd as gp
    from paper_2003_03590_amd import _lib as L
    lib = gp.lib()
    e = L.gp_energy()
    big = gp.Plan((128, 128, 128), 0.05, 40.0, 1e-3, "c128")     # 4 * 128^3 * 16 B > 64 MiB
    dummy = torch.zeros(8, dtype=torch.complex128, device=DEV)
    assert lib.gp_energies_static(big._h, C.c_void_p(dummy.data_ptr()), C.byref(e)) == L.GP_ERR_ARG
    assert "static workspace" in lib.gp_last_error().decode()
    assert lib.gp_energies_static(big._h, None, C.byref(e)) == L.GP_ERR_ARG
    big.close()
    bp = gp.BatchPlan([dict(n=16, alpha=0.3, beta=2.0, dt=0.01)], "c64")
    assert lib.gp_energies_static(bp._h, C.c_void_p(dummy.data_ptr()), C.byref(e)) == L.GP_ERR_STATE
    bp.close()
