"""Velocity statistics on the GPU against the oracle: longitudinal velocity
structure functions per axis (eq. strfunc-def), Mach numbers (eq. Mach-Number),
helicity and regularized helicity with their spectra (eq. helicity, eq. Hreg)."""
import math

import numpy as np
import pytest

import gp_inputs as I
from oracle import gp as O
from oracle import helicity as OH

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _plan(n, alpha, beta, prec):
    import paper_2003_03590_amd as gp
    return gp.Plan(n, alpha, beta, 1e-3, prec)


def _dev(a, prec):
    dt = torch.complex128 if prec == "c128" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dt).contiguous()


def _fields():
    x = 2 * np.pi * np.arange(16) / 16
    return {
        "random16": I.random_field(16, seed=41),
        "random24": I.random_field(24, seed=42),
        "tg32": I.tg_psi(32, 0.05, 1),                    # vortex lines (zeros of psi near the grid)
        "mode16": np.exp(0.5j * np.cos(x))[None, None, :] * np.ones((16, 16, 16)),
    }


@pytest.mark.parametrize("name", ["random16", "random24", "tg32", "mode16"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_velocity_structure_function_matches_oracle(name, prec):
    psi = _fields()[name]
    n, alpha, beta = psi.shape[0], 0.3, 2.0
    base = psi.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi
    s_ref, mv2_ref = O.structure_function_velocity(base, alpha)
    plan = _plan(n, alpha, beta, prec)
    s, mv2 = plan.structure_fn_velocity(_dev(psi, prec))
    scale = max(float(mv2_ref.max()), 1e-30)
    # complex128: FFT power sums vs direct lag sums, round-off only.  complex64: v is
    # formed from FP32 derivatives; near a vortex core v ~ 1/r amplifies their error
    tol = 1e-11 if prec == "c128" else (2e-3 if name == "tg32" else 2e-5)
    assert np.abs(s - s_ref).max() < tol * scale, (np.abs(s - s_ref).max(), scale)
    assert np.abs(mv2 - mv2_ref).max() < tol * scale
    plan.close()


@pytest.mark.parametrize("name", ["random16", "random24", "tg32"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_mach_numbers_match_oracle(name, prec):
    psi = _fields()[name]
    n, alpha, beta = psi.shape[0], 0.3, 2.0
    base = psi.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi
    mmax_ref, mrms_ref = O.mach_numbers(base, alpha, beta)
    plan = _plan(n, alpha, beta, prec)
    p = _dev(psi, prec)
    mmax, mrms = plan.mach(p)
    tol = 1e-12 if prec == "c128" else 2e-5
    assert abs(mmax - mmax_ref) < tol * mmax_ref and abs(mrms - mrms_ref) < tol * mrms_ref
    e = plan.energies(p)       # M_rms = sqrt(2 E_kin) / c on the same evaluation
    assert abs(mrms - math.sqrt(2 * e["e_kin"] / (2 * alpha * beta))) < 1e-9 * mrms
    plan.close()


def test_velocity_statistics_at_128_against_oracle():
    """A 128^3 Taylor-Green ansatz (several tiles per axis) in complex128: every lag of
    the three structure functions and both Mach numbers against the oracle."""
    n, alpha, beta = 128, 0.05, 40.0
    psi = I.tg_psi(n, math.sqrt(alpha / beta), 3)
    s_ref, mv2_ref = O.structure_function_velocity(psi, alpha)
    plan = _plan(n, alpha, beta, "c128")
    p = _dev(psi, "c128")
    s, mv2 = plan.structure_fn_velocity(p)
    assert np.abs(s - s_ref).max() < 1e-11 * mv2_ref.max()
    mm = plan.mach(p)
    ref = O.mach_numbers(psi, alpha, beta)
    assert abs(mm[0] - ref[0]) < 1e-12 * ref[0] and abs(mm[1] - ref[1]) < 1e-12 * ref[1]
    plan.close()


def test_velocity_statistics_errors():
    import paper_2003_03590_amd as gp
    plan = gp.Plan((16, 16, 8), 0.3, 2.0, 1e-3, "c128")
    p = _dev(I.random_field((8, 16, 16), seed=1), "c128")
    with pytest.raises(gp._lib.GPError):
        plan.structure_fn_velocity(p)            # not cubic
    plan.close()
    plan = _plan(16, 0.3, 2.0, "c128")
    with pytest.raises(gp._lib.GPError):
        plan.structure_fn_velocity(_dev(I.random_field(16, seed=1), "c128"), p_order=3)
    plan.close()


def _hel_fields():
    n = 16
    x = 2 * np.pi * (np.arange(n) + 0.5) / n          # cores between grid points
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    return {
        "random12": I.random_field(12, seed=43),
        "ragged": I.random_field((8, 12, 16), seed=44),     # (nz, ny, nx)
        "tg32": I.tg_psi(32, 0.05, 1),
        "lines16": (np.sin(X) + 1j * np.sin(Y)) * np.exp(2j * Z) * np.ones((n, n, n)),
    }


def _hel_scale(psi, alpha):
    """mean |v| |omega|: the size of the terms whose mean is H."""
    v = O.velocity(psi, alpha)
    om = OH.curl(v)
    return float(np.mean(np.sqrt(sum(c * c for c in v)) * np.sqrt(sum(c * c for c in om))))


@pytest.mark.parametrize("name", ["random12", "ragged", "tg32", "lines16"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_helicity_matches_oracle(name, prec):
    import paper_2003_03590_amd as gp
    psi = _hel_fields()[name]
    nz, ny, nx = psi.shape
    alpha, beta = 0.3, 2.0
    base = psi.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi
    ref = OH.helicity(base, alpha)
    scale = _hel_scale(base, alpha)
    plan = gp.Plan((nx, ny, nz), alpha, beta, 1e-3, prec)
    H, Hreg, spec = plan.helicity(_dev(psi, prec))
    # complex64: v and v_reg divide by |psi|^2 and |grad psi|^2, which amplifies the
    # FP32 rounding of the derivatives near cores and stagnation points
    tol = 1e-10 if prec == "c128" else 1e-3
    print(name, prec, "H", H, ref["H"], "H_reg", Hreg, ref["H_reg"], "scale", scale)
    assert abs(H - ref["H"]) < tol * scale and abs(Hreg - ref["H_reg"]) < tol * scale
    assert np.abs(spec - ref["spec"]).max() < tol * scale
    pt = 1e-9 if prec == "c128" else 1e-6        # spectra from FP32 transforms for complex64
    assert abs(spec[0].sum() - H) < pt * scale and abs(spec[1].sum() - Hreg) < pt * scale
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_helicity_of_a_planar_flow_vanishes(prec):
    """On a 2-D grid (nz = 1) v lies in the plane and omega = curl v is normal to it,
    so H = H_reg = 0 (the oracle to round-off).  complex128 likewise; complex64
    carries two real velocity components per transform, and FP32 rounding leaks
    ~1e-7 of one into the other, so it is zero to ~1e-6 of <|v||omega|>."""
    import paper_2003_03590_amd as gp
    psi = I.random_field((1, 16, 24), seed=45)
    ref = OH.helicity(psi, 0.3)
    scale = _hel_scale(psi, 0.3)
    plan = gp.Plan((24, 16, 1), 0.3, 2.0, 1e-3, prec)
    H, Hreg, spec = plan.helicity(_dev(psi, prec))
    assert abs(ref["H"]) < 1e-14 * scale and abs(ref["H_reg"]) < 1e-14 * scale
    tol = (1e-13 if prec == "c128" else 1e-6) * scale
    assert abs(H) < tol and abs(Hreg) < tol and np.abs(spec).max() < tol
    plan.close()
