"""Layout-rotating linear steps (gp_select_variant axis 5): every linear step as
x, z, y passes that each read whole contiguous pencils and write the state in a
turned layout, out of place between psi and one plan-owned state, or (mixed) as
two such passes and one in-place pass along the axis they leave innermost.  Against the
oracle on small cubes of both precisions (odd and even step counts, so both
buffer parities, and backward steps), against the fixed-layout form at 512^3 and 1024^3,
and the rejected shapes."""
import numpy as np
import pytest

import gp_inputs as I
from oracle import gp as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("mixed", [False, True], ids=["rotating", "mixed"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n", [16, 32, 48, 64])
def test_rotating_steps_match_oracle(n, prec, mixed):
    """Both rotating forms: every linear step as three rotating passes, or (mixed)
    as two rotating passes and one in-place pass, the layout advancing one place per
    step; step counts whose n + 1 leaves every remainder mod 2 and mod 3."""
    import paper_2003_03590_amd as gp
    alpha, beta, dt = 0.3, 4.0, 0.01
    plan = gp.Plan(n, alpha, beta, dt, prec)
    nrot = 1                                    # one rotating schedule per length
    plan.select_variant(5, 1 + nrot if mixed else 1)
    assert plan.schedule(5).startswith("layout: rotating+contiguous" if mixed else "layout: rotating N")
    psi0 = I.random_field(n, seed=600 + n)
    base = psi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi0
    tol = 1e-12 if prec == "c128" else 2e-6
    for nsteps in (1, 2, 3, 4, 5, -2):
        psi = torch.from_numpy(base).to(DEV).to(plan.dtype).contiguous()
        plan.step_n(psi, nsteps)
        ref = O.evolve(base, alpha, beta, dt, nsteps)
        rel = _rel(psi.to(torch.complex128).cpu().numpy(), ref)
        assert rel < tol, (n, prec, nsteps, rel)
    plan.select_variant(5, 0)                   # back to the fixed layout (workspace released)
    assert plan.schedule(5) == "layout: fixed"
    psi = torch.from_numpy(base).to(DEV).to(plan.dtype).contiguous()
    plan.step_n(psi, 2)
    assert _rel(psi.to(torch.complex128).cpu().numpy(), O.evolve(base, alpha, beta, dt, 2)) < tol
    plan.close()


def test_rotating_form_rejects_other_shapes():
    import paper_2003_03590_amd as gp
    from paper_2003_03590_amd import _lib as L
    for shape in ((32, 32, 16), (24, 24, 24)):          # not a cube; no rotating schedule
        plan = gp.Plan(shape, 0.3, 4.0, 0.01, "c128")
        with pytest.raises(gp.GPError) as ei:
            plan.select_variant(5, 1)
        assert ei.value.status == L.GP_ERR_UNSUPPORTED
        with pytest.raises(gp.GPError):
            plan.select_variant(5, 2)
        plan.close()


def test_rotating_1024_matches_fixed_layout():
    """1024^3 complex64 (the random-vortex-ring workload's parameters, white-noise
    field): two and three rotating steps against the fixed-layout passes (each
    parity-tested against the oracle), within FP32 rounding of the different
    operation order; mass conserved."""
    import paper_2003_03590_amd as gp
    w = I.WORKLOADS["rvr1024"]
    n = w["n"]
    g = torch.Generator(device=DEV).manual_seed(11)
    start = torch.randn((n, n, n), dtype=torch.complex64, device=DEV, generator=g)
    start += 1.0
    fixed = gp.Plan(n, w["alpha"], w["beta"], w["dt"], "c64")
    rot = gp.Plan(n, w["alpha"], w["beta"], w["dt"], "c64")
    m0 = float(torch.sum(torch.abs(start.to(torch.complex128)) ** 2))
    for variant in (1, 2):                      # rotating, mixed
        rot.select_variant(5, variant)
        for nsteps in (2, 3):
            a, b = start.clone(), start.clone()
            fixed.step_n(a, nsteps)
            rot.step_n(b, nsteps)
            rel = float(torch.linalg.vector_norm((a - b).to(torch.complex128)) /
                        torch.linalg.vector_norm(a.to(torch.complex128)))
            m1 = float(torch.sum(torch.abs(b.to(torch.complex128)) ** 2))
            print(f"1024^3 {rot.schedule(5)} vs fixed, {nsteps} steps: rel-L2 {rel:.2e}, "
                  f"mass change {abs(m1 - m0) / m0:.2e}")
            assert rel < 2e-6 and abs(m1 - m0) / m0 < 1e-6
            del a, b
    fixed.close()
    rot.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_rotating_512_matches_fixed_layout(prec):
    """512^3 (the rotating schedules 8x8x8 complex128 and 32x16 complex64, with the
    XOR-swizzled LDS regroup): two and three rotating and mixed steps against the
    fixed-layout passes, within rounding of the different operation order; mass
    conserved."""
    import paper_2003_03590_amd as gp
    w = I.WORKLOADS["rvr1024"]
    n = 512
    dt = torch.complex128 if prec == "c128" else torch.complex64
    tol = 1e-12 if prec == "c128" else 2e-6
    g = torch.Generator(device=DEV).manual_seed(12)
    start = torch.randn((n, n, n), dtype=dt, device=DEV, generator=g)
    start += 1.0
    fixed = gp.Plan(n, w["alpha"], w["beta"], w["dt"], prec)
    rot = gp.Plan(n, w["alpha"], w["beta"], w["dt"], prec)
    m0 = float(torch.sum(torch.abs(start.to(torch.complex128)) ** 2))
    for variant in (1, 2):                      # rotating, mixed
        rot.select_variant(5, variant)
        for nsteps in (2, 3):
            a, b = start.clone(), start.clone()
            fixed.step_n(a, nsteps)
            rot.step_n(b, nsteps)
            rel = float(torch.linalg.vector_norm((a - b).to(torch.complex128)) /
                        torch.linalg.vector_norm(a.to(torch.complex128)))
            m1 = float(torch.sum(torch.abs(b.to(torch.complex128)) ** 2))
            print(f"512^3 {prec} {rot.schedule(5)} vs fixed, {nsteps} steps: rel-L2 {rel:.2e}, "
                  f"mass change {abs(m1 - m0) / m0:.2e}")
            assert rel < tol and abs(m1 - m0) / m0 < tol
            del a, b
    fixed.close()
    rot.close()
