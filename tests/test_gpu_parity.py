"""GPU parity: every entry point of the C ABI against the CPU oracle on the same
seeded inputs.  Tolerances: complex128 1e-12 relative (rounding of the FFT
order only), complex64 a few FP32 ulps times the transform depth."""
import math

import numpy as np
import pytest

import gp_inputs as I
from oracle import gp as O
from oracle import adjoint as OA

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def _plan(n, alpha, beta, dt, prec="c128"):
    import paper_2003_03590_amd as gp
    return gp.Plan(n, alpha, beta, dt, prec)


def _to_dev(a, prec):
    dt = torch.complex128 if prec == "c128" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dt).contiguous()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


TOL = {"c128": 1e-13, "c64": 2e-6}
SHAPES = [(8, 8, 8), (16, 12, 8), (6, 24, 4), (32, 32, 32), (48, 8, 12), (64, 4, 6), (96, 6, 8), (3, 4, 128),
          (2, 256, 1), (192, 2, 2), (384, 1, 2), (1, 2, 512), (768, 1, 1), (1, 1024, 1)]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_substep_linear_each_axis(shape, prec):
    nx, ny, nz = shape
    psi0 = I.random_field((nz, ny, nx), seed=sum(shape))
    plan = _plan(shape, 0.37, 1.3, 0.01, prec)
    for axis in range(3):
        s = 0.05 * (axis + 1)
        psi = _to_dev(psi0, prec)
        plan.substep_linear(psi, axis, s)
        got = psi.cpu().numpy()
        ref = O.linear_substep_axis(psi0, 0.37, s, 2 - axis)
        assert rel_max(got, ref) < TOL[prec] * max(1, math.log2(max(shape))), (axis, rel_max(got, ref))


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_init_phase_and_nonlinear(prec):
    theta = I.srp_fourier_theta((8, 12, 16), 3, 1) * 3.0
    plan = _plan((16, 12, 8), 0.5, 2.0, 0.01, prec)
    psi = plan.init_phase(torch.from_numpy(theta).to(DEV))
    ref = np.exp(1j * theta)
    assert rel_max(psi.cpu().numpy(), ref) < TOL[prec]
    f0 = I.random_field((8, 12, 16), seed=3, amp_noise=0.5)
    psi = _to_dev(f0, prec)
    plan.substep_nonlinear(psi, 0.37)
    ref = O.nonlinear_substep(f0, 2.0, 0.37)
    assert rel_max(psi.cpu().numpy(), ref) < TOL[prec] * 4


@pytest.mark.parametrize("shape,steps", [((8, 8, 8), 7), ((16, 12, 8), 5), ((24, 24, 24), 4), ((48, 32, 16), 3),
                                         ((64, 64, 64), 2), ((96, 48, 12), 2), ((128, 16, 8), 2)])
def test_step_n_matches_literal_oracle(shape, steps):
    nx, ny, nz = shape
    psi0 = I.random_field((nz, ny, nx), seed=11)
    plan = _plan(shape, 0.3, 4.0, 0.01)
    psi = _to_dev(psi0, "c128")
    plan.step_n(psi, steps)
    ref = O.evolve(psi0, 0.3, 4.0, 0.01, steps)
    assert rel_l2(psi.cpu().numpy(), ref) < 1e-12


PLANE_CASES = [((16, 16, 16), "c64"), ((32, 32, 8), "c64"), ((48, 48, 6), "c64"), ((64, 64, 64), "c64"),
               ((96, 96, 4), "c64"), ((16, 16, 3), "c128"), ((32, 32, 32), "c128"), ((48, 48, 12), "c128"),
               ((64, 64, 8), "c128"), ((64, 64, 1), "c128")]


@pytest.mark.parametrize("shape,prec", PLANE_CASES, ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else v)
def test_plane_pass_steps_match_oracle(shape, prec):
    """gp_step_n with the xy-plane pass (both in-plane sub-steps in one kernel, the
    nonlinear rotation fused in front) against the oracle's literal steps, forward
    and backward."""
    nx, ny, nz = shape
    psi0 = I.random_field((nz, ny, nx), seed=21)
    plan = _plan(shape, 0.3, 4.0, 0.01, prec)
    plan.select_variant(3, 1)
    assert plan.schedule(3).startswith("xy: plane")
    base = psi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi0
    psi = _to_dev(psi0, prec)
    plan.step_n(psi, 3)
    ref = O.evolve(base, 0.3, 4.0, 0.01, 3)
    tol = 1e-12 if prec == "c128" else 5e-6
    assert rel_l2(psi.cpu().numpy().astype(np.complex128), ref) < tol
    plan.step_n(psi, -2)
    ref = O.evolve(ref, 0.3, 4.0, 0.01, -2)
    assert rel_l2(psi.cpu().numpy().astype(np.complex128), ref) < 2 * tol
    plan.select_variant(3, 0)
    assert plan.schedule(3) == "xy: separate passes"


def test_plane_pass_unavailable_shape_is_an_error():
    import paper_2003_03590_amd as gp
    plan = _plan((24, 16, 8), 0.3, 4.0, 0.01, "c64")
    with pytest.raises(gp._lib.GPError):
        plan.select_variant(3, 1)


def test_batch_plane_pass_matches_oracle():
    """The ensemble graph with the xy-plane pass in every run, replayed."""
    import paper_2003_03590_amd as gp
    runs = [dict(n=32, alpha=0.4, beta=2.0, dt=0.01), dict(n=16, alpha=0.3, beta=3.0, dt=0.01),
            dict(n=32, alpha=0.5, beta=1.0, dt=0.02), dict(n=48, alpha=0.2, beta=3.0, dt=0.01)]
    bp = gp.BatchPlan(runs, "c128")
    bp.select_xy(1)
    refs = [I.random_field(r["n"], seed=90 + i) for i, r in enumerate(runs)]
    states = [_to_dev(a, "c128") for a in refs]
    for rep in range(2):
        bp.step_n(states, 3)
        for i, r in enumerate(runs):
            refs[i] = O.evolve(refs[i], r["alpha"], r["beta"], r["dt"], 3)
            assert rel_l2(states[i].cpu().numpy(), refs[i]) < 1e-12, (rep, i)


def test_step_n_negative_is_backward_and_reversible():
    psi0 = I.random_field(16, seed=12)
    plan = _plan(16, 0.6, 2.0, 0.02)
    psi = _to_dev(psi0, "c128")
    plan.step_n(psi, -4)
    ref = O.evolve(psi0, 0.6, 2.0, 0.02, -4)
    assert rel_l2(psi.cpu().numpy(), ref) < 1e-12
    plan.step_n(psi, 4)
    assert rel_l2(psi.cpu().numpy(), psi0) < 1e-12


def test_config_srp32_full_run():
    """32^3 complex128, alpha = beta = 1, dt = 1e-3, 200 steps, SRP |k| <= 4 seed 0,
    diagnostics every 20 steps: psi and every diagnostic against the oracle."""
    w = I.WORKLOADS["srp32"]
    theta = I.srp_fourier_theta(32, 4, 0)
    plan = _plan(32, w["alpha"], w["beta"], w["dt"])
    psi = plan.init_phase(torch.from_numpy(theta).to(DEV))
    ref = np.exp(1j * theta)
    for blk in range(w["steps"] // w["diag_every"]):
        plan.step_n(psi, w["diag_every"])
        ref = O.evolve(ref, w["alpha"], w["beta"], w["dt"], w["diag_every"])
        spec, e = plan.spectra(psi)
        d = O.diagnostics(ref, w["alpha"], w["beta"])
        for k in ("mass", "energy", "e_kin", "e_kin_i", "e_kin_c", "e_q", "e_int"):
            assert abs(e[k] - d[k]) <= 1e-11 * max(abs(d[k]), 1e-3), (blk, k, e[k], d[k])
        assert np.abs(spec - d["spec"]).max() <= 1e-11 * np.abs(d["spec"]).max()
    assert rel_l2(psi.cpu().numpy(), ref) < 1e-12


def test_config_srp32_fp32_run():
    """The same 32^3 run in complex64 (FP32 transforms and propagators, FP64 tables
    and reductions): psi after 200 steps within 1e-5 relative L2 of the FP64
    oracle, every diagnostic within 1e-5 of the oracle's, mass and energy drift
    stated."""
    w = I.WORKLOADS["srp32"]
    theta = I.srp_fourier_theta(32, 4, 0)
    plan = _plan(32, w["alpha"], w["beta"], w["dt"], "c64")
    psi = plan.init_phase(torch.from_numpy(theta).to(DEV))
    ref = np.exp(1j * theta)
    e0 = plan.energies(psi)
    drift_n = drift_e = 0.0
    for blk in range(w["steps"] // w["diag_every"]):
        plan.step_n(psi, w["diag_every"])
        ref = O.evolve(ref, w["alpha"], w["beta"], w["dt"], w["diag_every"])
        spec, e = plan.spectra(psi)
        d = O.diagnostics(ref, w["alpha"], w["beta"])
        for k in ("mass", "energy", "e_kin", "e_kin_i", "e_kin_c", "e_q", "e_int"):
            assert abs(e[k] - d[k]) <= 1e-5 * max(abs(d[k]), 1e-3), (blk, k, e[k], d[k])
        assert np.abs(spec - d["spec"]).max() <= 1e-5 * np.abs(d["spec"]).max()
        drift_n = max(drift_n, abs(e["mass"] - e0["mass"]) / e0["mass"])
        drift_e = max(drift_e, abs(e["energy"] - e0["energy"]) / e0["energy"])
    err = rel_l2(psi.cpu().numpy().astype(np.complex128), ref)
    print(f"srp32 complex64: rel-L2 {err:.2e}, drift N {drift_n:.2e}, drift E {drift_e:.2e}")
    assert err < 1e-5
    assert drift_n < 1e-6 and drift_e < 1e-5


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 24, 8), (64, 32, 16), (96, 8, 4)], ids=lambda s: "x".join(map(str, s)))
def test_diagnostics(shape, prec):
    nx, ny, nz = shape
    psi0 = I.random_field((nz, ny, nx), seed=5, amp_noise=0.2)
    alpha, beta = 0.4, 3.0
    plan = _plan(shape, alpha, beta, 0.01, prec)
    psi = _to_dev(psi0, prec)
    spec, e = plan.spectra(psi)
    d = O.diagnostics(psi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi0, alpha, beta)
    tol = 1e-11 if prec == "c128" else 2e-5
    for k in ("mass", "energy", "e_kin", "e_kin_i", "e_kin_c", "e_q", "e_int"):
        assert abs(e[k] - d[k]) <= tol * max(abs(d[k]), 1e-3), (k, e[k], d[k])
    assert np.abs(spec - d["spec"]).max() <= tol * np.abs(d["spec"]).max()
    # run twice: bitwise identical (deterministic reductions)
    spec2, e2 = plan.spectra(psi)
    assert np.array_equal(spec, spec2) and e == e2


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_fft3_and_literal_step(prec):
    shape = (16, 24, 12)
    psi0 = I.random_field((12, 24, 16), seed=9)
    plan = _plan(shape, 0.5, 2.0, 0.01, prec)
    x = _to_dev(psi0, prec)
    c = plan.fft3(x, -1)
    from oracle.fft import fft3
    ref = fft3(psi0)
    assert rel_max(c.cpu().numpy(), ref) < TOL[prec] * 8
    back = plan.fft3(c, +1)
    assert rel_max(back.cpu().numpy(), psi0) < TOL[prec] * 8
    psi = _to_dev(psi0, prec)
    plan.step_literal_n(psi, 3)
    ref = O.evolve(psi0, 0.5, 2.0, 0.01, 3)
    assert rel_l2(psi.cpu().numpy(), ref) < (1e-12 if prec == "c128" else 2e-6)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(16, 12, 1), (24, 1, 1), (1, 8, 12), (1, 1, 1), (6, 4, 32)],
                         ids=lambda s: "x".join(map(str, s)))
def test_literal_step_last_forward_pass_carries_the_multiplier(shape, prec):
    """The literal form applies exp(-i alpha |k|^2 dt/2) in whichever forward pass is
    last (z, or y or x when the later axes have length 1); forward and backward steps
    against the oracle."""
    nx, ny, nz = shape
    psi0 = I.random_field((nz, ny, nx), seed=17)
    plan = _plan(shape, 0.3, 3.0, 0.02, prec)
    psi = _to_dev(psi0, prec)
    plan.step_literal_n(psi, 4)
    ref = O.evolve(psi0, 0.3, 3.0, 0.02, 4)
    tol = 1e-12 if prec == "c128" else 2e-6
    assert rel_l2(psi.cpu().numpy(), ref) < tol
    plan.step_literal_n(psi, -4)
    assert rel_l2(psi.cpu().numpy(), psi0) < 2 * tol
    plan.close()


def test_structure_function():
    psi0 = I.random_field(16, seed=21)
    plan = _plan(16, 0.5, 1.0, 0.01)
    s = plan.structure_fn(_to_dev(psi0, "c128"))
    ref = O.structure_function_density(psi0, 2)
    assert np.abs(s - ref).max() < 1e-12 * np.abs(ref).max()


def test_loss_gradient_matches_oracle():
    psi0 = I.random_field(12, seed=31, amp_noise=0.2)
    alpha = 0.3
    plan = _plan(12, alpha, 2.0, 0.01)
    J, lam = plan.loss_ekin_i_shells(_to_dev(psi0, "c128"), 1, 3)
    Jr, lamr = OA.loss_gradient(psi0, alpha, 1, 3)
    assert abs(J - Jr) < 1e-12 * Jr
    assert rel_max(lam.cpu().numpy(), lamr) < 1e-11


def test_adjoint_steps_match_oracle():
    psi0 = I.random_field((8, 12, 16), seed=41)
    lam0 = I.random_field((8, 12, 16), seed=42)
    alpha, beta, dt, n = 0.3, 2.0, 0.01, 5
    plan = _plan((16, 12, 8), alpha, beta, dt)
    lam = _to_dev(lam0, "c128")
    plan.adjoint_step_n(_to_dev(psi0, "c128"), lam, n)
    states = OA.forward_states(psi0, alpha, beta, dt, n)
    ref = lam0
    for k in range(n - 1, -1, -1):
        ref = OA.step_adjoint(states[k], ref, alpha, beta, dt)
    assert rel_l2(lam.cpu().numpy(), ref) < 1e-12


def test_autograd_gradient_matches_oracle_and_fd():
    import paper_2003_03590_amd as gp
    n, alpha, beta, dt, steps, smin, smax = 12, 0.3, 2.0, 0.01, 10, 1, 3
    theta = I.srp_fourier_theta(n, 2, 7)
    plan = _plan(n, alpha, beta, dt)
    th = torch.from_numpy(theta).to(DEV).requires_grad_(True)
    psi = gp.evolve(th, plan, steps, ckpt=4)
    J = gp.ekin_i_shells(psi, plan, smin, smax)
    J.backward()
    g = th.grad.cpu().numpy()
    Jr, gr, _ = OA.gradient_theta(theta, alpha, beta, dt, steps, smin, smax)
    assert abs(J.item() - Jr) < 1e-12 * Jr
    assert np.abs(g - gr).max() < 1e-10 * np.abs(gr).max()
    # central finite differences along random band-limited directions
    for s in range(3):
        d = I.srp_fourier_theta(n, 2, 1000 + s)
        h = 1e-6
        Jp = OA.loss_ekin_i_shells(O.evolve(np.exp(1j * (theta + h * d)), alpha, beta, dt, steps), alpha, smin, smax)
        Jm = OA.loss_ekin_i_shells(O.evolve(np.exp(1j * (theta - h * d)), alpha, beta, dt, steps), alpha, smin, smax)
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - float(np.sum(g * d))) < 1e-6 * abs(fd)


def test_batch_matches_single_runs():
    import paper_2003_03590_amd as gp
    runs = [dict(n=16, alpha=0.4, beta=2.0, dt=0.01), dict(n=12, alpha=0.3, beta=3.0, dt=0.01),
            dict(n=16, alpha=0.5, beta=1.0, dt=0.02)]
    bp = gp.BatchPlan(runs, "c128")
    init = [I.random_field(r["n"], seed=50 + i) for i, r in enumerate(runs)]
    states = [_to_dev(a, "c128") for a in init]
    bp.step_n(states, 3)
    bp.step_n(states, 3)          # graph replay
    e = bp.energies(states)
    for i, r in enumerate(runs):
        ref = O.evolve(init[i], r["alpha"], r["beta"], r["dt"], 6)
        assert rel_l2(states[i].cpu().numpy(), ref) < 1e-12
        assert abs(e[i, 0] - O.mass(ref)) < 1e-12
        assert abs(e[i, 1] - O.energy(ref, r["alpha"], r["beta"])) < 1e-10 * abs(e[i, 1])


def test_batch_graph_replays_with_eager_work_between():
    """The ensemble step is recorded once as a HIP graph and replayed; four
    replays with other GPU work (another plan's steps, the batch diagnostics,
    torch kernels) and synchronizations between them, every replay checked
    against the oracle advanced by the same number of steps."""
    import paper_2003_03590_amd as gp
    runs = [dict(n=16, alpha=0.4, beta=2.0, dt=0.01), dict(n=24, alpha=0.3, beta=3.0, dt=0.01),
            dict(n=16, alpha=0.5, beta=1.0, dt=0.02)]
    bp = gp.BatchPlan(runs, "c128")
    refs = [I.random_field(r["n"], seed=70 + i) for i, r in enumerate(runs)]
    states = [_to_dev(a, "c128") for a in refs]
    other = _plan(12, 0.3, 2.0, 0.01)
    x = _to_dev(I.random_field(12, seed=80), "c128")
    for rep in range(4):
        bp.step_n(states, 2)              # first call records the graph, later calls replay it
        other.step_n(x, 1)
        e = bp.energies(states)
        y = (x * 2.0).abs().sum()
        torch.cuda.synchronize()
        assert math.isfinite(float(y))
        for i, r in enumerate(runs):
            refs[i] = O.evolve(refs[i], r["alpha"], r["beta"], r["dt"], 2)
            assert rel_l2(states[i].cpu().numpy(), refs[i]) < 1e-12, (rep, i)
            assert abs(e[i, 0] - O.mass(refs[i])) < 1e-12


def test_errors_are_reported():
    import paper_2003_03590_amd as gp
    plan = _plan(8, 1.0, 1.0, 0.01)
    with pytest.raises(gp.GPError):
        plan.structure_fn(_to_dev(I.random_field(8, 1), "c128"), p_order=3)
    with pytest.raises(ValueError):
        plan.step_n(torch.zeros((8, 8, 4), dtype=torch.complex128, device=DEV), 1)
    with pytest.raises(gp.GPError):
        gp.Plan(10, 1.0, 1.0, 0.01)


def _variants(n, prec):
    import paper_2003_03590_amd as gp
    return int(gp.lib().gp_variant_count(n, 0 if prec == "c128" else 1))


VARIANT_CASES = [(n, p) for n in (64, 96, 128, 256, 512, 1024) for p in ("c128", "c64")]


@pytest.mark.parametrize("n,prec", VARIANT_CASES, ids=lambda v: str(v))
def test_every_schedule_variant(n, prec):
    """Each compiled schedule of a length is its own kernel: sub-steps on each
    axis, a forward/inverse 3-D transform and the diagnostics, per variant."""
    from oracle.fft import fft3
    nv = _variants(n, prec)
    assert nv >= 1
    tol = TOL[prec] * max(1, math.log2(n))
    for v in range(nv):
        for axis in range(3):
            shape = [6, 4, 2]
            shape[axis] = n
            nx, ny, nz = shape
            psi0 = I.random_field((nz, ny, nx), seed=n + v + axis)
            plan = _plan(tuple(shape), 0.21, 1.7, 0.01, prec)
            try:
                plan.select_variant(axis, v)
            except Exception:
                plan.close()
                continue           # this variant exists for another precision only
            psi = _to_dev(psi0, prec)
            plan.substep_linear(psi, axis, 0.03)
            ref = O.linear_substep_axis(psi0, 0.21, 0.03, 2 - axis)
            assert rel_max(psi.cpu().numpy(), ref) < tol, (v, axis)
            c = plan.fft3(_to_dev(psi0, prec), -1)
            assert rel_max(c.cpu().numpy(), fft3(psi0)) < tol * 4, (v, axis)
            e = plan.energies(_to_dev(psi0, prec))
            base = psi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi0
            d = O.diagnostics(base, 0.21, 1.7)
            for k in ("mass", "energy", "e_kin", "e_kin_i", "e_q"):
                assert abs(e[k] - d[k]) <= (1e-10 if prec == "c128" else 3e-5) * max(abs(d[k]), 1e-3), (v, axis, k)
            plan.close()


def test_autotune_and_cache(tmp_path):
    import json
    import paper_2003_03590_amd as gp
    cache = str(tmp_path / "tune.json")
    plan = _plan(64, 0.3, 4.0, 0.01, "c64")
    chosen = plan.autotune(reps=2, cache=cache)
    data = json.load(open(cache))
    # three axis schedules, the xy choice (plane pass or separate passes, single run)
    # and, with separate passes, the axis that carries the nonlinear rotation
    assert all(k.split("/")[1] == "c64" for k in data)
    assert any(k.endswith("/a3/r1") for k in data) and len(chosen) == 6
    # with separate passes also the nonlinear carrier and the layout form (64^3 has
    # a rotating schedule)
    assert len(data) == (6 if chosen[3].startswith("xy: separate") else 4)
    plan2 = _plan(64, 0.3, 4.0, 0.01, "c64")
    assert plan2.autotune(reps=2, cache=cache) == chosen
    psi0 = I.random_field(64, seed=77)
    psi = _to_dev(psi0, "c64")
    plan2.step_n(psi, 2)
    ref = O.evolve(psi0.astype(np.complex64).astype(np.complex128), 0.3, 4.0, 0.01, 2)
    assert rel_l2(psi.cpu().numpy(), ref) < 2e-6
    # a batch plan re-records its graph after tuning
    bp = gp.BatchPlan([dict(n=64, alpha=0.3, beta=4.0, dt=0.01), dict(n=96, alpha=0.2, beta=5.0, dt=0.01)], "c64")
    sts = [_to_dev(I.random_field(64, seed=1), "c64"), _to_dev(I.random_field(96, seed=2), "c64")]
    bp.step_n(sts, 1)
    bp.autotune(reps=2, cache=cache)
    bp.step_n(sts, 1)
    assert len(json.load(open(cache))) >= 8


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_nonlinear_carrier_axis(prec):
    """The nonlinear rotation may ride on any axis pass (the linear sub-steps commute):
    every choice gives the oracle's split step; bad choices are rejected."""
    import paper_2003_03590_amd as gp
    shape = (24, 16, 12)
    psi0 = I.random_field((12, 16, 24), seed=61)
    base = psi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi0
    ref = O.evolve(base, 0.3, 4.0, 0.01, 5)
    plan = gp.Plan(shape, 0.3, 4.0, 0.01, prec)
    for carrier in (0, 1, 2):
        plan.select_variant(4, carrier)
        assert plan.schedule(4) == "nl: " + "xyz"[carrier] + " pass"
        psi = _to_dev(psi0, prec)
        plan.step_n(psi, 5)
        assert rel_l2(psi.cpu().numpy(), ref) < (1e-12 if prec == "c128" else 2e-6)
        plan.step_n(psi, -5)
        assert rel_l2(psi.cpu().numpy(), base) < (1e-12 if prec == "c128" else 4e-6)
    with pytest.raises(gp._lib.GPError):
        plan.select_variant(4, 3)
    plan.close()
    flat = gp.Plan((16, 16, 1), 0.3, 4.0, 0.01, prec)
    with pytest.raises(gp._lib.GPError):
        flat.select_variant(4, 2)            # axis of length 1
    flat.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(3, 3, 3), (16, 16, 16), (64, 32, 8)], ids=lambda s: "x".join(map(str, s)))
def test_copy_state_is_exact(shape, prec):
    """gp_copy_state (the bandwidth reference): a bit-exact copy, including the odd
    8-byte tail of a complex64 state with an odd point count."""
    plan = _plan(shape, 0.05, 40.0, 1e-3, prec)
    rng = np.random.default_rng(3)
    fshape = shape[::-1]                  # [z][y][x]
    x = _to_dev(rng.standard_normal(fshape) + 1j * rng.standard_normal(fshape), prec)
    y = plan.copy_state(x)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(y), torch.view_as_real(x))
    plan.close()
