"""1024^3 complex64 workload (random vortex rings, spectra and structure functions)
and the full-size launch configurations: sampled outputs the oracle computes one
pencil at a time, invariants that hold at any size, and the initial-condition
generator against the host generator."""
import math

import numpy as np
import pytest

import gp_inputs as I
from oracle import gp as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _plan(n, alpha, beta, dt, prec):
    import paper_2003_03590_amd as gp
    return gp.Plan(n, alpha, beta, dt, prec)


def _pairs(n_pairs, seed):
    return [(p["R"], p["d"], p["X"], p["Y"], p["Z"], p["perm"]) for p in I.rvr_draws(n_pairs, seed)]


@pytest.mark.parametrize("n,npairs", [(24, 2), (32, 4)])
def test_rvr_generator_matches_host_generator(n, npairs):
    xi = 0.2
    plan = _plan(n, 0.1, 10.0, 1e-3, "c128")
    psi = plan.init_rvr(_pairs(npairs, 1), xi)
    ref = I.rvr_psi(n, xi, npairs, seed=1)
    assert np.abs(psi.cpu().numpy() - ref).max() < 1e-12


def _random_c64(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n, 2 * n), dtype=np.float32)
    return a.view(np.complex64)


@pytest.fixture(scope="module")
def field1024():
    n = 1024
    host = _random_c64(n, 5)
    dev = torch.from_numpy(host).to(DEV)
    return host, dev


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_1024_axis_pass_sampled_pencils(field1024, axis):
    """S(s, L_axis) at 1024^3 complex64 in the schedule the workload runs: eight
    pencils compared with the oracle's 1-D sub-step of the same input pencil."""
    host, dev = field1024
    w = I.WORKLOADS["rvr1024"]
    n = w["n"]
    plan = _plan(n, w["alpha"], w["beta"], w["dt"], "c64")
    plan.autotune(reps=2)
    psi = dev.clone()
    s = 0.5 * w["dt"]
    plan.substep_linear(psi, axis, s)
    rng = np.random.default_rng(axis)
    for _ in range(8):
        i, j = (int(v) for v in rng.integers(0, n, 2))
        if axis == 0:
            pin, pout = host[i, j, :], psi[i, j, :]
        elif axis == 1:
            pin, pout = host[i, :, j], psi[i, :, j]
        else:
            pin, pout = host[:, i, j], psi[:, i, j]
        ref = O.linear_substep_axis(pin.astype(np.complex128).reshape(1, 1, n), w["alpha"], s, 2)[0, 0]
        got = pout.cpu().numpy().astype(np.complex128)
        assert np.abs(got - ref).max() < 2e-6 * math.log2(n) * np.abs(ref).max()
    plan.close()


def test_1024_step_invariants(field1024):
    """Mass is conserved and n steps forward then n back return the start (FP32)."""
    _, dev = field1024
    w = I.WORKLOADS["rvr1024"]
    plan = _plan(w["n"], w["alpha"], w["beta"], w["dt"], "c64")
    psi = dev.clone()
    m0 = float(torch.sum(torch.abs(psi.to(torch.complex128)) ** 2))
    plan.step_n(psi, 3)
    m1 = float(torch.sum(torch.abs(psi.to(torch.complex128)) ** 2))
    assert abs(m1 - m0) / m0 < 1e-6
    plan.step_n(psi, -3)
    rel = float(torch.linalg.vector_norm((psi - dev).to(torch.complex128)) / torch.linalg.vector_norm(dev.to(torch.complex128)))
    assert rel < 1e-5
    plan.close()


def test_rvr1024_workload_segment():
    """1024^3 complex64, 40 random vortex-ring pairs (R in [0.3, 0.8], d = 2R, seed 1,
    xi = 3 (2 pi / 1024)), dt = 2.5e-4: 50 steps, then spectra and the density
    structure function; the spectra sum to the energies and mass is conserved."""
    w = I.WORKLOADS["rvr1024"]
    n = w["n"]
    plan = _plan(n, w["alpha"], w["beta"], w["dt"], "c64")
    psi = plan.init_rvr(_pairs(w["ic"][1]["n_pairs"], w["ic"][1]["seed"]), w["ic"][1]["xi"])
    amp = torch.abs(psi)
    assert float(amp.max()) <= 1.0 + 1e-5 and float(amp.min()) < 0.2
    e0 = plan.energies(psi)
    plan.step_n(psi, w["diag_every"])
    spec, e1 = plan.spectra(psi)
    sf = plan.structure_fn(psi)
    assert abs(e1["mass"] - e0["mass"]) / e0["mass"] < 1e-5
    assert abs(spec[0].sum() - e1["e_kin_i"]) < 1e-9 * e1["e_kin"]
    assert abs(spec[0].sum() + spec[1].sum() - e1["e_kin"]) < 1e-4 * e1["e_kin"]
    assert abs(spec[3].sum() - e1["e_int"]) < 1e-4 * e1["e_int"]
    assert np.all(np.isfinite(sf)) and np.all(sf >= 0) and sf[-1] > sf[0]
    print(f"rvr1024: E0 {e0['energy']:.8f} E1 {e1['energy']:.8f} dE {abs(e1['energy'] - e0['energy']) / e0['energy']:.2e}")
    plan.close()


@pytest.fixture(scope="module")
def tg256():
    """256^3 Taylor-Green state and one literal Strang step of the oracle from it."""
    w = I.WORKLOADS["tg256"]
    psi0 = I.tg_psi(w["n"], w["ic"][1]["xi"], w["ic"][1]["exponent"])
    return w, psi0, O.evolve(psi0, w["alpha"], w["beta"], w["dt"], 1)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_tg256_in_measured_configuration(tg256, prec):
    """256^3 Taylor-Green workload (alpha = 0.06942, beta = 28.81, dt = 5e-4) with
    the autotuned schedules of the throughput measurement: one Strang step over
    the whole field against the oracle's literal step, sampled pencils of each
    axis sub-step, and the spectra summing to the energies."""
    w, psi0, ref1 = tg256
    n = w["n"]
    plan = _plan(n, w["alpha"], w["beta"], w["dt"], prec)
    plan.autotune(reps=5)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    start = psi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi0
    dev0 = torch.from_numpy(start).to(DEV).to(dt).contiguous()
    psi = dev0.clone()
    plan.step_n(psi, 1)
    got = psi.cpu().numpy().astype(np.complex128)
    rel = float(np.linalg.norm(got - ref1) / np.linalg.norm(ref1))
    print(f"tg256 {prec} [{'; '.join(plan.schedule(a) for a in range(3))}]: one step rel-L2 {rel:.2e}")
    assert rel < (1e-12 if prec == "c128" else 2e-6)
    s = 0.5 * w["dt"]
    tol = 1e-13 if prec == "c128" else 2e-6 * math.log2(n)
    rng = np.random.default_rng(3)
    for axis in range(3):
        q = dev0.clone()
        plan.substep_linear(q, axis, s)
        for _ in range(6):
            i, j = (int(v) for v in rng.integers(0, n, 2))
            sl = [(i, j, slice(None)), (i, slice(None), j), (slice(None), i, j)][axis]
            ref = O.linear_substep_axis(start[sl].reshape(1, 1, n), w["alpha"], s, 2)[0, 0]
            assert np.abs(q[sl].cpu().numpy().astype(np.complex128) - ref).max() < tol * np.abs(ref).max()
    spec, e = plan.spectra(psi)
    rt = 1e-9 if prec == "c128" else 1e-6        # FP32 spectral fields for complex64
    assert abs(spec[0].sum() - e["e_kin_i"]) < rt * e["e_kin"]
    assert abs(spec[0].sum() + spec[1].sum() - e["e_kin"]) < rt * e["e_kin"]
    assert abs(spec[2].sum() - e["e_q"]) < rt * e["e_q"]
    assert abs(spec[3].sum() - e["e_int"]) < rt * e["e_int"]
    # E_kin + E_q = 2 alpha^2 sum |k~|^2 |c_k|^2 pointwise, so E_kin + E_q + E_int
    # differs from E only through the Nyquist entries of |k|^2 (negligible here)
    assert abs(e["e_kin"] + e["e_q"] + e["e_int"] - e["energy"]) < (1e-6 if prec == "c128" else 3e-6) * e["energy"]
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("field", ["tg", "random"])
def test_structure_fn_128_against_direct_lag_sums(prec, field):
    """gp_structure_fn at 128^3 (the density structure function of eq. strfunc-def,
    lags 1..64, mean over the three axes) against the oracle's direct lag sums of
    the same (precision-rounded) field.  Complex128 to 1e-12 of max S; complex64
    computes rho - 1 and its transform in FP32, an error of about (2 log2 N) u
    relative to the variance C(0) of rho (S runs up to about 2 C(0)), so 1e-5 of
    max S holds with margin."""
    n = 128
    psi0 = I.tg_psi(n, 2.0 * (2 * math.pi / n), 2) if field == "tg" else I.random_field(n, seed=8, amp_noise=0.2)
    start = psi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi0
    plan = _plan(n, 0.05, 40.0, 1e-3, prec)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    s = plan.structure_fn(torch.from_numpy(start).to(DEV).to(dt).contiguous())
    ref = O.structure_function_density(start, 2)
    err = np.abs(s - ref).max() / np.abs(ref).max()
    print(f"structure function 128^3 {field} {prec}: max error / max S = {err:.2e}")
    assert err < (1e-12 if prec == "c128" else 1e-5)
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_tg256_rotating_step_against_oracle(tg256, prec):
    """The 256^3 Taylor-Green workload with layout-rotating linear steps: one Strang
    step over the whole field against the oracle's literal step."""
    w, psi0, ref1 = tg256
    plan = _plan(w["n"], w["alpha"], w["beta"], w["dt"], prec)
    plan.select_variant(5, 1)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    start = psi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else psi0
    psi = torch.from_numpy(start).to(DEV).to(dt).contiguous()
    plan.step_n(psi, 1)
    rel = float(np.linalg.norm(psi.cpu().numpy().astype(np.complex128) - ref1) / np.linalg.norm(ref1))
    assert rel < (1e-12 if prec == "c128" else 2e-6), rel
    plan.close()
