"""The paper's own initial conditions of the SRP and RVR benchmarks in the
default GPU suite: the spline smoothed random phase (SRP section: uniform random
values at N_r^3 control points, periodic cubic splines) and the random vortex-ring
pairs of RVR_a (200 pairs, R = pi/2, d = pi; RVR section and its parameter table)
evolved against the oracle at small grids, and the paper-size RVR_c generator
(512^3, 800 pairs) against the host generator on sampled blocks, then 100 steps
with conservation.  The full-length paper runs stay in test_gpu_paper512.py."""
import math

import numpy as np
import pytest

import gp_inputs as I
from oracle import gp as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
SCALARS = ("mass", "energy", "e_kin", "e_kin_i", "e_kin_c", "e_q", "e_int")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_spline_srp_evolves_as_the_oracle(prec):
    """SRP phase of the paper at 64^3 (K = 8 pi as SRP_a, N_r = 4, seed 3), psi =
    exp(i theta) on the GPU, 20 steps of dt = 1/1024 with the parameter-table
    alpha, beta; psi and every diagnostic against the oracle."""
    import paper_2003_03590_amd as gp
    n, dt, steps = 64, 1.0 / 1024, 20
    alpha, beta = I.alpha_beta_table1(n)
    theta = I.srp_spline_theta(n, 8 * math.pi, 4, 3)
    plan = gp.Plan(n, alpha, beta, dt, prec)
    psi = plan.init_phase(torch.from_numpy(theta))
    start = np.exp(1j * theta)
    got0 = psi.to(torch.complex128).cpu().numpy()
    assert np.abs(got0 - start).max() < (1e-15 if prec == "c128" else 1e-7)
    plan.step_n(psi, steps)
    ref = O.evolve(got0, alpha, beta, dt, steps)
    rel = _rel(psi.to(torch.complex128).cpu().numpy(), ref)
    assert rel < (1e-12 if prec == "c128" else 1e-5), rel
    e = plan.energies(psi)
    d = O.diagnostics(ref, alpha, beta)
    for k in SCALARS:
        scale = max(abs(d[k]), 1e-3 * d["energy"])      # E_kin^i is tiny before vortices nucleate
        assert abs(e[k] - d[k]) <= (1e-10 if prec == "c128" else 1e-5) * scale, (k, e[k], d[k])
    plan.close()


def test_rvr_a_construction_evolves_as_the_oracle():
    """The RVR_a construction (200 ring pairs, R = pi/2, d = pi, seed 0) at 32^3 with
    the parameter-table alpha, beta and xi = sqrt(alpha/beta): the GPU generator
    against the host generator, then 20 steps against the oracle (complex128)."""
    import paper_2003_03590_amd as gp
    w = I.WORKLOADS["rvr128_paper"]
    n, dt, steps = 32, w["dt"], 20
    alpha, beta = I.alpha_beta_table1(n)
    xi = math.sqrt(alpha / beta)
    draws = I.rvr_draws(w["n_pairs"], 0, w["R"], w["R"])
    pairs = [(p["R"], p["d"], p["X"], p["Y"], p["Z"], p["perm"]) for p in draws]
    assert all(abs(p["d"] - math.pi) < 1e-15 for p in draws)
    plan = gp.Plan(n, alpha, beta, dt, "c128")
    psi = plan.init_rvr(pairs, xi)
    host = I.rvr_psi(n, xi, w["n_pairs"], 0, w["R"], w["R"])
    assert np.abs(psi.cpu().numpy() - host).max() < 1e-12
    plan.step_n(psi, steps)
    ref = O.evolve(host, alpha, beta, dt, steps)
    assert _rel(psi.cpu().numpy(), ref) < 1e-12
    plan.close()


def test_rvr_c_generator_and_steps_512():
    """RVR_c at the paper's size: 512^3 complex128, 800 ring pairs (R = pi/2,
    d = pi, seed 0), alpha = 0.0125, beta = 160, xi = sqrt(alpha/beta).  The GPU
    generator against the host generator on four sampled 8^3 blocks; then 100 steps
    of dt = 1/4096: N conserved to round-off, E to the run's own drift scale (the
    whole T_f = 4.5 run measured 5.8e-5), and the spectra summing to the energies."""
    import paper_2003_03590_amd as gp
    n, dt, npairs, R = 512, 1.0 / 4096, 800, math.pi / 2
    alpha, beta = I.alpha_beta_table1(n)
    xi = math.sqrt(alpha / beta)
    pairs = [(p["R"], p["d"], p["X"], p["Y"], p["Z"], p["perm"]) for p in I.rvr_draws(npairs, 0, R, R)]
    plan = gp.Plan(n, alpha, beta, dt, "c128")
    psi = plan.init_rvr(pairs, xi)
    rng = np.random.default_rng(7)
    for _ in range(4):
        z, y, x = (int(v) for v in rng.integers(0, n - 8, 3))
        host = I.rvr_psi(n, xi, npairs, 0, R, R, zslab=(z, z + 8), yslab=(y, y + 8), xslab=(x, x + 8))
        got = psi[z:z + 8, y:y + 8, x:x + 8].cpu().numpy()
        assert np.abs(got - host).max() < 1e-12, (z, y, x)
    e0 = plan.energies(psi)
    plan.step_n(psi, 100)
    spec, e1 = plan.spectra(psi)
    dn = abs(e1["mass"] - e0["mass"]) / e0["mass"]
    de = abs(e1["energy"] - e0["energy"]) / e0["energy"]
    print(f"RVR_c 512^3, 100 steps: dN {dn:.2e}, dE {de:.2e}")
    assert dn < 1e-12 and de < 6e-5
    for row, k in enumerate(("e_kin_i", "e_kin_c", "e_q", "e_int")):
        assert abs(spec[row].sum() - e1[k]) < 1e-9 * e1["energy"], k
    plan.close()
