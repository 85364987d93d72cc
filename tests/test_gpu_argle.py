"""Imaginary-time (ARGLE) preparation on the GPU: parity with the oracle, and the
Taylor-Green preparation against the energies the paper prints for it."""
import math
import os

import numpy as np
import pytest

import gp_inputs as I
from oracle import argle as A

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _plan(shape, alpha, beta, prec="c128"):
    import paper_2003_03590_amd as gp
    return gp.Plan(shape, alpha, beta, 1e-3, prec)


def _velocity(shape):
    """Taylor-Green velocity on an (nx, ny, nz) grid: oracle order [v_z, v_y, v_x]."""
    nx, ny, nz = shape
    x = 2 * np.pi * np.arange(nx) / nx
    y = 2 * np.pi * np.arange(ny) / ny
    z = 2 * np.pi * np.arange(nz) / nz
    vx = np.sin(x)[None, None, :] * np.cos(y)[None, :, None] * np.cos(z)[:, None, None]
    vy = -np.cos(x)[None, None, :] * np.sin(y)[None, :, None] * np.cos(z)[:, None, None]
    full = (nz, ny, nx)
    return [np.zeros(full), np.broadcast_to(vy, full).copy(), np.broadcast_to(vx, full).copy()]


def _to_dev_v(v, prec):
    """oracle order [v_z, v_y, v_x] -> device tensor (v_x, v_y, v_z)."""
    dt = torch.float64 if prec == "c128" else torch.float32
    return torch.from_numpy(np.stack([v[2], v[1], v[0]])).to(DEV).to(dt).contiguous()


def _to_dev(a, prec):
    dt = torch.complex128 if prec == "c128" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dt).contiguous()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("shape,prec", [((16, 16, 16), "c128"), ((24, 16, 12), "c128"), ((32, 8, 6), "c128"),
                                        ((16, 16, 16), "c64"), ((48, 24, 8), "c64")],
                         ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else v)
def test_argle_steps_and_energy_match_oracle(shape, prec):
    nx, ny, nz = shape
    alpha, beta, dtau = 0.2, 5.0, 0.02
    phi0 = I.random_field((nz, ny, nx), seed=31)
    v = _velocity(shape)
    plan = _plan(shape, alpha, beta, prec)
    base = phi0.astype(np.complex64).astype(np.complex128) if prec == "c64" else phi0
    vref = [c.astype(np.float32).astype(np.float64) for c in v] if prec == "c64" else v
    vd = _to_dev_v(v, prec)
    phi = _to_dev(phi0, prec)
    e = plan.argle_energy(phi, vd)
    e_ref = A.energy_v(base, vref, alpha, beta)
    tol = 1e-12 if prec == "c128" else 2e-5
    assert abs(e - e_ref) < tol * abs(e_ref)
    plan.argle_step(phi, vd, dtau, 6)
    ref = A.argle(base, vref, alpha, beta, dtau, 6)
    assert _rel(phi.cpu().numpy().astype(np.complex128), ref) < tol
    plan.close()


def test_argle_driven_plane_wave_stays_fixed():
    n, alpha, beta = 16, 0.3, 4.0
    k0 = (1, -2, 3)          # (kx, ky, kz)
    x = 2 * np.pi * np.arange(n) / n
    phi0 = np.exp(1j * (k0[0] * x[None, None, :] + k0[1] * x[None, :, None] + k0[2] * x[:, None, None]))
    v = torch.stack([torch.full((n, n, n), 2 * alpha * k, dtype=torch.float64) for k in k0]).to(DEV)
    plan = _plan(n, alpha, beta)
    phi = _to_dev(phi0, "c128")
    plan.argle_step(phi, v, 0.05, 20)
    assert np.abs(phi.cpu().numpy() - phi0).max() < 1e-12
    assert abs(plan.argle_energy(phi, v)) < 1e-12


def test_argle_errors():
    import paper_2003_03590_amd as gp
    plan = _plan(16, 0.3, 4.0)
    phi = _to_dev(I.random_field(16, seed=1), "c128")
    with pytest.raises(ValueError):
        plan.argle_step(phi, torch.zeros((2, 16, 16, 16), dtype=torch.float64, device=DEV), 0.01, 1)
    with pytest.raises(gp._lib.GPError):
        plan.argle_step(phi, torch.zeros((3, 16, 16, 16), dtype=torch.float64, device=DEV), -0.01, 1)


def test_argle_run_matches_oracle_stopping_rule():
    """gp_argle_run against the oracle's procedure: the criteria of eq. crit1 and
    eq. crit2 at every check, the step at which the run stops, and the field."""
    shape, alpha, beta, dtau = (16, 12, 8), 0.2, 5.0, 0.02
    nx, ny, nz = shape
    phi0 = I.random_field((nz, ny, nx), seed=33)
    v = _velocity(shape)
    plan = _plan(shape, alpha, beta)
    vd = _to_dev_v(v, "c128")
    # fixed number of steps (eps = 0): criteria of the last check (step 30)
    phi = _to_dev(phi0, "c128")
    r = plan.argle_run(phi, vd, dtau, 30, check_every=7, eps=0.0)
    ref, steps, cs, ce, ev, conv = A.argle_run(phi0, v, alpha, beta, dtau, 30, 7, 0.0)
    assert r["steps"] == steps == 30 and not r["converged"] and not conv
    assert abs(r["crit_sup"] - cs) < 1e-10 * cs and abs(r["crit_energy"] - ce) < 1e-8 * ce
    assert abs(r["e_v"] - ev) < 1e-12 * ev
    assert _rel(phi.cpu().numpy(), ref) < 1e-12
    # a threshold between two checks of the oracle's run: both stop at the same check
    crit = []
    p = phi0
    for k in range(1, 41):
        new = A.argle_step(p, v, alpha, beta, dtau)
        if k % 5 == 0:
            crit.append((k, A.crit_sup(new, p, dtau)))
        p = new
    # first check that falls clearly (10 %) below every earlier one
    j = next(j for j in range(1, len(crit)) if crit[j][1] < 0.9 * min(c for _, c in crit[:j]))
    k2 = crit[j][0]
    eps = 0.5 * (crit[j][1] + min(c for _, c in crit[:j]))
    phi = _to_dev(phi0, "c128")
    r = plan.argle_run(phi, vd, dtau, 1000, check_every=5, eps=eps)
    assert r["converged"] and r["steps"] == k2, (r, k2)
    # max_steps = 0: no check, E_v of the input
    phi = _to_dev(phi0, "c128")
    r = plan.argle_run(phi, vd, dtau, 0, check_every=5, eps=1.0)
    assert r["steps"] == 0 and math.isnan(r["crit_sup"]) and abs(r["e_v"] - A.energy_v(phi0, v, alpha, beta)) < 1e-12
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_argle_run_stops_where_the_scalar_recursion_converges(prec):
    """Uniform phi = c, v = 0: each step is c <- c + dtau beta (1 - |c|^2) c; the run
    stops at the first check whose |c_{n+1} - c_n| / dtau <= eps."""
    n, alpha, beta, dtau, eps, every = 16, 0.3, 2.0, 0.05, 1.2e-3, 4   # stop check at 0.99e-3, one before at 2.4e-3
    c0 = 0.4 * np.exp(-0.3j)
    c, k, want = c0, 0, None
    while want is None:
        cn = c + dtau * beta * (1 - abs(c) ** 2) * c
        k += 1
        if k % every == 0 and abs(cn - c) / dtau <= eps:
            want = (k, abs(cn - c) / dtau)
        c = cn
    plan = _plan(n, alpha, beta, prec)
    phi = _to_dev(np.full((n, n, n), c0), prec)
    dt = torch.float64 if prec == "c128" else torch.float32
    r = plan.argle_run(phi, torch.zeros((3, n, n, n), dtype=dt, device=DEV), dtau, 10 ** 5, every, eps)
    tol = 1e-9 if prec == "c128" else 5e-3        # FP32 field: |c_{n+1} - c_n| ~ 5e-5 to ~6e-8
    assert r["converged"] and r["steps"] == want[0]
    assert abs(r["crit_sup"] - want[1]) < tol * want[1]
    assert np.abs(phi.cpu().numpy() - c).max() < (1e-12 if prec == "c128" else 1e-6)
    plan.close()


def _golden(name="tg_argle_energies.txt"):
    rows = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows[f[0]] = [float(v) for v in f[1:]]
    return rows


def _energies_row(r):
    """N alpha beta E_kin^i E_kin^c E_q E_int E_v -> dict"""
    return dict(n=int(r[0]), alpha=r[1], beta=r[2], e_kin_i=r[3], e_kin_c=r[4], e_q=r[5], e_int=r[6], e_v=r[7])


def _prepare(n, alpha, beta, dtau, steps, ic="tg"):
    """The paper's preparation: ansatz, then ARGLE with the matching flow for
    `steps` steps (no early stop); returns the field, its energies, E_v / (2 alpha)
    (the printed normalisation) and the report of the last step."""
    plan = _plan(n, alpha, beta)
    if ic == "tg":
        expo = int(math.floor(1.0 / (2 * math.pi * alpha)))
        phi = _to_dev(I.tg_psi(n, math.sqrt(alpha / beta), expo), "c128")
        v = _to_dev_v(I.tg_velocity(n), "c128")
    else:
        phi = _to_dev(I.abc_psi(n, alpha), "c128")
        v = _to_dev_v(I.abc_velocity(n), "c128")
    rep = plan.argle_run(phi, v, dtau, steps, check_every=steps, eps=0.0)
    e = plan.energies(phi)
    e["e_v"] = rep["e_v"] / (2 * alpha)
    plan.close()
    return phi, e, rep


def _rels(e, g, keys=("e_kin_i", "e_kin_c", "e_q", "e_int", "e_v")):
    return {k: abs(e[k] - g[k]) / g[k] for k in keys if not math.isnan(g[k])}


def _evolve(phi, n, alpha, beta, dt, t_final, every):
    """GP run from a prepared field: N and E at 0 and T_f and the maximum relative
    changes, sampled every `every` steps."""
    import paper_2003_03590_amd as gp
    plan = gp.Plan(n, alpha, beta, dt, "c128")
    plan.autotune(reps=3)
    steps = int(round(t_final / dt))
    e0 = plan.energies(phi)
    dn = de = 0.0
    done = 0
    while done < steps:
        k = min(every, steps - done)
        plan.step_n(phi, k)
        done += k
        e = plan.energies(phi)
        dn = max(dn, abs(e["mass"] - e0["mass"]) / e0["mass"])
        de = max(de, abs(e["energy"] - e0["energy"]) / e0["energy"])
    plan.close()
    return e0, e, dn, de


@pytest.fixture(scope="module")
def tg_a_prepared():
    w = I.WORKLOADS["tg128_argle"]
    return _prepare(w["n"], w["alpha"], w["beta"], w["dtau"], w["steps"])


def test_taylor_green_preparation_reproduces_the_paper(tg_a_prepared):
    """TG_aIT (128^3, alpha = 0.05, beta = 40, dtau = 1.25e-2, tau_f = 60 from
    psi_4^3) against the paper's table of TG energies at tau_f, and its N and E
    against the t = 0 column of the TG conservation table.  Readings: the table's
    E_v column is E_v / (2 alpha), the mean of eq. energy-num-ext-vel without its
    2 alpha prefactor (a factor 10 here; the match is then 2e-5), and E_q is
    1/2 <|2 alpha grad |psi||^2> evaluated pointwise from psi's derivatives.  The
    compressible part is three orders of magnitude below the others and the least
    converged in tau, hence its looser bound."""
    _, e, rep = tg_a_prepared
    g = _energies_row(_golden()["TG_aIT"])
    rel = _rels(e, g)
    print("TG_aIT:", {k: (e[k], g[k]) for k in rel}, "relative differences:", rel, "last step:", rep)
    assert rel["e_kin_i"] < 1e-4 and rel["e_int"] < 1e-4 and rel["e_q"] < 5e-4 and rel["e_v"] < 1e-4
    assert rel["e_kin_c"] < 5e-3
    c = _golden("tg_conservation.txt")["TG_a"]
    assert abs(e["mass"] - c[5]) < 1e-6 and abs(e["energy"] - c[8]) < 3e-5 * c[8]


def test_taylor_green_run_conserves_as_printed(tg_a_prepared):
    """TG_a: the GP run from the TG_aIT field (dt = 1.25e-3, T_f = 12, 9600 Strang
    steps).  N is conserved to round-off (the paper prints delta(N) = 0.0); E(T_f)
    matches the printed value to 2e-5 and the maximum relative energy change
    (sampled every 200 steps) is of the printed size 7.97e-5 (within a factor 1.5:
    it depends on the sampling and on the last digits of the state)."""
    phi, _, _ = tg_a_prepared
    c = _golden("tg_conservation.txt")["TG_a"]
    n, alpha, beta, dt, tf = int(c[0]), c[1], c[2], c[3], c[4]
    e0, e, dn, de = _evolve(phi.clone(), n, alpha, beta, dt, tf, 200)
    print(f"TG_a: N0 {e0['mass']:.9f} N(T) {e['mass']:.9f} dN {dn:.2e}  E0 {e0['energy']:.9f} E(T) {e['energy']:.9f}"
          f" dE {de:.3e} (printed {c[8]} {c[9]} {c[10]})")
    assert dn < 1e-10
    assert abs(e["energy"] - c[9]) < 2e-5 * c[9]
    assert c[10] / 1.5 < de < 1.5 * c[10]


def test_taylor_green_grid_convergence_run_at_256():
    """TG_h (256^3, alpha = 0.05, beta = 40) of the grid-convergence table.  Reading:
    the table gives no dtau or tau_f for it; tau_f = 60 as for TG_aIT and
    dtau = 6.25e-3, the step of the 256^3 preparation TG_bIT (1.25e-2 is unstable at
    this resolution).  The run converges (eq. crit1 below 1e-6) and every printed
    digit is reproduced."""
    g = _energies_row(_golden()["TG_h"])
    _, e, rep = _prepare(256, g["alpha"], g["beta"], 6.25e-3, 9600)
    rel = _rels(e, g)
    print("TG_h:", {k: (e[k], g[k]) for k in rel}, "relative differences:", rel, "last step:", rep)
    assert rep["crit_sup"] < 1e-5
    assert rel["e_kin_i"] < 1e-4 and rel["e_q"] < 1e-4 and rel["e_int"] < 1e-4 and rel["e_v"] < 1e-5
    assert rel["e_kin_c"] < 1e-3


def test_taylor_green_256_preparation_and_run():
    """TG_bIT (256^3, alpha = 0.025, beta = 80, [gamma_d/4] = 6, dtau = 6.25e-3,
    tau_f = 60) against its printed energies, then TG_b (dt = 6.25e-4, T_f = 12)
    against the conservation table.  The preparation is not converged at tau_f
    (eq. crit1 about 5e-2), so the energies agree to 1e-3 (E_kin^c, 1e-3 of the
    total, to 6e-2) and E(0) to 1e-3; N(0), conservation of N and the size of
    delta(E) are checked as for TG_a."""
    g = _energies_row(_golden()["TG_bIT"])
    phi, e, rep = _prepare(256, g["alpha"], g["beta"], 6.25e-3, 9600)
    rel = _rels(e, g)
    print("TG_bIT:", {k: (e[k], g[k]) for k in rel}, "relative differences:", rel, "last step:", rep)
    assert rel["e_kin_i"] < 1e-3 and rel["e_q"] < 1e-3 and rel["e_int"] < 1e-3 and rel["e_kin_c"] < 6e-2
    c = _golden("tg_conservation.txt")["TG_b"]
    e0, e1, dn, de = _evolve(phi, 256, c[1], c[2], c[3], c[4], 400)
    print(f"TG_b: N0 {e0['mass']:.9f} E0 {e0['energy']:.9f} E(T) {e1['energy']:.9f} dN {dn:.2e} dE {de:.3e}"
          f" (printed {c[5]} {c[8]} {c[9]} {c[10]})")
    assert abs(e0["mass"] - c[5]) < 1e-5 and abs(e0["energy"] - c[8]) < 1e-3 * c[8]
    assert dn < 1e-10 and c[10] / 1.5 < de < 1.5 * c[10]


@pytest.fixture(scope="module")
def abc_a_prepared():
    r = _golden("abc_argle_energies.txt")["ABC_aIT"]
    n, alpha, beta, dtau, tau_f = int(r[0]), r[1], r[2], r[3], r[4]
    return _prepare(n, alpha, beta, dtau, int(round(tau_f / dtau)), ic="abc")


def test_abc_preparation_is_close_to_the_paper(abc_a_prepared):
    """ABC_aIT (128^3, alpha = 0.05, beta = 40, dtau = 4e-3, tau_f = 30 from the
    phase-only ansatz with v = v_ABC).  The paper stopped these runs before
    eq. crit1 was met, with eq. crit2 near 1e-3; the state at tau_f then depends on
    the path, so the check is closeness: E_kin^i, E_q, E_int within 1 %, E_kin^c
    (1e-3 of the total) within 10 %, and eq. crit2 at tau_f below 2e-3."""
    r = _golden("abc_argle_energies.txt")["ABC_aIT"]
    g = dict(e_kin_i=r[5], e_kin_c=r[6], e_q=r[7], e_int=r[8])
    _, e, rep = abc_a_prepared
    rel = _rels(e, g, keys=tuple(g))
    print("ABC_aIT:", {k: (e[k], g[k]) for k in rel}, "relative differences:", rel, "last step:", rep)
    assert rel["e_kin_i"] < 1e-2 and rel["e_q"] < 1e-2 and rel["e_int"] < 1e-2 and rel["e_kin_c"] < 0.1
    assert rep["crit_energy"] < 2e-3


def test_helicity_of_the_prepared_fields(tg_a_prepared, abc_a_prepared):
    """H and H_reg of the prepared fields against the paper's tables: the Taylor-Green
    state has none (printed 1.4e-13 and -1.9e-11; its symmetries cancel every
    contribution), the ABC state carries the helicity of the driving flow (printed
    H = 2.41, H_reg = 2.47 for ABC_aIT; the classical value is 3).  The ABC state is
    the not-converged preparation above (energies within 1 %).  H_reg, the quantity
    the paper builds for this purpose, agrees to 1 % (measured 0.3 %); the plain H
    samples v where it is singular (the paper calls it the noisier of the two) and
    is checked to 15 % (measured 10 %).  Also the GPU against the oracle on the same
    128^3 ABC field."""
    from oracle import helicity as OH
    import paper_2003_03590_amd as gp
    phi_tg, _, _ = tg_a_prepared
    w = I.WORKLOADS["tg128_argle"]
    plan = gp.Plan(w["n"], w["alpha"], w["beta"], 1e-3, "c128")
    H, Hreg, _ = plan.helicity(phi_tg)
    plan.close()
    print("TG_aIT helicity:", H, Hreg)
    assert abs(H) < 1e-8 and abs(Hreg) < 1e-8
    r = _golden("abc_argle_energies.txt")["ABC_aIT"]
    phi_abc, _, _ = abc_a_prepared
    plan = gp.Plan(int(r[0]), r[1], r[2], 1e-3, "c128")
    H, Hreg, spec = plan.helicity(phi_abc)
    plan.close()
    print("ABC_aIT helicity:", H, Hreg, "printed", r[9], r[10])
    assert abs(Hreg - r[10]) < 0.01 * r[10] and abs(H - r[9]) < 0.15 * r[9]
    ref = OH.helicity(phi_abc.cpu().numpy(), r[1])
    assert abs(H - ref["H"]) < 1e-9 * abs(ref["H"]) and abs(Hreg - ref["H_reg"]) < 1e-9 * abs(ref["H_reg"])


@pytest.mark.parametrize("shape", [(16, 12, 1), (1, 16, 8), (32, 1, 1)], ids=lambda s: "x".join(map(str, s)))
def test_argle_on_degenerate_grids(shape):
    """Grids with axes of length 1 (2-D and 1-D problems): that axis has only k = 0,
    so its derivative vanishes; steps, E_v and the stopping rule match the oracle."""
    nx, ny, nz = shape
    alpha, beta, dtau = 0.2, 5.0, 0.02
    phi0 = I.random_field((nz, ny, nx), seed=35)
    rng = np.random.default_rng(36)
    v = [0.3 * rng.standard_normal((nz, ny, nx)) for _ in range(3)]
    plan = _plan(shape, alpha, beta)
    vd = _to_dev_v(v, "c128")
    phi = _to_dev(phi0, "c128")
    r = plan.argle_run(phi, vd, dtau, 9, check_every=4, eps=0.0)
    ref, steps, cs, ce, ev, conv = A.argle_run(phi0, v, alpha, beta, dtau, 9, 4, 0.0)
    assert r["steps"] == steps and abs(r["e_v"] - ev) < 1e-12 * ev
    assert abs(r["crit_sup"] - cs) < 1e-10 * cs
    assert _rel(phi.cpu().numpy(), ref) < 1e-12
    plan.close()


def test_abc_run_conserves_as_printed(abc_a_prepared):
    """ABC_a: the GP run from the ABC_aIT field (dt = 8e-4, T_f = 10, 12500 steps)
    against the ABC conservation table: N(0) of the prepared field (1.2e-4 from the
    printed value; the preparation itself is within 1 %), N conserved to round-off,
    the maximum energy change of the printed size 5.98e-5 (within a factor 1.5)."""
    phi, _, _ = abc_a_prepared
    c = _golden("abc_conservation.txt")["ABC_a"]
    e0, e, dn, de = _evolve(phi.clone(), int(c[0]), c[1], c[2], c[3], c[4], 250)
    print(f"ABC_a: N0 {e0['mass']:.7f} E0 {e0['energy']:.7f} E(T) {e['energy']:.7f} dN {dn:.2e} dE {de:.3e}"
          f" (printed {c[5]} {c[8]} {c[9]} {c[10]})")
    assert abs(e0["mass"] - c[5]) < 5e-4 and dn < 1e-10
    assert c[10] / 1.5 < de < 1.5 * c[10]


def test_abc_256_preparation_run_and_helicity():
    """ABC_bIT (256^3, alpha = 0.025, beta = 80, dtau = 2e-3, tau_f = 30) against its
    printed energies and helicities, then ABC_b (dt = 4e-4, T_f = 10) against the
    conservation table.  Like ABC_aIT this preparation was stopped before
    convergence in the paper, so the energies and H_reg are compared at the level
    the not-converged state allows (measured values in the assertions' comments)."""
    import paper_2003_03590_amd as gp
    r = _golden("abc_argle_energies.txt")["ABC_bIT"]
    n, alpha, beta, dtau, tau_f = int(r[0]), r[1], r[2], r[3], r[4]
    phi, e, rep = _prepare(n, alpha, beta, dtau, int(round(tau_f / dtau)), ic="abc")
    g = dict(e_kin_i=r[5], e_kin_c=r[6], e_q=r[7], e_int=r[8])
    rel = _rels(e, g, keys=tuple(g))
    plan = gp.Plan(n, alpha, beta, 1e-3, "c128")
    H, Hreg, _ = plan.helicity(phi)
    plan.close()
    c = _golden("abc_conservation.txt")["ABC_b"]
    e0, e1, dn, de = _evolve(phi, n, c[1], c[2], c[3], c[4], 1250)
    print("ABC_bIT:", {k: (e[k], g[k]) for k in g}, "relative:", rel, "H", H, Hreg, "printed", r[9], r[10],
          "crit2", rep["crit_energy"])
    print(f"ABC_b: N0 {e0['mass']:.7f} E0 {e0['energy']:.7f} dN {dn:.2e} dE {de:.3e} (printed {c[5]} {c[8]} {c[10]})")
    # measured: E_kin^i 3.4e-3, E_kin^c 1.6e-3, E_q 7.7e-5, E_int 3.7e-4; H_reg 2.6480 vs 2.6533,
    # H 2.690 vs 2.744; N(0) 7e-5; delta(E) 6.06e-5 vs 6.18e-5
    assert rel["e_kin_i"] < 1e-2 and rel["e_q"] < 1e-3 and rel["e_int"] < 2e-3 and rel["e_kin_c"] < 1e-2
    assert abs(Hreg - r[10]) < 1e-2 * r[10] and abs(H - r[9]) < 5e-2 * r[9]
    assert abs(e0["mass"] - c[5]) < 5e-4
    assert dn < 1e-10 and c[10] / 1.5 < de < 1.5 * c[10]
