"""Benchmark of the Gross-Pitaevskii split step on one MI355X.

Workload (tg256): 256^3 periodic box, Taylor-Green vortex-lattice ansatz with
core width xi = 2 (2 pi / 256), alpha beta = 2 (alpha = 0.06942, beta = 28.81),
dt = 5e-4, energy decomposition and shell spectra every 100 steps, complex128
(headline) and complex64.  One bench "step" is one pass of the whole hot path:
100 Strang steps (gp_step_n) followed by the diagnostics (gp_spectra); the
default 10 timed bench steps are the workload's 1000 time steps.

Printed: one JSON line with the throughput in grid-point.steps/s; `roofline`,
the HBM roofline of the passes of the 1024^3 complex64 workload (an 8 GiB state,
32 times the last-level cache; HIP events over the timed region, a plain device
copy of the same bytes beside it); `roofline_tg256_c128`, the headline's axis pass
on its cache-resident state; the complex64 form at its measured energy drift, the
literal form, the 48-run ensemble, the 1024^3 layout forms, and the CPU oracle
timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
WORKLOAD = "tg256"
DIAG_EVERY = 100


def pass_traffic(name="axis_pass_tg256_traffic.json", schedules=None):
    """HBM bytes per axis-pass launch from a committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size), or None when
    the kernel sources changed since the counters were taken, or when `schedules`
    (the x, y, z schedule names of the timed plan) differ from the ones profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["source_files"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        if schedules is not None:
            for ax, sched in zip(rec["axes"], schedules):
                shape = " ".join(sched.split()[:4])          # "N=.. T=.. W=.. R=.."
                if shape not in ax["kernel"]:
                    return None
        return rec["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def run_form(gp, torch, psi0_np, w, prec, steps, warmup, tune=True):
    """Time `steps` bench steps (100 split steps + diagnostics each) after `warmup`."""
    n = w["n"]
    plan = gp.Plan(n, w["alpha"], w["beta"], w["dt"], prec)
    if tune:
        plan.autotune(reps=5)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    psi = torch.from_numpy(psi0_np).to("cuda").to(dt).contiguous()
    stream = torch.cuda.current_stream()
    e0 = plan.energies(psi)
    energies = [e0]
    for _ in range(warmup):
        plan.step_n(psi, DIAG_EVERY)
        plan.spectra(psi)
    # restart from the initial condition so the timed run is the workload itself
    psi.copy_(torch.from_numpy(psi0_np).to("cuda").to(dt))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    per_run = w["steps"] // DIAG_EVERY          # bench steps of one whole workload
    dev0 = torch.from_numpy(psi0_np).to("cuda").to(dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if i and i % per_run == 0:               # the workload again from its initial condition
            psi.copy_(dev0)
        ev[i][0].record(stream)
        plan.step_n(psi, DIAG_EVERY)
        ev[i][1].record(stream)
        spec, e = plan.spectra(psi)          # synchronizes the stream
        energies.append(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    passes_per_call = 3 * (DIAG_EVERY + 1)
    mean_pass_ms = sum(step_ms) / (passes_per_call * steps)
    E0 = e0["energy"]
    N0 = e0["mass"]
    dE = max(abs(e["energy"] - E0) for e in energies) / E0
    dN = max(abs(e["mass"] - N0) for e in energies) / N0
    out = psi.to(torch.complex128).cpu().numpy()
    del dev0
    return dict(plan=plan, wall=wall, step_ms=step_ms, mean_pass_ms=mean_pass_ms, dE=dE, dN=dN, psi=out,
                energies=energies, spec=spec)


def literal_form(torch, plan, psi0_np, step_ms_merged, steps=10):
    """The literal (un-merged) Strang step of the time-evolution section on the same
    plan and field: per step two 3-D linear half steps, each a forward 3-D FFT
    (3 passes, the last applying the 3-D multiplier before it stores) and an
    inverse 3-D FFT (3 passes), with the nonlinear rotation between them: 13 sweeps,
    26 N^3 S bytes per step against the merged form's 6 N^3 S."""
    S = 16 if plan.prec == 0 else 8
    dt = torch.complex128 if S == 16 else torch.complex64
    psi = torch.from_numpy(psi0_np).to("cuda").to(dt).contiguous()
    plan.step_literal_n(psi, 1)
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(st)
    plan.step_literal_n(psi, steps)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    npts = float(psi0_np.size)
    per_step = 26.0 * npts * S
    return {"steps": steps, "ms_per_step": ms, "value": npts / (ms / 1e3), "unit": "grid-point.steps/s",
            "bytes_per_step": per_step, "hbm_gbs": per_step / (ms / 1e3) / 1e9,
            "merged_over_literal": ms / step_ms_merged}


def ensemble_form(gp, torch, I):
    """The 48-run ensemble (32 at 64^3, 16 at 96^3, complex64, dt = 1e-3, 300 steps)
    advanced by one gp_step_n_batch call after autotuning (recorded step graphs:
    the opening half step, bodies of 128, 128, 32, 8, 2 and 1 applications, the
    closing half step; the two size groups on parallel branches);
    grid-point.steps/s summed over runs and the per-run drift of mass and energy."""
    import numpy as np
    w = I.WORKLOADS["ens48"]
    runs = [dict(r, dt=w["dt"]) for r in w["runs"]]
    bp = gp.BatchPlan(runs, "c64")
    bp.autotune(reps=3)
    init = [torch.from_numpy(np.exp(1j * I.srp_fourier_theta(r["n"], w["K"], r["seed"]))).to("cuda")
            .to(torch.complex64).contiguous() for r in runs]
    states = [x.clone() for x in init]
    bp.step_n(states, w["steps"])           # records and runs the graph once
    torch.cuda.synchronize()
    for s, x in zip(states, init):
        s.copy_(x)
    e0 = bp.energies(states)
    torch.cuda.synchronize()
    t = time.perf_counter()
    bp.step_n(states, w["steps"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    e1 = bp.energies(states)
    pts = sum(float(r["n"]) ** 3 for r in runs)
    # algorithmic bytes: a run on the xy-plane pass reads and writes its state twice per
    # step (plane pass + z pass), otherwise three times (x, y, z passes); the call's
    # opening half step adds one more step's worth
    plane = [bp.schedule(i, 3).startswith("xy: plane") for i in range(len(runs))]
    nbytes = sum((4.0 if pl else 6.0) * float(r["n"]) ** 3 * 8 for r, pl in zip(runs, plane)) * (w["steps"] + 1)
    return {"value": pts * w["steps"] / el, "unit": "grid-point.steps/s (summed over runs)",
            "runs": len(runs), "steps": w["steps"], "seconds": el,
            "hbm_GBs": nbytes / el / 1e9, "bytes": nbytes,
            "plane_pass_runs": int(sum(plane)),
            "max_dN": float(np.max(np.abs(e1[:, 0] - e0[:, 0]) / e0[:, 0])),
            "max_dE": float(np.max(np.abs(e1[:, 1] - e0[:, 1]) / e0[:, 1])),
            "launch": "8 launches of 8 recorded step graphs (opening half step, bodies of 128, 128, 32, 8, 2, 1 "
                      "applications, closing half step), each with one grouped pass launch per size group "
                      "and pass (the runs of a group on the second grid dimension) and the two size groups "
                      "on parallel branches",
            "copy_reference": "the 48 states total 0.18 GB and fit the 256 MB last-level cache, so this "
                              "rate is not an HBM figure; the HBM copy reference is "
                              "large_1024_c64.roofline.copy_gbs"}


def large_form(gp, torch, I, steps=5):
    """The 1024^3 complex64 workload (40 random vortex-ring pairs, alpha = 0.02603,
    beta = 76.83, dt = 2.5e-4) with autotuned schedules: `steps` Strang steps timed
    with HIP events on the plan's stream.  An 8 GiB state is far beyond the 256 MB
    last-level cache, so this is the HBM-bound form of the axis pass."""
    w = I.WORKLOADS["rvr1024"]
    n = w["n"]
    ic = w["ic"][1]
    plan = gp.Plan(n, w["alpha"], w["beta"], w["dt"], "c64")
    plan.autotune(reps=3)
    pairs = [(p["R"], p["d"], p["X"], p["Y"], p["Z"], p["perm"]) for p in I.rvr_draws(ic["n_pairs"], ic["seed"])]
    psi = plan.init_rvr(pairs, ic["xi"])
    plan.step_n(psi, 1)
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(st)
    plan.step_n(psi, steps)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    launches = 3 * (steps + 1)
    per_launch = 2.0 * float(n) ** 3 * 8
    gbs = per_launch * launches / (ms / 1e3) / 1e9
    # each axis pass alone (the propagator sub-step), and a device copy of the same
    # bytes (read 8 GiB, write 8 GiB): what this machine's HBM delivers to a plain stream
    axis = {}
    for ax in range(3):
        plan.substep_linear(psi, ax, w["dt"])
        torch.cuda.synchronize()
        a.record(st)
        for _ in range(3):
            plan.substep_linear(psi, ax, w["dt"])
        b.record(st)
        torch.cuda.synchronize()
        axis["xyz"[ax]] = per_launch / (a.elapsed_time(b) / 3 / 1e3) / 1e9
    x = torch.empty_like(psi)
    copies = {}
    for name, fn in (("gp_copy_state", lambda: plan.copy_state(psi, x)), ("torch_copy", lambda: x.copy_(psi))):
        fn()
        torch.cuda.synchronize()
        a.record(st)
        for _ in range(3):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        copies[name] = per_launch / (a.elapsed_time(b) / 3 / 1e3) / 1e9
    copy_gbs = copies["gp_copy_state"]
    del x
    # both forms of the linear steps, whichever the autotuner kept (fixed layout in
    # place, or layout-rotating passes through one more state)
    chosen = plan.schedule(5)
    forms = {}
    for v, name in ((0, "fixed"), (1, "rotating"), (2, "rotating+contiguous")):
        plan.select_variant(5, v)
        plan.step_n(psi, 2)
        torch.cuda.synchronize()
        a.record(st)
        plan.step_n(psi, steps)
        b.record(st)
        torch.cuda.synchronize()
        fms = a.elapsed_time(b)
        forms[name] = {"ms_per_step": fms / steps,
                       "axis_pass_gbs": per_launch * launches / (fms / 1e3) / 1e9,
                       "frac": per_launch * launches / (fms / 1e3) / 1e9 / HBM_PEAK_GBS}
    rot = chosen.startswith("layout: rotating")
    mixed = chosen.startswith("layout: rotating+contiguous")
    plan.select_variant(5, 2 if mixed else 1 if rot else 0)
    out = {"workload": "rvr1024: 1024^3 complex64, 40 random vortex-ring pairs (seed 1), dt = 2.5e-4",
           "steps": steps, "ms_per_step": ms / steps,
           "value": float(n) ** 3 * steps / (ms / 1e3), "unit": "grid-point.steps/s",
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "per_launch_bytes": per_launch,
                        "kernel": ("rot_pass twice and axis_pass (x kind, in place) once per step, mean of "
                                   "the three (the nonlinear rotation fused into the first rot_pass)") if mixed else
                                  ("rot_pass (layout-rotating propagator pass; the nonlinear rotation fused "
                                   "into the first pass of each step)") if rot else
                                  ("axis_pass (propagator; the nonlinear rotation fused into the carrier "
                                   "axis's pass)"),
                        "per_launch": "one axis pass: reads and writes the whole state once (2 N^3 S bytes)",
                        "traffic": (pass_traffic("mixed_pass_rvr1024_traffic.json") if mixed else
                                    pass_traffic("rot_pass_rvr1024_traffic.json") if rot else
                                    pass_traffic("axis_pass_rvr1024_traffic.json",
                                                 [plan.schedule(ax) for ax in range(3)])),
                        "traffic_source": "profiles/%s_pass_rvr1024_traffic.json (null once the kernel "
                                          "sources or schedules differ from the profiled ones)"
                                          % ("mixed" if mixed else "rot" if rot else "axis"),
                        "mean_launch_us": ms * 1e3 / launches,
                        "copy_gbs": copy_gbs, "frac_of_copy": gbs / copy_gbs,
                        "copy": "gp_copy_state: read 8 GiB, write 8 GiB, one 16-byte unit per lane "
                                f"(torch's copy_ of the same tensors: {copies['torch_copy']:.0f} GB/s)",
                        "axis_gbs": axis, "axis_frac": {k: v / HBM_PEAK_GBS for k, v in axis.items()},
                        "axis_frac_of_copy": {k: v / copy_gbs for k, v in axis.items()}},
           "layout_forms": forms,
           "schedule": [plan.schedule(ax) for ax in range(6)]}
    plan.close()
    del psi
    torch.cuda.empty_cache()
    return out


ARGLE_BYTES_PER_POINT = 30.5    # x S bytes per grid point and ARGLE step (see argle_form)


def argle_form(gp, torch, I, steps=200, warmup=20):
    """Imaginary-time (ARGLE) preparation at 256^3 complex128 in the configuration
    of the grid-convergence run TG_h (alpha = 0.05, beta = 40, dtau = 6.25e-3, Taylor-
    Green ansatz and flow): `steps` steps timed with HIP events on the plan's stream.
    Algorithmic bytes per step, in units of S = 16 bytes per point: the x and y
    derivative passes (read phi, write d_j: 4), the z-derivative pass that forms the
    explicit part in place of d_z (read phi, d_x, d_y and the three real velocity
    planes, write n: 5.5), forward 3-D transforms of phi and n (3 passes each, 12),
    the diagonal solve (read both, write phi: 3) and the inverse 3-D transform (6):
    30.5 S."""
    import numpy as np
    n, alpha, beta, dtau = 256, 0.05, 40.0, 6.25e-3
    plan = gp.Plan(n, alpha, beta, 1e-3, "c128")
    expo = int(math.floor(1.0 / (2 * math.pi * alpha)))
    phi = torch.from_numpy(I.tg_psi(n, math.sqrt(alpha / beta), expo)).to("cuda").contiguous()
    vz, vy, vx = I.tg_velocity(n)
    v = torch.from_numpy(np.stack([vx, vy, vz])).to("cuda").contiguous()
    plan.argle_step(phi, v, dtau, warmup)
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(st)
    plan.argle_step(phi, v, dtau, steps)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    per_step = ARGLE_BYTES_PER_POINT * 16.0 * float(n) ** 3
    gbs = per_step / (ms / 1e3) / 1e9
    out = {"workload": "TG_h preparation: 256^3 complex128, alpha = 0.05, beta = 40, dtau = 6.25e-3, "
                       "Taylor-Green ansatz and flow",
           "steps": steps, "ms_per_step": ms, "value": float(n) ** 3 / (ms / 1e3), "unit": "grid-point.steps/s",
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "per_step_bytes": per_step, "traffic": None,
                        "kernel": "whole ARGLE step (axis passes, explicit part, diagonal solve)"}}
    plan.close()
    del phi, v
    torch.cuda.empty_cache()
    return out


def passes_mode(gp, torch, spec, reps, tune=False, variants=None, rotating=False):
    """Each axis pass (propagator sub-step S(s, L_j)) `reps` times on a random
    N^3 field, then `reps` plain device copies of the same bytes (gp_copy_state:
    the bandwidth reference, and the calibration of the FETCH_SIZE / WRITE_SIZE
    counters); prints one JSON line of event timings.  With `tune`, the schedules
    are autotuned first; `variants` (one schedule variant per axis) fixes them
    instead, e.g. to those a timed run selected.  With `rotating`, the passes are
    the layout-rotating ones: `reps` calls of one Strang step (six passes)."""
    n, prec = spec.split(":")
    n = int(n)
    plan = gp.Plan(n, 0.05, 40.0, 1e-3, prec)
    if tune:
        plan.autotune(reps=3)
    if variants:
        for ax, v in enumerate(int(x) for x in variants.split(",")):
            plan.select_variant(ax, v)
    if rotating:
        plan.select_variant(5, 1)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    S = 16 if prec == "c128" else 8
    psi = torch.randn(n, n, n, dtype=dt, device="cuda")
    psi /= psi.abs()
    st = torch.cuda.current_stream()
    out = {"n": n, "prec": prec, "bytes_per_launch": 2 * n ** 3 * S,
           "schedule": [plan.schedule(ax) for ax in range(6)]}

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(k):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k * 1e3
    if rotating:
        us = timed(lambda: plan.step_n(psi, 1), reps) / 6
        out["rot_us"] = us
        out["rot_GBs"] = 2 * n ** 3 * S / us / 1e3
    else:
        for ax in range(3):
            us = timed(lambda: plan.substep_linear(psi, ax, 1e-3), reps)
            out[f"axis{ax}_us"] = us
            out[f"axis{ax}_GBs"] = 2 * n ** 3 * S / us / 1e3
    x = torch.empty_like(psi)
    us = timed(lambda: plan.copy_state(psi, x), reps)
    out["copy_us"] = us
    out["copy_GBs"] = 2 * n ** 3 * S / us / 1e3
    print(json.dumps(out))
    return 0


def _ensemble_member_step(args):
    """One literal Strang step of one ensemble member by the oracle (a pool task)."""
    import numpy as np
    import gp_inputs as I
    from oracle import gp as O
    from threadpoolctl import threadpool_limits
    r, K, dt = args
    psi = np.exp(1j * I.srp_fourier_theta(r["n"], K, r["seed"]))
    with threadpool_limits(1):              # one core per worker (the pool forks a threaded BLAS)
        t = time.perf_counter()
        O.strang_step(psi, r["alpha"], r["beta"], dt)
        return float(r["n"]) ** 3, time.perf_counter() - t


def oracle_sample(psi0_np, w, ensemble=True):
    """The CPU oracle on a bounded sample: one literal Strang step of the same 256^3 field;
    beside it, seconds per step at 32^3 ... 128^3 (the same construction), their
    N^3 log N extrapolation to the 1024^3 workload, and the ensemble's members run
    one per host core (a process pool started before the GPU is touched)."""
    import gp_inputs as I
    from oracle import gp as O
    out = {}
    if ensemble:
        # 16 members in the ensemble's size mix (10 at 64^3, 6 at 96^3), one process per
        # core, one step each; BLAS single-threaded in every worker
        import concurrent.futures as cf
        import multiprocessing as mp
        ew = I.WORKLOADS["ens48"]
        runs = ew["runs"][:10] + ew["runs"][32:38]
        procs = min(len(runs), os.cpu_count() or 1)
        t = time.perf_counter()
        with cf.ProcessPoolExecutor(procs, mp_context=mp.get_context("fork")) as ex:
            res = list(ex.map(_ensemble_member_step, [(r, ew["K"], ew["dt"]) for r in runs]))
        wall = time.perf_counter() - t
        pts = sum(p for p, _ in res)
        out["ensemble_aggregate"] = {
            "value": pts / wall, "unit": "grid-point.steps/s (summed over runs)", "cores": procs,
            "sample": f"one literal Strang step of each of {len(runs)} ensemble members (10 at 64^3, 6 at 96^3), "
                      f"one process per core, {wall:.2f} s wall (pool start included)",
            "seconds_per_member_step": {f"{r['n']}^3 seed {r['seed']}": s for r, (_, s) in zip(runs, res)}}
    t = time.perf_counter()
    O.strang_step(psi0_np, w["alpha"], w["beta"], w["dt"])
    dt = time.perf_counter() - t
    npts = float(psi0_np.size)
    sizes = {}
    for n in (32, 64, 96, 128):
        psi = I.tg_psi(n, w["ic"][1]["xi"], w["ic"][1]["exponent"])
        t1 = time.perf_counter()
        O.strang_step(psi, w["alpha"], w["beta"], w["dt"])
        sizes[str(n)] = time.perf_counter() - t1
    sizes["256"] = dt
    # the 1024^3 workload from the 256^3 time under N^3 log N (both FFT-path sizes)
    t1024 = dt * 64.0 * (10.0 / 8.0)
    base = {"value": npts / dt, "unit": "grid-point.steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one literal Strang step (4 3-D FFTs, numpy FP64, single thread) of the 256^3 "
                      f"tg256 field, {dt:.1f} s on {cpu_model()}; diagnostics (1 per 100 steps) not included",
            "seconds": dt, "seconds_per_step_by_n": sizes, "host_cpus": os.cpu_count(),
            "extrapolated_1024": {"seconds_per_step": t1024, "value": 1024.0 ** 3 / t1024,
                                  "rule": "256^3 time x (1024/256)^3 x log2(1024)/log2(256), one core"}}
    base.update(out)
    return base


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed bench steps (100 split steps + diagnostics each)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^3 complex64 HBM-bound form")
    ap.add_argument("--argle", action="store_true",
                    help="profiling mode: time only the 256^3 imaginary-time preparation, print its JSON, exit")
    ap.add_argument("--passes", default=None, metavar="N:PREC",
                    help="profiling mode: time each axis pass alone on an N^3 field (PREC c128|c64) "
                         "and one device copy of the same bytes, then exit")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--tune", action="store_true", help="with --passes: autotune the schedules first")
    ap.add_argument("--rotating", action="store_true", help="with --passes: the layout-rotating passes")
    ap.add_argument("--variants", default=None, metavar="VX,VY,VZ",
                    help="with --passes: schedule variant of each axis (as reported by a timed run)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU "
              "decomposition is a design, not a built path", file=sys.stderr)
        return 2

    import numpy as np

    import gp_inputs as I

    cpu = None
    if not (a.passes or a.argle or a.no_cpu_baseline):
        # the CPU oracle first: its process pool forks before the GPU runtime is loaded
        wb = I.WORKLOADS[WORKLOAD]
        cpu = oracle_sample(I.tg_psi(wb["n"], wb["ic"][1]["xi"], wb["ic"][1]["exponent"]), wb)

    import torch

    import paper_2003_03590_amd as gp

    if a.passes:
        return passes_mode(gp, torch, a.passes, a.reps, tune=a.tune, variants=a.variants, rotating=a.rotating)
    if a.argle:
        print(json.dumps(argle_form(gp, torch, I)))
        return 0

    w = I.WORKLOADS[WORKLOAD]
    n = w["n"]
    xi, expo = w["ic"][1]["xi"], w["ic"][1]["exponent"]
    psi0 = I.tg_psi(n, xi, expo)
    npts = float(n) ** 3

    f64 = run_form(gp, torch, psi0, w, "c128", a.steps, a.warmup, tune=not a.no_tune)
    split_steps = a.steps * DIAG_EVERY
    value = npts * split_steps / f64["wall"]
    step_only = npts * split_steps / (sum(f64["step_ms"]) / 1e3)
    S = 16
    bytes_per_pass = 2.0 * npts * S
    achieved = bytes_per_pass / (f64["mean_pass_ms"] / 1e3) / 1e9

    res = {
        "metric": "grid-point.steps/s (Strang split step incl. diagnostics every 100 steps)",
        "value": value,
        "unit": "grid-point.steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": f64["wall"] / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Taylor-Green ansatz, seedless closed form)",
        "config": {"workload": "tg256: 256^3 Taylor-Green ansatz psi_4^2, xi=2*(2pi/256), alpha=0.069420, "
                               "beta=28.810, dt=5e-4, 1000 steps, energy split + shell spectra every 100 steps",
                   "grid": [n, n, n], "prec": "complex128", "split_steps_timed": split_steps,
                   "workload_runs_timed": split_steps / w["steps"],
                   "bench_step": "100 Strang steps + gp_spectra; every 10 bench steps the workload "
                                 "restarts from its initial condition"},
        "value_step_only": step_only,
        "hbm_gbs_per_split_step": 6.0 * npts * S / (sum(f64["step_ms"]) / 1e3 / split_steps) / 1e9,
        "bytes_per_split_step_min": 6.0 * npts * S,
        "roofline_tg256_c128": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "cache_resident": "the 256 MiB state fits the 256 MB last-level cache; the HBM-bound "
                                       "form (the line's roofline) is the 1024^3 complex64 pass",
                     "traffic": pass_traffic(schedules=[f64["plan"].schedule(ax) for ax in range(3)]),
                     "kernel": "axis_pass (propagator; the nonlinear rotation fused into the carrier axis's pass), "
                               "mean of the three",
                     "per_launch_bytes": bytes_per_pass, "mean_launch_us": f64["mean_pass_ms"] * 1e3},
        "drift_f64": {"dE": f64["dE"], "dN": f64["dN"]},
        "schedule": [f64["plan"].schedule(ax) for ax in range(6)],
    }
    res["literal_form"] = literal_form(torch, f64["plan"], psi0, sum(f64["step_ms"]) / split_steps)
    if not a.no_fp32:
        f32 = run_form(gp, torch, psi0, w, "c64", a.steps, a.warmup, tune=not a.no_tune)
        v32 = npts * split_steps / f32["wall"]
        rel = float(np.linalg.norm(f32["psi"] - f64["psi"]) / np.linalg.norm(f64["psi"]))
        ach32 = 2.0 * npts * 8 / (f32["mean_pass_ms"] / 1e3) / 1e9
        res["fp32"] = {"value": v32, "ms_per_step": f32["wall"] / a.steps * 1e3, "speedup_vs_f64": v32 / value,
                       "value_step_only": npts * split_steps / (sum(f32["step_ms"]) / 1e3),
                       "dE": f32["dE"], "dN": f32["dN"], "rel_l2_psi_vs_f64_gpu": rel,
                       "axis_pass_gbs": ach32, "axis_pass_frac": ach32 / HBM_PEAK_GBS,
                       "mean_launch_us": f32["mean_pass_ms"] * 1e3,
                       "schedule": [f32["plan"].schedule(ax) for ax in range(6)]}
    if not a.no_ensemble:
        res["ensemble"] = ensemble_form(gp, torch, I)
    if not a.no_large:
        res["large_1024_c64"] = large_form(gp, torch, I)
        # the HBM roofline: the axis pass on a state 32x the last-level cache
        res["roofline"] = dict(res["large_1024_c64"]["roofline"],
                               workload="rvr1024: 1024^3 complex64, timed inside large_1024_c64")
    else:
        res["roofline"] = res["roofline_tg256_c128"]
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
