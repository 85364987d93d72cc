"""Writes the oracle fixtures of the long workloads (test infrastructure).

Every stored value comes from ``oracle/`` run on inputs from ``gp_inputs/``;
nothing else is imported.  The runs are the oracle's literal Strang step in
complex128 (time-evolution section, eq. adi_looptime) and its diagnostics
(energy-decomposition and spectra sections; density structure function of the
structure-function section).  To make runs of hours finish in reasonable wall
time, each 1-D FFT (lengths above 64) of a full 3-D field is split over a pool of
processes (independent pencils, each process calling the oracle's own
``transform_axis``),
and initial fields are built slab by slab; both leave every value unchanged
(``--selftest`` checks this bit for bit on small grids).

Fixtures (``tests/golden/oracle_<name>.npz``):

* ``tg256``  -- 256^3 Taylor-Green ansatz, 1000 steps of dt = 5e-4, every 100
  steps: mass, energy and its split, shell spectra, and psi on six pencils;
* ``rvr256`` -- the 40-pair random-vortex-ring construction at 256^3 (core width
  three grid spacings), 500 steps of dt = 2.5e-4, every 50 steps: the same
  diagnostics, the density structure function, psi on six pencils;
* ``ens48``  -- the 48 smoothed-random-phase ensemble members (complex64-rounded
  start, as the complex64 runs see it), 300 steps of dt = 1e-3: mass and energy
  every 50 steps and psi on six pencils at the end;
* ``tg256_libfft``, ``rvr256_libfft`` -- the first two runs again with every
  transform done by the library FFT (``oracle.fft.library_engine``), psi on the
  same pencils at every checkpoint: two correct FP64 implementations side by
  side, whose distance is the complex128 parity floor of the long runs.

Usage: python tests/golden/make_oracle_runs.py
       {tg256,rvr256,ens48,tg256-libfft,rvr256-libfft,--selftest}
       [--workers P] [--save-dir DIR]
``--save-dir`` keeps the full state at every checkpoint (for resuming: an
interrupted run restarts from the last saved state).
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time
from multiprocessing import shared_memory

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gp_inputs as I                      # noqa: E402
from oracle import fft as OF, gp as O      # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SCALARS = ("mass", "energy", "e_kin", "e_kin_i", "e_kin_c", "e_q", "e_int")

# --------------------------------------------------------------- process pool
_W = {}


def _attach(name_in, name_out, shape):
    _W["in"] = shared_memory.SharedMemory(name=name_in)
    _W["out"] = shared_memory.SharedMemory(name=name_out)
    _W["a"] = np.ndarray(shape, np.complex128, buffer=_W["in"].buf)
    _W["b"] = np.ndarray(shape, np.complex128, buffer=_W["out"].buf)


def _transform_chunk(axis, sign, split, lo, hi):
    sl = [slice(None)] * 3
    sl[split] = slice(lo, hi)
    sl = tuple(sl)
    _W["b"][sl] = OF.transform_axis(_W["a"][sl], axis, sign)
    return hi - lo


def _rvr_chunk(n, xi, n_pairs, seed, lo, hi):
    _W["b"][lo:hi] = I.rvr_psi(n, xi, n_pairs, seed, zslab=(lo, hi))
    return hi - lo


def _ranges(n, parts):
    cuts = [round(i * n / parts) for i in range(parts + 1)]
    return [(cuts[i], cuts[i + 1]) for i in range(parts) if cuts[i + 1] > cuts[i]]


class PoolEngine:
    """Callable transform engine for the oracle: splits the pencils of one 1-D
    transform of a full field over ``workers`` processes."""

    def __init__(self, shape, workers):
        self.shape = tuple(shape)
        nbytes = int(np.prod(shape)) * 16
        self.shm_in = shared_memory.SharedMemory(create=True, size=nbytes)
        self.shm_out = shared_memory.SharedMemory(create=True, size=nbytes)
        self.a = np.ndarray(self.shape, np.complex128, buffer=self.shm_in.buf)
        self.b = np.ndarray(self.shape, np.complex128, buffer=self.shm_out.buf)
        self.workers = workers
        self.pool = mp.get_context("fork").Pool(
            workers, initializer=_attach, initargs=(self.shm_in.name, self.shm_out.name, self.shape))

    def __call__(self, a, axis, sign):
        # the dense-DFT engine (n <= 64) is a BLAS product whose rounding depends
        # on the memory layout, so only the FFT engine's lengths are pooled
        if tuple(np.shape(a)) != self.shape or self.shape[axis] <= OF.NAIVE_MAX:
            return OF.transform_axis(a, axis, sign)
        self.a[...] = a
        split = (axis + 1) % 3
        jobs = [(axis, sign, split, lo, hi) for lo, hi in _ranges(self.shape[split], self.workers)]
        self.pool.starmap(_transform_chunk, jobs)
        return np.array(self.b)

    def rvr(self, n, xi, n_pairs, seed):
        jobs = [(n, xi, n_pairs, seed, lo, hi) for lo, hi in _ranges(n, self.workers)]
        self.pool.starmap(_rvr_chunk, jobs)
        return np.array(self.b)

    def close(self):
        self.pool.close()
        self.pool.join()
        for s in (self.shm_in, self.shm_out):
            s.close()
            s.unlink()


# --------------------------------------------------------------- helpers
def pencil_positions(n, per_axis=2, seed=20260):
    """(array axis, i, j) of the stored pencils: ``per_axis`` per axis."""
    rng = np.random.default_rng(seed)
    out = []
    for axis in (2, 1, 0):
        for _ in range(per_axis):
            i, j = (int(v) for v in rng.integers(0, n, 2))
            out.append((axis, i, j))
    return np.array(out, dtype=np.int64)


def take_pencil(psi, axis, i, j):
    if axis == 2:
        return psi[i, j, :]
    if axis == 1:
        return psi[i, :, j]
    return psi[:, i, j]


def _save(path, **arrays):
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, **arrays)
    os.replace(tmp, path)


def _state_path(save_dir, name, step):
    return os.path.join(save_dir, f"{name}_step{step:05d}.npy")


# --------------------------------------------------------------- long runs
def run_field(name, workers, save_dir):
    w = I.WORKLOADS[name]
    n, alpha, beta, dt, steps, every = w["n"], w["alpha"], w["beta"], w["dt"], w["steps"], w["diag_every"]
    kind, ic = w["ic"]
    eng = PoolEngine((n, n, n), workers)
    t0 = time.time()
    pos = pencil_positions(n)
    checks = list(range(0, steps + 1, every))
    rec = {"steps": np.array(checks), "scalars": np.full((len(checks), len(SCALARS)), np.nan),
           "spec": np.full((len(checks), 4, O.nshell((n, n, n))), np.nan),
           "pencils": np.full((len(checks), len(pos), n), np.nan + 0j),
           "pencil_pos": pos, "done": np.array(0)}
    if kind == "rvr":
        rec["sf"] = np.full((len(checks), n // 2), np.nan)
    out = os.path.join(HERE, f"oracle_{name}.npz")

    start, psi = 0, None
    if save_dir:
        saved = [c for c in checks if os.path.exists(_state_path(save_dir, name, c))]
        if saved and os.path.exists(out):
            start = max(saved)
            psi = np.load(_state_path(save_dir, name, start))
            old = np.load(out)
            for k in rec:
                if k in old.files:
                    rec[k] = old[k]
            print(f"{name}: resuming from step {start}", flush=True)
    if psi is None:
        if kind == "tg":
            psi = I.tg_psi(n, ic["xi"], ic["exponent"])
        else:
            psi = eng.rvr(n, ic["xi"], ic["n_pairs"], ic["seed"])
        print(f"{name}: initial field built ({time.time() - t0:.0f} s)", flush=True)

    def record(step, field):
        c = checks.index(step)
        d = O.diagnostics(field, alpha, beta, eng)
        rec["scalars"][c] = [d[k] for k in SCALARS]
        rec["spec"][c] = d["spec"]
        for p, (axis, i, j) in enumerate(pos):
            rec["pencils"][c, p] = take_pencil(field, axis, i, j)
        if kind == "rvr":
            rec["sf"][c] = O.structure_function_density(field)
        if save_dir:
            np.save(_state_path(save_dir, name, step), field)
        _save(out, **rec)
        print(f"{name}: step {step} E = {d['energy']:.15e} N = {d['mass']:.15e} "
              f"({time.time() - t0:.0f} s)", flush=True)

    if start == 0:
        record(0, psi)
    for blk_start in range(start, steps, every):
        psi = O.evolve(psi, alpha, beta, dt, every, engine=eng)
        record(blk_start + every, psi)
    rec["done"] = np.array(1)
    _save(out, **rec)
    eng.close()
    print(f"{name}: done in {time.time() - t0:.0f} s", flush=True)


def run_field_library(name, workers):
    """The same FP64 run with the oracle's transforms done by the library FFT
    (``oracle.fft.library_engine``): psi on the same pencils at every checkpoint.
    Against ``oracle_<name>.npz`` it measures how far two correct FP64
    implementations drift apart over the run (the complex128 parity floor)."""
    w = I.WORKLOADS[name]
    n, alpha, beta, dt, steps, every = w["n"], w["alpha"], w["beta"], w["dt"], w["steps"], w["diag_every"]
    kind, ic = w["ic"]
    t0 = time.time()
    pos = pencil_positions(n)
    checks = list(range(0, steps + 1, every))
    rec = {"steps": np.array(checks), "pencils": np.full((len(checks), len(pos), n), np.nan + 0j),
           "pencil_pos": pos, "done": np.array(0)}
    out = os.path.join(HERE, f"oracle_{name}_libfft.npz")
    if kind == "tg":
        psi = I.tg_psi(n, ic["xi"], ic["exponent"])
    else:
        gen = PoolEngine((n, n, n), workers)
        psi = gen.rvr(n, ic["xi"], ic["n_pairs"], ic["seed"])
        gen.close()
    eng = OF.library_engine(workers)
    for c, step in enumerate(checks):
        if step:
            psi = O.evolve(psi, alpha, beta, dt, every, engine=eng)
        for p, (axis, i, j) in enumerate(pos):
            rec["pencils"][c, p] = take_pencil(psi, axis, i, j)
        _save(out, **rec)
        print(f"{name} (library FFT): step {step} ({time.time() - t0:.0f} s)", flush=True)
    rec["done"] = np.array(1)
    _save(out, **rec)


def _ens_member(args):
    r, dt, steps, every, K = args
    n = r["n"]
    psi0 = np.exp(1j * I.srp_fourier_theta(n, K, r["seed"])).astype(np.complex64).astype(np.complex128)
    pos = pencil_positions(n, seed=20260 + r["seed"])
    hist = []

    def cb(step, psi):
        hist.append((O.mass(psi), O.energy(psi, r["alpha"], r["beta"])))

    end = O.evolve(psi0, r["alpha"], r["beta"], dt, steps, callback=cb, every=every)
    pens = np.array([take_pencil(end, a, i, j) for a, i, j in pos])
    return np.array(hist), pos, pens


def run_ensemble(workers):
    w = I.WORKLOADS["ens48"]
    t0 = time.time()
    jobs = [(r, w["dt"], w["steps"], w["diag_every"], w["K"]) for r in w["runs"]]
    with mp.get_context("fork").Pool(workers) as pool:
        res = []
        for k, r in enumerate(pool.imap(_ens_member, jobs)):
            res.append(r)
            print(f"ens48: run {k} done ({time.time() - t0:.0f} s)", flush=True)
    rec = {"seeds": np.array([r["seed"] for r in w["runs"]]),
           "energies": np.array([h for h, _, _ in res]),           # [run][check][mass, energy]
           "steps": np.arange(0, w["steps"] + 1, w["diag_every"]), "done": np.array(1)}
    for k, (_, pos, pens) in enumerate(res):
        rec[f"pos{k}"] = pos
        rec[f"pen{k}"] = pens
    _save(os.path.join(HERE, "oracle_ens48.npz"), **rec)
    print(f"ens48: done in {time.time() - t0:.0f} s", flush=True)


def selftest(workers):
    """The pooled transform, the slab-built ring field and a pooled Strang step
    equal the serial oracle bit for bit."""
    for n in (48, 96, 128):
        # 48: every transform falls back to the serial oracle (dense DFT)
        a = I.random_field(n, seed=n)
        eng = PoolEngine((n, n, n), workers)
        for axis in range(3):
            for sign in (-1, 1):
                assert np.array_equal(eng(a, axis, sign), OF.transform_axis(a, axis, sign)), (n, axis, sign)
        s1 = O.strang_step(a, 0.1, 20.0, 1e-3, eng)
        s0 = O.strang_step(a, 0.1, 20.0, 1e-3)
        assert np.array_equal(s1, s0), n
        d1, d0 = O.diagnostics(s1, 0.1, 20.0, eng), O.diagnostics(s0, 0.1, 20.0)
        assert all(d1[k] == d0[k] for k in SCALARS) and np.array_equal(d1["spec"], d0["spec"])
        r1 = eng.rvr(n, 0.2, 3, 1)
        assert np.array_equal(r1, I.rvr_psi(n, 0.2, 3, 1)), n
        eng.close()
        print(f"selftest {n}^3: pooled == serial", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["tg256", "rvr256", "ens48", "tg256-libfft", "rvr256-libfft",
                                     "--selftest", "selftest"])
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--save-dir", default="")
    a = ap.parse_args()
    if a.save_dir:
        os.makedirs(a.save_dir, exist_ok=True)
    if a.what in ("--selftest", "selftest"):
        selftest(a.workers)
    elif a.what == "ens48":
        run_ensemble(a.workers)
    elif a.what.endswith("-libfft"):
        run_field_library(a.what[:-len("-libfft")], a.workers)
    else:
        run_field(a.what, a.workers, a.save_dir)


if __name__ == "__main__":
    main()
