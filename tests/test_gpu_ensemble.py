"""Ensemble (batch) plans against the oracle and against single-grid plans:
backward steps, the largest ensemble lengths (96 with radix-3 stages, 128), and
stream ordering with the caller's stream (states written and read on torch's
stream around a long ensemble launch with no explicit synchronisation).

Two tests here belong to a persistent work-queue form of the ensemble step (one
launch per size group pulling (run, pass, tile) items, the groups on parallel
graph branches).  That form did not complete its first launch on the MI355X
(twice, the second time with every in-kernel wait bounded in time), so it is
switched off and its tests are skipped; the ensemble runs as a graph of grouped
pass launches."""
import numpy as np
import pytest

import gp_inputs as I
from oracle import gp as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(a, prec):
    t = torch.from_numpy(a).to(DEV)
    return (t if prec == "c128" else t.to(torch.complex64)).contiguous()


PERSISTENT_OFF = ("the persistent work-queue ensemble form did not complete its first launch on the "
                  "MI355X (five size groups on parallel graph branches); the form is switched off")


@pytest.mark.skip(reason=PERSISTENT_OFF)
@pytest.mark.parametrize("xy", [0, 1])
def test_ensemble_kinds_match_oracle(xy):
    """Five sizes in one batch (N = 12 has a ragged last tile), complex128, both
    kinds; step counts 1, 4, 2 in a row (one recorded graph, the step count is a
    launch parameter) against the oracle's literal steps."""
    import paper_2003_03590_amd as gp
    runs = [dict(n=12, alpha=0.4, beta=2.0, dt=0.01), dict(n=16, alpha=0.3, beta=3.0, dt=0.01),
            dict(n=24, alpha=0.5, beta=1.0, dt=0.02), dict(n=32, alpha=0.2, beta=3.0, dt=0.01),
            dict(n=16, alpha=0.6, beta=1.5, dt=0.01), dict(n=8, alpha=0.3, beta=2.0, dt=0.02)]
    bp = gp.BatchPlan(runs, "c128")
    bp.select_xy(xy)
    names = bp.schedules()
    assert len(names) == 5
    if xy:
        assert any(" plane " in nm for nm in names) and any(" xyz " in nm for nm in names)
    refs = [I.random_field(r["n"], seed=200 + i) for i, r in enumerate(runs)]
    states = [_dev(a, "c128") for a in refs]
    for nsteps in (1, 4, 2):
        bp.step_n(states, nsteps)
        for i, r in enumerate(runs):
            refs[i] = O.evolve(refs[i], r["alpha"], r["beta"], r["dt"], nsteps)
            assert _rel(states[i].cpu().numpy(), refs[i]) < 1e-12, (xy, nsteps, i, names)
    bp.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_ensemble_backward_steps_reverse(prec):
    import paper_2003_03590_amd as gp
    runs = [dict(n=48, alpha=0.2, beta=3.0, dt=0.01), dict(n=64, alpha=0.1, beta=20.0, dt=1e-3),
            dict(n=48, alpha=0.3, beta=2.0, dt=0.01)]
    bp = gp.BatchPlan(runs, prec)
    init = [I.random_field(r["n"], seed=300 + i) for i, r in enumerate(runs)]
    states = [_dev(a, prec) for a in init]
    bp.step_n(states, 5)
    bp.step_n(states, -5)
    tol = 1e-12 if prec == "c128" else 1e-5
    for i, a in enumerate(init):
        base = a if prec == "c128" else a.astype(np.complex64).astype(np.complex128)
        assert _rel(states[i].to(torch.complex128).cpu().numpy(), base) < tol
    # backward alone equals the oracle's steps of -dt
    states = [_dev(a, prec) for a in init]
    bp.step_n(states, -3)
    for i, r in enumerate(runs):
        base = init[i] if prec == "c128" else init[i].astype(np.complex64).astype(np.complex128)
        ref = O.evolve(base, r["alpha"], r["beta"], r["dt"], -3)
        assert _rel(states[i].to(torch.complex128).cpu().numpy(), ref) < (1e-12 if prec == "c128" else 3e-6)
    bp.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_ensemble_matches_single_plans_96_128(prec):
    """The largest ensemble lengths (96 with radix-3 stages, 128) against
    single-grid plans of the same runs."""
    import paper_2003_03590_amd as gp
    runs = [dict(n=96, alpha=6.4 / 96, beta=30.0, dt=1e-3), dict(n=128, alpha=0.05, beta=40.0, dt=1e-3),
            dict(n=96, alpha=6.4 / 96, beta=30.0, dt=1e-3)]
    bp = gp.BatchPlan(runs, prec)
    init = [I.random_field(r["n"], seed=400 + i, amp_noise=0.1) for i, r in enumerate(runs)]
    states = [_dev(a, prec) for a in init]
    bp.step_n(states, 6)
    for i, r in enumerate(runs):
        p = gp.Plan(r["n"], r["alpha"], r["beta"], r["dt"], "c128")
        ref = _dev(init[i] if prec == "c128" else init[i].astype(np.complex64).astype(np.complex128), "c128")
        p.step_n(ref, 6)
        rel = float(torch.linalg.vector_norm(states[i].to(torch.complex128) - ref) / torch.linalg.vector_norm(ref))
        assert rel < (1e-12 if prec == "c128" else 2e-6), (prec, i, rel)
        p.close()
    bp.close()


def test_ensemble_step_lengths_compose_from_recorded_graphs():
    """A call of n steps launches the recorded graphs of the opening half step, the
    body's n - 1 applications by binary digits (up to 128 per graph) and the
    closing half step: lengths 1, 2, 3, 130 and 257 forward and -5 backward, on
    three size groups (three capture branches), against single-grid plans."""
    import paper_2003_03590_amd as gp
    runs = [dict(n=32, alpha=0.2, beta=10.0, dt=1e-3), dict(n=48, alpha=6.4 / 48, beta=15.0, dt=1e-3),
            dict(n=32, alpha=0.2, beta=10.0, dt=1e-3), dict(n=64, alpha=0.1, beta=20.0, dt=1e-3)]
    bp = gp.BatchPlan(runs, "c128")
    init = [I.random_field(r["n"], seed=600 + i, amp_noise=0.1) for i, r in enumerate(runs)]
    states = [_dev(a, "c128") for a in init]
    refs = [_dev(a, "c128") for a in init]
    plans = [gp.Plan(r["n"], r["alpha"], r["beta"], r["dt"], "c128") for r in runs]
    for n in (1, 2, 3, 130, 257, -5):
        bp.step_n(states, n)
        for p, ref in zip(plans, refs):
            p.step_n(ref, n)
        torch.cuda.synchronize()
        for i in range(len(runs)):
            rel = float(torch.linalg.vector_norm(states[i] - refs[i]) / torch.linalg.vector_norm(refs[i]))
            assert rel < 1e-12, (n, i, rel)
    for p in plans:
        p.close()
    bp.close()


def test_ensemble_orders_with_the_callers_stream():
    """States written by torch on the current stream just before the call, and read
    right after a long ensemble launch, with no explicit synchronisation: the
    ensemble's own stream waits for the caller's stream and the caller's stream
    waits for the launch."""
    import paper_2003_03590_amd as gp
    runs = [dict(n=64, alpha=0.1, beta=20.0, dt=1e-3) for _ in range(8)] + \
           [dict(n=96, alpha=6.4 / 96, beta=30.0, dt=1e-3) for _ in range(4)]
    bp = gp.BatchPlan(runs, "c64")
    init = [_dev(I.random_field(r["n"], seed=500 + i, amp_noise=0.1), "c64") for i, r in enumerate(runs)]
    torch.cuda.synchronize()
    states = [torch.empty_like(x) for x in init]
    for s, x in zip(states, init):
        s.copy_(x)                      # enqueued on torch's stream, not waited for
    bp.step_n(states, 200)
    got = [s.cpu() for s in states]     # enqueued on torch's stream right after the launch
    for i, r in enumerate(runs):
        p = gp.Plan(r["n"], r["alpha"], r["beta"], r["dt"], "c64")
        ref = init[i].clone()
        p.step_n(ref, 200)
        rel = float(torch.linalg.vector_norm((got[i].to(DEV) - ref).to(torch.complex128))
                    / torch.linalg.vector_norm(ref.to(torch.complex128)))
        assert rel < 2e-5, (i, rel)
        p.close()
    bp.close()


@pytest.mark.skip(reason=PERSISTENT_OFF + " (the grouped form accepts every supported shape)")
def test_ensemble_rejects_unsupported_shapes():
    import paper_2003_03590_amd as gp
    from paper_2003_03590_amd import _lib as L
    for runs in ([dict(n=(16, 16, 8), alpha=0.3, beta=2.0, dt=0.01)],
                 [dict(n=16, alpha=0.3, beta=2.0, dt=0.01), dict(n=256, alpha=0.3, beta=2.0, dt=0.01)]):
        with pytest.raises(gp.GPError) as ei:
            gp.BatchPlan(runs, "c64")
        assert ei.value.status == L.GP_ERR_UNSUPPORTED
