"""MI355X-native Gross-Pitaevskii split step (arXiv:2003.03590).

Thin Python binding over the C ABI of ``include/gp.h``: every step of the
method runs in the gfx950 HIP kernels of ``libgp_mi355x.so``; PyTorch only
provides device memory and the stream.  The raw C functions are reachable as
``paper_2003_03590_amd.lib().gp_*``; ``Plan``/``BatchPlan`` marshal torch
tensors into them, and ``evolve``/``ekin_i_shells`` expose the adjoint through
``torch.autograd``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import GPError, GP_C128, GP_C64, gp_argle_report, gp_desc, gp_energy

__all__ = ["lib", "Plan", "BatchPlan", "evolve", "ekin_i_shells", "GPError", "GP_C128", "GP_C64"]

_LIB = None


def lib() -> C.CDLL:
    """The loaded C library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        _LIB = _lib.load()
    return _LIB


def _check(status: int) -> None:
    if status != _lib.GP_OK:
        raise GPError(status, lib().gp_last_error().decode())


def _torch():
    import torch
    return torch


def _prec_code(prec) -> int:
    if prec in ("c128", "complex128", GP_C128):
        return GP_C128
    if prec in ("c64", "complex64", GP_C64):
        return GP_C64
    raise ValueError(f"unknown precision {prec!r}")


def _ptr(t) -> int:
    return t.data_ptr()


class Plan:
    """One grid.  ``n`` = N or (Nx, Ny, Nz); fields are torch tensors of shape
    (Nz, Ny, Nx) (x contiguous) on the plan's device."""

    def __init__(self, n, alpha: float, beta: float, dt: float, prec="c128", device=None, stream=None):
        torch = _torch()
        if isinstance(n, int):
            n = (n, n, n)
        self.n = tuple(int(v) for v in n)
        self.alpha, self.beta, self.dt = float(alpha), float(beta), float(dt)
        self.prec = _prec_code(prec)
        self.dtype = torch.complex128 if self.prec == GP_C128 else torch.complex64
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        d = gp_desc((C.c_int32 * 3)(*self.n), self.alpha, self.beta, self.dt, self.prec, 0)
        h = C.c_void_p()
        _check(lib().gp_plan(C.byref(d), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.nshell = int(lib().gp_nshell(h))
        self._work = None
        self._hwork = None

    # ---------------------------------------------------------------- plumbing
    def close(self):
        if getattr(self, "_h", None):
            lib().gp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    def empty(self):
        return _torch().empty(self.shape, dtype=self.dtype, device=self.device)

    def work(self):
        if self._work is None:
            nb = int(lib().gp_work_bytes(self._h))
            self._work = _torch().empty(nb, dtype=_torch().uint8, device=self.device)
        return self._work

    def _field(self, t, name="psi"):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.dtype != self.dtype or tuple(t.shape) != self.shape \
                or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {self.shape} on {self.device}")
        return C.c_void_p(_ptr(t))

    def schedule(self, axis: int) -> str:
        return lib().gp_schedule_name(self._h, axis).decode()

    def select_variant(self, axis: int, variant: int):
        _check(lib().gp_select_variant(self._h, axis, variant))

    def autotune(self, reps: int = 5, cache: str | None = None):
        """Time every compiled schedule of each axis and keep the fastest."""
        scratch = _torch().zeros(self.shape, dtype=self.dtype, device=self.device)
        _check(lib().gp_autotune(self._h, C.c_void_p(_ptr(scratch)), int(reps),
                                 cache.encode() if cache else None))
        return [self.schedule(a) for a in range(6)]

    # ---------------------------------------------------------------- method
    def init_phase(self, theta, out=None):
        torch = _torch()
        theta = theta.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(theta.shape) != self.shape:
            raise ValueError("theta shape")
        psi = self.empty() if out is None else out
        _check(lib().gp_init_phase(self._h, C.c_void_p(_ptr(theta)), self._field(psi)))
        return psi

    def init_rvr(self, pairs, xi: float, out=None):
        """Random vortex-ring pairs: ``pairs`` is a sequence of (R, d, X, Y, Z, perm)."""
        arr = np.ascontiguousarray(np.asarray(pairs, dtype=np.float64).reshape(-1, 6))
        psi = self.empty() if out is None else out
        _check(lib().gp_init_rvr(self._h, arr.ctypes.data_as(C.POINTER(C.c_double)), int(arr.shape[0]),
                                 float(xi), self._field(psi)))
        return psi

    def step_n(self, psi, nsteps: int):
        _check(lib().gp_step_n(self._h, self._field(psi), int(nsteps)))
        return psi

    def step_literal_n(self, psi, nsteps: int):
        _check(lib().gp_step_literal_n(self._h, self._field(psi), int(nsteps)))
        return psi

    def substep_linear(self, psi, axis: int, s: float):
        _check(lib().gp_substep_linear(self._h, self._field(psi), int(axis), float(s)))
        return psi

    def substep_nonlinear(self, psi, s: float):
        _check(lib().gp_substep_nonlinear(self._h, self._field(psi), float(s)))
        return psi

    def fft3(self, x, direction: int = -1, out=None):
        out = self.empty() if out is None else out
        _check(lib().gp_fft3(self._h, self._field(x, "in"), self._field(out, "out"), int(direction)))
        return out

    def copy_state(self, src, out=None):
        """Plain device copy of one state (the bandwidth reference of the passes)."""
        out = self.empty() if out is None else out
        _check(lib().gp_copy_state(self._h, self._field(src, "in"), self._field(out, "out")))
        return out

    def energies(self, psi) -> dict:
        e = gp_energy()
        _check(lib().gp_energies(self._h, self._field(psi), C.c_void_p(_ptr(self.work())), C.byref(e)))
        return e.as_dict()

    def _velocity(self, v):
        """v: (3, Nz, Ny, Nx) real tensor, components (v_x, v_y, v_z), in the plan's
        real precision on its device."""
        torch = _torch()
        rdt = torch.float64 if self.prec == GP_C128 else torch.float32
        v = v.to(device=self.device, dtype=rdt).contiguous()
        if tuple(v.shape) != (3,) + tuple(self.shape):
            raise ValueError(f"velocity must have shape {(3,) + tuple(self.shape)}")
        return v

    def argle_step(self, phi, v, dtau: float, nsteps: int):
        """nsteps imaginary-time (ARGLE) steps of phi in place; v as in _velocity."""
        v = self._velocity(v)
        _check(lib().gp_argle_step(self._h, self._field(phi, "phi"), C.c_void_p(v.data_ptr()), float(dtau),
                                   int(nsteps), C.c_void_p(_ptr(self.work()))))
        return phi

    def argle_energy(self, phi, v) -> float:
        """Driven energy E_v per unit volume."""
        v = self._velocity(v)
        out = C.c_double()
        _check(lib().gp_argle_energy(self._h, self._field(phi, "phi"), C.c_void_p(v.data_ptr()),
                                     C.c_void_p(_ptr(self.work())), C.byref(out)))
        return out.value

    def argle_run(self, phi, v, dtau: float, max_steps: int, check_every: int = 100, eps: float = 0.0) -> dict:
        """The ARGLE procedure with its stopping rule: steps until
        ||phi^{n+1} - phi^n||_inf / dtau <= eps at a check (every check_every steps
        and the last step) or max_steps steps.  Returns steps, crit_sup, crit_energy,
        e_v and converged of the last check."""
        v = self._velocity(v)
        r = gp_argle_report()
        _check(lib().gp_argle_run(self._h, self._field(phi, "phi"), C.c_void_p(v.data_ptr()), float(dtau),
                                  int(max_steps), int(check_every), float(eps), C.c_void_p(_ptr(self.work())),
                                  C.byref(r)))
        out = r.as_dict()
        out["converged"] = bool(out["converged"])
        return out

    def spectra(self, psi):
        out = np.zeros((4, self.nshell), dtype=np.float64)
        e = gp_energy()
        _check(lib().gp_spectra(self._h, self._field(psi), C.c_void_p(_ptr(self.work())),
                                out.ctypes.data_as(C.POINTER(C.c_double)), self.nshell, C.byref(e)))
        return out, e.as_dict()

    def structure_fn(self, psi, p_order: int = 2):
        out = np.zeros(self.n[0] // 2, dtype=np.float64)
        _check(lib().gp_structure_fn(self._h, self._field(psi), C.c_void_p(_ptr(self.work())), int(p_order),
                                     out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def structure_fn_velocity(self, psi, p_order: int = 2):
        """Longitudinal velocity structure functions per axis: (S [3][N/2] in the
        order x, y, z, <v_j^2> [3])."""
        half = self.n[0] // 2
        out = np.zeros((3, half), dtype=np.float64)
        mv2 = np.zeros(3, dtype=np.float64)
        _check(lib().gp_structure_fn_velocity(self._h, self._field(psi), C.c_void_p(_ptr(self.work())), int(p_order),
                                              out.ctypes.data_as(C.POINTER(C.c_double)),
                                              mv2.ctypes.data_as(C.POINTER(C.c_double))))
        return out, mv2

    def helicity(self, psi, spectra: bool = True):
        """(H, H_reg) per unit volume and, with `spectra`, their shell spectra [2][nshell].
        Uses a workspace of gp_helicity_work_bytes (8 states), allocated on first use."""
        if self._hwork is None:
            nb = int(lib().gp_helicity_work_bytes(self._h))
            self._hwork = _torch().empty(nb, dtype=_torch().uint8, device=self.device)
        out = np.zeros(2, dtype=np.float64)
        spec = np.zeros((2, self.nshell), dtype=np.float64) if spectra else None
        _check(lib().gp_helicity(self._h, self._field(psi), C.c_void_p(_ptr(self._hwork)),
                                 out.ctypes.data_as(C.POINTER(C.c_double)),
                                 spec.ctypes.data_as(C.POINTER(C.c_double)) if spectra else None,
                                 self.nshell))
        return (float(out[0]), float(out[1]), spec) if spectra else (float(out[0]), float(out[1]))

    def mach(self, psi):
        """(M_max, M_rms)."""
        out = np.zeros(2, dtype=np.float64)
        _check(lib().gp_mach(self._h, self._field(psi), C.c_void_p(_ptr(self.work())),
                             out.ctypes.data_as(C.POINTER(C.c_double))))
        return float(out[0]), float(out[1])

    def loss_ekin_i_shells(self, psi, smin: int, smax: int, lam=None):
        lam = self.empty() if lam is None else lam
        J = C.c_double()
        _check(lib().gp_loss_ekin_i_shells(self._h, self._field(psi), C.c_void_p(_ptr(self.work())), int(smin),
                                           int(smax), C.byref(J), self._field(lam, "lam")))
        return J.value, lam

    def adjoint_step_n(self, psi_start, lam, nsteps: int, tape=None):
        torch = _torch()
        if tape is None or tape.numel() * tape.element_size() < nsteps * self.state_bytes():
            tape = torch.empty(max(1, nsteps) * self.state_bytes(), dtype=torch.uint8, device=self.device)
        _check(lib().gp_adjoint_step_n(self._h, self._field(psi_start), self._field(lam, "lam"), int(nsteps),
                                       C.c_void_p(_ptr(tape))))
        return lam, tape

    def phase_grad(self, psi0, lam0, out=None):
        torch = _torch()
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device) if out is None else out
        _check(lib().gp_phase_grad(self._h, self._field(psi0), self._field(lam0, "lam0"), C.c_void_p(_ptr(out))))
        return out

    def state_bytes(self) -> int:
        return int(lib().gp_state_bytes(self._h, 0))


class BatchPlan:
    """Ensemble of independent runs (sizes may differ) advanced by recorded HIP
    graphs: one grouped pass launch per size group and pass (runs of one size share
    it, run = second grid dimension), the size groups on parallel graph branches;
    a call of n steps replays the opening, 2^j-step body and closing graphs."""

    def __init__(self, runs, prec="c64", device=None, stream=None):
        torch = _torch()
        self.prec = _prec_code(prec)
        self.dtype = torch.complex128 if self.prec == GP_C128 else torch.complex64
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        descs = (gp_desc * len(runs))()
        self.shapes = []
        for i, r in enumerate(runs):
            n = r["n"]
            n = (n, n, n) if isinstance(n, int) else tuple(n)
            descs[i] = gp_desc((C.c_int32 * 3)(*n), float(r["alpha"]), float(r["beta"]), float(r["dt"]), self.prec, 0)
            self.shapes.append((n[2], n[1], n[0]))
        h = C.c_void_p()
        _check(lib().gp_plan_batch(descs, len(runs), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self._work = None

    def close(self):
        if getattr(self, "_h", None):
            lib().gp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, states):
        torch = _torch()
        if len(states) != len(self.shapes):
            raise ValueError("one state per run")
        for s, shp in zip(states, self.shapes):
            if not isinstance(s, torch.Tensor) or s.dtype != self.dtype or tuple(s.shape) != shp or not s.is_contiguous():
                raise ValueError(f"states must be contiguous {self.dtype} tensors of the run shapes")
        arr = (C.c_void_p * len(states))(*[s.data_ptr() for s in states])
        return arr

    def step_n(self, states, nsteps: int):
        _check(lib().gp_step_n_batch(self._h, self._ptrs(states), int(nsteps)))
        return states

    def schedule(self, run: int, axis: int) -> str:
        """Schedule name of one run's axis (0-2), its xy choice (3), its nonlinear
        carrier (4) or its layout form (5)."""
        return lib().gp_schedule_name(self._h, 6 * int(run) + int(axis)).decode()

    def select_xy(self, variant: int):
        """0: separate x and y passes; 1: one xy-plane pass for every run with a plane
        schedule (the next step call records a new graph)."""
        _check(lib().gp_select_variant(self._h, 3, int(variant)))

    def autotune(self, reps: int = 5, cache: str | None = None):
        """Autotune each size group on a scratch state of the largest run."""
        torch = _torch()
        big = max(self.shapes, key=lambda s: s[0] * s[1] * s[2])
        scratch = torch.zeros(big, dtype=self.dtype, device=self.device)
        _check(lib().gp_autotune(self._h, C.c_void_p(scratch.data_ptr()), int(reps),
                                 cache.encode() if cache else None))

    def energies(self, states):
        torch = _torch()
        if self._work is None:
            self._work = torch.empty(int(lib().gp_work_bytes(self._h)), dtype=torch.uint8, device=self.device)
        out = np.zeros(2 * len(states), dtype=np.float64)
        _check(lib().gp_energies_batch(self._h, self._ptrs(states), C.c_void_p(self._work.data_ptr()),
                                       out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(-1, 2)


# -------------------------------------------------------------------- autograd
def _functions():
    torch = _torch()

    class _Evolve(torch.autograd.Function):
        """theta -> psi_M = S^M exp(i theta); backward: adjoint segments of K steps
        recomputed from checkpoints psi_{jK}, then dJ/dtheta = Im(lam_0 conj psi_0)."""

        @staticmethod
        def forward(ctx, theta, plan, nsteps, ckpt):
            psi = plan.init_phase(theta.detach())
            ckpts = [psi.clone()]
            done = 0
            while done < nsteps:
                k = min(ckpt, nsteps - done)
                plan.step_n(psi, k)
                done += k
                if done < nsteps:
                    ckpts.append(psi.clone())
            ctx.plan, ctx.nsteps, ctx.ckpt = plan, nsteps, ckpt
            ctx.ckpts = ckpts
            return psi.clone()

        @staticmethod
        def backward(ctx, grad_psi):
            plan = ctx.plan
            lam = grad_psi.contiguous().clone()
            segs = []
            done = 0
            while done < ctx.nsteps:
                segs.append(min(ctx.ckpt, ctx.nsteps - done))
                done += segs[-1]
            tape = None
            for j in range(len(segs) - 1, -1, -1):
                lam, tape = plan.adjoint_step_n(ctx.ckpts[j], lam, segs[j], tape)
            dtheta = plan.phase_grad(ctx.ckpts[0], lam)
            return dtheta, None, None, None

    class _EkinI(torch.autograd.Function):
        """psi -> J = 1/2 sum_{smin <= s <= smax} |w^i_k|^2, backward grad_J * lam."""

        @staticmethod
        def forward(ctx, psi, plan, smin, smax):
            J, lam = plan.loss_ekin_i_shells(psi.detach().contiguous(), smin, smax)
            ctx.save_for_backward(lam)
            return torch.tensor(J, dtype=torch.float64, device=psi.device)

        @staticmethod
        def backward(ctx, gJ):
            (lam,) = ctx.saved_tensors
            return lam * gJ.to(lam.dtype), None, None, None

    return _Evolve, _EkinI


_FUNCS = None


def evolve(theta, plan: Plan, nsteps: int, ckpt: int = 20):
    """Differentiable psi_M(theta) (complex128 plans)."""
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _functions()
    return _FUNCS[0].apply(theta, plan, int(nsteps), int(ckpt))


def ekin_i_shells(psi, plan: Plan, smin: int, smax: int):
    """Differentiable incompressible kinetic energy summed over shells smin..smax."""
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _functions()
    return _FUNCS[1].apply(psi, plan, int(smin), int(smax))
