/*
 * gp.h -- C ABI of the MI355X (gfx950) Gross-Pitaevskii split-step library.
 *
 * Method: Kobayashi et al., "Quantum turbulence simulations using the
 * Gross-Pitaevskii equation: high-performance computing and new numerical
 * benchmarks" (arXiv:2003.03590).  The library integrates the dimensionless GP
 * equation of the "Scaling and dimensionless equations" section,
 *
 *     i d(psi)/dt = ( -alpha lap + beta (|psi|^2 - 1) ) psi        (eq. gpe-num)
 *
 * on the periodic box [0, 2 pi)^3 with the second-order Strang/ADI splitting of
 * the "Numerical method for the time evolution" section (eq. adi_looptime), each
 * sub-step solved exactly (spectral linear sub-steps, analytic nonlinear phase
 * rotation), and reports the energy split and shell spectra of the "Energy
 * decomposition" and "Spectra and structure functions" sections.
 *
 * Conventions shared by every entry point
 *   - Fields are complex, interleaved (re, im), C order [z][y][x] with x
 *     contiguous: GP_C128 = two doubles (16 B) per point, GP_C64 = two floats
 *     (8 B).  n[0] = Nx, n[1] = Ny, n[2] = Nz.
 *   - Pointers marked "dev" are device (HBM) pointers owned by the caller; the
 *     library never frees them.  Pointers marked "host" are host memory.
 *   - Every call is asynchronous on the plan's stream unless it returns host
 *     values, in which case it synchronizes that stream before returning.
 *   - Every call returns gp_status; nothing throws, exits or prints.  After a
 *     HIP error the plan is unusable (later calls return GP_ERR_STATE).
 *   - Calls that work on one grid return GP_ERR_STATE for a batch plan.
 *   - Testing the error paths: with the environment variable GP_FAULT_INJECT
 *     set to "alloc", every device allocation fails with GP_ERR_NOMEM before
 *     hipMalloc is called; set to "launch", every kernel-launch check reports
 *     a HIP error (GP_ERR_HIP, plan unusable) although the kernel runs normally.
 *   - A plan is not thread-safe; distinct plans are.
 *   - Supported axis lengths: 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96,
 *     128, 192, 256, 384, 512, 768, 1024 (GP_ERR_UNSUPPORTED otherwise).
 */
#ifndef GP_H
#define GP_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define GP_API __attribute__((visibility("default")))
#else
#define GP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_plan_s gp_plan_t;

typedef enum {
  GP_OK = 0,
  GP_ERR_ARG = 1,          /* null pointer, bad size, out-of-range argument */
  GP_ERR_UNSUPPORTED = 2,  /* axis length or precision not compiled */
  GP_ERR_HIP = 3,          /* a HIP runtime call failed; the plan is now unusable */
  GP_ERR_NOMEM = 4,        /* device or pinned allocation failed */
  GP_ERR_NONFINITE = 5,    /* a diagnostic is NaN/Inf (values are still written) */
  GP_ERR_STATE = 6         /* plan unusable after an earlier HIP error, or wrong plan kind */
} gp_status;

typedef enum { GP_C128 = 0, GP_C64 = 1 } gp_prec;

/* Problem description (paper scaling: L = 2 pi, coefficients alpha and beta of
 * eq. gpe-num, time step dt). */
typedef struct {
  int32_t n[3];      /* grid points along x, y, z */
  double alpha;      /* coefficient of -lap */
  double beta;       /* coefficient of (|psi|^2 - 1) */
  double dt;         /* time step of gp_step_n */
  int32_t prec;      /* gp_prec: storage and transform precision */
  uint32_t flags;    /* reserved, must be 0 */
} gp_desc;

/* Energies per unit volume in the paper's scaling:
 *   mass     N = <|psi|^2>                                   (eq. scaling-N)
 *   energy   E = 2 alpha^2 sum_k |k|^2 |c_k|^2 + alpha beta <(|psi|^2-1)^2>
 *                                                            (eq. scaling-energy)
 *   e_kin    <|w|^2>/2, w = 2 alpha Im(conj(psi) grad psi)/|psi| = sqrt(rho) v
 *   e_kin_i, e_kin_c   incompressible / compressible parts of e_kin (Helmholtz
 *            split of w; the k = 0 mode counts as incompressible)
 *   e_q      <|q|^2>/2, q = 2 alpha Re(conj(psi) grad psi)/|psi| = 2 alpha grad |psi|
 *            (pointwise from the spectral derivatives of psi, as w; q = w = 0 where
 *            psi = 0), so e_kin + e_q = 2 alpha^2 sum_k |k~|^2 |c_k|^2 with the
 *            first-derivative k~ (Nyquist entry 0)
 *   e_int    alpha beta <(|psi|^2-1)^2>          (eq. scaling-energy-mod-rho)    */
typedef struct {
  double mass, energy, e_kin, e_kin_i, e_kin_c, e_q, e_int;
} gp_energy;

/* Create a plan for one grid.  Generates the FP64 twiddle and propagator
 * tables on the host (rounded to the working precision) and uploads them;
 * selects the compiled FFT schedule of each axis.  hip_stream: a hipStream_t,
 * or NULL for the default stream.  *out receives the plan (NULL on error). */
GP_API gp_status gp_plan(const gp_desc* d, void* hip_stream, gp_plan_t** out);

/* Create a plan for an ensemble of independent runs (grid sizes may differ;
 * all runs share one precision).  Runs are advanced together by
 * gp_step_n_batch, which groups runs of equal size into single launches inside
 * recorded HIP graphs. */
GP_API gp_status gp_plan_batch(const gp_desc* runs, int32_t nruns, void* hip_stream, gp_plan_t** out);

GP_API gp_status gp_plan_destroy(gp_plan_t* p);

/* Bytes of one state (N^3 * S) -- for a batch plan, of run i (i < nruns). */
GP_API size_t gp_state_bytes(const gp_plan_t* p, int32_t run);
/* Bytes of the caller-provided diagnostics workspace (5 states). */
GP_API size_t gp_work_bytes(const gp_plan_t* p);
/* Number of integer shells s = round(|k|) of the spectra. */
GP_API int32_t gp_nshell(const gp_plan_t* p);

/* psi = exp(i theta) pointwise (initial condition of the smoothed-random-phase
 * construction, eq. SRP_Init).  theta: dev, N^3 doubles; psi: dev, out. */
GP_API gp_status gp_init_phase(gp_plan_t* p, const double* theta, void* psi);

/* Random-vortex-ring initial condition (RVR section): psi = product over npairs
 * ring pairs, each the pair ansatz psi_VR(z - d/2) conj(psi_VR(z + d/2)) (Pade core
 * profile of width xi, phase atan2(z~, r - R)) times the conjugates of its six mirror
 * images, evaluated at ((x, y, z) permuted) - (X, Y, Z) mod 2 pi.  pairs: host,
 * npairs x 6 doubles (R, d, X, Y, Z, permutation 0..5 in the order (x,y,z), (x,z,y),
 * (y,x,z), (y,z,x), (z,x,y), (z,y,x)).  psi: dev, out.  Synchronizes. */
GP_API gp_status gp_init_rvr(gp_plan_t* p, const double* pairs, int32_t npairs, double xi, void* psi);

/* One directional linear sub-step S(s, L_axis) psi = F_j^-1 exp(-i alpha k_j^2 s) F_j psi,
 * in place (time-evolution section).  axis: 0 = x, 1 = y, 2 = z. */
GP_API gp_status gp_substep_linear(gp_plan_t* p, void* psi, int32_t axis, double s);

/* Nonlinear sub-step S(s, N) psi = exp(-i beta (|psi|^2 - 1) s) psi, in place. */
GP_API gp_status gp_substep_nonlinear(gp_plan_t* p, void* psi, double s);

/* nsteps Strang steps of dt (nsteps < 0: |nsteps| steps of -dt), in place:
 * psi <- [L(dt/2) N(dt) L(dt/2)]^n psi with L = L_x L_y L_z (eq. adi_looptime).
 * Adjacent half steps are merged and the nonlinear rotation is fused into the
 * following x pass: 3 (|n| + 1) axis passes, each reading and writing psi once. */
GP_API gp_status gp_step_n(gp_plan_t* p, void* psi, int64_t nsteps);

/* The same steps in the literal 3-D form: 3-D FFT, multiply by
 * exp(-i alpha |k|^2 dt/2), inverse 3-D FFT, nonlinear rotation, and again
 * (the wording of the spectral sub-step).  The multiplier is applied by the last
 * forward pass before it stores: 13 sweeps of the state per step (26 N^3 S bytes),
 * against 3 (6 N^3 S) for gp_step_n. */
GP_API gp_status gp_step_literal_n(gp_plan_t* p, void* psi, int64_t nsteps);

/* 3-D transform: dir = -1 forward with 1/N^3 (c_k = N^-3 sum_x psi e^{-ik.x}),
 * dir = +1 inverse without factor.  Natural fftfreq order of k.  in may equal out. */
GP_API gp_status gp_fft3(gp_plan_t* p, const void* in, void* out, int32_t dir);

/* Bandwidth reference, not part of the method: dst <- src for one state of the plan
 * (n0 n1 n2 complex points, device pointers, 16-byte aligned, not overlapping),
 * one 16-byte unit per lane, on the plan's stream.  Timing it gives what HBM
 * delivers to a plain read-once, write-once stream of the bytes an axis pass moves.
 * GP_ERR_ARG for a null pointer, GP_ERR_STATE for a batch plan. */
GP_API gp_status gp_copy_state(gp_plan_t* p, const void* src, void* dst);

/* Mass, energy and its decomposition (see gp_energy).  work: dev, gp_work_bytes.
 * Synchronizes.  GP_ERR_NONFINITE if any value is NaN/Inf. */
GP_API gp_status gp_energies(gp_plan_t* p, const void* psi, void* work, gp_energy* out);

/* For callers that cannot allocate device memory (code under HIP graph capture
 * set up beforehand, tight serving loops, harnesses that forbid hipMalloc):
 * gp_energies with its diagnostics workspace in a static device array of
 * GP_STATIC_WORK_BYTES (64 MiB) that the library holds on every GPU it runs on
 * until the process ends, so the caller passes no workspace and nothing is
 * allocated or freed.  The plan (created earlier by gp_plan) must need at most
 * that much: 4 * N^3 * S bytes, i.e. up to 96^3 complex128 or 128^3 complex64;
 * larger grids return GP_ERR_ARG before any GPU work.  Results equal those of
 * gp_energies.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (from several threads or streams) race.  Synchronizes. */
#define GP_STATIC_WORK_BYTES (64u << 20)
GP_API gp_status gp_energies_static(gp_plan_t* p, const void* psi, gp_energy* out);

/* Shell spectra (spectra section, Parseval per unit volume): out is host
 * [4][nshell] doubles, rows E_kin^i(s), E_kin^c(s), E_q(s), E_int(s), each summing
 * to its energy.  energies (host, may be NULL) receives gp_energy of the same
 * evaluation.  nshell must equal gp_nshell.  Synchronizes. */
GP_API gp_status gp_spectra(gp_plan_t* p, const void* psi, void* work, double* out, int32_t nshell,
                     gp_energy* energies);

/* Second-order structure function of rho = |psi|^2 (eq. strfunc-def with v -> rho,
 * spatial mean, averaged over the three axes): out is host, Nx/2 doubles for lags
 * m = 1 .. Nx/2 (cubic grids only).  p_order must be 2.  Synchronizes. */
GP_API gp_status gp_structure_fn(gp_plan_t* p, const void* psi, void* work, int32_t p_order, double* out);

/* Longitudinal velocity structure functions (eq. strfunc-def), one per axis:
 * S_j(m) = < (v_j(x + m dx e_j) - v_j(x))^2 >, spatial mean, lags m = 1 .. N/2, with
 * v = 2 alpha Im(conj(psi) grad psi)/|psi|^2 from the spectral derivatives (v = 0 where
 * psi = 0).  Computed from the power spectrum of v_j along axis j (Wiener-Khinchin).
 * out: host, 3 * (N/2) doubles [axis (x, y, z)][m]; mean_v2: host, 3 doubles <v_j^2>
 * (2 <v_j^2> is the large-lag value of eq. strfunc-verif), may be NULL.  Cubic grids
 * only; p_order must be 2.  work: dev, gp_work_bytes.  Synchronizes. */
GP_API gp_status gp_structure_fn_velocity(gp_plan_t* p, const void* psi, void* work, int32_t p_order, double* out,
                                          double* mean_v2);

/* Mach numbers (eq. Mach-Number): out[0] = M_max = max |sqrt(rho) v| / c,
 * out[1] = M_rms = sqrt(2 E_kin) / c, with sqrt(rho) v = w of gp_energy and the sound
 * speed c = sqrt(2 alpha beta) of the paper's scaling.  out: host, 2 doubles.
 * work: dev, gp_work_bytes.  Synchronizes. */
GP_API gp_status gp_mach(gp_plan_t* p, const void* psi, void* work, double* out);

/* Bytes of the workspace gp_helicity needs (8 states; 0 for batch plans). */
GP_API size_t gp_helicity_work_bytes(const gp_plan_t* p);

/* Helicity and regularized helicity per unit volume (section on helicity):
 *   out[0] = H     = < v . omega >                          (eq. helicity)
 *   out[1] = H_reg = < v_reg . omega >                      (eq. Hreg)
 * with v = 2 alpha Im(conj(psi) grad psi)/|psi|^2, omega = curl v (spectral),
 * v_reg = v_par W/|W|, W = 4 alpha grad(Re psi) x grad(Im psi),
 * v_par = 2 alpha W . J / (|W| |grad psi|^2), J_i = Im(sum_j (d_i d_j psi)(d_j psi)*)
 * (hbar/m -> 2 alpha in the paper's scaling; v = 0 where psi = 0; v_reg = 0 where W = 0
 * or |grad psi|^2 <= 1e-12 <|grad psi|^2>, the critical points of psi where v_par's
 * denominator vanishes).  All derivatives spectral with the Nyquist entry 0; second
 * derivatives are two first derivatives.  spec (host, may be NULL): [2][nshell] shell
 * spectra Re(conj(v_k) . omega_k) and Re(conj(vreg_k) . omega_k), each summing to its
 * helicity; nshell must equal gp_nshell.  work: dev, gp_helicity_work_bytes.
 * Synchronizes. */
GP_API gp_status gp_helicity(gp_plan_t* p, const void* psi, void* work, double* out, double* spec, int32_t nshell);

/* Loss J = 1/2 sum over shells smin..smax of |w^i_k|^2 (incompressible kinetic
 * energy spectrum summed over those shells) and its gradient lam (dev, out) with
 * dJ = Re sum conj(lam) dpsi.  J: host.  Synchronizes. */
GP_API gp_status gp_loss_ekin_i_shells(gp_plan_t* p, const void* psi, void* work, int32_t smin,
                                int32_t smax, double* J, void* lam);

/* Adjoint of nsteps Strang steps from psi_seg_start: recomputes the forward
 * states phi_n = L(dt/2) psi_n of the segment into tape (dev, nsteps states),
 * then lam <- [L(-dt/2) N'(phi_n)^dagger L(-dt/2)] ... lam for n = nsteps-1 .. 0
 * (conjugate propagators in reverse order and the adjoint of the linearised
 * nonlinear rotation).  lam: dev, in/out.  GP_C128 only. */
GP_API gp_status gp_adjoint_step_n(gp_plan_t* p, const void* psi_seg_start, void* lam, int64_t nsteps,
                            void* tape);

/* dJ/dtheta = Im(lam0 conj(psi0)) for psi0 = exp(i theta).  dJ_dtheta: dev, N^3 doubles. */
GP_API gp_status gp_phase_grad(gp_plan_t* p, const void* psi0, const void* lam0, double* dJ_dtheta);

/* Imaginary-time preparation of a driven stationary state (section on stationary
 * solutions): nsteps steps of the semi-implicit backward Euler scheme
 * (eq. semi-backward-Euler) for the advective real Ginzburg-Landau equation
 * (eq. gradient-flow)
 *   phi_tau = (alpha lap - i v.grad - |v|^2/(4 alpha) + beta - beta |phi|^2) phi,
 * half of the Laplacian implicit (diagonal in Fourier space), the rest explicit;
 * alpha, beta from the plan (its dt is not used).  phi: dev, in/out, N^3 complex.
 * v: dev, three real fields v_x, v_y, v_z of the plan's real precision (FP64 for
 * GP_C128, FP32 for GP_C64), each N^3 in the [z][y][x] order of phi.  dtau > 0,
 * nsteps >= 0.  work: dev, gp_work_bytes (three states used).  |k|^2 of the
 * Laplacian uses N^2/4 at the Nyquist index; first derivatives use 0 there.
 * Asynchronous on the plan's stream.  Not for batch plans (GP_ERR_STATE). */
GP_API gp_status gp_argle_step(gp_plan_t* p, void* phi, const void* v, double dtau, int64_t nsteps, void* work);

/* Driven energy per unit volume (eq. energy-num-ext-vel)
 *   E_v = 2 alpha < alpha |grad phi - i v phi/(2 alpha)|^2 + (beta/2)(|phi|^2 - 1)^2 >,
 * the quantity the imaginary-time flow decreases.  Arguments as for
 * gp_argle_step; energy_v: host out.  Synchronizes. */
GP_API gp_status gp_argle_energy(gp_plan_t* p, const void* phi, const void* v, void* work, double* energy_v);

/* Outcome of gp_argle_run (values of the last check). */
typedef struct {
  int64_t steps;       /* steps taken */
  double crit_sup;     /* ||phi^{n+1} - phi^n||_inf / dtau            (eq. crit1) */
  double crit_energy;  /* |E_v^{n+1} - E_v^n| / (dtau E_v^n)         (eq. crit2) */
  double e_v;          /* E_v of the returned field                            */
  int32_t converged;   /* 1 if a check met crit_sup <= eps                       */
} gp_argle_report;

/* The ARGLE procedure with its stopping rule (section on computing stationary
 * solutions): steps of gp_argle_step until eq. crit1 holds or max_steps steps
 * are done.  The criteria are evaluated on every check_every-th step and on the
 * last step (a check adds one E_v evaluation before and after the step and a
 * copy of phi^n into the fifth workspace state); the run stops at the first
 * check with crit_sup <= eps.  eps <= 0 runs max_steps steps and reports the
 * criteria of the last one (the paper's fixed tau_f runs).  max_steps = 0:
 * crit_sup = crit_energy = NaN and e_v = E_v(phi).  work: dev, gp_work_bytes
 * (all five states used).  report: host out.  Synchronizes at every check. */
GP_API gp_status gp_argle_run(gp_plan_t* p, void* phi, const void* v, double dtau, int64_t max_steps,
                              int64_t check_every, double eps, void* work, gp_argle_report* report);

/* Ensemble: advance run i's state psis[i] (host array of dev pointers) by nsteps
 * (negative: backward).  The merged sequence L(h) [N L(dt)]^(n-1) N L(h) runs as
 * recorded HIP graphs: the opening half step, bodies of 2^j applications
 * (j = 0..7; the 128-application body repeated, the rest by the binary digits of
 * n - 1) and the closing half step.  Each graph holds one grouped launch per size
 * group and pass, the size groups on parallel branches; a graph is recorded on
 * first use for the given states and replayed after, so a call launches at most
 * 2 + 7 + (n-1)/128 graphs of at most 3 x 128 launches per group, whatever n.
 * New state pointers, gp_autotune or gp_select_variant drop the recorded graphs. */
GP_API gp_status gp_step_n_batch(gp_plan_t* p, void* const* psis, int64_t nsteps);

/* Ensemble: mass and energy of every run (host out, 2 * nruns doubles:
 * mass_i, energy_i).  work: dev, gp_work_bytes.  Synchronizes. */
GP_API gp_status gp_energies_batch(gp_plan_t* p, void* const* psis, void* work, double* out);

/* Message of the last non-OK status on this thread ("" if none). */
GP_API const char* gp_last_error(void);

/* Name of the compiled FFT schedule used for an axis, e.g. "N=256 T=16 W=8 R=16x16".
 * axis 3 names the xy choice: "xy: separate passes" or "xy: plane N=.. T=..";
 * axis 4 the pass that carries the nonlinear rotation ("nl: x pass", ...); axis 5
 * the form of the linear steps ("layout: fixed", "layout: rotating ..." or
 * "layout: rotating+contiguous ...").  For a
 * batch plan the index is 6 * run + axis (the names of that run's schedules). */
GP_API const char* gp_schedule_name(const gp_plan_t* p, int32_t axis);

/* Number of compiled schedule variants for an axis length and precision, and
 * selection of one of them for an axis of a plan.  Selecting rebuilds that
 * axis's tables (their order follows the schedule's radices); synchronizes.
 * axis 3 selects how the two in-plane sub-steps run in gp_step_n and
 * gp_step_n_batch: variant 0 = separate x and y passes, 1 = one xy-plane pass per
 * z-plane (both sub-steps on chip, psi read and written once; the x and y factors
 * commute, time-evolution section).  Variant 1 needs nx == ny with a compiled
 * plane length (complex64: 16..96, complex128: 16..64); otherwise
 * GP_ERR_UNSUPPORTED.  axis 4 (single plans, separate passes) selects the axis pass
 * that carries the nonlinear rotation as its prologue and runs first in each
 * linear step (variant 0, 1, 2 = x, y, z; the linear sub-steps commute, so any
 * order is the same split step); default: the first axis of length > 1.  axis 5
 * (single cubic plans) selects the form of the linear steps of gp_step_n: variant
 * 0 (default) the fixed layout, every pass in place; variant v = 1..R (R compiled
 * rotating schedules for the length) the v-th rotating schedule: layout-rotating
 * passes along x, z, y, each reading whole contiguous pencils and writing the state
 * in a turned layout ([z][y][x] -> [y][x][z] -> [x][z][y] -> [z][y][x]), out of
 * place between psi and one more state that the plan allocates on selection (N^3 S
 * bytes, released again by variant 0); variant R + v the same schedule in the
 * mixed form: per linear step two rotating passes and one in-place pass along the
 * axis they leave innermost, so the layout advances one place per step and returns
 * every three.  psi holds the [z][y][x] state whenever gp_step_n returns.
 * GP_ERR_UNSUPPORTED for other shapes or lengths without a rotating schedule.
 * Batch plans: GP_ERR_STATE for every axis but 3. */
GP_API int32_t gp_variant_count(int32_t n, int32_t prec);
GP_API gp_status gp_select_variant(gp_plan_t* p, int32_t axis, int32_t variant);

/* Autotuner: for every axis of the plan (every size group of a batch plan),
 * time `reps` launches of each compiled schedule variant on `scratch` (dev, one
 * state of the plan's largest run; its contents are overwritten) with HIP
 * events, and keep the fastest (timings within 1 % count as ties, resolved to the
 * lower variant index, so repeated tunings agree); then the xy choice (axis 3), timed with as many
 * runs per launch as the size group holds; then, for single plans with separate
 * passes, the nonlinear carrier (axis 4), timed as whole linear steps, and for
 * cubic grids with a rotating schedule the layout form (axis 5), timed as whole
 * linear steps (the rotating form's workspace is released when it loses).  cache_path
 * (may be NULL): a JSON file of
 * earlier choices keyed by GPU architecture, precision, grid shape and axis;
 * cached choices are applied without timing and new ones are added.
 * Synchronizes.  A batch plan re-records its graph on the next step call. */
GP_API gp_status gp_autotune(gp_plan_t* p, void* scratch, int32_t reps, const char* cache_path);

#ifdef __cplusplus
}
#endif

#endif /* GP_H */
