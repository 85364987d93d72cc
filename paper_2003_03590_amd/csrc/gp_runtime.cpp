// Host runtime of the Gross-Pitaevskii library: plans, FP64 table generation,
// pass sequencing of the split step, diagnostics and adjoint pipelines, the
// ensemble (batch) path with HIP graph capture, and the C ABI of include/gp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "gp.h"
#include "gp_point.h"

namespace gpk {

std::vector<PassEntry>& registry() {
  static std::vector<PassEntry> r;
  return r;
}

std::vector<PlaneEntry>& plane_registry() {
  static std::vector<PlaneEntry> r;
  return r;
}

std::vector<RotEntry>& rot_registry() {
  static std::vector<RotEntry> r;
  return r;
}

namespace {

thread_local std::string g_err;

gp_status fail(gp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

// ----------------------------------------------------------------- FP64 tables
// cos and sin of 2 pi num/den with the angle reduced exactly in integers to
// [0, pi/4] before calling the libm routines.
void cis2pi(long num, long den, double* c, double* s) {
  long m = ((num % den) + den) % den;
  // 8 m = oct * den + r, angle = (pi/4)(oct + r/den)
  const long oct = (8 * m) / den;
  const long r = 8 * m - oct * den;
  // reduce to the first octant
  double a;
  bool swap = false;
  if (oct % 2 == 0) { a = (M_PI / 4) * double(r) / double(den); }
  else { a = (M_PI / 4) * double(den - r) / double(den); swap = true; }
  const ct::Pair u = ct::unit_pair(std::cos(a), std::sin(a));    // norm-closest pair
  double cc = u.c, ss = u.s;
  if (swap) std::swap(cc, ss);        // angle in octant 2q+1 measured from the next axis
  const long q = oct / 2;              // quadrant
  switch (q) {
    case 0: *c = cc; *s = ss; break;
    case 1: *c = -ss; *s = cc; break;
    case 2: *c = -cc; *s = -ss; break;
    default: *c = ss; *s = -cc; break;
  }
}

int kfreq(int i, int n) { return (2 * i < n) ? i : i - n; }

// natural frequency index -> position of the DIF output (digit reversal)
int freq_pos(const PassEntry& e, int k) {
  int p = 0, K = 1;
  for (int s = 0; s < e.NS; ++s) {
    int M = 1;
    for (int i = s + 1; i < e.NS; ++i) M *= e.radix[i];
    p += ((k / K) % e.radix[s]) * M;
    K *= e.radix[s];
  }
  return p;
}

// table index of DIF output position pos: positions are g*R_last + r; the tables are
// stored r-major so that the lanes of one load instruction read consecutive entries
int lane_idx(const PassEntry& e, int pos) {
  const int rl = e.radix[e.NS - 1];
  return (pos % rl) * (e.n / rl) + pos / rl;
}

// index of natural frequency k in the multiplier tables of schedule e
int tab_idx(const PassEntry& e, int k) { return lane_idx(e, freq_pos(e, k)); }

// per-stage twiddles: stage s with M_s = R_{s+1}...R_{NS-1} > 1 stores
// W_{R_s M_s}^{lo k} = exp(-2 pi i lo k / (R_s M_s)) at off_s + (k-1) M_s + lo
std::vector<double> stage_twiddles(const PassEntry& e) {
  std::vector<double> tw;
  for (int s = 0; s < e.NS; ++s) {
    int M = 1;
    for (int i = s + 1; i < e.NS; ++i) M *= e.radix[i];
    if (M == 1) continue;
    const int R = e.radix[s], L = R * M;
    for (int k = 1; k < R; ++k)
      for (int lo = 0; lo < M; ++lo) {
        double c, sn;
        cis2pi(-(long)lo * k, L, &c, &sn);
        tw.push_back(c);
        tw.push_back(sn);
      }
  }
  if (tw.empty()) tw = {1.0, 0.0};     // single-stage schedules read no twiddle
  return tw;
}

const int kSupported[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};

const PassEntry* find_entry(int n, int prec, int variant) {
  for (const auto& e : registry())
    if (e.n == n && e.prec == prec && e.variant == variant) return &e;
  return nullptr;
}

enum Tau { TAU_H = 0, TAU_DT = 1, TAU_MH = 2, TAU_MDT = 3, NTAU = 4 };

struct Axis {
  int n = 1;
  int kind = CONTIG;
  const PassEntry* e = nullptr;
  long npencils = 0, inner = 1, outer = 0, es = 1;
  unsigned blocks = 0;
  // device tables (working precision unless noted)
  void* tw = nullptr;
  void* mult[NTAU] = {};    // exp(-i alpha k^2 tau)/n, lane order, FP64 complex
  void* deriv = nullptr;    // i k~/n, lane order, FP64 complex
  double* ksq = nullptr;    // k^2, position order (double)
  void* nat[NTAU] = {};     // exp(-i alpha k^2 tau)/n, natural order, FP64 complex
};

}  // namespace
}  // namespace gpk

using namespace gpk;

struct gp_plan_s {
  gp_desc d{};
  hipStream_t stream = nullptr;
  int prec = P_C128;
  size_t S = 16;
  long ntot = 0;
  int nshell = 0;
  Axis ax[3];
  std::vector<void*> allocs;       // device allocations owned by the plan
  std::map<std::pair<int, double>, void*> substep_tables;   // gp_substep_linear cache
  // reduction partials
  double* kin_part = nullptr;      // blocks(x) + blocks(y) + blocks(z)
  double* field_part = nullptr;    // 3 * field_blocks
  unsigned field_blocks = 0;
  double* bins_part = nullptr;     // spec_blocks * 4 * nshell
  unsigned spec_blocks = 0;
  long spec_chunk = 0;
  double* power_part = nullptr;    // 3 * pow_blocks * nx
  unsigned pow_blocks = 0;
  long pow_chunk = 0;
  double* loss_part = nullptr;     // field_blocks
  double* d_red = nullptr;         // 6 + 4 * nshell reduced sums
  double* d_pk = nullptr;          // 3 * nmax reduced axis power sums
  double* d_result = nullptr;      // 8 + 4 * nshell
  double* h_result = nullptr;      // pinned mirror
  bool broken = false;
  bool own_stream = false;         // stream created by the plan (batch plans on the null stream)
  std::string sched_name[6];       // x, y, z axis schedules; [3]: the xy-plane choice; [4]: the nonlinear
                                   // carrier; [5]: fixed-layout or layout-rotating linear steps
  int nl_axis = -1;                // axis pass that carries the nonlinear prologue (-1: first real axis)
  // xy-plane pass (x and y sub-steps fused; needs nx == ny with a compiled plane schedule)
  struct Plane {
    const PlaneEntry* e = nullptr;
    bool on = false;
    void* tw = nullptr;
    void* mx[NTAU] = {};
    void* my[NTAU] = {};
  } plane;
  // layout-rotating passes (cubic grids): every linear step as x, z, y passes that
  // turn the layout, out of place between psi and one state of workspace
  struct Rot {
    const RotEntry* e = nullptr;
    bool on = false;
    bool mixed = false;            // two rotating passes and one in-place x-kind pass per linear step
    void* work = nullptr;          // N^3 S bytes, allocated when first selected
    void* tw = nullptr;
    void* mult[NTAU] = {};
  } rot;
  RunPtrs* d_tune_ptrs = nullptr;  // autotuner: grouped timing launches
  size_t n_tune_ptrs = 0;
  // ensemble
  bool is_batch = false;
  std::vector<gp_plan_s*> runs;
  struct Group { int n; std::vector<int> members; RunPtrs* d_ptrs = nullptr; size_t nptrs = 0; };
  std::vector<Group> groups;
  // recorded step graphs, [sign: 0 forward, 1 backward][slot]: slot 0 the opening
  // half step L(h), 1 the closing [N, L(h)], 2 + j the body [N, L(dt)] x 2^j
  static constexpr int GPOW = 8, GSLOTS = 2 + GPOW;
  hipGraphExec_t gexec[2][GSLOTS] = {};
  std::vector<void*> graph_key;      // the states the recorded graphs and tables refer to
  std::vector<hipStream_t> side;     // capture branches of size groups 1, 2, ...
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
};

namespace gpk {
namespace {

#define HIPCHK(plan, expr)                                                                   \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) {                                                                  \
      if (plan) (plan)->broken = true;                                                       \
      return fail(GP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));                \
    }                                                                                        \
  } while (0)

// Host-side fault switch for testing the error paths: GP_FAULT_INJECT=alloc makes
// every device allocation of the library fail (GP_ERR_NOMEM) before hipMalloc is
// called; GP_FAULT_INJECT=launch makes every kernel-launch check report a HIP error
// (the kernel itself was launched and runs normally).  Unset, it costs one getenv.
bool fault_injected(const char* what) {
  const char* e = getenv("GP_FAULT_INJECT");
  return e && strcmp(e, what) == 0;
}

gp_status check_launch(gp_plan_s* p) {
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && fault_injected("launch")) e = hipErrorLaunchFailure;
  if (e != hipSuccess) {
    p->broken = true;
    return fail(GP_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  }
  return GP_OK;
}

gp_status dev_alloc(gp_plan_s* p, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 16;
  if (fault_injected("alloc")) return fail(GP_ERR_NOMEM, "hipMalloc(%zu) failed: injected fault", bytes);
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(GP_ERR_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  p->allocs.push_back(*ptr);
  return GP_OK;
}

// upload a complex FP64 table as Tab<Real> entries (16 B each): the FP64 value for
// complex128, the FP64 value split into FP32 hi + lo for complex64
gp_status upload_cplx(gp_plan_s* p, void** dst, const std::vector<double>& reim) {
  const size_t n = reim.size() / 2;
  gp_status st = dev_alloc(p, dst, n * 16);
  if (st != GP_OK) return st;
  if (p->prec == P_C128) {
    HIPCHK(p, hipMemcpy(*dst, reim.data(), n * 16, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(4 * n);
    for (size_t i = 0; i < n; ++i) {
      const float hx = (float)reim[2 * i], hy = (float)reim[2 * i + 1];
      f[4 * i] = hx;
      f[4 * i + 1] = hy;
      f[4 * i + 2] = (float)(reim[2 * i] - (double)hx);
      f[4 * i + 3] = (float)(reim[2 * i + 1] - (double)hy);
    }
    HIPCHK(p, hipMemcpy(*dst, f.data(), n * 16, hipMemcpyHostToDevice));
  }
  return GP_OK;
}

// upload a complex FP64 table as FP64 complex entries for either precision (the
// multipliers applied between forward and inverse transforms)
gp_status upload_c128(gp_plan_s* p, void** dst, const std::vector<double>& reim) {
  gp_status st = dev_alloc(p, dst, reim.size() * sizeof(double));
  if (st != GP_OK) return st;
  HIPCHK(p, hipMemcpy(*dst, reim.data(), reim.size() * sizeof(double), hipMemcpyHostToDevice));
  return GP_OK;
}

gp_status upload_f64(gp_plan_s* p, double** dst, const std::vector<double>& v) {
  gp_status st = dev_alloc(p, (void**)dst, v.size() * sizeof(double));
  if (st != GP_OK) return st;
  HIPCHK(p, hipMemcpy(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
  return GP_OK;
}

bool supported_n(int n) {
  for (int s : kSupported) if (s == n) return true;
  return false;
}

gp_status setup_axis(gp_plan_s* p, int a, int variant) {
  Axis& A = p->ax[a];
  const int n = A.n;
  const int nx = p->d.n[0], ny = p->d.n[1], nz = p->d.n[2];
  if (a == 0) { A.kind = CONTIG; A.npencils = (long)ny * nz; A.inner = 1; A.outer = nx; A.es = 1; }
  else if (a == 1) { A.kind = STRIDED; A.npencils = (long)nx * nz; A.inner = nx; A.outer = (long)nx * ny; A.es = nx; }
  else { A.kind = STRIDED; A.npencils = (long)nx * ny; A.inner = (long)nx * ny; A.outer = 0; A.es = (long)nx * ny; }
  if (n == 1) { A.e = nullptr; A.blocks = 0; p->sched_name[a] = "N=1 (identity)"; return GP_OK; }
  A.e = find_entry(n, p->prec, variant);
  if (!A.e) return fail(GP_ERR_UNSUPPORTED, "no compiled schedule for axis length %d (variant %d)", n, variant);
  A.blocks = (unsigned)((A.npencils + A.e->W - 1) / A.e->W);
  char nm[128];
  snprintf(nm, sizeof nm, "N=%d T=%d W=%d R=%dx%dx%d v%d", n, A.e->T, A.e->W, A.e->radix[0], A.e->radix[1],
           A.e->radix[2], variant);
  p->sched_name[a] = nm;
  return GP_OK;
}

// tables of one axis (FP64 on the host, rounded to working precision)
gp_status build_tables(gp_plan_s* p, int a) {
  Axis& A = p->ax[a];
  const int n = A.n;
  const double alpha = p->d.alpha, dt = p->d.dt;
  const double taus[NTAU] = {0.5 * dt, dt, -0.5 * dt, -dt};
  std::vector<int> pos(n);
  for (int k = 0; k < n; ++k) pos[k] = A.e ? tab_idx(*A.e, k) : k;
  gp_status st;
  if (A.e && (st = upload_cplx(p, &A.tw, stage_twiddles(*A.e))) != GP_OK) return st;
  for (int t = 0; t < NTAU; ++t) {
    std::vector<double> mp(2 * n), mn(2 * n);
    for (int k = 0; k < n; ++k) {
      const double kk = (double)kfreq(k, n);
      const double ph = alpha * kk * kk * taus[t];
      const ct::Pair u = ct::unit_pair(std::cos(ph), std::sin(ph));
      const double c = u.c / n, s = -u.s / n;
      mp[2 * pos[k]] = c; mp[2 * pos[k] + 1] = s;
      mn[2 * k] = c; mn[2 * k + 1] = s;
    }
    if ((st = upload_c128(p, &A.mult[t], mp)) != GP_OK) return st;
    if ((st = upload_c128(p, &A.nat[t], mn)) != GP_OK) return st;
  }
  std::vector<double> dv(2 * n), kq(n);
  for (int k = 0; k < n; ++k) {
    const int kf = kfreq(k, n);
    const int k1 = (n % 2 == 0 && 2 * k == n) ? 0 : kf;
    dv[2 * pos[k]] = 0.0; dv[2 * pos[k] + 1] = (double)k1 / n;       // i k~ / n
    kq[pos[k]] = (double)kf * kf;
  }
  if ((st = upload_c128(p, &A.deriv, dv)) != GP_OK) return st;
  if ((st = upload_f64(p, &A.ksq, kq)) != GP_OK) return st;
  return GP_OK;
}

const PlaneEntry* find_plane(int n, int prec) {
  for (const auto& e : plane_registry())
    if (e.n == n && e.prec == prec) return &e;
  return nullptr;
}

// a plane schedule described as an axis schedule (for the table-order helpers)
PassEntry plane_as_entry(const PlaneEntry& pe) {
  PassEntry e{};
  e.n = pe.n; e.prec = pe.prec; e.T = pe.T; e.W = pe.n; e.NS = pe.NS; e.threads = pe.threads;
  for (int i = 0; i < 3; ++i) e.radix[i] = pe.radix[i];
  return e;
}

// twiddles and x/y multipliers of the plane schedule (built once per plan; with
// nx == ny and one alpha the x and y multipliers are the same table)
gp_status build_plane_tables(gp_plan_s* p) {
  auto& P = p->plane;
  if (P.tw) return GP_OK;
  const PassEntry e = plane_as_entry(*P.e);
  gp_status st;
  if ((st = upload_cplx(p, &P.tw, stage_twiddles(e))) != GP_OK) return st;
  const double alpha = p->d.alpha, dt = p->d.dt;
  const double taus[NTAU] = {0.5 * dt, dt, -0.5 * dt, -dt};
  const int n = e.n;
  for (int t = 0; t < NTAU; ++t) {
    std::vector<double> m(2 * n);
    for (int k = 0; k < n; ++k) {
      const double kk = (double)kfreq(k, n);
      const double ph = alpha * kk * kk * taus[t];
      const int i = tab_idx(e, k);
      const ct::Pair u = ct::unit_pair(std::cos(ph), std::sin(ph));
      m[2 * i] = u.c / n;
      m[2 * i + 1] = -u.s / n;
    }
    if ((st = upload_c128(p, &P.mx[t], m)) != GP_OK) return st;
    P.my[t] = P.mx[t];
  }
  return GP_OK;
}

int shell_of_host(long k2) {
  const long q = 4 * k2;
  long r = (long)std::sqrt((double)q);
  while (r * r > q) --r;
  while ((r + 1) * (r + 1) <= q) ++r;
  return (int)((r + 1) / 2);
}

gp_status plan_init(gp_plan_s* p, const gp_desc* d, hipStream_t stream) {
  p->d = *d;
  p->stream = stream;
  p->prec = d->prec;
  p->S = d->prec == GP_C128 ? 16 : 8;
  for (int a = 0; a < 3; ++a) p->ax[a].n = d->n[a];
  p->ntot = (long)d->n[0] * d->n[1] * d->n[2];
  const long kmax2 = (long)(d->n[0] / 2) * (d->n[0] / 2) + (long)(d->n[1] / 2) * (d->n[1] / 2) +
                     (long)(d->n[2] / 2) * (d->n[2] / 2);
  p->nshell = shell_of_host(kmax2) + 1;
  gp_status st;
  for (int a = 0; a < 3; ++a) {
    if ((st = setup_axis(p, a, 0)) != GP_OK) return st;
    if ((st = build_tables(p, a)) != GP_OK) return st;
  }
  p->plane.e = (d->n[0] == d->n[1] && d->n[0] > 1) ? find_plane(d->n[0], p->prec) : nullptr;
  p->sched_name[3] = "xy: separate passes";
  p->sched_name[4] = "nl: first axis";
  p->sched_name[5] = "layout: fixed";
  // reduction partials
  const long kin_n = (long)p->ax[0].blocks + p->ax[1].blocks + p->ax[2].blocks;
  if ((st = dev_alloc(p, (void**)&p->kin_part, std::max(1L, kin_n) * sizeof(double))) != GP_OK) return st;
  p->field_blocks = (unsigned)std::min<long>(1024, std::max<long>(1, (p->ntot + 4095) / 4096));
  if ((st = dev_alloc(p, (void**)&p->field_part, 3 * p->field_blocks * sizeof(double))) != GP_OK) return st;
  if ((st = dev_alloc(p, (void**)&p->loss_part, p->field_blocks * sizeof(double))) != GP_OK) return st;
  p->spec_blocks = (unsigned)std::min<long>(2048, std::max<long>(1, (p->ntot + 4095) / 4096));
  p->spec_chunk = (p->ntot + p->spec_blocks - 1) / p->spec_blocks;
  if ((st = dev_alloc(p, (void**)&p->bins_part, (size_t)p->spec_blocks * 4 * p->nshell * sizeof(double))) != GP_OK)
    return st;
  p->pow_blocks = p->spec_blocks;
  p->pow_chunk = p->spec_chunk;
  const int nmax = std::max(d->n[0], std::max(d->n[1], d->n[2]));
  if ((st = dev_alloc(p, (void**)&p->power_part, 3 * (size_t)p->pow_blocks * nmax * sizeof(double))) != GP_OK)
    return st;
  if ((st = dev_alloc(p, (void**)&p->d_result, (8 + 4 * (size_t)p->nshell + nmax) * sizeof(double))) != GP_OK)
    return st;
  if ((st = dev_alloc(p, (void**)&p->d_red, (6 + 4 * (size_t)p->nshell) * sizeof(double))) != GP_OK) return st;
  if ((st = dev_alloc(p, (void**)&p->d_pk, 3 * (size_t)nmax * sizeof(double))) != GP_OK) return st;
  hipError_t e = hipHostMalloc((void**)&p->h_result, (8 + 4 * (size_t)p->nshell + nmax) * sizeof(double),
                               hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(GP_ERR_NOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
  }
  return GP_OK;
}

void plan_free(gp_plan_s* p) {
  if (!p) return;
  for (auto* r : p->runs) plan_free(r);
  for (auto& row : p->gexec)
    for (auto& x : row) if (x) (void)hipGraphExecDestroy(x);
  for (auto st : p->side) if (st) (void)hipStreamDestroy(st);
  for (auto ev : p->join_ev) if (ev) (void)hipEventDestroy(ev);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  for (void* a : p->allocs) (void)hipFree(a);
  for (auto& g : p->groups) if (g.d_ptrs) (void)hipFree(g.d_ptrs);
  if (p->h_result) (void)hipHostFree(p->h_result);
  if (p->rot.work) (void)hipFree(p->rot.work);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

// the recorded step graphs of a batch plan are stale (kernels, tables or states changed)
void drop_graphs(gp_plan_s* p) {
  for (auto& row : p->gexec)
    for (auto& x : row)
      if (x) { (void)hipGraphExecDestroy(x); x = nullptr; }
  p->graph_key.clear();
}

gp_status validate_desc(const gp_desc* d) {
  if (!d) return fail(GP_ERR_ARG, "null descriptor");
  for (int a = 0; a < 3; ++a) {
    if (d->n[a] < 1) return fail(GP_ERR_ARG, "n[%d] = %d must be >= 1", a, d->n[a]);
    if (!supported_n(d->n[a])) return fail(GP_ERR_UNSUPPORTED, "axis length n[%d] = %d is not supported", a, d->n[a]);
  }
  if (d->prec != GP_C128 && d->prec != GP_C64) return fail(GP_ERR_UNSUPPORTED, "precision %d", d->prec);
  if (!std::isfinite(d->alpha) || !std::isfinite(d->beta) || !std::isfinite(d->dt))
    return fail(GP_ERR_ARG, "alpha, beta and dt must be finite");
  if (d->flags != 0) return fail(GP_ERR_ARG, "flags must be 0");
  return GP_OK;
}

gp_status usable(const gp_plan_s* p) {
  if (!p) return fail(GP_ERR_ARG, "null plan");
  if (p->broken) return fail(GP_ERR_STATE, "plan is unusable after an earlier HIP error");
  return GP_OK;
}

// entry points that work on one grid: a batch plan has no tables of its own
gp_status usable_single(const gp_plan_s* p) {
  gp_status st = usable(p);
  if (st != GP_OK) return st;
  if (p->is_batch) return fail(GP_ERR_STATE, "batch plan: this call takes a single-grid plan");
  return GP_OK;
}

// ----------------------------------------------------------------- pass launch
gp_status pass(gp_plan_s* p, int a, int var, const void* in, void* out, const void* mult, double nl_coef = 0.0,
               const void* aux = nullptr, double scale = 1.0, double* kin = nullptr) {
  Axis& A = p->ax[a];
  if (A.n == 1) {
    // one point along the axis: the transform is the identity and k = 0, so the
    // propagator tables are 1 (derivatives are handled by the callers)
    if (var == V_PROP_NL || var == V_PROP_ADJ || var == V_FWD_DENSITY)
      return fail(GP_ERR_STATE, "internal: fused prologue on an axis of length 1");
    if (in != out || scale != 1.0) launch_scale_copy(p->prec, in, out, p->ntot, scale, p->stream);
    return check_launch(p);
  }
  PassArgs g{};
  g.batch = nullptr;
  g.in = in; g.out = out; g.mult = mult; g.tw = A.tw; g.aux = aux;
  g.ksq = A.ksq; g.kin_partial = kin; g.nl_coef = nl_coef; g.scale = scale;
  g.npencils = A.npencils; g.inner = A.inner; g.outer = A.outer; g.es = A.es;
  A.e->fn[A.kind][var](g, A.blocks, 1, p->stream);
  return check_launch(p);
}

int first_real_axis(const gp_plan_s* p) {
  for (int a = 0; a < 3; ++a) if (p->ax[a].n > 1) return a;
  return -1;
}

// L(tau) on psi in place, the nonlinear rotation of coefficient nl (if any) fused in front
// of the first pass
gp_status linear_all(gp_plan_s* p, void* psi, int tau, bool with_nl, double nl) {
  const int c = first_real_axis(p);
  gp_status st;
  if (c < 0) {   // 1x1x1 grid: only the nonlinear rotation acts (k = 0)
    if (with_nl) { launch_nonlinear(p->prec, psi, p->ntot, nl, p->stream); return check_launch(p); }
    return GP_OK;
  }
  if (p->plane.on) {          // x and y in one plane pass (nonlinear prologue there), then z
    PlaneArgs g{};
    g.in = psi; g.out = psi; g.multx = p->plane.mx[tau]; g.multy = p->plane.my[tau];
    g.tw = p->plane.tw; g.nl_coef = nl;
    p->plane.e->fn[with_nl ? 1 : 0](g, (unsigned)p->d.n[2], 1, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
    return p->ax[2].n > 1 ? pass(p, 2, V_PROP, psi, psi, p->ax[2].mult[tau]) : GP_OK;
  }
  // the linear sub-steps commute: the axis that carries the nonlinear prologue runs
  // first, the others follow in x, y, z order
  const int carrier = (p->nl_axis >= 0 && p->ax[p->nl_axis].n > 1) ? p->nl_axis : c;
  const int order[3] = {carrier, carrier == 0 ? 1 : 0, carrier == 2 ? 1 : 2};
  for (int q = 0; q < 3; ++q) {
    const int a = order[q];
    if (p->ax[a].n == 1) continue;
    const bool nl_here = with_nl && a == carrier;
    if ((st = pass(p, a, nl_here ? V_PROP_NL : V_PROP, psi, psi, p->ax[a].mult[tau], nl)) != GP_OK) return st;
  }
  return GP_OK;
}

// L(tau) as three layout-rotating passes x, z, y from `in` ([z][y][x]) through the
// workspace to `out` ([z][y][x]): in -> [y][x][z] -> [x][z][y] -> [z][y][x].  The
// passes alternate between the two states, so in = out only after an even number
// of such steps; `in` and `out` are psi and the workspace in turn.
// one layout-rotating pass: the innermost axis of `in` transformed, written to `out`
// turned ([A][B][C] -> [B][C][A])
gp_status rot_pass_one(gp_plan_s* p, const void* in, void* out, int tau, bool with_nl, double nl) {
  const RotEntry& e = *p->rot.e;
  const unsigned grid = (unsigned)((long)e.n * e.n / e.sched.W);
  RotArgs g{};
  g.in = in; g.out = out;
  g.mult = p->rot.mult[tau];
  g.tw = p->rot.tw;
  g.nl_coef = nl;
  e.fn[with_nl ? 1 : 0](g, grid, p->stream);
  return check_launch(p);
}

// L(tau) as three rotating passes x, z, y: from a to b, back in [z][y][x]
gp_status rot_linear(gp_plan_s* p, void* a, void* b, int tau, bool with_nl, double nl) {
  gp_status st;
  if ((st = rot_pass_one(p, a, b, tau, with_nl, nl)) != GP_OK) return st;   // x (nonlinear prologue)
  if ((st = rot_pass_one(p, b, a, tau, false, nl)) != GP_OK) return st;     // z
  return rot_pass_one(p, a, b, tau, false, nl);                             // y
}

// L(tau) as two rotating passes and one in-place pass along the axis they leave
// innermost (the x-kind kernel: a cube's axes share lengths and tables): from a
// through b back to a, the layout advanced by one place in the cycle
// [z][y][x] -> [x][z][y] -> [y][x][z] -> [z][y][x]
gp_status mixed_linear(gp_plan_s* p, void* a, void* b, int tau, bool with_nl, double nl) {
  gp_status st;
  if ((st = rot_pass_one(p, a, b, tau, with_nl, nl)) != GP_OK) return st;
  if ((st = rot_pass_one(p, b, a, tau, false, nl)) != GP_OK) return st;
  return pass(p, 0, V_PROP, a, a, p->ax[0].mult[tau]);
}

gp_status step_n(gp_plan_s* p, void* psi, int64_t nsteps) {
  if (nsteps == 0) return GP_OK;
  const bool back = nsteps < 0;
  const int64_t n = back ? -nsteps : nsteps;
  const int th = back ? TAU_MH : TAU_H, tf = back ? TAU_MDT : TAU_DT;
  const double nl = p->d.beta * (back ? -p->d.dt : p->d.dt);
  gp_status st;
  if (p->rot.on && p->rot.mixed) {
    // n + 1 linear steps; three mixed ones bring the layout back, each keeps the state
    // in psi; a remainder of one runs in place with the fixed-layout passes, of two as
    // two fully rotating steps (psi -> workspace -> psi); all before the cycles, while
    // the layout is [z][y][x]
    auto tau_of = [&](int64_t k) { return (k == 0 || k == n) ? th : tf; };
    const int64_t r = (n + 1) % 3;
    int64_t k = 0;
    if (r == 1) {
      if ((st = linear_all(p, psi, th, false, 0.0)) != GP_OK) return st;
      k = 1;
    } else if (r == 2) {
      if ((st = rot_linear(p, psi, p->rot.work, tau_of(0), false, nl)) != GP_OK) return st;
      if ((st = rot_linear(p, p->rot.work, psi, tau_of(1), true, nl)) != GP_OK) return st;
      k = 2;
    }
    for (; k <= n; ++k)
      if ((st = mixed_linear(p, psi, p->rot.work, tau_of(k), k > 0, nl)) != GP_OK) return st;
    return GP_OK;
  }
  if (p->rot.on) {
    // n + 1 linear steps; each rotating one moves the state to the other buffer, so
    // with an odd count the opening half step runs in place with the fixed-layout
    // passes and the state ends in psi
    int64_t first = 0;
    if ((n + 1) % 2 == 1) {
      if ((st = linear_all(p, psi, th, false, 0.0)) != GP_OK) return st;
      first = 1;
    }
    void* cur = psi;
    void* oth = p->rot.work;
    for (int64_t k = first; k <= n; ++k) {
      const int tau = (k == 0 || k == n) ? th : tf;
      if ((st = rot_linear(p, cur, oth, tau, k > 0, nl)) != GP_OK) return st;
      std::swap(cur, oth);
    }
    return GP_OK;
  }
  if ((st = linear_all(p, psi, th, false, 0.0)) != GP_OK) return st;
  for (int64_t s = 0; s < n; ++s)
    if ((st = linear_all(p, psi, s + 1 < n ? tf : th, true, nl)) != GP_OK) return st;
  return GP_OK;
}

// the v-th compiled rotating schedule of length n (registration order)
const RotEntry* find_rot(int n, int prec, int v = 0) {
  for (const auto& e : rot_registry())
    if (e.n == n && e.prec == prec && v-- == 0) return &e;
  return nullptr;
}

// tables of the rotating passes (the same for the three axes of a cube) and the
// workspace state
gp_status build_rot(gp_plan_s* p) {
  auto& R = p->rot;
  gp_status st;
  if (fault_injected("alloc")) return fail(GP_ERR_NOMEM, "rotating-pass workspace: injected fault");
  if (!R.tw && (st = upload_cplx(p, &R.tw, stage_twiddles(R.e->sched))) != GP_OK) return st;
  const double alpha = p->d.alpha, dt = p->d.dt;
  const double taus[NTAU] = {0.5 * dt, dt, -0.5 * dt, -dt};
  const int n = R.e->n;
  for (int t = 0; t < NTAU; ++t) {
    std::vector<double> m(2 * n);
    for (int k = 0; k < n; ++k) {
      const double kk = (double)kfreq(k, n);
      const double ph = alpha * kk * kk * taus[t];
      const int i = tab_idx(R.e->sched, k);
      const ct::Pair u = ct::unit_pair(std::cos(ph), std::sin(ph));
      m[2 * i] = u.c / n;
      m[2 * i + 1] = -u.s / n;
    }
    if (!R.mult[t] && (st = upload_c128(p, &R.mult[t], m)) != GP_OK) return st;
  }
  if (R.work) return GP_OK;
  hipError_t e = hipMalloc(&R.work, (size_t)p->ntot * p->S);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    R.work = nullptr;
    return fail(GP_ERR_NOMEM, "hipMalloc(%zu) of the rotating-pass workspace failed: %s", (size_t)p->ntot * p->S,
                hipGetErrorString(e));
  }
  return GP_OK;
}

gp_status fft3(gp_plan_s* p, const void* in, void* out, int dir) {
  gp_status st;
  const void* src = in;
  for (int a = 0; a < 3; ++a) {
    const double sc = dir < 0 ? 1.0 / p->ax[a].n : 1.0;
    if ((st = pass(p, a, dir < 0 ? V_FWD : V_INV, src, out, nullptr, 0.0, nullptr, sc)) != GP_OK) return st;
    src = out;
  }
  return GP_OK;
}

// unnormalised forward 3-D transform in place
gp_status fwd3_unnorm(gp_plan_s* p, void* f) {
  gp_status st;
  for (int a = 0; a < 3; ++a)
    if ((st = pass(p, a, V_FWD, f, f, nullptr, 0.0, nullptr, 1.0)) != GP_OK) return st;
  return GP_OK;
}
// unnormalised forward 3-D transform in place, the last pass multiplying by the 3-D
// propagator exp(-i alpha |k|^2 tau)/N^3 = m_x(k_x) m_y(k_y) m_z(k_z) before it stores
gp_status fwd3_mult3(gp_plan_s* p, void* f, int tau) {
  gp_status st;
  int last = -1;
  for (int a = 0; a < 3; ++a) if (p->ax[a].n > 1) last = a;
  for (int a = 0; a < last; ++a)
    if ((st = pass(p, a, V_FWD, f, f, nullptr, 0.0, nullptr, 1.0)) != GP_OK) return st;
  if (last < 0) {               // 1x1x1 grid: the multiplier alone
    launch_mult3(p->prec, f, 1, 1, 1, p->ax[0].nat[tau], p->ax[1].nat[tau], p->ax[2].nat[tau], p->stream);
    return check_launch(p);
  }
  const Axis& A = p->ax[last];
  PassArgs g{};
  g.in = f; g.out = f; g.tw = A.tw; g.scale = 1.0;
  g.aux = p->ax[0].nat[tau]; g.aux2 = p->ax[1].nat[tau]; g.aux3 = p->ax[2].nat[tau];
  g.npencils = A.npencils; g.inner = A.inner; g.outer = A.outer; g.es = A.es;
  g.axis = last; g.nx = p->d.n[0]; g.ny = p->d.n[1];
  A.e->fn[A.kind][V_FWD_MULT3](g, A.blocks, 1, p->stream);
  return check_launch(p);
}
gp_status inv3_unnorm(gp_plan_s* p, void* f) {
  gp_status st;
  for (int a = 0; a < 3; ++a)
    if ((st = pass(p, a, V_INV, f, f, nullptr, 0.0, nullptr, 1.0)) != GP_OK) return st;
  return GP_OK;
}

void* field(const gp_plan_s* p, void* work, int i) { return (char*)work + (size_t)i * p->ntot * p->S; }

// derivative passes psi -> F0..F2 with kinetic partials
gp_status derivatives(gp_plan_s* p, const void* psi, void* work, bool kin) {
  gp_status st;
  double* kp = p->kin_part;
  for (int a = 0; a < 3; ++a) {
    void* out = field(p, work, a);
    if (p->ax[a].n == 1) {
      HIPCHK(p, hipMemsetAsync(out, 0, p->ntot * p->S, p->stream));
      continue;
    }
    if ((st = pass(p, a, kin ? V_PROP_KIN : V_PROP, psi, out, p->ax[a].deriv, 0.0, nullptr, 1.0, kin ? kp : nullptr)) !=
        GP_OK)
      return st;
    kp += p->ax[a].blocks;
  }
  return GP_OK;
}

gp_status diagnose(gp_plan_s* p, const void* psi, void* work) {
  gp_status st;
  if ((st = derivatives(p, psi, work, true)) != GP_OK) return st;
  void* f0 = field(p, work, 0);
  void* f1 = field(p, work, 1);
  void* f2 = field(p, work, 2);
  void* f3 = field(p, work, 3);
  launch_diag_fields(p->prec, psi, f0, f1, f2, f3, p->ntot, p->d.alpha, p->field_part, p->field_blocks, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  for (void* f : {f0, f1, f2, f3})
    if ((st = fwd3_unnorm(p, f)) != GP_OK) return st;
  launch_spectral(p->prec, f0, f1, f2, f3, p->d.n[0], p->d.n[1], p->d.n[2], p->d.alpha, p->d.beta, p->nshell,
                  p->spec_blocks, p->bins_part, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  // fixed-order reductions of every partial into red = [kin_x, kin_y, kin_z, field[3], spectra[4][nshell]]
  const double nt = (double)p->ntot;
  double* red = p->d_red;
  double* kp = p->kin_part;
  for (int a = 0; a < 3; ++a) {
    if (p->ax[a].n > 1) {
      launch_segsum(kp, p->ax[a].blocks, 1, red + a, p->stream);
      kp += p->ax[a].blocks;
    } else {
      HIPCHK(p, hipMemsetAsync(red + a, 0, sizeof(double), p->stream));
    }
  }
  launch_segsum(p->field_part, p->field_blocks, 3, red + 3, p->stream);
  launch_segsum(p->bins_part, p->spec_blocks, 4 * p->nshell, red + 6, p->stream);
  launch_finalize_diag(red, 1.0 / (nt * p->ax[0].n), 1.0 / (nt * p->ax[1].n), 1.0 / (nt * p->ax[2].n), p->nshell,
                       p->d.alpha, p->d.beta, nt, p->d_result, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  const size_t bytes = (7 + 4 * (size_t)p->nshell) * sizeof(double);
  HIPCHK(p, hipMemcpyAsync(p->h_result, p->d_result, bytes, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return GP_OK;
}

gp_status copy_energies(gp_plan_s* p, gp_energy* out) {
  const double* r = p->h_result;
  gp_energy e{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
  if (out) *out = e;
  for (int i = 0; i < 7; ++i)
    if (!std::isfinite(r[i])) return fail(GP_ERR_NONFINITE, "diagnostic %d is not finite", i);
  return GP_OK;
}

}  // namespace

// Used by the entry point that allocates nothing (gp_noalloc.hip): argument checks
// of gp_energies for a workspace of at most max_bytes, the energies on a given
// workspace, and the error message of a failure found there.
size_t energies_work_bytes(const gp_plan_s* p) { return 4 * (size_t)p->ntot * p->S; }

gp_status energies_static_args(gp_plan_s* p, const void* psi, const gp_energy* out, size_t max_bytes) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi || !out) return fail(GP_ERR_ARG, "null argument");
  const size_t need = energies_work_bytes(p);
  if (need > max_bytes)
    return fail(GP_ERR_ARG, "grid needs %zu bytes of diagnostics workspace; the static workspace holds %zu", need,
                max_bytes);
  return GP_OK;
}

gp_status energies_on(gp_plan_s* p, const void* psi, void* work, gp_energy* out) {
  gp_status st = diagnose(p, psi, work);
  if (st != GP_OK) return st;
  return copy_energies(p, out);
}

gp_status report_error(gp_status st, const char* msg) { return fail(st, "%s", msg); }

}  // namespace gpk

// =================================================================== C ABI
extern "C" {

gp_status gp_plan(const gp_desc* d, void* hip_stream, gp_plan_t** out) {
  if (!out) return fail(GP_ERR_ARG, "null output pointer");
  *out = nullptr;
  gp_status st = validate_desc(d);
  if (st != GP_OK) return st;
  auto* p = new gp_plan_s();
  st = plan_init(p, d, (hipStream_t)hip_stream);
  if (st != GP_OK) {
    std::string msg = g_err;
    plan_free(p);
    g_err = msg;
    return st;
  }
  *out = p;
  g_err.clear();
  return GP_OK;
}

gp_status gp_plan_destroy(gp_plan_t* p) {
  if (!p) return fail(GP_ERR_ARG, "null plan");
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  plan_free(p);
  return GP_OK;
}

size_t gp_state_bytes(const gp_plan_t* p, int32_t run) {
  if (!p) return 0;
  if (p->is_batch) {
    if (run < 0 || run >= (int32_t)p->runs.size()) return 0;
    return p->runs[run]->ntot * p->runs[run]->S;
  }
  return p->ntot * p->S;
}

size_t gp_work_bytes(const gp_plan_t* p) {
  if (!p) return 0;
  if (p->is_batch) {
    size_t m = 0;
    for (auto* r : p->runs) m = std::max(m, gp_work_bytes(r));
    return m;
  }
  return 5 * p->ntot * p->S;
}

int32_t gp_nshell(const gp_plan_t* p) { return p ? p->nshell : 0; }

const char* gp_last_error(void) { return g_err.c_str(); }

const char* gp_schedule_name(const gp_plan_t* p, int32_t axis) {
  if (!p || axis < 0) return "";
  if (p->is_batch) {         // run-major: index 6 * run + axis
    const size_t r = (size_t)axis / 6;
    return r < p->runs.size() ? p->runs[r]->sched_name[axis % 6].c_str() : "";
  }
  if (axis > 5) return "";
  return p->sched_name[axis].c_str();
}

int32_t gp_variant_count(int32_t n, int32_t prec) {
  int c = 0;
  for (const auto& e : registry()) if (e.n == n && e.prec == prec) ++c;
  return c;
}

gp_status gp_select_variant(gp_plan_t* p, int32_t axis, int32_t variant) {
  gp_status st = usable(p);
  if (st != GP_OK) return st;
  if (p->is_batch) {   // the xy choice for every run that has a plane schedule
    if (axis != 3) return fail(GP_ERR_STATE, "batch plan: axis schedules are chosen by gp_autotune");
    for (auto* r : p->runs)
      if (r->plane.e || variant == 0)
        if ((st = gp_select_variant(r, 3, variant)) != GP_OK) return st;
    drop_graphs(p);
    return GP_OK;
  }
  if (axis == 3) {   // xy plane: 0 = separate x and y passes, 1 = one plane pass
    if (variant == 0) {
      p->plane.on = false;
      p->sched_name[3] = "xy: separate passes";
      return GP_OK;
    }
    if (variant != 1) return fail(GP_ERR_ARG, "xy variant %d (0 = separate passes, 1 = plane pass)", variant);
    if (!p->plane.e)
      return fail(GP_ERR_UNSUPPORTED, "no xy-plane schedule for %dx%d (needs nx == ny with a compiled plane length)",
                  p->d.n[0], p->d.n[1]);
    HIPCHK(p, p->stream ? hipStreamSynchronize(p->stream) : hipDeviceSynchronize());
    if ((st = build_plane_tables(p)) != GP_OK) return st;
    p->plane.on = true;
    char nm[128];
    snprintf(nm, sizeof nm, "xy: plane N=%d T=%d R=%dx%dx%d", p->plane.e->n, p->plane.e->T, p->plane.e->radix[0],
             p->plane.e->radix[1], p->plane.e->radix[2]);
    p->sched_name[3] = nm;
    return GP_OK;
  }
  if (axis == 5) {   // linear steps: 0 = fixed layout, in place; 1 = layout-rotating passes
    if (variant == 0) {
      if (p->rot.work) {
        HIPCHK(p, p->stream ? hipStreamSynchronize(p->stream) : hipDeviceSynchronize());
        (void)hipFree(p->rot.work);
        p->rot.work = nullptr;
      }
      p->rot.on = false;
      p->sched_name[5] = "layout: fixed";
      return GP_OK;
    }
    if (variant < 1)
      return fail(GP_ERR_ARG, "layout variant %d (0 = fixed, 1.. = rotating, then mixed, schedules)", variant);
    const int n = p->d.n[0];
    const bool cube = p->d.n[1] == n && p->d.n[2] == n;
    if (!cube || !find_rot(n, p->prec))
      return fail(GP_ERR_UNSUPPORTED, "no layout-rotating schedule for %dx%dx%d (cubes of a compiled length only)",
                  p->d.n[0], p->d.n[1], p->d.n[2]);
    const int nrot = [&] { int k = 0; while (find_rot(n, p->prec, k)) ++k; return k; }();
    const bool mixed = variant > nrot;
    const RotEntry* e = find_rot(n, p->prec, mixed ? variant - nrot - 1 : variant - 1);
    if (!e) return fail(GP_ERR_ARG, "layout variant %d: %d rotating schedules for n = %d", variant, nrot, n);
    HIPCHK(p, p->stream ? hipStreamSynchronize(p->stream) : hipDeviceSynchronize());
    if (p->rot.e && (p->rot.e->sched.NS != e->sched.NS || p->rot.e->sched.radix[0] != e->sched.radix[0] ||
                     p->rot.e->sched.radix[1] != e->sched.radix[1] || p->rot.e->sched.radix[2] != e->sched.radix[2])) {
      p->rot.tw = nullptr;           // another radix order: other tables (the old ones are freed with the plan)
      for (auto& m : p->rot.mult) m = nullptr;
    }
    p->rot.e = e;
    if ((st = build_rot(p)) != GP_OK) return st;
    p->rot.on = true;
    p->rot.mixed = mixed;
    char nm[128];
    snprintf(nm, sizeof nm, "layout: %s N=%d T=%d W=%d R=%dx%dx%d", mixed ? "rotating+contiguous" : "rotating", e->n,
             e->sched.T, e->sched.W, e->sched.radix[0], e->sched.radix[1], e->sched.radix[2]);
    p->sched_name[5] = nm;
    return GP_OK;
  }
  if (axis == 4) {   // which axis pass carries the nonlinear prologue: 0, 1, 2 = x, y, z
    if (variant < 0 || variant > 2) return fail(GP_ERR_ARG, "nonlinear carrier %d (0, 1, 2 = x, y, z)", variant);
    if (p->ax[variant].n == 1) return fail(GP_ERR_ARG, "nonlinear carrier: axis %d has length 1", variant);
    p->nl_axis = variant;
    p->sched_name[4] = std::string("nl: ") + "xyz"[variant] + " pass";
    return GP_OK;
  }
  if (axis < 0 || axis > 2) return fail(GP_ERR_ARG, "axis %d", axis);
  if (p->ax[axis].n == 1) return variant == 0 ? GP_OK : fail(GP_ERR_ARG, "axis of length 1 has one variant");
  const PassEntry* e = find_entry(p->ax[axis].n, p->prec, variant);
  if (!e) return fail(GP_ERR_ARG, "no variant %d for n = %d", variant, p->ax[axis].n);
  // the radix order defines the order of the tables: rebuild them, and drop the
  // one-off sub-step tables built for the previous order
  HIPCHK(p, p->stream ? hipStreamSynchronize(p->stream) : hipDeviceSynchronize());
  for (auto it = p->substep_tables.begin(); it != p->substep_tables.end();)
    it = it->first.first == axis ? p->substep_tables.erase(it) : std::next(it);
  const long old_blocks = p->ax[axis].blocks;
  if ((st = setup_axis(p, axis, variant)) != GP_OK) return st;
  if ((st = build_tables(p, axis)) != GP_OK) return st;
  if ((long)p->ax[axis].blocks > old_blocks) {
    const long kin_n = (long)p->ax[0].blocks + p->ax[1].blocks + p->ax[2].blocks;
    if ((st = dev_alloc(p, (void**)&p->kin_part, kin_n * sizeof(double))) != GP_OK) return st;
  }
  return GP_OK;
}

gp_status gp_init_phase(gp_plan_t* p, const double* theta, void* psi) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!theta || !psi) return fail(GP_ERR_ARG, "null theta or psi");
  launch_init_phase(p->prec, theta, psi, p->ntot, p->stream);
  return check_launch(p);
}

gp_status gp_init_rvr(gp_plan_t* p, const double* pairs, int32_t npairs, double xi, void* psi) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!pairs || !psi || npairs < 0) return fail(GP_ERR_ARG, "null argument or negative pair count");
  if (!(xi > 0.0) || !std::isfinite(xi)) return fail(GP_ERR_ARG, "core width xi must be positive");
  // host pair table -> device, in the layout of the kernel's ring parameters
  struct RP { double R, d, X, Y, Z; int perm; };
  if (ringpar_bytes() != sizeof(RP)) return fail(GP_ERR_STATE, "ring parameter layout mismatch");
  std::vector<RP> h(std::max(1, npairs));
  for (int q = 0; q < npairs; ++q) {
    const double* v = pairs + 6 * q;
    const int perm = (int)v[5];
    if (perm < 0 || perm > 5 || !(v[0] > 0.0)) return fail(GP_ERR_ARG, "pair %d: radius must be > 0, perm in 0..5", q);
    h[q] = RP{v[0], v[1], v[2], v[3], v[4], perm};
  }
  void* d = nullptr;
  HIPCHK(p, hipMalloc(&d, h.size() * sizeof(RP)));
  hipError_t e = hipMemcpyAsync(d, h.data(), h.size() * sizeof(RP), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) {
    const double s201 = std::sqrt(201.0);
    launch_init_rvr(p->prec, d, npairs, xi, (73.0 + 3.0 * s201) / 352.0, (6.0 + s201) / 528.0, (21.0 + s201) / 96.0,
                    p->d.n[0], p->d.n[1], p->d.n[2], psi, p->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  (void)hipFree(d);
  if (e != hipSuccess) { p->broken = true; return fail(GP_ERR_HIP, "gp_init_rvr: %s", hipGetErrorString(e)); }
  return GP_OK;
}

gp_status gp_substep_linear(gp_plan_t* p, void* psi, int32_t axis, double s) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi) return fail(GP_ERR_ARG, "null psi");
  if (axis < 0 || axis > 2) return fail(GP_ERR_ARG, "axis %d", axis);
  if (!std::isfinite(s)) return fail(GP_ERR_ARG, "non-finite s");
  Axis& A = p->ax[axis];
  if (A.n == 1) return GP_OK;
  if (p->substep_tables.size() > 256) return fail(GP_ERR_ARG, "too many distinct sub-step lengths on one plan");
  // table for this s (one-off; the step loop uses the cached dt/2 and dt tables)
  const int n = A.n;
  std::vector<double> m(2 * n);
  for (int k = 0; k < n; ++k) {
    const double kk = (double)kfreq(k, n);
    const double ph = p->d.alpha * kk * kk * s;
    const int ps = tab_idx(*A.e, k);
    const ct::Pair u = ct::unit_pair(std::cos(ph), std::sin(ph));
    m[2 * ps] = u.c / n;
    m[2 * ps + 1] = -u.s / n;
  }
  void*& tab = p->substep_tables[{axis, s}];
  if (!tab && (st = upload_c128(p, &tab, m)) != GP_OK) return st;
  return pass(p, axis, V_PROP, psi, psi, tab);
}

gp_status gp_substep_nonlinear(gp_plan_t* p, void* psi, double s) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi) return fail(GP_ERR_ARG, "null psi");
  if (!std::isfinite(s)) return fail(GP_ERR_ARG, "non-finite s");
  launch_nonlinear(p->prec, psi, p->ntot, p->d.beta * s, p->stream);
  return check_launch(p);
}

gp_status gp_step_n(gp_plan_t* p, void* psi, int64_t nsteps) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (p->is_batch) return fail(GP_ERR_STATE, "batch plan: use gp_step_n_batch");
  if (!psi) return fail(GP_ERR_ARG, "null psi");
  return step_n(p, psi, nsteps);
}

gp_status gp_step_literal_n(gp_plan_t* p, void* psi, int64_t nsteps) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi) return fail(GP_ERR_ARG, "null psi");
  const bool back = nsteps < 0;
  const int64_t n = back ? -nsteps : nsteps;
  const int th = back ? TAU_MH : TAU_H;
  const double nl = p->d.beta * (back ? -p->d.dt : p->d.dt);
  for (int64_t s = 0; s < n; ++s) {
    for (int half = 0; half < 2; ++half) {
      if ((st = fwd3_mult3(p, psi, th)) != GP_OK) return st;
      if ((st = inv3_unnorm(p, psi)) != GP_OK) return st;
      if (half == 0) {
        launch_nonlinear(p->prec, psi, p->ntot, nl, p->stream);
        if ((st = check_launch(p)) != GP_OK) return st;
      }
    }
  }
  return GP_OK;
}

gp_status gp_fft3(gp_plan_t* p, const void* in, void* out, int32_t dir) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!in || !out) return fail(GP_ERR_ARG, "null field");
  if (dir != -1 && dir != 1) return fail(GP_ERR_ARG, "dir must be -1 or +1");
  return fft3(p, in, out, dir);
}

gp_status gp_copy_state(gp_plan_t* p, const void* src, void* dst) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!src || !dst) return fail(GP_ERR_ARG, "null field");
  launch_copy16(src, dst, p->ntot * (p->prec == P_C128 ? 16L : 8L), p->stream);
  return check_launch(p);
}

gp_status gp_energies(gp_plan_t* p, const void* psi, void* work, gp_energy* out) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi || !work || !out) return fail(GP_ERR_ARG, "null argument");
  if ((st = diagnose(p, psi, work)) != GP_OK) return st;
  return copy_energies(p, out);
}

gp_status gp_spectra(gp_plan_t* p, const void* psi, void* work, double* out, int32_t nshell, gp_energy* energies) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi || !work || !out) return fail(GP_ERR_ARG, "null argument");
  if (nshell != p->nshell) return fail(GP_ERR_ARG, "nshell %d != %d", nshell, p->nshell);
  if ((st = diagnose(p, psi, work)) != GP_OK) return st;
  memcpy(out, p->h_result + 7, 4 * (size_t)p->nshell * sizeof(double));
  st = copy_energies(p, energies);
  for (int i = 0; i < 4 * p->nshell && st == GP_OK; ++i)
    if (!std::isfinite(out[i])) st = fail(GP_ERR_NONFINITE, "spectrum entry %d is not finite", i);
  return st;
}

gp_status gp_structure_fn(gp_plan_t* p, const void* psi, void* work, int32_t p_order, double* out) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi || !work || !out) return fail(GP_ERR_ARG, "null argument");
  if (p_order != 2) return fail(GP_ERR_UNSUPPORTED, "structure function order %d (only 2)", p_order);
  const int n = p->d.n[0];
  if (p->d.n[1] != n || p->d.n[2] != n) return fail(GP_ERR_UNSUPPORTED, "structure function needs a cubic grid");
  if (n < 2) return fail(GP_ERR_UNSUPPORTED, "structure function needs n >= 2");
  void* f = field(p, work, 0);
  const long div[3] = {1, n, (long)n * n};
  for (int a = 0; a < 3; ++a) {
    // F_a(|psi|^2 - 1), natural order along axis a
    if ((st = pass(p, a, V_FWD_DENSITY, psi, f, nullptr, 0.0, nullptr, 1.0)) != GP_OK) return st;
    launch_axis_power(p->prec, f, p->ntot, div[a], n, p->pow_blocks, p->pow_chunk,
                      p->power_part + (size_t)a * p->pow_blocks * n, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
  }
  // power_part = [axis][k][block] -> reduced pk[axis][k] (in d_red, which holds >= 3 n doubles)
  launch_segsum(p->power_part, p->pow_blocks, 3 * n, p->d_pk, p->stream);
  launch_structure_final(p->d_pk, n, (double)p->ntot, p->d_result, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  HIPCHK(p, hipMemcpyAsync(p->h_result, p->d_result, (n / 2) * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  memcpy(out, p->h_result, (n / 2) * sizeof(double));
  return GP_OK;
}

gp_status gp_structure_fn_velocity(gp_plan_t* p, const void* psi, void* work, int32_t p_order, double* out,
                                   double* mean_v2) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (p->is_batch) return fail(GP_ERR_STATE, "batch plan: diagnostics run on single plans");
  if (!psi || !work || !out) return fail(GP_ERR_ARG, "null argument");
  if (p_order != 2) return fail(GP_ERR_UNSUPPORTED, "structure function order %d (only 2)", p_order);
  const int n = p->d.n[0];
  if (p->d.n[1] != n || p->d.n[2] != n) return fail(GP_ERR_UNSUPPORTED, "structure function needs a cubic grid");
  if (n < 2) return fail(GP_ERR_UNSUPPORTED, "structure function needs n >= 2");
  if ((st = derivatives(p, psi, work, false)) != GP_OK) return st;
  void* f[3] = {field(p, work, 0), field(p, work, 1), field(p, work, 2)};
  launch_velocity_fields(p->prec, psi, f[0], f[1], f[2], p->ntot, p->d.alpha, p->field_part, p->field_blocks, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  const long div[3] = {1, n, (long)n * n};
  for (int a = 0; a < 3; ++a) {
    // F_a(v_a), natural order along axis a
    if ((st = pass(p, a, V_FWD, f[a], f[a], nullptr, 0.0, nullptr, 1.0)) != GP_OK) return st;
    launch_axis_power(p->prec, f[a], p->ntot, div[a], n, p->pow_blocks, p->pow_chunk,
                      p->power_part + (size_t)a * p->pow_blocks * n, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
  }
  const int half = n / 2;
  launch_segsum(p->power_part, p->pow_blocks, 3 * n, p->d_pk, p->stream);
  launch_structure_axes(p->d_pk, n, (double)p->ntot, p->d_result, p->stream);
  launch_segsum(p->field_part, p->field_blocks, 3, p->d_result + 3 * half, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  HIPCHK(p, hipMemcpyAsync(p->h_result, p->d_result, (3 * half + 3) * sizeof(double), hipMemcpyDeviceToHost,
                           p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  memcpy(out, p->h_result, 3 * half * sizeof(double));
  if (mean_v2)
    for (int a = 0; a < 3; ++a) mean_v2[a] = p->h_result[3 * half + a] / (double)p->ntot;
  for (int q = 0; q < 3 * half; ++q)
    if (!std::isfinite(out[q])) return fail(GP_ERR_NONFINITE, "velocity structure function is not finite");
  return GP_OK;
}

gp_status gp_mach(gp_plan_t* p, const void* psi, void* work, double* out) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (p->is_batch) return fail(GP_ERR_STATE, "batch plan: diagnostics run on single plans");
  if (!psi || !work || !out) return fail(GP_ERR_ARG, "null argument");
  if (!(p->d.alpha * p->d.beta > 0.0)) return fail(GP_ERR_ARG, "Mach numbers need alpha beta > 0");
  if ((st = derivatives(p, psi, work, false)) != GP_OK) return st;
  launch_mach_partials(p->prec, psi, field(p, work, 0), field(p, work, 1), field(p, work, 2), p->ntot, p->d.alpha,
                       p->loss_part, p->field_part, p->field_blocks, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  launch_segsum(p->loss_part, p->field_blocks, 1, p->d_result, p->stream);
  launch_segmax(p->field_part, p->field_blocks, p->d_result + 1, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  HIPCHK(p, hipMemcpyAsync(p->h_result, p->d_result, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  const double c = std::sqrt(2.0 * p->d.alpha * p->d.beta);
  out[0] = std::sqrt(p->h_result[1]) / c;
  out[1] = std::sqrt(p->h_result[0] / (double)p->ntot) / c;
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return fail(GP_ERR_NONFINITE, "Mach number is not finite");
  return GP_OK;
}

// out = d/dx_a in (spectral first derivative, Nyquist entry 0); in == out allowed
static gp_status deriv_pass(gp_plan_s* p, int a, const void* in, void* out) {
  if (p->ax[a].n == 1) {
    HIPCHK(p, hipMemsetAsync(out, 0, p->ntot * p->S, p->stream));
    return GP_OK;
  }
  return pass(p, a, V_PROP, in, out, p->ax[a].deriv, 0.0, nullptr, 1.0);
}

size_t gp_helicity_work_bytes(const gp_plan_t* p) {
  if (!p || p->is_batch) return 0;
  return 8 * p->ntot * p->S;
}

gp_status gp_helicity(gp_plan_t* p, const void* psi, void* work, double* out, double* spec, int32_t nshell) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (p->is_batch) return fail(GP_ERR_STATE, "batch plan: diagnostics run on single plans");
  if (!psi || !work || !out) return fail(GP_ERR_ARG, "null argument");
  if (spec && nshell != p->nshell) return fail(GP_ERR_ARG, "nshell %d != %d", nshell, p->nshell);
  void* S[8];
  for (int k = 0; k < 8; ++k) S[k] = field(p, work, k);
  const long n = p->ntot;
  const double al = p->d.alpha;
  // S0..S2 = grad psi
  if ((st = derivatives(p, psi, work, false)) != GP_OK) return st;
  // vorticity: S3..S5 = packed velocity components, differentiated in place, then
  // omega into S6 (x + i y) and S7 (z)
  launch_hel_pack(p->prec, psi, S[0], S[1], S[2], S[3], S[4], S[5], n, al, p->loss_part, p->field_blocks, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  double* g2_sum = p->d_result + 2 + 2 * (size_t)p->nshell;          // sum |grad psi|^2 (floor of v_reg)
  launch_segsum(p->loss_part, p->field_blocks, 1, g2_sum, p->stream);
  if ((st = deriv_pass(p, 1, S[3], S[3])) != GP_OK) return st;
  if ((st = deriv_pass(p, 2, S[4], S[4])) != GP_OK) return st;
  if ((st = deriv_pass(p, 0, S[5], S[5])) != GP_OK) return st;
  launch_hel_omega(p->prec, S[3], S[4], S[5], S[6], S[7], n, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  // J_i = Im(sum_j (d_i d_j psi)(d_j psi)*) into S4 (J_x + i J_y), S5 (J_z), one Hessian
  // entry at a time in S3: H_ij = d_i (d_j psi)
  struct Entry { int i, j; };
  const Entry hess[6] = {{0, 0}, {1, 1}, {2, 2}, {1, 0}, {2, 0}, {2, 1}};
  for (int e = 0; e < 6; ++e) {
    const int i = hess[e].i, j = hess[e].j;
    if ((st = deriv_pass(p, i, S[j], S[3])) != GP_OK) return st;
    // H_ij adds conj(d_j psi) H_ij to J_i and, off the diagonal, conj(d_i psi) H_ij to J_j
    launch_hel_acc(p->prec, S[3], S[j], i, i != j ? S[i] : S[j], i != j ? j : -1, e == 0, S[4], S[5], n, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
  }
  // v_reg into S3 (x + i y), S4 (z); physical-space sums of v.omega and v_reg.omega
  launch_hel_vreg(p->prec, psi, S[0], S[1], S[2], S[4], S[5], S[6], S[7], S[3], S[4], n, al, g2_sum,
                  p->field_part, p->field_blocks, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  launch_segsum(p->field_part, p->field_blocks, 2, p->d_result, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  if (spec) {
    // spectra: v into S0 (x + i y), S1 (z); transforms of v, v_reg, omega; shell bins
    launch_hel_vpack(p->prec, psi, S[0], S[1], S[2], n, al, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
    for (int k : {0, 1, 3, 4, 6, 7})
      if ((st = fwd3_unnorm(p, S[k])) != GP_OK) return st;
    launch_hel_spectral(p->prec, S[0], S[1], S[3], S[4], S[6], S[7], p->d.n[0], p->d.n[1], p->d.n[2], p->nshell,
                        p->spec_blocks, p->spec_chunk, p->bins_part, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
    launch_segsum(p->bins_part, p->spec_blocks, 2 * p->nshell, p->d_result + 2, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
  }
  const size_t cnt = 2 + (spec ? 2 * (size_t)p->nshell : 0);
  HIPCHK(p, hipMemcpyAsync(p->h_result, p->d_result, cnt * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  out[0] = p->h_result[0] / (double)n;
  out[1] = p->h_result[1] / (double)n;
  if (spec) memcpy(spec, p->h_result + 2, 2 * (size_t)p->nshell * sizeof(double));
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return fail(GP_ERR_NONFINITE, "helicity is not finite");
  return GP_OK;
}

// the z-derivative pass with the explicit part of the imaginary-time step fused after
// its inverse transform: out = n(phi, d/dx phi, d/dy phi, d/dz phi, v)
static gp_status argle_z_pass(gp_plan_s* p, const void* phi, const void* d0, const void* d1, const void* v,
                              void* out) {
  Axis& A = p->ax[2];
  PassArgs g{};
  g.in = phi; g.out = out; g.mult = A.deriv; g.tw = A.tw; g.aux = phi; g.aux2 = d0; g.aux3 = d1; g.vel = v;
  g.ksq = A.ksq; g.nl_coef = p->d.beta; g.q4a = 1.0 / (4.0 * p->d.alpha); g.scale = 1.0;
  g.npencils = A.npencils; g.inner = A.inner; g.outer = A.outer; g.es = A.es;
  A.e->fn[A.kind][V_PROP_ARGLE](g, A.blocks, 1, p->stream);
  return check_launch(p);
}

// nsteps steps of the semi-implicit backward Euler scheme; work slots 0..2.  With a
// z axis the explicit part n comes out of the z-derivative pass (d/dz never reaches
// memory); otherwise a pointwise kernel forms it and overwrites d/dz in place.
static gp_status argle_steps(gp_plan_s* p, void* phi, const void* v, double dtau, int64_t nsteps, void* work) {
  gp_status st;
  void* d0 = field(p, work, 0);
  void* d1 = field(p, work, 1);
  void* d2 = field(p, work, 2);
  void* q = d2;
  const bool fused = p->ax[2].n > 1;
  const double a = 0.5 * dtau * p->d.alpha, inv_n = 1.0 / (double)p->ntot;
  for (int64_t s = 0; s < nsteps; ++s) {
    if (fused) {
      for (int ax = 0; ax < 2; ++ax) {
        void* out = field(p, work, ax);
        if (p->ax[ax].n == 1) HIPCHK(p, hipMemsetAsync(out, 0, p->ntot * p->S, p->stream));
        else if ((st = pass(p, ax, V_PROP, phi, out, p->ax[ax].deriv)) != GP_OK) return st;
      }
      if ((st = argle_z_pass(p, phi, d0, d1, v, q)) != GP_OK) return st;
    } else {
      if ((st = derivatives(p, phi, work, false)) != GP_OK) return st;
      launch_argle_explicit(p->prec, phi, d0, d1, d2, v, q, p->ntot, p->d.alpha, p->d.beta, p->stream);
      if ((st = check_launch(p)) != GP_OK) return st;
    }
    if ((st = fwd3_unnorm(p, phi)) != GP_OK) return st;
    if ((st = fwd3_unnorm(p, q)) != GP_OK) return st;
    launch_argle_solve(p->prec, phi, q, p->d.n[0], p->d.n[1], p->d.n[2], a, dtau, inv_n, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
    if ((st = inv3_unnorm(p, phi)) != GP_OK) return st;
  }
  return GP_OK;
}

// E_v (synchronizes); work slots 0..2
static gp_status argle_energy(gp_plan_s* p, const void* phi, const void* v, void* work, double* energy_v) {
  gp_status st;
  if ((st = derivatives(p, phi, work, false)) != GP_OK) return st;
  launch_argle_energy(p->prec, phi, field(p, work, 0), field(p, work, 1), field(p, work, 2), v, p->ntot, p->d.alpha,
                      p->d.beta, p->loss_part, p->field_blocks, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  launch_segsum(p->loss_part, p->field_blocks, 1, p->d_result, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  HIPCHK(p, hipMemcpyAsync(p->h_result, p->d_result, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  *energy_v = 2.0 * p->d.alpha * p->h_result[0] / (double)p->ntot;
  if (!std::isfinite(*energy_v)) return fail(GP_ERR_NONFINITE, "E_v is not finite");
  return GP_OK;
}

static gp_status argle_args(gp_plan_s* p, const void* phi, const void* v, const void* work) {
  gp_status st = usable(p);
  if (st != GP_OK) return st;
  if (p->is_batch) return fail(GP_ERR_STATE, "batch plan: ARGLE runs on single plans");
  if (!phi || !v || !work) return fail(GP_ERR_ARG, "null argument");
  return GP_OK;
}

gp_status gp_argle_step(gp_plan_t* p, void* phi, const void* v, double dtau, int64_t nsteps, void* work) {
  gp_status st = argle_args(p, phi, v, work);
  if (st != GP_OK) return st;
  if (!std::isfinite(dtau) || dtau <= 0.0) return fail(GP_ERR_ARG, "dtau must be finite and positive");
  if (nsteps < 0) return fail(GP_ERR_ARG, "nsteps must be >= 0");
  return argle_steps(p, phi, v, dtau, nsteps, work);
}

gp_status gp_argle_energy(gp_plan_t* p, const void* phi, const void* v, void* work, double* energy_v) {
  gp_status st = argle_args(p, phi, v, work);
  if (st != GP_OK) return st;
  if (!energy_v) return fail(GP_ERR_ARG, "null argument");
  return argle_energy(p, phi, v, work, energy_v);
}

gp_status gp_argle_run(gp_plan_t* p, void* phi, const void* v, double dtau, int64_t max_steps, int64_t check_every,
                       double eps, void* work, gp_argle_report* report) {
  gp_status st = argle_args(p, phi, v, work);
  if (st != GP_OK) return st;
  if (!report) return fail(GP_ERR_ARG, "null argument");
  if (!std::isfinite(dtau) || dtau <= 0.0) return fail(GP_ERR_ARG, "dtau must be finite and positive");
  if (max_steps < 0) return fail(GP_ERR_ARG, "max_steps must be >= 0");
  if (check_every < 1) return fail(GP_ERR_ARG, "check_every must be >= 1");
  if (std::isnan(eps)) return fail(GP_ERR_ARG, "eps is NaN");
  gp_argle_report r{0, std::nan(""), std::nan(""), 0.0, 0};
  void* old = field(p, work, 4);
  const size_t bytes = (size_t)p->ntot * p->S;
  bool have_e = false;
  while (r.steps < max_steps) {
    const int64_t next = std::min<int64_t>((r.steps / check_every + 1) * check_every, max_steps);   // check step
    if ((st = argle_steps(p, phi, v, dtau, next - r.steps - 1, work)) != GP_OK) return st;
    double e_old, e_new, sup2;
    if ((st = argle_energy(p, phi, v, work, &e_old)) != GP_OK) return st;
    HIPCHK(p, hipMemcpyAsync(old, phi, bytes, hipMemcpyDeviceToDevice, p->stream));
    if ((st = argle_steps(p, phi, v, dtau, 1, work)) != GP_OK) return st;
    launch_sup_diff2(p->prec, phi, old, p->ntot, p->field_part, p->field_blocks, p->d_result, p->stream);
    if ((st = check_launch(p)) != GP_OK) return st;
    HIPCHK(p, hipMemcpyAsync(p->h_result, p->d_result, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
    sup2 = p->h_result[0];
    if ((st = argle_energy(p, phi, v, work, &e_new)) != GP_OK) return st;
    r.steps = next;
    r.crit_sup = std::sqrt(sup2) / dtau;
    r.crit_energy = std::fabs(e_new - e_old) / (dtau * e_old);
    r.e_v = e_new;
    have_e = true;
    if (!std::isfinite(r.crit_sup)) return fail(GP_ERR_NONFINITE, "ARGLE update is not finite at step %lld", (long long)next);
    if (r.crit_sup <= eps) { r.converged = 1; break; }
  }
  if (!have_e && (st = argle_energy(p, phi, v, work, &r.e_v)) != GP_OK) return st;
  *report = r;
  return GP_OK;
}

gp_status gp_loss_ekin_i_shells(gp_plan_t* p, const void* psi, void* work, int32_t smin, int32_t smax, double* J,
                                void* lam) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi || !work || !J || !lam) return fail(GP_ERR_ARG, "null argument");
  if (smin < 0 || smax < smin) return fail(GP_ERR_ARG, "bad shell range %d..%d", smin, smax);
  void* d0 = field(p, work, 0);
  void* d1 = field(p, work, 1);
  void* d2 = field(p, work, 2);
  void* g0 = field(p, work, 3);
  void* g1 = field(p, work, 4);
  if ((st = derivatives(p, psi, work, false)) != GP_OK) return st;
  launch_loss_fields(p->prec, psi, d0, d1, d2, g0, g1, p->ntot, p->d.alpha, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  if ((st = fwd3_unnorm(p, g0)) != GP_OK) return st;
  if ((st = fwd3_unnorm(p, g1)) != GP_OK) return st;
  launch_loss_spectral(p->prec, g0, g1, p->d.n[0], p->d.n[1], p->d.n[2], smin, smax, p->loss_part, p->field_blocks,
                       p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  if ((st = inv3_unnorm(p, g0)) != GP_OK) return st;
  if ((st = inv3_unnorm(p, g1)) != GP_OK) return st;
  launch_loss_lambda1(p->prec, psi, d0, d1, d2, g0, g1, lam, p->ntot, p->d.alpha, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  // d_j <- d/dj (h_j psi), in place
  for (int a = 0; a < 3; ++a) {
    void* f = field(p, work, a);
    if (p->ax[a].n == 1) {
      HIPCHK(p, hipMemsetAsync(f, 0, p->ntot * p->S, p->stream));
      continue;
    }
    if ((st = pass(p, a, V_PROP, f, f, p->ax[a].deriv)) != GP_OK) return st;
  }
  launch_loss_lambda2(p->prec, lam, d0, d1, d2, p->ntot, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  launch_segsum(p->loss_part, p->field_blocks, 1, p->d_result, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  HIPCHK(p, hipMemcpyAsync(p->h_result, p->d_result, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  *J = p->h_result[0];
  if (!std::isfinite(*J)) return fail(GP_ERR_NONFINITE, "loss is not finite");
  return GP_OK;
}

gp_status gp_adjoint_step_n(gp_plan_t* p, const void* psi_seg_start, void* lam, int64_t nsteps, void* tape) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi_seg_start || !lam || !tape) return fail(GP_ERR_ARG, "null argument");
  if (nsteps < 0) return fail(GP_ERR_ARG, "nsteps must be >= 0");
  if (p->prec != P_C128) return fail(GP_ERR_UNSUPPORTED, "the adjoint is compiled for complex128 only");
  if (nsteps == 0) return GP_OK;
  const size_t sb = p->ntot * p->S;
  auto slot = [&](int64_t i) { return (void*)((char*)tape + (size_t)i * sb); };
  const double nl = p->d.beta * p->d.dt;
  const int c = first_real_axis(p);
  // forward recompute: phi_0 = L(h) psi_0, phi_{n+1} = L(dt) N(phi_n), stored in the tape
  {
    const void* src = psi_seg_start;
    bool first = true;
    for (int a = 0; a < 3; ++a) {
      if (p->ax[a].n == 1) continue;
      if ((st = pass(p, a, V_PROP, first ? src : slot(0), slot(0), p->ax[a].mult[TAU_H])) != GP_OK) return st;
      first = false;
    }
    if (first) {  // 1x1x1 grid
      launch_scale_copy(p->prec, src, slot(0), p->ntot, 1.0, p->stream);
      if ((st = check_launch(p)) != GP_OK) return st;
    }
  }
  for (int64_t s = 0; s + 1 < nsteps; ++s) {
    if (c < 0) {
      launch_scale_copy(p->prec, slot(s), slot(s + 1), p->ntot, 1.0, p->stream);
      launch_nonlinear(p->prec, slot(s + 1), p->ntot, nl, p->stream);
      if ((st = check_launch(p)) != GP_OK) return st;
      continue;
    }
    for (int a = 0; a < 3; ++a) {
      if (p->ax[a].n == 1) continue;
      const bool carrier = (a == c);
      if ((st = pass(p, a, carrier ? V_PROP_NL : V_PROP, carrier ? slot(s) : slot(s + 1), slot(s + 1),
                     p->ax[a].mult[TAU_DT], nl)) != GP_OK)
        return st;
    }
  }
  // backward: lam <- L(-h); then per step n (reverse): N'(phi_n)^dagger fused, L(-dt) or L(-h)
  if ((st = linear_all(p, lam, TAU_MH, false, 0.0)) != GP_OK) return st;
  for (int64_t s = nsteps - 1; s >= 0; --s) {
    const int tau = s > 0 ? TAU_MDT : TAU_MH;
    if (c < 0) {
      return fail(GP_ERR_UNSUPPORTED, "adjoint on a 1x1x1 grid");
    }
    for (int a = 0; a < 3; ++a) {
      if (p->ax[a].n == 1) continue;
      const bool carrier = (a == c);
      if ((st = pass(p, a, carrier ? V_PROP_ADJ : V_PROP, lam, lam, p->ax[a].mult[tau], nl, carrier ? slot(s) : nullptr)) !=
          GP_OK)
        return st;
    }
  }
  return GP_OK;
}

gp_status gp_phase_grad(gp_plan_t* p, const void* psi0, const void* lam0, double* dJ_dtheta) {
  gp_status st = usable_single(p);
  if (st != GP_OK) return st;
  if (!psi0 || !lam0 || !dJ_dtheta) return fail(GP_ERR_ARG, "null argument");
  launch_phase_grad(p->prec, psi0, lam0, dJ_dtheta, p->ntot, p->stream);
  return check_launch(p);
}

// ----------------------------------------------------------------- ensemble
gp_status gp_plan_batch(const gp_desc* runs, int32_t nruns, void* hip_stream, gp_plan_t** out) {
  if (!out) return fail(GP_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!runs || nruns < 1) return fail(GP_ERR_ARG, "need at least one run");
  gp_status st;
  for (int i = 0; i < nruns; ++i) {
    if ((st = validate_desc(&runs[i])) != GP_OK) return st;
    if (runs[i].prec != runs[0].prec) return fail(GP_ERR_ARG, "all runs of a batch share one precision");
  }
  auto* p = new gp_plan_s();
  p->is_batch = true;
  p->prec = runs[0].prec;
  p->S = p->prec == GP_C128 ? 16 : 8;
  p->d = runs[0];
  p->stream = (hipStream_t)hip_stream;
  bool own_stream = false;
  if (!p->stream) {
    // graph capture needs a stream other than the legacy null stream; a blocking
    // stream keeps the null stream's order (work on either waits for the other), so
    // states written by the caller on the null stream before gp_step_n_batch, and
    // read on it afterwards, are ordered with the graph without any event
    hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamDefault);
    if (e != hipSuccess) { delete p; return fail(GP_ERR_HIP, "hipStreamCreate: %s", hipGetErrorString(e)); }
    own_stream = true;
  }
  for (int i = 0; i < nruns; ++i) {
    auto* r = new gp_plan_s();
    p->runs.push_back(r);
    if ((st = plan_init(r, &runs[i], p->stream)) != GP_OK) {
      std::string msg = g_err;
      p->own_stream = own_stream;
      plan_free(p);
      g_err = msg;
      return st;
    }
    // group runs of identical grid shape
    int g = -1;
    for (size_t j = 0; j < p->groups.size(); ++j) {
      const auto* r0 = p->runs[p->groups[j].members[0]];
      if (r0->d.n[0] == r->d.n[0] && r0->d.n[1] == r->d.n[1] && r0->d.n[2] == r->d.n[2]) g = (int)j;
    }
    if (g < 0) { p->groups.push_back({}); g = (int)p->groups.size() - 1; p->groups[g].n = r->d.n[0]; }
    p->groups[g].members.push_back(i);
  }
  p->nshell = p->runs[0]->nshell;
  p->ntot = p->runs[0]->ntot;
  p->own_stream = own_stream;
  // one capture branch per further size group, so the groups' launches of a step
  // graph are independent nodes that may run side by side
  for (size_t g = 1; g < p->groups.size(); ++g) {
    hipStream_t st2 = nullptr;
    hipEvent_t ev = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st2, hipStreamNonBlocking);
    if (e == hipSuccess) p->side.push_back(st2);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) p->join_ev.push_back(ev);
    if (e != hipSuccess) { plan_free(p); return fail(GP_ERR_HIP, "capture branch: %s", hipGetErrorString(e)); }
  }
  if (p->groups.size() > 1) {
    hipError_t e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
    if (e != hipSuccess) { plan_free(p); return fail(GP_ERR_HIP, "capture fork event: %s", hipGetErrorString(e)); }
  }
  *out = p;
  g_err.clear();
  return GP_OK;
}

// pointer tables of the grouped launches, both signs:
// RunPtrs[sign][axis][tau: 0 half step, 1 full step][member] per group
static gp_status batch_tables(gp_plan_s* p, void* const* psis) {
  // a launch of a recorded graph may still read the tables: let it finish
  HIPCHK(p, hipStreamSynchronize(p->stream));
  drop_graphs(p);
  for (auto& g : p->groups) {
    const size_t m = g.members.size();
    std::vector<RunPtrs> h(2 * 3 * 2 * m);
    for (int sg = 0; sg < 2; ++sg)
      for (int a = 0; a < 3; ++a)
        for (int t = 0; t < 2; ++t)
          for (size_t i = 0; i < m; ++i) {
            gp_plan_s* r = p->runs[g.members[i]];
            const int tau = sg ? (t == 0 ? TAU_MH : TAU_MDT) : (t == 0 ? TAU_H : TAU_DT);
            RunPtrs& e = h[((sg * 3 + a) * 2 + t) * m + i];
            e.in = psis[g.members[i]];
            e.out = psis[g.members[i]];
            e.mult = r->ax[a].mult[tau];
            e.nl_coef = r->d.beta * (sg ? -r->d.dt : r->d.dt);
            if (a == 0 && r->plane.on) {   // the x slot carries the plane pass's x and y tables
              e.mult = r->plane.mx[tau];
              e.mult2 = r->plane.my[tau];
            }
          }
    if (g.nptrs < h.size()) {
      if (g.d_ptrs) (void)hipFree(g.d_ptrs);
      g.d_ptrs = nullptr;
      g.nptrs = 0;
      HIPCHK(p, hipMalloc((void**)&g.d_ptrs, h.size() * sizeof(RunPtrs)));
      g.nptrs = h.size();
    }
    HIPCHK(p, hipMemcpy(g.d_ptrs, h.data(), h.size() * sizeof(RunPtrs), hipMemcpyHostToDevice));
  }
  p->graph_key.assign(psis, psis + p->runs.size());
  return GP_OK;
}

// record one step graph: slot 0 = L(h); 1 = N, L(h); 2 + j = (N, L(dt)) x 2^j, with the
// nonlinear rotation fused into each application's first pass; size group g > 0 is
// captured on its own branch (fork from and join into the plan's stream)
static gp_status batch_record(gp_plan_s* p, int sg, int slot) {
  const int64_t reps = slot < 2 ? 1 : (int64_t)1 << (slot - 2);
  const int t = slot < 2 ? 0 : 1;
  const bool nl = slot != 0;
  HIPCHK(p, hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  hipError_t ce = hipSuccess;
  if (p->groups.size() > 1) ce = hipEventRecord(p->fork_ev, p->stream);
  for (size_t gi = 0; gi < p->groups.size() && ce == hipSuccess; ++gi) {
    const auto& g = p->groups[gi];
    hipStream_t st = gi == 0 ? p->stream : p->side[gi - 1];
    if (gi > 0) ce = hipStreamWaitEvent(st, p->fork_ev, 0);
    if (ce != hipSuccess) break;
    gp_plan_s* r0 = p->runs[g.members[0]];
    const int c = first_real_axis(r0);
    const size_t m = g.members.size();
    auto ptrs = [&](int a) { return g.d_ptrs + ((sg * 3 + a) * 2 + t) * m; };
    for (int64_t k = 0; k < reps; ++k) {
      if (r0->plane.on) {      // every member of the group made the same choice
        PlaneArgs args{};
        args.batch = ptrs(0);
        args.tw = r0->plane.tw;
        r0->plane.e->fn[nl ? 1 : 0](args, (unsigned)r0->d.n[2], (unsigned)m, st);
        if (r0->ax[2].n > 1) {
          const Axis& A = r0->ax[2];
          PassArgs pa{};
          pa.batch = ptrs(2); pa.tw = A.tw; pa.ksq = A.ksq; pa.scale = 1.0;
          pa.npencils = A.npencils; pa.inner = A.inner; pa.outer = A.outer; pa.es = A.es;
          A.e->fn[A.kind][V_PROP](pa, A.blocks, (unsigned)m, st);
        }
        continue;
      }
      for (int a = 0; a < 3; ++a) {
        if (r0->ax[a].n == 1) continue;
        const Axis& A = r0->ax[a];
        PassArgs pa{};
        pa.batch = ptrs(a); pa.tw = A.tw; pa.ksq = A.ksq; pa.scale = 1.0;
        pa.npencils = A.npencils; pa.inner = A.inner; pa.outer = A.outer; pa.es = A.es;
        A.e->fn[A.kind][(nl && a == c) ? V_PROP_NL : V_PROP](pa, A.blocks, (unsigned)m, st);
      }
    }
    if (gi > 0) {
      ce = hipEventRecord(p->join_ev[gi - 1], st);
      if (ce == hipSuccess) ce = hipStreamWaitEvent(p->stream, p->join_ev[gi - 1], 0);
    }
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(p->stream, &graph);
  if (ce != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    p->broken = true;
    return fail(GP_ERR_HIP, "step graph capture: %s", hipGetErrorString(ce != hipSuccess ? ce : e));
  }
  e = hipGraphInstantiate(&p->gexec[sg][slot], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    p->gexec[sg][slot] = nullptr;
    p->broken = true;
    return fail(GP_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return GP_OK;
}

static gp_status batch_launch(gp_plan_s* p, int sg, int slot) {
  gp_status st;
  if (!p->gexec[sg][slot] && (st = batch_record(p, sg, slot)) != GP_OK) return st;
  HIPCHK(p, hipGraphLaunch(p->gexec[sg][slot], p->stream));
  return GP_OK;
}

gp_status gp_step_n_batch(gp_plan_t* p, void* const* psis, int64_t nsteps) {
  gp_status st = usable(p);
  if (st != GP_OK) return st;
  if (!p->is_batch) return fail(GP_ERR_STATE, "not a batch plan");
  if (!psis) return fail(GP_ERR_ARG, "null state array");
  for (size_t i = 0; i < p->runs.size(); ++i)
    if (!psis[i]) return fail(GP_ERR_ARG, "null state of run %zu", i);
  if (nsteps == 0) return GP_OK;
  for (const auto* r : p->runs)
    if (first_real_axis(r) < 0) return fail(GP_ERR_UNSUPPORTED, "1x1x1 runs cannot be batched");
  const bool same = p->graph_key.size() == p->runs.size() &&
                    std::equal(p->graph_key.begin(), p->graph_key.end(), psis);
  if (!same && (st = batch_tables(p, psis)) != GP_OK) return st;
  // L(h) [N L(dt)]^(n-1) N L(h): the body's n - 1 applications as recorded graphs of
  // 2^j applications each (the largest repeated, the rest by the binary digits), so a
  // call of any length launches a bounded set of graphs of bounded size
  const int sg = nsteps < 0 ? 1 : 0;
  int64_t rem = (nsteps < 0 ? -nsteps : nsteps) - 1;
  if ((st = batch_launch(p, sg, 0)) != GP_OK) return st;
  constexpr int top = gp_plan_s::GPOW - 1;
  while (rem >= ((int64_t)1 << top)) {
    if ((st = batch_launch(p, sg, 2 + top)) != GP_OK) return st;
    rem -= (int64_t)1 << top;
  }
  for (int j = top - 1; j >= 0; --j)
    if (rem & ((int64_t)1 << j))
      if ((st = batch_launch(p, sg, 2 + j)) != GP_OK) return st;
  return batch_launch(p, sg, 1);
}

gp_status gp_energies_batch(gp_plan_t* p, void* const* psis, void* work, double* out) {
  gp_status st = usable(p);
  if (st != GP_OK) return st;
  if (!p->is_batch) return fail(GP_ERR_STATE, "not a batch plan");
  if (!psis || !work || !out) return fail(GP_ERR_ARG, "null argument");
  for (size_t i = 0; i < p->runs.size(); ++i) {
    if (!psis[i]) return fail(GP_ERR_ARG, "null state of run %zu", i);
    gp_energy e{};
    if ((st = diagnose(p->runs[i], psis[i], work)) != GP_OK) { p->broken = p->runs[i]->broken; return st; }
    if ((st = copy_energies(p->runs[i], &e)) != GP_OK) return st;
    out[2 * i] = e.mass;
    out[2 * i + 1] = e.energy;
  }
  return GP_OK;
}

// ----------------------------------------------------------------- autotuner
// Cache: a flat JSON object {"<arch>/<prec>/<nx>x<ny>x<nz>/a<axis>": variant, ...}.
static std::map<std::string, int> read_cache(const char* path) {
  std::map<std::string, int> m;
  if (!path || !*path) return m;
  FILE* f = fopen(path, "r");
  if (!f) return m;
  std::string txt;
  char buf[4096];
  size_t k;
  while ((k = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, k);
  fclose(f);
  size_t i = 0;
  while ((i = txt.find('"', i)) != std::string::npos) {
    const size_t j = txt.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = txt.substr(i + 1, j - i - 1);
    size_t c = txt.find(':', j);
    if (c == std::string::npos) break;
    m[key] = atoi(txt.c_str() + c + 1);
    i = txt.find_first_of(",}", c);
    if (i == std::string::npos) break;
  }
  return m;
}

static void write_cache(const char* path, const std::map<std::string, int>& m) {
  if (!path || !*path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t n = 0;
  for (const auto& kv : m) fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++n < m.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

static std::string arch_name() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
  std::string a = pr.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

static std::string tune_key(const std::string& arch, const gp_plan_s* p, int axis) {
  char b[160];
  snprintf(b, sizeof b, "%s/%s/%dx%dx%d/a%d", arch.c_str(), p->prec == P_C128 ? "c128" : "c64", p->d.n[0], p->d.n[1],
           p->d.n[2], axis);
  return b;
}

// time `reps` in-place propagator passes of the selected schedule (microseconds per launch)
static gp_status time_axis(gp_plan_s* p, int axis, void* scratch, int reps, double* us) {
  hipEvent_t a, b;
  HIPCHK(p, hipEventCreate(&a));
  HIPCHK(p, hipEventCreate(&b));
  gp_status st = pass(p, axis, V_PROP, scratch, scratch, p->ax[axis].mult[TAU_DT]);
  if (st == GP_OK) {
    (void)hipEventRecord(a, p->stream);
    for (int r = 0; r < reps && st == GP_OK; ++r) st = pass(p, axis, V_PROP, scratch, scratch, p->ax[axis].mult[TAU_DT]);
    (void)hipEventRecord(b, p->stream);
  }
  float ms = 0.f;
  if (st == GP_OK) {
    hipError_t e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) { p->broken = true; st = fail(GP_ERR_HIP, "event timing: %s", hipGetErrorString(e)); }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *us = 1e3 * ms / std::max(1, reps);
  return st;
}

// time `reps` calls of launch() on the plan's stream (microseconds per call)
static gp_status time_calls(gp_plan_s* p, int reps, double* us, const std::function<void()>& launch) {
  hipEvent_t a, b;
  HIPCHK(p, hipEventCreate(&a));
  HIPCHK(p, hipEventCreate(&b));
  launch();                                    // warm-up
  (void)hipEventRecord(a, p->stream);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(b, p->stream);
  float ms = 0.f;
  hipError_t e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) { p->broken = true; return fail(GP_ERR_HIP, "event timing: %s", hipGetErrorString(e)); }
  *us = 1e3 * ms / std::max(1, reps);
  return check_launch(p);
}

// xy choice: separate x and y passes against one plane pass, both launched for
// `runs` copies of the scratch state at once (the ensemble launches a size group
// together, which changes how well each option fills the GPU; the copies all
// alias `scratch`, whose contents are undefined afterwards)
// Timings within 1 % count as ties, resolved to the candidate tried first (the lower
// variant index, the first axis, separate passes), so that repeated tunings agree.
constexpr double TUNE_TIE = 0.99;

// With GP_TUNE_LOG set, every timed candidate is reported on stderr.
static void tune_note(const gp_plan_s* p, const char* what, int axis, int cand, double us) {
  static const bool on = getenv("GP_TUNE_LOG") != nullptr;
  if (on)
    fprintf(stderr, "gp_autotune %dx%dx%d %s axis %d candidate %d: %.1f us\n", p->d.n[0], p->d.n[1], p->d.n[2],
            what, axis, cand, us);
}

static gp_status tune_xy(gp_plan_s* p, void* scratch, int reps, int runs, int* choice) {
  gp_status st;
  *choice = 0;
  if (!p->plane.e || p->ax[0].n == 1) return GP_OK;
  if ((st = build_plane_tables(p)) != GP_OK) return st;
  const size_t need = 3 * (size_t)runs;
  if (p->n_tune_ptrs < need) {
    if ((st = dev_alloc(p, (void**)&p->d_tune_ptrs, need * sizeof(RunPtrs))) != GP_OK) return st;
    p->n_tune_ptrs = need;
  }
  std::vector<RunPtrs> h(need);
  for (int i = 0; i < runs; ++i) {
    h[i] = RunPtrs{scratch, scratch, p->ax[0].mult[TAU_DT], nullptr, 0.0};
    h[runs + i] = RunPtrs{scratch, scratch, p->ax[1].mult[TAU_DT], nullptr, 0.0};
    h[2 * runs + i] = RunPtrs{scratch, scratch, p->plane.mx[TAU_DT], p->plane.my[TAU_DT], 0.0};
  }
  HIPCHK(p, hipMemcpy(p->d_tune_ptrs, h.data(), need * sizeof(RunPtrs), hipMemcpyHostToDevice));
  auto axis_launch = [&](int a, const RunPtrs* ptrs) {
    const Axis& A = p->ax[a];
    PassArgs g{};
    g.batch = ptrs; g.tw = A.tw; g.ksq = A.ksq; g.scale = 1.0;
    g.npencils = A.npencils; g.inner = A.inner; g.outer = A.outer; g.es = A.es;
    A.e->fn[A.kind][V_PROP](g, A.blocks, (unsigned)runs, p->stream);
  };
  double t_sep = 0, t_plane = 0;
  if ((st = time_calls(p, reps, &t_sep, [&] { axis_launch(0, p->d_tune_ptrs); axis_launch(1, p->d_tune_ptrs + runs); })) != GP_OK)
    return st;
  if ((st = time_calls(p, reps, &t_plane, [&] {
         PlaneArgs g{};
         g.batch = p->d_tune_ptrs + 2 * runs; g.tw = p->plane.tw;
         p->plane.e->fn[0](g, (unsigned)p->d.n[2], (unsigned)runs, p->stream);
       })) != GP_OK)
    return st;
  *choice = t_plane < TUNE_TIE * t_sep ? 1 : 0;
  return GP_OK;
}

// time the composed step L(dt) with the nonlinear prologue on each real axis in turn
// (state: psi = 1, the small-angle rotation of every real run); keep the fastest
static gp_status tune_nl(gp_plan_s* p, void* scratch, int reps, int* choice) {
  gp_status st;
  launch_fill(p->prec, scratch, p->ntot, 1.0, 0.0, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  const double nl = p->d.beta * p->d.dt;
  double best = 1e300;
  *choice = first_real_axis(p);
  for (int a = 0; a < 3; ++a) {
    if (p->ax[a].n == 1) continue;
    p->nl_axis = a;
    double us = 0;
    gp_status inner = GP_OK;
    if ((st = time_calls(p, reps, &us, [&] {
           if (inner == GP_OK) inner = linear_all(p, scratch, TAU_DT, true, nl);
         })) != GP_OK)
      return st;
    if (inner != GP_OK) return inner;
    tune_note(p, "nonlinear on", a, a, us);
    if (us < TUNE_TIE * best) { best = us; *choice = a; }
  }
  return GP_OK;
}

// linear steps: fixed-layout passes (in place) against layout-rotating passes (out of
// place through one more state); the rotating form is kept only if it wins by 1 %,
// otherwise its workspace is released
static gp_status tune_rot(gp_plan_s* p, void* scratch, int reps, int* choice) {
  gp_status st;
  *choice = 0;
  launch_fill(p->prec, scratch, p->ntot, 1.0, 0.0, p->stream);
  if ((st = check_launch(p)) != GP_OK) return st;
  const double nl = p->d.beta * p->d.dt;
  const int nrot = [&] { int k = 0; while (find_rot(p->d.n[0], p->prec, k)) ++k; return k; }();
  // the candidates are timed in alternation, twice each, keeping each one's best
  // time: the forms differ by ~10 % and clocks drift between measurements
  std::vector<double> t(1 + 2 * nrot, 1e300);
  gp_status inner = GP_OK;
  for (int round = 0; round < 2; ++round)
    for (int v = 0; v <= 2 * nrot; ++v) {
      double us = 0;
      if (v == 0) {
        if ((st = time_calls(p, reps, &us, [&] {
               if (inner == GP_OK) inner = linear_all(p, scratch, TAU_DT, true, nl);
             })) != GP_OK)
          return st;
      } else if (v <= nrot) {
        if ((st = gp_select_variant(p, 5, v)) != GP_OK) return st;
        if ((st = time_calls(p, reps, &us, [&] {       // two steps: back in `scratch`
               if (inner == GP_OK) inner = rot_linear(p, scratch, p->rot.work, TAU_DT, true, nl);
               if (inner == GP_OK) inner = rot_linear(p, p->rot.work, scratch, TAU_DT, true, nl);
             })) != GP_OK)
          return st;
        us *= 0.5;
      } else {
        if ((st = gp_select_variant(p, 5, v)) != GP_OK) return st;
        if ((st = time_calls(p, reps, &us, [&] {       // three steps: the layout's cycle
               for (int k = 0; k < 3 && inner == GP_OK; ++k)
                 inner = mixed_linear(p, scratch, p->rot.work, TAU_DT, true, nl);
             })) != GP_OK)
          return st;
        us /= 3.0;
      }
      if (inner != GP_OK) return inner;
      tune_note(p, "layout", 5, v, us);
      t[v] = std::min(t[v], us);
    }
  double best = t[0];
  for (int v = 1; v <= 2 * nrot; ++v)
    if (t[v] < TUNE_TIE * best) { best = t[v]; *choice = v; }
  return GP_OK;
}

static gp_status tune_plan(gp_plan_s* p, void* scratch, int reps, std::map<std::string, int>& cache,
                           const std::string& arch, int chosen[5], int runs) {
  gp_status st;
  for (int a = 0; a < 3; ++a) {
    chosen[a] = 0;
    if (p->ax[a].n == 1) continue;
    const std::string key = tune_key(arch, p, a);
    auto it = cache.find(key);
    if (it != cache.end() && find_entry(p->ax[a].n, p->prec, it->second)) {
      chosen[a] = it->second;
      if ((st = gp_select_variant(p, a, it->second)) != GP_OK) return st;
      continue;
    }
    const int nv = gp_variant_count(p->ax[a].n, p->prec);
    double best = 1e300;
    int bestv = 0;
    for (int v = 0; v < nv; ++v) {
      if (!find_entry(p->ax[a].n, p->prec, v)) continue;
      if ((st = gp_select_variant(p, a, v)) != GP_OK) return st;
      double us = 0;
      if ((st = time_axis(p, a, scratch, reps, &us)) != GP_OK) return st;
      tune_note(p, "schedule", a, v, us);
      if (us < TUNE_TIE * best) { best = us; bestv = v; }
    }
    if ((st = gp_select_variant(p, a, bestv)) != GP_OK) return st;
    cache[key] = bestv;
    chosen[a] = bestv;
  }
  chosen[3] = 0;
  if (p->plane.e) {
    char b[32];
    snprintf(b, sizeof b, "/r%d", runs);
    const std::string key = tune_key(arch, p, 3) + b;
    auto it = cache.find(key);
    if (it != cache.end() && (it->second == 0 || it->second == 1)) {
      chosen[3] = it->second;
    } else {
      if ((st = tune_xy(p, scratch, reps, runs, &chosen[3])) != GP_OK) return st;
      cache[key] = chosen[3];
    }
    if ((st = gp_select_variant(p, 3, chosen[3])) != GP_OK) return st;
  }
  // single plans with separate passes: the axis that carries the nonlinear prologue
  chosen[4] = first_real_axis(p);
  if (runs == 1 && !p->plane.on && chosen[4] >= 0) {
    const std::string key = tune_key(arch, p, 4);
    auto it = cache.find(key);
    if (it != cache.end() && it->second >= 0 && it->second <= 2 && p->ax[it->second].n > 1) {
      chosen[4] = it->second;
    } else {
      if ((st = tune_nl(p, scratch, reps, &chosen[4])) != GP_OK) return st;
      cache[key] = chosen[4];
    }
    if ((st = gp_select_variant(p, 4, chosen[4])) != GP_OK) return st;
  }
  // single cubic plans with separate passes: fixed-layout or layout-rotating steps
  const int n0 = p->d.n[0];
  if (runs == 1 && !p->plane.on && p->d.n[1] == n0 && p->d.n[2] == n0 && find_rot(n0, p->prec)) {
    const std::string key = tune_key(arch, p, 5);
    int c = 0;
    auto it = cache.find(key);
    const int nrot = [&] { int k = 0; while (find_rot(n0, p->prec, k)) ++k; return k; }();
    if (it != cache.end() && it->second >= 0 && it->second <= 2 * nrot) {
      c = it->second;
    } else {
      if ((st = tune_rot(p, scratch, reps, &c)) != GP_OK) return st;
      cache[key] = c;
    }
    if ((st = gp_select_variant(p, 5, c)) != GP_OK) return st;
  }
  return GP_OK;
}

gp_status gp_autotune(gp_plan_t* p, void* scratch, int32_t reps, const char* cache_path) {
  gp_status st = usable(p);
  if (st != GP_OK) return st;
  if (!scratch) return fail(GP_ERR_ARG, "null scratch state");
  if (reps < 1) return fail(GP_ERR_ARG, "reps must be >= 1");
  auto cache = read_cache(cache_path);
  const std::string arch = arch_name();
  if (!p->is_batch) {
    int chosen[5];
    if ((st = tune_plan(p, scratch, reps, cache, arch, chosen, 1)) != GP_OK) return st;
  } else {
    for (auto& g : p->groups) {
      gp_plan_s* r0 = p->runs[g.members[0]];
      int chosen[5];
      if ((st = tune_plan(r0, scratch, reps, cache, arch, chosen, (int)g.members.size())) != GP_OK) return st;
      for (size_t i = 1; i < g.members.size(); ++i)
        for (int a = 0; a < 4; ++a) {
          if (a == 3 && !p->runs[g.members[i]]->plane.e) continue;
          if ((st = gp_select_variant(p->runs[g.members[i]], a, chosen[a])) != GP_OK) return st;
        }
    }
    // kernels and tables changed: the recorded graphs are stale
    drop_graphs(p);
  }
  write_cache(cache_path, cache);
  return GP_OK;
}

}  // extern "C"
