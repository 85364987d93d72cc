// Registry of compiled axis-pass schedules (one entry per grid length, precision
// and variant).  Each instantiation unit registers its launchers at load time.
#pragma once

#include <vector>

#include "gp_pass.h"
#include "gp_plane.h"
#include "gp_rot.h"

namespace gpk {

enum Prec { P_C128 = 0, P_C64 = 1 };

struct PassEntry {
  int n, prec, variant;
  int T, W, NS, threads;
  int radix[3];
  PassLauncher fn[2][V_COUNT];   // [KIND][Variant]
};

std::vector<PassEntry>& registry();

// xy-plane schedules (one per grid length and precision; W = N)
struct PlaneEntry {
  int n, prec;
  int T, NS, threads;
  int radix[3];
  PlaneLauncher fn[2];           // [0] propagator, [1] with the nonlinear prologue
};

std::vector<PlaneEntry>& plane_registry();

struct PlaneRegistrar {
  explicit PlaneRegistrar(const PlaneEntry& e) { plane_registry().push_back(e); }
};

template <class Real, class S>
PlaneEntry make_plane_entry(int prec) {
  static_assert(S::THREADS % 64 == 0, "workgroup must be whole wavefronts");
  PlaneEntry e{};
  e.n = S::N; e.prec = prec;
  e.T = S::T; e.NS = S::NS; e.threads = S::THREADS;
  for (int s = 0; s < 3; ++s) e.radix[s] = s < S::NS ? S::rad(s) : 1;
  e.fn[0] = &launch_plane<Real, S, PRO_NONE>;
  e.fn[1] = &launch_plane<Real, S, PRO_NL>;
  return e;
}

struct Registrar {
  explicit Registrar(const PassEntry& e) { registry().push_back(e); }
};

template <class Real, class S, int KIND>
void fill(PassEntry& e) {
  e.fn[KIND][V_PROP] = &launch_pass<Real, S, KIND, PROP, PRO_NONE>;
  e.fn[KIND][V_PROP_NL] = &launch_pass<Real, S, KIND, PROP, PRO_NL>;
  e.fn[KIND][V_PROP_ADJ] = &launch_pass<Real, S, KIND, PROP, PRO_ADJ_NL>;
  e.fn[KIND][V_PROP_KIN] = &launch_pass<Real, S, KIND, PROP, PRO_KIN>;
  e.fn[KIND][V_FWD] = &launch_pass<Real, S, KIND, FWD, PRO_NONE>;
  e.fn[KIND][V_FWD_DENSITY] = &launch_pass<Real, S, KIND, FWD, PRO_DENSITY>;
  e.fn[KIND][V_INV] = &launch_pass<Real, S, KIND, INV, PRO_NONE>;
  e.fn[KIND][V_PROP_ARGLE] = &launch_pass<Real, S, KIND, PROP, PRO_ARGLE>;
  e.fn[KIND][V_FWD_MULT3] = &launch_pass<Real, S, KIND, FWD, PRO_MULT3>;
}

template <class Real, class S>
PassEntry make_entry(int prec, int variant) {
  static_assert(S::THREADS % 64 == 0, "workgroup must be whole wavefronts");
  PassEntry e{};
  e.n = S::N; e.prec = prec; e.variant = variant;
  e.T = S::T; e.W = S::W; e.NS = S::NS; e.threads = S::THREADS;
  for (int s = 0; s < 3; ++s) e.radix[s] = s < S::NS ? S::rad(s) : 1;
  fill<Real, S, CONTIG>(e);
  fill<Real, S, STRIDED>(e);
  return e;
}

// layout-rotating passes (cubic grids; one schedule serves all three axes)
struct RotEntry {
  int n, prec;
  PassEntry sched;         // schedule descriptor (table layout; no launchers)
  RotLauncher fn[2];       // [0] propagator, [1] with the nonlinear prologue
};

std::vector<RotEntry>& rot_registry();

struct RotRegistrar {
  explicit RotRegistrar(const RotEntry& e) { rot_registry().push_back(e); }
};

template <class Real, class S>
RotEntry make_rot_entry(int prec) {
  static_assert(S::THREADS % 64 == 0, "workgroup must be whole wavefronts");
  RotEntry e{};
  e.n = S::N; e.prec = prec;
  e.sched.n = S::N; e.sched.prec = prec; e.sched.variant = -1;
  e.sched.T = S::T; e.sched.W = S::W; e.sched.NS = S::NS; e.sched.threads = S::THREADS;
  for (int s = 0; s < 3; ++s) e.sched.radix[s] = s < S::NS ? S::rad(s) : 1;
  e.fn[0] = &launch_rot<Real, S, PRO_NONE>;
  e.fn[1] = &launch_rot<Real, S, PRO_NL>;
  return e;
}

}  // namespace gpk

#define GPK_CAT2(a, b) a##b
#define GPK_CAT(a, b) GPK_CAT2(a, b)
// GPK_SCHED(real, prec, variant, N, T, W, R0, R1, R2)
#define GPK_SCHED(REAL, PREC, VAR, N, T, W, R0, R1, R2)                                         \
  static ::gpk::Registrar GPK_CAT(gpk_reg_, __LINE__)(                                          \
      ::gpk::make_entry<REAL, ::gpk::Sched<N, T, W, R0, R1, R2>>(PREC, VAR));
// GPK_PLANE(real, prec, N, T, R0, R1, R2): xy-plane schedule with W = N
#define GPK_PLANE(REAL, PREC, N, T, R0, R1, R2)                                                  \
  static ::gpk::PlaneRegistrar GPK_CAT(gpk_plane_, __LINE__)(                                    \
      ::gpk::make_plane_entry<REAL, ::gpk::Sched<N, T, N, R0, R1, R2>>(PREC));
// GPK_ROT(real, prec, N, T, W, R0, R1, R2): layout-rotating pass schedule
#define GPK_ROT(REAL, PREC, N, T, W, R0, R1, R2)                                                  \
  static ::gpk::RotRegistrar GPK_CAT(gpk_rot_, __LINE__)(                                         \
      ::gpk::make_rot_entry<REAL, ::gpk::Sched<N, T, W, R0, R1, R2>>(PREC));
