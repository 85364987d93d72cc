// Axis-pass kernel: the directional spectral sub-step of the split step.
//
// One launch processes every pencil of the grid along one axis j and applies
//   PROP: v <- F_j^-1 ( m(k_j) * F_j v )         (S(s, L_j) with m = exp(-i alpha k_j^2 s)/N_j,
//                                                  or a spectral derivative with m = i k_j / N_j)
//   FWD : v <- scale * F_j v        (natural frequency order out)
//   INV : v <- scale * F_j^-1 v     (natural frequency order in, unnormalised inverse)
// with optional pointwise prologues (the nonlinear sub-step S(dt, N), its adjoint, the
// density rho - 1) fused in front of the transform.
//
// Transform structure (time-evolution section: each S(s, L_j) is exact in Fourier space):
// N = R_0 R_1 ... R_{S-1}; T threads per pencil each hold E = N/T points in registers.
// Forward stages are decimation-in-frequency butterflies done in registers, with an
// LDS exchange between stages; after the last stage position p holds the coefficient
// of the digit-reversed frequency.  PROP multiplies there by a table already stored in
// that order and runs the exact inverse (conjugate-twiddle DIT) stages in reverse, so
// no reordering pass is ever needed.  W pencils share one workgroup; for the strided
// axes (y, z) the W pencils are x-adjacent so each global access is a W*S-byte row.
//
// Table layouts (built on the host for the schedule in use): every table load of one
// instruction reads consecutive entries across the lanes, so it costs a few vector-L1
// requests instead of one per lane.
//   multiplier / k^2: the entry of position g*R_last + r is stored at r*(N/R_last) + g
//                     (g = t + T*j runs over the lanes of one load)
//   twiddles        : stage s keeps W_{R_s M_s}^{lo k} at TWOFF(s) + (k-1)*M_s + lo
#pragma once

#include "gp_device.h"

namespace gpk {

// global-memory pointers: accesses through them are global (not flat) instructions,
// which count on the vector-memory counter only (the qualifier is for the device
// compilation pass; the host pass only checks the kernel bodies)
#if defined(__HIP_DEVICE_COMPILE__)
#define GPK_GLOBAL __attribute__((address_space(1)))
#else
#define GPK_GLOBAL
#endif
template <class X>
__device__ __forceinline__ const GPK_GLOBAL X* gptr(const void* p) { return (const GPK_GLOBAL X*)p; }
template <class X>
__device__ __forceinline__ GPK_GLOBAL X* gptr_mut(void* p) { return (GPK_GLOBAL X*)p; }

enum PassKind { CONTIG = 0, STRIDED = 1 };
enum PassMode { PROP = 0, FWD = 1, INV = 2 };
// pointwise work fused in front of the transform (PRO_KIN: none, but accumulate
// sum k_j^2 |F_j v|^2 after the forward transform for the kinetic energy;
// PRO_ARGLE: none, but turn the derivative after the inverse transform into the
// explicit part of the imaginary-time step; PRO_MULT3: none, but multiply the
// forward transform by the separable 3-D propagator m_x(k_x) m_y(k_y) m_z(k_z) before
// it is stored -- the last forward pass of the literal 3-D form)
enum Prologue { PRO_NONE = 0, PRO_NL = 1, PRO_ADJ_NL = 2, PRO_DENSITY = 3, PRO_KIN = 4, PRO_ARGLE = 5, PRO_MULT3 = 6 };

// per-run pointers of a grouped (ensemble) launch: run = blockIdx.y
struct RunPtrs {
  const void* in;
  void* out;
  const void* mult;
  const void* mult2;       // plane pass: the y multipliers (mult holds the x ones)
  double nl_coef;
};

struct PassArgs {
  const RunPtrs* batch;    // grouped launch over runs of one size, or null
  const void* in;          // input field (complex, working precision)
  void* out;               // output field (may equal in)
  const void* mult;        // PROP: multiplier in lane order (N_j FP64 complex entries)
  const void* tw;          // per-stage twiddles W_{R M}^{lo k} (Tab<Real> entries, layout above)
  const void* aux;         // PRO_ADJ_NL, PRO_ARGLE: the state phi at the same points;
                           // PRO_MULT3: m_x in natural frequency order (FP64 complex)
  const void* aux2;        // PRO_ARGLE: d phi / dx and d phi / dy at the same points;
  const void* aux3;        // PRO_MULT3: m_y and m_z
  const void* vel;         // PRO_ARGLE: velocity planes v_x, v_y, v_z (Real, one field each)
  double q4a;              // PRO_ARGLE: 1 / (4 alpha)
  const double* ksq;       // k_j^2 in position order (kinetic accumulation)
  double* kin_partial;     // per-workgroup partial sum of k_j^2 |F_j v|^2 (or null)
  double nl_coef;          // beta * dt of the nonlinear prologue
  double scale;            // FWD/INV output scale
  long npencils;           // number of pencils along this axis
  long inner, outer;       // pencil p starts at (p / inner) * outer + (p % inner)
  long es;                 // element stride along the axis
  int axis;                // PRO_MULT3: the pass's axis (0 x, 1 y, 2 z) ...
  int nx, ny;              // ... and the grid's x and y lengths
};

template <int N_, int T_, int W_, int R0, int R1, int R2>
struct Sched {
  static constexpr int N = N_, T = T_, W = W_, E = N_ / T_;
  static constexpr int NS = (R0 > 1) + (R1 > 1) + (R2 > 1);
  static constexpr int rad(int s) { return s == 0 ? R0 : s == 1 ? R1 : R2; }
  // product of the radices after stage s (the digit weight of stage s)
  static constexpr int M(int s) { int m = 1; for (int i = s + 1; i < NS; ++i) m *= rad(i); return m; }
  // product of the radices before stage s (the frequency weight of stage s)
  static constexpr int K(int s) { int k = 1; for (int i = 0; i < s; ++i) k *= rad(i); return k; }
  // twiddle sub-table of stage s: entries W_{R M}^{lo k} at (k-1)*M(s) + lo, stages with
  // M(s) > 1 stored one after another
  static constexpr int TWOFF(int s) {
    int o = 0;
    for (int i = 0; i < s; ++i) if (M(i) > 1) o += (rad(i) - 1) * M(i);
    return o;
  }
  static constexpr bool valid() {
    if (T * E != N) return false;
    int p = 1;
    for (int s = 0; s < NS; ++s) { if (E % rad(s)) return false; p *= rad(s); }
    return p == N;
  }
  static_assert(valid(), "inconsistent FFT schedule");
  static constexpr int THREADS = T * W;
  static constexpr int RL = rad(NS > 0 ? NS - 1 : 0);     // radix of the last stage
};

// Lanes of one pencil in the contiguous mapping: TL consecutive lanes on one pencil
// (a 128-byte segment, or the whole pencil when it is shorter).
template <class S, int SZ>
constexpr int lanes_per_pencil() { return (S::T * SZ <= 128) ? S::T : 128 / SZ; }

// Smallest pitch >= n, in points of SZ bytes, that sets the rows of one LDS cycle
// apart by whole lane groups.  The LDS serves 128 bytes per cycle (16 lanes of a
// 64-bit access, 8 of a 128-bit one); with TL lanes per row, 128/(SZ TL) rows share a
// cycle and a pitch of TL modulo 128/SZ points puts each row on its own banks.  With
// one row per cycle the pitch is kept at 128 B modulo 256 B.
template <int SZ>
constexpr int row_pitch(int n, int TL) {
  int c = n;
  if (128 % SZ != 0) return c;
  const int slots = 128 / SZ;
  if (TL < slots) {
    while (c % slots != TL % slots) ++c;
  } else {
    while (c % (2 * slots) != slots) ++c;
  }
  return c;
}

// LDS layout of the stage exchanges (SZ = bytes per element).
//   CONTIG  [col][pos + pos/RL + pad]: one pad element every RL positions spreads the
//           stride-RL accesses of the last stage over the banks; the column pitch
//           (row_pitch) gives the pencils that share an LDS cycle different banks.
//   STRIDED [pos + pos/RL][col]: one pad row every RL rows, for the same reason.
template <class S, int SZ, int KIND>
struct Lds {
  static constexpr int PADN = S::N + S::N / S::RL;
  static constexpr int cpitch() { return row_pitch<SZ>(PADN, lanes_per_pencil<S, SZ>()); }
  static constexpr int CP = cpitch();
  static constexpr int ELEMS = (S::NS > 1) ? (KIND == CONTIG ? S::W * CP : PADN * S::W) : 1;
  static __device__ __forceinline__ int addr(int pos, int col) {
    if constexpr (KIND == CONTIG) return col * CP + pos + pos / S::RL;
    else return (pos + pos / S::RL) * S::W + col;
  }
};

// position held by register (j + B*r) of thread t at stage s
template <class S, int s>
__device__ __forceinline__ int stage_pos(int t, int j, int r) {
  constexpr int Ms = S::M(s);
  constexpr int Ls = S::rad(s) * Ms;
  const int g = t + S::T * j;
  return (g / Ms) * Ls + r * Ms + (g % Ms);
}

// position of natural frequency k (digit-reversal of the DIF output order)
template <class S>
__device__ __forceinline__ int freq_pos(int k) {
  int p = 0;
#pragma unroll
  for (int s = 0; s < S::NS; ++s) p += ((k / S::K(s)) % S::rad(s)) * S::M(s);
  return p;
}

template <class Real, class S, int KIND>
__device__ __forceinline__ int lds_addr(int pos, int col) {
  return Lds<S, (int)sizeof(cplx<Real>), KIND>::addr(pos, col);
}

// layout ids for exchanges: 0..NS-1 = stage layouts, -1 = natural frequency layout
template <class Real, class S, int KIND, int L>
__device__ __forceinline__ void put(cplx<Real>* lds, const cplx<Real>* v, int t, int col) {
  if constexpr (L < 0) {
#pragma unroll
    for (int e = 0; e < S::E; ++e) lds[lds_addr<Real, S, KIND>(freq_pos<S>(t + S::T * e), col)] = v[e];
  } else {
    constexpr int B = S::E / S::rad(L);
#pragma unroll
    for (int r = 0; r < S::rad(L); ++r)
#pragma unroll
      for (int j = 0; j < B; ++j) lds[lds_addr<Real, S, KIND>(stage_pos<S, L>(t, j, r), col)] = v[j + B * r];
  }
}
template <class Real, class S, int KIND, int L>
__device__ __forceinline__ void get(const cplx<Real>* lds, cplx<Real>* v, int t, int col) {
  if constexpr (L < 0) {
#pragma unroll
    for (int e = 0; e < S::E; ++e) v[e] = lds[lds_addr<Real, S, KIND>(freq_pos<S>(t + S::T * e), col)];
  } else {
    constexpr int B = S::E / S::rad(L);
#pragma unroll
    for (int r = 0; r < S::rad(L); ++r)
#pragma unroll
      for (int j = 0; j < B; ++j) v[j + B * r] = lds[lds_addr<Real, S, KIND>(stage_pos<S, L>(t, j, r), col)];
  }
}

template <class Real, class S, int KIND, int FROM, int TO>
__device__ __forceinline__ void exchange(cplx<Real>* lds, cplx<Real>* v, int t, int col) {
  __syncthreads();                          // previous readers of lds are done
  put<Real, S, KIND, FROM>(lds, v, t, col);
  __syncthreads();
  get<Real, S, KIND, TO>(lds, v, t, col);
}

// table entry i (32-bit index from the uniform table base; P is a global-memory or
// an LDS pointer)
template <class P>
__device__ __forceinline__ auto tab_at(P t, int i) {
  return t[(unsigned)i];
}

// forward DIF stage s: butterfly over digit s, then twiddle W_{L_s}^{lo*k}
template <class Real, class S, int s, class P>
__device__ __forceinline__ void fwd_stage(cplx<Real>* v, int t, P tw) {
  constexpr int R = S::rad(s), B = S::E / R, Ms = S::M(s);
#pragma unroll
  for (int j = 0; j < B; ++j) {
    cplx<Real> x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[j + B * r];
    Dft<R, -1, Real>::run(x);
    if constexpr (Ms > 1) {
      const int lo = (t + S::T * j) % Ms;
#pragma unroll
      for (int k = 1; k < R; ++k) x[k] = tmul(x[k], tab_at(tw, S::TWOFF(s) + (k - 1) * Ms + lo));
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[j + B * k] = x[k];
  }
}

// inverse of fwd_stage (up to the factor R): conjugate twiddle, then inverse butterfly
template <class Real, class S, int s, class P>
__device__ __forceinline__ void inv_stage(cplx<Real>* v, int t, P tw) {
  constexpr int R = S::rad(s), B = S::E / R, Ms = S::M(s);
#pragma unroll
  for (int j = 0; j < B; ++j) {
    cplx<Real> x[R];
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = v[j + B * k];
    if constexpr (Ms > 1) {
      const int lo = (t + S::T * j) % Ms;
#pragma unroll
      for (int k = 1; k < R; ++k) x[k] = tmulc(x[k], tab_at(tw, S::TWOFF(s) + (k - 1) * Ms + lo));
    }
    Dft<R, +1, Real>::run(x);
#pragma unroll
    for (int r = 0; r < R; ++r) v[j + B * r] = x[r];
  }
}

template <class Real, class S, int KIND, int s, class P>
__device__ __forceinline__ void forward_all(cplx<Real>* v, cplx<Real>* lds, int t, int col, P tw) {
  fwd_stage<Real, S, s, P>(v, t, tw);
  if constexpr (s + 1 < S::NS) {
    exchange<Real, S, KIND, s, s + 1>(lds, v, t, col);
    forward_all<Real, S, KIND, s + 1, P>(v, lds, t, col, tw);
  }
}

template <class Real, class S, int KIND, int s, class P>
__device__ __forceinline__ void inverse_all(cplx<Real>* v, cplx<Real>* lds, int t, int col, P tw) {
  inv_stage<Real, S, s, P>(v, t, tw);
  if constexpr (s > 0) {
    exchange<Real, S, KIND, s, s - 1>(lds, v, t, col);
    inverse_all<Real, S, KIND, s - 1, P>(v, lds, t, col, tw);
  }
}

// Complex64 tiles of whole contiguous pencils move between global memory and the
// lanes through the LDS exchange buffer with 16-byte accesses: unit u of the tile
// (u = tid + THREADS i) holds points 2q, 2q+1 of tile pencil u / (N/2), so one load or
// store instruction of a wavefront covers 1 KB of one pencil, against four 128-byte
// pieces of four pencils with one point per lane.  `pencil(pc)` is the element offset
// of tile pencil pc.  Complex128 points are 16 bytes already and move directly.
template <class S>
constexpr bool wide_io() { return S::NS > 1 && S::N % 2 == 0 && S::E % 2 == 0; }

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <class S, class F>
__device__ __forceinline__ void load_tile_wide(cplx<float>* v, cplx<float>* lds, const void* in, F pencil,
                                               int t, int col) {
  using L = Lds<S, 8, CONTIG>;
  constexpr int HN = S::N / 2, U = S::E / 2;
  const auto src = gptr<cplx<float>>(in);
  f32x4 r[U];
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int u = (int)threadIdx.x + S::THREADS * i, pc = u / HN, q = u % HN;
    r[i] = *(const GPK_GLOBAL f32x4*)(src + pencil(pc) + 2 * q);
  }
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int u = (int)threadIdx.x + S::THREADS * i, pc = u / HN, q = u % HN;
    lds[L::addr(2 * q, pc)] = mk(r[i].x, r[i].y);
    lds[L::addr(2 * q + 1, pc)] = mk(r[i].z, r[i].w);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::E; ++e) v[e] = lds[L::addr(t + S::T * e, col)];
}

template <class S, class F>
__device__ __forceinline__ void store_tile_wide(const cplx<float>* v, cplx<float>* lds, void* out, F pencil,
                                                int t, int col) {
  using L = Lds<S, 8, CONTIG>;
  constexpr int HN = S::N / 2, U = S::E / 2;
  const auto dst = gptr_mut<cplx<float>>(out);
  __syncthreads();                          // the last exchange has been read
#pragma unroll
  for (int e = 0; e < S::E; ++e) lds[L::addr(t + S::T * e, col)] = v[e];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int u = (int)threadIdx.x + S::THREADS * i, pc = u / HN, q = u % HN;
    const cplx<float> p0 = lds[L::addr(2 * q, pc)], p1 = lds[L::addr(2 * q + 1, pc)];
    *(GPK_GLOBAL f32x4*)(dst + pencil(pc) + 2 * q) = f32x4{p0.x, p0.y, p1.x, p1.y};
  }
}

// nonlinear sub-step S(dt, N): v <- v exp(-i beta (|v|^2 - 1) dt), in the working precision
template <class Real>
__device__ __forceinline__ cplx<Real> nl_rotate(cplx<Real> v, double coef) {
  Real s, c;
  sincos_rot(-Real(coef) * (cabs2(v) - Real(1)), &s, &c);
  return cmul(v, mk(c, s));
}
// FP32: v + v (cos a - 1 + i sin a), see sincos_m1; the small correction is formed
// first, so the result carries one rounding at the size of v
template <>
__device__ __forceinline__ cplx<float> nl_rotate<float>(cplx<float> v, double coef) {
  float s, cm1;
  sincos_m1(-float(coef) * (cabs2(v) - 1.0f), &s, &cm1);
  const float dx = fmaf(v.x, cm1, -v.y * s), dy = fmaf(v.y, cm1, v.x * s);
  return mk(v.x + dx, v.y + dy);
}

// adjoint of the linearised nonlinear sub-step at phi:
//   lam <- conj(u) lam + 2 beta dt Im(conj(lam) u phi) phi,  u = exp(-i beta (|phi|^2-1) dt)
template <class Real>
__device__ __forceinline__ cplx<Real> nl_adjoint(cplx<Real> lam, cplx<Real> phi, Real coef) {
  Real s, c;
  sincos_rot(-coef * (cabs2(phi) - Real(1)), &s, &c);
  const cplx<Real> u = mk(c, s);
  const cplx<Real> up = cmul(u, phi);
  const Real im = lam.x * up.y - lam.y * up.x;          // Im(conj(lam) * up)
  const cplx<Real> r = cmulc(lam, u);                    // conj(u) lam
  const Real f = Real(2) * coef * im;
  return mk(r.x + f * phi.x, r.y + f * phi.y);
}

template <class Real, class S, int KIND, int MODE, int PRO>
__global__ __launch_bounds__(S::THREADS) void axis_pass(PassArgs a) {
  using C = cplx<Real>;
  constexpr int T = S::T, W = S::W, E = S::E;
  __shared__ C lds[Lds<S, (int)sizeof(C), KIND>::ELEMS];
  __shared__ double red[S::THREADS / 64 + 1];

  if (a.batch) {                          // uniform per workgroup
    const RunPtrs r = a.batch[blockIdx.y];
    a.in = r.in; a.out = r.out; a.mult = r.mult; a.nl_coef = r.nl_coef;
  }
  const int tid = threadIdx.x;
  int t, col;
  if constexpr (KIND == CONTIG) {
    // TL consecutive points of one pencil form a 128-byte segment; a wavefront
    // covers several pencils per load instruction (spreads requests over channels)
    constexpr int TL = lanes_per_pencil<S, (int)sizeof(C)>();
    t = tid % TL + TL * (tid / (TL * W));
    col = (tid / TL) % W;
  } else {
    col = tid % W;
    t = tid / W;
  }
  // XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs;
  // give each XCD a contiguous run of tiles so tiles that share cache lines meet
  // in the same L2.
  const unsigned G = gridDim.x, b = blockIdx.x;
  const unsigned nfull = G / 8, rem = G % 8, xcd = b % 8;
  const long tile = (long)xcd * nfull + (xcd < rem ? xcd : rem) + b / 8;
  const long es = a.es;
  const long estep = (long)T * es * (long)sizeof(C);
  const auto tw = gptr<Tab<Real>>(a.tw);
  const auto mult = gptr<cplx<double>>(a.mult);     // FP64 multipliers for both precisions

  // Addressing: element e of this lane in tile tl sits at
  //   bbase + e*T*es   (uniform: first pencil of the tile, scalar registers)
  // + loff             (per lane, < 2^32 bytes for every supported shape)
  // so each access is a scalar-base + 32-bit-offset load or store.
  // A lane past the last pencil (ragged last tile) takes the last pencil: it loads,
  // transforms and stores exactly what that pencil's own lanes do, so every load and
  // store is issued unconditionally (no branch around memory instructions) and the
  // duplicate stores write equal bytes.
  struct Where { long bbase; unsigned loff; bool active; long pstart; };
  auto where = [&](long tl) {
    Where w;
    const long p = tl * W + col;
    w.active = p < a.npencils;
    const long pp = w.active ? p : a.npencils - 1;
    // pencil indices are below 2^20 for every supported shape: 32-bit division
    // (no 64-bit division subroutine with its branches)
    const unsigned inner = (unsigned)a.inner, q0 = (unsigned)(tl * W), q = (unsigned)pp;
    w.bbase = (long)(q0 / inner) * a.outer + (long)(q0 % inner);
    w.pstart = (long)(q / inner) * a.outer + (long)(q % inner);
    w.loff = (unsigned)(((long)(q / inner) * a.outer + (long)(q % inner) - w.bbase + (long)t * es) * (long)sizeof(C));
    return w;
  };
  auto load = [&](C* v, const Where& w) {
    const auto inb = gptr<char>(a.in) + w.bbase * (long)sizeof(C);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = *(const GPK_GLOBAL C*)(inb + e * estep + w.loff);
  };

  // x pencils of complex64 propagator passes: whole tiles of contiguous pencils,
  // moved with 16-byte accesses (a pencil past the last one takes the last one, as
  // the lanes do, so the duplicate stores write equal bytes)
  constexpr bool WIDE = sizeof(Real) == 4 && KIND == CONTIG && MODE == PROP &&
                        (PRO == PRO_NONE || PRO == PRO_NL) && wide_io<S>();
  auto tile_pencil = [&](int pc) {
    const long p = tile * W + pc;
    return (p < a.npencils ? p : a.npencils - 1) * (long)S::N;
  };

  double kin_acc = 0.0;
  // transform one tile held in v (prologue, transform, multiplier, inverse) and store it
  auto process = [&](C* v, const Where& cur) {
    if constexpr (MODE != INV) {
      if constexpr (PRO == PRO_NL) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = nl_rotate(v[e], a.nl_coef);
      } else if constexpr (PRO == PRO_ADJ_NL) {
        const auto phib = gptr<char>(a.aux) + cur.bbase * (long)sizeof(C);
        const Real coef = Real(a.nl_coef);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const C f = *(const GPK_GLOBAL C*)(phib + e * estep + cur.loff);
          v[e] = nl_adjoint(v[e], f, coef);
        }
      } else if constexpr (PRO == PRO_DENSITY) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = mk(cabs2(v[e]) - Real(1), Real(0));
      }
    }

    if constexpr (MODE == INV) {
      if constexpr (S::NS > 1) exchange<Real, S, KIND, -1, S::NS - 1>(lds, v, t, col);
      inverse_all<Real, S, KIND, S::NS - 1>(v, lds, t, col, tw);
      const Real sc = Real(a.scale);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cscale(v[e], sc);
    } else {
      forward_all<Real, S, KIND, 0>(v, lds, t, col, tw);
      constexpr int L = S::NS - 1;
      constexpr int B = E / S::rad(L);
      if constexpr (MODE == PROP) {
        if constexpr (PRO == PRO_KIN) {
          double acc = 0.0;
#pragma unroll
          for (int r = 0; r < S::rad(L); ++r)
#pragma unroll
            for (int j = 0; j < B; ++j) {
              const int li = r * (S::N / S::rad(L)) + t + T * j;
              const C x = v[j + B * r];
              acc += gptr<double>(a.ksq)[(unsigned)li] *
                     ((double)x.x * x.x + (double)x.y * x.y);
            }
          if (cur.active) kin_acc += acc;
        }
#pragma unroll
        for (int r = 0; r < S::rad(L); ++r)
#pragma unroll
          for (int j = 0; j < B; ++j)
            v[j + B * r] = pmul(v[j + B * r], tab_at(mult, r * (S::N / S::rad(L)) + t + T * j));
        inverse_all<Real, S, KIND, L>(v, lds, t, col, tw);
        if constexpr (PRO == PRO_ARGLE) {
          // v holds d phi / dz (this pass is the z derivative); replace it by the explicit
          // part of the imaginary-time step at the same points:
          //   n = -i v.grad phi + (beta - |v|^2/(4 alpha) - beta |phi|^2) phi
          const long ntot = a.npencils * (long)S::N;
          const auto vel = gptr<Real>(a.vel);
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const long idx = cur.bbase + (long)((e * estep + cur.loff) / (long)sizeof(C));
            const C f = gptr<C>(a.aux)[idx], gx = gptr<C>(a.aux2)[idx], gy = gptr<C>(a.aux3)[idx];
            const double ux = vel[idx], uy = vel[ntot + idx], uz = vel[2 * ntot + idx];
            const double gr = ux * gx.x + uy * gy.x + uz * v[e].x, gi = ux * gx.y + uy * gy.y + uz * v[e].y;
            const double pr = f.x, pi = f.y;
            const double c = a.nl_coef - (ux * ux + uy * uy + uz * uz) * a.q4a - a.nl_coef * (pr * pr + pi * pi);
            v[e] = mk(Real(gi + c * pr), Real(-gr + c * pi));
          }
        }
      } else {  // FWD: reorder to natural frequency order
        if constexpr (S::NS > 1) exchange<Real, S, KIND, L, -1>(lds, v, t, col);
        const Real sc = Real(a.scale);
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = cscale(v[e], sc);
        if constexpr (PRO == PRO_MULT3) {
          // v[e] holds frequency t + T e of the pencil starting at point cur.pstart;
          // the factors multiply in the order (m_x m_y) m_z, in FP64
          const auto mx = gptr<cplx<double>>(a.aux), my = gptr<cplx<double>>(a.aux2),
                     mz = gptr<cplx<double>>(a.aux3);
          const long nxy = (long)a.nx * a.ny;
          const int ix = (int)(cur.pstart % a.nx), iy = (int)((cur.pstart / a.nx) % a.ny),
                    iz = (int)(cur.pstart / nxy);
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int f = t + T * e;
            const cplx<double> m = cmul(cmul(mx[a.axis == 0 ? f : ix], my[a.axis == 1 ? f : iy]),
                                        mz[a.axis == 2 ? f : iz]);
            v[e] = pmul(v[e], m);
          }
        }
      }
    }

    if constexpr (WIDE) {
      store_tile_wide<S>(v, lds, a.out, tile_pencil, t, col);
    } else {
      const auto outb = gptr_mut<char>(a.out) + cur.bbase * (long)sizeof(C);
#pragma unroll
      for (int e = 0; e < E; ++e) *(GPK_GLOBAL C*)(outb + e * estep + cur.loff) = v[e];
    }
  };

  C v[E];
  const Where w = where(tile);
  if constexpr (WIDE) load_tile_wide<S>(v, lds, a.in, tile_pencil, t, col);
  else load(v, w);
  process(v, w);

  if constexpr (PRO == PRO_KIN) {
    // fixed-order reduction: wave butterfly, then waves in order (one partial per workgroup)
    double acc = kin_acc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < S::THREADS / 64 + (S::THREADS % 64 ? 1 : 0); ++w) s += red[w];
      gptr_mut<double>(a.kin_partial)[blockIdx.x] = s;
    }
  }
}

// launcher signature shared by every instantiation
using PassLauncher = void (*)(const PassArgs&, unsigned grid, unsigned runs, hipStream_t stream);

template <class Real, class S, int KIND, int MODE, int PRO>
void launch_pass(const PassArgs& a, unsigned grid, unsigned runs, hipStream_t stream) {
  hipLaunchKernelGGL((axis_pass<Real, S, KIND, MODE, PRO>), dim3(grid, runs), dim3(S::THREADS), 0, stream, a);
}

// kernel variants compiled for every schedule
enum Variant { V_PROP = 0, V_PROP_NL, V_PROP_ADJ, V_PROP_KIN, V_FWD, V_FWD_DENSITY, V_INV, V_PROP_ARGLE, V_FWD_MULT3,
               V_COUNT };

}  // namespace gpk
