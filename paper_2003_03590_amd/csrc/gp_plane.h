// xy-plane pass: the two in-plane sub-steps S(s, L_x) S(s, L_y) of the split step
// (time-evolution section; the axes commute, so the x and y factors may be applied
// together) on one z-plane per workgroup, reading and writing psi once.
//
// The plane (N x N points, N <= 128 for complex64, <= 64 for complex128) is small
// enough to stay on chip: the rows are loaded from global memory and transformed
// with the row (contiguous) mapping of the axis pass, written to LDS in natural
// order, read back as columns and transformed with the column (strided) mapping,
// then stored.  A Strang step then costs two sweeps of psi (this pass and the
// z pass) instead of three.  The transform stages, tables and the nonlinear
// prologue are those of the axis pass (same schedule type, W = N).
#pragma once

#include "gp_pass.h"

namespace gpk {

struct PlaneArgs {
  const RunPtrs* batch;    // grouped launch over runs of one size (mult = x, mult2 = y), or null
  const void* in;
  void* out;
  const void* multx;       // FP64 complex multipliers in the plane schedule's lane order
  const void* multy;
  const void* tw;          // per-stage twiddles of the plane schedule (Tab<Real>)
  double nl_coef;          // beta * dt for the fused nonlinear prologue
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <class Real, class S, int PRO>
__global__ __launch_bounds__(S::THREADS) void plane_pass(PlaneArgs a) {
  static_assert(S::W == S::N, "a plane workgroup holds all N rows");
  using C = cplx<Real>;
  constexpr int N = S::N, T = S::T, E = S::E;
  // plane row pitch in LDS: rows that share an LDS cycle in the row-major write get
  // their own banks (the column reads take consecutive points of one row)
  constexpr int SZ = (int)sizeof(C), TLX = lanes_per_pencil<S, SZ>();
  constexpr int P = (TLX < 128 / SZ) ? row_pitch<SZ>(N, TLX) : N + 1;
  constexpr int L = S::NS - 1, B = E / S::rad(L);
  constexpr int EX = Lds<S, (int)sizeof(C), CONTIG>::ELEMS, EY = Lds<S, (int)sizeof(C), STRIDED>::ELEMS;
  // one buffer serves the row exchanges, the plane and the column exchanges in turn
  __shared__ C lds[cmax(cmax(EX, EY), N * P)];

  const void* multx = a.multx;
  const void* multy = a.multy;
  if (a.batch) {                          // uniform per workgroup
    const RunPtrs r = a.batch[blockIdx.y];
    a.in = r.in; a.out = r.out; multx = r.mult; multy = r.mult2; a.nl_coef = r.nl_coef;
  }
  const int tid = threadIdx.x;
  const long base = (long)blockIdx.x * N * N;   // first point of this z-plane
  const auto tw = gptr<Tab<Real>>(a.tw);
  C v[E];

  {  // rows: S(s, L_x) (with the nonlinear prologue)
    constexpr int TL = TLX;
    const int t = tid % TL + TL * (tid / (TL * N));
    const int row = (tid / TL) % N;
    const auto src = gptr<C>(a.in) + base + (long)row * N + t;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[T * e];
    if constexpr (PRO == PRO_NL) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = nl_rotate(v[e], a.nl_coef);
    }
    forward_all<Real, S, CONTIG, 0>(v, lds, t, row, tw);
    const auto m = gptr<cplx<double>>(multx);
#pragma unroll
    for (int r = 0; r < S::rad(L); ++r)
#pragma unroll
      for (int j = 0; j < B; ++j) v[j + B * r] = pmul(v[j + B * r], m[(unsigned)(r * (N / S::rad(L)) + t + T * j)]);
    inverse_all<Real, S, CONTIG, L>(v, lds, t, row, tw);
    __syncthreads();                       // the last row exchange has been read
#pragma unroll
    for (int e = 0; e < E; ++e) lds[row * P + t + T * e] = v[e];
  }
  __syncthreads();
  {  // columns: S(s, L_y)
    const int col = tid % N;
    const int t = tid / N;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = lds[(t + T * e) * P + col];
    // the first column exchange starts with a barrier: every plane read is done by then
    forward_all<Real, S, STRIDED, 0>(v, lds, t, col, tw);
    const auto m = gptr<cplx<double>>(multy);
#pragma unroll
    for (int r = 0; r < S::rad(L); ++r)
#pragma unroll
      for (int j = 0; j < B; ++j) v[j + B * r] = pmul(v[j + B * r], m[(unsigned)(r * (N / S::rad(L)) + t + T * j)]);
    inverse_all<Real, S, STRIDED, L>(v, lds, t, col, tw);
    const auto dst = gptr_mut<C>(a.out) + base + col;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[(long)(t + T * e) * N] = v[e];
  }
}

using PlaneLauncher = void (*)(const PlaneArgs&, unsigned planes, unsigned runs, hipStream_t stream);

template <class Real, class S, int PRO>
void launch_plane(const PlaneArgs& a, unsigned planes, unsigned runs, hipStream_t stream) {
  hipLaunchKernelGGL((plane_pass<Real, S, PRO>), dim3(planes, runs), dim3(S::THREADS), 0, stream, a);
}

}  // namespace gpk
