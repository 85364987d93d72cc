// Layout-rotating axis pass: the spectral sub-step S(s, L_j) of the time-evolution
// section on a cubic grid whose layout turns with every pass.
//
// The input is a state in layout [A][B][C] (C, the transform axis, contiguous);
// the output is the same state in layout [B][C][A].  A workgroup takes W pencils
// with consecutive A at one B: it reads each pencil as one contiguous run of N
// points, transforms it exactly as the axis pass does (prologue, forward stages,
// multiplier, inverse stages), redistributes the tile through LDS so that
// neighbouring lanes hold neighbouring A, and writes rows of W consecutive A with
// a stride of N points between rows.  Three such passes along x, z, y take the
// layout [z][y][x] -> [y][x][z] -> [x][z][y] -> [z][y][x]: no access ever has the
// N^2 stride of a z pencil in the fixed layout, whose rows each fall in their own
// memory page.  The passes are out of place (a second state of workspace).
// Complex64 tiles are read with 16-byte loads staged through LDS (load_tile_wide);
// the turned rows are written one point per lane, which measured faster than
// 16-byte stores of the same 64-byte row pieces.
#pragma once

#include "gp_pass.h"
#include "gp_plane.h"

namespace gpk {

struct RotArgs {
  const void* in;          // layout [A][B][C]
  void* out;               // layout [B][C][A] (a different state)
  const void* mult;        // multipliers in the lane order of the schedule (FP64 complex)
  const void* tw;          // stage twiddles of the schedule (Tab<Real>)
  double nl_coef;          // beta * dt of the nonlinear prologue
};

template <class Real, class S, int PRO>
__global__ __launch_bounds__(S::THREADS) void rot_pass(RotArgs a) {
  using C = cplx<Real>;
  constexpr int T = S::T, W = S::W, E = S::E, N = S::N;
  constexpr int SZ = (int)sizeof(C);
  static_assert(N % W == 0 && (W & (W - 1)) == 0, "tiles cover whole rows of A; W a power of two");
  // stage exchanges, and the regrouping of the whole tile (which single-stage
  // schedules need although they have no exchange)
  constexpr int REGROUP = N * W;
  __shared__ C lds[cmax(cmax(Lds<S, SZ, CONTIG>::ELEMS, Lds<S, SZ, STRIDED>::ELEMS), REGROUP)];
  const int tid = threadIdx.x;

  // XCD-aware tile order (as the axis pass): each XCD takes a contiguous run of
  // tiles; tile = b * (N / W) + a0 / W
  const unsigned G = gridDim.x, bi = blockIdx.x;
  const unsigned nfull = G / 8, rem = G % 8, xcd = bi % 8;
  const unsigned tile = xcd * nfull + (xcd < rem ? xcd : rem) + bi / 8;
  constexpr unsigned NTA = N / W;
  const long b = tile / NTA, a0 = (long)(tile % NTA) * W;
  const long NN = (long)N * N;

  // load with the contiguous mapping: TL consecutive lanes on one pencil
  constexpr int TL = lanes_per_pencil<S, SZ>();
  const int t = tid % TL + TL * (tid / (TL * W));
  const int col = (tid / TL) % W;
  C v[E];
  if constexpr (sizeof(Real) == 4 && wide_io<S>()) {
    load_tile_wide<S>(v, lds, a.in, [&](int pc) { return (a0 + pc) * NN + b * N; }, t, col);
  } else {
    const auto in = gptr<C>(a.in) + (a0 + col) * NN + b * N + t;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = in[T * e];
  }

  if constexpr (PRO == PRO_NL) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = nl_rotate(v[e], a.nl_coef);
  }
  const auto tw = gptr<Tab<Real>>(a.tw);
  const auto mult = gptr<cplx<double>>(a.mult);
  forward_all<Real, S, CONTIG, 0>(v, lds, t, col, tw);
  constexpr int L = S::NS - 1;
  constexpr int B = E / S::rad(L);
#pragma unroll
  for (int r = 0; r < S::rad(L); ++r)
#pragma unroll
    for (int j = 0; j < B; ++j)
      v[j + B * r] = pmul(v[j + B * r], tab_at(mult, r * (N / S::rad(L)) + t + T * j));
  inverse_all<Real, S, CONTIG, L>(v, lds, t, col, tw);

  // v[e] holds position t + T e of pencil col; regroup so that lane (t2, col2)
  // holds positions t2 + T e of pencils col2 = tid % W (neighbouring lanes,
  // neighbouring A).  Regroup layout: row p of W columns with the column index
  // XOR-swizzled by the row.  The LDS serves 16 lanes of a 64-bit access (8 of a
  // 128-bit one) per cycle; with the swizzle neither the writes (consecutive rows of
  // one column) nor the reads (whole rows) of those lanes meet in a bank when
  // T >= 8, where the padded strided layout put 8 to 16 of them in one bank
  constexpr bool HALF = (W == 8 && SZ == 8);
  auto rg = [](int p, int c) { return p * W + (c ^ ((HALF ? (p >> 1) : 3 * p) & (W - 1))); };
  __syncthreads();                        // the last stage exchange has been read
#pragma unroll
  for (int e = 0; e < E; ++e) lds[rg(t + T * e, col)] = v[e];
  __syncthreads();
  const int col2 = tid % W, t2 = tid / W;
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = lds[rg(t2 + T * e, col2)];
  const auto out = gptr_mut<C>(a.out) + b * NN + (long)t2 * N + a0 + col2;
#pragma unroll
  for (int e = 0; e < E; ++e) out[(long)T * N * e] = v[e];
}

using RotLauncher = void (*)(const RotArgs&, unsigned grid, hipStream_t stream);

template <class Real, class S, int PRO>
void launch_rot(const RotArgs& a, unsigned grid, hipStream_t stream) {
  hipLaunchKernelGGL((rot_pass<Real, S, PRO>), dim3(grid), dim3(S::THREADS), 0, stream, a);
}

}  // namespace gpk
