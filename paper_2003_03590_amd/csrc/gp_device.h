// Device-side building blocks for the gfx950 Gross-Pitaevskii kernels:
// complex arithmetic, compile-time roots of unity and in-register DFTs.
//
// The in-register DFTs implement the radix butterflies of the Stockham-style
// axis passes (the spectral sub-steps S(s, L_j) of the time-evolution section
// are one forward 1-D transform, a diagonal multiply and one inverse transform
// along one axis).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace gpk {

template <class Real>
struct alignas(2 * sizeof(Real)) cplx {
  Real x, y;
};

template <class Real>
__device__ __forceinline__ cplx<Real> mk(Real a, Real b) { cplx<Real> r; r.x = a; r.y = b; return r; }
template <class Real>
__device__ __forceinline__ cplx<Real> operator+(cplx<Real> a, cplx<Real> b) { return mk(a.x + b.x, a.y + b.y); }
template <class Real>
__device__ __forceinline__ cplx<Real> operator-(cplx<Real> a, cplx<Real> b) { return mk(a.x - b.x, a.y - b.y); }
template <class Real>
__device__ __forceinline__ cplx<Real> cmul(cplx<Real> a, cplx<Real> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <class Real>
__device__ __forceinline__ cplx<Real> cmulc(cplx<Real> a, cplx<Real> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <class Real>
__device__ __forceinline__ cplx<Real> cscale(cplx<Real> a, Real s) { return mk(a.x * s, a.y * s); }
template <class Real>
__device__ __forceinline__ Real cabs2(cplx<Real> a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------------------
// Table entries.  complex128 tables hold the FP64 value.  complex64 tables hold
// the FP64 value as an unevaluated sum hi + lo of two FP32 complex numbers, so
// the FP32 kernels multiply by a constant accurate to ~1e-14: a constant
// rounded to FP32 would have |w| != 1 by up to 6e-8, a gain that repeats every
// pass and accumulates linearly over thousands of passes.
template <class Real> struct Tab;
template <> struct alignas(16) Tab<double> { cplx<double> v; };
template <> struct alignas(16) Tab<float> { cplx<float> hi, lo; };

__device__ __forceinline__ cplx<double> tmul(cplx<double> a, const Tab<double>& t) { return cmul(a, t.v); }
__device__ __forceinline__ cplx<double> tmulc(cplx<double> a, const Tab<double>& t) { return cmulc(a, t.v); }
// a * (hi + lo), the small products added first
__device__ __forceinline__ cplx<float> tmul(cplx<float> a, const Tab<float>& t) {
  const float sr = a.x * t.lo.x - a.y * t.lo.y, si = a.x * t.lo.y + a.y * t.lo.x;
  return mk(fmaf(a.x, t.hi.x, fmaf(-a.y, t.hi.y, sr)), fmaf(a.x, t.hi.y, fmaf(a.y, t.hi.x, si)));
}
// a * conj(hi + lo)
__device__ __forceinline__ cplx<float> tmulc(cplx<float> a, const Tab<float>& t) {
  const float sr = a.x * t.lo.x + a.y * t.lo.y, si = a.y * t.lo.x - a.x * t.lo.y;
  return mk(fmaf(a.x, t.hi.x, fmaf(a.y, t.hi.y, sr)), fmaf(a.y, t.hi.x, fmaf(-a.x, t.hi.y, si)));
}

// Multiplier between the forward and the inverse transform (propagator, spectral
// derivative): an FP64 complex table entry for both precisions.  FP32 data is
// widened, multiplied in FP64 and rounded once; the compensated FP32 product
// (tmul) leaves a rounding bias that grows the norm by about 1e-9 per pass when
// the multiplier is a nontrivial phase, which accumulates into mass and energy
// drift over a run.
__device__ __forceinline__ cplx<double> pmul(cplx<double> a, cplx<double> m) { return cmul(a, m); }
__device__ __forceinline__ cplx<float> pmul(cplx<float> a, cplx<double> m) {
  const double x = a.x, y = a.y;
  return mk(float(fma(x, m.x, -y * m.y)), float(fma(x, m.y, y * m.x)));
}

// ---------------------------------------------------------------------------
// Compile-time cos/sin of 2*pi*m/R.  The angle is reduced exactly in integers
// to [0, pi/4] and evaluated with a Taylor series in double (error ~1 ulp).
namespace ct {
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double sin_series(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 16; ++i) { term *= -x2 / double((2 * i) * (2 * i + 1)); sum += term; }
  return sum;
}
constexpr double cos_series(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 16; ++i) { term *= -x2 / double((2 * i - 1) * (2 * i)); sum += term; }
  return sum;
}
// cos(2 pi m / R)
constexpr double cos2pi(long m, long R) {
  long mm = ((m % R) + R) % R;               // [0, R)
  long q = (4 * mm) / R;                     // quadrant 0..3
  long r = 4 * mm - q * R;                   // angle within quadrant = (pi/2) r/R
  double c = 0, s = 0;
  if (2 * r <= R) {                          // (pi/2) r/R <= pi/4
    double a = (kPi / 2) * double(r) / double(R);
    c = cos_series(a); s = sin_series(a);
  } else {
    double a = (kPi / 2) * double(R - r) / double(R);
    c = sin_series(a); s = cos_series(a);
  }
  // rotate by q quadrants: (c, s) -> angle + q*pi/2
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}

// Unit complex constants as FP64 pairs whose norm is as close to 1 as the format
// allows.  The transform applies a constant w in the forward pass and conj(w) in
// the inverse, so every pass multiplies the modes on w's path by |w|^2; a rounded
// pair has |w|^2 - 1 of up to ~2e-16 (of one sign for the series values of a given
// radix), which repeats every pass and adds up over a run.  Among the pairs within
// two units in the last place of (c, s) the one with the smallest |c^2 + s^2 - 1|
// is taken: the angle moves by a few 1e-16 (a phase, which the inverse undoes), the
// norm error drops to ~1e-18.
constexpr void two_prod(double a, double b, double& p, double& e) {   // a b = p + e exactly
  p = a * b;
  const double sa = 134217729.0 * a, ah = sa - (sa - a), al = a - ah;
  const double sb = 134217729.0 * b, bh = sb - (sb - b), bl = b - bh;
  e = ((ah * bh - p) + ah * bl + al * bh) + al * bl;
}
constexpr double norm_err(double c, double s) {                        // c^2 + s^2 - 1
  double pc = 0, ec = 0, ps = 0, es = 0;
  two_prod(c, c, pc, ec);
  two_prod(s, s, ps, es);
  const double t = pc >= ps ? (pc - 1.0) + ps : (ps - 1.0) + pc;
  return t + (ec + es);
}
constexpr double ulp_step(double x, int k) {                           // k units in the last place
  return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, x) + (long long)k);
}
struct Pair { double c, s; };
constexpr Pair unit_pair(double c, double s) {
  Pair best{c, s};
  double be = norm_err(c, s);
  be = be < 0 ? -be : be;
  for (int i = -2; i <= 2; ++i)
    for (int j = -2; j <= 2; ++j) {
      if ((c == 0.0 && i != 0) || (s == 0.0 && j != 0)) continue;      // exact zeros stay
      const double cc = ulp_step(c, i), ss = ulp_step(s, j);
      double e = norm_err(cc, ss);
      e = e < 0 ? -e : e;
      if (e < be) { be = e; best = Pair{cc, ss}; }
    }
  return best;
}
}  // namespace ct

// exp(sgn * 2 pi i m / R) as compile-time constants; sgn = -1 forward, +1 inverse.
// sin(2 pi m/R) = cos(2 pi m/R - pi/2) = cos(2 pi (4m - R) / (4R)); the pair is the
// norm-closest one (ct::unit_pair), the same for both signs.
template <int M, int R, int SGN>
struct Root {
  static constexpr ct::Pair u = ct::unit_pair(ct::cos2pi(M, R), ct::cos2pi(4L * M - R, 4L * R));
  static constexpr double c = u.c;
  static constexpr double s = SGN * u.s;
};

// multiply v by exp(SGN * 2 pi i M / R), with exact special cases
template <int M, int R, int SGN, class Real>
__device__ __forceinline__ cplx<Real> rot(cplx<Real> v) {
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (2 * m == R) {
    return mk(-v.x, -v.y);
  } else if constexpr (4 * m == R) {            // exp(SGN i pi/2) = SGN * i
    return SGN < 0 ? mk(v.y, -v.x) : mk(-v.y, v.x);
  } else if constexpr (4 * m == 3 * R) {        // exp(SGN i 3pi/2) = -SGN * i
    return SGN < 0 ? mk(-v.y, v.x) : mk(v.y, -v.x);
  } else if constexpr (sizeof(Real) == 4) {
    // FP32: constant carried as hi + lo (see Tab<float>)
    constexpr double cd = Root<m, R, SGN>::c, sd = Root<m, R, SGN>::s;
    constexpr float ch = float(cd), sh = float(sd);
    constexpr float cl = float(cd - double(ch)), sl = float(sd - double(sh));
    const float sr = v.x * cl - v.y * sl, si = v.x * sl + v.y * cl;
    return mk(fmaf(v.x, ch, fmaf(-v.y, sh, sr)), fmaf(v.x, sh, fmaf(v.y, ch, si)));
  } else {
    constexpr double c = Root<m, R, SGN>::c, s = Root<m, R, SGN>::s;
    return mk(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// ---------------------------------------------------------------------------
// (cos a, sin a) for the nonlinear phase rotation.  The rotation angle
// beta (|psi|^2 - 1) dt is small in practice, so |a| <= 1/16 takes short Taylor
// series without reduction (FP64: through a^9 and a^8, truncation below 1e-18 of
// the result; FP32: through a^5 and a^4, below 1e-10).  Otherwise, for |a| < 1024,
// the angle is reduced as a = q pi/2 + r with pi/2 split into two doubles
// (hi = fl(pi/2), lo = fl(pi/2 - hi)) and fused multiply-adds, then sin r and
// cos r come from their Taylor series on |r| <= pi/4 (truncation below 1e-19).
// Larger angles use the library routine.  This keeps the fused prologue small in
// registers.
namespace ct {
constexpr double inv_fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= double(i); return 1.0 / f; }
}  // namespace ct

__device__ __forceinline__ void sincos_rot(double a, double* sn, double* cs) {
  if (fabs(a) <= 0.0625) {
    const double r2 = a * a;
    double ps = ct::inv_fact(9);
    ps = fma(ps, r2, -ct::inv_fact(7));
    ps = fma(ps, r2, ct::inv_fact(5));
    ps = fma(ps, r2, -ct::inv_fact(3));
    *sn = fma(ps * r2, a, a);
    double pc = ct::inv_fact(8);
    pc = fma(pc, r2, -ct::inv_fact(6));
    pc = fma(pc, r2, ct::inv_fact(4));
    pc = fma(pc, r2, -0.5);
    *cs = fma(pc, r2, 1.0);
  } else if (fabs(a) < 1024.0) {
    const double q = rint(a * 0.6366197723675814);
    double r = fma(-q, 1.5707963267948966, a);
    r = fma(-q, 6.123233995736766e-17, r);
    const double r2 = r * r;
    double ps = -ct::inv_fact(19);
    ps = fma(ps, r2, ct::inv_fact(17));
    ps = fma(ps, r2, -ct::inv_fact(15));
    ps = fma(ps, r2, ct::inv_fact(13));
    ps = fma(ps, r2, -ct::inv_fact(11));
    ps = fma(ps, r2, ct::inv_fact(9));
    ps = fma(ps, r2, -ct::inv_fact(7));
    ps = fma(ps, r2, ct::inv_fact(5));
    ps = fma(ps, r2, -ct::inv_fact(3));
    const double S = fma(ps * r2, r, r);
    double pc = ct::inv_fact(20);
    pc = fma(pc, r2, -ct::inv_fact(18));
    pc = fma(pc, r2, ct::inv_fact(16));
    pc = fma(pc, r2, -ct::inv_fact(14));
    pc = fma(pc, r2, ct::inv_fact(12));
    pc = fma(pc, r2, -ct::inv_fact(10));
    pc = fma(pc, r2, ct::inv_fact(8));
    pc = fma(pc, r2, -ct::inv_fact(6));
    pc = fma(pc, r2, ct::inv_fact(4));
    pc = fma(pc, r2, -0.5);
    const double C = fma(pc, r2, 1.0);
    const int n = int(q) & 3;
    *sn = n == 0 ? S : n == 1 ? C : n == 2 ? -S : -C;
    *cs = n == 0 ? C : n == 1 ? -S : n == 2 ? -C : S;
  } else {
    sincos(a, sn, cs);
  }
}

__device__ __forceinline__ void sincos_rot(float a, float* sn, float* cs) {
  if (fabsf(a) <= 0.0625f) {
    const float r2 = a * a;
    const float ps = fmaf(float(ct::inv_fact(5)), r2, float(-ct::inv_fact(3)));
    *sn = fmaf(ps * r2, a, a);
    float pc = fmaf(float(ct::inv_fact(4)), r2, -0.5f);
    *cs = fmaf(pc, r2, 1.0f);
  } else if (fabsf(a) < 1024.0f) {
    const float q = rintf(a * 0.63661975f);
    float r = fmaf(-q, 1.5707963705062866f, a);
    r = fmaf(-q, -4.371138828673793e-08f, r);
    const float r2 = r * r;
    float ps = float(-ct::inv_fact(11));
    ps = fmaf(ps, r2, float(ct::inv_fact(9)));
    ps = fmaf(ps, r2, float(-ct::inv_fact(7)));
    ps = fmaf(ps, r2, float(ct::inv_fact(5)));
    ps = fmaf(ps, r2, float(-ct::inv_fact(3)));
    const float S = fmaf(ps * r2, r, r);
    float pc = float(ct::inv_fact(12));
    pc = fmaf(pc, r2, float(-ct::inv_fact(10)));
    pc = fmaf(pc, r2, float(ct::inv_fact(8)));
    pc = fmaf(pc, r2, float(-ct::inv_fact(6)));
    pc = fmaf(pc, r2, float(ct::inv_fact(4)));
    pc = fmaf(pc, r2, -0.5f);
    const float C = fmaf(pc, r2, 1.0f);
    const int n = int(q) & 3;
    *sn = n == 0 ? S : n == 1 ? C : n == 2 ? -S : -C;
    *cs = n == 0 ? C : n == 1 ? -S : n == 2 ? -C : S;
  } else {
    sincosf(a, sn, cs);
  }
}

// exp(i a) - 1 = cm1 + i sn for FP32 data, with cm1 = cos a - 1 to full relative
// precision (the series gives it directly; larger angles use -2 sin^2(a/2)).
// The rotation is then applied as v + v (cm1 + i sn): the factor's norm is 1 to
// O(u a), where fl(cos a) + i fl(sin a) is off by up to u -- for |a| below
// ~2.4e-4, fl(cos a) = 1 while sin a != 0 -- a gain that repeats at a point
// every step with the slowly varying angle and so adds up coherently.
__device__ __forceinline__ void sincos_m1(float a, float* sn, float* cm1) {
  if (fabsf(a) <= 0.0625f) {
    const float r2 = a * a;
    const float ps = fmaf(float(ct::inv_fact(5)), r2, float(-ct::inv_fact(3)));
    *sn = fmaf(ps * r2, a, a);
    const float pc = fmaf(float(ct::inv_fact(4)), r2, -0.5f);
    *cm1 = pc * r2;
  } else {
    float sh, ch;
    sincos_rot(0.5f * a, &sh, &ch);
    *sn = 2.0f * sh * ch;
    *cm1 = -2.0f * sh * sh;
  }
}

constexpr int smallest_factor(int n) {
  if (n % 4 == 0) return 4;                        // radix-4 first: trivial internal rotations
  if (n % 2 == 0) return 2;
  if (n % 3 == 0) return 3;
  return n;
}

// In-register DFT of R points, natural order in and out:
//   X[k] = sum_n x[n] exp(SGN 2 pi i n k / R)
// Recursive Cooley-Tukey: R = A*B, n = B*n1 + n2, k = k1 + A*k2.
template <int R, int SGN, class Real>
struct Dft {
  static __device__ __forceinline__ void run(cplx<Real>* x);
};

template <int SGN, class Real>
struct Dft<1, SGN, Real> { static __device__ __forceinline__ void run(cplx<Real>*) {} };

template <int SGN, class Real>
struct Dft<2, SGN, Real> {
  static __device__ __forceinline__ void run(cplx<Real>* x) {
    cplx<Real> a = x[0], b = x[1];
    x[0] = a + b; x[1] = a - b;
  }
};

template <int SGN, class Real>
struct Dft<3, SGN, Real> {
  static __device__ __forceinline__ void run(cplx<Real>* x) {
    // c1 = cos(2pi/3) = -1/2, s1 = SGN*sin(2pi/3)
    constexpr Real h = Real(0.5);
    constexpr Real s = Real(SGN * 0.86602540378443864676372317075293618);
    cplx<Real> a = x[0], b = x[1], c = x[2];
    cplx<Real> t = b + c, d = b - c;
    cplx<Real> m = mk(a.x - h * t.x, a.y - h * t.y);
    x[0] = a + t;
    // X1 = a + b w + c w^2,  w = exp(SGN 2pi i/3) = -1/2 + i s
    Real sdx, sdy;
    if constexpr (sizeof(Real) == 4) {
      // s carried as hi + lo: an FP32-rounded s makes |w| != 1 by ~3e-8, a gain
      // on every mode not divisible by 3 that repeats in each radix-3 stage
      constexpr double sd = SGN * 0.86602540378443864676372317075293618;
      constexpr float shi = float(sd), slo = float(sd - double(shi));
      sdx = fmaf(shi, d.x, slo * d.x);
      sdy = fmaf(shi, d.y, slo * d.y);
    } else {
      sdx = s * d.x;
      sdy = s * d.y;
    }
    x[1] = mk(m.x - sdy, m.y + sdx);
    x[2] = mk(m.x + sdy, m.y - sdx);
  }
};

template <int SGN, class Real>
struct Dft<4, SGN, Real> {
  static __device__ __forceinline__ void run(cplx<Real>* x) {
    cplx<Real> a = x[0] + x[2], b = x[0] - x[2], c = x[1] + x[3], d = x[1] - x[3];
    // d * (SGN i)
    cplx<Real> di = SGN < 0 ? mk(d.y, -d.x) : mk(-d.y, d.x);
    x[0] = a + c; x[2] = a - c;
    x[1] = b + di; x[3] = b - di;
  }
};

template <int R, int SGN, class Real>
__device__ __forceinline__ void Dft<R, SGN, Real>::run(cplx<Real>* x) {
  constexpr int A = smallest_factor(R);
  constexpr int B = R / A;
  static_assert(A * B == R && A > 1 && B > 1, "unsupported radix");
  cplx<Real> y[R];
  // A-point DFTs over n1 for each n2, then twiddle W_R^{n2 k1}
#pragma unroll
  for (int n2 = 0; n2 < B; ++n2) {
    cplx<Real> t[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) t[n1] = x[B * n1 + n2];
    Dft<A, SGN, Real>::run(t);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) y[k1 * B + n2] = t[k1];
  }
  // twiddles (compile-time indices after unrolling)
  [&]<int... I>(std::integer_sequence<int, I...>) {
    ((y[I] = rot<(I % B) * (I / B), R, SGN>(y[I])), ...);
  }(std::make_integer_sequence<int, R>{});
  // B-point DFTs over n2 for each k1
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    Dft<B, SGN, Real>::run(&y[k1 * B]);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = y[k1 * B + k2];
  }
}

}  // namespace gpk
