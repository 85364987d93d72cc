// Pointwise and reduction kernels of the Gross-Pitaevskii library:
// the initial phase field, the standalone nonlinear sub-step, the
// hydrodynamic diagnostics (energy decomposition and shell spectra), the
// imaginary-time (ARGLE) step and its energy, the spectral loss and its
// gradient, the phase gradient, the density and velocity structure functions,
// the Mach numbers and the helicities.  All reductions are deterministic:
// fixed-order wave butterflies, per-workgroup partials, and a fixed-order final
// sum with Neumaier compensation (maxima are order-free); shell bins are
// accumulated per wavefront in LDS.
#include "gp_point.h"

namespace gpk {

// ----------------------------------------------------------------- helpers
struct Neu {          // Neumaier compensated sum
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ __forceinline__ double val() const { return s + c; }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block of 256 threads: sum of v in a fixed order, result valid in thread 0
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + (sh[2] + sh[3]));
  return r;
}

template <class Real>
__device__ __forceinline__ cplx<Real> ldc(const void* p, long i) { return reinterpret_cast<const cplx<Real>*>(p)[i]; }
template <class Real>
__device__ __forceinline__ void stc(void* p, long i, double re, double im) {
  reinterpret_cast<cplx<Real>*>(p)[i] = mk(Real(re), Real(im));
}

// integer shell s = round(|k|): (2s-1)^2 <= 4|k|^2 < (2s+1)^2
__device__ __forceinline__ int shell_of(long k2) {
  const long q = 4 * k2;
  long r = (long)sqrt((double)q);
  while (r * r > q) --r;
  while ((r + 1) * (r + 1) <= q) ++r;
  return (int)((r + 1) / 2);
}

__device__ __forceinline__ int kfreq(int i, int n) { return (2 * i < n) ? i : i - n; }  // fftfreq (Nyquist -> -n/2)

// Grid coordinates of linear index i (x fastest).  Indices below 2^32 use 32-bit
// unsigned division: a 64-bit division is a long software sequence on the GPU, and
// per point it cost more than the arithmetic of the kernels that need coordinates.
__device__ __forceinline__ void grid_xyz(long i, int nx, int ny, int& ix, int& iy, int& iz) {
  if ((unsigned long)i <= 0xFFFFFFFFul) {
    const unsigned u = (unsigned)i, r = u / (unsigned)nx, q = r / (unsigned)ny;
    ix = (int)(u - r * (unsigned)nx);
    iy = (int)(r - q * (unsigned)ny);
    iz = (int)q;
  } else {
    const long r = i / nx, q = r / ny;
    ix = (int)(i - r * nx);
    iy = (int)(r - q * ny);
    iz = (int)q;
  }
}
// index of the mirror point -x on a periodic axis of n points
__device__ __forceinline__ int mirror_of(int i, int n) { return i ? n - i : 0; }

// ----------------------------------------------------------------- elementwise
template <class Real>
__global__ void k_init_phase(const double* __restrict__ theta, void* psi, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double s, c;
    sincos(theta[i], &s, &c);
    stc<Real>(psi, i, c, s);
  }
}

template <class Real>
__global__ void k_nonlinear(void* psi, long n, double coef) {
  cplx<Real>* p = reinterpret_cast<cplx<Real>*>(psi);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = nl_rotate(p[i], coef);
}

template <class Real>
__global__ void k_scale_copy(const void* in, void* out, long n, double scale) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const cplx<Real> v = ldc<Real>(in, i);
    stc<Real>(out, i, (double)v.x * scale, (double)v.y * scale);
  }
}

// multiply by the separable 3-D propagator mx[kx] my[ky] mz[kz] (natural order tables)
template <class Real>
__global__ void k_mult3(void* f, int nx, int ny, int nz, const void* mx, const void* my, const void* mz) {
  const long n = (long)nx * ny * nz;
  cplx<Real>* p = reinterpret_cast<cplx<Real>*>(f);
  const cplx<double>* tx = reinterpret_cast<const cplx<double>*>(mx);
  const cplx<double>* ty = reinterpret_cast<const cplx<double>*>(my);
  const cplx<double>* tz = reinterpret_cast<const cplx<double>*>(mz);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    grid_xyz(i, nx, ny, ix, iy, iz);
    p[i] = pmul(p[i], cmul(cmul(tx[ix], ty[iy]), tz[iz]));      // product of the factors in FP64
  }
}

// ----------------------------------------------------- imaginary time (ARGLE)
// Section on stationary solutions: the advective real Ginzburg-Landau equation
// (eq. gradient-flow) advanced by the semi-implicit backward Euler scheme
// (eq. semi-backward-Euler).  v holds three real fields v_x, v_y, v_z of the working
// precision; d_x, d_y, d_z are the spectral first derivatives of phi.

// explicit part: n = -i v.grad phi + (beta - |v|^2/(4 alpha) - beta |phi|^2) phi.
// One point per thread (n <= 2^30, so 32-bit indices), q4a = 1/(4 alpha).
template <class Real>
__global__ __launch_bounds__(256) void k_argle_explicit(const void* phi, const void* dx, const void* dy,
                                                        const void* dz, const void* v, void* out, unsigned n,
                                                        double q4a, double beta) {
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const Real* vx = reinterpret_cast<const Real*>(v);
  const cplx<Real> p = ldc<Real>(phi, i), a = ldc<Real>(dx, i), b = ldc<Real>(dy, i), c = ldc<Real>(dz, i);
  const double ux = vx[i], uy = vx[n + i], uz = vx[2u * n + i];
  const double gr = ux * a.x + uy * b.x + uz * c.x, gi = ux * a.y + uy * b.y + uz * c.y;   // v.grad phi
  const double pr = p.x, pi = p.y;
  const double f = beta - (ux * ux + uy * uy + uz * uz) * q4a - beta * (pr * pr + pi * pi);
  stc<Real>(out, i, gi + f * pr, -gr + f * pi);                                             // -i (gr + i gi) + f phi
}

// the implicit half of the Laplacian, diagonal in Fourier space, on unnormalised
// transforms P = F(phi^n), Q = F(n): P <- ((1 - a k^2) P + dtau Q) / ((1 + a k^2) N^3),
// a = dtau alpha / 2, |k|^2 with the Nyquist entry N^2/4.  Grid: x = rows (y, z),
// y = 256-point chunks of a row.
template <class Real>
__global__ __launch_bounds__(256) void k_argle_solve(void* P, const void* Q, int nx, int ny, int nz, double a,
                                                     double dtau, double inv_n) {
  const int ix = blockIdx.y * 256 + threadIdx.x;
  if (ix >= nx) return;
  const unsigned row = blockIdx.x;                     // uniform: iy, iz on the scalar unit
  const int iy = (int)(row % (unsigned)ny), iz = (int)(row / (unsigned)ny);
  const unsigned i = row * (unsigned)nx + (unsigned)ix;
  const double kx = kfreq(ix, nx), ky = kfreq(iy, ny), kz = kfreq(iz, nz);
  const double k2 = kx * kx + ky * ky + kz * kz;
  const double num = 1.0 - a * k2, den = inv_n / (1.0 + a * k2);
  const cplx<Real> p = ldc<Real>(P, i), q = ldc<Real>(Q, i);
  stc<Real>(P, i, (num * (double)p.x + dtau * (double)q.x) * den, (num * (double)p.y + dtau * (double)q.y) * den);
}

// per-workgroup partial sums of alpha |grad phi - i v phi/(2 alpha)|^2 + (beta/2)(|phi|^2 - 1)^2
// (the integrand of eq. energy-num-ext-vel without its factor 2 alpha / L^3)
template <class Real>
__global__ __launch_bounds__(256) void k_argle_energy(const void* phi, const void* dx, const void* dy, const void* dz,
                                                      const void* v, long n, double alpha, double beta,
                                                      double* __restrict__ partial) {
  __shared__ double sh[4];
  const Real* vx = reinterpret_cast<const Real*>(v);
  const Real* vy = vx + n;
  const Real* vz = vy + n;
  const double h = 0.5 / alpha;
  Neu acc;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const cplx<Real> p = ldc<Real>(phi, i);
    const cplx<Real> d[3] = {ldc<Real>(dx, i), ldc<Real>(dy, i), ldc<Real>(dz, i)};
    const double u[3] = {(double)vx[i], (double)vy[i], (double)vz[i]};
    const double pr = p.x, pi = p.y, rho = pr * pr + pi * pi;
    double g = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double re = (double)d[j].x + u[j] * h * pi, im = (double)d[j].y - u[j] * h * pr;   // d_j - i v_j h phi
      g += re * re + im * im;
    }
    acc.add(alpha * g + 0.5 * beta * (rho - 1.0) * (rho - 1.0));
  }
  const double tot = block_sum256(acc.val(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// max |a - b|^2 over the field (sup norm of an update, eq. crit1): per-block maxima
// in partial[block]; the maximum is exact, so the result does not depend on order.
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double block_max256(double v, double* sh) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  return r;
}

template <class Real>
__global__ __launch_bounds__(256) void k_sup_diff2(const void* a, const void* b, long n,
                                                   double* __restrict__ partial) {
  __shared__ double sh[4];
  double m = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const cplx<Real> x = ldc<Real>(a, i), y = ldc<Real>(b, i);
    const double dr = (double)x.x - (double)y.x, di = (double)x.y - (double)y.y;
    m = fmax(m, dr * dr + di * di);
  }
  const double r = block_max256(m, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_segmax(const double* __restrict__ in, long len, double* __restrict__ out) {
  __shared__ double sh[4];
  double m = 0.0;
  for (long b = threadIdx.x; b < len; b += 256) m = fmax(m, in[b]);
  const double r = block_max256(m, sh);
  if (threadIdx.x == 0) out[0] = r;
}

// ----------------------------------------------------------------- diagnostics
// In: psi and its spectral derivatives d0 = d/dx, d1 = d/dy, d2 = d/dz (in f0, f1, f2).
// Out (in place): f0 = w_x + i w_y, f1 = w_z + i q_x, f2 = q_y + i q_z, f3 = (|psi|^2 - 1) + 0i,
// w = 2 alpha Im(conj(psi) grad psi)/|psi| and q = 2 alpha Re(conj(psi) grad psi)/|psi|
// (= 2 alpha grad sqrt(rho)); both 0 where psi = 0.
// Partials [quantity][block]: sum rho, sum (rho-1)^2, sum |w|^2.
template <class Real>
__global__ __launch_bounds__(256) void k_diag_fields(const void* psi, void* f0, void* f1, void* f2, void* f3, long n,
                                                     double alpha, double* __restrict__ partial) {
  __shared__ double sh[4];
  Neu a0, a1, a2;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const cplx<Real> p = ldc<Real>(psi, i);
    const cplx<Real> dx = ldc<Real>(f0, i), dy = ldc<Real>(f1, i), dz = ldc<Real>(f2, i);
    const double pr = p.x, pi = p.y;
    const double rho = pr * pr + pi * pi;
    const double amp = sqrt(rho);
    double wx = 0, wy = 0, wz = 0, qx = 0, qy = 0, qz = 0;
    if (amp > 0.0) {
      const double f = 2.0 * alpha / amp;
      wx = f * (pr * (double)dx.y - pi * (double)dx.x);
      wy = f * (pr * (double)dy.y - pi * (double)dy.x);
      wz = f * (pr * (double)dz.y - pi * (double)dz.x);
      qx = f * (pr * (double)dx.x + pi * (double)dx.y);
      qy = f * (pr * (double)dy.x + pi * (double)dy.y);
      qz = f * (pr * (double)dz.x + pi * (double)dz.y);
    }
    stc<Real>(f0, i, wx, wy);
    stc<Real>(f1, i, wz, qx);
    stc<Real>(f2, i, qy, qz);
    stc<Real>(f3, i, rho - 1.0, 0.0);
    a0.add(rho);
    a1.add((rho - 1.0) * (rho - 1.0));
    a2.add(wx * wx + wy * wy + wz * wz);
  }
  const double s0 = block_sum256(a0.val(), sh);
  const double s1 = block_sum256(a1.val(), sh);
  const double s2 = block_sum256(a2.val(), sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s0;
    partial[gridDim.x + blockIdx.x] = s1;
    partial[2 * gridDim.x + blockIdx.x] = s2;
  }
}

// Shell binning of the hydrodynamic spectra.  F0 = FFT(w_x + i w_y), F1 = FFT(w_z + i q_x),
// F2 = FFT(q_y + i q_z), F3 = FFT(rho - 1) (unnormalised, natural order).  Per k: unpack
// the real-field transforms with the mirror -k, normalise by 1/Ntot, split w into
// compressible (parallel to k) and incompressible parts, and add 1/2|w^i|^2, 1/2|w^c|^2,
// 1/2|q|^2, alpha beta |b|^2 to shell round(|k|).  One wavefront per workgroup; bins
// live in LDS.
// Shell densities of E_kin^i, E_kin^c, E_q, E_int at one point of the four packed
// transforms: z = F(k), zm = F(mirror point), (kx, ky, kz) the point's wavenumbers.
template <class Real>
__device__ __forceinline__ void spectral_terms(const cplx<Real>* z, const cplx<Real>* zm, int kx, int ky, int kz,
                                               double inv, double ab, double* d) {
  // A = (Z + conj Zm)/2, B = (Z - conj Zm)/(2i)
  const double wxr = 0.5 * ((double)z[0].x + zm[0].x) * inv, wxi = 0.5 * ((double)z[0].y - zm[0].y) * inv;
  const double wyr = 0.5 * ((double)z[0].y + zm[0].y) * inv, wyi = -0.5 * ((double)z[0].x - zm[0].x) * inv;
  const double wzr = 0.5 * ((double)z[1].x + zm[1].x) * inv, wzi = 0.5 * ((double)z[1].y - zm[1].y) * inv;
  const double qxr = 0.5 * ((double)z[1].y + zm[1].y) * inv, qxi = -0.5 * ((double)z[1].x - zm[1].x) * inv;
  const double qyr = 0.5 * ((double)z[2].x + zm[2].x) * inv, qyi = 0.5 * ((double)z[2].y - zm[2].y) * inv;
  const double qzr = 0.5 * ((double)z[2].y + zm[2].y) * inv, qzi = -0.5 * ((double)z[2].x - zm[2].x) * inv;
  const double br = 0.5 * ((double)z[3].x + zm[3].x) * inv, bi = 0.5 * ((double)z[3].y - zm[3].y) * inv;
  const long k2 = (long)kx * kx + (long)ky * ky + (long)kz * kz;
  double cr = 0, ci = 0;
  if (k2 > 0) {
    const double kdr = kx * wxr + ky * wyr + kz * wzr, kdi = kx * wxi + ky * wyi + kz * wzi;
    cr = kdr / (double)k2; ci = kdi / (double)k2;
  }
  const double cxr = kx * cr, cxi = kx * ci, cyr = ky * cr, cyi = ky * ci, czr = kz * cr, czi = kz * ci;
  d[1] = 0.5 * (cxr * cxr + cxi * cxi + cyr * cyr + cyi * cyi + czr * czr + czi * czi);
  const double ixr = wxr - cxr, ixi = wxi - cxi, iyr = wyr - cyr, iyi = wyi - cyi, izr = wzr - czr, izi = wzi - czi;
  d[0] = 0.5 * (ixr * ixr + ixi * ixi + iyr * iyr + iyi * iyi + izr * izr + izi * izi);
  d[2] = 0.5 * (qxr * qxr + qxi * qxi + qyr * qyr + qyi * qyi + qzr * qzr + qzi * qzi);
  d[3] = ab * (br * br + bi * bi);
}

template <class Real>
__global__ __launch_bounds__(64) void k_spectral(const void* F0, const void* F1, const void* F2, const void* F3,
                                                 int nx, int ny, int nz, double alpha, double beta, int nshell,
                                                 long chunk, double* __restrict__ bins_partial) {
  // The four transforms hold pairs of real fields, so the densities at -k equal
  // those at k (A(-k) = conj A(k), B(-k) = conj B(k), and the Helmholtz parts
  // follow), in the same shell.  Each pair {k, mirror} is visited once: only the
  // planes iz = 0 .. nz/2, and in the planes that are their own mirror only the
  // point of the pair with the smaller index.  The pair counts twice, except that a
  // point that is its own mirror counts once, and a point with a Nyquist component
  // (whose mirror index keeps the wavenumber -N/2, so it is not -k) has its mirror
  // evaluated with the mirror's own wavenumbers.  Consecutive lanes take
  // consecutive points (coalesced loads, the mirror loads in descending order);
  // a lane adds its points' terms in registers while they stay in one shell and
  // only then into the LDS bins.
  extern __shared__ double bins[];            // [4][nshell]
  for (int i = threadIdx.x; i < 4 * nshell; i += 64) bins[i] = 0.0;
  __syncthreads();
  const long n = (long)nx * ny * nz;
  const long nh = (long)(nz / 2 + 1) * nx * ny;
  const double inv = 1.0 / (double)n, ab = alpha * beta;
  const long i0 = (long)blockIdx.x * chunk;
  const long i1 = (i0 + chunk < nh) ? i0 + chunk : nh;
  const void* F[4] = {F0, F1, F2, F3};
  auto nyq = [](int i, int nn) { return (nn % 2 == 0) && 2 * i == nn; };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int cur = -1;
  {
    for (long i = i0 + threadIdx.x; i < i1; i += 64) {
      int ix, iy, iz;
      grid_xyz(i, nx, ny, ix, iy, iz);
      const int mx = mirror_of(ix, nx), my = mirror_of(iy, ny), mz = mirror_of(iz, nz);
      const long m = (long)mz * nx * ny + (long)my * nx + mx;
      if (m < i) continue;                    // counted with its mirror
      cplx<Real> z[4], zm[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) { z[f] = ldc<Real>(F[f], i); zm[f] = ldc<Real>(F[f], m); }
      const int kx = kfreq(ix, nx), ky = kfreq(iy, ny), kz = kfreq(iz, nz);
      double d[4];
      spectral_terms<Real>(z, zm, kx, ky, kz, inv, ab, d);
      if (m == i) {
        // own mirror: once
      } else if (nyq(ix, nx) || nyq(iy, ny) || nyq(iz, nz)) {
        double d2[4];
        spectral_terms<Real>(zm, z, kfreq(mx, nx), kfreq(my, ny), kfreq(mz, nz), inv, ab, d2);
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] += d2[q];
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] *= 2.0;
      }
      const int s = shell_of((long)kx * kx + (long)ky * ky + (long)kz * kz);
      if (s != cur) {
        if (cur >= 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q) atomicAdd(&bins[q * nshell + cur], acc[q]);
        }
        cur = s;
        acc[0] = acc[1] = acc[2] = acc[3] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += d[q];
    }
  }
  if (cur >= 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) atomicAdd(&bins[q * nshell + cur], acc[q]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * nshell; i += 64) bins_partial[(long)i * gridDim.x + blockIdx.x] = bins[i];
}

// Deterministic segmented sum: out[q] = sum_{b < len} in[q * len + b] for q < nseg.
// One block of 256 threads per segment: strided Neumaier partials per thread, then
// a fixed-order tree over the 256 threads (wave butterflies, then waves in order).
__global__ __launch_bounds__(256) void k_segsum(const double* __restrict__ in, long len, double* __restrict__ out) {
  __shared__ double sh[4];
  const double* seg = in + (long)blockIdx.x * len;
  Neu a;
  for (long b = threadIdx.x; b < len; b += 256) a.add(seg[b]);
  const double v = block_sum256(a.val(), sh);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// Energies from the reduced sums.  red = [kin_x, kin_y, kin_z, sum rho, sum (rho-1)^2,
// sum |w|^2, spectra[4][nshell]]; out[0..6] = gp_energy, out[7..] = spectra.
__global__ __launch_bounds__(256) void k_finalize_diag(const double* __restrict__ red, double kin_w0, double kin_w1,
                                                       double kin_w2, int nshell, double alpha, double beta,
                                                       double ntot, double* __restrict__ out) {
  const double* spec = red + 6;
  for (int q = threadIdx.x; q < 4 * nshell; q += 256) out[7 + q] = spec[q];
  if (threadIdx.x == 0) {
    Neu ei, ec, eq;
    for (int s = 0; s < nshell; ++s) { ei.add(spec[s]); ec.add(spec[nshell + s]); eq.add(spec[2 * nshell + s]); }
    const double kin_grad = red[0] * kin_w0 + red[1] * kin_w1 + red[2] * kin_w2;
    const double e_int = alpha * beta * red[4] / ntot;
    out[0] = red[3] / ntot;                           // mass
    out[1] = 2.0 * alpha * alpha * kin_grad + e_int;  // energy
    out[2] = 0.5 * red[5] / ntot;                     // e_kin
    out[3] = ei.val();
    out[4] = ec.val();
    out[5] = eq.val();
    out[6] = e_int;
  }
}

// ----------------------------------------------------------------- loss and its gradient
// f0 <- w_x + i w_y, f1 <- w_z (d0, d1, d2 keep the derivatives)
template <class Real>
__global__ __launch_bounds__(256) void k_loss_fields(const void* psi, const void* d0, const void* d1, const void* d2,
                                                     void* f0, void* f1, long n, double alpha) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const cplx<Real> p = ldc<Real>(psi, i);
    const cplx<Real> dx = ldc<Real>(d0, i), dy = ldc<Real>(d1, i), dz = ldc<Real>(d2, i);
    const double pr = p.x, pi = p.y, amp = sqrt(pr * pr + pi * pi);
    double wx = 0, wy = 0, wz = 0;
    if (amp > 0.0) {
      const double f = 2.0 * alpha / amp;
      wx = f * (pr * (double)dx.y - pi * (double)dx.x);
      wy = f * (pr * (double)dy.y - pi * (double)dy.x);
      wz = f * (pr * (double)dz.y - pi * (double)dz.x);
    }
    stc<Real>(f0, i, wx, wy);
    stc<Real>(f1, i, wz, 0.0);
  }
}

// For each pair {k, -k}: unpack w, project onto the incompressible part, keep
// shells smin..smax, add 1/2|g|^2 to J, and write back g/Ntot packed as
// F0 = g_x + i g_y, F1 = g_z (so the inverse transforms give N^-3 IFFT(g)).
template <class Real>
__global__ __launch_bounds__(256) void k_loss_spectral(void* F0, void* F1, int nx, int ny, int nz, int smin, int smax,
                                                       double* __restrict__ partial) {
  __shared__ double sh[4];
  const long n = (long)nx * ny * nz;
  const double inv = 1.0 / (double)n;
  Neu acc;
  cplx<Real>* P0 = reinterpret_cast<cplx<Real>*>(F0);
  cplx<Real>* P1 = reinterpret_cast<cplx<Real>*>(F1);
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    int ix, iy, iz;
    grid_xyz(i, nx, ny, ix, iy, iz);
    const long m = (long)mirror_of(iz, nz) * nx * ny + (long)mirror_of(iy, ny) * nx + mirror_of(ix, nx);
    if (m < i) continue;                       // the pair is handled at its smaller index
    const cplx<Real> z0 = P0[i], z0m = P0[m], z1 = P1[i], z1m = P1[m];
    const int kx = kfreq(ix, nx), ky = kfreq(iy, ny), kz = kfreq(iz, nz);
    const long k2 = (long)kx * kx + (long)ky * ky + (long)kz * kz;
    const int s = shell_of(k2);
    const bool in = (s >= smin && s <= smax);
    // w at k (normalised)
    const double wxr = 0.5 * ((double)z0.x + z0m.x) * inv, wxi = 0.5 * ((double)z0.y - z0m.y) * inv;
    const double wyr = 0.5 * ((double)z0.y + z0m.y) * inv, wyi = -0.5 * ((double)z0.x - z0m.x) * inv;
    const double wzr = 0.5 * ((double)z1.x + z1m.x) * inv, wzi = 0.5 * ((double)z1.y - z1m.y) * inv;
    double gxr = 0, gxi = 0, gyr = 0, gyi = 0, gzr = 0, gzi = 0;
    if (in) {
      double cr = 0, ci = 0;
      if (k2 > 0) {
        cr = (kx * wxr + ky * wyr + kz * wzr) / (double)k2;
        ci = (kx * wxi + ky * wyi + kz * wzi) / (double)k2;
      }
      gxr = wxr - kx * cr; gxi = wxi - kx * ci;
      gyr = wyr - ky * cr; gyi = wyi - ky * ci;
      gzr = wzr - kz * cr; gzi = wzi - kz * ci;
      const double e = 0.5 * (gxr * gxr + gxi * gxi + gyr * gyr + gyi * gyi + gzr * gzr + gzi * gzi);
      acc.add(m == i ? e : 2.0 * e);
    }
    // g(-k) = conj(g(k)) (real fields); pack: G0 = gx + i gy, G1 = gz
    P0[i] = mk(Real((gxr - gyi) * inv), Real((gxi + gyr) * inv));
    P1[i] = mk(Real(gzr * inv), Real(gzi * inv));
    if (m != i) {
      P0[m] = mk(Real((gxr + gyi) * inv), Real((-gxi + gyr) * inv));
      P1[m] = mk(Real(gzr * inv), Real(-gzi * inv));
    }
  }
  const double tot = block_sum256(acc.val(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// lam = sum_j [ -i h_j d_j - G_j w_j psi/|psi|^2 ],  h_j = 2 alpha G_j/|psi|;
// then d_j <- h_j psi (to be differentiated along j).  G0 = Gx + i Gy, G1 = Gz.
template <class Real>
__global__ __launch_bounds__(256) void k_loss_lambda1(const void* psi, void* d0, void* d1, void* d2, const void* G0,
                                                      const void* G1, void* lam, long n, double alpha) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const cplx<Real> p = ldc<Real>(psi, i);
    const double pr = p.x, pi = p.y, rho = pr * pr + pi * pi, amp = sqrt(rho);
    double lr = 0, li = 0;
    double hx = 0, hy = 0, hz = 0;
    if (amp > 0.0) {
      const cplx<Real> g0 = ldc<Real>(G0, i), g1 = ldc<Real>(G1, i);
      const double G[3] = {(double)g0.x, (double)g0.y, (double)g1.x};
      const void* dp[3] = {d0, d1, d2};
      double h[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const cplx<Real> d = ldc<Real>(dp[j], i);
        const double dr = d.x, di = d.y;
        const double w = 2.0 * alpha * (pr * di - pi * dr) / amp;
        h[j] = 2.0 * alpha * G[j] / amp;
        // -i h d = h * (di, -dr)
        lr += h[j] * di; li -= h[j] * dr;
        const double f = G[j] * w / rho;
        lr -= f * pr; li -= f * pi;
      }
      hx = h[0]; hy = h[1]; hz = h[2];
    }
    stc<Real>(lam, i, lr, li);
    stc<Real>(d0, i, hx * pr, hx * pi);
    stc<Real>(d1, i, hy * pr, hy * pi);
    stc<Real>(d2, i, hz * pr, hz * pi);
  }
}

// lam += -i (e0 + e1 + e2), e_j = d/dj (h_j psi)
template <class Real>
__global__ __launch_bounds__(256) void k_loss_lambda2(void* lam, const void* e0, const void* e1, const void* e2, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const cplx<Real> l = ldc<Real>(lam, i);
    const cplx<Real> a = ldc<Real>(e0, i), b = ldc<Real>(e1, i), c = ldc<Real>(e2, i);
    const double sr = (double)a.x + b.x + c.x, si = (double)a.y + b.y + c.y;
    stc<Real>(lam, i, (double)l.x + si, (double)l.y - sr);
  }
}

template <class Real>
__global__ void k_phase_grad(const void* psi0, const void* lam0, double* out, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const cplx<Real> p = ldc<Real>(psi0, i), l = ldc<Real>(lam0, i);
    out[i] = (double)l.y * p.x - (double)l.x * p.y;      // Im(lam conj(psi))
  }
}

// ----------------------------------------------------------------- structure function
// Per-axis power sums P_j(k) = sum over pencils |F_j(rho - 1)|^2 (natural order along
// axis j).  F holds the axis-j transform; axis j index of element i is (i / div) % nj.
__global__ __launch_bounds__(64) void k_axis_power_c128(const void* F, long n, long div, int nj, long chunk,
                                                        double* __restrict__ part);
__global__ __launch_bounds__(64) void k_axis_power_c64(const void* F, long n, long div, int nj, long chunk,
                                                       double* __restrict__ part);

template <class Real>
__device__ __forceinline__ void axis_power(const void* F, long n, long div, int nj, long chunk, double* part) {
  extern __shared__ double bins[];
  for (int i = threadIdx.x; i < nj; i += 64) bins[i] = 0.0;
  __syncthreads();
  const long i0 = (long)blockIdx.x * chunk;
  const long i1 = (i0 + chunk < n) ? i0 + chunk : n;
  for (long i = i0 + threadIdx.x; i < i1; i += 64) {
    const cplx<Real> z = ldc<Real>(F, i);
    atomicAdd(&bins[(i / div) % nj], (double)z.x * z.x + (double)z.y * z.y);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nj; i += 64) part[(long)i * gridDim.x + blockIdx.x] = bins[i];
}
__global__ __launch_bounds__(64) void k_axis_power_c128(const void* F, long n, long div, int nj, long chunk, double* part) {
  axis_power<double>(F, n, div, nj, chunk, part);
}
__global__ __launch_bounds__(64) void k_axis_power_c64(const void* F, long n, long div, int nj, long chunk, double* part) {
  axis_power<float>(F, n, div, nj, chunk, part);
}

// S(m) = (1/3) sum_j 2/(Ntot N_j) sum_k P_j(k) (1 - cos(2 pi k m / N_j)), m = 1..N/2,
// from the reduced power sums pk[axis][k].
__global__ __launch_bounds__(256) void k_structure_final(const double* __restrict__ pk, int nj, double ntot,
                                                         double* __restrict__ out) {
  for (int m = 1 + threadIdx.x; m <= nj / 2; m += 256) {
    Neu a;
    for (int ax = 0; ax < 3; ++ax)
      for (int k = 0; k < nj; ++k) {
        const long km = ((long)k * m) % nj;
        a.add(pk[ax * nj + k] * (1.0 - cospi(2.0 * (double)km / (double)nj)));
      }
    out[m - 1] = a.val() * 2.0 / (3.0 * ntot * (double)nj);
  }
}

// ----------------------------------------------------------------- velocity statistics
// Superfluid velocity v = 2 alpha Im(conj(psi) grad psi)/|psi|^2 (0 where psi = 0).
// In: d0, d1, d2 = spectral derivatives of psi along x, y, z.  Out (in place):
// d_a = v_a + 0i for the transform along axis a; partial[a][block] = sum v_a^2.
template <class Real>
__global__ __launch_bounds__(256) void k_velocity_fields(const void* psi, void* d0, void* d1, void* d2, unsigned n,
                                                         double alpha, double* __restrict__ partial) {
  __shared__ double sh[4];
  Neu acc[3];
  void* d[3] = {d0, d1, d2};
  for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
    const cplx<Real> p = ldc<Real>(psi, i);
    const double pr = p.x, pi = p.y, rho = pr * pr + pi * pi;
    const double f = rho > 0.0 ? 2.0 * alpha / rho : 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const cplx<Real> g = ldc<Real>(d[a], i);
      const double v = f * (pr * (double)g.y - pi * (double)g.x);
      stc<Real>(d[a], i, v, 0.0);
      acc[a].add(v * v);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double t = block_sum256(acc[a].val(), sh);
    if (threadIdx.x == 0) partial[(long)a * gridDim.x + blockIdx.x] = t;
  }
}

// Mach-number partials: sum |w|^2 and max |w|^2 per block, w = sqrt(rho) v.
template <class Real>
__global__ __launch_bounds__(256) void k_mach_partials(const void* psi, const void* d0, const void* d1, const void* d2,
                                                       unsigned n, double alpha, double* __restrict__ psum,
                                                       double* __restrict__ pmax) {
  __shared__ double sh[4];
  Neu acc;
  double mx = 0.0;
  for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
    const cplx<Real> p = ldc<Real>(psi, i);
    const cplx<Real> g[3] = {ldc<Real>(d0, i), ldc<Real>(d1, i), ldc<Real>(d2, i)};
    const double pr = p.x, pi = p.y, rho = pr * pr + pi * pi;
    double w2 = 0.0;
    if (rho > 0.0) {
      double im2 = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double im = pr * (double)g[a].y - pi * (double)g[a].x;
        im2 += im * im;
      }
      w2 = 4.0 * alpha * alpha * im2 / rho;
    }
    acc.add(w2);
    mx = fmax(mx, w2);
  }
  const double s = block_sum256(acc.val(), sh);
  const double m = block_max256(mx, sh);
  if (threadIdx.x == 0) { psum[blockIdx.x] = s; pmax[blockIdx.x] = m; }
}

// Per-axis structure functions S_a(m) = 2/(Ntot N) sum_k P_a(k) (1 - cos(2 pi k m / N)),
// m = 1..N/2, from the reduced power sums pk[axis][k] of v_a transformed along axis a.
__global__ __launch_bounds__(256) void k_structure_axes(const double* __restrict__ pk, int nj, double ntot,
                                                        double* __restrict__ out) {
  const int half = nj / 2;
  for (int q = threadIdx.x; q < 3 * half; q += 256) {
    const int ax = q / half, m = q % half + 1;
    Neu a;
    for (int k = 0; k < nj; ++k) {
      const long km = ((long)k * m) % nj;
      a.add(pk[ax * nj + k] * (1.0 - cospi(2.0 * (double)km / (double)nj)));
    }
    out[q] = a.val() * 2.0 / (ntot * (double)nj);
  }
}

// ----------------------------------------------------------------- helicity
// Section on helicity: H = <v . omega> (eq. helicity), H_reg = <v_reg . omega>
// (eq. Hreg), with hbar/m -> 2 alpha.  Real fields are carried two per complex
// state; every kernel is pointwise (one point per thread, 32-bit indices).

__device__ __forceinline__ void vel_at(double pr, double pi, const double* gr, const double* gi, double alpha,
                                       double* v) {
  const double rho = pr * pr + pi * pi;
  const double f = rho > 0.0 ? 2.0 * alpha / rho : 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = f * (pr * gi[a] - pi * gr[a]);
}

// S3 = v_z + i v_x, S4 = v_y + i v_x, S5 = v_z + i v_y (for d/dy, d/dz, d/dx of omega);
// partial[block] = sum |grad psi|^2
template <class Real>
__global__ __launch_bounds__(256) void k_hel_pack(const void* psi, const void* d0, const void* d1, const void* d2,
                                                  void* s3, void* s4, void* s5, unsigned n, double alpha,
                                                  double* __restrict__ partial) {
  __shared__ double sh[4];
  Neu acc;
  for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
    const cplx<Real> p = ldc<Real>(psi, i);
    const cplx<Real> g[3] = {ldc<Real>(d0, i), ldc<Real>(d1, i), ldc<Real>(d2, i)};
    const double gr[3] = {g[0].x, g[1].x, g[2].x}, gi[3] = {g[0].y, g[1].y, g[2].y};
    double v[3];
    vel_at(p.x, p.y, gr, gi, alpha, v);
    stc<Real>(s3, i, v[2], v[0]);
    stc<Real>(s4, i, v[1], v[0]);
    stc<Real>(s5, i, v[2], v[1]);
    acc.add(gr[0] * gr[0] + gi[0] * gi[0] + gr[1] * gr[1] + gi[1] * gi[1] + gr[2] * gr[2] + gi[2] * gi[2]);
  }
  const double t = block_sum256(acc.val(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// from T3 = d/dy (v_z + i v_x), T4 = d/dz (v_y + i v_x), T5 = d/dx (v_z + i v_y):
// S6 = omega_x + i omega_y, S7 = omega_z
template <class Real>
__global__ __launch_bounds__(256) void k_hel_omega(const void* t3, const void* t4, const void* t5, void* s6, void* s7,
                                                   unsigned n) {
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const cplx<Real> a = ldc<Real>(t3, i), b = ldc<Real>(t4, i), c = ldc<Real>(t5, i);
  const double ox = (double)a.x - (double)b.x;      // d_y v_z - d_z v_y
  const double oy = (double)b.y - (double)c.x;      // d_z v_x - d_x v_z
  const double oz = (double)c.y - (double)a.y;      // d_x v_y - d_y v_x
  stc<Real>(s6, i, ox, oy);
  stc<Real>(s7, i, oz, 0.0);
}

// J_i = Im(sum_j (d_i d_j psi)(d_j psi)*), accumulated from one Hessian entry H_ij:
// J[t1] += Im(conj(F1) H), and when t2 >= 0, J[t2] += Im(conj(F2) H).  J is packed as
// J0 = J_x + i J_y, J1 = J_z; `first` starts the sums from zero.
template <class Real>
__global__ __launch_bounds__(256) void k_hel_acc(const void* H, const void* F1, int t1, const void* F2, int t2,
                                                 int first, void* J0, void* J1, unsigned n) {
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  double j[3] = {0.0, 0.0, 0.0};
  if (!first) {
    const cplx<Real> a = ldc<Real>(J0, i), b = ldc<Real>(J1, i);
    j[0] = a.x; j[1] = a.y; j[2] = b.x;
  }
  const cplx<Real> h = ldc<Real>(H, i), f = ldc<Real>(F1, i);
  j[t1] += (double)f.x * (double)h.y - (double)f.y * (double)h.x;
  if (t2 >= 0) {
    const cplx<Real> g = ldc<Real>(F2, i);
    j[t2] += (double)g.x * (double)h.y - (double)g.y * (double)h.x;
  }
  stc<Real>(J0, i, j[0], j[1]);
  stc<Real>(J1, i, j[2], 0.0);
}

// v_reg = v_par W/|W|, W = 4 alpha grad(Re psi) x grad(Im psi),
// v_par = 2 alpha W.J/(|W| |grad psi|^2); v_reg = 0 where |W| = 0 or where
// |grad psi|^2 <= g2_floor = 1e-12 <|grad psi|^2> (critical points of psi, where the
// denominator vanishes; g2_sum[0] / n is the mean).
// Out: S3 = vreg_x + i vreg_y, S4 = vreg_z (S4 held J_x + i J_y: read first);
// partial[0][block] = sum v.omega, partial[1][block] = sum v_reg.omega.
template <class Real>
__global__ __launch_bounds__(256) void k_hel_vreg(const void* psi, const void* d0, const void* d1, const void* d2,
                                                  const void* j01, const void* j2, const void* w01, const void* w2,
                                                  void* s3, void* s4, unsigned n, double alpha,
                                                  const double* __restrict__ g2_sum, double* __restrict__ partial) {
  __shared__ double sh[4];
  Neu hv, hr;
  const double g2_floor = 1e-12 * g2_sum[0] / (double)n;
  for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
    const cplx<Real> p = ldc<Real>(psi, i);
    const cplx<Real> g[3] = {ldc<Real>(d0, i), ldc<Real>(d1, i), ldc<Real>(d2, i)};
    const double gr[3] = {g[0].x, g[1].x, g[2].x}, gi[3] = {g[0].y, g[1].y, g[2].y};
    double v[3];
    vel_at(p.x, p.y, gr, gi, alpha, v);
    const cplx<Real> ja = ldc<Real>(j01, i), jb = ldc<Real>(j2, i);
    const cplx<Real> oa = ldc<Real>(w01, i), ob = ldc<Real>(w2, i);
    const double J[3] = {ja.x, ja.y, jb.x}, om[3] = {oa.x, oa.y, ob.x};
    const double W[3] = {4.0 * alpha * (gr[1] * gi[2] - gr[2] * gi[1]), 4.0 * alpha * (gr[2] * gi[0] - gr[0] * gi[2]),
                         4.0 * alpha * (gr[0] * gi[1] - gr[1] * gi[0])};
    const double wn = sqrt(W[0] * W[0] + W[1] * W[1] + W[2] * W[2]);
    double g2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) g2 += gr[a] * gr[a] + gi[a] * gi[a];
    double vr[3] = {0.0, 0.0, 0.0};
    if (wn > 0.0 && g2 > g2_floor) {
      const double vpar = 2.0 * alpha * (W[0] * J[0] + W[1] * J[1] + W[2] * J[2]) / (wn * g2);
#pragma unroll
      for (int a = 0; a < 3; ++a) vr[a] = vpar * (W[a] / wn);
    }
    stc<Real>(s3, i, vr[0], vr[1]);
    stc<Real>(s4, i, vr[2], 0.0);
    hv.add(v[0] * om[0] + v[1] * om[1] + v[2] * om[2]);
    hr.add(vr[0] * om[0] + vr[1] * om[1] + vr[2] * om[2]);
  }
  const double a = block_sum256(hv.val(), sh);
  const double b = block_sum256(hr.val(), sh);
  if (threadIdx.x == 0) { partial[blockIdx.x] = a; partial[gridDim.x + blockIdx.x] = b; }
}

// in place: S0 = v_x + i v_y, S1 = v_z (from psi and its derivatives S0, S1, S2)
template <class Real>
__global__ __launch_bounds__(256) void k_hel_vpack(const void* psi, void* d0, void* d1, const void* d2, unsigned n,
                                                   double alpha) {
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const cplx<Real> p = ldc<Real>(psi, i);
  const cplx<Real> g[3] = {ldc<Real>(d0, i), ldc<Real>(d1, i), ldc<Real>(d2, i)};
  const double gr[3] = {g[0].x, g[1].x, g[2].x}, gi[3] = {g[0].y, g[1].y, g[2].y};
  double v[3];
  vel_at(p.x, p.y, gr, gi, alpha, v);
  stc<Real>(d0, i, v[0], v[1]);
  stc<Real>(d1, i, v[2], 0.0);
}

// Helicity spectra: from the unnormalised transforms of the packed real fields
// V01 = v_x + i v_y, V2 = v_z, R01, R2 (v_reg), O01, O2 (omega), per k
// Re(conj(v_k) . omega_k) and Re(conj(vreg_k) . omega_k) into shell round(|k|).
template <class Real>
__device__ __forceinline__ void unpack2(const void* F, long i, long m, double inv, double* ar, double* ai, double* br,
                                        double* bi) {
  const cplx<Real> z = ldc<Real>(F, i), zm = ldc<Real>(F, m);
  *ar = 0.5 * ((double)z.x + zm.x) * inv;  *ai = 0.5 * ((double)z.y - zm.y) * inv;
  *br = 0.5 * ((double)z.y + zm.y) * inv;  *bi = -0.5 * ((double)z.x - zm.x) * inv;
}

template <class Real>
__global__ __launch_bounds__(64) void k_hel_spectral(const void* V01, const void* V2, const void* R01, const void* R2,
                                                     const void* O01, const void* O2, int nx, int ny, int nz,
                                                     int nshell, long chunk, double* __restrict__ bins_partial) {
  extern __shared__ double bins[];            // [2][nshell]
  for (int i = threadIdx.x; i < 2 * nshell; i += 64) bins[i] = 0.0;
  __syncthreads();
  const long n = (long)nx * ny * nz;
  const double inv = 1.0 / (double)n;
  const long i0 = (long)blockIdx.x * chunk;
  const long i1 = (i0 + chunk < n) ? i0 + chunk : n;
  for (long i = i0 + threadIdx.x; i < i1; i += 64) {
    int ix, iy, iz;
    grid_xyz(i, nx, ny, ix, iy, iz);
    const long m = (long)mirror_of(iz, nz) * nx * ny + (long)mirror_of(iy, ny) * nx + mirror_of(ix, nx);
    double v[6], r[6], o[6], t0, t1;     // [x re, x im, y re, y im, z re, z im]
    unpack2<Real>(V01, i, m, inv, &v[0], &v[1], &v[2], &v[3]);
    unpack2<Real>(V2, i, m, inv, &v[4], &v[5], &t0, &t1);
    unpack2<Real>(R01, i, m, inv, &r[0], &r[1], &r[2], &r[3]);
    unpack2<Real>(R2, i, m, inv, &r[4], &r[5], &t0, &t1);
    unpack2<Real>(O01, i, m, inv, &o[0], &o[1], &o[2], &o[3]);
    unpack2<Real>(O2, i, m, inv, &o[4], &o[5], &t0, &t1);
    double hv = 0.0, hr = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      hv += v[2 * a] * o[2 * a] + v[2 * a + 1] * o[2 * a + 1];
      hr += r[2 * a] * o[2 * a] + r[2 * a + 1] * o[2 * a + 1];
    }
    const int kx = kfreq(ix, nx), ky = kfreq(iy, ny), kz = kfreq(iz, nz);
    const int s = shell_of((long)kx * kx + (long)ky * ky + (long)kz * kz);
    atomicAdd(&bins[s], hv);
    atomicAdd(&bins[nshell + s], hr);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * nshell; i += 64) bins_partial[(long)i * gridDim.x + blockIdx.x] = bins[i];
}

// every point <- (re, im)
template <class Real>
__global__ __launch_bounds__(256) void k_fill(void* f, unsigned n, double re, double im) {
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) stc<Real>(f, i, re, im);
}

// plain stream copy, one 16-byte unit per lane (the bandwidth reference of the passes);
// an odd 8-byte tail goes with the first lane
__global__ __launch_bounds__(256) void k_copy16(const void* __restrict__ src, void* __restrict__ dst, long units,
                                                int tail8) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < units) ((f4*)dst)[i] = ((const f4*)src)[i];
  if (tail8 && i == 0) ((double*)dst)[2 * units] = ((const double*)src)[2 * units];
}

// ----------------------------------------------------------------- launch wrappers
static unsigned grid_for(long n, int threads, unsigned cap = 4096) {
  long g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

void launch_init_phase(int prec, const double* theta, void* psi, long n, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_init_phase<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, theta, psi, n);
  else hipLaunchKernelGGL(k_init_phase<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, theta, psi, n);
}
void launch_nonlinear(int prec, void* psi, long n, double coef, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_nonlinear<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, psi, n, coef);
  else hipLaunchKernelGGL(k_nonlinear<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, psi, n, coef);
}
void launch_scale_copy(int prec, const void* in, void* out, long n, double scale, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_scale_copy<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, in, out, n, scale);
  else hipLaunchKernelGGL(k_scale_copy<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, in, out, n, scale);
}
void launch_mult3(int prec, void* f, int nx, int ny, int nz, const void* mx, const void* my, const void* mz, hipStream_t st) {
  const long n = (long)nx * ny * nz;
  if (prec == P_C128) hipLaunchKernelGGL(k_mult3<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, f, nx, ny, nz, mx, my, mz);
  else hipLaunchKernelGGL(k_mult3<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, f, nx, ny, nz, mx, my, mz);
}
void launch_diag_fields(int prec, const void* psi, void* f0, void* f1, void* f2, void* f3, long n, double alpha,
                        double* partial, unsigned blocks, hipStream_t st) {
  if (prec == P_C128)
    hipLaunchKernelGGL(k_diag_fields<double>, dim3(blocks), dim3(256), 0, st, psi, f0, f1, f2, f3, n, alpha, partial);
  else
    hipLaunchKernelGGL(k_diag_fields<float>, dim3(blocks), dim3(256), 0, st, psi, f0, f1, f2, f3, n, alpha, partial);
}
void launch_spectral(int prec, const void* F0, const void* F1, const void* F2, const void* F3, int nx, int ny, int nz,
                     double alpha, double beta, int nshell, unsigned blocks, double* bins, hipStream_t st) {
  const size_t sh = sizeof(double) * 4 * (size_t)nshell;
  // the kernel visits the planes iz = 0 .. nz/2 only (mirror pairs), in `blocks` chunks
  const long nh = (long)(nz / 2 + 1) * nx * ny;
  const long chunk = (nh + blocks - 1) / blocks;
  if (prec == P_C128)
    hipLaunchKernelGGL(k_spectral<double>, dim3(blocks), dim3(64), sh, st, F0, F1, F2, F3, nx, ny, nz, alpha, beta,
                       nshell, chunk, bins);
  else
    hipLaunchKernelGGL(k_spectral<float>, dim3(blocks), dim3(64), sh, st, F0, F1, F2, F3, nx, ny, nz, alpha, beta,
                       nshell, chunk, bins);
}
void launch_sup_diff2(int prec, const void* a, const void* b, long n, double* partial, unsigned blocks, double* out,
                      hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_sup_diff2<double>, dim3(blocks), dim3(256), 0, st, a, b, n, partial);
  else hipLaunchKernelGGL(k_sup_diff2<float>, dim3(blocks), dim3(256), 0, st, a, b, n, partial);
  hipLaunchKernelGGL(k_segmax, dim3(1), dim3(256), 0, st, partial, (long)blocks, out);
}
void launch_segsum(const double* in, long len, int nseg, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_segsum, dim3(nseg), dim3(256), 0, st, in, len, out);
}
void launch_finalize_diag(const double* red, double w0, double w1, double w2, int nshell, double alpha, double beta,
                          double ntot, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_diag, dim3(1), dim3(256), 0, st, red, w0, w1, w2, nshell, alpha, beta, ntot, out);
}
void launch_loss_fields(int prec, const void* psi, const void* d0, const void* d1, const void* d2, void* f0, void* f1,
                        long n, double alpha, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_loss_fields<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, psi, d0, d1, d2, f0, f1, n, alpha);
  else hipLaunchKernelGGL(k_loss_fields<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, psi, d0, d1, d2, f0, f1, n, alpha);
}
void launch_loss_spectral(int prec, void* F0, void* F1, int nx, int ny, int nz, int smin, int smax, double* partial,
                          unsigned blocks, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_loss_spectral<double>, dim3(blocks), dim3(256), 0, st, F0, F1, nx, ny, nz, smin, smax, partial);
  else hipLaunchKernelGGL(k_loss_spectral<float>, dim3(blocks), dim3(256), 0, st, F0, F1, nx, ny, nz, smin, smax, partial);
}
void launch_loss_lambda1(int prec, const void* psi, void* d0, void* d1, void* d2, const void* G0, const void* G1,
                         void* lam, long n, double alpha, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_loss_lambda1<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, psi, d0, d1, d2, G0, G1, lam, n, alpha);
  else hipLaunchKernelGGL(k_loss_lambda1<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, psi, d0, d1, d2, G0, G1, lam, n, alpha);
}
void launch_loss_lambda2(int prec, void* lam, const void* e0, const void* e1, const void* e2, long n, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_loss_lambda2<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, lam, e0, e1, e2, n);
  else hipLaunchKernelGGL(k_loss_lambda2<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, lam, e0, e1, e2, n);
}
void launch_argle_explicit(int prec, const void* phi, const void* dx, const void* dy, const void* dz, const void* v,
                           void* out, long n, double alpha, double beta, hipStream_t st) {
  const unsigned blocks = (unsigned)((n + 255) / 256), un = (unsigned)n;
  const double q4a = 1.0 / (4.0 * alpha);
  if (prec == P_C128)
    hipLaunchKernelGGL(k_argle_explicit<double>, dim3(blocks), dim3(256), 0, st, phi, dx, dy, dz, v, out, un, q4a, beta);
  else
    hipLaunchKernelGGL(k_argle_explicit<float>, dim3(blocks), dim3(256), 0, st, phi, dx, dy, dz, v, out, un, q4a, beta);
}
void launch_argle_solve(int prec, void* P, const void* Q, int nx, int ny, int nz, double a, double dtau, double inv_n,
                        hipStream_t st) {
  const dim3 grid((unsigned)(ny * nz), (unsigned)((nx + 255) / 256));
  if (prec == P_C128)
    hipLaunchKernelGGL(k_argle_solve<double>, grid, dim3(256), 0, st, P, Q, nx, ny, nz, a, dtau, inv_n);
  else
    hipLaunchKernelGGL(k_argle_solve<float>, grid, dim3(256), 0, st, P, Q, nx, ny, nz, a, dtau, inv_n);
}
void launch_argle_energy(int prec, const void* phi, const void* dx, const void* dy, const void* dz, const void* v,
                         long n, double alpha, double beta, double* partial, unsigned blocks, hipStream_t st) {
  if (prec == P_C128)
    hipLaunchKernelGGL(k_argle_energy<double>, dim3(blocks), dim3(256), 0, st, phi, dx, dy, dz, v, n, alpha, beta, partial);
  else
    hipLaunchKernelGGL(k_argle_energy<float>, dim3(blocks), dim3(256), 0, st, phi, dx, dy, dz, v, n, alpha, beta, partial);
}
void launch_phase_grad(int prec, const void* psi0, const void* lam0, double* out, long n, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_phase_grad<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, psi0, lam0, out, n);
  else hipLaunchKernelGGL(k_phase_grad<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, psi0, lam0, out, n);
}
void launch_axis_power(int prec, const void* F, long n, long div, int nj, unsigned blocks, long chunk, double* part,
                       hipStream_t st) {
  const size_t sh = sizeof(double) * (size_t)nj;
  if (prec == P_C128) hipLaunchKernelGGL(k_axis_power_c128, dim3(blocks), dim3(64), sh, st, F, n, div, nj, chunk, part);
  else hipLaunchKernelGGL(k_axis_power_c64, dim3(blocks), dim3(64), sh, st, F, n, div, nj, chunk, part);
}
void launch_velocity_fields(int prec, const void* psi, void* d0, void* d1, void* d2, long n, double alpha,
                            double* partial, unsigned blocks, hipStream_t st) {
  if (prec == P_C128)
    hipLaunchKernelGGL(k_velocity_fields<double>, dim3(blocks), dim3(256), 0, st, psi, d0, d1, d2, (unsigned)n, alpha, partial);
  else
    hipLaunchKernelGGL(k_velocity_fields<float>, dim3(blocks), dim3(256), 0, st, psi, d0, d1, d2, (unsigned)n, alpha, partial);
}
void launch_mach_partials(int prec, const void* psi, const void* d0, const void* d1, const void* d2, long n,
                          double alpha, double* psum, double* pmax, unsigned blocks, hipStream_t st) {
  if (prec == P_C128)
    hipLaunchKernelGGL(k_mach_partials<double>, dim3(blocks), dim3(256), 0, st, psi, d0, d1, d2, (unsigned)n, alpha, psum, pmax);
  else
    hipLaunchKernelGGL(k_mach_partials<float>, dim3(blocks), dim3(256), 0, st, psi, d0, d1, d2, (unsigned)n, alpha, psum, pmax);
}
#define GPK_PREC_LAUNCH(K, GRID, BLOCK, SH, ST, ...)                                   \
  do {                                                                                 \
    if (prec == P_C128) hipLaunchKernelGGL(K<double>, GRID, BLOCK, SH, ST, __VA_ARGS__); \
    else hipLaunchKernelGGL(K<float>, GRID, BLOCK, SH, ST, __VA_ARGS__);               \
  } while (0)
void launch_hel_pack(int prec, const void* psi, const void* d0, const void* d1, const void* d2, void* s3, void* s4,
                     void* s5, long n, double alpha, double* partial, unsigned blocks, hipStream_t st) {
  GPK_PREC_LAUNCH(k_hel_pack, dim3(blocks), dim3(256), 0, st, psi, d0, d1, d2, s3, s4, s5, (unsigned)n, alpha,
                  partial);
}
void launch_hel_omega(int prec, const void* t3, const void* t4, const void* t5, void* s6, void* s7, long n,
                      hipStream_t st) {
  GPK_PREC_LAUNCH(k_hel_omega, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, t3, t4, t5, s6, s7, (unsigned)n);
}
void launch_hel_acc(int prec, const void* H, const void* F1, int t1, const void* F2, int t2, int first, void* J0,
                    void* J1, long n, hipStream_t st) {
  GPK_PREC_LAUNCH(k_hel_acc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, H, F1, t1, F2, t2, first, J0, J1,
                  (unsigned)n);
}
void launch_hel_vreg(int prec, const void* psi, const void* d0, const void* d1, const void* d2, const void* j01,
                     const void* j2, const void* w01, const void* w2, void* s3, void* s4, long n, double alpha,
                     const double* g2_sum, double* partial, unsigned blocks, hipStream_t st) {
  GPK_PREC_LAUNCH(k_hel_vreg, dim3(blocks), dim3(256), 0, st, psi, d0, d1, d2, j01, j2, w01, w2, s3, s4,
                  (unsigned)n, alpha, g2_sum, partial);
}
void launch_hel_vpack(int prec, const void* psi, void* d0, void* d1, const void* d2, long n, double alpha,
                      hipStream_t st) {
  GPK_PREC_LAUNCH(k_hel_vpack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, psi, d0, d1, d2, (unsigned)n,
                  alpha);
}
void launch_hel_spectral(int prec, const void* V01, const void* V2, const void* R01, const void* R2, const void* O01,
                         const void* O2, int nx, int ny, int nz, int nshell, unsigned blocks, long chunk,
                         double* bins, hipStream_t st) {
  const size_t sh = sizeof(double) * 2 * (size_t)nshell;
  GPK_PREC_LAUNCH(k_hel_spectral, dim3(blocks), dim3(64), sh, st, V01, V2, R01, R2, O01, O2, nx, ny, nz, nshell,
                  chunk, bins);
}
#undef GPK_PREC_LAUNCH
void launch_fill(int prec, void* f, long n, double re, double im, hipStream_t st) {
  if (prec == P_C128) hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, f, (unsigned)n, re, im);
  else hipLaunchKernelGGL(k_fill<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, f, (unsigned)n, re, im);
}
void launch_copy16(const void* src, void* dst, long bytes, hipStream_t st) {
  const long units = bytes / 16;
  const unsigned grid = (unsigned)std::max(1L, (units + 255) / 256);
  hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, st, src, dst, units, (int)((bytes % 16) != 0));
}
void launch_segmax(const double* in, long len, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_segmax, dim3(1), dim3(256), 0, st, in, len, out);
}
void launch_structure_axes(const double* pk, int nj, double ntot, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_structure_axes, dim3(1), dim3(256), 0, st, pk, nj, ntot, out);
}
void launch_structure_final(const double* pk, int nj, double ntot, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_structure_final, dim3(1), dim3(256), 0, st, pk, nj, ntot, out);
}

// ----------------------------------------------------------------- random vortex rings
// Initial condition of the random-vortex-ring construction (RVR section): product over
// pairs of the periodised ring-pair ansatz, evaluated at translated, axis-permuted
// coordinates.
struct RingPar { double R, d, X, Y, Z; int perm; };

__device__ __forceinline__ void ring_eval(double x, double y, double z, double R, double xi, double pa1, double pa2,
                                          double pb1, double* re, double* im) {
  const double pi = 3.141592653589793238462643383279502884;
  const double xt = x - pi, yt = y - pi, zt = z - pi;
  const double dr = sqrt(xt * xt + yt * yt) - R;
  const double dist = sqrt(dr * dr + zt * zt);
  if (dist == 0.0) { *re = 0.0; *im = 0.0; return; }
  const double e2 = (dist / xi) * (dist / xi), e4 = e2 * e2;
  const double f = sqrt((pa1 * e2 + pa2 * e4) / (1.0 + pb1 * e2 + pa2 * e4));
  // f exp(i atan2(zt, dr)) = f (dr + i zt) / dist
  *re = f * dr / dist;
  *im = f * zt / dist;
}

// pair ring(z - d/2) * conj(ring(z + d/2))
__device__ __forceinline__ void pair_eval(double x, double y, double z, double R, double d, double xi, double a1,
                                          double a2, double b1, double* re, double* im) {
  double ar, ai, br, bi;
  ring_eval(x, y, z - 0.5 * d, R, xi, a1, a2, b1, &ar, &ai);
  ring_eval(x, y, z + 0.5 * d, R, xi, a1, a2, b1, &br, &bi);
  *re = ar * br + ai * bi;
  *im = ai * br - ar * bi;
}

template <class Real>
__global__ __launch_bounds__(256) void k_init_rvr(const RingPar* __restrict__ pairs, int npairs, double xi, double a1,
                                                  double a2, double b1, int nx, int ny, int nz, void* psi) {
  const double two_pi = 6.283185307179586476925286766559;
  const long n = (long)nx * ny * nz;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    grid_xyz(i, nx, ny, ix, iy, iz);
    const double c[3] = {two_pi * ix / nx, two_pi * iy / ny, two_pi * iz / nz};
    double pr = 1.0, pim = 0.0;
    for (int q = 0; q < npairs; ++q) {
      const RingPar P = pairs[q];
      // permuted coordinates (x, y, z) -> (c[o0], c[o1], c[o2])
      int o0, o1, o2;
      switch (P.perm) {
        case 0: o0 = 0; o1 = 1; o2 = 2; break;
        case 1: o0 = 0; o1 = 2; o2 = 1; break;
        case 2: o0 = 1; o1 = 0; o2 = 2; break;
        case 3: o0 = 1; o1 = 2; o2 = 0; break;
        case 4: o0 = 2; o1 = 0; o2 = 1; break;
        default: o0 = 2; o1 = 1; o2 = 0; break;
      }
      double sx = fmod(c[o0] - P.X, two_pi), sy = fmod(c[o1] - P.Y, two_pi), sz = fmod(c[o2] - P.Z, two_pi);
      if (sx < 0) sx += two_pi;
      if (sy < 0) sy += two_pi;
      if (sz < 0) sz += two_pi;
      // periodised pair: the pair times the conjugates of its six mirror images
      double tr, ti;
      pair_eval(sx, sy, sz, P.R, P.d, xi, a1, a2, b1, &tr, &ti);
      const double L2 = 2.0 * two_pi;
      const double img[6][3] = {{L2 - sx, sy, sz}, {-sx, sy, sz}, {sx, L2 - sy, sz},
                                {sx, -sy, sz},     {sx, sy, L2 - sz}, {sx, sy, -sz}};
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        double ur, ui;
        pair_eval(img[m][0], img[m][1], img[m][2], P.R, P.d, xi, a1, a2, b1, &ur, &ui);
        const double nr = tr * ur + ti * ui, ni = ti * ur - tr * ui;     // t * conj(u)
        tr = nr; ti = ni;
      }
      const double nr = pr * tr - pim * ti, ni = pr * ti + pim * tr;
      pr = nr; pim = ni;
    }
    stc<Real>(psi, i, pr, pim);
  }
}

void launch_init_rvr(int prec, const void* pairs, int npairs, double xi, double a1, double a2, double b1, int nx,
                     int ny, int nz, void* psi, hipStream_t st) {
  const long n = (long)nx * ny * nz;
  const RingPar* pp = reinterpret_cast<const RingPar*>(pairs);
  if (prec == P_C128)
    hipLaunchKernelGGL(k_init_rvr<double>, dim3(grid_for(n, 256, 1u << 20)), dim3(256), 0, st, pp, npairs, xi, a1, a2, b1, nx, ny, nz, psi);
  else
    hipLaunchKernelGGL(k_init_rvr<float>, dim3(grid_for(n, 256, 1u << 20)), dim3(256), 0, st, pp, npairs, xi, a1, a2, b1, nx, ny, nz, psi);
}
size_t ringpar_bytes() { return sizeof(RingPar); }

}  // namespace gpk
