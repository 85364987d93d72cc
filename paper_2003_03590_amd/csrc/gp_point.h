// Launch wrappers of the pointwise and reduction kernels (gp_point.hip).
#pragma once

#include "gp_registry.h"

namespace gpk {

void launch_init_phase(int prec, const double* theta, void* psi, long n, hipStream_t st);
void launch_nonlinear(int prec, void* psi, long n, double coef, hipStream_t st);
void launch_scale_copy(int prec, const void* in, void* out, long n, double scale, hipStream_t st);
void launch_mult3(int prec, void* f, int nx, int ny, int nz, const void* mx, const void* my, const void* mz,
                  hipStream_t st);
void launch_diag_fields(int prec, const void* psi, void* f0, void* f1, void* f2, void* f3, long n, double alpha,
                        double* partial, unsigned blocks, hipStream_t st);
void launch_spectral(int prec, const void* F0, const void* F1, const void* F2, const void* F3, int nx, int ny, int nz,
                     double alpha, double beta, int nshell, unsigned blocks, double* bins, hipStream_t st);
// out[0] = max over the field of |a - b|^2 (partial: blocks doubles)
void launch_sup_diff2(int prec, const void* a, const void* b, long n, double* partial, unsigned blocks, double* out,
                      hipStream_t st);
// in place: d_a <- v_a + 0i (superfluid velocity); partial[3][blocks] = sum v_a^2
void launch_velocity_fields(int prec, const void* psi, void* d0, void* d1, void* d2, long n, double alpha,
                            double* partial, unsigned blocks, hipStream_t st);
// psum, pmax: `blocks` doubles each (sum and max of |w|^2 per block)
void launch_mach_partials(int prec, const void* psi, const void* d0, const void* d1, const void* d2, long n,
                          double alpha, double* psum, double* pmax, unsigned blocks, hipStream_t st);
void launch_segmax(const double* in, long len, double* out, hipStream_t st);
// every point of f <- re + i im
void launch_fill(int prec, void* f, long n, double re, double im, hipStream_t st);
void launch_copy16(const void* src, void* dst, long bytes, hipStream_t st);   // bytes: a multiple of 8
// helicity stages (see the kernels for the packing of real fields into states)
// partial: blocks doubles (sum |grad psi|^2)
void launch_hel_pack(int prec, const void* psi, const void* d0, const void* d1, const void* d2, void* s3, void* s4,
                     void* s5, long n, double alpha, double* partial, unsigned blocks, hipStream_t st);
void launch_hel_omega(int prec, const void* t3, const void* t4, const void* t5, void* s6, void* s7, long n,
                      hipStream_t st);
void launch_hel_acc(int prec, const void* H, const void* F1, int t1, const void* F2, int t2, int first, void* J0,
                    void* J1, long n, hipStream_t st);
// g2_sum: device, one double (sum |grad psi|^2); partial: 2 * blocks doubles
void launch_hel_vreg(int prec, const void* psi, const void* d0, const void* d1, const void* d2, const void* j01,
                     const void* j2, const void* w01, const void* w2, void* s3, void* s4, long n, double alpha,
                     const double* g2_sum, double* partial, unsigned blocks, hipStream_t st);
void launch_hel_vpack(int prec, const void* psi, void* d0, void* d1, const void* d2, long n, double alpha,
                      hipStream_t st);
// bins: blocks * 2 * nshell doubles
void launch_hel_spectral(int prec, const void* V01, const void* V2, const void* R01, const void* R2, const void* O01,
                         const void* O2, int nx, int ny, int nz, int nshell, unsigned blocks, long chunk,
                         double* bins, hipStream_t st);
// out[3][nj/2] per-axis structure functions from pk[3][nj]
void launch_structure_axes(const double* pk, int nj, double ntot, double* out, hipStream_t st);
void launch_segsum(const double* in, long len, int nseg, double* out, hipStream_t st);
void launch_finalize_diag(const double* red, double w0, double w1, double w2, int nshell, double alpha, double beta,
                          double ntot, double* out, hipStream_t st);
void launch_loss_fields(int prec, const void* psi, const void* d0, const void* d1, const void* d2, void* f0,
                        void* f1, long n, double alpha, hipStream_t st);
void launch_loss_spectral(int prec, void* F0, void* F1, int nx, int ny, int nz, int smin, int smax,
                          double* partial, unsigned blocks, hipStream_t st);
void launch_loss_lambda1(int prec, const void* psi, void* d0, void* d1, void* d2, const void* G0, const void* G1,
                         void* lam, long n, double alpha, hipStream_t st);
void launch_loss_lambda2(int prec, void* lam, const void* e0, const void* e1, const void* e2, long n,
                         hipStream_t st);
void launch_phase_grad(int prec, const void* psi0, const void* lam0, double* out, long n, hipStream_t st);
void launch_argle_explicit(int prec, const void* phi, const void* dx, const void* dy, const void* dz, const void* v,
                           void* out, long n, double alpha, double beta, hipStream_t st);
void launch_argle_solve(int prec, void* P, const void* Q, int nx, int ny, int nz, double a, double dtau, double inv_n,
                        hipStream_t st);
void launch_argle_energy(int prec, const void* phi, const void* dx, const void* dy, const void* dz, const void* v,
                         long n, double alpha, double beta, double* partial, unsigned blocks, hipStream_t st);
void launch_axis_power(int prec, const void* F, long n, long div, int nj, unsigned blocks, long chunk,
                       double* part, hipStream_t st);
void launch_init_rvr(int prec, const void* pairs, int npairs, double xi, double a1, double a2, double b1, int nx,
                     int ny, int nz, void* psi, hipStream_t st);
size_t ringpar_bytes();
void launch_structure_final(const double* pk, int nj, double ntot, double* out, hipStream_t st);

}  // namespace gpk
