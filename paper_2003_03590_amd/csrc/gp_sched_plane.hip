// xy-plane schedules (lengths whose N x N plane fits in LDS beside the exchange
// layouts: complex64 up to 96, complex128 up to 64).  W = N; T * N threads.
// Chosen by timing against each other (more threads per plane paid at 32 and 64).
#include "gp_registry.h"

GPK_PLANE(float, gpk::P_C64, 16, 4, 4, 4, 1)
GPK_PLANE(float, gpk::P_C64, 32, 4, 8, 4, 1)
GPK_PLANE(float, gpk::P_C64, 48, 4, 12, 4, 1)
GPK_PLANE(float, gpk::P_C64, 64, 8, 8, 8, 1)
GPK_PLANE(float, gpk::P_C64, 96, 8, 6, 4, 4)
GPK_PLANE(double, gpk::P_C128, 16, 4, 4, 4, 1)
GPK_PLANE(double, gpk::P_C128, 32, 4, 8, 4, 1)
GPK_PLANE(double, gpk::P_C128, 48, 4, 12, 4, 1)
GPK_PLANE(double, gpk::P_C128, 64, 8, 8, 8, 1)
