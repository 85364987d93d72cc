// Axis-pass schedules for short axes (2 .. 48 points).
#include "gp_registry.h"

// c128
GPK_SCHED(double, gpk::P_C128, 0, 2, 1, 64, 2, 1, 1)
GPK_SCHED(double, gpk::P_C128, 0, 3, 1, 64, 3, 1, 1)
GPK_SCHED(double, gpk::P_C128, 0, 4, 1, 64, 4, 1, 1)
GPK_SCHED(double, gpk::P_C128, 0, 6, 1, 64, 6, 1, 1)
GPK_SCHED(double, gpk::P_C128, 0, 8, 1, 64, 8, 1, 1)
GPK_SCHED(double, gpk::P_C128, 0, 12, 1, 64, 12, 1, 1)
GPK_SCHED(double, gpk::P_C128, 0, 16, 1, 64, 16, 1, 1)
GPK_SCHED(double, gpk::P_C128, 0, 24, 2, 32, 12, 2, 1)
GPK_SCHED(double, gpk::P_C128, 0, 32, 4, 16, 8, 4, 1)
GPK_SCHED(double, gpk::P_C128, 0, 48, 4, 16, 12, 4, 1)
// c64
GPK_SCHED(float, gpk::P_C64, 0, 2, 1, 64, 2, 1, 1)
GPK_SCHED(float, gpk::P_C64, 0, 3, 1, 64, 3, 1, 1)
GPK_SCHED(float, gpk::P_C64, 0, 4, 1, 64, 4, 1, 1)
GPK_SCHED(float, gpk::P_C64, 0, 6, 1, 64, 6, 1, 1)
GPK_SCHED(float, gpk::P_C64, 0, 8, 1, 64, 8, 1, 1)
GPK_SCHED(float, gpk::P_C64, 0, 12, 1, 64, 12, 1, 1)
GPK_SCHED(float, gpk::P_C64, 0, 16, 1, 64, 16, 1, 1)
GPK_SCHED(float, gpk::P_C64, 0, 24, 1, 64, 24, 1, 1)
GPK_SCHED(float, gpk::P_C64, 0, 32, 2, 32, 16, 2, 1)
GPK_SCHED(float, gpk::P_C64, 0, 48, 2, 32, 24, 2, 1)
