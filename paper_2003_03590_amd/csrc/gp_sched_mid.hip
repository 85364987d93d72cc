// Axis-pass schedules for 64 .. 192 points.
#include "gp_registry.h"

GPK_SCHED(double, gpk::P_C128, 0, 64, 8, 8, 8, 8, 1)
GPK_SCHED(double, gpk::P_C128, 0, 96, 4, 16, 12, 8, 1)
GPK_SCHED(double, gpk::P_C128, 0, 128, 8, 8, 16, 8, 1)
GPK_SCHED(double, gpk::P_C128, 0, 192, 8, 8, 24, 8, 1)
GPK_SCHED(float, gpk::P_C64, 0, 64, 4, 16, 16, 4, 1)
GPK_SCHED(float, gpk::P_C64, 0, 96, 4, 16, 12, 8, 1)
GPK_SCHED(float, gpk::P_C64, 0, 128, 8, 16, 16, 8, 1)
GPK_SCHED(float, gpk::P_C64, 0, 192, 8, 16, 24, 8, 1)
