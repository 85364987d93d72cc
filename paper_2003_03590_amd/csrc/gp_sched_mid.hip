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

// alternative schedules (autotuner variants)
GPK_SCHED(float, gpk::P_C64, 1, 64, 8, 16, 8, 8, 1)
GPK_SCHED(float, gpk::P_C64, 2, 64, 1, 64, 64, 1, 1)
GPK_SCHED(float, gpk::P_C64, 1, 96, 4, 16, 24, 4, 1)
GPK_SCHED(float, gpk::P_C64, 2, 96, 2, 32, 16, 6, 1)
GPK_SCHED(double, gpk::P_C128, 1, 64, 4, 16, 16, 4, 1)
GPK_SCHED(double, gpk::P_C128, 1, 96, 4, 16, 24, 4, 1)
GPK_SCHED(double, gpk::P_C128, 1, 128, 8, 8, 8, 16, 1)
GPK_SCHED(double, gpk::P_C128, 2, 128, 8, 16, 16, 8, 1)
GPK_SCHED(float, gpk::P_C64, 1, 128, 8, 8, 16, 8, 1)
GPK_SCHED(float, gpk::P_C64, 2, 128, 4, 16, 32, 4, 1)
