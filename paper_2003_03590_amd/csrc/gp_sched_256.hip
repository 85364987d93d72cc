// Axis-pass schedules for 256 points.
#include "gp_registry.h"

GPK_SCHED(double, gpk::P_C128, 0, 256, 16, 8, 16, 16, 1)
GPK_SCHED(float, gpk::P_C64, 0, 256, 16, 16, 16, 16, 1)

// alternative schedules (autotuner variants)
GPK_SCHED(double, gpk::P_C128, 1, 256, 16, 4, 16, 16, 1)
GPK_SCHED(double, gpk::P_C128, 2, 256, 16, 16, 16, 16, 1)
GPK_SCHED(double, gpk::P_C128, 3, 256, 32, 4, 8, 8, 4)
GPK_SCHED(float, gpk::P_C64, 1, 256, 16, 8, 16, 16, 1)
GPK_SCHED(float, gpk::P_C64, 2, 256, 8, 16, 32, 8, 1)
GPK_SCHED(float, gpk::P_C64, 3, 256, 16, 32, 16, 16, 1)
