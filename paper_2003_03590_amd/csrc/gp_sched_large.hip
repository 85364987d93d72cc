// Axis-pass schedules for 384 .. 1024 points.
#include "gp_registry.h"

GPK_SCHED(double, gpk::P_C128, 0, 384, 16, 8, 8, 8, 6)
GPK_SCHED(double, gpk::P_C128, 0, 512, 32, 8, 8, 8, 8)
GPK_SCHED(double, gpk::P_C128, 0, 768, 32, 4, 8, 8, 12)
GPK_SCHED(double, gpk::P_C128, 0, 1024, 64, 4, 16, 16, 4)
GPK_SCHED(float, gpk::P_C64, 0, 384, 16, 16, 8, 8, 6)
GPK_SCHED(float, gpk::P_C64, 0, 512, 16, 16, 32, 16, 1)
GPK_SCHED(float, gpk::P_C64, 0, 768, 32, 8, 8, 8, 12)
GPK_SCHED(float, gpk::P_C64, 0, 1024, 32, 8, 32, 32, 1)
