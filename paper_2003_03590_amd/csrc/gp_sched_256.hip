// Axis-pass schedules for 256 points.
#include "gp_registry.h"

GPK_SCHED(double, gpk::P_C128, 0, 256, 16, 8, 16, 16, 1)
GPK_SCHED(float, gpk::P_C64, 0, 256, 16, 16, 16, 16, 1)
