// Axis-pass schedule variants for 1024 points (autotuner alternatives).
#include "gp_registry.h"

GPK_SCHED(float, gpk::P_C64, 1, 1024, 32, 16, 32, 32, 1)
GPK_SCHED(float, gpk::P_C64, 2, 1024, 64, 4, 16, 16, 4)
GPK_SCHED(float, gpk::P_C64, 3, 1024, 16, 8, 32, 32, 1)
GPK_SCHED(float, gpk::P_C64, 1, 512, 16, 8, 16, 32, 1)
GPK_SCHED(float, gpk::P_C64, 2, 512, 16, 8, 32, 16, 1)
GPK_SCHED(double, gpk::P_C128, 1, 512, 16, 8, 32, 16, 1)
