// Layout-rotating pass schedules (cubic grids).  Rows are written W points wide:
// W * S >= 64 bytes; W = 8 keeps two workgroups per compute unit at 1024 points
// (W = 16, full 128-byte rows but one workgroup per compute unit, measured 25.6 ms
// per 1024^3 complex64 step against 18.1 ms).
#include "gp_registry.h"

GPK_ROT(double, gpk::P_C128, 16, 4, 16, 4, 4, 1)
GPK_ROT(double, gpk::P_C128, 32, 4, 16, 8, 4, 1)
GPK_ROT(double, gpk::P_C128, 48, 4, 16, 12, 4, 1)
GPK_ROT(double, gpk::P_C128, 64, 8, 8, 8, 8, 1)
GPK_ROT(double, gpk::P_C128, 256, 16, 8, 16, 16, 1)
GPK_ROT(double, gpk::P_C128, 512, 32, 8, 8, 8, 8)
GPK_ROT(float, gpk::P_C64, 16, 4, 16, 4, 4, 1)
GPK_ROT(float, gpk::P_C64, 32, 4, 16, 8, 4, 1)
GPK_ROT(float, gpk::P_C64, 48, 4, 16, 12, 4, 1)
GPK_ROT(float, gpk::P_C64, 64, 4, 16, 16, 4, 1)
GPK_ROT(float, gpk::P_C64, 256, 16, 16, 16, 16, 1)
GPK_ROT(float, gpk::P_C64, 512, 16, 16, 32, 16, 1)
GPK_ROT(float, gpk::P_C64, 1024, 32, 8, 32, 32, 1)
