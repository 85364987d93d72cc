// Further axis-pass schedule variants (autotuner alternatives): 1024 points in
// complex64 with four pencils per workgroup, so that five workgroups (ten
// wavefronts) fit the LDS of a compute unit instead of two.
#include "gp_registry.h"

GPK_SCHED(float, gpk::P_C64, 4, 1024, 32, 4, 32, 32, 1)
