// The remeshing stage's mesh-to-volume step (Sec. 4.1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

#include "internal.hpp"

namespace pamo {

// Narrow-band unsigned distance field of the soup (V, F: nf triangles, device)
// at the voxel centres ((i + 1/2) / res, ...) of a res^3 grid, udf[(i res + j)
// res + k]: the smallest point-triangle distance when it is at most band,
// else +inf.  read_total synchronises, reads the 64-bit pair count from the
// device, checks the error bits (err: PAMO_EBIT_TILES when a triangle's
// banded box covers too many tiles) and that the count fits int32.
void udf_run(Workspace& ws, hipStream_t s, const double* V, const int* F, int nf, int res, double band, double* udf,
             int* err, const std::function<int64_t(const unsigned long long*)>& read_total);

// Dual Marching Cubes (Sec. 4.2) on the res^3 grid S (device float64, value
// S - iso, positive when >= 0) with linear (beta = 0) or smoothed crossings and the shared
// ambiguous-face fix.  Writes *nv vertices to V (float64 [*nv][3]) and *nf
// triangles to F (int32 [*nf][3]) when they fit vcap / fcap rows, else writes
// nothing and returns false.  res <= 512, at most 2^26 crossed cubes (else the
// scan throws).  Synchronises the stream.
bool dualmc_run(Workspace& ws, hipStream_t s, const double* S, int res, double iso, double beta, double* V,
                int64_t vcap, int32_t* F, int64_t fcap, int64_t* nv, int64_t* nf);

}  // namespace pamo
