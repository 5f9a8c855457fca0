// Deflation at the reduction level (Sec. 3.1): launch arguments and
// launchers of the kernels in orth_deflate.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "orth_internal.h"

namespace orth {

// Per-handle deflation state in the workspace: this 64-byte header, then the
// first sweep's W = V~ Lambda~^{-1/2} (s x s, row-major, columns t..s-1 zero).
struct DeflState {
    int32_t dropped;        // s - t of the latest step
    int32_t steps;          // steps with t < s
    int32_t total;          // directions dropped so far
    int32_t pad[13];
};
static_assert(sizeof(DeflState) == 64, "W starts 64 bytes in");

__host__ __device__ inline double *defl_W(DeflState *d) { return reinterpret_cast<double *>(d + 1); }
__host__ __device__ inline const double *defl_W(const DeflState *d) {
    return reinterpret_cast<const double *>(d + 1);
}
// doubles the state takes for block width s
constexpr int64_t defl_state_doubles(int s) { return 8 + (int64_t)s * s; }

struct DeflArgs {
    double delta2;          // squared relative tolerance
    DeflState *state;
};

// u1 <- u1 W over the logical rows of one level (only when the latest first
// sweep dropped directions)
struct DeflRowArgs {
    double *U;
    int64_t ld;
    LevelGeom geom;
    const DeflState *state;
    const DevStatus *status;
};

// The reduction level's factorisation for sweep a.sweep, launched in place
// of the Cholesky kernel; one workgroup (a.nleaf must be 1).
hipError_t launch_defl(int s, const CholArgs &a, const DeflArgs &d, hipStream_t st);
hipError_t launch_defl_rows(int s, const DeflRowArgs &a, hipStream_t st);

}  // namespace orth
