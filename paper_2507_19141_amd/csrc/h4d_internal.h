// Internal declarations shared by the host API and the HIP kernels of libhash4d.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hash4d.h"

namespace h4d {

// Grid description as the kernels see it: passed by value as a kernel argument,
// so every per-level field is a uniform (scalar) load from the kernarg segment.
struct DevGrid {
    int32_t L;
    int32_t F;
    uint32_t T;          // rows of a hashed level
    uint32_t tmask;      // T - 1 when T is a power of two, else 0
    uint32_t dense_bits; // bit l set: level l is dense
    uint32_t prime[4];
    int32_t res_s[H4D_MAX_LEVELS];
    int32_t res_t[H4D_MAX_LEVELS];
    uint32_t off[H4D_MAX_LEVELS]; // first row of level l (E F < 2^31, so rows fit 32 bits)
};

// Host-side conversion of a validated h4d_grid.
DevGrid to_device(const h4d_grid& g);

// ---- encoder launchers (encode.hip) ----
// out[l * lstride + q * qstride + f]; level-major grid (blockIdx.y = level).
hipError_t launch_encode(const DevGrid& g, h4d_dtype table_dt, const void* table, const float* xyzt, int n,
                         void* out, int64_t lstride, int64_t qstride, hipStream_t s);
hipError_t launch_encode_backward(const DevGrid& g, h4d_dtype grad_dt, const float* xyzt, int n,
                                  const void* d_feat, int64_t lstride, int64_t qstride, double scale,
                                  void* d_table, hipStream_t s);
hipError_t launch_corner_indices(const DevGrid& g, const float* xyzt, int n, int32_t* rows, float* w,
                                 hipStream_t s);

}  // namespace h4d
