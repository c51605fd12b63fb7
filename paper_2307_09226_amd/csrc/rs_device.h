// Device helpers shared by the gfx950 kernels: the binary64 geometry and
// phase-argument recipe and the work-item loop.
//
// Every file including this header is compiled with -ffp-contract=off so
// that the recipe below rounds exactly as written (IEEE binary64, round to
// nearest, correctly rounded sqrt on gfx950, no fused multiply-add): the
// plain form then reproduces binary64 reference sums to the last few ulp.
#pragma once
#include "rs_internal.h"

// Distance from a float32 pixel position to antenna `a` (metres).
__device__ __forceinline__ double rs_distance(float x, float y, float z, const double *a)
{
    double dx = (double)x - a[0];
    double dy = (double)y - a[1];
    double dz = (double)z - a[2];
    return __builtin_sqrt((dx * dx + dy * dy) + dz * dz);
}

// Fractional part v - floor(v), in [0, 1] (1 only by rounding of tiny
// negative v).
__device__ __forceinline__ double rs_frac(double v) { return v - __builtin_floor(v); }

// Per-pixel quantities of one virtual channel (Sec. II, eq. (1)):
//   R     = (|x - tx_m| + |x - rx_r|) / 2
//   psi_f = frac(R * Kc)      carrier phase of sigma, cycles mod 1
//   b     = R * Kb            beat frequency, cycles per fast-time sample
//   beta  = v * Kd            Doppler phase per block, cycles
struct rs_pixel_args {
    double psi_f, b, beta;
    float a;
};

__device__ __forceinline__ rs_pixel_args rs_pixel(const rs_job &J, const double *tx,
                                                  const double *rx, int64_t p)
{
    rs_pixel_args o;
    float x = J.x[p], y = J.y[p], z = J.z[p];
    double R = 0.5 * (rs_distance(x, y, z, tx) + rs_distance(x, y, z, rx));
    o.psi_f = rs_frac(R * J.Kc);
    o.b = R * J.Kb;
    o.beta = (double)J.vr[p] * J.Kd;
    o.a = J.amp[p];
    return o;
}

// Claim the next work item of a launch.  Persistent grids (counter != null)
// take items from an atomic counter; otherwise each workgroup runs item
// blockIdx.x once.  Returns -1 when no work is left.  Must be called by every
// thread of the workgroup (contains barriers in the persistent case).
__device__ __forceinline__ int64_t rs_next_item(const rs_launch &L, int64_t *slot, bool first)
{
    if (L.counter) {
        __syncthreads();
        if (threadIdx.x == 0) *slot = (int64_t)atomicAdd(L.counter, 1);
        __syncthreads();
        // uniform across the workgroup: keep it (and the job fields derived
        // from it) in scalar registers
        const int lo = __builtin_amdgcn_readfirstlane((int)(*slot & 0xffffffff));
        const int hi = __builtin_amdgcn_readfirstlane((int)(*slot >> 32));
        const int64_t it = ((int64_t)hi << 32) | (uint32_t)lo;
        return it < L.total ? it : -1;
    }
    if (!first) return -1;
    return (int64_t)blockIdx.x < L.total ? (int64_t)blockIdx.x : -1;
}
