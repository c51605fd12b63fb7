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

// Load p[i] from global memory.  Device pointers read out of a job table
// are generic (flat) to the compiler; a flat load also counts against the
// LDS wait counter, so a kernel waiting on its LDS operands would wait for
// the global load too.  Caller arrays are always global memory.
template <typename T>
__device__ __forceinline__ T rs_gload(const T *p, int64_t i)
{
    return ((const __attribute__((address_space(1))) T *)p)[i];
}

// Fractional part v - floor(v), in [0, 1] (1 only by rounding of tiny
// negative v).
__device__ __forceinline__ double rs_frac(double v) { return v - __builtin_floor(v); }

// Phase arguments of a pixel in virtual channel c = m N + r (Sec. II,
// eq. (1)): psi the carrier phase of sigma (cycles, not reduced), b the beat
// frequency (cycles per fast-time sample), beta the Doppler phase per block
// (cycles).  Without variant flags R = (|x - tx_m| + |x - rx_r|) / 2,
// psi = R Kc, b = R Kb, beta = v Kd.  The far-field flag uses eq. (2)'s
// range Rp = |x| and angle term instead: psi = Rp Kc - s Ka,
// s = u.(tx_m + rx_r)/2, u = x / Rp, b = Rp Kb (Ka = 2 fc / c0 even when
// the carrier phase is off, so that Kc = 0 gives eq. (2) as printed).  The
// other flags (rs_model_flags) change psi and b in the order below.
// J: an rs_job or any struct with its constants (model, M, Kc, Kb, Kd, Kf,
// Krvp, Ka).
template <typename JobConsts>
__device__ __forceinline__ void rs_chan_args(const JobConsts &J, float x, float y, float z, float v, int m,
                                             const double *tx, const double *rx, double *psi, double *b,
                                             double *beta)
{
    double Rb, ps;
    if (J.model & 1) {  // far field, eq. (2)
        const double xd = (double)x, yd = (double)y, zd = (double)z;
        const double Rp = __builtin_sqrt((xd * xd + yd * yd) + zd * zd);
        const double ux = xd / Rp, uy = yd / Rp, uz = zd / Rp;
        const double s = 0.5 * ((ux * (tx[0] + rx[0]) + uy * (tx[1] + rx[1])) + uz * (tx[2] + rx[2]));
        ps = Rp * J.Kc - s * J.Ka;
        Rb = Rp;
    } else {
        Rb = 0.5 * (rs_distance(x, y, z, tx) + rs_distance(x, y, z, rx));
        ps = Rb * J.Kc;
    }
    *beta = (double)v * J.Kd;
    *psi = ps;
    *b = Rb * J.Kb;
    if (J.model & 8) *psi = *psi - (Rb * Rb) * J.Krvp;                    // residual video phase
    if (J.model & 2) *psi = *psi - *beta * ((double)m / (double)J.M);     // Tx slot timing
    if (J.model & 4) *b = *b - (double)v * J.Kf;                          // Doppler within the chirp
}

// Per-item constants of the phase-argument recipe and the pixel arrays,
// copied to LDS once per work item by one thread: the job table is generic
// memory to the compiler, which reloads its fields after every LDS store
// (they might alias) and waits for each such load.
struct rs_item_consts {
    double Kc, Kb, Kd, Kf, Krvp, Ka;
    double tx[3], rx[3];            // antennas of the item's channel (Tx m, Rx r)
    const float *x, *y, *z, *amp, *vr;
    int64_t amp_lstride;
    int32_t model, M, L, pad_;
};

__device__ __forceinline__ void rs_item_consts_of(const rs_job &J, int m, int r, rs_item_consts &k)
{
    k.Kc = J.Kc;
    k.Kb = J.Kb;
    k.Kd = J.Kd;
    k.Kf = J.Kf;
    k.Krvp = J.Krvp;
    k.Ka = J.Ka;
    for (int i = 0; i < 3; ++i) {
        k.tx[i] = J.ant[3 * m + i];
        k.rx[i] = J.ant[3 * (J.M + r) + i];
    }
    k.x = J.x;
    k.y = J.y;
    k.z = J.z;
    k.amp = J.amp;
    k.vr = J.vr;
    k.amp_lstride = J.amp_lstride;
    k.model = J.model;
    k.M = J.M;
    k.L = J.L;
    k.pad_ = 0;
}

// Per-pixel quantities of one virtual channel: psi_f = frac(psi), b, beta, a.
struct rs_pixel_args {
    double psi_f, b, beta;
    float a;
};

__device__ __forceinline__ rs_pixel_args rs_pixel(const rs_job &J, int m, const double *tx,
                                                  const double *rx, int64_t p)
{
    rs_pixel_args o;
    double psi;
    rs_chan_args(J, J.x[p], J.y[p], J.z[p], J.vr[p], m, tx, rx, &psi, &o.b, &o.beta);
    o.psi_f = rs_frac(psi);
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
