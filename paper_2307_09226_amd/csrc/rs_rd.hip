// Range-Doppler maps and the strongest cell of each coherent processing
// interval (Sec. III): an FFT of every simulated cube gives its
// range-Doppler map, and the velocity of the map's maximum, one per CPI, is
// the Doppler-time series compared with the ground truth.
//
//   X_c[k][d] = sum_l sum_n Y[c][l][n] exp(-j2pi k n / Ns) exp(+j2pi d l / L)
//   power[k][d] = sum_c |X_c[k][d]|^2
//
// Three launches on the caller's stream:
//   k_range_fft      fast-time FFT of every (frame, channel, block) row in
//                    LDS -> rf[F][C][L][Ns] (float2 workspace)
//   k_doppler_power  per (frame, group of KB range bins): for each channel
//                    the inverse-sign FFT over blocks in LDS, |.|^2 summed in
//                    registers -> power[F][Ns][L]; plus the group's maximum
//   k_rd_peak        per frame: the maximum over the groups, its range and
//                    velocity, and the velocity spectrum at its range bin
// The FFTs are iterative radix-2 (decimation in time, bit-reversed load) in
// float32 with twiddles evaluated in binary64.  Memory bound: every cube
// entry is read once and the float2 intermediate written and read once.
#include "rs_api_internal.h"
#include "rs_fft.h"

#include <cmath>

namespace {

constexpr int kThreads = 256;
constexpr int kMaxPerThread = 16;   // power elements per thread in k_doppler_power
constexpr int kGroupElems = 4096;   // KB * L, at most (dynamic LDS <= 64 KiB)

struct rd_peak_part {
    float v;
    int32_t idx;   // k * L + d, -1 when the group has no eligible cell
};

template <typename IT>
__device__ __forceinline__ float2 load_c(const IT *p) { return make_float2((float)p->x, (float)p->y); }

// Fast-time FFT of `rows_total` rows of length Ns; `rpw` rows per workgroup.
template <typename IT>
__global__ __launch_bounds__(kThreads) void k_range_fft(const IT *cubes, float2 *rf, int64_t rows_total,
                                                        int logn, int rpw)
{
    extern __shared__ float2 smem[];
    const int n = 1 << logn;
    float2 *tw = smem;
    float2 *x = smem + n / 2;
    const int64_t r0 = (int64_t)blockIdx.x * rpw;
    const int rows = (int)min<int64_t>(rpw, rows_total - r0);
    if (rows <= 0) return;
    twiddles(tw, n, -1.0);
    const IT *src = cubes + r0 * n;
    for (int e = threadIdx.x; e < rows * n; e += blockDim.x) {
        const int row = e >> logn, col = e & (n - 1);
        x[row * n + bitrev(col, logn)] = load_c(src + e);
    }
    __syncthreads();
    fft_rows(x, rows, logn, tw);
    float2 *dst = rf + r0 * n;
    for (int e = threadIdx.x; e < rows * n; e += blockDim.x) dst[e] = x[e];
}

// Per (frame, group of kb range bins starting at k0): inverse-sign FFT over
// the L blocks for every channel, power summed over channels.
__global__ __launch_bounds__(kThreads) void k_doppler_power(const float2 *rf, float *power, rd_peak_part *parts,
                                                            int C, int logl, int Ns, int kb, int skip_static)
{
    extern __shared__ float2 smem[];
    const int L = 1 << logl;
    const int logkb = __builtin_ctz((unsigned)kb);
    const int groups = Ns / kb;
    const int f = blockIdx.x / groups;
    const int k0 = (blockIdx.x % groups) * kb;
    float2 *tw = smem;
    float2 *x = smem + L / 2;   // [kb][L]
    twiddles(tw, L, +1.0);
    const int ne = kb * L;      // elements of this group, <= kGroupElems
    float acc[kMaxPerThread];
#pragma unroll
    for (int i = 0; i < kMaxPerThread; ++i) acc[i] = 0.f;
    for (int c = 0; c < C; ++c) {
        const float2 *src = rf + (((int64_t)f * C + c) * L) * Ns + k0;
        // element e = l * kb + kk: kb consecutive range bins of one block row
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            const int l = e >> logkb, kk = e & (kb - 1);   // kb is a power of two
            x[kk * L + bitrev(l, logl)] = src[(int64_t)l * Ns + kk];
        }
        __syncthreads();
        fft_rows(x, kb, logl, tw);
#pragma unroll
        for (int i = 0; i < kMaxPerThread; ++i) {
            const int e = threadIdx.x + i * kThreads;
            if (e < ne) {
                const float2 v = x[e];
                acc[i] = __builtin_fmaf(v.x, v.x, __builtin_fmaf(v.y, v.y, acc[i]));
            }
        }
        __syncthreads();  // x is reloaded by the next channel
    }
    // write power[f][k0 + kk][d] (element e = kk * L + d) and find the
    // group's maximum; ties go to the smallest element index
    float best = -1.f;
    int bidx = -1;
    float *dst = power + ((int64_t)f * Ns + k0) * L;
#pragma unroll
    for (int i = 0; i < kMaxPerThread; ++i) {
        const int e = threadIdx.x + i * kThreads;
        if (e < ne) {
            dst[e] = acc[i];
            const int d = e & (L - 1);
            if (!(skip_static && d == 0) && acc[i] > best) {
                best = acc[i];
                bidx = e;
            }
        }
    }
    __shared__ float rv[kThreads];
    __shared__ int ri[kThreads];
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = bidx;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const float v2 = rv[threadIdx.x + o];
            const int i2 = ri[threadIdx.x + o];
            if (i2 >= 0 && (ri[threadIdx.x] < 0 || v2 > rv[threadIdx.x] ||
                            (v2 == rv[threadIdx.x] && i2 < ri[threadIdx.x]))) {
                rv[threadIdx.x] = v2;
                ri[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rd_peak_part p;
        p.v = rv[0];
        p.idx = ri[0] < 0 ? -1 : k0 * L + ri[0];
        parts[blockIdx.x] = p;
    }
}

// Per frame: maximum over the groups (smallest index on ties), the peak
// record and the velocity spectrum at the peak's range bin.
__global__ __launch_bounds__(kThreads) void k_rd_peak(const rd_peak_part *parts, const float *power, int groups,
                                                      int Ns, int L, float range_per_bin, float vel_per_bin,
                                                      rs_rd_peak *peaks, float *dtime)
{
    const int f = blockIdx.x;
    __shared__ float rv[kThreads];
    __shared__ int ri[kThreads];
    float best = -1.f;
    int bidx = -1;
    for (int g = threadIdx.x; g < groups; g += kThreads) {
        const rd_peak_part p = parts[(int64_t)f * groups + g];
        if (p.idx >= 0 && (bidx < 0 || p.v > best || (p.v == best && p.idx < bidx))) {
            best = p.v;
            bidx = p.idx;
        }
    }
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = bidx;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const float v2 = rv[threadIdx.x + o];
            const int i2 = ri[threadIdx.x + o];
            if (i2 >= 0 && (ri[threadIdx.x] < 0 || v2 > rv[threadIdx.x] ||
                            (v2 == rv[threadIdx.x] && i2 < ri[threadIdx.x]))) {
                rv[threadIdx.x] = v2;
                ri[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    const int idx = ri[0];
    const int k = idx < 0 ? 0 : idx / L;
    if (threadIdx.x == 0 && peaks) {
        rs_rd_peak p;
        const int d = idx < 0 ? 0 : idx % L;
        const int ds = d >= L / 2 ? d - L : d;
        p.range_bin = k;
        p.doppler_bin = ds;
        p.power = idx < 0 ? 0.f : rv[0];
        p.range_m = (float)k * range_per_bin;
        p.velocity_mps = (float)ds * vel_per_bin;
        p.reserved = 0.f;
        peaks[f] = p;
    }
    if (dtime) {
        const float *row = power + ((int64_t)f * Ns + k) * L;
        for (int d = threadIdx.x; d < L; d += kThreads) dtime[(int64_t)f * L + d] = row[d];
    }
}

int ilog2_exact(int v)
{
    if (v < 1 || (v & (v - 1))) return -1;
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

extern "C" rs_status rs_range_doppler(rs_plan *pl, const void *cubes, int32_t nframes, int32_t skip_static,
                                      float *power, float *doppler_time, rs_rd_peak *peaks, void *stream)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (nframes < 0) return rs_fail(RS_E_INVALID, "nframes < 0");
    if (nframes == 0) return RS_OK;
    if (!cubes) return rs_fail(RS_E_INVALID, "cubes is NULL");
    const int logn = ilog2_exact(pl->Ns), logl = ilog2_exact(pl->L);
    if (logn < 1 || logl < 1 || pl->Ns > 4096 || pl->L > 1024)
        return rs_fail(RS_E_UNSUPPORTED, "range-Doppler maps need Ns and L powers of two, 2 <= Ns <= 4096, "
                                         "2 <= L <= 1024 (got Ns = %d, L = %d)", pl->Ns, pl->L);
    device_guard g(pl->device);
    if (g.st != RS_OK) return g.st;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);

    const int Ns = pl->Ns, L = pl->L, C = pl->C;
    const int64_t rows = (int64_t)nframes * C * L;
    const int rpw = std::max(1, 2048 / Ns);
    int kb = std::min(16, kGroupElems / L);
    kb = std::min(kb, Ns);
    const int groups = Ns / kb;
    const size_t rf_bytes = (size_t)rows * Ns * sizeof(float2);
    const size_t pw_bytes = power ? 0 : (size_t)nframes * Ns * L * sizeof(float);
    const size_t part_bytes = (size_t)nframes * groups * sizeof(rd_peak_part);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t total = up(rf_bytes) + up(pw_bytes) + up(part_bytes);
    char *ws = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&ws), total, st) != hipSuccess)
        return rs_fail(RS_E_NOMEM, "stream-ordered workspace allocation of %zu bytes failed", total);
    float2 *rf = reinterpret_cast<float2 *>(ws);
    float *pw = power ? power : reinterpret_cast<float *>(ws + up(rf_bytes));
    rd_peak_part *parts = reinterpret_cast<rd_peak_part *>(ws + up(rf_bytes) + up(pw_bytes));

    rs_status s = RS_OK;
    const int64_t g1 = (rows + rpw - 1) / rpw;
    const size_t lds1 = (size_t)(Ns / 2 + rpw * Ns) * sizeof(float2);
    if (pl->dtype == RS_C128)
        hipLaunchKernelGGL(k_range_fft<double2>, dim3((unsigned)g1), dim3(kThreads), lds1, st,
                           reinterpret_cast<const double2 *>(cubes), rf, rows, logn, rpw);
    else
        hipLaunchKernelGGL(k_range_fft<float2>, dim3((unsigned)g1), dim3(kThreads), lds1, st,
                           reinterpret_cast<const float2 *>(cubes), rf, rows, logn, rpw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) s = rs_fail(RS_E_DEVICE, "range FFT launch: %s", hipGetErrorString(e));
    if (s == RS_OK) {
        const size_t lds2 = (size_t)(L / 2 + kb * L) * sizeof(float2);
        hipLaunchKernelGGL(k_doppler_power, dim3((unsigned)(nframes * groups)), dim3(kThreads), lds2, st, rf, pw,
                           parts, C, logl, Ns, kb, skip_static ? 1 : 0);
        e = hipGetLastError();
        if (e != hipSuccess) s = rs_fail(RS_E_DEVICE, "Doppler launch: %s", hipGetErrorString(e));
    }
    if (s == RS_OK && (peaks || doppler_time)) {
        const float rpb = pl->mu != 0.0 ? (float)(pl->c0 * pl->Fs / (2.0 * pl->mu * Ns)) : 0.f;
        const float vpb = pl->fc != 0.0 ? (float)(pl->c0 / (2.0 * pl->fc * pl->Tb * L)) : 0.f;
        hipLaunchKernelGGL(k_rd_peak, dim3((unsigned)nframes), dim3(kThreads), 0, st, parts, pw, groups, Ns, L, rpb,
                           vpb, peaks, doppler_time);
        e = hipGetLastError();
        if (e != hipSuccess) s = rs_fail(RS_E_DEVICE, "peak launch: %s", hipGetErrorString(e));
    }
    e = hipFreeAsync(ws, st);
    if (e != hipSuccess && s == RS_OK) s = rs_fail(RS_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    return s;
}
