// Range-Doppler maps and the strongest cell of each coherent processing
// interval (Sec. III): an FFT of every simulated cube gives its
// range-Doppler map, and the velocity of the map's maximum, one per CPI, is
// the Doppler-time series compared with the ground truth.
//
//   X_c[k][d] = sum_l sum_n Y[c][l][n] exp(-j2pi k n / Ns) exp(+j2pi d l / L)
//   power[k][d] = sum_c |X_c[k][d]|^2
//
// Fused path (Ns = 256, L = 16 D2 with D2 in {1, 2, 4, 8}): one workgroup
// holds a whole channel's L x 256 tile in registers, 64 entries a thread
// (4 rows of 16), and takes it through both FFTs without touching HBM in
// between:
//   k_rd_fused   per workgroup (at most one per compute unit) a contiguous
//                run of the (frame, channel) items; for each: fast-time
//                FFT as 16 x 16 (16-point DFTs in registers, a transpose
//                inside each wavefront through LDS), the tile's half
//                spectra moved through LDS into the slow-time layout, the
//                L-point inverse-sign FFT as 16 x D2 (the second factor
//                read back from LDS written in place), |.|^2 accumulated in
//                registers over the run's channels; one partial map per
//                (workgroup, frame) written at the run's frame boundaries
//   k_rd_merge   per (frame, block of 4096 cells): the partial maps of the
//                workgroups that cover the frame summed in workgroup order
//                -> power, and the block's maximum
//   k_rd_peak    per frame: the maximum over the blocks, its range and
//                velocity, and the velocity spectrum at its range bin
// HBM traffic: the cubes read once, plus one partial map per (workgroup,
// frame) written and read back, plus the map.
//
// Two-pass path (other shapes):
//   k_range_fft      fast-time FFT of every (frame, channel, block) row in
//                    LDS -> rf[F][C][L][Ns] (float2 workspace)
//   k_doppler_power  per (frame, group of KB range bins): for each channel
//                    the inverse-sign FFT over blocks in LDS, |.|^2 summed in
//                    registers -> power[F][Ns][L]; plus the group's maximum
//   k_rd_peak        as above
// The LDS FFTs are iterative radix-2 (decimation in time, bit-reversed
// load).  Both paths compute in float32 with twiddles evaluated in binary64;
// both are deterministic (fixed operation and summation order).
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

// ---------------------------------------------------------------------------
// Fused path
// ---------------------------------------------------------------------------
constexpr int kFNs = 256;                 // fast-time length of the fused path
constexpr int kFR = 16;                   // 256 = 16 x 16
constexpr int kFHalf = kFNs / 2;          // range bins per slow-time half
constexpr int kFX1 = kFR * (kFR + 1);     // one row of the fast-time transpose (padded, = 16 mod 32)
constexpr int kMergeCells = 4096;         // cells per k_rd_merge workgroup (256 threads, 4 float4 each)
constexpr int kFusedRows = 4;             // tile rows a thread holds (64 entries)

// cos(2 pi m / 16), m taken modulo 16
__host__ __device__ constexpr float cos16(int m)
{
    switch (m & 15) {
    case 0: return 1.0f;
    case 1: case 15: return 0.923879532511286756f;
    case 2: case 14: return 0.707106781186547524f;
    case 3: case 13: return 0.382683432365089772f;
    case 4: case 12: return 0.0f;
    case 5: case 11: return -0.382683432365089772f;
    case 6: case 10: return -0.707106781186547524f;
    case 7: case 9: return -0.923879532511286756f;
    default: return -1.0f;
    }
}
__host__ __device__ constexpr float sin16(int m) { return cos16(m + 12); }   // sin x = cos(x - pi/2)

__host__ __device__ constexpr int brev_c(int v, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
    return r;
}

// x * exp(SIGN j 2 pi m / 16) with the multiplications by 1 and +-j left out
template <int SIGN>
__device__ __forceinline__ float2 rot16(float2 x, int m)
{
    if (m == 0) return x;
    if (m == 4) return make_float2(-(float)SIGN * x.y, (float)SIGN * x.x);
    return cmul(x, make_float2(cos16(m), (float)SIGN * sin16(m)));
}

// In-register DFT of N <= 16 points, natural order in and out:
// v[k] <- sum_n v[n] exp(SIGN j 2 pi n k / N); radix-2 decimation in time,
// the bit reversal a renaming of registers.
template <int N, int SIGN>
__device__ __forceinline__ void dft_reg(float2 *v)
{
    constexpr int LOG = N >= 16 ? 4 : N >= 8 ? 3 : N >= 4 ? 2 : N >= 2 ? 1 : 0;
    static_assert((1 << LOG) == N && N <= 16, "N must be a power of two <= 16");
    float2 a[N];
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] = v[brev_c(i, LOG)];
#pragma unroll
    for (int s = 0; s < LOG; ++s) {
        const int half = 1 << s;
#pragma unroll
        for (int b = 0; b < N / 2; ++b) {
            const int pos = b & (half - 1);
            const int i = ((b >> s) << (s + 1)) + pos;
            const float2 t = rot16<SIGN>(a[i + half], pos * (8 / half));
            const float2 u = a[i];
            a[i] = make_float2(u.x + t.x, u.y + t.y);
            a[i + half] = make_float2(u.x - t.x, u.y - t.y);
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = a[i];
}

// LDS ordering among the lanes of one wavefront: the wavefront's LDS
// operations complete in issue order, so a fence that keeps the compiler
// from moving them across suffices.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int D2, int RPT>
struct rd_fused_shape {
    static constexpr int L = 16 * D2;
    static constexpr int T = 16 * L / RPT;          // threads: RPT rows of 16 tile entries each
    static constexpr int IPT = RPT / 2;             // slow-time problems per thread and half
    static constexpr int P = L + D2;                // padded row of the slow-time exchange
    static constexpr int NW = T / 64;
    static constexpr int X1 = NW * 4 * kFX1;        // fast-time transposes, 4 rows per wavefront
    static constexpr int XB = kFHalf * P > X1 ? kFHalf * P : X1;
    static constexpr size_t lds = (size_t)(XB + kFR * kFR + L) * sizeof(float2);
    static_assert(T % 64 == 0 && RPT % 2 == 0, "whole wavefronts, rows in pairs");
};

// Workgroup w takes items [w n / W, (w + 1) n / W) of the n = F C items
// (item = frame * C + channel, the cube order) and writes the power summed
// over each frame's items in its run to slots[w J + frame - first frame].
// Thread layouts (t = thread, T threads, RPT rows a thread):
//   fast time   rows g + s L / RPT (g = t / 16, s < RPT); pass 1 holds
//               n = q + 16 n1 (q = t % 16) and transforms over n1, pass 2
//               holds k = q + 16 k2 and transforms over the other factor
//   slow time   problems p = t + T i (i < RPT / 2) of half h: range bin
//               128 h + p / D2; pass 1 holds l = j + D2 l1 (j = p % D2) and
//               transforms over l1, pass 2 holds d1 = (16 / D2) j + e
//               (e < 16 / D2) and transforms over the D2 values of j;
//               cells (k, d = d1 + 16 d2)
template <int D2, int RPT, typename IT>
__global__ __launch_bounds__((rd_fused_shape<D2, RPT>::T)) void k_rd_fused(const IT *__restrict__ cubes,
                                                                        float *__restrict__ slots, int C,
                                                                        int64_t nitems, int W, int J)
{
    using S = rd_fused_shape<D2, RPT>;
    constexpr int L = S::L, P = S::P, T = S::T, IPT = S::IPT;
    constexpr int DI = 16 / D2;   // slow-time pass-2 problems per slow-time pass-1 problem
    constexpr int LD2 = D2 >= 8 ? 3 : D2 >= 4 ? 2 : D2 >= 2 ? 1 : 0;
    // LDS layouts (64 banks of 4 bytes: 32 float2 slots, 32 lanes served
    // together by a 64-bit access), all free of bank conflicts:
    //   slow-time exchange  entry (k, l) of a half at k P + (l ^ swz(k)),
    //                       swz(k) < D2 spreading the rows that the
    //                       16-lane groups of the write share a bank with
    //   pass 1 -> pass 2    row k rewritten in place: pass-1 problem j's
    //                       output d1 at D2 d1 + d1 / DI + j (one pad slot
    //                       after each 16)
    //   fast-time transpose rows of kFX1 = 16 (mod 32) slots
    auto swz = [](int k) { return (((k * D2) >> 5) << 1) & (D2 - 1); };
    extern __shared__ float2 smem[];
    float2 *buf = smem;
    // twiddles laid out so that a thread's own sit at fixed offsets from
    // one base: twr[k1][q] = exp(-j 2 pi q k1 / 256), twd[d1][j] =
    // exp(+j 2 pi j d1 / L)
    float2 *twr = smem + S::XB;
    float2 *twd = twr + kFR * kFR;
    const int t = threadIdx.x;
    const int g = t >> 4, q = t & 15, wv = t >> 6;
    const int jj = t % D2;
    const int sig = swz(q);   // = swz(q + 16 k2) for every k2
    for (int m = t; m < kFR * kFR; m += T) {
        double sn, cs;
        sincospi(2.0 * (double)((m >> 4) * (m & 15)) / (double)kFNs, &sn, &cs);
        twr[m] = make_float2((float)cs, (float)-sn);
    }
    for (int m = t; m < 16 * D2; m += T) {
        double sn, cs;
        sincospi(2.0 * (double)((m / D2) * (m % D2)) / (double)L, &sn, &cs);
        twd[m] = make_float2((float)cs, (float)sn);
    }
    const int64_t i0 = (int64_t)blockIdx.x * nitems / W, i1 = ((int64_t)blockIdx.x + 1) * nitems / W;
    const int64_t f0 = i0 / C;
    float acc[2][IPT][DI][D2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int e = 0; e < DI; ++e)
#pragma unroll
                for (int d = 0; d < D2; ++d) acc[h][i][e][d] = 0.f;

    // the first PF rows of each next item are loaded under the current
    // item's last slow-time pass (registers for more are not free)
    constexpr int PF = 1;
    float2 pre[PF][kFR];
    const IT *tile = cubes + g * kFNs + q;
#pragma unroll
    for (int r = 0; r < PF; ++r)
#pragma unroll
        for (int n1 = 0; n1 < kFR; ++n1) pre[r][n1] = load_c(tile + i0 * (int64_t)(L * kFNs) + r * (L / RPT) * kFNs + kFR * n1);
    for (int64_t it = i0; it < i1; ++it) {
        const IT *src = tile + it * (int64_t)(L * kFNs);
        float2 v[RPT][kFR];
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int n1 = 0; n1 < kFR; ++n1)
                v[r][n1] = r < PF ? pre[r][n1] : load_c(src + r * (L / RPT) * kFNs + kFR * n1);
        __syncthreads();   // the previous item's slow-time reads of buf are done (and the tables written)
        // fast time, one row at a time: 16-point DFT over n1, the product
        // with exp(-j 2 pi q k1 / 256) stored transposed, 16-point DFT over
        // the other factor -> v[r][k2] = X[row][q + 16 k2]
        float2 *x1 = buf + (wv * 4 + (g & 3)) * kFX1;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            dft_reg<kFR, -1>(v[r]);
            x1[q] = v[r][0];
#pragma unroll
            for (int k1 = 1; k1 < kFR; ++k1) x1[k1 * (kFR + 1) + q] = cmul(v[r][k1], twr[k1 * kFR + q]);
            wave_sync();
#pragma unroll
            for (int n2 = 0; n2 < kFR; ++n2) v[r][n2] = x1[q * (kFR + 1) + n2];
            wave_sync();
            dft_reg<kFR, -1>(v[r]);
            // finished spectra stay in registers: otherwise the compiler
            // defers the last butterflies of the second half past the
            // barriers below and holds both of their operands meanwhile
#pragma unroll
            for (int k = 0; k < kFR; ++k) asm volatile("" : "+v"(v[r][k].x), "+v"(v[r][k].y));
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __syncthreads();   // transposes / the other half's reads are done
#pragma unroll
            for (int r = 0; r < RPT; ++r)
#pragma unroll
                for (int k2 = 0; k2 < kFR / 2; ++k2)
                    buf[(q + kFR * k2) * P + (g ^ sig) + r * (L / RPT)] = v[r][h * (kFR / 2) + k2];
            if (h == 1) {
                // after the run's last item the load is a dummy one of item
                // 0's rows, which every workgroup shares through L2 (a
                // branch here would cost registers)
                const IT *nsrc = tile + (it + 1 < i1 ? it + 1 : 0) * (int64_t)(L * kFNs);
#pragma unroll
                for (int r = 0; r < PF; ++r)
#pragma unroll
                    for (int n1 = 0; n1 < kFR; ++n1) pre[r][n1] = load_c(nsrc + r * (L / RPT) * kFNs + kFR * n1);
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int kl = (t + T * i) / D2;
                // slow time, pass 1: 16-point DFT over l1, the product with
                // exp(+j 2 pi j d1 / L) written back in place
                float2 *row = buf + kl * P;
                const float2 *col = row + (jj ^ swz(kl));
                float2 u[16];
#pragma unroll
                for (int l1 = 0; l1 < 16; ++l1) u[l1] = col[D2 * l1];
                dft_reg<16, +1>(u);
                row += jj;
                row[0] = u[0];
#pragma unroll
                for (int d1 = 1; d1 < 16; ++d1) row[D2 * d1 + (d1 >> (4 - LD2))] = cmul(u[d1], twd[d1 * D2 + jj]);
            }
            wave_sync();   // the D2 threads of a range bin are lanes of one wavefront
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int kl = (t + T * i) / D2;
                // slow time, pass 2: D2-point DFT over j for d1 = DI jj + e
#pragma unroll
                for (int e = 0; e < DI; ++e) {
                    const float2 *z0 = buf + kl * P + 17 * jj + D2 * e;
                    float2 z[D2];
#pragma unroll
                    for (int j = 0; j < D2; ++j) z[j] = z0[j];
                    dft_reg<D2, +1>(z);
#pragma unroll
                    for (int d = 0; d < D2; ++d)
                        acc[h][i][e][d] =
                            __builtin_fmaf(z[d].x, z[d].x, __builtin_fmaf(z[d].y, z[d].y, acc[h][i][e][d]));
                }
            }
        }
        const int64_t f = it / C;
        if (it + 1 == i1 || (it + 1) / C != f) {
            float *dst = slots + ((int64_t)blockIdx.x * J + (f - f0)) * (int64_t)(kFNs * L);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    const int kl = (t + T * i) / D2;
#pragma unroll
                    for (int e = 0; e < DI; ++e)
#pragma unroll
                        for (int d = 0; d < D2; ++d) {
                            dst[(kFHalf * h + kl) * L + DI * jj + e + 16 * d] = acc[h][i][e][d];
                            acc[h][i][e][d] = 0.f;
                        }
                }
        }
    }
}

// Per (frame, block of 4096 cells): the frame's partial maps summed in
// workgroup order -> power, and the block's maximum (smallest cell index on
// ties; d = 0 skipped when skip_static).
__global__ __launch_bounds__(256) void k_rd_merge(const float *__restrict__ slots, float *__restrict__ power,
                                                 rd_peak_part *parts, int C, int64_t nitems, int W, int J,
                                                 int cells, int L, int skip_static)
{
    constexpr int V = kMergeCells / (4 * 256);   // float4 per thread
    const int nblk = cells / kMergeCells;
    const int64_t f = blockIdx.x / nblk;
    const int b = blockIdx.x % nblk;
    const int64_t wlo = ((f * C + 1) * W - 1) / nitems, whi = ((f * C + C) * W - 1) / nitems;
    float4 s[V];
#pragma unroll
    for (int v = 0; v < V; ++v) s[v] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t w = wlo; w <= whi; ++w) {
        const int64_t first = (w * nitems / W) / C;
        const float *src = slots + (w * J + (f - first)) * (int64_t)cells + b * kMergeCells + threadIdx.x * 4;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const float4 p = *reinterpret_cast<const float4 *>(src + v * 1024);
            s[v].x += p.x;
            s[v].y += p.y;
            s[v].z += p.z;
            s[v].w += p.w;
        }
    }
    float best = -1.f;
    int bidx = -1;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int e = b * kMergeCells + v * 1024 + threadIdx.x * 4;
        *reinterpret_cast<float4 *>(power + f * (int64_t)cells + e) = s[v];
        const float vals[4] = {s[v].x, s[v].y, s[v].z, s[v].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = e + i;
            if (!(skip_static && (c & (L - 1)) == 0) && vals[i] > best) {
                best = vals[i];
                bidx = c;
            }
        }
    }
    __shared__ float rv[256];
    __shared__ int ri[256];
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = bidx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
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
        p.idx = ri[0];
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

// Workgroups of the fused path: at most one per compute unit (a
// workgroup's LDS fills one), as few as keep the longest run at
// ceil(F C / compute units) items, the items split evenly over them; a
// frame's items can fall into several runs, whose partial maps k_rd_merge
// adds (fewer workgroups, fewer partial maps).
int64_t rd_fused_workgroups(int64_t nframes, int C, int ncu)
{
    const int64_t n = nframes * C;
    const int64_t per = (n + ncu - 1) / std::max(1, ncu);
    return std::max<int64_t>(1, (n + per - 1) / per);
}

template <int D2, typename IT>
hipError_t launch_fused(const void *cubes, float *slots, int C, int64_t nitems, int W, int J, hipStream_t st)
{
    constexpr int RPT = kFusedRows;
    using S = rd_fused_shape<D2, RPT>;
    // set on every launch: the attribute belongs to the device current now
    const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rd_fused<D2, RPT, IT>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_rd_fused<D2, RPT, IT>), dim3((unsigned)W), dim3(S::T), S::lds, st,
                       reinterpret_cast<const IT *>(cubes), slots, C, nitems, W, J);
    return hipGetLastError();
}

template <typename IT>
hipError_t launch_fused_l(int L, const void *cubes, float *slots, int C, int64_t nitems, int W, int J,
                          hipStream_t st)
{
    switch (L) {
    case 16: return launch_fused<1, IT>(cubes, slots, C, nitems, W, J, st);
    case 32: return launch_fused<2, IT>(cubes, slots, C, nitems, W, J, st);
    case 64: return launch_fused<4, IT>(cubes, slots, C, nitems, W, J, st);
    default: return launch_fused<8, IT>(cubes, slots, C, nitems, W, J, st);
    }
}

}  // namespace

namespace {

// Workspace of one call, in 256-byte aligned pieces.  Fused path: the
// partial maps [W][J][cells], the map when the caller wants none, the block
// maxima.  Two-pass path: the float2 fast-time spectra, the map when the
// caller wants none, the group maxima.
struct rd_layout {
    bool fused = false;
    int64_t W = 0, J = 0, nitems = 0;
    int groups = 0, kb = 0;
    size_t mid = 0, pw = 0, parts = 0, total = 0;   // byte offsets / sizes
};

rd_layout rd_plan_layout(const rs_plan *pl, int64_t nframes, bool power_given)
{
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    rd_layout y;
    const int Ns = pl->Ns, L = pl->L, C = pl->C;
    const int64_t cells = (int64_t)Ns * L;
    y.fused = Ns == kFNs && L >= 16 && L <= 128;
    size_t mid_bytes;
    if (y.fused) {
        y.nitems = nframes * C;
        y.W = rd_fused_workgroups(nframes, C, pl->ncu);
        const int64_t per = (y.nitems + y.W - 1) / y.W;
        y.J = (per - 1 + C - 1) / C + 1;   // frames a run of `per` items can touch
        y.groups = (int)(cells / kMergeCells);
        mid_bytes = (size_t)(y.W * y.J * cells) * sizeof(float);
    } else {
        y.kb = std::min(std::min(16, kGroupElems / L), Ns);
        y.groups = Ns / y.kb;
        mid_bytes = (size_t)(nframes * C * L * Ns) * sizeof(float2);
    }
    const size_t pw_bytes = power_given ? 0 : (size_t)(nframes * cells) * sizeof(float);
    const size_t part_bytes = (size_t)nframes * y.groups * sizeof(rd_peak_part);
    y.mid = 0;
    y.pw = up(mid_bytes);
    y.parts = y.pw + up(pw_bytes);
    y.total = y.parts + up(part_bytes);
    return y;
}

// Argument checks of both entry points; nframes = 0 passes (nothing to do).
rs_status rd_check(const rs_plan *pl, const void *cubes, int32_t nframes, int *logn, int *logl)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (nframes < 0) return rs_fail(RS_E_INVALID, "nframes < 0");
    if (nframes == 0) return RS_OK;
    if (!cubes) return rs_fail(RS_E_INVALID, "cubes is NULL");
    *logn = ilog2_exact(pl->Ns);
    *logl = ilog2_exact(pl->L);
    if (*logn < 1 || *logl < 1 || pl->Ns > 4096 || pl->L > 1024)
        return rs_fail(RS_E_UNSUPPORTED, "range-Doppler maps need Ns and L powers of two, 2 <= Ns <= 4096, "
                                         "2 <= L <= 1024 (got Ns = %d, L = %d)", pl->Ns, pl->L);
    return RS_OK;
}

// The launches of one call on `st` with the workspace `ws` laid out as y.
rs_status rd_run(const rs_plan *pl, const rd_layout &y, const void *cubes, int32_t nframes, int32_t skip_static,
                 float *power, float *doppler_time, rs_rd_peak *peaks, char *ws, int logn, int logl,
                 hipStream_t st)
{
    const int Ns = pl->Ns, L = pl->L, C = pl->C;
    const int64_t cells = (int64_t)Ns * L;
    const float rpb = pl->mu != 0.0 ? (float)(pl->c0 * pl->Fs / (2.0 * pl->mu * Ns)) : 0.f;
    const float vpb = pl->fc != 0.0 ? (float)(pl->c0 / (2.0 * pl->fc * pl->Tb * L)) : 0.f;
    float *pw = power ? power : reinterpret_cast<float *>(ws + y.pw);
    rd_peak_part *parts = reinterpret_cast<rd_peak_part *>(ws + y.parts);
    hipError_t e;
    if (y.fused) {
        float *slots = reinterpret_cast<float *>(ws + y.mid);
        e = pl->dtype == RS_C128
                ? launch_fused_l<double2>(L, cubes, slots, C, y.nitems, (int)y.W, (int)y.J, st)
                : launch_fused_l<float2>(L, cubes, slots, C, y.nitems, (int)y.W, (int)y.J, st);
        if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "fused range-Doppler launch: %s", hipGetErrorString(e));
        hipLaunchKernelGGL(k_rd_merge, dim3((unsigned)(nframes * y.groups)), dim3(256), 0, st, slots, pw, parts, C,
                           y.nitems, (int)y.W, (int)y.J, (int)cells, L, skip_static ? 1 : 0);
        e = hipGetLastError();
        if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "map merge launch: %s", hipGetErrorString(e));
    } else {
        float2 *rf = reinterpret_cast<float2 *>(ws + y.mid);
        const int64_t rows = (int64_t)nframes * C * L;
        const int rpw = std::max(1, 2048 / Ns);
        const int64_t g1 = (rows + rpw - 1) / rpw;
        const size_t lds1 = (size_t)(Ns / 2 + rpw * Ns) * sizeof(float2);
        if (pl->dtype == RS_C128)
            hipLaunchKernelGGL(k_range_fft<double2>, dim3((unsigned)g1), dim3(kThreads), lds1, st,
                               reinterpret_cast<const double2 *>(cubes), rf, rows, logn, rpw);
        else
            hipLaunchKernelGGL(k_range_fft<float2>, dim3((unsigned)g1), dim3(kThreads), lds1, st,
                               reinterpret_cast<const float2 *>(cubes), rf, rows, logn, rpw);
        e = hipGetLastError();
        if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "range FFT launch: %s", hipGetErrorString(e));
        const size_t lds2 = (size_t)(L / 2 + y.kb * L) * sizeof(float2);
        hipLaunchKernelGGL(k_doppler_power, dim3((unsigned)(nframes * y.groups)), dim3(kThreads), lds2, st, rf, pw,
                           parts, C, logl, Ns, y.kb, skip_static ? 1 : 0);
        e = hipGetLastError();
        if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "Doppler launch: %s", hipGetErrorString(e));
    }
    if (peaks || doppler_time) {
        hipLaunchKernelGGL(k_rd_peak, dim3((unsigned)nframes), dim3(kThreads), 0, st, parts, pw, y.groups, Ns, L, rpb,
                           vpb, peaks, doppler_time);
        e = hipGetLastError();
        if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "peak launch: %s", hipGetErrorString(e));
    }
    return RS_OK;
}

}  // namespace

extern "C" size_t rs_range_doppler_workspace_bytes(const rs_plan *pl, int32_t nframes, int32_t power_given)
{
    if (!pl || nframes <= 0) return 0;
    return rd_plan_layout(pl, nframes, power_given != 0).total;
}

extern "C" rs_status rs_range_doppler(rs_plan *pl, const void *cubes, int32_t nframes, int32_t skip_static,
                                      float *power, float *doppler_time, rs_rd_peak *peaks, void *stream)
{
    int logn = 0, logl = 0;
    const rs_status c = rd_check(pl, cubes, nframes, &logn, &logl);
    if (c != RS_OK || nframes == 0) return c;
    device_guard g(pl->device);
    if (g.st != RS_OK) return g.st;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const rd_layout y = rd_plan_layout(pl, nframes, power != nullptr);
    char *ws = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&ws), y.total, st) != hipSuccess)
        return rs_fail(RS_E_NOMEM, "stream-ordered workspace allocation of %zu bytes failed", y.total);
    rs_status s = rd_run(pl, y, cubes, nframes, skip_static, power, doppler_time, peaks, ws, logn, logl, st);
    const hipError_t e = hipFreeAsync(ws, st);
    if (e != hipSuccess && s == RS_OK) s = rs_fail(RS_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    return s;
}

extern "C" rs_status rs_range_doppler_ws(rs_plan *pl, const void *cubes, int32_t nframes, int32_t skip_static,
                                         float *power, float *doppler_time, rs_rd_peak *peaks, void *workspace,
                                         size_t workspace_bytes, void *stream)
{
    int logn = 0, logl = 0;
    const rs_status c = rd_check(pl, cubes, nframes, &logn, &logl);
    if (c != RS_OK || nframes == 0) return c;
    const rd_layout y = rd_plan_layout(pl, nframes, power != nullptr);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return rs_fail(RS_E_INVALID, "workspace is NULL or not 256-byte aligned");
    if (workspace_bytes < y.total)
        return rs_fail(RS_E_INVALID, "workspace of %zu bytes, %zu needed", workspace_bytes, y.total);
    device_guard g(pl->device);
    if (g.st != RS_OK) return g.st;
    return rd_run(pl, y, cubes, nframes, skip_static, power, doppler_time, peaks, static_cast<char *>(workspace),
                  logn, logl, reinterpret_cast<hipStream_t>(stream));
}
