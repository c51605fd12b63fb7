// Split-FP16 matrix-core form (gfx950, v_mfma_f32_32x32x16_f16).
//
// For one virtual channel c the cube is the complex contraction over pixels
//   Y_c[n][l] = sum_p F_c[p][n] * D[p][l]
//   F_c[p][n] = exp(j2pi (psi_{p,c} + b_{p,c} n))        unit magnitude
//   D[p][l]   = a_p exp(-j2pi beta_p l)                  shared by channels
// i.e. Y_c = F_c^T diag(sigma_c) D with the carrier phase of sigma folded into
// F (Sec. II, eq. (1) per channel, pixel sum of eq. (2)).  Phase arguments are
// evaluated and reduced mod 1 in binary64, phasors in binary32 with the
// hardware sin/cos (input in revolutions), and each binary32 value x is split
// into hi = rne16(x) and lo = rne16(x - hi).  The complex product is embedded
// in a real one: with k = (pixel, slot)
//   real column: A = (Fr, Fi), B = (Dr, -Di)  ->  Re(F D)
//   imag column: A = (Fr, Fi), B = (Di,  Dr)  ->  Im(F D)
// and hi*hi + hi*lo + lo*hi are accumulated in fp32 by the matrix cores
// (12 real MACs = 24 flop per term).
//
// Tiling (workgroup = 4 waves, one per SIMD):
//   item  = (channel, n tile of 4*WN rows, l tile of TL columns, pixel chunk)
//   wave  = WN rows x TL complex columns; WN/32 x 2TL/32 accumulator blocks
//   F     = A operand, evaluated by each lane for exactly the rows and pixels
//           it feeds to the matrix core (registers only, double-buffered so
//           the next step's phasors are computed while the matrix cores run)
//   D     = B operand, evaluated once per workgroup per 16-pixel step into
//           double-buffered LDS (both column arrangements, hi and lo)
// Phasor cost: per pixel and lane one binary64-reduced phasor; the other rows
// of the lane follow by binary32 rotation with exp(j2pi frac(32 b)), and the
// slow-time phasors of a thread by rotation with exp(j2pi frac(16 beta)) --
// every rotation factor is itself reduced in binary64, so the error stays at
// a few binary32 ulp (well below the fp16 hi/lo resolution of ~2^-22).
//
// Pixel strengths are scaled per chunk by an exact power of two (computed by
// k_chunk_scale) so that the largest maps into [2^14, 2^15) and fp16 keeps
// its relative precision for the small ones; the partial sum is scaled back
// exactly when it is written.
//
// Segments: a launch may cover only steps [seg_begin, seg_end) of every
// chunk.  The raw fp32 accumulators are then parked in the partial buffer
// and reloaded by the next segment, which makes the result independent of
// how a chunk is split into segments.
#include "rs_device.h"

#include <mutex>

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kKP = 16;        // pixels per step (two K=16 matrix steps)
constexpr int kPB = 256;       // pixels per parameter block
constexpr int kSPB = kPB / kKP;  // steps per parameter block
constexpr int kCS = 80;        // bytes per LDS column: 16 px * 2 halves * 2 B + 16 B pad
constexpr int kAmpExp = 14;    // largest scaled strength in [2^14, 2^15)

struct __align__(16) pix_par {
    double psi_f;         // frac(R Kc)
    double b;             // R Kb, cycles per fast-time sample
    double beta;          // v Kd, cycles per block
    float e32x, e32y;     // exp(j2pi frac(32 b)): rotation by 32 rows
    float s16x, s16y;     // exp(j2pi frac(16 beta)): rotation by 16 blocks
    float a;              // scaled strength
    float pad_;
};

template <int WN, int TL>
struct mfma_smem {
    static constexpr int NCOL = 2 * TL;
    char d[2][2][NCOL * kCS];   // [buffer][hi, lo][column][pixel-in-step][slot]
    pix_par par[2][kPB];
    int64_t item;
};

__device__ __forceinline__ unsigned pack2(_Float16 a, _Float16 b)
{
    half2v v = {a, b};
    return __builtin_bit_cast(unsigned, v);
}

__device__ __forceinline__ float frac32(double v) { return (float)rs_frac(v); }

template <int WN, int TL>
__global__ __launch_bounds__(256, 1) void k_mfma_split16(rs_launch Lc)
{
    constexpr int RB = WN / 32;          // 32-row blocks per wave
    constexpr int CB = 2 * TL / 32;      // 32-column blocks (re / im alternate)
    constexpr int TN = 4 * WN;
    constexpr int DPT = kKP * TL / 256;  // D phasors per thread per step
    extern __shared__ __align__(16) char smem_raw[];
    mfma_smem<WN, TL> &sm = *reinterpret_cast<mfma_smem<WN, TL> *>(smem_raw);

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int g = lane >> 5, li = lane & 31;

    bool first_item = true;
    for (;;) {
        const int64_t item = rs_next_item(Lc, &sm.item, first_item);
        first_item = false;
        if (item < 0) break;
        const int jidx = rs_find_job<RS_BY_ITEM>(Lc, item);
        const rs_job &J = rs_job_of(Lc, jidx);
        const rs_item it = rs_decode_item(J, J.item_first + (item - J.item_begin));
        const int n0 = it.nt * TN, l0 = it.lt * TL;
        const int64_t pb = (int64_t)it.s * J.chunk;
        const int64_t pe = min(J.P, pb + (int64_t)J.chunk);
        const int nsteps = (int)((pe - pb + kKP - 1) / kKP);
        const int nblocks = (nsteps + kSPB - 1) / kSPB;
        const int k0 = J.seg_begin;                 // multiple of kSPB
        const int k1 = min(J.seg_end, nsteps);
        if (k0 >= k1) continue;                      // chunk finished in an earlier segment
        const bool seg_first = k0 == 0, seg_last = k1 == nsteps;
        const int m = it.c / J.N, r = it.c % J.N;
        const double *tx = J.ant + 3 * m;
        const double *rx = J.ant + 3 * (J.M + r);
        const int sh = J.scale[it.s];
        const float a_scale = ldexpf(1.0f, sh);

        auto load_block = [&](int blk) {
            const int buf = blk & 1;
            for (int i = tid; i < kPB; i += 256) {
                const int64_t p = pb + (int64_t)blk * kPB + i;
                pix_par q;
                if (p < pe) {
                    rs_pixel_args a = rs_pixel(J, tx, rx, p);
                    q.psi_f = a.psi_f;
                    q.b = a.b;
                    q.beta = a.beta;
                    q.a = a.a * a_scale;
                } else {
                    q.psi_f = 0.0;
                    q.b = 0.0;
                    q.beta = 0.0;
                    q.a = 0.f;
                }
                const float fe = frac32(q.b * 32.0), fs = frac32(q.beta * 16.0);
                q.e32x = __builtin_amdgcn_cosf(fe);
                q.e32y = __builtin_amdgcn_sinf(fe);
                q.s16x = __builtin_amdgcn_cosf(fs);
                q.s16y = __builtin_amdgcn_sinf(fs);
                q.pad_ = 0.f;
                sm.par[buf][i] = q;
            }
        };

        const double nrow0 = (double)(n0 + wave * WN + li);

        // D phasors of step st -> LDS buffer st & 1.  Thread: pixel q, blocks
        // l = l0 + (tid >> 4) + 16 k; D = u - j w with u + j w = a exp(j2pi beta l).
        auto gen_d = [&](int st) {
            const int buf = (st / kSPB) & 1;
            const int q = tid & 15;
            const pix_par &pp = sm.par[buf][(st % kSPB) * kKP + q];
            const int lq = tid >> 4;
            const float f = frac32(pp.beta * (double)(l0 + lq));
            float u = pp.a * __builtin_amdgcn_cosf(f);
            float w = pp.a * __builtin_amdgcn_sinf(f);
            const float cx = pp.s16x, cy = pp.s16y;
            char *dh = sm.d[st & 1][0];
            char *dl = sm.d[st & 1][1];
#pragma unroll
            for (int k = 0; k < DPT; ++k) {
                const int ll = lq + 16 * k;
                const _Float16 uh = (_Float16)u, wh = (_Float16)w;
                const _Float16 ul = (_Float16)(u - (float)uh), wl = (_Float16)(w - (float)wh);
                const int colre = (ll >> 5) * 64 + (ll & 31);
                const int colim = colre + 32;
                *reinterpret_cast<unsigned *>(dh + colre * kCS + q * 4) = pack2(uh, wh);
                *reinterpret_cast<unsigned *>(dh + colim * kCS + q * 4) = pack2(-wh, uh);
                *reinterpret_cast<unsigned *>(dl + colre * kCS + q * 4) = pack2(ul, wl);
                *reinterpret_cast<unsigned *>(dl + colim * kCS + q * 4) = pack2(-wl, ul);
                const float un = u * cx - w * cy;
                w = u * cy + w * cx;
                u = un;
            }
        };

        float2 *part = reinterpret_cast<float2 *>(J.partial) +
                       ((int64_t)it.s * (J.M * J.N) + it.c) * (int64_t)J.L * J.Ns;

        f32x16 acc[RB][CB];
        if (seg_first) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[rb][cb][e] = 0.f;
        } else {
            // resume: raw accumulators parked by the previous segment
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int k = 0; k < CB / 2; ++k) {
                    const int l = l0 + 32 * k + li;
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int n = n0 + wave * WN + rb * 32 + 8 * (e >> 2) + 4 * g + (e & 3);
                        float2 v = make_float2(0.f, 0.f);
                        if (n < J.Ns && l < J.L) v = part[(int64_t)l * J.Ns + n];
                        acc[rb][2 * k][e] = v.x;
                        acc[rb][2 * k + 1][e] = v.y;
                    }
                }
        }

        // F phasors of step st, matrix step t only (see gen_f).
        auto gen_f_t = [&](int st, int t, half8 (&fh)[RB], half8 (&fl)[RB]) {
            const int buf = (st / kSPB) & 1;
            const int base = (st % kSPB) * kKP + 8 * t + 4 * g;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const pix_par &pp = sm.par[buf][base + j];
                const float f = frac32(pp.psi_f + rs_frac(pp.b * nrow0));
                float cv = __builtin_amdgcn_cosf(f);
                float sv = __builtin_amdgcn_sinf(f);
                const float ex = pp.e32x, ey = pp.e32y;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const _Float16 ch = (_Float16)cv, shh = (_Float16)sv;
                    fh[rb][2 * j] = ch;
                    fh[rb][2 * j + 1] = shh;
                    fl[rb][2 * j] = (_Float16)(cv - (float)ch);
                    fl[rb][2 * j + 1] = (_Float16)(sv - (float)shh);
                    if (rb + 1 < RB) {
                        const float cn = cv * ex - sv * ey;
                        sv = cv * ey + sv * ex;
                        cv = cn;
                    }
                }
            }
        };

        auto mfma_t = [&](int st, int t, const half8 (&fh)[RB], const half8 (&fl)[RB]) {
            const char *dh = sm.d[st & 1][0];
            const char *dl = sm.d[st & 1][1];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int off = (cb * 32 + li) * kCS + 32 * t + 16 * g;
                const half8 bh = *reinterpret_cast<const half8 *>(dh + off);
                const half8 bl = *reinterpret_cast<const half8 *>(dl + off);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fh[rb], bh, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fh[rb], bl, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fl[rb], bh, acc[rb][cb], 0, 0, 0);
                }
            }
        };

        // Operands of matrix step t: f0 (t = 0) and f1 (t = 1).  Each step
        // issues the matrix work of st while the next step's D (other LDS
        // buffer) and F (each half as soon as its registers are consumed)
        // are evaluated.  What is evaluated after the last step is unused.
        half8 f0h[RB], f0l[RB], f1h[RB], f1l[RB];
        __syncthreads();  // previous item's readers of the LDS buffers are done
        load_block(k0 / kSPB);
        __syncthreads();
        gen_d(k0);
        gen_f_t(k0, 0, f0h, f0l);
        gen_f_t(k0, 1, f1h, f1l);
        __syncthreads();
        for (int st = k0; st < k1; ++st) {
            if ((st % kSPB) == 0 && st / kSPB + 1 < nblocks) load_block(st / kSPB + 1);
            gen_d(st + 1);
            mfma_t(st, 0, f0h, f0l);
            gen_f_t(st + 1, 0, f0h, f0l);
            mfma_t(st, 1, f1h, f1l);
            gen_f_t(st + 1, 1, f1h, f1l);
            __syncthreads();
        }

        // ---- park or write the partial tile ---------------------------------
        const float osc = seg_last ? ldexpf(1.0f, -sh) : 1.0f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int k = 0; k < CB / 2; ++k) {
                const int l = l0 + 32 * k + li;
                if (l >= J.L) continue;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int n = n0 + wave * WN + rb * 32 + 8 * (e >> 2) + 4 * g + (e & 3);
                    if (n < J.Ns)
                        part[(int64_t)l * J.Ns + n] =
                            make_float2(acc[rb][2 * k][e] * osc, acc[rb][2 * k + 1][e] * osc);
                }
            }
    }
}

// Per-chunk strength scale: sh = 14 - floor(log2(max |a|)) so that the
// largest scaled strength of the chunk lies in [2^14, 2^15).
__global__ __launch_bounds__(256) void k_chunk_scale(rs_launch Lc)
{
    __shared__ float red[4];
    const int64_t gch = blockIdx.x;
    if (gch >= Lc.total) return;
    const int jidx = rs_find_job<RS_BY_CHUNK>(Lc, gch);
    const rs_job &J = rs_job_of(Lc, jidx);
    const int s = (int)(gch - J.chunk_begin);
    const int64_t pb = (int64_t)s * J.chunk;
    const int64_t pe = min(J.P, pb + (int64_t)J.chunk);
    float am = 0.f;
    for (int64_t p = pb + threadIdx.x; p < pe; p += 256) am = fmaxf(am, fabsf(J.amp[p]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) am = fmaxf(am, __shfl_xor(am, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = am;
    __syncthreads();
    if (threadIdx.x == 0) {
        am = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        int ex = (am > 0.f && am <= 3.4e38f) ? ilogbf(am) : kAmpExp;
        int sh = kAmpExp - ex;
        J.scale[s] = sh > 126 ? 126 : (sh < -126 ? -126 : sh);
    }
}

template <int WN, int TL>
void launch_one(const rs_launch &L, int grid, hipStream_t st)
{
    const size_t smem = sizeof(mfma_smem<WN, TL>);
    static std::once_flag once;
    std::call_once(once, [smem] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mfma_split16<WN, TL>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    });
    hipLaunchKernelGGL((k_mfma_split16<WN, TL>), dim3(grid), dim3(256), smem, st, L);
}

}  // namespace

void rs_launch_mfma(const rs_launch &L, int wn, int tl, int grid, hipStream_t st)
{
    if (tl == 64) {
        if (wn == 32) launch_one<32, 64>(L, grid, st);
        else if (wn == 64) launch_one<64, 64>(L, grid, st);
        else launch_one<128, 64>(L, grid, st);
    } else {
        if (wn == 32) launch_one<32, 128>(L, grid, st);
        else launch_one<64, 128>(L, grid, st);
    }
}

void rs_launch_chunk_scale(const rs_launch &L, hipStream_t st)
{
    if (L.total <= 0) return;
    hipLaunchKernelGGL(k_chunk_scale, dim3((unsigned)L.total), dim3(256), 0, st, L);
}
