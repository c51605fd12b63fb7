// Split-FP16 matrix-core form (gfx950, v_mfma_f32_32x32x16_f16).
//
// For one virtual channel c the cube is the complex contraction over pixels
//   Y_c[n][l] = sum_p F_c[p][n] * D[p][l]
//   F_c[p][n] = exp(j2pi (psi_{p,c} + b_{p,c} n))        unit magnitude
//   D[p][l]   = a_p exp(-j2pi beta_p l)                  shared by channels
// i.e. Y_c = F_c^T diag(sigma_c) D with the carrier phase of sigma folded into
// F (Sec. II, eq. (1) per channel, pixel sum of eq. (2)).  Phase arguments are
// evaluated and reduced mod 1 in binary64; the phasors in binary32 with the
// hardware sin/cos (input in revolutions); each binary32 value x is split
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
//           it feeds to the matrix core (registers only)
//   D     = B operand, evaluated once per workgroup per 16-pixel step into
//           double-buffered LDS (both column arrangements, hi and lo)
// Pixel strengths are scaled per chunk by an exact power of two so that the
// largest maps into [2^14, 2^15) (fp16 keeps its relative precision for the
// small ones); the partial sum is scaled back exactly before it is written.
#include "rs_device.h"

#include <mutex>

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kKP = 16;        // pixels per step (two K=16 matrix steps)
constexpr int kPB = 256;       // pixels per parameter block
constexpr int kCS = 80;        // bytes per LDS column: 16 px * 2 halves * 2 B + 16 B pad
constexpr int kAmpExp = 14;    // largest scaled strength in [2^14, 2^15)

struct __align__(16) pix_fd {
    double psi_f, b;
};

template <int WN, int TL>
struct mfma_smem {
    static constexpr int NCOL = 2 * TL;
    char d[2][2][NCOL * kCS];   // [buffer][hi, lo][column][pixel-in-step][slot]
    pix_fd fb[2][kPB];          // per parameter block: psi_f, b
    double beta[2][kPB];
    float amp[2][kPB];
    float red[4];
    int64_t item;
};

__device__ __forceinline__ unsigned pack2(_Float16 a, _Float16 b)
{
    half2v v = {a, b};
    return __builtin_bit_cast(unsigned, v);
}

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

    bool first = true;
    for (;;) {
        const int64_t item = rs_next_item(Lc, &sm.item, first);
        first = false;
        if (item < 0) break;
        const int jidx = rs_find_job<false>(Lc, item);
        const rs_job &J = rs_job_of(Lc, jidx);
        const rs_item it = rs_decode_item(J, J.item_first + (item - J.item_begin));
        const int n0 = it.nt * TN, l0 = it.lt * TL;
        const int64_t pb = (int64_t)it.s * J.chunk;
        const int64_t pe = min(J.P, pb + (int64_t)J.chunk);
        const int np = (int)(pe - pb);
        const int nsteps = (np + kKP - 1) / kKP;
        const int nblocks = (np + kPB - 1) / kPB;
        const int m = it.c / J.N, r = it.c % J.N;
        const double *tx = J.ant + 3 * m;
        const double *rx = J.ant + 3 * (J.M + r);

        // ---- chunk strength scale (exact power of two) ----------------------
        float am = 0.f;
        for (int64_t p = pb + tid; p < pe; p += 256) am = fmaxf(am, fabsf(J.amp[p]));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) am = fmaxf(am, __shfl_xor(am, o));
        __syncthreads();  // previous item's readers of sm.red are done
        if (lane == 0) sm.red[wave] = am;
        __syncthreads();
        am = fmaxf(fmaxf(sm.red[0], sm.red[1]), fmaxf(sm.red[2], sm.red[3]));
        int ex = (am > 0.f && am <= 3.4e38f) ? ilogbf(am) : kAmpExp;
        int sh = kAmpExp - ex;
        sh = sh > 126 ? 126 : (sh < -126 ? -126 : sh);
        const float a_scale = ldexpf(1.0f, sh);

        auto load_block = [&](int blk) {
            const int buf = blk & 1;
            for (int i = tid; i < kPB; i += 256) {
                const int64_t p = pb + (int64_t)blk * kPB + i;
                if (p < pe) {
                    rs_pixel_args a = rs_pixel(J, tx, rx, p);
                    sm.fb[buf][i].psi_f = a.psi_f;
                    sm.fb[buf][i].b = a.b;
                    sm.beta[buf][i] = a.beta;
                    sm.amp[buf][i] = a.a * a_scale;
                } else {
                    sm.fb[buf][i].psi_f = 0.0;
                    sm.fb[buf][i].b = 0.0;
                    sm.beta[buf][i] = 0.0;
                    sm.amp[buf][i] = 0.f;
                }
            }
        };

        // rows of this lane (A operand row = lane % 32)
        double nrow[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) nrow[rb] = (double)(n0 + wave * WN + rb * 32 + li);

        // D phasors of step st -> LDS buffer st & 1
        auto gen_d = [&](int st) {
            const int blk = st / (kPB / kKP), buf = blk & 1;
            const int q = tid & 15;
            const int pq = (st % (kPB / kKP)) * kKP + q;
            const double beta = sm.beta[buf][pq];
            const float a = sm.amp[buf][pq];
            char *dh = sm.d[st & 1][0];
            char *dl = sm.d[st & 1][1];
#pragma unroll 2
            for (int k = 0; k < DPT; ++k) {
                const int ll = (tid >> 4) + 16 * k;
                const double ph = rs_frac(beta * (double)(l0 + ll));
                const float f = (float)ph;
                const float u = a * __builtin_amdgcn_cosf(f);
                const float w = a * __builtin_amdgcn_sinf(f);
                const _Float16 uh = (_Float16)u, wh = (_Float16)w;
                const _Float16 ul = (_Float16)(u - (float)uh), wl = (_Float16)(w - (float)wh);
                const int colre = (ll >> 5) * 64 + (ll & 31);
                const int colim = colre + 32;
                *reinterpret_cast<unsigned *>(dh + colre * kCS + q * 4) = pack2(uh, wh);
                *reinterpret_cast<unsigned *>(dh + colim * kCS + q * 4) = pack2(-wh, uh);
                *reinterpret_cast<unsigned *>(dl + colre * kCS + q * 4) = pack2(ul, wl);
                *reinterpret_cast<unsigned *>(dl + colim * kCS + q * 4) = pack2(-wl, ul);
            }
        };

        // F phasors of matrix step t (pixels 8t + 4g .. 8t + 4g + 3 of step st)
        // for this lane's rows -> registers (hi, lo)
        auto gen_f = [&](int st, int t, half8 (&fh)[RB], half8 (&fl)[RB]) {
            const int blk = st / (kPB / kKP), buf = blk & 1;
            const int base = (st % (kPB / kKP)) * kKP + 8 * t + 4 * g;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const pix_fd pf = sm.fb[buf][base + j];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    double ph = pf.psi_f + rs_frac(pf.b * nrow[rb]);
                    ph = rs_frac(ph);
                    const float f = (float)ph;
                    const float cv = __builtin_amdgcn_cosf(f);
                    const float sv = __builtin_amdgcn_sinf(f);
                    const _Float16 ch = (_Float16)cv, shh = (_Float16)sv;
                    fh[rb][2 * j] = ch;
                    fh[rb][2 * j + 1] = shh;
                    fl[rb][2 * j] = (_Float16)(cv - (float)ch);
                    fl[rb][2 * j + 1] = (_Float16)(sv - (float)shh);
                }
            }
        };

        f32x16 acc[RB][CB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[rb][cb][e] = 0.f;

        if (nsteps > 0) {
            load_block(0);
            __syncthreads();
            half8 fh[2][RB], fl[2][RB];
            gen_d(0);
            gen_f(0, 0, fh[0], fl[0]);
            gen_f(0, 1, fh[1], fl[1]);
            __syncthreads();
            for (int st = 0; st < nsteps; ++st) {
                const int blk = st / (kPB / kKP);
                if ((st % (kPB / kKP)) == 0 && blk + 1 < nblocks) load_block(blk + 1);
                // Next step's D (into the other buffer) and F are evaluated
                // unconditionally so that the loop body stays one basic block
                // the scheduler can interleave with the matrix instructions;
                // after the last step they are simply not used.
                gen_d(st + 1);
                const char *dh = sm.d[st & 1][0];
                const char *dl = sm.d[st & 1][1];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        const int off = (cb * 32 + li) * kCS + 32 * t + 16 * g;
                        const half8 bh = *reinterpret_cast<const half8 *>(dh + off);
                        const half8 bl = *reinterpret_cast<const half8 *>(dl + off);
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb) {
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fh[t][rb], bh, acc[rb][cb], 0, 0, 0);
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fh[t][rb], bl, acc[rb][cb], 0, 0, 0);
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fl[t][rb], bh, acc[rb][cb], 0, 0, 0);
                        }
                    }
                    // the next step's operands for this matrix step, evaluated
                    // while the matrix cores drain the products above
                    gen_f(st + 1, t, fh[t], fl[t]);
                }
                __syncthreads();
            }
        }

        // ---- write the partial tile (strength scale undone exactly) ----------
        float2 *out = reinterpret_cast<float2 *>(J.partial) +
                      ((int64_t)it.s * (J.M * J.N) + it.c) * (int64_t)J.L * J.Ns;
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
                        out[(int64_t)l * J.Ns + n] = make_float2(ldexpf(acc[rb][2 * k][e], -sh),
                                                                 ldexpf(acc[rb][2 * k + 1][e], -sh));
                }
            }
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
