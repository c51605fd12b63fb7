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
// Tiling (workgroup = NW waves, NW/4 per SIMD):
//   item  = (channel, n tile of NW*WN rows, l tile of TL columns, pixel chunk)
//   wave  = WN rows x TL complex columns; WN/32 x 2TL/32 accumulator blocks
//   F     = A operand, evaluated by each lane for exactly the rows and pixels
//           it feeds to the matrix core (registers only: two sets in the
//           pipelined schedule, one in the phase-shifted one, where a wave
//           rewrites its F registers only around its own products)
//   D     = B operand, evaluated once per workgroup per 16-pixel step into
//           double-buffered LDS (both column arrangements, hi and lo; the
//           imaginary arrangement's split is the real one's times j)
// Two step schedules.  Phase-shifted waves (NW = 8): the two waves of a SIMD
// run their matrix and vector parts in opposite order, so the hardware
// interleaves one wave's matrix instructions with the other's phasor
// arithmetic.  Software-pipelined interleave (the other shapes, and NW = 8
// when the plan turns the phase shift off): every wave alternates one matrix
// group with one slice of vector work, the phasor evaluation cut into stages
// one slice apart so that no wave waits on its own vector results.
// Phasor cost: per pixel and lane one binary64-reduced phasor; the other rows
// of the lane follow by binary32 rotation with exp(j2pi frac(32 b)), and the
// slow-time phasors of a thread by rotation with exp(j2pi frac(LQ beta)), LQ
// the number of D threads per pixel (16 or 32) --
// every rotation factor is itself reduced in binary64, so the error stays at
// a few binary32 ulp (well below the fp16 hi/lo resolution of ~2^-22).
//
// Pixel strengths are scaled per chunk by an exact power of two (found by
// each work item from its chunk's strengths, or by k_chunk_scale for
// strengths per block) so that the largest maps into [2^14, 2^15) and fp16 keeps
// its relative precision for the small ones; the partial sum is scaled back
// exactly when it is written.
//
// Strengths per block (BS = true, jobs with amp_lstride != 0): D[p][l] =
// a_{p,l} exp(-j2pi beta_p l) is still one shared matrix per pixel chunk, so
// only its evaluation changes: the rotated phasor carries the chunk scale
// alone and each D entry is multiplied by its strength, read from global
// memory at the start of the step before it.  Jobs without per-block
// strengths in the same launch multiply by 1 (exact), so their cubes keep
// the bits of the launch without BS.
//
// Segments: a launch may cover only steps [seg_begin, seg_end) of every
// chunk.  The raw fp32 accumulators are then parked in the partial buffer
// and reloaded by the next segment, which makes the result independent of
// how a chunk is split into segments.
#include "rs_device.h"
#include "rs_split16.h"

#include <type_traits>

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
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
    float srx, sry;       // exp(j2pi frac(LQ beta)): rotation by LQ blocks
    float a;              // scaled strength
    float pad_;
};

typedef rs_half2v half2v;
__device__ __forceinline__ float frac32(double v) { return rs_frac32(v); }
__device__ __forceinline__ half2v hi2(float x, float y) { return rs_hi2(x, y); }
__device__ __forceinline__ half2v lo2(float x, float y, half2v h) { return rs_lo2(x, y, h); }
__device__ __forceinline__ unsigned bits(half2v v) { return rs_bits(v); }
__device__ __forceinline__ void pin(float &u, float &w) { rs_pin(u, w); }
__device__ __forceinline__ void rot(float &u, float &w, float rx, float ry) { rs_rot(u, w, rx, ry); }

// Both column arrangements of a D entry u + j w, real (u, w) and imaginary
// (-w, u), each split into hi and lo; the imaginary pair is the real one
// times j (rs_jmul), which saves a conversion and two mixed multiply-adds.
__device__ __forceinline__ void d_split(float u, float w, half2v &hre, half2v &him, half2v &lre, half2v &lim)
{
    hre = hi2(u, w);
    lre = lo2(u, w, hre);
    him = rs_jmul(hre);
    lim = rs_jmul(lre);
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

typedef std::integral_constant<int, 0> buf0_t;
typedef std::integral_constant<int, 1> buf1_t;

template <int WN, int TL, int NW, bool PHASE, bool BS>
__global__ __launch_bounds__(64 * NW, 1) void k_mfma_split16(rs_launch Lc)
{
    constexpr int NT = 64 * NW;          // threads per workgroup
    constexpr int RB = WN / 32;          // 32-row blocks per wave
    constexpr int CB = 2 * TL / 32;      // 32-column blocks (re / im alternate)
    constexpr int TN = NW * WN;          // tile rows
    constexpr int LQ = NT / 16;          // D threads per pixel (blocks l = lq + LQ k)
    constexpr int DPT = TL / LQ;         // D phasors per thread per step
    static_assert(LQ == 16 || LQ == 32, "D column mapping assumes 16 or 32 threads per pixel");
    static_assert(DPT >= 1 && DPT * LQ == TL, "TL must be a multiple of the D thread count");
    // Separate LDS objects for the two D buffers: the compiler then knows
    // that the next step's D stores never alias the operands being read.
    constexpr int DBYTES = 2 * TL * kCS;
    __shared__ __align__(16) char sD0[2][DBYTES];  // [hi, lo]
    __shared__ __align__(16) char sD1[2][DBYTES];
    __shared__ pix_par sPar[2][kPB];
    __shared__ rs_item_consts sK;
    __shared__ int64_t sItem;
    __shared__ float sRed[NW];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int g = lane >> 5, li = lane & 31;

    bool first_item = true;
    for (;;) {
        const int64_t item = rs_next_item(Lc, &sItem, first_item);
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
        const bool full_tile = n0 + TN <= J.Ns && l0 + TL <= J.L;
        const int m = it.c / J.N, r = it.c % J.N;
        // strength exponent shift of the chunk: from k_chunk_scale where the
        // job has a scale array (strengths per block), else found below
        int sh = J.scale ? J.scale[it.s] : 0;
        float a_scale = 1.0f;
        const bool per_block = BS && J.amp_lstride != 0;
        // every reader of the previous item's sK has passed a barrier since
        if (tid == 0) rs_item_consts_of(J, m, r, sK);

        // ---- pixel parameter blocks (256 pixels), raw data prefetched one
        // block ahead so that the global-memory latency stays hidden.  The
        // loads are unconditional (index clamped into the chunk) and their
        // validity is decided when the block is used: a conditional zero
        // would make the compiler wait for the loads right away. ----------
        float rxp, ryp, rzp, rap, rvp;
        auto fetch_block = [&](int blk) {
            if (tid < kPB) {
                const int64_t p = min(pb + (int64_t)blk * kPB + tid, pe - 1);
                rxp = rs_gload(sK.x, p);
                ryp = rs_gload(sK.y, p);
                rzp = rs_gload(sK.z, p);
                rap = rs_gload(sK.amp, p);
                rvp = rs_gload(sK.vr, p);
            }
        };
        auto load_block = [&](int blk) {
            if (tid < kPB) {
                const int64_t p = pb + (int64_t)blk * kPB + tid;
                pix_par q;
                if (p < pe) {
                    double psi;
                    rs_chan_args(sK, rxp, ryp, rzp, rvp, m, sK.tx, sK.rx, &psi, &q.b, &q.beta);
                    q.psi_f = rs_frac(psi);
                    q.a = per_block ? a_scale : rap * a_scale;
                } else {
                    q.psi_f = 0.0;
                    q.b = 0.0;
                    q.beta = 0.0;
                    q.a = 0.f;
                }
                const float fe = frac32(q.b * 32.0), fs = frac32(q.beta * (double)LQ);
                q.e32x = __builtin_amdgcn_cosf(fe);
                q.e32y = __builtin_amdgcn_sinf(fe);
                q.srx = __builtin_amdgcn_cosf(fs);
                q.sry = __builtin_amdgcn_sinf(fs);
                q.pad_ = 0.f;
                sPar[blk & 1][tid] = q;
            }
            fetch_block(blk + 1);
        };

        const double nrow0 = (double)(n0 + wave * WN + li);
        // D thread mapping: pixel q = lane % 16; block group lq such that the
        // four lq of one wave are 4 columns apart (80-byte columns: their
        // 16-dword write runs then fall into disjoint LDS banks)
        const int q = lane & 15;
        const int lq = (lane >> 4) * 4 + (wave & 3) + 16 * (wave >> 2);

        // D phasors of step st -> LDS buffer dbuf, all at once (prologue).
        // Thread: pixel q, blocks l = l0 + lq + LQ k; D = u - j w with
        // u + j w = a exp(j2pi beta l); real column (u, w), imaginary (-w, u).
        auto d_column = [](int k) { return ((LQ * k) >> 5) * 64 + ((LQ * k) & 31); };
        // strengths of this thread's D entries of step st (1 where the job
        // has none per block, or the pixel or block lies past the end)
        auto load_al = [&](int st, float (&al)[DPT]) {
            const int64_t p = pb + (int64_t)st * kKP + q;
#pragma unroll
            for (int k = 0; k < DPT; ++k) {
                const int l = l0 + lq + LQ * k;
                al[k] = per_block && p < pe && l < sK.L ? rs_gload(sK.amp, p + (int64_t)l * sK.amp_lstride) : 1.0f;
            }
        };
        // D entry (u, w) times its strength, pinned
        auto scaled = [&](float u, float w, float a, float &su, float &sw) {
            su = u * a;
            sw = w * a;
            pin(su, sw);
        };
        auto gen_d = [&](int st, auto dbuf) {
            const pix_par &pp = sPar[(st / kSPB) & 1][(st % kSPB) * kKP + q];
            float al[DPT];
            if constexpr (BS) load_al(st, al);
            const float f = frac32(pp.beta * (double)(l0 + lq));  // binary64 reduction
            float u = pp.a * __builtin_amdgcn_cosf(f);
            float w = pp.a * __builtin_amdgcn_sinf(f);
            pin(u, w);
            char (&db)[2][DBYTES] = decltype(dbuf)::value ? sD1 : sD0;
            char *dh = db[0] + lq * kCS + q * 4;
            char *dl = db[1] + lq * kCS + q * 4;
#pragma unroll
            for (int k = 0; k < DPT; ++k) {
                float su = u, sw = w;
                if constexpr (BS) scaled(u, w, al[k], su, sw);
                half2v hre, him, lre, lim;
                d_split(su, sw, hre, him, lre, lim);
                const int cre = d_column(k) * kCS, cim = cre + 32 * kCS;
                *reinterpret_cast<unsigned *>(dh + cre) = bits(hre);
                *reinterpret_cast<unsigned *>(dh + cim) = bits(him);
                *reinterpret_cast<unsigned *>(dl + cre) = bits(lre);
                *reinterpret_cast<unsigned *>(dl + cim) = bits(lim);
                rot(u, w, pp.srx, pp.sry);
            }
        };

        // One F pixel (matrix step ft, pixel j of the lane's group of four)
        // of step st for every row block of this lane -> hi and lo operands,
        // from the pixel's phase parameters (psi_f, b).
        struct fops {
            half8 h[2][RB], l[2][RB];
        };
        auto gen_f_reg = [&](int st, int ft, int j, double psi_f, double b, fops &fo) {
            const float f = frac32(__builtin_fma(b, nrow0, psi_f));
            float cv = __builtin_amdgcn_cosf(f);
            float sv = __builtin_amdgcn_sinf(f);
            float ex = 0.f, ey = 0.f;
            if constexpr (RB > 1) {
                const pix_par &pf = sPar[(st / kSPB) & 1][(st % kSPB) * kKP + 8 * ft + 4 * g + j];
                ex = pf.e32x;
                ey = pf.e32y;
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const half2v h = hi2(cv, sv);
                u32x4 vh = __builtin_bit_cast(u32x4, fo.h[ft][rb]);
                u32x4 vl = __builtin_bit_cast(u32x4, fo.l[ft][rb]);
                vh[j] = bits(h);
                vl[j] = bits(lo2(cv, sv, h));
                fo.h[ft][rb] = __builtin_bit_cast(half8, vh);
                fo.l[ft][rb] = __builtin_bit_cast(half8, vl);
                if (rb + 1 < RB) rot(cv, sv, ex, ey);
            }
        };
        auto gen_f_pixel = [&](int st, int ft, int j, fops &fo) {
            const pix_par &pf = sPar[(st / kSPB) & 1][(st % kSPB) * kKP + 8 * ft + 4 * g + j];
            gen_f_reg(st, ft, j, pf.psi_f, pf.b, fo);
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
            int rli = li, rg = g;
            asm volatile("" : "+v"(rli), "+v"(rg));
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int k = 0; k < CB / 2; ++k) {
                    const int l = l0 + 32 * k + rli;
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int n = n0 + wave * WN + rb * 32 + 8 * (e >> 2) + 4 * rg + (e & 3);
                        float2 v = make_float2(0.f, 0.f);
                        if (n < J.Ns && l < J.L) v = part[(int64_t)l * J.Ns + n];
                        acc[rb][2 * k][e] = v.x;
                        acc[rb][2 * k + 1][e] = v.y;
                    }
                }
        }

        // One step, written as an explicit software pipeline.  Matrix part:
        // NG = 2 CB groups, each the RB x 3 products of one column block and
        // one 16-deep matrix step, with its B operands (hi, lo) loaded kBD
        // groups ahead into a ring of registers; a scheduling fence after
        // every group keeps the loads where they are.  Vector part: NG
        // slices, the D phasors of the next step (into the other LDS buffer)
        // and the F pixels of step fstep (into fn).
        //   Phase-shifted waves (NW = 8): the two waves of a SIMD run the two
        // parts in opposite order, so one issues matrix instructions while
        // the other evaluates phasors.  The first wave evaluates F of the
        // next step after its products, the second F of the current step
        // before them; either way the F registers are dead when they are
        // rewritten, so one set suffices.  The vector part first issues all
        // its parameter reads (the D pixel's and the eight F pixels') and
        // only then starts the arithmetic, so that it waits for LDS once
        // instead of once per pixel pair; in the first wave that is after
        // its products, which then start right after the barrier.  (Without
        // the phase shift the steps run step_pipe below.)
        // What is evaluated after the last step is never used.
        constexpr int NG = 2 * CB;                  // groups per step
        constexpr int FG = NG - DPT;                // slices evaluating F
        constexpr int FPG = (8 + FG - 1) / FG;      // F pixels per such slice
        constexpr bool kShift = NW == 8 && PHASE;
        constexpr int kBD = kShift ? 2 : 1;         // B prefetch distance in groups
        auto step = [&](int st, auto cur, auto nxt, const fops &fc, fops &fn, int fstep) {
            if ((st % kSPB) == 0 && st / kSPB + 1 < nblocks) load_block(st / kSPB + 1);
            const int s1 = st + 1;
            float al[DPT];
            if constexpr (BS) load_al(s1, al);
            // parameters of the vector part, all read from LDS before any of
            // its arithmetic: D of step s1, F pixels of step fstep
            double dbeta = 0.0, fpsi[8], fbb[8];
            float da = 0.f, cx = 0.f, cy = 0.f, u = 0.f, w = 0.f;
            auto fetch = [&] {
                const pix_par &pd = sPar[(s1 / kSPB) & 1][(s1 % kSPB) * kKP + q];
                dbeta = pd.beta;
                da = pd.a;
                cx = pd.srx;
                cy = pd.sry;
#pragma unroll
                for (int fp = 0; fp < 8; ++fp) {
                    const pix_par &pf = sPar[(fstep / kSPB) & 1][(fstep % kSPB) * kKP + 8 * (fp >> 2) + 4 * g + (fp & 3)];
                    fpsi[fp] = pf.psi_f;
                    fbb[fp] = pf.b;
                }
            };
            auto d_start = [&] {
                const float fd = frac32(dbeta * (double)(l0 + lq));
                u = da * __builtin_amdgcn_cosf(fd);
                w = da * __builtin_amdgcn_sinf(fd);
                pin(u, w);
            };
            char (&dbn)[2][DBYTES] = decltype(nxt)::value ? sD1 : sD0;
            char *dwh = dbn[0] + lq * kCS + q * 4;
            char *dwl = dbn[1] + lq * kCS + q * 4;
            // lane offset through an empty asm statement: the per-block
            // constants then fold into the LDS instructions' offset fields
            int lo = li * kCS + 16 * g;
            asm volatile("" : "+v"(lo));
            const char (&dbc)[2][DBYTES] = decltype(cur)::value ? sD1 : sD0;
            const char *drh = dbc[0] + lo;
            const char *drl = dbc[1] + lo;
            auto boff = [](int gi) { return (gi % CB) * 32 * kCS + 32 * (gi / CB); };
            half8 bh[kBD + 1], bl[kBD + 1];
            auto load_b = [&](int gi) {
                bh[gi % (kBD + 1)] = *reinterpret_cast<const half8 *>(drh + boff(gi));
                bl[gi % (kBD + 1)] = *reinterpret_cast<const half8 *>(drl + boff(gi));
            };
            auto mfma_group = [&](int gi) {
                if (gi + kBD < NG) load_b(gi + kBD);
                const int t = gi / CB, cb = gi % CB;
                const half8 h = bh[gi % (kBD + 1)], l = bl[gi % (kBD + 1)];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fc.h[t][rb], h, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fc.h[t][rb], l, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fc.l[t][rb], h, acc[rb][cb], 0, 0, 0);
                }
            };
            auto mfma_prologue = [&] {
#pragma unroll
                for (int gi = 0; gi < kBD && gi < NG; ++gi) load_b(gi);
            };
            auto valu_slice = [&](int gi) {
                if (gi < DPT) {
                    float su = u, sw = w;
                    if constexpr (BS) scaled(u, w, al[gi], su, sw);
                    half2v hre, him, lre, lim;
                    d_split(su, sw, hre, him, lre, lim);
                    const int cre = d_column(gi) * kCS, cim = cre + 32 * kCS;
                    *reinterpret_cast<unsigned *>(dwh + cre) = bits(hre);
                    *reinterpret_cast<unsigned *>(dwh + cim) = bits(him);
                    *reinterpret_cast<unsigned *>(dwl + cre) = bits(lre);
                    *reinterpret_cast<unsigned *>(dwl + cim) = bits(lim);
                    rot(u, w, cx, cy);
                } else {
#pragma unroll
                    for (int k8 = 0; k8 < FPG; ++k8) {
                        const int fp = (gi - DPT) * FPG + k8;  // F pixel 0..7 of step fstep
                        if (fp < 8) gen_f_reg(fstep, fp >> 2, fp & 3, fpsi[fp], fbb[fp], fn);
                    }
                }
            };
            if (wave >= 4) {
                // second wave of each SIMD: phasor work first, then the
                // matrix work, so that it complements the first wave (with
                // strengths per block the F slices go first, giving the
                // strength loads time to arrive)
                fetch();
                __builtin_amdgcn_sched_barrier(0);
                d_start();
#pragma unroll
                for (int i = 0; i < NG; ++i) valu_slice(BS ? (i + DPT) % NG : i);
                __builtin_amdgcn_sched_barrier(0);
                mfma_prologue();
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) {
                    mfma_group(gi);
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                mfma_prologue();
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) {
                    mfma_group(gi);
                    __builtin_amdgcn_sched_barrier(0);
                }
                fetch();
                __builtin_amdgcn_sched_barrier(0);
                d_start();
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) valu_slice(gi);
            }
            __syncthreads();
        };

        // Software-pipelined interleave (no phase shift): every wave runs the
        // same stream, one matrix group then one vector slice.  The vector
        // work of the next step is cut into stages -- the pixel parameters
        // read from LDS, the binary64 phase, the sin / cos, the split and the
        // store -- and each stage sits one slice after the one producing its
        // operands, so that a wave never waits on its own vector results and
        // the matrix instructions of the two waves of a SIMD keep the matrix
        // core busy.  F pixel fp starts in slice f_slot(fp) and D entry k is
        // split and stored in slice d_slot(k); the phasors and their bits are
        // those of gen_f_pixel and gen_d.
        auto step_pipe = [&](int st, auto cur, auto nxt, const fops &fc, fops &fn) {
            if ((st % kSPB) == 0 && st / kSPB + 1 < nblocks) load_block(st / kSPB + 1);
            const int s1 = st + 1;
            const pix_par *ps1 = &sPar[(s1 / kSPB) & 1][(s1 % kSPB) * kKP];
            float al[DPT];
            if constexpr (BS) load_al(s1, al);
            char (&dbn)[2][DBYTES] = decltype(nxt)::value ? sD1 : sD0;
            char *dwh = dbn[0] + lq * kCS + q * 4;
            char *dwl = dbn[1] + lq * kCS + q * 4;
            int lo = li * kCS + 16 * g;
            asm volatile("" : "+v"(lo));
            const char (&dbc)[2][DBYTES] = decltype(cur)::value ? sD1 : sD0;
            const char *drh = dbc[0] + lo;
            const char *drl = dbc[1] + lo;
            constexpr int kBD = 1;
            auto boff = [](int gi) { return (gi % CB) * 32 * kCS + 32 * (gi / CB); };
            half8 bh[kBD + 1], bl[kBD + 1];
            auto load_b = [&](int gi) {
                bh[gi % (kBD + 1)] = *reinterpret_cast<const half8 *>(drh + boff(gi));
                bl[gi % (kBD + 1)] = *reinterpret_cast<const half8 *>(drl + boff(gi));
            };
            auto mfma_group = [&](int gi) {
                if (gi + kBD < NG) load_b(gi + kBD);
                const int t = gi / CB, cb = gi % CB;
                const half8 h = bh[gi % (kBD + 1)], l = bl[gi % (kBD + 1)];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fc.h[t][rb], h, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fc.h[t][rb], l, acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fc.l[t][rb], h, acc[rb][cb], 0, 0, 0);
                }
            };
            static_assert(NG >= 8, "the pipelined schedule needs 8 slices");
            // stage registers (indices are compile-time: registers, live only
            // between their stages)
            double dbeta = 0.0;
            float da = 0.f, dcx = 0.f, dcy = 0.f, dfr = 0.f, u = 0.f, w = 0.f;
            double fpsi[8], fbb[8];
            float fex[8], fey[8], fph[8], fcv[8], fsv[8];
            auto f_slot = [](int fp) { return (fp * (NG - 3)) / 8; };
            auto d_slot = [](int k) { return 3 + (k * (NG - 4)) / DPT; };
            auto slice = [&](int gi) {
                // D: parameters, binary64 phase, sin / cos, then the entries
                if (gi == 0) {
                    const pix_par &pd = ps1[q];
                    dbeta = pd.beta;
                    da = pd.a;
                    dcx = pd.srx;
                    dcy = pd.sry;
                }
                if (gi == 1) dfr = frac32(dbeta * (double)(l0 + lq));
                if (gi == 2) {
                    u = da * __builtin_amdgcn_cosf(dfr);
                    w = da * __builtin_amdgcn_sinf(dfr);
                    pin(u, w);
                }
#pragma unroll
                for (int k = 0; k < DPT; ++k) {
                    if (gi != d_slot(k)) continue;
                    float su = u, sw = w;
                    if constexpr (BS) scaled(u, w, al[k], su, sw);
                    half2v hre, him, lre, lim;
                    d_split(su, sw, hre, him, lre, lim);
                    const int cre = d_column(k) * kCS, cim = cre + 32 * kCS;
                    *reinterpret_cast<unsigned *>(dwh + cre) = bits(hre);
                    *reinterpret_cast<unsigned *>(dwh + cim) = bits(him);
                    *reinterpret_cast<unsigned *>(dwl + cre) = bits(lre);
                    *reinterpret_cast<unsigned *>(dwl + cim) = bits(lim);
                    if (k + 1 < DPT) rot(u, w, dcx, dcy);
                }
                // F of step s1: stages of earlier pixels first
#pragma unroll
                for (int fp = 0; fp < 8; ++fp) {
                    const int s0 = f_slot(fp), ft = fp >> 2, j = fp & 3;
                    if (gi == s0 + 3) {
                        float cv = fcv[fp], sv = fsv[fp];
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb) {
                            const half2v h = hi2(cv, sv);
                            u32x4 vh = __builtin_bit_cast(u32x4, fn.h[ft][rb]);
                            u32x4 vl = __builtin_bit_cast(u32x4, fn.l[ft][rb]);
                            vh[j] = bits(h);
                            vl[j] = bits(lo2(cv, sv, h));
                            fn.h[ft][rb] = __builtin_bit_cast(half8, vh);
                            fn.l[ft][rb] = __builtin_bit_cast(half8, vl);
                            if (rb + 1 < RB) rot(cv, sv, fex[fp], fey[fp]);
                        }
                    }
                    if (gi == s0 + 2) {
                        fcv[fp] = __builtin_amdgcn_cosf(fph[fp]);
                        fsv[fp] = __builtin_amdgcn_sinf(fph[fp]);
                    }
                    if (gi == s0 + 1) fph[fp] = frac32(__builtin_fma(fbb[fp], nrow0, fpsi[fp]));
                    if (gi == s0) {
                        const pix_par &pf = ps1[8 * ft + 4 * g + j];
                        fpsi[fp] = pf.psi_f;
                        fbb[fp] = pf.b;
                        if constexpr (RB > 1) {
                            fex[fp] = pf.e32x;
                            fey[fp] = pf.e32y;
                        }
                    }
                }
            };
#pragma unroll
            for (int gi = 0; gi < kBD; ++gi) load_b(gi);
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                mfma_group(gi);
                slice(gi);
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
        };

        // The chunk's exponent shift sh = 14 - floor(log2(max |a|)), as
        // k_chunk_scale computes it, found by the item itself while the first
        // parameter block is in flight (every item of the chunk finds the
        // same value).
        auto chunk_shift = [&]() {
            float am = 0.f;
            for (int64_t p = pb + tid; p < pe; p += NT) am = fmaxf(am, fabsf(rs_gload(sK.amp, p)));
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) am = fmaxf(am, __shfl_xor(am, o));
            if (lane == 0) sRed[wave] = am;
            __syncthreads();
            am = sRed[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) am = fmaxf(am, sRed[w]);
            const int ex = (am > 0.f && am <= 3.4e38f) ? ilogbf(am) : kAmpExp;
            const int v = kAmpExp - ex;
            return v > 126 ? 126 : (v < -126 ? -126 : v);
        };

        fops fa, fb;
        __syncthreads();  // previous item's readers of the LDS buffers are done
        fetch_block(k0 / kSPB);
        if (!J.scale) sh = chunk_shift();
        a_scale = ldexpf(1.0f, sh);
        load_block(k0 / kSPB);
        __syncthreads();
        gen_d(k0, buf0_t{});  // k0 is even: buffer 0
        if (!kShift || wave < 4) {
#pragma unroll
            for (int fp = 0; fp < 8; ++fp) gen_f_pixel(k0, fp >> 2, fp & 3, fa);
        }
        __syncthreads();
        if constexpr (kShift) {
            const int fofs = wave < 4 ? 1 : 0;  // F of the next step / of this step
            for (int st = k0; st < k1; st += 2) {
                step(st, buf0_t{}, buf1_t{}, fa, fa, st + fofs);
                if (st + 1 >= k1) break;
                step(st + 1, buf1_t{}, buf0_t{}, fa, fa, st + 1 + fofs);
            }
        } else {
            for (int st = k0; st < k1; st += 2) {
                step_pipe(st, buf0_t{}, buf1_t{}, fa, fb);
                if (st + 1 >= k1) break;
                step_pipe(st + 1, buf1_t{}, buf0_t{}, fb, fa);
            }
        }

        // ---- park or write the partial tile ---------------------------------
        // Lane coordinates pass through an empty asm statement so that the
        // store addresses are computed here, not hoisted above the step loop.
        int wli = li, wg = g;
        asm volatile("" : "+v"(wli), "+v"(wg));
        auto wn_of = [&](int rb, int e) { return n0 + wave * WN + rb * 32 + 8 * (e >> 2) + 4 * wg + (e & 3); };
        const float osc = seg_last ? ldexpf(1.0f, -sh) : 1.0f;
        if (full_tile) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int k = 0; k < CB / 2; ++k) {
                    float2 *row = part + (int64_t)(l0 + 32 * k + wli) * J.Ns;
#pragma unroll
                    for (int e = 0; e < 16; ++e)
                        row[wn_of(rb, e)] = make_float2(acc[rb][2 * k][e] * osc, acc[rb][2 * k + 1][e] * osc);
                }
        } else {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int k = 0; k < CB / 2; ++k) {
                    const int l = l0 + 32 * k + wli;
                    if (l >= J.L) continue;
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int n = wn_of(rb, e);
                        if (n < J.Ns)
                            part[(int64_t)l * J.Ns + n] =
                                make_float2(acc[rb][2 * k][e] * osc, acc[rb][2 * k + 1][e] * osc);
                    }
                }
        }
    }
}

// Largest |a| over 256 threads (every thread gets it).
__device__ __forceinline__ float block_max(float am, float *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) am = fmaxf(am, __shfl_xor(am, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = am;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Row groups of the strengths-per-block maximum: block l belongs to group
// l mod G.  G <= L keeps the G floats per chunk inside the chunk's share of
// the partial-sum buffer (C L Ns complex entries).
__device__ __forceinline__ int row_groups(const rs_job &J) { return min(16, J.L); }

// Strengths per block: the maximum of |a_{p,l}| over the pixels of a chunk
// and the blocks of one row group (blockIdx.y), written to the job's
// partial-sum buffer, which the main kernel overwrites only later.  Jobs
// without strengths per block are skipped.
__global__ __launch_bounds__(256) void k_chunk_rowmax(rs_launch Lc)
{
    __shared__ float red[4];
    const int64_t gch = blockIdx.x;
    if (gch >= Lc.total) return;
    const int jidx = rs_find_job<RS_BY_CHUNK>(Lc, gch);
    const rs_job &J = rs_job_of(Lc, jidx);
    const int G = row_groups(J);
    const int grp = blockIdx.y;
    if (J.amp_lstride == 0 || grp >= G) return;
    const int s = (int)(gch - J.chunk_begin);
    const int64_t pb = (int64_t)s * J.chunk;
    const int64_t pe = min(J.P, pb + (int64_t)J.chunk);
    float am = 0.f;
    for (int l = grp; l < J.L; l += G) {
        const float *a = J.amp + (int64_t)l * J.amp_lstride;
        for (int64_t p = pb + threadIdx.x; p < pe; p += 256) am = fmaxf(am, fabsf(rs_gload(a, p)));
    }
    am = block_max(am, red);
    if (threadIdx.x == 0) reinterpret_cast<float *>(J.partial)[(int64_t)s * G + grp] = am;
}

// Per-chunk strength scale: sh = 14 - floor(log2(max |a|)) so that the
// largest scaled strength of the chunk (over all blocks when strengths vary
// per block: the row-group maxima left by k_chunk_rowmax) lies in
// [2^14, 2^15).  Only jobs with strengths per block carry a scale array
// (the L x P strengths are too many to scan inside each work item); the
// main kernel finds the shift of the others itself.
__global__ __launch_bounds__(256) void k_chunk_scale(rs_launch Lc)
{
    __shared__ float red[4];
    const int64_t gch = blockIdx.x;
    if (gch >= Lc.total) return;
    const int jidx = rs_find_job<RS_BY_CHUNK>(Lc, gch);
    const rs_job &J = rs_job_of(Lc, jidx);
    if (!J.scale) return;  // the main kernel finds this job's shifts itself
    const int s = (int)(gch - J.chunk_begin);
    const int64_t pb = (int64_t)s * J.chunk;
    const int64_t pe = min(J.P, pb + (int64_t)J.chunk);
    float am = 0.f;
    if (J.amp_lstride) {
        const int G = row_groups(J);
        if ((int)threadIdx.x < G) am = reinterpret_cast<const float *>(J.partial)[(int64_t)s * G + threadIdx.x];
    } else {
        for (int64_t p = pb + threadIdx.x; p < pe; p += 256) am = fmaxf(am, fabsf(J.amp[p]));
    }
    am = block_max(am, red);
    if (threadIdx.x == 0) {
        int ex = (am > 0.f && am <= 3.4e38f) ? ilogbf(am) : kAmpExp;
        int sh = kAmpExp - ex;
        J.scale[s] = sh > 126 ? 126 : (sh < -126 ? -126 : sh);
    }
}

// interleave: the software-pipelined schedule for NW = 8 too (shapes with
// NW = 4 always use it)
template <int WN, int TL, int NW, bool BS>
void launch_one(const rs_launch &L, bool interleave, int grid, hipStream_t st)
{
    if (NW == 8 && !interleave)
        hipLaunchKernelGGL((k_mfma_split16<WN, TL, NW, true, BS>), dim3(grid), dim3(64 * NW), 0, st, L);
    else
        hipLaunchKernelGGL((k_mfma_split16<WN, TL, NW, false, BS>), dim3(grid), dim3(64 * NW), 0, st, L);
}

template <bool BS>
void launch_shape(const rs_launch &L, int wn, int tl, int nw, bool interleave, int grid, hipStream_t st)
{
    if (tl == 128) {
        if (wn == 64) launch_one<64, 128, 4, BS>(L, interleave, grid, st);
        else if (nw == 8) launch_one<32, 128, 8, BS>(L, interleave, grid, st);
        else launch_one<32, 128, 4, BS>(L, interleave, grid, st);
    } else {
        if (wn == 32 && nw == 8) launch_one<32, 64, 8, BS>(L, interleave, grid, st);
        else if (wn == 32) launch_one<32, 64, 4, BS>(L, interleave, grid, st);
        else if (wn == 64 && nw == 8) launch_one<64, 64, 8, BS>(L, interleave, grid, st);
        else if (wn == 64) launch_one<64, 64, 4, BS>(L, interleave, grid, st);
        else launch_one<128, 64, 4, BS>(L, interleave, grid, st);
    }
}

}  // namespace

// Tile shapes built into the library: rows per wave x columns x waves.
bool rs_mfma_shape_supported(int wn, int tl, int nw)
{
    return (tl == 128 && ((wn == 64 && nw == 4) || (wn == 32 && (nw == 4 || nw == 8)))) ||
           (tl == 64 && ((wn == 32 && (nw == 4 || nw == 8)) || (wn == 64 && (nw == 4 || nw == 8)) ||
                         (wn == 128 && nw == 4)));
}

void rs_launch_mfma(const rs_launch &L, int wn, int tl, int nw, bool interleave, bool block_strength, int grid,
                    hipStream_t st)
{
    if (block_strength)
        launch_shape<true>(L, wn, tl, nw, interleave, grid, st);
    else
        launch_shape<false>(L, wn, tl, nw, interleave, grid, st);
}

void rs_launch_chunk_scale(const rs_launch &L, bool block_strength, hipStream_t st)
{
    if (L.total <= 0) return;
    if (block_strength) hipLaunchKernelGGL(k_chunk_rowmax, dim3((unsigned)L.total, 16), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_chunk_scale, dim3((unsigned)L.total), dim3(256), 0, st, L);
}
