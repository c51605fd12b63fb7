// NUFFT form: the cube as one two-dimensional type-1 non-uniform FFT per
// virtual channel (gfx950).
//
// Per channel c the sum of Sec. II (eq. (1) per channel, pixel sum of
// eq. (2)) is
//   Y[c][l][n] = sum_p s_p exp(j2pi (u_p n + v_p l)),
//   s_p = a_p exp(j2pi psi_p),  u_p = b_p,  v_p = -beta_p,
// a type-1 NUFFT from the points (u_p, v_p) onto the Ns x L modes.  It is
// evaluated as such a transform is (Barnett, Magland and af Klinteberg,
// SIAM J. Sci. Comput. 41 (2019), "exponential of semicircle" kernel
// phi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1)) of width w cells, grid
// oversampled at least twofold):
//   k_nufft_zero    clear the n1 x n2 grid of every channel
//   k_nufft_spread  per (block of 256 pixels, channel): phase arguments in
//                   binary64 (the same recipe as the direct forms), reduced
//                   frequencies u' = u - rint(u), v' = v - rint(v), centring
//                   phase exp(j2pi (u' floor(Ns/2) + v' floor(L/2))), and the
//                   w x w kernel weights around (u' n1, v' n2); the points
//                   are sorted by window column in LDS and every cell of the
//                   block's bounding box gathers its sum in registers into
//                   the block's tile slot (boxes of up to 1,024 cells and
//                   512 columns; a box taller than 16 rows whose points form
//                   two row groups is split into two sub-boxes at the widest
//                   gap); larger boxes add their sums, and boxes wider than
//                   the grid (points over all beat frequencies, or across
//                   its periodic edge) each weight, to the grid with atomics
//   k_nufft_assemble  the tile slots added to the grid: one or four threads
//                   per cell sum, in block order, a share each of the tiles
//                   whose box covers it, and the shares are added in a fixed
//                   order (no atomics on the cells every block touches)
//   k_nufft_rows    FFT (+ sign) of every grid row of length n1 in LDS that
//                   some block wrote to; the Ns kept modes times the
//                   deconvolution factor h / phi_hat go to a row buffer
//                   [C][n2][Ns]
//   k_nufft_cols    FFT (+ sign) of every column of length n2 (rows no block
//                   wrote to read as zero), the L kept modes times their
//                   deconvolution factor into the cube
// Arithmetic: phase arguments binary64; strengths, weights, grid and FFTs
// float32.  The sums are formed in a fixed order when every box fits a tile
// slot; boxes that do not are added with atomics, and then the order of the
// additions, and the last bits of the result, vary from run to run.
#include "rs_api_internal.h"
#include "rs_device.h"
#include "rs_fft.h"

#include <climits>
#include <cmath>
#include <type_traits>
#include <vector>

namespace {

constexpr int kSpreadThreads = 256;
constexpr int kBlockPts = 256;                        // pixels per spreading workgroup (power of two)
constexpr int kMaxCols = 512;                         // widest box gathered per cell
constexpr int kSlot = 1024;                           // tile cells kept per (block, channel)
constexpr int kAccCells = 2048;                       // LDS accumulator cells of the column gather
constexpr int kRowsReg = 16;                          // box rows held in registers by the column gather
constexpr int kGapRows = 1024;                        // tallest box searched for a row gap to split at
constexpr int kMaskBlocks = 1024;                     // descriptor entries per coverage pass of a row
constexpr int kAsmGroups = 8192;                      // assembly workgroups enough for 256 columns each
constexpr int kAsmRows = 8;                           // grid rows per assembly workgroup
constexpr int kFftThreads = 256;
constexpr int kFftElems = 4096;                       // complex values per FFT workgroup

struct nu_args {
    const float *x, *y, *z, *amp, *vr;
    int64_t P;
    const double *ant;          // tx[M][3] then rx[N][3]
    double Kc, Kb, Kd, Kf, Krvp, Ka;
    int32_t M, N, Ns, L, model;
    int32_t n1, n2;             // grid size along n and l (powers of two)
    float beta;                 // kernel shape
    float2 *grid;               // [C][n2][n1]: weights of boxes that do not fit a tile slot
    float2 *rows;               // [C][n2][Ns]
    float2 *tiles;              // [C][nblk][kSlot]: each block's (sub-)box sums, row-major e1 x e2
    int4 *desc;                 // [C][nblk][2]: sub-boxes (lo1, lo2, e1 | e2 << 16, tile offset);
                                //   e1 = 0 when not in a slot (the second one when unused)
    int *rowcov;                // [C][n2]: nonzero when some block wrote to the grid row
    int32_t nblk;               // pixel blocks
    const float *d1, *d2;       // deconvolution factors [Ns], [L]
    void *cube;                 // [C][L][Ns]
};

__device__ __forceinline__ void gatomic_add(float *p, float v)
{
    __hip_atomic_fetch_add((__attribute__((address_space(1))) float *)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// a mod n in [0, n) for the grid sizes, which are powers of two (two's
// complement makes the mask right for negative a too)
__device__ __forceinline__ int pmod(int a, int n) { return a & (n - 1); }

// Global load of a complex float32 value (one 8-byte load; rs_gload cannot
// copy the vector class out of the global address space).
__device__ __forceinline__ float2 rs_gload2(const float2 *p, int64_t i)
{
    const unsigned long long v = rs_gload(reinterpret_cast<const unsigned long long *>(p), i);
    return make_float2(__uint_as_float((unsigned)(v & 0xffffffffu)), __uint_as_float((unsigned)(v >> 32)));
}

// Kernel weight at offset t (cells) from the point; zero outside |t| <= w/2.
template <int W>
__device__ __forceinline__ float es_weight(float t, float beta)
{
    const float z = t * (2.0f / W);
    const float q = 1.0f - z * z;
    return q > 0.0f ? expf(beta * (__builtin_sqrtf(q) - 1.0f)) : 0.0f;
}

__global__ __launch_bounds__(256) void k_nufft_zero(float4 *p, int64_t n4)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Block-wide minimum (is_min) or maximum of v; every thread gets it.
__device__ __forceinline__ int block_reduce(int v, int *red, bool is_min)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int w = __shfl_xor(v, o);
        v = is_min ? min(v, w) : max(v, w);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = red[0];
    for (int i = 1; i < kSpreadThreads / 64; ++i) r = is_min ? min(r, red[i]) : max(r, red[i]);
    __syncthreads();
    return r;
}

// Block-wide component-wise minimum of v; every thread gets it (a maximum
// is taken as the minimum of ~x, which is order-reversing and cannot
// overflow).
__device__ __forceinline__ int4 block_min4(int4 v, int4 *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x = min(v.x, __shfl_xor(v.x, o));
        v.y = min(v.y, __shfl_xor(v.y, o));
        v.z = min(v.z, __shfl_xor(v.z, o));
        v.w = min(v.w, __shfl_xor(v.w, o));
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int4 r = red[0];
    for (int i = 1; i < kSpreadThreads / 64; ++i) {
        const int4 t = red[i];
        r = make_int4(min(r.x, t.x), min(r.y, t.y), min(r.z, t.z), min(r.w, t.w));
    }
    __syncthreads();
    return r;
}

// Spreading of one pixel block onto one channel's grid, gathered per cell.
//   1. A thread per pixel evaluates its point into LDS: the first cells
//      (m1, m2) of its W x W window, its strength c and the 2 W kernel
//      weights; the block's bounding box of cells follows by reduction (and
//      a tall box of two row groups is split into two sub-boxes).
//   2. The points are sorted by (sub-box, window column, index) -- a rank
//      sort of unique keys, so the order is fixed -- and cs[k] marks where
//      column k starts.
//   3. A thread per box column (and share of its candidates) sums, in
//      registers, c w1[x - m1] w2[y - m2] over the points whose window
//      covers it -- those with m1 - lo1 in [x - W + 1, x], a contiguous run
//      of the sorted order -- and the shares are added in a fixed order into
//      the block's tile slot; boxes that fit no slot add to the grid with
//      global atomics.
// No LDS atomics: neighbouring pixels share most of their window, and
// atomics on the same LDS cells from successive instructions serialise.
// Under 40 KB of LDS for W <= 7 and under 128 VGPRs: four workgroups per CU.
template <int W>
__global__ __launch_bounds__(kSpreadThreads) void k_nufft_spread(nu_args A)
{
    __shared__ int pm1[kBlockPts], pm2[kBlockPts];
    __shared__ float pw1[kBlockPts * W], pw2[kBlockPts * W];
    __shared__ int cs[kMaxCols + 1];
    __shared__ int2 srec[kBlockPts];      // sorted: ((m1 - lo1) | (m2 - lo2) << 16, point index)
    __shared__ float2 spc[kBlockPts];     // sorted strengths
    // per-share accumulators [share][row][column]; before them, in the same
    // space, each sorted point's w2 placed at its row of the box (16 rows).
    // Until the sorted records are complete the space holds the points'
    // strengths, the sort keys and the start-row occupancy of the split.
    __shared__ __align__(16) float accbuf[2 * kAccCells];   // read as float4
    float *accr = accbuf, *acci = accbuf + kAccCells, *spw2r = accbuf;
    float2 *pc = reinterpret_cast<float2 *>(accbuf);                          // [kBlockPts]
    int *key = reinterpret_cast<int *>(accbuf + 2 * kBlockPts);               // [kBlockPts], read as int4
    unsigned *occ = reinterpret_cast<unsigned *>(accbuf + 3 * kBlockPts);     // [kGapRows / 32]
    static_assert(3 * kBlockPts + kGapRows / 32 <= 2 * kAccCells, "aliases fit the accumulator space");
    __shared__ int red[kSpreadThreads / 64];
    __shared__ int4 red4[kSpreadThreads / 64];
    const int tid = threadIdx.x;
    const int c = blockIdx.y;
    const int m = c / A.N, r = c % A.N;
    double tx[3], rx[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        tx[i] = rs_gload(A.ant, 3 * m + i);
        rx[i] = rs_gload(A.ant, 3 * (A.M + r) + i);
    }
    const int64_t p0 = (int64_t)blockIdx.x * kBlockPts;
    const int npts = (int)min<int64_t>(kBlockPts, A.P - p0);
    int lo1 = INT_MAX, hi1 = INT_MIN, lo2 = INT_MAX, hi2 = INT_MIN;
    for (int q = tid; q < npts; q += kSpreadThreads) {
        const int64_t p = p0 + q;
        double psi, b, beta;
        rs_chan_args(A, rs_gload(A.x, p), rs_gload(A.y, p), rs_gload(A.z, p), rs_gload(A.vr, p), m, tx, rx, &psi,
                     &b, &beta);
        const double u = b - __builtin_rint(b);
        const double v = -beta - __builtin_rint(-beta);
        double th = rs_frac(psi) + u * (double)(A.Ns / 2) + v * (double)(A.L / 2);
        th = rs_frac(th);
        float sn, cs_;
        sincospif(2.0f * (float)th, &sn, &cs_);
        const float a = rs_gload(A.amp, p);
        pc[q] = make_float2(a * cs_, a * sn);
        // first cell of the W-cell window and the weights at its cells; the
        // offset from the point is formed in binary64 so that the weights see
        // it to float32 precision whatever the grid size
        const double t1 = u * (double)A.n1, t2 = v * (double)A.n2;
        const double s1 = __builtin_ceil(t1 - 0.5 * W), s2 = __builtin_ceil(t2 - 0.5 * W);
        const int c1 = (int)s1, c2 = (int)s2;
        pm1[q] = c1;
        pm2[q] = c2;
        const float o1 = (float)(s1 - t1), o2 = (float)(s2 - t2);
#pragma unroll
        for (int i = 0; i < W; ++i) {
            pw1[q * W + i] = es_weight<W>(o1 + (float)i, A.beta);
            pw2[q * W + i] = es_weight<W>(o2 + (float)i, A.beta);
        }
        lo1 = min(lo1, c1);
        hi1 = max(hi1, c1);
        lo2 = min(lo2, c2);
        hi2 = max(hi2, c2);
    }
    int4 *dsc = A.desc + ((int64_t)c * A.nblk + blockIdx.x) * 2;
    {   // the barriers also publish the points
        const int4 b = block_min4(make_int4(lo1, ~hi1, lo2, ~hi2), red4);
        lo1 = b.x;
        hi1 = ~b.y;
        lo2 = b.z;
        hi2 = ~b.w;
    }
    if (lo1 == INT_MAX) {                 // no pixel in this block (uniform)
        if (tid < 2) dsc[tid] = make_int4(0, 0, 0, 0);
        return;
    }
    const int e1 = hi1 - lo1 + W, e2 = hi2 - lo2 + W;   // box of cells touched
    float2 *grid = A.grid + (int64_t)c * A.n2 * A.n1;

    // ---- a box taller than the register rows whose window start rows fall
    // into two groups apart (static and moving scatterers in one block) is
    // split at the widest gap between occupied start rows, into two
    // sub-boxes that each take the register gather below -------------------
    int nsb = 1, split = 0;
    int blo1[2] = {lo1, 0}, blo2[2] = {lo2, 0}, be1[2] = {e1, 0}, be2[2] = {e2, 0};
    if (e2 > kRowsReg && hi2 - lo2 < kGapRows) {   // uniform
        for (int w = tid; w < kGapRows / 32; w += kSpreadThreads) occ[w] = 0u;
        __syncthreads();
        for (int q = tid; q < npts; q += kSpreadThreads) {
            const int rr = pm2[q] - lo2;
            atomicOr(&occ[rr >> 5], 1u << (rr & 31));
        }
        __syncthreads();
        // every run of occupied rows that ends at r < span - 1 is followed by
        // a gap up to the next occupied row (row span - 1 is occupied); key:
        // widest gap first, then lowest r
        const int span = hi2 - lo2 + 1;
        int best = -1;
        for (int rr = tid; rr < span - 1; rr += kSpreadThreads) {
            const bool run_end = (occ[rr >> 5] >> (rr & 31) & 1u) && !(occ[(rr + 1) >> 5] >> ((rr + 1) & 31) & 1u);
            if (run_end) {
                int wi = (rr + 2) >> 5;
                unsigned bits = occ[wi] & (~0u << ((rr + 2) & 31));
                while (!bits) bits = occ[++wi];
                const int nx = wi * 32 + __builtin_ctz(bits);
                best = max(best, (nx - rr) * kGapRows + (kGapRows - 1 - rr));
            }
        }
        best = block_reduce(best, red, false);
        if (best >= 0) {
            const int gap = best / kGapRows, rsp = kGapRows - 1 - best % kGapRows;
            const int e2a = rsp + W, e2b = (span - 1) - (rsp + gap) + W;
            if (e2a <= kRowsReg && e2b <= kRowsReg && e2a <= A.n2 && e2b <= A.n2) {   // uniform
                int alo = INT_MAX, ahi = INT_MIN, blo = INT_MAX, bhi = INT_MIN;
                for (int q = tid; q < npts; q += kSpreadThreads) {
                    if (pm2[q] - lo2 <= rsp) {
                        alo = min(alo, pm1[q]);
                        ahi = max(ahi, pm1[q]);
                    } else {
                        blo = min(blo, pm1[q]);
                        bhi = max(bhi, pm1[q]);
                    }
                }
                const int4 ab = block_min4(make_int4(alo, ~ahi, blo, ~bhi), red4);
                alo = ab.x;
                ahi = ~ab.y;
                blo = ab.z;
                bhi = ~ab.w;
                const int e1a = ahi - alo + W, e1b = bhi - blo + W;
                if (e1a * e2a + e1b * e2b <= kSlot && (ahi - alo + 1) + (bhi - blo + 1) <= kMaxCols &&
                    e1a + e1b <= kSpreadThreads && e1a <= A.n1 && e1b <= A.n1) {
                    nsb = 2;
                    split = rsp;
                    blo1[0] = alo;
                    blo1[1] = blo;
                    blo2[1] = lo2 + rsp + gap;
                    be1[0] = e1a;
                    be1[1] = e1b;
                    be2[0] = e2a;
                    be2[1] = e2b;
                }
            }
        }
    }

    const bool slot = nsb == 2 || (e1 * e2 <= kSlot && hi1 - lo1 < kMaxCols && e1 <= A.n1 && e2 <= A.n2);
    if (tid == 0) {
        dsc[0] = make_int4(blo1[0], blo2[0], slot ? be1[0] | be2[0] << 16 : 0, 0);
        dsc[1] = make_int4(blo1[1], blo2[1], nsb == 2 ? be1[1] | be2[1] << 16 : 0, be1[0] * be2[0]);
    }
    // flag the grid rows this block writes to (every row when the box is
    // taller than the grid): the FFT passes skip the rows no block touches
    // (every writer stores the same 1 into a cleared flag: plain stores)
    for (int sb = 0; sb < nsb; ++sb)
        for (int t = tid; t < min(be2[sb], A.n2); t += kSpreadThreads)
            A.rowcov[(int64_t)c * A.n2 + pmod(blo2[sb] + t, A.n2)] = 1;
    if (nsb == 1 && (hi1 - lo1 >= kMaxCols || e1 > A.n1 || e2 > A.n2)) {
        // box wider than the grid or the column table: scatter each weight
        // to the grid (a lane per window cell, a wave per point)
        const int lane = tid & 63, wave = tid >> 6;
        const int i = lane % W, j = lane / W;
        if (lane < W * W) {
            for (int q = wave; q < npts; q += kSpreadThreads / 64) {
                const float w = pw1[q * W + i] * pw2[q * W + j];
                const float2 cv = pc[q];
                float2 *cell = grid + (int64_t)pmod(pm2[q] + j, A.n2) * A.n1 + pmod(pm1[q] + i, A.n1);
                gatomic_add(&cell->x, cv.x * w);
                gatomic_add(&cell->y, cv.y * w);
            }
        }
        return;
    }

    // ---- 2. sort by sub-box and window column: key = column * kBlockPts + q,
    // the columns of the second sub-box numbered after those of the first;
    // a rank sort (no barriers inside) ----------------------------------------
    const int ncolA = be1[0] - W + 1;
    const int ncol = ncolA + (nsb == 2 ? be1[1] - W + 1 : 0);
    auto group = [&](int q) { return nsb == 2 && pm2[q] - lo2 > split ? 1 : 0; };
    for (int q = tid; q < kBlockPts; q += kSpreadThreads) {
        if (q < npts) {
            const int g = group(q);
            key[q] = ((g ? ncolA : 0) + pm1[q] - blo1[g]) * kBlockPts + q;
        } else {
            key[q] = INT_MAX;
        }
    }
    __syncthreads();
    // the sorted position of a point is the number of smaller keys (the keys
    // are unique, so the ranks are a permutation); every lane of a wave
    // reads the same keys at once, which the LDS broadcasts.  The records
    // (offsets from their sub-box's corner) are stored in sorted order so
    // that the gather reads them without an indirection.
    // Each point also lays out its w2 at its row of the (sub-)box, 16 rows
    // from its sorted position (what the register gather reads), into the
    // space that held the keys and strengths: both are read first.
    static_assert(kSpreadThreads == kBlockPts, "one point per thread");
    int rank = 0;
    float2 cq = make_float2(0.f, 0.f);
    if (tid < npts) {
        const int k = key[tid];
        const int4 *k4 = reinterpret_cast<const int4 *>(key);
#pragma unroll 4
        for (int i = 0; i < kBlockPts / 4; ++i) {
            const int4 v = k4[i];
            rank += (v.x < k) + (v.y < k) + (v.z < k) + (v.w < k);
        }
        cq = pc[tid];
    }
    __syncthreads();   // every key and strength has been read
    if (tid < npts) {
        const int g = group(tid);
        const int row = pm2[tid] - blo2[g];
        srec[rank] = make_int2((pm1[tid] - blo1[g]) | (row << 16), tid);
        spc[rank] = cq;
        float4 *dst = reinterpret_cast<float4 *>(spw2r + rank * kRowsReg);
#pragma unroll
        for (int r4 = 0; r4 < kRowsReg / 4; ++r4) {
            float w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int d = 4 * r4 + j - row;
                w[j] = d >= 0 && d < W ? pw2[tid * W + d] : 0.f;
            }
            dst[r4] = make_float4(w[0], w[1], w[2], w[3]);
        }
    }
    __syncthreads();
    // cs[k] = first sorted position whose column is >= k, k = 0 .. ncol
    auto column = [&](int s) {
        const int2 rec = srec[s];
        return (group(rec.y) ? ncolA : 0) + (rec.x & 0xffff);
    };
    for (int s = tid; s < npts; s += kSpreadThreads) {
        const int col = column(s);
        const int prev = s == 0 ? -1 : column(s - 1);
        for (int k = prev + 1; k <= col; ++k) cs[k] = s;
        if (s == npts - 1)
            for (int k = col + 1; k <= ncol; ++k) cs[k] = npts;
    }
    __syncthreads();

    // ---- 3a. boxes that fit a tile slot: a thread per (column, share of its
    // candidates) forms c w1 once per point and adds c w1 w2[j] to the W rows
    // of its private LDS accumulator; the shares are then added in a fixed
    // order per cell ---------------------------------------------------------
    const int E = e1 * e2;
    const int nparts = slot ? min(kSpreadThreads / e1, kAccCells / E) : 0;
    // (Sub-)boxes of at most 16 rows: the row sums of a column live in
    // registers, and each point's w2 is laid out at its row offset (by the
    // sort) so that a candidate costs four LDS vector reads and 32 FMAs.  TWO
    // (two sub-boxes) is a compile-time flag, so that the one-box case keeps
    // its simple indexing.
    auto register_gather = [&](auto two_t) {
        constexpr bool TWO = decltype(two_t)::value;
        // threads, shares and accumulator cells of the sub-boxes: the first
        // takes threads in proportion to its points (at least a column's
        // worth each), its shares leave room for one of the second
        const int EA = be1[0] * be2[0], EB = TWO ? be1[1] * be2[1] : 0;
        const int nA = TWO ? cs[ncolA] : npts;   // points of the first sub-box
        const int tA = TWO ? min(max(kSpreadThreads * nA / npts, be1[0]), kSpreadThreads - be1[1]) : kSpreadThreads;
        const int pA = min(tA / be1[0], (kAccCells - EB) / EA);
        const int pB = TWO ? min((kSpreadThreads - tA) / be1[1], (kAccCells - pA * EA) / EB) : 0;
        const int g = TWO && tid >= tA ? 1 : 0;
        const int tl = g ? tid - tA : tid;
        const int ex = g ? be1[1] : be1[0], ey = g ? be2[1] : be2[0];
        const int x = tl % ex, p = tl / ex;
        const int np = g ? pB : pA;
        const int coff = g ? ncolA : 0, ncg = g ? ncol - ncolA : ncolA;
        float ar[kRowsReg], ai[kRowsReg];
#pragma unroll
        for (int r = 0; r < kRowsReg; ++r) ar[r] = ai[r] = 0.f;
        if (p < np) {
            const int k0 = max(0, x - W + 1), k1 = min(x, ncg - 1);
            const int sb = cs[coff + k0], len = cs[coff + k1 + 1] - sb;
            const int s_beg = sb + len * p / np, s_end = sb + len * (p + 1) / np;
            for (int s = s_beg; s < s_end; ++s) {
                const int2 rec = srec[s];
                const float2 cv = spc[s];
                const float w1 = pw1[rec.y * W + x - (rec.x & 0xffff)];   // dx in [0, W) for this column range
                const float cr = cv.x * w1, ci = cv.y * w1;
                const float4 *wv = reinterpret_cast<const float4 *>(spw2r + s * kRowsReg);
#pragma unroll
                for (int r4 = 0; r4 < kRowsReg / 4; ++r4) {
                    const float4 w = wv[r4];
                    ar[4 * r4 + 0] = __builtin_fmaf(cr, w.x, ar[4 * r4 + 0]);
                    ai[4 * r4 + 0] = __builtin_fmaf(ci, w.x, ai[4 * r4 + 0]);
                    ar[4 * r4 + 1] = __builtin_fmaf(cr, w.y, ar[4 * r4 + 1]);
                    ai[4 * r4 + 1] = __builtin_fmaf(ci, w.y, ai[4 * r4 + 1]);
                    ar[4 * r4 + 2] = __builtin_fmaf(cr, w.z, ar[4 * r4 + 2]);
                    ai[4 * r4 + 2] = __builtin_fmaf(ci, w.z, ai[4 * r4 + 2]);
                    ar[4 * r4 + 3] = __builtin_fmaf(cr, w.w, ar[4 * r4 + 3]);
                    ai[4 * r4 + 3] = __builtin_fmaf(ci, w.w, ai[4 * r4 + 3]);
                }
            }
        }
        __syncthreads();   // spw2r is overwritten by the accumulators below
        if (p < np) {
            const int ab = g ? pA * EA + p * EB : p * EA;
#pragma unroll
            for (int r = 0; r < kRowsReg; ++r) {
                if (r < ey) {
                    accr[ab + r * ex + x] = ar[r];
                    acci[ab + r * ex + x] = ai[r];
                }
            }
        }
        __syncthreads();
        // the slot holds the first sub-box's cells, then the second's
        float2 *slotp = A.tiles + ((int64_t)c * A.nblk + blockIdx.x) * kSlot;
        for (int cell = tid; cell < EA + EB; cell += kSpreadThreads) {
            const bool inB = TWO && cell >= EA;
            const int base = inB ? pA * EA + (cell - EA) : cell, stride = inB ? EB : EA, n = inB ? pB : pA;
            float sr = 0.f, si = 0.f;
            for (int q = 0; q < n; ++q) {
                sr += accr[base + q * stride];
                si += acci[base + q * stride];
            }
            slotp[cell] = make_float2(sr, si);   // the assembly adds the slot to the grid rows it covers
        }
    };
    if (nsb == 2) {
        register_gather(std::true_type{});
        return;
    }
    if (nparts > 0 && e2 <= kRowsReg) {
        register_gather(std::false_type{});
        return;
    }
    if (nparts > 0) {
        for (int k = tid; k < nparts * E; k += kSpreadThreads) {
            accr[k] = 0.f;
            acci[k] = 0.f;
        }
        __syncthreads();
        const int x = tid % e1, p = tid / e1;
        if (p < nparts) {
            const int k0 = max(0, x - W + 1), k1 = min(x, ncol - 1);
            const int sb = cs[k0], len = cs[k1 + 1] - sb;
            const int s_beg = sb + len * p / nparts, s_end = sb + len * (p + 1) / nparts;
            float *ar = accr + p * E + x, *ai = acci + p * E + x;
            for (int s = s_beg; s < s_end; ++s) {
                const int2 rec = srec[s];
                const float2 cv = spc[s];
                const int base = rec.y * W;
                const float w1 = pw1[base + x - (rec.x & 0xffff)];   // dx in [0, W) for this column range
                const float cr = cv.x * w1, ci = cv.y * w1;
                const int r0 = (rec.x >> 16) * e1;
                float w2[W];
#pragma unroll
                for (int j = 0; j < W; ++j) w2[j] = pw2[base + j];
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    ar[r0 + j * e1] = __builtin_fmaf(cr, w2[j], ar[r0 + j * e1]);
                    ai[r0 + j * e1] = __builtin_fmaf(ci, w2[j], ai[r0 + j * e1]);
                }
            }
        }
        __syncthreads();
        float2 *slotp = A.tiles + ((int64_t)c * A.nblk + blockIdx.x) * kSlot;
        for (int cell = tid; cell < E; cell += kSpreadThreads) {
            float sr = 0.f, si = 0.f;
            for (int q = 0; q < nparts; ++q) {
                sr += accr[q * E + cell];
                si += acci[q * E + cell];
            }
            slotp[cell] = make_float2(sr, si);   // the assembly adds the slot to the grid rows it covers
        }
        return;
    }

    // ---- 3b. other boxes: gather per cell, one atomic pair per nonzero cell -
    for (int cell = tid; cell < e1 * e2; cell += kSpreadThreads) {
        const int y = cell / e1, x = cell - y * e1;
        const int k0 = max(0, x - W + 1), k1 = min(x, ncol - 1);
        const int sb = cs[k0], se = cs[k1 + 1];
        float sr = 0.f, si = 0.f;
        // kU candidates per round, their reads issued together; the points
        // of this column range have dx in [0, W) by construction
        constexpr int kU = 8;
        for (int s0 = sb; s0 < se; s0 += kU) {
            int2 rec[kU];
            float2 cv[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int si_ = min(s0 + u, se - 1);
                rec[u] = srec[si_];
                cv[u] = spc[si_];
            }
            float w1v[kU], w2v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int dx = x - (rec[u].x & 0xffff), dy = y - (rec[u].x >> 16);
                const bool hit = s0 + u < se && dy >= 0 && dy < W;
                const int base = rec[u].y * W;
                w1v[u] = pw1[base + (hit ? dx : 0)];
                w2v[u] = hit ? pw2[base + dy] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const float w = w1v[u] * w2v[u];
                sr = __builtin_fmaf(cv[u].x, w, sr);
                si = __builtin_fmaf(cv[u].y, w, si);
            }
        }
        if (slot) {
            // the assembly adds the slot to the grid rows it covers
            A.tiles[((int64_t)c * A.nblk + blockIdx.x) * kSlot + cell] = make_float2(sr, si);
        } else if (sr != 0.f || si != 0.f) {
            float2 *g = grid + (int64_t)pmod(lo2 + y, A.n2) * A.n1 + pmod(lo1 + x, A.n1);
            gatomic_add(&g->x, sr);
            gatomic_add(&g->y, si);
        }
    }
}

// Adds the tile slots to the grid: a workgroup per (channel, 8 grid rows n2/8
// apart, 256 / SPLIT columns), SPLIT threads per cell (SPLIT = 4 where the
// launch is small, so that more workgroups share it; 1 where channels are
// many, so that fewer column groups repeat the scan of the descriptors).
// The (sub-)boxes that cover the
// row and overlap the workgroup's columns are listed in LDS in block order
// (a coverage bitmask over the two descriptor entries of every block, set in
// any order, read in order), and every cell sums its tiles in that order, so
// the result does not depend on scheduling.
// Rows no block wrote to (their flag, set by the spreading kernel, is zero)
// are skipped.
template <int SPLIT>
__global__ __launch_bounds__(kFftThreads) void k_nufft_assemble(nu_args A)
{
    constexpr int kSplit = SPLIT, kAsmCols = kFftThreads / SPLIT;
    constexpr int kWords = kMaskBlocks / 32;
    static_assert(kWords <= 64 && kMaskBlocks % kFftThreads == 0, "one wave scans the words; whole entries per thread");
    __shared__ unsigned mask[kWords];
    __shared__ int woff[kWords];
    __shared__ int4 ldesc[kMaskBlocks];   // descriptors of the covering sub-boxes, in block order
    __shared__ int lid[kMaskBlocks];      // their entries: 2 block + sub-box
    __shared__ int ncov;
    __shared__ float2 part[kSplit][kAsmCols];
    const int c = blockIdx.z;
    // thread = (column, share of the covering list): the SPLIT partial sums
    // of a cell are added in a fixed order at the end
    const int lc = threadIdx.x % kAsmCols, sp = threadIdx.x / kAsmCols;
    const int c0 = blockIdx.x * kAsmCols;
    const int col = c0 + lc;
    const int4 *dc = A.desc + (int64_t)c * A.nblk * 2;
    const float2 *tc = A.tiles + (int64_t)c * A.nblk * kSlot;
    const int nent = 2 * A.nblk;
    // rows blockIdx.y + k gridDim.y (k < kAsmRows): the covered rows, which
    // lie together around the scene's Doppler band, go to different
    // workgroups.  Their flags are read at once; rows no block wrote to are
    // skipped.
    __shared__ unsigned rows_live;
    if (threadIdx.x < 64) {
        const int m2 = blockIdx.y + threadIdx.x * gridDim.y;
        const bool live = (int)threadIdx.x < kAsmRows && m2 < A.n2 && rs_gload(A.rowcov, (int64_t)c * A.n2 + m2) != 0;
        const unsigned long long bal = __ballot(live);
        if (threadIdx.x == 0) rows_live = (unsigned)bal;
    }
    __syncthreads();
    for (unsigned live = rows_live; live; live &= live - 1u) {
        const int m2 = blockIdx.y + __builtin_ctz(live) * gridDim.y;
        float2 acc = make_float2(0.f, 0.f);
        for (int b0 = 0; b0 < nent; b0 += kMaskBlocks) {
            const int nb = min(kMaskBlocks, nent - b0);
            const int nw = (nb + 31) / 32;
            for (int w = threadIdx.x; w < nw; w += blockDim.x) mask[w] = 0u;
            __syncthreads();
            // entries b = threadIdx.x + kFftThreads i: their descriptors stay in
            // registers until they are placed in the list
            constexpr int kPer = kMaskBlocks / kFftThreads;
            int4 dv[kPer];
            bool hit[kPer];
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int b = threadIdx.x + kFftThreads * i;
                hit[i] = false;
                if (b < nb) {
                    dv[i] = dc[b0 + b];
                    const int4 d = dv[i];
                    // the box covers this row and overlaps this workgroup's columns
                    // c0 .. c0 + kAsmCols - 1 (both taken around the periodic grid)
                    hit[i] = d.z > 0 && pmod(m2 - d.y, A.n2) < (d.z >> 16) &&
                             (pmod(c0 - d.x, A.n1) < (d.z & 0xffff) || pmod(d.x - c0, A.n1) < kAsmCols);
                    if (hit[i]) atomicOr(&mask[b >> 5], 1u << (b & 31));
                }
            }
            __syncthreads();
            // word offsets: an inclusive scan of the words' bit counts over the
            // first wave (kWords <= 64)
            if (threadIdx.x < 64) {
                const int cnt = (int)threadIdx.x < nw ? __builtin_popcount(mask[threadIdx.x]) : 0;
                int incl = cnt;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int v = __shfl_up(incl, off);
                    if ((int)threadIdx.x >= off) incl += v;
                }
                if ((int)threadIdx.x < nw) woff[threadIdx.x] = incl - cnt;
                if (threadIdx.x == 63) ncov = incl;
            }
            __syncthreads();
            const int nc = ncov;
            if (nc > 0) {
                // each covering entry goes to its place in block order
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    if (hit[i]) {
                        const int b = threadIdx.x + kFftThreads * i;
                        const int w = b >> 5;
                        const int o = woff[w] + __builtin_popcount(mask[w] & ((1u << (b & 31)) - 1u));
                        lid[o] = b0 + b;
                        ldesc[o] = dv[i];
                    }
                }
                __syncthreads();
                if (col < A.n1) {
                    const int kb = (int)((int64_t)nc * sp / kSplit), ke = (int)((int64_t)nc * (sp + 1) / kSplit);
                    // kU covering sub-boxes per round: their tile loads are in flight together
                    constexpr int kU = 8;
                    for (int k0 = kb; k0 < ke; k0 += kU) {
                        float2 t[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            t[u] = make_float2(0.f, 0.f);
                            if (k0 + u < ke) {
                                const int4 d = ldesc[k0 + u];
                                const int xx = pmod(col - d.x, A.n1), ex = d.z & 0xffff;
                                if (xx < ex)
                                    t[u] = rs_gload2(tc + (int64_t)(lid[k0 + u] >> 1) * kSlot + d.w,
                                                     pmod(m2 - d.y, A.n2) * ex + xx);
                            }
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            acc.x += t[u].x;
                            acc.y += t[u].y;
                        }
                    }
                }
            }
            __syncthreads();   // mask and list are rebuilt for the next block range
        }
        part[sp][lc] = acc;
        __syncthreads();
        if (sp == 0 && col < A.n1) {
            float2 *g = A.grid + ((int64_t)c * A.n2 + m2) * A.n1 + col;
            float2 v = rs_gload2(g, 0);
#pragma unroll
            for (int k = 0; k < kSplit; ++k) {
                v.x += part[k][lc].x;
                v.y += part[k][lc].y;
            }
            *g = v;
        }
        __syncthreads();   // part is rewritten for the next row
    }
}

// FFT (+ sign) of `rows` grid rows of length n1 per workgroup; the Ns kept
// modes k = n - floor(Ns/2) (index k mod n1) times d1[n] into the row buffer.
__global__ __launch_bounds__(kFftThreads) void k_nufft_rows(nu_args A, int logn1, int rpw, int64_t rows_total)
{
    extern __shared__ float2 smem[];
    const int n1 = 1 << logn1;
    float2 *tw = smem;
    float2 *x = smem + n1 / 2;
    const int64_t r0 = (int64_t)blockIdx.x * rpw;
    const int rows = (int)min<int64_t>(rpw, rows_total - r0);
    if (rows <= 0) return;
    // grid rows no block touched are zero, and so are their transforms: the
    // column pass reads them as zero, so they are neither read nor written
    __shared__ int live[kFftElems / 16];   // rows per workgroup <= kFftElems / 16 (n1 >= 16)
    int mine = 0;
    for (int row = threadIdx.x; row < rows; row += blockDim.x) {
        live[row] = rs_gload(A.rowcov, r0 + row);
        mine |= live[row];
    }
    if (!__syncthreads_or(mine)) return;
    twiddles(tw, n1, +1.0);
    const float2 *src = A.grid + r0 * n1;
    for (int e = threadIdx.x; e < rows * n1; e += blockDim.x) {
        const int row = e >> logn1, col = e & (n1 - 1);
        x[row * n1 + bitrev(col, logn1)] = live[row] ? rs_gload2(src, e) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_rows(x, rows, logn1, tw);
    const int h = A.Ns / 2;
    float2 *dst = A.rows + r0 * A.Ns;
    for (int e = threadIdx.x; e < rows * A.Ns; e += blockDim.x) {
        const int row = e / A.Ns, n = e - row * A.Ns;
        if (!live[row]) continue;
        const int k = n - h;
        const float2 v = x[row * n1 + (k < 0 ? k + n1 : k)];
        const float d = rs_gload(A.d1, n);
        dst[e] = make_float2(v.x * d, v.y * d);
    }
}

// FFT (+ sign) along l of kb columns n0 .. n0 + kb - 1 of one channel's row
// buffer; the L kept modes k = l - floor(L/2) times d2[l] into the cube.
template <typename OT>
__global__ __launch_bounds__(kFftThreads) void k_nufft_cols(nu_args A, int logn2, int kb, int groups)
{
    extern __shared__ float2 smem[];
    const int n2 = 1 << logn2;
    float2 *tw = smem;
    // [kb][n2 + 1]: the padding puts the columns' equal offsets in different banks
    const int xs = n2 + 1;
    float2 *x = smem + n2 / 2;
    const int c = blockIdx.x / groups;
    const int n0 = (blockIdx.x % groups) * kb;
    const int kn = min(kb, A.Ns - n0);
    const int logkb = __builtin_ctz((unsigned)kb);   // kb is a power of two
    __shared__ int live[kFftElems];        // grid rows of this channel some block wrote to (n2 <= kFftElems)
    for (int m2 = threadIdx.x; m2 < n2; m2 += blockDim.x) live[m2] = rs_gload(A.rowcov, (int64_t)c * n2 + m2);
    twiddles(tw, n2, +1.0);
    __syncthreads();
    const float2 *src = A.rows + (int64_t)c * n2 * A.Ns + n0;
    for (int e = threadIdx.x; e < n2 * kb; e += blockDim.x) {
        const int m2 = e >> logkb, kk = e & (kb - 1);
        // untouched rows are zero (their row-buffer entries were never written)
        x[kk * xs + bitrev(m2, logn2)] =
            kk < kn && live[m2] ? rs_gload2(src, (int64_t)m2 * A.Ns + kk) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_rows(x, kb, logn2, tw, xs);
    const int h = A.L / 2;
    OT *out = reinterpret_cast<OT *>(A.cube) + (int64_t)c * A.L * A.Ns + n0;
    for (int e = threadIdx.x; e < A.L * kb; e += blockDim.x) {
        const int l = e >> logkb, kk = e & (kb - 1);
        if (kk >= kn) continue;
        const int k = l - h;
        const float2 v = x[kk * xs + (k < 0 ? k + n2 : k)];
        const float d = rs_gload(A.d2, l);
        OT o;
        o.x = v.x * d;
        o.y = v.y * d;
        out[(int64_t)l * A.Ns + kk] = o;
    }
}

template <int W>
void launch_spread(const nu_args &A, int C, hipStream_t st)
{
    const dim3 grid((unsigned)((A.P + kBlockPts - 1) / kBlockPts), (unsigned)C);
    hipLaunchKernelGGL(k_nufft_spread<W>, grid, dim3(kSpreadThreads), 0, st, A);
}

int log2i(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton's method on the
// Legendre polynomial from the Chebyshev-like first guesses).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

// Kernel parameters for a tolerance (twofold oversampling): width
// w = ceil(log10(1/tol)) + 1 cells (2 .. 8 for the tolerances a plan
// accepts), shape beta = 2.30 w (2.20 w, 2.26 w, 2.38 w for w = 2, 3, 4).
void rs_nufft_params(double tol, int *w, double *beta)
{
    int ww = (int)std::ceil(std::log10(1.0 / tol)) + 1;
    ww = ww < 2 ? 2 : (ww > 8 ? 8 : ww);
    const double per = ww == 2 ? 2.20 : ww == 3 ? 2.26 : ww == 4 ? 2.38 : 2.30;
    *w = ww;
    *beta = per * ww;
}

int rs_nufft_fine(int N, int w)
{
    int n = 1;
    while (n < 2 * N || n < 2 * w) n *= 2;
    return n;
}

// h / phi_hat(k) for the centred modes k = i - floor(N/2), i < N, on an
// n-point grid: phi_hat(k) = integral of phi(x) cos(k x) over radians x,
// by 200-node Gauss-Legendre quadrature in binary64.
void rs_nufft_deconv(int N, int n, int w, double beta, float *out)
{
    std::vector<double> z, q;
    gauss_legendre(200, z, q);
    const double h = 2.0 * M_PI / n, half = 0.5 * w * h;
    for (int i = 0; i < N; ++i) {
        const double k = (double)(i - N / 2);
        double s = 0.0;
        for (size_t j = 0; j < z.size(); ++j)
            s += q[j] * std::exp(beta * (std::sqrt(1.0 - z[j] * z[j]) - 1.0)) * std::cos(k * half * z[j]);
        out[i] = (float)(h / (half * s));
    }
}

// Workspace: grid, row buffer, tile slots and box descriptors.
size_t rs_nufft_workspace(const rs_plan *pl, int64_t P)
{
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t nblk = (P + kBlockPts - 1) / kBlockPts;
    return up((size_t)pl->C * pl->nu_n1 * pl->nu_n2 * 8) + up((size_t)pl->C * pl->nu_n2 * 4) +
           up((size_t)pl->C * pl->nu_n2 * pl->Ns * 8) + up((size_t)pl->C * nblk * kSlot * 8) +
           up((size_t)pl->C * nblk * 2 * sizeof(int4));
}

rs_status rs_nufft_enqueue(const rs_plan *pl, const rs_pixels *px, void *cube, void *ws, hipStream_t st)
{
    nu_args A;
    A.x = px->x;
    A.y = px->y;
    A.z = px->z;
    A.amp = px->amp;
    A.vr = px->vr;
    A.P = px->P;
    A.ant = pl->d_ant;
    A.Kc = pl->Kc;
    A.Kb = pl->Kb;
    A.Kd = pl->Kd;
    A.Kf = pl->Kf;
    A.Krvp = pl->Krvp;
    A.Ka = pl->Ka;
    A.M = pl->M;
    A.N = pl->N;
    A.Ns = pl->Ns;
    A.L = pl->L;
    A.model = pl->model;
    A.n1 = pl->nu_n1;
    A.n2 = pl->nu_n2;
    A.beta = (float)pl->nu_beta;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    A.nblk = (int32_t)((px->P + kBlockPts - 1) / kBlockPts);
    char *w = static_cast<char *>(ws);
    A.grid = reinterpret_cast<float2 *>(w);
    w += up((size_t)pl->C * pl->nu_n1 * pl->nu_n2 * 8);
    A.rowcov = reinterpret_cast<int *>(w);
    w += up((size_t)pl->C * pl->nu_n2 * 4);
    const size_t zero_bytes = (size_t)(w - static_cast<char *>(ws));   // grid and row flags
    A.rows = reinterpret_cast<float2 *>(w);
    w += up((size_t)pl->C * pl->nu_n2 * pl->Ns * 8);
    A.tiles = reinterpret_cast<float2 *>(w);
    w += up((size_t)pl->C * A.nblk * kSlot * 8);
    A.desc = reinterpret_cast<int4 *>(w);
    A.d1 = pl->d_deconv;
    A.d2 = pl->d_deconv + pl->Ns;
    A.cube = cube;

    const int64_t n4 = (int64_t)(zero_bytes / 16);
    const int zgrid = (int)std::min<int64_t>((n4 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_nufft_zero, dim3(zgrid), dim3(256), 0, st, reinterpret_cast<float4 *>(A.grid), n4);
    if (A.P > 0) {
        switch (pl->nu_w) {
        case 2: launch_spread<2>(A, pl->C, st); break;
        case 3: launch_spread<3>(A, pl->C, st); break;
        case 4: launch_spread<4>(A, pl->C, st); break;
        case 5: launch_spread<5>(A, pl->C, st); break;
        case 6: launch_spread<6>(A, pl->C, st); break;
        case 7: launch_spread<7>(A, pl->C, st); break;
        case 8: launch_spread<8>(A, pl->C, st); break;
        default: return rs_fail(RS_E_UNSUPPORTED, "NUFFT kernel width %d not built", pl->nu_w);
        }
    }
    if (A.nblk > 0) {
        const int gy = std::max(1, pl->nu_n2 / kAsmRows);
        const int64_t wide = (int64_t)((pl->nu_n1 + kFftThreads - 1) / kFftThreads) * gy * pl->C;
        if (wide >= kAsmGroups)
            hipLaunchKernelGGL(k_nufft_assemble<1>, dim3((unsigned)((pl->nu_n1 + kFftThreads - 1) / kFftThreads),
                                                         (unsigned)gy, (unsigned)pl->C),
                               dim3(kFftThreads), 0, st, A);
        else
            hipLaunchKernelGGL(k_nufft_assemble<4>,
                               dim3((unsigned)((pl->nu_n1 + kFftThreads / 4 - 1) / (kFftThreads / 4)), (unsigned)gy,
                                    (unsigned)pl->C),
                               dim3(kFftThreads), 0, st, A);
    }
    const int logn1 = log2i(pl->nu_n1), logn2 = log2i(pl->nu_n2);
    // few rows or columns per workgroup: only the rows some block wrote to
    // carry work, and each pass then takes about one workgroup's time
    // (measured on the frame: 8 rows of 512 per workgroup 18.7 us, 1 row
    // 10.1 us; 16 columns of 256 13.9 us, 4 columns 8.2 us)
    const int rpw = std::max(1, 512 / pl->nu_n1);
    const int64_t rows_total = (int64_t)pl->C * pl->nu_n2;
    const size_t lds1 = (size_t)(pl->nu_n1 / 2 + rpw * pl->nu_n1) * sizeof(float2);
    hipLaunchKernelGGL(k_nufft_rows, dim3((unsigned)((rows_total + rpw - 1) / rpw)), dim3(kFftThreads), lds1, st, A,
                       logn1, rpw, rows_total);
    const int kb = std::max(1, std::min(4, 1024 / pl->nu_n2));
    const int groups = (pl->Ns + kb - 1) / kb;
    const size_t lds2 = (size_t)(pl->nu_n2 / 2 + kb * (pl->nu_n2 + 1)) * sizeof(float2);
    if (pl->dtype == RS_C128)
        hipLaunchKernelGGL(k_nufft_cols<double2>, dim3((unsigned)(pl->C * groups)), dim3(kFftThreads), lds2, st, A,
                           logn2, kb, groups);
    else
        hipLaunchKernelGGL(k_nufft_cols<float2>, dim3((unsigned)(pl->C * groups)), dim3(kFftThreads), lds2, st, A,
                           logn2, kb, groups);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "NUFFT launch: %s", hipGetErrorString(e));
    return RS_OK;
}
