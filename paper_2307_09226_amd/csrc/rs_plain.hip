// Plain form: binary64 direct sum on the vector ALUs (gfx950).
//
// Y[c][l][n] = sum_p a_p exp(j2pi(psi_{p,c} + b_{p,c} n - beta_p l))  (Sec. II,
// eq. (1) per virtual channel, pixel sum of eq. (2)).  Each term is the
// product F[p][n] * D[p][l] with
//   F[p][n] = exp(j2pi wrap(psi_f + frac(b n)))
//   D[p][l] = a_p exp(-j2pi frac(beta l))
// in binary64, accumulated with four binary64 FMAs (8 flop per term).
//
// Work item = (channel, 64-row n tile, TL-column l tile, pixel chunk).  Per
// step of 16 pixels the workgroup evaluates the 16 x 64 F and 16 x TL D
// phasors once into LDS (each of a pixel's 16 threads finds the pixel's
// phase arguments itself, so the step has no serial parameter stage); each
// thread then owns a 4 (n) x TL/16 (l) block of binary64 accumulators.  A thread evaluates a run of consecutive phasors of
// one pixel: the first directly (binary64 sincospi of the reduced phase),
// the others by binary64 rotation with exp(j2pi frac(b)) or
// exp(-j2pi frac(beta)), at most 7 rotations (~1e-15 relative).  With
// strengths per block (amp_lstride != 0) the slow-time run rotates the unit
// phasor and multiplies each entry by a_{p,l}.  Chunks
// write binary64 partial tiles that the reduce kernel sums in a fixed
// order.
#include "rs_device.h"

namespace {

constexpr int kTN = 64;  // n rows per tile
constexpr int kKP = 16;  // pixels per step

template <int TL>
__global__ __launch_bounds__(256, 2) void k_plain_fp64(rs_launch Lc)
{
    constexpr int NJ = TL / 16;
    __shared__ double2 sF[kKP][kTN];
    __shared__ double2 sD[kKP][TL];
    __shared__ rs_item_consts sK;
    __shared__ int64_t s_item;

    const int tid = threadIdx.x;
    const int tn = tid & 15, tl = tid >> 4;
    bool first = true;
    for (;;) {
        const int64_t item = rs_next_item(Lc, &s_item, first);
        first = false;
        if (item < 0) break;
        const int jidx = rs_find_job<RS_BY_ITEM>(Lc, item);
        const rs_job &J = rs_job_of(Lc, jidx);
        const rs_item it = rs_decode_item(J, J.item_first + (item - J.item_begin));
        const int n0 = it.nt * kTN, l0 = it.lt * TL;
        const int64_t pb = (int64_t)it.s * J.chunk;
        const int64_t pe = min(J.P, pb + (int64_t)J.chunk);
        const int m = it.c / J.N, r = it.c % J.N;
        // every reader of the previous item's sK has passed a barrier since
        if (tid == 0) rs_item_consts_of(J, m, r, sK);
        __syncthreads();
        // raw values of this thread's pixel of the next step (the 16 threads
        // of a pixel load the same values), loaded a step ahead; the index is
        // clamped into the chunk and the pixel's validity decided when it is
        // used
        float nx, ny, nz, na, nv;
        auto fetch = [&](int64_t p0) {
            const int64_t p = min(p0 + (tid >> 4), pe - 1);
            nx = rs_gload(sK.x, p);
            ny = rs_gload(sK.y, p);
            nz = rs_gload(sK.z, p);
            na = rs_gload(sK.amp, p);
            nv = rs_gload(sK.vr, p);
        };
        fetch(pb);

        double2 acc[4][NJ];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][j] = make_double2(0.0, 0.0);

        for (int64_t p0 = pb; p0 < pe; p0 += kKP) {
            {
                // thread = (pixel q, run r of consecutive rows / columns); each
                // of the pixel's 16 threads finds its phase arguments
                const int q = tid >> 4, r = tid & 15;
                double psi_f = 0.0, b = 0.0, beta = 0.0, a = 0.0;
                if (p0 + q < pe) {
                    double psi;
                    rs_chan_args(sK, nx, ny, nz, nv, m, sK.tx, sK.rx, &psi, &b, &beta);
                    psi_f = rs_frac(psi);
                    a = (double)na;
                }
                fetch(p0 + kKP);
                // fast-time phasors F = exp(j 2pi phi), phi = wrap(psi_f + frac(b n)),
                // rows n0 + 4r .. n0 + 4r + 3
                constexpr int FR = kTN / 16;
                double phi = psi_f + rs_frac(b * (double)(n0 + FR * r));
                phi = phi - __builtin_floor(phi + 0.5);
                double fs, fc, rs_, rc;
                sincospi(2.0 * phi, &fs, &fc);
                sincospi(2.0 * rs_frac(b), &rs_, &rc);
#pragma unroll
                for (int k = 0; k < FR; ++k) {
                    sF[q][FR * r + k] = make_double2(fc, fs);
                    const double cn = __builtin_fma(fc, rc, -(fs * rs_));
                    fs = __builtin_fma(fc, rs_, fs * rc);
                    fc = cn;
                }
                // slow-time phasors D = a exp(-j 2pi frac(beta l)), columns
                // l0 + DR r .. l0 + DR r + DR - 1
                constexpr int DR = TL / 16;
                double ds, dc, ts, tc;
                sincospi(2.0 * rs_frac(beta * (double)(l0 + DR * r)), &ds, &dc);
                sincospi(2.0 * rs_frac(beta), &ts, &tc);
                if (sK.amp_lstride == 0) {
                    dc *= a;
                    ds *= a;
#pragma unroll
                    for (int k = 0; k < DR; ++k) {
                        sD[q][DR * r + k] = make_double2(dc, -ds);
                        const double cn = __builtin_fma(dc, tc, -(ds * ts));
                        ds = __builtin_fma(dc, ts, ds * tc);
                        dc = cn;
                    }
                } else {
                    // strength per block: the unit phasor is rotated and
                    // each entry multiplied by a_{p,l}
                    const int64_t p = p0 + q;
#pragma unroll
                    for (int k = 0; k < DR; ++k) {
                        const int l = l0 + DR * r + k;
                        const double al =
                            p < pe && l < sK.L ? (double)rs_gload(sK.amp, p + (int64_t)l * sK.amp_lstride) : 0.0;
                        sD[q][DR * r + k] = make_double2(dc * al, -(ds * al));
                        const double cn = __builtin_fma(dc, tc, -(ds * ts));
                        ds = __builtin_fma(dc, ts, ds * tc);
                        dc = cn;
                    }
                }
            }
            __syncthreads();
#pragma unroll 2
            for (int q = 0; q < kKP; ++q) {
                double2 f[4], d[NJ];
#pragma unroll
                for (int i = 0; i < 4; ++i) f[i] = sF[q][tn + 16 * i];
#pragma unroll
                for (int j = 0; j < NJ; ++j) d[j] = sD[q][tl + 16 * j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        acc[i][j].x = __builtin_fma(f[i].x, d[j].x, acc[i][j].x);
                        acc[i][j].x = __builtin_fma(-f[i].y, d[j].y, acc[i][j].x);
                        acc[i][j].y = __builtin_fma(f[i].x, d[j].y, acc[i][j].y);
                        acc[i][j].y = __builtin_fma(f[i].y, d[j].x, acc[i][j].y);
                    }
            }
            __syncthreads();
        }

        double2 *out = reinterpret_cast<double2 *>(J.partial) +
                       ((int64_t)it.s * (J.M * J.N) + it.c) * (int64_t)J.L * J.Ns;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n = n0 + tn + 16 * i;
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int l = l0 + tl + 16 * j;
                if (n < J.Ns && l < J.L) out[(int64_t)l * J.Ns + n] = acc[i][j];
            }
        }
    }
}

}  // namespace

void rs_launch_plain(const rs_launch &L, int tl, int grid, hipStream_t st)
{
    if (tl == 64)
        hipLaunchKernelGGL(k_plain_fp64<64>, dim3(grid), dim3(256), 0, st, L);
    else
        hipLaunchKernelGGL(k_plain_fp64<128>, dim3(grid), dim3(256), 0, st, L);
}
