// Split-K reduction: cube[c][l][n] = sum_{s=0}^{S-1} partial[s][c][l][n], summed
// in increasing s in binary64 and stored as complex64 or complex128.  The
// fixed order makes a cube independent of how work items were scheduled.
#include "rs_device.h"

namespace {

template <typename PT>
__global__ __launch_bounds__(256) void k_reduce(rs_launch Lc)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= Lc.total) return;
    const int jidx = rs_find_job<RS_BY_OUT>(Lc, g);
    const rs_job &J = rs_job_of(Lc, jidx);
    const int64_t idx = g - J.out_begin;
    const int64_t cln = (int64_t)(J.M * J.N) * J.L * J.Ns;
    const PT *p = reinterpret_cast<const PT *>(J.partial) + idx;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < J.S; ++s) {
        const PT v = p[(int64_t)s * cln];
        re += (double)v.x;
        im += (double)v.y;
    }
    if (J.dtype == 1)
        reinterpret_cast<double2 *>(J.cube)[idx] = make_double2(re, im);
    else
        reinterpret_cast<float2 *>(J.cube)[idx] = make_float2((float)re, (float)im);
}

__device__ __forceinline__ void store_entry(const rs_job &J, int64_t idx, double re, double im)
{
    if (J.dtype == 1)
        reinterpret_cast<double2 *>(J.cube)[idx] = make_double2(re, im);
    else
        reinterpret_cast<float2 *>(J.cube)[idx] = make_float2((float)re, (float)im);
}

// Matrix-core partials (complex64): two neighbouring entries per thread with
// 16-byte loads, the chunk loop unrolled for loads in flight; the sum of
// each entry is formed in the same order as k_reduce forms it.
__global__ __launch_bounds__(256) void k_reduce_pairs(rs_launch Lc)
{
    const int64_t g = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
    if (g >= Lc.total) return;
    const int jidx = rs_find_job<RS_BY_OUT>(Lc, g);
    const rs_job &J = rs_job_of(Lc, jidx);
    const int64_t idx = g - J.out_begin;
    const int64_t cln = (int64_t)(J.M * J.N) * J.L * J.Ns;
    const int S = J.S;
    if (((idx | cln) & 1) == 0) {
        // both entries in this job, 16-byte aligned in every partial
        const float4 *p = reinterpret_cast<const float4 *>(reinterpret_cast<const float2 *>(J.partial) + idx);
        const int64_t stride = cln / 2;
        double r0 = 0.0, i0 = 0.0, r1 = 0.0, i1 = 0.0;
#pragma unroll 4
        for (int s = 0; s < S; ++s) {
            const float4 v = p[(int64_t)s * stride];
            r0 += (double)v.x;
            i0 += (double)v.y;
            r1 += (double)v.z;
            i1 += (double)v.w;
        }
        store_entry(J, idx, r0, i0);
        store_entry(J, idx + 1, r1, i1);
        return;
    }
    // an odd-sized job: each entry on its own (the second may open the next job)
    for (int k = 0; k < 2 && g + k < Lc.total; ++k) {
        const rs_job &Jk = rs_job_of(Lc, rs_find_job<RS_BY_OUT>(Lc, g + k));
        const int64_t ik = g + k - Jk.out_begin;
        const int64_t ck = (int64_t)(Jk.M * Jk.N) * Jk.L * Jk.Ns;
        const float2 *p = reinterpret_cast<const float2 *>(Jk.partial) + ik;
        double re = 0.0, im = 0.0;
        for (int s = 0; s < Jk.S; ++s) {
            const float2 v = p[(int64_t)s * ck];
            re += (double)v.x;
            im += (double)v.y;
        }
        store_entry(Jk, ik, re, im);
    }
}

__global__ void k_zero_int(int *p, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

void rs_launch_reduce(const rs_launch &L, int form, hipStream_t st)
{
    const int64_t blocks = (L.total + 255) / 256;
    if (blocks <= 0) return;
    if (form == 0)
        hipLaunchKernelGGL(k_reduce<double2>, dim3((unsigned)blocks), dim3(256), 0, st, L);
    else
        hipLaunchKernelGGL(k_reduce_pairs, dim3((unsigned)((L.total + 511) / 512)), dim3(256), 0, st, L);
}

void rs_launch_zero_int(int *p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
}
