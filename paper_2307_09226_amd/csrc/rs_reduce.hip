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
        hipLaunchKernelGGL(k_reduce<float2>, dim3((unsigned)blocks), dim3(256), 0, st, L);
}

void rs_launch_zero_int(int *p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
}
