// Radix-2 FFT helpers in LDS, float32 data with twiddles from binary64,
// used by the range-Doppler maps and the NUFFT form.  Every thread of the
// workgroup must call twiddles and fft_rows (fft_rows contains barriers).
#pragma once
#include <hip/hip_runtime.h>

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// exp(sign j 2pi j / n) for j < n/2 into tw (binary64 evaluation)
static __device__ void twiddles(float2 *tw, int n, double sign)
{
    for (int j = threadIdx.x; j < n / 2; j += blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)j / (double)n, &s, &c);
        tw[j] = make_float2((float)c, (float)(sign * s));
    }
}

// In-place radix-2 DIT over `rows` rows of length n = 2^logn, stored with
// row stride `stride` (n when 0) in LDS, input in bit-reversed order.
// tw = twiddles of n.
static __device__ void fft_rows(float2 *x, int rows, int logn, const float2 *tw, int stride = 0)
{
    const int n = 1 << logn;
    const int rs = stride ? stride : n;
    const int nb = rows * (n >> 1);  // butterflies per stage
    for (int s = 0; s < logn; ++s) {
        const int half = 1 << s;
        const int tstride = (n >> 1) >> s;  // twiddle index step
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            const int row = b >> (logn - 1);
            const int bb = b & ((n >> 1) - 1);
            const int pos = bb & (half - 1);
            const int i = ((bb >> s) << (s + 1)) + pos;
            float2 *r = x + row * rs;
            const float2 t = cmul(tw[pos * tstride], r[i + half]);
            const float2 u = r[i];
            r[i] = make_float2(u.x + t.x, u.y + t.y);
            r[i + half] = make_float2(u.x - t.x, u.y - t.y);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bitrev(int v, int logn) { return (int)(__brev((unsigned)v) >> (32 - logn)); }

