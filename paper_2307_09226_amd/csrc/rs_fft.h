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

__device__ __forceinline__ int bitrev(int v, int logn) { return (int)(__brev((unsigned)v) >> (32 - logn)); }

// In-place radix-2 DIT over `rows` rows of length n = 2^logn, stored with
// row stride `stride` (n when 0) in LDS, input in bit-reversed order;
// tw = twiddles of n.  The stages are taken two at a time: a thread takes
// the four elements (i, i+h, i+2h, i+3h) of a block of 4h, applies stage s
// to the pairs (i, i+h) and (i+2h, i+3h) and stage s+1 to (i, i+2h) and
// (i+h, i+3h), the butterflies of the one-stage-at-a-time form in the same
// order with half the barriers and LDS round trips.  An odd number of
// stages ends with one radix-2 stage.
static __device__ void fft_rows(float2 *x, int rows, int logn, const float2 *tw, int stride = 0)
{
    const int n = 1 << logn;
    const int rs = stride ? stride : n;
    int s = 0;
    for (; s + 1 < logn; s += 2) {
        const int h = 1 << s;
        const int t2 = (n >> 1) >> s;  // twiddle index step of stage s
        const int t4 = t2 >> 1;        // ... of stage s + 1
        const int nq = rows * (n >> 2);
        for (int b = threadIdx.x; b < nq; b += blockDim.x) {
            const int row = b >> (logn - 2);
            const int bb = b & ((n >> 2) - 1);
            const int pos = bb & (h - 1);
            const int i = ((bb >> s) << (s + 2)) + pos;
            float2 *r = x + row * rs;
            const float2 w2 = tw[pos * t2];
            const float2 tb = cmul(w2, r[i + h]);
            const float2 td = cmul(w2, r[i + 3 * h]);
            const float2 a = r[i], c = r[i + 2 * h];
            const float2 a1 = make_float2(a.x + tb.x, a.y + tb.y), b1 = make_float2(a.x - tb.x, a.y - tb.y);
            const float2 c1 = make_float2(c.x + td.x, c.y + td.y), d1 = make_float2(c.x - td.x, c.y - td.y);
            const float2 tc = cmul(tw[pos * t4], c1);
            const float2 te = cmul(tw[(pos + h) * t4], d1);
            r[i] = make_float2(a1.x + tc.x, a1.y + tc.y);
            r[i + 2 * h] = make_float2(a1.x - tc.x, a1.y - tc.y);
            r[i + h] = make_float2(b1.x + te.x, b1.y + te.y);
            r[i + 3 * h] = make_float2(b1.x - te.x, b1.y - te.y);
        }
        __syncthreads();
    }
    if (s < logn) {
        const int half = 1 << s;
        const int tstride = (n >> 1) >> s;
        const int nb = rows * (n >> 1);
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
