// Test-only gfx950 library: runs the device primitives the synthesis kernels
// rely on, element by element, so that tests can compare them with the host.
//   prim_distance   rs_distance (binary64 recipe, correctly rounded sqrt)
//   prim_sqrt       binary64 sqrt as the kernels compile it
//   prim_fract      __builtin_amdgcn_fract (v_fract_f64) and rs_frac
//   prim_sincos     the binary32 hardware sin / cos, input in revolutions
//   prim_split16    the fp16 hi / lo split of a binary32 pair
//   prim_split16j   that split times j (rs_jmul): the split of (-y, x)
// Every function enqueues one kernel on `stream` and returns 0, or the HIP
// error code of the launch.  All pointers are device memory of n elements
// (prim_distance: ant holds 3 doubles).  Built with the library's flags.
#include "rs_device.h"
#include "rs_split16.h"

namespace {

__global__ void k_distance(const float *x, const float *y, const float *z, const double *ant, double *out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = rs_distance(x[i], y[i], z[i], ant);
}

__global__ void k_sqrt(const double *in, double *out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = __builtin_sqrt(in[i]);
}

__global__ void k_fract(const double *in, double *hw, double *sub, float *f32, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        hw[i] = __builtin_amdgcn_fract(in[i]);
        sub[i] = rs_frac(in[i]);
        f32[i] = rs_frac32(in[i]);
    }
}

__global__ void k_sincos(const float *in, float *s, float *c, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        s[i] = __builtin_amdgcn_sinf(in[i]);
        c[i] = __builtin_amdgcn_cosf(in[i]);
    }
}

// in: n pairs (x, y); hi, lo: n packed fp16 pairs (x in bits 15:0)
__global__ void k_split16(const float2 *in, unsigned *hi, unsigned *lo, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        float x = in[i].x, y = in[i].y;
        rs_pin(x, y);
        const rs_half2v h = rs_hi2(x, y);
        hi[i] = rs_bits(h);
        lo[i] = rs_bits(rs_lo2(x, y, h));
    }
}

// as k_split16, then both packed pairs times j
__global__ void k_split16j(const float2 *in, unsigned *hi, unsigned *lo, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        float x = in[i].x, y = in[i].y;
        rs_pin(x, y);
        const rs_half2v h = rs_hi2(x, y);
        hi[i] = rs_bits(rs_jmul(h));
        lo[i] = rs_bits(rs_jmul(rs_lo2(x, y, h)));
    }
}

int launched() { return (int)hipGetLastError(); }

unsigned blocks(int n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" int prim_distance(const float *x, const float *y, const float *z, const double *ant, double *out,
                             int n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_distance, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, x, y, z, ant, out, n);
    return launched();
}

extern "C" int prim_sqrt(const double *in, double *out, int n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_sqrt, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, in, out, n);
    return launched();
}

extern "C" int prim_fract(const double *in, double *hw, double *sub, float *f32, int n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fract, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, in, hw, sub, f32, n);
    return launched();
}

extern "C" int prim_sincos(const float *in, float *s, float *c, int n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_sincos, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, in, s, c, n);
    return launched();
}

extern "C" int prim_split16(const float *in, unsigned *hi, unsigned *lo, int n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_split16, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float2 *>(in), hi, lo, n);
    return launched();
}

extern "C" int prim_split16j(const float *in, unsigned *hi, unsigned *lo, int n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_split16j, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float2 *>(in), hi, lo, n);
    return launched();
}
