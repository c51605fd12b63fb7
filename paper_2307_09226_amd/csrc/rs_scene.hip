// Synthetic scenes on the device: each pixel of a g_az x g_el grid casts a
// ray from the origin into an axis-aligned room and an optional ellipsoid
// pedestrian (the stand-in for the rendered image whose pixels the paper
// turns into scatterers, Sec. II).  A thread takes one pixel of a few
// frames (its ray direction, two binary64 sincospi, is shared by them);
// binary64 geometry, float32 structure-of-arrays output (20 bytes written
// and 4 read per pixel and frame).
#include "rs_api_internal.h"

#include <cmath>
#include <vector>

namespace {

constexpr int kFramesPerThread = 4;  // frames one thread casts along its pixel's ray

// The ray of one pixel against one frame's room and pedestrian; writes the
// pixel's scatterer at index g of the output arrays.
__device__ __forceinline__ void cast(const rs_scene &S, const double (&u)[3], int64_t g, const float *noise,
                                     float *ox, float *oy, float *oz, float *oamp, float *ovr)
{
    // nearest wall: planes x = +-W/2, y = D, z = +-H/2
    const double inf = __builtin_huge_val();
    const double tx = u[0] > 0 ? (S.room_w / 2) / u[0] : (u[0] < 0 ? (-S.room_w / 2) / u[0] : inf);
    const double ty = u[1] > 0 ? S.room_d / u[1] : inf;
    const double tz = u[2] > 0 ? (S.room_h / 2) / u[2] : (u[2] < 0 ? (-S.room_h / 2) / u[2] : inf);
    double t = tx, cosi = fabs(u[0]);
    if (ty < t) {
        t = ty;
        cosi = fabs(u[1]);
    }
    if (tz < t) {
        t = tz;
        cosi = fabs(u[2]);
    }
    double v = 0.0;
    if (S.pedestrian) {
        // |(t u - c) / s| = 1:  a t^2 + b t + cc = 0 with d = u / s, o = -c / s
        double d[3], o[3];
        for (int k = 0; k < 3; ++k) {
            d[k] = u[k] / S.semi_axes[k];
            o[k] = -S.centre[k] / S.semi_axes[k];
        }
        const double a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double b = 2.0 * (d[0] * o[0] + d[1] * o[1] + d[2] * o[2]);
        const double cc = (o[0] * o[0] + o[1] * o[1] + o[2] * o[2]) - 1.0;
        const double disc = b * b - 4.0 * a * cc;
        if (disc > 0) {
            const double sq = sqrt(disc);
            const double t1 = (-b - sq) / (2.0 * a), t2 = (-b + sq) / (2.0 * a);
            const double te = t1 > 0 ? t1 : t2;
            if (te > 0 && te < t) {
                // outward normal (x - c) / s^2 at the hit, normalised
                double nrm[3], nn = 0.0;
                for (int k = 0; k < 3; ++k) {
                    nrm[k] = (u[k] * te - S.centre[k]) / (S.semi_axes[k] * S.semi_axes[k]);
                    nn += nrm[k] * nrm[k];
                }
                nn = sqrt(nn);
                t = te;
                cosi = fabs((u[0] * nrm[0] + u[1] * nrm[1] + u[2] * nrm[2]) / nn);
                v = -(u[0] * S.velocity[0] + u[1] * S.velocity[1] + u[2] * S.velocity[2]);
            }
        }
    }
    const double nz = noise ? (double)noise[g] : 1.0;
    ox[g] = (float)(u[0] * t);
    oy[g] = (float)(u[1] * t);
    oz[g] = (float)(u[2] * t);
    oamp[g] = (float)(cosi / (t * t) * nz);
    ovr[g] = (float)v;
}

// Thread = (pixel p, group of kFramesPerThread frames): the pixel's ray
// direction is evaluated once and cast into each frame of the group.
__global__ __launch_bounds__(256) void k_render(const rs_scene *scenes, int64_t P, int nframes, int64_t threads,
                                                int g_az, int g_el, const float *noise, float *ox, float *oy,
                                                float *oz, float *oamp, float *ovr)
{
    const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gi >= threads) return;
    const int64_t p = gi % P;
    const int f0 = (int)(gi / P) * kFramesPerThread;
    const int i = (int)(p % g_az), j = (int)(p / g_az);
    // ray direction of the pixel centre (angles in degrees / 180 = half turns)
    const double az = (-60.0 + 120.0 * ((double)i + 0.5) / (double)g_az) / 180.0;
    const double el = (-30.0 + 60.0 * ((double)j + 0.5) / (double)g_el) / 180.0;
    double saz, caz, sel, cel;
    sincospi(az, &saz, &caz);
    sincospi(el, &sel, &cel);
    const double u[3] = {cel * saz, cel * caz, sel};
    const int f1 = min(nframes, f0 + kFramesPerThread);
    for (int f = f0; f < f1; ++f) cast(scenes[f], u, (int64_t)f * P + p, noise, ox, oy, oz, oamp, ovr);
}

bool pos_finite(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

extern "C" rs_status rs_render_scenes(const rs_scene *scenes, int32_t nframes, int32_t g_az, int32_t g_el,
                                      const float *noise, float *x, float *y, float *z, float *amp, float *vr,
                                      void *stream)
{
    if (nframes < 0) return rs_fail(RS_E_INVALID, "nframes < 0");
    if (nframes == 0) return RS_OK;
    if (!scenes || !x || !y || !z || !amp || !vr) return rs_fail(RS_E_INVALID, "NULL scene or output array");
    if (g_az < 1 || g_el < 1) return rs_fail(RS_E_INVALID, "grid sides must be >= 1");
    const int64_t P = (int64_t)g_az * g_el;
    if (P * nframes > ((int64_t)1 << 31)) return rs_fail(RS_E_INVALID, "more than 2^31 pixels");
    for (int f = 0; f < nframes; ++f) {
        const rs_scene &S = scenes[f];
        if (!pos_finite(S.room_w) || !pos_finite(S.room_d) || !pos_finite(S.room_h))
            return rs_fail(RS_E_INVALID, "frame %d: room sides must be finite and > 0", f);
        if (S.pedestrian)
            for (int k = 0; k < 3; ++k)
                if (!pos_finite(S.semi_axes[k]) || !std::isfinite(S.centre[k]) || !std::isfinite(S.velocity[k]))
                    return rs_fail(RS_E_INVALID, "frame %d: bad pedestrian", f);
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rs_scene *d = nullptr;
    const size_t bytes = sizeof(rs_scene) * (size_t)nframes;
    if (hipMallocAsync(reinterpret_cast<void **>(&d), bytes, st) != hipSuccess)
        return rs_fail(RS_E_NOMEM, "stream-ordered allocation of %zu bytes failed", bytes);
    rs_status s = RS_OK;
    hipError_t e = hipMemcpyAsync(d, scenes, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) s = rs_fail(RS_E_DEVICE, "scene copy: %s", hipGetErrorString(e));
    if (s == RS_OK) {
        const int64_t threads = P * ((nframes + kFramesPerThread - 1) / kFramesPerThread);
        const bool timed = rs_timer_begin(st);
        hipLaunchKernelGGL(k_render, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, d, P, nframes,
                           threads, g_az, g_el, noise, x, y, z, amp, vr);
        e = hipGetLastError();
        if (e != hipSuccess) s = rs_fail(RS_E_DEVICE, "render launch: %s", hipGetErrorString(e));
        else if (timed) rs_timer_end(st);
    }
    e = hipFreeAsync(d, st);
    if (e != hipSuccess && s == RS_OK) s = rs_fail(RS_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    return s;
}
