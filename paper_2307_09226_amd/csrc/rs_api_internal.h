// Host-side internals shared by rs_api.hip and rs_session.hip.
#pragma once
#include "../../include/rs.h"
#include "rs_internal.h"

struct rs_plan {
    int device = 0;
    int ncu = 0;
    int32_t M = 0, N = 0, C = 0, Ns = 0, L = 0, carrier = 1;
    double fc = 0, mu = 0, Fs = 0, Tb = 0, c0 = 0;
    double Kc = 0, Kb = 0, Kd = 0;  // binary64 phase constants
    double Kf = 0, Krvp = 0;        // ... of the intra-chirp Doppler and video-phase variants
    double Ka = 0;                  // 2 fc / c0, the far-field angle term (not switched by carrier)
    int32_t model = 0;              // rs_model_flags
    double *d_ant = nullptr;        // device tx[M][3] then rx[N][3]
    rs_form form = RS_FORM_MFMA_SPLIT16;
    rs_dtype dtype = RS_C64;
    int64_t max_pixels = 0;
    // tile configuration
    int tn = 0, tl = 0, wn = 0;     // tile rows (n), tile columns (l), rows per wave (MFMA)
    int nw = 4;                     // waves per workgroup (MFMA)
    int interleave = 0;             // MFMA, NW = 8: 1 = software-pipelined schedule, 0 = phase-shifted waves
    int n_tiles = 0, l_tiles = 0;
    int64_t items_target = 0;       // work items aimed at for one cube
    int min_chunk = 0;              // smallest pixel chunk
    int occupancy = 1;              // resident workgroups per CU of the main kernel
    // NUFFT form
    double nu_tol = 0;              // requested tolerance
    int nu_w = 0;                   // kernel width (cells)
    double nu_beta = 0;             // kernel shape
    int nu_n1 = 0, nu_n2 = 0;       // grid size along n and l
    float *d_deconv = nullptr;      // device: h / phi_hat for n [Ns] then for l [L]
};

rs_status rs_fail(rs_status s, const char *fmt, ...);

// Makes `dev` current for a call and restores the caller's device on exit.
struct device_guard {
    int prev = -1;
    rs_status st = RS_OK;
    explicit device_guard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev && hipSetDevice(dev) != hipSuccess)
            st = rs_fail(RS_E_DEVICE, "hipSetDevice(%d) failed", dev);
    }
    ~device_guard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};
void rs_choose_tiles(rs_plan *pl);
rs_status rs_plan_chunking(const rs_plan *pl, int64_t P, int32_t *S, int32_t *chunk);
size_t rs_partial_bytes(const rs_plan *pl, int32_t S);
size_t rs_workspace_bytes(const rs_plan *pl, int32_t S);   // partials (+ chunk scales with strengths per block)
size_t rs_scale_bytes(int32_t S);                            // a chunk-scale array
int32_t rs_steps_per_chunk(const rs_plan *pl, int32_t chunk);
rs_status rs_launch_scale_checked(const rs_launch &L, bool block_strength, hipStream_t st);
rs_job rs_make_job(const rs_plan *pl, const rs_pixels *px, void *cube, void *partial,
                   int32_t S, int32_t chunk);
rs_status rs_check_pixels(const rs_plan *pl, const rs_pixels *px);
// The calling thread's kernel timer (rs_kernel_timer_attach): an event
// before a launch on st when the timer has room (returns whether it took
// one), and the closing event after it.
bool rs_timer_begin(hipStream_t st);
void rs_timer_end(hipStream_t st);
// block_strength: some job of the launch has strengths per block
rs_status rs_launch_main(const rs_plan *pl, const rs_launch &L, bool block_strength, int grid, hipStream_t st);
rs_status rs_launch_reduce_checked(const rs_plan *pl, const rs_launch &L, hipStream_t st);
// NUFFT form (rs_nufft.hip)
void rs_nufft_params(double tol, int *w, double *beta);
int rs_nufft_fine(int N, int w);
void rs_nufft_deconv(int N, int n, int w, double beta, float *out);
size_t rs_nufft_workspace(const rs_plan *pl, int64_t P);
rs_status rs_nufft_enqueue(const rs_plan *pl, const rs_pixels *px, void *cube, void *ws, hipStream_t st);
