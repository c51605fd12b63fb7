// Internal definitions shared by the host library and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

// One cube request inside a launch.  Every field is plain data so that a
// table of jobs can be copied to the device or passed by value.
struct rs_job {
    const float *x, *y, *z, *amp, *vr; // device SoA pixels
    int64_t P;
    void *cube;                // output [C][L][Ns] complex64/complex128
    void *partial;             // split-K partials [S][C][L][Ns] complex (f32 or f64)
    const double *ant;         // device antenna table: tx[M][3] then rx[N][3]
    double Kc, Kb, Kd;         // phase constants of the binary64 recipe
    double Kf, Krvp;           // constants of the intra-chirp / video-phase variants
    double Ka;                 // 2 fc / c0 whatever the carrier switch (far-field angle term)
    int32_t M, N, Ns, L;
    int32_t n_tiles, l_tiles;  // output tiles along n and l
    int32_t S, chunk;          // pixel chunks and pixels per chunk
    int64_t item_begin;        // first launch-global work item of this job
    int64_t item_first;        // first job-local work item covered by this launch
    int64_t item_count;        // job-local work items covered by this launch
    int64_t out_begin;         // first launch-global output entry (reduce launches)
    int64_t chunk_begin;       // first launch-global pixel chunk (chunk-scale launches)
    int32_t *scale;            // [S] per-chunk strength exponent shift (matrix-core form)
    int32_t seg_begin, seg_end;  // 16-pixel steps of every chunk covered by this launch
    int32_t dtype;             // 0 = complex64, 1 = complex128
    int32_t model;             // signal-model variant flags (rs_model_flags)
    int64_t amp_lstride;       // P when strengths vary over the blocks (amp[l * P + p]), else 0
};

// Job table of one launch.  With jobs == nullptr the single job `inline_job`
// (passed by value) is used.  counter != nullptr selects a persistent grid
// whose workgroups claim items with an atomic counter; otherwise work item =
// blockIdx.x.
struct rs_launch {
    const rs_job *jobs;
    int32_t njobs;
    int32_t pad_;
    int64_t total;      // work items (main kernels) or output entries (reduce)
    int *counter;
    rs_job inline_job;
};

__device__ __forceinline__ const rs_job &rs_job_of(const rs_launch &L, int j)
{
    return L.jobs ? L.jobs[j] : L.inline_job;
}

enum { RS_BY_ITEM = 0, RS_BY_OUT = 1, RS_BY_CHUNK = 2 };

// Largest j with begin(j) <= g (jobs sorted by begin); begin = item_begin,
// out_begin or chunk_begin.
template <int BY>
__device__ __forceinline__ int rs_find_job(const rs_launch &L, int64_t g)
{
    if (!L.jobs) return 0;
    int lo = 0, hi = L.njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        const rs_job &J = L.jobs[mid];
        int64_t b = BY == RS_BY_ITEM ? J.item_begin : (BY == RS_BY_OUT ? J.out_begin : J.chunk_begin);
        if (b <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Work-item decomposition, identical for every form: local item index ->
// (channel c, n tile, l tile, chunk s), chunk fastest.
struct rs_item {
    int c, nt, lt, s;
};

__device__ __forceinline__ rs_item rs_decode_item(const rs_job &J, int64_t local)
{
    rs_item it;
    it.s = (int)(local % J.S);
    int64_t t = local / J.S;
    it.lt = (int)(t % J.l_tiles);
    t /= J.l_tiles;
    it.nt = (int)(t % J.n_tiles);
    it.c = (int)(t / J.n_tiles);
    return it;
}

// Kernel entry points (defined in the .hip files, launched by rs_api.hip).
void rs_launch_plain(const rs_launch &L, int tl, int grid, hipStream_t st);
// block_strength: some job of the launch has amp_lstride != 0
// interleave: software-pipelined schedule also for NW = 8 (else phase-shifted waves)
void rs_launch_mfma(const rs_launch &L, int wn, int tl, int nw, bool interleave, bool block_strength, int grid,
                    hipStream_t st);
bool rs_mfma_shape_supported(int wn, int tl, int nw);
void rs_launch_reduce(const rs_launch &L, int form, hipStream_t st);
// block_strength: some job of the launch has strengths per block
void rs_launch_chunk_scale(const rs_launch &L, bool block_strength, hipStream_t st);
void rs_launch_zero_int(int *p, int n, hipStream_t st);
