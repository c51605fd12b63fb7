// Host side of the C ABI (include/rs.h): plans, single-frame and batched
// synthesis.  All device work is enqueued on the caller's stream.
#include "rs_api_internal.h"

#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

static thread_local std::string tl_error;

rs_status rs_fail(rs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    tl_error = buf;
    return s;
}

extern "C" const char *rs_last_error(void) { return tl_error.c_str(); }
extern "C" const char *rs_version(void) { return "rs 0.1 gfx950"; }

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int64_t round_up(int64_t v, int64_t m) { return ((v + m - 1) / m) * m; }

}  // namespace

// ---------------------------------------------------------------- plans ----

rs_status rs_plan_chunking(const rs_plan *pl, int64_t P, int32_t *S, int32_t *chunk)
{
    if (P <= 0) {
        *S = 0;
        *chunk = pl->min_chunk;
        return RS_OK;
    }
    const int64_t tiles = (int64_t)pl->C * pl->n_tiles * pl->l_tiles;
    int64_t s_target = pl->items_target / tiles;
    if (s_target < 1) s_target = 1;
    int64_t ch = (P + s_target - 1) / s_target;
    ch = round_up(ch, 16);
    if (ch < pl->min_chunk) ch = pl->min_chunk;
    if (ch > (int64_t)1 << 30) return rs_fail(RS_E_INVALID, "pixel count too large");
    *chunk = (int32_t)ch;
    *S = (int32_t)((P + ch - 1) / ch);
    return RS_OK;
}

size_t rs_partial_bytes(const rs_plan *pl, int32_t S)
{
    const size_t elem = pl->form == RS_FORM_FP64_DIRECT ? 16 : 8;
    const size_t b = (size_t)S * pl->C * pl->L * pl->Ns * elem;
    return (b + 255) & ~(size_t)255;
}

size_t rs_scale_bytes(int32_t S) { return ((size_t)S * 4 + 255) & ~(size_t)255; }

size_t rs_workspace_bytes(const rs_plan *pl, int32_t S)
{
    size_t scale = pl->form == RS_FORM_MFMA_SPLIT16 && (pl->model & RS_MODEL_BLOCK_STRENGTH)
                       ? (((size_t)S * 4 + 255) & ~(size_t)255)
                       : 0;
    return rs_partial_bytes(pl, S) + scale;
}

int32_t rs_steps_per_chunk(const rs_plan *pl, int32_t chunk)
{
    (void)pl;
    return (chunk + 15) / 16;
}

rs_job rs_make_job(const rs_plan *pl, const rs_pixels *px, void *cube, void *partial,
                   int32_t S, int32_t chunk)
{
    rs_job j;
    std::memset(&j, 0, sizeof j);
    j.x = px->x;
    j.y = px->y;
    j.z = px->z;
    j.amp = px->amp;
    j.vr = px->vr;
    j.P = px->P;
    j.cube = cube;
    j.partial = partial;
    j.ant = pl->d_ant;
    j.Kc = pl->Kc;
    j.Kb = pl->Kb;
    j.Kd = pl->Kd;
    j.Kf = pl->Kf;
    j.Krvp = pl->Krvp;
    j.Ka = pl->Ka;
    j.model = pl->model;
    j.amp_lstride = (pl->model & RS_MODEL_BLOCK_STRENGTH) ? px->P : 0;
    j.M = pl->M;
    j.N = pl->N;
    j.Ns = pl->Ns;
    j.L = pl->L;
    j.n_tiles = pl->n_tiles;
    j.l_tiles = pl->l_tiles;
    j.S = S;
    j.chunk = chunk;
    j.item_count = (int64_t)S * pl->C * pl->n_tiles * pl->l_tiles;
    j.dtype = pl->dtype == RS_C128 ? 1 : 0;
    j.seg_begin = 0;
    j.seg_end = 0x7fffffff;
    // chunk scales come from k_chunk_scale only for strengths per block; the
    // main kernel finds the others itself
    j.scale = pl->form == RS_FORM_MFMA_SPLIT16 && partial && (pl->model & RS_MODEL_BLOCK_STRENGTH)
                  ? reinterpret_cast<int32_t *>(static_cast<char *>(partial) + rs_partial_bytes(pl, S))
                  : nullptr;
    return j;
}

rs_status rs_launch_scale_checked(const rs_launch &L, bool block_strength, hipStream_t st)
{
    rs_launch_chunk_scale(L, block_strength, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "chunk-scale launch: %s", hipGetErrorString(e));
    return RS_OK;
}

rs_status rs_check_pixels(const rs_plan *pl, const rs_pixels *px)
{
    if (!px) return rs_fail(RS_E_INVALID, "pixels is NULL");
    if (px->P < 0) return rs_fail(RS_E_INVALID, "P < 0");
    if (px->P > pl->max_pixels)
        return rs_fail(RS_E_INVALID, "P = %lld exceeds the plan's max_pixels = %lld",
                       (long long)px->P, (long long)pl->max_pixels);
    if (px->P > 0 && (!px->x || !px->y || !px->z || !px->amp || !px->vr))
        return rs_fail(RS_E_INVALID, "NULL pixel array with P > 0");
    return RS_OK;
}

// ---------------------------------------------------------- kernel timer --

struct rs_kernel_timer {
    int device = 0;
    int cap = 0, used = 0;
    std::vector<hipEvent_t> ev;  // begin/end pairs
};

static thread_local rs_kernel_timer *tl_timer = nullptr;

extern "C" rs_status rs_kernel_timer_create(int32_t capacity, rs_kernel_timer **out)
{
    if (!out || capacity < 1 || capacity > (1 << 20)) return rs_fail(RS_E_INVALID, "bad argument");
    *out = nullptr;
    rs_kernel_timer *t = new (std::nothrow) rs_kernel_timer();
    if (!t) return rs_fail(RS_E_NOMEM, "host allocation failed");
    (void)hipGetDevice(&t->device);
    t->cap = capacity;
    t->ev.resize(2 * (size_t)capacity, nullptr);
    for (auto &e : t->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            rs_kernel_timer_destroy(t);
            return rs_fail(RS_E_DEVICE, "hipEventCreate failed");
        }
    *out = t;
    return RS_OK;
}

extern "C" rs_status rs_kernel_timer_attach(rs_kernel_timer *t)
{
    tl_timer = t;
    return RS_OK;
}

extern "C" rs_status rs_kernel_timer_read(rs_kernel_timer *t, double *ms, int32_t max, int32_t *count)
{
    if (!t || !count || max < 0) return rs_fail(RS_E_INVALID, "bad argument");
    for (int i = 0; i < t->used; ++i) {
        float v = 0.f;
        if (hipEventSynchronize(t->ev[2 * i + 1]) != hipSuccess ||
            hipEventElapsedTime(&v, t->ev[2 * i], t->ev[2 * i + 1]) != hipSuccess)
            return rs_fail(RS_E_DEVICE, "event timing failed");
        if (ms && i < max) ms[i] = v;
    }
    *count = t->used;
    t->used = 0;
    return RS_OK;
}

extern "C" void rs_kernel_timer_destroy(rs_kernel_timer *t)
{
    if (!t) return;
    if (tl_timer == t) tl_timer = nullptr;
    for (auto &e : t->ev)
        if (e) (void)hipEventDestroy(e);
    delete t;
}

bool rs_timer_begin(hipStream_t st)
{
    rs_kernel_timer *tm = tl_timer;
    if (!tm || tm->used >= tm->cap) return false;
    (void)hipEventRecord(tm->ev[2 * tm->used], st);
    return true;
}

void rs_timer_end(hipStream_t st)
{
    rs_kernel_timer *tm = tl_timer;
    (void)hipEventRecord(tm->ev[2 * tm->used + 1], st);
    tm->used++;
}

rs_status rs_launch_main(const rs_plan *pl, const rs_launch &L, bool block_strength, int grid, hipStream_t st)
{
    if (L.total <= 0) return RS_OK;
    const bool timed = rs_timer_begin(st);
    if (pl->form == RS_FORM_FP64_DIRECT)
        rs_launch_plain(L, pl->tl, grid, st);
    else
        rs_launch_mfma(L, pl->wn, pl->tl, pl->nw, pl->interleave != 0, block_strength, grid, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "main kernel launch: %s", hipGetErrorString(e));
    if (timed) rs_timer_end(st);
    return RS_OK;
}

rs_status rs_launch_reduce_checked(const rs_plan *pl, const rs_launch &L, hipStream_t st)
{
    rs_launch_reduce(L, pl->form == RS_FORM_FP64_DIRECT ? 0 : 1, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rs_fail(RS_E_DEVICE, "reduce launch: %s", hipGetErrorString(e));
    return RS_OK;
}

static rs_status plan_common(const rs_radar *r, rs_form form, rs_dtype dtype, int64_t max_pixels, double tol,
                             rs_plan **out);

extern "C" rs_status rs_cube_plan(const rs_radar *r, rs_form form, rs_dtype dtype,
                                  int64_t max_pixels, rs_plan **out)
{
    return plan_common(r, form, dtype, max_pixels, 1e-6, out);
}

extern "C" rs_status rs_cube_plan_nufft(const rs_radar *r, rs_dtype dtype, int64_t max_pixels, double tolerance,
                                        rs_plan **out)
{
    if (!(tolerance >= 1e-7 && tolerance < 0.5))
        return rs_fail(RS_E_INVALID, "NUFFT tolerance must lie in [1e-7, 0.5)");
    return plan_common(r, RS_FORM_NUFFT, dtype, max_pixels, tolerance, out);
}

static rs_status plan_common(const rs_radar *r, rs_form form, rs_dtype dtype, int64_t max_pixels, double tol,
                             rs_plan **out)
{
    if (!out) return rs_fail(RS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!r) return rs_fail(RS_E_INVALID, "radar is NULL");
    if (r->M < 1 || r->N < 1 || r->Ns < 1 || r->L < 1)
        return rs_fail(RS_E_INVALID, "M, N, Ns and L must be >= 1");
    const int64_t cells = (int64_t)r->M * r->N * r->L * r->Ns;
    if (cells > ((int64_t)1 << 31)) return rs_fail(RS_E_INVALID, "cube larger than 2^31 entries");
    if (r->M > 256 || r->N > 256) return rs_fail(RS_E_INVALID, "at most 256 Tx and 256 Rx");
    if (!finite_pos(r->Fs) || !finite_pos(r->Tb) || !finite_pos(r->c0))
        return rs_fail(RS_E_INVALID, "Fs, Tb and c0 must be finite and > 0");
    if (!std::isfinite(r->fc) || !std::isfinite(r->mu))
        return rs_fail(RS_E_INVALID, "fc and mu must be finite");
    if (!r->tx_xyz || !r->rx_xyz) return rs_fail(RS_E_INVALID, "tx_xyz / rx_xyz is NULL");
    for (int i = 0; i < 3 * r->M; ++i)
        if (!std::isfinite(r->tx_xyz[i])) return rs_fail(RS_E_INVALID, "non-finite Tx position");
    for (int i = 0; i < 3 * r->N; ++i)
        if (!std::isfinite(r->rx_xyz[i])) return rs_fail(RS_E_INVALID, "non-finite Rx position");
    if (form != RS_FORM_FP64_DIRECT && form != RS_FORM_MFMA_SPLIT16 && form != RS_FORM_NUFFT)
        return rs_fail(RS_E_INVALID, "unknown form");
    if (dtype != RS_C64 && dtype != RS_C128) return rs_fail(RS_E_INVALID, "unknown dtype");
    if (r->model < 0 || (r->model & ~(RS_MODEL_FAR_FIELD | RS_MODEL_TDM_SLOT | RS_MODEL_INTRA_CHIRP | RS_MODEL_RVP |
                                      RS_MODEL_BLOCK_STRENGTH)))
        return rs_fail(RS_E_INVALID, "unknown model flags 0x%x", (unsigned)r->model);
    if (max_pixels < 0) return rs_fail(RS_E_INVALID, "max_pixels < 0");
    if (max_pixels > ((int64_t)1 << 40)) return rs_fail(RS_E_INVALID, "max_pixels too large");
    if (form == RS_FORM_NUFFT) {
        if (r->model & RS_MODEL_BLOCK_STRENGTH)
            return rs_fail(RS_E_UNSUPPORTED, "the NUFFT form needs strengths constant over the blocks");
        if (r->Ns > 2048 || r->L > 2048) return rs_fail(RS_E_UNSUPPORTED, "the NUFFT form serves Ns, L <= 2048");
        if ((int64_t)r->M * r->N > 65535) return rs_fail(RS_E_UNSUPPORTED, "the NUFFT form serves <= 65535 channels");
        if (max_pixels > ((int64_t)1 << 31) - 1)
            return rs_fail(RS_E_UNSUPPORTED, "the NUFFT form serves max_pixels < 2^31");
        // its FFT passes launch up to one workgroup of 256 per grid row and
        // per fast-time sample and channel: both counts stay below 2^24
        int w = 0;
        double beta = 0.0;
        rs_nufft_params(tol, &w, &beta);
        const int64_t C = (int64_t)r->M * r->N;
        if (C * rs_nufft_fine(r->L, w) >= ((int64_t)1 << 24) || C * r->Ns >= ((int64_t)1 << 24))
            return rs_fail(RS_E_UNSUPPORTED, "the NUFFT form serves channels x grid rows and channels x Ns below 2^24");
    }

    rs_plan *pl = new (std::nothrow) rs_plan();
    if (!pl) return rs_fail(RS_E_NOMEM, "host allocation failed");
    if (hipGetDevice(&pl->device) != hipSuccess) {
        delete pl;
        return rs_fail(RS_E_DEVICE, "no HIP device");
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess ||
        ncu <= 0) {
        delete pl;
        return rs_fail(RS_E_DEVICE, "cannot query the compute-unit count");
    }
    pl->ncu = ncu;
    pl->M = r->M;
    pl->N = r->N;
    pl->C = r->M * r->N;
    pl->Ns = r->Ns;
    pl->L = r->L;
    pl->fc = r->fc;
    pl->mu = r->mu;
    pl->Fs = r->Fs;
    pl->Tb = r->Tb;
    pl->c0 = r->c0;
    pl->carrier = r->carrier_phase ? 1 : 0;
    // binary64 phase constants of the recipe (same expressions as the
    // reference definition: Kc = 2 fc / c0, Kb = 2 mu / (c0 Fs),
    // Kd = 2 fc Tb / c0)
    pl->Kc = pl->carrier ? (2.0 * r->fc) / r->c0 : 0.0;
    pl->Kb = (2.0 * r->mu) / (r->c0 * r->Fs);
    pl->Kd = ((2.0 * r->fc) * r->Tb) / r->c0;
    pl->Kf = (2.0 * r->fc) / (r->c0 * r->Fs);
    pl->Krvp = (2.0 * r->mu) / (r->c0 * r->c0);
    pl->Ka = (2.0 * r->fc) / r->c0;
    pl->model = r->model;
    pl->form = form;
    pl->dtype = dtype;
    pl->max_pixels = max_pixels;
    rs_choose_tiles(pl);
    std::vector<float> deconv;
    if (form == RS_FORM_NUFFT) {
        pl->nu_tol = tol;
        rs_nufft_params(tol, &pl->nu_w, &pl->nu_beta);
        pl->nu_n1 = rs_nufft_fine(r->Ns, pl->nu_w);
        pl->nu_n2 = rs_nufft_fine(r->L, pl->nu_w);
        deconv.resize((size_t)r->Ns + r->L);
        rs_nufft_deconv(r->Ns, pl->nu_n1, pl->nu_w, pl->nu_beta, deconv.data());
        rs_nufft_deconv(r->L, pl->nu_n2, pl->nu_w, pl->nu_beta, deconv.data() + r->Ns);
    }

    std::vector<double> ant(3 * (r->M + r->N));
    std::memcpy(ant.data(), r->tx_xyz, sizeof(double) * 3 * r->M);
    std::memcpy(ant.data() + 3 * r->M, r->rx_xyz, sizeof(double) * 3 * r->N);
    if (hipMalloc(&pl->d_ant, ant.size() * sizeof(double)) != hipSuccess) {
        delete pl;
        return rs_fail(RS_E_NOMEM, "hipMalloc of the antenna table failed");
    }
    if (hipMemcpy(pl->d_ant, ant.data(), ant.size() * sizeof(double), hipMemcpyHostToDevice) !=
        hipSuccess) {
        (void)hipFree(pl->d_ant);
        delete pl;
        return rs_fail(RS_E_DEVICE, "copy of the antenna table failed");
    }
    if (!deconv.empty()) {
        const size_t nb = deconv.size() * sizeof(float);
        if (hipMalloc(&pl->d_deconv, nb) != hipSuccess) {
            pl->d_deconv = nullptr;
            rs_plan_destroy(pl);
            return rs_fail(RS_E_NOMEM, "hipMalloc of the NUFFT deconvolution table failed");
        }
        if (hipMemcpy(pl->d_deconv, deconv.data(), nb, hipMemcpyHostToDevice) != hipSuccess) {
            rs_plan_destroy(pl);
            return rs_fail(RS_E_DEVICE, "copy of the NUFFT deconvolution table failed");
        }
    }
    *out = pl;
    return RS_OK;
}

void rs_choose_tiles(rs_plan *pl)
{
    if (pl->form == RS_FORM_FP64_DIRECT) {
        pl->tn = 64;
        pl->tl = pl->L <= 64 ? 64 : 128;
        pl->wn = 0;
        pl->items_target = (int64_t)pl->ncu * 4;
        pl->min_chunk = 256;
        pl->occupancy = 2;
    } else {
        // Matrix-core tiles: TL columns (l), NW waves of WN rows (n).
        //   L > 64: 128 columns; 8 waves x 32 rows (two waves per SIMD) when
        //           Ns > 128, else 4 waves x 32 rows
        //   L <= 64: 64 columns; 4 waves x 64 rows (Ns > 128) or x 32 rows
        int wn, tl, nw;
        if (pl->L > 64) {
            tl = 128;
            wn = 32;
            nw = pl->Ns > 128 ? 8 : 4;
        } else {
            tl = 64;
            nw = 4;
            wn = pl->Ns > 128 ? 64 : 32;
        }
        pl->wn = wn;
        pl->tl = tl;
        pl->nw = nw;
        pl->interleave = 0;
        pl->tn = nw * wn;
        pl->items_target = pl->ncu;
        pl->min_chunk = 1024;
        pl->occupancy = 1;
    }
    pl->n_tiles = (pl->Ns + pl->tn - 1) / pl->tn;
    pl->l_tiles = (pl->L + pl->tl - 1) / pl->tl;
}

extern "C" void rs_plan_destroy(rs_plan *pl)
{
    if (!pl) return;
    if (pl->d_ant || pl->d_deconv) {
        device_guard g(pl->device);
        if (pl->d_ant) (void)hipFree(pl->d_ant);
        if (pl->d_deconv) (void)hipFree(pl->d_deconv);
    }
    delete pl;
}

extern "C" rs_status rs_plan_workspace_bytes(const rs_plan *pl, int64_t P, size_t *bytes)
{
    if (!pl || !bytes) return rs_fail(RS_E_INVALID, "NULL argument");
    if (P < 0 || P > pl->max_pixels) return rs_fail(RS_E_INVALID, "P out of range");
    if (pl->form == RS_FORM_NUFFT) {
        *bytes = rs_nufft_workspace(pl, P);
        return RS_OK;
    }
    int32_t S, chunk;
    rs_status s = rs_plan_chunking(pl, P, &S, &chunk);
    if (s != RS_OK) return s;
    *bytes = rs_workspace_bytes(pl, S);
    return RS_OK;
}

extern "C" rs_status rs_plan_describe(const rs_plan *pl, int64_t P, char *buf, size_t len)
{
    if (!pl || !buf) return rs_fail(RS_E_INVALID, "NULL argument");
    if (P < 0) return rs_fail(RS_E_INVALID, "P < 0");
    int32_t S = 0, chunk = 0;
    rs_status s = rs_plan_chunking(pl, P, &S, &chunk);
    if (s != RS_OK) return s;
    if (len == 0) return RS_OK;
    if (pl->form == RS_FORM_NUFFT) {
        snprintf(buf, len,
                 "{\"form\": \"nufft\", \"dtype\": \"%s\", \"C\": %d, \"Ns\": %d, \"L\": %d, "
                 "\"tolerance\": %.3g, \"kernel_width\": %d, \"kernel_beta\": %.4g, \"grid_n\": %d, "
                 "\"grid_l\": %d, \"pixel_blocks\": %lld, \"cus\": %d, \"model\": %d}",
                 pl->dtype == RS_C128 ? "complex128" : "complex64", pl->C, pl->Ns, pl->L, pl->nu_tol, pl->nu_w,
                 pl->nu_beta, pl->nu_n1, pl->nu_n2, (long long)((P + 255) / 256), pl->ncu, pl->model);
        return RS_OK;
    }
    snprintf(buf, len,
             "{\"form\": \"%s\", \"dtype\": \"%s\", \"C\": %d, \"Ns\": %d, \"L\": %d, "
             "\"tile_n\": %d, \"tile_l\": %d, \"wave_rows\": %d, \"waves\": %d, \"n_tiles\": %d, \"l_tiles\": %d, "
             "\"schedule\": \"%s\", \"chunks\": %d, \"chunk_pixels\": %d, \"items\": %lld, \"cus\": %d, "
             "\"model\": %d}",
             pl->form == RS_FORM_FP64_DIRECT ? "fp64_direct" : "mfma_split16",
             pl->dtype == RS_C128 ? "complex128" : "complex64", pl->C, pl->Ns, pl->L, pl->tn,
             pl->tl, pl->wn, pl->form == RS_FORM_FP64_DIRECT ? 4 : pl->nw, pl->n_tiles, pl->l_tiles,
             pl->form == RS_FORM_FP64_DIRECT ? "lds_blocks"
                                              : (pl->nw == 8 && !pl->interleave ? "phase_shifted" : "pipelined"),
             S, chunk, (long long)S * pl->C * pl->n_tiles * pl->l_tiles, pl->ncu, pl->model);
    return RS_OK;
}

// ----------------------------------------------------------- tile tuning ----

static void set_mfma_shape(rs_plan *pl, int wn, int tl, int nw, int interleave)
{
    pl->wn = wn;
    pl->tl = tl;
    pl->nw = nw;
    pl->interleave = nw == 8 ? interleave : 0;
    pl->tn = nw * wn;
    pl->n_tiles = (pl->Ns + pl->tn - 1) / pl->tn;
    pl->l_tiles = (pl->L + pl->tl - 1) / pl->tl;
}

// Tile configurations as text: "WNxTLxNW" (rows per wave x columns x
// waves), with an 'i' suffix for the software-pipelined schedule on 8-wave
// shapes, which otherwise run phase-shifted waves (4-wave shapes always run
// the pipelined schedule and take the suffix without effect).
static bool parse_tile(const char *s, int *wn, int *tl, int *nw, int *il)
{
    int a = 0, b = 0, c = 0, n = 0;
    if (!s || std::sscanf(s, "%dx%dx%d%n", &a, &b, &c, &n) != 3) return false;
    int i = 0;
    if (s[n] == 'i') {
        i = 1;
        ++n;
    }
    if (s[n] != '\0' || !rs_mfma_shape_supported(a, b, c)) return false;
    *wn = a;
    *tl = b;
    *nw = c;
    *il = c == 8 ? i : 0;
    return true;
}

static void format_tile(const rs_plan *pl, char *buf, size_t len)
{
    snprintf(buf, len, "%dx%dx%d%s", pl->wn, pl->tl, pl->nw, pl->nw == 8 && pl->interleave ? "i" : "");
}

extern "C" rs_status rs_plan_set_tile(rs_plan *pl, const char *tile)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (pl->form != RS_FORM_MFMA_SPLIT16) return rs_fail(RS_E_UNSUPPORTED, "tile configurations belong to matrix-core plans");
    int wn, tl, nw, il;
    if (!parse_tile(tile, &wn, &tl, &nw, &il))
        return rs_fail(RS_E_INVALID, "tile \"%s\" is not a built configuration", tile ? tile : "(null)");
    set_mfma_shape(pl, wn, tl, nw, il);
    return RS_OK;
}

extern "C" rs_status rs_plan_tune(rs_plan *pl, const rs_pixels *px, void *cube, int32_t reps, void *stream,
                                  char *chosen, size_t chosen_len)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (reps < 1) return rs_fail(RS_E_INVALID, "reps < 1");
    if (!cube) return rs_fail(RS_E_INVALID, "cube is NULL");
    rs_status s = rs_check_pixels(pl, px);
    if (s != RS_OK) return s;
    if (pl->form == RS_FORM_MFMA_SPLIT16) {
        // every built shape; 8-wave shapes with both schedules
        static const int shapes[][4] = {{64, 128, 4, 0}, {32, 128, 4, 0}, {32, 128, 8, 0}, {32, 128, 8, 1},
                                        {32, 64, 4, 0},  {32, 64, 8, 0},  {32, 64, 8, 1},  {64, 64, 4, 0},
                                        {64, 64, 8, 0},  {64, 64, 8, 1},  {128, 64, 4, 0}};
        device_guard g(pl->device);
        if (g.st != RS_OK) return g.st;
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return rs_fail(RS_E_DEVICE, "hipEventCreate failed");
        }
        const int wn0 = pl->wn, tl0 = pl->tl, nw0 = pl->nw, il0 = pl->interleave;
        int best = -1;
        float best_ms = 0.f;
        for (int i = 0; i < (int)(sizeof shapes / sizeof shapes[0]) && s == RS_OK; ++i) {
            if (!rs_mfma_shape_supported(shapes[i][0], shapes[i][1], shapes[i][2])) continue;
            set_mfma_shape(pl, shapes[i][0], shapes[i][1], shapes[i][2], shapes[i][3]);
            if ((s = rs_beat_synthesize(pl, px, cube, stream)) != RS_OK) break;
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps && s == RS_OK; ++r) s = rs_beat_synthesize(pl, px, cube, stream);
            (void)hipEventRecord(e1, st);
            float ms = 0.f;
            if (s == RS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                s = rs_fail(RS_E_DEVICE, "event timing failed");
            if (s == RS_OK && (best < 0 || ms < best_ms)) {
                best = i;
                best_ms = ms;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (s != RS_OK || best < 0) {
            set_mfma_shape(pl, wn0, tl0, nw0, il0);
            return s != RS_OK ? s : rs_fail(RS_E_UNSUPPORTED, "no tile shape could run");
        }
        set_mfma_shape(pl, shapes[best][0], shapes[best][1], shapes[best][2], shapes[best][3]);
        // leave the cube computed with the chosen shape
        if ((s = rs_beat_synthesize(pl, px, cube, stream)) != RS_OK) return s;
        if (hipStreamSynchronize(st) != hipSuccess) return rs_fail(RS_E_DEVICE, "stream synchronisation failed");
    }
    if (chosen && chosen_len > 0) {
        if (pl->form == RS_FORM_MFMA_SPLIT16) format_tile(pl, chosen, chosen_len);
        else chosen[0] = '\0';
    }
    return RS_OK;
}

extern "C" rs_status rs_plan_tune_cached(rs_plan *pl, const rs_pixels *px, void *cube, int32_t reps, void *stream,
                                         const char *cache_path, char *chosen, size_t chosen_len)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (!cache_path) return rs_fail(RS_E_INVALID, "cache_path is NULL");
    if (reps < 1) return rs_fail(RS_E_INVALID, "reps < 1");
    if (!cube) return rs_fail(RS_E_INVALID, "cube is NULL");
    rs_status s = rs_check_pixels(pl, px);
    if (s != RS_OK) return s;
    if (pl->form != RS_FORM_MFMA_SPLIT16) {
        if (chosen && chosen_len > 0) chosen[0] = '\0';
        return RS_OK;
    }
    long long pb = 1;
    while (pb < px->P) pb <<= 1;
    // the last well-formed entry with this key and a built shape wins
    int hit_wn = 0, hit_tl = 0, hit_nw = 0, hit_il = 0;
    if (std::FILE *f = std::fopen(cache_path, "r")) {
        char line[256];
        while (std::fgets(line, sizeof line, f)) {
            int c = 0, ns = 0, l = 0, wn = 0, tl = 0, nw = 0, il = 0;
            long long b = 0;
            char tile[64];
            if (std::sscanf(line, "%d %d %d %lld %63s", &c, &ns, &l, &b, tile) == 5 && c == pl->C &&
                ns == pl->Ns && l == pl->L && b == pb && parse_tile(tile, &wn, &tl, &nw, &il)) {
                hit_wn = wn;
                hit_tl = tl;
                hit_nw = nw;
                hit_il = il;
            }
        }
        const bool bad = std::ferror(f) != 0;
        std::fclose(f);
        if (bad) return rs_fail(RS_E_INVALID, "cannot read the tile cache %s", cache_path);
    } else if (errno != ENOENT) {
        return rs_fail(RS_E_INVALID, "cannot open the tile cache %s", cache_path);
    }
    if (hit_wn) {
        set_mfma_shape(pl, hit_wn, hit_tl, hit_nw, hit_il);
        if (chosen && chosen_len > 0) format_tile(pl, chosen, chosen_len);
        return RS_OK;
    }
    if ((s = rs_plan_tune(pl, px, cube, reps, stream, chosen, chosen_len)) != RS_OK) return s;
    char tile[32], entry[128];
    format_tile(pl, tile, sizeof tile);
    snprintf(entry, sizeof entry, "%d %d %d %lld %s\n", pl->C, pl->Ns, pl->L, pb, tile);
    std::FILE *f = std::fopen(cache_path, "a");
    const bool ok = f && std::fputs(entry, f) >= 0;
    if (f && std::fclose(f) != 0) return rs_fail(RS_E_INVALID, "cannot append to the tile cache %s", cache_path);
    if (!ok) return rs_fail(RS_E_INVALID, "cannot append to the tile cache %s", cache_path);
    return RS_OK;
}

// ------------------------------------------------------------ synthesis ----

extern "C" rs_status rs_beat_synthesize_ws(rs_plan *pl, const rs_pixels *px, void *cube,
                                           void *ws, size_t ws_bytes, void *stream)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (!cube) return rs_fail(RS_E_INVALID, "cube is NULL");
    rs_status s = rs_check_pixels(pl, px);
    if (s != RS_OK) return s;
    int32_t S, chunk;
    if ((s = rs_plan_chunking(pl, px->P, &S, &chunk)) != RS_OK) return s;
    const size_t need = pl->form == RS_FORM_NUFFT ? rs_nufft_workspace(pl, px->P) : rs_workspace_bytes(pl, S);
    if (need > 0 && (!ws || ws_bytes < need))
        return rs_fail(RS_E_INVALID, "workspace too small: need %zu bytes", need);
    if (need > 0 && (reinterpret_cast<uintptr_t>(ws) & 255))
        return rs_fail(RS_E_INVALID, "workspace must be 256-byte aligned");
    device_guard g(pl->device);
    if (g.st != RS_OK) return g.st;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (pl->form == RS_FORM_NUFFT) return rs_nufft_enqueue(pl, px, cube, ws, st);

    rs_launch L;
    std::memset(&L, 0, sizeof L);
    L.inline_job = rs_make_job(pl, px, cube, ws, S, chunk);
    L.njobs = 1;
    if (pl->form == RS_FORM_MFMA_SPLIT16 && S > 0 && (pl->model & RS_MODEL_BLOCK_STRENGTH)) {
        rs_launch Sc = L;
        Sc.total = S;
        if ((s = rs_launch_scale_checked(Sc, (pl->model & RS_MODEL_BLOCK_STRENGTH) != 0, st)) != RS_OK) return s;
    }
    L.total = L.inline_job.item_count;
    if ((s = rs_launch_main(pl, L, (pl->model & RS_MODEL_BLOCK_STRENGTH) != 0, (int)L.total, st)) != RS_OK)
        return s;
    rs_launch R = L;
    R.total = (int64_t)pl->C * pl->L * pl->Ns;
    R.counter = nullptr;
    return rs_launch_reduce_checked(pl, R, st);
}

extern "C" rs_status rs_beat_synthesize(rs_plan *pl, const rs_pixels *px, void *cube, void *stream)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (!cube) return rs_fail(RS_E_INVALID, "cube is NULL");
    rs_status s = rs_check_pixels(pl, px);
    if (s != RS_OK) return s;
    size_t need = 0;
    if ((s = rs_plan_workspace_bytes(pl, px->P, &need)) != RS_OK) return s;
    device_guard g(pl->device);
    if (g.st != RS_OK) return g.st;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    void *ws = nullptr;
    if (need > 0 && hipMallocAsync(&ws, need, st) != hipSuccess)
        return rs_fail(RS_E_NOMEM, "stream-ordered workspace allocation of %zu bytes failed", need);
    s = rs_beat_synthesize_ws(pl, px, cube, ws, need, stream);
    if (ws) {
        hipError_t e = hipFreeAsync(ws, st);
        if (e != hipSuccess && s == RS_OK) s = rs_fail(RS_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    }
    return s;
}

// ------------------------------------------------ allocation-free call ----
// rs_beat_synthesize_noalloc keeps its workspace (split-K partial sums and
// chunk scales, or the NUFFT grid) in this file-scope device array, one copy
// per device the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy: the name is a host
// stand-in, not a device address.  The address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) char scratch[RS_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices];

// The device address of `scratch` on `dev`, which the caller has made
// current.
rs_status scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxScratchDevices)
        return rs_fail(RS_E_UNSUPPORTED, "device %d beyond the %d the static scratch serves", dev,
                       kMaxScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return rs_fail(RS_E_DEVICE, "hipGetSymbolAddress of the static scratch on device %d: %s", dev,
                           hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RS_OK;
}

}  // namespace

extern "C" rs_status rs_beat_synthesize_noalloc(rs_plan *pl, const rs_pixels *px, void *cube, void *stream)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (!cube) return rs_fail(RS_E_INVALID, "cube is NULL");
    rs_status s = rs_check_pixels(pl, px);
    if (s != RS_OK) return s;
    size_t need = 0;
    if ((s = rs_plan_workspace_bytes(pl, px->P, &need)) != RS_OK) return s;
    if (need > (size_t)RS_STATIC_SCRATCH_BYTES)
        return rs_fail(RS_E_INVALID,
                       "workspace of %zu bytes exceeds the static scratch of %zu bytes (P = %lld): use "
                       "rs_beat_synthesize or rs_beat_synthesize_ws",
                       need, (size_t)RS_STATIC_SCRATCH_BYTES, (long long)px->P);
    void *ws = nullptr;
    {
        device_guard g(pl->device);
        if (g.st != RS_OK) return g.st;
        if ((s = scratch_address(pl->device, &ws)) != RS_OK) return s;
    }
    return rs_beat_synthesize_ws(pl, px, cube, ws, (size_t)RS_STATIC_SCRATCH_BYTES, stream);
}

extern "C" rs_status rs_beat_synthesize_batch(rs_plan *pl, const rs_pixels *frames, int32_t nframes,
                                              void *cubes, void *stream)
{
    if (!pl) return rs_fail(RS_E_INVALID, "plan is NULL");
    if (nframes < 0) return rs_fail(RS_E_INVALID, "nframes < 0");
    if (nframes == 0) return RS_OK;
    if (!frames || !cubes) return rs_fail(RS_E_INVALID, "NULL frames or cubes");
    rs_status s;
    for (int f = 0; f < nframes; ++f)
        if ((s = rs_check_pixels(pl, &frames[f])) != RS_OK) return s;
    device_guard g(pl->device);
    if (g.st != RS_OK) return g.st;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t cube_bytes_f = (size_t)pl->C * pl->L * pl->Ns * (pl->dtype == RS_C128 ? 16 : 8);
    if (pl->form == RS_FORM_NUFFT) {
        // the frames one after another on one workspace sized for the largest
        int64_t pmax = 0;
        for (int f = 0; f < nframes; ++f) pmax = frames[f].P > pmax ? frames[f].P : pmax;
        const size_t need = rs_nufft_workspace(pl, pmax);
        void *ws = nullptr;
        if (need > 0 && hipMallocAsync(&ws, need, st) != hipSuccess)
            return rs_fail(RS_E_NOMEM, "stream-ordered workspace allocation of %zu bytes failed", need);
        s = RS_OK;
        for (int f = 0; f < nframes && s == RS_OK; ++f)
            s = rs_nufft_enqueue(pl, &frames[f], static_cast<char *>(cubes) + f * cube_bytes_f, ws, st);
        if (ws) {
            const hipError_t e = hipFreeAsync(ws, st);
            if (e != hipSuccess && s == RS_OK) s = rs_fail(RS_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
        }
        return s;
    }

    const size_t cube_bytes = (size_t)pl->C * pl->L * pl->Ns * (pl->dtype == RS_C128 ? 16 : 8);
    std::vector<rs_job> jobs(nframes);
    const size_t head = 256 + (((size_t)nframes * sizeof(rs_job) + 255) & ~(size_t)255);
    size_t off = head;
    int64_t items = 0, outs = 0, chunks = 0;
    std::vector<size_t> offs(nframes);
    for (int f = 0; f < nframes; ++f) {
        int32_t S, chunk;
        if ((s = rs_plan_chunking(pl, frames[f].P, &S, &chunk)) != RS_OK) return s;
        offs[f] = off;
        jobs[f] = rs_make_job(pl, &frames[f], static_cast<char *>(cubes) + f * cube_bytes, nullptr,
                              S, chunk);
        jobs[f].item_begin = items;
        jobs[f].out_begin = outs;
        jobs[f].chunk_begin = chunks;
        items += jobs[f].item_count;
        outs += (int64_t)pl->C * pl->L * pl->Ns;
        chunks += S;
        off += rs_workspace_bytes(pl, S);
    }
    char *ws = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&ws), off, st) != hipSuccess)
        return rs_fail(RS_E_NOMEM, "stream-ordered workspace allocation of %zu bytes failed", off);
    for (int f = 0; f < nframes; ++f) {
        rs_job j = rs_make_job(pl, &frames[f], jobs[f].cube, ws + offs[f], jobs[f].S, jobs[f].chunk);
        j.item_begin = jobs[f].item_begin;
        j.out_begin = jobs[f].out_begin;
        j.chunk_begin = jobs[f].chunk_begin;
        jobs[f] = j;
    }
    rs_job *djobs = reinterpret_cast<rs_job *>(ws + 256);
    // The host job table is pageable: the runtime stages it before returning.
    hipError_t e = hipMemcpyAsync(djobs, jobs.data(), jobs.size() * sizeof(rs_job),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)hipFreeAsync(ws, st);
        return rs_fail(RS_E_DEVICE, "job table copy: %s", hipGetErrorString(e));
    }
    rs_launch L;
    std::memset(&L, 0, sizeof L);
    L.jobs = djobs;
    L.njobs = nframes;
    L.total = items;
    L.counter = reinterpret_cast<int *>(ws);
    s = RS_OK;
    if (pl->form == RS_FORM_MFMA_SPLIT16 && chunks > 0 && (pl->model & RS_MODEL_BLOCK_STRENGTH)) {
        rs_launch Sc = L;
        Sc.counter = nullptr;
        Sc.total = chunks;
        s = rs_launch_scale_checked(Sc, (pl->model & RS_MODEL_BLOCK_STRENGTH) != 0, st);
    }
    if (s == RS_OK && items > 0) {
        rs_launch_zero_int(L.counter, 1, st);
        int64_t grid = (int64_t)pl->ncu * pl->occupancy;
        if (grid > items) grid = items;
        s = rs_launch_main(pl, L, (pl->model & RS_MODEL_BLOCK_STRENGTH) != 0, (int)grid, st);
    }
    if (s == RS_OK) {
        rs_launch R = L;
        R.counter = nullptr;
        R.total = outs;
        s = rs_launch_reduce_checked(pl, R, st);
    }
    e = hipFreeAsync(ws, st);
    if (e != hipSuccess && s == RS_OK) s = rs_fail(RS_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    return s;
}
