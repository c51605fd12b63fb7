/*
 * CPU FP64 oracle for per-pixel TDM-MIMO beat-cube synthesis.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or constant with the GPU
 * library.
 *
 * What it computes (Sec. II, eq. (1) read per virtual channel, summed over
 * pixels as in eq. (2), with exact per-channel ranges instead of eq. (2)'s
 * far-field angle term):
 *
 *   Y[c][l][n] = sum_p a_p * exp(j 2 pi (psi_{p,c} + b_{p,c} n - beta_p l))
 *
 *   c = m*N + r            virtual channel (Tx m, Rx r), 0-based
 *   n = 0..Ns-1            fast-time sample (eq. (1)'s n_s - 1)
 *   l = 0..L-1             TDM block (eq. (1)'s l - 1)
 *   R_{p,c}   = (|x_p - tx_m| + |x_p - rx_r|) / 2        eq. (1)'s R_{m,n}
 *   psi_{p,c} = 2 fc R / c0      carrier phase held in sigma (0 if disabled)
 *   b_{p,c}   = 2 mu R / (c0 Fs) beat frequency in cycles per sample, eq. (1)
 *   beta_p    = 2 fc Tb v_p / c0 Doppler f_D = 2 v fc / c0 times Tb, eq. (1)
 *
 * The floating-point recipe is fixed (IEEE binary64, round to nearest, no
 * contraction: build with -ffp-contract=off -fno-fast-math):
 *   Kc = (2*fc)/c0 (0 when carrier_phase == 0), Kb = (2*mu)/(c0*Fs),
 *   Kd = ((2*fc)*Tb)/c0
 *   rt = sqrt((dx*dx + dy*dy) + dz*dz) with dx = (double)x - tx.x, rr likewise
 *   R = 0.5*(rt + rr)
 *   psi_f = frac(R*Kc); th_f = frac((R*Kb)*n); ph_f = frac(((double)v*Kd)*l)
 *   phi = psi_f + th_f - ph_f wrapped to [-1/2, 1/2)
 *   term = (double)a * (cos(2 pi phi), sin(2 pi phi)), summed in increasing p.
 *
 * Signal-model variants (bit flags in orc_radar.model; 0 = the model above).
 * Each changes only the per-(pixel, channel) arguments psi and b, evaluated
 * in binary64 in this order:
 *   FAR_FIELD (1)   eq. (2): the range is the one from the array origin,
 *                   Rp = |x|, for the beat frequency (b = Rp Kb) and the
 *                   carrier phase, and the channels differ by eq. (2)'s
 *                   angle-of-arrival term, the first-order path change
 *                   across the array -u.(tx_m + rx_r)/2 (u = x/Rp) in
 *                   wavelengths:  psi = Rp Kc - s Ka,
 *                   s = u.(tx_m + rx_r)/2, Ka = (2 fc)/c0 whatever
 *                   carrier_phase says.  With carrier_phase == 0 this is
 *                   eq. (2) as printed (sigma = a, no common phase
 *                   2 Rp / lambda); with carrier_phase == 1 it is the
 *                   far-field limit of the exact model above
 *   RVP (8)         residual video phase of the dechirped signal,
 *                   -mu tau^2 / 2 with tau = 2 R / c0:  psi -= (R R) Krvp,
 *                   Krvp = (2 mu)/(c0 c0), R the beat range
 *   TDM_SLOT (2)    Tx m transmits in slot m of each block, at l Tb + m Tb/M:
 *                   psi -= beta (m / M)
 *   INTRA_CHIRP (4) Doppler shift within the chirp, with the sign of the
 *                   slow-time term (the echo delay shrinks as an approaching
 *                   scatterer closes in): b -= v Kf, Kf = (2 fc)/(c0 Fs)
 * One variant changes the strength instead of the phase arguments:
 *   BLOCK_STRENGTH (16)  eq. (1)'s sigma depends on the TDM block l: the
 *                   strength of pixel p in block l is amp[l*P + p] (amp holds
 *                   L rows of P values), the same for every channel, so
 *                   a_p becomes a_{p,l} in the sum above.
 *
 * Output layout: interleaved (re, im) doubles, [C][L][Ns] row-major, n fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t M, N, Ns, L;
    double fc, mu, Fs, Tb, c0;
    const double *tx; /* [M][3] */
    const double *rx; /* [N][3] */
    int32_t carrier_phase;
    int32_t model;    /* signal-model variant flags, see above */
} orc_radar;

enum { ORC_FAR_FIELD = 1, ORC_TDM_SLOT = 2, ORC_INTRA_CHIRP = 4, ORC_RVP = 8, ORC_BLOCK_STRENGTH = 16,
       ORC_MODEL_ALL = 31 };

typedef struct {
    int64_t P;
    const float *x, *y, *z, *amp, *vr;
} orc_pixels;

static const double PI = 3.14159265358979323846264338327950288;
static const double TWO_PI = 6.283185307179586476925286766559;

static void orc_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Plan constants of the recipe. */
typedef struct {
    double Kc, Kb, Kd, Kf, Krvp, Ka;
} orc_consts;

static void constants(const orc_radar *r, orc_consts *k)
{
    k->Kc = r->carrier_phase ? (2.0 * r->fc) / r->c0 : 0.0;
    k->Kb = (2.0 * r->mu) / (r->c0 * r->Fs);
    k->Kd = ((2.0 * r->fc) * r->Tb) / r->c0;
    k->Kf = (2.0 * r->fc) / (r->c0 * r->Fs);
    k->Krvp = (2.0 * r->mu) / (r->c0 * r->c0);
    k->Ka = (2.0 * r->fc) / r->c0;
}

/* Euclidean distance from a float32 pixel position to an antenna. */
static double distance(float x, float y, float z, const double *ant)
{
    double dx = (double)x - ant[0];
    double dy = (double)y - ant[1];
    double dz = (double)z - ant[2];
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

/* Phase arguments of pixel p in channel c = m*N + r (Sec. II, eq. (1)):
 * psi the carrier phase of sigma (cycles, not reduced), b the beat frequency
 * (cycles per fast-time sample), beta the Doppler phase per block (cycles).
 * Without variant flags R = (|x - tx_m| + |x - rx_r|) / 2, psi = R Kc,
 * b = R Kb, beta = v Kd. */
static void chan_args(const orc_radar *r, const orc_consts *k, const orc_pixels *px, int64_t p, int c,
                      double *psi, double *b, double *beta)
{
    int m = c / r->N, rr = c % r->N;
    const double *tx = r->tx + 3 * m, *rx = r->rx + 3 * rr;
    double v = (double)px->vr[p];
    double Rb, ps;
    if (r->model & ORC_FAR_FIELD) {
        double x = (double)px->x[p], y = (double)px->y[p], z = (double)px->z[p];
        double Rp = sqrt((x * x + y * y) + z * z);
        double ux = x / Rp, uy = y / Rp, uz = z / Rp;
        double s = 0.5 * ((ux * (tx[0] + rx[0]) + uy * (tx[1] + rx[1])) + uz * (tx[2] + rx[2]));
        ps = Rp * k->Kc - s * k->Ka;
        Rb = Rp;
    } else {
        double rt = distance(px->x[p], px->y[p], px->z[p], tx);
        double rv = distance(px->x[p], px->y[p], px->z[p], rx);
        Rb = 0.5 * (rt + rv);
        ps = Rb * k->Kc;
    }
    *beta = v * k->Kd;
    *psi = ps;
    *b = Rb * k->Kb;
    if (r->model & ORC_RVP) *psi = *psi - (Rb * Rb) * k->Krvp;
    if (r->model & ORC_TDM_SLOT) *psi = *psi - *beta * ((double)m / (double)r->M);
    if (r->model & ORC_INTRA_CHIRP) *b = *b - v * k->Kf;
}

static double frac(double v) { return v - floor(v); }

/* Strength of pixel p in TDM block l: a_p, or a_{p,l} with BLOCK_STRENGTH. */
static double strength(const orc_radar *r, const orc_pixels *px, int64_t p, int l)
{
    if (r->model & ORC_BLOCK_STRENGTH) return (double)px->amp[(int64_t)l * px->P + p];
    return (double)px->amp[p];
}

/* One term a * exp(j 2 pi (psi + b n - beta l)) by the fixed recipe. */
static void term(double psi, double b, double beta, double a, int n, int l, double *re, double *im)
{
    double psi_f = frac(psi);
    double th_f = frac(b * (double)n);
    double ph_f = frac(beta * (double)l);
    double phi = (psi_f + th_f) - ph_f;
    phi = phi - floor(phi + 0.5);
    double ang = TWO_PI * phi;
    *re = a * cos(ang);
    *im = a * sin(ang);
}

static int valid(const orc_radar *r, const orc_pixels *px)
{
    if (!r || !px) return 0;
    if (r->M < 1 || r->N < 1 || r->Ns < 1 || r->L < 1) return 0;
    if (!(r->Fs > 0) || !(r->Tb > 0) || !(r->c0 > 0)) return 0;
    if (px->P < 0) return 0;
    if (px->P > 0 && (!px->x || !px->y || !px->z || !px->amp || !px->vr)) return 0;
    if (!r->tx || !r->rx) return 0;
    if (r->model < 0 || (r->model & ~ORC_MODEL_ALL)) return 0;
    return 1;
}

/* Full cube, direct sum over pixels in increasing p for every (c, l, n). */
int orc_cube(const orc_radar *r, const orc_pixels *px, double *out, int nthreads)
{
    if (!valid(r, px) || !out) return 1;
    orc_consts k;
    constants(r, &k);
    const int C = r->M * r->N, L = r->L, Ns = r->Ns;
    const int64_t P = px->P;
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t row = 0; row < (int64_t)C * L; ++row) {
        int c = (int)(row / L), l = (int)(row % L);
        double *o = out + 2 * row * Ns;
        for (int n = 0; n < Ns; ++n) { o[2 * n] = 0.0; o[2 * n + 1] = 0.0; }
        for (int64_t p = 0; p < P; ++p) {
            double psi, b, beta;
            chan_args(r, &k, px, p, c, &psi, &b, &beta);
            double a = strength(r, px, p, l);
            for (int n = 0; n < Ns; ++n) {
                double re, im;
                term(psi, b, beta, a, n, l, &re, &im);
                o[2 * n] += re;
                o[2 * n + 1] += im;
            }
        }
    }
    return 0;
}

/* Selected entries Y[c_k][l_k][n_k], k = 0..K-1; same recipe and order. */
int orc_entries(const orc_radar *r, const orc_pixels *px, int64_t K,
                const int32_t *cs, const int32_t *ls, const int32_t *ns,
                double *out, int nthreads)
{
    if (!valid(r, px) || K < 0 || (K > 0 && (!cs || !ls || !ns || !out))) return 1;
    const int C = r->M * r->N;
    for (int64_t k = 0; k < K; ++k)
        if (cs[k] < 0 || cs[k] >= C || ls[k] < 0 || ls[k] >= r->L || ns[k] < 0 || ns[k] >= r->Ns)
            return 1;
    orc_consts kk;
    constants(r, &kk);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < K; ++k) {
        double sre = 0.0, sim = 0.0;
        for (int64_t p = 0; p < px->P; ++p) {
            double psi, b, beta;
            chan_args(r, &kk, px, p, cs[k], &psi, &b, &beta);
            double re, im;
            term(psi, b, beta, strength(r, px, p, ls[k]), ns[k], ls[k], &re, &im);
            sre += re;
            sim += im;
        }
        out[2 * k] = sre;
        out[2 * k + 1] = sim;
    }
    return 0;
}

/*
 * Geometric-series kernel G_N(x) = sum_{k=0}^{N-1} exp(j 2 pi x k)
 *                               = exp(j pi (N-1) x) sin(pi N x) / sin(pi x),
 * equal to N where x is an integer.  Used by the marginals below, which sum
 * the cube over one axis in closed form instead of term by term.
 */
static void geom(int N, double x, double *re, double *im)
{
    double xr = x - floor(x + 0.5); /* the kernel has period 1 in x */
    double s = sin(PI * xr);
    double mag;
    if (fabs(s) < 1e-300) {
        mag = (double)N;
    } else {
        double t = fmod((double)N * xr, 2.0);
        mag = sin(PI * t) / s;
    }
    double ang = PI * fmod((double)(N - 1) * xr, 2.0);
    *re = mag * cos(ang);
    *im = mag * sin(ang);
}

/* Fast-time marginal S[c][l] = sum_n Y[c][l][n] in closed form:
 * sum_p a_p exp(j 2 pi (psi - beta l)) G_Ns(b). */
int orc_marginal_n(const orc_radar *r, const orc_pixels *px, double *out, int nthreads)
{
    if (!valid(r, px) || !out) return 1;
    orc_consts k;
    constants(r, &k);
    const int C = r->M * r->N, L = r->L;
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t row = 0; row < (int64_t)C * L; ++row) {
        int c = (int)(row / L), l = (int)(row % L);
        double sre = 0.0, sim = 0.0;
        for (int64_t p = 0; p < px->P; ++p) {
            double psi, b, beta;
            chan_args(r, &k, px, p, c, &psi, &b, &beta);
            double ph = frac(psi) - frac(beta * (double)l);
            double gr, gi;
            geom(r->Ns, b, &gr, &gi);
            double cr = cos(TWO_PI * ph), ci = sin(TWO_PI * ph);
            double a = strength(r, px, p, l);
            sre += a * (cr * gr - ci * gi);
            sim += a * (cr * gi + ci * gr);
        }
        out[2 * row] = sre;
        out[2 * row + 1] = sim;
    }
    return 0;
}

/* Slow-time marginal S[c][n] = sum_l Y[c][l][n] in closed form:
 * sum_p a_p exp(j 2 pi (psi + b n)) G_L(-beta).  With BLOCK_STRENGTH the
 * slow-time factor sum_l a_{p,l} exp(-j 2 pi beta l) has no closed form and
 * is summed over l per pixel, still apart from the fast-time phasor. */
int orc_marginal_l(const orc_radar *r, const orc_pixels *px, double *out, int nthreads)
{
    if (!valid(r, px) || !out) return 1;
    orc_consts k;
    constants(r, &k);
    const int C = r->M * r->N, Ns = r->Ns;
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t row = 0; row < (int64_t)C * Ns; ++row) {
        int c = (int)(row / Ns), n = (int)(row % Ns);
        double sre = 0.0, sim = 0.0;
        for (int64_t p = 0; p < px->P; ++p) {
            double psi, b, beta;
            chan_args(r, &k, px, p, c, &psi, &b, &beta);
            double ph = frac(psi) + frac(b * (double)n);
            double gr = 0.0, gi = 0.0, a = 1.0;
            if (r->model & ORC_BLOCK_STRENGTH) {
                for (int l = 0; l < r->L; ++l) {
                    double al = strength(r, px, p, l), th = TWO_PI * frac(beta * (double)l);
                    gr += al * cos(th);
                    gi -= al * sin(th);
                }
            } else {
                geom(r->L, -beta, &gr, &gi);
                a = (double)px->amp[p];
            }
            double cr = cos(TWO_PI * ph), ci = sin(TWO_PI * ph);
            sre += a * (cr * gr - ci * gi);
            sim += a * (cr * gi + ci * gr);
        }
        out[2 * row] = sre;
        out[2 * row + 1] = sim;
    }
    return 0;
}

/* Phase arguments of every pixel in channel c by the recipe above: psi (not
 * reduced), b and beta, each an array of P doubles.  Serves the NUFFT
 * oracle, which needs the arguments rather than the sum. */
int orc_chan_args(const orc_radar *r, const orc_pixels *px, int c, double *psi, double *b, double *beta)
{
    if (!valid(r, px) || c < 0 || c >= r->M * r->N || (px->P > 0 && (!psi || !b || !beta))) return 1;
    orc_consts k;
    constants(r, &k);
    for (int64_t p = 0; p < px->P; ++p) chan_args(r, &k, px, p, c, &psi[p], &b[p], &beta[p]);
    return 0;
}

/* Number of OpenMP threads a parallel region would use. */
int orc_max_threads(int nthreads)
{
#ifdef _OPENMP
    orc_set_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}
