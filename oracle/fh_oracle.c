/*
 * CPU oracle for the frequency-Hough (FH) transform -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the package smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header or table with the GPU
 * library; the two agree only through the written definition below.
 *
 * What it computes (Astone et al., "Method for all-sky searches of continuous
 * gravitational wave signals using the frequency-Hough transform"):
 *
 *   For one sky direction n, every peak (FFT i, natural bin k) of the peakmap
 *   is Doppler corrected, f' = f / (1 + v_i . n)            (Eq. fdopp)
 *   and mapped into the (f0, fdot) plane as the stripe
 *       f' - fdot tau_i - df/2  <=  f0  <  f' - fdot tau_i + df/2
 *   with tau_i = t_i - t0                                    (Eqs. uno, due)
 *   Each fine bin (K_f per natural bin, Eq. freqres) of each spin-down row
 *   whose label lies in the stripe gains w_i (1 when unweighted)
 *                                                     (Eqs. ncount, ncountadap)
 *
 * The stripe edge is evaluated in an exactly specified fixed point with
 * Q = 2^16 steps per fine bin, so that integer maps can be compared bit for
 * bit.  Every row s has its own spin-down fdot_s = fdot0 + s*dfdot (Eq.
 * sdstep), and its shift is rounded once per row and FFT:
 *   S      = (K_f * T_FFT) * Q
 *   G_is   = llrint(((fdot0 + s*dfdot) * tau_i) * S)       (row s, FFT i)
 *   D      = 1 + ((vx*nx + vy*ny) + vz*nz),  r = 1 / D
 *   X      = floor(((double)(K_f*k) * r) * Q)             (corrected centre)
 *   L_s    = X - b0*Q - K_f*Q/2 - G_is                    (left edge, row s)
 *   bin b is touched  iff  L_s <= b*Q < L_s + K_f*Q
 * All double operations are IEEE binary64, round to nearest even, evaluated in
 * the order written and never contracted into FMAs (build with
 * -ffp-contract=off).  Against the real-valued edge of Eq. due (the same
 * inputs in exact arithmetic) L_s lies within [-1.5, +0.5] quanta: the floor
 * of X loses less than one quantum, the rounding of G_is at most half of one,
 * and the binary64 products add ~1e-3 quanta at most.
 *
 * Per-FFT shift variant (the Doppler removal read as a plain shift of each
 * FFT's bins, computed at one reference frequency f_ref for the whole band):
 *   q      = ((double)K_f * T_FFT) * f_ref                 (reference, fine bins)
 *   X      = K_f*k*Q - llrint((q * (1 - r)) * Q)
 * which equals the exact centre at k = f_ref T_FFT and drifts from it by
 * (K_f k - q)(1 - r) fine bins elsewhere.
 *
 * The oracle fills every touched fine bin directly (K_f additions per peak and
 * row), accumulating in double; it is deliberately slow.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* fixed-point steps per fine bin */
#define QD 65536.0
#define QI ((int64_t)1 << 16)

/* floor(a / Q) for any int64 a, written without relying on >> of negatives */
static int64_t floor_div_q(int64_t a)
{
    int64_t q = a / QI; /* truncates toward zero */
    if (a % QI != 0 && a < 0) q -= 1;
    return q;
}

/* Spin-down shift of row s for an FFT at tau = t_i - t0, in fixed-point fine
 * bins (Eqs. uno and sdstep): the row's spin-down times tau, rounded once. */
static int64_t row_shift(double tau, double S, double fdot0, double dfdot, int32_t s)
{
    double fs = fdot0 + (double)s * dfdot;
    return llrint((fs * tau) * S);
}

/* Shifts of row s for every FFT: out[i] = G_is. */
void fho_row_shifts(int32_t n_fft, const double *t, double t0, double t_fft, int32_t kf,
                    double fdot0, double dfdot, int32_t s, int64_t *out)
{
    double S = ((double)kf * t_fft) * QD;
    for (int32_t i = 0; i < n_fft; ++i) out[i] = row_shift(t[i] - t0, S, fdot0, dfdot, s);
}

/* Doppler factor inverse r = 1/(1 + v.n) per FFT (Eq. fdopp). */
void fho_inv_doppler(int32_t n_fft, const double *v, const double *nhat, double *r)
{
    for (int32_t i = 0; i < n_fft; ++i) {
        const double *vi = v + 3 * (int64_t)i;
        double d = 1.0 + ((vi[0] * nhat[0] + vi[1] * nhat[1]) + vi[2] * nhat[2]);
        r[i] = 1.0 / d;
    }
}

/* Corrected peak centre in fixed-point fine bins. */
int64_t fho_center(int32_t k, int32_t kf, double r)
{
    double x = ((double)((int64_t)kf * (int64_t)k) * r) * QD;
    return (int64_t)floor(x);
}

/* Corrected peak centre of the per-FFT shift variant. */
int64_t fho_shift_center(int32_t k, int32_t kf, double q, double r)
{
    return (int64_t)kf * (int64_t)k * QI - llrint((q * (1.0 - r)) * QD);
}

/* Stripe left edge at fdot = 0: E = X - b0*Q - K_f*Q/2. */
static int64_t zero_spin_edge(int32_t k, int32_t kf, double r, int64_t b0, int32_t shift_mode, double q)
{
    int64_t x = shift_mode ? fho_shift_center(k, kf, q, r) : fho_center(k, kf, r);
    return x - b0 * QI - (int64_t)kf * (QI / 2);
}

/*
 * Left stripe edges L_s (fixed point) of sampled (peak, row) pairs of one sky
 * direction, by the same steps as the map: out[j] = L for peak peak[j] in row
 * row[j] (exact Doppler correction).  Returns 0, or -1 on a bad index.
 */
int fho_left_edges(int32_t n_fft, const int64_t *offsets, const int32_t *bins, const double *t,
                   const double *v, double t_fft, const double *nhat, int32_t kf, int64_t b0,
                   double fdot0, double dfdot, double t0, int64_t n_pairs, const int64_t *peak,
                   const int32_t *row, int64_t *out)
{
    const double S = ((double)kf * t_fft) * QD;
    const int64_t n_peaks = offsets[n_fft];
    for (int64_t j = 0; j < n_pairs; ++j) {
        int64_t p = peak[j];
        if (p < 0 || p >= n_peaks) return -1;
        /* FFT of the peak: last i with offsets[i] <= p */
        int32_t lo = 0, hi = n_fft;
        while (hi - lo > 1) {
            int32_t m = lo + (hi - lo) / 2;
            if (offsets[m] <= p) lo = m; else hi = m;
        }
        double r;
        fho_inv_doppler(1, v + 3 * (int64_t)lo, nhat, &r);
        out[j] = zero_spin_edge(bins[p], kf, r, b0, 0, 0.0) - row_shift(t[lo] - t0, S, fdot0, dfdot, row[j]);
    }
    return 0;
}

/*
 * Hough map of one sky direction, rows [row_lo, row_hi) only (the other rows
 * of `out` are left untouched).  out is [ns][nf] row-major, double, and is
 * zeroed on the selected rows first.  w may be NULL (all weights 1).
 * shift = 0: exact per-peak Doppler correction; 1: per-FFT shift at f_ref.
 * Returns 0, or -1 on invalid arguments.
 */
int fho_hough_map_mode(int32_t n_fft, const int64_t *offsets, const int32_t *bins,
                       const double *t, const double *v, double t_fft, const double *nhat,
                       const double *w, int32_t kf, int64_t b0, int32_t nf, int32_t ns,
                       double fdot0, double dfdot, double t0, int32_t row_lo, int32_t row_hi,
                       int32_t shift_mode, double f_ref, double *out)
{
    if (n_fft < 0 || kf < 1 || nf < 0 || ns < 0 || row_lo < 0 || row_hi > ns || row_lo > row_hi)
        return -1;
    int64_t n_peaks = offsets[n_fft];
    double *tau = (double *)malloc(sizeof(double) * (size_t)(n_fft + 1));
    double *r = (double *)malloc(sizeof(double) * (size_t)(n_fft + 1));
    int64_t *edge = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_peaks + 1));
    if (!tau || !r || !edge) {
        free(tau); free(r); free(edge);
        return -1;
    }
    for (int32_t i = 0; i < n_fft; ++i) tau[i] = t[i] - t0;
    const double S = ((double)kf * t_fft) * QD;
    fho_inv_doppler(n_fft, v, nhat, r);
    const double q = ((double)kf * t_fft) * f_ref;
    for (int32_t i = 0; i < n_fft; ++i)
        for (int64_t p = offsets[i]; p < offsets[i + 1]; ++p)
            edge[p] = zero_spin_edge(bins[p], kf, r[i], b0, shift_mode, q);

    const int64_t width = (int64_t)kf * QI;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t s = row_lo; s < row_hi; ++s) {
        double *row = out + (int64_t)s * nf;
        memset(row, 0, sizeof(double) * (size_t)nf);
        for (int32_t i = 0; i < n_fft; ++i) {
            int64_t shift = row_shift(tau[i], S, fdot0, dfdot, s);
            double wi = w ? w[i] : 1.0;
            for (int64_t p = offsets[i]; p < offsets[i + 1]; ++p) {
                int64_t L = edge[p] - shift;
                /* candidate bins around the edge; membership decided by the test */
                int64_t first = floor_div_q(L);
                for (int64_t b = first; b <= first + kf; ++b) {
                    if (b < 0 || b >= nf) continue;
                    int64_t lab = b * QI;
                    if (L <= lab && lab < L + width) row[b] += wi;
                }
            }
        }
    }
    free(tau); free(r); free(edge);
    return 0;
}

int fho_hough_map(int32_t n_fft, const int64_t *offsets, const int32_t *bins,
                  const double *t, const double *v, double t_fft, const double *nhat,
                  const double *w, int32_t kf, int64_t b0, int32_t nf, int32_t ns,
                  double fdot0, double dfdot, double t0, int32_t row_lo, int32_t row_hi,
                  double *out)
{
    return fho_hough_map_mode(n_fft, offsets, bins, t, v, t_fft, nhat, w, kf, b0, nf, ns, fdot0, dfdot, t0,
                              row_lo, row_hi, 0, 0.0, out);
}

/*
 * Candidates of one map by exhaustive scan (Sec. "Selection of first level
 * candidates"): the map's fine-bin axis is cut into sub-bands of `width` bins
 * (the last one may be shorter).  In each sub-band, over all rows:
 *   first  = cell with the largest value; ties -> smaller bin, then smaller row
 *   second = same order over cells with |b - b_first| > excl; it is reported
 *            only when |b_second - b_first| >= sep (sep < 0 disables it)
 * out_idx: [n_sb][2][3] = (valid, bin, row); out_val: [n_sb][2].
 * Returns the number of sub-bands.
 */
static int better(double v, int32_t b, int32_t s, double bv, int32_t bb, int32_t bs)
{
    if (v != bv) return v > bv;
    if (b != bb) return b < bb;
    return s < bs;
}

int32_t fho_candidates(const double *map, int32_t ns, int32_t nf, int32_t width, int32_t excl,
                       int32_t sep, int32_t *out_idx, double *out_val)
{
    if (width < 1) return -1;
    int32_t n_sb = (nf + width - 1) / width;
    for (int32_t j = 0; j < n_sb; ++j) {
        int32_t lo = j * width, hi = lo + width < nf ? lo + width : nf;
        int found = 0;
        double bv = 0;
        int32_t bb = -1, bs = -1;
        for (int32_t s = 0; s < ns; ++s)
            for (int32_t b = lo; b < hi; ++b) {
                double x = map[(int64_t)s * nf + b];
                if (!found || better(x, b, s, bv, bb, bs)) {
                    found = 1; bv = x; bb = b; bs = s;
                }
            }
        int32_t *o = out_idx + 6 * (int64_t)j;
        o[0] = found; o[1] = bb; o[2] = bs;
        out_val[2 * j] = bv;
        int found2 = 0;
        double cv = 0;
        int32_t cb = -1, cs = -1;
        if (found && sep >= 0) {
            for (int32_t s = 0; s < ns; ++s)
                for (int32_t b = lo; b < hi; ++b) {
                    int32_t d = b > bb ? b - bb : bb - b;
                    if (d <= excl) continue;
                    double x = map[(int64_t)s * nf + b];
                    if (!found2 || better(x, b, s, cv, cb, cs)) {
                        found2 = 1; cv = x; cb = b; cs = s;
                    }
                }
            if (found2) {
                int32_t d = cb > bb ? cb - bb : bb - cb;
                if (d < sep) found2 = 0;
            }
        }
        o[3] = found2; o[4] = found2 ? cb : -1; o[5] = found2 ? cs : -1;
        out_val[2 * j + 1] = found2 ? cv : 0.0;
    }
    return n_sb;
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* thread control for timing runs */
void fho_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t fho_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
