/*
 * fh.h -- C ABI of the MI355X (gfx950) frequency-Hough library.
 *
 * The library computes the frequency-Hough (FH) transform of Astone et al.,
 * "Method for all-sky searches of continuous gravitational wave signals using
 * the frequency-Hough transform": for each sky direction it Doppler-corrects
 * a time-frequency peakmap (Eq. fdopp), maps every peak into the source
 * (f0, fdot) plane as a stripe one natural bin wide (Eqs. uno, due) at K_f
 * fine bins per natural bin (Eq. freqres), accumulates the number count or its
 * weighted form (Eqs. ncount, ncountadap) on a spin-down grid (Eq. sdstep),
 * and selects candidates per frequency sub-band (Sec. "Selection of first
 * level candidates").
 *
 * Exact integer definition (shared by every entry point), stripe edges in
 * units of Q = 2^-16 fine bins:
 *   tau_i = t_i - t0;  S = (K_f * T_FFT) * 2^16
 *   G_is  = llrint(((fdot0 + s*dfdot) * tau_i) * S)           (row s, FFT i)
 *   D     = 1 + ((vx*nx + vy*ny) + vz*nz);  r = 1 / D        (IEEE binary64,
 *   X     = floor(((double)(K_f * k) * r) * 2^16)             no FMA contraction)
 *   L_s   = X - b0*2^16 - K_f*2^15 - G_is
 *   fine bin b (0 <= b < nf) of row s (0 <= s < ns) gains w_i for peak (i, k)
 *   iff L_s <= b*2^16 < L_s + K_f*2^16.
 *   Bin b is labelled f0 = (b0 + b) / (K_f T_FFT); row s is fdot0 + s*dfdot.
 *   L_s is within [-1.5, +0.5] Q of the real-valued stripe edge of Eq. due
 *   for the same inputs, so a cell's membership differs from the exact
 *   geometry only where a bin label lies within 1.5 Q of a stripe edge.
 *   Rejected with FH_E_UNSUPPORTED: a grid whose largest step
 *   |dfdot tau_i| K_f T_FFT reaches 128 fine bins per row (the tiles keep
 *   tile-relative stripe edges in 32 bits), a peakmap with an FFT of 65536
 *   peaks or more, n_fft * ceil(ns / 16) reaching 2^28 (the per-row shift
 *   records are addressed with 31-bit byte offsets), n_fft above
 *   524 160 (a tile run of every 16th FFT holds at most 32767), and
 *   n_peaks + 16 n_fft reaching 2^30 (a direction's stripe edges are
 *   addressed with 32-bit byte offsets).
 *
 * Conventions
 *   - Every pointer named d_* is device memory on the context's device and is
 *     owned by the caller; it must stay valid until the work enqueued on the
 *     given stream has completed.  Pointers without the prefix are host memory,
 *     read before the call returns.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Compute calls are
 *     asynchronous with respect to the host: they validate their host-visible
 *     arguments, enqueue kernels on `stream` and return.
 *   - Library workspaces are owned by the context and grow on demand; a call
 *     that has to grow one first synchronises `stream`.
 *   - A context may be used by one host thread at a time.
 *   - Errors: functions return a negative fh_status and set a thread-local
 *     message read with fh_last_error().  Nothing is enqueued after a failed
 *     validation.  Conditions that can only be seen on the device (invalid
 *     weights) set a device-side flag that fh_ctx_check() reports.
 */
#ifndef FH_H
#define FH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FH_OK = 0,
    FH_E_INVALID = -1,     /* an argument fails validation                     */
    FH_E_NOMEM = -2,       /* device or host allocation failed                 */
    FH_E_DEVICE = -3,      /* a HIP runtime call failed                        */
    FH_E_UNSUPPORTED = -4, /* valid but outside what this build supports       */
    FH_E_BUSY = -5,        /* serving: request not admissible right now        */
    FH_E_CANCELLED = -6    /* serving: request was cancelled                   */
} fh_status;

typedef struct fh_ctx fh_ctx;
typedef struct fh_peakmap fh_peakmap;

/* Peakmap in CSR form (Sec. "Peakmap", Eq. pm): FFT i owns the natural-bin
 * indices bins[offsets[i] .. offsets[i+1]).  All arrays are host memory. */
typedef struct {
    int32_t n_fft;          /* N >= 1                                               */
    int64_t n_peaks;        /* P = offsets[N] >= 0                                  */
    const int64_t *offsets; /* [N+1], offsets[0] = 0, non-decreasing                */
    const int32_t *bins;    /* [P], k >= 0, strictly ascending within each FFT      */
    const double *t;        /* [N] FFT time tags t_i in s (finite)                  */
    const double *v;        /* [N][3] detector velocity / c, equatorial, |v| < 1e-2 */
    double t_fft;           /* T_FFT in s, > 0                                      */
} fh_peakmap_desc;

/* Search grid of one Hough map (Sec. "Coarse grid in the parameter space"). */
typedef struct {
    int32_t kf;    /* K_f fine bins per natural bin, 1 .. 64                   */
    int64_t b0;    /* absolute index of fine bin 0, 0 <= b0 < 2^28             */
    int32_t nf;    /* fine bins, 1 .. 2^22                                     */
    int32_t ns;    /* spin-down rows, 1 .. 2^15                                */
    double fdot0;  /* spin-down of row 0 [Hz/s]                                */
    double dfdot;  /* row step [Hz/s]                                          */
    double t0;     /* reference time [s]                                       */
} fh_grid;

/* Candidate selection (Sec. "Selection of first level candidates"): the map
 * is cut into sub-bands of `width` fine bins (the last may be shorter); per
 * sub-band the best cell over all rows is rank 0; rank 1 is the best cell
 * with |b - b_rank0| > excl, kept only if |b - b_rank0| >= sep (sep < 0
 * disables it).  Ties: larger value, then smaller bin, then smaller row. */
typedef struct {
    int32_t width;  /* >= 1                                               */
    int32_t excl;   /* >= 0, e.g. 4                                       */
    int32_t sep;    /* e.g. 8; < 0 disables rank 1                        */
    double theta;   /* peak threshold for the critical ratio, e.g. 2.5    */
} fh_select;

/* One candidate.  f0 = (b0 + bin)/(K_f T_FFT); fdot = fdot0 + row*dfdot.
 * value: number count, or weighted count; cr: critical ratio (Eq. cr) --
 * (n - N p0)/sqrt(N p0 (1-p0)), weighted (n - p0 sum w)/sqrt(p0 (1-p0) sum w^2),
 * with p0 = e^-t - e^-2t + e^-3t / 3 (Eq. p0).  valid = 0 marks an absent
 * rank-1 candidate (all other fields are then 0 / -1). */
typedef struct {
    int32_t sky, subband, rank, bin, row;
    float value, cr;
    int32_t valid;
} fh_candidate;

/* Scheduling of a multi-sky search. */
typedef enum {
    FH_SCHED_PLAIN = 0,      /* one launch sequence per sky direction            */
    FH_SCHED_PERSISTENT = 1  /* all skies' tiles in one persistent launch        */
} fh_schedule;

typedef struct {
    int32_t schedule;    /* fh_schedule                                            */
    int32_t tile_bins;   /* fine bins per LDS tile; 0 = library choice (autotuned).
                            A requested width is rounded up to a multiple of 64
                            and capped at what one 16-row tile holds in LDS */
    int32_t sky_chunk;   /* sky directions per workspace chunk; 0 = library choice */
    int32_t use_graph;   /* 1: capture the whole search in a hipGraph on first use
                            and replay it while every pointer and shape argument
                            (and the stream) is unchanged                       */
} fh_options;

/* Tile / workspace plan reported by fh_plan_query. */
typedef struct {
    int32_t tile_rows;       /* spin-down rows per LDS tile (16)           */
    int32_t tile_bins;       /* fine bins per LDS tile                     */
    int32_t n_row_blocks;    /* 16-row blocks run as tiles: ceil(ns / 16),
                                less one when the grid's last block holds
                                1-3 rows and the tile width leaves room for
                                them, in which case the tiles of the block
                                before it also accumulate those rows      */
    int32_t n_bin_blocks;
    int64_t workspace_bytes; /* library workspace for one sky direction   */
    int64_t cell_updates;    /* peaks x rows, per sky direction           */
} fh_plan_info;

/* ---- context ----------------------------------------------------------- */

/* Library version string (static storage). */
const char *fh_version(void);

/* Message of the last failed call on this thread (static storage, never NULL). */
const char *fh_last_error(void);

/* Create a context on HIP device `device`.  *out receives the handle. */
fh_status fh_ctx_create(int32_t device, fh_ctx **out);

/* Destroy a context; waits for its device work and frees its workspaces.
 * Peakmaps uploaded through it must be released first.  NULL is a no-op. */
void fh_ctx_destroy(fh_ctx *ctx);

/* Synchronise `stream` and report (then clear) the device-side error flag:
 * FH_E_INVALID if a weight vector used since the last check held a value that
 * is not finite or outside (0, 65536); FH_E_DEVICE if a per-row spin-down
 * residual left its 2-bit code (excluded by the shifts' error bound; a
 * broken invariant, not an input error). */
fh_status fh_ctx_check(fh_ctx *ctx, void *stream);

/* Tuning knobs of a context, for experiments and tests.  Results never
 * depend on them.  Names: "window_method" (0 = two binary searches per peak
 * window, 1 = one sweep per FFT, 2 = stripe edges and windows in one kernel
 * with the edges of a few FFTs staged in LDS, default 2; it falls back to 1
 * when one FFT holds too many peaks for the LDS).  FH_E_INVALID for an
 * unknown name or value. */
fh_status fh_ctx_set_option(fh_ctx *ctx, const char *name, int64_t value);

/* Doppler correction used by every later search of the context (Sec. "The
 * frequency-Hough transform": removing the Doppler effect amounts to
 * shifting each FFT's bins).  mode 0 (default): exact per peak, the centre
 * X = floor(((double)(K_f k) r) 2^16) with r = 1 / (1 + v_i . n).  mode 1: one
 * shift per FFT computed at the reference frequency f_ref [Hz] (f_ref <= 0:
 * each map's band centre (b0 + nf / 2) / (K_f T_FFT)):
 *   q = ((double)K_f * T_FFT) * f_ref,  X = K_f k 2^16 - llrint((q (1 - r)) 2^16)
 * which is exact at f_ref and drifts by (K_f k - q)(1 - r) fine bins away
 * from it (up to half the band times |v| natural bins).  FH_E_INVALID for
 * another mode or a non-finite f_ref. */
fh_status fh_ctx_set_doppler(fh_ctx *ctx, int32_t mode, double f_ref);

/* ---- peakmaps ---------------------------------------------------------- */

/* Validate a host peakmap and copy it to device memory owned by the returned
 * handle (the copy completes before the call returns; the caller keeps its
 * arrays).  Rejects unsorted or negative bins, bad offsets, non-finite times
 * or velocities, |v| >= 1e-2, T_FFT <= 0. */
fh_status fh_peakmap_upload(fh_ctx *ctx, const fh_peakmap_desc *desc, void *stream,
                            fh_peakmap **out);

/* Build a device-resident peakmap from equalised spectra (Sec. "Peakmap",
 * Eq. pm): per FFT i and row bin j, R = d_sp[i][j] / d_sar[i][j] (float32,
 * correctly rounded; d_sar = NULL means d_sp already holds R); bin j
 * (1 <= j <= n_bins - 2; the first and last bins of a row are guards) is a
 * peak of natural bin k0 + j when R > theta and R is strictly larger than
 * both neighbours.  d_sp / d_sar: device [n_fft][ld] float32, ld >= n_bins.
 * t, v, t_fft: host arrays as in fh_peakmap_desc.  Synchronises `stream`
 * (the peak count sizes the result). */
fh_status fh_peakmap_from_spectra(fh_ctx *ctx, int32_t n_fft, int32_t n_bins, int64_t ld,
                                  const float *d_sp, const float *d_sar, int32_t k0, float theta,
                                  const double *t, const double *v, double t_fft, void *stream,
                                  fh_peakmap **out);

/* Copy a peakmap's CSR back to host arrays: offsets [n_fft+1] and bins
 * [n_peaks] (either may be NULL).  Synchronous. */
fh_status fh_peakmap_download(fh_ctx *ctx, const fh_peakmap *pm, int64_t *offsets, int32_t *bins);

/* Number of FFTs and peaks of a peakmap. */
fh_status fh_peakmap_shape(const fh_peakmap *pm, int32_t *n_fft, int64_t *n_peaks);

/* Free a peakmap's device memory (after work using it has completed). */
void fh_peakmap_release(fh_ctx *ctx, fh_peakmap *pm);

/* Device bytes held by a peakmap. */
int64_t fh_peakmap_bytes(const fh_peakmap *pm);

/* ---- planning ---------------------------------------------------------- */

/* Tile shape and workspace size the library will use for (pm, grid);
 * tile_bins = 0 lets the library choose. */
fh_status fh_plan_query(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *grid,
                        int32_t tile_bins, fh_plan_info *out);

/* ---- Hough maps (one sky direction) ------------------------------------- */

/* Unweighted number-count map (Eq. ncount): d_map is [ns][nf] int32 row-major
 * and is fully overwritten.  Bit-exact with the definition above.  nhat is a
 * host unit vector (| |n| - 1 | < 1e-9). */
fh_status fh_hough_map_i32(fh_ctx *ctx, const fh_peakmap *pm, const double nhat[3],
                           const fh_grid *grid, int32_t *d_map, void *stream);

/* Weighted map (Eq. ncountadap): d_w is the device float32 weight of each FFT
 * [N]; d_map is [ns][nf] float32.  Weights are rounded to fixed point with
 * F = floor(log2((2^32-1) / (m * sum w))) fractional bits (m = 1, or 2 when
 * a peakmap has adjacent bins), accumulated exactly in 32-bit integers and
 * converted to float32 once, so each cell is within
 * (#contributions) * 2^-(F+1) + 2^-24 |value| of the exact sum. */
fh_status fh_hough_map_f32(fh_ctx *ctx, const fh_peakmap *pm, const double nhat[3],
                           const float *d_w, const fh_grid *grid, float *d_map,
                           void *stream);

/* Allocation-free variant of fh_hough_map_i32, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and the same bit-exact map;
 * it calls no allocating routine.  Its workspace (shift table, stripe edges,
 * peak windows) lives in a static 64 MiB device array that each GPU holds
 * until the process ends; the array's address on each device is taken when
 * the first context on that device is created.  A map needing more than
 * 64 MiB is rejected with FH_E_UNSUPPORTED before anything is enqueued: the
 * need is about 4 (n_peaks + 16 n_fft) + 16 x (row groups of 64 rows) x (tiles
 * along the band) x (n_fft rounded up to 192) + 8 n_fft ceil(ns / 16) +
 * 80 n_fft bytes.
 * Every call on a GPU shares that GPU's array and leaves its contents there:
 * calls that overlap on one GPU (different streams or contexts without
 * ordering) race, so serialise them, e.g. on one stream. */
fh_status fh_hough_map_i32_static(fh_ctx *ctx, const fh_peakmap *pm, const double nhat[3],
                                  const fh_grid *grid, int32_t *d_map, void *stream);

/* ---- candidates (many sky directions) ------------------------------------ */

/* Sub-band candidates of n_sky maps without materialising them.
 * sky:    host [n_sky][3] unit vectors.
 * d_w:    NULL (unweighted), or device float32 weights: w_stride = 0 means one
 *         [N] vector shared by all directions, w_stride = N means [n_sky][N].
 * d_out:  device [n_sky][n_sb][2] candidates, n_sb = ceil(nf / sel->width).
 * opts:   NULL for defaults (persistent schedule, autotuned tile width, library
 *         chunking, no graph capture).
 * Unweighted results are bit-exact with the definition above and identical for
 * both schedules; weighted results are identical for both schedules. */
fh_status fh_hough_candidates(fh_ctx *ctx, const fh_peakmap *pm, int32_t n_sky,
                              const double *sky, const float *d_w, int32_t w_stride,
                              const fh_grid *grid, const fh_select *sel,
                              const fh_options *opts, fh_candidate *d_out, void *stream);

/* Column maxima of n_sky maps without materialising them: for every
 * direction and fine bin b, the largest map value over the spin-down rows
 * and the smallest row holding it -- what candidate selection ranks over
 * "all the possible spin-down values" (Sec. "Selection of first level
 * candidates"), and the map's projection on the frequency axis by maximum.
 * Arguments as fh_hough_candidates (use_graph is ignored).
 * d_value: device float32 [n_sky][nf]: the count (exact) or the weighted
 *          sum (the fixed-point sum times 2^-F, rounded to float32 as the
 *          candidates' value);
 * d_row:   device int32 [n_sky][nf]: smallest row s with H[s][b] = max.
 * Unweighted results are bit-exact with the definition above. */
fh_status fh_hough_colmax(fh_ctx *ctx, const fh_peakmap *pm, int32_t n_sky, const double *sky,
                          const float *d_w, int32_t w_stride, const fh_grid *grid,
                          const fh_options *opts, float *d_value, int32_t *d_row, void *stream);

/* ---- refined grid ---------------------------------------------------- */

/* The peaks of `pm` whose natural bin k lies in [k_lo, k_hi), as a new device
 * peakmap with the same FFTs, times and velocities (a narrow band for a small
 * search).  Runs on `stream` and waits for it (the exact peak count is read
 * back); the new handle is owned by the caller and released with
 * fh_peakmap_release.  Errors: FH_E_INVALID for k_lo < 0 or k_hi <= k_lo,
 * FH_E_NOMEM, FH_E_DEVICE (nothing is allocated on failure). */
fh_status fh_peakmap_slice(fh_ctx *ctx, const fh_peakmap *pm, int32_t k_lo, int32_t k_hi,
                           void *stream, fh_peakmap **out);

/* A coarse candidate to refine: frequency f0 [Hz] and spin-down fdot [Hz/s]
 * at the reference time t0 of fh_refine_opts, ecliptic longitude and latitude
 * [rad] of its sky point, and the coarse sky spacings there (longitude step of
 * its ring, latitude distance to the adjacent ring). */
typedef struct fh_coarse_cand {
    double f0, fdot, lambda, beta, dlambda, dbeta;
} fh_coarse_cand;

/* Refinement (Sec. "Refined Grid in the parameter space"): frequency over
 * K_f fine bins per natural bin, +-1 natural bin around f0 (2 K_f + 1 bins);
 * spin-down step dfdot / k_fdot with 2 k_fdot steps below fdot and
 * 2 k_fdot - 1 above (4 k_fdot rows, row 2 k_fdot = fdot); k_sky x k_sky sky
 * points (k_sky odd) at steps dlambda / k_sky, dbeta / k_sky around the
 * candidate.  theta is the peakmap threshold used for the critical ratio. */
typedef struct fh_refine_opts {
    int32_t kf, k_fdot, k_sky, pad;
    double dfdot, t0, theta;
} fh_refine_opts;

/* One refined candidate per coarse one: the best cell over the refined sky
 * points, frequency bins and spin-down rows (larger value, then smaller sky
 * index, bin and row); sky = j * k_sky + i for latitude step j and longitude
 * step i (both from -(k_sky-1)/2); bin and row index the refined grid. */
typedef struct fh_refined {
    int32_t cand, sky, bin, row;
    float value, cr;
    int32_t valid, pad;
    double f0, fdot, lambda, beta;
} fh_refined;

/* Refine n_cand coarse candidates (host array) against `pm`; d_w: NULL or
 * FP32 weights [N] (shared).  Each candidate is searched on the peaks within
 * its band plus the Doppler and spin-down margin, so the result equals the
 * search of the full peakmap.  Writes d_out[n_cand] (device).  FH_E_INVALID
 * for bad options (kf, k_fdot >= 1, k_sky odd >= 1, dfdot > 0, finite
 * candidates). */
fh_status fh_refine(fh_ctx *ctx, const fh_peakmap *pm, int32_t n_cand, const fh_coarse_cand *cands,
                    const fh_refine_opts *opts, const float *d_w, fh_refined *d_out, void *stream);

/* ---- peakmap cleaning ------------------------------------------------------
 * Sec. "Removal of time and frequency domain disturbances".  Every function
 * here runs on `stream`; those returning a new peakmap wait for it (the
 * surviving peak count sizes the result), and the new handle is owned by the
 * caller (fh_peakmap_release).  FH_E_INVALID for bad arguments. */

/* Cells of the gross histogram (subsection on spectral wandering lines).
 * FFT i lies in time cell floor((t_i - t_origin) / dt_h) and a peak of
 * natural bin k in frequency cell floor(k / (df_h T_FFT)) - c0 (FP64: one
 * product df_h T_FFT, one division and a floor each); the histogram holds
 * the cells [0, n_t) x [0, n_f).  dt_h, df_h > 0, n_t, n_f >= 1. */
typedef struct fh_gross {
    double t_origin, dt_h, df_h;
    int64_t c0;
    int32_t n_t, n_f;
} fh_gross;

/* d_hist: device int32 [n_t][n_f] (row-major), overwritten with the number
 * of peaks in each cell; peaks outside the cells are not counted. */
fh_status fh_gross_histogram(fh_ctx *ctx, const fh_peakmap *pm, const fh_gross *geo, int32_t *d_hist,
                             void *stream);

/* Wandering-line veto: a new peakmap without the peaks whose cell holds more
 * than `threshold` peaks (the paper takes E_H + 2-3 sigma_H); peaks outside
 * the cells are kept.  d_hist (device int32 [n_t][n_f], caller-owned) holds
 * the gross histogram on return. */
fh_status fh_clean_gross(fh_ctx *ctx, const fh_peakmap *pm, const fh_gross *geo, double threshold,
                         int32_t *d_hist, void *stream, fh_peakmap **out);

/* Persistency (subsection on lines of constant frequency): d_counts (device
 * int32 [k_hi - k_lo]) = number of peaks at each natural bin k in
 * [k_lo, k_hi), i.e. of FFTs holding a peak there. */
fh_status fh_bin_counts(fh_ctx *ctx, const fh_peakmap *pm, int32_t k_lo, int32_t k_hi, int32_t *d_counts,
                        void *stream);

/* Robust statistic (appendix "Robust statistic"): out[0] = m1 = median of
 * d_x[0 .. n), out[1] = m2 = median(|x - m1|) / 0.6745, a median of an even
 * count being the mean of the two middle values.  Exact (integer ranks).
 * Requires n >= 1 and 0 <= x <= x_max (checked on the device: FH_E_INVALID).
 * out: host array; waits for `stream`. */
fh_status fh_robust_stats(fh_ctx *ctx, const int32_t *d_x, int32_t n, int32_t x_max, double out[2],
                          void *stream);

/* Lines of constant frequency without Doppler correction (the third option
 * of that subsection): per fine bin of `g`, the largest count over the grid's
 * spin-down rows of the unweighted Hough map of pm computed with v . n = 0
 * (rows around zero spin-down admit a slowly drifting line).  d_out: device
 * int32 [g->nf]. */
fh_status fh_line_counts(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, int32_t *d_out, void *stream);

/* Veto of natural bins: a new peakmap without the peaks of natural bin k in
 * [k_lo, k_hi) for which idx = step (k - k_lo) + offset lies in [0, n_x) and
 * d_x[idx] > threshold (d_x: device int32 [n_x], e.g. fh_bin_counts with
 * step 1, or fh_line_counts with step K_f and offset K_f k_lo - b0). */
fh_status fh_veto_bins(fh_ctx *ctx, const fh_peakmap *pm, int32_t k_lo, int32_t k_hi, const int32_t *d_x,
                       int64_t n_x, int32_t step, int64_t offset, double threshold, void *stream,
                       fh_peakmap **out);

/* ---- serving ------------------------------------------------------------ */

/* A continuous-batching request server over one context.  Requests
 * (band = a resident peakmap + grid, sky patch, spin-down range) queue on the
 * host; fh_server_poll admits queued requests in arrival order whenever a lane
 * (a HIP stream) is free and a block of the request's HBM footprint is free in
 * the server's arena, launches them, and returns finished ones.  The arena
 * is hbm_budget bytes of device memory allocated once by fh_server_create;
 * each running request's workspace is a block of it, returned when the
 * request finishes, so admission never allocates or frees device memory and
 * the server holds exactly the budget.  Admitted requests run concurrently on
 * separate streams, so requests that arrive while others are on the GPU
 * overlap with them.  Results are identical to running each request alone
 * with fh_hough_candidates (same kernels, same integer arithmetic).
 * All server calls must come from the thread that owns the context. */
typedef struct fh_server fh_server;

typedef struct {
    const fh_peakmap *pm;  /* resident peakmap of the request's band            */
    fh_grid grid;          /* band (b0, nf), spin-down rows, reference time     */
    fh_select sel;
    int32_t n_sky;         /* >= 1                                              */
    const double *sky;     /* host [n_sky][3]; copied by fh_server_submit       */
    const float *d_w;      /* device weights or NULL (see fh_hough_candidates)  */
    int32_t w_stride;      /* 0 or N                                            */
    fh_candidate *d_out;   /* device [n_sky][n_sb][2], caller-owned; valid once
                              the request's completion has been returned       */
    uint64_t tag;          /* caller's tag, echoed in the completion            */
} fh_request;

typedef struct {
    uint64_t id;
    uint64_t tag;
    int32_t status;        /* FH_OK, FH_E_CANCELLED, or the launch error        */
    int32_t lane;          /* lane that ran it (-1 if never admitted)           */
    double queue_ms;       /* submit -> admission                               */
    double latency_ms;     /* submit -> completion seen by fh_server_poll       */
    double device_ms;      /* device time of the request's launches             */
    int64_t footprint;     /* HBM bytes charged against the budget              */
    int64_t cell_updates;
} fh_completion;

/* hbm_budget: bytes of the device arena that in-flight requests share (rounded
 * down to 256; FH_E_NOMEM if it cannot be allocated); lanes: concurrent
 * requests (streams), 1 .. 16; max_queue: pending requests accepted before
 * fh_server_submit returns FH_E_BUSY. */
fh_status fh_server_create(fh_ctx *ctx, int64_t hbm_budget, int32_t lanes, int32_t max_queue,
                           fh_server **out);

/* Validate and queue a request; *id receives its id.  Its directions run in
 * chunks sized so that one chunk's workspace fits budget / lanes where it
 * can.  FH_E_BUSY when the queue is full; FH_E_UNSUPPORTED when the request's
 * workspace for one direction at a time exceeds the budget. */
fh_status fh_server_submit(fh_server *srv, const fh_request *req, uint64_t *id);

/* Make progress (retire finished lanes, admit and launch queued requests) and
 * copy up to max finished requests into out; *n receives how many. */
fh_status fh_server_poll(fh_server *srv, fh_completion *out, int32_t max, int32_t *n);

/* Cancel a queued request (its completion reports FH_E_CANCELLED); FH_E_BUSY
 * if it is already running, FH_E_INVALID if the id is unknown or finished. */
fh_status fh_server_cancel(fh_server *srv, uint64_t id);

/* Requests queued, running, and finished but not yet returned. */
fh_status fh_server_stats(const fh_server *srv, int32_t *queued, int32_t *running,
                          int32_t *finished, int64_t *bytes_in_flight);

/* Admit and run every queued request and wait until none is running; their
 * completions stay available to fh_server_poll.  FH_E_DEVICE if a wait
 * fails. */
fh_status fh_server_drain(fh_server *srv);

/* Wait for all queued and running requests to finish, then free the server
 * (completions not yet polled are dropped).  NULL is a no-op. */
void fh_server_destroy(fh_server *srv);

/* ---- measurement ---------------------------------------------------------- */

/* Device time of the kernels of this context, measured with HIP events
 * recorded on the stream each kernel is launched on. */
typedef struct {
    double tiles_ms;          /* LDS-histogram tile kernels                  */
    int64_t tiles_launches;
    double front_ms;          /* shifts, weights, stripe edges, windows      */
    int64_t front_launches;
    double select_ms;         /* candidate selection                         */
    int64_t select_launches;
    int64_t cell_updates;     /* peaks x rows x directions of timed calls    */
    double graph_ms;          /* replays of captured searches (use_graph)    */
    int64_t graph_launches;
} fh_profile;

/* enable = 1 starts recording (and clears the totals); 0 stops. */
fh_status fh_ctx_profile(fh_ctx *ctx, int32_t enable);

/* Synchronise the device and read the totals recorded so far. */
fh_status fh_ctx_profile_read(fh_ctx *ctx, fh_profile *out);

#ifdef __cplusplus
}
#endif
#endif /* FH_H */
