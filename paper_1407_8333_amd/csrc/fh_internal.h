// Internal declarations shared by the HIP kernels and the host runtime of the
// frequency-Hough library.  Not part of the public C ABI (include/fh.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fh.h"

namespace fh {

// Rows of one LDS tile (lanes 0-15 of each 16-lane group of a wave hold one
// spin-down row each; the four groups of a wave process four peaks).
constexpr int kTileRows = 16;
// Row blocks sharing one peak-window table entry.
constexpr int kRowBlocksPerGroup = 4;
// Threads per tile workgroup (16 waves).
constexpr int kTileThreads = 1024;
constexpr int kTileWaves = kTileThreads / 64;
// FFTs per tile wave and the padded FFT count of a window row: every wave of
// a tile takes the same number of FFTs, a multiple of 12 (blocks of four FFTs
// in a ring of three blocks), and the window entries past the last FFT are
// empty.
__host__ __device__ inline int32_t wave_ffts(int32_t n_fft) {
    const int32_t per = (n_fft + kTileWaves - 1) / kTileWaves;
    return (per + 11) / 12 * 12;
}
__host__ __device__ inline int32_t win_stride(int32_t n_fft) { return kTileWaves * wave_ffts(n_fft); }
// LDS bytes available to one tile workgroup on gfx950.
constexpr int kLdsBytes = 163840;
// Bytes of LDS reserved for the scheduler slot and alignment.
constexpr int kLdsReserve = 256;
// dump columns after a tile's W + K_f - 1 columns (one per lane group)
constexpr int kDumpCols = 4;
// A last row block of at most kTailRows grid rows is not run as tiles of its
// own: the tiles of the row block before it also accumulate those rows, one
// atomic per peak and row, in LDS rows after their 16.
constexpr int kTailRows = 3;
// dump words after a tail row's W + K_f - 1 columns (one per lane of a wave)
constexpr int kTailDump = 64;
// Number of XCDs of an MI355X; workgroup w is dispatched to XCD w % 8.
constexpr int kXcds = 8;
// Padding entries after each FFT's stripe edges (never inside a window).
constexpr int kYPad = 16;
// Stripe edges per sky direction: every peak plus kYPad per FFT, plus one
// block of slack at the end (a block load reads up to 63 past a window start).
__host__ __device__ inline int64_t y_stride(int64_t n_peaks, int32_t n_fft) {
    return n_peaks + (int64_t)kYPad * n_fft + 64;
}

// Per-weight-vector statistics computed on the device.
struct WeightStats {
    double sum_w;   // sum of w_i
    double sum_w2;  // sum of w_i^2
    int32_t frac_bits;  // F: fixed-point fractional bits of the weights
    int32_t bad;        // 1 if a weight is not finite or outside (0, 65536)
};

// Arguments of the tile kernels.
struct TileArgs {
    int32_t n_fft;
    int64_t n_peaks;
    int32_t kf, nf, ns, W;        // W: fine bins per tile
    int32_t nrb, nbb, nrbg;       // row blocks run by the tiles, bin blocks, row-block groups
    int32_t tail;                 // grid rows past the last run row block (0..kTailRows), done by its tiles
    int32_t n_slots;              // sky directions in this chunk
    const uint32_t *Y;            // [slot][P] low words of the stripe edges (2^-16 fine bins)
    const int2 *win;              // [slot][nrbg][nbb][win_stride(N)] sorted windows
    const uint2 *rec;             // [nrb][N] low word of G_{i,s0} and the rows' residual codes
    const uint32_t *step;         // [N][16] floor(j q_i / 2^16): the rows' linear steps
    const uint32_t *wq;           // [slot][N] fixed-point weights or nullptr
    const WeightStats *ws;        // [slot * ws_stride] or nullptr
    int32_t ws_stride;            // 0: one shared weight vector, 1: one per slot
    int32_t *map_i32;             // [ns][nf] (plain map, single slot)
    float *map_f32;               // [ns][nf]
    unsigned long long *colmax;   // [slot][nf] packed (value << 32 | ~row)
    // persistent scheduling
    int32_t *queue_ctr;           // [kXcds] claimed positions of the tile queues
    int32_t tile_base;            // first tile id of a plain launch
};

// ---- launchers (fh_kernels.hip) ----
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
// p[0..2] = (x, y, z), written by a kernel (no copy from host memory)
hipError_t launch_set_f64x3(double *p, double x, double y, double z, hipStream_t st);
// spin-down shift tables of G_is = rint(((fdot0 + s dfdot) (t_i - t0)) (K_f T_FFT) 2^16):
// gwin [N][nrbg][2] (first and last grid row of each row group), rec [nrb][N],
// step [N][16] (see k_shift_tables); err bit 2 if a residual code overflows
// (nrb row blocks of records; windows for the row groups of the first
// nrb_run blocks, the last group reaching the grid's last row)
hipError_t launch_shift_tables(int32_t n_fft, int32_t nrb, int32_t nrb_run, int32_t ns, const double *t, double t0,
                               double t_fft,
                               int32_t kf, double fdot0, double dfdot, int64_t *gwin, uint2 *rec, uint32_t *step,
                               int32_t *err, hipStream_t st);
hipError_t launch_weight_stats(int32_t n_fft, int32_t n_vec, const float *w, int32_t w_stride,
                               int32_t mult, WeightStats *ws, int32_t *err_flag, hipStream_t st);
hipError_t launch_prep(int32_t n_fft, int64_t n_peaks, const int64_t *offsets, const int32_t *bins,
                       const double *v, const double *sky, int32_t n_slots, int32_t kf, int64_t b0,
                       int64_t *Y, const float *w, int32_t w_stride,
                       const WeightStats *ws, int32_t ws_stride, uint32_t *wq, uint32_t *Y32,
                       int32_t shift_mode, double q, hipStream_t st);
// fused stripe edges + weights + windows (LDS-staged edges of F FFTs per
// workgroup); F = front_ffts_per_block(max peaks of one FFT), 0 when even one
// FFT's edges do not fit (then use launch_prep + launch_windows).  FFTs of
// kFrontBigFft peaks or more go at most four to a workgroup: the front is
// latency-bound, and more, smaller workgroups per CU hide more of it.
constexpr int kFrontLdsBytes = 48 * 1024;
constexpr int kFrontBigFft = 256;
constexpr int kFrontMaxF = 16;
int front_ffts_per_block(int32_t max_per_fft);
hipError_t launch_front(int32_t n_fft, int64_t n_peaks, const int64_t *offsets, const int32_t *bins,
                        const double *v, const double *sky, int32_t n_slots, int32_t kf, int64_t b0,
                        const int64_t *gwin, uint32_t *Y, const float *w,
                        int32_t w_stride, const WeightStats *ws, int32_t ws_stride, uint32_t *wq,
                        int32_t ns, int32_t nrbg, int32_t nbb, int32_t W, int32_t F, int32_t max_per_fft,
                        int2 *win, int32_t shift_mode, double q, hipStream_t st);
// shift_mode 1: Doppler correction as a per-FFT shift computed at the
// reference q = (K_f T_FFT) f_ref fine bins (0: exact per peak)
// window rows sorted by window size per tile-wave run (see k_sort_windows)
hipError_t launch_sort_windows(int32_t n_fft, int32_t nrbg, int32_t nbb, int32_t n_slots, const int2 *win,
                               int2 *wsorted, hipStream_t st);
// method 0: two binary searches per entry; 1: one sweep per FFT
hipError_t launch_windows(int32_t n_fft, const int64_t *offsets, const int64_t *Y, int64_t n_peaks,
                          const int64_t *gwin, int32_t nrbg, int32_t nbb, int32_t W,
                          int32_t kf, int32_t n_slots, int2 *win, int method, hipStream_t st);
hipError_t launch_tiles(const TileArgs &a, bool weighted, bool want_map, bool want_colmax,
                        bool persistent, int32_t n_tiles, int32_t grid_blocks, hipStream_t st);
hipError_t launch_select(const unsigned long long *colmax, int32_t nf, int32_t n_slots,
                         const fh_select &sel, int32_t sky_base, int32_t n_fft,
                         const WeightStats *ws, int32_t ws_stride, fh_candidate *out,
                         hipStream_t st);
// peakmap construction from equalised spectra
hipError_t launch_pm_rows(int32_t n_fft, int32_t n_bins, int64_t ld, const float *sp, const float *sar,
                          int32_t k0, float theta, int32_t cap, int32_t *scratch, int32_t *counts,
                          hipStream_t st);
hipError_t launch_pm_scan(int32_t n_fft, const int32_t *counts, int64_t *offsets, hipStream_t st);
hipError_t launch_pm_pack(int32_t n_fft, int32_t cap, const int32_t *scratch, const int64_t *offsets,
                          int32_t *bins, hipStream_t st);
// peaks of each FFT with natural bin in [k_lo, k_hi) into a new CSR
hipError_t launch_slice(int32_t n_fft, const int64_t *offsets, const int32_t *bins, int32_t k_lo, int32_t k_hi,
                        int64_t *first, int32_t *counts, int64_t *out_offsets, int32_t *out_bins,
                        hipStream_t st);
// best of the first candidates of each refined direction, per coarse candidate
hipError_t launch_refine_pick(int32_t n_cand, int32_t n_dir, const fh_candidate *cands, const double *params,
                              const double *lamb, fh_refined *out, hipStream_t st);
// peakmap cleaning
hipError_t launch_gross_hist(int32_t n_fft, const int64_t *offsets, const int32_t *bins, const double *t,
                             double t_fft, const fh_gross &geo, int32_t *hist, hipStream_t st);
// filter of the peaks of a peakmap (mode 0: gross cells over thr; mode 1:
// natural bins whose statistic exceeds thr); phase 0 counts survivors per
// FFT and scans them into out_offsets, phase 1 packs the survivors
struct FilterSpec {
    int mode;
    const double *t;
    double t_fft;
    fh_gross geo;
    const int32_t *hist;
    int32_t k_lo, k_hi, step;
    int64_t offset, n_x;
    const int32_t *x;
    double thr;
};
hipError_t launch_filter(int32_t n_fft, const int64_t *offsets, const int32_t *bins, const FilterSpec &spec,
                         int32_t *counts, int64_t *out_offsets, int32_t *out_bins, int phase, hipStream_t st);
hipError_t launch_bin_counts(int32_t n_fft, const int64_t *offsets, const int32_t *bins, int32_t k_lo,
                             int32_t k_hi, int32_t *counts, hipStream_t st);
// robust statistic: hist needs 2 x_max + 1 entries; out[0] = m1, out[1] = m2
hipError_t launch_robust(const int32_t *x, int32_t n, int32_t x_max, int32_t *hist, int64_t *s2, double *out,
                         int32_t *err, hipStream_t st);
// decoded column maxima of n_slots directions: value [slot][nf], row [slot][nf]
hipError_t launch_colmax_decode(const unsigned long long *colmax, int32_t nf, int32_t n_slots, const WeightStats *ws,
                                int32_t ws_stride, float *value, int32_t *row, hipStream_t st);
hipError_t launch_colmax_values(const unsigned long long *colmax, int32_t nf, int32_t *out, hipStream_t st);
// LDS bytes of a tile of 16 + tail rows
int tile_lds_bytes(int W, int kf, int tail);
// Raise the dynamic-LDS limit of the tile kernels (once per device).
hipError_t init_kernel_attributes();
// widest tile (multiple of 64) of `rows` LDS rows that the LDS holds and
// that keeps 32-bit tile-relative stripe edges exact when a row's spin-down
// step is at most step_bins fine bins; 0 when no tile does
int max_tile_bins(int kf, double step_bins, int rows);

}  // namespace fh
