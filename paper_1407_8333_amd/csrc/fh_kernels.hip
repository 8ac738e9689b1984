// HIP kernels of the frequency-Hough (FH) library for gfx950 (MI355X).
//
// Pipeline for one chunk of sky directions (Sec. "Frequency-Hough transform"):
//   k_shift_tables per (FFT, row block): the rows' shifts G_is in 2^-16 fine
//                  bins (Eqs. uno, sdstep) as compact tables.  sky independent
//   k_weight_stats per weight vector: sum w, sum w^2, fixed-point bits F.
//   k_prep         per (sky, peak): Doppler-corrected stripe edge Y (Eq.
//                  fdopp, Eq. due) and per (sky, FFT) fixed-point weights.
//   k_windows      per (sky, row-block group, bin block, FFT): the contiguous
//                  range of that FFT's peaks whose stripes reach the tile.
//   k_tiles_*      per tile of 16 rows x W fine bins: LDS histogram of stripe
//                  starts (one ds_add_u32 per peak and row), then the
//                  differential +w/-w sum along each row as a width-K_f window
//                  (Eqs. ncount, ncountadap, freqres); writes the map and/or the
//                  per-bin maximum over rows.
//   k_select       per (sky, sub-band): first and second-order candidates
//                  (Sec. "Selection of first level candidates").
//
// All FP64 arithmetic is IEEE round-to-nearest-even with contraction off, so
// the integer stripe edges agree bit for bit with any other implementation of
// the same definition.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fh_internal.h"

#pragma clang fp contract(off)

namespace fh {

namespace {

// Fixed point of stripe edges: kQ = 2^kFrac steps per fine bin.
constexpr int kFrac = 16;
constexpr double kQd = 65536.0;
constexpr int64_t kQ = (int64_t)1 << kFrac;

__device__ __forceinline__ int64_t shrq(int64_t a) { return a >> kFrac; }  // floor(a / kQ)

// Stripe edge stored in the kYPad slots after each FFT's peaks (never inside
// a window; the slots keep every FFT's run of edges followed by readable
// memory).
constexpr int64_t kYSentinel = (int64_t)1 << 61;

// Tile-relative edges are 32-bit: with kFrac = 16 fractional bits a column is
// the upper half-word, inside +-2^15.  A peak of a window starts within 64
// rows' worth of spin-down steps of the tile (the window covers a group of
// 64 rows, the last group up to kTailRows more; the last row block may reach
// 16 rows past the grid), so max_tile_bins bounds W + K_f + 80 (step + 1) +
// 64 below 2^15.  kFarEdge
// (16384 bins) then stays in range and beyond the dump column for every row.
constexpr uint32_t kFarEdge = 16384u << kFrac;

// ----------------------------------------------------------------------------
// fills (graph-safe replacements for memset)

__global__ void k_fill_u64(unsigned long long *__restrict__ p, int64_t n, unsigned long long v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_set_f64x3(double *__restrict__ p, double x, double y, double z) {
    if (threadIdx.x == 0) {
        p[0] = x;
        p[1] = y;
        p[2] = z;
    }
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ----------------------------------------------------------------------------
// spin-down shifts (Eqs. uno, sdstep): row s has the spin-down
// fdot_s = fdot0 + s dfdot, and FFT i's stripes in that row are shifted by
//   G_is = rint((fdot_s tau_i) S),  tau_i = t_i - t0,  S = (K_f T_FFT) kQ
// rounded once per row (rows past the grid, up to the end of the last row
// block, follow the same formula and never reach the output).

__device__ __forceinline__ int64_t row_shift(double tau, double S, double fdot0, double dfdot, int32_t s) {
    double fs = (double)s * dfdot;
    fs = fdot0 + fs;
    double a = fs * tau;
    a = a * S;
    return (int64_t)rint(a);
}

// The tiles need, for FFT i and the 16 rows s0 + j of a row block, the
// offsets G_{i,s0} - G_{i,s0+j}.  With q_i = rint(((dfdot tau_i) S) 2^16) the
// row step in 2^-32 fine bins, floor(j q_i / 2^16) is within (-1, 1] + 1e-3
// of j's exact step, and each G within 0.5 of its exact value, so
//   c_ij = G_{i,s0+j} - G_{i,s0} - floor(j q_i / 2^16)  lies in {-1, 0, 1, 2}.
// Tables (all sky independent):
//   step[i][j]  = low word of floor(j q_i / 2^16)                  [N][16]
//   rec[rb][i]  = (low word of G_{i,s0}, sum_j (c_ij + 1) << 2j)   [nrb][N]
//   gwin[i][g]  = (G_is at the first and at the last grid row of row
//                 group g), for the peak windows                   [N][nrbg][2]
// A code outside {-1 .. 2} (impossible by the bound above) sets bit 2 of the
// error flag.
__global__ void k_shift_tables(int32_t n_fft, int32_t nrb, int32_t nrb_run, int32_t ns,
                               const double *__restrict__ t, double t0,
                               double S, double fdot0, double dfdot, int64_t *__restrict__ gwin,
                               uint2 *__restrict__ rec, uint32_t *__restrict__ step,
                               int32_t *__restrict__ err) {
    // row groups of the row blocks the tiles run; the last one reaches the
    // grid's last row (the rows of a folded last block included)
    const int32_t nrbg = (nrb_run + kRowBlocksPerGroup - 1) / kRowBlocksPerGroup;
    const int64_t n = (int64_t)n_fft * nrb;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t rb = (int32_t)(x / n_fft);
        const int32_t i = (int32_t)(x - (int64_t)rb * n_fft);
        const double tau = t[i] - t0;
        double sig = dfdot * tau;
        sig = sig * S;
        const int64_t q = (int64_t)rint(sig * 65536.0);
        const int32_t s0 = rb * kTileRows;
        const int64_t g0 = row_shift(tau, S, fdot0, dfdot, s0);
        uint32_t codes = 0;
        bool bad = false;
        for (int j = 0; j < kTileRows; ++j) {
            const int64_t lin = ((int64_t)j * q) >> 16;  // floor (arithmetic shift)
            const int64_t c = row_shift(tau, S, fdot0, dfdot, s0 + j) - g0 - lin;
            bad = bad || c < -1 || c > 2;
            codes |= (uint32_t)((c + 1) & 3) << (2 * j);
            if (rb == 0) step[(int64_t)i * kTileRows + j] = (uint32_t)(uint64_t)lin;
        }
        rec[(int64_t)rb * n_fft + i] = make_uint2((uint32_t)(uint64_t)g0, codes);
        if (bad) atomicOr(err, 2);
        if (rb < nrb_run && rb % kRowBlocksPerGroup == 0) {
            const int32_t g = rb / kRowBlocksPerGroup;
            const int32_t s_hi = g == nrbg - 1 ? ns - 1 : s0 + kRowBlocksPerGroup * kTileRows - 1;
            gwin[((int64_t)i * nrbg + g) * 2] = g0;
            gwin[((int64_t)i * nrbg + g) * 2 + 1] = row_shift(tau, S, fdot0, dfdot, s_hi);
        }
    }
}

// ----------------------------------------------------------------------------
// weight statistics and fixed-point scale (Eq. ncountadap)

__global__ void k_weight_stats(int32_t n, const float *__restrict__ w, int32_t w_stride,
                               int32_t mult, WeightStats *__restrict__ ws,
                               int32_t *__restrict__ err_flag) {
    const float *wv = w + (int64_t)blockIdx.x * w_stride;
    double s1 = 0.0, s2 = 0.0;
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double x = (double)wv[i];
        if (!(x > 0.0 && x < 65536.0)) bad = 1;  // also catches NaN
        s1 += x;
        s2 += x * x;
    }
    __shared__ double r1[256], r2[256];
    __shared__ int rb[256];
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    rb[threadIdx.x] = bad;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
            rb[threadIdx.x] |= rb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        WeightStats st;
        st.sum_w = r1[0];
        st.sum_w2 = r2[0];
        st.bad = rb[0];
        // a cell holds at most mult * sum_i rint(w_i 2^F) <= mult (2^F sum w + N/2)
        double lim = (4294967295.0 / (double)mult - 0.5 * (double)n) / r1[0];
        int F = -1;
        if (!rb[0] && lim >= 1.0) {
            F = 0;
            while (F < 40 && ldexp(1.0, F + 1) <= lim) ++F;
        }
        if (F < 0) st.bad = 1;
        st.frac_bits = F < 0 ? 0 : F;
        ws[blockIdx.x] = st;
        if (st.bad) atomicOr(err_flag, 1);
    }
}

// ----------------------------------------------------------------------------
// per-peak stripe edge.  For peak (i, k) and sky n:
//   r = 1 / (1 + ((vx nx + vy ny) + vz nz))                     (Eq. fdopp)
//   X = floor(((double)(K_f k) r) kQ)
//   Y = X - b0 kQ - K_f kQ/2 + (kQ - 1)
// so that the first fine bin of the stripe in row s is
//   a_s = ceil((X - b0 kQ - K_f kQ/2 - G_is) / kQ)
//       = floor((Y - G_is) / kQ).
// One wave per FFT; grid.y = sky slot.

__global__ void __launch_bounds__(256) k_prep(
    int32_t n_fft, int64_t n_peaks, const int64_t *__restrict__ offsets,
    const int32_t *__restrict__ bins, const double *__restrict__ v,
    const double *__restrict__ sky, int32_t kf, int64_t b0,
    int64_t *__restrict__ Y, const float *__restrict__ w, int32_t w_stride,
    const WeightStats *__restrict__ ws, int32_t ws_stride, uint32_t *__restrict__ wq,
    uint32_t *__restrict__ Y32, int32_t shift_mode, double q) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int slot = blockIdx.y;
    if (i >= n_fft) return;
    const double *n = sky + 3 * (int64_t)slot;
    const double *vi = v + 3 * (int64_t)i;
    double d = vi[0] * n[0];
    d = d + vi[1] * n[1];
    d = d + vi[2] * n[2];
    d = 1.0 + d;
    const double r = 1.0 / d;
    int64_t c = -b0 * kQ - (int64_t)kf * (kQ / 2) + (kQ - 1);
    if (shift_mode) c -= llrint((q * (1.0 - r)) * kQd);  // per-FFT shift at the reference
    // FFT i's edges start at offsets[i] + kYPad * i and are followed by kYPad
    // sentinels
    int64_t *Ys = Y + (int64_t)slot * y_stride(n_peaks, n_fft) + (int64_t)kYPad * i;
    uint32_t *Ys32 = Y32 + (int64_t)slot * y_stride(n_peaks, n_fft) + (int64_t)kYPad * i;
    const int64_t e = offsets[i + 1];
    for (int64_t p = offsets[i] + lane; p < e; p += 64) {
        int64_t y;
        if (shift_mode) {
            y = (int64_t)kf * (int64_t)bins[p] * kQ + c;
        } else {
            double x = (double)((int64_t)kf * (int64_t)bins[p]) * r;
            x = x * kQd;
            y = (int64_t)floor(x) + c;
        }
        Ys[p] = y;
        Ys32[p] = (uint32_t)y;
    }
    if (lane < kYPad) {
        Ys[e + lane] = kYSentinel;
        Ys32[e + lane] = (uint32_t)kYSentinel;
    }
    if (w != nullptr && lane == 0) {
        const WeightStats st = ws[(int64_t)slot * ws_stride];
        double wi = (double)w[(int64_t)slot * w_stride + i];
        wq[(int64_t)slot * n_fft + i] = st.bad ? 0u : (uint32_t)rint(ldexp(wi, st.frac_bits));
    }
}

// ----------------------------------------------------------------------------
// Fused front: for one direction slot and F consecutive FFTs f0 .. f0+F-1
// (grid.x over the padded FFT count, grid.y = slot), the stripe edges of
// their peaks (written out for the tiles and staged in LDS), their
// fixed-point weights, and every window entry (row group, bin block, FFT) by
// two binary searches over the staged edges.  The window of a tile is the run
// of peaks p with
//   max_s a_s(p) >= jb W - (K_f - 1)   and   min_s a_s(p) < (jb + 1) W
// over the group's rows s (a_s is monotone in Y, Y ascending within an FFT;
// G_is is monotone in s, so its extremes over the rows are those of the
// first and last row).  Consecutive threads write consecutive FFTs of a
// window row.

__global__ void __launch_bounds__(256) k_front(
    int32_t n_fft, int64_t n_peaks, const int64_t *__restrict__ offsets,
    const int32_t *__restrict__ bins, const double *__restrict__ v,
    const double *__restrict__ sky, int32_t kf, int64_t b0, const int64_t *__restrict__ gwin,
    uint32_t *__restrict__ Y, const float *__restrict__ w,
    int32_t w_stride, const WeightStats *__restrict__ ws, int32_t ws_stride,
    uint32_t *__restrict__ wq, int32_t ns, int32_t nrbg, int32_t nbb, int32_t W, int32_t F,
    int32_t search_top, int2 *__restrict__ win, int32_t shift_mode, double q) {
    extern __shared__ int64_t ys[];
    __shared__ int64_t s_off[kFrontMaxF + 1];  // offsets of the block's FFTs
    __shared__ int32_t s_loc[kFrontMaxF + 1];  // the same, from the block's first peak
    __shared__ int64_t s_c[kFrontMaxF];        // per-FFT constant of the edge
    __shared__ double s_r[kFrontMaxF];         // per-FFT inverse Doppler factor
    const int slot = blockIdx.y;
    const int f0 = blockIdx.x * F;
    const int fe = min(f0 + F, n_fft);
    const int nfl = fe - f0;  // FFTs of this block (<= 0 for padding blocks)
    const int32_t n_pad = win_stride(n_fft);
    uint32_t *Yslot = Y + (int64_t)slot * y_stride(n_peaks, n_fft);
    // padded index of the first staged edge
    const int64_t pb = f0 < n_fft ? offsets[f0] + (int64_t)kYPad * f0 : 0;

    // per-FFT terms (r, constant, weight), one thread per FFT
    const double *n = sky + 3 * (int64_t)slot;
    if ((int)threadIdx.x <= nfl) {
        const int64_t o = offsets[f0 + threadIdx.x];
        s_off[threadIdx.x] = o;
        s_loc[threadIdx.x] = (int32_t)(o - offsets[f0]);
    }
    if ((int)threadIdx.x < nfl) {
        const int i = f0 + threadIdx.x;
        const double *vi = v + 3 * (int64_t)i;
        double d = vi[0] * n[0];
        d = d + vi[1] * n[1];
        d = d + vi[2] * n[2];
        d = 1.0 + d;
        const double r = 1.0 / d;
        s_r[threadIdx.x] = r;
        int64_t c = -b0 * kQ - (int64_t)kf * (kQ / 2) + (kQ - 1);
        if (shift_mode) c -= llrint((q * (1.0 - r)) * kQd);  // per-FFT shift at the reference
        s_c[threadIdx.x] = c;
        if (w != nullptr) {
            const WeightStats wst = ws[(int64_t)slot * ws_stride];
            double wi = (double)w[(int64_t)slot * w_stride + i];
            wq[(int64_t)slot * n_fft + i] = wst.bad ? 0u : (uint32_t)rint(ldexp(wi, wst.frac_bits));
        }
    }
    __syncthreads();

    // stripe edges (as k_prep) of all the block's peaks: wave w takes FFTs w,
    // w + 4, ..., its lanes that FFT's consecutive peaks, so no lane searches
    // for its FFT and its Doppler factor and constant are read once per FFT
    if (nfl > 0) {
        const int64_t P0 = s_off[0];
        // peak indices local to the block (32-bit: a block holds at most
        // 48 KB of edges); K_f k < 2^28 (checked at upload), so the natural
        // frequency in fine bins converts to double from 32 bits exactly
        const int32_t *__restrict__ kbins = bins + P0;
        uint32_t *__restrict__ Yb = Yslot + P0 + (int64_t)kYPad * f0;
        const int lane = (int)threadIdx.x & 63, nw = (int)blockDim.x >> 6;
        constexpr int kU = 4;  // peaks per lane and round, their natural bins requested together
        for (int l = (int)threadIdx.x >> 6; l < nfl; l += nw) {
            const int pa = s_loc[l], pe = s_loc[l + 1];
            const double r = s_r[l];
            const int64_t c = s_c[l];
            for (int lb = pa + lane; lb < pe; lb += 64 * kU) {
                int32_t kb[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int lp = lb + 64 * u;
                    kb[u] = lp < pe ? kbins[lp] : 0;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int lp = lb + 64 * u;
                    if (lp >= pe) break;
                    int64_t y;
                    if (shift_mode) {
                        y = (int64_t)(kf * kb[u]) * kQ + c;
                    } else {
                        double x = (double)(kf * kb[u]) * r;
                        x = x * kQd;
                        y = (int64_t)floor(x) + c;
                    }
                    const int li = lp + kYPad * l;
                    Yb[li] = (uint32_t)y;  // the tiles use the low word
                    ys[li] = y;
                }
            }
        }
        for (int t = threadIdx.x; t < nfl * kYPad; t += blockDim.x) {
            const int fl = t / kYPad;
            Yslot[s_off[fl + 1] + (int64_t)kYPad * (f0 + fl) + (t - fl * kYPad)] = (uint32_t)kYSentinel;
        }
    }
    __syncthreads();

    // Window entries e = tid + k blockDim, e = (g nbb + jb) F + fl: F divides
    // blockDim, so a thread keeps one FFT fl, and its row index g nbb + jb
    // advances by blockDim / F per entry (no division per entry).  Each of
    // the two searches is a branchless binary lifting over the FFT's staged
    // edges: powers of two from search_top (the largest power of two up to
    // the longest FFT's peak count) down to 1, a step taken while the edge
    // it passes is below the bound.
    const int fl = (int)threadIdx.x & (F - 1);
    const int step_r = (int)blockDim.x / F;
    const int n_rows = nrbg * nbb;
    int rest = (int)threadIdx.x / F;
    int g = rest / nbb, jb = rest - g * nbb;
    const int dg = step_r / nbb, djb = step_r - dg * nbb;
    const int f = f0 + fl;
    const bool live = fl < nfl;
    int a0 = 0, end = 0;
    if (live) {
        a0 = s_loc[fl] + kYPad * fl;
        end = s_loc[fl + 1] + kYPad * fl;
    }
    const int64_t *__restrict__ gq = gwin + (int64_t)f * nrbg * 2;
    int2 *__restrict__ wp = win + (int64_t)slot * n_rows * n_pad + f;
    for (; rest < n_rows; rest += step_r) {
        int2 out = make_int2(0, 0);
        if (live) {
            // shifts of the group's first and last grid rows
            const int64_t q_lo = gq[2 * g], q_hi = gq[2 * g + 1];
            // max_s a_s = floor((Y - min G) / kQ) >= t  <=>  Y >= t kQ + min G
            // min_s a_s = floor((Y - max G) / kQ) >= t  <=>  Y >= t kQ + max G
            const int64_t y_lo = ((int64_t)jb * W - (kf - 1)) * kQ + (q_lo < q_hi ? q_lo : q_hi);
            const int64_t y_hi = (int64_t)(jb + 1) * W * kQ + (q_lo < q_hi ? q_hi : q_lo);
            int lo = a0, hi = a0;  // first peaks with Y >= y_lo and with Y >= y_hi
            for (int stp = search_top; stp > 0; stp >>= 1) {
                const int t1 = lo + stp - 1, t2 = hi + stp - 1;
                const int64_t v1 = ys[t1 < end ? t1 : a0], v2 = ys[t2 < end ? t2 : a0];
                lo += (t1 < end && v1 < y_lo) ? stp : 0;
                hi += (t2 < end && v2 < y_hi) ? stp : 0;
            }
            out = make_int2((int)(lo + pb), (int)(hi + pb));
        }
        wp[(int64_t)rest * n_pad] = out;
        g += dg;
        jb += djb;
        if (jb >= nbb) {
            jb -= nbb;
            ++g;
        }
    }
}

// ----------------------------------------------------------------------------
// peak windows.  A peak reaches tile (row group g, bin block jb) when its
// stripe start, over the group's rows, meets the tile's LDS columns
// [0, W + K_f - 1) measured from fine bin jb*W - (K_f - 1).  Stripe starts are
// monotone in Y, and Y is ascending within an FFT, so the peaks that reach a
// tile form one contiguous range, found by two binary searches.

__global__ void k_windows(int32_t n_fft, const int64_t *__restrict__ offsets,
                          const int64_t *__restrict__ Y, int64_t n_peaks,
                          const int64_t *__restrict__ gwin, int32_t nrbg,
                          int32_t nbb, int32_t W, int32_t kf, int2 *__restrict__ win) {
    const int32_t n_pad = win_stride(n_fft);
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nbb * n_pad) return;
    const int32_t jb = (int32_t)(idx / n_pad);
    const int32_t i = (int32_t)(idx - (int64_t)jb * n_pad);
    const int32_t g = blockIdx.y, slot = blockIdx.z;
    int2 *out = win + (((int64_t)slot * nrbg + g) * nbb + jb) * n_pad + i;
    if (i >= n_fft) {  // padding: empty window
        *out = make_int2(0, 0);
        return;
    }
    const int64_t c0 = (int64_t)jb * W - (kf - 1);
    const int64_t wc = (int64_t)W + kf - 1;
    const int64_t q_lo = gwin[((int64_t)i * nrbg + g) * 2] + c0 * kQ;
    const int64_t q_hi = gwin[((int64_t)i * nrbg + g) * 2 + 1] + c0 * kQ;
    const int64_t *Ys = Y + (int64_t)slot * y_stride(n_peaks, n_fft);
    const int64_t p0 = offsets[i] + (int64_t)kYPad * i, p1 = offsets[i + 1] + (int64_t)kYPad * i;
    // lo: first peak whose larger column is >= 0
    int64_t a = p0, b = p1;
    while (a < b) {
        int64_t m = (a + b) >> 1;
        int64_t y = Ys[m];
        int64_t c1 = shrq(y - q_lo), c2 = shrq(y - q_hi);
        int64_t cmax = c1 > c2 ? c1 : c2;
        if (cmax >= 0) b = m; else a = m + 1;
    }
    const int64_t lo = a;
    // hi: first peak whose smaller column is >= W + K_f - 1
    b = p1;
    while (a < b) {
        int64_t m = (a + b) >> 1;
        int64_t y = Ys[m];
        int64_t c1 = shrq(y - q_lo), c2 = shrq(y - q_hi);
        int64_t cmin = c1 < c2 ? c1 : c2;
        if (cmin >= wc) b = m; else a = m + 1;
    }
    *out = make_int2((int)lo, (int)a);
}

// Same windows by one sweep over each FFT's peaks (one wave per FFT, every
// row group): with jhi(p) / jlo(p) the last / first bin block that peak p
// reaches over a group's rows (non-decreasing in p),
//   lo[jb] = first p with jhi(p) >= jb,   hi[jb] = first p with jlo(p) > jb,
// and each lane writes the entries whose boundary falls on its peak.

__device__ __forceinline__ int floor_div_w(int64_t x, int W, float inv_w) {
    int q = (int)floorf((float)x * inv_w);
    if ((int64_t)q * W > x) --q;
    else if ((int64_t)(q + 1) * W <= x) ++q;
    return q;
}

__global__ void __launch_bounds__(256) k_windows_sweep(
    int32_t n_fft, const int64_t *__restrict__ offsets, const int64_t *__restrict__ Y,
    int64_t n_peaks, const int64_t *__restrict__ gwin, int32_t nrbg, int32_t nbb,
    int32_t W, int32_t kf, int2 *__restrict__ win) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int slot = blockIdx.y;
    const int32_t n_pad = win_stride(n_fft);
    if (i >= n_pad) return;
    if (i >= n_fft) {  // padding: empty windows
        for (int e = lane; e < nrbg * nbb; e += 64)
            win[((int64_t)slot * nrbg * nbb + e) * n_pad + i] = make_int2(0, 0);
        return;
    }
    const int64_t *Ys = Y + (int64_t)slot * y_stride(n_peaks, n_fft);
    const int p0 = (int)(offsets[i] + (int64_t)kYPad * i);
    const int p1 = (int)(offsets[i + 1] + (int64_t)kYPad * i);
    const int64_t *gi = gwin + (int64_t)i * nrbg * 2;
    const float inv_w = 1.0f / (float)W;
    for (int g = 0; g < nrbg; ++g) {
        int2 *wg = win + ((int64_t)slot * nrbg + g) * nbb * (int64_t)n_pad + i;
        const int64_t q_lo = gi[2 * g], q_hi = gi[2 * g + 1];
        int prev_hi = -1;  // jhi of the peak before this chunk
        int prev_lo = 0;   // jlo of the peak before this chunk
        for (int pb = p0; pb < p1; pb += 64) {
            const int p = pb + lane;
            int jhi = nbb - 1, jlo = nbb;  // past the segment end
            if (p < p1) {
                const int64_t y = Ys[p];
                const int64_t a1 = shrq(y - q_lo), a2 = shrq(y - q_hi);
                const int64_t amin = a1 < a2 ? a1 : a2, amax = a1 < a2 ? a2 : a1;
                jhi = max(-1, min(nbb - 1, floor_div_w(amax + kf - 1, W, inv_w)));
                jlo = max(0, min(nbb, floor_div_w(amin, W, inv_w)));
            }
            int before_hi = __shfl_up(jhi, 1);
            int before_lo = __shfl_up(jlo, 1);
            if (lane == 0) {
                before_hi = prev_hi;
                before_lo = prev_lo;
            }
            if (p < p1) {
                for (int jb = before_hi + 1; jb <= jhi; ++jb) wg[(int64_t)jb * n_pad].x = p;
                for (int jb = before_lo; jb < jlo; ++jb) wg[(int64_t)jb * n_pad].y = p;
            }
            const int last = min(63, p1 - 1 - pb);
            prev_hi = __shfl(jhi, last);
            prev_lo = __shfl(jlo, last);
        }
        // bin blocks past the last peak's reach end at the segment end
        for (int jb = prev_hi + 1 + lane; jb < nbb; jb += 64) wg[(int64_t)jb * n_pad].x = p1;
        for (int jb = prev_lo + lane; jb < nbb; jb += 64) wg[(int64_t)jb * n_pad].y = p1;
    }
}

// ----------------------------------------------------------------------------
// tiles

// Window rows ordered for the tiles.  Run w of a row holds every
// kTileWaves-th FFT, w, w + 16, w + 32, ... (so that every run spans the
// whole observation, whose windows widen with |t - t0|); its wave_ffts(N)
// FFTs are sorted by window size, largest first (a counting sort over sizes
// clipped to 127; the few windows of 127 peaks or more, which share the first
// bucket, are ranked exactly among themselves), so that the four FFTs of a
// tile block (four consecutive entries of a run) have nearly equal windows
// and the first holds the largest, which the tiles rely on.  An entry becomes
// (lo, m << 16 | count): FFT m * 16 + w of the row.  One workgroup per window
// row (grid.x = row group * bin blocks, grid.y = slot), one wave per run.
constexpr int kSortBuckets = 128;
// rows of at most this many bytes are first copied into LDS with 16-byte
// loads (the runs read the row with a 128-byte stride, twice)
constexpr int kSortStageBytes = 128 * 1024;

// Place of a window of c >= 127 peaks (entry e of a run of `per`) among the
// run's windows of 127 peaks or more, which fill the run's first places:
// larger first, equal sizes in run order.  entry(j) reads entry j of the run.
// Such windows are rare (dense peakmaps, K_f = 1), so a scan of the run is
// cheap enough.
template <typename Entry>
__device__ __forceinline__ int big_window_rank(int c, int e, int per, Entry entry) {
    int pos = 0;
    for (int j = 0; j < per; ++j) {
        const int2 o = entry(j);
        const int cj = o.y - o.x;
        pos += (cj > c || (cj == c && j < e)) ? 1 : 0;
    }
    return pos;
}

__global__ void __launch_bounds__(kTileThreads) k_sort_windows(int32_t n_fft, int32_t nrows,
                                                               const int2 *__restrict__ win,
                                                               int2 *__restrict__ wsorted) {
    extern __shared__ int4 s_row4[];
    __shared__ int hist[kTileWaves][kSortBuckets];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = wave_ffts(n_fft);
    const int n_pad = win_stride(n_fft);  // a multiple of 64 entries
    const int64_t row = (int64_t)blockIdx.y * nrows + blockIdx.x;
    const int2 *rowp = win + row * n_pad;
    {
        const int4 *g4 = reinterpret_cast<const int4 *>(rowp);
        for (int i = threadIdx.x; i < n_pad / 2; i += blockDim.x) s_row4[i] = g4[i];
    }
    // FFT m * kTileWaves + wave of the row is entry m of run `wave`
    const int2 *src = reinterpret_cast<const int2 *>(s_row4) + wave;
    int2 *dst = wsorted + row * n_pad + (int64_t)wave * per;
    int *h = hist[wave];
    for (int b = lane; b < kSortBuckets; b += 64) h[b] = 0;
    __syncthreads();
    // entries are read four per lane and round (one memory latency per round)
    constexpr int kU = 4;
    for (int e0 = lane; e0 < per; e0 += kU * 64) {
        int2 w2[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + 64 * u;
            w2[u] = e < per ? src[(int64_t)e * kTileWaves] : make_int2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (e0 + 64 * u < per) atomicAdd(&h[kSortBuckets - 1 - min(w2[u].y - w2[u].x, kSortBuckets - 1)], 1);
    }
    __syncthreads();
    // exclusive prefix sum over the buckets (lane L holds buckets 2L, 2L+1)
    const int a0 = h[2 * lane], a1 = h[2 * lane + 1];
    int incl = a0 + a1;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    const int excl = incl - (a0 + a1);
    __syncthreads();
    h[2 * lane] = excl;
    h[2 * lane + 1] = excl + a0;
    __syncthreads();
    for (int e0 = lane; e0 < per; e0 += kU * 64) {
        int2 w2[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + 64 * u;
            w2[u] = e < per ? src[(int64_t)e * kTileWaves] : make_int2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + 64 * u;
            if (e >= per) break;
            const int c = w2[u].y - w2[u].x;
            int pos;
            if (c >= kSortBuckets - 1) {
                pos = big_window_rank(c, e, per, [&](int j) { return src[(int64_t)j * kTileWaves]; });
            } else {
                pos = atomicAdd(&h[kSortBuckets - 1 - c], 1);
            }
            dst[pos] = make_int2(w2[u].x, (e << 16) | c);
        }
    }
}

// Rows longer than kSortStageEntries entries: the same sort, the row copied
// into LDS in pieces of kSortStageEntries (128 KB), once per pass.
constexpr int kSortStageEntries = 16384;

__global__ void __launch_bounds__(kTileThreads) k_sort_windows_long(int32_t n_fft, int32_t nrows,
                                                               const int2 *__restrict__ win,
                                                               int2 *__restrict__ wsorted) {
    extern __shared__ int4 s_row4[];
    __shared__ int hist[kTileWaves][kSortBuckets];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = wave_ffts(n_fft);
    const int n_pad = win_stride(n_fft);  // a multiple of 64 entries
    const int piece = kSortStageEntries;
    const int64_t row = (int64_t)blockIdx.y * nrows + blockIdx.x;
    const int2 *rowp = win + row * n_pad;
    const int2 *s_row = reinterpret_cast<const int2 *>(s_row4);
    int2 *dst = wsorted + row * n_pad + (int64_t)wave * per;
    int *h = hist[wave];
    // entries [p0, p0 + piece) of the row into LDS (both multiples of 64)
    auto stage = [&](int p0) {
        const int n = min(piece, n_pad - p0);
        const int4 *g4 = reinterpret_cast<const int4 *>(rowp + p0);
        for (int i = threadIdx.x; i < n / 2; i += blockDim.x) s_row4[i] = g4[i];
    };
    for (int b = lane; b < kSortBuckets; b += 64) h[b] = 0;
    __syncthreads();
    // Entry e of run `wave` is row entry e * kTileWaves + wave; a piece
    // starting at p0 holds the run's entries [p0 / 16, (p0 + piece) / 16).
    // Entries are read four per lane and round.
    constexpr int kU = 4;
    for (int p0 = 0; p0 < n_pad; p0 += piece) {
        if (p0 > 0) __syncthreads();
        stage(p0);
        __syncthreads();
        const int e_lo = p0 / kTileWaves, e_hi = min(per, (p0 + piece) / kTileWaves);
        for (int e0 = e_lo + lane; e0 < e_hi; e0 += kU * 64) {
            int2 w2[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int e = e0 + 64 * u;
                w2[u] = e < e_hi ? s_row[(e - e_lo) * kTileWaves + wave] : make_int2(0, 0);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (e0 + 64 * u < e_hi)
                    atomicAdd(&h[kSortBuckets - 1 - min(w2[u].y - w2[u].x, kSortBuckets - 1)], 1);
        }
    }
    __syncthreads();
    // exclusive prefix sum over the buckets (lane L holds buckets 2L, 2L+1)
    const int a0 = h[2 * lane], a1 = h[2 * lane + 1];
    int incl = a0 + a1;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    const int excl = incl - (a0 + a1);
    __syncthreads();
    h[2 * lane] = excl;
    h[2 * lane + 1] = excl + a0;
    __syncthreads();
    for (int p0 = 0; p0 < n_pad; p0 += piece) {
        if (p0 > 0) __syncthreads();
        stage(p0);
        __syncthreads();
        const int e_lo = p0 / kTileWaves, e_hi = min(per, (p0 + piece) / kTileWaves);
        for (int e0 = e_lo + lane; e0 < e_hi; e0 += kU * 64) {
            int2 w2[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int e = e0 + 64 * u;
                w2[u] = e < e_hi ? s_row[(e - e_lo) * kTileWaves + wave] : make_int2(0, 0);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int e = e0 + 64 * u;
                if (e >= e_hi) break;
                const int c = w2[u].y - w2[u].x;
                int pos;
                if (c >= kSortBuckets - 1) {
                    // the run's other pieces are not staged: read the row in memory
                    pos = big_window_rank(c, e, per, [&](int j) { return rowp[(int64_t)j * kTileWaves + wave]; });
                } else {
                    pos = atomicAdd(&h[kSortBuckets - 1 - c], 1);
                }
                dst[pos] = make_int2(w2[u].x, (e << 16) | c);
            }
        }
    }
}

// Raw buffer access with 32-bit byte offsets (no 64-bit address arithmetic
// per load); the records limit is never reached by the offsets used here.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, 0x7FFFFFFF, 0x00020000);
}
__device__ __forceinline__ uint32_t ld_u32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
}

// s_waitcnt operand that waits for every vector-memory access of the wave
// (vmcnt 0) and leaves the export and LDS/scalar counters alone.
constexpr int kWaitVmcnt0 = (0x7 << 4) | (0xF << 8);

// Workgroup barrier that orders LDS accesses only: global stores and atomics
// still in flight are not waited for.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS tile: word (c, j) = c * 16 + j holds the stripe starts of column c
// (fine bin jb*W - (K_f-1) + c) in row s0 + j; column W + K_f - 1 is a dump
// column for updates that fall outside the tile.  The 16 lanes of a group
// address 16 consecutive words, so a group's part of an LDS atomic never
// conflicts with itself (the four groups of a wave can still collide on the
// bank halves that their columns map to).
// One step of the accumulation.  Lane (group g, row j) adds the stripe of the
// peak held by lane (g, U): its edge, already made relative to the tile
// (v = Y - c0 kQ - G_{i,s0}, exact in 32 bits for every peak of a window),
// reaches the group's 16 lanes through DPP row_newbcast:U fused into the add
// of the lane's row term t = G_{i,s0} - G_{i,s0+j}.  col = floor((v + t) / kQ) is the tile
// column of the stripe start in row s0 + j; columns outside
// [0, W + K_f - 1) (negative ones wrap to large unsigned values) go to the
// group's dump column.
template <int U>
__device__ __forceinline__ uint32_t stripe_word(uint32_t v, uint32_t t, uint32_t dump, uint32_t lane_off) {
    const uint32_t b = __builtin_amdgcn_update_dpp(0u, v, 0x150 + U, 0xF, 0xF, true);
    // the column is the upper half-word (negative columns read as 2^15 and
    // more); one SDWA min takes it and clamps it to the dump column
    const uint16_t col = (uint16_t)((b + t) >> kFrac);
    const uint32_t cu = col < (uint16_t)dump ? col : (uint16_t)dump;
    return cu * kTileRows + lane_off;
}

// Steps U .. E-1, two at a time (independent address chains interleave).
template <int U, int E>
__device__ __forceinline__ void stripe_run(uint32_t v, uint32_t t, uint32_t dump,
                                           uint32_t lane_off, uint32_t val,
                                           uint32_t *__restrict__ lds) {
    if constexpr (U + 1 < E) {
        const uint32_t a0 = stripe_word<U>(v, t, dump, lane_off);
        const uint32_t a1 = stripe_word<U + 1>(v, t, dump, lane_off);
        atomicAdd(lds + a0, val);
        atomicAdd(lds + a1, val);
        stripe_run<U + 2, E>(v, t, dump, lane_off, val, lds);
    } else if constexpr (U < E) {
        atomicAdd(lds + stripe_word<U>(v, t, dump, lane_off), val);
    }
}

// A chunk of up to 16 peaks of each group's FFT occupies the lanes named by
// a 16-bit pattern m(n), n = min(peaks left in the block's largest window,
// 16), built from fixed runs so that each run is one straight sequence of
// steps: lanes 0-7 (n & 8), 8-11 (n & 4), 12-13 (n & 2), 14 (n & 1); n = 16
// uses all 16.  Pattern lane j of a group holds its FFT's peak q (plus the
// chunk's first peak), q = the number of pattern lanes below j; lanes
// outside the pattern take part in the steps only as rows.
__device__ __forceinline__ uint32_t chunk_pattern(int n) {
    if (n >= 16) return 0xFFFFu;
    return ((1u << (n & 8)) - 1u) | (((1u << (n & 4)) - 1u) << 8) |
           (((1u << (n & 2)) - 1u) << 12) | (((1u << (n & 1)) - 1u) << 14);
}

__device__ __forceinline__ void stripe_chunk(uint32_t m, uint32_t v, uint32_t t, uint32_t dump,
                                             uint32_t lane_off, uint32_t val,
                                             uint32_t *__restrict__ lds) {
    if (m & 0x00FFu) stripe_run<0, 8>(v, t, dump, lane_off, val, lds);
    if (m & 0x0F00u) stripe_run<8, 12>(v, t, dump, lane_off, val, lds);
    if (m & 0x3000u) stripe_run<12, 14>(v, t, dump, lane_off, val, lds);
    if (m & 0x4000u) stripe_run<14, 15>(v, t, dump, lane_off, val, lds);
    if (m & 0x8000u) stripe_run<15, 16>(v, t, dump, lane_off, val, lds);
}

// Tail rows (rows 16 .. 16 + A.tail - 1 of the tiles of the last run row
// block): every pattern lane adds its own peak's stripe start in each tail
// row, one atomic per peak and row, in the row-major tail region `lt` (row
// stride `stride` words).  Lane r of a group holds the group's tail row term
// of row 16 + r, broadcast to the group by DPP row_newbcast:r fused into the
// add; lanes outside the chunk's pattern (which may repeat a pattern lane's
// peak) and starts outside the tile go to the lane's own dump word, so that
// no two lanes of an atomic update one word.
template <int R>
__device__ __forceinline__ void tail_row(uint32_t v, uint32_t tt, uint32_t dump, uint32_t val,
                                         uint32_t *__restrict__ lt) {
    const uint32_t b = __builtin_amdgcn_update_dpp(0u, tt, 0x150 + R, 0xF, 0xF, true);
    const uint16_t col = (uint16_t)((v + b) >> kFrac);
    const uint32_t cu = col < (uint16_t)dump ? col : (uint16_t)dump;
    atomicAdd(lt + cu, val);
}

__device__ __forceinline__ void tail_steps(int rows, uint32_t m, uint32_t j, uint32_t v, uint32_t tt,
                                           uint32_t dump, uint32_t stride, uint32_t val,
                                           uint32_t *__restrict__ lt) {
    static_assert(kTailRows == 3, "tail_steps unrolls kTailRows rows");
    const uint32_t vv = (m >> j) & 1u ? v : kFarEdge;
    tail_row<0>(vv, tt, dump, val, lt);
    if (rows > 1) tail_row<1>(vv, tt, dump, val, lt + stride);
    if (rows > 2) tail_row<2>(vv, tt, dump, val, lt + 2 * stride);
}

// One block: four consecutive FFTs of a sorted run, entry 4 b + g in lane
// group g.  Lane (g, j) holds its group's window, row term and weight, and
// the stripe edges of its peaks in up to two chunks of 16.
struct Quad {
    int g, run;          // block id claimed from the tile's counter; its run g % 16
    int lo, pk;          // window start; FFT place in the run << 16 | peak count
    uint32_t gb;         // G_{i,s0} of the group's FFT i (mod 2^32)
    uint32_t t, wq;      // row term G_{i,s0} - G_{i,s0+j} (mod 2^32); fixed-point weight
    uint32_t tt;         // tail row term G_{i,s0} - G_{i,s0+16+j} (mod 2^32), tiles with tail rows
    int cnt;             // peaks in the window (0 past the tile's blocks)
    int32_t q1, q2;      // chunk positions of the lane's peaks
    uint32_t y0, y1;     // low words of their stripe edges
    uint32_t m1, m2;     // lane patterns of the two chunks
    int cmax;            // largest window of the four groups
};

__device__ __forceinline__ void decode_tile(const TileArgs &A, int t, int &slot, int &rb, int &jb) {
    jb = t % A.nbb;
    const int r = t / A.nbb;
    rb = r % A.nrb;
    slot = r / A.nrb;
}

// Persistent form.  Tile groups (sky, bin block) are dealt round-robin to
// kXcds queues (workgroups are dispatched round-robin over the XCDs, so
// workgroup w serves queue w % 8 and the tiles of one group, which read the
// same stripe edges, stay in one XCD's L2); a queue holds its groups in order,
// each with all its row blocks.  Position pos of queue qi is therefore
// group qi + 8 (pos / nrb), row block pos % nrb.
__device__ __forceinline__ int queue_len(const TileArgs &A, int qi) {
    const int groups = A.n_slots * A.nbb;
    return qi < groups ? A.nrb * ((groups - qi + kXcds - 1) / kXcds) : 0;
}

__device__ __forceinline__ int queue_tile(const TileArgs &A, int qi, int pos) {
    const int k = pos / A.nrb, rb = pos - k * A.nrb;
    const int grp = qi + kXcds * k;
    const int sl = grp / A.nbb, jb = grp - sl * A.nbb;
    return (sl * A.nrb + rb) * A.nbb + jb;
}

// A tile from the first queue, starting at `home`, that is not exhausted; -1
// when all are.
__device__ int steal_tile(const TileArgs &A, int home) {
    for (int k = 0; k < kXcds; ++k) {
        const int qi = (home + k) % kXcds;
        const int len = queue_len(A, qi);
        if (__hip_atomic_load(A.queue_ctr + qi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len)
            continue;
        const int pos = atomicAdd(A.queue_ctr + qi, 1);
        if (pos < len) return queue_tile(A, qi, pos);
    }
    return -1;
}

// LDS words of a tile: W + K_f - 1 columns plus the dump columns, 16 rows
// (column-major), then A.tail rows of W + K_f - 1 + kTailDump words
// (row-major).
__device__ __forceinline__ int tile_words(const TileArgs &A) {
    return kTileRows * (A.W + A.kf - 1 + kDumpCols) + A.tail * (A.W + A.kf - 1 + kTailDump);
}

__device__ __forceinline__ void tile_zero(const TileArgs &A, uint32_t *__restrict__ lds) {
    const int nwords = tile_words(A);
    for (int x = threadIdx.x * 4; x < nwords; x += blockDim.x * 4) {
        if (x + 3 < nwords) {
            *reinterpret_cast<uint4 *>(lds + x) = make_uint4(0, 0, 0, 0);
        } else {
            for (int y = x; y < nwords; ++y) lds[y] = 0;
        }
    }
}

// Output phase of tile (slot, rb, jb): per-row window sums of the start
// histogram, written as a map and/or reduced to per-bin column maxima.
// Column maxima: a lane group owns a segment [x0, x1) of columns.  Its first
// K_f - 1 columns are still read by the previous group's window sums, so
// their maxima are reduced across the group's 16 lanes at once (DPP); every
// later column is read by its own group only, and its window sums replace
// its start counts in place.  After a barrier one thread per such column
// reduces the 16 rows in registers and updates the global maximum.
template <bool WEIGHTED, bool MAP, bool COLMAX>
__device__ __forceinline__ void tile_output(const TileArgs &A, int slot, int rb, int jb,
                                            uint32_t *__restrict__ lds) {
    const int tid = threadIdx.x;
    const int j = tid & 15;
    const int W = A.W, kf = A.kf;
    const int s0 = rb * kTileRows;
    // Row sums: H(x) = sum_{c = x}^{x + K_f - 1} P(c), x in [0, W): the +w at
    // the stripe start and the -w K_f bins later, prefix-summed along the row.
    const int nseg = blockDim.x / kTileRows;
    const int seg = tid >> 4;
    const int len = (W + nseg - 1) / nseg;
    const int64_t bbase = (int64_t)jb * W;
    const int xend = (int)min((int64_t)W, (int64_t)A.nf - bbase);  // columns of the map
    const int x0 = seg * len;
    const int x1 = min(x0 + len, xend);
    const int xs = x0 + kf - 1;  // first column rewritten in place
    const int s = s0 + j;
    const bool row_ok = s < A.ns;
    uint32_t *__restrict__ P = lds + j;
    unsigned long long *__restrict__ cm = A.colmax + (int64_t)slot * A.nf + bbase;
    float scale = 1.0f;
    if (WEIGHTED) scale = ldexpf(1.0f, -A.ws[(int64_t)slot * A.ws_stride].frac_bits);
    uint32_t acc = 0;
    if (x0 < x1)
        for (int c = x0; c < x0 + kf - 1; ++c) acc += P[c * kTileRows];
    for (int x = x0; x < x1; ++x) {
        acc += P[(x + kf - 1) * kTileRows];
        const int64_t b = bbase + x;
        if (MAP && row_ok) {
            if (WEIGHTED) A.map_f32[(int64_t)s * A.nf + b] = (float)acc * scale;
            else A.map_i32[(int64_t)s * A.nf + b] = (int32_t)acc;
        }
        const uint32_t trail = P[x * kTileRows];
        if (COLMAX && x < xs) {
            // largest value over the 16 rows (DPP row_shr prefix max: lane 15
            // ends with it), then the smallest row holding it (prefix min)
            const uint32_t a = row_ok ? acc : 0u;
            uint32_t mx = a;
            mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x111, 0xF, 0xF, false));
            mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x112, 0xF, 0xF, false));
            mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x114, 0xF, 0xF, false));
            mx = max(mx, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x118, 0xF, 0xF, false));
            const uint32_t top = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)mx, 0x15F, 0xF, 0xF, true);
            int r = row_ok && a == top ? j : kTileRows;
            r = min(r, __builtin_amdgcn_update_dpp(r, r, 0x111, 0xF, 0xF, false));
            r = min(r, __builtin_amdgcn_update_dpp(r, r, 0x112, 0xF, 0xF, false));
            r = min(r, __builtin_amdgcn_update_dpp(r, r, 0x114, 0xF, 0xF, false));
            r = min(r, __builtin_amdgcn_update_dpp(r, r, 0x118, 0xF, 0xF, false));
            if (j == kTileRows - 1)
                atomicMax(cm + x, ((unsigned long long)top << 32) | (0xFFFFFFFFull - (unsigned)(s0 + r)));
        } else if (COLMAX) {
            P[x * kTileRows] = row_ok ? acc : 0u;
        }
        acc -= trail;
    }
    if (!COLMAX) return;
    lds_barrier();
    // columns rewritten in place: x in [x0 + K_f - 1, x1) of each segment
    for (int x = tid; x < xend; x += blockDim.x) {
        const int sx = x / len;
        if (x < sx * len + kf - 1) continue;
        const uint4 *q = reinterpret_cast<const uint4 *>(lds + x * kTileRows);
        const uint4 h0 = q[0], h1 = q[1], h2 = q[2], h3 = q[3];
        const uint32_t h[16] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w,
                                h2.x, h2.y, h2.z, h2.w, h3.x, h3.y, h3.z, h3.w};
        uint32_t top = h[0];
#pragma unroll
        for (int k = 1; k < kTileRows; ++k) top = max(top, h[k]);
        // smallest row holding the maximum (rows past the grid hold 0, and
        // row 0 always exists, so a row past the grid is never chosen)
        int r = kTileRows - 1;
#pragma unroll
        for (int k = kTileRows - 2; k >= 0; --k) r = h[k] == top ? k : r;
        atomicMax(cm + x, ((unsigned long long)top << 32) | (0xFFFFFFFFull - (unsigned)(s0 + r)));
    }
}

// Column-maximum output of tile (slot, rb, jb) that also clears the tile for
// the next one: the output of the candidate search for K_f <= kHold + 1.
// Phase 1, lane group = segment of columns, lane = row: the window sums H(x)
// along each row.  The first K_f - 1 columns of a segment are still read by
// the previous segment, so their sums wait in registers; the later ones are
// rewritten in place, eight columns per round with every LDS read of a round
// issued before the first is used.  After a barrier the held sums go back in
// place, and after another one, phase 2: one thread per column reduces its
// 16 rows, updates the global maximum and clears the column (dump columns
// and columns past the map are only cleared).  `mid` runs between the
// phases (the caller's prefetch of the next tile); the caller's barrier then
// separates the clearing from the next tile's updates.
constexpr int kHold = 9;  // held columns per lane: K_f - 1 <= kHold
constexpr int kRound = 8;  // columns per round of the first output phase

// The whole rounds of the first phase from column x of a segment ending at
// x1: window sums written in place, with no test per column; MASK writes
// zeros for a row past the grid (only the last row block has such rows).
// Returns the first column not done (fewer than kRound remain).
template <bool MASK>
__device__ __forceinline__ int colmax_rounds(uint32_t *__restrict__ P, int x, int x1, int kf,
                                             uint32_t &acc, bool row_ok) {
    for (; x + kRound <= x1; x += kRound) {
        const uint32_t *ph = P + (x + kf - 1) * kTileRows;
        uint32_t *pt = P + x * kTileRows;
        uint32_t h[kRound], t[kRound], o[kRound];
#pragma unroll
        for (int c = 0; c < kRound; ++c) {
            h[c] = ph[c * kTileRows];
            t[c] = pt[c * kTileRows];
        }
#pragma unroll
        for (int c = 0; c < kRound; ++c) {
            acc += h[c];
            o[c] = MASK && !row_ok ? 0u : acc;
            acc -= t[c];
        }
        // a round's writes follow all of its reads: column x + c is read as a
        // head by earlier rounds only, and as a trail by this round
#pragma unroll
        for (int c = 0; c < kRound; ++c) pt[c * kTileRows] = o[c];
    }
    return x;
}

template <typename Mid>
__device__ __forceinline__ void tile_colmax(const TileArgs &A, int slot, int rb, int jb,
                                            uint32_t *__restrict__ lds, Mid mid) {
    const int tid = threadIdx.x;
    const int j = tid & 15;
    const int W = A.W, kf = A.kf;
    const int s0 = rb * kTileRows;
    const int nseg = blockDim.x / kTileRows;
    const int seg = tid >> 4;
    const int len = (W + nseg - 1) / nseg;
    const int64_t bbase = (int64_t)jb * W;
    const int xend = (int)min((int64_t)W, (int64_t)A.nf - bbase);  // columns of the map
    const int x0 = seg * len;
    const int x1 = min(x0 + len, xend);
    const int nh = max(0, min(kf - 1, x1 - x0));  // held columns [x0, x0 + nh)
    const bool row_ok = s0 + j < A.ns;
    uint32_t *__restrict__ P = lds + j;
    unsigned long long *__restrict__ cm = A.colmax + (int64_t)slot * A.nf + bbase;

    // Phase 1.  Reads past a segment's end are clamped to its last column
    // (their values are not used); W is a multiple of 64, so a segment starts
    // at column 63 len <= W even past the map, and no read passes column
    // W + K_f - 1 (the first dump column).
    uint32_t acc = 0;
    if (x0 < x1)
        for (int c = x0; c < x0 + kf - 1; ++c) acc += P[c * kTileRows];
    uint32_t hold[kHold];
    {
        uint32_t h[kHold], t[kHold];
#pragma unroll
        for (int c = 0; c < kHold; ++c) {
            const int xc = x0 + min(c, max(nh - 1, 0));
            h[c] = P[(xc + kf - 1) * kTileRows];
            t[c] = P[xc * kTileRows];
        }
#pragma unroll
        for (int c = 0; c < kHold; ++c) {
            const uint32_t v = acc + h[c];
            hold[c] = row_ok ? v : 0u;
            if (c < nh) acc = v - t[c];
        }
    }
    int x = x0 + nh;
    if (s0 + kTileRows <= A.ns) x = colmax_rounds<false>(P, x, x1, kf, acc, true);
    else x = colmax_rounds<true>(P, x, x1, kf, acc, row_ok);
    if (x < x1) {  // the segment's last, partial round
        uint32_t h[kRound], t[kRound], o[kRound];
#pragma unroll
        for (int c = 0; c < kRound; ++c) {
            const int xc = min(x + c, x1 - 1);
            h[c] = P[(xc + kf - 1) * kTileRows];
            t[c] = P[xc * kTileRows];
        }
#pragma unroll
        for (int c = 0; c < kRound; ++c) {
            acc += h[c];
            o[c] = row_ok ? acc : 0u;
            acc -= t[c];
        }
#pragma unroll
        for (int c = 0; c < kRound; ++c)
            if (x + c < x1) P[(x + c) * kTileRows] = o[c];
    }
    mid();
    lds_barrier();
#pragma unroll
    for (int c = 0; c < kHold; ++c)
        if (c < nh) P[(x0 + c) * kTileRows] = hold[c];
    lds_barrier();

    // Phase 2.  Lane l reads the four 16-byte quarters of its column starting
    // at quarter (l >> 1) & 3: with columns 64 bytes apart, every eight lanes
    // then cover the 32 banks once.
    const int ncols = W + kf - 1 + kDumpCols;
    const int st = ((tid & 63) >> 1) & 3;
    int qo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) qo[k] = (k + st) & 3;
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int c = tid; c < ncols; c += blockDim.x) {
        uint4 *q = reinterpret_cast<uint4 *>(lds + c * kTileRows);
        if (c < xend) {
            uint4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = q[qo[k]];
            uint32_t top = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) top = max(max(top, max(v[k].x, v[k].y)), max(v[k].z, v[k].w));
            // smallest row holding the maximum (rows past the grid hold 0,
            // and row 0 always exists, so a row past the grid is never chosen)
            int r = kTileRows;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int rk = v[k].x == top ? 0 : v[k].y == top ? 1 : v[k].z == top ? 2 : v[k].w == top ? 3 : 4;
                r = min(r, rk < 4 ? 4 * qo[k] + rk : kTileRows);
            }
            atomicMax(cm + c, ((unsigned long long)top << 32) | (0xFFFFFFFFull - (unsigned)(s0 + r)));
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) q[qo[k]] = z;
    }
}

// Output of the tail rows of a tile (rows (rb + 1) 16 + r, r < A.tail): their
// window sums, one thread per column summing K_f start counts per row, as a
// map and/or raised into the column maxima; then, after a barrier, the tail
// region is cleared for the next tile.  Reads only the tail region, so it
// may follow either output phase of the 16 rows without a barrier between.
template <bool WEIGHTED, bool MAP, bool COLMAX>
__device__ __forceinline__ void tail_output(const TileArgs &A, int slot, int rb, int jb,
                                            uint32_t *__restrict__ lt) {
    const int W = A.W, kf = A.kf;
    const int stride = W + kf - 1 + kTailDump;
    const int s_t = (rb + 1) * kTileRows;  // first tail row
    const int64_t bbase = (int64_t)jb * W;
    const int xend = (int)min((int64_t)W, (int64_t)A.nf - bbase);
    unsigned long long *__restrict__ cm = A.colmax + (int64_t)slot * A.nf + bbase;
    float scale = 1.0f;
    if (WEIGHTED) scale = ldexpf(1.0f, -A.ws[(int64_t)slot * A.ws_stride].frac_bits);
    for (int x = threadIdx.x; x < xend; x += blockDim.x) {
        uint32_t top = 0;
        int brow = 0;
        for (int r = 0; r < A.tail; ++r) {
            const uint32_t *P = lt + r * stride + x;
            uint32_t acc = 0;
            for (int c = 0; c < kf; ++c) acc += P[c];
            if (MAP) {
                const int64_t idx = (int64_t)(s_t + r) * A.nf + bbase + x;
                if (WEIGHTED) A.map_f32[idx] = (float)acc * scale;
                else A.map_i32[idx] = (int32_t)acc;
            }
            if (acc > top) {  // the smallest row holding the maximum
                top = acc;
                brow = r;
            }
        }
        if (COLMAX) atomicMax(cm + x, ((unsigned long long)top << 32) | (0xFFFFFFFFull - (unsigned)(s_t + brow)));
    }
    lds_barrier();
    const int nwords = A.tail * stride;
    for (int x = threadIdx.x; x < nwords; x += blockDim.x) lt[x] = 0;
}

// The tiles of one workgroup.  The waves take the tile's blocks (four FFTs
// of a sorted run, one per lane group; windows past the last FFT are empty)
// from a counter in LDS, so that each wave takes as many as it can process.
// A block's window data are loaded two blocks ahead and its stripe edges one
// block ahead (a ring of three blocks), so that the accumulation of a block
// never waits for memory; the first two blocks of the next tile are loaded
// during the output phase of the current one.  Every load is issued on every
// path so that the wait counts stay exact.  PERSISTENT: tiles come from the
// XCD queues until all are exhausted; otherwise the workgroup runs tile
// tile_base + blockIdx.x only.
template <bool WEIGHTED, bool MAP, bool COLMAX, bool PERSISTENT, bool TAIL>
__device__ __forceinline__ void run_tiles(const TileArgs &A, uint32_t *__restrict__ lds, int *s_next,
                                          int *s_cnt) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int j = lane & 15;
    const int grp = lane >> 4;
    const int W = A.W, kf = A.kf;
    const int wc = W + kf - 1;
    // LDS column c holds fine bin c0 + c, c in [0, wc); columns wc + g are
    // the dumps of the four lane groups.
    const uint32_t dump = (uint32_t)(wc + grp);
    const uint32_t lane_off = (uint32_t)j;
    const uint32_t below = (1u << j) - 1u;           // pattern lanes below j
    const uint32_t mtab = chunk_pattern(lane);       // lane n holds m(n), n <= 16
    const int32_t n_pad = win_stride(A.n_fft);
    const int per = wave_ffts(A.n_fft);
    const int nblk = per >> 2;
    const int total = kTileWaves * nblk;  // blocks of a tile
    const int i_last = A.n_fft - 1;
    const int home = blockIdx.x % kXcds;
    const __amdgpu_buffer_rsrc_t r_rec = buf(A.rec), r_step = buf(A.step);
    const uint32_t lane_code = 2u * (uint32_t)j;  // bit offset of this row's residual code
    // tail rows after the 16-row tile (row-major, rows of wc + kTailDump
    // words; every lane of a wave has its own dump word in each row)
    const uint32_t t_stride = (uint32_t)(wc + kTailDump);
    const uint32_t t_dump = (uint32_t)(wc + lane);
    uint32_t *__restrict__ const ltail = lds + kTileRows * (wc + kDumpCols);

    // per-tile buffers: window row, stripe edges and weights of the slot
    struct Bufs {
        __amdgpu_buffer_rsrc_t win, y, wq;
        uint32_t rb;  // row block of the tile
    };
    auto tile_bufs = [&](int t) {
        int slot, rb, jb;
        decode_tile(A, t, slot, rb, jb);
        const int g = rb / kRowBlocksPerGroup;
        Bufs b;
        b.win = buf(A.win + (((int64_t)slot * A.nrbg + g) * A.nbb + jb) * n_pad);
        // low 32 bits of the stripe edges (all the tile needs: see stripe_word)
        b.y = buf(A.Y + (int64_t)slot * y_stride(A.n_peaks, A.n_fft));
        b.wq = buf(WEIGHTED ? (const void *)(A.wq + (int64_t)slot * A.n_fft) : (const void *)A.step);
        b.rb = (uint32_t)rb;
        return b;
    };
    // Blocks are handed out dynamically: block g of a tile is block g / 16 of
    // run g % 16 (four consecutive entries of that run), so the counter walks
    // the runs' largest windows first, and a wave that the SIMD arbiter
    // serves less simply takes fewer blocks.  `claim` takes n blocks and
    // returns the first in lane 0; it is read (and waited for) only when the
    // blocks are staged.
    auto claim = [&](int par, int n) {
        int g = 0;
        if (lane == 0) g = atomicAdd(s_cnt + par, n);
        return g;
    };
    // window data of block g (stage 1).  Blocks past the last one (claims
    // after the counter ran out) read the row's last entry, an empty window.
    auto stage_w = [&](Quad &Q, int gv, const Bufs &B) {
        Q.g = __builtin_amdgcn_readfirstlane(gv);
        Q.run = Q.g & (kTileWaves - 1);
        const uint32_t e = (uint32_t)(Q.run * per + 4 * (Q.g >> 4) + grp);
        const auto w2 = __builtin_amdgcn_raw_buffer_load_b64(
            B.win, (Q.g < total ? e : (uint32_t)(n_pad - 1)) * 8u, 0, 0);
        Q.lo = (int)w2[0];
        Q.pk = (int)w2[1];
    };
    // stripe edges, row terms and weights of block bb (stage 2): the chunk
    // sizes follow the largest window of the four groups, group 0's (the runs
    // are sorted by window size, exactly).  The row term of row s0 + j,
    // G_{i,s0} - G_{i,s0+j} = 1 - step[i][j] - code_j (mod 2^32), comes from the
    // FFT's step table and the row block's record (the host keeps N nrb below
    // 2^28, so the byte offsets fit 31 bits).
    auto stage_y = [&](Quad &Q, const Bufs &B) {
        Q.cnt = Q.pk & 0xFFFF;
        const uint32_t fc = min((uint32_t)((Q.pk >> 16) * kTileWaves + Q.run), (uint32_t)i_last);
        const auto r = __builtin_amdgcn_raw_buffer_load_b64(r_rec, (B.rb * (uint32_t)A.n_fft + fc) * 8u, 0, 0);
        Q.gb = (uint32_t)r[0];
        const uint32_t code = __builtin_amdgcn_ubfe((uint32_t)r[1], lane_code, 2u);
        Q.t = (1u - ld_u32(r_step, (fc * kTileRows + (uint32_t)j) * 4u)) - code;
        // tiles with tail rows: G_{i,s0} - G_{i,s0+16+j} from the next row
        // block's record, whose rows share this block's linear steps (other
        // row blocks read their own record and leave the term unused; no
        // branch, so that nothing here waits for the loads)
        Q.tt = 0u;
        if (TAIL) {
            const uint32_t rb2 = B.rb + (B.rb == (uint32_t)(A.nrb - 1) ? 1u : 0u);
            const auto r2 = __builtin_amdgcn_raw_buffer_load_b64(r_rec, (rb2 * (uint32_t)A.n_fft + fc) * 8u, 0, 0);
            const uint32_t code2 = __builtin_amdgcn_ubfe((uint32_t)r2[1], lane_code, 2u);
            Q.tt = Q.t + code - code2 + (Q.gb - (uint32_t)r2[0]);
        }
        Q.wq = WEIGHTED ? ld_u32(B.wq, fc * 4u) : 1u;
        Q.cmax = __builtin_amdgcn_readlane(Q.cnt, 0);
        const int n1 = min(Q.cmax, 16);
        const int n2 = min(max(Q.cmax - 16, 0), 16);
        Q.m1 = __builtin_amdgcn_readlane(mtab, n1);
        Q.m2 = __builtin_amdgcn_readlane(mtab, n2);
        Q.q1 = (int32_t)__builtin_popcount(Q.m1 & below);
        Q.q2 = 16 + (int32_t)__builtin_popcount(Q.m2 & below);
        Q.y0 = ld_u32(B.y, (uint32_t)(Q.lo + Q.q1) * 4u);
        Q.y1 = ld_u32(B.y, (uint32_t)(Q.lo + Q.q2) * 4u);
    };

    int t;
    if (PERSISTENT) {
        if (tid == 0) s_next[0] = steal_tile(A, home);
    }
    if (tid < 2) s_cnt[tid] = 0;
    tile_zero(A, lds);
    lds_barrier();
    t = PERSISTENT ? s_next[0] : A.tile_base + (int)blockIdx.x;
    if (t < 0 || nblk == 0) return;  // nblk > 0 whenever there is an FFT
    Quad qa, qb, qc;
    Bufs cur = tile_bufs(t);
    stage_w(qa, claim(0, 1), cur);
    stage_w(qb, claim(0, 1), cur);
    stage_y(qa, cur);
    for (int it = 0;; ++it) {
        const int par = it & 1;  // block counter of this tile; the other is the next tile's
        int pos = 0;
        if (PERSISTENT && tid == 0) pos = atomicAdd(A.queue_ctr + home, 1);
        // the next tile's counter was last used by the previous tile, whose
        // claims all came before the barrier that ended its accumulation
        if (tid == 0) s_cnt[par ^ 1] = 0;
        int slot, rb, jb;
        decode_tile(A, t, slot, rb, jb);
        const uint32_t c0q = (uint32_t)(jb * W - (kf - 1)) << kFrac;
        const bool tailed = TAIL && rb == A.nrb - 1;  // this tile also does the tail rows
        auto consume = [&](const Quad &Q) {
            const uint32_t base = c0q + Q.gb;
            uint32_t val = Q.wq;
            asm volatile("" : "+v"(val));
            const uint32_t v0 = Q.q1 < Q.cnt ? Q.y0 - base : kFarEdge;
            stripe_chunk(Q.m1, v0, Q.t, dump, lane_off, val, lds);
            if (tailed) tail_steps(A.tail, Q.m1, lane_off, v0, Q.tt, t_dump, t_stride, val, ltail);
            if (Q.cmax > 16) {
                const uint32_t v1 = Q.q2 < Q.cnt ? Q.y1 - base : kFarEdge;
                stripe_chunk(Q.m2, v1, Q.t, dump, lane_off, val, lds);
                if (tailed) tail_steps(A.tail, Q.m2, lane_off, v1, Q.tt, t_dump, t_stride, val, ltail);
            }
            // windows longer than 32 peaks: further chunks, loaded here
            for (int off = 32; off < Q.cmax; off += 16) {
                const uint32_t m = __builtin_amdgcn_readlane(mtab, min(Q.cmax - off, 16));
                const int32_t q = off + (int32_t)__builtin_popcount(m & below);
                uint32_t v = kFarEdge;
                if (q < Q.cnt) v = ld_u32(cur.y, (uint32_t)(Q.lo + q) * 4u) - base;
                stripe_chunk(m, v, Q.t, dump, lane_off, val, lds);
                if (tailed) tail_steps(A.tail, m, lane_off, v, Q.tt, t_dump, t_stride, val, ltail);
            }
        };
        // Ring of three blocks: a block's window is loaded two blocks ahead,
        // its stripe edges one block ahead.  Blocks are claimed three at a
        // time, one round ahead, so a wave drains its LDS queue to read a
        // claim once per three blocks.  A wave's claims grow, so once one
        // block is past the end, so are the blocks staged after it.
        int gv = claim(par, 3);
        for (;;) {
            const int g3 = __builtin_amdgcn_readfirstlane(gv);
            gv = claim(par, 3);
            stage_w(qc, g3, cur);
            stage_y(qb, cur);
            if (qa.g >= total) break;
            consume(qa);
            stage_w(qa, g3 + 1, cur);
            stage_y(qc, cur);
            if (qb.g >= total) break;
            consume(qb);
            stage_w(qb, g3 + 2, cur);
            stage_y(qa, cur);
            if (qc.g >= total) break;
            consume(qc);
        }
        int tn = -1;
        if (PERSISTENT) {
            if (tid == 0)
                s_next[(it + 1) & 1] = pos < queue_len(A, home) ? queue_tile(A, home, pos) : steal_tile(A, home);
        }
        // Drain this wave's vector-memory queue here, where the workgroup
        // waits anyway: otherwise the compiler cannot tell that the tile
        // claim above has returned on every path, and the output phase would
        // open with a full wait that also covers the next tile's prefetch.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        lds_barrier();
        if (PERSISTENT) tn = s_next[(it + 1) & 1];
        Bufs nxt = cur;
        if (tn >= 0) {
            nxt = tile_bufs(tn);
            stage_w(qa, claim(par ^ 1, 1), nxt);
            stage_w(qb, claim(par ^ 1, 1), nxt);
        }
        // candidate search: clearing fused into the output, and the next
        // tile's stripe edges requested while the output still runs
        const bool fused = COLMAX && !MAP && kf <= kHold + 1;
        if (fused) {
            tile_colmax(A, slot, rb, jb, lds, [&] {
                if (tn >= 0) stage_y(qa, nxt);
            });
        } else {
            tile_output<WEIGHTED, MAP, COLMAX>(A, slot, rb, jb, lds);
        }
        if (TAIL && tailed) tail_output<WEIGHTED, MAP, COLMAX>(A, slot, rb, jb, ltail);
        if (tn < 0) break;
        if (!fused) stage_y(qa, nxt);
        lds_barrier();
        if (!fused) {
            tile_zero(A, lds);
            lds_barrier();
        }
        cur = nxt;
        t = tn;
    }
}

template <bool WEIGHTED, bool MAP, bool COLMAX, bool TAIL>
__global__ void __launch_bounds__(kTileThreads) k_tiles_plain(TileArgs A) {
    extern __shared__ uint32_t lds[];
    __shared__ int s_cnt[2];
    run_tiles<WEIGHTED, MAP, COLMAX, false, TAIL>(A, lds, nullptr, s_cnt);
}

// One workgroup per CU.  The next tile of the home queue is claimed when a
// tile starts (its counter update overlaps the tile's work) and used when it
// ends; an exhausted home queue sends the workgroup to the others.  Every
// workgroup leaves the loop once all queues are exhausted.
template <bool WEIGHTED, bool MAP, bool COLMAX, bool TAIL>
__global__ void __launch_bounds__(kTileThreads) k_tiles_persistent(TileArgs A) {
    extern __shared__ uint32_t lds[];
    __shared__ int s_next[2];
    __shared__ int s_cnt[2];
    run_tiles<WEIGHTED, MAP, COLMAX, true, TAIL>(A, lds, s_next, s_cnt);
}

// ----------------------------------------------------------------------------
// candidates per (sky, sub-band)

struct Best {
    uint32_t val;
    int32_t bin;
    int32_t row;
};

__device__ __forceinline__ bool better(const Best &a, const Best &b) {
    if (a.val != b.val) return a.val > b.val;
    if (a.bin != b.bin) return a.bin < b.bin;
    return a.row < b.row;
}

__device__ Best block_best(Best m, Best *red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        Best o2;
        o2.val = __shfl_xor(m.val, o);
        o2.bin = __shfl_xor(m.bin, o);
        o2.row = __shfl_xor(m.row, o);
        if (better(o2, m)) m = o2;
    }
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = m;
    __syncthreads();
    Best r = red[0];
    for (int k = 1; k < nw; ++k)
        if (better(red[k], r)) r = red[k];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) k_select(const unsigned long long *__restrict__ colmax,
                                                int32_t nf, fh_select sel, int32_t sky_base,
                                                int32_t n_fft, const WeightStats *__restrict__ ws,
                                                int32_t ws_stride, fh_candidate *__restrict__ out) {
    __shared__ Best red[16];
    const int sb = blockIdx.x, slot = blockIdx.y;
    const int n_sb = gridDim.x;
    const int lo = sb * sel.width;
    const int hi = lo + sel.width < nf ? lo + sel.width : nf;
    const unsigned long long *cm = colmax + (int64_t)slot * nf;
    const Best none = {0u, 0x7fffffff, 0x7fffffff};
    Best m = none;
    bool any = false;
    for (int b = lo + threadIdx.x; b < hi; b += blockDim.x) {
        const unsigned long long k = cm[b];
        Best c = {(uint32_t)(k >> 32), b, (int32_t)(0xFFFFFFFFu - (uint32_t)k)};
        if (!any || better(c, m)) { m = c; any = true; }
    }
    const Best b1 = block_best(m, red);
    m = none;
    any = false;
    if (sel.sep >= 0) {
        for (int b = lo + threadIdx.x; b < hi; b += blockDim.x) {
            const int d = b > b1.bin ? b - b1.bin : b1.bin - b;
            if (d <= sel.excl) continue;
            const unsigned long long k = cm[b];
            Best c = {(uint32_t)(k >> 32), b, (int32_t)(0xFFFFFFFFu - (uint32_t)k)};
            if (!any || better(c, m)) { m = c; any = true; }
        }
    }
    const Best b2 = block_best(m, red);
    if (threadIdx.x == 0) {
        const double th = sel.theta;
        const double p0 = exp(-th) - exp(-2.0 * th) + exp(-3.0 * th) / 3.0;
        double scale = 1.0, mu, sd;
        if (ws != nullptr) {
            const WeightStats st = ws[(int64_t)slot * ws_stride];
            scale = ldexp(1.0, -st.frac_bits);
            mu = p0 * st.sum_w;
            sd = sqrt(p0 * (1.0 - p0) * st.sum_w2);
        } else {
            mu = (double)n_fft * p0;
            sd = sqrt((double)n_fft * p0 * (1.0 - p0));
        }
        fh_candidate *o = out + ((int64_t)(sky_base + slot) * n_sb + sb) * 2;
        const Best bs[2] = {b1, b2};
        for (int r = 0; r < 2; ++r) {
            fh_candidate c;
            c.sky = sky_base + slot;
            c.subband = sb;
            c.rank = r;
            bool valid = bs[r].bin != 0x7fffffff && hi > lo;
            if (r == 1) {
                const int d = bs[1].bin > b1.bin ? bs[1].bin - b1.bin : b1.bin - bs[1].bin;
                valid = valid && sel.sep >= 0 && d >= sel.sep;
            }
            c.valid = valid ? 1 : 0;
            if (valid) {
                const double value = ws != nullptr ? (double)(float)((float)bs[r].val * (float)scale)
                                                   : (double)bs[r].val;
                c.bin = bs[r].bin;
                c.row = bs[r].row;
                c.value = (float)value;
                c.cr = (float)((value - mu) / sd);
            } else {
                c.bin = -1;
                c.row = -1;
                c.value = 0.0f;
                c.cr = 0.0f;
            }
            o[r] = c;
        }
    }
}

// ----------------------------------------------------------------------------
// peakmap construction (Sec. "Peakmap", Eq. pm): R = S_P / S_AR bin by bin; a
// peak is a bin above theta that is strictly larger than both neighbours.
// One workgroup per FFT writes its peaks compactly into a per-FFT scratch run
// (at most one peak in every two bins) and its count; after a scan of the
// counts a second kernel packs the runs into the CSR.

__global__ void __launch_bounds__(256) k_pm_rows(int32_t n_bins, int64_t ld,
                                                 const float *__restrict__ sp,
                                                 const float *__restrict__ sar, int32_t k0,
                                                 float theta, int32_t cap,
                                                 int32_t *__restrict__ scratch,
                                                 int32_t *__restrict__ counts) {
    __shared__ int wsum[4];
    const int i = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float *P = sp + (int64_t)i * ld;
    const float *A = sar ? sar + (int64_t)i * ld : nullptr;
    int32_t *out = scratch + (int64_t)i * cap;
    int base = 0;
    for (int j0 = 1; j0 < n_bins - 1; j0 += blockDim.x) {
        const int j = j0 + threadIdx.x;
        bool pk = false;
        if (j < n_bins - 1) {
            float l = P[j - 1], c = P[j], r = P[j + 1];
            if (A) {
                l = l / A[j - 1];
                c = c / A[j];
                r = r / A[j + 1];
            }
            pk = c > theta && c > l && c > r;
        }
        const uint64_t m = __ballot(pk);
        if (lane == 0) wsum[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < 4; ++w) {
            before += w < wave ? wsum[w] : 0;
            total += wsum[w];
        }
        if (pk) {
            const int pos = base + before + __popcll(m & ((1ull << lane) - 1ull));
            out[pos] = k0 + j;
        }
        base += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[i] = base;
}

// exclusive scan of per-FFT counts into CSR offsets (one workgroup)
__global__ void __launch_bounds__(1024) k_pm_scan(int32_t n, const int32_t *__restrict__ counts,
                                                  int64_t *__restrict__ offsets) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b = 0; b < n; b += blockDim.x) {
        const int i = b + threadIdx.x;
        const int64_t v = i < n ? counts[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < (int)blockDim.x; o <<= 1) {
            const int64_t add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n) offsets[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += part[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[n] = carry;
}

__global__ void __launch_bounds__(256) k_pm_pack(int32_t cap, const int32_t *__restrict__ scratch,
                                                 const int64_t *__restrict__ offsets,
                                                 int32_t *__restrict__ bins) {
    const int i = blockIdx.x;
    const int64_t o = offsets[i];
    const int c = (int)(offsets[i + 1] - o);
    const int32_t *src = scratch + (int64_t)i * cap;
    for (int t = threadIdx.x; t < c; t += blockDim.x) bins[o + t] = src[t];
}

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 16) g = 65535 * 16;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int tile_lds_bytes(int W, int kf, int tail) {
    return (kTileRows * (W + kf - 1 + kDumpCols) + tail * (W + kf - 1 + kTailDump)) * 4;
}

int max_tile_bins(int kf, double step_bins, int rows) {
    // rows past 16 are tail rows, with kTailDump dump words each
    const int words = (kLdsBytes - kLdsReserve) / 4 - kDumpCols * kTileRows - kTailDump * (rows - kTileRows);
    int w = words / rows - kf + 1;  // rows (W + kf - 1) + dump words <= words
    // supported row steps: below 128 fine bins
    if (step_bins * kQd + 1.0 >= 8388608.0) return 0;
    // 32-bit tile-relative edges (see kFarEdge)
    const double m = ceil(step_bins) + 1.0;
    const double wr = (double)(1 << (31 - kFrac)) - 64.0 - kf - 80.0 * m;
    if (wr < (double)w) w = wr < 0.0 ? 0 : (int)wr;
    return (w / 64) * 64;
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_set_f64x3(double *p, double x, double y, double z, hipStream_t st) {
    k_set_f64x3<<<1, 64, 0, st>>>(p, x, y, z);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_shift_tables(int32_t n_fft, int32_t nrb, int32_t nrb_run, int32_t ns, const double *t, double t0,
                               double t_fft,
                               int32_t kf, double fdot0, double dfdot, int64_t *gwin, uint2 *rec, uint32_t *step,
                               int32_t *err, hipStream_t st) {
    const int64_t n = (int64_t)n_fft * nrb;
    if (n <= 0) return hipSuccess;
    if (nrb_run < 1 || nrb_run > nrb) return hipErrorInvalidValue;
    const double S = ((double)kf * t_fft) * kQd;
    k_shift_tables<<<grid_for(n, 256), 256, 0, st>>>(n_fft, nrb, nrb_run, ns, t, t0, S, fdot0, dfdot, gwin, rec,
                                                     step, err);
    return hipGetLastError();
}

hipError_t launch_weight_stats(int32_t n_fft, int32_t n_vec, const float *w, int32_t w_stride,
                               int32_t mult, WeightStats *ws, int32_t *err_flag, hipStream_t st) {
    k_weight_stats<<<n_vec, 256, 0, st>>>(n_fft, w, w_stride, mult, ws, err_flag);
    return hipGetLastError();
}

hipError_t launch_prep(int32_t n_fft, int64_t n_peaks, const int64_t *offsets, const int32_t *bins,
                       const double *v, const double *sky, int32_t n_slots, int32_t kf, int64_t b0,
                       int64_t *Y, const float *w, int32_t w_stride,
                       const WeightStats *ws, int32_t ws_stride, uint32_t *wq, uint32_t *Y32,
                       int32_t shift_mode, double q, hipStream_t st) {
    dim3 grid((n_fft + 3) / 4, n_slots);
    k_prep<<<grid, 256, 0, st>>>(n_fft, n_peaks, offsets, bins, v, sky, kf, b0, Y, w, w_stride,
                                 ws, ws_stride, wq, Y32, shift_mode, q);
    return hipGetLastError();
}

int front_ffts_per_block(int32_t max_per_fft) {
    for (int F = max_per_fft >= kFrontBigFft ? 4 : kFrontMaxF; F >= 1; F >>= 1)
        if ((int64_t)F * (max_per_fft + kYPad) * 8 <= kFrontLdsBytes) return F;
    return 0;
}

hipError_t launch_front(int32_t n_fft, int64_t n_peaks, const int64_t *offsets, const int32_t *bins,
                        const double *v, const double *sky, int32_t n_slots, int32_t kf, int64_t b0,
                        const int64_t *gwin, uint32_t *Y, const float *w,
                        int32_t w_stride, const WeightStats *ws, int32_t ws_stride, uint32_t *wq,
                        int32_t ns, int32_t nrbg, int32_t nbb, int32_t W, int32_t F, int32_t max_per_fft,
                        int2 *win, int32_t shift_mode, double q, hipStream_t st) {
    if (F < 1 || win_stride(n_fft) % F != 0) return hipErrorInvalidValue;
    dim3 grid(win_stride(n_fft) / F, n_slots);
    const size_t lds = ((size_t)F * (max_per_fft + kYPad) * 8 + 255) / 256 * 256;
    if (F > kFrontMaxF || lds > (size_t)kFrontLdsBytes) return hipErrorInvalidValue;
    int32_t top = 0;  // largest power of two up to max_per_fft (0 when no FFT has a peak)
    while (top * 2 <= max_per_fft && top < (1 << 30)) top = top ? 2 * top : 1;
    k_front<<<grid, 256, lds, st>>>(n_fft, n_peaks, offsets, bins, v, sky, kf, b0, gwin, Y,
                                               w, w_stride, ws, ws_stride, wq, ns, nrbg, nbb, W, F, top, win,
                                               shift_mode, q);
    return hipGetLastError();
}

hipError_t launch_sort_windows(int32_t n_fft, int32_t nrbg, int32_t nbb, int32_t n_slots, const int2 *win,
                               int2 *wsorted, hipStream_t st) {
    dim3 grid(nrbg * nbb, n_slots);
    const size_t row_bytes = (size_t)win_stride(n_fft) * sizeof(int2);
    if (row_bytes <= (size_t)kSortStageBytes)
        k_sort_windows<<<grid, kTileThreads, row_bytes, st>>>(n_fft, nrbg * nbb, win, wsorted);
    else
        k_sort_windows_long<<<grid, kTileThreads, (size_t)kSortStageEntries * sizeof(int2), st>>>(
            n_fft, nrbg * nbb, win, wsorted);
    return hipGetLastError();
}

hipError_t launch_windows(int32_t n_fft, const int64_t *offsets, const int64_t *Y, int64_t n_peaks,
                          const int64_t *gwin, int32_t nrbg, int32_t nbb, int32_t W,
                          int32_t kf, int32_t n_slots, int2 *win, int method, hipStream_t st) {
    if (method == 0) {
        dim3 grid(grid_for((int64_t)nbb * win_stride(n_fft), 256), nrbg, n_slots);
        k_windows<<<grid, 256, 0, st>>>(n_fft, offsets, Y, n_peaks, gwin, nrbg, nbb, W, kf, win);
    } else {
        dim3 grid((win_stride(n_fft) + 3) / 4, n_slots);
        k_windows_sweep<<<grid, 256, 0, st>>>(n_fft, offsets, Y, n_peaks, gwin, nrbg, nbb, W, kf, win);
    }
    return hipGetLastError();
}

template <bool Wt, bool M, bool C, bool T>
static hipError_t set_tile_attrs_t() {
    const int lds = kLdsBytes - kLdsReserve;
    hipError_t e = hipFuncSetAttribute((const void *)k_tiles_persistent<Wt, M, C, T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_tiles_plain<Wt, M, C, T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

template <bool Wt, bool M, bool C>
static hipError_t set_tile_attrs() {
    const hipError_t e = set_tile_attrs_t<Wt, M, C, false>();
    return e != hipSuccess ? e : set_tile_attrs_t<Wt, M, C, true>();
}

// Tiles with tail rows run the TAIL form of the kernels; without, the plain
// form has no trace of them.
template <bool Wt, bool M, bool C>
static hipError_t launch_tiles_t(const TileArgs &a, bool persistent, int32_t n_tiles,
                                 int32_t grid_blocks, hipStream_t st) {
    if (a.tail < 0 || a.tail > kTailRows) return hipErrorInvalidValue;
    const int lds = tile_lds_bytes(a.W, a.kf, a.tail);
    if (lds > kLdsBytes - kLdsReserve) return hipErrorInvalidValue;
    if (a.tail > 0) {
        if (persistent)
            k_tiles_persistent<Wt, M, C, true><<<grid_blocks, kTileThreads, lds, st>>>(a);
        else
            k_tiles_plain<Wt, M, C, true><<<n_tiles, kTileThreads, lds, st>>>(a);
    } else {
        if (persistent)
            k_tiles_persistent<Wt, M, C, false><<<grid_blocks, kTileThreads, lds, st>>>(a);
        else
            k_tiles_plain<Wt, M, C, false><<<n_tiles, kTileThreads, lds, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t init_kernel_attributes() {
    hipError_t e;
    if ((e = set_tile_attrs<true, true, true>()) != hipSuccess) return e;
    if ((e = set_tile_attrs<true, true, false>()) != hipSuccess) return e;
    if ((e = set_tile_attrs<true, false, true>()) != hipSuccess) return e;
    if ((e = set_tile_attrs<false, true, true>()) != hipSuccess) return e;
    if ((e = set_tile_attrs<false, true, false>()) != hipSuccess) return e;
    if ((e = set_tile_attrs<false, false, true>()) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_sort_windows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kSortStageBytes)) != hipSuccess)
        return e;
    return hipFuncSetAttribute((const void *)k_sort_windows_long, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kSortStageEntries * (int)sizeof(int2));
}

hipError_t launch_tiles(const TileArgs &a, bool weighted, bool want_map, bool want_colmax,
                        bool persistent, int32_t n_tiles, int32_t grid_blocks, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    if (weighted) {
        if (want_map && want_colmax) return launch_tiles_t<true, true, true>(a, persistent, n_tiles, grid_blocks, st);
        if (want_map) return launch_tiles_t<true, true, false>(a, persistent, n_tiles, grid_blocks, st);
        return launch_tiles_t<true, false, true>(a, persistent, n_tiles, grid_blocks, st);
    }
    if (want_map && want_colmax) return launch_tiles_t<false, true, true>(a, persistent, n_tiles, grid_blocks, st);
    if (want_map) return launch_tiles_t<false, true, false>(a, persistent, n_tiles, grid_blocks, st);
    return launch_tiles_t<false, false, true>(a, persistent, n_tiles, grid_blocks, st);
}

hipError_t launch_select(const unsigned long long *colmax, int32_t nf, int32_t n_slots,
                         const fh_select &sel, int32_t sky_base, int32_t n_fft,
                         const WeightStats *ws, int32_t ws_stride, fh_candidate *out,
                         hipStream_t st) {
    const int n_sb = (nf + sel.width - 1) / sel.width;
    dim3 grid(n_sb, n_slots);
    k_select<<<grid, 256, 0, st>>>(colmax, nf, sel, sky_base, n_fft, ws, ws_stride, out);
    return hipGetLastError();
}

hipError_t launch_pm_rows(int32_t n_fft, int32_t n_bins, int64_t ld, const float *sp, const float *sar,
                          int32_t k0, float theta, int32_t cap, int32_t *scratch, int32_t *counts,
                          hipStream_t st) {
    k_pm_rows<<<n_fft, 256, 0, st>>>(n_bins, ld, sp, sar, k0, theta, cap, scratch, counts);
    return hipGetLastError();
}

namespace {

// ----------------------------------------------------------------------------
// peakmap slice: the peaks of each FFT with natural bin in [k_lo, k_hi)

__global__ void k_slice_count(int32_t n_fft, const int64_t *__restrict__ offsets,
                              const int32_t *__restrict__ bins, int32_t k_lo, int32_t k_hi,
                              int64_t *__restrict__ first, int32_t *__restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_fft) return;
    const int64_t p0 = offsets[i], p1 = offsets[i + 1];
    int64_t a = p0, b = p1;
    while (a < b) {  // first bin >= k_lo
        const int64_t m = (a + b) >> 1;
        if (bins[m] >= k_lo) b = m; else a = m + 1;
    }
    const int64_t lo = a;
    b = p1;
    while (a < b) {  // first bin >= k_hi
        const int64_t m = (a + b) >> 1;
        if (bins[m] >= k_hi) b = m; else a = m + 1;
    }
    first[i] = lo;
    counts[i] = (int32_t)(a - lo);
}

__global__ void k_slice_pack(const int64_t *__restrict__ first, const int32_t *__restrict__ counts,
                             const int64_t *__restrict__ offsets, const int32_t *__restrict__ bins,
                             int32_t *__restrict__ out) {
    const int i = blockIdx.x;
    const int64_t src = first[i], dst = offsets[i];
    for (int k = threadIdx.x; k < counts[i]; k += blockDim.x) out[dst + k] = bins[src + k];
}

// ----------------------------------------------------------------------------
// refined candidates: the best of the k_sky^2 directions' first candidates

__global__ void k_refine_pick(int32_t n_cand, int32_t n_dir, const fh_candidate *__restrict__ cands,
                              const double *__restrict__ params, const double *__restrict__ lamb,
                              fh_refined *__restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cand) return;
    const fh_candidate *cc = cands + (int64_t)c * n_dir * 2;
    int best = -1;
    for (int s = 0; s < n_dir; ++s) {
        const fh_candidate &x = cc[2 * s];
        if (!x.valid) continue;
        if (best < 0 || x.value > cc[2 * best].value) best = s;
    }
    fh_refined r{};
    r.cand = c;
    if (best >= 0) {
        const fh_candidate &x = cc[2 * best];
        const double *pr = params + 4 * (int64_t)c;  // f0 of bin 0, bin width, fdot of row 0, row step
        r.sky = best;
        r.bin = x.bin;
        r.row = x.row;
        r.value = x.value;
        r.cr = x.cr;
        r.valid = 1;
        r.f0 = pr[0] + x.bin * pr[1];
        r.fdot = pr[2] + x.row * pr[3];
        r.lambda = lamb[2 * ((int64_t)c * n_dir + best)];
        r.beta = lamb[2 * ((int64_t)c * n_dir + best) + 1];
    } else {
        r.sky = r.bin = r.row = -1;
    }
    out[c] = r;
}

// ----------------------------------------------------------------------------
// peakmap cleaning

// Filters on the peaks of a peakmap: mode 0 drops the peaks of gross cells
// holding more than thr peaks; mode 1 drops the peaks of natural bins k in
// [k_lo, k_hi) whose statistic x[step (k - k_lo) + offset] exceeds thr.
struct PeakFilter {
    int mode;
    // mode 0
    const double *t;
    double t_origin, dt_h, B;  // B = df_h T_FFT
    int64_t c0;
    int32_t n_t, n_f;
    const int32_t *hist;
    // mode 1
    int32_t k_lo, k_hi, step;
    int64_t offset, n_x;
    const int32_t *x;
    double thr;
};

__device__ __forceinline__ int gross_time_cell(const PeakFilter &f, int i) {
    return (int)floor((f.t[i] - f.t_origin) / f.dt_h);
}

// frequency cell of natural bin k, -1 when outside [0, n_f)
__device__ __forceinline__ int64_t gross_freq_cell(const PeakFilter &f, int32_t k) {
    const int64_t c = (int64_t)floor((double)k / f.B) - f.c0;
    return c >= 0 && c < f.n_f ? c : -1;
}

__device__ __forceinline__ bool filter_drop(const PeakFilter &f, int ct, int32_t k) {
    if (f.mode == 0) {
        if (ct < 0 || ct >= f.n_t) return false;
        const int64_t cf = gross_freq_cell(f, k);
        return cf >= 0 && (double)f.hist[(int64_t)ct * f.n_f + cf] > f.thr;
    }
    if (k < f.k_lo || k >= f.k_hi) return false;
    const int64_t idx = (int64_t)f.step * (k - f.k_lo) + f.offset;
    return idx >= 0 && idx < f.n_x && (double)f.x[idx] > f.thr;
}

// one wave per FFT: cells of its peaks counted into the gross histogram
__global__ void __launch_bounds__(256) k_gross_hist(int32_t n_fft, const int64_t *__restrict__ offsets,
                                                    const int32_t *__restrict__ bins, PeakFilter f,
                                                    int32_t *__restrict__ hist) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n_fft) return;
    const int ct = gross_time_cell(f, i);
    if (ct < 0 || ct >= f.n_t) return;
    for (int64_t p = offsets[i] + lane; p < offsets[i + 1]; p += 64) {
        const int64_t cf = gross_freq_cell(f, bins[p]);
        if (cf >= 0) atomicAdd(hist + (int64_t)ct * f.n_f + cf, 1);
    }
}

// one wave per FFT: surviving peaks counted
__global__ void __launch_bounds__(256) k_filter_count(int32_t n_fft, const int64_t *__restrict__ offsets,
                                                      const int32_t *__restrict__ bins, PeakFilter f,
                                                      int32_t *__restrict__ counts) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n_fft) return;
    const int ct = f.mode == 0 ? gross_time_cell(f, i) : 0;
    int kept = 0;
    for (int64_t p = offsets[i] + lane; p < offsets[i + 1]; p += 64) kept += filter_drop(f, ct, bins[p]) ? 0 : 1;
    for (int o = 32; o >= 1; o >>= 1) kept += __shfl_xor(kept, o);
    if (lane == 0) counts[i] = kept;
}

// one wave per FFT: surviving peaks packed in order
__global__ void __launch_bounds__(256) k_filter_pack(int32_t n_fft, const int64_t *__restrict__ offsets,
                                                     const int32_t *__restrict__ bins, PeakFilter f,
                                                     const int64_t *__restrict__ out_offsets,
                                                     int32_t *__restrict__ out_bins) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n_fft) return;
    const int ct = f.mode == 0 ? gross_time_cell(f, i) : 0;
    int64_t dst = out_offsets[i];
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t pb = offsets[i]; pb < offsets[i + 1]; pb += 64) {
        const int64_t p = pb + lane;
        const bool in = p < offsets[i + 1];
        const int32_t k = in ? bins[p] : 0;
        const bool keep = in && !filter_drop(f, ct, k);
        const uint64_t m = __ballot(keep);
        if (keep) out_bins[dst + __popcll(m & below)] = k;
        dst += __popcll(m);
    }
}

// one wave per FFT: peaks per natural bin in [k_lo, k_hi)
__global__ void __launch_bounds__(256) k_bin_counts(int32_t n_fft, const int64_t *__restrict__ offsets,
                                                    const int32_t *__restrict__ bins, int32_t k_lo,
                                                    int32_t k_hi, int32_t *__restrict__ counts) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n_fft) return;
    for (int64_t p = offsets[i] + lane; p < offsets[i + 1]; p += 64) {
        const int32_t k = bins[p];
        if (k >= k_lo && k < k_hi) atomicAdd(counts + (k - k_lo), 1);
    }
}

// value histograms for the robust statistic: pass 0 counts x, pass 1 counts
// |2 x - s| (s = twice the median, an integer)
__global__ void k_value_hist(const int32_t *__restrict__ x, int32_t n, int32_t x_max, int pass,
                             const int64_t *__restrict__ s2, int32_t *__restrict__ hist,
                             int32_t *__restrict__ err) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int32_t v = x[e];
    if (v < 0 || v > x_max) {
        atomicOr(err, 1);
        return;
    }
    if (pass == 0) {
        atomicAdd(hist + v, 1);
    } else {
        int64_t d = 2 * (int64_t)v - s2[0];
        d = d < 0 ? -d : d;
        if (d <= 2 * (int64_t)x_max) atomicAdd(hist + d, 1);
    }
}

// One block: the values at 1-based ranks ra and rb of a value histogram of
// m bins; writes their sum to s2[0] and, for pass 0, m1 = sum / 2 to out[0],
// for pass 1, m2 = sum / 4 / 0.6745 to out[1].
__global__ void __launch_bounds__(1024) k_rank_pick(const int32_t *__restrict__ hist, int32_t m, int64_t ra,
                                                    int64_t rb, int pass, int64_t *__restrict__ s2,
                                                    double *__restrict__ out) {
    __shared__ int64_t part[1024];
    __shared__ int32_t val[2];
    const int tid = threadIdx.x;
    if (tid < 2) val[tid] = 0;  // stays 0 for a rank past the total (invalid data)
    const int chunk = (m + 1023) / 1024;
    const int v0 = tid * chunk, v1 = min(v0 + chunk, m);
    int64_t sum = 0;
    for (int v = v0; v < v1; ++v) sum += hist[v];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan
        const int64_t a = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += a;
        __syncthreads();
    }
    const int64_t before = part[tid] - sum;
    for (int q = 0; q < 2; ++q) {
        const int64_t r = q == 0 ? ra : rb;
        if (r > before && r <= before + sum) {
            int64_t c = before;
            for (int v = v0; v < v1; ++v) {
                c += hist[v];
                if (c >= r) {
                    val[q] = v;
                    break;
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int64_t t = (int64_t)val[0] + (int64_t)val[1];
        if (pass == 0) {
            s2[0] = t;
            out[0] = 0.5 * (double)t;
        } else {
            // median of |x - m1| = (t / 2) / 2: both halves exact
            out[1] = 0.5 * (0.5 * (double)val[0] + 0.5 * (double)val[1]) / 0.6745;
        }
    }
}

// fine-bin counts of a column-maximum buffer (value << 32 | ~row)
__global__ void k_colmax_values(const unsigned long long *__restrict__ colmax, int32_t nf,
                                int32_t *__restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nf) out[b] = (int32_t)(colmax[b] >> 32);
}

// Column maxima of n_slots directions decoded: value (the count, or the
// weighted sum as k_select forms it from the fixed point) and smallest row.
__global__ void k_colmax_decode(const unsigned long long *__restrict__ colmax, int32_t nf, int32_t n_slots,
                                const WeightStats *__restrict__ ws, int32_t ws_stride,
                                float *__restrict__ value, int32_t *__restrict__ row) {
    const int64_t n = (int64_t)n_slots * nf;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = colmax[x];
        const uint32_t v = (uint32_t)(k >> 32);
        float f = (float)v;
        if (ws != nullptr) {
            const int64_t slot = x / nf;
            f = f * (float)ldexp(1.0, -ws[slot * ws_stride].frac_bits);
        }
        value[x] = f;
        row[x] = (int32_t)(0xFFFFFFFFu - (uint32_t)k);
    }
}

}  // namespace

hipError_t launch_colmax_decode(const unsigned long long *colmax, int32_t nf, int32_t n_slots, const WeightStats *ws,
                                int32_t ws_stride, float *value, int32_t *row, hipStream_t st) {
    const int64_t n = (int64_t)n_slots * nf;
    if (n <= 0) return hipSuccess;
    k_colmax_decode<<<grid_for(n, 256) > 8192 ? 8192 : grid_for(n, 256), 256, 0, st>>>(colmax, nf, n_slots, ws,
                                                                                       ws_stride, value, row);
    return hipGetLastError();
}

hipError_t launch_slice(int32_t n_fft, const int64_t *offsets, const int32_t *bins, int32_t k_lo, int32_t k_hi,
                        int64_t *first, int32_t *counts, int64_t *out_offsets, int32_t *out_bins,
                        hipStream_t st) {
    k_slice_count<<<grid_for(n_fft, 256), 256, 0, st>>>(n_fft, offsets, bins, k_lo, k_hi, first, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pm_scan<<<1, 1024, 0, st>>>(n_fft, counts, out_offsets);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_slice_pack<<<n_fft, 256, 0, st>>>(first, counts, out_offsets, bins, out_bins);
    return hipGetLastError();
}

hipError_t launch_refine_pick(int32_t n_cand, int32_t n_dir, const fh_candidate *cands, const double *params,
                              const double *lamb, fh_refined *out, hipStream_t st) {
    if (n_cand <= 0) return hipSuccess;
    k_refine_pick<<<grid_for(n_cand, 64), 64, 0, st>>>(n_cand, n_dir, cands, params, lamb, out);
    return hipGetLastError();
}

hipError_t launch_gross_hist(int32_t n_fft, const int64_t *offsets, const int32_t *bins, const double *t,
                             double t_fft, const fh_gross &geo, int32_t *hist, hipStream_t st) {
    hipError_t e = launch_fill_i32(hist, (int64_t)geo.n_t * geo.n_f, 0, st);
    if (e != hipSuccess || n_fft == 0) return e;
    PeakFilter f{};
    f.mode = 0;
    f.t = t;
    f.t_origin = geo.t_origin;
    f.dt_h = geo.dt_h;
    f.B = geo.df_h * t_fft;
    f.c0 = geo.c0;
    f.n_t = geo.n_t;
    f.n_f = geo.n_f;
    k_gross_hist<<<(n_fft + 3) / 4, 256, 0, st>>>(n_fft, offsets, bins, f, hist);
    return hipGetLastError();
}

hipError_t launch_filter(int32_t n_fft, const int64_t *offsets, const int32_t *bins, const FilterSpec &spec,
                         int32_t *counts, int64_t *out_offsets, int32_t *out_bins, int phase, hipStream_t st) {
    PeakFilter f{};
    f.mode = spec.mode;
    f.t = spec.t;
    f.t_origin = spec.geo.t_origin;
    f.dt_h = spec.geo.dt_h;
    f.B = spec.geo.df_h * spec.t_fft;
    f.c0 = spec.geo.c0;
    f.n_t = spec.geo.n_t;
    f.n_f = spec.geo.n_f;
    f.hist = spec.hist;
    f.k_lo = spec.k_lo;
    f.k_hi = spec.k_hi;
    f.step = spec.step;
    f.offset = spec.offset;
    f.n_x = spec.n_x;
    f.x = spec.x;
    f.thr = spec.thr;
    if (n_fft == 0) return hipSuccess;
    if (phase == 0) {
        k_filter_count<<<(n_fft + 3) / 4, 256, 0, st>>>(n_fft, offsets, bins, f, counts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_pm_scan<<<1, 1024, 0, st>>>(n_fft, counts, out_offsets);
    } else {
        k_filter_pack<<<(n_fft + 3) / 4, 256, 0, st>>>(n_fft, offsets, bins, f, out_offsets, out_bins);
    }
    return hipGetLastError();
}

hipError_t launch_bin_counts(int32_t n_fft, const int64_t *offsets, const int32_t *bins, int32_t k_lo,
                             int32_t k_hi, int32_t *counts, hipStream_t st) {
    hipError_t e = launch_fill_i32(counts, (int64_t)k_hi - k_lo, 0, st);
    if (e != hipSuccess || n_fft == 0) return e;
    k_bin_counts<<<(n_fft + 3) / 4, 256, 0, st>>>(n_fft, offsets, bins, k_lo, k_hi, counts);
    return hipGetLastError();
}

hipError_t launch_robust(const int32_t *x, int32_t n, int32_t x_max, int32_t *hist, int64_t *s2, double *out,
                         int32_t *err, hipStream_t st) {
    const int64_t ra = (int64_t)(n + 1) / 2, rb = (int64_t)n / 2 + 1;  // odd n: both the middle
    for (int pass = 0; pass < 2; ++pass) {
        const int32_t m = pass == 0 ? x_max + 1 : 2 * x_max + 1;
        hipError_t e = launch_fill_i32(hist, m, 0, st);
        if (e != hipSuccess) return e;
        k_value_hist<<<grid_for(n, 256), 256, 0, st>>>(x, n, x_max, pass, s2, hist, err);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_rank_pick<<<1, 1024, 0, st>>>(hist, m, ra, rb, pass, s2, out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_colmax_values(const unsigned long long *colmax, int32_t nf, int32_t *out, hipStream_t st) {
    k_colmax_values<<<grid_for(nf, 256), 256, 0, st>>>(colmax, nf, out);
    return hipGetLastError();
}

hipError_t launch_pm_scan(int32_t n_fft, const int32_t *counts, int64_t *offsets, hipStream_t st) {
    k_pm_scan<<<1, 1024, 0, st>>>(n_fft, counts, offsets);
    return hipGetLastError();
}

hipError_t launch_pm_pack(int32_t n_fft, int32_t cap, const int32_t *scratch, const int64_t *offsets,
                          int32_t *bins, hipStream_t st) {
    k_pm_pack<<<n_fft, 256, 0, st>>>(cap, scratch, offsets, bins);
    return hipGetLastError();
}

}  // namespace fh
