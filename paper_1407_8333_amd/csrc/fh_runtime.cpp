// Host runtime of the frequency-Hough library: contexts, device-resident
// peakmaps, validation, tile planning, workspace management and the launch
// sequences behind the C ABI of include/fh.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fh_internal.h"

using namespace fh;

// Scratch memory of fh_hough_map_i32_static (callers that cannot allocate):
// one copy of this array per GPU, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy: the device address of
// each GPU's copy is taken once, with that device current, when the first
// context on it is created (scratch_init), and only that address is used.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

thread_local std::string g_err = "no error";

fh_status fail(fh_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_OK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(FH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

// Device address of each GPU's copy of `scratch` (nullptr until taken).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Take the address of the current device's copy of `scratch` (once per
// device).  Devices past kMaxDevices keep no address; the entry point that
// needs it then reports FH_E_UNSUPPORTED.
fh_status scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return FH_OK;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return FH_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(FH_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return FH_OK;
}

// A device buffer that only grows.  Growing synchronises the stream first so
// that no enqueued kernel still uses the old allocation.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    fh_status ensure(size_t want, hipStream_t st) {
        if (want <= bytes) return FH_OK;
        if (ptr) {
            hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess) return fail(FH_E_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
            (void)hipFree(ptr);
            ptr = nullptr;
            bytes = 0;
        }
        size_t n = std::max(want, (size_t)256);
        if (hipMalloc(&ptr, n) != hipSuccess) {
            ptr = nullptr;
            return fail(FH_E_NOMEM, "hipMalloc of %zu bytes failed", n);
        }
        bytes = n;
        return FH_OK;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
};

struct PinnedBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    fh_status ensure(size_t want, hipStream_t st) {
        if (want <= bytes) return FH_OK;
        if (ptr) {
            hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess) return fail(FH_E_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
            (void)hipHostFree(ptr);
            ptr = nullptr;
        }
        size_t n = std::max(want, (size_t)4096);
        if (hipHostMalloc(&ptr, n, hipHostMallocDefault) != hipSuccess) {
            ptr = nullptr;
            bytes = 0;
            return fail(FH_E_NOMEM, "hipHostMalloc of %zu bytes failed", n);
        }
        bytes = n;
        return FH_OK;
    }
    void release() {
        if (ptr) (void)hipHostFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
};

}  // namespace

struct fh_peakmap {
    int32_t n_fft = 0;
    int64_t n_peaks = 0;
    double t_fft = 0;
    double t_min = 0, t_max = 0;
    double v_max = 0;
    int32_t k_min = 0, k_max = 0;
    int32_t adjacent = 0;  // 1 if some FFT holds two peaks one natural bin apart
    int32_t max_per_fft = 0;
    int64_t *d_offsets = nullptr;
    int32_t *d_bins = nullptr;
    double *d_t = nullptr;
    double *d_v = nullptr;
    int64_t bytes = 0;
};

// Device and pinned buffers of one in-flight search.  A context owns one;
// each serving lane owns another.
struct Workspace {
    DevBuf sht, Y, Y64, win, wsort, colmax, wq, ws, sky, qctr;
    PinnedBuf h_sky;
    size_t device_bytes() const {
        size_t n = 0;
        for (const DevBuf *b : {&sht, &Y, &Y64, &win, &wsort, &colmax, &wq, &ws, &sky, &qctr})
            n += b->bytes;
        return n;
    }
    void release() {
        for (DevBuf *b : {&sht, &Y, &Y64, &win, &wsort, &colmax, &wq, &ws, &sky, &qctr})
            b->release();
        h_sky.release();
    }
};

struct fh_ctx {
    int32_t device = 0;
    int32_t n_cu = 256;
    Workspace main_ws;
    Workspace *cur = &main_ws;  // workspace used by the launch sequences
    int32_t window_method = 2;  // peak windows: 0 binary searches, 1 sweep, 2 fused front
    // Doppler correction: 0 exact per peak, 1 per-FFT shift at doppler_fref
    // (<= 0: each map's band centre)
    int32_t doppler_mode = 0;
    double doppler_fref = 0.0;
    DevBuf err;
    // refinement: sliced peakmap and per-call scratch
    DevBuf rf_offsets, rf_bins, rf_t, rf_v, rf_first, rf_counts, rf_cands, rf_aux;
    // cleaning: robust-statistic histogram, its rank sum and results
    DevBuf cl_hist, cl_s2, cl_out;
    // autotuned tile width per problem shape (shared by weighted and
    // unweighted searches: the two kernels differ only in the added value)
    std::map<std::tuple<int, int, int, int>, int> tuned;
    // captured searches (fh_options.use_graph), keyed by every argument and
    // workspace pointer they bake in
    struct GraphEntry {
        std::vector<uint64_t> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;
    // event-based timing (fh_ctx_profile)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Span { hipEvent_t a, b; int kind; };
    std::vector<Span> spans;
    int64_t prof_updates = 0;
};

namespace {

// nrb: row blocks the tiles run (the last one also takes `tail` rows past it
// when the grid's last 16-row block holds at most kTailRows rows); nrb_tab:
// every 16-row block of the grid (the shift records cover them all).
struct Plan {
    int W, nrb, nbb, nrbg;
    int nrb_tab, tail;
    int64_t tiles_per_sky;
};

// Spin-down shift tables of one search (see k_shift_tables), one buffer:
// gwin int64 [N][nrbg][2] | rec uint2 [nrb][N] | step u32 [N][16].
struct ShiftLayout {
    size_t gwin, rec, step, total;
};

ShiftLayout shift_layout(int64_t n_fft, int nrb, int nrbg) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    ShiftLayout L;
    size_t o = 0;
    L.gwin = o; o += al((size_t)16 * n_fft * nrbg);
    L.rec = o;  o += al((size_t)8 * n_fft * nrb);
    L.step = o; o += al((size_t)4 * kTileRows * n_fft);
    L.total = o;
    return L;
}

// Rows of the grid's last 16-row block when the tiles of the block before
// it take them (at most kTailRows, and a block before it exists), else 0.
int tail_rows(const fh_grid &g) {
    const int nrb = (g.ns + kTileRows - 1) / kTileRows;
    const int r = g.ns - (nrb - 1) * kTileRows;
    return nrb >= 2 && r <= kTailRows ? r : 0;
}

Plan make_plan(const fh_grid &g, int W) {
    Plan p;
    p.W = W;
    p.nrb_tab = (g.ns + kTileRows - 1) / kTileRows;
    // the tail rows are folded only where the wider tile still fits the LDS
    p.tail = tail_rows(g);
    if (p.tail && tile_lds_bytes(W, g.kf, p.tail) > kLdsBytes - kLdsReserve) p.tail = 0;
    p.nrb = p.nrb_tab - (p.tail ? 1 : 0);
    p.nbb = (g.nf + W - 1) / W;
    p.nrbg = (p.nrb + kRowBlocksPerGroup - 1) / kRowBlocksPerGroup;
    p.tiles_per_sky = (int64_t)p.nrb * p.nbb;
    return p;
}

fh_status check_ctx(fh_ctx *ctx) {
    if (!ctx) return fail(FH_E_INVALID, "context is NULL");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(FH_E_DEVICE, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
    return FH_OK;
}

// Largest spin-down step of one row, in fine bins: |dfdot tau| K_f T_FFT
// (Eq. sdstep) over the FFTs' reference-time offsets tau, plus rounding.
double row_step_bins(const fh_peakmap *pm, const fh_grid *g) {
    const double tau = std::max(std::fabs(pm->t_min - g->t0), std::fabs(pm->t_max - g->t0));
    return std::fabs(g->dfdot) * tau * ((double)g->kf * pm->t_fft) + 1e-6;
}

// Widest tile for the grid: its LDS also holds the tail rows when the grid
// has some, unless that leaves no tile of 64 bins (then they run as a row
// block of their own).
int tile_bins_limit(const fh_peakmap *pm, const fh_grid *g) {
    const int w = max_tile_bins(g->kf, row_step_bins(pm, g), kTileRows + tail_rows(*g));
    return w >= 64 ? w : max_tile_bins(g->kf, row_step_bins(pm, g), kTileRows);
}

fh_status check_grid(const fh_peakmap *pm, const fh_grid *g) {
    if (!pm) return fail(FH_E_INVALID, "peakmap is NULL");
    if (!g) return fail(FH_E_INVALID, "grid is NULL");
    if (g->kf < 1 || g->kf > 64) return fail(FH_E_INVALID, "kf=%d outside 1..64", g->kf);
    if (g->nf < 1 || g->nf > (1 << 22)) return fail(FH_E_INVALID, "nf=%d outside 1..2^22", g->nf);
    if (g->ns < 1 || g->ns > (1 << 15)) return fail(FH_E_INVALID, "ns=%d outside 1..2^15", g->ns);
    if (g->b0 < 0 || g->b0 >= ((int64_t)1 << 28)) return fail(FH_E_INVALID, "b0 outside [0, 2^28)");
    if (!std::isfinite(g->fdot0) || !std::isfinite(g->dfdot) || !std::isfinite(g->t0))
        return fail(FH_E_INVALID, "grid has a non-finite fdot0, dfdot or t0");
    // fixed-point range: |K_f k| < 2^28 and every shift far below 2^62
    if ((int64_t)pm->k_max * g->kf >= ((int64_t)1 << 28))
        return fail(FH_E_INVALID, "K_f * k reaches 2^28 (fixed-point range)");
    const double tau = std::max(std::fabs(pm->t_min - g->t0), std::fabs(pm->t_max - g->t0));
    const double S = (double)g->kf * pm->t_fft;
    const double gmax = (std::fabs(g->fdot0) + std::fabs(g->dfdot) * g->ns) * tau * S;
    if (!(gmax < 1e12)) return fail(FH_E_INVALID, "spin-down shifts exceed the fixed-point range");
    if (pm->max_per_fft >= 65536)
        return fail(FH_E_UNSUPPORTED, "an FFT holds %d peaks; at most 65535 are supported", pm->max_per_fft);
    // a window entry holds its FFT's place in a tile run in 15 bits, and the
    // tiles address a direction's stripe edges with 32-bit byte offsets
    if (wave_ffts(pm->n_fft) >= 32768)
        return fail(FH_E_UNSUPPORTED, "n_fft=%d: a tile run would hold more than 32767 FFTs", pm->n_fft);
    if (y_stride(pm->n_peaks, pm->n_fft) >= ((int64_t)1 << 30))
        return fail(FH_E_UNSUPPORTED, "n_peaks + 16 n_fft reaches 2^30");
    // the tiles address the shift records [row blocks][N] with 31-bit byte offsets
    const int64_t nrb = (int64_t)(g->ns + kTileRows - 1) / kTileRows;
    if ((int64_t)pm->n_fft * nrb >= ((int64_t)1 << 28))
        return fail(FH_E_UNSUPPORTED, "n_fft x row blocks = %lld reaches 2^28", (long long)pm->n_fft * nrb);
    if (max_tile_bins(g->kf, row_step_bins(pm, g), kTileRows) < 64)
        return fail(FH_E_UNSUPPORTED, "spin-down step of %.6g fine bins per row is too large for a tile",
                    row_step_bins(pm, g));
    return FH_OK;
}

fh_status check_sky(const double *n) {
    if (!n) return fail(FH_E_INVALID, "sky vector is NULL");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(n[k])) return fail(FH_E_INVALID, "sky vector is not finite");
    const double r = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (std::fabs(r - 1.0) > 1e-9) return fail(FH_E_INVALID, "sky vector is not a unit vector (|n| = %.17g)", r);
    return FH_OK;
}

std::tuple<int, int, int, int> tune_key(const fh_peakmap *pm, const fh_grid *g) {
    return std::make_tuple(pm->n_fft, g->nf, g->ns, g->kf);
}

// Tile width: the requested one (multiple of 64, at most what a 16-row tile
// holds; a width too wide for the tail rows runs them as a row block of
// their own), else the autotuned one, else the widest that also holds the
// tail rows.
int choose_tile_bins(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, int requested) {
    const int wmax = tile_bins_limit(pm, g);
    if (requested > 0)
        return std::min(((requested + 63) / 64) * 64, max_tile_bins(g->kf, row_step_bins(pm, g), kTileRows));
    auto it = ctx->tuned.find(tune_key(pm, g));
    if (it != ctx->tuned.end()) return it->second;
    // a tile never needs to be wider than the map
    int w = std::min(wmax, ((g->nf + 63) / 64) * 64);
    return std::max(64, w);
}

// kinds of timed spans
enum { kSpanFront = 0, kSpanTiles = 1, kSpanSelect = 2, kSpanGraph = 3 };

hipEvent_t next_event(fh_ctx *ctx) {
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ctx->ev_used++];
}

// Records an event before a group of launches and another after it.
// Profiling span.  A record that fails leaves an unrecorded event, which
// fh_ctx_profile_read then reports through hipEventElapsedTime.
struct Timed {
    fh_ctx *ctx;
    hipStream_t st;
    int kind;
    hipEvent_t a = nullptr;
    Timed(fh_ctx *c, hipStream_t s, int k) : ctx(c), st(s), kind(k) {
        if (ctx->profiling) {
            a = next_event(ctx);
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~Timed() {
        if (a) {
            hipEvent_t b = next_event(ctx);
            if (b) {
                (void)hipEventRecord(b, st);
                ctx->spans.push_back({a, b, kind});
            }
        }
    }
};

struct ChunkBufs {
    int64_t *gwin;   // spin-down shift tables (ShiftLayout)
    uint2 *rec;
    uint32_t *step;
    uint32_t *Y;   // low words of the stripe edges (what the tiles read)
    int64_t *Y64;  // full stripe edges, only for the unfused window methods
    int2 *win, *wsort;
    unsigned long long *colmax;
    uint32_t *wq;
    WeightStats *ws;
    double *sky;
    int32_t *qctr, *err;
};

// the unfused window methods (chosen, or forced when one FFT's edges do not
// fit the fused front's LDS) search the full 64-bit edges in device memory
bool needs_full_edges(const fh_ctx *ctx, const fh_peakmap *pm) {
    return !(ctx->window_method == 2 && front_ffts_per_block(pm->max_per_fft) > 0);
}

// device bytes of the stripe edges of one direction
int64_t edge_bytes_per_sky(const fh_ctx *ctx, const fh_peakmap *pm) {
    return (needs_full_edges(ctx, pm) ? 12 : 4) * y_stride(pm->n_peaks, pm->n_fft);
}

fh_status ensure_workspace(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p,
                           int slots, int n_sky, bool weighted, hipStream_t st, ChunkBufs &b) {
    const int64_t N = pm->n_fft;
    fh_status s;
    const ShiftLayout sl = shift_layout(N, p.nrb_tab, p.nrbg);
    if ((s = ctx->cur->sht.ensure(sl.total, st))) return s;
    if ((s = ctx->cur->Y.ensure((size_t)4 * y_stride(pm->n_peaks, pm->n_fft) * slots, st))) return s;
    if (needs_full_edges(ctx, pm) &&
        (s = ctx->cur->Y64.ensure((size_t)8 * y_stride(pm->n_peaks, pm->n_fft) * slots, st)))
        return s;
    if ((s = ctx->cur->win.ensure((size_t)8 * slots * p.nrbg * p.nbb * win_stride(N), st))) return s;
    if ((s = ctx->cur->wsort.ensure((size_t)8 * slots * p.nrbg * p.nbb * win_stride(N), st))) return s;
    if ((s = ctx->cur->colmax.ensure((size_t)8 * slots * g->nf, st))) return s;
    if ((s = ctx->cur->wq.ensure(weighted ? (size_t)4 * slots * N : 4, st))) return s;
    if ((s = ctx->cur->ws.ensure(sizeof(WeightStats) * (size_t)slots, st))) return s;
    if ((s = ctx->cur->sky.ensure((size_t)24 * n_sky, st))) return s;
    if ((s = ctx->cur->qctr.ensure(4 * kXcds, st))) return s;
    if ((s = ctx->err.ensure(4, st))) return s;
    b.gwin = reinterpret_cast<int64_t *>((char *)ctx->cur->sht.ptr + sl.gwin);
    b.rec = reinterpret_cast<uint2 *>((char *)ctx->cur->sht.ptr + sl.rec);
    b.step = reinterpret_cast<uint32_t *>((char *)ctx->cur->sht.ptr + sl.step);
    b.Y = (uint32_t *)ctx->cur->Y.ptr;
    b.Y64 = (int64_t *)ctx->cur->Y64.ptr;
    b.win = (int2 *)ctx->cur->win.ptr;
    b.wsort = (int2 *)ctx->cur->wsort.ptr;
    b.colmax = (unsigned long long *)ctx->cur->colmax.ptr;
    b.wq = (uint32_t *)ctx->cur->wq.ptr;
    b.ws = (WeightStats *)ctx->cur->ws.ptr;
    b.sky = (double *)ctx->cur->sky.ptr;
    b.qctr = (int32_t *)ctx->cur->qctr.ptr;
    b.err = (int32_t *)ctx->err.ptr;
    return FH_OK;
}

TileArgs tile_args(const fh_peakmap *pm, const fh_grid *g, const Plan &p, int slots,
                   const ChunkBufs &b, bool weighted, int ws_stride) {
    TileArgs a{};
    a.n_fft = pm->n_fft;
    a.n_peaks = pm->n_peaks;
    a.kf = g->kf;
    a.nf = g->nf;
    a.ns = g->ns;
    a.W = p.W;
    a.nrb = p.nrb;
    a.tail = p.tail;
    a.nbb = p.nbb;
    a.nrbg = p.nrbg;
    a.n_slots = slots;
    a.Y = b.Y;
    a.win = b.wsort;
    a.rec = b.rec;
    a.step = b.step;
    a.wq = weighted ? b.wq : nullptr;
    a.ws = weighted ? b.ws : nullptr;
    a.ws_stride = ws_stride;
    a.colmax = b.colmax;
    a.queue_ctr = b.qctr;
    return a;
}

// Copy all sky directions of a call to the device in one go.
fh_status upload_sky(fh_ctx *ctx, const double *sky_host, int n_sky, const ChunkBufs &b,
                     hipStream_t st) {
    fh_status s = ctx->cur->h_sky.ensure((size_t)24 * n_sky, st);
    if (s) return s;
    // the pinned staging buffer may still feed an earlier copy on this stream
    HIP_OK(hipStreamSynchronize(st));
    std::memcpy(ctx->cur->h_sky.ptr, sky_host, (size_t)24 * n_sky);
    HIP_OK(hipMemcpyAsync(b.sky, ctx->cur->h_sky.ptr, (size_t)24 * n_sky, hipMemcpyHostToDevice, st));
    return FH_OK;
}

// Shared front half of every path: shifts, weights, stripe edges, windows.
// Reference of the per-FFT shift variant, in fine bins: (K_f T_FFT) f_ref.
double shift_reference_bins(const fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g) {
    const double f_ref = ctx->doppler_fref > 0
                             ? ctx->doppler_fref
                             : ((double)g->b0 + 0.5 * (double)g->nf) / ((double)g->kf * pm->t_fft);
    return ((double)g->kf * pm->t_fft) * f_ref;
}

fh_status enqueue_front(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p,
                        int slots, const double *d_sky, const float *d_w, int w_stride,
                        const ChunkBufs &b, hipStream_t st) {
    Timed timed(ctx, st, kSpanFront);
    HIP_OK(launch_shift_tables(pm->n_fft, p.nrb_tab, p.nrb, g->ns, pm->d_t, g->t0, pm->t_fft, g->kf, g->fdot0, g->dfdot,
                               b.gwin, b.rec, b.step, b.err, st));
    const bool weighted = d_w != nullptr;
    const int n_vec = weighted ? (w_stride == 0 ? 1 : slots) : 0;
    if (weighted)
        HIP_OK(launch_weight_stats(pm->n_fft, n_vec, d_w, w_stride, pm->adjacent ? 2 : 1, b.ws, b.err, st));
    const int F = ctx->window_method == 2 ? front_ffts_per_block(pm->max_per_fft) : 0;
    const int32_t sm = ctx->doppler_mode;
    const double q = sm ? shift_reference_bins(ctx, pm, g) : 0.0;
    if (F > 0) {
        HIP_OK(launch_front(pm->n_fft, pm->n_peaks, pm->d_offsets, pm->d_bins, pm->d_v, d_sky, slots, g->kf,
                            g->b0, b.gwin, b.Y, d_w, w_stride, b.ws, w_stride == 0 ? 0 : 1, b.wq, g->ns,
                            p.nrbg, p.nbb, p.W, F, pm->max_per_fft, b.win, sm, q, st));
        HIP_OK(launch_sort_windows(pm->n_fft, p.nrbg, p.nbb, slots, b.win, b.wsort, st));
        return FH_OK;
    }
    HIP_OK(launch_prep(pm->n_fft, pm->n_peaks, pm->d_offsets, pm->d_bins, pm->d_v, d_sky, slots,
                       g->kf, g->b0, b.Y64, d_w, w_stride, b.ws, w_stride == 0 ? 0 : 1, b.wq, b.Y, sm, q,
                       st));
    HIP_OK(launch_windows(pm->n_fft, pm->d_offsets, b.Y64, pm->n_peaks, b.gwin, p.nrbg, p.nbb,
                          p.W, g->kf, slots, b.win, ctx->window_method == 0 ? 0 : 1, st));
    HIP_OK(launch_sort_windows(pm->n_fft, p.nrbg, p.nbb, slots, b.win, b.wsort, st));
    return FH_OK;
}

fh_status enqueue_map(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p, const float *d_w,
                      const ChunkBufs &b, void *out, hipStream_t st);

fh_status hough_map_common(fh_ctx *ctx, const fh_peakmap *pm, const double nhat[3],
                           const float *d_w, const fh_grid *g, void *out, void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if ((s = check_grid(pm, g))) return s;
    if ((s = check_sky(nhat))) return s;
    if (!out) return fail(FH_E_INVALID, "output map pointer is NULL");
    hipStream_t st = (hipStream_t)stream;
    const bool weighted = d_w != nullptr;
    const Plan p = make_plan(*g, choose_tile_bins(ctx, pm, g, 0));
    ChunkBufs b;
    if ((s = ensure_workspace(ctx, pm, g, p, 1, 1, weighted, st, b))) return s;
    if ((s = upload_sky(ctx, nhat, 1, b, st))) return s;
    return enqueue_map(ctx, pm, g, p, d_w, b, out, st);
}

// Front and tiles of one direction's map (the direction already in b.sky).
fh_status enqueue_map(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p, const float *d_w,
                      const ChunkBufs &b, void *out, hipStream_t st) {
    fh_status s;
    const bool weighted = d_w != nullptr;
    if ((s = enqueue_front(ctx, pm, g, p, 1, b.sky, d_w, 0, b, st))) return s;
    TileArgs a = tile_args(pm, g, p, 1, b, weighted, 0);
    a.map_i32 = weighted ? nullptr : (int32_t *)out;
    a.map_f32 = weighted ? (float *)out : nullptr;
    a.tile_base = 0;
    {
        Timed timed(ctx, st, kSpanTiles);
        HIP_OK(launch_tiles(a, weighted, true, false, false, (int32_t)p.tiles_per_sky, 0, st));
    }
    if (ctx->profiling) ctx->prof_updates += pm->n_peaks * (int64_t)g->ns;
    return FH_OK;
}

// chunk: as many directions as a 48 GiB workspace holds (a sixth of the
// MI355X's HBM), at most 4096: fewer launches, more tiles per persistent
// launch (the 256 Hz batch of 1024 directions, 27 GB, is one launch)
// Directions whose tiles one launch can number (tile ids are 32-bit).
int64_t chunk_by_tiles(const Plan &p) {
    return std::max<int64_t>(1, (((int64_t)1 << 31) - 1) / std::max<int64_t>(1, p.tiles_per_sky));
}

int default_chunk(const fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p, int requested) {
    if (requested > 0) return (int)std::min<int64_t>(requested, chunk_by_tiles(p));
    const int64_t per_sky = edge_bytes_per_sky(ctx, pm) + 16 * (int64_t)p.nrbg * p.nbb * win_stride(pm->n_fft) + 8 * (int64_t)g->nf;
    const int64_t by_mem = std::max<int64_t>(1, ((int64_t)48 << 30) / std::max<int64_t>(1, per_sky));
    return (int)std::min<int64_t>(std::min<int64_t>(by_mem, 4096), chunk_by_tiles(p));
}

// Enqueue the search of n_sky directions (already uploaded to b.sky) in
// chunks of `chunk`; sel == nullptr skips candidate selection.
// Optional per-bin column maxima of every direction, decoded: value [n_sky][nf]
// and smallest row holding it [n_sky][nf].
struct ColmaxOut {
    float *value = nullptr;
    int32_t *row = nullptr;
};

fh_status run_search(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p, int chunk,
                     int n_sky, const float *d_w, int w_stride, int schedule, const fh_select *sel,
                     fh_candidate *d_out, const ChunkBufs &b, hipStream_t st, ColmaxOut cm_out = {}) {
    fh_status s;
    const bool weighted = d_w != nullptr;
    for (int32_t base = 0; base < n_sky; base += chunk) {
        const int slots = std::min(chunk, n_sky - base);
        const float *w = weighted ? d_w + (w_stride ? (int64_t)base * w_stride : 0) : nullptr;
        if ((s = enqueue_front(ctx, pm, g, p, slots, b.sky + 3 * (int64_t)base, w, w_stride, b, st))) return s;
        HIP_OK(launch_fill_u64(b.colmax, (int64_t)slots * g->nf, 0ull, st));
        TileArgs a = tile_args(pm, g, p, slots, b, weighted, w_stride == 0 ? 0 : 1);
        const int64_t n_tiles = p.tiles_per_sky * slots;
        if (schedule == FH_SCHED_PERSISTENT) {
            HIP_OK(launch_fill_i32(b.qctr, kXcds, 0, st));
            const int grid_blocks = (int)std::min<int64_t>(ctx->n_cu, n_tiles);
            Timed timed(ctx, st, kSpanTiles);
            HIP_OK(launch_tiles(a, weighted, false, true, true, (int32_t)n_tiles, grid_blocks, st));
        } else {
            a.tile_base = 0;
            Timed timed(ctx, st, kSpanTiles);
            HIP_OK(launch_tiles(a, weighted, false, true, false, (int32_t)n_tiles, 0, st));
        }
        if (ctx->profiling) ctx->prof_updates += pm->n_peaks * (int64_t)g->ns * slots;
        if (cm_out.value)
            HIP_OK(launch_colmax_decode(b.colmax, g->nf, slots, weighted ? b.ws : nullptr,
                                        weighted ? (w_stride == 0 ? 0 : 1) : 0,
                                        cm_out.value + (int64_t)base * g->nf, cm_out.row + (int64_t)base * g->nf,
                                        st));
        if (sel) {
            Timed timed_sel(ctx, st, kSpanSelect);
            HIP_OK(launch_select(b.colmax, g->nf, slots, *sel, base, pm->n_fft, weighted ? b.ws : nullptr,
                                 weighted ? (w_stride == 0 ? 0 : 1) : 0, d_out, st));
        }
    }
    return FH_OK;
}

// Tile-width autotuner: times the persistent search of a sample of the
// directions for each candidate width (multiples of 64 up to what the LDS
// holds) and keeps the fastest per problem shape and weighting.  With tail
// rows, the widest 16-row tile (too wide to hold them, so they run as a row
// block of their own) is a candidate too.
fh_status autotune(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, int n_sky,
                   const double *sky, const float *d_w, int w_stride, hipStream_t st) {
    const bool weighted = d_w != nullptr;
    const int wmax = tile_bins_limit(pm, g);
    const int wmap = std::max(64, ((g->nf + 63) / 64) * 64);  // a tile never needs to be wider than the map
    const int wcap = std::min(wmax, wmap);
    std::vector<int> cands;
    for (int w : {512, 832, 1280, 1792, 2176})
        if (w < wcap) cands.push_back(w);
    cands.push_back(wcap);
    const int w16 = std::min(max_tile_bins(g->kf, row_step_bins(pm, g), kTileRows), wmap);
    if (w16 > wcap) cands.push_back(w16);
    const int sample = std::min(n_sky, 128);
    const bool was = ctx->profiling;
    ctx->profiling = false;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    int best_w = wcap;
    float best_ms = 0.f;
    fh_status s = FH_OK;
    for (int w : cands) {
        const Plan p = make_plan(*g, w);
        ChunkBufs b;
        if ((s = ensure_workspace(ctx, pm, g, p, sample, n_sky, weighted, st, b))) break;
        if ((s = upload_sky(ctx, sky, sample, b, st))) break;
        float ms = 0.f;
        for (int rep = 0; rep < 2 && s == FH_OK; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) { s = fail(FH_E_DEVICE, "hipEventRecord"); break; }
            s = run_search(ctx, pm, g, p, sample, sample, d_w, w_stride, FH_SCHED_PERSISTENT, nullptr,
                           nullptr, b, st);
            if (s) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                s = fail(FH_E_DEVICE, "autotune timing failed");
                break;
            }
        }
        if (s) break;
        if (best_ms == 0.f || ms < best_ms) {
            best_ms = ms;
            best_w = w;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->profiling = was;
    if (s) return s;
    ctx->tuned[tune_key(pm, g)] = best_w;
    return FH_OK;
}

}  // namespace

// peakmap cleaning helpers
namespace {

fh_status check_gross(const fh_gross *geo) {
    if (!geo) return fail(FH_E_INVALID, "gross geometry is NULL");
    if (!(geo->dt_h > 0) || !(geo->df_h > 0) || !std::isfinite(geo->dt_h) || !std::isfinite(geo->df_h) ||
        !std::isfinite(geo->t_origin))
        return fail(FH_E_INVALID, "gross cells need finite dt_h > 0, df_h > 0 and t_origin");
    if (geo->n_t < 1 || geo->n_f < 1 || (int64_t)geo->n_t * geo->n_f > ((int64_t)1 << 31))
        return fail(FH_E_INVALID, "gross histogram of %d x %d cells", geo->n_t, geo->n_f);
    return FH_OK;
}

// A new peakmap holding the peaks of pm that `spec` keeps.
fh_status filter_peakmap(fh_ctx *ctx, const fh_peakmap *pm, const FilterSpec &spec, hipStream_t st,
                         fh_peakmap **out) {
    fh_status s;
    const int32_t N = pm->n_fft;
    if ((s = ctx->rf_counts.ensure(4 * (size_t)std::max(1, N), st))) return s;
    fh_peakmap *q = new fh_peakmap(*pm);
    q->d_offsets = nullptr;
    q->d_bins = nullptr;
    q->d_t = nullptr;
    q->d_v = nullptr;
    const size_t b_off = 8 * (size_t)(N + 1);
    if (hipMalloc(&q->d_offsets, b_off) != hipSuccess || hipMalloc(&q->d_t, 8 * (size_t)N) != hipSuccess ||
        hipMalloc(&q->d_v, 24 * (size_t)N) != hipSuccess) {
        fh_peakmap_release(ctx, q);
        return fail(FH_E_NOMEM, "device allocation for the cleaned peakmap failed");
    }
    std::vector<int64_t> h_off((size_t)N + 1, 0);
    hipError_t e = hipSuccess;
    if (N > 0) {
        e = launch_filter(N, pm->d_offsets, pm->d_bins, spec, (int32_t *)ctx->rf_counts.ptr, q->d_offsets,
                          nullptr, 0, st);
        if (e == hipSuccess) e = hipMemcpyAsync(h_off.data(), q->d_offsets, b_off, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    } else {
        e = hipMemcpyAsync(q->d_offsets, h_off.data(), b_off, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    const int64_t P = e == hipSuccess ? h_off[N] : 0;
    if (e == hipSuccess && hipMalloc(&q->d_bins, 4 * (size_t)std::max<int64_t>(1, P)) != hipSuccess)
        e = hipErrorOutOfMemory;
    if (e == hipSuccess && N > 0)
        e = launch_filter(N, pm->d_offsets, pm->d_bins, spec, nullptr, q->d_offsets, q->d_bins, 1, st);
    if (e == hipSuccess) e = hipMemcpyAsync(q->d_t, pm->d_t, 8 * (size_t)N, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(q->d_v, pm->d_v, 24 * (size_t)N, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
        fh_peakmap_release(ctx, q);
        return fail(e == hipErrorOutOfMemory ? FH_E_NOMEM : FH_E_DEVICE, "filtering the peakmap failed: %s",
                    hipGetErrorString(e));
    }
    q->n_peaks = P;
    q->max_per_fft = 0;
    for (int32_t i = 0; i < N; ++i) q->max_per_fft = std::max<int32_t>(q->max_per_fft, (int32_t)(h_off[i + 1] - h_off[i]));
    q->bytes = (int64_t)(b_off + 4 * (size_t)std::max<int64_t>(1, P) + 32 * (size_t)N);
    *out = q;
    return FH_OK;
}

}  // namespace

extern "C" {

const char *fh_version(void) { return "fh-mi355x 0.1 (gfx950)"; }

const char *fh_last_error(void) { return g_err.c_str(); }

fh_status fh_ctx_create(int32_t device, fh_ctx **out) {
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(FH_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(FH_E_INVALID, "device %d not in [0, %d)", device, n);
    HIP_OK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(FH_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    HIP_OK(init_kernel_attributes());
    fh_status ss = scratch_init(device);
    if (ss) return ss;
    fh_ctx *c = new fh_ctx();
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    fh_status s = c->err.ensure(4, nullptr);
    if (s) {
        delete c;
        return s;
    }
    if (hipMemset(c->err.ptr, 0, 4) != hipSuccess) {
        c->err.release();
        delete c;
        return fail(FH_E_DEVICE, "hipMemset failed");
    }
    *out = c;
    return FH_OK;
}

void fh_ctx_destroy(fh_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &e : ctx->graphs) {
        (void)hipGraphExecDestroy(e.exec);
        (void)hipGraphDestroy(e.graph);
    }
    ctx->graphs.clear();
    ctx->main_ws.release();
    ctx->err.release();
    for (DevBuf *b : {&ctx->rf_offsets, &ctx->rf_bins, &ctx->rf_t, &ctx->rf_v, &ctx->rf_first, &ctx->rf_counts,
                      &ctx->rf_cands, &ctx->rf_aux, &ctx->cl_hist, &ctx->cl_s2, &ctx->cl_out})
        b->release();
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

fh_status fh_ctx_set_doppler(fh_ctx *ctx, int32_t mode, double f_ref) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (mode != 0 && mode != 1) return fail(FH_E_INVALID, "Doppler mode must be 0 (exact) or 1 (per-FFT shift)");
    if (!std::isfinite(f_ref)) return fail(FH_E_INVALID, "reference frequency is not finite");
    ctx->doppler_mode = mode;
    ctx->doppler_fref = f_ref;
    return FH_OK;
}

fh_status fh_ctx_set_option(fh_ctx *ctx, const char *name, int64_t value) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (!name) return fail(FH_E_INVALID, "option name is NULL");
    if (std::strcmp(name, "window_method") == 0) {
        if (value < 0 || value > 2) return fail(FH_E_INVALID, "window_method must be 0, 1 or 2");
        ctx->window_method = (int32_t)value;
        return FH_OK;
    }
    return fail(FH_E_INVALID, "unknown option '%s'", name);
}

fh_status fh_ctx_check(fh_ctx *ctx, void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_OK(hipStreamSynchronize(st));
    int32_t flag = 0;
    HIP_OK(hipMemcpy(&flag, ctx->err.ptr, 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemset(ctx->err.ptr, 0, 4));
    if (flag & 2) return fail(FH_E_DEVICE, "internal: a spin-down residual code left its 2-bit range");
    if (flag) return fail(FH_E_INVALID, "a weight vector held a value that is not finite or outside (0, 65536), or whose sum is too large");
    return FH_OK;
}

fh_status fh_peakmap_upload(fh_ctx *ctx, const fh_peakmap_desc *d, void *stream, fh_peakmap **out) {
    fh_status s;
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    *out = nullptr;
    if ((s = check_ctx(ctx))) return s;
    if (!d) return fail(FH_E_INVALID, "descriptor is NULL");
    const int32_t N = d->n_fft;
    if (N < 1) return fail(FH_E_INVALID, "n_fft=%d < 1", N);
    if (!d->offsets || !d->t || !d->v || (d->n_peaks > 0 && !d->bins))
        return fail(FH_E_INVALID, "a peakmap array is NULL");
    if (!(d->t_fft > 0) || !std::isfinite(d->t_fft)) return fail(FH_E_INVALID, "t_fft must be finite and > 0");
    if (d->offsets[0] != 0) return fail(FH_E_INVALID, "offsets[0] != 0");
    if (d->offsets[N] != d->n_peaks) return fail(FH_E_INVALID, "offsets[N] != n_peaks");
    if (d->n_peaks < 0 || d->n_peaks >= ((int64_t)1 << 31)) return fail(FH_E_INVALID, "n_peaks outside [0, 2^31)");
    fh_peakmap *pm = new fh_peakmap();
    pm->n_fft = N;
    pm->n_peaks = d->n_peaks;
    pm->t_fft = d->t_fft;
    pm->t_min = d->t[0];
    pm->t_max = d->t[0];
    pm->k_min = 0x7fffffff;
    pm->k_max = 0;
    for (int32_t i = 0; i < N; ++i) {
        const int64_t a = d->offsets[i], e = d->offsets[i + 1];
        if (e < a) { delete pm; return fail(FH_E_INVALID, "offsets decrease at FFT %d", i); }
        if (!std::isfinite(d->t[i])) { delete pm; return fail(FH_E_INVALID, "t[%d] is not finite", i); }
        pm->t_min = std::min(pm->t_min, d->t[i]);
        pm->t_max = std::max(pm->t_max, d->t[i]);
        const double *v = d->v + 3 * (int64_t)i;
        if (!std::isfinite(v[0]) || !std::isfinite(v[1]) || !std::isfinite(v[2])) {
            delete pm;
            return fail(FH_E_INVALID, "v[%d] is not finite", i);
        }
        const double vn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (vn >= 1e-2) { delete pm; return fail(FH_E_INVALID, "|v[%d]| = %g >= 1e-2", i, vn); }
        pm->v_max = std::max(pm->v_max, vn);
        pm->max_per_fft = std::max<int32_t>(pm->max_per_fft, (int32_t)(e - a));
        for (int64_t p = a; p < e; ++p) {
            const int32_t k = d->bins[p];
            if (k < 0) { delete pm; return fail(FH_E_INVALID, "negative bin at peak %lld", (long long)p); }
            if (p > a) {
                if (k <= d->bins[p - 1]) {
                    delete pm;
                    return fail(FH_E_INVALID, "bins not strictly ascending in FFT %d", i);
                }
                if (k == d->bins[p - 1] + 1) pm->adjacent = 1;
            }
            pm->k_min = std::min(pm->k_min, k);
            pm->k_max = std::max(pm->k_max, k);
        }
    }
    if (pm->n_peaks == 0) pm->k_min = pm->k_max = 0;
    hipStream_t st = (hipStream_t)stream;
    const size_t b_off = 8 * (size_t)(N + 1), b_bins = 4 * (size_t)std::max<int64_t>(1, d->n_peaks);
    const size_t b_t = 8 * (size_t)N, b_v = 24 * (size_t)N;
    if (hipMalloc(&pm->d_offsets, b_off) != hipSuccess || hipMalloc(&pm->d_bins, b_bins) != hipSuccess ||
        hipMalloc(&pm->d_t, b_t) != hipSuccess || hipMalloc(&pm->d_v, b_v) != hipSuccess) {
        fh_peakmap_release(ctx, pm);
        return fail(FH_E_NOMEM, "device allocation for the peakmap failed");
    }
    pm->bytes = (int64_t)(b_off + b_bins + b_t + b_v);
    hipError_t e = hipMemcpyAsync(pm->d_offsets, d->offsets, b_off, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && d->n_peaks > 0)
        e = hipMemcpyAsync(pm->d_bins, d->bins, 4 * (size_t)d->n_peaks, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pm->d_t, d->t, b_t, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pm->d_v, d->v, b_v, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        fh_peakmap_release(ctx, pm);
        return fail(FH_E_DEVICE, "peakmap upload failed: %s", hipGetErrorString(e));
    }
    *out = pm;
    return FH_OK;
}

fh_status fh_peakmap_from_spectra(fh_ctx *ctx, int32_t n_fft, int32_t n_bins, int64_t ld,
                                  const float *d_sp, const float *d_sar, int32_t k0, float theta,
                                  const double *t, const double *v, double t_fft, void *stream,
                                  fh_peakmap **out) {
    fh_status s;
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    *out = nullptr;
    if ((s = check_ctx(ctx))) return s;
    if (n_fft < 1 || n_fft > (1 << 24)) return fail(FH_E_INVALID, "n_fft=%d outside 1..2^24", n_fft);
    if (n_bins < 3 || ld < n_bins) return fail(FH_E_INVALID, "need n_bins >= 3 and ld >= n_bins");
    if (!d_sp || !t || !v) return fail(FH_E_INVALID, "a spectrum or time/velocity array is NULL");
    if (k0 < 0 || (int64_t)k0 + n_bins >= ((int64_t)1 << 31)) return fail(FH_E_INVALID, "k0 out of range");
    if (!std::isfinite(theta)) return fail(FH_E_INVALID, "theta is not finite");
    if (!(t_fft > 0) || !std::isfinite(t_fft)) return fail(FH_E_INVALID, "t_fft must be finite and > 0");
    fh_peakmap *pm = new fh_peakmap();
    pm->n_fft = n_fft;
    pm->t_fft = t_fft;
    pm->t_min = pm->t_max = t[0];
    for (int32_t i = 0; i < n_fft; ++i) {
        if (!std::isfinite(t[i])) { delete pm; return fail(FH_E_INVALID, "t[%d] is not finite", i); }
        pm->t_min = std::min(pm->t_min, t[i]);
        pm->t_max = std::max(pm->t_max, t[i]);
        const double *vi = v + 3 * (int64_t)i;
        if (!std::isfinite(vi[0]) || !std::isfinite(vi[1]) || !std::isfinite(vi[2])) {
            delete pm;
            return fail(FH_E_INVALID, "v[%d] is not finite", i);
        }
        const double vn = std::sqrt(vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
        if (vn >= 1e-2) { delete pm; return fail(FH_E_INVALID, "|v[%d]| = %g >= 1e-2", i, vn); }
        pm->v_max = std::max(pm->v_max, vn);
    }
    hipStream_t st = (hipStream_t)stream;
    const int32_t cap = n_bins / 2 + 1;  // strict local maxima are never adjacent
    int32_t *rows_buf = nullptr, *counts = nullptr;
    const size_t b_off = 8 * (size_t)(n_fft + 1), b_t = 8 * (size_t)n_fft, b_v = 24 * (size_t)n_fft;
    if (hipMalloc(&rows_buf, 4 * (size_t)n_fft * cap) != hipSuccess || hipMalloc(&counts, 4 * (size_t)n_fft) != hipSuccess ||
        hipMalloc(&pm->d_offsets, b_off) != hipSuccess || hipMalloc(&pm->d_t, b_t) != hipSuccess ||
        hipMalloc(&pm->d_v, b_v) != hipSuccess) {
        if (rows_buf) (void)hipFree(rows_buf);
        if (counts) (void)hipFree(counts);
        fh_peakmap_release(ctx, pm);
        return fail(FH_E_NOMEM, "device allocation for the peakmap failed");
    }
    std::vector<int64_t> h_off(n_fft + 1);
    hipError_t e = launch_pm_rows(n_fft, n_bins, ld, d_sp, d_sar, k0, theta, cap, rows_buf, counts, st);
    if (e == hipSuccess) e = launch_pm_scan(n_fft, counts, pm->d_offsets, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h_off.data(), pm->d_offsets, b_off, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const int64_t P = e == hipSuccess ? h_off[n_fft] : 0;
    if (e == hipSuccess && hipMalloc(&pm->d_bins, 4 * (size_t)std::max<int64_t>(1, P)) != hipSuccess)
        e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = launch_pm_pack(n_fft, cap, rows_buf, pm->d_offsets, pm->d_bins, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pm->d_t, t, b_t, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pm->d_v, v, b_v, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(rows_buf);
    (void)hipFree(counts);
    if (e != hipSuccess) {
        fh_peakmap_release(ctx, pm);
        return fail(e == hipErrorOutOfMemory ? FH_E_NOMEM : FH_E_DEVICE, "peakmap construction failed: %s",
                    hipGetErrorString(e));
    }
    pm->n_peaks = P;
    pm->k_min = k0 + 1;
    pm->k_max = k0 + n_bins - 2;
    pm->adjacent = 0;
    for (int32_t i = 0; i < n_fft; ++i)
        pm->max_per_fft = std::max<int32_t>(pm->max_per_fft, (int32_t)(h_off[i + 1] - h_off[i]));
    pm->bytes = (int64_t)(b_off + 4 * (size_t)std::max<int64_t>(1, P) + b_t + b_v);
    *out = pm;
    return FH_OK;
}

fh_status fh_peakmap_download(fh_ctx *ctx, const fh_peakmap *pm, int64_t *offsets, int32_t *bins) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (!pm) return fail(FH_E_INVALID, "peakmap is NULL");
    if (offsets) HIP_OK(hipMemcpy(offsets, pm->d_offsets, 8 * (size_t)(pm->n_fft + 1), hipMemcpyDeviceToHost));
    if (bins && pm->n_peaks > 0)
        HIP_OK(hipMemcpy(bins, pm->d_bins, 4 * (size_t)pm->n_peaks, hipMemcpyDeviceToHost));
    return FH_OK;
}

fh_status fh_peakmap_shape(const fh_peakmap *pm, int32_t *n_fft, int64_t *n_peaks) {
    if (!pm) return fail(FH_E_INVALID, "peakmap is NULL");
    if (n_fft) *n_fft = pm->n_fft;
    if (n_peaks) *n_peaks = pm->n_peaks;
    return FH_OK;
}

void fh_peakmap_release(fh_ctx *ctx, fh_peakmap *pm) {
    if (!pm) return;
    if (ctx) (void)hipSetDevice(ctx->device);
    if (pm->d_offsets) (void)hipFree(pm->d_offsets);
    if (pm->d_bins) (void)hipFree(pm->d_bins);
    if (pm->d_t) (void)hipFree(pm->d_t);
    if (pm->d_v) (void)hipFree(pm->d_v);
    delete pm;
}

int64_t fh_peakmap_bytes(const fh_peakmap *pm) { return pm ? pm->bytes : 0; }

fh_status fh_peakmap_slice(fh_ctx *ctx, const fh_peakmap *pm, int32_t k_lo, int32_t k_hi, void *stream,
                           fh_peakmap **out) {
    fh_status s;
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    *out = nullptr;
    if ((s = check_ctx(ctx))) return s;
    if (!pm) return fail(FH_E_INVALID, "peakmap is NULL");
    if (k_lo < 0 || k_hi <= k_lo) return fail(FH_E_INVALID, "need 0 <= k_lo < k_hi");
    hipStream_t st = (hipStream_t)stream;
    const int32_t N = pm->n_fft;
    const int64_t cap = std::min<int64_t>((int64_t)N * (k_hi - k_lo), pm->n_peaks);
    if ((s = ctx->rf_first.ensure(8 * (size_t)N, st)) || (s = ctx->rf_counts.ensure(4 * (size_t)N, st)))
        return s;
    fh_peakmap *q = new fh_peakmap(*pm);
    q->d_offsets = nullptr;
    q->d_bins = nullptr;
    q->d_t = nullptr;
    q->d_v = nullptr;
    q->n_peaks = cap;
    q->k_min = k_lo;
    q->k_max = k_hi - 1;
    q->max_per_fft = std::min<int32_t>(pm->max_per_fft, k_hi - k_lo);
    const size_t b_off = 8 * (size_t)(N + 1), b_bins = 4 * (size_t)std::max<int64_t>(1, cap);
    if (hipMalloc(&q->d_offsets, b_off) != hipSuccess || hipMalloc(&q->d_bins, b_bins) != hipSuccess ||
        hipMalloc(&q->d_t, 8 * (size_t)N) != hipSuccess || hipMalloc(&q->d_v, 24 * (size_t)N) != hipSuccess) {
        fh_peakmap_release(ctx, q);
        return fail(FH_E_NOMEM, "device allocation for the sliced peakmap failed");
    }
    q->bytes = (int64_t)(b_off + b_bins + 32 * (size_t)N);
    hipError_t e = launch_slice(N, pm->d_offsets, pm->d_bins, k_lo, k_hi, (int64_t *)ctx->rf_first.ptr,
                                (int32_t *)ctx->rf_counts.ptr, q->d_offsets, q->d_bins, st);
    if (e == hipSuccess) e = hipMemcpyAsync(q->d_t, pm->d_t, 8 * (size_t)N, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(q->d_v, pm->d_v, 24 * (size_t)N, hipMemcpyDeviceToDevice, st);
    // exact peak count and longest FFT of the slice (the allocation keeps the bound)
    std::vector<int64_t> h_off((size_t)N + 1);
    if (e == hipSuccess) e = hipMemcpyAsync(h_off.data(), q->d_offsets, b_off, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        fh_peakmap_release(ctx, q);
        return fail(FH_E_DEVICE, "slicing the peakmap failed: %s", hipGetErrorString(e));
    }
    q->n_peaks = h_off[N];
    q->max_per_fft = 0;
    for (int32_t i = 0; i < N; ++i) q->max_per_fft = std::max<int32_t>(q->max_per_fft, (int32_t)(h_off[i + 1] - h_off[i]));
    *out = q;
    return FH_OK;
}

fh_status fh_refine(fh_ctx *ctx, const fh_peakmap *pm, int32_t n_cand, const fh_coarse_cand *cands,
                    const fh_refine_opts *o, const float *d_w, fh_refined *d_out, void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (!pm || !o) return fail(FH_E_INVALID, "peakmap or options is NULL");
    if (n_cand < 0 || (n_cand > 0 && (!cands || !d_out))) return fail(FH_E_INVALID, "bad candidate arrays");
    if (o->kf < 1 || o->kf > 64 || o->k_fdot < 1 || o->k_sky < 1 || o->k_sky % 2 == 0 || o->k_sky > 63)
        return fail(FH_E_INVALID, "refine options need 1 <= kf <= 64, k_fdot >= 1, odd 1 <= k_sky <= 63");
    if (!(o->dfdot > 0) || !std::isfinite(o->dfdot) || !std::isfinite(o->t0) || !(o->theta > 0))
        return fail(FH_E_INVALID, "refine options need dfdot > 0, finite t0 and theta > 0");
    if (n_cand == 0) return FH_OK;
    hipStream_t st = (hipStream_t)stream;
    const int kf = o->kf, ks = o->k_sky, n_dir = ks * ks, L = (ks - 1) / 2;
    const int ns = 4 * o->k_fdot, nf = 2 * kf + 1;
    const double T = pm->t_fft, dfd = o->dfdot / o->k_fdot;
    const double tau = std::max(std::fabs(pm->t_min - o->t0), std::fabs(pm->t_max - o->t0));
    const double ce = std::cos(23.44 * M_PI / 180.0), se = std::sin(23.44 * M_PI / 180.0);
    std::vector<fh_grid> grids((size_t)n_cand);
    std::vector<int32_t> klo((size_t)n_cand), khi((size_t)n_cand);
    std::vector<double> sky((size_t)n_cand * n_dir * 3), aux((size_t)n_cand * (4 + 2 * n_dir));
    double *prm = aux.data(), *lamb = aux.data() + 4 * (size_t)n_cand;
    int32_t width = 1, kmin = 0x7fffffff, kmax = 0;
    for (int c = 0; c < n_cand; ++c) {
        const fh_coarse_cand &q = cands[c];
        if (!std::isfinite(q.f0) || !(q.f0 > 0) || !std::isfinite(q.fdot) || !std::isfinite(q.lambda) ||
            !std::isfinite(q.beta) || !std::isfinite(q.dlambda) || !std::isfinite(q.dbeta))
            return fail(FH_E_INVALID, "candidate %d is not finite", c);
        fh_grid &g = grids[c];
        g.kf = kf;
        g.b0 = (int64_t)std::llround(q.f0 * kf * T) - kf;
        g.nf = nf;
        g.ns = ns;
        g.fdot0 = q.fdot - 2.0 * o->dfdot;
        g.dfdot = dfd;
        g.t0 = o->t0;
        if (g.b0 < 0) return fail(FH_E_INVALID, "candidate %d lies below the first fine bin", c);
        prm[4 * c + 0] = (double)g.b0 / (kf * T);
        prm[4 * c + 1] = 1.0 / (kf * T);
        prm[4 * c + 2] = g.fdot0;
        prm[4 * c + 3] = dfd;
        // peaks whose stripes can reach the refined bins: Doppler and
        // spin-down drift over the observation, plus one bin each side
        const double f_lo = (double)g.b0 / (kf * T), f_hi = (double)(g.b0 + nf) / (kf * T);
        const double fd_max = std::max(std::fabs(g.fdot0), std::fabs(g.fdot0 + (ns - 1) * dfd));
        const int64_t margin = (int64_t)std::ceil((f_hi * pm->v_max * 1.01 + fd_max * tau) * T) + 2;
        klo[c] = (int32_t)std::max<int64_t>(0, (int64_t)std::floor(f_lo * T) - margin);
        khi[c] = (int32_t)std::min<int64_t>((int64_t)1 << 30, (int64_t)std::ceil(f_hi * T) + margin + 1);
        width = std::max(width, khi[c] - klo[c]);
        kmin = std::min(kmin, klo[c]);
        kmax = std::max(kmax, khi[c] - 1);
        for (int j = -L; j <= L; ++j)
            for (int i = -L; i <= L; ++i) {
                const int d = (j + L) * ks + (i + L);
                double lam = q.lambda + i * (q.dlambda / ks), bet = q.beta + j * (q.dbeta / ks);
                if (std::fabs(bet) > 0.5 * M_PI) {  // over a pole
                    lam += M_PI;
                    bet = (bet > 0 ? M_PI : -M_PI) - bet;
                }
                lam = std::fmod(lam, 2.0 * M_PI);
                if (lam < 0) lam += 2.0 * M_PI;
                lamb[2 * ((size_t)c * n_dir + d)] = lam;
                lamb[2 * ((size_t)c * n_dir + d) + 1] = bet;
                const double x = std::cos(bet) * std::cos(lam), ye = std::cos(bet) * std::sin(lam),
                             ze = std::sin(bet);
                double n[3] = {x, ye * ce - ze * se, ye * se + ze * ce};
                const double r = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                for (int k = 0; k < 3; ++k) sky[3 * ((size_t)c * n_dir + d) + k] = n[k] / r;
            }
    }
    // the sliced peakmap (context-owned arrays, reused by every candidate)
    const int32_t N = pm->n_fft;
    const int64_t cap = std::min<int64_t>((int64_t)N * width, pm->n_peaks);
    if ((s = ctx->rf_offsets.ensure(8 * (size_t)(N + 1), st)) || (s = ctx->rf_bins.ensure(4 * (size_t)cap + 4, st)) ||
        (s = ctx->rf_t.ensure(8 * (size_t)N, st)) || (s = ctx->rf_v.ensure(24 * (size_t)N, st)) ||
        (s = ctx->rf_first.ensure(8 * (size_t)N, st)) || (s = ctx->rf_counts.ensure(4 * (size_t)N, st)) ||
        (s = ctx->rf_cands.ensure(sizeof(fh_candidate) * 2 * (size_t)n_cand * n_dir, st)) ||
        (s = ctx->rf_aux.ensure(8 * aux.size(), st)))
        return s;
    fh_peakmap sub(*pm);
    sub.d_offsets = (int64_t *)ctx->rf_offsets.ptr;
    sub.d_bins = (int32_t *)ctx->rf_bins.ptr;
    sub.d_t = (double *)ctx->rf_t.ptr;
    sub.d_v = (double *)ctx->rf_v.ptr;
    sub.n_peaks = cap;
    sub.k_min = kmin;
    sub.k_max = kmax;
    sub.max_per_fft = std::min<int32_t>(pm->max_per_fft, width);
    for (int c = 0; c < n_cand; ++c)
        if ((s = check_grid(&sub, &grids[c]))) return s;
    HIP_OK(hipMemcpyAsync(sub.d_t, pm->d_t, 8 * (size_t)N, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(sub.d_v, pm->d_v, 24 * (size_t)N, hipMemcpyDeviceToDevice, st));
    const bool weighted = d_w != nullptr;
    const Plan p = make_plan(grids[0], choose_tile_bins(ctx, &sub, &grids[0], 0));
    ChunkBufs b;
    if ((s = ensure_workspace(ctx, &sub, &grids[0], p, n_dir, n_cand * n_dir, weighted, st, b))) return s;
    if ((s = upload_sky(ctx, sky.data(), n_cand * n_dir, b, st))) return s;
    // the auxiliary arrays go through the (now idle) pinned sky buffer
    if ((s = ctx->cur->h_sky.ensure(8 * aux.size(), st))) return s;
    HIP_OK(hipStreamSynchronize(st));
    std::memcpy(ctx->cur->h_sky.ptr, aux.data(), 8 * aux.size());
    HIP_OK(hipMemcpyAsync(ctx->rf_aux.ptr, ctx->cur->h_sky.ptr, 8 * aux.size(), hipMemcpyHostToDevice, st));
    fh_select sel{nf, nf, -1, o->theta};
    fh_candidate *dc = (fh_candidate *)ctx->rf_cands.ptr;
    for (int c = 0; c < n_cand; ++c) {
        HIP_OK(launch_slice(N, pm->d_offsets, pm->d_bins, klo[c], khi[c], (int64_t *)ctx->rf_first.ptr,
                            (int32_t *)ctx->rf_counts.ptr, sub.d_offsets, sub.d_bins, st));
        ChunkBufs bc = b;
        bc.sky = b.sky + 3 * (int64_t)c * n_dir;
        if ((s = run_search(ctx, &sub, &grids[c], p, n_dir, n_dir, d_w, 0, FH_SCHED_PERSISTENT, &sel,
                            dc + 2 * (int64_t)c * n_dir, bc, st)))
            return s;
    }
    const double *daux = (const double *)ctx->rf_aux.ptr;
    HIP_OK(launch_refine_pick(n_cand, n_dir, dc, daux, daux + 4 * (size_t)n_cand, d_out, st));
    return FH_OK;
}


// ---- peakmap cleaning ----

fh_status fh_gross_histogram(fh_ctx *ctx, const fh_peakmap *pm, const fh_gross *geo, int32_t *d_hist,
                             void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (!pm) return fail(FH_E_INVALID, "peakmap is NULL");
    if ((s = check_gross(geo))) return s;
    if (!d_hist) return fail(FH_E_INVALID, "histogram pointer is NULL");
    HIP_OK(launch_gross_hist(pm->n_fft, pm->d_offsets, pm->d_bins, pm->d_t, pm->t_fft, *geo, d_hist,
                             (hipStream_t)stream));
    return FH_OK;
}

fh_status fh_clean_gross(fh_ctx *ctx, const fh_peakmap *pm, const fh_gross *geo, double threshold,
                         int32_t *d_hist, void *stream, fh_peakmap **out) {
    fh_status s;
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    *out = nullptr;
    if (std::isnan(threshold)) return fail(FH_E_INVALID, "threshold is NaN");
    if ((s = fh_gross_histogram(ctx, pm, geo, d_hist, stream))) return s;
    FilterSpec f{};
    f.mode = 0;
    f.t = pm->d_t;
    f.t_fft = pm->t_fft;
    f.geo = *geo;
    f.hist = d_hist;
    f.thr = threshold;
    return filter_peakmap(ctx, pm, f, (hipStream_t)stream, out);
}

fh_status fh_bin_counts(fh_ctx *ctx, const fh_peakmap *pm, int32_t k_lo, int32_t k_hi, int32_t *d_counts,
                        void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (!pm) return fail(FH_E_INVALID, "peakmap is NULL");
    if (k_lo < 0 || k_hi <= k_lo) return fail(FH_E_INVALID, "need 0 <= k_lo < k_hi");
    if (!d_counts) return fail(FH_E_INVALID, "counts pointer is NULL");
    HIP_OK(launch_bin_counts(pm->n_fft, pm->d_offsets, pm->d_bins, k_lo, k_hi, d_counts, (hipStream_t)stream));
    return FH_OK;
}

fh_status fh_robust_stats(fh_ctx *ctx, const int32_t *d_x, int32_t n, int32_t x_max, double out[2],
                          void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (!d_x || !out) return fail(FH_E_INVALID, "data or output pointer is NULL");
    if (n < 1) return fail(FH_E_INVALID, "robust statistic of %d values", n);
    if (x_max < 0 || x_max > (1 << 28)) return fail(FH_E_INVALID, "x_max=%d outside 0..2^28", x_max);
    hipStream_t st = (hipStream_t)stream;
    if ((s = ctx->cl_hist.ensure(4 * (2 * (size_t)x_max + 1), st)) || (s = ctx->cl_s2.ensure(8, st)) ||
        (s = ctx->cl_out.ensure(16, st)) || (s = ctx->err.ensure(4, st)))
        return s;
    int32_t *err = (int32_t *)ctx->err.ptr;
    HIP_OK(launch_fill_i32(err, 1, 0, st));
    HIP_OK(launch_robust(d_x, n, x_max, (int32_t *)ctx->cl_hist.ptr, (int64_t *)ctx->cl_s2.ptr,
                         (double *)ctx->cl_out.ptr, err, st));
    int32_t h_err = 0;
    double h_out[2];
    HIP_OK(hipMemcpyAsync(&h_err, err, 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(h_out, ctx->cl_out.ptr, 16, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (h_err) return fail(FH_E_INVALID, "a value lies outside [0, x_max=%d]", x_max);
    out[0] = h_out[0];
    out[1] = h_out[1];
    return FH_OK;
}

fh_status fh_line_counts(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, int32_t *d_out, void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if ((s = check_grid(pm, g))) return s;
    if (!d_out) return fail(FH_E_INVALID, "output pointer is NULL");
    hipStream_t st = (hipStream_t)stream;
    const Plan p = make_plan(*g, choose_tile_bins(ctx, pm, g, 0));
    ChunkBufs b;
    if ((s = ensure_workspace(ctx, pm, g, p, 1, 1, false, st, b))) return s;
    const double zero[3] = {0.0, 0.0, 0.0};  // v . n = 0: no Doppler correction
    if ((s = upload_sky(ctx, zero, 1, b, st))) return s;
    if ((s = run_search(ctx, pm, g, p, 1, 1, nullptr, 0, FH_SCHED_PERSISTENT, nullptr, nullptr, b, st))) return s;
    HIP_OK(launch_colmax_values(b.colmax, g->nf, d_out, st));
    return FH_OK;
}

fh_status fh_veto_bins(fh_ctx *ctx, const fh_peakmap *pm, int32_t k_lo, int32_t k_hi, const int32_t *d_x,
                       int64_t n_x, int32_t step, int64_t offset, double threshold, void *stream,
                       fh_peakmap **out) {
    fh_status s;
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    *out = nullptr;
    if ((s = check_ctx(ctx))) return s;
    if (!pm) return fail(FH_E_INVALID, "peakmap is NULL");
    if (k_lo < 0 || k_hi <= k_lo) return fail(FH_E_INVALID, "need 0 <= k_lo < k_hi");
    if (!d_x || n_x < 1) return fail(FH_E_INVALID, "statistic array is NULL or empty");
    if (std::isnan(threshold)) return fail(FH_E_INVALID, "threshold is NaN");
    FilterSpec f{};
    f.mode = 1;
    f.k_lo = k_lo;
    f.k_hi = k_hi;
    f.step = step;
    f.offset = offset;
    f.n_x = n_x;
    f.x = d_x;
    f.thr = threshold;
    return filter_peakmap(ctx, pm, f, (hipStream_t)stream, out);
}

fh_status fh_plan_query(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, int32_t tile_bins,
                        fh_plan_info *out) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if ((s = check_grid(pm, g))) return s;
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    if (tile_bins < 0) return fail(FH_E_INVALID, "tile_bins < 0");
    const Plan p = make_plan(*g, choose_tile_bins(ctx, pm, g, tile_bins));
    out->tile_rows = kTileRows;
    out->tile_bins = p.W;
    out->n_row_blocks = p.nrb;
    out->n_bin_blocks = p.nbb;
    out->workspace_bytes = edge_bytes_per_sky(ctx, pm) + 16 * (int64_t)p.nrbg * p.nbb * win_stride(pm->n_fft) +
                           8 * (int64_t)g->nf + 4 * (int64_t)pm->n_fft + 4 * p.tiles_per_sky +
                           (int64_t)shift_layout(pm->n_fft, p.nrb_tab, p.nrbg).total;
    out->cell_updates = pm->n_peaks * (int64_t)g->ns;
    return FH_OK;
}

fh_status fh_hough_map_i32(fh_ctx *ctx, const fh_peakmap *pm, const double nhat[3],
                           const fh_grid *grid, int32_t *d_map, void *stream) {
    return hough_map_common(ctx, pm, nhat, nullptr, grid, d_map, stream);
}

fh_status fh_hough_map_f32(fh_ctx *ctx, const fh_peakmap *pm, const double nhat[3],
                           const float *d_w, const fh_grid *grid, float *d_map, void *stream) {
    if (!d_w) return fail(FH_E_INVALID, "weights pointer is NULL");
    return hough_map_common(ctx, pm, nhat, d_w, grid, d_map, stream);
}

}  // extern "C"

namespace {

// Pieces of the unweighted map path carved out of `scratch` (256-byte aligned
// byte offsets).  Every piece a kernel reads is written earlier in the same
// call (edges, their padding, every window entry including the padding FFTs,
// the shift table and the direction), so nothing has to start at zero; the
// error flag and the queue counters are only read on paths this call does not
// take (weights, the persistent schedule).
struct StaticLayout {
    size_t sky, err, qctr, sht, y, y64, win, wsort, total;
    ShiftLayout shl;
};

StaticLayout static_layout(const fh_ctx *ctx, const fh_peakmap *pm, const Plan &p) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t ys = (size_t)y_stride(pm->n_peaks, pm->n_fft);
    const size_t wins = (size_t)8 * p.nrbg * p.nbb * win_stride(pm->n_fft);
    StaticLayout L{};
    size_t o = 0;
    L.sky = o;   o += al(24);
    L.err = o;   o += al(4);
    L.qctr = o;  o += al(4 * kXcds);
    L.shl = shift_layout(pm->n_fft, p.nrb_tab, p.nrbg);
    L.sht = o;   o += L.shl.total;
    L.y = o;     o += al(4 * ys);
    L.y64 = o;   if (needs_full_edges(ctx, pm)) o += al(8 * ys);
    L.win = o;   o += al(wins);
    L.wsort = o; o += al(wins);
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

fh_status fh_hough_map_i32_static(fh_ctx *ctx, const fh_peakmap *pm, const double nhat[3],
                                  const fh_grid *g, int32_t *d_map, void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if ((s = check_grid(pm, g))) return s;
    if ((s = check_sky(nhat))) return s;
    if (!d_map) return fail(FH_E_INVALID, "output map pointer is NULL");
    hipStream_t st = (hipStream_t)stream;
    const Plan p = make_plan(*g, choose_tile_bins(ctx, pm, g, 0));
    const StaticLayout L = static_layout(ctx, pm, p);
    if (L.total > kStaticScratchBytes)
        return fail(FH_E_UNSUPPORTED, "this map needs %zu bytes of scratch; the static scratch holds %zu",
                    L.total, kStaticScratchBytes);
    void *base = ctx->device < kMaxDevices ? g_scratch_ptr[ctx->device] : nullptr;
    if (!base) return fail(FH_E_UNSUPPORTED, "no static scratch on device %d", ctx->device);
    char *c = static_cast<char *>(base);
    ChunkBufs b{};
    b.sky = reinterpret_cast<double *>(c + L.sky);
    b.err = reinterpret_cast<int32_t *>(c + L.err);
    b.qctr = reinterpret_cast<int32_t *>(c + L.qctr);
    b.colmax = reinterpret_cast<unsigned long long *>(c + L.qctr);  // not written by the map path
    b.gwin = reinterpret_cast<int64_t *>(c + L.sht + L.shl.gwin);
    b.rec = reinterpret_cast<uint2 *>(c + L.sht + L.shl.rec);
    b.step = reinterpret_cast<uint32_t *>(c + L.sht + L.shl.step);
    b.Y = reinterpret_cast<uint32_t *>(c + L.y);
    b.Y64 = reinterpret_cast<int64_t *>(c + L.y64);
    b.win = reinterpret_cast<int2 *>(c + L.win);
    b.wsort = reinterpret_cast<int2 *>(c + L.wsort);
    HIP_OK(launch_set_f64x3(b.sky, nhat[0], nhat[1], nhat[2], st));
    // no profiling spans here: recording one can create an event
    const bool was = ctx->profiling;
    ctx->profiling = false;
    s = enqueue_map(ctx, pm, g, p, nullptr, b, d_map, st);
    ctx->profiling = was;
    return s;
}

fh_status fh_hough_candidates(fh_ctx *ctx, const fh_peakmap *pm, int32_t n_sky, const double *sky,
                              const float *d_w, int32_t w_stride, const fh_grid *g,
                              const fh_select *sel, const fh_options *opts, fh_candidate *d_out,
                              void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if ((s = check_grid(pm, g))) return s;
    if (n_sky < 1) return fail(FH_E_INVALID, "n_sky=%d < 1", n_sky);
    if (!sky) return fail(FH_E_INVALID, "sky is NULL");
    for (int32_t k = 0; k < n_sky; ++k)
        if ((s = check_sky(sky + 3 * (int64_t)k))) return s;
    if (!sel || sel->width < 1 || sel->excl < 0 || !std::isfinite(sel->theta) || !(sel->theta > 0))
        return fail(FH_E_INVALID, "selection needs width >= 1, excl >= 0, theta > 0");
    if (!d_out) return fail(FH_E_INVALID, "output pointer is NULL");
    if (d_w && w_stride != 0 && w_stride != pm->n_fft)
        return fail(FH_E_INVALID, "w_stride must be 0 or n_fft");
    fh_options o{FH_SCHED_PERSISTENT, 0, 0, 0};
    if (opts) o = *opts;
    if (o.schedule != FH_SCHED_PLAIN && o.schedule != FH_SCHED_PERSISTENT)
        return fail(FH_E_INVALID, "unknown schedule %d", o.schedule);
    if (o.tile_bins < 0 || o.sky_chunk < 0) return fail(FH_E_INVALID, "negative option");
    hipStream_t st = (hipStream_t)stream;
    const bool weighted = d_w != nullptr;
    if (o.tile_bins == 0 && ctx->tuned.find(tune_key(pm, g)) == ctx->tuned.end())
        if ((s = autotune(ctx, pm, g, n_sky, sky, d_w, w_stride, st))) return s;
    const Plan p = make_plan(*g, choose_tile_bins(ctx, pm, g, o.tile_bins));
    int chunk = o.schedule == FH_SCHED_PLAIN ? 1 : default_chunk(ctx, pm, g, p, o.sky_chunk);
    chunk = std::min(chunk, n_sky);
    ChunkBufs b;
    if ((s = ensure_workspace(ctx, pm, g, p, chunk, n_sky, weighted, st, b))) return s;
    if ((s = upload_sky(ctx, sky, n_sky, b, st))) return s;
    if (!o.use_graph)
        return run_search(ctx, pm, g, p, chunk, n_sky, d_w, w_stride, o.schedule, sel, d_out, b, st);
    if (st == nullptr) return fail(FH_E_INVALID, "use_graph needs a created stream, not the default stream");

    // hipGraph: capture the whole search once, replay it while every argument
    // and workspace pointer it bakes in is unchanged (sky vectors and weights
    // are read from device memory at replay time, so their contents may change).
    auto bits = [](double x) { uint64_t u; std::memcpy(&u, &x, 8); return u; };
    std::vector<uint64_t> key = {
        (uint64_t)(uintptr_t)pm, (uint64_t)g->kf, (uint64_t)g->b0, (uint64_t)g->nf, (uint64_t)g->ns,
        bits(g->fdot0), bits(g->dfdot), bits(g->t0), (uint64_t)sel->width, (uint64_t)(uint32_t)sel->excl,
        (uint64_t)(uint32_t)sel->sep, bits(sel->theta), (uint64_t)o.schedule, (uint64_t)p.W,
        (uint64_t)chunk, (uint64_t)n_sky, (uint64_t)(uintptr_t)d_w, (uint64_t)(uint32_t)w_stride,
        (uint64_t)(uintptr_t)d_out, (uint64_t)(uintptr_t)st, (uint64_t)(uintptr_t)b.Y,
        (uint64_t)(uintptr_t)b.win, (uint64_t)(uintptr_t)b.wsort, (uint64_t)(uintptr_t)b.colmax, (uint64_t)(uintptr_t)b.wq,
        (uint64_t)(uintptr_t)b.ws, (uint64_t)(uintptr_t)b.sky,
        (uint64_t)(uintptr_t)b.gwin,
        (uint64_t)(uintptr_t)b.qctr, (uint64_t)(uintptr_t)b.Y64, (uint64_t)ctx->window_method,
        (uint64_t)ctx->doppler_mode, bits(ctx->doppler_fref)};
    fh_ctx::GraphEntry *ge = nullptr;
    for (auto &e : ctx->graphs)
        if (e.key == key) ge = &e;
    if (!ge) {
        const bool was = ctx->profiling;
        ctx->profiling = false;  // no event records inside the capture
        HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        s = run_search(ctx, pm, g, p, chunk, n_sky, d_w, w_stride, o.schedule, sel, d_out, b, st);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(st, &graph);
        ctx->profiling = was;
        if (s) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess) return fail(FH_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(FH_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        if (ctx->graphs.size() >= 16) {
            (void)hipGraphExecDestroy(ctx->graphs.front().exec);
            (void)hipGraphDestroy(ctx->graphs.front().graph);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back({key, graph, exec});
        ge = &ctx->graphs.back();
    }
    {
        Timed timed(ctx, st, kSpanGraph);
        HIP_OK(hipGraphLaunch(ge->exec, st));
    }
    if (ctx->profiling) ctx->prof_updates += pm->n_peaks * (int64_t)g->ns * n_sky;
    return FH_OK;
}

fh_status fh_hough_colmax(fh_ctx *ctx, const fh_peakmap *pm, int32_t n_sky, const double *sky, const float *d_w,
                          int32_t w_stride, const fh_grid *g, const fh_options *opts, float *d_value,
                          int32_t *d_row, void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if ((s = check_grid(pm, g))) return s;
    if (n_sky < 1) return fail(FH_E_INVALID, "n_sky=%d < 1", n_sky);
    if (!sky) return fail(FH_E_INVALID, "sky is NULL");
    for (int32_t k = 0; k < n_sky; ++k)
        if ((s = check_sky(sky + 3 * (int64_t)k))) return s;
    if (!d_value || !d_row) return fail(FH_E_INVALID, "output pointer is NULL");
    if (d_w && w_stride != 0 && w_stride != pm->n_fft)
        return fail(FH_E_INVALID, "w_stride must be 0 or n_fft");
    fh_options o{FH_SCHED_PERSISTENT, 0, 0, 0};
    if (opts) o = *opts;
    if (o.schedule != FH_SCHED_PLAIN && o.schedule != FH_SCHED_PERSISTENT)
        return fail(FH_E_INVALID, "unknown schedule %d", o.schedule);
    if (o.tile_bins < 0 || o.sky_chunk < 0) return fail(FH_E_INVALID, "negative option");
    hipStream_t st = (hipStream_t)stream;
    const bool weighted = d_w != nullptr;
    if (o.tile_bins == 0 && ctx->tuned.find(tune_key(pm, g)) == ctx->tuned.end())
        if ((s = autotune(ctx, pm, g, n_sky, sky, d_w, w_stride, st))) return s;
    const Plan p = make_plan(*g, choose_tile_bins(ctx, pm, g, o.tile_bins));
    int chunk = o.schedule == FH_SCHED_PLAIN ? 1 : default_chunk(ctx, pm, g, p, o.sky_chunk);
    chunk = std::min(chunk, n_sky);
    ChunkBufs b;
    if ((s = ensure_workspace(ctx, pm, g, p, chunk, n_sky, weighted, st, b))) return s;
    if ((s = upload_sky(ctx, sky, n_sky, b, st))) return s;
    ColmaxOut cm;
    cm.value = d_value;
    cm.row = d_row;
    return run_search(ctx, pm, g, p, chunk, n_sky, d_w, w_stride, o.schedule, nullptr, nullptr, b, st, cm);
}

fh_status fh_ctx_profile(fh_ctx *ctx, int32_t enable) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (enable) {
        HIP_OK(hipDeviceSynchronize());
        ctx->spans.clear();
        ctx->ev_used = 0;
        ctx->prof_updates = 0;
    }
    ctx->profiling = enable != 0;
    return FH_OK;
}

fh_status fh_ctx_profile_read(fh_ctx *ctx, fh_profile *out) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    HIP_OK(hipDeviceSynchronize());
    fh_profile p{};
    for (const auto &sp : ctx->spans) {
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, sp.a, sp.b));
        if (sp.kind == kSpanTiles) { p.tiles_ms += ms; p.tiles_launches++; }
        else if (sp.kind == kSpanFront) { p.front_ms += ms; p.front_launches++; }
        else if (sp.kind == kSpanGraph) { p.graph_ms += ms; p.graph_launches++; }
        else { p.select_ms += ms; p.select_launches++; }
    }
    p.cell_updates = ctx->prof_updates;
    *out = p;
    return FH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// continuous-batching server

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Byte layout of one search's workspace inside a block of the server's
// arena: the same buffers ensure_workspace provides, 256-byte aligned.
struct SearchLayout {
    size_t sht = 0, y = 0, y64 = 0, win = 0, wsort = 0, colmax = 0, wq = 0, ws = 0, sky = 0, qctr = 0, total = 0;
    ShiftLayout shl{};
};

SearchLayout search_layout(const fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p, int chunk,
                           int n_sky, bool weighted) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t N = (size_t)pm->n_fft, c = (size_t)chunk;
    const size_t ys = (size_t)y_stride(pm->n_peaks, pm->n_fft);
    const size_t wins = (size_t)8 * c * p.nrbg * p.nbb * win_stride(pm->n_fft);
    SearchLayout L;
    size_t o = 0;
    L.shl = shift_layout((int64_t)N, p.nrb_tab, p.nrbg);
    L.sht = o;    o += L.shl.total;
    L.y = o;      o += al(4 * ys * c);
    L.y64 = o;    if (needs_full_edges(ctx, pm)) o += al(8 * ys * c);
    L.win = o;    o += al(wins);
    L.wsort = o;  o += al(wins);
    L.colmax = o; o += al(8 * c * (size_t)g->nf);
    L.wq = o;     o += al(weighted ? 4 * c * N : 4);
    L.ws = o;     o += al(sizeof(WeightStats) * c);
    L.sky = o;    o += al(24 * (size_t)n_sky);
    L.qctr = o;   o += al(4 * kXcds);
    L.total = o;
    return L;
}

ChunkBufs carve(char *base, const SearchLayout &L, int32_t *err) {
    ChunkBufs b{};
    b.gwin = reinterpret_cast<int64_t *>(base + L.sht + L.shl.gwin);
    b.rec = reinterpret_cast<uint2 *>(base + L.sht + L.shl.rec);
    b.step = reinterpret_cast<uint32_t *>(base + L.sht + L.shl.step);
    b.Y = reinterpret_cast<uint32_t *>(base + L.y);
    b.Y64 = reinterpret_cast<int64_t *>(base + L.y64);
    b.win = reinterpret_cast<int2 *>(base + L.win);
    b.wsort = reinterpret_cast<int2 *>(base + L.wsort);
    b.colmax = reinterpret_cast<unsigned long long *>(base + L.colmax);
    b.wq = reinterpret_cast<uint32_t *>(base + L.wq);
    b.ws = reinterpret_cast<WeightStats *>(base + L.ws);
    b.sky = reinterpret_cast<double *>(base + L.sky);
    b.qctr = reinterpret_cast<int32_t *>(base + L.qctr);
    b.err = err;
    return b;
}

// First-fit allocator over the server's device arena (host bookkeeping
// only; block sizes are multiples of 256 bytes).
struct Arena {
    char *base = nullptr;
    size_t bytes = 0;
    std::map<size_t, size_t> free_;  // offset -> size, never adjacent
    void reset(char *p, size_t n) {
        base = p;
        bytes = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, o2 = it->first + n;
            free_.erase(it);
            if (rest) free_[o2] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + n == nx->first) {  // merge with the next block
            n += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {  // merge with the previous block
                pv->second += n;
                return;
            }
        }
        free_[off] = n;
    }
};

struct ServerRequest {
    uint64_t id = 0;
    fh_request r{};
    std::vector<double> sky;
    Clock::time_point t_submit, t_admit;
    SearchLayout layout;
    int64_t footprint = 0;
    size_t arena_off = 0;
    int32_t chunk = 1;
    int32_t W = 64;
    int32_t lane = -1;
    int32_t status = FH_OK;
    double device_ms = 0.0, latency_ms = 0.0, queue_ms = 0.0;
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t ev_start = nullptr, ev_done = nullptr;
    uint64_t req = 0;  // 0 = idle
};

}  // namespace

struct fh_server {
    fh_ctx *ctx = nullptr;
    int64_t budget = 0;
    Arena arena;  // budget bytes of device memory, allocated once at creation
    int32_t max_queue = 0;
    std::vector<Lane> lanes;
    std::deque<uint64_t> queue;
    std::map<uint64_t, ServerRequest> reqs;  // queued, running, finished-unreported
    std::deque<uint64_t> finished;
    uint64_t next_id = 1;
    int64_t in_flight = 0;
};

namespace {

void retire_lanes(fh_server *srv) {
    for (size_t li = 0; li < srv->lanes.size(); ++li) {
        Lane &L = srv->lanes[li];
        if (!L.req) continue;
        hipError_t q = hipEventQuery(L.ev_done);
        if (q == hipErrorNotReady) continue;
        ServerRequest &R = srv->reqs[L.req];
        const Clock::time_point now = Clock::now();
        if (q != hipSuccess) {
            R.status = FH_E_DEVICE;
        } else {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, L.ev_start, L.ev_done) == hipSuccess) R.device_ms = ms;
        }
        R.latency_ms = ms_between(R.t_submit, now);
        srv->arena.release(R.arena_off, (size_t)R.footprint);
        srv->in_flight -= R.footprint;
        srv->finished.push_back(R.id);
        L.req = 0;
    }
}

void admit(fh_server *srv) {
    fh_ctx *ctx = srv->ctx;
    while (!srv->queue.empty()) {
        const uint64_t id = srv->queue.front();
        ServerRequest &R = srv->reqs[id];
        int li = -1;
        for (size_t k = 0; k < srv->lanes.size(); ++k)
            if (!srv->lanes[k].req) { li = (int)k; break; }
        if (li < 0) break;  // wait for a lane
        // arrival order: the head waits until a block of its footprint is free
        size_t off = 0;
        if (!srv->arena.alloc((size_t)R.footprint, &off)) break;
        srv->queue.pop_front();
        Lane &L = srv->lanes[li];
        R.lane = li;
        R.arena_off = off;
        R.t_admit = Clock::now();
        R.queue_ms = ms_between(R.t_submit, R.t_admit);
        const fh_request &q = R.r;
        const Plan p = make_plan(q.grid, R.W);
        // the workspace is the arena block: nothing is allocated or freed here
        ChunkBufs b = carve(srv->arena.base + off, R.layout, (int32_t *)ctx->err.ptr);
        fh_status s = FH_OK;
        if (hipMemcpyAsync(b.sky, R.sky.data(), (size_t)24 * q.n_sky, hipMemcpyHostToDevice, L.st) != hipSuccess)
            s = fail(FH_E_DEVICE, "copying the request's sky vectors failed");
        if (!s && hipEventRecord(L.ev_start, L.st) != hipSuccess) s = fail(FH_E_DEVICE, "hipEventRecord");
        if (!s)
            s = run_search(ctx, q.pm, &q.grid, p, R.chunk, q.n_sky, q.d_w, q.w_stride,
                           FH_SCHED_PERSISTENT, &q.sel, q.d_out, b, L.st);
        if (hipEventRecord(L.ev_done, L.st) != hipSuccess && !s) s = fail(FH_E_DEVICE, "hipEventRecord");
        R.status = s;
        srv->in_flight += R.footprint;
        L.req = id;
    }
}

}  // namespace

extern "C" {

fh_status fh_server_create(fh_ctx *ctx, int64_t hbm_budget, int32_t lanes, int32_t max_queue,
                           fh_server **out) {
    fh_status s;
    if (!out) return fail(FH_E_INVALID, "out is NULL");
    *out = nullptr;
    if ((s = check_ctx(ctx))) return s;
    if (hbm_budget <= 0) return fail(FH_E_INVALID, "hbm_budget must be > 0");
    if (lanes < 1 || lanes > 16) return fail(FH_E_INVALID, "lanes=%d outside 1..16", lanes);
    if (max_queue < 1) return fail(FH_E_INVALID, "max_queue must be >= 1");
    // the arena is carved in 256-byte pieces
    const int64_t budget = hbm_budget / 256 * 256;
    if (budget <= 0) return fail(FH_E_INVALID, "hbm_budget must be at least 256 bytes");
    void *mem = nullptr;
    if (hipMalloc(&mem, (size_t)budget) != hipSuccess)
        return fail(FH_E_NOMEM, "allocating the server's %lld-byte arena failed", (long long)budget);
    fh_server *srv = new fh_server();
    srv->ctx = ctx;
    srv->budget = budget;
    srv->arena.reset(static_cast<char *>(mem), (size_t)budget);
    srv->max_queue = max_queue;
    srv->lanes.resize(lanes);
    for (Lane &L : srv->lanes) {
        if (hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&L.ev_start) != hipSuccess || hipEventCreate(&L.ev_done) != hipSuccess) {
            fh_server_destroy(srv);
            return fail(FH_E_DEVICE, "creating the server's streams failed");
        }
    }
    *out = srv;
    return FH_OK;
}

fh_status fh_server_submit(fh_server *srv, const fh_request *req, uint64_t *id) {
    fh_status s;
    if (!srv) return fail(FH_E_INVALID, "server is NULL");
    if (!req || !id) return fail(FH_E_INVALID, "request or id is NULL");
    fh_ctx *ctx = srv->ctx;
    if ((s = check_ctx(ctx))) return s;
    if ((s = check_grid(req->pm, &req->grid))) return s;
    if (req->n_sky < 1 || !req->sky) return fail(FH_E_INVALID, "request needs n_sky >= 1 and sky");
    for (int32_t k = 0; k < req->n_sky; ++k)
        if ((s = check_sky(req->sky + 3 * (int64_t)k))) return s;
    const fh_select &sel = req->sel;
    if (sel.width < 1 || sel.excl < 0 || !std::isfinite(sel.theta) || !(sel.theta > 0))
        return fail(FH_E_INVALID, "selection needs width >= 1, excl >= 0, theta > 0");
    if (!req->d_out) return fail(FH_E_INVALID, "output pointer is NULL");
    if (req->d_w && req->w_stride != 0 && req->w_stride != req->pm->n_fft)
        return fail(FH_E_INVALID, "w_stride must be 0 or n_fft");
    if ((int32_t)srv->queue.size() >= srv->max_queue) return fail(FH_E_BUSY, "request queue is full");
    ServerRequest R;
    R.id = srv->next_id++;
    R.r = *req;
    R.sky.assign(req->sky, req->sky + 3 * (int64_t)req->n_sky);
    R.r.sky = nullptr;
    R.t_submit = Clock::now();
    R.W = choose_tile_bins(ctx, req->pm, &req->grid, 0);
    const Plan p = make_plan(req->grid, R.W);
    // the largest chunk whose footprint fits one lane's share of the budget
    const bool weighted = req->d_w != nullptr;
    const int64_t share = srv->budget / (int64_t)srv->lanes.size();
    int chunk = (int)std::min<int64_t>(std::min<int>(req->n_sky, 256), chunk_by_tiles(p));
    while (chunk > 1 &&
           (int64_t)search_layout(ctx, req->pm, &req->grid, p, chunk, req->n_sky, weighted).total > share)
        chunk = (chunk + 1) / 2;
    R.chunk = chunk;
    R.layout = search_layout(ctx, req->pm, &req->grid, p, chunk, req->n_sky, weighted);
    R.footprint = (int64_t)R.layout.total;
    if (R.footprint > srv->budget) {
        srv->next_id--;
        return fail(FH_E_UNSUPPORTED, "request needs %lld workspace bytes, over the %lld-byte budget",
                    (long long)R.footprint, (long long)srv->budget);
    }
    *id = R.id;
    srv->reqs[R.id] = std::move(R);
    srv->queue.push_back(*id);
    return FH_OK;
}

fh_status fh_server_poll(fh_server *srv, fh_completion *out, int32_t max, int32_t *n) {
    fh_status s;
    if (!srv || !n) return fail(FH_E_INVALID, "server or n is NULL");
    *n = 0;
    if (max > 0 && !out) return fail(FH_E_INVALID, "out is NULL");
    if ((s = check_ctx(srv->ctx))) return s;
    retire_lanes(srv);
    admit(srv);
    int32_t k = 0;
    while (k < max && !srv->finished.empty()) {
        const uint64_t id = srv->finished.front();
        srv->finished.pop_front();
        const ServerRequest &R = srv->reqs[id];
        fh_completion c{};
        c.id = R.id;
        c.tag = R.r.tag;
        c.status = R.status;
        c.lane = R.lane;
        c.queue_ms = R.queue_ms;
        c.latency_ms = R.latency_ms;
        c.device_ms = R.device_ms;
        c.footprint = R.footprint;
        c.cell_updates = R.r.pm->n_peaks * (int64_t)R.r.grid.ns * R.r.n_sky;
        out[k++] = c;
        srv->reqs.erase(id);
    }
    *n = k;
    return FH_OK;
}

fh_status fh_server_cancel(fh_server *srv, uint64_t id) {
    if (!srv) return fail(FH_E_INVALID, "server is NULL");
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) return fail(FH_E_INVALID, "unknown request id %llu", (unsigned long long)id);
    for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q) {
        if (*q == id) {
            srv->queue.erase(q);
            it->second.status = FH_E_CANCELLED;
            it->second.latency_ms = ms_between(it->second.t_submit, Clock::now());
            srv->finished.push_back(id);
            return FH_OK;
        }
    }
    for (const Lane &L : srv->lanes)
        if (L.req == id) return fail(FH_E_BUSY, "request %llu is running", (unsigned long long)id);
    return fail(FH_E_INVALID, "request %llu has finished", (unsigned long long)id);
}

fh_status fh_server_stats(const fh_server *srv, int32_t *queued, int32_t *running, int32_t *finished,
                          int64_t *bytes_in_flight) {
    if (!srv) return fail(FH_E_INVALID, "server is NULL");
    int32_t r = 0;
    for (const Lane &L : srv->lanes) r += L.req ? 1 : 0;
    if (queued) *queued = (int32_t)srv->queue.size();
    if (running) *running = r;
    if (finished) *finished = (int32_t)srv->finished.size();
    if (bytes_in_flight) *bytes_in_flight = srv->in_flight;
    return FH_OK;
}

fh_status fh_server_drain(fh_server *srv) {
    fh_status s;
    if (!srv) return fail(FH_E_INVALID, "server is NULL");
    if ((s = check_ctx(srv->ctx))) return s;
    // admit and run everything accepted; completions stay for fh_server_poll
    for (;;) {
        retire_lanes(srv);
        admit(srv);
        bool busy = !srv->queue.empty();
        for (const Lane &L : srv->lanes) busy = busy || L.req != 0;
        if (!busy) return FH_OK;
        for (const Lane &L : srv->lanes)
            if (L.req) HIP_OK(hipEventSynchronize(L.ev_done));
    }
}

void fh_server_destroy(fh_server *srv) {
    if (!srv) return;
    if (srv->ctx) (void)hipSetDevice(srv->ctx->device);
    // run everything that was accepted, then release
    fh_server_drain(srv);
    for (Lane &L : srv->lanes) {
        if (L.st) (void)hipStreamSynchronize(L.st);
        if (L.ev_start) (void)hipEventDestroy(L.ev_start);
        if (L.ev_done) (void)hipEventDestroy(L.ev_done);
        if (L.st) (void)hipStreamDestroy(L.st);
    }
    if (srv->arena.base) (void)hipFree(srv->arena.base);
    delete srv;
}

}  // extern "C"
