// Host runtime of the frequency-Hough library: contexts, device-resident
// peakmaps, validation, tile planning, workspace management and the launch
// sequences behind the C ABI of include/fh.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "fh_internal.h"

using namespace fh;

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
            hipFree(ptr);
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
        if (ptr) hipFree(ptr);
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
            hipHostFree(ptr);
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
        if (ptr) hipHostFree(ptr);
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

struct fh_ctx {
    int32_t device = 0;
    int32_t n_cu = 256;
    // workspaces
    DevBuf g0, dg, Y, win, colmax, wq, ws, sky, order, qstart, qctr, err;
    PinnedBuf h_sky, h_order;
    // autotuned tile width per problem shape
    std::map<std::tuple<int, int, int, int, int>, int> tuned;
    // event-based timing (fh_ctx_profile)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Span { hipEvent_t a, b; int kind; };
    std::vector<Span> spans;
    int64_t prof_updates = 0;
};

namespace {

struct Plan {
    int W, nrb, nbb, nrbg;
    int64_t tiles_per_sky;
};

Plan make_plan(const fh_grid &g, int W) {
    Plan p;
    p.W = W;
    p.nrb = (g.ns + kTileRows - 1) / kTileRows;
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

int choose_tile_bins(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, int requested) {
    const int wmax = max_tile_bins(g->kf);
    if (requested > 0) return std::min(((requested + 63) / 64) * 64, wmax);
    auto key = std::make_tuple(pm->n_fft, g->nf, g->ns, g->kf, 0);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second;
    // a tile never needs to be wider than the map
    int w = std::min(wmax, ((g->nf + 63) / 64) * 64);
    return std::max(64, w);
}

// kinds of timed spans
enum { kSpanFront = 0, kSpanTiles = 1, kSpanSelect = 2 };

hipEvent_t next_event(fh_ctx *ctx) {
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ctx->ev_used++];
}

// Records an event before a group of launches and another after it.
struct Timed {
    fh_ctx *ctx;
    hipStream_t st;
    int kind;
    hipEvent_t a = nullptr;
    Timed(fh_ctx *c, hipStream_t s, int k) : ctx(c), st(s), kind(k) {
        if (ctx->profiling) {
            a = next_event(ctx);
            if (a) hipEventRecord(a, st);
        }
    }
    ~Timed() {
        if (a) {
            hipEvent_t b = next_event(ctx);
            if (b) {
                hipEventRecord(b, st);
                ctx->spans.push_back({a, b, kind});
            }
        }
    }
};

struct ChunkBufs {
    int64_t *g0, *dg, *Y;
    int2 *win;
    unsigned long long *colmax;
    uint32_t *wq;
    WeightStats *ws;
    double *sky;
    int32_t *order, *qstart, *qctr, *err;
};

fh_status ensure_workspace(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p,
                           int slots, bool weighted, hipStream_t st, ChunkBufs &b) {
    const int64_t N = pm->n_fft;
    fh_status s;
    if ((s = ctx->g0.ensure(8 * N, st))) return s;
    if ((s = ctx->dg.ensure(8 * N, st))) return s;
    // the tile kernels read up to 15 stripe edges past a window's end
    if ((s = ctx->Y.ensure((size_t)8 * (std::max<int64_t>(1, pm->n_peaks) * slots + 16), st))) return s;
    if ((s = ctx->win.ensure((size_t)8 * slots * p.nrbg * p.nbb * N, st))) return s;
    if ((s = ctx->colmax.ensure((size_t)8 * slots * g->nf, st))) return s;
    if ((s = ctx->wq.ensure(weighted ? (size_t)4 * slots * N : 4, st))) return s;
    if ((s = ctx->ws.ensure(sizeof(WeightStats) * (size_t)slots, st))) return s;
    if ((s = ctx->sky.ensure((size_t)24 * slots, st))) return s;
    if ((s = ctx->order.ensure((size_t)4 * p.tiles_per_sky * slots, st))) return s;
    if ((s = ctx->qstart.ensure(4 * (kXcds + 1), st))) return s;
    if ((s = ctx->qctr.ensure(4 * kXcds, st))) return s;
    if ((s = ctx->err.ensure(4, st))) return s;
    b.g0 = (int64_t *)ctx->g0.ptr;
    b.dg = (int64_t *)ctx->dg.ptr;
    b.Y = (int64_t *)ctx->Y.ptr;
    b.win = (int2 *)ctx->win.ptr;
    b.colmax = (unsigned long long *)ctx->colmax.ptr;
    b.wq = (uint32_t *)ctx->wq.ptr;
    b.ws = (WeightStats *)ctx->ws.ptr;
    b.sky = (double *)ctx->sky.ptr;
    b.order = (int32_t *)ctx->order.ptr;
    b.qstart = (int32_t *)ctx->qstart.ptr;
    b.qctr = (int32_t *)ctx->qctr.ptr;
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
    a.nbb = p.nbb;
    a.nrbg = p.nrbg;
    a.n_slots = slots;
    a.Y = b.Y;
    a.win = b.win;
    a.dg = b.dg;
    a.wq = weighted ? b.wq : nullptr;
    a.ws = weighted ? b.ws : nullptr;
    a.ws_stride = ws_stride;
    a.colmax = b.colmax;
    a.order = b.order;
    a.queue_start = b.qstart;
    a.queue_ctr = b.qctr;
    return a;
}

// Shared front half of every path: shifts, weights, stripe edges, windows.
fh_status enqueue_front(fh_ctx *ctx, const fh_peakmap *pm, const fh_grid *g, const Plan &p,
                        int slots, const double *sky_host, const float *d_w, int w_stride,
                        const ChunkBufs &b, hipStream_t st) {
    fh_status s = ctx->h_sky.ensure((size_t)24 * slots, st);
    if (s) return s;
    // the pinned staging buffer may still feed an earlier copy on this stream
    HIP_OK(hipStreamSynchronize(st));
    std::memcpy(ctx->h_sky.ptr, sky_host, (size_t)24 * slots);
    HIP_OK(hipMemcpyAsync(b.sky, ctx->h_sky.ptr, (size_t)24 * slots, hipMemcpyHostToDevice, st));
    Timed timed(ctx, st, kSpanFront);
    HIP_OK(launch_shifts(pm->n_fft, pm->d_t, g->t0, pm->t_fft, g->kf, g->fdot0, g->dfdot, b.g0, b.dg, st));
    const bool weighted = d_w != nullptr;
    const int n_vec = weighted ? (w_stride == 0 ? 1 : slots) : 0;
    if (weighted)
        HIP_OK(launch_weight_stats(pm->n_fft, n_vec, d_w, w_stride, pm->adjacent ? 2 : 1, b.ws, b.err, st));
    HIP_OK(launch_prep(pm->n_fft, pm->n_peaks, pm->d_offsets, pm->d_bins, pm->d_v, b.sky, slots,
                       g->kf, g->b0, b.g0, b.Y, d_w, w_stride, b.ws, w_stride == 0 ? 0 : 1, b.wq, st));
    HIP_OK(launch_windows(pm->n_fft, pm->d_offsets, b.Y, pm->n_peaks, b.dg, g->ns, p.nrbg, p.nbb,
                          p.W, g->kf, slots, b.win, st));
    return FH_OK;
}

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
    if ((s = ensure_workspace(ctx, pm, g, p, 1, weighted, st, b))) return s;
    if ((s = enqueue_front(ctx, pm, g, p, 1, nhat, d_w, 0, b, st))) return s;
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
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    for (DevBuf *b : {&ctx->g0, &ctx->dg, &ctx->Y, &ctx->win, &ctx->colmax, &ctx->wq, &ctx->ws,
                      &ctx->sky, &ctx->order, &ctx->qstart, &ctx->qctr, &ctx->err})
        b->release();
    ctx->h_sky.release();
    ctx->h_order.release();
    for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
    delete ctx;
}

fh_status fh_ctx_check(fh_ctx *ctx, void *stream) {
    fh_status s;
    if ((s = check_ctx(ctx))) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_OK(hipStreamSynchronize(st));
    int32_t flag = 0;
    HIP_OK(hipMemcpy(&flag, ctx->err.ptr, 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemset(ctx->err.ptr, 0, 4));
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

void fh_peakmap_release(fh_ctx *ctx, fh_peakmap *pm) {
    if (!pm) return;
    if (ctx) hipSetDevice(ctx->device);
    if (pm->d_offsets) hipFree(pm->d_offsets);
    if (pm->d_bins) hipFree(pm->d_bins);
    if (pm->d_t) hipFree(pm->d_t);
    if (pm->d_v) hipFree(pm->d_v);
    delete pm;
}

int64_t fh_peakmap_bytes(const fh_peakmap *pm) { return pm ? pm->bytes : 0; }

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
    out->workspace_bytes = 8 * (int64_t)pm->n_peaks + 8 * (int64_t)p.nrbg * p.nbb * pm->n_fft +
                           8 * (int64_t)g->nf + 4 * (int64_t)pm->n_fft + 4 * p.tiles_per_sky;
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
    const Plan p = make_plan(*g, choose_tile_bins(ctx, pm, g, o.tile_bins));
    // chunk: enough tiles to keep every CU busy, bounded workspace
    int chunk = o.sky_chunk;
    if (chunk == 0) {
        const int64_t per_sky = 8 * pm->n_peaks + 8 * (int64_t)p.nrbg * p.nbb * pm->n_fft + 8 * (int64_t)g->nf;
        const int64_t by_mem = std::max<int64_t>(1, ((int64_t)3 << 30) / std::max<int64_t>(1, per_sky));
        const int64_t by_tiles = std::max<int64_t>(1, (int64_t)16 * ctx->n_cu / std::max<int64_t>(1, p.tiles_per_sky));
        chunk = (int)std::min<int64_t>({by_mem, std::max<int64_t>(by_tiles, 4), 256});
    }
    if (o.schedule == FH_SCHED_PLAIN) chunk = 1;
    chunk = std::min(chunk, n_sky);
    ChunkBufs b;
    if ((s = ensure_workspace(ctx, pm, g, p, chunk, weighted, st, b))) return s;
    for (int32_t base = 0; base < n_sky; base += chunk) {
        const int slots = std::min(chunk, n_sky - base);
        const float *w = weighted ? d_w + (w_stride ? (int64_t)base * w_stride : 0) : nullptr;
        if ((s = enqueue_front(ctx, pm, g, p, slots, sky + 3 * (int64_t)base, w, w_stride, b, st))) return s;
        HIP_OK(launch_fill_u64(b.colmax, (int64_t)slots * g->nf, 0ull, st));
        TileArgs a = tile_args(pm, g, p, slots, b, weighted, w_stride == 0 ? 0 : 1);
        const int64_t n_tiles = p.tiles_per_sky * slots;
        if (o.schedule == FH_SCHED_PERSISTENT) {
            // order: tiles sharing (sky, bin block) go to the same XCD queue
            if ((s = ctx->h_order.ensure(4 * (size_t)(n_tiles + kXcds + 1), st))) return s;
            int32_t *ho = (int32_t *)ctx->h_order.ptr;
            std::vector<std::vector<int32_t>> q(kXcds);
            int64_t grp = 0;
            for (int sl = 0; sl < slots; ++sl)
                for (int jb = 0; jb < p.nbb; ++jb, ++grp)
                    for (int rb = 0; rb < p.nrb; ++rb)
                        q[grp % kXcds].push_back((int32_t)(((int64_t)sl * p.nrb + rb) * p.nbb + jb));
            int32_t *hs = ho + n_tiles;
            int64_t pos = 0;
            for (int x = 0; x < kXcds; ++x) {
                hs[x] = (int32_t)pos;
                for (int32_t t : q[x]) ho[pos++] = t;
            }
            hs[kXcds] = (int32_t)pos;
            HIP_OK(hipMemcpyAsync(b.order, ho, 4 * (size_t)n_tiles, hipMemcpyHostToDevice, st));
            HIP_OK(hipMemcpyAsync(b.qstart, hs, 4 * (kXcds + 1), hipMemcpyHostToDevice, st));
            HIP_OK(launch_fill_i32(b.qctr, kXcds, 0, st));
            const int grid_blocks = (int)std::min<int64_t>(ctx->n_cu, n_tiles);
            {
                Timed timed(ctx, st, kSpanTiles);
                HIP_OK(launch_tiles(a, weighted, false, true, true, (int32_t)n_tiles, grid_blocks, st));
            }
            // the pinned order buffer is reused by the next chunk
            HIP_OK(hipStreamSynchronize(st));
        } else {
            a.tile_base = 0;
            Timed timed(ctx, st, kSpanTiles);
            HIP_OK(launch_tiles(a, weighted, false, true, false, (int32_t)n_tiles, 0, st));
        }
        if (ctx->profiling) ctx->prof_updates += pm->n_peaks * (int64_t)g->ns * slots;
        Timed timed_sel(ctx, st, kSpanSelect);
        HIP_OK(launch_select(b.colmax, g->nf, slots, *sel, base, pm->n_fft, weighted ? b.ws : nullptr,
                             weighted ? (w_stride == 0 ? 0 : 1) : 0, d_out, st));
    }
    return FH_OK;
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
        else { p.select_ms += ms; p.select_launches++; }
    }
    p.cell_updates = ctx->prof_updates;
    *out = p;
    return FH_OK;
}

}  // extern "C"
