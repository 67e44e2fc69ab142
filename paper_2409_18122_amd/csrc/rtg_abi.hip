// Host runtime behind the C ABI declared in include/rtg.h: argument checks,
// a caching device-memory pool, frames (projected records, sorted tile lists,
// per-pixel state), the batched and per-view scorers, the captured scoring
// graph and the tile autotuner.  All device work is in rtg_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rtg.h"
#include "rtg_internal.h"

using namespace rtg;

namespace {

thread_local std::string g_err;

rtg_status set_err(rtg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_err(e_ == hipErrorOutOfMemory ? RTG_ERR_OOM : RTG_ERR_HIP,            \
                           "%s failed: %s (%d)", #expr, hipGetErrorString(e_), (int)e_);     \
    } while (0)

#define RTG_TRY(expr)                    \
    do {                                 \
        rtg_status s_ = (expr);          \
        if (s_ != RTG_OK) return s_;     \
    } while (0)

rtg_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(RTG_ERR_HIP, "%s launch failed: %s (%d)", what, hipGetErrorString(e), (int)e);
    return RTG_OK;
}

// ------------------------------------------------------------------- pool
// Grow-only caching allocator: released blocks are kept and reused for
// requests of at most their size (and at least half of it).  Blocks are
// reused in stream order, which is safe because a context serves one stream.
// Blocks come from hipMalloc, or from the caller's allocator when one is set.
struct Pool {
    std::multimap<size_t, void*> free_;
    std::map<void*, size_t> size_;
    size_t bytes_live = 0, bytes_cached = 0;
    rtg_alloc_fn alloc_fn = nullptr;
    rtg_free_fn free_fn = nullptr;
    void* user = nullptr;

    void* raw_alloc(size_t bytes) {
        if (alloc_fn) return alloc_fn(user, bytes);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void raw_free(void* p) {
        if (free_fn) free_fn(user, p);
        else (void)hipFree(p);
    }

    rtg_status get(size_t bytes, void** out) {
        bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && it->first <= 2 * bytes) {
            *out = it->second;
            bytes_cached -= it->first;
            bytes_live += it->first;
            free_.erase(it);
            return RTG_OK;
        }
        void* p = raw_alloc(bytes);
        if (!p) {
            // release the cache and retry once
            trim();
            p = raw_alloc(bytes);
            if (!p) return set_err(RTG_ERR_OOM, "device allocation of %zu bytes failed", bytes);
        }
        size_[p] = bytes;
        bytes_live += bytes;
        *out = p;
        return RTG_OK;
    }
    void put(void* p) {
        if (!p) return;
        auto it = size_.find(p);
        if (it == size_.end()) return;
        free_.emplace(it->second, p);
        bytes_live -= it->second;
        bytes_cached += it->second;
    }
    void trim() {
        for (auto& kv : free_) {
            raw_free(kv.second);
            size_.erase(kv.second);
        }
        free_.clear();
        bytes_cached = 0;
    }
    ~Pool() {
        trim();
        for (auto& kv : size_) raw_free(kv.first);
    }
};

}  // namespace


constexpr int N_TIMERS = 9;

struct PendingTimer {
    int id;
    hipEvent_t a, b;
};

struct rtg_ctx {
    int device = 0;
    int cu = 0;
    void* scratch = nullptr;  // this device's fixed scratch array (device address), or NULL
    Pool pool;
    uint32_t* pinned = nullptr;  // small host readback area
    int last_tw = 16, last_th = 16, last_batch = 0;
    // measurement
    bool timing = false;
    bool capturing = false;
    std::vector<PendingTimer> pending;
    std::vector<hipEvent_t> spare_events;
    double timer_ms[N_TIMERS] = {};
    int64_t timer_n[N_TIMERS] = {};
};

namespace {

hipEvent_t take_event(rtg_ctx* c) {
    if (!c->spare_events.empty()) {
        hipEvent_t e = c->spare_events.back();
        c->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Brackets the kernels enqueued during its lifetime with events on `s`.
struct Timer {
    rtg_ctx* c;
    int id;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Timer(rtg_ctx* c_, int id_, hipStream_t s_) : c(c_), id(id_), s(s_) {
        if (c->timing && !c->capturing) {
            a = take_event(c);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Timer() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) {
            c->spare_events.push_back(a);
            return;
        }
        (void)hipEventRecord(b, s);
        c->pending.push_back(PendingTimer{id, a, b});
    }
};

void drain_timers(rtg_ctx* c) {
    for (auto& p : c->pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->timer_ms[p.id] += ms;
            c->timer_n[p.id] += 1;
        }
        (void)hipGetLastError();
        c->spare_events.push_back(p.a);
        c->spare_events.push_back(p.b);
    }
    c->pending.clear();
}

// A device buffer taken from the context pool.
struct Buf {
    rtg_ctx* ctx = nullptr;
    void* p = nullptr;
    size_t bytes = 0;
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    ~Buf() { release(); }
    void release() {
        if (p && ctx) ctx->pool.put(p);
        p = nullptr;
        bytes = 0;
    }
    rtg_status ensure(rtg_ctx* c, size_t need) {
        if (p && bytes >= need) return RTG_OK;
        release();
        ctx = c;
        RTG_TRY(c->pool.get(need, &p));
        bytes = need;
        return RTG_OK;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

bool valid_tile(int tw, int th) { return (tw == 8 && th == 8) || (tw == 16 && th == 16) || (tw == 32 && th == 8); }

int bits_for(uint64_t n) {
    int b = 1;
    while ((1ull << b) < n) b++;
    return b;
}

rtg_status check_gauss(const rtg_gaussians* g, bool need_colors, bool need_unc) {
    if (!g) return set_err(RTG_ERR_INVALID, "gaussians is NULL");
    if (g->n < 0) return set_err(RTG_ERR_INVALID, "n = %lld < 0", (long long)g->n);
    if (g->n >= (int64_t)1 << 31) return set_err(RTG_ERR_UNSUPPORTED, "n = %lld exceeds 2^31 - 1", (long long)g->n);
    if (g->n > 0) {
        if (!g->means || !g->log_scales || !g->opacity)
            return set_err(RTG_ERR_INVALID, "a required Gaussian array (means, log_scales, opacity) is NULL");
        if (need_colors && !g->colors) return set_err(RTG_ERR_INVALID, "colors is NULL");
        if (need_unc && !g->uncert) return set_err(RTG_ERR_INVALID, "uncert is NULL");
    }
    return RTG_OK;
}

rtg_status check_cams(const rtg_camera* cams, int n_views) {
    if (!cams) return set_err(RTG_ERR_INVALID, "cams is NULL");
    if (n_views < 1 || n_views > MAX_VIEWS) return set_err(RTG_ERR_INVALID, "n_views = %d not in [1, %d]", n_views, MAX_VIEWS);
    for (int v = 0; v < n_views; v++) {
        const rtg_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0) return set_err(RTG_ERR_INVALID, "camera %d: size %dx%d", v, c.width, c.height);
        if (c.width > 16384 || c.height > 16384)
            return set_err(RTG_ERR_UNSUPPORTED, "camera %d: size %dx%d above 16384", v, c.width, c.height);
        bool fin = std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) && std::isfinite(c.cy);
        for (int k = 0; k < 9; k++) fin = fin && std::isfinite(c.R[k]);
        for (int k = 0; k < 3; k++) fin = fin && std::isfinite(c.T[k]);
        if (!fin) return set_err(RTG_ERR_INVALID, "camera %d has a non-finite value", v);
        if (!(c.fx > 0.0f) || !(c.fy > 0.0f)) return set_err(RTG_ERR_INVALID, "camera %d: focal length must be > 0", v);
    }
    return RTG_OK;
}

rtg_status resolve_settings(rtg_ctx* ctx, const rtg_settings* in, rtg_settings* out) {
    if (!in) return set_err(RTG_ERR_INVALID, "settings is NULL");
    *out = *in;
    if (out->tile_w == 0 && out->tile_h == 0) {
        out->tile_w = ctx->last_tw;
        out->tile_h = ctx->last_th;
        if (out->batch == 0) out->batch = ctx->last_batch;
    }
    if (!valid_tile(out->tile_w, out->tile_h))
        return set_err(RTG_ERR_INVALID, "tile %dx%d not one of 8x8, 16x16, 32x8", out->tile_w, out->tile_h);
    bool fin = std::isfinite(out->T_min) && std::isfinite(out->alpha_min) && std::isfinite(out->alpha_max) &&
               std::isfinite(out->z_near) && std::isfinite(out->eps2d);
    if (!fin) return set_err(RTG_ERR_INVALID, "settings hold a non-finite value");
    if (!(out->alpha_min > 0.0f) || !(out->alpha_max < 1.0f) || !(out->alpha_min < out->alpha_max))
        return set_err(RTG_ERR_INVALID, "need 0 < alpha_min < alpha_max < 1");
    if (!(out->T_min > 0.0f) || !(out->T_min < 1.0f)) return set_err(RTG_ERR_INVALID, "need 0 < T_min < 1");
    if (!(out->z_near > 0.0f)) return set_err(RTG_ERR_INVALID, "need z_near > 0");
    if (out->eps2d < 0.0f) return set_err(RTG_ERR_INVALID, "need eps2d >= 0");
    if (out->isotropic != 0 && out->isotropic != 1) return set_err(RTG_ERR_INVALID, "isotropic must be 0 or 1");
    const int b = out->batch;
    if (b != 0 && ((b != 32 && b != 64 && b != 128 && b != 256) || b > out->tile_w * out->tile_h))
        return set_err(RTG_ERR_INVALID, "batch %d is not 0 or one of 32, 64, 128, 256 within the tile's %d pixels", b,
                       out->tile_w * out->tile_h);
    return RTG_OK;
}

SetDev to_dev(const rtg_settings& s) {
    return SetDev{s.T_min, s.alpha_min, s.alpha_max, s.z_near, s.eps2d, (float)std::log2((double)s.alpha_min),
                  s.isotropic};
}

GaussDev to_dev(const rtg_gaussians& g) {
    return GaussDev{g.n, g.means, g.log_scales, g.quats, g.opacity, g.colors, g.uncert};
}

// Tile and pixel layout of a batch of views.
struct Layout {
    std::vector<ViewDev> views;
    Header hdr{};
    int max_pix = 0;
};

void make_layout(const rtg_camera* cams, int n, int tw, int th, Layout& L) {
    L.views.resize(n);
    uint64_t tiles = 0, pix = 0;
    int maxp = 0;
    for (int v = 0; v < n; v++) {
        const rtg_camera& c = cams[v];
        ViewDev& d = L.views[v];
        for (int k = 0; k < 9; k++) d.R[k] = (double)c.R[k];
        for (int k = 0; k < 3; k++) d.T[k] = (double)c.T[k];
        d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
        for (int k = 0; k < 9; k++) d.Rf[k] = c.R[k];
        for (int k = 0; k < 3; k++) d.Tf[k] = c.T[k];
        d.fxf = c.fx; d.fyf = c.fy; d.cxf = c.cx; d.cyf = c.cy;
        d.W = c.width; d.H = c.height;
        d.tiles_x = (c.width + tw - 1) / tw;
        d.tiles_y = (c.height + th - 1) / th;
        d.tile_off = (uint32_t)tiles;
        d.pad = 0;
        d.pix_off = pix;
        tiles += (uint64_t)d.tiles_x * d.tiles_y;
        pix += (uint64_t)c.width * c.height;
        maxp = std::max(maxp, c.width * c.height);
    }
    L.hdr.n_views = (uint32_t)n;
    L.hdr.tiles_total = (uint32_t)tiles;
    L.hdr.pix_total = pix;
    L.max_pix = maxp;
}

// Counters kept on the device: [0] records, [1] instances, [2] flags,
// [3] work queue, [4] number of Gaussians.
enum { C_REC = 0, C_INST = 1, C_FLAGS = 2, C_QUEUE = 3, C_NG = 4, C_COUNT = 8 };

}  // namespace

// All device state of one projection of the map into a batch of views.
struct rtg_frame {
    rtg_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    rtg_gaussians g{};
    rtg_settings st{};
    Layout L;
    int n_views = 0;
    int views_cap = 0;  // words of the visibility mask
    uint32_t R = 0;     // records
    int64_t K = -1;     // instances (-1 before binning)
    uint32_t rec_cap = 0, inst_cap = 0, tiles_cap = 0;
    bool rendered = false;
    bool scoring = false;  // only scored: records carry no colour / depth attributes
    int order_in_alt = 0, inst_in_alt = 0;

    Buf views, hdr, counters, cnt, mask, rec_off, scan_ws, sort_hist, chunk_g;
    Buf emit, q64, attr, ntiles, skey, skey2, order, order2;
    Buf inst_off, tkey, tkey2, irec, irec2, ranges, tile_ord, tile_ord_ws;
    Buf T_final, n_last, g2d, loss_part, score_part, ssim_maps;

    Records records() const {
        return Records{emit.as<EmitRec>(), q64.as<double4>(), attr.as<float4>(), ntiles.as<uint32_t>()};
    }
    uint32_t* sorted_order() const { return order_in_alt ? order2.as<uint32_t>() : order.as<uint32_t>(); }
    uint32_t* sorted_tkey() const { return inst_in_alt ? tkey2.as<uint32_t>() : tkey.as<uint32_t>(); }
    uint32_t* sorted_irec() const { return inst_in_alt ? irec2.as<uint32_t>() : irec.as<uint32_t>(); }
    uint32_t* ctr(int k) const { return counters.as<uint32_t>() + k; }
    Buf n_contrib, stats, d_img;
};

namespace {

rtg_status flags_status(uint32_t flags) {
    if (flags & FLAG_COUNT_OVERFLOW)
        return set_err(RTG_ERR_UNSUPPORTED, "2^31 or more records or pairs: the 32-bit list offsets cannot hold them");
    if (flags & (FLAG_REC_OVERFLOW | FLAG_INST_OVERFLOW))
        return set_err(RTG_ERR_CAPACITY, "buffers overflowed (flags 0x%x)", flags);
    if (flags) return set_err(RTG_ERR_HIP, "pair emission disagreed with the pair count (flags 0x%x)", flags);
    return RTG_OK;
}

// Reads the device counters (a synchronisation point) and reports any flag.
rtg_status read_counter(rtg_ctx* ctx, const uint32_t* dev, uint32_t* host, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(ctx->pinned, dev, sizeof(uint32_t) * C_COUNT, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(host, ctx->pinned, sizeof(uint32_t) * C_COUNT);
    return flags_status(host[C_FLAGS]);
}

// Allocates the view-side and per-Gaussian buffers of a frame and uploads
// the layout.  Used by the eager frame path and the captured graph.
rtg_status frame_setup(rtg_frame* f, int views_cap, hipStream_t s) {
    rtg_ctx* ctx = f->ctx;
    const int64_t n = f->g.n;
    f->views_cap = views_cap;
    int words = (views_cap + 31) / 32;
    RTG_TRY(f->views.ensure(ctx, sizeof(ViewDev) * views_cap));
    RTG_TRY(f->hdr.ensure(ctx, sizeof(Header)));
    RTG_TRY(f->counters.ensure(ctx, sizeof(uint32_t) * C_COUNT));
    RTG_TRY(f->cnt.ensure(ctx, sizeof(uint32_t) * std::max<int64_t>(n, 1)));
    RTG_TRY(f->rec_off.ensure(ctx, sizeof(uint32_t) * std::max<int64_t>(n, 1)));
    RTG_TRY(f->mask.ensure(ctx, sizeof(uint32_t) * std::max<int64_t>(n, 1) * words));
    RTG_TRY(f->scan_ws.ensure(ctx, sizeof(uint32_t) * 1088));
    return RTG_OK;
}

rtg_status upload_layout(rtg_frame* f, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(f->views.p, f->L.views.data(), sizeof(ViewDev) * f->L.views.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(f->hdr.p, &f->L.hdr, sizeof(Header), hipMemcpyHostToDevice, s));
    return RTG_OK;
}

// Records buffers for capacity rc.
rtg_status alloc_records(rtg_frame* f, uint32_t rc) {
    rtg_ctx* ctx = f->ctx;
    size_t r = std::max<uint32_t>(rc, 1);
    RTG_TRY(f->emit.ensure(ctx, sizeof(EmitRec) * r));
    RTG_TRY(f->q64.ensure(ctx, 32 * r));
    if (!f->scoring) RTG_TRY(f->attr.ensure(ctx, 16 * r));
    RTG_TRY(f->ntiles.ensure(ctx, 4 * r));
    RTG_TRY(f->skey.ensure(ctx, 4 * r));
    RTG_TRY(f->skey2.ensure(ctx, 4 * r));
    RTG_TRY(f->order.ensure(ctx, 4 * r));
    RTG_TRY(f->order2.ensure(ctx, 4 * r));
    RTG_TRY(f->inst_off.ensure(ctx, 4 * r));
    RTG_TRY(f->chunk_g.ensure(ctx, 4 * pe_chunk_words((uint32_t)r)));
    f->rec_cap = rc;
    return RTG_OK;
}

rtg_status alloc_instances(rtg_frame* f, uint32_t kc, uint32_t tiles_cap) {
    rtg_ctx* ctx = f->ctx;
    size_t k = std::max<uint32_t>(kc, 1);
    RTG_TRY(f->tkey.ensure(ctx, 4 * k));
    RTG_TRY(f->tkey2.ensure(ctx, 4 * k));
    RTG_TRY(f->irec.ensure(ctx, 4 * k));
    RTG_TRY(f->irec2.ensure(ctx, 4 * k));
    RTG_TRY(f->ranges.ensure(ctx, 8 * (size_t)std::max<uint32_t>(tiles_cap, 1)));
    RTG_TRY(f->tile_ord.ensure(ctx, 4 * (size_t)std::max<uint32_t>(tiles_cap, 1)));
    RTG_TRY(f->tile_ord_ws.ensure(ctx, 4 * (size_t)TILE_ORDER_WS));
    uint64_t big = std::max<uint64_t>(std::max<uint64_t>(kc, f->rec_cap), 1);
    RTG_TRY(f->sort_hist.ensure(ctx, sizeof(uint32_t) * sort_hist_words(big)));
    f->inst_cap = kc;
    f->tiles_cap = tiles_cap;
    return RTG_OK;
}

// Projection kernels (count, scan, emit).  In eager mode the record count is
// read back and the record buffers sized exactly.
rtg_status enqueue_project(rtg_frame* f, bool eager, hipStream_t s) {
    GaussDev gd = to_dev(f->g);
    SetDev sd = to_dev(f->st);
    const ViewDev* views = f->views.as<ViewDev>();
    const Header* hdr = f->hdr.as<Header>();
    uint32_t n = (uint32_t)f->g.n;
    Timer tm(f->ctx, 0, s);
    // a captured graph keeps its flags word across replays (an overflow stays
    // reported until the graph is destroyed); an eager frame starts clean
    if (eager) fill_u32(f->ctr(0), 0u, C_COUNT, s);
    else fill_u32(f->ctr(0), 0u, C_FLAGS, s);  // records and pairs counters
    fill_u32(f->ctr(C_NG), n, 1, s);
    project_count(gd, views, hdr, f->views_cap, sd, f->cnt.as<uint32_t>(), f->mask.as<uint32_t>(), s);
    scan_u32(f->cnt.as<uint32_t>(), nullptr, f->rec_off.as<uint32_t>(), f->ctr(C_NG), std::max<uint32_t>(n, 1),
             f->ctr(C_REC), f->ctr(C_FLAGS), ScanWs{f->scan_ws.as<uint32_t>()}, s);
    RTG_TRY(check_launch("projection count"));
    if (eager) {
        uint32_t c[C_COUNT];
        RTG_TRY(read_counter(f->ctx, f->ctr(0), c, s));
        f->R = c[C_REC];
        RTG_TRY(alloc_records(f, f->R));
    }
    project_emit(gd, views, hdr, f->views_cap, sd, f->st.tile_w, f->st.tile_h, f->mask.as<uint32_t>(),
                 f->cnt.as<uint32_t>(), f->rec_off.as<uint32_t>(), f->ctr(C_REC), f->rec_cap, f->records(),
                 f->skey.as<uint32_t>(), f->order.as<uint32_t>(), !f->scoring, f->chunk_g.as<uint32_t>(),
                 f->ctr(C_FLAGS), s);
    return check_launch("projection emit");
}

// Digit widths of the two sorts (measured): the 32-bit depth keys in 4 passes
// of 8 bits; tile keys (ceil(log2 tiles) bits) in passes of up to 8 bits too.
// 11-bit tile digits (one pass up to 2048 tiles) were as fast on a 640x480
// frame and 1-2% slower on batches of views: their scatter spreads a block's
// pairs over 2048 buckets, so more writes are partial cache lines.
constexpr int DEPTH_SORT_DIGIT = 8;
constexpr int TILE_SORT_DIGIT = 8;

rtg_status enqueue_bin(rtg_frame* f, bool eager, hipStream_t s) {
    const uint32_t rc = std::max<uint32_t>(f->rec_cap, 1);
    SortWs ws{f->sort_hist.as<uint32_t>(), f->scan_ws.as<uint32_t>()};
    if (eager) {
        // the histogram table must fit the larger of the two sorts; size it for the records now
        RTG_TRY(f->sort_hist.ensure(f->ctx, sizeof(uint32_t) * sort_hist_words(rc)));
        ws.hist = f->sort_hist.as<uint32_t>();
    }
    {
        Timer tm(f->ctx, 1, s);
        // the last pass also lays the records' pair counts out in depth order
        // (into inst_off), so that the scan below reads them in sequence
        f->order_in_alt = radix_sort(f->skey.as<uint32_t>(), f->order.as<uint32_t>(), f->skey2.as<uint32_t>(),
                                     f->order2.as<uint32_t>(), f->ctr(C_REC), rc, 32, DEPTH_SORT_DIGIT, ws, s,
                                     f->ntiles.as<uint32_t>(), f->inst_off.as<uint32_t>());
    }
    scan_u32(f->inst_off.as<uint32_t>(), nullptr, f->inst_off.as<uint32_t>(), f->ctr(C_REC), rc, f->ctr(C_INST),
             f->ctr(C_FLAGS), ScanWs{f->scan_ws.as<uint32_t>()}, s);
    RTG_TRY(check_launch("depth sort"));
    if (eager) {
        uint32_t c[C_COUNT];
        RTG_TRY(read_counter(f->ctx, f->ctr(0), c, s));
        f->K = c[C_INST];
        RTG_TRY(alloc_instances(f, (uint32_t)f->K, f->L.hdr.tiles_total));
        ws.hist = f->sort_hist.as<uint32_t>();
    }
    const uint32_t kc = std::max<uint32_t>(f->inst_cap, 1);
    Timer tm(f->ctx, 2, s);
    emit_instances(f->sorted_order(), f->ctr(C_REC), rc, f->ctr(C_INST), f->records(), f->views.as<ViewDev>(),
                   f->inst_off.as<uint32_t>(), f->st.tile_w, f->st.tile_h, to_dev(f->st), f->inst_cap,
                   f->tkey.as<uint32_t>(), f->irec.as<uint32_t>(), f->ranges.as<uint2>(), f->tiles_cap,
                   f->ctr(C_FLAGS), s);
    int tbits = bits_for(std::max<uint32_t>(f->tiles_cap, 2));
    f->inst_in_alt = radix_sort(f->tkey.as<uint32_t>(), f->irec.as<uint32_t>(), f->tkey2.as<uint32_t>(),
                                f->irec2.as<uint32_t>(), f->ctr(C_INST), kc, tbits, TILE_SORT_DIGIT, ws, s);
    tile_ranges(f->sorted_tkey(), f->ctr(C_INST), kc, f->ranges.as<uint2>(), f->tiles_cap, f->ctr(C_FLAGS), s);
    tile_order(f->ranges.as<uint2>(), f->hdr.as<Header>(), f->tiles_cap, f->tile_ord_ws.as<uint32_t>(),
               f->tile_ord.as<uint32_t>(), s);
    return check_launch("tile binning");
}

rtg_status new_frame(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int n_views,
                     const rtg_settings* settings, rtg_frame** out, hipStream_t s) {
    std::unique_ptr<rtg_frame> f(new (std::nothrow) rtg_frame());
    if (!f) return set_err(RTG_ERR_OOM, "host allocation failed");
    f->ctx = ctx;
    f->stream = s;
    f->g = *g;
    RTG_TRY(resolve_settings(ctx, settings, &f->st));
    if (!f->st.isotropic && g->n > 0 && !g->quats)
        return set_err(RTG_ERR_INVALID, "quats is NULL (required unless isotropic)");
    make_layout(cams, n_views, f->st.tile_w, f->st.tile_h, f->L);
    f->n_views = n_views;
    RTG_TRY(frame_setup(f.get(), n_views, s));
    RTG_TRY(upload_layout(f.get(), s));
    *out = f.release();
    return RTG_OK;
}

rtg_status ensure_pixel_state(rtg_frame* f) {
    size_t P = std::max<uint64_t>(f->L.hdr.pix_total, 1);
    RTG_TRY(f->T_final.ensure(f->ctx, 4 * P));
    RTG_TRY(f->n_last.ensure(f->ctx, 4 * P));
    RTG_TRY(f->n_contrib.ensure(f->ctx, 4 * P));
    return RTG_OK;
}

rtg_status ctx_ok(rtg_ctx* ctx) {
    if (!ctx) return set_err(RTG_ERR_INVALID, "context is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    return RTG_OK;
}

}  // namespace

// ======================================================== fixed scratch
// Device scratch for the entry points that allocate nothing: one array per
// GPU, resident from the code object's load until the process ends.  Host
// code must never pass the array's own name to a kernel or a copy (it names
// a host-side stand-in); it uses the device address that hipGetSymbolAddress
// returns for the current device, taken once per device at context creation.
constexpr size_t SCRATCH_BYTES = (size_t)96 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[SCRATCH_MAX_DEVICES] = {};

// With `device` current: its scratch address, looked up on first use.
rtg_status scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= SCRATCH_MAX_DEVICES)
        return set_err(RTG_ERR_UNSUPPORTED, "fixed scratch: device %d beyond %d", device, SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_err(RTG_ERR_HIP, "hipGetSymbolAddress of the fixed scratch failed: %s (%d)",
                           hipGetErrorString(e), (int)e);
        }
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return RTG_OK;
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

rtg_status collision_args(const rtg_gaussians* g, const float* points, int64_t n_points, float r_robot,
                          float lambda_g, int32_t* collide) {
    if (!g) return set_err(RTG_ERR_INVALID, "gaussians is NULL");
    if (g->n < 0 || n_points < 0) return set_err(RTG_ERR_INVALID, "n = %lld, n_points = %lld", (long long)g->n,
                                                 (long long)n_points);
    if (g->n >= (int64_t)1 << 31 || n_points >= (int64_t)1 << 31)
        return set_err(RTG_ERR_UNSUPPORTED, "n = %lld, n_points = %lld: 2^31 or more", (long long)g->n,
                       (long long)n_points);
    if (g->n > 0 && (!g->means || !g->log_scales)) return set_err(RTG_ERR_INVALID, "means and log_scales are required");
    if (n_points > 0 && (!points || !collide)) return set_err(RTG_ERR_INVALID, "points and collide must be non-NULL");
    if (!std::isfinite(r_robot) || !(r_robot >= 0.0f)) return set_err(RTG_ERR_INVALID, "r_robot must be finite and >= 0");
    if (!std::isfinite(lambda_g) || !(lambda_g >= 0.0f))
        return set_err(RTG_ERR_INVALID, "lambda_g must be finite and >= 0");
    return RTG_OK;
}

}  // namespace

// =================================================================== ABI

extern "C" {

const char* rtg_last_error(void) { return g_err.c_str(); }

rtg_status rtg_default_settings(rtg_settings* s) {
    if (!s) return set_err(RTG_ERR_INVALID, "settings is NULL");
    s->tile_w = 16;
    s->tile_h = 16;
    s->batch = 0;
    s->T_min = 1e-4f;
    s->alpha_min = 1.0f / 255.0f;
    s->alpha_max = 0.99f;
    s->z_near = 0.2f;
    s->eps2d = 0.0f;
    s->max_instances = 0;
    s->isotropic = 0;
    s->reserved = 0;
    return RTG_OK;
}

int32_t rtg_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

rtg_status rtg_create(int32_t device, rtg_ctx** out) {
    if (!out) return set_err(RTG_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int n = rtg_device_count();
    if (device < 0 || device >= n) return set_err(RTG_ERR_HIP, "no HIP device %d (%d present)", device, n);
    HIP_TRY(hipSetDevice(device));
    std::unique_ptr<rtg_ctx> c(new (std::nothrow) rtg_ctx());
    if (!c) return set_err(RTG_ERR_OOM, "host allocation failed");
    c->device = device;
    c->cu = device_cu_count();
    // the fixed scratch of the allocation-free entry points; a failure here
    // is reported by those entry points, the rest of the library works
    if (scratch_address(device, &c->scratch) != RTG_OK) c->scratch = nullptr;
    HIP_TRY(hipHostMalloc((void**)&c->pinned, sizeof(uint32_t) * 64, hipHostMallocDefault));
    *out = c.release();
    return RTG_OK;
}

rtg_status rtg_set_allocator(rtg_ctx* ctx, rtg_alloc_fn alloc, rtg_free_fn free, void* user) {
    RTG_TRY(ctx_ok(ctx));
    if ((alloc == nullptr) != (free == nullptr))
        return set_err(RTG_ERR_INVALID, "alloc and free must both be set or both be NULL");
    if (ctx->pool.bytes_live)
        return set_err(RTG_ERR_INVALID, "%zu bytes are in use by frames or graphs of this context; destroy them first",
                       ctx->pool.bytes_live);
    HIP_TRY(hipDeviceSynchronize());
    ctx->pool.trim();  // cached blocks go back to the allocator they came from
    ctx->pool.alloc_fn = alloc;
    ctx->pool.free_fn = free;
    ctx->pool.user = user;
    return RTG_OK;
}

void rtg_destroy(rtg_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    drain_timers(ctx);
    for (auto e : ctx->spare_events) (void)hipEventDestroy(e);
    delete ctx;
}

rtg_status rtg_project(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int32_t n_views,
                       const rtg_settings* settings, rtg_frame** out, void* stream) {
    if (!out) return set_err(RTG_ERR_INVALID, "out is NULL");
    *out = nullptr;
    RTG_TRY(ctx_ok(ctx));
    RTG_TRY(check_gauss(g, false, false));
    RTG_TRY(check_cams(cams, n_views));
    hipStream_t s = (hipStream_t)stream;
    rtg_frame* f = nullptr;
    RTG_TRY(new_frame(ctx, g, cams, n_views, settings, &f, s));
    rtg_status st = enqueue_project(f, true, s);
    if (st != RTG_OK) {
        delete f;
        return st;
    }
    *out = f;
    return RTG_OK;
}

rtg_status rtg_bin_sort(rtg_ctx* ctx, rtg_frame* f, int64_t* n_instances, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!f) return set_err(RTG_ERR_INVALID, "frame is NULL");
    RTG_TRY(enqueue_bin(f, true, (hipStream_t)stream));
    f->rendered = false;
    if (n_instances) *n_instances = f->K;
    return RTG_OK;
}

rtg_status rtg_render(rtg_ctx* ctx, rtg_frame* f, float* rgb, float* depth, float* alpha, float* unc,
                      void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!f) return set_err(RTG_ERR_INVALID, "frame is NULL");
    if (f->K < 0) return set_err(RTG_ERR_INVALID, "rtg_bin_sort must run before rtg_render");
    if (rgb && f->g.n > 0 && !f->g.colors) return set_err(RTG_ERR_INVALID, "rgb requested but the map has no colors");
    if (unc && f->g.n > 0 && !f->g.uncert)
        return set_err(RTG_ERR_INVALID, "unc requested but the map has no uncertainty");
    hipStream_t s = (hipStream_t)stream;
    RTG_TRY(ensure_pixel_state(f));
    RenderOut o{rgb, depth, alpha, unc, f->T_final.as<float>(), f->n_last.as<uint32_t>(),
                f->n_contrib.as<uint32_t>()};
    Timer tm(ctx, 3, s);
    render_forward(f->st.tile_w, f->st.tile_h, f->st.batch, f->views.as<ViewDev>(), f->n_views,
                   f->L.hdr.tiles_total, f->ranges.as<uint2>(), f->tile_ord.as<uint32_t>(), f->sorted_irec(), f->records(), to_dev(f->st), o,
                   f->ctr(C_FLAGS), s);
    RTG_TRY(check_launch("render"));
    f->rendered = true;
    return RTG_OK;
}

rtg_status rtg_loss(rtg_ctx* ctx, rtg_frame* f, const float* rgb, const float* depth, const float* target_rgb,
                    const float* target_depth, float w_depth, float* d_rgb, float* d_depth, double* loss,
                    void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!f) return set_err(RTG_ERR_INVALID, "frame is NULL");
    if (!rgb || !depth || !target_rgb || !target_depth || !loss)
        return set_err(RTG_ERR_INVALID, "rgb, depth, targets and loss must be non-NULL");
    if (!std::isfinite(w_depth)) return set_err(RTG_ERR_INVALID, "w_depth is not finite");
    int bx = (f->L.max_pix + 255) / 256;
    RTG_TRY(f->loss_part.ensure(ctx, sizeof(double) * (size_t)std::max(1, bx * f->n_views)));
    Timer tm(ctx, 4, (hipStream_t)stream);
    loss_l1(f->views.as<ViewDev>(), f->n_views, f->L.max_pix, rgb, depth, target_rgb, target_depth, w_depth, d_rgb,
            d_depth, f->loss_part.as<double>(), bx * f->n_views, loss, (hipStream_t)stream);
    return check_launch("loss");
}

rtg_status rtg_loss_ssim(rtg_ctx* ctx, rtg_frame* f, const float* rgb, const float* depth, const float* target_rgb,
                         const float* target_depth, float w_depth, float lambda_1, float lambda_2, float* d_rgb,
                         float* d_depth, double* loss, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!f) return set_err(RTG_ERR_INVALID, "frame is NULL");
    if (!rgb || !depth || !target_rgb || !target_depth || !loss)
        return set_err(RTG_ERR_INVALID, "rgb, depth, targets and loss must be non-NULL");
    if (!std::isfinite(w_depth) || !std::isfinite(lambda_1) || !std::isfinite(lambda_2))
        return set_err(RTG_ERR_INVALID, "w_depth, lambda_1 and lambda_2 must be finite");
    int max_w = 0, max_h = 0;
    for (const ViewDev& v : f->L.views) {
        max_w = std::max(max_w, (int)v.W);
        max_h = std::max(max_h, (int)v.H);
    }
    const int bpv = ssim_blocks_per_view(max_w, max_h);
    const uint64_t P = f->L.hdr.pix_total;
    RTG_TRY(f->loss_part.ensure(ctx, sizeof(double) * (size_t)std::max(1, bpv * f->n_views)));
    RTG_TRY(f->ssim_maps.ensure(ctx, sizeof(float) * 9 * (size_t)std::max<uint64_t>(P, 1)));
    Timer tm(ctx, 4, (hipStream_t)stream);
    loss_ssim(f->views.as<ViewDev>(), f->n_views, bpv, P, rgb, depth, target_rgb, target_depth, w_depth, lambda_1,
              lambda_2, f->ssim_maps.as<float>(), f->loss_part.as<double>(), d_rgb, d_depth, loss,
              (hipStream_t)stream);
    return check_launch("loss with SSIM");
}

rtg_status rtg_render_backward(rtg_ctx* ctx, rtg_frame* f, const float* d_rgb, const float* d_depth,
                               const float* d_alpha, const float* d_unc, const rtg_grads* out, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!f) return set_err(RTG_ERR_INVALID, "frame is NULL");
    if (!out) return set_err(RTG_ERR_INVALID, "grads is NULL");
    if (!f->rendered) return set_err(RTG_ERR_INVALID, "rtg_render must run on this frame before the backward");
    if (d_unc && f->g.n > 0 && !f->g.uncert) return set_err(RTG_ERR_INVALID, "d_unc given but the map has no uncertainty");
    hipStream_t s = (hipStream_t)stream;
    size_t R = std::max<uint32_t>(f->R, 1);
    RTG_TRY(f->g2d.ensure(ctx, sizeof(double) * G2D_STRIDE * R));
    fill_u32(f->g2d.as<uint32_t>(), 0u, (uint64_t)2 * G2D_STRIDE * R, s);
    {
    Timer tm(ctx, 5, s);
    render_backward(f->st.tile_w, f->st.tile_h, f->st.batch, f->views.as<ViewDev>(), f->n_views,
                    f->L.hdr.tiles_total, f->ranges.as<uint2>(), f->tile_ord.as<uint32_t>(), f->sorted_irec(), f->records(), to_dev(f->st),
                    f->T_final.as<float>(), f->n_last.as<uint32_t>(), d_rgb, d_depth, d_alpha, d_unc,
                    f->g2d.as<double>(), f->ctr(C_FLAGS), s);
    }
    RTG_TRY(check_launch("render backward"));
    Timer tm(ctx, 6, s);
    project_backward(to_dev(f->g), f->views.as<ViewDev>(), to_dev(f->st), f->rec_off.as<uint32_t>(),
                     f->cnt.as<uint32_t>(), f->emit.as<EmitRec>(), f->g2d.as<double>(), out->d_means,
                     out->d_log_scales, out->d_quats, out->d_opacity, out->d_colors, f->ctr(C_FLAGS), s);
    return check_launch("projection backward");
}

void rtg_frame_destroy(rtg_frame* f) { delete f; }

rtg_status rtg_frame_export(rtg_ctx* ctx, rtg_frame* f, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                            void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!f) return set_err(RTG_ERR_INVALID, "frame is NULL");
    if (f->K < 0) return set_err(RTG_ERR_INVALID, "rtg_bin_sort must run before rtg_frame_export");
    hipStream_t s = (hipStream_t)stream;
    if ((keys || vals) && f->K > 0)
        export_pairs(f->sorted_tkey(), f->sorted_irec(), f->ctr(C_INST), f->records(), keys, vals, f->inst_cap, s);
    if (ranges && f->L.hdr.tiles_total)
        HIP_TRY(hipMemcpyAsync(ranges, f->ranges.p, 8 * (size_t)f->L.hdr.tiles_total, hipMemcpyDeviceToDevice, s));
    return check_launch("export");
}

rtg_status rtg_frame_export_records(rtg_ctx* ctx, rtg_frame* f, double* mean2d, double* conic, int32_t* pbox,
                                    uint32_t* depth_bits, uint32_t* gid, uint32_t* view, uint32_t* ntiles,
                                    void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!f) return set_err(RTG_ERR_INVALID, "frame is NULL");
    if (f->R == 0) return RTG_OK;
    export_records(f->ctr(C_REC), f->rec_cap, f->records(), mean2d, conic, pbox, depth_bits, gid, view, ntiles,
                   (hipStream_t)stream);
    return check_launch("export records");
}

rtg_status rtg_frame_stats(rtg_ctx* ctx, rtg_frame* f, int64_t out[4], void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!f || !out) return set_err(RTG_ERR_INVALID, "frame or out is NULL");
    if (!f->rendered) return set_err(RTG_ERR_INVALID, "rtg_render must run before rtg_frame_stats");
    hipStream_t s = (hipStream_t)stream;
    RTG_TRY(f->stats.ensure(ctx, 2 * sizeof(unsigned long long)));
    fill_u32(f->stats.as<uint32_t>(), 0u, 4, s);
    sum_u32_pair(f->n_contrib.as<uint32_t>(), f->n_last.as<uint32_t>(), f->L.hdr.pix_total,
                 f->stats.as<unsigned long long>(), s);
    RTG_TRY(check_launch("frame stats"));
    unsigned long long h[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(ctx->pinned, f->stats.p, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ctx->pinned + 4, f->ctr(C_FLAGS), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(h, ctx->pinned, sizeof(h));
    RTG_TRY(flags_status(ctx->pinned[4]));
    out[0] = f->R;
    out[1] = f->K;
    out[2] = (int64_t)h[0];
    out[3] = (int64_t)h[1];
    return RTG_OK;
}

rtg_status rtg_timing_enable(rtg_ctx* ctx, int32_t on) {
    if (!ctx) return set_err(RTG_ERR_INVALID, "context is NULL");
    ctx->timing = on != 0;
    return RTG_OK;
}

rtg_status rtg_timing_read(rtg_ctx* ctx, int32_t id, double* total_ms, int64_t* count) {
    if (!ctx) return set_err(RTG_ERR_INVALID, "context is NULL");
    if (id < 0 || id >= N_TIMERS) return set_err(RTG_ERR_INVALID, "timer id %d", id);
    HIP_TRY(hipSetDevice(ctx->device));
    drain_timers(ctx);
    if (total_ms) *total_ms = ctx->timer_ms[id];
    if (count) *count = ctx->timer_n[id];
    return RTG_OK;
}

rtg_status rtg_timing_reset(rtg_ctx* ctx) {
    if (!ctx) return set_err(RTG_ERR_INVALID, "context is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    drain_timers(ctx);
    for (int i = 0; i < N_TIMERS; i++) {
        ctx->timer_ms[i] = 0.0;
        ctx->timer_n[i] = 0;
    }
    return RTG_OK;
}

rtg_status rtg_frame_info(const rtg_frame* f, int64_t info[6]) {
    if (!f || !info) return set_err(RTG_ERR_INVALID, "frame or info is NULL");
    info[0] = f->R;
    info[1] = f->K;
    info[2] = f->L.hdr.tiles_total;
    info[3] = (int64_t)f->L.hdr.pix_total;
    info[4] = f->st.tile_w;
    info[5] = f->st.tile_h;
    return RTG_OK;
}

}  // extern "C"

// ================================================================ scoring

namespace {

rtg_status score_batched(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int n_views,
                         const rtg_settings* settings, int mode, double* scores, hipStream_t s) {
    rtg_frame* fp = nullptr;
    RTG_TRY(new_frame(ctx, g, cams, n_views, settings, &fp, s));
    std::unique_ptr<rtg_frame> f(fp);
    f->scoring = true;
    RTG_TRY(enqueue_project(f.get(), true, s));
    RTG_TRY(enqueue_bin(f.get(), true, s));
    RTG_TRY(f->score_part.ensure(ctx, sizeof(double) * std::max<uint32_t>(f->L.hdr.tiles_total, 1)));
    int grid = score_persistent_blocks(f->st.tile_w, f->st.tile_h, f->st.batch);
    Timer tm(ctx, 7, s);
    score_tiles(f->st.tile_w, f->st.tile_h, f->st.batch, mode, true, grid, f->views.as<ViewDev>(), f->n_views,
                f->hdr.as<Header>(), 0, f->L.hdr.tiles_total, f->ranges.as<uint2>(), f->tile_ord.as<uint32_t>(), f->sorted_irec(), f->records(),
                to_dev(f->st), f->score_part.as<double>(), f->ctr(C_QUEUE), f->ctr(C_FLAGS), s);
    score_reduce(f->views.as<ViewDev>(), f->hdr.as<Header>(), n_views, f->score_part.as<double>(), scores,
                 f->ctr(C_FLAGS), s);
    return check_launch("persistent scoring");
}

rtg_status score_plain(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int n_views,
                       const rtg_settings* settings, int mode, double* scores, hipStream_t s) {
    for (int v = 0; v < n_views; v++) {
        rtg_frame* fp = nullptr;
        RTG_TRY(new_frame(ctx, g, cams + v, 1, settings, &fp, s));
        std::unique_ptr<rtg_frame> f(fp);
        f->scoring = true;
        RTG_TRY(enqueue_project(f.get(), true, s));
        RTG_TRY(enqueue_bin(f.get(), true, s));
        RTG_TRY(f->score_part.ensure(ctx, sizeof(double) * std::max<uint32_t>(f->L.hdr.tiles_total, 1)));
        Timer tm(ctx, 7, s);
        score_tiles(f->st.tile_w, f->st.tile_h, f->st.batch, mode, false, 0, f->views.as<ViewDev>(), 1,
                    f->hdr.as<Header>(),
                    0, f->L.hdr.tiles_total, f->ranges.as<uint2>(), f->tile_ord.as<uint32_t>(), f->sorted_irec(), f->records(), to_dev(f->st),
                    f->score_part.as<double>(), f->ctr(C_QUEUE), f->ctr(C_FLAGS), s);
        score_reduce(f->views.as<ViewDev>(), f->hdr.as<Header>(), 1, f->score_part.as<double>(), scores + v,
                     f->ctr(C_FLAGS), s);
        RTG_TRY(check_launch("plain scoring"));
    }
    return RTG_OK;
}

}  // namespace

extern "C" rtg_status rtg_score_views(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams,
                                      int32_t n_views, const rtg_settings* settings, double* scores,
                                      int32_t persistent, int32_t mode, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    RTG_TRY(check_gauss(g, false, true));
    RTG_TRY(check_cams(cams, n_views));
    if (!scores) return set_err(RTG_ERR_INVALID, "scores is NULL");
    if (mode != 0 && mode != 1) return set_err(RTG_ERR_INVALID, "score mode %d not in {0, 1}", mode);
    hipStream_t s = (hipStream_t)stream;
    return persistent ? score_batched(ctx, g, cams, n_views, settings, mode, scores, s)
                      : score_plain(ctx, g, cams, n_views, settings, mode, scores, s);
}

// ================================================================== graph

struct rtg_graph {
    int kind = 0;  // 0 scoring, 1 mapping
    rtg_ctx* ctx = nullptr;
    std::unique_ptr<rtg_frame> f;
    int max_views = 0, max_w = 0, max_h = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // Two camera staging slots, so that a launch waits only for the replay
    // before the previous one (which has normally finished) before it
    // rewrites a slot; done[k] completes with the last replay that used slot k.
    static constexpr int SLOTS = 2;
    hipEvent_t done[SLOTS] = {nullptr, nullptr};
    ViewDev* staging[SLOTS] = {nullptr, nullptr};  // pinned
    Header* staging_hdr[SLOTS] = {nullptr, nullptr};
    uint32_t* flag_host = nullptr;  // pinned, written at the end of every replay
    Buf scores;
    int grid = 0;
    int mode = 0;  // scoring: 0 rendered proxy, 1 binary-J trace
    int last_views = 0;
    int64_t launches = 0;
    bool launched = false;
    int last_slot() const { return (int)((launches - 1) % SLOTS); }
};

namespace {

void graph_free(rtg_graph* gr) {
    if (!gr) return;
    (void)hipSetDevice(gr->ctx->device);
    for (int k = 0; k < rtg_graph::SLOTS; k++)
        if (gr->done[k]) (void)hipEventSynchronize(gr->done[k]);
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    if (gr->cap_stream) (void)hipStreamDestroy(gr->cap_stream);
    for (int k = 0; k < rtg_graph::SLOTS; k++) {
        if (gr->done[k]) (void)hipEventDestroy(gr->done[k]);
        if (gr->staging[k]) (void)hipHostFree(gr->staging[k]);
        if (gr->staging_hdr[k]) (void)hipHostFree(gr->staging_hdr[k]);
    }
    if (gr->flag_host) (void)hipHostFree(gr->flag_host);
    delete gr;
}

// Pinned flag word, events and the capture stream of a graph; the device
// flags word starts clear and is never cleared by a replay.
rtg_status graph_host_setup(rtg_graph* gr, bool staging, hipStream_t s) {
    hipError_t e = hipSuccess;
    const int max_views = std::max(gr->max_views, 1);
    for (int k = 0; k < rtg_graph::SLOTS && e == hipSuccess; k++) {
        if (staging) {
            e = hipHostMalloc((void**)&gr->staging[k], sizeof(ViewDev) * max_views, hipHostMallocDefault);
            if (e == hipSuccess)
                e = hipHostMalloc((void**)&gr->staging_hdr[k], sizeof(Header), hipHostMallocDefault);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&gr->done[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipHostMalloc((void**)&gr->flag_host, sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&gr->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return set_err(RTG_ERR_HIP, "graph setup failed: %s", hipGetErrorString(e));
    *gr->flag_host = 0;
    fill_u32(gr->f->ctr(0), 0u, C_COUNT, s);
    RTG_TRY(check_launch("graph counters"));
    HIP_TRY(hipStreamSynchronize(s));
    return RTG_OK;
}

// RTG_ERR_CAPACITY (RTG_ERR_UNSUPPORTED for counts of 2^31 or more) once a
// replay has reported an overflow.  Never waits: the device flags word is
// sticky and copied to the pinned word at the end of every replay, so the
// pinned word only ever goes from zero to non-zero, and reading it at any time
// reports every overflow of the replays whose copy has landed.
rtg_status graph_check_flags(rtg_graph* gr) {
    const uint32_t fl = *(volatile uint32_t*)gr->flag_host;
    if (!fl) return RTG_OK;
    if (fl & FLAG_COUNT_OVERFLOW) return flags_status(fl);
    return set_err(RTG_ERR_CAPACITY, "a replay overflowed the graph's buffers (flags 0x%x); create a larger graph",
                   fl);
}

// The batched scoring pipeline with fixed grids and device-side sizes.
rtg_status enqueue_graph_body(rtg_graph* gr, hipStream_t s) {
    rtg_frame* f = gr->f.get();
    RTG_TRY(enqueue_project(f, false, s));
    RTG_TRY(enqueue_bin(f, false, s));
    score_tiles(f->st.tile_w, f->st.tile_h, f->st.batch, gr->mode, true, gr->grid, f->views.as<ViewDev>(),
                gr->max_views,
                f->hdr.as<Header>(), 0, 0, f->ranges.as<uint2>(), f->tile_ord.as<uint32_t>(), f->sorted_irec(), f->records(), to_dev(f->st),
                f->score_part.as<double>(), f->ctr(C_QUEUE), f->ctr(C_FLAGS), s);
    score_reduce(f->views.as<ViewDev>(), f->hdr.as<Header>(), gr->max_views, f->score_part.as<double>(),
                 gr->scores.as<double>(), f->ctr(C_FLAGS), s);
    HIP_TRY(hipMemcpyAsync(gr->flag_host, f->ctr(C_FLAGS), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    return check_launch("graph body");
}

rtg_status graph_layout(rtg_graph* gr, const rtg_camera* cams, int n_views) {
    rtg_frame* f = gr->f.get();
    for (int v = 0; v < n_views; v++)
        if (cams[v].width > gr->max_w || cams[v].height > gr->max_h)
            return set_err(RTG_ERR_INVALID, "camera %d (%dx%d) exceeds the graph's %dx%d", v, cams[v].width,
                           cams[v].height, gr->max_w, gr->max_h);
    make_layout(cams, n_views, f->st.tile_w, f->st.tile_h, f->L);
    f->n_views = n_views;
    return RTG_OK;
}

}  // namespace

extern "C" {

rtg_status rtg_score_graph_create(rtg_ctx* ctx, const rtg_gaussians* g, int32_t max_views, int32_t max_width,
                                  int32_t max_height, const rtg_settings* settings, int32_t mode,
                                  const rtg_camera* probe, int32_t n_probe, rtg_graph** out, void* stream) {
    if (!out) return set_err(RTG_ERR_INVALID, "out is NULL");
    *out = nullptr;
    RTG_TRY(ctx_ok(ctx));
    if (mode != 0 && mode != 1) return set_err(RTG_ERR_INVALID, "score mode %d not in {0, 1}", mode);
    RTG_TRY(check_gauss(g, false, true));
    if (max_views < 1 || max_views > MAX_VIEWS) return set_err(RTG_ERR_INVALID, "max_views = %d", max_views);
    if (max_width < 1 || max_height < 1 || max_width > 16384 || max_height > 16384)
        return set_err(RTG_ERR_INVALID, "max size %dx%d", max_width, max_height);
    rtg_settings st;
    RTG_TRY(resolve_settings(ctx, settings, &st));
    hipStream_t s = (hipStream_t)stream;
    int64_t inst_cap = st.max_instances;
    int64_t rec_cap = 0;
    if (inst_cap <= 0) {
        if (!probe || n_probe < 1) return set_err(RTG_ERR_INVALID, "probe cameras needed when max_instances = 0");
        RTG_TRY(check_cams(probe, n_probe));
        rtg_frame* fp = nullptr;
        RTG_TRY(new_frame(ctx, g, probe, n_probe, &st, &fp, s));
        std::unique_ptr<rtg_frame> pf(fp);
        pf->scoring = true;
        RTG_TRY(enqueue_project(pf.get(), true, s));
        RTG_TRY(enqueue_bin(pf.get(), true, s));
        double scale = 2.0 * (double)max_views / (double)n_probe;
        inst_cap = (int64_t)std::ceil(scale * (double)std::max<int64_t>(pf->K, 1)) + 4096;
        rec_cap = (int64_t)std::ceil(scale * (double)std::max<uint32_t>(pf->R, 1)) + 4096;
    }
    int64_t full = g->n * (int64_t)max_views;
    if (rec_cap <= 0) rec_cap = std::min<int64_t>(full, inst_cap);
    rec_cap = std::min<int64_t>(rec_cap, std::max<int64_t>(full, 1));
    if (inst_cap >= ((int64_t)1 << 31) || rec_cap >= ((int64_t)1 << 31))
        return set_err(RTG_ERR_UNSUPPORTED, "capacity above 2^31 pairs");

    rtg_graph* gr = new (std::nothrow) rtg_graph();
    if (!gr) return set_err(RTG_ERR_OOM, "host allocation failed");
    gr->ctx = ctx;
    gr->mode = mode;
    gr->max_views = max_views;
    gr->max_w = max_width;
    gr->max_h = max_height;
    gr->f.reset(new (std::nothrow) rtg_frame());
    if (!gr->f) {
        graph_free(gr);
        return set_err(RTG_ERR_OOM, "host allocation failed");
    }
    rtg_frame* f = gr->f.get();
    f->ctx = ctx;
    f->g = *g;
    f->st = st;
    f->scoring = true;
    uint32_t tiles_per = (uint32_t)(((max_width + st.tile_w - 1) / st.tile_w) * ((max_height + st.tile_h - 1) / st.tile_h));
    uint32_t tiles_cap = tiles_per * (uint32_t)max_views;
    rtg_status rs = RTG_OK;
    auto fail = [&](rtg_status code) {
        graph_free(gr);
        return code;
    };
    if ((rs = frame_setup(f, max_views, s)) != RTG_OK) return fail(rs);
    if ((rs = alloc_records(f, (uint32_t)rec_cap)) != RTG_OK) return fail(rs);
    if ((rs = alloc_instances(f, (uint32_t)inst_cap, tiles_cap)) != RTG_OK) return fail(rs);
    if ((rs = f->score_part.ensure(ctx, sizeof(double) * tiles_cap)) != RTG_OK) return fail(rs);
    if ((rs = gr->scores.ensure(ctx, sizeof(double) * max_views)) != RTG_OK) return fail(rs);
    f->R = (uint32_t)rec_cap;
    f->K = inst_cap;
    // a placeholder layout for capture (kernels read the real one at replay)
    std::vector<rtg_camera> dummy(max_views);
    for (auto& c : dummy) {
        std::memset(&c, 0, sizeof(c));
        c.width = max_width;
        c.height = max_height;
        c.fx = c.fy = 1.0f;
        c.R[0] = c.R[4] = c.R[8] = 1.0f;
    }
    make_layout(dummy.data(), max_views, st.tile_w, st.tile_h, f->L);
    f->n_views = max_views;
    gr->grid = score_persistent_blocks(st.tile_w, st.tile_h, st.batch);
    if ((rs = graph_host_setup(gr, true, s)) != RTG_OK) return fail(rs);
    hipError_t e;
    if ((e = hipStreamBeginCapture(gr->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        graph_free(gr);
        return set_err(RTG_ERR_HIP, "begin capture failed: %s", hipGetErrorString(e));
    }
    ctx->capturing = true;
    rs = enqueue_graph_body(gr, gr->cap_stream);
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(gr->cap_stream, &graph);
    if (rs != RTG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        graph_free(gr);
        return rs;
    }
    if (e != hipSuccess) {
        graph_free(gr);
        return set_err(RTG_ERR_HIP, "end capture failed: %s", hipGetErrorString(e));
    }
    gr->graph = graph;
    if ((e = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        graph_free(gr);
        return set_err(RTG_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    *out = gr;
    return RTG_OK;
}

rtg_status rtg_score_graph_launch(rtg_graph* gr, const rtg_camera* cams, int32_t n_views, double* scores,
                                  void* stream) {
    if (!gr || gr->kind != 0) return set_err(RTG_ERR_INVALID, "not a scoring graph");
    RTG_TRY(ctx_ok(gr->ctx));
    RTG_TRY(check_cams(cams, n_views));
    if (n_views > gr->max_views) return set_err(RTG_ERR_INVALID, "n_views %d > graph capacity %d", n_views, gr->max_views);
    if (!scores) return set_err(RTG_ERR_INVALID, "scores is NULL");
    RTG_TRY(graph_check_flags(gr));
    hipStream_t s = (hipStream_t)stream;
    RTG_TRY(graph_layout(gr, cams, n_views));
    // this slot's pinned area may still feed the upload of the replay before
    // the previous one
    const int slot = (int)(gr->launches % rtg_graph::SLOTS);
    if (gr->launches >= rtg_graph::SLOTS) HIP_TRY(hipEventSynchronize(gr->done[slot]));
    std::memcpy(gr->staging[slot], gr->f->L.views.data(), sizeof(ViewDev) * n_views);
    *gr->staging_hdr[slot] = gr->f->L.hdr;
    HIP_TRY(hipMemcpyAsync(gr->f->views.p, gr->staging[slot], sizeof(ViewDev) * n_views, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(gr->f->hdr.p, gr->staging_hdr[slot], sizeof(Header), hipMemcpyHostToDevice, s));
    {
        Timer tm(gr->ctx, 7, s);
        HIP_TRY(hipGraphLaunch(gr->exec, s));
    }
    HIP_TRY(hipMemcpyAsync(scores, gr->scores.p, sizeof(double) * n_views, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipEventRecord(gr->done[slot], s));
    gr->launches++;
    gr->launched = true;
    gr->last_views = n_views;
    return RTG_OK;
}

rtg_status rtg_score_graph_status(rtg_graph* gr) {
    if (!gr) return set_err(RTG_ERR_INVALID, "graph is NULL");
    if (!gr->launched) return RTG_OK;
    HIP_TRY(hipEventSynchronize(gr->done[gr->last_slot()]));
    return graph_check_flags(gr);
}

void rtg_score_graph_destroy(rtg_graph* gr) { graph_free(gr); }

// The captured mapping iteration, with the loss of rtg_loss (eq4 false) or rtg_loss_ssim (eq4 true).
static rtg_status map_graph_build(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int32_t n_views,
                                  const rtg_settings* settings, const float* target_rgb, const float* target_depth,
                                  float w_depth, bool eq4, float lambda_1, float lambda_2, float* rgb, float* depth,
                                  double* loss, const rtg_grads* grads, rtg_graph** out, void* stream) {
    if (!out) return set_err(RTG_ERR_INVALID, "out is NULL");
    *out = nullptr;
    RTG_TRY(ctx_ok(ctx));
    RTG_TRY(check_gauss(g, true, false));
    RTG_TRY(check_cams(cams, n_views));
    if (!target_rgb || !target_depth || !rgb || !depth || !loss || !grads)
        return set_err(RTG_ERR_INVALID, "targets, outputs, loss and grads must be non-NULL");
    if (!std::isfinite(w_depth) || !std::isfinite(lambda_1) || !std::isfinite(lambda_2))
        return set_err(RTG_ERR_INVALID, "w_depth, lambda_1 and lambda_2 must be finite");
    rtg_settings st;
    RTG_TRY(resolve_settings(ctx, settings, &st));
    hipStream_t s = (hipStream_t)stream;
    // eager pass to size the capacities
    int64_t R0, K0;
    {
        rtg_frame* fp = nullptr;
        RTG_TRY(new_frame(ctx, g, cams, n_views, &st, &fp, s));
        std::unique_ptr<rtg_frame> pf(fp);
        RTG_TRY(enqueue_project(pf.get(), true, s));
        RTG_TRY(enqueue_bin(pf.get(), true, s));
        R0 = pf->R;
        K0 = pf->K;
    }
    int64_t rec_cap = std::min<int64_t>(g->n * (int64_t)n_views, R0 + R0 / 2 + 4096);
    int64_t inst_cap = K0 + K0 / 2 + 16384;
    if (st.max_instances > 0) {  // explicit capacity
        inst_cap = st.max_instances;
        rec_cap = std::min<int64_t>(rec_cap, inst_cap);
    }
    rec_cap = std::max<int64_t>(rec_cap, 1);
    if (inst_cap >= ((int64_t)1 << 31)) return set_err(RTG_ERR_UNSUPPORTED, "capacity above 2^31 pairs");

    rtg_graph* gr = new (std::nothrow) rtg_graph();
    if (!gr) return set_err(RTG_ERR_OOM, "host allocation failed");
    gr->kind = 1;
    gr->ctx = ctx;
    rtg_frame* fp = nullptr;
    rtg_status rs = new_frame(ctx, g, cams, n_views, &st, &fp, s);
    if (rs != RTG_OK) {
        graph_free(gr);
        return rs;
    }
    gr->f.reset(fp);
    rtg_frame* f = fp;
    auto fail = [&](rtg_status code) {
        graph_free(gr);
        return code;
    };
    const uint64_t P = f->L.hdr.pix_total;
    const int bx = (f->L.max_pix + 255) / 256;
    int max_w = 0, max_h = 0;
    for (const ViewDev& v : f->L.views) {
        max_w = std::max(max_w, (int)v.W);
        max_h = std::max(max_h, (int)v.H);
    }
    const int bpv = ssim_blocks_per_view(max_w, max_h);
    const int n_part = std::max(1, (eq4 ? bpv : bx) * n_views);
    if (eq4 && (rs = f->ssim_maps.ensure(ctx, sizeof(float) * 9 * (size_t)std::max<uint64_t>(P, 1))) != RTG_OK)
        return fail(rs);
    if ((rs = alloc_records(f, (uint32_t)rec_cap)) != RTG_OK) return fail(rs);
    if ((rs = alloc_instances(f, (uint32_t)inst_cap, f->L.hdr.tiles_total)) != RTG_OK) return fail(rs);
    if ((rs = ensure_pixel_state(f)) != RTG_OK) return fail(rs);
    if ((rs = f->g2d.ensure(ctx, sizeof(double) * G2D_STRIDE * (size_t)rec_cap)) != RTG_OK) return fail(rs);
    if ((rs = f->loss_part.ensure(ctx, sizeof(double) * (size_t)n_part)) != RTG_OK) return fail(rs);
    if ((rs = f->d_img.ensure(ctx, sizeof(float) * 4 * (size_t)std::max<uint64_t>(P, 1))) != RTG_OK) return fail(rs);
    f->R = (uint32_t)rec_cap;
    f->K = inst_cap;
    if ((rs = graph_host_setup(gr, false, s)) != RTG_OK) return fail(rs);
    hipError_t e;
    if ((e = hipStreamBeginCapture(gr->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        graph_free(gr);
        return set_err(RTG_ERR_HIP, "begin capture failed: %s", hipGetErrorString(e));
    }
    ctx->capturing = true;
    hipStream_t cs = gr->cap_stream;
    float* d_rgb = f->d_img.as<float>();
    float* d_dep = d_rgb + 3 * P;
    rs = enqueue_project(f, false, cs);
    if (rs == RTG_OK) rs = enqueue_bin(f, false, cs);
    if (rs == RTG_OK) {
        RenderOut o{rgb, depth, nullptr, nullptr, f->T_final.as<float>(), f->n_last.as<uint32_t>(),
                    f->n_contrib.as<uint32_t>()};
        render_forward(st.tile_w, st.tile_h, st.batch, f->views.as<ViewDev>(), n_views, f->L.hdr.tiles_total,
                       f->ranges.as<uint2>(), f->tile_ord.as<uint32_t>(), f->sorted_irec(), f->records(), to_dev(st), o, f->ctr(C_FLAGS), cs);
        if (eq4)
            loss_ssim(f->views.as<ViewDev>(), n_views, bpv, P, rgb, depth, target_rgb, target_depth, w_depth,
                      lambda_1, lambda_2, f->ssim_maps.as<float>(), f->loss_part.as<double>(), d_rgb, d_dep, loss,
                      cs);
        else
            loss_l1(f->views.as<ViewDev>(), n_views, f->L.max_pix, rgb, depth, target_rgb, target_depth, w_depth,
                    d_rgb, d_dep, f->loss_part.as<double>(), bx * n_views, loss, cs);
        fill_u32(f->g2d.as<uint32_t>(), 0u, (uint64_t)2 * G2D_STRIDE * rec_cap, cs);
        render_backward(st.tile_w, st.tile_h, st.batch, f->views.as<ViewDev>(), n_views, f->L.hdr.tiles_total,
                        f->ranges.as<uint2>(), f->tile_ord.as<uint32_t>(), f->sorted_irec(), f->records(), to_dev(st), f->T_final.as<float>(),
                        f->n_last.as<uint32_t>(), d_rgb, d_dep, nullptr, nullptr, f->g2d.as<double>(), f->ctr(C_FLAGS),
                        cs);
        project_backward(to_dev(f->g), f->views.as<ViewDev>(), to_dev(st), f->rec_off.as<uint32_t>(),
                         f->cnt.as<uint32_t>(), f->emit.as<EmitRec>(), f->g2d.as<double>(), grads->d_means,
                         grads->d_log_scales, grads->d_quats, grads->d_opacity, grads->d_colors, f->ctr(C_FLAGS), cs);
        e = hipMemcpyAsync(gr->flag_host, f->ctr(C_FLAGS), sizeof(uint32_t), hipMemcpyDeviceToHost, cs);
        if (e != hipSuccess) rs = set_err(RTG_ERR_HIP, "flag copy failed: %s", hipGetErrorString(e));
        if (rs == RTG_OK) rs = check_launch("mapping graph body");
    }
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (rs != RTG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        graph_free(gr);
        return rs;
    }
    if (e != hipSuccess) {
        graph_free(gr);
        return set_err(RTG_ERR_HIP, "end capture failed: %s", hipGetErrorString(e));
    }
    gr->graph = graph;
    if ((e = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        graph_free(gr);
        return set_err(RTG_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    *out = gr;
    return RTG_OK;
}

rtg_status rtg_map_graph_create(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int32_t n_views,
                                const rtg_settings* settings, const float* target_rgb, const float* target_depth,
                                float w_depth, float* rgb, float* depth, double* loss, const rtg_grads* grads,
                                rtg_graph** out, void* stream) {
    return map_graph_build(ctx, g, cams, n_views, settings, target_rgb, target_depth, w_depth, false, 1.0f, 0.0f,
                           rgb, depth, loss, grads, out, stream);
}

rtg_status rtg_map_graph_create_ssim(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int32_t n_views,
                                     const rtg_settings* settings, const float* target_rgb, const float* target_depth,
                                     float w_depth, float lambda_1, float lambda_2, float* rgb, float* depth,
                                     double* loss, const rtg_grads* grads, rtg_graph** out, void* stream) {
    return map_graph_build(ctx, g, cams, n_views, settings, target_rgb, target_depth, w_depth, true, lambda_1,
                           lambda_2, rgb, depth, loss, grads, out, stream);
}

rtg_status rtg_map_graph_launch(rtg_graph* gr, void* stream) {
    if (!gr || gr->kind != 1) return set_err(RTG_ERR_INVALID, "not a mapping graph");
    RTG_TRY(ctx_ok(gr->ctx));
    RTG_TRY(graph_check_flags(gr));
    hipStream_t s = (hipStream_t)stream;
    {
        Timer tm(gr->ctx, 8, s);
        HIP_TRY(hipGraphLaunch(gr->exec, s));
    }
    const int slot = (int)(gr->launches % rtg_graph::SLOTS);
    HIP_TRY(hipEventRecord(gr->done[slot], s));
    gr->launches++;
    gr->launched = true;
    return RTG_OK;
}

rtg_status rtg_map_graph_status(rtg_graph* gr) {
    if (!gr || gr->kind != 1) return set_err(RTG_ERR_INVALID, "not a mapping graph");
    return rtg_score_graph_status(gr);
}

void rtg_map_graph_destroy(rtg_graph* gr) { graph_free(gr); }

// ============================================================== autotune

rtg_status rtg_autotune(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int32_t n_views, int32_t mode,
                        rtg_settings* settings, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    RTG_TRY(check_gauss(g, mode != 2, mode == 2));
    RTG_TRY(check_cams(cams, n_views));
    if (!settings) return set_err(RTG_ERR_INVALID, "settings is NULL");
    if (mode < 0 || mode > 2) return set_err(RTG_ERR_INVALID, "mode %d not in {0, 1, 2}", mode);
    hipStream_t s = (hipStream_t)stream;
    static const int tiles[3][2] = {{8, 8}, {16, 16}, {32, 8}};
    uint64_t pix = 0;
    for (int v = 0; v < n_views; v++) pix += (uint64_t)cams[v].width * cams[v].height;
    // scratch images and gradients for the timed runs
    Buf img, grads, scores, dimg;
    RTG_TRY(img.ensure(ctx, sizeof(float) * 6 * std::max<uint64_t>(pix, 1)));
    RTG_TRY(dimg.ensure(ctx, sizeof(float) * 4 * std::max<uint64_t>(pix, 1)));
    RTG_TRY(grads.ensure(ctx, sizeof(float) * 14 * std::max<int64_t>(g->n, 1)));
    RTG_TRY(scores.ensure(ctx, sizeof(double) * n_views));
    float* im = img.as<float>();
    fill_u32(dimg.as<uint32_t>(), 0x3a800000u /* 2^-10 */, 4 * pix, s);
    fill_u32(grads.as<uint32_t>(), 0u, 14 * (uint64_t)std::max<int64_t>(g->n, 1), s);
    float* gp = grads.as<float>();
    rtg_grads gr{gp, gp + 3 * g->n, gp + 6 * g->n, gp + 10 * g->n, gp + 11 * g->n};
    // The cost of a candidate is the device time of its kernels, read from
    // the library's per-group event timers: the eager calls' host reads of
    // the pair counts are left out, so this is the work a captured graph of
    // the same call replays.  The caller's timer totals are kept aside.
    drain_timers(ctx);
    const bool was_timing = ctx->timing;
    double saved_ms[N_TIMERS];
    int64_t saved_n[N_TIMERS];
    for (int i = 0; i < N_TIMERS; i++) {
        saved_ms[i] = ctx->timer_ms[i];
        saved_n[i] = ctx->timer_n[i];
    }
    ctx->timing = true;
    auto device_ms = [&]() {
        drain_timers(ctx);
        double t = 0.0;
        for (int i = 0; i < N_TIMERS; i++) t += ctx->timer_ms[i];
        return t;
    };
    auto run_once = [&](const rtg_settings& st) -> rtg_status {
        if (mode == 2) return rtg_score_views(ctx, g, cams, n_views, &st, scores.as<double>(), 1, 0, stream);
        rtg_frame* f = nullptr;
        rtg_status r = rtg_project(ctx, g, cams, n_views, &st, &f, stream);
        if (r == RTG_OK) r = rtg_bin_sort(ctx, f, nullptr, stream);
        if (r == RTG_OK) r = rtg_render(ctx, f, im, im + 3 * pix, im + 4 * pix, g->uncert ? im + 5 * pix : nullptr, stream);
        if (r == RTG_OK && mode == 1) {
            float* d = dimg.as<float>();
            r = rtg_render_backward(ctx, f, d, d + 3 * pix, nullptr, nullptr, &gr, stream);
        }
        rtg_frame_destroy(f);
        return r;
    };
    // one warm-up call, then the median of three timed ones
    auto time_it = [&](const rtg_settings& st, double& ms) -> rtg_status {
        double t[3];
        for (int rep = 0; rep < 4; rep++) {
            const double before = device_ms();
            RTG_TRY(run_once(st));
            const double after = device_ms();
            if (rep > 0) t[rep - 1] = after - before;
        }
        std::sort(t, t + 3);
        ms = t[1];
        return RTG_OK;
    };
    // every tile with every staging batch below its pixel count (0: one
    // splat per thread of the tile)
    static const int batches[4] = {0, 32, 64, 128};
    double best = 1e300;
    int bi = 1, bb = 0;
    rtg_status rs = RTG_OK;
    for (int t = 0; t < 3 && rs == RTG_OK; t++) {
        for (int k = 0; k < 4 && rs == RTG_OK; k++) {
            if (batches[k] >= tiles[t][0] * tiles[t][1]) continue;
            rtg_settings st = *settings;
            st.tile_w = tiles[t][0];
            st.tile_h = tiles[t][1];
            st.batch = batches[k];
            double ms = 0.0;
            rs = time_it(st, ms);
            if (rs == RTG_OK && ms < best) {
                best = ms;
                bi = t;
                bb = batches[k];
            }
        }
    }
    drain_timers(ctx);
    ctx->timing = was_timing;
    for (int i = 0; i < N_TIMERS; i++) {
        ctx->timer_ms[i] = saved_ms[i];
        ctx->timer_n[i] = saved_n[i];
    }
    if (rs != RTG_OK) return rs;
    settings->tile_w = tiles[bi][0];
    settings->tile_h = tiles[bi][1];
    settings->batch = bb;
    ctx->last_tw = tiles[bi][0];
    ctx->last_th = tiles[bi][1];
    ctx->last_batch = bb;
    return RTG_OK;
}

}  // extern "C"

// ========================================================== view utility

extern "C" {

rtg_status rtg_uncertainty_thresholds(rtg_ctx* ctx, const float* uncert, int64_t n, double k_std, double* lo_hi,
                                      void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (n < 0) return set_err(RTG_ERR_INVALID, "n < 0");
    if (n > 0 && !uncert) return set_err(RTG_ERR_INVALID, "uncert is NULL");
    if (!lo_hi) return set_err(RTG_ERR_INVALID, "lo_hi is NULL");
    if (!std::isfinite(k_std)) return set_err(RTG_ERR_INVALID, "k_std is not finite");
    Buf scratch;
    RTG_TRY(scratch.ensure(ctx, sizeof(double) * 520));
    uncertainty_thresholds(uncert, n, k_std, scratch.as<double>(), lo_hi, (hipStream_t)stream);
    return check_launch("uncertainty thresholds");
}

rtg_status rtg_view_utility(rtg_ctx* ctx, const rtg_gaussians* g, const rtg_camera* cams, int32_t n_views,
                            const rtg_settings* settings, float range, const double* lo_hi, double lambda_xi,
                            int64_t* n_high, int64_t* n_low, double* sum_u, double* xi, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    RTG_TRY(check_gauss(g, false, true));
    RTG_TRY(check_cams(cams, n_views));
    if (!lo_hi) return set_err(RTG_ERR_INVALID, "lo_hi is NULL");
    if (!(range > 0.0f) || !std::isfinite(range)) return set_err(RTG_ERR_INVALID, "range must be finite and > 0");
    if (!std::isfinite(lambda_xi)) return set_err(RTG_ERR_INVALID, "lambda_xi is not finite");
    rtg_settings st;
    RTG_TRY(resolve_settings(ctx, settings, &st));
    hipStream_t s = (hipStream_t)stream;
    Layout L;
    make_layout(cams, n_views, st.tile_w, st.tile_h, L);
    Buf views, acc;
    RTG_TRY(views.ensure(ctx, sizeof(ViewDev) * n_views));
    RTG_TRY(acc.ensure(ctx, sizeof(unsigned long long) * 3 * n_views));
    HIP_TRY(hipMemcpyAsync(views.p, L.views.data(), sizeof(ViewDev) * n_views, hipMemcpyHostToDevice, s));
    view_utility(to_dev(*g), views.as<ViewDev>(), n_views, st.z_near, range, lo_hi, acc.as<unsigned long long>(),
                 lambda_xi, n_high, n_low, sum_u, xi, s);
    return check_launch("view utility");
}

rtg_status rtg_uncertainty_update(rtg_ctx* ctx, int64_t n, const float* means_prev, const float* means_cur,
                                  const float* u_prev, int32_t squared, float* u_out, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (n < 0) return set_err(RTG_ERR_INVALID, "n = %lld < 0", (long long)n);
    if (n > 0 && (!means_prev || !means_cur || !u_prev || !u_out))
        return set_err(RTG_ERR_INVALID, "means_prev, means_cur, u_prev and u_out must be non-NULL");
    uncertainty_update(n, means_prev, means_cur, u_prev, squared ? 1 : 0, u_out, (hipStream_t)stream);
    return check_launch("uncertainty update");
}

rtg_status rtg_region_grid(const double* box, double size, int32_t* dims) {
    if (!box || !dims) return set_err(RTG_ERR_INVALID, "box and dims must be non-NULL");
    if (!(size > 0.0) || !std::isfinite(size)) return set_err(RTG_ERR_INVALID, "size must be finite and > 0");
    int64_t nr = 1;
    for (int a = 0; a < 3; a++) {
        const double e = (box[3 + a] - box[a]) / size;
        if (!(e > 0.0) || !(e <= 65536.0)) return set_err(RTG_ERR_INVALID, "box axis %d: extent / size = %g", a, e);
        dims[a] = (int32_t)std::ceil(e);
        nr *= dims[a];
    }
    if (nr > ((int64_t)1 << 28)) return set_err(RTG_ERR_UNSUPPORTED, "%lld regions", (long long)nr);
    return RTG_OK;
}

rtg_status rtg_region_utility(rtg_ctx* ctx, int64_t n, const float* means, const float* u, const double* box,
                              double size, int64_t* count, double* sum, double* mean, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (n < 0) return set_err(RTG_ERR_INVALID, "n = %lld < 0", (long long)n);
    if (n > 0 && (!means || !u)) return set_err(RTG_ERR_INVALID, "means and u must be non-NULL");
    int32_t dims[3];
    RTG_TRY(rtg_region_grid(box, size, dims));
    const int64_t nr = (int64_t)dims[0] * dims[1] * dims[2];
    hipStream_t s = (hipStream_t)stream;
    Buf acc;
    RTG_TRY(acc.ensure(ctx, (2 * sizeof(unsigned long long) + sizeof(unsigned int)) * (size_t)nr));
    unsigned long long* cnt = acc.as<unsigned long long>();
    int dm[3] = {dims[0], dims[1], dims[2]};
    region_utility(n, means, u, box, size, dm, cnt, cnt + nr, reinterpret_cast<unsigned int*>(cnt + 2 * nr), count,
                   sum, mean, s);
    return check_launch("region utility");
}

rtg_status rtg_collision_check(rtg_ctx* ctx, const rtg_gaussians* g, const float* points, int64_t n_points,
                               float r_robot, float lambda_g, int32_t* collide, float* clearance, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    RTG_TRY(collision_args(g, points, n_points, r_robot, lambda_g, collide));
    if (n_points == 0) return RTG_OK;
    hipStream_t s = (hipStream_t)stream;
    Buf packed, bound, key;
    RTG_TRY(packed.ensure(ctx, sizeof(float4) * (size_t)std::max<int64_t>(g->n, 1)));
    RTG_TRY(bound.ensure(ctx, sizeof(float2) * (size_t)std::max<int64_t>(g->n, 1)));
    RTG_TRY(key.ensure(ctx, sizeof(uint32_t) * (size_t)n_points));
    collision_check(to_dev(*g), points, n_points, r_robot, lambda_g, packed.as<float4>(), bound.as<float2>(), collide,
                    key.as<uint32_t>(), clearance, s);
    return check_launch("collision check");
}

rtg_status rtg_collision_check_noalloc(rtg_ctx* ctx, const rtg_gaussians* g, const float* points, int64_t n_points,
                                       float r_robot, float lambda_g, int32_t* collide, float* clearance,
                                       void* stream) {
    RTG_TRY(ctx_ok(ctx));
    RTG_TRY(collision_args(g, points, n_points, r_robot, lambda_g, collide));
    // the same three scratch arrays as rtg_collision_check, carved from the
    // fixed array: packed (16 B per Gaussian), bound (8 B), clear_key (4 B
    // per point); the kernels write all of them before reading them
    const size_t n = (size_t)g->n, np = (size_t)n_points;
    const size_t off_bound = align256(16 * n), off_key = off_bound + align256(8 * n);
    const size_t need = off_key + align256(4 * np);
    if (need > SCRATCH_BYTES)
        return set_err(RTG_ERR_UNSUPPORTED,
                       "%lld Gaussians and %lld points need %zu bytes of scratch, above the fixed %zu "
                       "(24 bytes per Gaussian + 4 per point); use rtg_collision_check",
                       (long long)g->n, (long long)n_points, need, SCRATCH_BYTES);
    if (n_points == 0) return RTG_OK;
    if (!ctx->scratch) {
        void* p = nullptr;
        RTG_TRY(scratch_address(ctx->device, &p));
        ctx->scratch = p;
    }
    unsigned char* base = static_cast<unsigned char*>(ctx->scratch);
    collision_check(to_dev(*g), points, n_points, r_robot, lambda_g, reinterpret_cast<float4*>(base),
                    reinterpret_cast<float2*>(base + off_bound), collide, reinterpret_cast<uint32_t*>(base + off_key),
                    clearance, (hipStream_t)stream);
    return check_launch("collision check (fixed scratch)");
}

rtg_status rtg_trajectory_select(rtg_ctx* ctx, const double* xi, const int32_t* offsets, int32_t n_traj,
                                 double* traj_utility, int32_t* best, void* stream) {
    RTG_TRY(ctx_ok(ctx));
    if (!xi || !offsets || !best) return set_err(RTG_ERR_INVALID, "xi, offsets and best must be non-NULL");
    if (n_traj < 1) return set_err(RTG_ERR_INVALID, "n_traj = %d < 1", n_traj);
    trajectory_select(xi, offsets, n_traj, traj_utility, best, (hipStream_t)stream);
    return check_launch("trajectory select");
}

}  // extern "C"
