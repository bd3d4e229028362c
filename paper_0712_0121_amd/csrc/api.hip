// C interface: argument checks, decomposition of an operation into kernel
// launches, workspace sizing, batch plans.  Declarations and the contract
// of every entry point are in include/morph.h.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

namespace morph {

static thread_local char g_hip_err[256] = "";

bool trace_pause();                 // tracing off; returns the previous state
void trace_resume(bool prev);        // (both defined with the tracing code)

void set_hip_error(hipError_t e)
{
    std::snprintf(g_hip_err, sizeof g_hip_err, "%s (%d)", hipGetErrorString(e), (int)e);
}

// ------------------------------------------------------------ pass planning
// A rectangle operation is a sequence of erosion passes, each in the image
// domain (dom 0) or in the complement domain (dom 1: dilation by B is the
// complement of erosion of the complement by the reflected element B^).
// An element whose origin is more than 64 pixels from a side of the row
// window, or taller than the vertical limit, is split by the composition
// law  op_{B1 (+) B2} = op_{B2} . op_{B1}  with
// B1 (+) B2 = (w1+w2-1, h1+h2-1, cx1+cx2, cy1+cy2).
struct Pass {
    Stage st;
    int dom;
};

constexpr int kVReachMax = 128;

static void decompose(Stage B, int dom, std::vector<Pass> &out)
{
    int l = B.cx, r = B.w - 1 - B.cx, t = B.cy, b = B.h - 1 - B.cy;
    bool first = true;
    while (first || l > 0 || r > 0 || t > 0 || b > 0) {
        const int pl = std::min(l, kReachMax), pr = std::min(r, kReachMax);
        const int pt = std::min(t, kVReachMax), pb = std::min(b, kVReachMax);
        out.push_back({Stage{pl + pr + 1, pt + pb + 1, pl, pt}, dom});
        l -= pl; r -= pr; t -= pt; b -= pb;
        first = false;
    }
}

static std::vector<Pass> op_passes(int op, morph_se_t se)
{
    const Stage B{se.w, se.h, se.cx, se.cy};
    const Stage R{se.w, se.h, se.w - 1 - se.cx, se.h - 1 - se.cy};
    std::vector<Pass> v;
    switch (op) {
    case MORPH_ERODE: decompose(B, 0, v); break;
    case MORPH_DILATE: decompose(R, 1, v); break;
    case MORPH_OPEN: decompose(B, 0, v); decompose(R, 1, v); break;
    case MORPH_CLOSE: decompose(R, 1, v); decompose(B, 0, v); break;
    }
    return v;
}

struct Launch {
    RectPage p;
};

// Groups passes into launches (two per launch when a tile fits both) and
// fills in complement flags and tile shapes.  Buffers are set by the caller.
// With small_tiles, a one-stage launch whose halo rows stay under a fifth
// of a small tile runs four 256-thread workgroups per CU instead of two
// 512-thread ones (measured a few percent faster for short elements; the
// number of launches does not change).  With by_halo (single operations and
// their workspace query, not batch pages, which need one launch each), two
// stages whose halo rows pass 0.6 of a fused tile's rows run as two launches.
static bool plan_launches(int op, morph_se_t se, int W, int H, int npages, int tile_rows,
                          int strip_words, std::vector<Launch> &out, bool small_tiles = false,
                          bool by_halo = false)
{
    const std::vector<Pass> ps = op_passes(op, se);
    const int nw = (W + 63) / 64;
    RectPage base{};
    base.W = W;
    base.H = H;
    base.nw = nw;
    base.padmask = (W % 64) ? ((1ull << (W % 64)) - 1) : ~0ull;
    int stored_dom = 0;
    size_t i = 0;
    while (i < ps.size()) {
        RectPage p = base;
        bool fused = false;
        if (i + 1 < ps.size()) {
            p.nst = 2;
            p.st[0] = ps[i].st;
            p.st[1] = ps[i + 1].st;
            RectPage q = p;
            bool share = plan_tiles(q, tile_rows, strip_words, npages);
            if (share) {
                // whether two stages share a tile depends on the element and
                // the page width only, never on the page height: the
                // workspace query sees a stack's total rows, the operation
                // one page's.  r.TR is the most output rows a fused tile
                // can hold.  With by_halo, the stages share a tile only
                // while their halo rows (h1 - 1 + h2 - 1) stay within 0.6 of
                // those: beyond that the first stage recomputes more rows
                // than two single-stage launches cost with the
                // intermediate's round trip through HBM.  Letter pages:
                // opening by 51 x 51, 100 halo rows over fused tiles of 120
                // rows, 0.42 ms fused and 0.35 ms as two launches; by 31 x 1,
                // 60 over 160, 0.23 ms fused and 0.28 ms as two launches.
                RectPage r = p;
                r.H = 1 << 30;
                share = plan_tiles(r, 1 << 30, strip_words, npages) && r.TR >= 8 &&
                        (!by_halo || 5 * (ps[i].st.h - 1 + ps[i + 1].st.h - 1) <= 3 * r.TR);
            }
            if (share) {
                p = q;
                fused = true;
            }
        }
        if (!fused) {
            p.nst = 1;
            p.st[0] = ps[i].st;
            if (!plan_tiles(p, tile_rows, strip_words, npages)) return false;
        }
        if (small_tiles && tile_rows == 0 && strip_words == 0 && p.nst == 1) {
            int hsum = 0;
            for (int k = 0; k < p.nst; k++) hsum += p.st[k].h - 1;
            RectPage q = p;
            if (plan_tiles(q, 0, 0, npages, kThreadsSmall) && q.TR >= 32 && 5 * hsum <= q.TR) p = q;
        }
        const size_t last = i + p.nst - 1;
        const int out_dom = (last + 1 < ps.size()) ? ps[last + 1].dom : 0;
        p.in_c = ps[i].dom != stored_dom;
        p.mid_c = (p.nst == 2) && (ps[i + 1].dom != ps[i].dom);
        p.out_c = ps[last].dom != out_dom;
        stored_dom = out_dom;
        out.push_back(Launch{p});
        i = last + 1;
    }
    return true;
}

static size_t image_bytes(int W, int rows) { return (size_t)((W + 63) / 64) * (size_t)rows * 8; }

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

static bool se_ok(morph_se_t se)
{
    return se.w >= 1 && se.h >= 1 && se.cx >= 0 && se.cy >= 0 && se.cx < se.w && se.cy < se.h;
}

static bool bitmap_ok(const morph_bitmap_t *b)
{
    if (!b || !b->words) return false;
    if (b->width < 1 || b->height < 1 || b->npages < 1) return false;
    if (b->stride_words < (b->width + 63) / 64) return false;
    if (((uintptr_t)b->words) & 7) return false;
    if ((long long)b->height * b->npages > 0x7fffffffLL) return false;
    return true;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

static size_t bitmap_extent(const morph_bitmap_t *b)
{
    const size_t rows = (size_t)b->height * b->npages;
    return ((rows - 1) * b->stride_words + (b->width + 63) / 64) * 8;
}

static int rect_packed(int op, const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                       void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!bitmap_ok(dst) || !bitmap_ok(src) || !se_ok(se)) return MORPH_E_INVAL;
    if (dst->width != src->width || dst->height != src->height || dst->npages != src->npages)
        return MORPH_E_SHAPE;
    if (overlap(dst->words, bitmap_extent(dst), src->words, bitmap_extent(src))) return MORPH_E_ALIAS;
    std::vector<Launch> L;
    if (!plan_launches(op, se, src->width, src->height, src->npages, 0, 0, L, true, true))
        return MORPH_E_UNSUPPORTED;
    const int W = src->width, H = src->height, P = src->npages, nw = (W + 63) / 64;
    const size_t img = round256(image_bytes(W, H * P));
    const size_t need = L.size() <= 1 ? 0 : (L.size() == 2 ? img : 2 * img);
    if (need > 0 && (ws == nullptr || ws_bytes < need)) return MORPH_E_WORKSPACE;
    uint64_t *tmp[2] = {(uint64_t *)ws, (uint64_t *)((char *)ws + img)};
    const uint64_t *in = src->words;
    int in_stride = src->stride_words;
    for (size_t k = 0; k < L.size(); k++) {
        RectPage p = L[k].p;
        const bool lastl = k + 1 == L.size();
        uint64_t *out = lastl ? dst->words : tmp[k & 1];
        const int out_stride = lastl ? dst->stride_words : nw;
        p.src = in;
        p.dst = out;
        p.sstride = in_stride;
        p.dstride = out_stride;
        p.src_page_words = (long long)in_stride * H;
        p.dst_page_words = (long long)out_stride * H;
        hipError_t e = launch_rect(p, P, stream);
        if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
        in = out;
        in_stride = out_stride;
    }
    return MORPH_OK;
}

// ------------------------------------------------------------------ batches
}  // namespace morph

struct morph_batch_plan {
    morph::RectPage *pages_dev = nullptr;
    morph::TileRef *tiles_dev = nullptr;
    int *queue_dev = nullptr;
    int ntiles = 0;
    int nblocks = 0;
    double alg_bytes = 0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace morph;

extern "C" {

const char *morph_version(void) { return "morph 0.1 (gfx950, HIP)"; }

int morph_copy_async(void *dst, const void *src, size_t bytes, morph_stream_t stream)
{
    if (bytes == 0) return MORPH_OK;
    if (!dst || !src) return MORPH_E_INVAL;
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

const char *morph_strerror(int code)
{
    switch (code) {
    case MORPH_OK: return "ok";
    case MORPH_E_INVAL: return "invalid argument";
    case MORPH_E_SHAPE: return "dst and src sizes differ";
    case MORPH_E_ALIAS: return "dst overlaps src";
    case MORPH_E_WORKSPACE: return "workspace too small";
    case MORPH_E_NONCANONICAL: return "run-length image not canonical";
    case MORPH_E_CAPACITY: return "run capacity too small";
    case MORPH_E_HIP: return "HIP call failed";
    case MORPH_E_UNSUPPORTED: return "not supported";
    default: return "unknown error";
    }
}

const char *morph_last_hip_error(void) { return g_hip_err; }

int morph_erode_rect_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                            void *ws, size_t ws_bytes, morph_stream_t stream)
{
    return rect_packed(MORPH_ERODE, dst, src, se, ws, ws_bytes, (hipStream_t)stream);
}
int morph_dilate_rect_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                             void *ws, size_t ws_bytes, morph_stream_t stream)
{
    return rect_packed(MORPH_DILATE, dst, src, se, ws, ws_bytes, (hipStream_t)stream);
}
int morph_open_rect_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                           void *ws, size_t ws_bytes, morph_stream_t stream)
{
    return rect_packed(MORPH_OPEN, dst, src, se, ws, ws_bytes, (hipStream_t)stream);
}
int morph_close_rect_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_se_t se,
                            void *ws, size_t ws_bytes, morph_stream_t stream)
{
    return rect_packed(MORPH_CLOSE, dst, src, se, ws, ws_bytes, (hipStream_t)stream);
}

int64_t morph_rle_max_runs(int32_t width, int32_t height)
{
    if (width < 1 || height < 1) return 0;
    return (int64_t)height * ((width + 1) / 2);
}

size_t morph_workspace_bytes(int op, int repr, int32_t width, int32_t height, morph_se_t se)
{
    if (width < 1 || height < 1 || !se_ok(se) || op < MORPH_ERODE || op > MORPH_CLOSE) return 0;
    if (repr == MORPH_PACKED) {
        std::vector<Launch> L;
        if (!plan_launches(op, se, width, height, 1, 0, 0, L, false, true)) return 0;
        const size_t img = round256(image_bytes(width, height));
        return L.size() <= 1 ? 0 : (L.size() == 2 ? img : 2 * img);
    }
    return rle_op_workspace(op, width, height, height, se);
}

// ---- batch plans
}  // extern "C"

namespace morph {

// Plans a batch: one fused launch per page, tiles ordered with the most
// expensive pages first (their tiles leave the queue first) and each page's
// tiles in band order so neighbours run close together in time.
static int build_batch(const morph_page_desc_t *descs, int32_t n, std::vector<RectPage> &pages,
                       std::vector<TileRef> &tiles)
{
    if ((!descs && n > 0) || n < 0) return MORPH_E_INVAL;
    std::vector<double> cost;
    pages.clear();
    tiles.clear();
    for (int i = 0; i < n; i++) {
        const morph_page_desc_t &d = descs[i];
        if (!bitmap_ok(&d.dst) || !bitmap_ok(&d.src) || !se_ok(d.se) || d.op < MORPH_ERODE ||
            d.op > MORPH_CLOSE || d.src.npages != 1 || d.dst.npages != 1)
            return MORPH_E_INVAL;
        if (d.dst.width != d.src.width || d.dst.height != d.src.height) return MORPH_E_SHAPE;
        if (overlap(d.dst.words, bitmap_extent(&d.dst), d.src.words, bitmap_extent(&d.src)))
            return MORPH_E_ALIAS;
        std::vector<Launch> L;
        if (!plan_launches(d.op, d.se, d.src.width, d.src.height, n, d.tile_rows, d.strip_words, L) ||
            L.size() != 1)
            return MORPH_E_UNSUPPORTED;
        RectPage p = L[0].p;
        if (p.nt != kThreads || !tile_fits(p)) return MORPH_E_UNSUPPORTED;
        p.src = d.src.words;
        p.dst = d.dst.words;
        p.sstride = d.src.stride_words;
        p.dstride = d.dst.stride_words;
        p.src_page_words = 0;
        p.dst_page_words = 0;
        pages.push_back(p);
        double hs = 0, lg = 0;
        for (int s = 0; s < p.nst; s++) {
            hs += p.st[s].h - 1;
            lg += 2 + std::log2((double)p.st[s].w) + std::log2((double)p.st[s].h);
        }
        cost.push_back((double)p.nw * (p.H + hs * p.nbands) * lg);
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int i : order)
        for (int b = 0; b < pages[i].nbands; b++)
            for (int s = 0; s < pages[i].nstrips; s++) tiles.push_back(TileRef{i, b, s, 0});
    if (tiles.size() > 0x7fffffff) return MORPH_E_UNSUPPORTED;
    return MORPH_OK;
}

static double batch_alg_bytes(const std::vector<RectPage> &pages)
{
    double b = 0;
    for (const RectPage &p : pages) b += 16.0 * p.nw * (double)p.H;
    return b;
}

// Device layout of an uploaded batch: queue counter, page table, tile list.
static size_t batch_bytes(size_t npages, size_t ntiles)
{
    return 256 + round256(npages * sizeof(RectPage)) + round256(ntiles * sizeof(TileRef));
}

}  // namespace morph

extern "C" {

int morph_batch_plan_create(morph_batch_plan_t **plan, const morph_page_desc_t *descs, int32_t n,
                            morph_stream_t stream)
{
    (void)stream;
    if (!plan) return MORPH_E_INVAL;
    *plan = nullptr;
    std::vector<RectPage> pages;
    std::vector<TileRef> tiles;
    const int rc = build_batch(descs, n, pages, tiles);
    if (rc != MORPH_OK) return rc;
    morph_batch_plan_t *pl = new (std::nothrow) morph_batch_plan_t();
    if (!pl) return MORPH_E_HIP;
    hipError_t e = hipSuccess;
    const size_t pb = std::max<size_t>(1, pages.size()) * sizeof(RectPage);
    const size_t tb = std::max<size_t>(1, tiles.size()) * sizeof(TileRef);
    if ((e = hipMalloc(&pl->pages_dev, pb)) != hipSuccess ||
        (e = hipMalloc(&pl->tiles_dev, tb)) != hipSuccess ||
        (e = hipMalloc(&pl->queue_dev, 256)) != hipSuccess ||
        (n > 0 && (e = hipMemcpy(pl->pages_dev, pages.data(), pages.size() * sizeof(RectPage),
                                 hipMemcpyHostToDevice)) != hipSuccess) ||
        (!tiles.empty() && (e = hipMemcpy(pl->tiles_dev, tiles.data(), tiles.size() * sizeof(TileRef),
                                          hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipStreamCreateWithFlags(&pl->capture_stream, hipStreamNonBlocking)) != hipSuccess) {
        set_hip_error(e);
        morph_batch_plan_destroy(pl);
        return MORPH_E_HIP;
    }
    pl->ntiles = (int)tiles.size();
    pl->nblocks = std::max(1, std::min(pl->ntiles, 2 * device_cu_count()));
    for (const RectPage &p : pages) pl->alg_bytes += 16.0 * p.nw * (double)p.H;
    *plan = pl;
    return MORPH_OK;
}

int64_t morph_batch_workspace_bytes(const morph_page_desc_t *descs, int32_t n)
{
    std::vector<RectPage> pages;
    std::vector<TileRef> tiles;
    if (build_batch(descs, n, pages, tiles) != MORPH_OK) return -1;
    return (int64_t)batch_bytes(pages.size(), tiles.size());
}

int morph_batch_launch(const morph_page_desc_t *descs, int32_t n, void *ws, size_t ws_bytes,
                       void *host_staging, size_t staging_bytes, morph_stream_t stream)
{
    std::vector<RectPage> pages;
    std::vector<TileRef> tiles;
    const int rc = build_batch(descs, n, pages, tiles);
    if (rc != MORPH_OK) return rc;
    if (tiles.empty()) return MORPH_OK;
    const size_t need = batch_bytes(pages.size(), tiles.size());
    if (!ws || ws_bytes < need || (((uintptr_t)ws) & 255)) return MORPH_E_WORKSPACE;
    if (host_staging && staging_bytes < need) return MORPH_E_WORKSPACE;
    // table image: [256 bytes: counter] [pages] [tiles]
    const size_t po = 256, to = 256 + round256(pages.size() * sizeof(RectPage));
    std::vector<char> local;
    char *img;
    if (host_staging) {
        img = (char *)host_staging;
    } else {
        local.resize(need);
        img = local.data();
    }
    std::memcpy(img + po, pages.data(), pages.size() * sizeof(RectPage));
    std::memcpy(img + to, tiles.data(), tiles.size() * sizeof(TileRef));
    hipStream_t s = (hipStream_t)stream;
    char *d = (char *)ws;
    hipError_t e;
    if ((e = hipMemcpyAsync(d + po, img + po, need - po, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (!host_staging && (e = hipStreamSynchronize(s)) != hipSuccess) ||
        (e = launch_reset_counter((int *)d, s)) != hipSuccess ||
        (e = launch_rect_batch((const RectPage *)(d + po), (const TileRef *)(d + to), (int)tiles.size(),
                               (int *)d, std::max(1, std::min((int)tiles.size(), 2 * device_cu_count())), s,
                               batch_alg_bytes(pages))) != hipSuccess) {
        set_hip_error(e);
        return MORPH_E_HIP;
    }
    return MORPH_OK;
}

int64_t morph_batch_tiles(const morph_batch_plan_t *plan) { return plan ? plan->ntiles : 0; }

int morph_batch_run(morph_batch_plan_t *plan, int32_t use_graph, morph_stream_t stream)
{
    if (!plan) return MORPH_E_INVAL;
    if (plan->ntiles == 0) return MORPH_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (!use_graph) {
        if ((e = launch_reset_counter(plan->queue_dev, s)) != hipSuccess ||
            (e = launch_rect_batch(plan->pages_dev, plan->tiles_dev, plan->ntiles, plan->queue_dev,
                                   plan->nblocks, s, plan->alg_bytes)) != hipSuccess) {
            set_hip_error(e);
            return MORPH_E_HIP;
        }
        return MORPH_OK;
    }
    if (!plan->exec) {
        // the queue counter is cleared by a kernel inside the graph (no memset node)
        hipStream_t cs = plan->capture_stream;
        if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            set_hip_error(e);
            return MORPH_E_HIP;
        }
        hipError_t e1 = launch_reset_counter(plan->queue_dev, cs);
        const bool was_on = trace_pause();      // no event records inside the graph
        hipError_t e2 = launch_rect_batch(plan->pages_dev, plan->tiles_dev, plan->ntiles, plan->queue_dev,
                                          plan->nblocks, cs, plan->alg_bytes);
        trace_resume(was_on);
        e = hipStreamEndCapture(cs, &plan->graph);
        if (e1 != hipSuccess || e2 != hipSuccess || e != hipSuccess) {
            set_hip_error(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e));
            if (plan->graph) { hipGraphDestroy(plan->graph); plan->graph = nullptr; }
            return MORPH_E_HIP;
        }
        if ((e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0)) != hipSuccess) {
            set_hip_error(e);
            plan->exec = nullptr;
            return MORPH_E_HIP;
        }
    }
    trace_before(MORPH_K_RECT_BATCH, s);
    if ((e = hipGraphLaunch(plan->exec, s)) != hipSuccess) {
        set_hip_error(e);
        return MORPH_E_HIP;
    }
    trace_after(MORPH_K_RECT_BATCH, s, plan->alg_bytes);
    return MORPH_OK;
}

void morph_batch_plan_destroy(morph_batch_plan_t *plan)
{
    if (!plan) return;
    if (plan->exec) hipGraphExecDestroy(plan->exec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    if (plan->capture_stream) hipStreamDestroy(plan->capture_stream);
    if (plan->pages_dev) hipFree(plan->pages_dev);
    if (plan->tiles_dev) hipFree(plan->tiles_dev);
    if (plan->queue_dev) hipFree(plan->queue_dev);
    delete plan;
}

}  // extern "C"

// ------------------------------------------------------------ run-length API
namespace morph {

static bool rle_ok(const morph_rle_t *r)
{
    if (!r || !r->row_ptr) return false;
    if (r->width < 1 || r->height < 1 || r->npages < 1 || r->capacity < 0) return false;
    if (r->capacity > 0 && !r->runs) return false;
    if (((uintptr_t)r->runs) & 7 || ((uintptr_t)r->row_ptr) & 3) return false;   // runs are read as pairs
    if ((long long)r->height * r->npages >= 0x7fffffffLL) return false;
    return true;
}

static size_t rle_extent_rp(const morph_rle_t *r) { return ((size_t)r->height * r->npages + 1) * 4; }
static size_t rle_extent_runs(const morph_rle_t *r) { return (size_t)r->capacity * 8; }

static bool rle_alias(const morph_rle_t *a, const morph_rle_t *b)
{
    const size_t ar = rle_extent_rp(a), br = rle_extent_rp(b);
    const size_t an = rle_extent_runs(a), bn = rle_extent_runs(b);
    if (overlap(a->row_ptr, ar, b->row_ptr, br)) return true;
    if (an && bn && overlap(a->runs, an, b->runs, bn)) return true;
    if (bn && overlap(a->row_ptr, ar, b->runs, bn)) return true;
    if (an && overlap(a->runs, an, b->row_ptr, br)) return true;
    return false;
}

static int rect_rle(int op, const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se, void *ws,
                    size_t ws_bytes, hipStream_t stream)
{
    if (!rle_ok(dst) || !rle_ok(src) || !se_ok(se)) return MORPH_E_INVAL;
    if (dst->width != src->width || dst->height != src->height || dst->npages != src->npages)
        return MORPH_E_SHAPE;
    if (rle_alias(dst, src)) return MORPH_E_ALIAS;
    // Two forms.  The slot form (the fast one) keeps every intermediate row
    // in a workspace slot sized for the worst case and indexes slot rows in
    // 32 bits.  The band form keeps the intermediates in LDS and needs only
    // the row counts; it runs when the workspace given is too small for the
    // slot form, or the image too large for it, and the band form takes
    // the element and width.
    const long long ext =
        (long long)src->npages * (src->height + (long long)se.h - 1) * (rle_uses_scan(se) ? 2 : 1);
    const bool slot_ok = ext < 0x7fffffffLL &&
                         (long long)src->npages * src->height * (((long long)src->width + 1) / 2) < 0x7fffffffLL;
    const size_t need = slot_ok ? rle_op_workspace(op, src->width, src->height * src->npages, src->height, se) : 0;
    const bool band_ok = rle_band_applies(op, src->width, se);
    const size_t need_band = band_ok ? rle_band_workspace(op, src->width, (long long)src->height * src->npages, se) : 0;
    hipError_t e;
    if (slot_ok && ws && ws_bytes >= need) {
        e = rle_rect_op(op, *dst, *src, se, ws, ws_bytes, stream);
    } else if (band_ok && ws && ws_bytes >= need_band && !(((uintptr_t)ws) & 255)) {
        e = rle_band_op(op, *dst, *src, se, ws, stream);
    } else {
        if (!slot_ok && !band_ok) return MORPH_E_UNSUPPORTED;
        return MORPH_E_WORKSPACE;
    }
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

}  // namespace morph

extern "C" {

int morph_erode_rect_rle(const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se, void *ws,
                         size_t ws_bytes, morph_stream_t stream)
{
    return rect_rle(MORPH_ERODE, dst, src, se, ws, ws_bytes, (hipStream_t)stream);
}
int morph_dilate_rect_rle(const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se, void *ws,
                          size_t ws_bytes, morph_stream_t stream)
{
    return rect_rle(MORPH_DILATE, dst, src, se, ws, ws_bytes, (hipStream_t)stream);
}
int morph_open_rect_rle(const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se, void *ws,
                        size_t ws_bytes, morph_stream_t stream)
{
    return rect_rle(MORPH_OPEN, dst, src, se, ws, ws_bytes, (hipStream_t)stream);
}
int morph_close_rect_rle(const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se, void *ws,
                         size_t ws_bytes, morph_stream_t stream)
{
    return rect_rle(MORPH_CLOSE, dst, src, se, ws, ws_bytes, (hipStream_t)stream);
}

size_t morph_rle_workspace_bytes(int op, int32_t width, int32_t height, int32_t npages, morph_se_t se)
{
    if (width < 1 || height < 1 || npages < 1 || !se_ok(se) || op < MORPH_ERODE || op > MORPH_CLOSE)
        return 0;
    const long long ext = (long long)npages * (height + (long long)se.h - 1) * (rle_uses_scan(se) ? 2 : 1);
    if (ext >= 0x7fffffffLL || (long long)npages * height * (((long long)width + 1) / 2) >= 0x7fffffffLL)
        return morph_rle_workspace_bytes_compact(op, width, height, npages, se);
    return rle_op_workspace(op, width, height * npages, height, se);
}

size_t morph_rle_workspace_bytes_compact(int op, int32_t width, int32_t height, int32_t npages, morph_se_t se)
{
    if (width < 1 || height < 1 || npages < 1 || !se_ok(se) || op < MORPH_ERODE || op > MORPH_CLOSE)
        return 0;
    if (!rle_band_applies(op, width, se) || (long long)height * npages >= 0x7fffffffLL) return 0;
    return rle_band_workspace(op, width, (long long)height * npages, se);
}

size_t morph_pack_to_rle_workspace_bytes(int32_t width, int32_t height)
{
    if (width < 1 || height < 1) return 0;
    return ((size_t)height * 4 + 255) / 256 * 256 + scan_workspace(height);
}

int morph_pack_to_rle(const morph_rle_t *dst, const morph_bitmap_t *src, void *ws, size_t ws_bytes,
                      morph_stream_t stream)
{
    if (!rle_ok(dst) || !bitmap_ok(src)) return MORPH_E_INVAL;
    if (dst->width != src->width || dst->height != src->height || dst->npages != src->npages)
        return MORPH_E_SHAPE;
    const size_t ext = bitmap_extent(src);
    if (overlap(dst->row_ptr, rle_extent_rp(dst), src->words, ext) ||
        (dst->capacity && overlap(dst->runs, rle_extent_runs(dst), src->words, ext)))
        return MORPH_E_ALIAS;
    const size_t need = morph_pack_to_rle_workspace_bytes(src->width, src->height * src->npages);
    if (!ws || ws_bytes < need) return MORPH_E_WORKSPACE;
    hipError_t e = rle_from_packed(*dst, *src, ws, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

int morph_pack_to_rle_noalloc(const morph_rle_t *dst, const morph_bitmap_t *src, morph_stream_t stream)
{
    if (!rle_ok(dst) || !bitmap_ok(src)) return MORPH_E_INVAL;
    if (dst->width != src->width || dst->height != src->height || dst->npages != src->npages)
        return MORPH_E_SHAPE;
    const size_t ext = bitmap_extent(src);
    if (overlap(dst->row_ptr, rle_extent_rp(dst), src->words, ext) ||
        (dst->capacity && overlap(dst->runs, rle_extent_runs(dst), src->words, ext)))
        return MORPH_E_ALIAS;
    if ((long long)src->height * src->npages > MORPH_NOALLOC_MAX_ROWS) return MORPH_E_UNSUPPORTED;
    hipError_t e = rle_from_packed_noalloc(*dst, *src, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

int morph_rle_to_pack(const morph_bitmap_t *dst, const morph_rle_t *src, morph_stream_t stream)
{
    if (!bitmap_ok(dst) || !rle_ok(src)) return MORPH_E_INVAL;
    if (dst->width != src->width || dst->height != src->height || dst->npages != src->npages)
        return MORPH_E_SHAPE;
    const size_t ext = bitmap_extent(dst);
    if (overlap(src->row_ptr, rle_extent_rp(src), dst->words, ext) ||
        (src->capacity && overlap(src->runs, rle_extent_runs(src), dst->words, ext)))
        return MORPH_E_ALIAS;
    // one thread per output word, indexed in 32 bits
    if ((long long)dst->height * dst->npages * ((dst->width + 63) / 64) >= 0xffffffffLL) return MORPH_E_UNSUPPORTED;
    hipError_t e = rle_to_packed(*dst, *src, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

}  // extern "C"

// ---------------------------------------------------------- transposition
namespace morph {

static bool transposed_shape(int dw, int dh, int dp, int sw, int sh, int sp)
{
    return dw == sh && dh == sw && dp == sp;
}

// Workspace of a run-length transpose: the transposed bitmap, the scratch
// of the re-encoding, then the source decoded in its own orientation (rows
// of up to 128 words are decoded there and transposed as a bitmap).
// Whether the runs of the transpose of a W x H image (P pages) take the
// short path: the runs decoded into a bitmap in their own orientation (rows
// of up to 128 words), its transpose made together with the run counts of
// its rows (rows of up to 128 words too), and the runs encoded from it.
static bool direct_transposed(int W, int H, int P)
{
    return (W + 63) / 64 <= 128 && (H + 63) / 64 <= 128 && (long long)W * P < 0x7fffffffLL;
}

// Workspace of the run-length transpose: the transposed bitmap (the path
// through it only), the encoding scratch of either path, and the decoded
// image in its own orientation.
static size_t transpose_rle_ws(int W, int H, int P)
{
    const size_t rows = (size_t)W * P;
    return round256(image_bytes(H, (int)rows)) +
           round256(std::max(morph_pack_to_rle_workspace_bytes(H, (int)rows), transposed_rle_workspace(W, H, P))) +
           round256(image_bytes(W, H * P));
}

// Workspace of the transpose-based rectangle operation: one bitmap buffer
// (the transposed image, later the image back in its own orientation), one
// run-length buffer (the transposed runs; for opening and closing its run
// array later holds the bitmap after the last within-line pass), the
// re-encoding scratch and, for opening and closing, that last pass's
// workspace.
struct RletWs {
    size_t bm, rp, runs, p2r, rowop, tmp, total;
    long long cap;
};

static RletWs rlet_ws(int op, int W, int H, int P, morph_se_t se)
{
    RletWs w{};
    const long long rowsT = (long long)W * P, rows = (long long)H * P;
    w.bm = round256(std::max(image_bytes(H, (int)rowsT), image_bytes(W, (int)rows)));
    w.cap = rowsT * ((H + 1) / 2);
    w.rp = round256((size_t)(rowsT + 1) * 4);
    w.runs = round256(std::max((size_t)w.cap * 8, image_bytes(W, (int)rows)));
    w.p2r = round256(std::max({morph_pack_to_rle_workspace_bytes(H, (int)rowsT),
                               morph_pack_to_rle_workspace_bytes(W, (int)rows), transposed_rle_workspace(W, H, P),
                               transposed_rle_workspace(H, W, P)}));
    if (op == MORPH_OPEN || op == MORPH_CLOSE) {
        // the last within-line pass along the rows, on the image in its own
        // orientation or, as a pass along the columns, on its transpose
        const int op2 = op == MORPH_OPEN ? MORPH_DILATE : MORPH_ERODE;
        const morph_se_t row{se.w, 1, se.cx, 0}, col{1, se.w, 0, se.cx};
        w.rowop = round256(std::max(morph_workspace_bytes(op2, MORPH_PACKED, W, (int)rows, row),
                                    morph_workspace_bytes(op2, MORPH_PACKED, H, (int)rowsT, col)));
    }
    // each decode's source in its own orientation, before the transpose
    w.tmp = round256(std::max(image_bytes(W, (int)rows), image_bytes(H, (int)rowsT)));
    w.total = w.bm + w.rp + w.runs + w.p2r + w.rowop + w.tmp;
    return w;
}

// Rectangle operation by within-line operations and transposition: the
// operation along the rows is applied while the runs are decoded into the
// transposed bitmap, which is re-encoded; the operation along the former
// columns is applied while those runs are decoded back.  Opening is E_w,
// then the column opening, then D_w (closing the reverse): the row and
// column passes of a rectangle commute, so two transpositions suffice, and
// the last row pass runs on the decoded bitmap before it is re-encoded.
static int rlet_run(int op, const morph_rle_t &dst, const morph_rle_t &src, morph_se_t se, char *ws,
                    const RletWs &L, hipStream_t s)
{
    const int W = src.width, H = src.height, P = src.npages;
    const morph_bitmap_t T1{(uint64_t *)ws, H, W, (H + 63) / 64, P};
    const morph_rle_t R1{H, W, P, (int *)(ws + L.bm), (int *)(ws + L.bm + L.rp), L.cap};
    const morph_bitmap_t T2{(uint64_t *)ws, W, H, (W + 63) / 64, P};
    const morph_bitmap_t T3{(uint64_t *)(ws + L.bm + L.rp), W, H, (W + 63) / 64, P};
    void *p2r = ws + L.bm + L.rp + L.runs;
    const bool ero_first = (op == MORPH_ERODE || op == MORPH_OPEN);
    const LineOp row{ero_first ? kLineErode : kLineDilate, se.w, se.cx, 0};
    LineOp col{};
    switch (op) {
    case MORPH_ERODE: col = LineOp{kLineErode, se.h, se.cy, 0}; break;
    case MORPH_DILATE: col = LineOp{kLineDilate, se.h, se.cy, 0}; break;
    case MORPH_OPEN: col = LineOp{kLineOpen, se.h, se.cy, 0}; break;
    default: col = LineOp{kLineOpen, se.h, se.h - 1 - se.cy, 1}; break;   // closing: the gaps' opening
    }
    uint64_t *tmp = (uint64_t *)(ws + L.bm + L.rp + L.runs + L.p2r + L.rowop);
    const bool one = (op == MORPH_ERODE || op == MORPH_DILATE);
    hipError_t e;
    // each decode into tmp in the runs' own orientation, then the runs of
    // its transpose encoded straight from it (where the rows allow)
    if (direct_transposed(W, H, P)) {
        const morph_bitmap_t D{tmp, W, H, (W + 63) / 64, P};
        e = rle_decode_rows(D, src, row, s);
        if (e == hipSuccess) e = rle_from_packed_transposed(R1, D, (uint64_t *)ws, p2r, s);
    } else {
        e = rle_decode_transposed(T1, src, row, s, tmp);
        if (e == hipSuccess) e = rle_from_packed(R1, T1, p2r, s);
    }
    const int op2 = op == MORPH_OPEN ? MORPH_DILATE : MORPH_ERODE;
    void *rowop_ws = L.rowop ? ws + L.bm + L.rp + L.runs + L.p2r : nullptr;
    if (e == hipSuccess && direct_transposed(H, W, P)) {
        const morph_bitmap_t D{tmp, H, W, (H + 63) / 64, P};
        e = rle_decode_rows(D, R1, col, s);
        if (e == hipSuccess && one) e = rle_from_packed_transposed(dst, D, (uint64_t *)ws, p2r, s);
        if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
        if (one) return MORPH_OK;
        // opening and closing: the last pass along the rows runs down the
        // columns of the decoded transpose, which is then encoded back
        const morph_bitmap_t V{(uint64_t *)ws, H, W, (H + 63) / 64, P};
        const int rc = rect_packed(op2, &V, &D, morph_se_t{1, se.w, 0, se.cx}, rowop_ws, L.rowop, s);
        if (rc != MORPH_OK) return rc;
        e = rle_from_packed_transposed(dst, V, tmp, p2r, s);
        if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
        return MORPH_OK;
    } else if (e == hipSuccess) {
        e = rle_decode_transposed(T2, R1, col, s, tmp);
        if (e == hipSuccess && one) e = rle_from_packed(dst, T2, p2r, s);
    }
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    if (one) return MORPH_OK;
    const morph_se_t last{se.w, 1, se.cx, 0};
    const int rc = rect_packed(op2, &T3, &T2, last, rowop_ws, L.rowop, s);
    if (rc != MORPH_OK) return rc;
    e = rle_from_packed(dst, T3, p2r, s);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

}  // namespace morph

extern "C" {

int morph_transpose_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, morph_stream_t stream)
{
    if (!bitmap_ok(dst) || !bitmap_ok(src)) return MORPH_E_INVAL;
    if (!transposed_shape(dst->width, dst->height, dst->npages, src->width, src->height, src->npages))
        return MORPH_E_SHAPE;
    if (overlap(dst->words, bitmap_extent(dst), src->words, bitmap_extent(src))) return MORPH_E_ALIAS;
    hipError_t e = packed_transpose(*dst, *src, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

int morph_popcount_pages(const morph_bitmap_t *src, int64_t *counts, morph_stream_t stream)
{
    if (!bitmap_ok(src) || !counts || (((uintptr_t)counts) & 7)) return MORPH_E_INVAL;
    if (overlap(counts, (size_t)src->npages * 8, src->words, bitmap_extent(src))) return MORPH_E_ALIAS;
    hipError_t e = popcount_pages(*src, (unsigned long long *)counts, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

size_t morph_transpose_rle_workspace_bytes(int32_t width, int32_t height, int32_t npages)
{
    if (width < 1 || height < 1 || npages < 1 || (long long)width * npages > 0x7fffffffLL) return 0;
    return transpose_rle_ws(width, height, npages);
}

int morph_transpose_rle(const morph_rle_t *dst, const morph_rle_t *src, void *ws, size_t ws_bytes,
                        morph_stream_t stream)
{
    if (!rle_ok(dst) || !rle_ok(src)) return MORPH_E_INVAL;
    if (!transposed_shape(dst->width, dst->height, dst->npages, src->width, src->height, src->npages))
        return MORPH_E_SHAPE;
    if (rle_alias(dst, src)) return MORPH_E_ALIAS;
    if (dst->capacity < morph_rle_max_runs(dst->width, dst->height * dst->npages)) return MORPH_E_CAPACITY;
    const size_t need = morph_transpose_rle_workspace_bytes(src->width, src->height, src->npages);
    if (!ws || (((uintptr_t)ws) & 255) || ws_bytes < need) return MORPH_E_WORKSPACE;
    const int W = src->width, H = src->height, P = src->npages;
    char *w = (char *)ws;
    const morph_bitmap_t T{(uint64_t *)w, H, W, (H + 63) / 64, P};
    char *enc = w + round256(image_bytes(H, W * P));
    uint64_t *tmp = (uint64_t *)(enc + round256(std::max(morph_pack_to_rle_workspace_bytes(H, W * P),
                                                         transposed_rle_workspace(W, H, P))));
    const LineOp none{kLineNone, 1, 0, 0};
    hipError_t e;
    if (direct_transposed(W, H, P)) {
        const morph_bitmap_t D{tmp, W, H, (W + 63) / 64, P};
        e = rle_decode_rows(D, *src, none, (hipStream_t)stream);
        if (e == hipSuccess) e = rle_from_packed_transposed(*dst, D, (uint64_t *)w, enc, (hipStream_t)stream);
    } else {
        e = rle_decode_transposed(T, *src, none, (hipStream_t)stream, tmp);
        if (e == hipSuccess) e = rle_from_packed(*dst, T, enc, (hipStream_t)stream);
    }
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

size_t morph_rlet_workspace_bytes(int op, int32_t width, int32_t height, int32_t npages, morph_se_t se)
{
    if (width < 1 || height < 1 || npages < 1 || !se_ok(se) || op < MORPH_ERODE || op > MORPH_CLOSE)
        return 0;
    if ((long long)width * npages > 0x7fffffffLL || (long long)height * npages > 0x7fffffffLL) return 0;
    return rlet_ws(op, width, height, npages, se).total;
}

int morph_rect_rlet(int op, const morph_rle_t *dst, const morph_rle_t *src, morph_se_t se, void *ws,
                    size_t ws_bytes, morph_stream_t stream)
{
    if (!rle_ok(dst) || !rle_ok(src) || !se_ok(se) || op < MORPH_ERODE || op > MORPH_CLOSE)
        return MORPH_E_INVAL;
    if (dst->width != src->width || dst->height != src->height || dst->npages != src->npages)
        return MORPH_E_SHAPE;
    if (rle_alias(dst, src)) return MORPH_E_ALIAS;
    if (dst->capacity < morph_rle_max_runs(dst->width, dst->height * dst->npages)) return MORPH_E_CAPACITY;
    const int W = src->width, H = src->height, P = src->npages;
    if ((long long)W * P > 0x7fffffffLL) return MORPH_E_UNSUPPORTED;
    const RletWs L = rlet_ws(op, W, H, P, se);
    if (L.cap >= 0x7fffffffLL) return MORPH_E_UNSUPPORTED;
    if (!ws || (((uintptr_t)ws) & 255) || ws_bytes < L.total) return MORPH_E_WORKSPACE;
    return rlet_run(op, *dst, *src, se, (char *)ws, L, (hipStream_t)stream);
}

size_t morph_rle_label_workspace_bytes(int32_t rows, int64_t max_runs)
{
    if (rows < 1 || max_runs < 0 || max_runs >= 0x7fffffffLL) return 0;
    return cc_workspace(rows, max_runs);
}

int morph_rle_label(const morph_rle_t *src, int32_t connectivity, int32_t *labels, int64_t max_runs,
                    int32_t *comp_ptr, void *ws, size_t ws_bytes, morph_stream_t stream)
{
    if (!rle_ok(src) || (connectivity != 4 && connectivity != 8) || !comp_ptr || max_runs < 0 ||
        (max_runs > 0 && !labels) || (((uintptr_t)labels) & 3) || (((uintptr_t)comp_ptr) & 3))
        return MORPH_E_INVAL;
    if (max_runs >= 0x7fffffffLL) return MORPH_E_UNSUPPORTED;
    const long long R = (long long)src->height * src->npages;
    const size_t need = cc_workspace(R, max_runs);
    if (!ws || (((uintptr_t)ws) & 255) || ws_bytes < need) return MORPH_E_WORKSPACE;
    const size_t lb = (size_t)max_runs * 4, cb = ((size_t)src->npages + 1) * 4;
    if ((lb && (overlap(labels, lb, src->runs, rle_extent_runs(src)) ||
                overlap(labels, lb, src->row_ptr, rle_extent_rp(src)) || overlap(labels, lb, comp_ptr, cb))) ||
        overlap(comp_ptr, cb, src->row_ptr, rle_extent_rp(src)) ||
        (src->capacity && overlap(comp_ptr, cb, src->runs, rle_extent_runs(src))))
        return MORPH_E_ALIAS;
    hipError_t e = cc_label(*src, connectivity, labels, max_runs, comp_ptr, ws, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

int morph_rle_component_stats(const morph_rle_t *src, const int32_t *labels, int64_t max_runs,
                              const int32_t *comp_ptr, morph_component_t *stats, int64_t max_components,
                              morph_stream_t stream)
{
    if (!rle_ok(src) || !comp_ptr || max_runs < 0 || max_components < 0 || (max_runs > 0 && !labels) ||
        (max_components > 0 && !stats) || (((uintptr_t)stats) & 7))
        return MORPH_E_INVAL;
    if (max_runs >= 0x7fffffffLL) return MORPH_E_UNSUPPORTED;
    hipError_t e = cc_stats(*src, labels, max_runs, comp_ptr, stats, max_components, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

int morph_rle_run_histograms(const morph_rle_t *src, int32_t *black, int32_t *white, morph_stream_t stream)
{
    if (!rle_ok(src) || !black || !white || (((uintptr_t)black) & 3) || (((uintptr_t)white) & 3))
        return MORPH_E_INVAL;
    const size_t hb = (size_t)src->npages * ((size_t)src->width + 1) * 4;
    if (overlap(black, hb, white, hb) || overlap(black, hb, src->row_ptr, rle_extent_rp(src)) ||
        overlap(white, hb, src->row_ptr, rle_extent_rp(src)) ||
        (src->capacity && (overlap(black, hb, src->runs, rle_extent_runs(src)) ||
                           overlap(white, hb, src->runs, rle_extent_runs(src)))))
        return MORPH_E_ALIAS;
    hipError_t e = run_histograms(*src, black, white, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

size_t morph_histogram_percentile_workspace_bytes(int32_t nbins)
{
    return nbins < 1 ? 0 : percentile_workspace(nbins);
}

int morph_histogram_percentile(const int32_t *hist, int32_t nrows, int32_t nbins, int32_t num, int32_t den,
                               int32_t *out, void *ws, size_t ws_bytes, morph_stream_t stream)
{
    if (!hist || !out || nrows < 1 || nbins < 1 || num < 1 || den < num || den > (1 << 20) ||
        (((uintptr_t)hist) & 3) || (((uintptr_t)out) & 3))
        return MORPH_E_INVAL;
    if (!ws || (((uintptr_t)ws) & 255) || ws_bytes < percentile_workspace(nbins)) return MORPH_E_WORKSPACE;
    const size_t hb = (size_t)nrows * nbins * 4;
    if (overlap(ws, percentile_workspace(nbins), hist, hb) || overlap(ws, percentile_workspace(nbins), out, 4))
        return MORPH_E_ALIAS;
    hipError_t e = histogram_percentile(hist, nrows, nbins, num, den, out, ws, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ masks
namespace morph {

static bool mask_ok(const morph_mask_t *m)
{
    return m && m->bits && m->w >= 1 && m->h >= 1 && m->w < 32768 && m->h < 32768 && m->cx >= 0 &&
           m->cy >= 0 && m->cx < m->w && m->cy < m->h;
}

// The horizontal runs of the mask (or of its reflection), longest first.
static bool mask_runs(const morph_mask_t &m, bool reflected, MaskRunsArg &out)
{
    struct Run { int dx, dy, len; };
    std::vector<Run> v;
    for (int j = 0; j < m.h; j++) {
        int i = 0;
        while (i < m.w) {
            if (!m.bits[(size_t)j * m.w + i]) { i++; continue; }
            int k = i;
            while (k < m.w && m.bits[(size_t)j * m.w + k]) k++;
            if (reflected)      // pixel (i, j) -> (w-1-i, h-1-j), origin -> (w-1-cx, h-1-cy)
                v.push_back({(m.w - k) - (m.w - 1 - m.cx), (m.h - 1 - j) - (m.h - 1 - m.cy), k - i});
            else
                v.push_back({i - m.cx, j - m.cy, k - i});
            i = k;
        }
    }
    if ((int)v.size() > kMaskMaxRuns) return false;
    std::stable_sort(v.begin(), v.end(), [](const Run &x, const Run &y) { return x.len > y.len; });
    out.n = (int)v.size();
    for (int q = 0; q < out.n; q++) {
        out.dx[q] = (short)v[q].dx;
        out.dy[q] = (short)v[q].dy;
        out.len[q] = (short)v[q].len;
    }
    return true;
}

static bool mask_page(MaskPage &p, const morph_bitmap_t &dst, const morph_bitmap_t &src, int in_c, int out_c,
                      const MaskRunsArg &m)
{
    p = MaskPage{};
    p.src = src.words;
    p.dst = dst.words;
    p.W = src.width;
    p.H = src.height;
    p.nw = (src.width + 63) / 64;
    p.sstride = src.stride_words;
    p.dstride = dst.stride_words;
    p.spw = (long long)src.stride_words * src.height;
    p.dpw = (long long)dst.stride_words * dst.height;
    p.in_c = in_c;
    p.out_c = out_c;
    p.padmask = (src.width % 64) ? ((1ull << (src.width % 64)) - 1) : ~0ull;
    return plan_mask(p, m);
}

}  // namespace morph

extern "C" {

size_t morph_mask_workspace_bytes(int op, int repr, int32_t width, int32_t height, int32_t npages,
                                  const morph_mask_t *mask)
{
    if (width < 1 || height < 1 || npages < 1 || !mask_ok(mask) || op < MORPH_ERODE || op > MORPH_CLOSE)
        return 0;
    const long long rows = (long long)height * npages;
    if (repr == MORPH_PACKED)
        return (op == MORPH_OPEN || op == MORPH_CLOSE) ? round256(image_bytes(width, (int)rows)) : 0;
    return rle_mask_workspace(width, rows);
}

int morph_mask_packed(int op, const morph_bitmap_t *dst, const morph_bitmap_t *src, const morph_mask_t *mask,
                      void *ws, size_t ws_bytes, morph_stream_t stream)
{
    if (!bitmap_ok(dst) || !bitmap_ok(src) || !mask_ok(mask) || op < MORPH_ERODE || op > MORPH_CLOSE)
        return MORPH_E_INVAL;
    if (dst->width != src->width || dst->height != src->height || dst->npages != src->npages)
        return MORPH_E_SHAPE;
    if (overlap(dst->words, bitmap_extent(dst), src->words, bitmap_extent(src))) return MORPH_E_ALIAS;
    MaskRunsArg m, mr;
    if (!mask_runs(*mask, false, m) || !mask_runs(*mask, true, mr)) return MORPH_E_UNSUPPORTED;
    const int W = src->width, H = src->height, P = src->npages;
    const bool two = op == MORPH_OPEN || op == MORPH_CLOSE;
    const size_t need = two ? round256(image_bytes(W, H * P)) : 0;
    if (two && (!ws || (((uintptr_t)ws) & 255) || ws_bytes < need)) return MORPH_E_WORKSPACE;
    const morph_bitmap_t tmp{(uint64_t *)ws, W, H, (W + 63) / 64, P};
    if (two && (overlap(ws, need, dst->words, bitmap_extent(dst)) || overlap(ws, need, src->words, bitmap_extent(src))))
        return MORPH_E_ALIAS;
    // erosion by M; dilation = not erosion by the reflected mask of not A
    struct Step { const morph_bitmap_t *d, *s; int in_c, out_c; const MaskRunsArg *m; };
    Step steps[2];
    int ns = 0;
    switch (op) {
    case MORPH_ERODE: steps[ns++] = {dst, src, 0, 0, &m}; break;
    case MORPH_DILATE: steps[ns++] = {dst, src, 1, 1, &mr}; break;
    case MORPH_OPEN: steps[ns++] = {&tmp, src, 0, 0, &m}; steps[ns++] = {dst, &tmp, 1, 1, &mr}; break;
    default: steps[ns++] = {&tmp, src, 1, 1, &mr}; steps[ns++] = {dst, &tmp, 0, 0, &m}; break;
    }
    for (int k = 0; k < ns; k++) {
        MaskPage p;
        if (!mask_page(p, *steps[k].d, *steps[k].s, steps[k].in_c, steps[k].out_c, *steps[k].m))
            return MORPH_E_UNSUPPORTED;
        hipError_t e = launch_mask(p, *steps[k].m, P, (hipStream_t)stream);
        if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    }
    return MORPH_OK;
}

int morph_mask_rle(int op, const morph_rle_t *dst, const morph_rle_t *src, const morph_mask_t *mask, void *ws,
                   size_t ws_bytes, morph_stream_t stream)
{
    if (!rle_ok(dst) || !rle_ok(src) || !mask_ok(mask) || op < MORPH_ERODE || op > MORPH_CLOSE)
        return MORPH_E_INVAL;
    if (dst->width != src->width || dst->height != src->height || dst->npages != src->npages)
        return MORPH_E_SHAPE;
    if (rle_alias(dst, src)) return MORPH_E_ALIAS;
    const long long rows = (long long)src->height * src->npages;
    if (rows * ((((long long)src->width + 1) / 2 + 15) & ~15LL) >= 0x7fffffffLL) return MORPH_E_UNSUPPORTED;
    if (dst->capacity < morph_rle_max_runs(dst->width, dst->height * dst->npages)) return MORPH_E_CAPACITY;
    MaskRunsArg m, mr;
    if (!mask_runs(*mask, false, m) || !mask_runs(*mask, true, mr)) return MORPH_E_UNSUPPORTED;
    if (!ws || (((uintptr_t)ws) & 255) || ws_bytes < rle_mask_workspace(src->width, rows)) return MORPH_E_WORKSPACE;
    hipError_t e = rle_mask_op(op, *dst, *src, m, mr, ws, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

int morph_shift_rows_packed(const morph_bitmap_t *dst, const morph_bitmap_t *src, const int32_t *shifts,
                            int32_t fill, morph_stream_t stream)
{
    if (!bitmap_ok(dst) || !bitmap_ok(src) || !shifts || (((uintptr_t)shifts) & 3) || (fill != 0 && fill != 1))
        return MORPH_E_INVAL;
    if (dst->height != src->height || dst->npages != src->npages) return MORPH_E_SHAPE;
    if (overlap(dst->words, bitmap_extent(dst), src->words, bitmap_extent(src)) ||
        overlap(dst->words, bitmap_extent(dst), shifts, (size_t)src->height * src->npages * 4))
        return MORPH_E_ALIAS;
    hipError_t e = shift_rows_packed(*dst, *src, shifts, fill, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

size_t morph_shift_rows_rle_workspace_bytes(int32_t rows)
{
    return rows < 1 ? 0 : shift_rows_rle_workspace(rows);
}

int morph_shift_rows_rle(const morph_rle_t *dst, const morph_rle_t *src, const int32_t *shifts, int32_t fill,
                         void *ws, size_t ws_bytes, morph_stream_t stream)
{
    if (!rle_ok(dst) || !rle_ok(src) || !shifts || (((uintptr_t)shifts) & 3) || (fill != 0 && fill != 1))
        return MORPH_E_INVAL;
    if (dst->height != src->height || dst->npages != src->npages) return MORPH_E_SHAPE;
    if (rle_alias(dst, src)) return MORPH_E_ALIAS;
    if (dst->capacity < morph_rle_max_runs(dst->width, dst->height * dst->npages)) return MORPH_E_CAPACITY;
    const long long R = (long long)src->height * src->npages;
    if (!ws || (((uintptr_t)ws) & 255) || ws_bytes < shift_rows_rle_workspace(R)) return MORPH_E_WORKSPACE;
    hipError_t e = shift_rows_rle(*dst, *src, shifts, fill, ws, (hipStream_t)stream);
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

int morph_rle_validate(const morph_rle_t *r, morph_stream_t stream)
{
    if (!rle_ok(r)) return MORPH_E_INVAL;
    hipError_t e = hipSuccess;
    const int rc = rle_validate(*r, (hipStream_t)stream, &e);
    if (rc == MORPH_E_HIP) set_hip_error(e);
    return rc;
}

}  // extern "C"

// ------------------------------------------------------------------ tracing
namespace morph {

namespace {
struct TraceRec {
    hipEvent_t a, b;
    int kernel;
    double bytes;
};
struct Trace {
    bool on = false;
    unsigned long long *dev = nullptr;
    std::vector<TraceRec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t pending = nullptr;
} g_trace;

hipEvent_t trace_event()
{
    hipEvent_t e = nullptr;
    if (!g_trace.pool.empty()) {
        e = g_trace.pool.back();
        g_trace.pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

__global__ void zero_kernel(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
}  // namespace

bool trace_on() { return g_trace.on; }

bool trace_pause()
{
    const bool prev = g_trace.on;
    g_trace.on = false;
    return prev;
}

void trace_resume(bool prev) { g_trace.on = prev; }

unsigned long long *trace_counters() { return g_trace.on ? g_trace.dev : nullptr; }

void trace_before(int kernel, hipStream_t s)
{
    (void)kernel;
    if (!g_trace.on) return;
    g_trace.pending = trace_event();
    if (g_trace.pending) hipEventRecord(g_trace.pending, s);
}

void trace_after(int kernel, hipStream_t s, double alg_bytes)
{
    if (!g_trace.on || !g_trace.pending) return;
    hipEvent_t b = trace_event();
    if (!b) return;
    hipEventRecord(b, s);
    g_trace.recs.push_back(TraceRec{g_trace.pending, b, kernel, alg_bytes});
    g_trace.pending = nullptr;
}

}  // namespace morph

extern "C" {

const char *morph_kernel_name(int k)
{
    static const char *names[MORPH_K_COUNT] = {"rect_kernel", "rect_batch_kernel", "pack_to_rle_kernel",
                                               "rle_to_pack_kernel", "row_erode_kernel", "col_and_kernel",
                                               "pack_rows_kernel", "transpose_kernel",
                                               "decode_transpose_kernel", "components",
                                               "component_stats_kernel", "run_hist_kernel", "mask_kernel",
                                               "mask_and_kernel", "shift_rows_kernel", "shift_rows_rle_kernel",
                                               "col_scan_kernel", "rle_band_kernel", "rle_band_count_kernel",
                                               "transpose_to_rle"};
    return (k >= 0 && k < MORPH_K_COUNT) ? names[k] : "?";
}

int morph_trace_begin(void *dev_counters, size_t bytes, morph_stream_t stream)
{
    if (!dev_counters || bytes < MORPH_TRACE_BYTES || (((uintptr_t)dev_counters) & 127)) return MORPH_E_INVAL;
    g_trace.on = true;
    g_trace.dev = (unsigned long long *)dev_counters;
    g_trace.recs.clear();
    const int n = MORPH_TRACE_BYTES / 8;
    hipLaunchKernelGGL(zero_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, g_trace.dev, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

int morph_trace_end(morph_kernel_trace_t *out, morph_stream_t stream)
{
    if (!out) return MORPH_E_INVAL;
    for (int k = 0; k < MORPH_K_COUNT; k++) out[k] = morph_kernel_trace_t{0, 0.0, 0.0};
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    std::vector<unsigned long long> raw(MORPH_TRACE_BYTES / 8, 0);
    if (e == hipSuccess && g_trace.dev)
        e = hipMemcpy(raw.data(), g_trace.dev, MORPH_TRACE_BYTES, hipMemcpyDeviceToHost);
    // per kernel: 2 counters (read, written) x 256 slots, one slot every 16 words
    unsigned long long runs[2 * MORPH_K_COUNT] = {0};
    for (int c = 0; c < 2 * MORPH_K_COUNT; c++)
        for (int sl = 0; sl < 256; sl++) runs[c] += raw[((size_t)c * 256 + sl) * 16];
    for (const TraceRec &r : g_trace.recs) {
        float ms = 0.f;
        if (e == hipSuccess) hipEventElapsedTime(&ms, r.a, r.b);
        out[r.kernel].launches++;
        out[r.kernel].ms += ms;
        out[r.kernel].bytes += r.bytes;
        g_trace.pool.push_back(r.a);
        g_trace.pool.push_back(r.b);
    }
    // run-length kernels: 8 bytes per run read and written on top of the
    // row counts the host added
    for (int k = 0; k < MORPH_K_COUNT; k++) out[k].bytes += 8.0 * (double)(runs[2 * k] + runs[2 * k + 1]);
    g_trace.recs.clear();
    g_trace.on = false;
    g_trace.dev = nullptr;
    if (e != hipSuccess) { set_hip_error(e); return MORPH_E_HIP; }
    return MORPH_OK;
}

}  // extern "C"
