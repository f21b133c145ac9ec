// scalp_abi.hip -- the extern "C" entry points of libscalp.so: argument
// validation, workspace layout, kernel sequencing and hipGraph capture.
// Declarations and their contracts are in include/scalp.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <vector>

#include "scalp.h"
#include "scalp_internal.h"

using namespace scalp;

// The scratch of scalp_run_static: the workspace that scalp_run takes from
// its caller, as a device array of this library (one per GPU).  In host code
// `scratch` names a host-side stand-in, not a device address: every use goes
// through the per-device address that hipGetSymbolAddress returns
// (static_scratch below).
static __device__ __align__(256) unsigned char scratch[SCALP_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

std::once_flag g_init_once;
void library_init() { std::call_once(g_init_once, [] { lift_lds_limits(); }); }

// r = sqrt(N / k) in FP64 (Sec. II-A), with the requested k.
double grid_r(int W, int H, int k) { return std::sqrt((double)W * (double)H / (double)k); }

bool grid_valid(const scalp_grid_t* g) {
    if (!g) return false;
    scalp_grid_t ref;
    if (scalp_make_grid(g->width, g->height, g->k_requested, &ref) != SCALP_OK) return false;
    return ref.nx == g->nx && ref.ny == g->ny && ref.num_sp == g->num_sp;
}

bool params_valid(const scalp_params_t* p) {
    if (!p) return false;
    if (!std::isfinite(p->m) || p->m < 0.0f) return false;
    if (!(p->lambda >= 0.0f && p->lambda <= 1.0f)) return false;
    if (!(p->sigma > 0.0f) || !std::isfinite(p->sigma)) return false;
    if (!std::isfinite(p->gamma)) return false;
    if (p->iterations < 0) return false;
    if (p->lds_pixels < 0 || p->lds_pixels > kMaxLdsPixels) return false;
    if (p->wg_size != 0 && p->wg_size != 256 && p->wg_size != 512 && p->wg_size != 1024)
        return false;
    if (p->assign_mode != SCALP_ASSIGN_GRID3X3 && p->assign_mode != SCALP_ASSIGN_WINDOW)
        return false;
    if (p->contour_source != SCALP_CONTOUR_INPUT && p->contour_source != SCALP_CONTOUR_GRADIENT)
        return false;
    if (p->exact_pruning != 0 && p->exact_pruning != 1) return false;
    if (p->persistent_blocks < 0 || p->persistent_blocks > 16) return false;
    if (p->table_mode != 0 && p->table_mode != 1) return false;
    return true;
}

// The pointers a packing step reads are present.
bool pack_inputs_ok(const scalp_params_t* p, const float* lab, const float* contour) {
    return lab && (contour || p->contour_source == SCALP_CONTOUR_GRADIENT);
}

Tuning tuning_of(const scalp_params_t* p) {
    Tuning t;
    t.wg = p->wg_size == 0 ? 1024 : p->wg_size;
    t.lds_pixels = p->lds_pixels > 0 ? p->lds_pixels : default_lds_pixels();
    t.blocks_per_cu = p->persistent_blocks;
    t.voted = p->table_mode;
    return t;
}

// Assignment work items per cell for workgroups of wg lanes: the largest cell
// is ceil(W / nx) x ceil(H / ny) pixels, in ceil(. / 64) chunks of 64, split
// evenly so that no item has more than wg / 64 chunks.
int slices_of(const scalp_grid_t* g, int wg) {
    const long long cw = (g->width + g->nx - 1) / g->nx, ch = (g->height + g->ny - 1) / g->ny;
    const long long chunks = (cw * ch + 63) / 64, per = wg / 64;
    return (int)std::max<long long>(1, (chunks + per - 1) / per);
}

Img img_of(const scalp_grid_t* g, const scalp_params_t* p, long long pix, int sp) {
    Img im;
    im.W = g->width;
    im.H = g->height;
    im.nx = g->nx;
    im.ny = g->ny;
    im.pix = pix;
    im.sp = sp;
    const double r = grid_r(g->width, g->height, g->k_requested);
    im.spw = (float)(((double)p->m * (double)p->m) / (r * r));          // Eq. (3)
    im.gamma = p->gamma < 0.0f ? (float)(2.0 * r) : p->gamma;           // Sec. III-A.3
    im.spl = slices_of(g, tuning_of(p).wg);
    im.rad = (int)std::floor(r + 0.5);
    im.prune = p->exact_pruning;
    // Each XCD (own L2) takes a contiguous run of the cell order; strips of
    // width about sqrt(nx ny / 8) make those runs near-square blocks of
    // cells, so fewer table texels sit in cells that another XCD reads too.
    im.strips = std::max(1, std::min({8, g->nx,
        (int)std::lround(std::sqrt(8.0 * g->nx / std::max(1, g->ny)))}));
    return im;
}

// Single-image workspace: [packed float4 N][acc int64 8K][ctrl int32 64][plist int32 K]
// [window minima uint64 N]
struct Layout {
    size_t packed, acc, ctrl, plist, keys, total;
};

Layout layout_of(long long N, long long K) {
    Layout L;
    L.packed = 0;
    L.acc = align_up((size_t)N * 16);
    L.ctrl = L.acc + (size_t)K * kAccStride * 8;   // acc and ctrl are contiguous (cleared together)
    L.plist = align_up(L.ctrl + kCtrlWords * 4);
    L.keys = align_up(L.plist + (size_t)K * 4);
    L.total = align_up(L.keys + (size_t)N * 8);
    return L;
}

struct Views {
    float4* packed;
    long long* acc;
    int* ctrl;
    int* plist;
    unsigned long long* keys;
};

Views views_of(void* ws, const Layout& L) {
    char* b = static_cast<char*>(ws);
    return Views{reinterpret_cast<float4*>(b + L.packed), reinterpret_cast<long long*>(b + L.acc),
                 reinterpret_cast<int*>(b + L.ctrl), reinterpret_cast<int*>(b + L.plist),
                 reinterpret_cast<unsigned long long*>(b + L.keys)};
}

// Half-width of Algorithm 1's window: r = sqrt(N/k) rounded to whole pixels.
int window_radius(const scalp_grid_t* g) {
    return (int)std::floor(grid_r(g->width, g->height, g->k_requested) + 0.5);
}

long long clear_words(const Layout& L) { return (long long)((L.ctrl + kCtrlWords * 4 - L.acc) / 8); }

// Device address of the current device's scratch, resolved once per device
// with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

int static_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SCALP_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return SCALP_ERR_HIP;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return SCALP_OK;
}

#define CHECK_HIP(expr)                            \
    do {                                           \
        if ((expr) != hipSuccess) return SCALP_ERR_HIP; \
    } while (0)

int check_common(const scalp_grid_t* g, const scalp_params_t* p, void* ws, size_t ws_bytes) {
    if (!grid_valid(g) || !params_valid(p)) return SCALP_ERR_ARG;
    if (!ws || ws_bytes < scalp_workspace_bytes(g)) return SCALP_ERR_WORKSPACE;
    return SCALP_OK;
}

// Enqueue helpers (no validation).
int enq_prepare(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                const float* contour, const Views& v, hipStream_t s) {
    if (p->contour_source == SCALP_CONTOUR_GRADIENT)
        return launch_prepare_gradient(g->width, g->height, lab, p->sigma, v.packed,
                                       reinterpret_cast<unsigned long long*>(v.ctrl + kCtrlGradMax), s);
    return launch_prepare((long long)g->width * g->height, lab, contour, p->sigma, v.packed, s);
}

int enq_init(const Img& im, const Views& v, float* centers, int* endpoints, int* counts,
             int* labels, hipStream_t s) {
    int e = launch_init_cells(im, v.packed, labels, v.acc, s);
    if (e == hipSuccess)
        e = launch_finalize(im, centers, endpoints, counts, v.acc, labels, v.ctrl, v.plist, false, s);
    return e;
}

// One window-form pass and its sums (the update cannot be fused: a pixel's
// label is known only after every window covering it).  The sums pass takes
// the labels from the window minima and resets them, so consecutive passes
// need no fill in between; first: fill the minima and clear the sums first
// (the keys of a workspace hold all ones only after a window pass or a fill;
// within a run the finalize step leaves every sum at zero, as the grid form
// relies on).
int enq_window_pass(const Img& im, const scalp_params_t* p, const Views& v, int R,
                    const float* centers, const int* endpoints, int* labels, long long clear_n,
                    bool first, hipStream_t s) {
    int e = first ? launch_fill_keys(im, v.keys, s) : (int)hipSuccess;
    if (e == hipSuccess && first) e = launch_clear(v.acc, clear_n, s);
    if (e == hipSuccess)
        e = launch_assign_window(im, v.packed, centers, endpoints, labels, v.keys, R, p->lambda,
                                 false, tuning_of(p), s);
    if (e == hipSuccess)
        e = launch_accumulate_window(im, v.packed, labels, v.keys, v.ctrl, v.acc, s);
    return e;
}

int enq_iterations(const Img& im, const scalp_params_t* p, const Views& v, float* centers,
                   int* endpoints, int* labels, int* counts, hipStream_t s, int R,
                   long long clear_n) {
    const Tuning t = tuning_of(p);
    for (int it = 0; it < p->iterations; ++it) {
        int e = p->assign_mode == SCALP_ASSIGN_WINDOW
                    ? enq_window_pass(im, p, v, R, centers, endpoints, labels, clear_n, it == 0, s)
                    : launch_assign(im, v.packed, centers, endpoints, labels, v.acc, v.ctrl,
                                    p->lambda, true, t, s);
        if (e == hipSuccess)
            e = p->project ? launch_finalize_project(im, centers, endpoints, counts, v.acc, labels, s)
                           : launch_finalize(im, centers, endpoints, counts, v.acc, labels, v.ctrl,
                                             v.plist, false, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

struct scalp_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" int scalp_graph_destroy(scalp_graph_handle h);

namespace {

int capture(scalp_graph_handle* out, const std::function<int(hipStream_t)>& body) {
    hipStream_t cs = nullptr;
    CHECK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    scalp_graph* h = new (std::nothrow) scalp_graph();
    if (!h) {
        static_cast<void>(hipStreamDestroy(cs));
        return SCALP_ERR_HIP;
    }
    int rc = SCALP_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = SCALP_ERR_HIP;
    if (rc == SCALP_OK) {
        const int e = body(cs);
        const hipError_t ee = hipStreamEndCapture(cs, &h->graph);
        if (e != hipSuccess || ee != hipSuccess) rc = SCALP_ERR_HIP;
    }
    if (rc == SCALP_OK && hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = SCALP_ERR_HIP;
    static_cast<void>(hipStreamDestroy(cs));
    if (rc != SCALP_OK) {
        scalp_graph_destroy(h);
        return rc;
    }
    *out = h;
    return SCALP_OK;
}

}  // namespace

extern "C" {

int scalp_default_params(scalp_params_t* out) {
    if (!out) return SCALP_ERR_ARG;
    out->m = 10.0f;
    out->lambda = 0.5f;
    out->sigma = 0.25f;
    out->gamma = -1.0f;
    out->iterations = 10;
    out->project = 1;
    out->reuse_prepared = 0;
    out->lds_pixels = 0;
    out->wg_size = 0;
    out->assign_mode = SCALP_ASSIGN_GRID3X3;
    out->contour_source = SCALP_CONTOUR_INPUT;
    out->exact_pruning = 1;
    out->persistent_blocks = 0;
    out->table_mode = 0;
    return SCALP_OK;
}

int scalp_make_grid(int32_t W, int32_t H, int32_t k, scalp_grid_t* out) {
    if (!out || W < 1 || H < 1 || k < 1) return SCALP_ERR_ARG;
    const long long N = (long long)W * H;
    if (N >= (1LL << 31) || (long long)k > N) return SCALP_ERR_ARG;
    const double r = grid_r(W, H, k);
    long gx = std::lround((double)W / r), gy = std::lround((double)H / r);
    gx = gx < 1 ? 1 : (gx > W ? W : gx);
    gy = gy < 1 ? 1 : (gy > H ? H : gy);
    out->width = W;
    out->height = H;
    out->k_requested = k;
    out->nx = (int32_t)gx;
    out->ny = (int32_t)gy;
    out->num_sp = (int32_t)(gx * gy);
    out->r = (float)r;
    return SCALP_OK;
}

size_t scalp_workspace_bytes(const scalp_grid_t* g) {
    if (!grid_valid(g)) return 0;
    return layout_of((long long)g->width * g->height, g->num_sp).total;
}

int scalp_prepare(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                  const float* contour, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(g, p, ws, ws_bytes);
    if (rc != SCALP_OK) return rc;
    if (!pack_inputs_ok(p, lab, contour)) return SCALP_ERR_ARG;
    library_init();
    const Views v = views_of(ws, layout_of((long long)g->width * g->height, g->num_sp));
    CHECK_HIP(enq_prepare(g, p, lab, contour, v, (hipStream_t)stream));
    return SCALP_OK;
}

int scalp_init_grid(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                    const float* contour, float* centers, int32_t* endpoints, int32_t* labels,
                    void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(g, p, ws, ws_bytes);
    if (rc != SCALP_OK) return rc;
    if (!centers || !endpoints || !labels) return SCALP_ERR_ARG;
    if (!p->reuse_prepared && !pack_inputs_ok(p, lab, contour)) return SCALP_ERR_ARG;
    library_init();
    const hipStream_t s = (hipStream_t)stream;
    const Layout L = layout_of((long long)g->width * g->height, g->num_sp);
    const Views v = views_of(ws, L);
    if (!p->reuse_prepared) CHECK_HIP(enq_prepare(g, p, lab, contour, v, s));
    // counts are not an output of this call: the projection list area holds them
    CHECK_HIP(enq_init(img_of(g, p, 0, 0), v, centers, endpoints, v.plist, labels, s));
    return SCALP_OK;
}

int scalp_assign(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                 const float* contour, const float* centers, const int32_t* endpoints,
                 int32_t* labels, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(g, p, ws, ws_bytes);
    if (rc != SCALP_OK) return rc;
    if (!centers || !endpoints || !labels) return SCALP_ERR_ARG;
    if (!p->reuse_prepared && !pack_inputs_ok(p, lab, contour)) return SCALP_ERR_ARG;
    library_init();
    const hipStream_t s = (hipStream_t)stream;
    const Views v = views_of(ws, layout_of((long long)g->width * g->height, g->num_sp));
    if (!p->reuse_prepared) CHECK_HIP(enq_prepare(g, p, lab, contour, v, s));
    if (p->assign_mode == SCALP_ASSIGN_WINDOW)
        CHECK_HIP(launch_assign_window(img_of(g, p, 0, 0), v.packed, centers, endpoints, labels,
                                       v.keys, window_radius(g), p->lambda, true, tuning_of(p),
                                       s));
    else
        CHECK_HIP(launch_assign(img_of(g, p, 0, 0), v.packed, centers, endpoints, labels, v.acc,
                                v.ctrl, p->lambda, false, tuning_of(p), s));
    return SCALP_OK;
}

int scalp_update(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                 const int32_t* labels, float* centers, int32_t* endpoints, int32_t* counts,
                 void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(g, p, ws, ws_bytes);
    if (rc != SCALP_OK) return rc;
    if (!lab || !labels || !centers || !endpoints || !counts) return SCALP_ERR_ARG;
    library_init();
    const hipStream_t s = (hipStream_t)stream;
    const Layout L = layout_of((long long)g->width * g->height, g->num_sp);
    const Views v = views_of(ws, L);
    const Img im = img_of(g, p, 0, 0);
    CHECK_HIP(launch_clear(v.acc, clear_words(L), s));
    CHECK_HIP(launch_accumulate(im, lab, labels, v.acc, s));
    CHECK_HIP(launch_finalize(im, centers, endpoints, counts, v.acc, labels, v.ctrl, v.plist,
                              p->project != 0, s));
    if (p->project)
        CHECK_HIP(launch_project(im, centers, counts, labels, endpoints, v.ctrl, v.plist, s));
    return SCALP_OK;
}

int scalp_assign_accumulate(const scalp_grid_t* g, const scalp_params_t* p, const float* centers,
                            const int32_t* endpoints, int32_t* labels, void* ws, size_t ws_bytes,
                            void* stream) {
    int rc = check_common(g, p, ws, ws_bytes);
    if (rc != SCALP_OK) return rc;
    if (!centers || !endpoints || !labels) return SCALP_ERR_ARG;
    library_init();
    const Layout L = layout_of((long long)g->width * g->height, g->num_sp);
    const Views v = views_of(ws, L);
    if (p->assign_mode == SCALP_ASSIGN_WINDOW)
        CHECK_HIP(enq_window_pass(img_of(g, p, 0, 0), p, v, window_radius(g), centers, endpoints,
                                  labels, clear_words(L), true, (hipStream_t)stream));
    else
        CHECK_HIP(launch_assign(img_of(g, p, 0, 0), v.packed, centers, endpoints, labels, v.acc,
                                v.ctrl, p->lambda, true, tuning_of(p), (hipStream_t)stream));
    return SCALP_OK;
}

int scalp_finalize(const scalp_grid_t* g, const scalp_params_t* p, const int32_t* labels,
                   float* centers, int32_t* endpoints, int32_t* counts, void* ws,
                   size_t ws_bytes, void* stream) {
    int rc = check_common(g, p, ws, ws_bytes);
    if (rc != SCALP_OK) return rc;
    if (!labels || !centers || !endpoints || !counts) return SCALP_ERR_ARG;
    library_init();
    const hipStream_t s = (hipStream_t)stream;
    const Views v = views_of(ws, layout_of((long long)g->width * g->height, g->num_sp));
    const Img im = img_of(g, p, 0, 0);
    CHECK_HIP(launch_finalize(im, centers, endpoints, counts, v.acc, labels, v.ctrl, v.plist,
                              p->project != 0, s));
    if (p->project)
        CHECK_HIP(launch_project(im, centers, counts, labels, endpoints, v.ctrl, v.plist, s));
    return SCALP_OK;
}

int scalp_run(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
              const float* contour, float* centers, int32_t* endpoints, int32_t* labels,
              int32_t* counts, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(g, p, ws, ws_bytes);
    if (rc != SCALP_OK) return rc;
    if (!centers || !endpoints || !labels || !counts) return SCALP_ERR_ARG;
    if (!p->reuse_prepared && !pack_inputs_ok(p, lab, contour)) return SCALP_ERR_ARG;
    library_init();
    const hipStream_t s = (hipStream_t)stream;
    const Layout L = layout_of((long long)g->width * g->height, g->num_sp);
    const Views v = views_of(ws, L);
    const Img im = img_of(g, p, 0, 0);
    if (!p->reuse_prepared) CHECK_HIP(enq_prepare(g, p, lab, contour, v, s));
    CHECK_HIP(enq_init(im, v, centers, endpoints, counts, labels, s));
    CHECK_HIP(enq_iterations(im, p, v, centers, endpoints, labels, counts, s, window_radius(g),
                             clear_words(L)));
    return SCALP_OK;
}

int scalp_run_static(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                     const float* contour, float* centers, int32_t* endpoints, int32_t* labels,
                     int32_t* counts, void* stream) {
    if (!grid_valid(g) || !params_valid(p) || p->reuse_prepared) return SCALP_ERR_ARG;
    if (scalp_workspace_bytes(g) > SCALP_STATIC_SCRATCH_BYTES) return SCALP_ERR_WORKSPACE;
    if (!centers || !endpoints || !labels || !counts || !pack_inputs_ok(p, lab, contour))
        return SCALP_ERR_ARG;
    void* ws = nullptr;
    const int rc = static_scratch(&ws);
    if (rc != SCALP_OK) return rc;
    return scalp_run(g, p, lab, contour, centers, endpoints, labels, counts, ws,
                     SCALP_STATIC_SCRATCH_BYTES, stream);
}

int scalp_graph_create(const scalp_grid_t* g, const scalp_params_t* p, float* centers,
                       int32_t* endpoints, int32_t* labels, int32_t* counts, void* ws,
                       size_t ws_bytes, scalp_graph_handle* out) {
    int rc = check_common(g, p, ws, ws_bytes);
    if (rc != SCALP_OK) return rc;
    if (!centers || !endpoints || !labels || !counts || !out) return SCALP_ERR_ARG;
    library_init();
    const Layout L = layout_of((long long)g->width * g->height, g->num_sp);
    const Views v = views_of(ws, L);
    const Img im = img_of(g, p, 0, 0);
    const scalp_params_t pc = *p;
    const int R = window_radius(g);
    const long long cw = clear_words(L);
    return capture(out, [&](hipStream_t s) {
        return enq_iterations(im, &pc, v, centers, endpoints, labels, counts, s, R, cw);
    });
}

int scalp_graph_launch(scalp_graph_handle h, void* stream) {
    if (!h || !h->exec) return SCALP_ERR_ARG;
    CHECK_HIP(hipGraphLaunch(h->exec, (hipStream_t)stream));
    return SCALP_OK;
}

int scalp_graph_destroy(scalp_graph_handle h) {
    if (!h) return SCALP_OK;
    int rc = SCALP_OK;
    if (h->exec && hipGraphExecDestroy(h->exec) != hipSuccess) rc = SCALP_ERR_HIP;
    if (h->graph && hipGraphDestroy(h->graph) != hipSuccess) rc = SCALP_ERR_HIP;
    delete h;
    return rc;
}

// ------------------------------------------------------------------ batched

namespace {

// Batched workspace: [packed][acc][ctrl][plist][imgs][cell_start][item_start]
struct BatchLayout {
    Layout base;
    size_t imgs, starts, items, total;
    long long N, K, items_total;
};

bool batch_layout(const scalp_batch_desc_t* d, int n, BatchLayout* out) {
    if (!d || n < 1) return false;
    long long N = 0, K = 0, I = 0;
    for (int i = 0; i < n; ++i) {
        if (!grid_valid(&d[i].grid)) return false;
        if (d[i].pix_offset != N || d[i].sp_offset != K) return false;
        N += (long long)d[i].grid.width * d[i].grid.height;
        K += d[i].grid.num_sp;
        I += (long long)d[i].grid.num_sp * slices_of(&d[i].grid, kMinAssignWG);   // most items
        if (N >= (1LL << 40) || K >= (1LL << 31) || I >= (1LL << 31)) return false;
    }
    out->items_total = I;
    out->base = layout_of(N, K);
    out->imgs = out->base.total;
    out->starts = align_up(out->imgs + sizeof(Img) * (size_t)n);
    out->items = align_up(out->starts + sizeof(int) * (size_t)(n + 1));
    out->total = align_up(out->items + sizeof(int) * 9 * (size_t)(n + 1));   // starts + 8 XCD runs
    out->N = N;
    out->K = K;
    return true;
}

int enq_batched(const scalp_batch_desc_t* d, int n, const scalp_params_t* p, const float* lab,
                const float* contour, float* centers, int* endpoints, int* labels, int* counts,
                void* ws, const BatchLayout& BL, int grid, hipStream_t s) {
    const Views v = views_of(ws, BL.base);
    char* b = static_cast<char*>(ws);
    Img* imgs = reinterpret_cast<Img*>(b + BL.imgs);
    int* starts = reinterpret_cast<int*>(b + BL.starts);
    int* items = reinterpret_cast<int*>(b + BL.items);
    std::vector<Img> himg((size_t)n);
    std::vector<int> hstart((size_t)n + 1), hitem(9 * ((size_t)n + 1));
    long long total_items = 0;
    for (int i = 0; i < n; ++i) {
        himg[(size_t)i] = img_of(&d[i].grid, p, d[i].pix_offset, d[i].sp_offset);
        hstart[(size_t)i] = d[i].sp_offset;
        hitem[(size_t)i] = (int)total_items;
        total_items += (long long)d[i].grid.num_sp * himg[(size_t)i].spl;   // < 2^31: batch_layout
    }
    hstart[(size_t)n] = (int)BL.K;
    hitem[(size_t)n] = (int)total_items;
    // the persistent assignment's run of XCD x: the x-th eighth of each image's items
    for (int x = 0; x < 8; ++x) {
        int* run = hitem.data() + ((size_t)n + 1) * (size_t)(1 + x);
        run[0] = 0;
        for (int i = 0; i < n; ++i) {
            const long long ni = (long long)hitem[(size_t)i + 1] - hitem[(size_t)i];
            run[i + 1] = run[i] + (int)((ni * (x + 1) >> 3) - (ni * x >> 3));
        }
    }
    int e = launch_write_bytes(imgs, himg.data(), sizeof(Img) * (size_t)n, s);
    if (e == hipSuccess) e = launch_write_bytes(starts, hstart.data(), sizeof(int) * (size_t)(n + 1), s);
    if (e == hipSuccess) e = launch_write_bytes(items, hitem.data(), sizeof(int) * hitem.size(), s);
    if (e == hipSuccess && !p->reuse_prepared) {
        if (p->contour_source == SCALP_CONTOUR_GRADIENT) {
            // the prior is normalised per image: one max + pack per image
            unsigned long long* mx = reinterpret_cast<unsigned long long*>(v.ctrl + kCtrlGradMax);
            for (int i = 0; e == hipSuccess && i < n; ++i)
                e = launch_prepare_gradient(d[i].grid.width, d[i].grid.height,
                                            lab + 3 * d[i].pix_offset, p->sigma,
                                            v.packed + d[i].pix_offset, mx, s);
        } else {
            e = launch_prepare(BL.N, lab, contour, p->sigma, v.packed, s);
        }
    }
    if (e == hipSuccess) e = launch_init_cells_batched(imgs, starts, n, (int)BL.K, v.packed, labels, v.acc, s);
    if (e == hipSuccess)
        e = launch_finalize_batched(imgs, starts, n, (int)BL.K, centers, endpoints, counts, v.acc,
                                    labels, v.ctrl, v.plist, false, s);
    const Tuning t = tuning_of(p);
    long long max_block = 0;
    for (int i = 0; i < n; ++i)
        max_block = std::max(max_block, block_pixels(d[i].grid.width, d[i].grid.height,
                                                     d[i].grid.nx, d[i].grid.ny));
    for (int it = 0; e == hipSuccess && it < p->iterations; ++it) {
        e = launch_assign_persistent(imgs, items, n, (int)total_items, v.packed, centers, endpoints,
                                     labels, v.acc, v.ctrl, p->lambda, t, grid, s);
        if (e == hipSuccess)
            e = p->project ? launch_finalize_project_batched(imgs, starts, n, (int)BL.K, max_block,
                                                             centers, endpoints, counts, v.acc,
                                                             labels, v.ctrl, s)
                           : launch_finalize_batched(imgs, starts, n, (int)BL.K, centers,
                                                     endpoints, counts, v.acc, labels, v.ctrl,
                                                     v.plist, false, s);
    }
    return e;
}

}  // namespace

size_t scalp_batch_workspace_bytes(const scalp_batch_desc_t* descs, int32_t n) {
    BatchLayout BL;
    if (!batch_layout(descs, n, &BL)) return 0;
    return BL.total;
}

int scalp_run_batched(const scalp_batch_desc_t* descs, int32_t n, const scalp_params_t* p,
                      const float* lab, const float* contour, float* centers, int32_t* endpoints,
                      int32_t* labels, int32_t* counts, void* ws, size_t ws_bytes,
                      void* stream) {
    BatchLayout BL;
    if (!batch_layout(descs, n, &BL) || !params_valid(p)) return SCALP_ERR_ARG;
    if (p->assign_mode != SCALP_ASSIGN_GRID3X3) return SCALP_ERR_UNSUPPORTED;
    if (!centers || !endpoints || !labels || !counts) return SCALP_ERR_ARG;
    if (!p->reuse_prepared && !pack_inputs_ok(p, lab, contour)) return SCALP_ERR_ARG;
    if (!ws || ws_bytes < BL.total) return SCALP_ERR_WORKSPACE;
    library_init();
    const int grid = persistent_grid(tuning_of(p));
    if (grid < 1) return SCALP_ERR_HIP;
    CHECK_HIP(enq_batched(descs, n, p, lab, contour, centers, endpoints, labels, counts, ws, BL,
                          grid, (hipStream_t)stream));
    return SCALP_OK;
}

int scalp_batched_graph_create(const scalp_batch_desc_t* descs, int32_t n, const scalp_params_t* p,
                               const float* lab, const float* contour, float* centers,
                               int32_t* endpoints, int32_t* labels, int32_t* counts, void* ws,
                               size_t ws_bytes, scalp_graph_handle* out) {
    BatchLayout BL;
    if (!batch_layout(descs, n, &BL) || !params_valid(p)) return SCALP_ERR_ARG;
    if (p->assign_mode != SCALP_ASSIGN_GRID3X3) return SCALP_ERR_UNSUPPORTED;
    if (!centers || !endpoints || !labels || !counts || !out) return SCALP_ERR_ARG;
    if (!p->reuse_prepared && !pack_inputs_ok(p, lab, contour)) return SCALP_ERR_ARG;
    if (!ws || ws_bytes < BL.total) return SCALP_ERR_WORKSPACE;
    library_init();
    // the occupancy query runs before the capture
    const int grid = persistent_grid(tuning_of(p));
    if (grid < 1) return SCALP_ERR_HIP;
    return capture(out, [&](hipStream_t s) {
        return enq_batched(descs, n, p, lab, contour, centers, endpoints, labels, counts, ws, BL,
                           grid, s);
    });
}

// ------------------------------------------------------------------ soft

}  // extern "C"

namespace {

// saved: [A: T][B][9][N] float, [Bf: T][B][9][N] float, [Z: T][B][K] double
struct SoftSaved {
    size_t a, bf, z, total;
};

SoftSaved soft_saved_layout(const scalp_grid_t* g, long long B, long long T) {
    const long long N = (long long)g->width * g->height, K = g->num_sp;
    SoftSaved s;
    s.a = 0;
    s.bf = align_up((size_t)(T * B * 9 * N) * 4);
    s.z = s.bf + align_up((size_t)(T * B * 9 * N) * 4);
    s.total = s.z + align_up((size_t)(T * B * K) * 8);
    return s;
}

// workspace: [packed B*N float4][gd B*9*N][gf B*N float4][gth 2 x B*K*5 double]
// [cand B*K*2 float4][gmask B*N uint16]
struct SoftWs {
    size_t packed, gd, gf, gth0, gth1, cand, gmask, total;
};

SoftWs soft_ws_layout(const scalp_grid_t* g, long long B) {
    const long long N = (long long)g->width * g->height, K = g->num_sp;
    SoftWs w;
    w.packed = 0;
    w.gd = align_up((size_t)(B * N) * 16);
    w.gf = w.gd + align_up((size_t)(B * 9 * N) * 4);
    w.gth0 = w.gf + align_up((size_t)(B * N) * 16);
    w.gth1 = w.gth0 + align_up((size_t)(B * K * 5) * 8);
    w.cand = w.gth1 + align_up((size_t)(B * K * 5) * 8);
    w.gmask = w.cand + align_up((size_t)(B * K * 2) * 16);
    w.total = w.gmask + align_up((size_t)(B * N) * 2);
    return w;
}

bool soft_args_ok(const scalp_grid_t* g, const scalp_params_t* p, float temperature,
                  int32_t batch) {
    if (!grid_valid(g) || !params_valid(p)) return false;
    if (p->assign_mode != SCALP_ASSIGN_GRID3X3) return false;   // soft slots are the 3x3 cells
    if (!(temperature > 0.0f) || !std::isfinite(temperature)) return false;
    if (batch < 1 || batch > 65535 || p->iterations < 1) return false;
    const long long N = (long long)g->width * g->height;
    if ((long long)batch * N >= (1LL << 40)) return false;
    // one workgroup per (image, cell, slice) must fit a 32-bit grid
    const long long items = (long long)batch * g->num_sp *
                            soft_slices(g->width, g->height, g->nx, g->ny, kMinAssignWG);
    return items <= 0x7fffffffLL;
}

int soft_cap_bytes(const scalp_params_t* p) {
    return (p->lds_pixels > 0 ? p->lds_pixels : default_lds_pixels()) * 16;
}

std::once_flag g_soft_once;

}  // namespace

extern "C" {

size_t scalp_soft_saved_bytes(const scalp_grid_t* g, int32_t batch, int32_t iterations) {
    if (!grid_valid(g) || batch < 1 || iterations < 1) return 0;
    return soft_saved_layout(g, batch, iterations).total;
}

size_t scalp_soft_workspace_bytes(const scalp_grid_t* g, int32_t batch) {
    if (!grid_valid(g) || batch < 1) return 0;
    return soft_ws_layout(g, batch).total;
}

int scalp_soft_forward(const scalp_grid_t* g, const scalp_params_t* p, float temperature,
                       int32_t batch, const float* lab, const float* contour, float* centers_t,
                       float* q_t, void* saved, void* ws, size_t ws_bytes, void* stream) {
    if (!soft_args_ok(g, p, temperature, batch)) return SCALP_ERR_ARG;
    if (p->contour_source != SCALP_CONTOUR_INPUT) return SCALP_ERR_UNSUPPORTED;
    if (!centers_t || !q_t || !saved) return SCALP_ERR_ARG;
    if (!p->reuse_prepared && !pack_inputs_ok(p, lab, contour)) return SCALP_ERR_ARG;
    const SoftWs W = soft_ws_layout(g, batch);
    if (!ws || ws_bytes < W.total) return SCALP_ERR_WORKSPACE;
    library_init();
    std::call_once(g_soft_once, [] { lift_soft_lds_limits(); });
    const hipStream_t s = (hipStream_t)stream;
    const long long N = (long long)g->width * g->height, K = g->num_sp, B = batch;
    const int T = p->iterations;
    const Img im = img_of(g, p, 0, 0);
    const SoftGeom geo = soft_geom(g->width, g->height, g->nx, g->ny, batch, im.spw, im.gamma,
                                   p->lambda, temperature, tuning_of(p).wg,
                                   p->exact_pruning);
    const SoftSaved S = soft_saved_layout(g, B, T);
    char* wb = static_cast<char*>(ws);
    char* sb = static_cast<char*>(saved);
    float4* packed = reinterpret_cast<float4*>(wb + W.packed);
    float* fa = reinterpret_cast<float*>(sb + S.a);
    float* fb = reinterpret_cast<float*>(sb + S.bf);
    double* z = reinterpret_cast<double*>(sb + S.z);
    const int cap = soft_cap_bytes(p) / 16;
    if (!p->reuse_prepared) CHECK_HIP(launch_prepare(B * N, lab, contour, p->sigma, packed, s));
    CHECK_HIP(launch_soft_init(geo, packed, centers_t, s));
    for (int t = 0; t < T; ++t) {
        const long long qo = (long long)t * B * 9 * N;
        CHECK_HIP(launch_soft_assign(geo, packed, centers_t + (long long)t * B * K * 5, q_t + qo,
                                     fa + qo, fb + qo, cap, s));
        CHECK_HIP(launch_soft_update(geo, q_t + qo, packed, centers_t + (long long)t * B * K * 5,
                                     centers_t + (long long)(t + 1) * B * K * 5,
                                     z + (long long)t * B * K, s));
    }
    return SCALP_OK;
}

int scalp_soft_backward(const scalp_grid_t* g, const scalp_params_t* p, float temperature,
                        int32_t batch, const float* lab, const float* contour,
                        const float* centers_t, const float* q_t, const void* saved,
                        const float* grad_q, const float* grad_centers, float* grad_lab,
                        float* grad_contour, void* ws, size_t ws_bytes, void* stream) {
    if (!soft_args_ok(g, p, temperature, batch)) return SCALP_ERR_ARG;
    if (p->contour_source != SCALP_CONTOUR_INPUT) return SCALP_ERR_UNSUPPORTED;
    if (!centers_t || !q_t || !saved || !grad_q || !grad_centers || !grad_lab || !grad_contour ||
        !contour)
        return SCALP_ERR_ARG;
    if (!p->reuse_prepared && !lab) return SCALP_ERR_ARG;
    const SoftWs W = soft_ws_layout(g, batch);
    if (!ws || ws_bytes < W.total) return SCALP_ERR_WORKSPACE;
    library_init();
    std::call_once(g_soft_once, [] { lift_soft_lds_limits(); });
    const hipStream_t s = (hipStream_t)stream;
    const long long N = (long long)g->width * g->height, K = g->num_sp, B = batch;
    const int T = p->iterations;
    const Img im = img_of(g, p, 0, 0);
    const SoftGeom geo = soft_geom(g->width, g->height, g->nx, g->ny, batch, im.spw, im.gamma,
                                   p->lambda, temperature, tuning_of(p).wg,
                                   p->exact_pruning);
    const SoftSaved S = soft_saved_layout(g, B, T);
    char* wb = static_cast<char*>(ws);
    const char* sb = static_cast<const char*>(saved);
    float4* packed = reinterpret_cast<float4*>(wb + W.packed);
    float* gd = reinterpret_cast<float*>(wb + W.gd);
    float4* gf = reinterpret_cast<float4*>(wb + W.gf);
    double* gth[2] = {reinterpret_cast<double*>(wb + W.gth0),
                      reinterpret_cast<double*>(wb + W.gth1)};
    float4* cand = reinterpret_cast<float4*>(wb + W.cand);
    unsigned short* gmask = reinterpret_cast<unsigned short*>(wb + W.gmask);
    const float* fa = reinterpret_cast<const float*>(sb + S.a);
    const float* fb = reinterpret_cast<const float*>(sb + S.bf);
    const double* z = reinterpret_cast<const double*>(sb + S.z);
    const int cap = soft_cap_bytes(p);
    if (!p->reuse_prepared) CHECK_HIP(launch_prepare(B * N, lab, contour, p->sigma, packed, s));
    CHECK_HIP(launch_clear(reinterpret_cast<long long*>(gf), B * N * 2, s));
    CHECK_HIP(launch_widen_f32(grad_centers, gth[0], B * K * 5, s));
    int cur = 0;
    for (int t = T - 1; t >= 0; --t) {
        const long long qo = (long long)t * B * 9 * N;
        const double* zt = z + (long long)t * B * K;
        CHECK_HIP(launch_soft_bwd_update(geo, t == T - 1, q_t + qo, zt,
                                         centers_t + (long long)(t + 1) * B * K * 5, packed,
                                         gth[cur], grad_q, gd, gmask, gf, cand, s));
        CHECK_HIP(launch_soft_bwd_pass(geo, zt, gth[cur], gth[1 - cur], s));
        CHECK_HIP(launch_soft_bwd_path(geo, packed, centers_t + (long long)t * B * K * 5, fa + qo,
                                       fb + qo, gd, gmask, gf, gth[1 - cur], cap, s));
        cur = 1 - cur;
    }
    CHECK_HIP(launch_soft_bwd_finish(geo, gf, gth[cur], contour, p->sigma, grad_lab, grad_contour,
                                     s));
    return SCALP_OK;
}

// ------------------------------------------------------------------ metrics

static bool metrics_args_ok(int32_t W, int32_t H, int32_t K, int32_t R) {
    if (W < 1 || H < 1 || K < 1 || R < 1) return false;
    if ((long long)W * H >= (1LL << 31)) return false;
    return (long long)K * R <= (1LL << 30);
}

size_t scalp_metrics_workspace_bytes(int32_t width, int32_t height, int32_t num_sp,
                                     int32_t num_regions) {
    if (!metrics_args_ok(width, height, num_sp, num_regions)) return 0;
    return metrics_workspace_bytes(width, height, num_sp, num_regions);
}

int scalp_metrics(int32_t width, int32_t height, const int32_t* labels, int32_t num_sp,
                  const int32_t* gt, int32_t num_regions, float epsilon, double* out,
                  void* ws, size_t ws_bytes, void* stream) {
    if (!metrics_args_ok(width, height, num_sp, num_regions)) return SCALP_ERR_ARG;
    if (!labels || !gt || !out) return SCALP_ERR_ARG;
    if (!(epsilon > 0.0f) || epsilon > 64.0f) return SCALP_ERR_ARG;
    if (!ws || ws_bytes < metrics_workspace_bytes(width, height, num_sp, num_regions))
        return SCALP_ERR_WORKSPACE;
    CHECK_HIP(launch_metrics(width, height, labels, num_sp, gt, num_regions, epsilon, out, ws,
                             (hipStream_t)stream));
    return SCALP_OK;
}

// ------------------------------------------------------------------ maps

int scalp_boundary_map(int32_t width, int32_t height, const int32_t* labels, int32_t n, float* out,
                       void* stream) {
    if (width < 1 || height < 1 || n < 1 || !labels || !out) return SCALP_ERR_ARG;
    if ((long long)width * height >= (1LL << 31)) return SCALP_ERR_ARG;
    CHECK_HIP(launch_boundary_frequency(width, height, n, labels, out, (hipStream_t)stream));
    return SCALP_OK;
}

int scalp_contour_from_lab(int32_t width, int32_t height, const float* lab, float* out, void* ws,
                           size_t ws_bytes, void* stream) {
    if (width < 1 || height < 1 || !lab || !out) return SCALP_ERR_ARG;
    if ((long long)width * height >= (1LL << 31)) return SCALP_ERR_ARG;
    if (!ws || ws_bytes < (size_t)kGradBytes) return SCALP_ERR_WORKSPACE;
    CHECK_HIP(launch_contour_from_lab(width, height, lab, out, ws, (hipStream_t)stream));
    return SCALP_OK;
}

const char* scalp_strerror(int code) {
    switch (code) {
        case SCALP_OK: return "ok";
        case SCALP_ERR_ARG: return "invalid argument";
        case SCALP_ERR_WORKSPACE: return "workspace missing or too small";
        case SCALP_ERR_HIP: return "HIP runtime error";
        case SCALP_ERR_UNSUPPORTED: return "unsupported request";
        default: return "unknown error code";
    }
}

}  // extern "C"
