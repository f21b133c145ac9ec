// scalp_internal.h -- shared declarations of the HIP kernels and the host ABI
// layer of libscalp.so (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scalp {

// Fixed point of the colour sums in the update: values are rounded to
// multiples of 2^-24 and summed as 64-bit integers, so the sum does not
// depend on the order in which pixels arrive (atomics, workgroups).
constexpr float kFixScaleF = 16777216.0f;
constexpr double kFixInv = 1.0 / 16777216.0;

// Per-superpixel accumulator stride (int64 words): count, sum x, sum y,
// sum l, sum a, sum b, 2 pad -> one 64-byte line per superpixel.
constexpr int kAccStride = 8;

// Control words in the workspace.
enum Ctrl : int {
    kCtrlProjCount = 0,   // entries in the projection list
    kCtrlGradMax = 64,    // words 64-1087: kGradSlots partial maxima of the squared
                          // gradient magnitude (FP64 bits), one per 128-byte line
    kCtrlQueue = 1088,    // words 1088-1343: the persistent assignment's 8 queue heads
                          // (one per XCD's run of items), one per 128-byte line
    kCtrlWords = 1344
};

// The gradient maximum is kept in kGradSlots 64-bit slots kGradStride words
// apart (one per 128-byte cache line; block b of the maximum pass updates
// slot b mod kGradSlots), so that the atomics of thousands of blocks do not
// queue on one line; readers take the largest.
constexpr int kGradSlots = 32, kGradStride = 16;
constexpr int kGradBytes = kGradSlots * kGradStride * 8;

// One image as the kernels see it.
struct Img {
    int W, H, nx, ny;
    long long pix;    // first pixel in the concatenated pixel arrays
    int sp;           // first superpixel in the concatenated superpixel arrays
    float spw;        // m^2 / r^2 of Eq. (3)
    float gamma;      // gamma of Eq. (2)
    int spl;          // assignment work items per grid cell (at most WG pixels each)
    int rad;          // R = r rounded to whole pixels (the window form's half-width)
    int prune;        // 1: skip the walks that the exact lower bound of D rules out
    int strips;       // column strips of the grid assignment's cell order (see cell_in_strips)
};

// An assignment work item has at most as many pixels as its workgroup has
// lanes (one pixel per lane): cells larger than that are split into several
// items, which also spreads images with few, large superpixels over the chip.
constexpr int kMinAssignWG = 256;

struct Tuning {
    int wg;           // workgroup size of the assignment kernel (256, 512 or 1024)
    int lds_pixels;   // LDS table budget in 16-byte units
    int blocks_per_cu = 0;   // persistent launch: workgroups per CU (0: as many as fit)
    int voted = 0;           // 1: voted per-candidate tables (one buffer, two barriers)
};

int default_lds_pixels();
// LDS budget of the assignment kernels in 16-byte units (two 8-byte tables of
// this many entries for the grid form; one table of twice as many for the
// window form): 152 KiB of the 160 KiB of a gfx950 CU.
constexpr int kMaxLdsPixels = 9728;

// Raises the per-kernel dynamic LDS limit of the assignment kernels (once per
// process, before any launch or capture).
void lift_lds_limits();
int launch_write_bytes(void* dst, const void* src, size_t n, hipStream_t s);

// Launchers (return hipError_t as int).  All enqueue on `s`.
int launch_prepare(long long n, const float* lab, const float* contour, float sigma,
                   float4* packed, hipStream_t s);
int launch_clear(long long* p, long long n_words, hipStream_t s);
int launch_init_cells(const Img& im, const float4* packed, int* labels, long long* acc,
                      hipStream_t s);
int launch_assign(const Img& im, const float4* packed, const float* centres,
                  const int* endpoints, int* labels, long long* acc, int* ctrl, float lambda,
                  bool accumulate, const Tuning& t, hipStream_t s);
int launch_accumulate(const Img& im, const float* lab, const int* labels, long long* acc,
                      hipStream_t s);
// Window form of the assignment (candidate rule of Algorithm 1).  keys: one
// 64-bit minimum per pixel.  labels_out: fill the keys, then write the labels
// (labels in/out); else the keys must hold all ones on entry and keep the
// pass's minima for launch_accumulate_window.
int launch_assign_window(const Img& im, const float4* packed, const float* centres,
                         const int* endpoints, int* labels, unsigned long long* keys, int R,
                         float lambda, bool labels_out, const Tuning& t, hipStream_t s);
int launch_fill_keys(const Img& im, unsigned long long* keys, hipStream_t s);
// The update sums of a window pass: labels from the keys where a window
// covered the pixel, keys reset to all ones, the projection queue emptied.
int launch_accumulate_window(const Img& im, const float4* packed, int* labels,
                             unsigned long long* keys, int* ctrl, long long* acc, hipStream_t s);
int launch_finalize(const Img& im, float* centres, int* endpoints, int* counts,
                    long long* acc, const int* labels, int* ctrl, int* plist, bool project,
                    hipStream_t s);
// finalize + projection in one launch (one workgroup per superpixel)
// (max_block_px: the most pixels of any superpixel's 3x3 cell block in the batch)
int launch_finalize_project_batched(const Img* imgs, const int* sp_start, int n_img,
                                    int total_sp, long long max_block_px, float* centres,
                                    int* endpoints, int* counts, long long* acc, const int* labels,
                                    int* ctrl, hipStream_t s);
long long block_pixels(int W, int H, int nx, int ny);
int launch_finalize_project(const Img& im, float* centres, int* endpoints, int* counts,
                            long long* acc, const int* labels, hipStream_t s);
int launch_project(const Img& im, const float* centres, const int* counts, const int* labels,
                   int* endpoints, const int* ctrl, const int* plist, hipStream_t s);

// Batched variants: imgs/cell_start/sp_start are device arrays in the workspace.
int launch_init_cells_batched(const Img* imgs, const int* cell_start, int n_img, int total_cells,
                              const float4* packed, int* labels, long long* acc, hipStream_t s);
int launch_assign_persistent(const Img* imgs, const int* item_start, int n_img, int total_items,
                             const float4* packed, const float* centres, const int* endpoints,
                             int* labels, long long* acc, int* ctrl, float lambda,
                             const Tuning& t, int grid, hipStream_t s);
int launch_finalize_batched(const Img* imgs, const int* sp_start, int n_img, int total_sp,
                            float* centres, int* endpoints, int* counts, long long* acc,
                            const int* labels, int* ctrl, int* plist, bool project,
                            hipStream_t s);
int persistent_grid(const Tuning& t);

// ---- soft SCALP (scalp_soft.hip)
struct SoftGeom {
    int W, H, nx, ny, B;
    int wg;   // workgroup size of the path kernels (256, 512 or 1024)
    float spw, gamma, lambda, temperature;
    int prune;  // 1: skip the walks of slots whose softmax weight is provably 0
};
SoftGeom soft_geom(int W, int H, int nx, int ny, int B, float spw, float gamma, float lambda,
                   float temperature, int wg, int prune);
void lift_soft_lds_limits();
// Work items per cell of the soft assignment at workgroup size wg: a cell
// is cut into slices of whole 64-pixel chunks, at most wg pixels each.
int soft_slices(int W, int H, int nx, int ny, int wg);
int launch_soft_init(const SoftGeom& g, const float4* packed, float* theta0, hipStream_t st);
int launch_soft_assign(const SoftGeom& g, const float4* packed, const float* theta_prev, float* q,
                       float* fa, float* fb, int cap, hipStream_t st);
int launch_soft_update(const SoftGeom& g, const float* q, const float4* packed,
                       const float* theta_prev, float* theta_next, double* z, hipStream_t st);
// cand: scratch of 2 * B * K float4 (per-superpixel terms of the update backward);
// gd receives the nonzero dL/dD only, gmask ([B][N]) which of the 9 slots they are
int launch_soft_bwd_update(const SoftGeom& g, int first, const float* q, const double* z,
                           const float* theta, const float4* packed, const double* gth,
                           const float* gq_in, float* gd, unsigned short* gmask, float4* gf,
                           float4* cand, hipStream_t st);
int launch_soft_bwd_pass(const SoftGeom& g, const double* z, const double* gth, double* gth_prev,
                         hipStream_t st);
// dL/dTheta (gth, gth_prev, gth0) is FP64; cap_bytes: LDS tile budget of the path pass
int launch_soft_bwd_path(const SoftGeom& g, const float4* packed, const float* theta_prev,
                         const float* fa, const float* fb, const float* gd,
                         const unsigned short* gmask, float4* gf, double* gth_prev,
                         int cap_bytes, hipStream_t st);
int launch_soft_bwd_finish(const SoftGeom& g, const float4* gf, const double* gth0,
                           const float* contour, float sigma, float* glab, float* gcon,
                           hipStream_t st);
int launch_widen_f32(const float* src, double* dst, long long n, hipStream_t st);

// ---- per-pixel maps (scalp_maps.hip)
int launch_boundary_frequency(int W, int H, int n, const int* labels, float* out, hipStream_t s);
int launch_contour_from_lab(int W, int H, const float* lab, float* out, void* ws, hipStream_t s);
// prepare with the contour prior computed from lab (same values as
// launch_contour_from_lab followed by launch_prepare); mx: 8 bytes of scratch
int launch_prepare_gradient(int W, int H, const float* lab, float sigma, float4* packed,
                            unsigned long long* mx, hipStream_t s);

// ---- quality metrics (scalp_metrics.hip)
size_t metrics_workspace_bytes(int W, int H, int K, int R);
int launch_metrics(int W, int H, const int* S, int K, const int* G, int R, float eps, double* out,
                   void* ws, hipStream_t st);

}  // namespace scalp
