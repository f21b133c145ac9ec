/*
 * scalp.h -- C ABI of libscalp.so, the MI355X (gfx950) implementation of the
 * iterative clustering of SCALP ("Superpixels with Contour Adherence using
 * Linear Path", Giraud, Ta, Papadakis, ICPR 2018, arXiv 1903.07149).
 *
 * Conventions for every entry point
 *   - Array arguments are DEVICE pointers (e.g. torch tensor data pointers)
 *     unless marked "host".  All arrays are row-major and contiguous:
 *       lab      float32 [H][W][3]  CIELab features (l, a, b) of Sec. II-A
 *       contour  float32 [H][W]     soft contour prior C in [0, 1] of Sec. II-D
 *       labels   int32   [H][W]     superpixel index in [0, K')
 *       centers  float32 [K'][5]    cluster C_k = (l_k, a_k, b_k, x_k, y_k)
 *       endpoints int32  [K'][2]    path end pixel (x, y) of each cluster: the
 *                                   rounded barycenter, or its projection X_k*
 *                                   of Eq. (4)
 *       counts   int32   [K']       |S_k|
 *   - The caller owns every buffer, including the workspace.  The library
 *     never allocates device memory and never synchronises: every call only
 *     enqueues work on `stream` (a hipStream_t passed as void*; NULL is the
 *     null stream) and returns.  Kernel faults surface at the caller's next
 *     synchronisation.
 *   - Return value: SCALP_OK (0) or a negative SCALP_ERR_* code.  Argument
 *     errors are detected on the host before anything is enqueued.  Nothing
 *     is thrown across the ABI.
 *   - workspace / workspace_bytes: caller-allocated device scratch and its
 *     size; SCALP_ERR_WORKSPACE if it is NULL or smaller than the matching
 *     *_workspace_bytes() value.  Its contents persist between calls (the
 *     packed image, see reuse_prepared) but are otherwise opaque.
 *   - Calls that share a workspace must be ordered (same stream, or the
 *     caller synchronises); calls on distinct workspaces are independent.
 *
 * Grid (Sec. II-A): r = sqrt(N / k) with N = W*H and the requested k;
 * nx = max(1, lround(W / r)), ny = max(1, lround(H / r)), K' = nx * ny
 * (K' may differ from k; every K'-sized buffer uses K').  Pixel (x, y)
 * belongs to cell (floor(y*ny/H), floor(x*nx/W)), cluster index
 * i * nx + j.
 */
#ifndef SCALP_H
#define SCALP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SCALP_OK = 0,
    SCALP_ERR_ARG = -1,          /* invalid argument (null pointer, size, parameter range) */
    SCALP_ERR_WORKSPACE = -2,    /* workspace pointer null or smaller than required        */
    SCALP_ERR_HIP = -3,          /* a HIP runtime call or kernel launch reported an error  */
    SCALP_ERR_UNSUPPORTED = -4   /* valid request this build does not support              */
};

typedef struct {
    int32_t width, height;   /* W, H (pixels), both >= 1                     */
    int32_t k_requested;     /* k, 1 <= k <= W*H                             */
    int32_t nx, ny;          /* grid columns / rows                          */
    int32_t num_sp;          /* K' = nx * ny                                 */
    float r;                 /* sqrt(N / k), informational                  */
} scalp_grid_t;

typedef struct {
    float m;                 /* compactness of Eq. (3); paper default 10     */
    float lambda;            /* weight of Eq. (1), in [0, 1]; default 0.5    */
    float sigma;             /* scale of Eq. (2), > 0; default 0.25          */
    float gamma;             /* weight of Eq. (2), >= 0; < 0 selects 2r      */
    int32_t iterations;      /* clustering iterations (Algorithm 1); >= 0    */
    int32_t project;         /* 1: Eq. (4) projection after each update      */
    int32_t reuse_prepared;  /* 1: the workspace already holds this image's
                                packed (l, a, b, w) from an earlier call with
                                the same lab/contour/sigma; skip re-packing  */
    int32_t lds_pixels;      /* tuning: LDS budget of the assignment in 16-byte
                                units (per-candidate tables of 8-byte entries,
                                two of this many; one table of twice as many
                                with table_mode 1 and for the window form),
                                0..9728; 0 selects the default (4800)        */
    int32_t wg_size;         /* tuning: assignment workgroup size, 0 (default
                                1024), 256, 512 or 1024                      */
    int32_t assign_mode;     /* SCALP_ASSIGN_GRID3X3 (default) or
                                SCALP_ASSIGN_WINDOW, see below               */
    int32_t contour_source;  /* SCALP_CONTOUR_INPUT (default) or
                                SCALP_CONTOUR_GRADIENT, see below            */
    int32_t exact_pruning;   /* 1 (default): the 3x3 assignment skips the path
                                walk of a candidate whose exact FP32 lower
                                bound of D (lambda dcp + spatial term of
                                Eq. (3)) cannot beat the best so far, and the
                                soft forward skips the walk of a slot whose
                                softmax weight that bound proves to be 0; 0:
                                every candidate is walked.  The results are
                                the same either way; 0 or 1, else
                                SCALP_ERR_ARG                                */
    int32_t persistent_blocks; /* tuning: workgroups per compute unit of the
                                batched persistent launch, 0 (default: as many
                                as fit) or 1..16 (capped at what fits); the
                                results do not depend on it                  */
    int32_t table_mode;      /* tuning of the 3x3 assignment: 0 (default): a
                                (colour distance, w) table per candidate over
                                the rectangle of the work item's pixels and the
                                endpoint, two tables of lds_pixels entries
                                alternating, one barrier per candidate; 1: the
                                waves with a lane that walks the candidate vote
                                the table down to the box of their pixels and
                                the endpoint, one table of twice as many
                                entries, two barriers per candidate, no table
                                when no lane walks (pays off for cells much
                                larger than the workgroup).  The results do
                                not depend on it; 0 or 1, else SCALP_ERR_ARG */
} scalp_params_t;

/* Candidate rule of the assignment.
 *   SCALP_ASSIGN_GRID3X3: every pixel compares the superpixels of the 3x3 grid
 *     cells around its own cell (pixel-centric; labels are always grid
 *     neighbours).
 *   SCALP_ASSIGN_WINDOW: the window rule of Algorithm 1: the candidates of a
 *     pixel are the superpixels whose (2R+1) x (2R+1) window, centred on the
 *     rounded barycenter with R = r rounded to a whole pixel, contains it; a
 *     pixel takes the smallest D over them (the smallest k among equal D)
 *     and keeps its previous label where no window contains it (labels are
 *     then in/out for scalp_assign).  Single-image entry points only. */
enum { SCALP_ASSIGN_GRID3X3 = 0, SCALP_ASSIGN_WINDOW = 1 };

/* Where the contour prior C of Sec. II-D comes from when an entry point packs
 * the image.
 *   SCALP_CONTOUR_INPUT: the caller's contour map (float32 [H][W] in [0, 1]).
 *   SCALP_CONTOUR_GRADIENT: computed from lab while packing, with the values
 *     scalp_contour_from_lab gives (normalised gradient magnitude, per image);
 *     the contour argument is ignored and may be NULL.  Not for the soft
 *     entry points (SCALP_ERR_UNSUPPORTED): their backward returns dL/dC
 *     for a given C. */
enum { SCALP_CONTOUR_INPUT = 0, SCALP_CONTOUR_GRADIENT = 1 };

/* Fills the paper's defaults (Sec. III-A.3: m = 10, lambda = 0.5,
 * sigma = 0.25, gamma = 2r) with 10 iterations, projection on, the 3x3 grid
 * candidate rule and the caller's contour map.
 * out: host pointer.  Returns SCALP_ERR_ARG if out is NULL. */
int scalp_default_params(scalp_params_t* out);

/* Host-only grid arithmetic (Sec. II-A; see the header comment).
 * out: host pointer.  SCALP_ERR_ARG if W, H < 1, k < 1, k > W*H or
 * W*H >= 2^31. */
int scalp_make_grid(int32_t width, int32_t height, int32_t k, scalp_grid_t* out);

/* Bytes of device workspace the single-image entry points need for grid g:
 * the packed (l, a, b, w) image (16 B per pixel), 8 B per pixel of window
 * minima, 68 B per superpixel (integer accumulators, projection queue) and
 * 5376 B of control words (projection queue length, partial maxima of the
 * computed contour prior, the batched assignment's per-XCD queue heads).
 * 0 if g is invalid. */
size_t scalp_workspace_bytes(const scalp_grid_t* g);

/* Packs lab and contour into the workspace as float4 (l, a, b, w) with
 * w = 1 - exp(-C^2 / sigma^2), the summand of Eq. (2), evaluated in FP64 and
 * rounded once to FP32. */
int scalp_prepare(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                  const float* contour, void* workspace, size_t workspace_bytes, void* stream);

/* Algorithm 1, initialisation: packs the image (unless reuse_prepared), sets
 * labels to the cell index of every pixel, centers to each cell's mean
 * colour and barycenter, and endpoints to the rounded barycenters
 * floor(x + 0.5).  Means use exact integer sums of the positions and of the
 * colours in 2^-24 fixed point, divided in FP64 and rounded once to FP32. */
int scalp_init_grid(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                    const float* contour, float* centers, int32_t* endpoints, int32_t* labels,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Algorithm 1, one assignment pass from the given centers and endpoints
 * (endpoints outside the image are clamped into it): every pixel compares the distance D of Eqs. (1)-(3), computed along the
 * Bresenham path from the pixel to each candidate's endpoint (Sec. II-B),
 * over the superpixels of the 3x3 grid cells around its own cell, and takes
 * the first strict minimum in ascending superpixel order.  FP32 arithmetic
 * in a fixed per-pixel order (no contraction), so labels are reproducible
 * bit for bit.  labels: output (in/out with SCALP_ASSIGN_WINDOW). */
int scalp_assign(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                 const float* contour, const float* centers, const int32_t* endpoints,
                 int32_t* labels, void* workspace, size_t workspace_bytes, void* stream);

/* Algorithm 1, cluster update, then (if p->project) the projection of
 * Eq. (4): centers (in/out) become the mean colour and barycenter of each
 * superpixel of `labels` (empty superpixels keep their center); endpoints
 * (in/out) become the rounded barycenter, or, when that pixel's label is
 * not k, the member pixel nearest to the barycenter (ties: lowest raster
 * index); counts: output.  Labels outside [0, K') are ignored. */
int scalp_update(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                 const int32_t* labels, float* centers, int32_t* endpoints, int32_t* counts,
                 void* workspace, size_t workspace_bytes, void* stream);

/* The two halves of one fused iteration of scalp_run, for callers that step
 * the loop themselves.  scalp_assign_accumulate: one assignment pass exactly
 * as scalp_assign (on the packed image already in the workspace) that also
 * adds each pixel's position and 2^-24 fixed-point colour to its
 * superpixel's integer sums in the workspace.  scalp_finalize: the update of
 * scalp_update computed from those sums (centers, endpoints with the Eq. (4)
 * projection if p->project, counts), which then clears the sums.  The sums
 * are zero after scalp_init_grid, scalp_update, scalp_finalize and
 * scalp_run. */
int scalp_assign_accumulate(const scalp_grid_t* g, const scalp_params_t* p, const float* centers,
                            const int32_t* endpoints, int32_t* labels, void* workspace,
                            size_t workspace_bytes, void* stream);
int scalp_finalize(const scalp_grid_t* g, const scalp_params_t* p, const int32_t* labels,
                   float* centers, int32_t* endpoints, int32_t* counts, void* workspace,
                   size_t workspace_bytes, void* stream);

/* Algorithm 1 end to end: prepare, init, then p->iterations x (assign,
 * update, projection).  The update is fused into the assignment kernel.
 * centers, endpoints, labels, counts: outputs. */
int scalp_run(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
              const float* contour, float* centers, int32_t* endpoints, int32_t* labels,
              int32_t* counts, void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): scalp_run
 * without a workspace argument.  The same computation and outputs, with
 * scalp_run's workspace replaced by a scratch array the library keeps in
 * device memory: SCALP_STATIC_SCRATCH_BYTES (64 MiB), held on every GPU the
 * library runs on until the process ends.  It allocates and frees nothing.
 * Limits: scalp_workspace_bytes(g) must not exceed the scratch (1920x1080
 * fits, 3840x2160 does not), else SCALP_ERR_WORKSPACE before anything is
 * enqueued; p->reuse_prepared must be 0 (SCALP_ERR_ARG).  All calls on one
 * GPU share that GPU's scratch, which keeps the last call's contents (each
 * call clears what it needs on its own stream): calls on one GPU that
 * overlap in time (other streams, other host threads) race, and their
 * results are undefined.  Other arguments as for scalp_run. */
#define SCALP_STATIC_SCRATCH_BYTES (64ull << 20)
int scalp_run_static(const scalp_grid_t* g, const scalp_params_t* p, const float* lab,
                     const float* contour, float* centers, int32_t* endpoints, int32_t* labels,
                     int32_t* counts, void* stream);

/* The iteration loop of scalp_run (assign, update, projection, repeated
 * p->iterations times) captured once into a hipGraph for fixed buffers, and
 * replayed with scalp_graph_launch.  The graph reads centers and endpoints
 * and leaves the next state in them, so each replay continues the run.
 * *out receives an opaque handle (host pointer).  The packed image must
 * already be in the workspace (scalp_prepare or scalp_init_grid). */
typedef struct scalp_graph* scalp_graph_handle;
int scalp_graph_create(const scalp_grid_t* g, const scalp_params_t* p, float* centers,
                       int32_t* endpoints, int32_t* labels, int32_t* counts, void* workspace,
                       size_t workspace_bytes, scalp_graph_handle* out);
int scalp_graph_launch(scalp_graph_handle h, void* stream);
int scalp_graph_destroy(scalp_graph_handle h);

/* ---- Batched hard SCALP: many images of different sizes and k ---------- */

/* One image of a batch.  Pixel data of image i starts at pixel pix_offset
 * in the concatenated lab (x3 floats), contour and labels arrays; its
 * superpixels start at sp_offset in the concatenated centers (x5),
 * endpoints (x2) and counts arrays.  grid must come from scalp_make_grid. */
typedef struct {
    int64_t pix_offset;
    int32_t sp_offset;
    int32_t reserved;
    scalp_grid_t grid;
} scalp_batch_desc_t;

/* Workspace bytes for a batch (descs: host array of n_images); 0 if a
 * descriptor is invalid or the images are not concatenated in order
 * (pix_offset and sp_offset must be the running sums of W*H and K'). */
size_t scalp_batch_workspace_bytes(const scalp_batch_desc_t* descs, int32_t n_images);

/* Algorithm 1 on every image of the batch: prepare, init and
 * p->iterations x (assign + update, projection), each iteration one
 * persistent launch over a work queue of (image, cell, slice) items (a
 * cell larger than the workgroup is cut into slices of whole 64-pixel
 * chunks).  Results are identical to scalp_run on each image alone.
 * descs: host array; all other arrays are device arrays concatenated as
 * described above.  gamma < 0 selects 2r per image. */
int scalp_run_batched(const scalp_batch_desc_t* descs, int32_t n_images, const scalp_params_t* p,
                      const float* lab, const float* contour, float* centers,
                      int32_t* endpoints, int32_t* labels, int32_t* counts, void* workspace,
                      size_t workspace_bytes, void* stream);

/* The same run captured once into a hipGraph (prepare, init and all
 * iterations), replayed with scalp_graph_launch; each replay recomputes the
 * whole run from lab/contour. */
int scalp_batched_graph_create(const scalp_batch_desc_t* descs, int32_t n_images,
                               const scalp_params_t* p, const float* lab, const float* contour,
                               float* centers, int32_t* endpoints, int32_t* labels,
                               int32_t* counts, void* workspace, size_t workspace_bytes,
                               scalp_graph_handle* out);

/* ---- Soft SCALP (differentiable extension, not in the paper) ------------ */
/*
 * B images of the same size.  Q_pj = softmax_j(-D_pj / T) over the 3x3
 * candidate slots j = (di+1)*3 + (dj+1) (slots outside the grid get 0), D of
 * Eqs. (1)-(3) with paths to floor(X_k + 0.5) (no projection); soft update
 * f_k = sum Q f_p / sum Q, X_k = sum Q X_p / sum Q (a superpixel whose
 * sum Q is below 1e-6 keeps its centre); Theta_0 = cell means.  D is
 * evaluated in FP32 exactly as in the hard path; the softmax and the update
 * sums run in FP64; Q and Theta are stored as FP32.  Slot-major layouts:
 *   centers_t : float32 [iters+1][B][K'][5]   (output; Theta_0 .. Theta_T)
 *   q_t       : float32 [iters][B][9][H][W]   (output)
 *   saved     : scalp_soft_saved_bytes() bytes (output of forward, input of
 *               backward): per-iteration factors A, B of Eqs. (1)-(2) and
 *               the FP64 masses sum Q (A and B are written only for slots
 *               inside the grid whose Q the exact bound does not prove to
 *               be 0: the only ones the backward reads).
 * lab: float32 [B][H][W][3]; contour: float32 [B][H][W]; 1 <= B <= 65535.
 * The soft entry points support only SCALP_ASSIGN_GRID3X3 and
 * SCALP_CONTOUR_INPUT.
 */
size_t scalp_soft_saved_bytes(const scalp_grid_t* g, int32_t batch, int32_t iterations);
size_t scalp_soft_workspace_bytes(const scalp_grid_t* g, int32_t batch);
int scalp_soft_forward(const scalp_grid_t* g, const scalp_params_t* p, float temperature,
                       int32_t batch, const float* lab, const float* contour, float* centers_t,
                       float* q_t, void* saved, void* workspace, size_t workspace_bytes, void* stream);
/* Gradient of L given dL/dQ_T (grad_q: [B][9][H][W]) and dL/dTheta_T
 * (grad_centers: [B][K'][5]) with respect to lab (grad_lab: [B][H][W][3],
 * output) and contour (grad_contour: [B][H][W], output).  Path samples are
 * recomputed, not stored; slots whose Q is below 2^-24 contribute no path
 * terms (each is proportional to Q).  Per cell, each slot's per-sample
 * weights go to an LDS tile over the box of its walked paths (FP64, at most
 * min(16 lds_pixels, 58 KiB) bytes of tiles in all); a slot whose tile does
 * not fit scatters to global memory instead.  contour is always required (dw/dC
 * needs it); lab may be null when reuse_prepared is set and the workspace
 * holds the packed image of the forward call.  FP32 with float atomics, the
 * centre gradients summed in FP64: not bit-reproducible. */
int scalp_soft_backward(const scalp_grid_t* g, const scalp_params_t* p, float temperature,
                        int32_t batch, const float* lab, const float* contour,
                        const float* centers_t, const float* q_t, const void* saved,
                        const float* grad_q, const float* grad_centers, float* grad_lab,
                        float* grad_contour, void* workspace, size_t workspace_bytes,
                        void* stream);

/* ---- Quality metrics (Sec. III-A.2) ------------------------------------ */

/* Boundary recall (Eq. (5)), achievable segmentation accuracy (Eq. (6)),
 * undersegmentation error (Eq. (7)) and compactness (Eq. (8)) of the label
 * map `labels` (int32 [H][W], values in [0, num_sp)) against the
 * ground-truth partition `gt` (int32 [H][W], values in [0, num_regions)).
 * A pixel is a boundary pixel when a 4-neighbour inside the image has
 * another label; BR counts ground-truth boundary pixels with a superpixel
 * boundary pixel at Euclidean distance < epsilon (the paper uses 2;
 * 0 < epsilon <= 64, else SCALP_ERR_ARG);
 * perimeters count 4-connected pixel edges, the image border included.
 * Pixels whose label or region is out of range are left out of the overlap
 * table and the perimeters.  out: device double[6] = {BR, ASA, UE, CO,
 * number of ground-truth boundary pixels, number of superpixel boundary
 * pixels}.  Sums are integers, or FP64 in a fixed order: the result is
 * deterministic.  SCALP_ERR_ARG if num_sp * num_regions > 2^30. */
size_t scalp_metrics_workspace_bytes(int32_t width, int32_t height, int32_t num_sp,
                                     int32_t num_regions);
int scalp_metrics(int32_t width, int32_t height, const int32_t* labels, int32_t num_sp,
                  const int32_t* gt, int32_t num_regions, float epsilon, double* out,
                  void* workspace, size_t workspace_bytes, void* stream);

/* ---- Per-pixel maps -------------------------------------------------------- */

/* Multi-scale boundary map: labels holds n label maps int32 [n][H][W] of one
 * image (e.g. decompositions at several k, Sec. III-A.2 uses 12 scales from 6
 * to 600 superpixels); out float32 [H][W] receives, per pixel, the fraction
 * c/n (FP32 division) of maps in which it is a boundary pixel (a 4-neighbour
 * inside the image has another label). */
int scalp_boundary_map(int32_t width, int32_t height, const int32_t* labels, int32_t n,
                       float* out, void* stream);

/* A soft contour prior C in [0, 1] (Sec. II-D) computed from the image: the
 * central-difference gradient magnitude of lab (float32 [H][W][3];
 * replicated borders; sqrt of the sum over channels of gx^2 + gy^2 with
 * g = (f(+1) - f(-1)) / 2) divided by its maximum over the image, in FP64
 * and rounded once to FP32; all zeros for a constant image.  A detector-free
 * stand-in for the learned detectors of Sec. II-E.  workspace: at least
 * 4096 bytes of device memory (8-byte aligned), else SCALP_ERR_WORKSPACE.
 * out: float32 [H][W]. */
int scalp_contour_from_lab(int32_t width, int32_t height, const float* lab, float* out,
                           void* workspace, size_t workspace_bytes, void* stream);

/* Static description of a code. */
const char* scalp_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SCALP_H */
