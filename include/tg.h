/*
 * tg.h -- C ABI of libtg, the MI355X (gfx950) library for TrackerSplat's
 * tracking-to-Gaussian motion transfer and its differentiable rasteriser.
 *
 * Paper: "TrackerSplat: Exploiting Point Tracking for Fast and Robust Dynamic
 * 3D Gaussians Reconstruction", SIGGRAPH Asia 2025.
 *
 * One frame of motion transfer is the call sequence
 *     tg_preprocess -> tg_bin_sort -> tg_splat_accumulate
 *                   -> tg_solve_views -> tg_triangulate
 * and the post-relocation refinement uses
 *     tg_preprocess -> tg_bin_sort -> tg_raster_fwd / tg_raster_bwd
 *                   -> tg_l1_loss_grad (+ tg_ssim_loss_grad for the 3DGS
 *                      objective) -> tg_adam_step / tg_adam_step_rows.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns tg_status.  Argument errors (null pointers,
 *    negative sizes, misaligned records, too many views) are detected on the
 *    host before anything is launched and leave all buffers untouched.
 *  - Every call is asynchronous on the caller's HIP stream (`stream`, a
 *    hipStream_t; NULL means the default stream).  No call synchronises the
 *    device.  Conditions only the device can see (pair-list overflow) are
 *    written to caller-visible device words that the caller reads after it
 *    synchronises.
 *  - The caller owns every buffer.  Pointers marked "device" must be device
 *    memory (e.g. torch tensors); pointers marked "host" are read during the
 *    call only.  The library keeps no pointer after it returns and allocates
 *    no device memory: scratch space comes from a caller workspace whose size
 *    is returned by a query call (ws == NULL).
 *  - Arrays are C-contiguous, float32 unless stated; "[V,N,k]" means view
 *    major, then Gaussian, then component.  Record arrays (rec, acc) must be
 *    16-byte aligned.
 *  - Calls on different streams with disjoint output buffers may run
 *    concurrently.  No exception crosses the ABI.
 */
#ifndef TG_H
#define TG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TG_ABI_VERSION 1
#define TG_TILE 16          /* pixels per tile side (16x16 = 256 pixels)      */
#define TG_MAX_VIEWS 32     /* views per launch; more views are chunked       */
#define TG_ACC_STRIDE 16    /* floats per accumulator record                  */
#define TG_REC_STRIDE 8     /* floats per splat record                        */
#define TG_MAX_SLOTS 8      /* Gaussian sets per batched accumulate launch    */
#define TG_MAX_FRAMES 4     /* frames sharing one alpha/T evaluation          */
#define TG_REG_K_MAX 8      /* neighbours of the regularisation               */

typedef enum tg_status {
    TG_OK = 0,
    TG_ERR_INVALID_ARG = 1,  /* null pointer, bad size or mode               */
    TG_ERR_ALIGNMENT = 2,    /* record array not 16-byte aligned              */
    TG_ERR_WORKSPACE = 3,    /* workspace missing or smaller than required    */
    TG_ERR_OVERFLOW = 4,     /* host-detected capacity problem                */
    TG_ERR_DEVICE = 5,       /* a HIP runtime call failed                     */
    TG_ERR_BUDGET = 6,       /* serving: request does not fit the budget      */
    TG_ERR_UNSUPPORTED = 7   /* size outside what this build supports         */
} tg_status;

/* Pinhole camera (80 bytes).  p_cam = R x + t with R row-major world->camera;
 * pixel = (fx p_x/p_z + cx, fy p_y/p_z + cy); pixel (row r, column c) is
 * sampled at (c, r).  x right, y down, z forward. */
typedef struct tg_camera {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float pad[2];
} tg_camera;

/* Method constants.  tg_default_params() fills the values used throughout:
 * renderer constants (alpha clamp 0.99, alpha_min 1/255, T_min 1e-4,
 * dilation 0.3 px^2, 3-sigma extent, near plane 0.2, Jacobian clamp 1.3x the
 * half field of view) and the unsolvable thresholds of Sec. 5.2 (determinant
 * of V1 below 1e-12, accumulated alpha below 1e-3, fewer than 2 pixels per
 * view; fewer than 2 views, total alpha below 1e-3, fewer than 3 pixels
 * across views).  iso_min (1e-4) makes "near-singular V1" (Sec. 4.3.5)
 * scale-invariant: the covered pixels must not lie (nearly) on one line. */
typedef struct tg_params {
    float near_z;
    float dilation;
    float extent;
    float j_clamp;
    float alpha_min;
    float alpha_max;
    float t_min;
    float static_px;        /* |x' - x| below this counts as static (Sec. 4.5.2) */
    double det_min;
    double iso_min;         /* near-singular V1: 4 det(C)/tr(C)^2 below this,
                               C the weighted covariance of the pixel offsets  */
    double wsum_min;
    double wsum_total_min;
    int32_t pix_min;
    int32_t views_min;
    int32_t pix_total_min;
    int32_t coarse_shift;   /* log2 of tiles per coarse-bin side (default 3)  */
    /* motion regularisation (Sec. 4.5, Sec. 5.2) */
    int32_t reg_k;          /* neighbours, 1..TG_REG_K_MAX (default 8)        */
    int32_t static_min_pix; /* static in a view: more than this many pixels  */
    double static_frac;     /* ... of which more than this fraction static   */
    int32_t static_views;   /* static Gaussian: static in at least this many views */
    int32_t reserved;
} tg_params;

/* 3D Gaussians (Sec. 3.1): mean, rotation, scale, opacity, optional SH
 * colour.  All device pointers. */
typedef struct tg_gaussians {
    float* means;        /* [N,3]                                             */
    float* quats;        /* [N,4] (w,x,y,z); need not be normalised           */
    float* scales;       /* [N,3] linear (scale_mode 0) or log (scale_mode 1) */
    float* opacity;      /* [N]   in (0,1) (opacity_mode 0) or logit (mode 1) */
    float* sh;           /* [N,(d+1)^2,3] SH coefficients or NULL             */
    int32_t sh_degree;   /* 0..3                                              */
    int32_t scale_mode;
    int32_t opacity_mode;
    int32_t pad;
} tg_gaussians;

/* Per-(view, Gaussian) splats written by tg_preprocess.  All device. */
typedef struct tg_splats {
    float* rec;          /* [V,N,8]: mu_x, mu_y, conic a, b, c, opacity,
                            depth, 0.  mu is the splat centre; conic is the
                            inverse of the dilated 2D covariance.  16B aligned */
    float* cov2d;        /* [V,N,3]: undilated Sigma_2D (a, b, c) of Eq. 1    */
    uint16_t* rect;      /* [V,N,4]: tile rectangle tx0, ty0, tx1, ty1
                            (half-open; all zero when culled)                 */
    uint32_t* key;       /* [V,N]: FP32 bits of the camera-space depth, or
                            0xFFFFFFFF when culled                            */
    float* colors;       /* [V,N,3] view-dependent RGB or NULL                */
    uint8_t* clamped;    /* [V,N,3] 1 where the colour was clamped at 0, or NULL */
} tg_splats;

/* Depth-ordered coarse-bin lists written by tg_bin_sort.  All device. */
typedef struct tg_bins {
    uint32_t* order;       /* [V,N]: Gaussian ids by (depth key, id)          */
    uint32_t* cell_ids;    /* [capacity]: per coarse bin, the ids of the
                              Gaussians whose tile rectangle meets the bin,
                              in depth order                                  */
    uint32_t* cell_ranges; /* [n_cells,2]: [start, end) into cell_ids         */
    int64_t* n_pairs;      /* [1]: number of (bin, Gaussian) pairs            */
    int32_t* overflow;     /* [1]: set to 1 when n_pairs > capacity           */
    int64_t capacity;
} tg_bins;

/* ---------------------------------------------------------------------- */
int tg_abi_version(void);
const char* tg_status_string(tg_status s);
void tg_default_params(tg_params* p);

/* Number of coarse bins over V views for N Gaussians (host arithmetic
 * only; the coarse size grows past p->coarse_shift when bin and rank bits
 * would exceed 32).  -1 on invalid arguments. */
int64_t tg_num_cells(const tg_camera* cams, int32_t V, int64_t N, const tg_params* p);
/* Number of 16x16 tiles over V views. */
int64_t tg_num_tiles(const tg_camera* cams, int32_t V);

/*
 * tg_preprocess -- EWA projection of every Gaussian into every view
 * (Sec. 3.1, Eq. 1).
 *
 * For view v and Gaussian i: p = R_v mu + t_v; culled if p_z <= near_z;
 * Sigma_3D = R S S^T R^T; Sigma_2D = J W Sigma_3D W^T J^T (W = R_v, J the
 * Jacobian of the perspective map at p, its x/y ratios clamped to j_clamp
 * times the half field of view); the dilated Sigma_2D + dilation*I gives the
 * conic and a 3-sigma radius; the tile rectangle covers the centre +- radius.
 * The integer-deciding quantities (centre, radius, rectangle, depth key) use
 * FP32 in a fixed operation order; Sigma_2D and the conic are formed in FP64
 * and rounded.  A Gaussian with a non-finite mean, quaternion, scale or
 * opacity (as passed in) is culled in every view.  With g->sh != NULL and out->colors != NULL, colours are the
 * degree-d SH evaluated in the viewing direction, +0.5, clamped at 0.
 *
 * cams: host [V] (any V >= 1; launched in chunks of TG_MAX_VIEWS).
 * Errors: TG_ERR_INVALID_ARG for null buffers, N < 0, V < 1, bad modes;
 *         TG_ERR_ALIGNMENT if out->rec is not 16-byte aligned.
 */
tg_status tg_preprocess(const tg_gaussians* g, int64_t N, const tg_camera* cams, int32_t V,
                        const tg_params* p, tg_splats* out, void* stream);

/*
 * tg_bin_sort -- depth ordering and coarse binning of the splats
 * (Sec. 3.1: blending follows depth order).
 *
 * Step 1: per view, a device LSD radix sort of the N depth keys (ties by
 * Gaussian id) gives bins->order.  Step 2: every non-culled Gaussian emits a
 * key (coarse bin | Gaussian id) for each coarse bin (2^coarse_shift tiles a
 * side) its tile rectangle meets, in (view, depth rank) order; a stable device
 * radix sort of those keys over the bin bits gives, per bin, the Gaussians in
 * depth order.  The renderer reads a tile's list as
 * the entries of its bin whose rectangle contains the tile, which is exactly
 * the depth-ordered per-tile list.
 *
 * ws/ws_bytes: workspace.  With ws == NULL the required size is written to
 * *ws_bytes and nothing runs.  bins->capacity bounds the pair count; if the
 * device count exceeds it, *bins->overflow is set, no list is written and the
 * later stages of the frame do nothing (the caller re-sizes and re-runs).
 * Errors: TG_ERR_WORKSPACE if *ws_bytes is smaller than required;
 *         TG_ERR_UNSUPPORTED if bin and id bits exceed 32 at every
 *         coarse size.
 */
tg_status tg_bin_sort(const tg_splats* s, int64_t N, const tg_camera* cams, int32_t V,
                      const tg_params* p, tg_bins* bins, void* ws, size_t* ws_bytes,
                      void* stream);

/*
 * tg_bin_sort_static -- tg_bin_sort for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that forbid
 * hipMalloc): the same results, with the workspace taken from a scratch
 * array that the library holds on each device it runs on (allocated when the
 * library's code object is loaded, kept until the process ends).  The call
 * allocates nothing and does no device synchronisation; the first call on a
 * device looks the array's address up once (no allocation).
 *
 * Limit: the workspace tg_bin_sort would ask for (query it with ws == NULL)
 * must be at most TG_BIN_SORT_STATIC_BYTES (64 MiB: about 2.4M (view,
 * Gaussian) pairs with a pair capacity of 4M); larger requests return
 * TG_ERR_WORKSPACE before anything runs.  Every call on a device shares that
 * device's array, so calls whose executions overlap on one device (several
 * streams or threads at once) race and must be serialised by the caller; a
 * call's stream order alone makes consecutive calls on one stream safe.
 * Other errors as tg_bin_sort, plus TG_ERR_DEVICE if the array's address
 * cannot be found.
 */
#define TG_BIN_SORT_STATIC_BYTES (64u << 20)
tg_status tg_bin_sort_static(const tg_splats* s, int64_t N, const tg_camera* cams, int32_t V,
                             const tg_params* p, tg_bins* bins, void* stream);

/*
 * tg_splat_accumulate -- PWI-LS statistics (Sec. 4.3.3, 4.3.4 Eq. 4,
 * Sec. 4.3.5; static-pixel counters of Sec. 4.5.2).
 *
 * For every pixel x of every view, in depth order: alpha = min(alpha_max,
 * o exp(-1/2 d^T conic d)); skip when alpha < alpha_min; stop when
 * T (1 - alpha) < t_min (that Gaussian excluded); w = alpha T.  When the
 * pixel's track is visible, add to acc[v,i] the record
 *   [w, w ux, w uy, w ux ux, w ux uy, w uy uy, w dx, w dy,
 *    w ux dx, w ux dy, w uy dx, w uy dy, 1, s, s alpha, (pad)]
 * with u = x - mu (centre of the splat), d = disp = x' - x and s = 1 when
 * |d| < static_px.  These are the centred entries of V1 = sum w P_i and
 * V2 = sum w Q_i (the paper's raw-coordinate V1, V2 follow by an exact
 * change of origin).  Then T <- T (1 - alpha).
 *
 * disp: device [V,H,W,2] float32 (x' - x in pixels).  vis: device [V,H,W]
 * uint8 or NULL (all visible).  All views must share one resolution.
 * acc: device [V,N,16] float32, zeroed by the caller (results are added);
 * no other stream may read or write it until the launch completes (an
 * unsynchronised reader on another stream has cost additions here).
 * t_final: device [V,H,W] or NULL: final transmittance per pixel.  With
 * t_final NULL, a pixel whose track is hidden (vis 0) is not visited at all:
 * it adds to no sum, and only t_final would need its transmittance.
 * stats: device int64 [4] or NULL: adds (pairs evaluated, pairs
 * contributing, pixel steps, list refill rounds) over the launch.  Evaluated pairs count the
 * depth-ordered list entries visited up to each visited pixel's termination, after
 * exact culling of Gaussians whose alpha stays below alpha_min on the whole
 * tile; a pixel step evaluates one pixel against up to 64 Gaussians.
 * Counting is a diagnostic: each wave adds its counts with atomics on the
 * same words, which serialise, so a counted launch runs about twice as long.
 */
tg_status tg_splat_accumulate(const tg_splats* s, const tg_bins* bins, int64_t N,
                              const tg_camera* cams, int32_t V, const float* disp,
                              const uint8_t* vis, const tg_params* p, float* acc,
                              float* t_final, int64_t* stats, void* stream);

/*
 * tg_acc_zero -- clear n_records accumulator records (16 floats each), the
 * zero start of the per-(view, Gaussian) sums that tg_splat_accumulate adds
 * into (Sec. 4.3.3, Eq. 4).  acc: device float32, 16-byte aligned (NULL
 * allowed when n_records is 0).  One 16-byte store per thread over as many
 * workgroups as it takes (the layout that reaches the highest HBM write rate
 * for a fill).  Errors: TG_ERR_INVALID_ARG for n_records < 0 (or so large
 * that its bytes overflow int64) or a null acc;
 * TG_ERR_ALIGNMENT; TG_ERR_DEVICE on a failed launch.
 */
tg_status tg_acc_zero(float* acc, int64_t n_records, void* stream);

/*
 * tg_splat_accumulate_batch -- the same statistics for several Gaussian sets
 * and several frames per set in one launch.
 *
 * Each target frame of a clip is transferred from the clip's first frame
 * (Sec. 4.7: motion compensation of a frame depends only on the tracks and
 * on the first frame's Gaussians), so the F frames of a slot share its
 * splats, bins, alpha and T, and differ only in their tracks: the kernel
 * evaluates alpha T once per (pixel, Gaussian) and adds frame f's record
 * (defined as for tg_splat_accumulate, with frame f's disp and vis) to
 * acc[f].  The slots form one ragged list of (slot, view, tile)
 * work; slots may differ in N, V and resolution (the views of one slot share
 * one resolution).
 *
 * slots: host [n_slots], n_slots <= TG_MAX_SLOTS, read during the call.
 * Per slot: s, bins (as from tg_preprocess / tg_bin_sort for that set),
 * cams host [V]; F in 1..TG_MAX_FRAMES; for each frame f < F: disp[f]
 * device [V,H,W,2], vis[f] device [V,H,W] uint8 or NULL, acc[f] device
 * [V,N,16] zeroed by the caller (frames are separate buffers, so each can
 * be uploaded and retired on its own); t_final device [V,H,W] or NULL.
 * Slots with N = 0 are skipped.  A slot whose bins overflowed is skipped by
 * the device (see tg_bin_sort).
 * stats as for tg_splat_accumulate, summed over every slot (frames share
 * the evaluation, so pairs count once per slot).  Results equal F separate
 * tg_splat_accumulate calls up to the order of the FP32 atomic additions.
 */
typedef struct tg_acc_slot {
    const tg_splats* s;
    const tg_bins* bins;
    const tg_camera* cams;
    int64_t N;
    int32_t V;
    int32_t F;
    const float* disp[TG_MAX_FRAMES];
    const uint8_t* vis[TG_MAX_FRAMES];
    float* acc[TG_MAX_FRAMES];
    float* t_final;
} tg_acc_slot;

tg_status tg_splat_accumulate_batch(const tg_acc_slot* slots, int32_t n_slots, const tg_params* p,
                                    int64_t* stats, void* stream);

/*
 * tg_solve_views -- per (view, Gaussian) 2D affine motion (Sec. 4.3.4 Eq. 4,
 * Sec. 4.2 Eq. 2) in FP64.
 *
 * From the centred record: V1 = [[Suu, Su],[Su^T, Sw]], V2 = [[Sud],[Sd^T]],
 * Theta = V1^{-1} V2 = [G^T; c^T]; A = I + G; mu' = mu + c (the paper's
 * A mu + b); Sigma' = A Sigma A^T with the undilated Sigma_2D.  Flags per
 * (view, Gaussian): 1 solved, 2 culled, 4 fewer than pix_min pixels,
 * 8 accumulated alpha below wsum_min, 16 near-singular V1: det V1 below
 * det_min, or 4 det(C)/tr(C)^2 below iso_min with C = Suu/Sw - (Su/Sw)(Su/Sw)^T
 * the weighted covariance of the pixel offsets, 32 a non-finite statistic
 * (a non-finite track reached the record) (bits 2-32 may combine).
 * Unsolved entries get zero mu'/Sigma'.
 * mu2d_new [V,N,2], cov2d_new [V,N,3] float32, vflags [V,N] uint8: device.
 * wn: device [V,N,2] float32 or NULL: receives each record's accumulated
 * alpha (slot 0) and pixel count (slot 12), the compact totals that
 * tg_triangulate reads (8-byte aligned).
 */
tg_status tg_solve_views(const float* acc, const tg_splats* s, int64_t N, int32_t V,
                         const tg_params* p, float* mu2d_new, float* cov2d_new,
                         uint8_t* vflags, float* wn, void* stream);

/*
 * tg_triangulate -- multi-view update of each Gaussian (Sec. 4.4) in FP64.
 *
 * Needs at least views_min solved views, total alpha >= wsum_total_min and
 * total pixels >= pix_total_min (Sec. 5.2).  Mean: homogeneous DLT over the
 * solved views' mu' in K^{-1}-normalised coordinates, smallest eigenvector
 * of the 4x4 normal matrix (Jacobi), rejected when |h_w| < 1e-12 or behind
 * a used camera.  Covariance: the 3 equations per view of
 * Sigma_2D' = J W Sigma_3D' W^T J^T (J at the new mean) in 6 unknowns,
 * unweighted normal equations, Cholesky.  Decomposition: Jacobi eigen;
 * rejected when an eigenvalue is <= 0; eigenpairs re-ordered so the scale
 * ranks match the input Gaussian's, columns sign-aligned to the old rotation,
 * det +1, quaternion with w >= 0, scales = sqrt(eigenvalues).
 * Status bits: 1 mean updated, 2 rotation/scale updated, 4 few views,
 * 8 low total alpha, 16 few total pixels, 32 non-positive eigenvalue or
 * singular covariance system, 64 degenerate DLT, 128 behind a camera,
 * 256 non-finite input: a non-finite parameter of the Gaussian (culled in
 * every view by tg_preprocess, so never updated) or a view whose statistics
 * were non-finite (left out of the update like any unsolved view).
 * Everything not updated is copied from g_in.  g_out may alias g_in (in-place
 * update).  cams: host [V]; V <= TG_MAX_VIEWS.  wn: device [V,N,2] from
 * tg_solve_views (accumulated alpha and pixel count per view, summed here
 * into the per-Gaussian totals).
 */
tg_status tg_triangulate(const float* mu2d_new, const float* cov2d_new, const uint8_t* vflags,
                         const float* wn, const tg_splats* s, const tg_gaussians* g_in,
                         int64_t N, const tg_camera* cams, int32_t V, const tg_params* p,
                         tg_gaussians* g_out, uint32_t* status, void* stream);

/*
 * tg_solve_triangulate -- tg_solve_views followed by tg_triangulate in one
 * launch (Sec. 4.3.4 Eq. 4, Sec. 4.2 Eq. 2, Sec. 4.4, thresholds of
 * Sec. 5.2): each Gaussian's per-view solves are computed from its
 * accumulator records where the update needs them, with the same FP64
 * arithmetic and the same FP32 rounding of mu' and Sigma' as the two calls,
 * and nothing is stored in between (no mu2d_new, cov2d_new, vflags, wn).
 * Outputs, statuses and errors as tg_triangulate; acc and s as for
 * tg_solve_views.  cams: host [V], V <= TG_MAX_VIEWS.
 */
tg_status tg_solve_triangulate(const float* acc, const tg_splats* s, const tg_gaussians* g_in, int64_t N,
                               const tg_camera* cams, int32_t V, const tg_params* p, tg_gaussians* g_out,
                               uint32_t* status, void* stream);

/*
 * tg_solve_triangulate_batch -- the fused update of tg_solve_triangulate for
 * several Gaussian sets and several frames per set in one launch (the
 * per-step update of a serving loop whose accumulation ran as one
 * tg_splat_accumulate_batch).  Per slot: s (the set's splats), g_in (its
 * Gaussians, shared by its frames), cams: DEVICE [V] cameras (4-byte
 * aligned; the launch reads them, so they must stay valid until it has
 * run), N, V, F in 1..TG_MAX_FRAMES; per frame f < F: acc[f] device
 * [V,N,16], g_out[f] (host struct of device pointers) and status[f] (device
 * [N] or NULL).  n_slots <= TG_MAX_SLOTS.  Every argument is checked before
 * anything is launched.
 */
typedef struct tg_upd_slot {
    const tg_splats* s;
    const tg_gaussians* g_in;
    const tg_camera* cams;
    int64_t N;
    int32_t V;
    int32_t F;
    const float* acc[TG_MAX_FRAMES];
    tg_gaussians* g_out[TG_MAX_FRAMES];
    uint32_t* status[TG_MAX_FRAMES];
} tg_upd_slot;

tg_status tg_solve_triangulate_batch(const tg_upd_slot* slots, int32_t n_slots, const tg_params* p, void* stream);

/*
 * tg_serve_* -- continuous-batching motion-transfer server on one GPU (the
 * one-GPU share of the frame-parallel pipeline, Sec. 4.7; clips of a first
 * frame and several target frames, Sec. 5.1).
 *
 * Every target frame of a clip (a "stream" here) is transferred from the
 * clip's first frame, so a stream's Gaussians are projected and binned once
 * when it is admitted and stay resident while its frames arrive.  Each
 * tg_serve_step retires finished work, admits waiting streams (first in,
 * first out, no overtaking) whose resident set plus one frame's working set
 * fit in the arena, uploads the tracks of admitted streams' frames as
 * working sets fit (copy stream), and launches steps: a step takes the
 * streams whose oldest ready frame is oldest, up to max_frames of their ready
 * frames (in entries of at most TG_MAX_FRAMES), up to TG_MAX_SLOTS entries,
 * and runs one tg_splat_accumulate_batch (alpha and T evaluated once per
 * entry for its frames) and one tg_solve_triangulate_batch.  Up to
 * max_inflight steps are in flight.  An admitted stream keeps one frame's
 * working set reserved for its lifetime, so it can always progress.
 *
 * Memory: the caller owns everything.  `arena` (device, arena_bytes, the
 * HBM budget) holds every buffer the server needs (splats, bins, binning
 * workspace while binning, device cameras, per-frame accumulators and track
 * copies), sub-allocated on the host; `host_scratch` (pinned host memory,
 * at least TG_SERVE_HOST_BYTES) receives the pair counts of each binning.
 * Gaussians (tg_serve_open_stream), tracks and outputs (tg_serve_submit)
 * stay the caller's and must stay valid until the frame is reported done
 * (the Gaussians until the stream's last frame is done).  Host tracks must
 * be pinned (their upload is asynchronous).
 *
 * Times are seconds on the server's clock (tg_serve_now: host time since
 * creation, aligned with the GPU clock by an event at creation); a frame's
 * done time is when the GPU finished its step (an event), so latency =
 * done - arrival.  The server is not thread-safe: one host thread drives it.
 *
 * Dry mode (arena == NULL, dry = 1): the same policy with no device at all
 * (the arena is an address range that is never touched, uploads complete at
 * once and steps when tg_serve_dry_complete says so), for testing the
 * policy without a GPU.
 */
#define TG_SERVE_HOST_BYTES 4096
typedef struct tg_server tg_server;

typedef struct tg_serve_config {
    void* arena;            /* device memory to sub-allocate (NULL in dry mode)   */
    size_t arena_bytes;     /* its size: the HBM budget                           */
    void* host_scratch;     /* pinned host memory, >= TG_SERVE_HOST_BYTES         */
    void* compute_stream;   /* hipStream_t for every kernel                       */
    void* copy_stream;      /* hipStream_t for track uploads (may equal compute)  */
    int32_t max_inflight;   /* steps in flight, >= 1                              */
    int32_t max_frames;     /* frames of one stream per step, 1..2*TG_MAX_FRAMES  */
    int32_t max_slots;      /* entries per step, 1..TG_MAX_SLOTS                  */
    int32_t dry;            /* 1: dry mode (no device)                            */
} tg_serve_config;

typedef struct tg_serve_done {
    int64_t stream_id;
    int64_t frame_id;
    int64_t step;           /* the step that ran it (0, 1, ...; -1 if none)   */
    double arrival;
    double done;
    int32_t status;         /* TG_OK, or the error that ended the frame        */
    int32_t entry;          /* its entry within the step                       */
} tg_serve_done;

typedef struct tg_serve_stats {
    int64_t steps;              /* steps launched                                */
    int64_t entries;            /* stream entries over all steps                 */
    int64_t frames;             /* frames over all steps                         */
    int64_t rebins;             /* bindings repeated after a pair overflow       */
    int64_t max_admitted;       /* most streams admitted at once                 */
    int64_t arena_used;         /* bytes allocated now                           */
    int64_t arena_peak;         /* most bytes allocated at once                  */
    int64_t waiting_streams;    /* opened, not yet admitted                      */
    int64_t admitted_streams;   /* admitted, not yet finished                    */
    int64_t inflight_steps;
} tg_serve_stats;

/* Creates a server.  Errors: TG_ERR_INVALID_ARG for out-of-range config
 * values or a missing arena / host_scratch outside dry mode. */
tg_status tg_serve_create(const tg_serve_config* cfg, const tg_params* p, tg_server** out);
/* Waits for the work in flight, then frees the host state (the caller's
 * buffers stay the caller's). */
tg_status tg_serve_destroy(tg_server* srv);
/* Host seconds since creation (the clock of arrival and done times). */
double tg_serve_now(const tg_server* srv);
/* Opens a stream (a clip's first-frame Gaussians, N, cams host [V] with one
 * resolution, V <= TG_MAX_VIEWS; g device, linear or log scales) that
 * arrived at `arrival`; *stream_id receives its id.  TG_ERR_BUDGET when its
 * resident set plus one frame's working set exceeds the whole arena. */
tg_status tg_serve_open_stream(tg_server* srv, const tg_gaussians* g, int64_t N, const tg_camera* cams, int32_t V,
                               double arrival, int64_t* stream_id);
/* Submits target frame `frame_id` of a stream: disp [V,H,W,2] and vis
 * [V,H,W] uint8 (or NULL: all visible), on the host (host_tracks = 1,
 * pinned) or the device; the update goes to g_out (means, quats, scales;
 * the opacity is the stream's) and status [N] (device, or NULL).  Errors:
 * TG_ERR_INVALID_ARG for an unknown or closed stream. */
tg_status tg_serve_submit(tg_server* srv, int64_t stream_id, int64_t frame_id, const float* disp,
                          const uint8_t* vis, int32_t host_tracks, tg_gaussians* g_out, uint32_t* status,
                          double arrival);
/* No more frames for this stream: its resident set is released once its
 * submitted frames are done. */
tg_status tg_serve_close_stream(tg_server* srv, int64_t stream_id);
/* Retire, admit, upload, launch; never waits for the device.  *launched
 * (nullable) receives the number of steps launched. */
tg_status tg_serve_step(tg_server* srv, int32_t* launched);
/* Moves up to max finished frames into out (oldest first); *n receives the
 * count. */
tg_status tg_serve_poll(tg_server* srv, tg_serve_done* out, int32_t max, int32_t* n);
tg_status tg_serve_get_stats(const tg_server* srv, tg_serve_stats* st);
/* Dry mode only: completes the oldest n steps in flight at time `now`
 * (uploads complete at once in dry mode). */
tg_status tg_serve_dry_complete(tg_server* srv, int32_t n, double now);
/* Host-only sizing of a stream as the server allocates it: the resident set
 * (with the binning workspace and the first pair-list guess), and one
 * frame's working set with host tracks (track copies included) or with
 * device tracks.  Admission needs resident + frame_host bytes of the arena.
 * Any output may be NULL. */
tg_status tg_serve_stream_bytes(const tg_camera* cams, int32_t V, int64_t N, const tg_params* p,
                                int64_t* resident, int64_t* frame_host, int64_t* frame_device);

/*
 * tg_regularize -- motion regularisation after the multi-view update
 * (Sec. 4.5; K = 8 neighbours, Sec. 5.2).
 *
 * A Gaussian is static when, in at least p->static_views views, it is hit by
 * more than p->static_min_pix pixels of which more than p->static_frac are
 * static (acc slots 12 and 13 of tg_splat_accumulate); static Gaussians keep
 * g_ref.  Solved Gaussians (status bits 1 and 2, not static) take the
 * component-wise median, over their p->reg_k nearest solved Gaussians
 * (themselves included; distances between g_ref means, FP64, ties by index),
 * of the change against g_ref: d_mu = mu' - mu, d_S = s' - s and the Euler
 * angles (phi, theta, psi) of R' R^T = Rz(psi) Ry(theta) Rx(phi).  Every
 * other Gaussian takes the mean of its nearest solved Gaussians' filtered
 * changes.  The change is added to g_ref (rotation: R = Q R_ref); a scale
 * component that would not stay positive keeps g_ref's.  With no solved
 * Gaussian at all, nothing moves.
 *
 * g_ref, g_upd, g_out: device, linear scales (scale_mode 0); g_out may alias
 * either input; only means, quats and scales are written.  status: device
 * uint32 [N] from tg_triangulate.  acc: device [V,N,16].  reg_status:
 * device uint32 [N]: 1 static, 2 filtered, 4 propagated, 0 unchanged.
 * Workspace: query with ws == NULL (about 190 B per Gaussian plus 16 MB).
 */
tg_status tg_regularize(const tg_gaussians* g_ref, const tg_gaussians* g_upd, const uint32_t* status,
                        const float* acc, int64_t N, int32_t V, const tg_params* p, void* ws,
                        size_t* ws_bytes, tg_gaussians* g_out, uint32_t* reg_status, void* stream);

/*
 * tg_raster_fwd -- forward rasteriser for the refinement (Sec. 4.6), same
 * compositing rules as the motion path (Sec. 3.1): per pixel, in depth order,
 * C = sum_i c_i alpha_i T_i + T_final bg.  s->colors must be filled
 * (tg_preprocess with SH).  bg: host float[3] or NULL (black).
 * image: device [V,H,W,3]; t_final: device [V,H,W] or NULL; n_proc: device
 * int32 [V,H,W], the number of the tile's filtered depth-ordered entries the
 * pixel processed (the backward replays exactly these).
 */
tg_status tg_raster_fwd(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams, int32_t V,
                        const float* bg, const tg_params* p, float* image, float* t_final, int32_t* n_proc,
                        void* stream);

/*
 * tg_raster_fwd_counted -- tg_raster_fwd that also adds, to stats (device
 * int64 [2], nullable), the (pixel, Gaussian) pairs evaluated (the pixel,
 * not yet terminated, tests the tile-list entry) and contributing (the entry
 * passes every test of Sec. 3.1 and is composited).  Same outputs as
 * tg_raster_fwd.  A diagnostic: every wave adds its counts with atomics on
 * the same two words, which serialise, so a counted launch runs several
 * times longer than tg_raster_fwd; time the plain call.
 */
tg_status tg_raster_fwd_counted(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                int32_t V, const float* bg, const tg_params* p, float* image, float* t_final,
                                int32_t* n_proc, int64_t* stats, void* stream);

/*
 * tg_raster_bwd -- gradients of a loss w.r.t. the 2D splats, given dL/dimage
 * and the forward's image and n_proc.  grad2d: device [V,N,9], zeroed by the
 * caller, receives (adds) per (view, Gaussian): dL/dmu_x, dL/dmu_y, dL/dconic
 * (a, b, c; power = -1/2 (a dx^2 + c dy^2) - b dx dy), dL/dopacity (activated),
 * dL/dcolour (r, g, b).  Clamped alpha (alpha_max) passes no gradient.
 */
tg_status tg_raster_bwd(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams, int32_t V,
                        const float* image, const float* dl_dimage, const int32_t* n_proc, const tg_params* p,
                        float* grad2d, void* stream);

/*
 * tg_raster_bwd_counted -- tg_raster_bwd that also adds, to stats (device
 * int64 [3], nullable): pixel steps (one pixel against one batch of up to 64
 * Gaussians of the tile's list), pairs evaluated (entries the forward
 * processed for the pixel) and pairs contributing (entries that reach the
 * pixel and carry gradient terms).  Same outputs as tg_raster_bwd; a
 * diagnostic, slower than tg_raster_bwd for the same reason as
 * tg_raster_fwd_counted.
 */
tg_status tg_raster_bwd_counted(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                int32_t V, const float* image, const float* dl_dimage, const int32_t* n_proc,
                                const tg_params* p, float* grad2d, int64_t* stats, void* stream);

/*
 * tg_project_bwd -- chain rule from the 2D splat gradients (grad2d) through
 * Eq. 1 (EWA projection, Jacobian clamp, dilation), the SH colour (including
 * the viewing-direction term; clamped channels pass nothing), the opacity and
 * scale activations and the quaternion normalisation, summed over views.
 * grads: device buffers with the layout of g (written, not added).
 */
tg_status tg_project_bwd(const tg_gaussians* g, const tg_splats* s, int64_t N, const tg_camera* cams, int32_t V,
                         const float* grad2d, const tg_params* p, tg_gaussians* grads, void* stream);

/* L1 loss: grad[i] = scale * sign(image[i] - target[i]); adds
 * scale * sum |image - target| to *loss_sum (device float, nullable). */
tg_status tg_l1_loss_grad(const float* image, const float* target, int64_t n, float scale, float* grad,
                          float* loss_sum, void* stream);

/* Chain rule by a device scalar: out[i] = in[i] * factor[0] (factor: device
 * float, e.g. the upstream gradient of a scalar loss; out may equal in). */
tg_status tg_scale_by(float* out, const float* in, int64_t n, const float* factor, void* stream);

/* out[0] = c + sum_{i<k} w[i] x[i]: assembles a scalar objective from the
 * sums the loss kernels accumulated (x: device [k]; w: host [k], k <= 8;
 * out: device float). */
tg_status tg_scalar_affine(float* out, const float* x, int32_t k, const float* w, float c, void* stream);

/*
 * tg_ssim_loss_grad -- the structural-similarity term of the 3DGS objective
 * the refinement optimises (Sec. 4.6: (1 - lambda) L1 + lambda (1 - SSIM),
 * lambda = 0.2, as in 3DGS).  SSIM per pixel and channel over an 11x11
 * Gaussian window (sigma 1.5, zero padding at the borders) with
 * C1 = 0.01^2, C2 = 0.03^2.
 * image, target: device [B,H,W,3].  Adds scale * d(sum of the SSIM map)/d image
 * to grad (device [B,H,W,3]; so tg_l1_loss_grad, which writes grad, runs
 * first, and the caller passes scale = -lambda / (B*H*W*3) for the objective
 * above).  Adds the sum of the SSIM map (unscaled) to *ssim_sum (device
 * float, nullable).  ws: three [B,H,W,3] float maps; query with ws == NULL.
 * Errors: TG_ERR_INVALID_ARG for null buffers or negative sizes,
 *         TG_ERR_WORKSPACE if *ws_bytes is smaller than required.
 */
tg_status tg_ssim_loss_grad(const float* image, const float* target, int32_t B, int32_t H, int32_t W, float scale,
                            float* grad, float* ssim_sum, void* ws, size_t* ws_bytes, void* stream);

/* Adam (bias-corrected, step >= 1), in place on param, m, v. */
tg_status tg_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                       float beta2, float eps, int32_t step, void* stream);

/* Adam as above over n / row rows of row floats, with two learning rates:
 * the first `head` floats of every row step with lr_head, the rest with
 * lr_tail.  3DGS steps the DC SH coefficients (head = 3 of row = 3 (D+1)^2)
 * 20x faster than the higher bands.  TG_ERR_INVALID_ARG unless
 * 0 <= head <= row and n is a multiple of row. */
tg_status tg_adam_step_rows(float* param, const float* grad, float* m, float* v, int64_t n, int32_t row,
                            int32_t head, float lr_head, float lr_tail, float beta1, float beta2, float eps,
                            int32_t step, void* stream);

/* Linear index of tiles and coarse bins, for tests and tools: expands the
 * coarse lists into the per-tile depth-ordered lists.  tile_ranges [T,2]
 * start/end into tile_ids (capacity entries).  Runs two passes (count, fill)
 * using the workspace; query with ws == NULL. */
tg_status tg_bin_expand(const tg_splats* s, const tg_bins* bins, int64_t N,
                        const tg_camera* cams, int32_t V, const tg_params* p,
                        uint32_t* tile_ids, uint32_t* tile_ranges, int64_t capacity,
                        int64_t* n_out, void* ws, size_t* ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TG_H */
