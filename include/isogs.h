/*
 * isogs.h - C ABI of the MI355X (gfx950) rasterizer for isotropic Gaussian splatting.
 *
 * Method: Gong, Yu, Yue, "Isotropic Gaussian Splatting for Real-Time Radiance Field
 * Rendering" (arXiv 2403.14244). A pixel's colour is the front-to-back composite of eq. 4,
 * C = sum_k c_k alpha_k prod_{j<k}(1 - alpha_j), with the isotropic kernel of eq. 8,
 * g = exp(-|x - mu|^2 / sigma^2). On the image plane the kernel is a circle of screen
 * scale s = f sigma / z: by Section 2 ("View Dependency", and Table 1) an isotropic
 * kernel's size depends only on its distance to the view point. alpha = min(0.99, o g);
 * an entry contributes only where alpha >= 1/255 (the compact support of eq. 2); a pixel
 * stops after the entry that takes its transmittance T below 1e-4.
 *
 * Pipeline (one call each, all asynchronous on the caller's HIP stream):
 *   isogs_project    particles -> screen footprints and per-particle tile counts
 *   isogs_bin_sort   footprints -> (tile, depth)-sorted entry lists per 16x16 tile
 *   isogs_render_fwd entry lists -> image, final transmittance, last contributor
 *                    (isogs_render_fwd_ordered: the same with the tiles dispatched
 *                    longest list first)
 *   isogs_render_bwd dL/dimage -> dL/d(particle parameters), for back-propagation
 *                    (the optimisation mode of Section 3, "Optimization")
 * and, for the 2D kernel-sum representation of Section 3 (no compositing),
 * isogs_field2d_bin / isogs_field2d_fwd / isogs_field2d_bwd on the same bins, with its
 * quadtree initialisation and multiscale edits (isogs_field2d_tree_init / _prune /
 * _split), and the loss terms, isogs_ssim_fwd / _bwd and isogs_l1_fwd / _bwd.
 *
 * Conventions shared by every call:
 *   - Every buffer pointer is DEVICE memory owned by the caller, except the arrays of
 *     isogs_scene / isogs_camera structs themselves, which are HOST memory read during
 *     the call only. The library keeps no pointer after a call returns and allocates no
 *     device memory; scratch space comes from the caller's workspace (query with
 *     ws == NULL).
 *   - A batch holds V views. View v renders scene scenes[v] with camera cams[v]; views
 *     may share a scene and may have different resolutions. Per-view arrays are packed
 *     back to back in view order: particles (sum of n_v), tiles (sum of TX_v * TY_v with
 *     TX = ceil(W/16), TY = ceil(H/16)), pixels (sum of H_v * W_v).
 *   - Return codes: ISOGS_OK, or ISOGS_ERR_* below; isogs_last_error() then describes the
 *     failure. Data-dependent failures (entry capacity) cannot be known at launch time;
 *     they are reported through the device-side status word of isogs_bins. Every later
 *     call that takes those bins reads the word on the device and, unless it is ISOGS_OK,
 *     skips its work, so a caller may queue a whole forward and backward pass before it
 *     reads the status: the compositing calls then write NaN colour and transmittance and
 *     n_last 0 for every pixel (no stale image can pass for a render), the others leave
 *     their outputs unwritten.
 *   - Per-particle garbage (non-finite values, sigma <= 0, o < 1/255, depth <= near) is
 *     not an error: such a particle is culled (tile count 0).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 */
#ifndef ISOGS_H
#define ISOGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISOGS_OK 0
#define ISOGS_ERR_INVALID (-1)   /* bad argument: NULL pointer, V <= 0, n < 0, degree > 3, ... */
#define ISOGS_ERR_CAPACITY (-2)  /* entry count exceeds isogs_bins.capacity (device status) */
#define ISOGS_ERR_WORKSPACE (-3) /* workspace NULL-sized or too small */
#define ISOGS_ERR_DEVICE (-4)    /* a HIP launch failed */

/* Method constants (readings of the paper; the oracle states the same values). */
#define ISOGS_TILE 16            /* tile edge, pixels */
#define ISOGS_ALPHA_MIN_INV 255  /* entries with alpha < 1/255 are skipped (eq. 2 support) */
#define ISOGS_ALPHA_MAX 0.99f    /* alpha clamp */
#define ISOGS_T_MIN 1e-4f        /* termination threshold on transmittance */
#define ISOGS_NEAR_DEFAULT 0.2f
#define ISOGS_MAX_SH_DEGREE 3

/* A scene: structure-of-arrays FP32 particle parameters (device memory).
 *   pos      [3][n]     centres mu, rows x, y, z
 *   scale    [n]        isotropic scale sigma > 0 (linear; eq. 8)
 *   opacity  [n]        activated opacity o
 *   color    [3K][n]    colour coefficients, K = (sh_degree + 1)^2; row 3k + ch holds
 *                       coefficient k (k = l^2 + l + m) of channel ch. Colour seen along
 *                       the unit direction d = (mu - eye)/|mu - eye| is
 *                       max(0, c_0 + sum_{l>=1} c_lm Y_lm(d)) with real orthonormal
 *                       spherical harmonics Y_lm without the Condon-Shortley phase.
 * In isogs_render_bwd the same struct describes gradient OUTPUT buffers (non-const use). */
typedef struct {
    const float* pos;
    const float* scale;
    const float* opacity;
    const float* color;
    int32_t n;
    int32_t sh_degree;
} isogs_scene;

/* A pinhole camera (host struct). World point mu maps to p = R mu + t (R row-major,
 * rows = camera x right, y down, z forward); depth z = p_z; pixel coordinates
 * u = f p_x / z + cx, v = f p_y / z + cy; pixel (i, j) has its centre at (i + 1/2, j + 1/2).
 * eye is the camera centre in world space (used for the colour direction). */
typedef struct {
    float R[9];
    float t[3];
    float eye[3];
    float f;
    float cx;
    float cy;
    float near_z;   /* particles with depth <= near_z are culled; must be > 0 */
    int32_t width;
    int32_t height;
} isogs_camera;

/* Screen footprints, one record per (view, particle), packed over views (device memory).
 *   record      [N][8]  {u, v, 1/s^2, o, r, g, b, radius}, 32-byte aligned: one aligned
 *                       32-byte gather per entry when compositing. radius is the binning
 *                       radius s sqrt(ln(255 o)) (1 + 2^-10) + 2^-6 pixels; a culled particle
 *                       has an all-zero record
 *   depth       [N]     z (FP32)
 *   tile_count  [N]     number of member tiles (0 if culled)
 * A tile is a member when the FP32 distance from (u, v) to the rectangle of its pixel
 * centres, evaluated as dx = max(max(x_lo - u, u - x_hi), 0), dy likewise,
 * dx*dx + dy*dy <= radius*radius, one rounded operation at a time, holds. */
typedef struct {
    float* record;
    float* depth;
    uint32_t* tile_count;
} isogs_projected;

/* Binned and sorted entries (device memory).
 *   keys        [capacity]  optional (NULL: not written): (global tile id << 32) |
 *                           bits(depth), ascending; ties in emit order (view, particle,
 *                           row-major tile), i.e. a stable sort
 *   pidx        [capacity]  packed particle index (into isogs_projected) of each entry, in
 *                           the order of the keys
 *   ranges      [T][2]      [start, end) of each global tile's entries; [0, 0) if empty
 *   offsets     [N]         first emit position of each particle (exclusive scan of
 *                           tile_count); entry (particle p, j-th member tile in row-major
 *                           order) has emit position offsets[p] + j
 *   capacity    number of entries the two entry arrays can hold
 *   count       [1]         written: total entries (even when it exceeds capacity)
 *   status      [1]         written: ISOGS_OK, or ISOGS_ERR_CAPACITY when count > capacity
 *                           (then every later call on these bins skips its work - the
 *                           compositing calls write NaN images, see above; re-run
 *                           isogs_bin_sort with a larger capacity) */
typedef struct {
    uint64_t* keys;
    uint32_t* pidx;
    uint32_t* ranges;
    uint32_t* offsets;
    uint64_t capacity;
    uint32_t* count;
    int32_t* status;
} isogs_bins;

/* Projects every particle of every view (eq. 8 kernel as a circle of scale s = f sigma/z),
 * evaluates its colour for the view direction and counts its member tiles.
 *   scenes, cams  host arrays of V structs; out  packed over views (sum n_v records).
 * Errors: ISOGS_ERR_INVALID for NULL arrays, V <= 0, n < 0, sh_degree outside 0..3,
 * width/height <= 0, near_z <= 0, f <= 0, or a NULL buffer with n > 0. */
int isogs_project(const isogs_scene* scenes, const isogs_camera* cams, int32_t n_views,
                  const isogs_projected* out, void* stream);

/* Bins the footprints into 16x16 tiles and sorts the entries stably by (tile, depth): a
 * device LSD radix sort on the tile id, then a stable sort of every tile's segment on the
 * depth bits; fills tile ranges, per-entry particle indices and, if requested, the keys.
 *   n_per_view  host array [V]: particles of each view (the n of its scene)
 *   ws, ws_bytes  workspace; with ws == NULL only *ws_bytes is written (the bytes needed
 *                 for this capacity and these views), and nothing is launched.
 * Errors: ISOGS_ERR_INVALID (bad arguments), ISOGS_ERR_WORKSPACE (ws too small),
 * ISOGS_ERR_DEVICE; overflow of `capacity` is reported in *status on the device. */
int isogs_bin_sort(const isogs_projected* proj, const int32_t* n_per_view,
                   const isogs_camera* cams, int32_t n_views, const isogs_bins* bins,
                   void* ws, size_t* ws_bytes, void* stream);

/* isogs_bin_sort for callers that cannot allocate device memory or hand over a workspace:
 * code under HIP graph capture, tight serving loops, harnesses that forbid allocation. The
 * same kernels and outputs as isogs_bin_sort (bit for bit), with the scratch taken from a
 * static device array of ISOGS_STATIC_SCRATCH_BYTES that the library holds on each GPU it
 * runs on until the process ends (its address is looked up once per device, on the first
 * call with that device current). The caller still owns and passes proj and bins.
 *   - Limit: the call needs the scratch isogs_bin_sort reports for the same arguments
 *     (about 21 bytes per entry of capacity, 20 bytes per tile and 0.3 MB); above
 *     ISOGS_STATIC_SCRATCH_BYTES it returns ISOGS_ERR_WORKSPACE and launches nothing
 *     (128 MiB: about 6M entries, three 1080p views of a 1M-particle scene).
 *   - No hipMalloc, hipFree or allocating library call is made; the bookkeeping that must
 *     start at zero is cleared by a kernel on `stream` at every call.
 *   - Every call on one GPU shares that GPU's array, which keeps the last call's contents:
 *     calls that overlap on one GPU (other streams, other host threads) race and must be
 *     serialised by the caller.
 * Errors: as isogs_bin_sort, plus ISOGS_ERR_DEVICE if the array's address cannot be found. */
#define ISOGS_STATIC_SCRATCH_BYTES (128u << 20)
int isogs_bin_sort_static(const isogs_projected* proj, const int32_t* n_per_view,
                          const isogs_camera* cams, int32_t n_views, const isogs_bins* bins,
                          void* stream);

/* Compositing checkpoints, for isogs_render_bwd on long tile lists (at least
 * 2 * ISOGS_CKPT_CHUNK entries): at list positions k * ISOGS_CKPT_CHUNK (k >= 1) of such a
 * tile, each pixel's state before that entry - float4 {T, accumulated r, g, b} - is stored
 * at slot start / ISOGS_CKPT_CHUNK + k of the buffer (start: the tile's first entry), 256
 * float4 per slot in the tile's thread order. Slots of different tiles never overlap. A
 * buffer for bins of a given capacity takes isogs_checkpoint_bytes(capacity) bytes (device
 * memory, caller-owned). */
#define ISOGS_CKPT_CHUNK 256
size_t isogs_checkpoint_bytes(uint64_t capacity);

/* Front-to-back compositing (eq. 4) of every pixel over its tile's sorted entries.
 *   bg        host [3] background colour added as T_final * bg
 *   image     [sum 3 H_v W_v]  planar per view: [V][3][H][W]
 *   T_final   [sum H_v W_v]    transmittance left after the last composited entry
 *   n_last    [sum H_v W_v]    1 + tile-list position of the last contributing entry
 *                              (0 if none); the backward pass starts there. NULL: not
 *                              written (a forward that no backward pass follows; the
 *                              longest-first walks then do not track it)
 *   checkpoints  NULL, or a buffer of isogs_checkpoint_bytes(bins->capacity) bytes that
 *                receives the compositing checkpoints (see above)
 * Errors: ISOGS_ERR_INVALID, ISOGS_ERR_DEVICE. */
int isogs_render_fwd(const isogs_projected* proj, const int32_t* n_per_view,
                     const isogs_bins* bins, const isogs_camera* cams, int32_t n_views,
                     const float* bg, float* image, float* T_final, uint32_t* n_last,
                     float* checkpoints, void* stream);

/* Flags of isogs_render_fwd_ordered. */
#define ISOGS_FWD_WIDE 1u   /* wide walk for the longest tiles of small launches (see below) */
#define ISOGS_FWD_TIMES 2u  /* per-workgroup clock stamps in the workspace (see below) */

/* Same outputs as isogs_render_fwd (bitwise), with the tiles dispatched longest entry list
 * first: a queue of the tiles sorted by list length is built on the device and workgroup b
 * composites the tile at queue position b, so that the few very long tiles of skewed scenes
 * start first instead of trailing the launch. Launches of few tiles (at most 24576 per group
 * of 16 views) use a software-pipelined walk that shortens the longest tiles; larger ones a
 * compact walk that keeps more workgroups resident.
 *   flags  0, or ISOGS_FWD_WIDE: every tile of at least 2048 entries is composited by
 *          four workgroups, one per 8x8 quadrant, with four lanes per pixel that take the
 *          four entries of a list step together (transmittance products scanned across
 *          the lanes, the stopping entry found exactly, colour terms summed). Those tiles
 *          then agree with isogs_render_fwd up to rounding (products and sums associated
 *          per step) instead of bitwise; a single 1080p view composites about twice as
 *          fast. With or without the flag, a view's result does not depend on the other
 *          views of the launch. ISOGS_FWD_TIMES (with either walk) adds a measurement of
 *          load balance: the workspace grows by 80 bytes per tile of the call, and from byte
 *          offset (the size queried without ISOGS_FWD_TIMES) - 256 it receives one
 *          {start, end} pair of uint64 stamps of the GPU's constant 100 MHz clock per
 *          workgroup: the workgroups of the launch for the group of views whose first tile
 *          is the call's tile t occupy pairs 5t, 5t + 1, ...; a workgroup whose list was
 *          empty, or that had no tile, leaves {0, 0}. The images are the same as without it.
 *   ws, ws_bytes  workspace (query with ws == NULL, with the same flags): the queue, 4 bytes
 *                 per tile of the largest group of 16 views, plus bookkeeping
 * Errors: ISOGS_ERR_INVALID, ISOGS_ERR_WORKSPACE, ISOGS_ERR_DEVICE. */
int isogs_render_fwd_ordered(const isogs_projected* proj, const int32_t* n_per_view,
                             const isogs_bins* bins, const isogs_camera* cams, int32_t n_views,
                             const float* bg, float* image, float* T_final, uint32_t* n_last,
                             float* checkpoints, uint32_t flags, void* ws, size_t* ws_bytes,
                             void* stream);

/* Gradients of a scalar loss L with respect to the particle parameters, given dL/dimage.
 * Walks each pixel's entries in reverse from n_last, recovering the transmittance before
 * each entry as T / (1 - alpha) (no per-entry state is stored by the forward pass), and
 * sums each entry's gradient over the tile's pixels with wavefront reductions in a fixed
 * order (no floating-point atomics: results are bitwise reproducible). With the forward's
 * checkpoints, a tile of at least 2 * ISOGS_CKPT_CHUNK entries is walked as independent
 * chunks on different workgroups, each starting from the checkpoint at its end (the light
 * from behind a chunk is image - accumulated colour there).
 *   scenes, cams   the same arrays as given to isogs_project
 *   image          the forward's image (may be NULL when checkpoints is NULL)
 *   dL_dimage      [sum 3 H_v W_v], same layout as image
 *   checkpoints    NULL, or the buffer the forward filled for these bins
 *   grads          host array [V] of output buffers in scene layout; views whose scene
 *                  pointers (pos) are equal must pass equal grads entries: their
 *                  gradients are summed in view order. Outputs are overwritten.
 *   ws, ws_bytes   workspace (query with ws == NULL, 256-byte aligned): 32 bytes per
 *                  entry of capacity - each entry's gradient record is stored at its emit
 *                  position, so a particle's records are contiguous - plus a tile queue of
 *                  4 bytes per tile of the largest group of 16 views (one workgroup per
 *                  chunk of a long tile, then per tile, longest entry list first), and
 *                  the chunk list, 8 bytes per ISOGS_CKPT_CHUNK entries of capacity and
 *                  per tile
 * Errors: ISOGS_ERR_INVALID, ISOGS_ERR_WORKSPACE, ISOGS_ERR_DEVICE. */
int isogs_render_bwd(const isogs_scene* scenes, const isogs_camera* cams, int32_t n_views,
                     const isogs_projected* proj, const isogs_bins* bins, const float* bg,
                     const float* image, const float* dL_dimage, const float* T_final,
                     const uint32_t* n_last, const float* checkpoints, const isogs_scene* grads,
                     void* ws, size_t* ws_bytes, void* stream);

/* ---- Anisotropic variant (Section 1: eq. 5, eq. 6, eq. 7) ----------------------------
 * The kernels the paper sets its isotropic ones against, on the same pipeline: a particle
 * carries a rotation and three scales, its covariance is Sigma = R S S^T R^T (eq. 6), its
 * screen covariance Sigma_2D = J V Sigma V^T J^T (eq. 7: V the camera rotation, J the
 * Jacobian of the pinhole map at the centre, no low-pass term), and the screen kernel is
 * eq. 5 with Sigma_2D, g = exp(-(A dx^2 + 2 B dx dy + C dy^2)) where [[A, B], [B, C]] =
 * Sigma_2D^-1 (the conic) and (dx, dy) = pixel centre - projected centre (no factor 1/2,
 * as in eq. 8). alpha = min(0.99, o g) and everything after it - the 1/255 support, the
 * compositing of eq. 4, the stop at T < 1e-4, 16x16 tiles, the depth order - is the
 * isotropic path's. With Sigma = sigma^2 I the footprint is the full projection
 * sigma^2 J J^T of an isotropic particle (on the optical axis, the circle of scale
 * f sigma / z that isogs_project uses).
 *
 * A scene (device memory, structure of arrays, FP32):
 *   pos      [3][n]   centres
 *   rot      [4][n]   quaternions (w, x, y, z), any non-zero length (normalised inside)
 *   scale    [3][n]   linear per-axis scales > 0
 *   opacity  [n], color [3K][n]  as in isogs_scene
 * In isogs_aniso_render_bwd the same struct describes gradient OUTPUT buffers. */
typedef struct {
    const float* pos;
    const float* rot;
    const float* scale;
    const float* opacity;
    const float* color;
    int32_t n;
    int32_t sh_degree;
} isogs_aniso_scene;

/* Anisotropic footprints, packed over views like isogs_projected:
 *   fp.record  [N][8]  {u, v, A, o, r, g, b, radius} (32-byte aligned); radius is the
 *                      radius of the disk around the support ellipse A dx^2 + 2 B dx dy +
 *                      C dy^2 <= ln(255 o), sqrt(lambda_max(Sigma_2D) ln(255 o)) (1 + 2^-10)
 *                      + 2^-6 pixels; a culled particle has an all-zero record
 *   fp.depth, fp.tile_count  as in isogs_projected
 *   conic      [N][2]  {B, C} (8-byte aligned)
 * fp has the isotropic record's layout where binning reads it (centre, radius, depth,
 * tile count): isogs_bin_sort and isogs_bin_sort_static take &fp unchanged. */
typedef struct {
    isogs_projected fp;
    float* conic;
} isogs_aniso_projected;

/* Projects every particle of every view: centre, conic and binning radius of eq. 7 (FP64
 * inside, rounded once to FP32), colour as isogs_project, member-tile count. A particle
 * is culled when a parameter is non-finite, a scale <= 0, |q| = 0, o < 1/255, depth <=
 * near_z, det Sigma_2D <= 0, or its footprint has no normal FP32 form (centre, conic or
 * radius overflowing, A or C below the smallest normal FP32 value).
 * Errors: as isogs_project (rot must be non-NULL with n > 0; conic 8-byte aligned). */
int isogs_aniso_project(const isogs_aniso_scene* scenes, const isogs_camera* cams, int32_t n_views,
                        const isogs_aniso_projected* out, void* stream);

/* isogs_render_fwd_ordered for anisotropic footprints binned by isogs_bin_sort(&proj->fp):
 * the same outputs, workspace, checkpoints and flags (ISOGS_FWD_WIDE). */
int isogs_aniso_render_fwd(const isogs_aniso_projected* proj, const int32_t* n_per_view,
                           const isogs_bins* bins, const isogs_camera* cams, int32_t n_views,
                           const float* bg, float* image, float* T_final, uint32_t* n_last,
                           float* checkpoints, uint32_t flags, void* ws, size_t* ws_bytes,
                           void* stream);

/* isogs_render_bwd for the anisotropic family: gradients of the centre, the quaternion
 * (through its normalisation), the three scales, the opacity and the colour coefficients.
 * The workspace holds 48 bytes per entry of capacity (each entry's nine gradient sums)
 * instead of 32; everything else as isogs_render_bwd. */
int isogs_aniso_render_bwd(const isogs_aniso_scene* scenes, const isogs_camera* cams, int32_t n_views,
                           const isogs_aniso_projected* proj, const isogs_bins* bins, const float* bg,
                           const float* image, const float* dL_dimage, const float* T_final,
                           const uint32_t* n_last, const float* checkpoints,
                           const isogs_aniso_scene* grads, void* ws, size_t* ws_bytes, void* stream);

/* ---- 2D kernel-sum representation (Section 3, "Our Method") --------------------------
 * An image signal represented by K weighted isotropic kernels, with no compositing:
 *   f_c(x) = sum over k with |x - mu_k| < D of A_kc exp(-|x - mu_k|^2 / sigma_k^2)
 * (the reconstruction equation of Section 3, the support region of eq. 2, the kernel of
 * eq. 8), for pixel centres x = (i + 1/2, j + 1/2), x right and y down, channels
 * c = 0, 1, 2. The support test is strict and taken in FP32 one operation at a time:
 * dx = x - mu_x, dy likewise, include iff dx*dx + dy*dy < D*D. A particle with a
 * non-finite parameter or sigma <= 0 contributes nothing and gets zero gradients.
 * The calls reuse the splatting path's footprints, bins and sort: every particle is a
 * disk of radius D (record {mu_x, mu_y, 1/sigma^2, 0, A_0, A_1, A_2, D}, depth 1), so each
 * tile's list keeps particle order and every pixel's sum is taken in that fixed order. */
typedef struct {
    float* mu;      /* [2][K] centres, pixels */
    float* sigma;   /* [K] scales sigma > 0, pixels */
    float* amp;     /* [3][K] amplitudes A_k (the particle's colour) */
    int32_t K;
} isogs_field2d;

/* Footprints and tile lists of a 2D signal on a width x height image with support D.
 *   field       host struct of device arrays (read only here)
 *   fp          output footprints: record [K][8] (32-byte aligned), depth [K], tile_count [K]
 *   bins        as for isogs_bin_sort: one view of ceil(W/16) * ceil(H/16) tiles
 *   ws, ws_bytes  the isogs_bin_sort workspace of this capacity and one view (query with
 *                 ws == NULL)
 * Errors: ISOGS_ERR_INVALID (NULL arrays with K > 0, K < 0, width/height <= 0, D not
 * finite or <= 0), ISOGS_ERR_WORKSPACE, ISOGS_ERR_DEVICE; capacity overflow is reported
 * in *bins->status on the device. */
int isogs_field2d_bin(const isogs_field2d* field, int32_t width, int32_t height, float support,
                      const isogs_projected* fp, const isogs_bins* bins, void* ws, size_t* ws_bytes,
                      void* stream);

/* The image [3][H][W] of the signal binned by isogs_field2d_bin (same width, height, D):
 * one workgroup per tile, one lane per pixel, kernels added in list (particle) order.
 * Errors: ISOGS_ERR_INVALID, ISOGS_ERR_DEVICE. */
int isogs_field2d_fwd(const isogs_projected* fp, int32_t K, const isogs_bins* bins, int32_t width,
                      int32_t height, float support, float* image, void* stream);

/* Gradients of a loss with respect to mu, sigma and A, given dL/dimage [3][H][W]:
 *   dL/dA_kc  = sum_x w_c(x) g_k(x),  with w = dL/dimage and g_k the kernel of particle k
 *   dL/dmu_k  = sum_x (sum_c w_c A_kc) g_k(x) 2 (x - mu_k) / sigma_k^2
 *   dL/dsigma = sum_x (sum_c w_c A_kc) g_k(x) 2 |x - mu_k|^2 / sigma_k^3
 * Each (tile, particle) entry's six sums over the tile's pixels are formed in a fixed
 * order and stored at its emit position; each particle then adds its entries in
 * row-major tile order (bitwise reproducible, no atomics).
 *   grads       host struct of device OUTPUT arrays of the field's shapes (overwritten)
 *   ws, ws_bytes  32 bytes per entry of capacity (query with ws == NULL, 256-byte aligned)
 * Errors: ISOGS_ERR_INVALID, ISOGS_ERR_WORKSPACE, ISOGS_ERR_DEVICE. */
int isogs_field2d_bwd(const isogs_projected* fp, int32_t K, const isogs_bins* bins, int32_t width,
                      int32_t height, float support, const float* dL_dimage, const isogs_field2d* grads,
                      void* ws, size_t* ws_bytes, void* stream);

/* The 2D kernel sum with anisotropic kernels, the variant the paper times its isotropic
 * kernels against (Table 2, the settings (D, K) of the 2D fit): particle k has centre mu_k,
 * rotation angle theta_k, scales s1_k, s2_k > 0 and amplitude A_k, and the kernel of eq. 5
 * with the 2D form of eq. 6, Sigma = R(theta) diag(s1^2, s2^2) R(theta)^T,
 *   f_c(x) = sum over |x - mu_k| < D of A_kc exp(-(x - mu_k)^T Sigma_k^-1 (x - mu_k)),
 * the support, pixel grid, order of the sum and binning being those of the isotropic calls
 * above. The conic Sigma^-1 = [[P00, P01], [P01, P11]] is formed in FP64 and rounded once;
 * the exponent is evaluated in FP32. A particle with a non-finite parameter, a scale <= 0
 * or a conic entry overflowing contributes nothing and gets zero gradients. */
typedef struct {
    float* mu;      /* [2][K] centres, pixels */
    float* theta;   /* [K] rotation angles, radians */
    float* scale;   /* [2][K] scales s1, s2 > 0, pixels */
    float* amp;     /* [3][K] amplitudes */
    int32_t K;
} isogs_field2d_aniso;

/* Footprints and tile lists: fp as for isogs_field2d_bin with {mu_x, mu_y, P00, P01} in
 * the record's first half, conic_c [K] (device) receives P11.
 * Errors: as isogs_field2d_bin (conic_c NULL with K > 0 is invalid). */
int isogs_field2d_aniso_bin(const isogs_field2d_aniso* field, int32_t width, int32_t height,
                            float support, const isogs_projected* fp, float* conic_c,
                            const isogs_bins* bins, void* ws, size_t* ws_bytes, void* stream);

/* The image [3][H][W] of the binned anisotropic signal. Errors: as isogs_field2d_fwd. */
int isogs_field2d_aniso_fwd(const isogs_projected* fp, const float* conic_c, int32_t K,
                            const isogs_bins* bins, int32_t width, int32_t height, float support,
                            float* image, void* stream);

/* Gradients for dL/dimage [3][H][W]: per entry the eight sums over its tile's pixels
 * (the amplitude terms, t dx, t dy, t dx^2, t dx dy, t dy^2 with t = (sum_c w_c A_c) g),
 * stored at the entry's emit position; per particle their sum in emit order, chained in
 * FP64 to mu, theta and the scales. `field` is the binned signal (for theta and the
 * scales); grads: device OUTPUT arrays of its shapes. ws: 32 bytes per entry of capacity.
 * Errors: as isogs_field2d_bwd. */
int isogs_field2d_aniso_bwd(const isogs_field2d_aniso* field, const isogs_projected* fp,
                            const float* conic_c, const isogs_bins* bins, int32_t width,
                            int32_t height, float support, const float* dL_dimage,
                            const isogs_field2d_aniso* grads, void* ws, size_t* ws_bytes,
                            void* stream);

/* Quadtree initialisation of a 2D signal (Section 3, "Initial with Tree Structure"): the
 * leaves of a quadtree over `target` [3][height][width] become particles with the mean
 * colour of their pixels as amplitude, half the cell width as sigma and the centre of the
 * cell's in-image rectangle as mu. The tree starts from a grid of root cells of side
 * `root` (a power of two; border cells clipped to the image); a cell of side s splits into
 * its in-image quadrants when its colour variance (the mean over channels of the
 * population variance of its pixels, in FP64) exceeds tau and s/2 >= min_side. Levels
 * grow one at a time; a level whose splits would let the leaf count exceed K splits no
 * cell. Leaves are numbered by level (root first), row-major within a level.
 *   out    host struct of device arrays of capacity out->K >= K (row stride out->K)
 *   count  device int32: the number of particles written (<= K)
 *   ws, ws_bytes  workspace (query with ws == NULL, 256-byte aligned)
 * Errors: ISOGS_ERR_INVALID (sizes, root not a power of two >= min_side >= 1, tau not
 * finite or < 0, K below the number of root cells, NULL buffers), ISOGS_ERR_WORKSPACE,
 * ISOGS_ERR_DEVICE. */
int isogs_field2d_tree_init(const float* target, int32_t height, int32_t width, int32_t root,
                            int32_t min_side, float tau, int32_t K, const isogs_field2d* out,
                            int32_t* count, void* ws, size_t* ws_bytes, void* stream);

/* Multiscale edits (Section 2, "Multiscale": isotropic kernels are easily deleted or
 * divided according to their scale), order-preserving:
 *   prune  keeps the particles whose largest amplitude magnitude max_c |A_kc| >= amp_min
 *          (and drops those with a non-finite parameter or sigma <= 0);
 *   split  replaces every particle with sigma > sigma_max, in place, by four of scale
 *          sigma/2 centred at mu + (-h, -h), (+h, -h), (-h, +h), (+h, +h), h = sigma/2
 *          (one FP32 rounding each), with its amplitude; copies the others.
 *   in     host struct of device arrays (in->K particles)
 *   out    host struct of device arrays of capacity out->K (row stride out->K); outputs
 *          past the capacity are not written
 *   count  device int32: the number of outputs (may exceed the capacity)
 *   ws, ws_bytes  workspace (query with ws == NULL, 256-byte aligned)
 * Errors: ISOGS_ERR_INVALID, ISOGS_ERR_WORKSPACE, ISOGS_ERR_DEVICE. */
int isogs_field2d_prune(const isogs_field2d* in, float amp_min, const isogs_field2d* out,
                        int32_t* count, void* ws, size_t* ws_bytes, void* stream);
int isogs_field2d_split(const isogs_field2d* in, float sigma_max, const isogs_field2d* out,
                        int32_t* count, void* ws, size_t* ws_bytes, void* stream);

/* Merge (Section 2, "Multiscale": isotropic kernels are easily merged or divided according
 * to their scale; Section 3, "Optimization"), the inverse of the split: particles with
 * sigma <= sigma_max (finite parameters, sigma > 0, centre inside the width x height image)
 * are grouped by the square cell of edge `cell` holding their centre (floor(mu / cell), in
 * FP64); every group of two or more particles becomes one that keeps the kernels' mass per
 * channel (pi A sigma^2): sigma_m^2 = sum sigma_k^2, mu_m and A_m the sigma_k^2-weighted
 * means; it takes the place of the group's first member, the other particles keep their
 * order. The four children of a split merge back into their parent. Group sums are FP64
 * (their terms may be added in any order: the merged values can differ in their last FP64
 * bits between calls, rounded to FP32 they practically never do); membership and order are
 * exact.
 *   in, out, count  as isogs_field2d_prune (count: outputs, <= in->K)
 *   ws, ws_bytes    workspace (query with ws == NULL, 256-byte aligned): 56 bytes per cell
 *                   of the width x height grid plus the scan's block sums
 * Errors: ISOGS_ERR_INVALID (sizes, cell not finite or <= 0, a grid of more than 2^26 cells,
 * NULL buffers), ISOGS_ERR_WORKSPACE, ISOGS_ERR_DEVICE. */
int isogs_field2d_merge(const isogs_field2d* in, int32_t width, int32_t height, float cell,
                        float sigma_max, const isogs_field2d* out, int32_t* count, void* ws,
                        size_t* ws_bytes, void* stream);

/* ---- Octree initialisation of 3D particles (Section 3, "Initial with Tree Structure") -
 * The 3D counterpart of isogs_field2d_tree_init: an octree over a coloured point cloud (the
 * points a reconstruction starts from), every leaf cell a particle with the mean colour of
 * its points and a scale of half the cell width.
 *   - The domain is a grid of roots[0] x roots[1] x roots[2] cubic root cells of edge
 *     root_side with corner lo; the tree has `levels` levels, level l having cells of edge
 *     root_side / 2^l; a point belongs to the finest cell floor((p - lo) / h) per axis (FP64,
 *     h the finest edge) and is ignored outside the grid.
 *   - Statistics are exact integers: each colour channel clamped to [0, 1] and quantised to
 *     q = rint(65535 c); a cell keeps its point count and the sums of q and q^2 per channel
 *     (coarser cells add their eight children), so they do not depend on the order points
 *     are added in. Its colour variance, in FP64 from those integers,
 *     (1/3) sum_ch (S2/n - (S1/n)^2), is compared with tau * 65535^2.
 *   - A cell with no point never splits and carries no particle; a non-empty cell of a
 *     level below the last splits into its octants when its variance exceeds tau. Levels
 *     grow one at a time; a level whose splits would let the particle count (leaves so far,
 *     the level's non-empty cells that do not split, the non-empty children of those that
 *     do) exceed K splits no cell.
 *   - Leaves are numbered level by level, x fastest, then y, then z; particle: centre = the
 *     cell centre lo + (i + 1/2) edge (FP64, rounded), scale = edge / 2, opacity = `opacity`,
 *     colour = the mean quantised colour / 65535 as coefficient 0 (the scene's higher
 *     coefficients are set to 0).
 *   points, colors  device [3][n_points] each (FP32)
 *   out    host struct of device arrays with capacity out->n >= K (the row stride), any
 *          sh_degree; at most K particles are written
 *   count  device int32: the number of leaves (above K only when the non-empty root cells
 *          alone exceed it; particles past K are not written)
 *   ws, ws_bytes  workspace (query with ws == NULL, 256-byte aligned): 58 bytes per cell of
 *          all levels and the scan's block sums
 * Errors: ISOGS_ERR_INVALID (n_points < 0, levels outside 1..12, a root count < 1,
 * root_side or lo not finite, root_side <= 0, 2^28 cells or more, K < 1, out->n < K, tau
 * not finite or < 0, opacity outside (0, 1), NULL buffers), ISOGS_ERR_WORKSPACE,
 * ISOGS_ERR_DEVICE. */
typedef struct {
    float lo[3];
    float root_side;
    int32_t roots[3];
    int32_t levels;
} isogs_octree_grid;

int isogs_octree_init(const float* points, const float* colors, int32_t n_points,
                      const isogs_octree_grid* grid, float tau, int32_t K, float opacity,
                      const isogs_scene* out, int32_t* count, void* ws, size_t* ws_bytes,
                      void* stream);

/* ---- SSIM term of the loss (Section 3) -----------------------------------------------
 * The paper's loss adds lambda times an SSIM term to the L1 error (lambda = 0.2); read as
 * lambda (1 - SSIM). SSIM is the structural similarity of Wang et al. (2004): per channel,
 * local statistics under an 11 x 11 Gaussian window of standard deviation 1.5 normalised
 * to sum 1, the image counted as zero outside its borders (no renormalisation),
 * C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1),
 *   S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
 * and the reported value is the mean of S over channels and pixels.
 *   image, target  device [channels][height][width] (any number of planes: views and
 *                  colour channels alike)
 *   ssim           device [1]: the mean, written by the forward (block sums added in
 *                  FP64 in a fixed order: reproducible)
 *   ws, ws_bytes   workspace (query with ws == NULL, 256-byte aligned): the three
 *                  derivative maps of S (12 bytes per pixel and channel) and the block
 *                  sums; the backward reads what the forward left there
 * Errors: ISOGS_ERR_INVALID (sizes <= 0, more than 2^31 values or 65535 planes, NULL
 * buffers), ISOGS_ERR_WORKSPACE, ISOGS_ERR_DEVICE. */
int isogs_ssim_fwd(const float* image, const float* target, int32_t channels, int32_t height,
                   int32_t width, float* ssim, void* ws, size_t* ws_bytes, void* stream);

/* dL/dimage = dL/dSSIM * dSSIM/dimage for the same image, target and workspace as the
 * forward (the target is constant); dL_dssim is a device scalar. Output overwritten. */
int isogs_ssim_bwd(const float* image, const float* target, int32_t channels, int32_t height,
                   int32_t width, const float* dL_dssim, const void* ws, size_t ws_bytes,
                   float* dL_dimage, void* stream);

/* The paper's loss (Section 3), (1 - lambda) L1 + lambda (1 - SSIM) with the two terms as
 * defined for isogs_l1_fwd and isogs_ssim_fwd (lambda = 0.2 in the paper; the sign of the
 * SSIM term read so that the loss falls as the images agree).
 *   loss      device [2]: written, {the loss, the mean SSIM}; the L1 mean is added in FP64
 *             from fixed-order block sums, as isogs_l1_fwd does
 *   ws, ws_bytes  workspace (query with ws == NULL, 256-byte aligned): the SSIM workspace
 *             plus the L1 block sums; isogs_loss_bwd reads what the forward left there
 * isogs_loss_bwd writes dL/dimage = dL_dloss ((1 - lambda) sign(image - target) / n -
 * lambda dSSIM/dimage) in one kernel (dL_dloss a device scalar; sign(0) = 0).
 * Errors: as isogs_ssim_fwd / _bwd, and ISOGS_ERR_INVALID for lambda outside [0, 1]. */
int isogs_loss_fwd(const float* image, const float* target, int32_t channels, int32_t height,
                   int32_t width, float lambda, float* loss, void* ws, size_t* ws_bytes, void* stream);
int isogs_loss_bwd(const float* image, const float* target, int32_t channels, int32_t height,
                   int32_t width, float lambda, const float* dL_dloss, const void* ws, size_t ws_bytes,
                   float* dL_dimage, void* stream);

/* The L1 term of the loss (Section 3): loss = mean |image - target| over n values (FP32
 * per element, block sums added in FP64 in a fixed order), and its gradient
 * dL/dimage = dL/dloss * sign(image - target) / n with sign(0) = 0. `loss` and `dL_dloss`
 * are device scalars; ws holds one FP64 partial sum per 4096 values (query with
 * ws == NULL). Errors: ISOGS_ERR_INVALID (n < 0 or >= 2^40, NULL buffers),
 * ISOGS_ERR_WORKSPACE, ISOGS_ERR_DEVICE. */
int isogs_l1_fwd(const float* image, const float* target, int64_t n, float* loss, void* ws,
                 size_t* ws_bytes, void* stream);
int isogs_l1_bwd(const float* image, const float* target, int64_t n, const float* dL_dloss,
                 float* dL_dimage, void* stream);

/* A HIP stream of default priority on the current device with a hardware queue of its own,
 * for callers that run work on several streams at once and need it to overlap on the device:
 * a plain stream takes the least used queue of the process's shared pool when it is
 * created, so that two streams made one after the other can share a queue, which then runs
 * their work in turn. The stream is created with a CU mask that enables every CU, which
 * gives it a queue outside that pool. Like a stream from hipStreamCreate it is ordered with
 * the null stream (work on either waits for earlier work on the other). The stream is the
 * caller's to destroy with isogs_stream_destroy once its work is done. Errors:
 * ISOGS_ERR_INVALID (NULL stream), ISOGS_ERR_DEVICE. */
int isogs_stream_create(void** stream);
int isogs_stream_destroy(void* stream);

/* Message describing the last error returned on the calling thread ("" if none). */
const char* isogs_last_error(void);

/* Library version string. */
const char* isogs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ISOGS_H */
