// Launchers of the device kernels, called by the C ABI layer (abi.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/isogs.h"

namespace isogs {

int launch_project(const isogs_scene* scenes, const isogs_camera* cams, int32_t nv, const isogs_projected* out,
                   hipStream_t stream);

// Workspace layout of isogs_bin_sort for a given capacity and batch.
struct BinSortPlan {
    uint64_t capacity;
    uint32_t n_total;       // packed particles over all views
    uint32_t tiles_total;   // global tiles over all views
    int passes;             // radix passes (digits of at most 9 bits) over the tile id
    int tile_bits;          // bits of the largest global tile id
    uint32_t sort_tiles;    // 4096-entry sort tiles for `capacity`
    uint32_t scan_blocks;   // 2048-particle scan blocks
    uint32_t chunk_h_max;   // segments sorted in chunks by all workgroups, at most
    uint32_t chunk_max;     // their 4096-entry chunks, at most
    size_t off_keys_a, off_keys_b, off_vals_alt, off_z_a, off_z_b, off_hist, off_long_counts,
        off_block_sums, off_long_lists, off_tcount, off_chunk_tables, off_chunk_seg, off_chunk_cnt, bytes;
};

BinSortPlan plan_bin_sort(const int32_t* n_per_view, const isogs_camera* cams, int32_t nv, uint64_t capacity);

int launch_bin_sort(const BinSortPlan& plan, const isogs_projected* proj, const int32_t* n_per_view,
                    const isogs_camera* cams, int32_t nv, const isogs_bins* bins, void* ws, hipStream_t stream);

int launch_render_fwd(const isogs_projected* proj, const int32_t* n_per_view, const isogs_bins* bins,
                      const isogs_camera* cams, int32_t nv, const float* bg, float* image, float* T_final,
                      uint32_t* n_last, float* ckpt, hipStream_t stream);

size_t render_fwd_ordered_ws(const isogs_camera* cams, int32_t nv, uint32_t flags);

// Longest-list-first tile queue of one launch group: words needed, the largest group, the
// launch. The queue holds the length-class histogram (its first kBuckets words, read by
// the compositing kernels), the class cursors, and the order array (returned).
size_t tile_queue_words(uint32_t n_tiles);
uint32_t max_group_tiles(const isogs_camera* cams, int32_t nv);
// The tiles of a launch in longest-list-first order (length classes 0 and 32 - clz(len)).
uint32_t* launch_tile_queue(uint32_t* q, const uint32_t* ranges, uint32_t tile0, uint32_t n_tiles, uint32_t cap,
                            hipStream_t stream);
// Workgroups of `threads` threads of `kernel` resident on the whole GPU at once.
int resident_blocks(const void* kernel, int threads);

// an: the anisotropic family (48-byte entry records instead of 32)
size_t render_bwd_ws(uint64_t capacity, const isogs_camera* cams, int32_t nv, bool an);

// conic: NULL for the isotropic family; the {B, C} array of anisotropic footprints.
int launch_render_fwd_ordered(const isogs_projected* proj, const float* conic, const int32_t* n_per_view,
                              const isogs_bins* bins, const isogs_camera* cams, int32_t nv, const float* bg,
                              float* image, float* T_final, uint32_t* n_last, float* ckpt, uint32_t flags, void* ws,
                              hipStream_t stream);

int launch_render_bwd(const isogs_scene* scenes, const isogs_camera* cams, int32_t nv,
                      const isogs_projected* proj, const isogs_bins* bins, const float* bg,
                      const float* image, const float* dL_dimage, const float* T_final, const uint32_t* n_last,
                      const float* ckpt, const isogs_scene* grads, void* ws, hipStream_t stream);

// The anisotropic family (eq. 5-7): projection to conic footprints, and the backward
// (the forward is launch_render_fwd_ordered with the conic array).
int launch_aniso_project(const isogs_aniso_scene* scenes, const isogs_camera* cams, int32_t nv,
                         const isogs_aniso_projected* out, hipStream_t stream);
int launch_aniso_render_bwd(const isogs_aniso_scene* scenes, const isogs_camera* cams, int32_t nv,
                            const isogs_aniso_projected* proj, const isogs_bins* bins, const float* bg,
                            const float* image, const float* dL_dimage, const float* T_final,
                            const uint32_t* n_last, const float* ckpt, const isogs_aniso_scene* grads, void* ws,
                            hipStream_t stream);

// The 2D kernel-sum representation (no compositing) on the same footprints and bins.
BinSortPlan plan_field2d_bin(int32_t K, int32_t width, int32_t height, uint64_t capacity);
int launch_field2d_bin(const BinSortPlan& plan, const isogs_field2d* f, int32_t width, int32_t height,
                       float support, const isogs_projected* fp, const isogs_bins* bins, void* ws,
                       hipStream_t stream);
int launch_field2d_fwd(const isogs_projected* fp, const isogs_bins* bins, int32_t width, int32_t height,
                       float support, float* image, hipStream_t stream);
size_t field2d_bwd_ws(uint64_t capacity);
int launch_field2d_bwd(const isogs_projected* fp, int32_t K, const isogs_bins* bins, int32_t width, int32_t height,
                       float support, const float* dL_dimage, const isogs_field2d* grads, void* ws,
                       hipStream_t stream);

int launch_field2d_aniso_bin(const BinSortPlan& plan, const isogs_field2d_aniso* f, int32_t width, int32_t height,
                             float support, const isogs_projected* fp, float* conic_c, const isogs_bins* bins,
                             void* ws, hipStream_t stream);
int launch_field2d_aniso_fwd(const isogs_projected* fp, const float* conic_c, const isogs_bins* bins, int32_t width,
                             int32_t height, float support, float* image, hipStream_t stream);
int launch_field2d_aniso_bwd(const isogs_field2d_aniso* f, const isogs_projected* fp, const float* conic_c,
                             const isogs_bins* bins, int32_t width, int32_t height, float support,
                             const float* dL_dimage, const isogs_field2d_aniso* grads, void* ws, hipStream_t stream);

// The SSIM term of the loss: forward (mean SSIM and the derivative maps kept in the
// workspace) and backward.
size_t ssim_ws_bytes(int32_t channels, int32_t height, int32_t width);
int launch_ssim_fwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                    float* ssim, void* ws, hipStream_t stream);
int launch_ssim_bwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                    const float* dL_dssim, const void* ws, float* dL_dimage, hipStream_t stream);

int launch_ssim_bwd_weighted(const float* image, const float* target, int32_t channels, int32_t height,
                             int32_t width, const float* dL_dssim, const void* ws, float ssim_w, float l1_w,
                             float* dL_dimage, hipStream_t stream);
// The paper's combined loss (1 - lambda) L1 + lambda (1 - SSIM): loss[0] the value, loss[1]
// the SSIM mean; the backward is one fused kernel.
size_t loss_ws_bytes(int32_t channels, int32_t height, int32_t width);
int launch_loss_fwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                    float lambda, float* loss, void* ws, hipStream_t stream);
int launch_loss_bwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                    float lambda, const float* dL_dloss, const void* ws, float* dL_dimage, hipStream_t stream);
uint32_t launch_l1_partial(const float* image, const float* target, uint64_t n, double* blocks, hipStream_t stream);

// Quadtree initialisation, prune and split of 2D particles.
int tree_levels_ok(int32_t width, int32_t height, int32_t root, int32_t min_side, uint64_t* root_cells);
size_t tree_init_ws(int32_t width, int32_t height, int32_t root, int32_t min_side);
int launch_tree_init(const float* target, int32_t width, int32_t height, int32_t root, int32_t min_side, float tau,
                     int32_t K, const isogs_field2d* out, int32_t* count, void* ws, hipStream_t stream);
size_t edit_ws(int32_t K);
// mode 0: prune (keep max |A| >= thr), mode 1: split (sigma > thr into four)
int launch_edit(int mode, float thr, const isogs_field2d* in, const isogs_field2d* out, int32_t cap, int32_t* count,
                void* ws, hipStream_t stream);

// Octree initialisation of 3D particles from a coloured point cloud; merge of 2D particles.
int octree_grid_ok(const isogs_octree_grid* g);
size_t octree_init_ws(const isogs_octree_grid* g);
int launch_octree_init(const float* points, const float* colors, int32_t P, const isogs_octree_grid* grid, float tau,
                       int32_t K, float opacity, const isogs_scene* out, int32_t* count, void* ws,
                       hipStream_t stream);
int merge_cells_ok(int32_t width, int32_t height, float cell);
size_t merge_ws(int32_t K, int32_t width, int32_t height, float cell);
int launch_merge(const isogs_field2d* in, int32_t width, int32_t height, float cell, float sigma_max,
                 const isogs_field2d* out, int32_t* count, void* ws, hipStream_t stream);

// The L1 term of the loss: mean |image - target| and its gradient.
size_t l1_ws_bytes(uint64_t n);
int launch_l1_fwd(const float* image, const float* target, uint64_t n, float* loss, void* ws, hipStream_t stream);
int launch_l1_bwd(const float* image, const float* target, uint64_t n, const float* dL_dloss, float* dL_dimage,
                  hipStream_t stream);

}  // namespace isogs
