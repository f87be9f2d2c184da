// C ABI entry points: argument validation, workspace sizing and dispatch.
#include <algorithm>
#include <math.h>
#include <mutex>
#include <stdarg.h>
#include <stdio.h>

#include "kernels.h"

namespace {

thread_local char g_error[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof(g_error), fmt, ap);
    va_end(ap);
    return code;
}

int device_fail(const char* where) {
    const hipError_t e = hipGetLastError();
    return fail(ISOGS_ERR_DEVICE, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

constexpr int32_t kMaxBatchViews = 4096;

int check_cameras(const isogs_camera* cams, int32_t nv) {
    if (!cams) return fail(ISOGS_ERR_INVALID, "cams is NULL");
    for (int v = 0; v < nv; ++v) {
        const isogs_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 32768 || c.height > 32768)
            return fail(ISOGS_ERR_INVALID, "view %d: image size %dx%d outside 1..32768", v, c.width, c.height);
        if (!(c.f > 0.0f) || !isfinite(c.f))
            return fail(ISOGS_ERR_INVALID, "view %d: focal length must be positive and finite", v);
        if (!(c.near_z > 0.0f) || !isfinite(c.near_z))
            return fail(ISOGS_ERR_INVALID, "view %d: near_z must be positive and finite", v);
        bool ok = isfinite(c.cx) && isfinite(c.cy);
        for (int k = 0; k < 9; ++k) ok = ok && isfinite(c.R[k]);
        for (int k = 0; k < 3; ++k) ok = ok && isfinite(c.t[k]) && isfinite(c.eye[k]);
        if (!ok) return fail(ISOGS_ERR_INVALID, "view %d: non-finite camera parameter", v);
    }
    return ISOGS_OK;
}

int check_views(int32_t nv) {
    if (nv <= 0 || nv > kMaxBatchViews) return fail(ISOGS_ERR_INVALID, "n_views = %d outside 1..%d", nv, kMaxBatchViews);
    return ISOGS_OK;
}

int check_totals(const int32_t* n_per_view, const isogs_camera* cams, int32_t nv, uint64_t* n_total,
                 uint64_t* tiles, uint64_t* pixels) {
    uint64_t n = 0, t = 0, p = 0;
    for (int v = 0; v < nv; ++v) {
        if (n_per_view[v] < 0) return fail(ISOGS_ERR_INVALID, "view %d: negative particle count", v);
        n += (uint64_t)n_per_view[v];
        t += (uint64_t)((cams[v].width + 15) / 16) * (uint64_t)((cams[v].height + 15) / 16);
        p += (uint64_t)cams[v].width * (uint64_t)cams[v].height;
    }
    if (n >= (1ull << 31)) return fail(ISOGS_ERR_INVALID, "total particles over all views must be < 2^31");
    if (t >= (1ull << 31)) return fail(ISOGS_ERR_INVALID, "total tiles over all views must be < 2^31");
    if (p >= (1ull << 32)) return fail(ISOGS_ERR_INVALID, "total pixels over all views must be < 2^32");
    if (n_total) *n_total = n;
    if (tiles) *tiles = t;
    if (pixels) *pixels = p;
    return ISOGS_OK;
}

int check_projected(const isogs_projected* p, uint64_t n) {
    if (!p) return fail(ISOGS_ERR_INVALID, "projected is NULL");
    if (n && (!p->record || !p->depth || !p->tile_count)) return fail(ISOGS_ERR_INVALID, "projected buffer is NULL");
    if ((uintptr_t)p->record & 31) return fail(ISOGS_ERR_INVALID, "projected record must be 32-byte aligned");
    return ISOGS_OK;
}

int check_bins(const isogs_bins* b, uint64_t n, uint64_t tiles) {
    if (!b) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    if (!b->count || !b->status) return fail(ISOGS_ERR_INVALID, "bins count/status is NULL");
    if (tiles && !b->ranges) return fail(ISOGS_ERR_INVALID, "bins ranges is NULL");
    if (n && !b->offsets) return fail(ISOGS_ERR_INVALID, "bins offsets is NULL");
    if (b->capacity && !b->pidx) return fail(ISOGS_ERR_INVALID, "bins pidx is NULL");
    if (b->capacity >= (1ull << 30) - 1) return fail(ISOGS_ERR_INVALID, "bins capacity must be < 2^30 - 1");
    return ISOGS_OK;
}

int check_scene(const isogs_scene& s, int v, bool grads) {
    if (s.n < 0) return fail(ISOGS_ERR_INVALID, "%s %d: n < 0", grads ? "grads" : "scene", v);
    if (s.sh_degree < 0 || s.sh_degree > ISOGS_MAX_SH_DEGREE)
        return fail(ISOGS_ERR_INVALID, "%s %d: sh_degree %d outside 0..3", grads ? "grads" : "scene", v, s.sh_degree);
    if (s.n > 0 && (!s.pos || !s.scale || !s.opacity || !s.color))
        return fail(ISOGS_ERR_INVALID, "%s %d: NULL parameter buffer", grads ? "grads" : "scene", v);
    return ISOGS_OK;
}

int check_aniso_scene(const isogs_aniso_scene& s, int v, bool grads) {
    const char* what = grads ? "grads" : "scene";
    if (s.n < 0) return fail(ISOGS_ERR_INVALID, "%s %d: n < 0", what, v);
    if (s.sh_degree < 0 || s.sh_degree > ISOGS_MAX_SH_DEGREE)
        return fail(ISOGS_ERR_INVALID, "%s %d: sh_degree %d outside 0..3", what, v, s.sh_degree);
    if (s.n > 0 && (!s.pos || !s.rot || !s.scale || !s.opacity || !s.color))
        return fail(ISOGS_ERR_INVALID, "%s %d: NULL parameter buffer", what, v);
    return ISOGS_OK;
}

int check_aniso_projected(const isogs_aniso_projected* p, uint64_t n) {
    if (!p) return fail(ISOGS_ERR_INVALID, "projected is NULL");
    int rc = check_projected(&p->fp, n);
    if (rc) return rc;
    if (n && !p->conic) return fail(ISOGS_ERR_INVALID, "projected conic is NULL");
    if ((uintptr_t)p->conic & 7) return fail(ISOGS_ERR_INVALID, "projected conic must be 8-byte aligned");
    return ISOGS_OK;
}

int check_field2d_sizes(int32_t K, int32_t width, int32_t height, float support, uint64_t* tiles) {
    if (K < 0) return fail(ISOGS_ERR_INVALID, "K < 0");
    if (width <= 0 || height <= 0) return fail(ISOGS_ERR_INVALID, "width and height must be positive");
    if (!(support > 0.0f) || !isfinite(support)) return fail(ISOGS_ERR_INVALID, "support must be finite and > 0");
    const uint64_t t = (uint64_t)((width + 15) / 16) * (uint64_t)((height + 15) / 16);
    if (t >= (1ull << 31) || (uint64_t)width * (uint64_t)height >= (1ull << 32))
        return fail(ISOGS_ERR_INVALID, "image too large");
    *tiles = t;
    return ISOGS_OK;
}

}  // namespace

extern "C" {

int isogs_stream_create(void** stream) {
    g_error[0] = 0;
    if (!stream) return fail(ISOGS_ERR_INVALID, "stream is NULL");
    // A stream with a CU mask gets a hardware queue created for it alone; streams without
    // one share the process's pool of queues, where two of them can land on the same queue
    // (the least used one at creation) and then run in turn. The mask enables every CU.
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return device_fail("isogs_stream_create");
    uint32_t mask[32] = {};
    const int words = std::min((cus + 31) / 32, 32);
    for (int c = 0; c < std::min(cus, 32 * 32); ++c) mask[c / 32] |= 1u << (c % 32);
    hipStream_t s = nullptr;
    if (hipExtStreamCreateWithCUMask(&s, (uint32_t)words, mask) != hipSuccess) return device_fail("isogs_stream_create");
    *stream = s;
    return ISOGS_OK;
}

int isogs_stream_destroy(void* stream) {
    g_error[0] = 0;
    if (!stream) return fail(ISOGS_ERR_INVALID, "stream is NULL");
    if (hipStreamDestroy(static_cast<hipStream_t>(stream)) != hipSuccess) return device_fail("isogs_stream_destroy");
    return ISOGS_OK;
}

const char* isogs_last_error(void) { return g_error; }

const char* isogs_version(void) { return "isogs 0.1 gfx950"; }

int isogs_project(const isogs_scene* scenes, const isogs_camera* cams, int32_t n_views, const isogs_projected* out,
                  void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!scenes) return fail(ISOGS_ERR_INVALID, "scenes is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    int32_t npv[kMaxBatchViews];
    for (int v = 0; v < n_views; ++v) {
        if ((rc = check_scene(scenes[v], v, false))) return rc;
        npv[v] = scenes[v].n;
    }
    uint64_t n;
    if ((rc = check_totals(npv, cams, n_views, &n, nullptr, nullptr))) return rc;
    if ((rc = check_projected(out, n))) return rc;
    if (isogs::launch_project(scenes, cams, n_views, out, (hipStream_t)stream)) return device_fail("isogs_project");
    return ISOGS_OK;
}

int isogs_bin_sort(const isogs_projected* proj, const int32_t* n_per_view, const isogs_camera* cams, int32_t n_views,
                   const isogs_bins* bins, void* ws, size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!n_per_view) return fail(ISOGS_ERR_INVALID, "n_per_view is NULL");
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    uint64_t n, tiles;
    if ((rc = check_totals(n_per_view, cams, n_views, &n, &tiles, nullptr))) return rc;
    if (!bins) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    const isogs::BinSortPlan plan = isogs::plan_bin_sort(n_per_view, cams, n_views, bins->capacity);
    if (!ws) {
        *ws_bytes = plan.bytes;
        return ISOGS_OK;
    }
    if (*ws_bytes < plan.bytes)
        return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, plan.bytes);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if ((rc = check_projected(proj, n))) return rc;
    if ((rc = check_bins(bins, n, tiles))) return rc;
    if (isogs::launch_bin_sort(plan, proj, n_per_view, cams, n_views, bins, ws, (hipStream_t)stream))
        return device_fail("isogs_bin_sort");
    return ISOGS_OK;
}

size_t isogs_checkpoint_bytes(uint64_t capacity) {
    return (size_t)(capacity / ISOGS_CKPT_CHUNK + 1) * 256 * 4 * sizeof(float);
}

int isogs_render_fwd(const isogs_projected* proj, const int32_t* n_per_view, const isogs_bins* bins,
                     const isogs_camera* cams, int32_t n_views, const float* bg, float* image, float* T_final,
                     uint32_t* n_last, float* checkpoints, void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!n_per_view) return fail(ISOGS_ERR_INVALID, "n_per_view is NULL");
    if (!bg) return fail(ISOGS_ERR_INVALID, "bg is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    uint64_t n, tiles;
    if ((rc = check_totals(n_per_view, cams, n_views, &n, &tiles, nullptr))) return rc;
    if ((rc = check_projected(proj, n))) return rc;
    if ((rc = check_bins(bins, n, tiles))) return rc;
    if (!image || !T_final) return fail(ISOGS_ERR_INVALID, "output buffer is NULL");
    if (isogs::launch_render_fwd(proj, n_per_view, bins, cams, n_views, bg, image, T_final, n_last, checkpoints,
                                 (hipStream_t)stream))
        return device_fail("isogs_render_fwd");
    return ISOGS_OK;
}

int isogs_render_fwd_ordered(const isogs_projected* proj, const int32_t* n_per_view, const isogs_bins* bins,
                             const isogs_camera* cams, int32_t n_views, const float* bg, float* image,
                             float* T_final, uint32_t* n_last, float* checkpoints, uint32_t flags, void* ws,
                             size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!n_per_view) return fail(ISOGS_ERR_INVALID, "n_per_view is NULL");
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    if (flags & ~(ISOGS_FWD_WIDE | ISOGS_FWD_TIMES)) return fail(ISOGS_ERR_INVALID, "unknown flags %u", flags);
    const size_t need = isogs::render_fwd_ordered_ws(cams, n_views, flags);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!bg) return fail(ISOGS_ERR_INVALID, "bg is NULL");
    uint64_t n, tiles;
    if ((rc = check_totals(n_per_view, cams, n_views, &n, &tiles, nullptr))) return rc;
    if ((rc = check_projected(proj, n))) return rc;
    if ((rc = check_bins(bins, n, tiles))) return rc;
    if (!image || !T_final) return fail(ISOGS_ERR_INVALID, "output buffer is NULL");
    if (isogs::launch_render_fwd_ordered(proj, nullptr, n_per_view, bins, cams, n_views, bg, image, T_final, n_last,
                                         checkpoints, flags, ws, (hipStream_t)stream))
        return device_fail("isogs_render_fwd_ordered");
    return ISOGS_OK;
}

int isogs_render_bwd(const isogs_scene* scenes, const isogs_camera* cams, int32_t n_views,
                     const isogs_projected* proj, const isogs_bins* bins, const float* bg, const float* image,
                     const float* dL_dimage, const float* T_final, const uint32_t* n_last, const float* checkpoints,
                     const isogs_scene* grads, void* ws, size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!scenes || !grads) return fail(ISOGS_ERR_INVALID, "scenes or grads is NULL");
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!bins) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    const size_t need = isogs::render_bwd_ws(bins->capacity, cams, n_views, false);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    int32_t npv[kMaxBatchViews];
    for (int v = 0; v < n_views; ++v) {
        if ((rc = check_scene(scenes[v], v, false))) return rc;
        if ((rc = check_scene(grads[v], v, true))) return rc;
        if (grads[v].n != scenes[v].n || grads[v].sh_degree != scenes[v].sh_degree)
            return fail(ISOGS_ERR_INVALID, "view %d: grads must match the scene's n and sh_degree", v);
        npv[v] = scenes[v].n;
    }
    for (int v = 0; v < n_views; ++v)
        for (int u = 0; u < v; ++u)
            if (scenes[u].pos == scenes[v].pos &&
                (grads[u].pos != grads[v].pos || scenes[u].n != scenes[v].n ||
                 scenes[u].sh_degree != scenes[v].sh_degree || scenes[u].color != scenes[v].color))
                return fail(ISOGS_ERR_INVALID, "views %d and %d share a scene but not its grads buffers", u, v);
    uint64_t n, tiles;
    if ((rc = check_totals(npv, cams, n_views, &n, &tiles, nullptr))) return rc;
    if ((rc = check_projected(proj, n))) return rc;
    if ((rc = check_bins(bins, n, tiles))) return rc;
    if (!bg || !dL_dimage || !T_final || !n_last) return fail(ISOGS_ERR_INVALID, "input buffer is NULL");
    if (checkpoints && !image) return fail(ISOGS_ERR_INVALID, "checkpoints given without the image");
    if (isogs::launch_render_bwd(scenes, cams, n_views, proj, bins, bg, image, dL_dimage, T_final, n_last,
                                 checkpoints, grads, ws, (hipStream_t)stream))
        return device_fail("isogs_render_bwd");
    return ISOGS_OK;
}

int isogs_aniso_project(const isogs_aniso_scene* scenes, const isogs_camera* cams, int32_t n_views,
                        const isogs_aniso_projected* out, void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!scenes) return fail(ISOGS_ERR_INVALID, "scenes is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    int32_t npv[kMaxBatchViews];
    for (int v = 0; v < n_views; ++v) {
        if ((rc = check_aniso_scene(scenes[v], v, false))) return rc;
        npv[v] = scenes[v].n;
    }
    uint64_t n;
    if ((rc = check_totals(npv, cams, n_views, &n, nullptr, nullptr))) return rc;
    if ((rc = check_aniso_projected(out, n))) return rc;
    if (isogs::launch_aniso_project(scenes, cams, n_views, out, (hipStream_t)stream))
        return device_fail("isogs_aniso_project");
    return ISOGS_OK;
}

int isogs_aniso_render_fwd(const isogs_aniso_projected* proj, const int32_t* n_per_view, const isogs_bins* bins,
                           const isogs_camera* cams, int32_t n_views, const float* bg, float* image, float* T_final,
                           uint32_t* n_last, float* checkpoints, uint32_t flags, void* ws, size_t* ws_bytes,
                           void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!n_per_view) return fail(ISOGS_ERR_INVALID, "n_per_view is NULL");
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    if (flags & ~(ISOGS_FWD_WIDE | ISOGS_FWD_TIMES)) return fail(ISOGS_ERR_INVALID, "unknown flags %u", flags);
    const size_t need = isogs::render_fwd_ordered_ws(cams, n_views, flags);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!bg) return fail(ISOGS_ERR_INVALID, "bg is NULL");
    uint64_t n, tiles;
    if ((rc = check_totals(n_per_view, cams, n_views, &n, &tiles, nullptr))) return rc;
    if ((rc = check_aniso_projected(proj, n))) return rc;
    if ((rc = check_bins(bins, n, tiles))) return rc;
    if (!image || !T_final) return fail(ISOGS_ERR_INVALID, "output buffer is NULL");
    // a NULL conic selects the isotropic walk: give the anisotropic one a valid address
    // even when there is no particle
    static float no_conic[2];
    const float* conic = proj->conic ? proj->conic : no_conic;
    if (isogs::launch_render_fwd_ordered(&proj->fp, conic, n_per_view, bins, cams, n_views, bg, image, T_final,
                                         n_last, checkpoints, flags, ws, (hipStream_t)stream))
        return device_fail("isogs_aniso_render_fwd");
    return ISOGS_OK;
}

int isogs_aniso_render_bwd(const isogs_aniso_scene* scenes, const isogs_camera* cams, int32_t n_views,
                           const isogs_aniso_projected* proj, const isogs_bins* bins, const float* bg,
                           const float* image, const float* dL_dimage, const float* T_final, const uint32_t* n_last,
                           const float* checkpoints, const isogs_aniso_scene* grads, void* ws, size_t* ws_bytes,
                           void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!scenes || !grads) return fail(ISOGS_ERR_INVALID, "scenes or grads is NULL");
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!bins) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    const size_t need = isogs::render_bwd_ws(bins->capacity, cams, n_views, true);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    int32_t npv[kMaxBatchViews];
    for (int v = 0; v < n_views; ++v) {
        if ((rc = check_aniso_scene(scenes[v], v, false))) return rc;
        if ((rc = check_aniso_scene(grads[v], v, true))) return rc;
        if (grads[v].n != scenes[v].n || grads[v].sh_degree != scenes[v].sh_degree)
            return fail(ISOGS_ERR_INVALID, "view %d: grads must match the scene's n and sh_degree", v);
        npv[v] = scenes[v].n;
    }
    for (int v = 0; v < n_views; ++v)
        for (int u = 0; u < v; ++u)
            if (scenes[u].pos == scenes[v].pos &&
                (grads[u].pos != grads[v].pos || scenes[u].n != scenes[v].n || scenes[u].rot != scenes[v].rot ||
                 scenes[u].scale != scenes[v].scale || scenes[u].sh_degree != scenes[v].sh_degree ||
                 scenes[u].color != scenes[v].color))
                return fail(ISOGS_ERR_INVALID, "views %d and %d share a scene but not its grads buffers", u, v);
    uint64_t n, tiles;
    if ((rc = check_totals(npv, cams, n_views, &n, &tiles, nullptr))) return rc;
    if ((rc = check_aniso_projected(proj, n))) return rc;
    if ((rc = check_bins(bins, n, tiles))) return rc;
    if (!bg || !dL_dimage || !T_final || !n_last) return fail(ISOGS_ERR_INVALID, "input buffer is NULL");
    if (checkpoints && !image) return fail(ISOGS_ERR_INVALID, "checkpoints given without the image");
    if (isogs::launch_aniso_render_bwd(scenes, cams, n_views, proj, bins, bg, image, dL_dimage, T_final, n_last,
                                       checkpoints, grads, ws, (hipStream_t)stream))
        return device_fail("isogs_aniso_render_bwd");
    return ISOGS_OK;
}

int isogs_field2d_bin(const isogs_field2d* field, int32_t width, int32_t height, float support,
                      const isogs_projected* fp, const isogs_bins* bins, void* ws, size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    int rc;
    if (!field) return fail(ISOGS_ERR_INVALID, "field is NULL");
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!bins) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    uint64_t tiles;
    if ((rc = check_field2d_sizes(field->K, width, height, support, &tiles))) return rc;
    const isogs::BinSortPlan plan = isogs::plan_field2d_bin(field->K, width, height, bins->capacity);
    if (!ws) {
        *ws_bytes = plan.bytes;
        return ISOGS_OK;
    }
    if (*ws_bytes < plan.bytes)
        return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, plan.bytes);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (field->K > 0 && (!field->mu || !field->sigma || !field->amp))
        return fail(ISOGS_ERR_INVALID, "field parameter buffer is NULL");
    if ((rc = check_projected(fp, (uint64_t)field->K))) return rc;
    if ((rc = check_bins(bins, (uint64_t)field->K, tiles))) return rc;
    if (isogs::launch_field2d_bin(plan, field, width, height, support, fp, bins, ws, (hipStream_t)stream))
        return device_fail("isogs_field2d_bin");
    return ISOGS_OK;
}

int isogs_field2d_fwd(const isogs_projected* fp, int32_t K, const isogs_bins* bins, int32_t width, int32_t height,
                      float support, float* image, void* stream) {
    g_error[0] = 0;
    int rc;
    uint64_t tiles;
    if ((rc = check_field2d_sizes(K, width, height, support, &tiles))) return rc;
    if ((rc = check_projected(fp, (uint64_t)K))) return rc;
    if ((rc = check_bins(bins, (uint64_t)K, tiles))) return rc;
    if (!image) return fail(ISOGS_ERR_INVALID, "image is NULL");
    if (isogs::launch_field2d_fwd(fp, bins, width, height, support, image, (hipStream_t)stream))
        return device_fail("isogs_field2d_fwd");
    return ISOGS_OK;
}

int isogs_field2d_bwd(const isogs_projected* fp, int32_t K, const isogs_bins* bins, int32_t width, int32_t height,
                      float support, const float* dL_dimage, const isogs_field2d* grads, void* ws, size_t* ws_bytes,
                      void* stream) {
    g_error[0] = 0;
    int rc;
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!bins) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    uint64_t tiles;
    if ((rc = check_field2d_sizes(K, width, height, support, &tiles))) return rc;
    const size_t need = isogs::field2d_bwd_ws(bins->capacity);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if ((rc = check_projected(fp, (uint64_t)K))) return rc;
    if ((rc = check_bins(bins, (uint64_t)K, tiles))) return rc;
    if (!dL_dimage) return fail(ISOGS_ERR_INVALID, "dL_dimage is NULL");
    if (!grads || grads->K != K) return fail(ISOGS_ERR_INVALID, "grads must describe K particles");
    if (K > 0 && (!grads->mu || !grads->sigma || !grads->amp))
        return fail(ISOGS_ERR_INVALID, "grads buffer is NULL");
    if (isogs::launch_field2d_bwd(fp, K, bins, width, height, support, dL_dimage, grads, ws, (hipStream_t)stream))
        return device_fail("isogs_field2d_bwd");
    return ISOGS_OK;
}

int isogs_ssim_fwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                   float* ssim, void* ws, size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (channels <= 0 || height <= 0 || width <= 0) return fail(ISOGS_ERR_INVALID, "sizes must be positive");
    if ((uint64_t)channels * (uint64_t)height * (uint64_t)width >= (1ull << 31) || channels > 65535)
        return fail(ISOGS_ERR_INVALID, "image too large");
    const size_t need = isogs::ssim_ws_bytes(channels, height, width);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!image || !target || !ssim) return fail(ISOGS_ERR_INVALID, "buffer is NULL");
    if (isogs::launch_ssim_fwd(image, target, channels, height, width, ssim, ws, (hipStream_t)stream))
        return device_fail("isogs_ssim_fwd");
    return ISOGS_OK;
}

int isogs_ssim_bwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                   const float* dL_dssim, const void* ws, size_t ws_bytes, float* dL_dimage, void* stream) {
    g_error[0] = 0;
    if (channels <= 0 || height <= 0 || width <= 0) return fail(ISOGS_ERR_INVALID, "sizes must be positive");
    if ((uint64_t)channels * (uint64_t)height * (uint64_t)width >= (1ull << 31) || channels > 65535)
        return fail(ISOGS_ERR_INVALID, "image too large");
    const size_t need = isogs::ssim_ws_bytes(channels, height, width);
    if (!ws || ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "the forward's workspace of %zu bytes is needed", need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!image || !target || !dL_dssim || !dL_dimage) return fail(ISOGS_ERR_INVALID, "buffer is NULL");
    if (isogs::launch_ssim_bwd(image, target, channels, height, width, dL_dssim, ws, dL_dimage, (hipStream_t)stream))
        return device_fail("isogs_ssim_bwd");
    return ISOGS_OK;
}

int isogs_field2d_aniso_bin(const isogs_field2d_aniso* field, int32_t width, int32_t height, float support,
                            const isogs_projected* fp, float* conic_c, const isogs_bins* bins, void* ws,
                            size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    int rc;
    if (!field) return fail(ISOGS_ERR_INVALID, "field is NULL");
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!bins) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    uint64_t tiles;
    if ((rc = check_field2d_sizes(field->K, width, height, support, &tiles))) return rc;
    const isogs::BinSortPlan plan = isogs::plan_field2d_bin(field->K, width, height, bins->capacity);
    if (!ws) {
        *ws_bytes = plan.bytes;
        return ISOGS_OK;
    }
    if (*ws_bytes < plan.bytes)
        return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, plan.bytes);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (field->K > 0 && (!field->mu || !field->theta || !field->scale || !field->amp || !conic_c))
        return fail(ISOGS_ERR_INVALID, "field parameter buffer or conic_c is NULL");
    if ((rc = check_projected(fp, (uint64_t)field->K))) return rc;
    if ((rc = check_bins(bins, (uint64_t)field->K, tiles))) return rc;
    if (isogs::launch_field2d_aniso_bin(plan, field, width, height, support, fp, conic_c, bins, ws,
                                        (hipStream_t)stream))
        return device_fail("isogs_field2d_aniso_bin");
    return ISOGS_OK;
}

int isogs_field2d_aniso_fwd(const isogs_projected* fp, const float* conic_c, int32_t K, const isogs_bins* bins,
                            int32_t width, int32_t height, float support, float* image, void* stream) {
    g_error[0] = 0;
    int rc;
    uint64_t tiles;
    if ((rc = check_field2d_sizes(K, width, height, support, &tiles))) return rc;
    if ((rc = check_projected(fp, (uint64_t)K))) return rc;
    if ((rc = check_bins(bins, (uint64_t)K, tiles))) return rc;
    if (!image || (K > 0 && !conic_c)) return fail(ISOGS_ERR_INVALID, "image or conic_c is NULL");
    if (isogs::launch_field2d_aniso_fwd(fp, conic_c, bins, width, height, support, image, (hipStream_t)stream))
        return device_fail("isogs_field2d_aniso_fwd");
    return ISOGS_OK;
}

int isogs_field2d_aniso_bwd(const isogs_field2d_aniso* field, const isogs_projected* fp, const float* conic_c,
                            const isogs_bins* bins, int32_t width, int32_t height, float support,
                            const float* dL_dimage, const isogs_field2d_aniso* grads, void* ws, size_t* ws_bytes,
                            void* stream) {
    g_error[0] = 0;
    int rc;
    if (!field || !grads) return fail(ISOGS_ERR_INVALID, "field or grads is NULL");
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!bins) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    uint64_t tiles;
    if ((rc = check_field2d_sizes(field->K, width, height, support, &tiles))) return rc;
    const size_t need = isogs::field2d_bwd_ws(bins->capacity);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if ((rc = check_projected(fp, (uint64_t)field->K))) return rc;
    if ((rc = check_bins(bins, (uint64_t)field->K, tiles))) return rc;
    if (!dL_dimage) return fail(ISOGS_ERR_INVALID, "dL_dimage is NULL");
    if (grads->K != field->K) return fail(ISOGS_ERR_INVALID, "grads must describe K particles");
    if (field->K > 0 && (!field->theta || !field->scale || !conic_c || !grads->mu || !grads->theta ||
                         !grads->scale || !grads->amp))
        return fail(ISOGS_ERR_INVALID, "buffer is NULL");
    if (isogs::launch_field2d_aniso_bwd(field, fp, conic_c, bins, width, height, support, dL_dimage, grads, ws,
                                        (hipStream_t)stream))
        return device_fail("isogs_field2d_aniso_bwd");
    return ISOGS_OK;
}

int isogs_field2d_merge(const isogs_field2d* in, int32_t width, int32_t height, float cell, float sigma_max,
                        const isogs_field2d* out, int32_t* count, void* ws, size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!in || !out) return fail(ISOGS_ERR_INVALID, "in or out is NULL");
    if (in->K < 0 || out->K < 0) return fail(ISOGS_ERR_INVALID, "K < 0");
    if (width <= 0 || height <= 0) return fail(ISOGS_ERR_INVALID, "width and height must be positive");
    if (!(cell > 0.0f) || !isfinite(cell)) return fail(ISOGS_ERR_INVALID, "cell must be finite and > 0");
    if (!isogs::merge_cells_ok(width, height, cell)) return fail(ISOGS_ERR_INVALID, "the cell grid is too large");
    const size_t need = isogs::merge_ws(in->K, width, height, cell);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!count) return fail(ISOGS_ERR_INVALID, "count is NULL");
    if (in->K > 0 && (!in->mu || !in->sigma || !in->amp)) return fail(ISOGS_ERR_INVALID, "input buffer is NULL");
    if (out->K > 0 && (!out->mu || !out->sigma || !out->amp)) return fail(ISOGS_ERR_INVALID, "output buffer is NULL");
    if (isogs::launch_merge(in, width, height, cell, sigma_max, out, count, ws, (hipStream_t)stream))
        return device_fail("isogs_field2d_merge");
    return ISOGS_OK;
}

int isogs_octree_init(const float* points, const float* colors, int32_t n_points, const isogs_octree_grid* grid,
                      float tau, int32_t K, float opacity, const isogs_scene* out, int32_t* count, void* ws,
                      size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!grid) return fail(ISOGS_ERR_INVALID, "grid is NULL");
    if (!isogs::octree_grid_ok(grid))
        return fail(ISOGS_ERR_INVALID, "octree grid: levels 1..12, roots >= 1, finite lo, root_side > 0, < 2^28 cells");
    const size_t need = isogs::octree_init_ws(grid);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (n_points < 0) return fail(ISOGS_ERR_INVALID, "n_points < 0");
    if (n_points > 0 && (!points || !colors)) return fail(ISOGS_ERR_INVALID, "points or colors is NULL");
    if (!(tau >= 0.0f) || !isfinite(tau)) return fail(ISOGS_ERR_INVALID, "tau must be finite and >= 0");
    if (!(opacity > 0.0f && opacity < 1.0f)) return fail(ISOGS_ERR_INVALID, "opacity must be in (0, 1)");
    if (K < 1) return fail(ISOGS_ERR_INVALID, "K must be >= 1");
    if (!out || out->n < K) return fail(ISOGS_ERR_INVALID, "out must hold K particles");
    if (out->sh_degree < 0 || out->sh_degree > ISOGS_MAX_SH_DEGREE)
        return fail(ISOGS_ERR_INVALID, "out sh_degree outside 0..3");
    if (!out->pos || !out->scale || !out->opacity || !out->color || !count)
        return fail(ISOGS_ERR_INVALID, "output buffer is NULL");
    if (isogs::launch_octree_init(points, colors, n_points, grid, tau, K, opacity, out, count, ws, (hipStream_t)stream))
        return device_fail("isogs_octree_init");
    return ISOGS_OK;
}

int isogs_loss_fwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                   float lambda, float* loss, void* ws, size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (channels <= 0 || height <= 0 || width <= 0) return fail(ISOGS_ERR_INVALID, "sizes must be positive");
    if ((uint64_t)channels * (uint64_t)height * (uint64_t)width >= (1ull << 31) || channels > 65535)
        return fail(ISOGS_ERR_INVALID, "image too large");
    if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(ISOGS_ERR_INVALID, "lambda must be in [0, 1]");
    const size_t need = isogs::loss_ws_bytes(channels, height, width);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!image || !target || !loss) return fail(ISOGS_ERR_INVALID, "buffer is NULL");
    if (isogs::launch_loss_fwd(image, target, channels, height, width, lambda, loss, ws, (hipStream_t)stream))
        return device_fail("isogs_loss_fwd");
    return ISOGS_OK;
}

int isogs_loss_bwd(const float* image, const float* target, int32_t channels, int32_t height, int32_t width,
                   float lambda, const float* dL_dloss, const void* ws, size_t ws_bytes, float* dL_dimage,
                   void* stream) {
    g_error[0] = 0;
    if (channels <= 0 || height <= 0 || width <= 0) return fail(ISOGS_ERR_INVALID, "sizes must be positive");
    if ((uint64_t)channels * (uint64_t)height * (uint64_t)width >= (1ull << 31) || channels > 65535)
        return fail(ISOGS_ERR_INVALID, "image too large");
    if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(ISOGS_ERR_INVALID, "lambda must be in [0, 1]");
    const size_t need = isogs::loss_ws_bytes(channels, height, width);
    if (!ws || ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "the forward's workspace of %zu bytes is needed", need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!image || !target || !dL_dloss || !dL_dimage) return fail(ISOGS_ERR_INVALID, "buffer is NULL");
    if (isogs::launch_loss_bwd(image, target, channels, height, width, lambda, dL_dloss, ws, dL_dimage,
                               (hipStream_t)stream))
        return device_fail("isogs_loss_bwd");
    return ISOGS_OK;
}

int isogs_field2d_tree_init(const float* target, int32_t height, int32_t width, int32_t root, int32_t min_side,
                            float tau, int32_t K, const isogs_field2d* out, int32_t* count, void* ws, size_t* ws_bytes,
                            void* stream) {
    g_error[0] = 0;
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (height <= 0 || width <= 0) return fail(ISOGS_ERR_INVALID, "width and height must be positive");
    if ((uint64_t)width * (uint64_t)height * 3 >= (1ull << 31)) return fail(ISOGS_ERR_INVALID, "image too large");
    uint64_t roots = 0;
    if (!isogs::tree_levels_ok(width, height, root, min_side, &roots))
        return fail(ISOGS_ERR_INVALID, "root must be a power of two >= min_side >= 1");
    if (!(tau >= 0.0f) || !isfinite(tau)) return fail(ISOGS_ERR_INVALID, "tau must be finite and >= 0");
    if (K <= 0 || (uint64_t)K < roots) return fail(ISOGS_ERR_INVALID, "K must allow one particle per root cell");
    const size_t need = isogs::tree_init_ws(width, height, root, min_side);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!target || !out || !count || !out->mu || !out->sigma || !out->amp)
        return fail(ISOGS_ERR_INVALID, "buffer is NULL");
    if (out->K < K) return fail(ISOGS_ERR_INVALID, "out must hold K particles");
    isogs_field2d o = *out;
    o.K = K;
    if (isogs::launch_tree_init(target, width, height, root, min_side, tau, K, &o, count, ws, (hipStream_t)stream))
        return device_fail("isogs_field2d_tree_init");
    return ISOGS_OK;
}

static int field2d_edit(int mode, const char* name, const isogs_field2d* in, float thr, const isogs_field2d* out,
                        int32_t* count, void* ws, size_t* ws_bytes, void* stream) {
    g_error[0] = 0;
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (!in || in->K < 0) return fail(ISOGS_ERR_INVALID, "in must describe K >= 0 particles");
    if (isnan(thr)) return fail(ISOGS_ERR_INVALID, "threshold is NaN");
    const size_t need = isogs::edit_ws(in->K);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!out || !count || out->K < 0) return fail(ISOGS_ERR_INVALID, "out or count is NULL");
    if (in->K > 0 && (!in->mu || !in->sigma || !in->amp)) return fail(ISOGS_ERR_INVALID, "in buffer is NULL");
    if (out->K > 0 && (!out->mu || !out->sigma || !out->amp)) return fail(ISOGS_ERR_INVALID, "out buffer is NULL");
    if (isogs::launch_edit(mode, thr, in, out, out->K, count, ws, (hipStream_t)stream)) return device_fail(name);
    return ISOGS_OK;
}

int isogs_field2d_prune(const isogs_field2d* in, float amp_min, const isogs_field2d* out, int32_t* count, void* ws,
                        size_t* ws_bytes, void* stream) {
    return field2d_edit(0, "isogs_field2d_prune", in, amp_min, out, count, ws, ws_bytes, stream);
}

int isogs_field2d_split(const isogs_field2d* in, float sigma_max, const isogs_field2d* out, int32_t* count, void* ws,
                        size_t* ws_bytes, void* stream) {
    return field2d_edit(1, "isogs_field2d_split", in, sigma_max, out, count, ws, ws_bytes, stream);
}

int isogs_l1_fwd(const float* image, const float* target, int64_t n, float* loss, void* ws, size_t* ws_bytes,
                 void* stream) {
    g_error[0] = 0;
    if (!ws_bytes) return fail(ISOGS_ERR_INVALID, "ws_bytes is NULL");
    if (n < 0 || (uint64_t)n >= (1ull << 40)) return fail(ISOGS_ERR_INVALID, "n must be in [0, 2^40)");
    const size_t need = isogs::l1_ws_bytes((uint64_t)n);
    if (!ws) {
        *ws_bytes = need;
        return ISOGS_OK;
    }
    if (*ws_bytes < need) return fail(ISOGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(ISOGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (!loss || (n > 0 && (!image || !target))) return fail(ISOGS_ERR_INVALID, "buffer is NULL");
    if (isogs::launch_l1_fwd(image, target, (uint64_t)n, loss, ws, (hipStream_t)stream)) return device_fail("isogs_l1_fwd");
    return ISOGS_OK;
}

int isogs_l1_bwd(const float* image, const float* target, int64_t n, const float* dL_dloss, float* dL_dimage,
                 void* stream) {
    g_error[0] = 0;
    if (n < 0 || (uint64_t)n >= (1ull << 40)) return fail(ISOGS_ERR_INVALID, "n must be in [0, 2^40)");
    if (!dL_dloss || (n > 0 && (!image || !target || !dL_dimage))) return fail(ISOGS_ERR_INVALID, "buffer is NULL");
    if (isogs::launch_l1_bwd(image, target, (uint64_t)n, dL_dloss, dL_dimage, (hipStream_t)stream))
        return device_fail("isogs_l1_bwd");
    return ISOGS_OK;
}

}  // extern "C"

// ---- Bin sort without a caller workspace ---------------------------------------------------
// The scratch of isogs_bin_sort_static lives in a file-scope device array, one copy per GPU,
// held until the process ends. Host code never passes the array's name to a kernel (on the
// host it only stands in for the symbol): its device address is looked up once per device
// with hipGetSymbolAddress and cached.
namespace {

constexpr size_t kStaticScratchBytes = (size_t)ISOGS_STATIC_SCRATCH_BYTES;
static_assert(kStaticScratchBytes % 256 == 0, "the scratch holds 256-byte aligned sections");

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch (the current device's), or NULL with the error set.
void* device_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        fail(ISOGS_ERR_DEVICE, "isogs_bin_sort_static: no current device (or device index >= %d)", kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(ISOGS_ERR_DEVICE, "isogs_bin_sort_static: hipGetSymbolAddress failed on device %d: %s", dev,
                 hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int isogs_bin_sort_static(const isogs_projected* proj, const int32_t* n_per_view, const isogs_camera* cams,
                          int32_t n_views, const isogs_bins* bins, void* stream) {
    g_error[0] = 0;
    int rc;
    if ((rc = check_views(n_views))) return rc;
    if (!n_per_view) return fail(ISOGS_ERR_INVALID, "n_per_view is NULL");
    if ((rc = check_cameras(cams, n_views))) return rc;
    uint64_t n, tiles;
    if ((rc = check_totals(n_per_view, cams, n_views, &n, &tiles, nullptr))) return rc;
    if (!bins) return fail(ISOGS_ERR_INVALID, "bins is NULL");
    const isogs::BinSortPlan plan = isogs::plan_bin_sort(n_per_view, cams, n_views, bins->capacity);
    if (plan.bytes > kStaticScratchBytes)
        return fail(ISOGS_ERR_WORKSPACE,
                    "isogs_bin_sort_static: %zu bytes of scratch needed for capacity %llu and %llu tiles, "
                    "the static scratch holds %zu",
                    plan.bytes, (unsigned long long)bins->capacity, (unsigned long long)tiles, kStaticScratchBytes);
    if ((rc = check_projected(proj, n))) return rc;
    if ((rc = check_bins(bins, n, tiles))) return rc;
    void* ws = device_scratch();
    if (!ws) return ISOGS_ERR_DEVICE;
    if (isogs::launch_bin_sort(plan, proj, n_per_view, cams, n_views, bins, ws, (hipStream_t)stream))
        return device_fail("isogs_bin_sort_static");
    return ISOGS_OK;
}

}  // extern "C"
