// Projection of isotropic particles to circular screen footprints (+ colour, tile count).
#include "common.h"
#include "kernels.h"

namespace isogs {

// Real orthonormal spherical harmonics up to degree 3 in Cartesian form (unit direction
// x, y, z), without the Condon-Shortley phase: Y_{1,-1}, Y_{1,0}, Y_{1,1} are positive
// multiples of y, z, x. Index k = l^2 + l + m. The degree-0 term is not used: the base
// colour c_0 enters with weight 1.
struct SHConst {
    static constexpr float c1 = 0.48860251190291992f;    // sqrt(3 / 4pi)
    static constexpr float c2a = 1.09254843059207907f;   // sqrt(15 / 4pi)
    static constexpr float c2b = 0.31539156525252005f;   // sqrt(5 / 16pi)
    static constexpr float c2c = 0.54627421529603959f;   // sqrt(15 / 16pi)
    static constexpr float c3a = 0.59004358992664352f;   // sqrt(35 / 32pi)
    static constexpr float c3b = 2.89061144264055405f;   // sqrt(105 / 4pi)
    static constexpr float c3c = 0.45704579946446573f;   // sqrt(21 / 32pi)
    static constexpr float c3d = 0.37317633259011540f;   // sqrt(7 / 16pi)
    static constexpr float c3e = 1.44530572132027702f;   // sqrt(105 / 16pi)
};

__device__ __forceinline__ void sh_eval(int deg, float x, float y, float z, float Y[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) Y[k] = 0.0f;
    Y[0] = 1.0f;
    if (deg < 1) return;
    Y[1] = SHConst::c1 * y;
    Y[2] = SHConst::c1 * z;
    Y[3] = SHConst::c1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SHConst::c2a * x * y;
    Y[5] = SHConst::c2a * y * z;
    Y[6] = SHConst::c2b * (3.0f * zz - 1.0f);
    Y[7] = SHConst::c2a * x * z;
    Y[8] = SHConst::c2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = SHConst::c3a * y * (3.0f * xx - yy);
    Y[10] = SHConst::c3b * x * y * z;
    Y[11] = SHConst::c3c * y * (5.0f * zz - 1.0f);
    Y[12] = SHConst::c3d * z * (5.0f * zz - 3.0f);
    Y[13] = SHConst::c3c * x * (5.0f * zz - 1.0f);
    Y[14] = SHConst::c3e * z * (xx - yy);
    Y[15] = SHConst::c3a * x * (xx - 3.0f * yy);
}

struct ProjViewArgs {
    const float* pos;
    const float* scale;
    const float* opacity;
    const float* color;
    uint32_t n;
    int32_t sh_degree;
    uint32_t p_off;
    int32_t width, height;
    float R[9], t[3], eye[3], f, cx, cy, near_z;
};

struct ProjPack {
    int32_t nv;
    uint32_t block_begin[kMaxViews + 1];
    ProjViewArgs v[kMaxViews];
};

// One thread per particle of one view; blocks are grouped by view. Parameters are read
// structure-of-arrays (consecutive lanes read consecutive floats of each plane).
// Geometry (camera transform, pixel position, screen scale, radius) is evaluated in FP64
// and rounded once to FP32: this memory-bound kernel has FP64 throughput to spare, and
// the stored footprints then differ from the exact values by half an FP32 ulp.
__global__ void __launch_bounds__(256) project_kernel(const ProjPack pk, float4* __restrict__ footprint,
                                                      float4* __restrict__ color_radius,
                                                      float* __restrict__ depth,
                                                      uint32_t* __restrict__ tile_count) {
    int vi = 0;
    for (int i = 1; i < pk.nv; ++i) vi = (blockIdx.x >= pk.block_begin[i]) ? i : vi;
    vi = __builtin_amdgcn_readfirstlane(vi);
    const ProjViewArgs& pv = pk.v[vi];
    const uint32_t i = (blockIdx.x - pk.block_begin[vi]) * blockDim.x + threadIdx.x;
    if (i >= pv.n) return;
    const uint32_t n = pv.n;
    const uint32_t o = pv.p_off + i;

    const float mx = pv.pos[i], my = pv.pos[n + i], mz = pv.pos[2 * n + i];
    const float sigma = pv.scale[i], opa = pv.opacity[i];

    const double px = (double)pv.R[0] * mx + (double)pv.R[1] * my + (double)pv.R[2] * mz + (double)pv.t[0];
    const double py = (double)pv.R[3] * mx + (double)pv.R[4] * my + (double)pv.R[5] * mz + (double)pv.t[1];
    const double pz = (double)pv.R[6] * mx + (double)pv.R[7] * my + (double)pv.R[8] * mz + (double)pv.t[2];
    const double f = (double)pv.f;
    const double u64 = f * px / pz + (double)pv.cx;
    const double v64 = f * py / pz + (double)pv.cy;
    const double s64 = f * (double)sigma / pz;

    bool vis = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(sigma) && isfinite(opa) &&
               sigma > 0.0f && (double)opa >= 1.0 / 255.0 && pz > (double)pv.near_z;
    vis = vis && isfinite(u64) && isfinite(v64) && isfinite(s64) && s64 > 0.0;

    // colour for the direction from the camera centre to the particle (world frame)
    const int K = (pv.sh_degree + 1) * (pv.sh_degree + 1);
    float rgb[3] = {0.0f, 0.0f, 0.0f};
    {
        const float dx = mx - pv.eye[0], dy = my - pv.eye[1], dz = mz - pv.eye[2];
        const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
        float Y[16];
        sh_eval(pv.sh_degree, dx * inv, dy * inv, dz * inv, Y);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc = pv.color[(size_t)ch * n + i];
#pragma unroll
            for (int k = 1; k < 16; ++k)
                if (k < K) acc = fmaf(pv.color[(size_t)(3 * k + ch) * n + i], Y[k], acc);
            rgb[ch] = fmaxf(acc, 0.0f);
            vis = vis && isfinite(acc);
        }
    }

    float4 fp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 cr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float z32 = 1.0f;
    uint32_t cnt = 0;
    if (vis) {
        const float u = (float)u64, v = (float)v64;
        const double r64 = s64 * sqrt(log(255.0 * (double)opa)) * (1.0 + 0x1p-10) + 0x1p-6;
        const float r = (float)r64;
        z32 = (float)pz;
        fp = make_float4(u, v, (float)(1.0 / (s64 * s64)), opa);
        cr = make_float4(rgb[0], rgb[1], rgb[2], r);
        int tx0, tx1, ty0, ty1;
        const int TX = (pv.width + kTile - 1) / kTile, TY = (pv.height + kTile - 1) / kTile;
        tile_box(u, v, r, TX, TY, tx0, tx1, ty0, ty1);
        const float r2 = r * r;
        const float w_lim = (float)pv.width - 0.5f, h_lim = (float)pv.height - 0.5f;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) cnt += tile_member(u, v, r2, tx, ty, w_lim, h_lim) ? 1u : 0u;
    }
    footprint[o] = fp;
    color_radius[o] = cr;
    depth[o] = z32;
    tile_count[o] = cnt;
}

int launch_project(const isogs_scene* scenes, const isogs_camera* cams, int32_t nv, const isogs_projected* out,
                   hipStream_t stream) {
    uint32_t p_off = 0;
    for (int v0 = 0; v0 < nv; v0 += kMaxViews) {
        ProjPack pk{};
        pk.nv = min(kMaxViews, nv - v0);
        uint32_t blocks = 0;
        for (int j = 0; j < pk.nv; ++j) {
            const isogs_scene& sc = scenes[v0 + j];
            const isogs_camera& cam = cams[v0 + j];
            ProjViewArgs& a = pk.v[j];
            a.pos = sc.pos;
            a.scale = sc.scale;
            a.opacity = sc.opacity;
            a.color = sc.color;
            a.n = (uint32_t)sc.n;
            a.sh_degree = sc.sh_degree;
            a.p_off = p_off;
            a.width = cam.width;
            a.height = cam.height;
            for (int k = 0; k < 9; ++k) a.R[k] = cam.R[k];
            for (int k = 0; k < 3; ++k) a.t[k] = cam.t[k], a.eye[k] = cam.eye[k];
            a.f = cam.f;
            a.cx = cam.cx;
            a.cy = cam.cy;
            a.near_z = cam.near_z;
            pk.block_begin[j] = blocks;
            blocks += (a.n + 255u) / 256u;
            p_off += a.n;
        }
        pk.block_begin[pk.nv] = blocks;
        if (blocks == 0) continue;
        hipLaunchKernelGGL(project_kernel, dim3(blocks), dim3(256), 0, stream, pk,
                           reinterpret_cast<float4*>(out->footprint), reinterpret_cast<float4*>(out->color_radius),
                           out->depth, out->tile_count);
        if (hipPeekAtLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace isogs
