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

// A view's camera as the projection uses it: the geometry in FP64 (converted once on the
// host), with 1/f^2 for the footprint scale.
struct ProjCam {
    double R[9], t[3], f, inv_f2, cx, cy, near_z;
    float eye[3];
    int32_t width, height;
    uint32_t p_off;   // first packed record of this view
};

// All views of one launch render the same scene.
struct ProjPack {
    const float* pos;
    const float* scale;
    const float* opacity;
    const float* color;
    uint32_t n;
    int32_t nv;
    ProjCam c[kMaxViews];
};

// One thread per particle: its parameters are read once (structure of arrays, coalesced)
// and projected into every view of the launch. Geometry (camera transform, pixel position,
// screen scale, radius) is evaluated in FP64 and rounded once to FP32: this memory-bound
// kernel has FP64 throughput to spare, and the stored footprints then differ from the
// exact values by half an FP32 ulp. DEG is the SH degree of the scene.
template <int DEG>
__global__ void __launch_bounds__(256) project_kernel(const ProjPack pk, float4* __restrict__ record,
                                                      float* __restrict__ depth,
                                                      uint32_t* __restrict__ tile_count) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pk.n) return;
    const uint32_t n = pk.n;
    const float mx = pk.pos[i], my = pk.pos[n + i], mz = pk.pos[2 * n + i];
    const float sigma = pk.scale[i], opa = pk.opacity[i];
    float coef[3 * K];
    bool finite_in = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(sigma) && isfinite(opa);
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) {
        coef[k] = pk.color[(size_t)k * n + i];
        finite_in = finite_in && isfinite(coef[k]);
    }
    const bool param_ok = finite_in && sigma > 0.0f && (double)opa >= 1.0 / 255.0;
    const double root = param_ok ? sqrt(log(255.0 * (double)opa)) : 0.0;
    const double sig = (double)sigma, inv_sig2 = 1.0 / (sig * sig);
    const double dx = mx, dy = my, dz = mz;

    for (int vi = 0; vi < pk.nv; ++vi) {
        const ProjCam& pv = pk.c[vi];
        const uint32_t o = pv.p_off + i;
        const double px = pv.R[0] * dx + pv.R[1] * dy + pv.R[2] * dz + pv.t[0];
        const double py = pv.R[3] * dx + pv.R[4] * dy + pv.R[5] * dz + pv.t[1];
        const double pz = pv.R[6] * dx + pv.R[7] * dy + pv.R[8] * dz + pv.t[2];
        // one division per view: u = f px / z + cx, v = f py / z + cy, s = f sigma / z and
        // 1/s^2 = z^2 / (f^2 sigma^2), each within a few FP64 ulps before the FP32 rounding
        const double inv_z = 1.0 / pz;
        const double u64 = pv.f * px * inv_z + pv.cx;
        const double v64 = pv.f * py * inv_z + pv.cy;
        const double s64 = pv.f * sig * inv_z;
        // the stored footprint must have a normal FP32 form: centre, 1/s^2 and radius
        // finite, 1/s^2 at least the smallest normal value (a denormal may be flushed)
        const float u = (float)u64, v = (float)v64;
        const float inv_s2 = (float)(pz * pz * (pv.inv_f2 * inv_sig2));
        const float r = (float)(s64 * root * (1.0 + 0x1p-10) + 0x1p-6);
        const bool vis = param_ok && pz > pv.near_z && isfinite(u) && isfinite(v) && isfinite(s64) &&
                         s64 > 0.0 && isfinite(inv_s2) && inv_s2 >= 0x1p-126f && isfinite(r);
        float4 fp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float4 cr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float z32 = 1.0f;
        uint32_t cnt = 0;
        if (vis) {
            // colour for the direction from the camera centre to the particle (world frame)
            const float ex = mx - pv.eye[0], ey = my - pv.eye[1], ez = mz - pv.eye[2];
            const float inv = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
            float Y[16];
            sh_eval(DEG, ex * inv, ey * inv, ez * inv, Y);
            float rgb[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = coef[ch];
#pragma unroll
                for (int k = 1; k < K; ++k) acc = fmaf(coef[3 * k + ch], Y[k], acc);
                rgb[ch] = fmaxf(acc, 0.0f);
            }
            z32 = (float)pz;
            fp = make_float4(u, v, inv_s2, opa);
            cr = make_float4(rgb[0], rgb[1], rgb[2], r);
            int tx0, tx1, ty0, ty1;
            const int TX = (pv.width + kTile - 1) / kTile, TY = (pv.height + kTile - 1) / kTile;
            tile_box(u, v, r, TX, TY, tx0, tx1, ty0, ty1);
            const float r2 = r * r;
            const float w_lim = (float)pv.width - 0.5f, h_lim = (float)pv.height - 0.5f;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) cnt += tile_member(u, v, r2, tx, ty, w_lim, h_lim) ? 1u : 0u;
        }
        record[2 * (size_t)o] = fp;
        record[2 * (size_t)o + 1] = cr;
        depth[o] = z32;
        tile_count[o] = cnt;
    }
}

static void fill_proj_cam(ProjCam& c, const isogs_camera& cam, uint32_t p_off) {
    for (int k = 0; k < 9; ++k) c.R[k] = cam.R[k];
    for (int k = 0; k < 3; ++k) c.t[k] = cam.t[k], c.eye[k] = cam.eye[k];
    c.f = cam.f;
    c.inv_f2 = 1.0 / ((double)cam.f * (double)cam.f);
    c.cx = cam.cx;
    c.cy = cam.cy;
    c.near_z = cam.near_z;
    c.width = cam.width;
    c.height = cam.height;
    c.p_off = p_off;
}

int launch_project(const isogs_scene* scenes, const isogs_camera* cams, int32_t nv, const isogs_projected* out,
                   hipStream_t stream) {
    // record offset of every view
    uint32_t off[4096];
    if (nv > 4096) return -1;
    uint32_t p = 0;
    for (int v = 0; v < nv; ++v) {
        off[v] = p;
        p += (uint32_t)scenes[v].n;
    }
    // views grouped by scene (same parameter buffers), up to kMaxViews per launch
    bool done[4096] = {false};
    for (int v = 0; v < nv; ++v) {
        if (done[v]) continue;
        const isogs_scene& sc = scenes[v];
        ProjPack pk{};
        pk.pos = sc.pos;
        pk.scale = sc.scale;
        pk.opacity = sc.opacity;
        pk.color = sc.color;
        pk.n = (uint32_t)sc.n;
        auto flush = [&]() -> int {
            if (pk.nv == 0 || pk.n == 0) return 0;
            const dim3 grid((pk.n + 255) / 256);
            float4* rec = reinterpret_cast<float4*>(out->record);
            switch (sc.sh_degree) {
                case 0: hipLaunchKernelGGL(project_kernel<0>, grid, dim3(256), 0, stream, pk, rec, out->depth, out->tile_count); break;
                case 1: hipLaunchKernelGGL(project_kernel<1>, grid, dim3(256), 0, stream, pk, rec, out->depth, out->tile_count); break;
                case 2: hipLaunchKernelGGL(project_kernel<2>, grid, dim3(256), 0, stream, pk, rec, out->depth, out->tile_count); break;
                default: hipLaunchKernelGGL(project_kernel<3>, grid, dim3(256), 0, stream, pk, rec, out->depth, out->tile_count); break;
            }
            pk.nv = 0;
            return hipPeekAtLastError() == hipSuccess ? 0 : -1;
        };
        for (int u = v; u < nv; ++u) {
            const isogs_scene& su = scenes[u];
            if (done[u] || su.pos != sc.pos || su.scale != sc.scale || su.opacity != sc.opacity ||
                su.color != sc.color || su.n != sc.n || su.sh_degree != sc.sh_degree)
                continue;
            done[u] = true;
            fill_proj_cam(pk.c[pk.nv++], cams[u], off[u]);
            if (pk.nv == kMaxViews && flush()) return -1;
        }
        if (flush()) return -1;
    }
    return 0;
}

// ---- Anisotropic footprints (eq. 5-7) ------------------------------------------------------

struct AnisoProjPack {
    const float* pos;
    const float* rot;
    const float* scale;
    const float* opacity;
    const float* color;
    uint32_t n;
    int32_t nv;
    ProjCam c[kMaxViews];
};

// One thread per particle, every view of the launch. Sigma = R diag(s^2) R^T (eq. 6) is
// formed once per particle; per view, Sigma_2D = T Sigma T^T with T = J V (eq. 7), its
// inverse (the conic), the larger eigenvalue (the binning radius) - all in FP64, the
// stored footprint rounded once to FP32.
template <int DEG>
__global__ void __launch_bounds__(256) aniso_project_kernel(const AnisoProjPack pk, float4* __restrict__ record,
                                                            float2* __restrict__ conic, float* __restrict__ depth,
                                                            uint32_t* __restrict__ tile_count) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pk.n) return;
    const uint32_t n = pk.n;
    const float mx = pk.pos[i], my = pk.pos[n + i], mz = pk.pos[2 * n + i];
    const float q0 = pk.rot[i], q1 = pk.rot[n + i], q2 = pk.rot[2 * n + i], q3 = pk.rot[3 * n + i];
    const float s0 = pk.scale[i], s1 = pk.scale[n + i], s2 = pk.scale[2 * n + i];
    const float opa = pk.opacity[i];
    float coef[3 * K];
    bool finite_in = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(q0) && isfinite(q1) && isfinite(q2) &&
                     isfinite(q3) && isfinite(s0) && isfinite(s1) && isfinite(s2) && isfinite(opa);
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) {
        coef[k] = pk.color[(size_t)k * n + i];
        finite_in = finite_in && isfinite(coef[k]);
    }
    const double qw = q0, qx = q1, qy = q2, qz = q3;
    const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const bool param_ok = finite_in && s0 > 0.0f && s1 > 0.0f && s2 > 0.0f && qn > 0.0 &&
                          (double)opa >= 1.0 / 255.0;
    const double root = param_ok ? sqrt(log(255.0 * (double)opa)) : 0.0;
    // Sigma (symmetric): S00 S01 S02 S11 S12 S22
    double Sg[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (param_ok) {
        const double w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
        const double R[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                             2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                             2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
        const double d[3] = {(double)s0 * s0, (double)s1 * s1, (double)s2 * s2};
        int k = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b)
                Sg[k++] = R[3 * a] * d[0] * R[3 * b] + R[3 * a + 1] * d[1] * R[3 * b + 1] + R[3 * a + 2] * d[2] * R[3 * b + 2];
    }

    for (int vi = 0; vi < pk.nv; ++vi) {
        const ProjCam& pv = pk.c[vi];
        const uint32_t o = pv.p_off + i;
        double V[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) V[k] = pv.R[k];
        const double px = V[0] * mx + V[1] * my + V[2] * mz + pv.t[0];
        const double py = V[3] * mx + V[4] * my + V[5] * mz + pv.t[1];
        const double pz = V[6] * mx + V[7] * my + V[8] * mz + pv.t[2];
        const double f = pv.f;
        const double u64 = f * px / pz + pv.cx;
        const double v64 = f * py / pz + pv.cy;
        // T = J V, J = [[f/z, 0, -f p_x/z^2], [0, f/z, -f p_y/z^2]]
        const double j0 = f / pz, j2 = -f * px / (pz * pz), j5 = -f * py / (pz * pz);
        double T0[3], T1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T0[c] = j0 * V[c] + j2 * V[6 + c];
            T1[c] = j0 * V[3 + c] + j5 * V[6 + c];
        }
        // Sigma_2D = [[a, b], [b, c]] = T Sigma T^T
        double ST0[3], ST1[3];
        ST0[0] = Sg[0] * T0[0] + Sg[1] * T0[1] + Sg[2] * T0[2];
        ST0[1] = Sg[1] * T0[0] + Sg[3] * T0[1] + Sg[4] * T0[2];
        ST0[2] = Sg[2] * T0[0] + Sg[4] * T0[1] + Sg[5] * T0[2];
        ST1[0] = Sg[0] * T1[0] + Sg[1] * T1[1] + Sg[2] * T1[2];
        ST1[1] = Sg[1] * T1[0] + Sg[3] * T1[1] + Sg[4] * T1[2];
        ST1[2] = Sg[2] * T1[0] + Sg[4] * T1[1] + Sg[5] * T1[2];
        const double a = T0[0] * ST0[0] + T0[1] * ST0[1] + T0[2] * ST0[2];
        const double b = T0[0] * ST1[0] + T0[1] * ST1[1] + T0[2] * ST1[2];
        const double c = T1[0] * ST1[0] + T1[1] * ST1[1] + T1[2] * ST1[2];
        const double det = a * c - b * b;
        const double lam = 0.5 * (a + c) + sqrt(0.25 * (a - c) * (a - c) + b * b);
        const float u = (float)u64, v = (float)v64;
        const float A = (float)(c / det), B = (float)(-b / det), C = (float)(a / det);
        const float r = (float)(sqrt(lam) * root * (1.0 + 0x1p-10) + 0x1p-6);
        const bool vis = param_ok && pz > pv.near_z && isfinite(u) && isfinite(v) && isfinite(det) &&
                         det > 0.0 && isfinite(A) && isfinite(B) && isfinite(C) && A >= 0x1p-126f &&
                         C >= 0x1p-126f && isfinite(r);
        float4 fp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float4 cr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float2 bc = make_float2(0.0f, 0.0f);
        float z32 = 1.0f;
        uint32_t cnt = 0;
        if (vis) {
            const float ex = mx - pv.eye[0], ey = my - pv.eye[1], ez = mz - pv.eye[2];
            const float inv = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
            float Y[16];
            sh_eval(DEG, ex * inv, ey * inv, ez * inv, Y);
            float rgb[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = coef[ch];
#pragma unroll
                for (int k = 1; k < K; ++k) acc = fmaf(coef[3 * k + ch], Y[k], acc);
                rgb[ch] = fmaxf(acc, 0.0f);
            }
            z32 = (float)pz;
            fp = make_float4(u, v, A, opa);
            cr = make_float4(rgb[0], rgb[1], rgb[2], r);
            bc = make_float2(B, C);
            int tx0, tx1, ty0, ty1;
            const int TX = (pv.width + kTile - 1) / kTile, TY = (pv.height + kTile - 1) / kTile;
            tile_box(u, v, r, TX, TY, tx0, tx1, ty0, ty1);
            const float r2 = r * r;
            const float w_lim = (float)pv.width - 0.5f, h_lim = (float)pv.height - 0.5f;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) cnt += tile_member(u, v, r2, tx, ty, w_lim, h_lim) ? 1u : 0u;
        }
        record[2 * (size_t)o] = fp;
        record[2 * (size_t)o + 1] = cr;
        conic[o] = bc;
        depth[o] = z32;
        tile_count[o] = cnt;
    }
}

int launch_aniso_project(const isogs_aniso_scene* scenes, const isogs_camera* cams, int32_t nv,
                         const isogs_aniso_projected* out, hipStream_t stream) {
    uint32_t off[4096];
    if (nv > 4096) return -1;
    uint32_t p = 0;
    for (int v = 0; v < nv; ++v) {
        off[v] = p;
        p += (uint32_t)scenes[v].n;
    }
    bool done[4096] = {false};
    for (int v = 0; v < nv; ++v) {
        if (done[v]) continue;
        const isogs_aniso_scene& sc = scenes[v];
        AnisoProjPack pk{};
        pk.pos = sc.pos;
        pk.rot = sc.rot;
        pk.scale = sc.scale;
        pk.opacity = sc.opacity;
        pk.color = sc.color;
        pk.n = (uint32_t)sc.n;
        auto flush = [&]() -> int {
            if (pk.nv == 0 || pk.n == 0) return 0;
            const dim3 grid((pk.n + 255) / 256);
            float4* rec = reinterpret_cast<float4*>(out->fp.record);
            float2* cn = reinterpret_cast<float2*>(out->conic);
            switch (sc.sh_degree) {
                case 0: hipLaunchKernelGGL(aniso_project_kernel<0>, grid, dim3(256), 0, stream, pk, rec, cn, out->fp.depth, out->fp.tile_count); break;
                case 1: hipLaunchKernelGGL(aniso_project_kernel<1>, grid, dim3(256), 0, stream, pk, rec, cn, out->fp.depth, out->fp.tile_count); break;
                case 2: hipLaunchKernelGGL(aniso_project_kernel<2>, grid, dim3(256), 0, stream, pk, rec, cn, out->fp.depth, out->fp.tile_count); break;
                default: hipLaunchKernelGGL(aniso_project_kernel<3>, grid, dim3(256), 0, stream, pk, rec, cn, out->fp.depth, out->fp.tile_count); break;
            }
            pk.nv = 0;
            return hipPeekAtLastError() == hipSuccess ? 0 : -1;
        };
        for (int u = v; u < nv; ++u) {
            const isogs_aniso_scene& su = scenes[u];
            if (done[u] || su.pos != sc.pos || su.rot != sc.rot || su.scale != sc.scale || su.opacity != sc.opacity ||
                su.color != sc.color || su.n != sc.n || su.sh_degree != sc.sh_degree)
                continue;
            done[u] = true;
            fill_proj_cam(pk.c[pk.nv++], cams[u], off[u]);
            if (pk.nv == kMaxViews && flush()) return -1;
        }
        if (flush()) return -1;
    }
    return 0;
}

}  // namespace isogs
