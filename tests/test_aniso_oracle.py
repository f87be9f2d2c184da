"""Pins of the anisotropic oracle (eq. 5-7) against what the paper and the mathematics fix:
quaternion rotations in closed form, the isotropic special case (sigma^2 I gives the
circle of scale f sigma / z on the optical axis, sigma^2 J J^T off it, with J checked by
finite differences of the pinhole map), a quarter turn about the optical axis swapping
the conic's axes, the support disk containing every pixel that the kernel reaches,
tiled == untiled, agreement with the isotropic walk for circular conics, and central
finite differences of every parameter gradient."""
import math

import numpy as np
import pytest

import oracle as O
import scenegen as S

A64 = O.aniso64


def _one(pos, rot, scale, opacity=0.8, rgb=(0.2, 0.5, 0.9)):
    return S.AnisoScene(pos=np.asarray(pos, np.float32).reshape(3, 1), rot=np.asarray(rot, np.float32).reshape(4, 1),
                        scale=np.asarray(scale, np.float32).reshape(3, 1), opacity=np.asarray([opacity], np.float32),
                        color=np.asarray(rgb, np.float32).reshape(3, 1), sh_degree=0)


def test_quaternion_rotations():
    rng = np.random.default_rng(0)
    q = rng.normal(size=(4, 50))
    q /= np.linalg.norm(q, axis=0)
    R = A64.quat_to_rot(q)
    for k in range(50):
        M = R[:, :, k]
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(M) - 1.0) < 1e-13
        assert np.allclose(M, A64.quat_to_rot(-q[:, k:k + 1])[:, :, 0], atol=1e-14)
    th = 0.7
    Rz = A64.quat_to_rot(np.array([[math.cos(th / 2)], [0.0], [0.0], [math.sin(th / 2)]]))[:, :, 0]
    assert np.allclose(Rz, [[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]], atol=1e-15)
    # Rodrigues' formula for a general axis
    ax = np.array([1.0, -2.0, 0.5])
    ax /= np.linalg.norm(ax)
    Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    Rr = np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * Kx @ Kx
    qa = np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * ax])[:, None]
    assert np.allclose(A64.quat_to_rot(qa)[:, :, 0], Rr, atol=1e-14)


def test_isotropic_covariance_and_on_axis_circle():
    """Sigma = sigma^2 I for any rotation (eq. 6); on the optical axis eq. 7 gives the
    circle of scale s = f sigma / z: conic I / s^2, the isotropic path's footprint and
    binning radius."""
    cam = S.look_at_camera((0.0, 0.0, 3.0), width=64, height=64)
    rng = np.random.default_rng(1)
    q = rng.normal(size=4)
    sig = 0.05
    sc = _one((0.0, 0.0, 0.4), q, (sig, sig, sig))
    R = A64.quat_to_rot((q / np.linalg.norm(q))[:, None])
    Sig = A64.covariance3d(R, np.full((3, 1), np.float32(sig), np.float64))[:, :, 0]
    assert np.allclose(Sig, np.float32(sig) ** 2 * np.eye(3), atol=1e-17)
    pa = A64.project_aniso64(sc, cam)
    iso = S.Scene(pos=sc.pos, scale=np.asarray([sig], np.float32), opacity=sc.opacity, color=sc.color, sh_degree=0)
    pi = O.project64(iso, cam)
    s = pi.s[0]
    assert abs(pi.u[0] - 32.0) < 1e-12 and abs(pi.v[0] - 32.0) < 1e-12     # on the axis
    A, B, C = pa.conic[:, 0]
    assert abs(A * s * s - 1.0) < 1e-12 and abs(C * s * s - 1.0) < 1e-12 and abs(B) < 1e-9 / (s * s)
    assert abs(pa.radius[0] - pi.radius[0]) < 1e-12 * pi.radius[0]
    assert abs(s - cam.f * float(np.float32(sig)) / (3.0 - float(np.float32(0.4)))) < 1e-12


def test_screen_covariance_against_a_numerical_jacobian():
    """Off the axis an isotropic Gaussian projects to sigma^2 J J^T: J from central
    differences of the pinhole map, independent of the closed form."""
    cam = S.orbit_camera(0.4, 4.0, 320, 240)
    V = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    rng = np.random.default_rng(2)
    for _ in range(5):
        mu = rng.uniform(-0.8, 0.8, size=3)
        sig = 0.03
        sc = _one(mu, (1.0, 0.0, 0.0, 0.0), (sig, sig, sig))
        pa = A64.project_aniso64(sc, cam)
        p = V @ sc.pos[:, 0].astype(np.float64) + t

        def pin(pp):
            return np.array([cam.f * pp[0] / pp[2], cam.f * pp[1] / pp[2]])
        h = 1e-6
        J = np.stack([(pin(p + h * e) - pin(p - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        cov = float(np.float32(sig)) ** 2 * J @ J.T
        assert np.allclose(pa.cov[:, 0], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-7, atol=0)


def test_quarter_turn_about_the_axis_swaps_the_conic_axes():
    cam = S.look_at_camera((0.0, 0.0, 3.0), width=64, height=64)
    # camera looks down -z (world); a rotation about world z is a rotation about the view axis
    sc = _one((0.0, 0.0, 0.0), (1.0, 0.0, 0.0, 0.0), (0.08, 0.02, 0.05))
    th = math.pi / 2
    sr = _one((0.0, 0.0, 0.0), (math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)), (0.08, 0.02, 0.05))
    a = A64.project_aniso64(sc, cam).conic[:, 0]
    b = A64.project_aniso64(sr, cam).conic[:, 0]
    assert abs(a[1]) < 1e-9 * a[0] and abs(b[1]) < 1e-6 * b[0]
    assert abs(a[0] - b[2]) < 1e-6 * a[0] and abs(a[2] - b[0]) < 1e-6 * a[2]
    assert a[0] < a[2]        # the long axis (x) has the smaller conic coefficient


def test_support_disk_contains_every_reached_pixel():
    """Brute force: every pixel centre where alpha >= 1/255 (FP64) lies within the binning
    radius and in a member tile."""
    sc = S.aniso_mixture_scene(300, seed=3, log_scale_mean=math.log(0.03), axis_log_std=0.8, sh_degree=0)
    cam = S.orbit_camera(1.0, 2.5, 96, 80)
    pr = A64.project_aniso64(sc, cam)
    X, Y = np.meshgrid(np.arange(96) + 0.5, np.arange(80) + 0.5)
    views = A64.f32_views_aniso([pr], [cam])
    gi, ty, tx = O.member_tiles(views[0]["u"], views[0]["v"], views[0]["r"], 96, 80)
    member = set(zip(gi.tolist(), ty.tolist(), tx.tolist()))
    hits = 0
    for g in np.nonzero(pr.visible)[0]:
        dx, dy = X - pr.u[g], Y - pr.v[g]
        a = pr.opacity[g] * np.exp(-A64.kernel_exponent(dx, dy, pr.conic[:, g]))
        ys, xs = np.nonzero(a >= O.ALPHA_MIN)
        for y, x in zip(ys, xs):
            assert math.hypot(X[y, x] - pr.u[g], Y[y, x] - pr.v[g]) <= pr.radius[g]
            assert (int(g), int(y) // 16, int(x) // 16) in member
            hits += 1
    assert hits > 1000


def test_tiled_equals_untiled_bitwise():
    for seed in (4, 5):
        sc = S.aniso_mixture_scene(150, seed=seed, log_scale_mean=math.log(0.04), axis_log_std=0.6, sh_degree=1)
        cam = S.orbit_camera(0.3 * seed, 2.5, 48, 40)
        img_t, T_t, _, _, projs, _ = A64.render_aniso_views([sc], [cam], bg=(0.1, 0.2, 0.3))
        img_u, T_u = A64.render_aniso_untiled(projs[0], 48, 40, bg=(0.1, 0.2, 0.3))
        assert np.array_equal(img_t[0], img_u) and np.array_equal(T_t[0], T_u)
        assert (T_u < 0.999).mean() > 0.3


def test_circular_conics_composite_like_the_isotropic_walk():
    """The same footprints through both walks: the anisotropic one with conic I / s^2."""
    rng = np.random.default_rng(6)
    n = 40
    u, v = rng.uniform(0, 32, n), rng.uniform(0, 32, n)
    s = rng.uniform(1.0, 6.0, n)
    o = rng.uniform(0.05, 0.99, n)
    rgb = rng.uniform(0, 1, (3, n))
    conic = np.array([1 / s ** 2, np.zeros(n), 1 / s ** 2])
    X, Y = np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5)
    seq = np.arange(n)
    Ci, Ti, ni = O.composite_pixels(X.ravel(), Y.ravel(), seq, u, v, s, o, rgb, (0.0, 0.0, 0.0))
    Ca, Ta, na = A64.composite_pixels_aniso(X.ravel(), Y.ravel(), seq, u, v, conic, o, rgb, (0.0, 0.0, 0.0))
    assert np.abs(Ci - Ca).max() < 1e-13 and np.abs(Ti - Ta).max() < 1e-13 and np.array_equal(ni, na)


def test_white_partition_of_unity():
    sc = S.aniso_mixture_scene(200, seed=7, log_scale_mean=math.log(0.05), sh_degree=0)
    sc.color[:] = 1.0
    cam = S.orbit_camera(2.0, 2.5, 40, 32)
    img, T, _, _, _, _ = A64.render_aniso_views([sc], [cam])
    assert np.abs(img[0] - (1.0 - T[0])[None]).max() < 1e-12


@pytest.mark.parametrize("deg", [0, 2])
def test_gradients_match_central_differences(deg):
    """Every parameter of a small scene: analytic FP64 gradients of L = <W, C> against
    central differences, skipping parameters whose +-h renders take a different decision."""
    rng = np.random.default_rng(10 + deg)
    n = 12
    sc = S.aniso_mixture_scene(n, seed=20 + deg, log_scale_mean=math.log(0.12), log_scale_std=0.2,
                               axis_log_std=0.4, sh_degree=deg)
    sc.pos[:] = (rng.uniform(-0.4, 0.4, size=(3, n))).astype(np.float32)
    sc.opacity[:] = rng.uniform(0.3, 0.9, n).astype(np.float32)
    cam = S.orbit_camera(0.5, 2.2, 24, 20)
    W = rng.normal(size=(3, 20, 24))
    bg = (0.05, 0.1, 0.2)
    g = A64.scene_grads_aniso(sc, [cam], [W], bg)

    def loss(s2):
        pr = A64.project_aniso64(s2, cam)
        img, _ = A64.render_aniso_untiled(pr, 24, 20, bg)
        return float((W * img).sum()), A64.decision_signature_aniso(pr, 24, 20, bg)

    def with_param(name, idx, delta):
        s2 = S.AnisoScene(pos=sc.pos.astype(np.float64), rot=sc.rot.astype(np.float64),
                          scale=sc.scale.astype(np.float64), opacity=sc.opacity.astype(np.float64),
                          color=sc.color.astype(np.float64), sh_degree=deg)
        getattr(s2, name)[idx] += delta
        return s2

    checked = 0
    for name in ("pos", "rot", "scale", "opacity", "color"):
        arr = getattr(sc, name)
        for idx in np.ndindex(arr.shape):
            base = float(arr[idx])
            h = 1e-6 * max(1.0, abs(base))
            lp, sp = loss(with_param(name, idx, h))
            lm, sm = loss(with_param(name, idx, -h))
            if sp != sm:
                continue
            fd = (lp - lm) / (2 * h)
            an = float(g[name][idx])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (name, idx, fd, an)
            checked += 1
    assert checked > 0.8 * sum(getattr(sc, k).size for k in ("pos", "rot", "scale", "opacity", "color"))


def test_centre_growth_bounds_every_shift_and_reduces_to_the_circle():
    """The band growth for a centre rounded to FP32: brute force over shifts of at most e in
    x and y (corners, edges, a random interior set) never changes Q by more than
    centre_growth, the bound is reached at a corner to first order, and for a circular
    conic it is the isotropic walk's (2 (|dx| + |dy|) e + 2 e^2) / s^2."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        a, c = rng.uniform(0.01, 2.0, 2)
        b = rng.uniform(-0.99, 0.99) * math.sqrt(a * c)
        conic = np.array([a, b, c])
        dx, dy = rng.uniform(-20, 20, 2)
        e = rng.uniform(1e-6, 0.1)
        Q0 = A64.kernel_exponent(dx, dy, conic)
        bound = A64.centre_growth(dx, dy, conic, e)
        sx = np.concatenate([[-e, -e, e, e, 0, 0, e, -e], rng.uniform(-e, e, 64)])
        sy = np.concatenate([[-e, e, -e, e, e, -e, 0, 0], rng.uniform(-e, e, 64)])
        dQ = np.abs(A64.kernel_exponent(dx - sx, dy - sy, conic) - Q0)
        assert dQ.max() <= bound * (1 + 1e-12) + 1e-15
        assert dQ[:4].max() >= 0.5 * bound
    s = 2.5
    dx, dy, e = 3.0, -1.5, 0.01
    iso = (2.0 * (abs(dx) + abs(dy)) * e + 2.0 * e * e) / (s * s)
    assert abs(A64.centre_growth(dx, dy, np.array([1 / s ** 2, 0.0, 1 / s ** 2]), e) - iso) < 1e-15


def test_rounded_flags_cover_the_rounded_footprints():
    """A render of the FP32-rounded footprints differs from the FP64 one by at most 1e-4 on
    every pixel that the rounded-footprint flags leave unflagged."""
    sc = S.aniso_mixture_scene(400, seed=12, log_scale_mean=math.log(0.03), axis_log_std=0.7, sh_degree=1)
    cam = S.orbit_camera(0.9, 2.6, 64, 48)
    img, T, _, flags, projs, bins = A64.render_aniso_views([sc], [cam], rounded=True, q_err=2.0 ** -20)
    pr = projs[0]
    v = pr.visible
    r32 = lambda x: np.where(v, x, 0.0).astype(np.float32).astype(np.float64)
    conic32 = np.array([r32(x) for x in pr.conic])
    img32, T32, _, _ = A64.render_aniso_tiled(r32(pr.u), r32(pr.v), conic32, pr.opacity, pr.rgb, bins, 0, 64, 48)
    d = np.maximum(np.abs(img32 - img[0]).max(axis=0), np.abs(T32 - T[0]))
    assert d[~flags[0]].max() <= 1e-4
    assert flags[0].mean() < 0.05
