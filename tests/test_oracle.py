"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the plausible oracle mistake it is there to catch. None of them compares
the oracle with itself: they use hand-worked values, closed forms, invariants, brute
force, library routines and finite differences.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from scenegen import Camera, Scene, look_at_camera, uniform_cube_scene, mixture_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def axis_camera(f=100.0, cx=16.5, cy=16.5, w=32, h=32, near=0.2):
    """Camera at the world origin looking down +z with x right, y down."""
    return Camera(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), eye=np.zeros(3, np.float32),
                  f=float(np.float32(f)), cx=float(np.float32(cx)), cy=float(np.float32(cy)),
                  width=w, height=h, near=near)


def make_scene(pos, sigma, opacity, rgb, dtype=np.float32):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    return Scene(pos=np.ascontiguousarray(pos.T).astype(dtype), scale=np.asarray(sigma, dtype),
                 opacity=np.asarray(opacity, dtype), color=np.ascontiguousarray(np.asarray(rgb, np.float64).reshape(-1, 3).T).astype(dtype),
                 sh_degree=0)


def render_both(scene, cam, bg=(0.0, 0.0, 0.0)):
    pr = O.project64(scene, cam)
    un, Tun = O.render64_untiled(pr, cam.width, cam.height, bg)
    bins = O.bin_sort_ref(O.f32_views([pr], [cam]))
    ti, Tti, nl = O.render64_tiled(pr.u, pr.v, pr.s, pr.opacity, pr.rgb, bins, 0, cam.width, cam.height, bg)
    return pr, un, Tun, ti, Tti, nl, bins


# ---------------------------------------------------------------------------------------
# eq. 8 + isotropic footprint: single-particle closed forms
# ---------------------------------------------------------------------------------------

def test_single_gaussian_peak_and_falloff_exact_e_minus_1():
    """Catches: a 1/2 in the exponent, s^2 vs s, a wrong focal scaling, a pixel-centre
    offset. sigma is chosen so s = f sigma / z = 2 px; the pixel 2 px from the centre must
    see exactly o e^-1 (with a 1/2 in the exponent it would be o e^-1/2)."""
    cam = axis_camera()
    o, rgb = 0.8, (0.3, 0.6, 0.9)
    sc = make_scene([0, 0, 5.0], [0.1], [o], [rgb])
    pr, un, Tun, ti, Tti, _, _ = render_both(sc, cam)
    rgb = np.array(rgb, np.float32).astype(np.float64)
    s = 100.0 * float(np.float32(0.1)) / 5.0
    assert abs(pr.s[0] - 2.0) < 1e-6
    for img, T in ((un, Tun), (ti, Tti)):
        np.testing.assert_allclose(img[:, 16, 16], rgb * float(np.float32(o)), rtol=1e-12)
        assert abs(T[16, 16] - (1 - float(np.float32(o)))) < 1e-12
        a2 = float(np.float32(o)) * math.exp(-4.0 / (s * s))
        assert abs(a2 - float(np.float32(o)) / math.e) < 1e-7
        for (j, i) in ((16, 18), (16, 14), (18, 16), (14, 16)):
            np.testing.assert_allclose(img[:, j, i], rgb * a2, rtol=1e-12)
        # diagonal neighbour at distance sqrt(2): exp(-2/4)
        np.testing.assert_allclose(img[:, 17, 17], rgb * float(np.float32(o)) * math.exp(-2.0 / (s * s)),
                                   rtol=1e-12)


def test_support_cutoff_alpha_threshold():
    """Catches: a missing 1/255 cutoff or a cutoff on the wrong quantity. A pixel at
    distance d contributes iff o exp(-d^2/s^2) >= 1/255."""
    cam = axis_camera(w=48, h=16, cx=0.5, cy=8.5)
    o = 0.5
    sc = make_scene([0, 0, 5.0], [0.1], [o], [(1, 1, 1)])
    pr, un, *_ = render_both(sc, cam)
    s = pr.s[0]
    d_cut = s * math.sqrt(math.log(255 * float(np.float32(o))))
    row = un[0, 8, :]
    for i in range(48):
        d = i  # pixel i centre is at i + 0.5 = u + i
        a = float(np.float32(o)) * math.exp(-d * d / (s * s))
        if d < d_cut - 1e-9:
            assert row[i] == pytest.approx(a, rel=1e-12)
        elif d > d_cut + 1e-9:
            assert row[i] == 0.0


def test_distance_scaling_identical_footprint():
    """Catches: s computed from sigma alone or from the Euclidean distance to the eye.
    Twice the depth with twice the scale gives the same circle (eq. 8 with s = f sigma/z):
    doubling an FP32 value is exact, so the images are identical."""
    cam = axis_camera(w=40, h=40, cx=20.0, cy=20.0)
    near = make_scene([[0.3, -0.2, 5.0]], [0.1], [0.7], [(0.2, 0.5, 0.9)])
    far = make_scene([[0.6, -0.4, 10.0]], [0.2], [0.7], [(0.2, 0.5, 0.9)])
    a = O.render64_untiled(O.project64(near, cam), 40, 40)[0]
    b = O.render64_untiled(O.project64(far, cam), 40, 40)[0]
    assert a.max() > 0.3
    np.testing.assert_array_equal(a, b)


def test_projection_camera_conventions():
    """Catches: a transposed rotation, a sign error in t, flipped image axes. A point
    above the target (world +y) must appear above the image centre (smaller v), a point
    to the camera's right must have larger u, and a camera-space point built from a pixel
    must project back to that pixel."""
    cam = look_at_camera((0.0, 0.0, 3.0), width=64, height=64)
    sc = make_scene([[0, 0.5, 0], [0.5, 0, 0], [0, 0, 0]], [0.01] * 3, [0.5] * 3, [(1, 1, 1)] * 3)
    pr = O.project64(sc, cam)
    assert pr.v[0] < cam.cy - 5 and abs(pr.u[0] - cam.cx) < 1e-9
    assert pr.u[1] > cam.cx + 5 and abs(pr.v[1] - cam.cy) < 1e-9
    assert abs(pr.z[2] - 3.0) < 1e-6
    # an oblique camera: back-project chosen pixels at chosen depths
    cam2 = look_at_camera((2.0, 1.0, 3.0), target=(0.1, -0.2, 0.3), width=96, height=64)
    R = cam2.R.astype(np.float64)
    t = cam2.t.astype(np.float64)
    uv = np.array([[10.25, 5.5], [80.0, 60.0], [48.0, 32.0]])
    zz = np.array([2.0, 3.5, 5.0])
    pc = np.stack([(uv[:, 0] - cam2.cx) * zz / cam2.f, (uv[:, 1] - cam2.cy) * zz / cam2.f, zz])
    mu = np.linalg.solve(R, pc - t[:, None])
    sc2 = Scene(pos=mu, scale=np.full(3, 0.01), opacity=np.full(3, 0.5), color=np.ones((3, 3)), sh_degree=0)
    pr2 = O.project64(sc2, cam2)
    np.testing.assert_allclose(pr2.u, uv[:, 0], atol=1e-9)
    np.testing.assert_allclose(pr2.v, uv[:, 1], atol=1e-9)
    np.testing.assert_allclose(pr2.z, zz, atol=1e-9)


def test_culling_rules():
    """Catches: rendering particles behind the near plane, with sigma <= 0, with an
    opacity that can never reach 1/255, or with non-finite parameters."""
    cam = axis_camera()
    pos = [[0, 0, 5], [0, 0, 0.1], [0, 0, -5], [0, 0, 5], [0, 0, 5], [0, 0, 5], [np.nan, 0, 5], [0, 0, 5]]
    sig = [0.1, 0.1, 0.1, 0.0, -0.1, 0.1, 0.1, 0.1]
    opa = [0.5, 0.5, 0.5, 0.5, 0.5, 1 / 256, 0.5, 0.5]
    sc = make_scene(pos, sig, opa, [(1, 1, 1)] * 8)
    sc.scale[7] = np.inf
    pr = O.project64(sc, cam)
    assert pr.visible.tolist() == [True] + [False] * 7
    bins = O.bin_sort_ref(O.f32_views([pr], [cam]))
    assert bins.tile_count.tolist()[1:] == [0] * 7 and bins.tile_count[0] > 0


def test_culling_of_footprints_without_fp32_form():
    """Catches: a footprint stored with 1/s^2 = inf (0 * inf = NaN in any later product)
    or a denormal 1/s^2 (flushed to 0 by some FP32 units: a kernel of constant value) or an
    infinite binning radius. With f = 100 and z = 5, sigma = 1e-22 gives s = 2e-21 px
    (1/s^2 = 2.5e41 overflows FP32) and sigma = 1e19 gives s = 2e20 px (1/s^2 = 2.5e-41,
    below the smallest normal FP32 value); both are culled, while sigma = 1e-17
    (1/s^2 = 2.5e31) and sigma = 1e17 (1/s^2 = 2.5e-37, normal) stay visible."""
    cam = axis_camera()
    sc = make_scene([[0, 0, 5]] * 4, [1e-22, 1e19, 1e-17, 1e17], [0.5] * 4, [(1, 1, 1)] * 4)
    pr = O.project64(sc, cam)
    assert pr.visible.tolist() == [False, False, True, True]
    assert (pr.radius[:2] == 0).all()


# ---------------------------------------------------------------------------------------
# eq. 4: compositing
# ---------------------------------------------------------------------------------------

def test_golden_two_gaussians_hand_worked():
    """Hand-worked eq. 4 values (tests/golden/two_gaussians.json). Catches: back-to-front
    order, a product over the wrong index range, a missing background term, the 0.99
    clamp, and termination before rather than after the entry that crosses 1e-4."""
    d = json.load(open(os.path.join(GOLDEN, "two_gaussians.json")))
    c = d["camera"]
    cam = axis_camera(c["f"], c["cx"], c["cy"], c["width"], c["height"])
    for case in d["cases"]:
        ps = case["particles"]
        sc = make_scene([p["pos"] for p in ps], [p["sigma"] for p in ps], [p["opacity"] for p in ps],
                        [p["rgb"] for p in ps])
        pr, un, Tun, ti, Tti, nl, _ = render_both(sc, cam, tuple(case["bg"]))
        j, i = case["pixel"]
        for img, T in ((un, Tun), (ti, Tti)):
            np.testing.assert_allclose(img[:, j, i], case["C"], rtol=1e-6, atol=1e-12, err_msg=case["name"])
            assert T[j, i] == pytest.approx(case["T"], rel=1e-6), case["name"]
        if "n_last" in case:
            assert nl[j, i] == case["n_last"]


def test_white_scene_partition_of_unity():
    """Catches: a weight other than alpha T, T updated before use, a dropped (1 - alpha).
    With every colour 1 and no background, C = 1 - T_final at every pixel."""
    sc = uniform_cube_scene(300, seed=3, log_scale_mean=math.log(0.08))
    sc.color[:] = 1.0
    cam = look_at_camera((0, 0, 3.0), width=40, height=40)
    pr, un, Tun, ti, Tti, _, _ = render_both(sc, cam)
    assert (Tun < 0.5).mean() > 0.15
    for ch in range(3):
        np.testing.assert_allclose(un[ch], 1.0 - Tun, atol=1e-12)
        np.testing.assert_allclose(ti[ch], 1.0 - Tti, atol=1e-12)


def test_transmittance_monotone_positive_and_stop_rule():
    """Catches: T increasing, T reaching 0, or a pixel going on after T < 1e-4."""
    sc = uniform_cube_scene(600, seed=4, log_scale_mean=math.log(0.15))
    sc.opacity[:] = np.float32(0.9)
    cam = look_at_camera((0, 0, 3.0), width=32, height=32)
    pr = O.project64(sc, cam)
    seq = O.depth_order(pr)
    X, Y = np.meshgrid(np.arange(32), np.arange(32))
    C, T, nl, tr = O.composite_pixels(X.ravel() + 0.5, Y.ravel() + 0.5, seq, pr.u, pr.v, pr.s,
                                      pr.opacity, pr.rgb, (0, 0, 0), trace=True)
    prev = np.ones(T.shape[0])
    stopped = np.zeros(T.shape[0], bool)
    for pos, g, a, Tk, use, G in tr["records"]:
        assert not (use & stopped).any()
        assert (Tk[use] <= prev[use] + 0.0).all() and (Tk > 0).all()
        prev = np.where(use, Tk * (1 - a), prev)
        stopped |= use & (prev < O.T_MIN)
    assert (T > 0).all()
    assert stopped.sum() > 10
    assert ((T < O.T_MIN) == stopped).all()


# ---------------------------------------------------------------------------------------
# View independence (Section 2): rolling the camera rotates the image into itself
# ---------------------------------------------------------------------------------------

def test_roll_invariance():
    """Catches: an anisotropic or orientation-dependent footprint. A 90 degree roll about
    the optical axis maps pixel centres onto pixel centres; every isotropic footprint
    keeps its size, so the image is the rotated image."""
    sc = uniform_cube_scene(200, seed=5, log_scale_mean=math.log(0.05))
    a = look_at_camera((0, 0, 3.0), up=(0, 1, 0), width=48, height=48)
    b = look_at_camera((0, 0, 3.0), up=(1, 0, 0), width=48, height=48)
    A = O.render64_untiled(O.project64(sc, a), 48, 48)[0]
    B = O.render64_untiled(O.project64(sc, b), 48, 48)[0]
    assert A.max() > 0.2
    for ch in range(3):
        np.testing.assert_allclose(B[ch], np.rot90(A[ch], 1), atol=1e-12)


# ---------------------------------------------------------------------------------------
# Tiling, membership, sort
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed,w,h,n", [(0, 64, 64, 200), (1, 40, 24, 150), (2, 33, 17, 120), (3, 16, 16, 60)])
def test_tiled_equals_untiled_bitwise(seed, w, h, n):
    """Catches: a binning radius that misses part of the support, a wrong tile rectangle
    at ragged image edges, a sort that breaks depth order. In FP64 the tiled render must
    be bit-identical to the plain definition."""
    sc = uniform_cube_scene(n, seed=seed, log_scale_mean=math.log(0.05), log_scale_std=0.5)
    cam = look_at_camera((0.4, 0.3, 2.6), width=w, height=h)
    pr, un, Tun, ti, Tti, _, bins = render_both(sc, cam, bg=(0.1, 0.2, 0.3))
    z = np.sort(pr.z[pr.visible])
    assert np.all(np.diff(z) / z[1:] > 2.0 ** -20)      # no near-ties in these scenes
    assert un.max() > 0.1 and bins.keys.shape[0] > n // 2
    np.testing.assert_array_equal(un, ti)
    np.testing.assert_array_equal(Tun, Tti)


def test_membership_superset_brute_force():
    """Catches: a radius without the FP32 margin, or a tile test on the wrong corner.
    Every (pixel, particle) pair with alpha >= 1/255 in FP64 must have the particle in the
    pixel's tile."""
    sc = uniform_cube_scene(150, seed=7, log_scale_mean=math.log(0.06), log_scale_std=0.6)
    cam = look_at_camera((0.2, -0.3, 2.4), width=50, height=37)
    pr = O.project64(sc, cam)
    gi, ty, tx = O.member_tiles(*[O.f32_views([pr], [cam])[0][k] for k in ("u", "v", "r")], 50, 37)
    member = set(zip(gi.tolist(), ty.tolist(), tx.tolist()))
    X, Y = np.meshgrid(np.arange(50) + 0.5, np.arange(37) + 0.5)
    n_pairs = 0
    for g in np.nonzero(pr.visible)[0]:
        a = pr.opacity[g] * np.exp(-((X - pr.u[g]) ** 2 + (Y - pr.v[g]) ** 2) / pr.s[g] ** 2)
        jj, ii = np.nonzero(a >= O.ALPHA_MIN)
        for j, i in zip(jj, ii):
            assert (int(g), int(j) // 16, int(i) // 16) in member
            n_pairs += 1
    assert n_pairs > 1000


def test_member_tiles_bbox_equals_brute_force():
    """Catches: a candidate box that is too small near image borders."""
    for seed in range(3):
        u, v, z, r = __import__("scenegen").random_projected(300, 70, 45, seed=seed, max_radius=30.0)
        a = O.member_tiles(u, v, r, 70, 45)
        b = O.member_tiles(u, v, r, 70, 45, brute_force=True)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_tile_member_matches_exact_geometry():
    """Catches: a wrong tile rectangle (pixel edges instead of pixel centres, the last
    ragged column) or a wrong distance formula. The FP32 test must agree with the exact
    rational distance from (u, v) to the clamped nearest point of the tile's pixel-centre
    rectangle wherever the exact margin exceeds FP32 rounding."""
    from fractions import Fraction as F
    import scenegen
    W, H = 70, 45
    u, v, z, r = scenegen.random_projected(400, W, H, seed=21, max_radius=25.0)
    TX, TY = O.tile_grid(W, H)
    rng = np.random.default_rng(0)
    tx = rng.integers(0, TX, 400)
    ty = rng.integers(0, TY, 400)
    got = O.tile_member_f32(u, v, r, tx, ty, W, H)
    decided = 0
    for i in range(400):
        xl, xh = F(16 * int(tx[i])) + F(1, 2), min(F(16 * int(tx[i])) + F(31, 2), F(W) - F(1, 2))
        yl, yh = F(16 * int(ty[i])) + F(1, 2), min(F(16 * int(ty[i])) + F(31, 2), F(H) - F(1, 2))
        uu, vv, rr = F(float(u[i])), F(float(v[i])), F(float(r[i]))
        px = min(max(uu, xl), xh)
        py = min(max(vv, yl), yh)
        d2 = (uu - px) ** 2 + (vv - py) ** 2
        if abs(d2 - rr * rr) > F(1, 10 ** 4) * (rr * rr + 1):
            assert bool(got[i]) == (d2 <= rr * rr), i
            decided += 1
    assert decided > 390 and 20 < got.sum() < 380


@pytest.mark.parametrize("ties", [False, True])
def test_bin_sort_against_python_sorted(ties):
    """Catches: an unstable sort, wrong key packing, wrong range ends or a wrong offset
    scan. The reference here is Python's sorted() over (tile, depth bits, emit index)
    and itertools.accumulate over the counts."""
    import scenegen
    views = []
    for k, (w, h) in enumerate([(64, 48), (33, 20)]):
        u, v, z, r = scenegen.random_projected(200, w, h, seed=10 + k, depth_ties=ties)
        views.append(dict(u=u, v=v, z=z, r=r, width=w, height=h))
    bins = O.bin_sort_ref(views)
    entries = []
    base, nb = 0, 0
    for vw in views:
        TX, TY = O.tile_grid(vw["width"], vw["height"])
        for g in range(200):
            for ty in range(TY):
                for tx in range(TX):
                    if O.tile_member_f32(vw["u"][g:g + 1], vw["v"][g:g + 1], vw["r"][g:g + 1],
                                         np.array([tx]), np.array([ty]), vw["width"], vw["height"])[0] \
                            and vw["r"][g] > 0:
                        entries.append((base + ty * TX + tx, int(vw["z"][g:g + 1].view(np.uint32)[0]),
                                        len(entries), nb + g))
        base += TX * TY
        nb += 200
    srt = sorted(entries, key=lambda e: (e[0], e[1], e[2]))
    assert [(e[0] << 32) | e[1] for e in srt] == bins.keys.tolist()
    assert [e[2] for e in srt] == bins.emit_index.tolist()
    assert [e[3] for e in srt] == bins.pidx.tolist()
    counts = np.zeros(400, np.int64)
    for e in entries:
        counts[e[3]] += 1
    assert counts.tolist() == bins.tile_count.tolist()
    assert [0] + list(itertools.accumulate(counts.tolist()))[:-1] == bins.offsets.tolist()
    for t in range(base):
        idx = [i for i, e in enumerate(srt) if e[0] == t]
        exp = (idx[0], idx[-1] + 1) if idx else (0, 0)
        assert tuple(bins.ranges[t].tolist()) == exp
    if ties:
        assert len(set(e[1] for e in entries)) <= 4


# ---------------------------------------------------------------------------------------
# Spherical harmonics
# ---------------------------------------------------------------------------------------

def _sphere_quadrature(nt=24, nphi=48):
    zq, wq = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    Z, P = np.meshgrid(zq, phi, indexing="ij")
    W = np.repeat(wq[:, None], nphi, axis=1) * (2 * np.pi / nphi)
    st = np.sqrt(1 - Z ** 2)
    d = np.stack([st * np.cos(P), st * np.sin(P), Z]).reshape(3, -1)
    return d, W.ravel()


def test_sh_orthonormal_by_quadrature():
    """Catches: a wrong normalisation constant, a wrong Legendre derivative order, a
    cos/sin mix-up. Gauss-Legendre x uniform-phi quadrature is exact for these degrees."""
    d, w = _sphere_quadrature()
    Y = O.sh_basis(3, d)
    G = (Y * w[None, :]) @ Y.T
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_addition_theorem_and_sign_convention():
    """Catches: a per-m scale error (sum over m of Y_lm^2 = (2l+1)/(4 pi) for every
    direction) and a Condon-Shortley sign (Y_{1,-1}, Y_{1,0}, Y_{1,1} = c (y, z, x),
    c = sqrt(3/(4 pi)))."""
    rng = np.random.default_rng(0)
    d = rng.normal(size=(3, 50))
    d /= np.linalg.norm(d, axis=0)
    Y = O.sh_basis(3, d)
    for l in range(4):
        np.testing.assert_allclose((Y[l * l:(l + 1) ** 2] ** 2).sum(0), (2 * l + 1) / (4 * np.pi), rtol=1e-12)
    c = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y[1:4], c * d[[1, 2, 0]], rtol=1e-12)
    np.testing.assert_allclose(Y[0], 0.5 / math.sqrt(math.pi), rtol=1e-12)


def test_sh_gradient_finite_difference():
    """Catches: a wrong derivative of (x + iy)^m or of the Legendre factor."""
    rng = np.random.default_rng(1)
    d = rng.normal(size=(3, 20))
    d /= np.linalg.norm(d, axis=0)
    Gr = O.sh_basis_grad(3, d)
    h = 1e-6
    for a in range(3):
        e = np.zeros((3, 1))
        e[a] = h
        fd = (O.sh_basis(3, d + e) - O.sh_basis(3, d - e)) / (2 * h)
        np.testing.assert_allclose(Gr[:, a], fd, atol=1e-8)


def test_sh_colour_direction_dependence():
    """Catches: SH evaluated in camera space or with the direction reversed. A degree-1
    coefficient on Y_{1,1} (x) brightens the particle seen from +x (view direction
    mu - eye has negative x) less than from -x."""
    sc = Scene(pos=np.zeros((3, 1), np.float32), scale=np.full(1, 0.05, np.float32),
               opacity=np.full(1, 0.9, np.float32), color=np.zeros((12, 1), np.float32), sh_degree=1)
    sc.color[0:3] = 0.5
    sc.color[9:12] = 0.2          # coefficient k = 3 (l=1, m=1) for each channel
    from_px = look_at_camera((3.0, 0, 0), width=16, height=16)
    from_nx = look_at_camera((-3.0, 0, 0), width=16, height=16)
    c = math.sqrt(3 / (4 * math.pi))
    assert O.project64(sc, from_px).rgb[0, 0] == pytest.approx(0.5 - 0.2 * c, rel=1e-6)
    assert O.project64(sc, from_nx).rgb[0, 0] == pytest.approx(0.5 + 0.2 * c, rel=1e-6)


# ---------------------------------------------------------------------------------------
# Gradients: FP64 analytic vs central finite differences
# ---------------------------------------------------------------------------------------

def _fd_scene(seed, n, deg):
    rng = np.random.default_rng(seed)
    K = (deg + 1) ** 2
    pos = np.stack([rng.uniform(-0.25, 0.25, n), rng.uniform(-0.25, 0.25, n), rng.uniform(-0.3, 0.3, n)])
    color = np.zeros((3 * K, n))
    color[0:3] = rng.uniform(0.1, 0.9, (3, n))
    color[3:] = rng.normal(0, 0.15, (3 * K - 3, n))
    return Scene(pos=pos, scale=np.exp(rng.normal(math.log(0.07), 0.3, n)),
                 opacity=1 / (1 + np.exp(-rng.normal(0.5, 1.5, n))), color=color, sh_degree=deg)


def _loss(scene, cams, Ws, bg):
    tot = 0.0
    for cam, W in zip(cams, Ws):
        img, _ = O.render64_untiled(O.project64(scene, cam), cam.width, cam.height, bg)
        tot += float((img * W).sum())
    return tot


@pytest.mark.parametrize("deg", [0, 2])
def test_gradients_match_central_differences(deg):
    """Catches: any sign, factor or missing term in the backward pass (compositing,
    alpha clamp, kernel, projection, SH chain through the view direction), and views of
    one scene not being summed. L = sum_v <W_v, C_v> with random W."""
    sc = _fd_scene(11 + deg, 10, deg)
    cams = [look_at_camera((0.3, 0.2, 2.0), width=24, height=20),
            look_at_camera((-0.5, 0.1, 1.8), width=20, height=24)]
    rng = np.random.default_rng(3)
    Ws = [rng.normal(size=(3, c.height, c.width)) for c in cams]
    bg = (0.1, 0.2, 0.05)
    g = O.scene_grads(sc, cams, Ws, bg)
    sigs0 = [O.decision_signature(O.project64(sc, c), c.width, c.height, bg) for c in cams]
    checked = skipped = 0
    for name in ("pos", "scale", "opacity", "color"):
        arr = getattr(sc, name)
        for idx in np.ndindex(arr.shape):
            h = 1e-6 * max(1.0, abs(arr[idx]))
            vals = []
            same = True
            for sgn in (1, -1):
                arr[idx] += sgn * h
                vals.append(_loss(sc, cams, Ws, bg))
                same &= all(O.decision_signature(O.project64(sc, c), c.width, c.height, bg) == s0
                            for c, s0 in zip(cams, sigs0))
                arr[idx] -= sgn * h
            if not same:
                skipped += 1
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = g[name][idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)
            checked += 1
    assert checked > 0.9 * (checked + skipped)
    assert np.abs(g["pos"]).max() > 1e-3 and np.abs(g["opacity"]).max() > 1e-3
