"""Pins of the oracle's handling of borderline decisions ("several results are correct").

An FP32 walk of eq. 4 may take a decision differently from the FP64 walk when the FP64
value lies within rounding of the threshold: alpha against 1/255 (the compact support of
eq. 2), T against 1e-4 (termination), and the order of two depths one FP32 ulp apart.
``pixel_outcomes`` lists every correct result of such a pixel; these tests fix it with
closed forms of eq. 4 written out by hand for one decision at a time, with brute force,
and with the plain walk where nothing is in band. A plausible mistake - a missing branch,
a branch on the wrong entry, a stop taken one entry late, a band formula that does not
bound the change it claims to - fails one of them.
"""
import math

import numpy as np
import pytest

import oracle as O
from scenegen import uniform_cube_scene, look_at_camera

A_MIN = 1.0 / 255.0


def one_pixel(parts):
    """Arrays for particles given as (dx, o, rgb) around the pixel centre (0.5, 0.5), s = 1."""
    n = len(parts)
    u = np.array([0.5 + p[0] for p in parts], np.float64)
    v = np.full(n, 0.5)
    s = np.ones(n)
    o = np.array([p[1] for p in parts], np.float64)
    rgb = np.array([p[2] for p in parts], np.float64).T.reshape(3, n)
    return u, v, s, o, rgb


def has(outs, C, T, tol=1e-13):
    return any(np.abs(c - np.asarray(C)).max() <= tol and abs(t - T) <= tol * max(1.0, T) for c, t, _ in outs)


def test_nothing_in_band_gives_the_plain_walk_only():
    """Catches: spurious alternatives, or outcomes that differ from the walk itself. On a
    random tiled scene, every pixel that the walk does not flag has exactly one outcome,
    equal to the walk's (C, T, n_last); every flagged pixel's outcomes include the walk's."""
    sc = uniform_cube_scene(300, seed=3, log_scale_mean=math.log(0.06), log_scale_std=0.4)
    cam = look_at_camera((0.2, 0.1, 3.0), width=40, height=32)
    pr = O.project64(sc, cam)
    bins = O.bin_sort_ref(O.f32_views([pr], [cam]))
    TX, TY = O.tile_grid(cam.width, cam.height)
    n_flag = n_plain = 0
    for ty in range(TY):
        for tx in range(TX):
            a, b = bins.ranges[ty * TX + tx]
            seq = bins.pidx[a:b].astype(np.int64)
            X, Y = O.tile_pixels(tx, ty, cam.width, cam.height)
            C, T, nl, tr = O.composite_pixels(X + 0.5, Y + 0.5, seq, pr.u, pr.v, pr.s, pr.opacity, pr.rgb,
                                              (0.1, 0.2, 0.3), trace=True, alpha_band=2.0 ** -8, term_band=2.0 ** -4)
            fl = tr["near_alpha"] | tr["near_term"]
            for p in range(X.shape[0]):
                outs, ok = O.pixel_outcomes(X[p] + 0.5, Y[p] + 0.5, seq, pr.u, pr.v, pr.s, pr.opacity, pr.rgb,
                                            (0.1, 0.2, 0.3), alpha_band=2.0 ** -8, term_band=2.0 ** -4)
                assert ok
                assert has(outs, C[:, p], T[p])
                if not fl[p]:
                    assert len(outs) == 1 and outs[0][2] == nl[p]
                    n_plain += 1
                else:
                    n_flag += 1
    assert n_plain > 500 and n_flag > 0      # wide bands here, so that both kinds occur


def test_alpha_decision_taken_both_ways_closed_form():
    """Catches: an in-band entry not branched, or branched on the wrong entry. Front entry
    alpha1 = 0.5; the entry behind it has alpha2 = (1/255)(1 + 1e-7), inside the band: the
    outcomes are exactly c1 a1 + c2 a2 (1 - a1) (T = (1 - a1)(1 - a2)) and c1 a1 (T = 1 - a1)."""
    a2 = A_MIN * (1 + 1e-7)
    d = math.sqrt(math.log(0.5 / a2))
    c1, c2 = (0.2, 0.4, 0.6), (0.9, 0.1, 0.5)
    u, v, s, o, rgb = one_pixel([(0.0, 0.5, c1), (d, 0.5, c2)])
    outs, ok = O.pixel_outcomes(0.5, 0.5, [0, 1], u, v, s, o, rgb)
    assert ok and len(outs) == 2
    c1, c2 = np.array(c1), np.array(c2)
    assert has(outs, c1 * 0.5 + c2 * a2 * 0.5, 0.5 * (1 - a2))
    assert has(outs, c1 * 0.5, 0.5)
    # the same entry far outside the band: one outcome
    u2, *_ = one_pixel([(0.0, 0.5, c1), (d * 1.01, 0.5, c2)])
    outs, ok = O.pixel_outcomes(0.5, 0.5, [0, 1], u2, v, s, o, rgb)
    assert ok and len(outs) == 1


def test_stop_decision_taken_both_ways_closed_form():
    """Catches: a stop taken one entry early or late, or the end of the list lost. With
    alpha 0.9, 0.9 and then a3 = 0.99 (1 - 1e-11), T after the third entry is
    1e-4 (1 + ~1e-9): in band. The walk may stop there, or composite the fourth entry
    (alpha 0.5) and stop after it (T clearly below 1e-4), never later."""
    a3 = 0.99 * (1 - 1e-11)
    cs = [np.array(c) for c in ((0.1, 0.2, 0.3), (0.4, 0.5, 0.6), (0.7, 0.8, 0.9), (1.0, 0.0, 0.5), (0.3, 0.3, 0.3))]
    u, v, s, o, rgb = one_pixel([(0.0, 0.9, cs[0]), (0.0, 0.9, cs[1]), (0.0, a3, cs[2]), (0.0, 0.5, cs[3]),
                                 (0.0, 0.5, cs[4])])
    outs, ok = O.pixel_outcomes(0.5, 0.5, [0, 1, 2, 3, 4], u, v, s, o, rgb)
    assert ok and len(outs) == 2
    T1, T2 = 0.1, 0.01
    T3 = T2 * (1 - a3)
    C3 = cs[0] * 0.9 + cs[1] * 0.9 * T1 + cs[2] * a3 * T2
    assert abs(T3 / 1e-4 - 1) < 1e-8
    assert has(outs, C3, T3)
    assert has(outs, C3 + cs[3] * 0.5 * T3, T3 * 0.5)
    assert sorted(x[2] for x in outs) == [3, 4]


def test_insignificant_flip_kept_on_the_fp64_side():
    """Catches: branching on decisions that cannot matter (combinatorial blow-up). Behind
    alpha 0.99 and 0.98 (T = 2e-4) an in-band entry changes the colour by at most
    2 (1/255)(2e-4) < 1e-5: one outcome, the plain walk's."""
    u, v, s, o, rgb = one_pixel([(0.0, 0.99, (1, 1, 1)), (0.0, 0.98, (1, 1, 1)),
                                 (math.sqrt(math.log(0.5 * 255 / (1 + 1e-7))), 0.5, (1, 1, 1))])
    outs, ok = O.pixel_outcomes(0.5, 0.5, [0, 1, 2], u, v, s, o, rgb)
    C, T, nl = O.composite_pixels(np.array([0.5]), np.array([0.5]), [0, 1, 2], u, v, s, o, rgb, (0, 0, 0))
    assert ok and len(outs) == 1
    assert np.abs(outs[0][0] - C[:, 0]).max() < 1e-15 and outs[0][1] == T[0]


def test_depth_order_taken_both_ways_closed_form():
    """Catches: a missing order branch. Two entries whose FP32 depths are one ulp apart may
    be composited in either order: c1 a1 + c2 a2 (1 - a1) and c2 a2 + c1 a1 (1 - a2)."""
    c1, c2 = np.array((0.9, 0.1, 0.1)), np.array((0.1, 0.1, 0.9))
    u, v, s, o, rgb = one_pixel([(0.0, 0.5, c1), (0.0, 0.3, c2)])
    z = np.array([2.0, np.nextafter(np.float32(2.0), np.float32(3.0))], np.float32)
    outs, ok = O.pixel_outcomes(0.5, 0.5, [0, 1], u, v, s, o, rgb, z32=z)
    assert ok and len(outs) == 2
    assert has(outs, c1 * 0.5 + c2 * 0.3 * 0.5, 0.35)
    assert has(outs, c2 * 0.3 + c1 * 0.5 * 0.7, 0.35)
    z[1] = np.float32(2.001)
    outs, ok = O.pixel_outcomes(0.5, 0.5, [0, 1], u, v, s, o, rgb, z32=z)
    assert ok and len(outs) == 1


def test_unresolved_beyond_the_branch_limit():
    """Catches: silent truncation of the enumeration. Thirteen significant in-band entries
    exceed a limit of twelve decisions: reported unresolved, with no outcome."""
    d = math.sqrt(math.log(0.5 * 255 / (1 + 1e-7)))
    u, v, s, o, rgb = one_pixel([(d, 0.5, (1, 1, 1))] * 13)
    outs, ok = O.pixel_outcomes(0.5, 0.5, list(range(13)), u, v, s, o, rgb, max_branch=12)
    assert not ok and outs == []
    outs, ok = O.pixel_outcomes(0.5, 0.5, list(range(4)), u, v, s, o, rgb, max_branch=12)
    # 0..4 of four equal entries composited: five colours (n_last tells the subsets apart)
    assert ok and len({round(float(c[0]), 12) for c, _, _ in outs}) == 5 and len(outs) == 11


def test_position_band_bounds_the_kernel_change_brute_force():
    """Catches: a band growth that does not bound what a shifted centre does. For random
    offsets, scales and centre errors e, every shift of the centre within [-e, e]^2 changes
    d^2 / s^2 (hence ln alpha) by at most (2 (|dx| + |dy|) e + 2 e^2) / s^2."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        dx, dy = rng.uniform(-6, 6, 2)
        s = rng.uniform(0.2, 4)
        e = rng.uniform(1e-5, 0.05)
        grow = (2 * (abs(dx) + abs(dy)) * e + 2 * e * e) / (s * s)
        g = np.linspace(-e, e, 41)
        sx, sy = np.meshgrid(g, g)
        change = np.abs(((dx - sx) ** 2 + (dy - sy) ** 2) - (dx * dx + dy * dy)) / (s * s)
        assert change.max() <= grow * (1 + 1e-12)


def test_position_band_flags_and_branches():
    """Catches: pos_err ignored by the flags or by the outcomes. An entry with
    alpha = (1/255)(1 + 1e-3) is outside the rounding band, but a centre error of 0.01 px at
    distance ~2.3 s changes alpha by ~5%: flagged, and both sides are outcomes."""
    d = math.sqrt(math.log(0.5 * 255 / (1 + 1e-3)))
    u, v, s, o, rgb = one_pixel([(0.0, 0.5, (0.2, 0.2, 0.2)), (d, 0.5, (1, 0, 0))])
    C, T, nl, tr = O.composite_pixels(np.array([0.5]), np.array([0.5]), [0, 1], u, v, s, o, rgb, (0, 0, 0),
                                      trace=True)
    assert not tr["near_alpha"][0]
    pe = np.full(2, 0.01)
    C, T, nl, tr = O.composite_pixels(np.array([0.5]), np.array([0.5]), [0, 1], u, v, s, o, rgb, (0, 0, 0),
                                      trace=True, pos_err=pe)
    assert tr["near_alpha"][0]
    outs, ok = O.pixel_outcomes(0.5, 0.5, [0, 1], u, v, s, o, rgb, pos_err=pe)
    assert ok and len(outs) == 2


def test_footprint_uncertainty_bounds_the_fp32_rounding():
    """Catches: a bound in the wrong units or one that misses the rounding into the next
    binade. For every visible particle, both FP32 neighbours of each FP64 coordinate (the
    two values a rounding can give) lie within the bound of it."""
    sc = uniform_cube_scene(400, seed=1)
    cam = look_at_camera((0, 0, 2.2), width=1920, height=1080)
    pr = O.project64(sc, cam)
    pe, z32 = O.footprint_uncertainty(pr)
    vis = pr.visible
    for c in (pr.u[vis], pr.v[vis]):
        lo = c.astype(np.float32)
        lo = np.where(lo.astype(np.float64) > c, np.nextafter(lo, np.float32(-np.inf)), lo)
        hi = np.nextafter(lo, np.float32(np.inf))
        near = np.where(np.abs(lo - c) <= np.abs(hi - c), lo, hi).astype(np.float64)
        assert (np.abs(near - c) <= pe[vis]).all()
    assert (pe[vis] < 1e-3).all()
    np.testing.assert_array_equal(z32[vis], pr.z[vis].astype(np.float32))


@pytest.mark.parametrize("seed", [0, 1])
def test_screen_gradients_tiled_equal_untiled(seed):
    """Catches: a tiling mistake in the backward (an entry's gradient summed over a tile it
    does not belong to, or a pixel missed). Per-particle screen gradients summed tile by
    tile equal those of every pixel walking every particle, up to the summation order."""
    sc = uniform_cube_scene(120, seed=seed, log_scale_mean=math.log(0.08), log_scale_std=0.4)
    cam = look_at_camera((0.1, -0.2, 3.0), width=37, height=29)
    pr = O.project64(sc, cam)
    bins = O.bin_sort_ref(O.f32_views([pr], [cam]))
    dC = np.random.default_rng(seed).normal(size=(3, cam.height, cam.width))
    gt = O.screen_grads_tiled(pr.u, pr.v, pr.s, pr.opacity, pr.rgb, bins, 0, cam.width, cam.height, dC,
                              (0.2, 0.1, 0.0))
    gu = O.screen_grads_untiled(pr, cam.width, cam.height, dC, (0.2, 0.1, 0.0))
    for k in ("du", "dv", "ds", "do", "drgb"):
        scale = np.abs(gu[k]).max()
        assert scale > 0
        np.testing.assert_allclose(gt[k], gu[k], rtol=1e-10, atol=1e-12 * scale)
