"""Pins of the oracle's measurement preprocessing (Eq. 3): depth image D = F r and height
image H = F (z + O) of a sensor-frame point cloud.

Closed forms: a scan rebuilt as points, one on every pixel's ray (Eq. 3's pixel centres),
maps back one point per pixel with D = |p| and H = z; the scalars F and O act as written.
The depth buffer keeps the nearest point and, between points of bit-identical range, the
first in input order (seen through H).  Invalid points (non-finite, r = 0, r > r_max,
outside the vertical field of view) write nothing.  A small random cloud matches a
per-pixel brute-force minimum over the points the pinned pixel rule assigns there.
"""
import numpy as np

import oracle
import synth


def _norm32(p):
    p = np.asarray(p, dtype=np.float32).reshape(-1, 3)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    return np.sqrt((x * x + y * y) + z * z).astype(np.float32)


def test_scan_round_trip_one_point_per_pixel():
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    rng = np.random.Generator(np.random.PCG64(11))
    r = rng.uniform(1.0, 35.0, size=lidar.rows * lidar.cols)
    pts = (lidar.directions() * r[:, None]).astype(np.float32)
    D, H, n = oracle.range_image(lidar.rows, lidar.cols, lidar.elev_rad, lidar.r_max, pts)
    assert n == lidar.rows * lidar.cols  # a bijection: no pixel empty, none shared
    np.testing.assert_array_equal(D.reshape(-1), _norm32(pts))
    np.testing.assert_array_equal(H.reshape(-1), pts[:, 2])
    np.testing.assert_allclose(D.reshape(-1), r, rtol=1e-6)


def test_scalars_F_and_O():
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    rng = np.random.Generator(np.random.PCG64(12))
    pts = (lidar.directions() * rng.uniform(1.0, 35.0, size=(lidar.rows * lidar.cols, 1))).astype(np.float32)
    D1, H1, _ = oracle.range_image(lidar.rows, lidar.cols, lidar.elev_rad, lidar.r_max, pts)
    F, O = np.float32(250.0), np.float32(1.73)
    D, H, _ = oracle.range_image(lidar.rows, lidar.cols, lidar.elev_rad, lidar.r_max, pts, F=F, O=O)
    np.testing.assert_array_equal(D, (F * D1).astype(np.float32))
    np.testing.assert_array_equal(H, (F * (H1 + O).astype(np.float32)).astype(np.float32))


def _same_range_pair():
    """Two points on one pixel with bit-identical fp32 range and different z."""
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    d = lidar.directions()[5 * lidar.cols + 700]
    rng = np.random.Generator(np.random.PCG64(13))
    cand = (10.0 * (d[None, :] + rng.normal(0.0, 1e-4, size=(4000, 3)))).astype(np.float32)
    r = _norm32(cand)
    for i in range(len(cand)):
        same = np.nonzero((r == r[i]) & (cand[:, 2] != cand[i, 2]))[0]
        for j in same:
            pi = oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, cand[i])
            pj = oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, cand[j])
            if pi is not None and pi == pj:
                return lidar, cand[i], cand[j], pi
    raise AssertionError("no equal-range pair found")


def test_nearest_point_wins_and_ties_keep_the_first():
    lidar, a, b, (row, col) = _same_range_pair()
    far = (a * np.float32(1.5)).astype(np.float32)
    near = (a * np.float32(0.5)).astype(np.float32)
    assert oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, near) == (row, col)
    for order, want_z in (([far, a, b], a[2]), ([far, b, a], b[2]), ([a, near, b], near[2])):
        D, H, n = oracle.range_image(lidar.rows, lidar.cols, lidar.elev_rad, lidar.r_max, np.stack(order))
        assert n == 1
        assert H[row, col] == want_z
        assert D[row, col] == min(_norm32(np.stack(order)))


def test_invalid_points_write_nothing():
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    nan = np.float32(np.nan)
    pts = np.array([[nan, 1, 0], [np.inf, 0, 0], [0, 0, 0],
                    [50.0, 0, 0],            # beyond r_max
                    [5.0, 0, 5.0],           # 45 degrees up: above the field of view
                    [5.0, 0, -5.0],          # 45 degrees down: below it
                    [0, 0, 3.0]],            # on the axis: no azimuth
                   dtype=np.float32)
    D, H, n = oracle.range_image(lidar.rows, lidar.cols, lidar.elev_rad, lidar.r_max, pts)
    assert n == 0 and not D.any() and not H.any()


def test_small_cloud_brute_force():
    lidar = synth.uniform_lidar(8, 64, 10.0, -10.0, 20.0)
    rng = np.random.Generator(np.random.PCG64(14))
    n = 3000
    az = rng.uniform(-np.pi, np.pi, n)
    el = rng.uniform(np.deg2rad(-13.0), np.deg2rad(13.0), n)
    rr = rng.uniform(0.5, 22.0, n)
    pts = np.stack([rr * np.cos(el) * np.cos(az), rr * np.cos(el) * np.sin(az), rr * np.sin(el)], 1)
    pts = pts.astype(np.float32)
    pts[rng.choice(n, 300)] = pts[rng.choice(n, 300)]  # repeated points
    D, H, written = oracle.range_image(lidar.rows, lidar.cols, lidar.elev_rad, lidar.r_max, pts, F=2.0, O=0.5)
    r = _norm32(pts)
    best = {}
    for i in range(n):
        if not (0.0 < r[i] <= np.float32(lidar.r_max)):
            continue
        px = oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, pts[i])
        if px is None:
            continue
        if px not in best or r[i] < r[best[px]]:
            best[px] = i
    assert written == len(best)
    want_D = np.zeros_like(D)
    want_H = np.zeros_like(H)
    for (k, c), i in best.items():
        want_D[k, c] = np.float32(2.0) * r[i]
        want_H[k, c] = np.float32(2.0) * (pts[i, 2] + np.float32(0.5))
    np.testing.assert_array_equal(D, want_D)
    np.testing.assert_array_equal(H, want_H)
