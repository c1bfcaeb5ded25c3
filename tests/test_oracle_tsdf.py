"""Pins of the oracle's projective TSDF update (Sec. IV-C.2, Eq. 5).

Closed form: a sensor inside a sphere of radius R centred on it reads R on every pixel,
so the projective distance of every voxel is psi = R - |x - o| whichever pixel it maps
to; after one frame D = min(psi, tau) and W = min((psi + tau) / (2 tau), 1), and after n
identical frames W = n w with D unchanged.  The nearest-pixel choice is pinned against a
brute-force angular search and the boundary tie rule; the invariants of Eq. 5 (bounded
D, monotone W, untouched voxels unchanged) on a real scene.
"""
import numpy as np
import pytest

import oracle
import synth

NU, TAU = 0.2, 0.6


def _tilted_pose():
    a = np.deg2rad(20.0)
    Rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    return synth.pose_matrix(synth.rot_z(np.deg2rad(30.0)) @ Rx, [1.3, -2.1, 0.4])


def _voxel_centres(b):
    i = np.arange(512)
    loc = np.stack([i & 7, (i >> 3) & 7, i >> 6], axis=1)
    return (np.asarray(b)[None, :] * 8 + loc).astype(np.float64)


@pytest.mark.parametrize("pose", ["identity", "tilted"])
def test_sphere_closed_form(pose):
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    T = synth.pose_matrix(np.eye(3), [0, 0, 0]) if pose == "identity" else _tilted_pose()
    R = 4.0
    m = oracle.OracleMap(NU, TAU, 3)
    rimg = synth.constant_range(lidar, R)
    assert m.integrate_lidar(lidar, rimg, T) == oracle.OK
    Td = T.astype(np.float64)
    nu = float(np.float32(NU))
    tau = float(np.float32(TAU))
    top = lidar.elev_rad[0] + 0.5 * (lidar.elev_rad[0] - lidar.elev_rad[1])
    bot = lidar.elev_rad[-1] - 0.5 * (lidar.elev_rad[-2] - lidar.elev_rad[-1])
    n_checked = n_updated = 0
    for b in m.touched():
        blk = m.block(b)
        x = _voxel_centres(b) * nu
        p = (x - Td[:3, 3]) @ Td[:3, :3]          # R^T (x - t)
        dist = np.linalg.norm(p, axis=1)
        el = np.arctan2(p[:, 2], np.hypot(p[:, 0], p[:, 1]))
        psi = R - dist
        in_fov = (el < top) & (el > bot)
        expect = in_fov & (psi >= -tau)
        clear = (np.abs(el - top) > 1e-5) & (np.abs(el - bot) > 1e-5) & (np.abs(psi + tau) > 1e-4)
        w = np.minimum((psi + tau) / (2 * tau), 1.0)
        sel = expect & clear
        np.testing.assert_allclose(blk["D"][sel], np.minimum(psi, tau)[sel], atol=2e-6)
        np.testing.assert_allclose(blk["W"][sel], w[sel], atol=2e-6)
        bclear = sel & (np.abs(np.abs(psi) - tau) > 1e-5)
        np.testing.assert_array_equal(blk["band"][bclear].astype(bool), (np.abs(psi) <= tau)[bclear])
        off = ~expect & clear
        assert np.all(blk["W"][off] == 0) and np.all(blk["D"][off] == 0)
        n_checked += int(clear.sum())
        n_updated += int(sel.sum())
    assert n_updated > 10000 and n_checked > n_updated
    assert m.stats()["updates"] >= n_updated


def test_repeated_frames_accumulate_weight():
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    T = _tilted_pose()
    rimg = synth.constant_range(lidar, 3.0)
    m = oracle.OracleMap(NU, TAU, 3)
    m.integrate_lidar(lidar, rimg, T)
    first = {tuple(b): m.block(b) for b in m.touched()}
    n = 5
    for _ in range(n - 1):
        assert m.integrate_lidar(lidar, rimg, T) == oracle.OK
    for b, d1 in first.items():
        dn = m.block(b)
        np.testing.assert_allclose(dn["W"], n * d1["W"], rtol=1e-6)
        np.testing.assert_allclose(dn["D"], d1["D"], atol=1e-6)


def _uniform_boundaries(lidar):
    e = lidar.elev_rad.astype(np.float64)
    C = lidar.cols
    col_b = np.pi - (np.arange(C) - 0.5) * (2 * np.pi / C)
    row_b = np.concatenate([[e[0] + 0.5 * (e[0] - e[1])], 0.5 * (e[:-1] + e[1:]), [e[-1] - 0.5 * (e[-2] - e[-1])]])
    return col_b, row_b


def test_pixel_choice_is_nearest_pixel():
    lidar = synth.uniform_lidar(64, 2048, 2.0, -24.8, 100.0)
    rng = np.random.Generator(np.random.PCG64(9))
    col_b, row_b = _uniform_boundaries(lidar)
    phis = np.pi - np.arange(lidar.cols) * (2 * np.pi / lidar.cols)
    n = 0
    for _ in range(3000):
        az = rng.uniform(-np.pi, np.pi)
        el = rng.uniform(-0.45, 0.05)
        rr = rng.uniform(0.5, 80)
        p = np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)]) * rr
        p32 = p.astype(np.float32)
        pd = p32.astype(np.float64)
        az = np.arctan2(pd[1], pd[0])
        el = np.arctan2(pd[2], np.hypot(pd[0], pd[1]))
        dcol = np.abs(np.angle(np.exp(1j * (az - col_b))))
        if dcol.min() < 1e-6 or np.abs(el - row_b).min() < 1e-6:
            continue
        got = oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, p32)
        if el > row_b[0] or el < row_b[-1]:
            assert got is None
            continue
        want_c = int(np.argmin(np.abs(np.angle(np.exp(1j * (az - phis))))))
        want_r = int(np.argmin(np.abs(el - lidar.elev_rad.astype(np.float64))))
        assert got == (want_r, want_c), (p32, got, want_r, want_c)
        n += 1
    assert n > 2000


def test_pixel_boundary_ties_go_to_higher_index():
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    col_b, row_b = _uniform_boundaries(lidar)
    for c in (1, 17, 450, 899, 1799):
        bx, by = np.float32(np.cos(col_b[c])), np.float32(np.sin(col_b[c]))
        p = np.array([bx * 4, by * 4, 0.0], np.float32)  # exactly on boundary c (power-of-2 scale)
        assert oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, p)[1] == c
    for k in (1, 5, 8, 15):
        rc, rs = np.float32(np.cos(row_b[k])), np.float32(np.sin(row_b[k]))
        p = np.array([rc * 8, 0.0, rs * 8], np.float32)  # on row boundary k, azimuth 0
        got = oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, p)
        assert got == (k, lidar.cols // 2)
    # on the bottom boundary: outside (the next row would not exist); on the top: row 0
    rc, rs = np.float32(np.cos(row_b[16])), np.float32(np.sin(row_b[16]))
    assert oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, np.array([rc * 8, 0, rs * 8], np.float32)) is None
    rc, rs = np.float32(np.cos(row_b[0])), np.float32(np.sin(row_b[0]))
    assert oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, np.array([rc * 8, 0, rs * 8], np.float32))[0] == 0
    # straight up / at the sensor: no pixel
    assert oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, np.array([0, 0, 1], np.float32)) is None


def test_invariants_on_scene():
    """|D| <= tau, W monotone and <= frame count, voxels outside T_k unchanged."""
    w = synth.tiny_workload()
    m = oracle.OracleMap(w.voxel, w.trunc, w.n_classes)
    tau = np.float32(w.trunc)
    prev = {}
    rng = np.random.Generator(np.random.PCG64(2))
    for k in range(4):
        R = synth.rot_z(rng.normal(0, 0.05))
        T = synth.pose_matrix(R, rng.normal(0, 0.3, size=3))
        f = w.frame(0, with_labels=False)
        assert m.integrate_lidar(w.lidar, f.range, T) == oracle.OK
        touched = {tuple(b) for b in m.touched()}
        cur = {tuple(b): m.block(b) for b in m.block_coords()}
        for b, d in cur.items():
            assert np.all(np.abs(d["D"]) <= tau * (1 + 2 ** -20))
            assert np.all(d["W"] <= k + 1 + 1e-6)
            if b in prev:
                assert np.all(d["W"] >= prev[b]["W"])
                if b not in touched:
                    np.testing.assert_array_equal(d["D"], prev[b]["D"])
                    np.testing.assert_array_equal(d["W"], prev[b]["W"])
            else:
                assert b in touched
        prev = cur
