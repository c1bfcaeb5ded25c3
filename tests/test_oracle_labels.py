"""Pins of the oracle's label fusion (Sec. IV-C.3, Eq. 6).

Reading: a hard label per pixel with a symmetric likelihood (p for the observed class,
(1-p)/(L-1) for the others).  The recursive Bayes posterior after the votes is then
proportional to p^n_l ((1-p)/(L-1))^(N-n_l), whose argmax is the argmax of the vote
counts n_l for any p > 1/L; ties go to the lowest class id.  Here a textbook recursive
Bayes filter in fp64 (normalised product of prior and likelihood, one image at a time)
is run on the same vote sequences and must give the same most probable class.
"""
import numpy as np
import pytest

import oracle
import synth


def _sphere_map(L, R=3.0, lidar=None):
    lidar = lidar or synth.uniform_lidar(16, 360, 15.0, -15.0, 40.0)
    m = oracle.OracleMap(0.2, 0.6, L)
    T = synth.pose_matrix(np.eye(3), [0, 0, 0])
    assert m.integrate_lidar(lidar, synth.constant_range(lidar, R), T) == oracle.OK
    return m, T


def _visible(x, T, cam, margin=1e-3):
    """fp64 projection of world points into a pinhole camera (z forward); pixel or -1."""
    Td = T.astype(np.float64)
    p = (x - Td[:3, 3]) @ Td[:3, :3]
    z = p[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam.fx * p[:, 0] / z + cam.cx
        v = cam.fy * p[:, 1] / z + cam.cy
        ok = (z > 1e-6) & (u >= 0) & (u < cam.width) & (v >= 0) & (v < cam.height)
        near = (np.abs(u - np.round(u)) < margin) | (np.abs(v - np.round(v)) < margin) | (np.abs(z) < 1e-4)
    return ok, near, u, v


def _band_voxels(m):
    out = []
    for b in m.touched():
        blk = m.block(b)
        i = np.arange(512)
        v = np.stack([i & 7, (i >> 3) & 7, i >> 6], axis=1) + 8 * np.asarray(b)
        out.append((tuple(b), blk, v.astype(np.float64) * float(np.float32(0.2))))
    return out


def test_counts_exact_and_bayes_equivalence():
    L = 6
    m, _ = _sphere_map(L)
    rng = np.random.Generator(np.random.PCG64(4))
    cam = synth.Camera(640, 480, 120.0, 120.0, 320.0, 240.0)
    seq = []
    for k in range(14):
        yaw = rng.uniform(-np.pi, np.pi)
        T = synth.pose_matrix(synth.rot_z(yaw) @ synth.camera_yaw(0.0), [0, 0, 0])
        l = int(rng.integers(0, L)) if k % 5 else 255  # every fifth image is 'ignore'
        seq.append((T, l))
        assert m.integrate_labels(cam, np.full((480, 640), l, np.uint8), T) == oracle.OK
    n_voxels = 0
    for b, blk, x in _band_voxels(m):
        want = np.zeros((L, 512), np.int64)
        amb = np.zeros(512, bool)
        sel = (blk["band"] > 0) & (blk["W"] > 0)
        for T, l in seq:
            ok, near, _, _ = _visible(x, T, cam)
            amb |= near & sel
            if l < L:
                want[l] += (ok & sel)
        good = sel & ~amb
        np.testing.assert_array_equal(blk["counts"][:, good], want[:, good])
        # textbook recursive Bayes filter, fp64, on each voxel's vote sequence
        for p in (0.6, 0.9):
            for j in np.nonzero(good)[0][::7]:
                post = np.full(L, 1.0 / L)
                for T, l in seq:
                    ok, _, _, _ = _visible(x[j:j + 1], T, cam)
                    if l < L and ok[0]:
                        like = np.full(L, (1 - p) / (L - 1))
                        like[l] = p
                        post = post * like
                        post /= post.sum()
                if want[:, j].sum() == 0:
                    assert blk["fused"][j] == 255
                    continue
                best = np.nonzero(post >= post.max() * (1 - 1e-9))[0].min()
                assert blk["fused"][j] == best
                n_voxels += 1
    assert n_voxels > 500


def test_single_class_counts_equal_frames():
    """A single-class world: each visible band voxel holds exactly (#images seeing it) votes."""
    L = 4
    m, T = _sphere_map(L, R=5.0)
    cam = synth.Camera(320, 240, 60.0, 60.0, 160.0, 120.0)
    Tc = synth.pose_matrix(synth.camera_yaw(0.0), [0, 0, 0])
    for _ in range(3):
        m.integrate_labels(cam, np.full((240, 320), 2, np.uint8), Tc)
    tot = 0
    for b, blk, x in _band_voxels(m):
        ok, near, _, _ = _visible(x, Tc, cam)
        sel = (blk["band"] > 0) & ~near
        np.testing.assert_array_equal(blk["counts"][2, sel], 3 * ok[sel])
        assert np.all(blk["counts"][[0, 1, 3]] == 0)
        assert np.all(blk["fused"][sel & ok] == 2)
        assert np.all(blk["fused"][~ok & ~near] == 255)
        tot += int((sel & ok).sum())
    assert tot > 100
    assert m.stats()["votes"] >= tot  # the last call's votes include the ambiguous voxels


def test_pixel_floor_and_image_rows():
    """Pixel (i, j) spans [i, i+1) x [j, j+1): a voxel's vote reads img[floor v][floor u]."""
    L = 200
    m, _ = _sphere_map(L, R=4.0)
    cam = synth.Camera(64, 48, 20.0, 20.0, 32.0, 24.0)
    Tc = synth.pose_matrix(synth.camera_yaw(0.3), [0, 0, 0])
    img = (np.arange(64 * 48) % 199).astype(np.uint8).reshape(48, 64)
    m.integrate_labels(cam, img, Tc)
    n = 0
    for b, blk, x in _band_voxels(m):
        ok, near, u, v = _visible(x, Tc, cam, margin=1e-4)
        sel = (blk["band"] > 0) & ok & ~near
        for j in np.nonzero(sel)[0]:
            l = img[int(np.floor(v[j])), int(np.floor(u[j]))]
            assert blk["counts"][l, j] == 1 and blk["counts"][:, j].sum() == 1
            assert blk["fused"][j] == l
            n += 1
    assert n > 100


def test_count_saturation_and_tie_rule():
    lidar = synth.uniform_lidar(2, 8, 1.0, -1.0, 10.0)
    m, _ = _sphere_map(10, R=2.0, lidar=lidar)
    cam = synth.Camera(16, 16, 2.0, 2.0, 8.0, 8.0)
    Tc = synth.pose_matrix(synth.camera_yaw(0.0), [0, 0, 0])
    img = lambda l: np.full((16, 16), l, np.uint8)  # noqa: E731
    for _ in range(65535):
        m.integrate_labels(cam, img(7), Tc)
    for _ in range(65536 + 3):
        m.integrate_labels(cam, img(2), Tc)
    seen = 0
    for b, blk, x in _band_voxels(m):
        sel = blk["counts"][7] > 0
        assert np.all(blk["counts"][7][sel] == 65535)
        assert np.all(blk["counts"][2][sel] == 65535)   # saturated
        assert np.all(blk["fused"][sel] == 2)           # tie at 65535: lowest id wins
        seen += int(sel.sum())
    assert seen > 0
    # the other order: the lower id first, the higher id never overtakes it
    m2, _ = _sphere_map(10, R=2.0, lidar=lidar)
    for _ in range(3):
        m2.integrate_labels(cam, img(1), Tc)
    for _ in range(3):
        m2.integrate_labels(cam, img(4), Tc)
    for b, blk, x in _band_voxels(m2):
        sel = blk["counts"][1] > 0
        assert np.all(blk["fused"][sel] == 1)
