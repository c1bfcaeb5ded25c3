"""Pins of the oracle's LiDAR-label fusion: a label range image (the scan's pixel layout)
under the scan's pose, each visible voxel of the last scan voting with the label at its
nearest pixel (Sec. V-A's point-cloud segmentation labels; the vote of Eq. 6 with hard
labels).

Closed forms: a constant label gives every visible voxel exactly one vote for it; a label
image that encodes the pixel gives each voxel the label of the pixel the pinned pixel rule
assigns to its centre; labels >= L give no vote; no scan, no fusion.
"""
import numpy as np

import oracle
import synth


def _scan(w):
    m = oracle.OracleMap(w.voxel, w.trunc, w.n_classes)
    f = w.frame(0, with_labels=False)
    assert m.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    return m, f


def _visible(m):
    out = []
    for b in m.touched():
        d = m.block(b)
        idx = np.nonzero((d["band"] != 0) & (d["W"] > 0))[0]
        out.append((tuple(int(v) for v in b), idx, d))
    return out


def test_constant_label_one_vote_per_visible_voxel():
    w = synth.tiny_workload()
    m, f = _scan(w)
    vis = _visible(m)
    n_vis = sum(len(i) for _, i, _ in vis)
    assert n_vis > 1000
    v0 = m.stats()["votes"]
    lab = np.full((w.lidar.rows, w.lidar.cols), 3, np.uint8)
    assert m.integrate_labels_lidar(w.lidar, lab, f.T_wl) == oracle.OK
    assert m.stats()["votes"] - v0 == n_vis
    for b, idx, _ in vis:
        d = m.block(b)
        assert np.all(d["counts"][3, idx] == 1) and np.all(d["fused"][idx] == 3)
        rest = np.delete(d["counts"], 3, axis=0)
        assert not rest[:, idx].any()


def test_pixel_encoding_label_is_the_nearest_pixel():
    w = synth.tiny_workload()
    m, f = _scan(w)
    R, C, L = w.lidar.rows, w.lidar.cols, w.n_classes
    rows, cols = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    lab = ((rows * 7 + cols) % L).astype(np.uint8)
    assert m.integrate_labels_lidar(w.lidar, lab, f.T_wl) == oracle.OK
    T = f.T_wl.astype(np.float32)
    nu = np.float32(w.voxel)
    rng = np.random.Generator(np.random.PCG64(5))
    checked = 0
    for b, idx, _ in _visible(m)[::7]:
        d = m.block(b)
        for li in rng.choice(idx, size=min(len(idx), 8), replace=False):
            v = np.array([8 * b[0] + (li & 7), 8 * b[1] + ((li >> 3) & 7), 8 * b[2] + (li >> 6)], np.float32)
            x = v * nu
            dd = (x - T[:3, 3]).astype(np.float32)
            p = np.array([(T[0, j] * dd[0] + T[1, j] * dd[1]) + T[2, j] * dd[2] for j in range(3)], np.float32)
            px = oracle.pixel_of(R, C, w.lidar.elev_rad, p)
            assert px is not None
            assert d["fused"][li] == lab[px], (b, li)
            checked += 1
    assert checked > 200


def test_labels_at_or_above_L_do_not_vote_and_no_scan():
    w = synth.tiny_workload()
    lab = np.full((w.lidar.rows, w.lidar.cols), 255, np.uint8)
    empty = oracle.OracleMap(w.voxel, w.trunc, w.n_classes)
    assert empty.integrate_labels_lidar(w.lidar, lab, np.eye(4, dtype=np.float32)) == oracle.NO_SCAN
    m, f = _scan(w)
    lab[:] = w.n_classes
    v0 = m.stats()["votes"]
    assert m.integrate_labels_lidar(w.lidar, lab, f.T_wl) == oracle.OK
    assert m.stats()["votes"] == v0


def test_segmentation_labels_accumulate_with_the_camera_rule():
    w = synth.tiny_workload()
    m, f = _scan(w)
    lab = w.lidar_labels(0)
    for _ in range(2):
        assert m.integrate_labels_lidar(w.lidar, lab, f.T_wl) == oracle.OK
    for b, idx, _ in _visible(m)[::5]:
        d = m.block(b)
        c = d["counts"][:, idx].astype(np.int64)
        tot = c.sum(axis=0)
        assert np.all((tot == 2) | (tot == 0))  # each visible voxel voted twice, or never
        voted = tot == 2
        assert np.all(d["fused"][idx][voted] == np.argmax(c[:, voted], axis=0))
