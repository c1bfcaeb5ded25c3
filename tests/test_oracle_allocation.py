"""Pins of the oracle's block allocation (the blocks a return's truncation band meets).

The band segment of a return is [max(r - tau, 0), r + tau] along the ray (reading of
Sec. IV-C.2: only voxels near the measured surface are touched); blocks are the 8^3
voxel blocks of Sec. IV-C.2.  The segment-vs-block test is checked against hand-derived
cases and against an independent exact enumeration with Python fractions.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

BLOCK = 1 << 19  # one block in 2^-16-voxel fixed point
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    cases = []
    with open(os.path.join(HERE, "golden", "segment_blocks.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            lhs, rhs = line.split(":")
            v = [float(x) for x in lhs.split()]
            q0 = [int(round(x * BLOCK)) for x in v[:3]]
            q1 = [int(round(x * BLOCK)) for x in v[3:]]
            blocks = {tuple(int(x) for x in b.split()) for b in rhs.split("/")}
            cases.append((q0, q1, blocks))
    return cases


@pytest.mark.parametrize("q0,q1,expected", _golden())
def test_segment_blocks_hand_cases(q0, q1, expected):
    got = {tuple(b) for b in oracle.segment_blocks(q0, q1)}
    assert got == expected


def _cells_exact(q0, q1):
    """Independent enumeration: the cell is constant between consecutive plane crossings,
    so the cells at every crossing parameter and every midpoint cover the segment."""
    q0 = [Fraction(x) for x in q0]
    q1 = [Fraction(x) for x in q1]
    ts = {Fraction(0), Fraction(1)}
    for a in range(3):
        d = q1[a] - q0[a]
        if d == 0:
            continue
        lo, hi = min(q0[a], q1[a]), max(q0[a], q1[a])
        k0 = (lo // BLOCK)
        k1 = (hi // BLOCK) + 1
        for k in range(int(k0), int(k1) + 1):
            t = (k * BLOCK - q0[a]) / d
            if 0 <= t <= 1:
                ts.add(t)
    ts = sorted(ts)
    samples = list(ts) + [(a + b) / 2 for a, b in zip(ts[:-1], ts[1:])]
    cells = set()
    for t in samples:
        p = [q0[a] + t * (q1[a] - q0[a]) for a in range(3)]
        cells.add(tuple(int(x // BLOCK) for x in p))
    return cells


def test_segment_blocks_vs_exact_enumeration():
    rng = np.random.Generator(np.random.PCG64(11))
    for i in range(400):
        # endpoints on a coarse lattice half the time, so planes, edges and corners are hit
        if i % 2 == 0:
            q0 = rng.integers(-12, 12, size=3) * (BLOCK // 4)
            q1 = q0 + rng.integers(-6, 7, size=3) * (BLOCK // 4)
        else:
            q0 = rng.integers(-3 * BLOCK, 3 * BLOCK, size=3)
            q1 = q0 + rng.integers(-BLOCK, BLOCK, size=3)
        got = {tuple(b) for b in oracle.segment_blocks(q0, q1)}
        assert got == _cells_exact(q0.tolist(), q1.tolist()), (q0, q1)


def test_ray_segment_geometry():
    """Fixed-point endpoints equal (o + s R d) / nu + 1/2 within fp32 error, s = max(r-tau,0), r+tau."""
    lidar = synth.uniform_lidar(16, 360, 15.0, -15.0, 60.0)
    ang = np.deg2rad([20.0, -35.0, 50.0])
    R = synth.rot_z(ang[2]) @ np.array([[1, 0, 0], [0, np.cos(ang[0]), -np.sin(ang[0])],
                                       [0, np.sin(ang[0]), np.cos(ang[0])]])
    T = synth.pose_matrix(R, [3.3, -1.7, 0.9])
    m = oracle.OracleMap(0.1, 0.3, 5)
    Td = T.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(300):
        k, c = int(rng.integers(0, 16)), int(rng.integers(0, 360))
        r = float(np.float32(rng.uniform(0.05, 59.0)))
        q0, q1 = m.ray_segment(lidar, k, c, r, T)
        e = float(lidar.elev_rad[k])
        phi = np.pi - c * 2 * np.pi / 360
        d = Td[:3, :3] @ np.array([np.cos(e) * np.cos(phi), np.cos(e) * np.sin(phi), np.sin(e)])
        for s, q in ((max(r - 0.3, 0.0), q0), (r + 0.3, q1)):
            want = (Td[:3, 3] + s * d) / np.float32(0.1) + 0.5
            assert np.all(np.abs(q / 65536.0 - want) < 2e-3), (k, c, r)
    assert m.ray_segment(lidar, 0, 0, 0.0, T) is None       # dropout
    assert m.ray_segment(lidar, 0, 0, 61.0, T) is None      # beyond r_max
    assert m.ray_segment(lidar, 0, 0, float("nan"), T) is None


def test_scan_touched_set_is_union_of_ray_sets():
    """T_k equals the union of the per-return block sets; N_k counts the new ones."""
    lidar = synth.uniform_lidar(8, 64, 10.0, -20.0, 30.0)
    T = synth.pose_matrix(synth.rot_z(0.3), [0.4, -0.2, 1.1])
    rng = np.random.Generator(np.random.PCG64(5))
    rimg = rng.uniform(0.1, 25.0, size=(8, 64)).astype(np.float32)
    rimg[rng.random(size=rimg.shape) < 0.1] = 0.0
    m = oracle.OracleMap(0.2, 0.6, 4)
    want = set()
    for k in range(8):
        for c in range(64):
            seg = m.ray_segment(lidar, k, c, float(rimg[k, c]), T)
            if seg is not None:
                want |= {tuple(b) for b in oracle.segment_blocks(*seg)}
    assert m.integrate_lidar(lidar, rimg, T) == oracle.OK
    got = {tuple(b) for b in m.touched()}
    assert got == want
    st = m.stats()
    assert st["touched"] == len(want) and st["new_blocks"] == len(want) and st["allocated"] == len(want)
    coords = m.block_coords()
    assert len({tuple(b) for b in coords}) == len(coords)   # no duplicate keys
    # the same frame again: nothing new
    assert m.integrate_lidar(lidar, rimg, T) == oracle.OK
    assert m.stats()["new_blocks"] == 0 and m.num_blocks() == len(want)


def test_capacity_rejects_frame_and_leaves_map_unchanged():
    lidar = synth.uniform_lidar(8, 64, 10.0, -20.0, 30.0)
    T = synth.pose_matrix(np.eye(3), [0.0, 0.0, 0.0])
    rimg = np.full((8, 64), 5.0, np.float32)
    m = oracle.OracleMap(0.2, 0.6, 4, max_blocks=10)
    cam = synth.Camera(8, 8, 4.0, 4.0, 4.0, 4.0)
    # labels before any frame was submitted
    assert m.integrate_labels(cam, np.zeros((8, 8), np.uint8), T) == oracle.NO_SCAN
    assert m.integrate_lidar(lidar, rimg, T) == oracle.CAPACITY
    assert m.num_blocks() == 0
    # a rejected frame leaves an empty scan: label calls after it vote nowhere and succeed
    assert m.integrate_labels(cam, np.zeros((8, 8), np.uint8), T) == oracle.OK
    st = m.stats()
    assert st["votes"] == 0 and st["touched"] == 0 and m.num_blocks() == 0


def test_invalid_arguments():
    lidar = synth.uniform_lidar(8, 64, 10.0, -20.0, 30.0)
    rimg = np.full((8, 64), 5.0, np.float32)
    m = oracle.OracleMap(0.2, 0.6, 4)
    bad = synth.pose_matrix(np.eye(3), [0, 0, 0])
    bad[0, 0] = 1.01  # not orthonormal
    assert m.integrate_lidar(lidar, rimg, bad) == oracle.INVALID
    nanpose = synth.pose_matrix(np.eye(3), [0, 0, 0])
    nanpose[1, 3] = np.nan
    assert m.integrate_lidar(lidar, rimg, nanpose) == oracle.INVALID
    rev = synth.Lidar(8, 64, lidar.elev_rad[::-1].copy(), 30.0)  # elevations must decrease
    assert m.integrate_lidar(rev, rimg, synth.pose_matrix(np.eye(3), [0, 0, 0])) == oracle.INVALID
    far = synth.pose_matrix(np.eye(3), [0.2 * (1 << 19), 0, 0])  # outside the map domain
    assert m.integrate_lidar(lidar, rimg, far) == oracle.INVALID
    with pytest.raises(ValueError):
        oracle.OracleMap(0.1, 10.0, 4)  # truncation above 64 voxels
