"""GPU parity on adversarial micro-scenes: band segments that start or end exactly on block
faces, run inside block faces, and pass exactly through block edges and corners, and
voxel centres that lie exactly on pixel boundaries.

The device walks each band segment block by block with hand-written tie rules (positive
moves at the crossing, negative moves just after it, equal-parameter axes together); the
oracle tests every block of the segment's bounding box with an exact rational slab test
(the half-open cells of Sec. IV-C.2's 8^3 blocks).  Natural scans almost never hit an
exact fixed-point tie, so these scenes are built to: a binary voxel size (0.25 m), the
sensor on a block corner, a voxel centre or a block edge, exact rotations (multiples of
90 degrees), rows at 0 and +-45 degrees and columns at multiples of 45 degrees (whose
fp32 cosines and sines are equal), ranges on the voxel lattice, and a 12-column model
whose column boundaries are the diagonals.  Block sets, touched sets, D and W are compared
bit for bit and the meshes as multisets, after every frame.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import compare_mesh, compare_state, gpu_mesh, lidar_model, step_log

pytestmark = pytest.mark.gpu

NU = 0.25           # binary voxel: block edges at nu (8 b - 1/2) are exact in fp32
TAU = 3 * NU
BLOCK_FX = 1 << 19  # one block edge in the 2^-16-voxel fixed point of the walk

ROT = {
    "identity": np.eye(3),
    "yaw90": np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]),
    "roll180": np.diag([1.0, -1.0, -1.0]),
}


def corner(b):
    """World position of block corner b (the fixed-point cell boundary 8 b)."""
    return NU * (8.0 * np.asarray(b, np.float64) - 0.5)


MODELS = {
    # rows at 45, 0 and -45 degrees among others; columns every 45 degrees among 1024
    "deg45x1024": synth.lidar_from_degrees([45, 30, 15, 0, -15, -30, -45], 1024, 30.0),
    # column boundaries at +-45 and +-135 degrees (pi - (c - 1/2) 30 degrees)
    "deg30x12": synth.lidar_from_degrees([30, 0, -30], 12, 30.0),
    "deg45x8": synth.lidar_from_degrees([45, 0, -45], 8, 30.0),
}


def tie_counts(om, lidar, rng_img, T):
    """Independent census of a frame's exact ties from the oracle's fixed-point band
    segments: endpoints on a block plane, segments inside a block plane, and segments that
    cross two axes' block planes at the same points (through block edges or corners)."""
    on_plane = in_plane = through_edge = 0
    rows, cols = rng_img.shape
    for k in range(rows):
        for c in range(cols):
            seg = om.ray_segment(lidar, k, c, float(rng_img[k, c]), T)
            if seg is None:
                continue
            Q0, Q1 = (np.asarray(q, np.int64) for q in seg)
            d = Q1 - Q0
            on_plane += bool(np.any(Q0 % BLOCK_FX == 0) or np.any(Q1 % BLOCK_FX == 0))
            in_plane += bool(np.any((d == 0) & (Q0 % BLOCK_FX == 0)))
            for a in range(3):
                for b in range(a + 1, 3):
                    crosses = (Q0[a] // BLOCK_FX) != (Q1[a] // BLOCK_FX)
                    if not crosses or d[a] == 0:
                        continue
                    if (d[a] == d[b] and (Q0[a] - Q0[b]) % BLOCK_FX == 0) or \
                       (d[a] == -d[b] and (Q0[a] + Q0[b]) % BLOCK_FX == 0):
                        through_edge += 1
    return on_plane, in_plane, through_edge


def _run(torch, frames, lidar, check_ties=True, max_blocks=1 << 16):
    from paper_2412_00291_amd import Map
    m = Map(NU, TAU, 4, max_blocks)
    om = oracle.OracleMap(NU, TAU, 4, max_blocks)
    census = np.zeros(3, np.int64)
    for i, (rng_img, T) in enumerate(frames):
        step_log(f"ties: {lidar.rows}x{lidar.cols} frame {i}")
        m.integrate_lidar(lidar_model(lidar), torch.from_numpy(rng_img).cuda(), T)
        assert om.integrate_lidar(lidar, rng_img, T) == oracle.OK
        assert m.sync() == 0
        if check_ties:
            census += tie_counts(om, lidar, rng_img, T)
        # touched set of this frame, the whole block set, D and W, counters
        assert {tuple(b) for b in m.touched_coords()} == {tuple(b) for b in om.touched()}, i
        rep = compare_state(m, om)
        assert rep["non_identical"] == 0, rep
        st, s = m.stats()
        o = om.stats()
        for key in ("touched", "new_blocks", "updates", "allocated"):
            assert s[key] == o[key], (i, key, s[key], o[key])
        gm = gpu_mesh(m, 0)
        st_, pos, lab, keys, n = om.extract_mesh(oracle.MESH_DIRTY)
        compare_mesh(gm, (pos, lab, keys), voxel=NU)
    gm = gpu_mesh(m, 1)
    st_, pos, lab, keys, n = om.extract_mesh(oracle.MESH_ALL)
    compare_mesh(gm, (pos, lab, keys), voxel=NU)
    m.close()
    om.close()
    return census, rep


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch


@pytest.mark.parametrize("model", sorted(MODELS))
def test_lattice_ranges_from_block_corners_edges_and_voxel_centres(torch_mod, model):
    """Lattice ranges (multiples of nu up to 20 m) from sensors on a block corner, on a
    block edge and at a voxel centre, under exact rotations; five frames into one map."""
    lidar = MODELS[model]
    poses = [
        synth.pose_matrix(ROT["identity"], corner((0, 0, 0))),
        synth.pose_matrix(ROT["yaw90"], corner((1, -1, 0))),
        synth.pose_matrix(ROT["roll180"], corner((0, 0, 1))),
        # on a block edge: x and y on block planes, z at a voxel centre
        synth.pose_matrix(ROT["identity"], corner((2, 1, 0)) + np.array([0.0, 0.0, 1.5 * NU])),
        # at a voxel centre: voxel centres then lie exactly on the diagonal boundaries
        synth.pose_matrix(ROT["yaw90"], NU * np.array([3.0, -5.0, 1.0])),
    ]
    frames = [(synth.lattice_ranges(lidar, seed=40 + i, step=NU, n_max=80, p_drop=0.02), T)
              for i, T in enumerate(poses)]
    census, rep = _run(torch_mod, frames, lidar)
    on_plane, in_plane, through_edge = census
    assert on_plane > 0 and in_plane > 0, census
    # the 12-column model has no diagonal rays (its ties are the diagonal pixel boundaries)
    assert through_edge > 0 or model == "deg30x12", census
    assert rep["blocks"] > 50


def test_sensor_inside_box_room(torch_mod):
    """A closed box room whose walls lie on block planes, seen from a block corner and
    from a voxel centre after a quarter turn: the meshes are compared after each frame and
    the whole (closed) room at the end."""
    lidar = synth.lidar_from_degrees(list(range(60, -61, -4)), 1024, 40.0)
    lo = corner((-4, -3, -1))
    hi = corner((5, 3, 2))
    poses = [synth.pose_matrix(ROT["identity"], corner((0, 0, 0))),
             synth.pose_matrix(ROT["yaw90"], NU * np.array([2.0, 1.0, 0.0])),
             synth.pose_matrix(ROT["roll180"], corner((1, 1, 1)))]
    frames = [(synth.box_room_range(lidar, T, lo, hi), T) for T in poses]
    for r, _ in frames:
        assert np.all(r > 0), "every ray meets a wall"
    census, rep = _run(torch_mod, frames, lidar, check_ties=False)
    assert rep["blocks"] > 200
