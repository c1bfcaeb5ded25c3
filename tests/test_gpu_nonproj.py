"""GPU parity of the non-projective distance (the paper's "Ours", Sec. IV-C.2, Eq. 4) with
the oracle, through the C ABI: the normal image and point filter of each scan, the block
sets, D, W and the per-voxel gradients (bit for bit: the same fp32 operations in the same
order), label counts and meshes.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import camera_model, compare_mesh, compare_state, gpu_mesh, lidar_model, step_log

pytestmark = pytest.mark.gpu

INC = float(np.deg2rad(80.0))


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch


def _pair(voxel, trunc, n_classes, max_blocks, inc=INC):
    from paper_2412_00291_amd import Map, MAP_DIST_NONPROJECTIVE
    m = Map(voxel, trunc, n_classes, max_blocks)
    m.set_distance(MAP_DIST_NONPROJECTIVE, inc)
    om = oracle.OracleMap(voxel, trunc, n_classes, max_blocks, variant="omp")
    assert om.set_distance(oracle.DIST_NONPROJECTIVE, inc) == oracle.OK
    return m, om


def compare_gradients(m, om):
    """Per-voxel gradients of every block bit-identical to the oracle's."""
    g = m.download(with_counts=False)
    aux = m.download_aux(grad=True, logpost=False)
    n_nonzero = 0
    for i, b in enumerate(g["coords"]):
        og = om.block_gradient(tuple(b))
        assert og is not None, b
        np.testing.assert_array_equal(aux["grad"][i], og, err_msg=str(b))
        n_nonzero += int(np.count_nonzero(np.any(og != 0, axis=0)))
    return n_nonzero


def compare_normals(m, lidar, rng_img, T, inc=INC):
    kept, nrm = oracle.normal_image(lidar, rng_img, T, inc)
    gn = m.frame_normals()
    assert gn is not None and gn.shape == (lidar.rows * lidar.cols, 4)
    np.testing.assert_array_equal(gn[:, 3].reshape(lidar.rows, lidar.cols), kept)
    np.testing.assert_array_equal(gn[:, :3].reshape(lidar.rows, lidar.cols, 3), nrm)
    return int(np.count_nonzero(kept))


def _frame(torch, m, om, w, f, labels=True):
    m.integrate_lidar(lidar_model(w.lidar), torch.from_numpy(f.range).cuda(), f.T_wl)
    assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    if labels:
        for T, lab, cam in f.cams:
            m.integrate_labels(camera_model(cam), torch.from_numpy(np.ascontiguousarray(lab)).cuda(), T)
            assert om.integrate_labels(cam, lab, T) == oracle.OK


def _check_frame(m, om, w, k):
    st_, s = m.stats()
    o = om.stats()
    for key in ("touched", "new_blocks", "updates", "votes", "allocated"):
        assert s[key] == o[key], (k, key, s[key], o[key])
    assert {tuple(b) for b in m.touched_coords()} == {tuple(b) for b in om.touched()}
    gm = gpu_mesh(m, 0)
    st, pos, lab, keys, n = om.extract_mesh(oracle.MESH_DIRTY)
    return compare_mesh(gm, (pos, lab, keys), voxel=w.voxel)


def test_street_frames_nonprojective(torch_mod):
    """Five 64x2048 street frames with four 1280x720 label images each: normal image,
    counters, touched sets and dirty meshes after every frame; D, W, labels and gradients
    after frames 0, 2 and 4."""
    torch = torch_mod
    w = synth.street_workload(n_frames=5)
    m, om = _pair(w.voxel, w.trunc, w.n_classes, 1 << 18)
    for k in range(5):
        step_log(f"nonproj street frame {k}")
        f = w.frame(k)
        _frame(torch, m, om, w, f)
        kept = compare_normals(m, w.lidar, f.range, f.T_wl)
        assert kept > 0.5 * np.count_nonzero(f.range)
        mr = _check_frame(m, om, w, k)
        if k in (0, 2, 4):
            rep = compare_state(m, om)
            assert rep["non_identical"] == 0, rep
            assert compare_gradients(m, om) > 100000
    # the point filter drops grazing returns (the far ground), so fewer blocks than projective
    assert rep["blocks"] > 3000 and mr["triangles"] > 10000
    m.close()


def test_tiny_frame_sphere_and_plane(torch_mod):
    """The tiny frame (16x1800, 0.2 m voxels, one camera), the sensor inside a sphere, and
    an oblique plane, each against the oracle."""
    torch = torch_mod
    w = synth.tiny_workload()
    m, om = _pair(w.voxel, w.trunc, w.n_classes, 1 << 16)
    f = w.frame(0)
    _frame(torch, m, om, w, f)
    compare_normals(m, w.lidar, f.range, f.T_wl)
    _check_frame(m, om, w, 0)
    assert compare_state(m, om)["non_identical"] == 0
    compare_gradients(m, om)
    m.close()

    lidar = synth.uniform_lidar(48, 720, 40.0, -40.0, 40.0)
    for rimg, T in ((synth.constant_range(lidar, 3.0), synth.pose_matrix(np.eye(3), [0.0, 0.0, 0.0])),
                    (None, synth.pose_matrix(np.eye(3), [0.0, 0.0, 1.5]))):
        if rimg is None:
            rimg = synth.plane_range(lidar, T, np.array([0.0, 0.0, 1.0]), 0.0)
        m, om = _pair(0.1, 0.3, 4, 1 << 16)
        m.integrate_lidar(lidar_model(lidar), torch.from_numpy(rimg).cuda(), T)
        assert om.integrate_lidar(lidar, rimg, T) == oracle.OK
        compare_normals(m, lidar, rimg, T)
        rep = compare_state(m, om)
        assert rep["non_identical"] == 0 and rep["voxels"] > 1000
        compare_gradients(m, om)
        gm = gpu_mesh(m, 1)
        st, pos, lab, keys, n = om.extract_mesh(oracle.MESH_ALL)
        compare_mesh(gm, (pos, lab, keys), voxel=0.1)
        m.close()


def test_switch_from_projective_and_incidence_limits(torch_mod):
    """Projective frames first, then the non-projective distance (gradients start at zero)
    with a tight incidence limit (60 degrees), then a second map with no limit (90)."""
    torch = torch_mod
    from paper_2412_00291_amd import Map, MAP_DIST_NONPROJECTIVE
    w = synth.street_workload(n_frames=4, n_cams=1)
    m = Map(w.voxel, w.trunc, w.n_classes, 1 << 18)
    om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, 1 << 18, variant="omp")
    for k in range(4):
        if k == 2:
            m.set_distance(MAP_DIST_NONPROJECTIVE, float(np.deg2rad(60.0)))
            assert om.set_distance(oracle.DIST_NONPROJECTIVE, float(np.deg2rad(60.0))) == oracle.OK
        f = w.frame(k)
        _frame(torch, m, om, w, f)
        if k >= 2:
            compare_normals(m, w.lidar, f.range, f.T_wl, float(np.deg2rad(60.0)))
        _check_frame(m, om, w, k)
    assert compare_state(m, om)["non_identical"] == 0
    compare_gradients(m, om)
    m.close()
    m, om = _pair(w.voxel, w.trunc, w.n_classes, 1 << 18, inc=float(np.pi / 2))
    f = w.frame(0)
    _frame(torch, m, om, w, f)
    compare_normals(m, w.lidar, f.range, f.T_wl, float(np.pi / 2))
    assert compare_state(m, om)["non_identical"] == 0
    compare_gradients(m, om)
    m.close()


def test_set_distance_rejects_bad_arguments(torch_mod):
    from paper_2412_00291_amd import Map, MAP_ERR_INVALID_ARG, map_set_distance
    m = Map(0.1, 0.3, 4, 1 << 10)
    assert map_set_distance(m.h, 2, 1.0) == MAP_ERR_INVALID_ARG
    assert map_set_distance(m.h, 1, float("nan")) == MAP_ERR_INVALID_ARG
    assert map_set_distance(m.h, 1, -0.5) == MAP_ERR_INVALID_ARG
    assert m.frame_normals() is None  # projective: no normal image
    m.close()
