"""GPU parity of label fusion from a label range image (the scan's points labelled by a
point-cloud segmentation) against the CPU oracle, through the C ABI.  Bar: label counts
and fused labels bit-exact (compare_state), vote counts equal."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import camera_model, compare_state, lidar_model, step_log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch, torch.device("cuda:0")


def _pair(w):
    from paper_2412_00291_amd import Map
    return Map(w.voxel, w.trunc, w.n_classes, w.max_blocks), oracle.OracleMap(w.voxel, w.trunc, w.n_classes,
                                                                                w.max_blocks)


def test_street_frames_lidar_and_camera_labels(torch_dev):
    torch, dev = torch_dev
    w = synth.street_workload(n_frames=3, n_cams=1)
    m, om = _pair(w)
    lid = lidar_model(w.lidar)
    for k in range(3):
        step_log(f"lidar labels: street frame {k}")
        f = w.frame(k)
        m.integrate_lidar(lid, torch.from_numpy(f.range).to(dev), f.T_wl)
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
        lab = w.lidar_labels(k)
        m.integrate_labels_lidar(lid, torch.from_numpy(lab).to(dev), f.T_wl)
        assert om.integrate_labels_lidar(w.lidar, lab, f.T_wl) == oracle.OK
        T, cl, cam = f.cams[0]  # a camera after the LiDAR labels, in the same frame
        m.integrate_labels(camera_model(cam), torch.from_numpy(np.ascontiguousarray(cl)).to(dev), T)
        assert om.integrate_labels(cam, cl, T) == oracle.OK
        assert m.sync() == 0
        _, s = m.stats()
        assert s["votes"] == om.stats()["votes"]
    rep = compare_state(m, om)
    assert rep["blocks"] > 1000


def test_pixel_encoding_labels_tiny_frame(torch_dev):
    torch, dev = torch_dev
    w = synth.tiny_workload()
    m, om = _pair(w)
    f = w.frame(0, with_labels=False)
    lid = lidar_model(w.lidar)
    m.integrate_lidar(lid, torch.from_numpy(f.range).to(dev), f.T_wl)
    assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    R, C = w.lidar.rows, w.lidar.cols
    rows, cols = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    lab = ((rows * 7 + cols) % (w.n_classes + 3)).astype(np.uint8)  # some labels >= L: no vote
    step_log("lidar labels: tiny frame, pixel-encoding labels")
    for _ in range(2):
        m.integrate_labels_lidar(lid, torch.from_numpy(lab).to(dev), f.T_wl)
        assert om.integrate_labels_lidar(w.lidar, lab, f.T_wl) == oracle.OK
    assert m.sync() == 0
    _, s = m.stats()
    assert s["votes"] == om.stats()["votes"] > 1000
    compare_state(m, om)


def test_no_scan_is_reported(torch_dev):
    torch, dev = torch_dev
    from paper_2412_00291_amd import MAP_ERR_NO_SCAN, Map, map_integrate_labels_lidar
    w = synth.tiny_workload()
    m = Map(w.voxel, w.trunc, w.n_classes, 1 << 12)
    lab = torch.zeros(w.lidar.rows, w.lidar.cols, dtype=torch.uint8, device=dev)
    assert map_integrate_labels_lidar(m.h, lidar_model(w.lidar), lab, np.eye(4, dtype=np.float32)) == MAP_ERR_NO_SCAN


def test_invalid_arguments_are_rejected(torch_dev):
    torch, dev = torch_dev
    from paper_2412_00291_amd import MAP_ERR_INVALID_ARG, map_integrate_labels_lidar
    w = synth.tiny_workload()
    m, _ = _pair(w)
    f = w.frame(0, with_labels=False)
    lid = lidar_model(w.lidar)
    m.integrate_lidar(lid, torch.from_numpy(f.range).to(dev), f.T_wl)
    lab = torch.zeros(w.lidar.rows, w.lidar.cols, dtype=torch.uint8, device=dev)
    sheared = f.T_wl.copy()
    sheared[0, 1] += 0.1  # not a rotation
    assert map_integrate_labels_lidar(m.h, lid, lab, sheared) == MAP_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        map_integrate_labels_lidar(m.h, lid, lab[:3], f.T_wl)
    assert m.sync() == 0
