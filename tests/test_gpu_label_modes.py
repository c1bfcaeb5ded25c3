"""GPU parity of the label fusion modes with the oracle, through the C ABI (Sec. IV-C.3,
Eq. 6, and the Ours-wo-Bay ablation of Sec. V-C):

* latest label wins: camera and LiDAR label images; fused labels bit-exact, counts untouched;
* Eq. 6 on per-pixel class log-probability images: the L fp32 log-posteriors of every voxel
  bit-exact (the same fp32 sums in the same class order), the most probable labels exact;
* the modes' argument checks.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import camera_model, compare_state, lidar_model, step_log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch


def _pair(w, mode, max_blocks):
    from paper_2412_00291_amd import Map
    m = Map(w.voxel, w.trunc, w.n_classes, max_blocks)
    m.set_label_fusion(mode)
    om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, max_blocks, variant="omp")
    assert om.set_label_fusion(mode) == oracle.OK
    return m, om


def _votes(m, om):
    st, s = m.stats()
    assert s["votes"] == om.stats()["votes"], (s["votes"], om.stats()["votes"])
    return s["votes"]


def test_latest_label_camera_and_lidar(torch_mod):
    """Three street frames: four camera label images per frame, then the frame's label
    range image; after each call the fused labels equal the oracle's and counts stay 0."""
    torch = torch_mod
    from paper_2412_00291_amd import MAP_LABELS_LATEST
    w = synth.street_workload(n_frames=3)
    m, om = _pair(w, MAP_LABELS_LATEST, 1 << 18)
    lid = lidar_model(w.lidar)
    for k in range(3):
        step_log(f"latest labels: street frame {k}")
        f = w.frame(k)
        m.integrate_lidar(lid, torch.from_numpy(f.range).cuda(), f.T_wl)
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
        cams = [camera_model(c) for _, _, c in f.cams]
        labs = [torch.from_numpy(np.ascontiguousarray(l)).cuda() for _, l, _ in f.cams]
        m.integrate_labels_multi(cams, labs, [T for T, _, _ in f.cams])
        for T, lab, cam in f.cams:
            assert om.integrate_labels(cam, lab, T) == oracle.OK
        assert _votes(m, om) > 10000
        rep = compare_state(m, om)
        lr = w.lidar_labels(k)
        m.integrate_labels_lidar(lid, torch.from_numpy(lr).cuda(), f.T_wl)
        assert om.integrate_labels_lidar(w.lidar, lr, f.T_wl) == oracle.OK
        _votes(m, om)
        rep = compare_state(m, om)
    g = m.download(with_counts=True)
    assert not g["counts"].any()
    assert np.count_nonzero(g["fused"] != 255) > 100000 and rep["blocks"] > 5000
    m.close()


def _compare_logpost(m, om):
    g = m.download(with_counts=False)
    aux = m.download_aux(grad=False, logpost=True)
    n_voted = 0
    for i, b in enumerate(g["coords"]):
        lp = om.block_logpost(tuple(b))
        np.testing.assert_array_equal(aux["logpost"][i], lp, err_msg=str(b))
        n_voted += int(np.count_nonzero(np.any(lp != 0, axis=0)))
    return n_voted


@pytest.mark.parametrize("scene", ["tiny", "street"])
def test_bayes_logprob_images(torch_mod, scene):
    """Log-softmax images of noisy logits (and, for the tiny scene, hard-label images with
    p = 0.9): log-posteriors, fused labels and vote counts equal the oracle's."""
    torch = torch_mod
    from paper_2412_00291_amd import MAP_LABELS_BAYES
    if scene == "tiny":
        w = synth.tiny_workload()
        nfr, mb = 1, 1 << 15
    else:
        w = synth.street_workload(n_frames=2, n_cams=2)
        nfr, mb = 2, 1 << 16
    m, om = _pair(w, MAP_LABELS_BAYES, mb)
    lid = lidar_model(w.lidar)
    for k in range(nfr):
        step_log(f"bayes labels: {scene} frame {k}")
        f = w.frame(k)
        m.integrate_lidar(lid, torch.from_numpy(f.range).cuda(), f.T_wl)
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
        for i, (T, lab, cam) in enumerate(f.cams):
            lps = [synth.logprob_image(lab, w.n_classes, seed=100 * k + i)]
            if scene == "tiny":
                lps.append(synth.hard_logprob_image(lab, w.n_classes, 0.9))
            for lp in lps:
                m.integrate_logprobs(camera_model(cam), torch.from_numpy(lp).cuda(), T)
                assert om.integrate_logprobs(cam, lp, T) == oracle.OK
        assert _votes(m, om) > 1000
        rep = compare_state(m, om)
        assert _compare_logpost(m, om) > 1000
    assert rep["blocks"] > 500
    m.close()


def test_label_mode_arguments(torch_mod):
    torch = torch_mod
    from paper_2412_00291_amd import (MAP_ERR_INVALID_ARG, MAP_ERR_NO_SCAN, MAP_LABELS_BAYES, MAP_OK, Map,
                                      map_integrate_labels, map_integrate_labels_lidar, map_integrate_logprobs,
                                      map_set_label_fusion)
    w = synth.tiny_workload()
    cam = w.cameras[0]
    T = synth.pose_matrix(np.eye(3), [0, 0, 0])
    lab = torch.zeros((cam.height, cam.width), dtype=torch.uint8, device="cuda")
    lp = torch.zeros((cam.height, cam.width, w.n_classes), dtype=torch.float32, device="cuda")
    m = Map(w.voxel, w.trunc, w.n_classes, 1 << 12)
    assert map_set_label_fusion(m.h, 3) == MAP_ERR_INVALID_ARG
    # counts mode: log-probabilities are refused
    assert map_integrate_logprobs(m.h, camera_model(cam), lp, T, w.n_classes) == MAP_ERR_INVALID_ARG
    assert map_set_label_fusion(m.h, MAP_LABELS_BAYES) == MAP_OK
    assert map_integrate_logprobs(m.h, camera_model(cam), lp, T, w.n_classes) == MAP_ERR_NO_SCAN
    m.integrate_lidar(lidar_model(w.lidar), torch.from_numpy(w.frame(0, with_labels=False).range).cuda(), T)
    assert map_integrate_labels(m.h, camera_model(cam), lab, T) == MAP_ERR_INVALID_ARG
    lr = torch.zeros((w.lidar.rows, w.lidar.cols), dtype=torch.uint8, device="cuda")
    assert map_integrate_labels_lidar(m.h, lidar_model(w.lidar), lr, T) == MAP_ERR_INVALID_ARG
    assert map_integrate_logprobs(m.h, camera_model(cam), lp, T, w.n_classes) == MAP_OK
    assert m.sync() == MAP_OK
    m.close()
