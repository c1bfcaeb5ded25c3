"""GPU parity of the measurement preprocessing (Eq. 3) against the CPU oracle, through
the C ABI.  Bar: depth and height images bit-exact (the pixel choice and the depth buffer
are exact decisions on the same fp32 range; D and H are one fp32 operation each on the
same operands)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import lidar_model, step_log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def street():
    return synth.street_workload(n_frames=3, n_cams=1)


def _map():
    from paper_2412_00291_amd import Map
    return Map(0.1, 0.3, 19, 1 << 12)


def _gpu(torch, m, lidar, pts, F=1.0, O=0.0, height=True):
    dev = torch.device("cuda:0")
    P = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)).to(dev)
    D = torch.full((lidar.rows, lidar.cols), -1.0, dtype=torch.float32, device=dev)
    H = torch.full((lidar.rows, lidar.cols), -1.0, dtype=torch.float32, device=dev) if height else None
    m.range_image(lidar_model(lidar), P, D, H, F, O)
    torch.cuda.synchronize()
    return D.cpu().numpy(), (H.cpu().numpy() if height else None)


def _check(torch, m, lidar, pts, F=1.0, O=0.0):
    D, H = _gpu(torch, m, lidar, pts, F, O)
    oD, oH, n = oracle.range_image(lidar.rows, lidar.cols, lidar.elev_rad, lidar.r_max, pts, F=F, O=O)
    np.testing.assert_array_equal(D, oD)
    np.testing.assert_array_equal(H, oH)
    return n


def test_street_clouds_bit_exact(torch_dev, street):
    torch, _ = torch_dev
    m = _map()
    for k, (F, O) in enumerate([(1.0, 0.0), (250.0, 1.73), (1.0, 0.0)]):
        step_log(f"range image: street cloud frame {k}, F={F}, O={O}")
        pts = synth.cloud_points(street, k, 100 + k)
        n = _check(torch, m, street.lidar, pts, F, O)
        assert n > 0.95 * street.lidar.rows * street.lidar.cols


def test_scan_as_points_round_trip(torch_dev, street):
    torch, _ = torch_dev
    lidar = street.lidar
    f = street.frame(0, with_labels=False)
    r = f.range.reshape(-1).astype(np.float64)
    pts = (lidar.directions() * r[:, None]).astype(np.float32)  # dropouts land at the origin
    step_log("range image: street scan as points")
    _check(torch, _map(), lidar, pts)
    D, _ = _gpu(torch, _map(), lidar, pts, height=False)
    valid = f.range > 0
    assert np.array_equal(D > 0, valid)
    np.testing.assert_allclose(D[valid], f.range[valid], rtol=1e-6)


def _same_range_pair(lidar):
    d = lidar.directions()[5 * lidar.cols + 700]
    rng = np.random.Generator(np.random.PCG64(13))
    cand = (10.0 * (d[None, :] + rng.normal(0.0, 1e-4, size=(4000, 3)))).astype(np.float32)
    x, y, z = cand[:, 0], cand[:, 1], cand[:, 2]
    r = np.sqrt((x * x + y * y) + z * z)
    for i in range(len(cand)):
        for j in np.nonzero((r == r[i]) & (z != z[i]))[0]:
            pi = oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, cand[i])
            if pi is not None and pi == oracle.pixel_of(lidar.rows, lidar.cols, lidar.elev_rad, cand[j]):
                return cand[i], cand[j], pi
    raise AssertionError("no equal-range pair found")


def test_equal_ranges_keep_the_first_point(torch_dev):
    torch, _ = torch_dev
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    a, b, (row, col) = _same_range_pair(lidar)
    m = _map()
    filler = (lidar.directions()[::7] * 20.0).astype(np.float32)  # other pixels, to spread the launch
    for first, second in ((a, b), (b, a)):
        step_log("range image: equal-range pair")
        pts = np.concatenate([filler, first[None], second[None], filler[:50] * np.float32(1.5)])
        _check(torch, m, lidar, pts)
        D, H = _gpu(torch, m, lidar, pts)
        assert H[row, col] == first[2]


def test_empty_cloud_and_model_changes(torch_dev, street):
    torch, _ = torch_dev
    tiny = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    m = _map()
    step_log("range image: empty cloud")
    D, H = _gpu(torch, m, street.lidar, np.zeros((0, 3), np.float32))
    assert not D.any() and not H.any()
    pts = synth.cloud_points(street, 1, 7)
    # a large image, a smaller model, the large one again: the per-pixel keys are reset by
    # every call, whatever the model
    for lidar, p in ((street.lidar, pts), (tiny, pts), (street.lidar, pts[: len(pts) // 3])):
        step_log(f"range image: {lidar.rows}x{lidar.cols}, {len(p)} points")
        _check(torch, m, lidar, p)


def test_depth_only(torch_dev, street):
    torch, _ = torch_dev
    pts = synth.cloud_points(street, 2, 9)
    D, _ = _gpu(torch, _map(), street.lidar, pts, F=3.0, height=False)
    oD, _, _ = oracle.range_image(street.lidar.rows, street.lidar.cols, street.lidar.elev_rad,
                                  street.lidar.r_max, pts, F=3.0)
    np.testing.assert_array_equal(D, oD)


def test_invalid_arguments_are_rejected_before_any_launch(torch_dev):
    torch, dev = torch_dev
    from paper_2412_00291_amd import MAP_ERR_INVALID_ARG, map_range_image
    from paper_2412_00291_amd.mapcore import LidarModel
    lidar = synth.uniform_lidar(16, 1800, 15.0, -15.0, 40.0)
    m = _map()
    P = torch.zeros(10, 3, dtype=torch.float32, device=dev)
    D = torch.zeros(16, 1800, dtype=torch.float32, device=dev)
    good = lidar_model(lidar)
    assert map_range_image(m.h, good, P, D, None, float("inf"), 0.0) == MAP_ERR_INVALID_ARG
    assert map_range_image(m.h, good, P, D, None, 1.0, float("nan")) == MAP_ERR_INVALID_ARG
    no_range = LidarModel(16, 1800, np.ascontiguousarray(lidar.elev_rad, np.float32), 0.0)
    assert map_range_image(m.h, no_range, P, D, None) == MAP_ERR_INVALID_ARG
    rising = LidarModel(16, 1800, np.ascontiguousarray(lidar.elev_rad[::-1], np.float32), 40.0)
    assert map_range_image(m.h, rising, P, D, None) == MAP_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        map_range_image(m.h, good, P, torch.zeros(5, dtype=torch.float32, device=dev), None)
