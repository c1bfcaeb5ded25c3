"""The allocation-free pose adjoint (map_sdf_pose_adjoint_noalloc, for callers that cannot
allocate) against map_sdf_pose_adjoint, through the C ABI: the same kernels with the
partial sums in the library's static device scratch, so the loss, dL/dxi and dL/dp are
bit-identical; two calls in a row, the second smaller, and a size beyond the scratch
rejected."""
import numpy as np
import pytest

import synth
from tests.gpu_helpers import lidar_model, step_log

pytestmark = pytest.mark.gpu


def test_noalloc_adjoint_equals_allocating_call():
    import torch
    from paper_2412_00291_amd import MAP_ERR_INVALID_ARG, MAP_OK, Map, map_last_error, map_sdf_pose_adjoint_noalloc
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    w = synth.tiny_workload()
    f = w.frame(0, with_labels=False)
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    m.integrate_lidar(lidar_model(w.lidar), torch.from_numpy(f.range).to(dev), f.T_wl)
    pts = synth.scan_points(w, synth.uniform_lidar(64, 2048, 15.0, -15.0, 40.0), f.T_wl, 131072, seed=4)
    xi = synth.perturbed_poses(64, seed=4)
    for B, N in ((64, 131072), (5, 1000)):  # the second call is smaller
        step_log(f"noalloc adjoint: B={B} N={N}")
        P = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(pts[:N], (B, N, 3)))).to(dev)
        X = torch.from_numpy(np.ascontiguousarray(xi[:B])).to(dev)
        outs = []
        for noalloc in (False, True):
            loss = torch.full((B,), float("nan"), device=dev)
            gxi = torch.full((B, 6), float("nan"), device=dev)
            gp = torch.full_like(P, float("nan"))
            if noalloc:
                assert map_sdf_pose_adjoint_noalloc(m.h, X, P, loss, gxi, gp) == MAP_OK
            else:
                m.sdf_pose_adjoint(X, P, loss, gxi, gp)
            torch.cuda.synchronize()
            outs.append((loss.cpu().numpy(), gxi.cpu().numpy(), gp.cpu().numpy()))
        for a, b in zip(*outs):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert np.isfinite(outs[1][0]).all() and outs[1][0].sum() > 0
    # beyond the static scratch: B * ceil(N / 256) > 131072 chunks
    B, N = 2, 256 * 65537
    X = torch.zeros((B, 6), device=dev)
    P = torch.zeros((B, N, 3), device=dev)
    loss = torch.empty(B, device=dev)
    gxi = torch.empty(B, 6, device=dev)
    assert map_sdf_pose_adjoint_noalloc(m.h, X, P, loss, gxi, None) == MAP_ERR_INVALID_ARG
    assert "static scratch" in map_last_error(m.h)
    m.close()
