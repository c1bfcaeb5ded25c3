"""GPU checks of the batched step's concurrent schedule (each map's own kernels, the maps
spread over several streams) at its edges: maps without cameras next to maps with several,
a map whose frame is rejected for capacity, steps that leave maps out, and the schedule's
argument checks.  Every map must end as its own plain calls leave it: state, per-step
meshes (as multisets) and statuses."""
import numpy as np
import pytest

import synth
from tests.gpu_helpers import camera_model, canonical_mesh, lidar_model, sorted_download, step_log

pytestmark = pytest.mark.gpu

CAP = 1 << 20


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch


def _setup(torch):
    """Four maps on the street sequence: 0.1 m with two cameras, 0.2 m without cameras,
    0.4 m with one camera, and a 0.2 m map with room for 300 blocks (its first frame fits
    nowhere near: rejected)."""
    w = synth.street_workload(n_frames=4, n_cams=2)
    frames = [w.frame(k) for k in range(4)]
    lid = lidar_model(w.lidar)
    cams = [camera_model(c) for c in w.cameras]
    dev = [(torch.from_numpy(f.range).cuda(), [torch.from_numpy(np.ascontiguousarray(l)).cuda() for _, l, _ in f.cams],
            f.T_wl, [T for T, _, _ in f.cams]) for f in frames]
    specs = [(0.1, 0.3, 2, 1 << 19), (0.2, 0.6, 0, 1 << 18), (0.4, 1.2, 1, 1 << 17), (0.2, 0.6, 1, 300)]
    return w, lid, cams, dev, specs


def _items(k, dev, lid, cams, specs, bufs, skip=()):
    out = []
    for mi, (nu, tau, nc, mb) in enumerate(specs):
        if mi in skip:
            continue
        r, labs, T, Tcs = dev[k]
        out.append({"map_index": mi, "lidar": lid, "range": r, "T_wl": T, "cams": cams[:nc], "labels": labs[:nc],
                    "T_wc": Tcs[:nc], "pos": bufs[mi][0], "lab": bufs[mi][1], "keys": bufs[mi][2]})
    return out


def _bufs(torch, n):
    return [(torch.zeros((CAP, 3, 3), dtype=torch.float32, device="cuda"),
             torch.zeros((CAP, 3), dtype=torch.uint8, device="cuda"),
             torch.zeros((CAP, 3), dtype=torch.int64, device="cuda")) for _ in range(n)]


def _mesh(bufs, n):
    pos, lab, keys = bufs
    return canonical_mesh(pos[:n].cpu().numpy(), lab[:n].cpu().numpy(), keys[:n].cpu().numpy())


def test_concurrent_schedule_equals_plain_calls(torch_mod):
    torch = torch_mod
    from paper_2412_00291_amd import MAP_ERR_CAPACITY, MAP_MESH_DIRTY, Batch, Map
    w, lid, cams, dev, specs = _setup(torch)
    L = w.n_classes
    plain = [Map(nu, tau, L, mb) for nu, tau, nc, mb in specs]
    conc = [Map(nu, tau, L, mb) for nu, tau, nc, mb in specs]
    pb, cb = _bufs(torch, len(specs)), _bufs(torch, len(specs))
    batch = Batch(conc, schedule=4, grid=3, use_graph=False)
    stream = torch.cuda.Stream()
    skips = {0: (), 1: (2,), 2: (), 3: (0, 1)}  # steps that leave maps out
    for k in range(4):
        step_log(f"batch concurrent: step {k}")
        items = _items(k, dev, lid, cams, specs, cb, skips[k])
        with torch.cuda.stream(stream):
            st, ns = batch.step(items)
        stream.synchronize()
        for it, n in zip(items, ns):
            mi = it["map_index"]
            m = plain[mi]
            m.integrate_lidar(lid, it["range"], it["T_wl"])
            if it["cams"]:
                m.integrate_labels_multi(it["cams"], it["labels"], it["T_wc"])
            st_p, n_p = m.extract_mesh(MAP_MESH_DIRTY, *pb[mi])
            assert n == n_p, (k, mi, n, n_p)
            assert np.array_equal(_mesh(cb[mi], n), _mesh(pb[mi], n_p)), (k, mi)
    for mi in range(len(specs)):
        sp, sc = plain[mi].sync(), conc[mi].sync()
        assert sp == sc, (mi, sp, sc)
        a, b = sorted_download(plain[mi]), sorted_download(conc[mi])
        for key in ("coords", "D", "W", "fused", "counts"):
            assert np.array_equal(a[key], b[key]), (mi, key)
        _, s_p = plain[mi].stats()
        _, s_c = conc[mi].stats()
        for key in ("touched", "new_blocks", "updates", "votes", "allocated", "frames", "mesh_blocks", "triangles"):
            assert s_p[key] == s_c[key], (mi, key, s_p[key], s_c[key])
    # the map with room for 300 blocks rejected its frames; the others took theirs
    assert conc[3].stats()[1]["allocated"] == 0 and conc[3].stats()[1]["frames"] == 0
    assert all(conc[mi].stats()[1]["frames"] > 0 for mi in range(3))
    batch.close()
    for m in plain + conc:
        m.close()


def test_concurrent_schedule_arguments(torch_mod):
    from paper_2412_00291_amd import MAP_ERR_INVALID_ARG, Map
    from paper_2412_00291_amd.mapcore import map_batch_configure, map_batch_create, map_batch_destroy
    maps = [Map(0.2, 0.6, 4, 1024) for _ in range(2)]
    st, h = map_batch_create([m.h for m in maps])
    assert st == 0
    assert map_batch_configure(h, 4, 0, 0) == MAP_ERR_INVALID_ARG
    assert map_batch_configure(h, 4, 17, 0) == MAP_ERR_INVALID_ARG
    assert map_batch_configure(h, 5, 4, 0) == MAP_ERR_INVALID_ARG
    assert map_batch_configure(h, 3, 32, 1) == MAP_ERR_INVALID_ARG
    assert map_batch_configure(h, 4, 16, 0) == 0
    assert map_batch_configure(h, 4, 2, 1) == 0
    assert map_batch_configure(h, 3, 1024, 1) == 0
    map_batch_destroy(h)
    for m in maps:
        m.close()
