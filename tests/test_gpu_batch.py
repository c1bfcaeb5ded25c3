"""GPU checks of the batched step (many maps of uneven size, one launch per phase,
replayed from a captured hipGraph): every map ends bit-identical to its own sequence of
plain calls, per-step meshes are equal, for both schedules; one map is also compared
with the oracle directly."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import camera_model, canonical_mesh, compare_state, lidar_model, sorted_download, step_log

pytestmark = pytest.mark.gpu

N_MAPS = 16
MAX_BLOCKS = 1 << 16
CAP = 1 << 21


@pytest.fixture(scope="module")
def batch_data():
    import torch
    ws = synth.batched_workloads(seed=3, n_maps=N_MAPS)
    data = []
    for m, w in enumerate(ws):
        nfr = 2 + (m % 3)  # uneven frame counts
        frames = []
        for k in range(nfr):
            f = w.frame(k)
            T, lab, cam = f.cams[0]
            frames.append({"range": torch.from_numpy(f.range).cuda(), "T_wl": f.T_wl,
                           "labels": torch.from_numpy(np.ascontiguousarray(lab)).cuda(), "T_wc": T,
                           "host": f})
        data.append((w, frames))
    torch.cuda.synchronize()
    step_log(f"batch: generated {sum(len(f) for _, f in data)} frames over {N_MAPS} maps")
    return data


def _mesh_bufs(torch):
    return (torch.empty((CAP, 3, 3), dtype=torch.float32, device="cuda"),
            torch.empty((CAP, 3), dtype=torch.uint8, device="cuda"),
            torch.empty((CAP, 3), dtype=torch.int64, device="cuda"))


def _mesh_multiset(pos, lab, keys, n):
    return canonical_mesh(pos[:n].cpu().numpy(), lab[:n].cpu().numpy(), keys[:n].cpu().numpy())


def _run_sequential(torch, data):
    from paper_2412_00291_amd import Map, MAP_MESH_DIRTY
    maps = [Map(w.voxel, w.trunc, w.n_classes, MAX_BLOCKS) for w, _ in data]
    pos, lab, keys = _mesh_bufs(torch)
    meshes = {}
    n_steps = max(len(f) for _, f in data)
    for k in range(n_steps):
        for mi, (w, frames) in enumerate(data):
            if k >= len(frames):
                continue
            fr = frames[k]
            m = maps[mi]
            m.integrate_lidar(lidar_model(w.lidar), fr["range"], fr["T_wl"])
            m.integrate_labels_multi([camera_model(w.cameras[0])], [fr["labels"]], [fr["T_wc"]])
            st, n = m.extract_mesh(MAP_MESH_DIRTY, pos, lab, keys)
            meshes[(mi, k)] = _mesh_multiset(pos, lab, keys, n)
    return maps, meshes


def _run_batched(torch, data, schedule, grid):
    from paper_2412_00291_amd import Batch, Map
    maps = [Map(w.voxel, w.trunc, w.n_classes, MAX_BLOCKS) for w, _ in data]
    batch = Batch(maps, schedule=schedule, grid=grid, use_graph=True)
    bufs = [_mesh_bufs(torch) for _ in data]
    stream = torch.cuda.Stream()
    meshes = {}
    n_steps = max(len(f) for _, f in data)
    with torch.cuda.stream(stream):
        for k in range(n_steps):
            items = []
            for mi, (w, frames) in enumerate(data):
                if k >= len(frames):
                    continue
                fr = frames[k]
                pos, lab, keys = bufs[mi]
                items.append({"map_index": mi, "lidar": lidar_model(w.lidar), "range": fr["range"],
                              "T_wl": fr["T_wl"], "cams": [camera_model(w.cameras[0])], "labels": [fr["labels"]],
                              "T_wc": [fr["T_wc"]], "pos": pos, "lab": lab, "keys": keys})
            st, ns = batch.step(items)
            for it, n in zip(items, ns):
                pos, lab, keys = bufs[it["map_index"]]
                meshes[(it["map_index"], k)] = _mesh_multiset(pos, lab, keys, n)
            step_log(f"batch: schedule {schedule} step {k} done ({len(items)} maps)")
    stream.synchronize()
    return maps, batch, meshes


@pytest.mark.parametrize("schedule,grid", [(0, 2048), (1, 1024), (2, 4096), (3, 1024)])
def test_batched_equals_sequential(torch_dev_batch, batch_data, schedule, grid):
    torch = torch_dev_batch
    seq_maps, seq_meshes = _run_sequential(torch, batch_data)
    bat_maps, batch, bat_meshes = _run_batched(torch, batch_data, schedule, grid)
    assert set(seq_meshes) == set(bat_meshes)
    for key in seq_meshes:
        assert np.array_equal(seq_meshes[key], bat_meshes[key]), key
    n_blocks = 0
    for mi in range(N_MAPS):
        a, b = sorted_download(seq_maps[mi]), sorted_download(bat_maps[mi])
        for k in ("coords", "D", "W", "fused", "counts"):
            assert np.array_equal(a[k], b[k]), (mi, k)
        st_a, sa = seq_maps[mi].stats()
        st_b, sb = bat_maps[mi].stats()
        for k in ("touched", "new_blocks", "updates", "votes", "allocated", "frames", "triangles"):
            assert sa[k] == sb[k], (mi, k, sa[k], sb[k])
        n_blocks += len(a["coords"])
    assert n_blocks > 10000
    # one map of the batch against the oracle
    w, frames = batch_data[0]
    om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, MAX_BLOCKS)
    for fr in frames:
        f = fr["host"]
        om.integrate_lidar(w.lidar, f.range, f.T_wl)
        T, lab, cam = f.cams[0]
        om.integrate_labels(cam, lab, T)
    compare_state(bat_maps[0], om)
    batch.close()
    for m in seq_maps + bat_maps:
        m.close()


@pytest.fixture(scope="module")
def torch_dev_batch():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch
