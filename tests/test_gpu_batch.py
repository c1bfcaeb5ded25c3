"""GPU checks of the batched step (many maps of uneven size, one launch per phase,
replayed from a captured hipGraph).

* Every map of the batch (voxels 0.05 to 0.4 m, 16/32/64 beams, 1024 to 2048 columns) is
  run for 10 to 12 frames by plain calls next to the CPU oracle: per-frame counters and
  dirty meshes after every frame, and the whole state (blocks, D, W, label counts, fused
  labels) at the end, are compared with the oracle.
* The batched step, for each schedule, leaves every map bit-identical to those plain calls,
  with per-step meshes equal as multisets.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import camera_model, compare_mesh, compare_state, lidar_model, sorted_download, step_log

pytestmark = pytest.mark.gpu

N_MAPS = 16
MAX_BLOCKS = 1 << 16
CAP = 1 << 21


def frames_of(m):
    return 10 + (m % 3)  # uneven frame counts, at least 10 per map


@pytest.fixture(scope="module")
def batch_data():
    import torch
    ws = synth.batched_workloads(seed=3, n_maps=N_MAPS)
    data = []
    for m, w in enumerate(ws):
        frames = []
        for k in range(frames_of(m)):
            f = w.frame(k)
            T, lab, cam = f.cams[0]
            frames.append({"range": torch.from_numpy(f.range).cuda(), "T_wl": f.T_wl,
                           "labels": torch.from_numpy(np.ascontiguousarray(lab)).cuda(), "T_wc": T,
                           "host": f})
        data.append((w, frames))
        step_log(f"batch: map {m} ({w.name}) {len(frames)} frames generated")
    torch.cuda.synchronize()
    return data


def _mesh_bufs(torch):
    return (torch.empty((CAP, 3, 3), dtype=torch.float32, device="cuda"),
            torch.empty((CAP, 3), dtype=torch.uint8, device="cuda"),
            torch.empty((CAP, 3), dtype=torch.int64, device="cuda"))


_MIX = np.array([0x9E3779B97F4A7C15, 0xC2B2AE3D27D4EB4F, 0x165667B19E3779F9, 0xD6E8FEB86659FD93,
                 0xFF51AFD7ED558CCD, 0xC4CEB9FE1A85EC53, 0x94D049BB133111EB, 0xBF58476D1CE4E5B9,
                 0x2545F4914F6CDD1D, 0x9FB21C651E98DF25, 0xA0761D6478BD642F, 0xE7037ED1A0B428DB,
                 0x8EBC6AF09C88C6E3, 0x589965CC75374CC3, 0x1D8E4E27C47D124F], dtype=np.uint64)


def _multiset_digest(pos, lab, keys):
    """Order-independent digest of a triangle soup: each triangle's (3 edge keys, 3 labels,
    9 position bit patterns) mixed into 64 bits, summed modulo 2^64, with the count."""
    n = len(keys)
    rows = np.concatenate([np.asarray(keys, np.int64).reshape(n, 3).view(np.uint64),
                           np.asarray(lab, np.uint64).reshape(n, 3),
                           np.ascontiguousarray(pos, np.float32).reshape(n, 9).view(np.uint32).astype(np.uint64)],
                          axis=1)
    with np.errstate(over="ignore"):
        h = (rows * _MIX).sum(axis=1, dtype=np.uint64)
        h ^= h >> np.uint64(31)
        h *= np.uint64(0x7FB5D329728EA185)
        h ^= h >> np.uint64(27)
        return n, int(h.sum(dtype=np.uint64))


def _download_mesh(bufs, n):
    pos, lab, keys = bufs
    return pos[:n].cpu().numpy(), lab[:n].cpu().numpy(), keys[:n].cpu().numpy()


@pytest.fixture(scope="module")
def sequential(torch_dev_batch, batch_data):
    """Every map by plain calls, map after map, next to the oracle (OpenMP build: the
    results are those of the plain build); per-frame meshes compared with the oracle's."""
    torch = torch_dev_batch
    from paper_2412_00291_amd import Map, MAP_MESH_DIRTY
    maps = [Map(w.voxel, w.trunc, w.n_classes, MAX_BLOCKS) for w, _ in batch_data]
    bufs = _mesh_bufs(torch)
    digests = {}
    for mi, (w, frames) in enumerate(batch_data):
        m = maps[mi]
        om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, MAX_BLOCKS, variant="omp")
        for k, fr in enumerate(frames):
            f = fr["host"]
            m.integrate_lidar(lidar_model(w.lidar), fr["range"], fr["T_wl"])
            m.integrate_labels_multi([camera_model(w.cameras[0])], [fr["labels"]], [fr["T_wc"]])
            st, n = m.extract_mesh(MAP_MESH_DIRTY, *bufs)
            assert st == 0
            gpos, glab, gkeys = _download_mesh(bufs, n)
            digests[(mi, k)] = _multiset_digest(gpos, glab, gkeys)
            assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
            T, lab, cam = f.cams[0]
            assert om.integrate_labels(cam, lab, T) == oracle.OK
            ost, opos, olab, okeys, on = om.extract_mesh(oracle.MESH_DIRTY)
            compare_mesh({"n": n, "pos": gpos, "lab": glab, "keys": gkeys}, (opos, olab, okeys), voxel=w.voxel)
            st_, s = m.stats()
            o = om.stats()
            for key in ("touched", "new_blocks", "updates", "votes", "allocated", "mesh_blocks", "triangles"):
                assert s[key] == o[key], (mi, k, key, s[key], o[key])
        rep = compare_state(m, om)
        assert rep["non_identical"] == 0, (mi, rep)
        om.close()
        step_log(f"batch: map {mi} ({w.name}) equals the oracle over {len(frames)} frames: {rep}")
    yield maps, digests
    for m in maps:
        m.close()


def _run_batched(torch, data, schedule, grid):
    from paper_2412_00291_amd import Batch, Map
    maps = [Map(w.voxel, w.trunc, w.n_classes, MAX_BLOCKS) for w, _ in data]
    batch = Batch(maps, schedule=schedule, grid=grid, use_graph=True)
    bufs = [_mesh_bufs(torch) for _ in data]
    stream = torch.cuda.Stream()
    digests = {}
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
                digests[(it["map_index"], k)] = _multiset_digest(*_download_mesh(bufs[it["map_index"]], n))
            step_log(f"batch: schedule {schedule} step {k} done ({len(items)} maps)")
    stream.synchronize()
    return maps, batch, digests


@pytest.mark.parametrize("schedule,grid", [(0, 2048), (1, 1024), (2, 4096), (3, 1024), (4, 4)])
def test_batched_equals_plain_calls_and_oracle(torch_dev_batch, batch_data, sequential, schedule, grid):
    torch = torch_dev_batch
    seq_maps, seq_digests = sequential
    bat_maps, batch, bat_digests = _run_batched(torch, batch_data, schedule, grid)
    assert set(seq_digests) == set(bat_digests)
    for key in seq_digests:
        assert seq_digests[key] == bat_digests[key], key
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
    batch.close()
    for m in bat_maps:
        m.close()


@pytest.fixture(scope="module")
def torch_dev_batch():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch
