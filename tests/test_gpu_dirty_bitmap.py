"""GPU checks of dirty meshing's two candidate searches: the sweep of the allocated slots
and the dirty bitmap that the TSDF pass keeps once a map is large (forced here on street
maps by a threshold of 0 blocks).

Every extraction of the bitmap map is compared with the oracle's dirty mesh (triangles
as multisets of edge keys and labels, vertices within 1e-4 voxel) and with a map that
sweeps, and the stats say which search ran.  The sequence covers what must fall back to a
sweep: an extraction that does not fit its buffer (the dirty set is kept, the bitmap was
cleared by the counting pass), a frame integrated above the threshold (its marks are not
in the bitmap), a change of meshing schedule (the bitmap's layout follows the counting
grid), two frames meshed by one extraction, ALL extractions in between, and batched steps
(which mark the bitmap but mesh by their own sweep) followed by plain calls.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import camera_model, compare_mesh, lidar_model, step_log

pytestmark = pytest.mark.gpu

N_FRAMES = 10
NEVER = 1 << 40  # a threshold no pool reaches


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    import paper_2412_00291_amd  # noqa: F401
    return torch


def _mesh(torch, m, cap=None):
    """DIRTY extraction with room for every triangle (counted by an ALL extraction first,
    which leaves the dirty set alone) or for `cap` triangles."""
    from paper_2412_00291_amd import MAP_MESH_ALL, MAP_MESH_DIRTY
    if cap is None:
        _, n_all = m.extract_mesh(MAP_MESH_ALL, None, None, allow_small=True)
        cap = max(n_all, 1)
    pos = torch.zeros((cap, 3, 3), dtype=torch.float32, device="cuda")
    lab = torch.zeros((cap, 3), dtype=torch.uint8, device="cuda")
    key = torch.zeros((cap, 3), dtype=torch.int64, device="cuda")
    st, n = m.extract_mesh(MAP_MESH_DIRTY, pos, lab, key, allow_small=True)
    k = min(n, cap)
    return {"status": st, "n": n, "pos": pos[:k].cpu().numpy(), "lab": lab[:k].cpu().numpy(),
            "keys": key[:k].cpu().numpy()}


def test_bitmap_equals_sweep_and_oracle(torch_mod):
    torch = torch_mod
    from paper_2412_00291_amd import MAP_ERR_BUFFER_TOO_SMALL, MAP_OK, Map
    w = synth.street_workload(n_frames=N_FRAMES, n_cams=1)
    lid = lidar_model(w.lidar)
    cam = camera_model(w.cameras[0])
    m_bits = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    m_bits.set_dirty_bitmap(0)
    m_sweep = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    m_sweep.set_dirty_bitmap(NEVER)
    om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    seen = {0: 0, 1: 0}
    for k in range(N_FRAMES):
        f = w.frame(k)
        step_log(f"dirty bitmap: street frame {k}")
        rng = torch.from_numpy(f.range).cuda()
        T, lab, c = f.cams[0]
        labd = torch.from_numpy(np.ascontiguousarray(lab)).cuda()
        if k == 5:
            m_bits.set_dirty_bitmap(NEVER)  # this frame's marks stay out of the bitmap
        if k == 7:
            m_bits.set_schedule(0, 0, 0)    # the counting grid (and the layout) may change
        for m in (m_bits, m_sweep):
            m.integrate_lidar(lid, rng, f.T_wl)
            m.integrate_labels(cam, labd, T)
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
        assert om.integrate_labels(c, lab, T) == oracle.OK
        if k == 5:
            m_bits.set_dirty_bitmap(0)
        if k == 8:
            continue  # frames 8 and 9 are meshed by one extraction
        expect_bits = {0: 1, 1: 1, 2: 0, 3: 1, 4: 1, 5: 0, 6: 1, 7: None, 9: 1}[k]
        if k == 2:  # too small a buffer: the dirty set is kept, and the retry must sweep
            small = _mesh(torch, m_bits, cap=1)
            assert small["status"] == MAP_ERR_BUFFER_TOO_SMALL and small["n"] > 1
            assert m_bits.stats()[1]["mesh_from_bitmap"] == 1
        gb = _mesh(torch, m_bits)
        gs = _mesh(torch, m_sweep)
        assert gb["status"] == MAP_OK and gs["status"] == MAP_OK
        _, opos, olab, okeys, on = om.extract_mesh(oracle.MESH_DIRTY)
        rb = compare_mesh(gb, (opos, olab, okeys), voxel=w.voxel)
        compare_mesh(gs, (opos, olab, okeys), voxel=w.voxel)
        sb, ss = m_bits.stats()[1], m_sweep.stats()[1]
        o = om.stats()
        for key in ("mesh_blocks", "triangles", "allocated"):
            assert sb[key] == ss[key] == o[key], (k, key, sb[key], ss[key], o[key])
        assert ss["mesh_from_bitmap"] == 0
        if expect_bits is not None:
            assert sb["mesh_from_bitmap"] == expect_bits, (k, sb["mesh_from_bitmap"])
        seen[sb["mesh_from_bitmap"]] += 1
        step_log(f"dirty bitmap: frame {k} {rb['triangles']} triangles, bitmap {sb['mesh_from_bitmap']}")
    assert seen[1] >= 6 and seen[0] >= 2
    om.close()
    m_bits.close()
    m_sweep.close()


def test_bitmap_after_batched_steps(torch_mod):
    """Batched steps mark the bitmap of a map above its threshold and mesh by their own
    sweep; plain frames and bitmap extractions afterwards still equal the oracle."""
    torch = torch_mod
    from paper_2412_00291_amd import MAP_OK, Batch, Map
    w = synth.street_workload(n_frames=6, n_cams=1)
    lid = lidar_model(w.lidar)
    cam = camera_model(w.cameras[0])
    m = Map(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    m.set_dirty_bitmap(0)
    om = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, w.max_blocks)
    cap = 1 << 21
    bufs = (torch.empty((cap, 3, 3), dtype=torch.float32, device="cuda"),
            torch.empty((cap, 3), dtype=torch.uint8, device="cuda"),
            torch.empty((cap, 3), dtype=torch.int64, device="cuda"))
    batch = Batch([m], schedule=0, grid=1024, use_graph=True)
    stream = torch.cuda.Stream()
    for k in range(6):
        f = w.frame(k)
        step_log(f"dirty bitmap: batched/plain frame {k}")
        T, lab, c = f.cams[0]
        rng = torch.from_numpy(f.range).cuda()
        labd = torch.from_numpy(np.ascontiguousarray(lab)).cuda()
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
        assert om.integrate_labels(c, lab, T) == oracle.OK
        _, opos, olab, okeys, on = om.extract_mesh(oracle.MESH_DIRTY)
        if k < 3:
            with torch.cuda.stream(stream):
                st, ns = batch.step([{"map_index": 0, "lidar": lid, "range": rng, "T_wl": f.T_wl, "cams": [cam],
                                      "labels": [labd], "T_wc": [T], "pos": bufs[0], "lab": bufs[1],
                                      "keys": bufs[2]}])
            stream.synchronize()
            n = ns[0]
            g = {"n": n, "pos": bufs[0][:n].cpu().numpy(), "lab": bufs[1][:n].cpu().numpy(),
                 "keys": bufs[2][:n].cpu().numpy()}
            if k == 2:
                batch.close()
        else:
            m.integrate_lidar(lid, rng, f.T_wl)
            m.integrate_labels(cam, labd, T)
            g = _mesh(torch, m)
            assert g["status"] == MAP_OK
            assert m.stats()[1]["mesh_from_bitmap"] == 1
        compare_mesh(g, (opos, olab, okeys), voxel=w.voxel)
    om.close()
    m.close()
