"""The OpenMP build of the oracle (used only to time the CPU baseline) computes exactly
what the plain build computes: the same block sets, distances, weights, label counts,
most probable labels, statistics and meshes, over street frames with four cameras."""
import numpy as np

import oracle
import synth


def _run(variant, w, frames):
    m = oracle.OracleMap(w.voxel, w.trunc, w.n_classes, w.max_blocks, variant=variant)
    out = []
    for f in frames:
        assert m.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
        for T, lab, cam in f.cams:
            assert m.integrate_labels(cam, lab, T) == oracle.OK
        st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_DIRTY)
        assert st == oracle.OK
        out.append((m.stats(), pos.copy(), lab.copy(), keys.copy()))
    blocks = {tuple(b): m.block(b) for b in m.block_coords()}
    m.close()
    return out, blocks


def test_openmp_build_equals_plain_build():
    w = synth.street_workload(n_frames=2, n_cams=4)
    frames = [w.frame(k) for k in range(2)]
    assert oracle.threads("plain") == 1
    a, ba = _run("plain", w, frames)
    b, bb = _run("omp", w, frames)
    for (sa, pa, la, ka), (sb, pb, lb, kb) in zip(a, b):
        assert sa == sb
        assert np.array_equal(pa.view(np.int32), pb.view(np.int32))  # same order, same bits
        assert np.array_equal(la, lb) and np.array_equal(ka, kb)
    assert list(ba) == list(bb)  # same blocks in the same slot order
    for k in ba:
        for f in ("D", "W", "fused", "counts", "band"):
            assert np.array_equal(ba[k][f].view(np.uint8), bb[k][f].view(np.uint8)), (k, f)
