"""Helpers for GPU parity tests: model conversion, GPU/oracle state and mesh comparison."""
import os
import time

import numpy as np

import oracle


def step_log(msg):
    """Append a progress line (naming the step before it runs) to the file that
    $MAPCORE_STEP_LOG names, if it is set."""
    path = os.environ.get("MAPCORE_STEP_LOG")
    if not path:
        return
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path, "a") as fh:
        fh.write(f"{time.strftime('%H:%M:%S')} {msg}\n")


def lidar_model(l):
    from paper_2412_00291_amd import LidarModel
    return LidarModel(l.rows, l.cols, np.ascontiguousarray(l.elev_rad, np.float32), float(l.r_max))


def camera_model(c):
    from paper_2412_00291_amd import CameraModel
    return CameraModel(c.width, c.height, float(c.fx), float(c.fy), float(c.cx), float(c.cy))


def compare_state(m, om, d_tol=1e-5, exact_labels=True):
    """GPU map vs oracle map: identical block sets; D, W within 1e-5 relative (D on the
    truncation scale); label counts and fused labels bit-exact.  Returns a report."""
    g = m.download(with_counts=True)
    gkeys = [tuple(b) for b in g["coords"]]
    okeys = [tuple(b) for b in om.block_coords()]
    assert len(set(gkeys)) == len(gkeys), "duplicate block on the GPU"
    assert set(gkeys) == set(okeys), (len(set(gkeys) - set(okeys)), len(set(okeys) - set(gkeys)))
    tau = np.float32(om.trunc)
    n_obs = 0
    n_diff = 0
    for i, b in enumerate(gkeys):
        ob = om.block(b)
        Dg, Wg = g["D"][i], g["W"][i]
        assert np.all(np.abs(Wg - ob["W"]) <= d_tol * np.maximum(np.abs(ob["W"]), 1e-30)), b
        assert np.all(np.abs(Dg - ob["D"]) <= d_tol * tau), b
        n_diff += int(np.count_nonzero((Dg != ob["D"]) | (Wg != ob["W"])))
        if exact_labels:
            np.testing.assert_array_equal(g["counts"][i], ob["counts"], err_msg=str(b))
            np.testing.assert_array_equal(g["fused"][i], ob["fused"], err_msg=str(b))
        n_obs += int(np.count_nonzero(ob["W"] > 0))
    return {"blocks": len(gkeys), "voxels": n_obs, "non_identical": n_diff}


def canonical_mesh(pos, lab, keys):
    """Triangles as rows [3 edge keys, 3 labels, 9 position bit patterns], lexicographically
    sorted: two meshes are equal as multisets iff these matrices are equal."""
    n = len(keys)
    rows = np.concatenate([np.asarray(keys, np.int64).reshape(n, 3),
                           np.asarray(lab, np.int64).reshape(n, 3),
                           np.ascontiguousarray(pos, np.float32).reshape(n, 9).view(np.int32).astype(np.int64)], axis=1)
    if n == 0:
        return rows
    order = np.lexsort(rows.T[::-1])
    return rows[order]


def sorted_download(m):
    d = m.download()
    order = np.lexsort(d["coords"].T[::-1])
    return {k: v[order] for k, v in d.items()}


def gpu_mesh(m, mode, cap=None):
    import torch
    from paper_2412_00291_amd import MAP_OK, MAP_ERR_BUFFER_TOO_SMALL
    if cap is None:
        st, n = m.extract_mesh(1, None, None, allow_small=True)  # ALL: count only (no dirty change)
        cap = max(n, 1)
        if mode == 0:
            cap = max(cap, 1)
    pos = torch.zeros((cap, 3, 3), dtype=torch.float32, device="cuda")
    lab = torch.zeros((cap, 3), dtype=torch.uint8, device="cuda")
    key = torch.zeros((cap, 3), dtype=torch.int64, device="cuda")
    st, n = m.extract_mesh(mode, pos, lab, key, allow_small=True)
    k = min(n, cap)
    return {"status": st, "n": n, "pos": pos[:k].cpu().numpy(), "lab": lab[:k].cpu().numpy(),
            "keys": key[:k].cpu().numpy()}


def compare_mesh(gm, om_mesh, tol_vox=1e-4, voxel=None):
    """Triangles equal as multisets of (edge-key triple, label triple); vertices at the
    same edge key within tol_vox voxel."""
    pos, lab, keys = om_mesh
    assert gm["n"] == len(keys), (gm["n"], len(keys))
    a = canonical_mesh(np.zeros((gm["n"], 3, 3), np.float32), gm["lab"], gm["keys"])[:, :6]
    b = canonical_mesh(np.zeros((len(keys), 3, 3), np.float32), lab, keys)[:, :6]
    assert np.array_equal(a, b)
    err = 0.0
    if len(keys):
        gk, gi = np.unique(gm["keys"].reshape(-1), return_index=True)
        ok_, oi = np.unique(keys.reshape(-1), return_index=True)
        assert np.array_equal(gk, ok_)
        err = float(np.abs(gm["pos"].reshape(-1, 3)[gi].astype(np.float64) -
                           pos.reshape(-1, 3)[oi].astype(np.float64)).max())
    if voxel is not None:
        assert err <= tol_vox * voxel, err
    return {"triangles": gm["n"], "max_err_vox": err / voxel if voxel else err}
