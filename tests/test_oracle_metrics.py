"""Pins of the oracle's map-quality metrics (Sec. V-C, Eq. 7, Eq. 8; RC, mIoU, Acc):
closed forms on shifted copies and far-away clouds, brute-force nearest neighbours with
the tie rule on lattices, a known confusion matrix, and a reconstructed sphere against
points on the analytic sphere."""
import numpy as np

import oracle
import synth
from oracle import metrics

NU = 0.1


def _spread_points(rng, n, spacing):
    """n points on a jittered lattice of the given spacing (nearest distinct points are at
    least 0.6 spacing apart)."""
    side = int(np.ceil(n ** (1 / 3))) + 1
    g = np.stack(np.meshgrid(*[np.arange(side)] * 3, indexing="ij"), -1).reshape(-1, 3)[:n]
    return (g + rng.uniform(-0.2, 0.2, size=g.shape)) * spacing


def test_shifted_copy_closed_form():
    rng = np.random.default_rng(0)
    G = _spread_points(rng, 5000, 1.0)
    u = rng.normal(size=G.shape)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    delta = 0.07
    M = G + delta * u
    lab = rng.integers(0, 5, size=len(G)).astype(np.uint8)
    r = metrics.mesh_metrics(M, lab, G, lab, NU, 5)
    assert abs(r["re"] - delta) < 1e-12 and abs(r["cd"] - delta) < 1e-12 and r["rc"] == 1.0
    assert r["miou"] == 1.0 and r["acc"] == 1.0 and r["n_eval"] == len(G)
    # beyond the cap every distance counts 2 nu and nothing is covered
    far = G + 0.5 * u
    r = metrics.mesh_metrics(far, lab, G, lab, NU, 5)
    assert abs(r["re"] - 2 * NU) < 1e-12 and abs(r["cd"] - 2 * NU) < 1e-12 and r["rc"] == 0.0
    assert r["n_eval"] == 0


def test_nearest_matches_brute_force_with_ties():
    rng = np.random.default_rng(1)
    dst = np.stack(np.meshgrid(*[np.arange(6)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.float64) * 0.1
    # queries at lattice points, edge midpoints, face centres and cube centres (many ties)
    src = np.concatenate([dst[:40] + 0.05 * rng.integers(0, 2, size=(40, 3)), rng.uniform(0, 0.5, size=(300, 3))])
    d, i = metrics.nearest(src, dst)
    D = np.linalg.norm(src[:, None, :] - dst[None, :, :], axis=2)
    dmin = D.min(axis=1)
    want = np.array([np.nonzero(D[k] == dmin[k])[0].min() for k in range(len(src))])
    np.testing.assert_allclose(d, dmin, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(i, want)


def test_known_confusion():
    """G of three classes; the vertices' labels are G's except: 30 points of class 0 labelled
    1, 20 of class 2 unlabelled (255).  TP, FP, FN and both scores follow."""
    rng = np.random.default_rng(2)
    G = _spread_points(rng, 300, 1.0)
    G_lab = np.repeat(np.arange(3), 100).astype(np.uint8)
    M_lab = G_lab.copy()
    M_lab[:30] = 1
    M_lab[200:220] = 255
    M = G + 0.01
    r = metrics.mesh_metrics(M, M_lab, G, G_lab, NU, 3)
    tp = np.array([70, 100, 80])
    fp = np.array([0, 30, 0])
    fn = np.array([30, 0, 20])
    np.testing.assert_array_equal(np.diag(r["confusion"][:3]), tp)
    assert abs(r["miou"] - np.mean(tp / (tp + fp + fn))) < 1e-12
    assert abs(r["acc"] - tp.sum() / 300) < 1e-12


def test_sphere_reconstruction_against_analytic_surface():
    """The oracle's mesh of a sphere seen from inside, against points sampled on the
    sphere: every vertex within the marching-cubes error bound nu^2 / (8 (R - nu)) of the
    surface (plus the sampling gap), full coverage of the scanned part."""
    lidar = synth.uniform_lidar(64, 720, 40.0, -40.0, 40.0)
    R = 3.0
    om = oracle.OracleMap(NU, 3 * NU, 2, 1 << 18)
    T = synth.pose_matrix(np.eye(3), [0, 0, 0])
    assert om.integrate_lidar(lidar, synth.constant_range(lidar, R), T) == oracle.OK
    st, pos, lab, keys, n = om.extract_mesh(oracle.MESH_ALL)
    V = np.unique(pos.reshape(-1, 3).astype(np.float64), axis=0)
    # ground truth: the sphere sampled densely inside the scanned band of elevations
    rng = np.random.default_rng(3)
    g = rng.normal(size=(400000, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    g = g[np.abs(np.arcsin(g[:, 2])) < np.deg2rad(38.0)] * R
    gl = np.zeros(len(g), np.uint8)
    r = metrics.mesh_metrics(V, np.zeros(len(V), np.uint8), g, gl, NU, 2)
    gap = np.sqrt(4 * np.pi * R * R / 400000) * 2
    assert r["re"] < NU * NU / (8 * (R - NU)) + gap and r["rc"] > 0.999
