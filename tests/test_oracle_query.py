"""Pins of the oracle's trilinear SDF query and its SE(3) pose / point adjoint.

The query interpolates the stored distances at voxel centres x = nu v (Sec. IV-C.2)
trilinearly; the loss of a posed scan is sum_j D(Exp(w) p_j + t)^2.  Pinned by: exact
values at voxel centres, exact reproduction of a linear field and its gradient, and fp64
central differences (step 1e-4) of the loss with respect to the pose and the points,
excluding stencils that cross a cell face or a validity change.
"""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def tiny_map():
    w = synth.tiny_workload()
    m = oracle.OracleMap(w.voxel, w.trunc, w.n_classes)
    f = w.frame(0, with_labels=False)
    assert m.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    return w, m


def test_exact_at_voxel_centres(tiny_map):
    w, m = tiny_map
    nu = float(np.float32(w.voxel))
    n = 0
    for b in m.touched()[:200]:
        blk = m.block(b)
        i = np.arange(512)
        v = np.stack([i & 7, (i >> 3) & 7, i >> 6], 1) + 8 * np.asarray(b)
        x = v.astype(np.float64) * nu
        sdf, grad, valid = m.query_sdf(x, mode=0)
        np.testing.assert_allclose(sdf[valid], blk["D"][valid].astype(np.float64), atol=1e-12)
        assert np.all(blk["W"][valid] > 0)
        n += int(valid.sum())
    assert n > 1000


def test_linear_field_value_and_gradient():
    nu = np.float32(0.1)
    m = oracle.OracleMap(float(nu), 0.3, 2)
    a = np.array([0.25, -0.5, 0.125])  # dyadic: every stored value is exact in fp32
    b0 = 0.75
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                i = np.arange(512)
                v = np.stack([i & 7, (i >> 3) & 7, i >> 6], 1) + 8 * np.array([bx, by, bz])
                m.set_block((bx, by, bz), D=(v @ a + b0).astype(np.float32), W=np.ones(512, np.float32))
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.uniform(0.0, 14.99, size=(2000, 3)) * float(nu)
    sdf, grad, valid = m.query_sdf(x, mode=0)
    assert valid.all()
    np.testing.assert_allclose(sdf, (x / float(nu)) @ a + b0, atol=1e-12)
    np.testing.assert_allclose(grad, np.broadcast_to(a / float(nu), grad.shape), rtol=1e-12)
    # outside the allocated blocks: invalid, zero
    sdf, grad, valid = m.query_sdf(np.array([[-0.05, 0.3, 0.3], [1.55, 0.3, 0.3]]), mode=0)
    assert not valid.any() and np.all(sdf == 0)


def _loss_at(m, xi, p):
    loss, _, _, margin = m.pose_adjoint(xi[None], p[None, None])
    return loss[0], margin[0, 0]


def _richardson(m, xi, p, h, kind, i):
    """Central differences at h and h/2, Richardson-extrapolated (O(h^4) error); None if
    the stencil leaves the cell or changes validity."""
    vals, ok = {}, set()
    for s in (-1.0, -0.5, 0.0, 0.5, 1.0):
        x2, p2 = xi.copy(), p.copy()
        if kind == "xi":
            x2[i] += s * h
        else:
            p2[i] = np.float32(p2[i] + np.float32(s * h))
        v, mg = _loss_at(m, x2, p2)
        if mg < 0.01:
            return None
        vals[s] = v
        ok.add(v != 0.0)
    if len(ok) != 1:
        return None
    d1 = (vals[1.0] - vals[-1.0]) / (2 * h)
    d2 = (vals[0.5] - vals[-0.5]) / h
    return (4 * d2 - d1) / 3, d1


def test_pose_and_point_gradients_vs_central_differences(tiny_map):
    w, m = tiny_map
    pts = synth.scan_points(w, synth.uniform_lidar(64, 2048, 15.0, -15.0, 40.0), w.poses[0], 131072, seed=4)
    rng = np.random.Generator(np.random.PCG64(6))
    sel = pts[rng.choice(len(pts), size=120, replace=False)]
    xis = [np.zeros(6), np.array([0.02, -0.01, 0.015, 0.01, -0.02, 0.03]),
           np.array([0.05, 0.1, -0.05, 0.2, -0.15, 0.1])]  # zero, series and closed-form branches
    h_xi = 1e-4
    h_p = 2.0 ** -13  # p +- h and p +- h/2 are exact in fp32 for |p| < 512
    n_checked = 0
    for xi in xis:
        for p in sel:
            loss, gxi, gpts, margin = m.pose_adjoint(xi[None], p[None, None])
            if loss[0] == 0.0 or margin[0, 0] < 0.05:
                continue
            for i in range(6):
                r = _richardson(m, xi, p, h_xi, "xi", i)
                if r is None:
                    continue
                ext, fd = r
                g = gxi[0, i]
                assert abs(ext - g) <= 1e-6 * max(1.0, abs(g)), (xi, p, i, ext, fd, g)
                assert abs(fd - g) <= 2e-3 * max(1.0, abs(g))  # plain central difference, step 1e-4
                n_checked += 1
            for i in range(3):
                r = _richardson(m, xi, p.astype(np.float32), h_p, "p", i)
                if r is None:
                    continue
                ext, fd = r
                g = gpts[0, 0, i]
                assert abs(ext - g) <= 1e-6 * max(1.0, abs(g)), (xi, p, i, ext, fd, g)
                n_checked += 1
    assert n_checked > 500


def test_batch_sums_and_query_consistency(tiny_map):
    w, m = tiny_map
    pts = synth.scan_points(w, synth.uniform_lidar(64, 2048, 15.0, -15.0, 40.0), w.poses[0], 131072, seed=4)
    sub = pts[::97][:1000]
    xi = np.array([0.03, -0.02, 0.01, 0.01, 0.02, -0.01])
    loss, gxi, gpts, _ = m.pose_adjoint(np.stack([np.zeros(6), xi]), np.stack([sub, sub]))
    sdf, grad, valid = m.query_sdf(sub.astype(np.float64), mode=0)
    assert abs(loss[0] - np.sum(sdf[valid] ** 2)) <= 1e-12 * max(1, loss[0])
    np.testing.assert_allclose(gpts[0], 2 * sdf[:, None] * grad, atol=1e-12)  # R = I at xi = 0
    np.testing.assert_allclose(gxi[0, :3], gpts[0].sum(0), rtol=1e-10, atol=1e-12)
    per = np.array([m.pose_adjoint(xi[None], p[None, None])[1][0] for p in sub[:200]])
    l200, g200, _, _ = m.pose_adjoint(xi[None], sub[None, :200])
    np.testing.assert_allclose(g200[0], per.sum(0), rtol=1e-9, atol=1e-10)
