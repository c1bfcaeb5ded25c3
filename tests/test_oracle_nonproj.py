"""Pins of the oracle's non-projective distance (the paper's "Ours", Sec. IV-C.2, Eq. 4):
the normal image and point filter, Eq. 4 as read (the printed second term restored with
its missing factor psi and its sign from the surface's bend), the gradient as the
weighted average of normals, and the whole update against closed forms.

Each pin is fixed by geometry, not by the oracle: a plane's distance along its normal,
the exact distance to a sphere or a cylinder (convex or concave, in front of or behind
the surface), a plane's normal, the incidence angle of a ray on a known plane, and the
sensor inside a sphere, where every ray is along the normal and the two distances agree.
"""
import numpy as np
import pytest

import oracle
import synth

NU, TAU = 0.1, 0.3


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------------------------------
# Eq. 4
# ---------------------------------------------------------------------------------------

def test_plane_gives_the_distance_along_the_normal():
    rng = np.random.default_rng(1)
    for _ in range(500):
        n = _unit(rng.normal(size=3)).astype(np.float32)
        u = _unit(rng.normal(size=3))
        if u @ n > -0.05:
            u = -u if u @ n > 0.05 else _unit(u - 0.5 * n)
        u = u.astype(np.float32)
        psi = np.float32(rng.uniform(-0.3, 0.3))
        d = oracle.nonproj_distance(psi, u, n, n)
        want = -float(psi) * float(u.astype(np.float64) @ n.astype(np.float64))
        assert abs(d - want) <= 2e-6 * abs(float(psi)) + 1e-9, (d, want)


def _sphere_case(rng, concave, in_front, cylinder=False):
    """A surface point p on a sphere (or a cylinder along z), the normal n there facing the
    free side, a ray u that reaches p from the free side, the voxel x = p - psi u, its
    exact signed distance (positive on the free side) and the gradient of that distance."""
    R = rng.uniform(0.5, 8.0)
    C = rng.normal(size=3) * 3
    v = rng.normal(size=3)
    if cylinder:
        v[2] = 0.0
    v = _unit(v)
    p = C + R * v
    n = -v if concave else v
    u = _unit(rng.normal(size=3))
    if u @ n > 0:
        u = -u
    psi = rng.uniform(0.01, 0.3) * (1 if in_front else -1)
    x = p - psi * u
    r = x - C
    if cylinder:
        r[2] = 0.0
    rho = np.linalg.norm(r)
    if concave:
        return psi, u, n, R - rho, -r / rho
    return psi, u, n, rho - R, r / rho


@pytest.mark.parametrize("cylinder", [False, True])
def test_sphere_and_cylinder_distances_are_exact(cylinder):
    """The printed second term, multiplied by psi and signed by the bend, makes Eq. 4 the
    exact distance to a sphere (or a cylinder) whose normal at p and gradient at x are
    the surface's; a dropped psi, a dropped term or a wrong sign fails it."""
    rng = np.random.default_rng(2 + cylinder)
    n_checked = 0
    for trial in range(4000):
        concave, in_front = bool(trial & 1), bool(trial & 2)
        psi, u, n, d_true, g = _sphere_case(rng, concave, in_front, cylinder)
        if n @ g <= 0.05 or abs(u @ n) < 0.1:
            continue
        d = oracle.nonproj_distance(psi, u, g, n)
        scale = abs(psi) + abs(d_true)
        assert abs(d - d_true) <= 2e-5 * scale, (trial, concave, in_front, d, d_true)
        n_checked += 1
    assert n_checked > 2000


def test_bend_term_changes_the_distance_on_curved_surfaces():
    """On a tightly curved surface seen obliquely the distance differs from the planar
    |cos theta| psi, in the direction of the bend: smaller in front of a convex surface,
    larger in front of a concave one."""
    rng = np.random.default_rng(5)
    signs = {True: [], False: []}
    for trial in range(2000):
        concave = bool(trial & 1)
        psi, u, n, d_true, g = _sphere_case(rng, concave, True)
        if n @ g <= 0.05 or abs(u @ n) < 0.1:
            continue
        d = oracle.nonproj_distance(psi, u, g, n)
        planar = -psi * float(u @ g)
        if abs(d - planar) > 1e-4 * abs(psi):
            signs[concave].append(np.sign(d - planar))
    assert len(signs[True]) > 100 and len(signs[False]) > 100
    assert np.all(np.array(signs[False]) < 0) and np.all(np.array(signs[True]) > 0)


def test_gradient_opposing_the_normal_is_replaced_by_it():
    rng = np.random.default_rng(6)
    for _ in range(200):
        n = _unit(rng.normal(size=3))
        g = _unit(-n + 0.3 * rng.normal(size=3))
        if n @ g > 0:
            continue
        u = _unit(-n + 0.2 * rng.normal(size=3))
        psi = rng.uniform(-0.3, 0.3)
        d = oracle.nonproj_distance(psi, u, g, n)
        assert abs(d - (-psi * (u @ n))) <= 2e-6 * abs(psi) + 1e-9


# ---------------------------------------------------------------------------------------
# normal image and point filter
# ---------------------------------------------------------------------------------------

def _lidar():
    return synth.uniform_lidar(32, 360, 15.0, -30.0, 60.0)


def _rz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


@pytest.mark.parametrize("yaw", [0.0, 0.7])
def test_plane_normals_face_the_sensor(yaw):
    lidar = _lidar()
    T = synth.pose_matrix(_rz(yaw), [0.5, -0.3, 1.2])
    n_w = _unit([0.3, -0.2, 1.0])           # a tilted ground plane below the sensor
    rng_img = synth.plane_range(lidar, T, n_w, -0.5)
    kept, nrm = oracle.normal_image(lidar, rng_img, T, max_incidence=np.pi / 2)
    valid = rng_img > 0
    has = np.zeros_like(valid)
    has[1:] = valid[1:] & valid[:-1] & np.roll(valid, 1, axis=1)[1:]
    # exactly the pixels with a valid return, a valid one above and one to the left have
    # a normal (the left neighbour of column 0 is the last column)
    assert np.array_equal(kept > 0, has) and has.sum() > 3000
    assert not np.any(kept[0])
    got = nrm[has].astype(np.float64)
    # world plane normal, facing the sensor (its origin is above the plane)
    assert np.all(np.linalg.norm(got - n_w, axis=1) < 1e-3), np.abs(got - n_w).max()
    assert np.array_equal(kept[has], rng_img[has])
    assert not np.any(nrm[~has])


def test_point_filter_drops_grazing_returns():
    lidar = _lidar()
    T = synth.pose_matrix(np.eye(3), [0.0, 0.0, 1.7])
    rng_img = synth.plane_range(lidar, T, [0.0, 0.0, 1.0], 0.0)  # flat ground
    limit = np.deg2rad(75.0)
    kept, _ = oracle.normal_image(lidar, rng_img, T, max_incidence=limit)
    kept_all, _ = oracle.normal_image(lidar, rng_img, T, max_incidence=np.pi / 2)
    # incidence of each ray on the ground: the angle between the ray and the vertical
    d = lidar.directions().reshape(lidar.rows, lidar.cols, 3)
    inc = np.arccos(np.abs(d[..., 2]))
    has = kept_all > 0
    clear = np.abs(inc - limit) > 2e-3
    assert np.array_equal((kept > 0)[has & clear], (inc <= limit)[has & clear])
    assert (kept > 0).sum() < has.sum() and (kept > 0).sum() > 0
    assert not np.any((kept > 0) & ~has)


def test_dropouts_remove_their_neighbours_normals():
    lidar = _lidar()
    T = synth.pose_matrix(np.eye(3), [0.0, 0.0, 0.0])
    rng_img = synth.constant_range(lidar, 5.0)
    rng_img[10, 20] = 0.0
    kept, nrm = oracle.normal_image(lidar, rng_img, T, max_incidence=np.pi / 2)
    assert kept[10, 20] == 0 and kept[11, 20] == 0 and kept[10, 21] == 0   # below and right of it
    assert kept[9, 20] > 0 and kept[10, 19] > 0 and kept[11, 21] > 0
    assert kept[0].sum() == 0 and kept[1:].astype(bool).sum() == (lidar.rows - 1) * lidar.cols - 3
    # inside a sphere every normal points back at the sensor along the ray
    d = lidar.directions().reshape(lidar.rows, lidar.cols, 3)
    m = kept > 0
    assert np.all(np.abs(np.einsum("ijk,ijk->ij", nrm, d)[m] + 1.0) < 2e-3)


# ---------------------------------------------------------------------------------------
# the update
# ---------------------------------------------------------------------------------------

def _pair():
    a = oracle.OracleMap(NU, TAU, 4, 1 << 18)
    b = oracle.OracleMap(NU, TAU, 4, 1 << 18)
    assert b.set_distance(oracle.DIST_NONPROJECTIVE, np.pi / 2) == oracle.OK
    return a, b


def test_sensor_inside_sphere_agrees_with_projective():
    """Every pixel's normal is along its ray up to the pixel spacing (alpha = 0 on the first
    frame), so d = psi cos theta with theta under 1.5 pixels: both modes give the same map
    to that bound, with gradients pointing back at the sensor."""
    lidar = synth.uniform_lidar(48, 720, 40.0, -40.0, 40.0)
    # a pixel's normal is that of the plane through its point and the points above and to
    # its left: on the sphere, the direction of that triangle's circumcentre, within a
    # pixel of the pixel's ray, which is within half a pixel of the voxel's ray
    one_pixel = 1.5 * np.hypot(np.deg2rad(80.0 / 47), 2 * np.pi / 720)
    proj, ours = _pair()
    rimg = synth.constant_range(lidar, 3.0)
    T = synth.pose_matrix(np.eye(3), [0.0, 0.0, 0.0])
    for om in (proj, ours):
        assert om.integrate_lidar(lidar, rimg, T) == oracle.OK
    assert proj.stats()["updates"] > 10000
    blocks = proj.block_coords()
    assert len(blocks) == len(ours.block_coords())
    n_band = 0
    for b in blocks:
        a, o = proj.block(b), ours.block(b)
        # only returns with a normal are kept: the top row's rays are dropped, and with
        # them the voxels whose nearest pixel is in the top row; the others have the
        # projective weight (it is the linear weight of psi in both modes)
        assert np.all((o["W"] == a["W"]) | (o["W"] == 0))
        upd = o["W"] > 0
        # d = psi cos(angle between the voxel's ray and its pixel's normal)
        assert np.all(np.abs(a["D"] - o["D"])[upd] <= TAU * (1.0 - np.cos(one_pixel)) + 2e-6 * TAU)
        G = ours.block_gradient(b)
        idx = np.nonzero(o["band"])[0]
        v = np.stack([8 * b[0] + idx % 8, 8 * b[1] + (idx // 8) % 8, 8 * b[2] + idx // 64], 1) * NU
        radial = -v / np.linalg.norm(v, axis=1, keepdims=True)
        # the gradient is the pixel's normal, along the pixel's ray (half a pixel from the voxel's)
        assert np.all(np.einsum("ij,ij->i", G[:, idx].T, radial) > np.cos(np.deg2rad(3.0)))
        n_band += len(idx)
    assert n_band > 1000


def test_plane_at_incidence_gives_the_perpendicular_distance():
    """A plane seen obliquely: the projective distance overstates the distance by
    1 / cos(incidence); the non-projective one is the perpendicular distance, up to the
    nearest pixel's angular offset (at most half a pixel in each direction)."""
    lidar = synth.uniform_lidar(64, 1024, 10.0, -30.0, 60.0)
    proj, ours = _pair()
    n_w = _unit([0.0, 0.0, 1.0])
    T = synth.pose_matrix(np.eye(3), [0.0, 0.0, 1.5])
    rimg = synth.plane_range(lidar, T, n_w, 0.0)
    for om in (proj, ours):
        assert om.integrate_lidar(lidar, rimg, T) == oracle.OK
    d_pix = np.hypot(np.deg2rad(40.0 / 63), 2 * np.pi / 1024) / 2
    worst_o, worst_p, n = 0.0, 0.0, 0
    for b in ours.block_coords():
        o, a = ours.block(b), proj.block(b)
        # voxels inside the band after one frame: the projective D is psi itself
        m = (o["W"] > 0) & (np.abs(a["D"]) < 0.9 * TAU)
        if not m.any():
            continue
        idx = np.nonzero(m)[0]
        v = np.stack([8 * b[0] + idx % 8, 8 * b[1] + (idx // 8) % 8, 8 * b[2] + idx // 64], 1) * NU
        perp = v[:, 2]                               # signed distance to the ground plane z = 0
        # the pixel's ray meets the plane at range dist + psi; the voxel's ray is within
        # d_pix of it, which moves the distance along the normal by at most that range
        # times d_pix
        r_pix = np.linalg.norm(v - [0.0, 0.0, 1.5], axis=1) + np.abs(a["D"][idx])
        bound = r_pix * d_pix * 1.05 + 1e-5
        err = np.abs(o["D"][idx] - perp)
        assert np.all(err <= bound), (b, err.max(), bound[err.argmax()])
        worst_o = max(worst_o, float((err / bound).max()))
        worst_p = max(worst_p, float((np.abs(a["D"][idx] - perp) / bound).max()))
        n += len(idx)
    assert n > 5000 and worst_p > 3.0 * worst_o


def test_gradient_is_the_normalised_weighted_average_of_normals():
    """Two frames of a plane from different poses: the gradient of every observed voxel is
    the plane's normal, and a second plane's normals average in by weight."""
    lidar = synth.uniform_lidar(32, 512, 10.0, -30.0, 40.0)
    _, ours = _pair()
    n_w = _unit([0.2, 0.1, 1.0])
    for x in (0.0, 0.35):
        T = synth.pose_matrix(_rz(0.3 * x), [x, 0.1, 1.5])
        assert ours.integrate_lidar(lidar, synth.plane_range(lidar, T, n_w, 0.0), T) == oracle.OK
    n_obs = 0
    for b in ours.block_coords():
        o = ours.block(b)
        G = ours.block_gradient(b)
        m = o["W"] > 0
        assert np.all(np.linalg.norm(G[:, m].T - n_w, axis=1) < 2e-3)
        n_obs += int(m.sum())
    assert n_obs > 5000


def test_projective_mode_is_unchanged_by_the_option():
    """Switching the mode on and back off leaves the projective update as it was."""
    w = synth.tiny_workload()
    f = w.frame(0, with_labels=False)
    a = oracle.OracleMap(w.voxel, w.trunc, w.n_classes)
    b = oracle.OracleMap(w.voxel, w.trunc, w.n_classes)
    assert b.set_distance(oracle.DIST_NONPROJECTIVE) == oracle.OK
    assert b.set_distance(oracle.DIST_PROJECTIVE) == oracle.OK
    for om in (a, b):
        assert om.integrate_lidar(w.lidar, f.range, f.T_wl) == oracle.OK
    assert a.stats() == b.stats()
    for blk in a.block_coords()[::50]:
        np.testing.assert_array_equal(a.block(blk)["D"], b.block(blk)["D"])
    assert b.set_distance(5) == oracle.INVALID
