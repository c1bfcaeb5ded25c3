"""Pins of the oracle's marching cubes (end of Sec. IV-C.3).

The triangulation is fixed by a rule (face segments, inside corners kept apart on
ambiguous faces, cycles oriented toward D >= 0, fan from the smallest edge id), so it is
pinned by what any correct rule must satisfy: every surface of a closed sign field is a
closed, consistently oriented 2-manifold (each directed edge appears once and its
reverse once); a linear field's zero set is reproduced exactly; the sphere seen from
inside is one closed surface of Euler characteristic 2, facing the sensor, within the
interpolation error bound nu^2 / (8 (R - nu)) of the true radius; and meshing the dirty
blocks after every frame gives the same mesh as meshing everything at the end.
"""
from collections import Counter

import numpy as np
import pytest

import oracle
import synth


def _edge_axis_base(key):
    key = np.asarray(key, dtype=np.int64)
    axis = key & 3
    off = 1 << 19
    v = np.stack([(key >> 42) & 0xFFFFF, (key >> 22) & 0xFFFFF, (key >> 2) & 0xFFFFF], -1) - off
    return axis, v


def _directed_edges(keys):
    c = Counter()
    for a, b, d in keys:
        c[(a, b)] += 1
        c[(b, d)] += 1
        c[(d, a)] += 1
    return c


def _assert_closed_oriented(keys):
    """Every directed edge once, its reverse once: closed and consistently oriented."""
    tri = [tuple(int(x) for x in t) for t in keys]
    for t in tri:
        assert len(set(t)) == 3
    c = _directed_edges(tri)
    for (a, b), n in c.items():
        assert n == 1, ("edge used twice in one direction", a, b)
        assert c.get((b, a), 0) == 1, ("open edge", a, b)
    return tri


def _euler(tri):
    verts = {v for t in tri for v in t}
    edges = {tuple(sorted(e)) for t in tri for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    return len(verts) - len(edges) + len(tri)


def test_rule_cases_use_crossing_edges_only():
    for mask in range(256):
        tris = oracle.cube_triangles(mask)
        used = set(tris.ravel().tolist())
        crossing = set()
        for e in range(12):
            ax, j = e // 4, e % 4
            base = [0, 0, 0]
            others = [a for a in range(3) if a != ax]
            base[others[0]], base[others[1]] = j & 1, j >> 1
            tip = list(base)
            tip[ax] = 1
            ia = (mask >> (base[0] + 2 * base[1] + 4 * base[2])) & 1
            ib = (mask >> (tip[0] + 2 * tip[1] + 4 * tip[2])) & 1
            if ia != ib:
                crossing.add(e)
        assert used == crossing, mask


def _closed_field_map(seed, bad_corners=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    nu = 0.25
    m = oracle.OracleMap(nu, 0.75, 3)
    D = rng.choice([-1.0, 1.0], size=(16, 16, 16)) * rng.uniform(0.05, 0.7, size=(16, 16, 16))
    D[[0, -1], :, :] = 0.5
    D[:, [0, -1], :] = 0.5
    D[:, :, [0, -1]] = 0.5
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                sub = D[8 * bx:8 * bx + 8, 8 * by:8 * by + 8, 8 * bz:8 * bz + 8]
                m.set_block((bx, by, bz), D=sub.transpose(2, 1, 0).astype(np.float32),
                            W=np.ones(512, np.float32), fused=np.full(512, 1, np.uint8))
    return m, D


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_closed_fields_are_watertight(seed):
    m, _ = _closed_field_map(seed)
    st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_ALL)
    assert st == oracle.OK and n > 100
    _assert_closed_oriented(keys)


def test_linear_field_zero_set_exact():
    nu = np.float32(0.2)
    m = oracle.OracleMap(float(nu), 0.6, 3)
    a = np.array([0.37, 0.21, -0.15])
    b0 = -(0.37 * 7.3 + 0.21 * 8.1 - 0.15 * 6.6)
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                i = np.arange(512)
                v = np.stack([i & 7, (i >> 3) & 7, i >> 6], 1) + 8 * np.array([bx, by, bz])
                D = (v @ a + b0).astype(np.float32)
                m.set_block((bx, by, bz), D=D, W=np.ones(512, np.float32))
    st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_ALL)
    assert st == oracle.OK and n > 50
    val = pos.reshape(-1, 3).astype(np.float64) / float(nu) @ a + b0
    assert np.abs(val).max() < 2e-5
    # vertices lie on their edges, at the recorded edge key
    axis, base = _edge_axis_base(keys.reshape(-1))
    p = pos.reshape(-1, 3).astype(np.float64) / float(nu)
    for k in range(3):
        on = axis == k
        assert np.all(np.abs(p[~on, k] - base[~on, k]) < 1e-5)
        assert np.all((p[on, k] >= base[on, k] - 1e-6) & (p[on, k] <= base[on, k] + 1 + 1e-6))
    # normals point toward increasing D
    P = pos.astype(np.float64)
    nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    big = np.linalg.norm(nrm, axis=1) > 1e-6
    assert np.all(nrm[big] @ a > 0)


def _sphere_three_views(R=3.0, nu=0.2, tau=0.6):
    lidar = synth.uniform_lidar(64, 1800, 60.0, -60.0, 40.0)
    m = oracle.OracleMap(nu, tau, 4)
    rx = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], float)
    ry = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], float)
    for Rm in (np.eye(3), rx, ry):
        assert m.integrate_lidar(lidar, synth.constant_range(lidar, R), synth.pose_matrix(Rm, [0, 0, 0])) == 0
    return m


def test_sphere_from_inside_closed_and_accurate():
    R, nu = 3.0, 0.2
    m = _sphere_three_views(R, nu)
    st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_ALL)
    assert st == oracle.OK and n > 1000
    tri = _assert_closed_oriented(keys)
    assert _euler(tri) == 2
    r = np.linalg.norm(pos.reshape(-1, 3).astype(np.float64), axis=1)
    assert np.abs(r - R).max() <= nu * nu / (8 * (R - nu)) + 1e-5
    P = pos.astype(np.float64)
    nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    big = np.linalg.norm(nrm, axis=1) > 1e-3 * nu * nu  # slivers at a corner have no direction
    cen = P.mean(axis=1)
    assert big.mean() > 0.9
    assert np.all(np.einsum("ij,ij->i", nrm[big], -cen[big]) > 0)  # facing the sensor
    assert np.all(lab == 255)  # no label image was integrated


def _cube_base(keys):
    axis, base = _edge_axis_base(keys)
    return base.min(axis=0)


def test_incremental_equals_full_remesh():
    w = synth.tiny_workload()
    m = oracle.OracleMap(w.voxel, w.trunc, w.n_classes)
    f = w.frame(0)
    acc = {}
    pending = set()
    rng = np.random.Generator(np.random.PCG64(8))
    for k in range(5):
        T = synth.pose_matrix(synth.rot_z(rng.normal(0, 0.1)), [0.6 * k, rng.normal(0, 0.2), 0.0])
        assert m.integrate_lidar(w.lidar, f.range, T) == oracle.OK
        for Tc, lab, cam in f.cams:
            m.integrate_labels(cam, lab, T @ np.linalg.inv(f.T_wl) @ Tc)
        allocated = {tuple(b) for b in m.block_coords()}
        for b in m.touched():
            for e in range(8):
                nb = (b[0] - (e & 1), b[1] - ((e >> 1) & 1), b[2] - ((e >> 2) & 1))
                if nb in allocated:
                    pending.add(nb)
        if k % 2 == 1:
            continue  # dirty blocks accumulate across frames until the next extraction
        st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_DIRTY)
        assert st == oracle.OK
        assert m.stats()["mesh_blocks"] == len(pending)
        for b in pending:
            acc[b] = []
        for t in range(n):
            blk = tuple(int(x) for x in np.floor_divide(_cube_base(keys[t]), 8))
            assert blk in pending
            acc[blk].append((tuple(keys[t]), tuple(lab[t]), pos[t].tobytes()))
        pending = set()
    st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_ALL)
    full = Counter((tuple(keys[t]), tuple(lab[t]), pos[t].tobytes()) for t in range(n))
    inc = Counter(x for v in acc.values() for x in v)
    assert full == inc and n > 1000


def test_buffer_too_small_keeps_dirty_set():
    m = _sphere_three_views()
    n_all = m.extract_mesh(oracle.MESH_ALL)[4]
    st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_DIRTY, cap=10)
    assert st == oracle.BUFFER and n == n_all
    st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_DIRTY)
    assert st == oracle.OK and n == n_all
    st, pos, lab, keys, n = m.extract_mesh(oracle.MESH_DIRTY)
    assert st == oracle.OK and n == 0
