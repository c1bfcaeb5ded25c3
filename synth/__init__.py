"""Seeded synthetic inputs for the mapping path (test and benchmark input generator).

This module turns a seeded scene recipe into posed LiDAR range images and camera
label images.  It holds none of the mapping method's arithmetic: it only lays
out primitive shapes with NumPy ``PCG64`` and ray-casts them (``raycast.c``).
Both the CPU oracle and the GPU library consume what it produces, so neither
side ever sees the other's output as an input.

Sensor conventions follow the paper's range-image geometry (Sec. IV-C.1, Eq. 3):
column ``c`` of a ``rows x cols`` range image looks along azimuth
``pi - c * 2 pi / cols``; row ``k`` along elevation ``elev[k]`` (top row first).
Cameras are undistorted pinholes with z forward, x right, y down.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

OBJ_BOX, OBJ_CYL, OBJ_CONE, OBJ_SPHERE = 0, 1, 2, 3


# The sanitizer tests build a second copy with AddressSanitizer and
# UndefinedBehaviorSanitizer (no OpenMP) and name it in MAPCORE_SYNTH_LIB for a child process.
SAN_LIB_PATH = os.path.join(_HERE, "libsynth_san.so")


def build_lib(force: bool = False, sanitize: bool = False) -> str:
    """Compile the ray caster (host C, OpenMP; or sanitized and single-threaded)."""
    src = os.path.join(_HERE, "raycast.c")
    out = SAN_LIB_PATH if sanitize else _LIB_PATH
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        extra = (["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
                 if sanitize else ["-fopenmp"])
        subprocess.check_call(["gcc", "-O2", *extra, "-fPIC", "-shared", "-std=c11", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("MAPCORE_SYNTH_LIB")
        if not path:
            path = _LIB_PATH
            if not os.path.exists(path):
                build_lib()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.synth_scene_new.restype = P
        lib.synth_scene_new.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int, P, P, ctypes.c_int, ctypes.c_double]
        lib.synth_scene_set_heightfield.argtypes = [P, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, P]
        lib.synth_scene_free.argtypes = [P]
        lib.synth_cast.argtypes = [P, ctypes.c_int64, P, P, ctypes.c_double, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class Scene:
    """A set of primitives plus a ground, with an xy grid for ray casting."""

    def __init__(self, objects, ground_kind=1, ground_z=0.0, bands=(), ground_default_cls=0,
                 cell=4.0, heightfield=None):
        lib = _load()
        n = len(objects)
        self.objects = list(objects)
        types = np.array([o[0] for o in objects] or [0], dtype=np.int32)
        cls = np.array([o[1] for o in objects] or [0], dtype=np.int32)
        params = np.zeros((max(n, 1), 6), dtype=np.float64)
        for i, o in enumerate(objects):
            params[i, :len(o[2])] = o[2]
        band_y = np.array([b[0] for b in bands] or [0.0], dtype=np.float64)
        band_c = np.array([b[1] for b in bands] or [0], dtype=np.int32)
        self._keep = (types, cls, params, band_y, band_c)
        self.h = lib.synth_scene_new(n, _ptr(types), _ptr(cls), _ptr(params), int(ground_kind),
                                     float(ground_z), len(bands), _ptr(band_y), _ptr(band_c),
                                     int(ground_default_cls), float(cell))
        if heightfield is not None:
            x0, y0, hstep, z = heightfield
            z = np.ascontiguousarray(z, dtype=np.float32)
            lib.synth_scene_set_heightfield(self.h, float(x0), float(y0), float(hstep),
                                            int(z.shape[1]), int(z.shape[0]), _ptr(z))

    def cast(self, origin, dirs, tmax):
        """First-hit distance (inf on miss) and class id (255 on miss) per ray."""
        dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        origin = np.ascontiguousarray(origin, dtype=np.float64).reshape(3)
        n = dirs.shape[0]
        t = np.empty(n, dtype=np.float64)
        c = np.empty(n, dtype=np.uint8)
        _load().synth_cast(self.h, n, _ptr(origin), _ptr(dirs), float(tmax), _ptr(t), _ptr(c))
        return t, c

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _load().synth_scene_free(self.h)
                self.h = None
        except Exception:
            pass


@dataclass
class Lidar:
    rows: int
    cols: int
    elev_rad: np.ndarray  # float32 [rows], top row first, strictly decreasing
    r_max: float

    def directions(self) -> np.ndarray:
        """Unit ray directions in the sensor frame, double, [rows*cols, 3]."""
        e = self.elev_rad.astype(np.float64)[:, None]
        c = np.arange(self.cols, dtype=np.float64)[None, :]
        phi = np.pi - c * (2.0 * np.pi / self.cols)
        d = np.stack([np.cos(e) * np.cos(phi), np.cos(e) * np.sin(phi),
                      np.sin(e) * np.ones_like(phi)], axis=-1)
        return d.reshape(-1, 3)


def uniform_lidar(rows, cols, top_deg, bottom_deg, r_max) -> Lidar:
    e = np.linspace(np.deg2rad(top_deg), np.deg2rad(bottom_deg), rows)
    return Lidar(rows, cols, e.astype(np.float32), float(r_max))


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R_lc: np.ndarray = field(default_factory=lambda: camera_yaw(0.0))  # camera -> LiDAR rotation

    def pixel_dirs(self) -> np.ndarray:
        """Camera-frame ray directions through pixel centres, [H*W, 3]."""
        u = (np.arange(self.width, dtype=np.float64) + 0.5 - self.cx) / self.fx
        v = (np.arange(self.height, dtype=np.float64) + 0.5 - self.cy) / self.fy
        uu, vv = np.meshgrid(u, v)
        return np.stack([uu, vv, np.ones_like(uu)], axis=-1).reshape(-1, 3)


def camera_yaw(yaw_rad: float) -> np.ndarray:
    """Rotation camera->LiDAR for a camera co-located with the LiDAR, optical axis
    horizontal at the given yaw (0 = along LiDAR +x), image y pointing down."""
    cy, sy = np.cos(yaw_rad), np.sin(yaw_rad)
    fwd = np.array([cy, sy, 0.0])
    right = np.array([sy, -cy, 0.0])
    down = np.array([0.0, 0.0, -1.0])
    return np.stack([right, down, fwd], axis=1)


def pose_matrix(R, t) -> np.ndarray:
    """4x4 float32 row-major pose (the exact value every consumer sees)."""
    T = np.eye(4, dtype=np.float64)
    T[:3, :3] = R
    T[:3, 3] = t
    return T.astype(np.float32)


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


@dataclass
class Frame:
    T_wl: np.ndarray            # float32 4x4
    range: np.ndarray           # float32 [rows, cols]
    cams: list                  # list of (T_wc float32 4x4, labels uint8 [H, W], Camera)


@dataclass
class Workload:
    name: str
    voxel: float
    trunc: float
    n_classes: int
    lidar: Lidar
    cameras: list
    scene: Scene
    poses: list                 # float32 4x4 T_wl per frame
    seed: int
    noise_sigma: float = 0.02
    dropout: float = 0.02
    max_blocks: int = 1 << 20

    @property
    def n_frames(self):
        return len(self.poses)

    def frame(self, k: int, with_labels: bool = True) -> Frame:
        T = self.poses[k]
        Td = T.astype(np.float64)
        o = Td[:3, 3]
        d = self.lidar.directions() @ Td[:3, :3].T
        t, _ = self.scene.cast(o, d, self.lidar.r_max)
        rng = np.random.Generator(np.random.PCG64(self.seed * 1000 + k))
        r = t + rng.normal(0.0, self.noise_sigma, size=t.shape) if self.noise_sigma > 0 else t.copy()
        drop = rng.random(size=t.shape) < self.dropout
        r[~np.isfinite(t)] = 0.0
        r[t > self.lidar.r_max] = 0.0
        r[drop] = 0.0
        rng_img = r.astype(np.float32).reshape(self.lidar.rows, self.lidar.cols)
        cams = []
        if with_labels:
            for cam in self.cameras:
                R_wc = Td[:3, :3] @ cam.R_lc
                T_wc = pose_matrix(R_wc, o)
                Rc = T_wc.astype(np.float64)
                dirs = cam.pixel_dirs() @ Rc[:3, :3].T
                _, cl = self.scene.cast(Rc[:3, 3], dirs, 1.0e4)
                cams.append((T_wc, cl.reshape(cam.height, cam.width), cam))
        return Frame(T, rng_img, cams)


    def lidar_labels(self, k: int, flip: float = 0.05) -> np.ndarray:
        """Label range image of frame k (uint8 [rows, cols], the range image's layout): the
        class of each LiDAR ray's first hit (255 on a miss), a fraction `flip` of the hits
        replaced by a uniformly drawn class, as a point-cloud segmentation would give."""
        Td = self.poses[k].astype(np.float64)
        d = self.lidar.directions() @ Td[:3, :3].T
        t, cl = self.scene.cast(Td[:3, 3], d, self.lidar.r_max)
        lab = np.where(np.isfinite(t) & (t <= self.lidar.r_max), cl, 255).astype(np.int64)
        rng = np.random.Generator(np.random.PCG64(self.seed * 1000 + 500 + k))
        hit = lab != 255
        flip_m = hit & (rng.random(lab.shape) < flip)
        lab[flip_m] = rng.integers(0, self.n_classes, size=int(flip_m.sum()))
        return lab.astype(np.uint8).reshape(self.lidar.rows, self.lidar.cols)


# ----------------------------------------------------------------------------------------
# Scene recipes
# ----------------------------------------------------------------------------------------

def _annulus_xy(rng, rmin, rmax):
    rho = rng.uniform(rmin, rmax)
    th = rng.uniform(0, 2 * np.pi)
    return rho * np.cos(th), rho * np.sin(th)


def tiny_scene(seed=1):
    """16-beam tiny scene: ground 1.73 m below the sensor, 20 boxes, 5 cylinders."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gz = -1.73
    objs = []
    while len([o for o in objs if o[0] == OBJ_BOX]) < 20:
        sx, sy, sz = rng.uniform(1, 5, size=3)
        cx, cy = _annulus_xy(rng, 3, 35)
        x0, x1, y0, y1 = cx - sx / 2, cx + sx / 2, cy - sy / 2, cy + sy / 2
        dx = max(x0, -x1, 0.0)
        dy = max(y0, -y1, 0.0)
        if np.hypot(dx, dy) < 0.5:
            continue  # keep the sensor out of every box
        objs.append((OBJ_BOX, int(rng.integers(1, 20)), [x0, y0, gz, x1, y1, gz + sz]))
    for _ in range(5):
        r = rng.uniform(0.3, 1.0)
        h = rng.uniform(1, 4)
        while True:
            cx, cy = _annulus_xy(rng, 3, 35)
            if np.hypot(cx, cy) > r + 0.5:
                break
        objs.append((OBJ_CYL, int(rng.integers(1, 20)), [cx, cy, r, gz, gz + h]))
    return Scene(objs, ground_kind=1, ground_z=gz, bands=(), ground_default_cls=0, cell=4.0)


# street scene classes (19 classes)
ROAD, SIDEWALK, BUILDING, TERRAIN, POLE, TRUNK, VEGETATION = 0, 1, 2, 3, 4, 5, 6


def street_scene(seed=2):
    """Street: ground split in road / sidewalk / terrain bands, 200 box buildings set back
    at |y| >= 10 m, 500 poles and trees (trunk cylinder + cone crown)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    objs = []
    for _ in range(200):
        fx, fy, h = rng.uniform(5, 30, size=3)
        side = 1 if rng.random() < 0.5 else -1
        ynear = rng.uniform(10, 30)
        x0 = rng.uniform(-120, 130 - fx)
        y0, y1 = (ynear, ynear + fy) if side > 0 else (-ynear - fy, -ynear)
        cls = BUILDING if rng.random() < 0.5 else int(rng.integers(7, 19))
        objs.append((OBJ_BOX, cls, [x0, y0, 0.0, x0 + fx, y1, h]))
    for _ in range(500):
        x = rng.uniform(-120, 130)
        y = (1 if rng.random() < 0.5 else -1) * rng.uniform(5.0, 9.5)
        if rng.random() < 0.5:
            r = rng.uniform(0.1, 0.3)
            h = rng.uniform(3, 8)
            objs.append((OBJ_CYL, POLE, [x, y, r, 0.0, h]))
        else:
            rt = rng.uniform(0.1, 0.3)
            ht = rng.uniform(2, 4)
            rc = rng.uniform(1, 3)
            hc = rng.uniform(2, 6)
            objs.append((OBJ_CYL, TRUNK, [x, y, rt, 0.0, ht]))
            objs.append((OBJ_CONE, VEGETATION, [x, y, rc, ht, ht + hc]))
    bands = ((4.0, ROAD), (7.0, SIDEWALK))
    return Scene(objs, ground_kind=1, ground_z=0.0, bands=bands, ground_default_cls=TERRAIN, cell=5.0)


def campus_scene(seed=5):
    """Tiled 50 m campus around a 300 x 200 m loop: heightfield ground with N(0, 0.1 m)
    heights on a 1 m lattice, box buildings, cone and sphere vegetation, 0.15 m curbs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x0, y0, nx, ny = -220.0, -170.0, 441, 341
    z = rng.normal(0.0, 0.1, size=(ny, nx)).astype(np.float32)
    objs = []
    # loop: rounded rectangle with straight sides at x=+-150, y=+-100 (path width 8 m)
    def near_path(x, y, margin):
        ax, ay = abs(x), abs(y)
        dx = abs(ax - 150) if ay <= 100 else np.hypot(ax - 150, ay - 100) if ax > 150 else abs(ay - 100)
        dy = abs(ay - 100) if ax <= 150 else dx
        return min(dx, dy) < margin
    for tx in range(-4, 4):
        for ty in range(-3, 3):
            bx, by = tx * 50 + 25, ty * 50 + 25
            for _ in range(2):
                fx, fy, h = rng.uniform(8, 25), rng.uniform(8, 25), rng.uniform(4, 20)
                cx, cy = bx + rng.uniform(-15, 15), by + rng.uniform(-15, 15)
                if near_path(cx, cy, max(fx, fy) / 2 + 8):
                    continue
                objs.append((OBJ_BOX, BUILDING, [cx - fx / 2, cy - fy / 2, -0.5, cx + fx / 2, cy + fy / 2, h]))
            for _ in range(12):
                cx, cy = bx + rng.uniform(-25, 25), by + rng.uniform(-25, 25)
                if near_path(cx, cy, 6):
                    continue
                if rng.random() < 0.5:
                    objs.append((OBJ_CONE, VEGETATION, [cx, cy, rng.uniform(1, 3), -0.2, rng.uniform(3, 8)]))
                else:
                    r = rng.uniform(0.8, 2.5)
                    objs.append((OBJ_SPHERE, 7, [cx, cy, r * 0.8, r]))
    # curbs: thin boxes 0.15 m high along both sides of the straight path segments
    for sgn in (-1, 1):
        for off in (-4.0, 4.0):
            objs.append((OBJ_BOX, SIDEWALK, [-150, sgn * 100 + off - 0.5, -0.3, 150, sgn * 100 + off + 0.5, 0.15]))
            objs.append((OBJ_BOX, SIDEWALK, [sgn * 150 + off - 0.5, -100, -0.3, sgn * 150 + off + 0.5, 100, 0.15]))
    return Scene(objs, ground_kind=2, ground_z=0.0, bands=(), ground_default_cls=TERRAIN, cell=5.0,
                 heightfield=(x0, y0, 1.0, z))


# ----------------------------------------------------------------------------------------
# Workload recipes (the five configurations, sizes as stated in the method's workloads)
# ----------------------------------------------------------------------------------------

def tiny_workload(seed=1) -> Workload:
    lidar = Lidar(16, 1800, np.deg2rad(np.arange(15, -16, -2, dtype=np.float64)).astype(np.float32), 40.0)
    cam = Camera(640, 480, 500.0, 500.0, 320.0, 240.0, camera_yaw(0.0))
    return Workload("tiny-16x1800-v0.2", 0.2, 0.6, 20, lidar, [cam], tiny_scene(seed),
                    [pose_matrix(np.eye(3), np.zeros(3))], seed, max_blocks=1 << 18)


def street_poses(seed, n_frames, start_x=0.0, speed_per_frame=0.1, z=1.73):
    rng = np.random.Generator(np.random.PCG64(seed * 7919 + 17))
    poses = []
    for k in range(n_frames):
        yaw = rng.normal(0.0, np.deg2rad(0.5))
        poses.append(pose_matrix(rot_z(yaw), np.array([start_x + k * speed_per_frame, 0.0, z])))
    return poses


def street_workload(seed=2, n_frames=100, n_cams=4) -> Workload:
    lidar = uniform_lidar(64, 2048, 2.0, -24.8, 100.0)
    cams = [Camera(1280, 720, 640.0, 640.0, 640.0, 360.0, camera_yaw(np.deg2rad(a)))
            for a in (0, 90, 180, 270)[:n_cams]]
    return Workload("street-64x2048-v0.1", 0.1, 0.3, 19, lidar, cams, street_scene(seed),
                    street_poses(seed, n_frames), seed, max_blocks=1 << 21)


def batched_workloads(seed=3, n_maps=16, frame_cap=None):
    """16 uneven maps over the street scene: voxel in {0.05,0.1,0.2,0.4}, 16/32/64 beams,
    1024-2048 columns, 10-200 frames, staggered start offsets, one front camera."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = street_scene(2)
    out = []
    for m in range(n_maps):
        nu = float(rng.choice([0.05, 0.1, 0.2, 0.4]))
        beams = int(rng.choice([16, 32, 64]))
        cols = int(rng.integers(1024, 2049))
        nfr = int(rng.integers(10, 201))
        if frame_cap is not None:
            nfr = min(nfr, frame_cap)
        if beams == 16:
            lidar = uniform_lidar(16, cols, 15.0, -15.0, 100.0)
        elif beams == 32:
            lidar = uniform_lidar(32, cols, 10.0, -30.0, 100.0)
        else:
            lidar = uniform_lidar(64, cols, 2.0, -24.8, 100.0)
        cam = Camera(1280, 720, 640.0, 640.0, 640.0, 360.0, camera_yaw(0.0))
        start = float(rng.uniform(-80, 80))
        w = Workload(f"batched-map{m}-{beams}x{cols}-v{nu}", nu, 3.0 * nu, 19, lidar, [cam], scene,
                     street_poses(seed * 100 + m, nfr, start_x=start), seed * 100 + m,
                     max_blocks=1 << 20)
        out.append(w)
    return out


def campus_poses(n_frames, step=0.5, z=1.8):
    """Rounded-rectangle loop, 300 x 200 m straights with 25 m corner radius."""
    a, b, rc = 150.0, 100.0, 25.0
    segs = []
    # build polyline of the loop densely, then resample by arc length
    pts = []
    for th in np.linspace(0, 2 * np.pi, 4000, endpoint=False):
        c, s = np.cos(th), np.sin(th)
        # superellipse-like rounded rectangle via clamping
        x = np.clip(1.6 * a * c, -a, a)
        y = np.clip(1.6 * b * s, -b, b)
        pts.append((x, y))
    pts = np.array(pts)
    seg = np.linalg.norm(np.diff(np.vstack([pts, pts[:1]]), axis=0), axis=1)
    cum = np.concatenate([[0], np.cumsum(seg)])
    total = cum[-1]
    poses = []
    for k in range(n_frames):
        s = (k * step) % total
        i = int(np.searchsorted(cum, s, side="right") - 1)
        i = min(i, len(pts) - 1)
        p0, p1 = pts[i], pts[(i + 1) % len(pts)]
        f = (s - cum[i]) / max(seg[i], 1e-9)
        p = p0 + f * (p1 - p0)
        yaw = np.arctan2(p1[1] - p0[1], p1[0] - p0[0])
        poses.append(pose_matrix(rot_z(yaw), np.array([p[0], p[1], z])))
    del segs, rc
    return poses


def campus_workload(seed=5, n_frames=2000) -> Workload:
    lidar = uniform_lidar(128, 2048, 22.5, -22.5, 100.0)
    cams = [Camera(1920, 1080, 960.0, 960.0, 960.0, 540.0, camera_yaw(np.deg2rad(a))) for a in (0, 180)]
    return Workload("campus-128x2048-v0.1", 0.1, 0.3, 20, lidar, cams, campus_scene(seed),
                    campus_poses(n_frames), seed, max_blocks=2_000_000)


def scan_points(w: Workload, lidar: Lidar, frame_pose, n_points, seed):
    """Noiseless scan of the workload's scene as sensor-frame points (float32 [n,3]);
    invalid returns are replaced by seeded re-draws of valid ones."""
    Td = frame_pose.astype(np.float64)
    d = lidar.directions()
    t, _ = w.scene.cast(Td[:3, 3], d @ Td[:3, :3].T, lidar.r_max)
    ok = np.isfinite(t) & (t <= lidar.r_max)
    pts = d * np.where(ok, t, 0.0)[:, None]
    rng = np.random.Generator(np.random.PCG64(seed))
    valid_idx = np.nonzero(ok)[0]
    bad = np.nonzero(~ok)[0]
    pts[bad] = pts[rng.choice(valid_idx, size=bad.size)]
    assert pts.shape[0] == n_points
    return pts.astype(np.float32)


def cloud_points(w: Workload, k: int, seed: int, jitter=0.45, extra=0.1, invalid=0.01):
    """Raw sensor-frame point cloud of frame k (float32 [n, 3], shuffled): one return per
    beam and column cast at an angle drawn uniformly within +-jitter of a pixel spacing
    around the pixel centre, with the workload's range noise; plus a fraction `extra` of
    second returns (nearer and farther along drawn returns' directions) and a fraction
    `invalid` of points no scan keeps (non-finite, at the origin, beyond r_max, above the
    field of view)."""
    lidar = w.lidar
    R, C = lidar.rows, lidar.cols
    rng = np.random.Generator(np.random.PCG64(seed))
    e = lidar.elev_rad.astype(np.float64)
    de = np.abs(np.diff(e))
    de = np.concatenate([de[:1], de])  # spacing at each row
    row = np.repeat(np.arange(R), C)
    col = np.tile(np.arange(C), R)
    el = e[row] + rng.uniform(-jitter, jitter, R * C) * de[row]
    dphi = 2.0 * np.pi / C
    phi = np.pi - col * dphi + rng.uniform(-jitter, jitter, R * C) * dphi
    d = np.stack([np.cos(el) * np.cos(phi), np.cos(el) * np.sin(phi), np.sin(el)], axis=1)
    Td = w.poses[k].astype(np.float64)
    t, _ = w.scene.cast(Td[:3, 3], d @ Td[:3, :3].T, lidar.r_max)
    ok = np.isfinite(t) & (t <= lidar.r_max)
    r = t[ok] + rng.normal(0.0, w.noise_sigma, size=int(ok.sum()))
    pts = d[ok] * r[:, None]
    m = int(extra * len(pts))
    pick = rng.choice(len(pts), size=m)
    scale = np.where(rng.random(m) < 0.5, rng.uniform(0.5, 0.95, m), rng.uniform(1.05, 2.0, m))
    more = pts[pick] * scale[:, None]
    q = max(int(invalid * len(pts)), 8)
    bad = np.zeros((q, 3))
    kind = np.arange(q) % 4
    bad[kind == 0] = np.nan
    far = d[rng.choice(R * C, size=int((kind == 2).sum()))] * (lidar.r_max * 1.5)
    bad[kind == 2] = far
    up = np.deg2rad(80.0)
    bad[kind == 3] = np.array([np.cos(up), 0.0, np.sin(up)]) * 5.0
    allp = np.concatenate([pts, more, bad])
    return allp[rng.permutation(len(allp))].astype(np.float32)


def perturbed_poses(n, seed, rot_sigma=0.05, trans_sigma=0.2):
    """n pose 6-vectors (t, omega) drawn around the identity, float32 [n,6]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = rng.normal(0, trans_sigma, size=(n, 3))
    w = rng.normal(0, rot_sigma, size=(n, 3))
    return np.concatenate([t, w], axis=1).astype(np.float32)


def constant_range(lidar: Lidar, r: float) -> np.ndarray:
    """Range image where every return reads r (sensor inside a sphere of radius r)."""
    return np.full((lidar.rows, lidar.cols), r, dtype=np.float32)


# ----------------------------------------------------------------------------------------
# Micro-scenes with exact ties (block edges and corners, pixel boundaries)
# ----------------------------------------------------------------------------------------

def lidar_from_degrees(elev_deg, cols, r_max) -> Lidar:
    """Scan model with the given row elevations (degrees, top row first)."""
    e = np.deg2rad(np.asarray(elev_deg, dtype=np.float64))
    return Lidar(len(e), int(cols), e.astype(np.float32), float(r_max))


def lattice_ranges(lidar: Lidar, seed: int, step: float, n_max: int, p_drop=0.0) -> np.ndarray:
    """Range image whose every return is a multiple of `step` in [step, n_max*step]
    (seeded): with a binary voxel size and a sensor on a block corner, axis-aligned rays
    then end, or start, exactly on block faces, edges and corners."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.integers(1, n_max + 1, size=(lidar.rows, lidar.cols)).astype(np.float64) * step
    if p_drop > 0:
        r[rng.random(r.shape) < p_drop] = 0.0
    return r.astype(np.float32)


def box_room_range(lidar: Lidar, T_wl, lo, hi) -> np.ndarray:
    """Noiseless range image of a sensor inside the axis-aligned box room [lo, hi]
    (world frame): each ray's distance to the first wall it meets, in float64, rounded
    once to float32."""
    Td = np.asarray(T_wl, dtype=np.float64)
    o = Td[:3, 3]
    d = lidar.directions() @ Td[:3, :3].T
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(d > 0, (hi - o) / d, np.where(d < 0, (lo - o) / d, np.inf))
    r = t.min(axis=1)
    r[~np.isfinite(r) | (r > lidar.r_max)] = 0.0
    return r.astype(np.float32).reshape(lidar.rows, lidar.cols)


def plane_range(lidar: Lidar, T_wl, normal, offset) -> np.ndarray:
    """Noiseless range image of the plane {x : normal . x = offset} (world frame): each
    ray's distance to it in float64 (rays that miss it, or meet it beyond r_max, read 0),
    rounded once to float32."""
    Td = np.asarray(T_wl, dtype=np.float64)
    o = Td[:3, 3]
    d = lidar.directions() @ Td[:3, :3].T
    n = np.asarray(normal, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (float(offset) - n @ o) / (d @ n)
    t[~np.isfinite(t) | (t <= 0) | (t > lidar.r_max)] = 0.0
    return t.astype(np.float32).reshape(lidar.rows, lidar.cols)


def logprob_image(labels: np.ndarray, n_classes: int, seed: int, boost: float = 3.0, sigma: float = 1.0):
    """Per-pixel class log-probabilities [H, W, L] float32, as a segmentation network's
    log-softmax output: logits N(0, sigma) per class plus `boost` on the pixel's label
    (none where the label is 255 or >= L), normalised in float64, rounded once."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = labels.shape
    z = rng.normal(0.0, sigma, size=(H, W, n_classes))
    lab = labels.astype(np.int64)
    ok = lab < n_classes
    ii, jj = np.nonzero(ok)
    z[ii, jj, lab[ok]] += boost
    zmax = z.max(axis=2, keepdims=True)
    lse = zmax + np.log(np.exp(z - zmax).sum(axis=2, keepdims=True))
    return (z - lse).astype(np.float32)


def hard_logprob_image(labels: np.ndarray, n_classes: int, p: float) -> np.ndarray:
    """Log-probabilities of a hard label with a symmetric likelihood: log p for the
    pixel's label and log((1 - p) / (L - 1)) for the others (uniform where the label is
    255 or >= L), float32 [H, W, L]."""
    H, W = labels.shape
    lo, hi = np.float32(np.log((1.0 - p) / (n_classes - 1))), np.float32(np.log(p))
    out = np.full((H, W, n_classes), lo, np.float32)
    lab = labels.astype(np.int64)
    ok = lab < n_classes
    ii, jj = np.nonzero(ok)
    out[ii, jj, lab[ok]] = hi
    out[~ok] = np.float32(-np.log(n_classes))
    return out


def ground_truth_cloud(w: Workload, frames, lidar: Lidar = None):
    """Ground-truth point cloud of a sequence, as the paper's datasets build theirs
    (labelled scans accumulated with their true poses): the noiseless first hits of every
    ray of the given frames (within r_max) in the world frame, float32 [n, 3], with the hit
    object's class, uint8 [n]."""
    lidar = lidar or w.lidar
    pts, cls = [], []
    d0 = lidar.directions()
    for k in frames:
        Td = w.poses[k].astype(np.float64)
        o = Td[:3, 3]
        d = d0 @ Td[:3, :3].T
        t, c = w.scene.cast(o, d, lidar.r_max)
        hit = np.isfinite(t) & (t <= lidar.r_max)
        pts.append(o + t[hit, None] * d[hit])
        cls.append(c[hit])
    return np.concatenate(pts).astype(np.float32), np.concatenate(cls).astype(np.uint8)
