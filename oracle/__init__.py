"""CPU oracle of the mapping path -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper over ``liboracle.so`` (plain C in ``oracle.c``).  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import this package; the
GPU library and its Python binding never do.  It shares no code with them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
# Builds of the one source: plain (the parity reference), OpenMP (the same results on
# several threads, for the CPU timing baseline) and, for the sanitizer tests, plain with
# AddressSanitizer and UndefinedBehaviorSanitizer.  MAPCORE_ORACLE_LIB names a library to
# load in place of the plain build (the sanitizer tests set it in a child process).
VARIANTS = {
    "plain": ("liboracle.so", []),
    "omp": ("liboracle_omp.so", ["-fopenmp"]),
    "san": ("liboracle_san.so", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                 "-fno-omit-frame-pointer", "-g"]),
}
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]
_libs = {}

OK, INVALID, CAPACITY, BUFFER, NO_SCAN = 0, -1, -2, -3, -4
MESH_DIRTY, MESH_ALL = 0, 1
DIST_PROJECTIVE, DIST_NONPROJECTIVE = 0, 1
LABELS_COUNTS, LABELS_LATEST, LABELS_BAYES = 0, 1, 2
DEFAULT_MAX_INCIDENCE = float(np.deg2rad(80.0))  # point filter of the non-projective mode


def normal_image(lidar, range_img, T_wl, max_incidence=DEFAULT_MAX_INCIDENCE):
    """Normal image and point filter of one scan: (kept ranges [R, C], world normals [R, C, 3])."""
    e = _f32(lidar.elev_rad)
    r = _f32(range_img)
    T = _f32(T_wl).reshape(16)
    kept = np.zeros((lidar.rows, lidar.cols), np.float32)
    nrm = np.zeros((lidar.rows, lidar.cols, 3), np.float32)
    st = _load().om_normal_image(lidar.rows, lidar.cols, _p(e), float(lidar.r_max), float(max_incidence),
                                 _p(r), _p(T), _p(kept), _p(nrm))
    if st != OK:
        raise ValueError("invalid scan model")
    return kept, nrm


def nonproj_distance(psi, u, g, n):
    """Eq. 4 as read here, in fp32 (for pins)."""
    u, g, n = _f32(u), _f32(g), _f32(n)  # kept alive across the call
    return float(_load().om_nonproj_distance(float(psi), _p(u), _p(g), _p(n)))


def lib_path(variant: str = "plain") -> str:
    return os.path.join(_HERE, VARIANTS[variant][0])


def build(force: bool = False, variant: str = "plain") -> str:
    src = os.path.join(_HERE, "oracle.c")
    hdr = os.path.join(_HERE, "oracle.h")
    out = lib_path(variant)
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    if force or not os.path.exists(out) or os.path.getmtime(out) < newest:
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *VARIANTS[variant][1], "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def build_all(force: bool = False):
    for v in ("plain", "omp"):
        build(force, v)


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("touched", "new_blocks", "updates", "votes", "mesh_blocks", "triangles", "allocated")]


def _load(variant: str = "plain"):
    L = _libs.get(variant)
    if L is None:
        path = os.environ.get("MAPCORE_ORACLE_LIB") if variant == "plain" else None
        if not path:
            path = lib_path(variant)
            if not os.path.exists(path):
                build(variant=variant)
        L = ctypes.CDLL(path)
        P, I, I64, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
        L.om_create.restype = P
        L.om_create.argtypes = [F, F, I, I64]
        L.om_destroy.argtypes = [P]
        L.om_integrate_lidar.argtypes = [P, I, I, P, F, P, P]
        L.om_integrate_labels.argtypes = [P, I, I, F, F, F, F, P, P]
        L.om_extract_mesh.argtypes = [P, I, I64, P, P, P, P]
        L.om_get_stats.argtypes = [P, P]
        L.om_num_blocks.restype = I64
        L.om_num_blocks.argtypes = [P]
        L.om_block_coords.argtypes = [P, P]
        L.om_touched.restype = I64
        L.om_touched.argtypes = [P, P, I64]
        L.om_block_data.argtypes = [P, I, I, I, P, P, P, P, P]
        L.om_segment_blocks.restype = I64
        L.om_segment_blocks.argtypes = [P, P, P, I64]
        L.om_ray_segment.argtypes = [P, I, I, P, F, I, I, F, P, P, P]
        L.om_pixel_of.argtypes = [I, I, P, P, P, P]
        L.om_integrate_labels_lidar.argtypes = [P, I, I, P, P, P]
        L.om_range_image.restype = I64
        L.om_range_image.argtypes = [I, I, P, F, P, I64, F, F, P, P]
        L.om_query_sdf.argtypes = [P, P, I64, P, P, P, I]
        L.om_pose_adjoint.argtypes = [P, P, P, I, I64, P, P, P, P]
        L.om_set_block.argtypes = [P, I, I, I, P, P, P]
        L.om_cube_triangles.argtypes = [I, P]
        L.om_threads.restype = I
        L.om_threads.argtypes = []
        L.om_set_distance.argtypes = [P, I, F]
        L.om_normal_image.argtypes = [I, I, P, F, F, P, P, P, P]
        L.om_nonproj_distance.restype = F
        L.om_nonproj_distance.argtypes = [F, P, P, P]
        L.om_block_gradient.argtypes = [P, I, I, I, P]
        L.om_set_label_fusion.argtypes = [P, I]
        L.om_integrate_logprobs.argtypes = [P, I, I, F, F, F, F, P, P]
        L.om_block_logpost.argtypes = [P, I, I, I, P]
        _libs[variant] = L
    return L


def threads(variant: str = "plain") -> int:
    """Threads the given build uses (OpenMP's maximum for the omp build, else 1)."""
    return int(_load(variant).om_threads())


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def segment_blocks(Q0, Q1) -> np.ndarray:
    """Blocks met by a closed fixed-point segment (brute-force slab test)."""
    L = _load()
    q0 = np.ascontiguousarray(Q0, dtype=np.int64)
    q1 = np.ascontiguousarray(Q1, dtype=np.int64)
    out = np.zeros((4096, 3), dtype=np.int32)
    n = L.om_segment_blocks(_p(q0), _p(q1), _p(out), 4096)
    assert n <= 4096
    return out[:n].copy()


def cube_triangles(mask: int) -> np.ndarray:
    """Edge-id triples the marching-cubes rule gives for one inside-corner mask."""
    out = np.zeros((12, 3), dtype=np.int32)
    n = _load().om_cube_triangles(int(mask), _p(out))
    return out[:n].copy()


def pixel_of(lidar_rows, lidar_cols, elev, p):
    L = _load()
    e = _f32(elev)
    pp = _f32(p)
    r, c = ctypes.c_int(), ctypes.c_int()
    ok = L.om_pixel_of(lidar_rows, lidar_cols, _p(e), _p(pp), ctypes.byref(r), ctypes.byref(c))
    return (r.value, c.value) if ok else None


def range_image(lidar_rows, lidar_cols, elev, r_max, pts, F=1.0, O=0.0):
    """Depth and height images (Eq. 3) of sensor-frame points [n, 3]: (D, H, pixels written)."""
    L = _load()
    e = _f32(elev)
    p = _f32(pts).reshape(-1, 3)
    D = np.zeros((lidar_rows, lidar_cols), dtype=np.float32)
    H = np.zeros((lidar_rows, lidar_cols), dtype=np.float32)
    w = L.om_range_image(lidar_rows, lidar_cols, _p(e), float(r_max), _p(p), p.shape[0], float(F), float(O),
                         _p(D), _p(H))
    if w < 0:
        raise ValueError("invalid scan model")
    return D, H, int(w)


class OracleMap:
    """One map held by the CPU oracle."""

    def __init__(self, voxel, trunc, n_classes, max_blocks=1 << 22, variant="plain"):
        self._L = _load(variant)
        self.voxel, self.trunc, self.n_classes = float(voxel), float(trunc), int(n_classes)
        self.h = self._L.om_create(voxel, trunc, n_classes, max_blocks)
        if not self.h:
            raise ValueError("invalid oracle map parameters")

    def close(self):
        if self.h:
            self._L.om_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_distance(self, mode, max_incidence=None) -> int:
        """mode DIST_PROJECTIVE or DIST_NONPROJECTIVE; max_incidence in radians."""
        inc = DEFAULT_MAX_INCIDENCE if max_incidence is None else max_incidence
        return self._L.om_set_distance(self.h, int(mode), float(inc))

    def set_label_fusion(self, mode) -> int:
        return self._L.om_set_label_fusion(self.h, int(mode))

    def integrate_logprobs(self, cam, logp, T_wc) -> int:
        """logp: float32 [H, W, L] per-pixel class log-probabilities."""
        lp = _f32(logp)
        assert lp.shape == (cam.height, cam.width, self.n_classes)
        T = _f32(T_wc).reshape(16)
        return self._L.om_integrate_logprobs(self.h, cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                                             _p(lp), _p(T))

    def block_logpost(self, b):
        LP = np.zeros((self.n_classes, 512), np.float32)
        ok = self._L.om_block_logpost(self.h, int(b[0]), int(b[1]), int(b[2]), _p(LP))
        return LP if ok else None

    def block_gradient(self, b):
        G = np.zeros((3, 512), np.float32)
        ok = self._L.om_block_gradient(self.h, int(b[0]), int(b[1]), int(b[2]), _p(G))
        return G if ok else None

    def integrate_lidar(self, lidar, range_img, T_wl) -> int:
        e = _f32(lidar.elev_rad)
        r = _f32(range_img)
        T = _f32(T_wl).reshape(16)
        return self._L.om_integrate_lidar(self.h, lidar.rows, lidar.cols, _p(e), float(lidar.r_max),
                                          _p(r), _p(T))

    def integrate_labels(self, cam, labels, T_wc) -> int:
        lab = np.ascontiguousarray(labels, dtype=np.uint8)
        T = _f32(T_wc).reshape(16)
        return self._L.om_integrate_labels(self.h, cam.width, cam.height, cam.fx, cam.fy, cam.cx,
                                           cam.cy, _p(lab), _p(T))

    def integrate_labels_lidar(self, lidar, labels, T_wl) -> int:
        e = _f32(lidar.elev_rad)
        lab = np.ascontiguousarray(labels, dtype=np.uint8)
        assert lab.size == lidar.rows * lidar.cols
        T = _f32(T_wl).reshape(16)
        return self._L.om_integrate_labels_lidar(self.h, lidar.rows, lidar.cols, _p(e), _p(lab), _p(T))

    def extract_mesh(self, mode=MESH_DIRTY, cap=None, with_keys=True):
        """Returns (status, pos [T,3,3] f32, labels [T,3] u8, keys [T,3] i64 or None, n)."""
        n = ctypes.c_int64(0)
        if cap is None:
            # size the buffers with a zero-capacity call (it leaves the dirty set alone
            # whenever there is anything to return)
            self._L.om_extract_mesh(self.h, mode, 0, None, None, None, ctypes.byref(n))
            cap = n.value
        pos = np.zeros((max(cap, 1), 3, 3), dtype=np.float32)
        lab = np.zeros((max(cap, 1), 3), dtype=np.uint8)
        keys = np.zeros((max(cap, 1), 3), dtype=np.int64) if with_keys else None
        st = self._L.om_extract_mesh(self.h, mode, cap, _p(pos), _p(lab), _p(keys), ctypes.byref(n))
        k = min(n.value, cap)
        return st, pos[:k], lab[:k], (keys[:k] if keys is not None else None), n.value

    def stats(self) -> dict:
        s = _Stats()
        self._L.om_get_stats(self.h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in _Stats._fields_}

    def num_blocks(self) -> int:
        return self._L.om_num_blocks(self.h)

    def block_coords(self) -> np.ndarray:
        n = self.num_blocks()
        out = np.zeros((max(n, 1), 3), dtype=np.int32)
        self._L.om_block_coords(self.h, _p(out))
        return out[:n]

    def touched(self) -> np.ndarray:
        n = self._L.om_touched(self.h, None, 0)
        out = np.zeros((max(n, 1), 3), dtype=np.int32)
        self._L.om_touched(self.h, _p(out), n)
        return out[:n]

    def block(self, b):
        D = np.zeros(512, np.float32)
        W = np.zeros(512, np.float32)
        F = np.zeros(512, np.uint8)
        C = np.zeros((self.n_classes, 512), np.uint16)
        band = np.zeros(512, np.uint8)
        ok = self._L.om_block_data(self.h, int(b[0]), int(b[1]), int(b[2]), _p(D), _p(W), _p(F), _p(C), _p(band))
        if not ok:
            return None
        return {"D": D, "W": W, "fused": F, "counts": C, "band": band}

    def set_block(self, b, D=None, W=None, fused=None):
        """Test hook: overwrite one block (created if absent) and mark it dirty."""
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=t).reshape(512)
                for a, t in ((D, np.float32), (W, np.float32), (fused, np.uint8))]
        ok = self._L.om_set_block(self.h, int(b[0]), int(b[1]), int(b[2]), *[_p(a) for a in arrs])
        if not ok:
            raise RuntimeError("oracle map is full")

    def ray_segment(self, lidar, row, col, r, T_wl):
        e = _f32(lidar.elev_rad)
        T = _f32(T_wl).reshape(16)
        q0 = np.zeros(3, np.int64)
        q1 = np.zeros(3, np.int64)
        ok = self._L.om_ray_segment(self.h, lidar.rows, lidar.cols, _p(e), float(lidar.r_max), row, col,
                                    float(r), _p(T), _p(q0), _p(q1))
        return (q0, q1) if ok else None

    def query_sdf(self, pts, mode=0):
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        n = pts.shape[0]
        sdf = np.zeros(n, np.float64)
        grad = np.zeros((n, 3), np.float64)
        valid = np.zeros(n, np.uint8)
        self._L.om_query_sdf(self.h, _p(pts), n, _p(sdf), _p(grad), _p(valid), mode)
        return sdf, grad, valid.astype(bool)

    def pose_adjoint(self, xi, pts):
        xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 6)
        B = xi.shape[0]
        pts = _f32(pts).reshape(B, -1, 3)
        N = pts.shape[1]
        loss = np.zeros(B, np.float64)
        gxi = np.zeros((B, 6), np.float64)
        gpts = np.zeros((B, N, 3), np.float64)
        margin = np.zeros((B, N), np.float64)
        self._L.om_pose_adjoint(self.h, _p(xi), _p(pts), B, N, _p(loss), _p(gxi), _p(gpts), _p(margin))
        return loss, gxi, gpts, margin
