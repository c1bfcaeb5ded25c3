"""ctypes binding of the mapcore C ABI (argument marshalling only).

Function names mirror the C entry points.  Device buffers are torch CUDA tensors (HIP
on ROCm); the stream defaults to torch's current stream.  The binding never computes
anything itself and raises if ``libmapcore.so`` is absent: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_FILE = os.path.join(_HERE, "libmapcore.so")

MAP_OK, MAP_ERR_INVALID_ARG, MAP_ERR_CAPACITY = 0, -1, -2
MAP_ERR_BUFFER_TOO_SMALL, MAP_ERR_NO_SCAN, MAP_ERR_DEVICE = -3, -4, -5
MAP_MESH_DIRTY, MAP_MESH_ALL = 0, 1
MAP_DIST_PROJECTIVE, MAP_DIST_NONPROJECTIVE = 0, 1
MAP_LABELS_COUNTS, MAP_LABELS_LATEST, MAP_LABELS_BAYES = 0, 1, 2


def lib_path() -> str:
    return _LIB_FILE


if not os.path.exists(_LIB_FILE):
    raise ImportError(f"mapcore HIP library not built: {_LIB_FILE} is missing "
                      "(run `python -c 'import __graft_entry__ as g; g.build()'` from the repo root)")

# torch first: the library then binds to the HIP runtime torch ships (same soname), so
# torch's tensors and streams and this library share one runtime whatever the caller
# imported first.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(_LIB_FILE)


class _Params(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_float), ("truncation", ctypes.c_float),
                ("max_blocks", ctypes.c_int64), ("n_classes", ctypes.c_int32), ("device", ctypes.c_int32)]


class _Lidar(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("elev_rad", ctypes.c_void_p), ("r_max", ctypes.c_float)]


class _Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class _BatchItem(ctypes.Structure):
    _fields_ = [("map_index", ctypes.c_int32), ("lidar", ctypes.c_void_p), ("range_dev", ctypes.c_void_p),
                ("T_wl", ctypes.c_void_p), ("n_cams", ctypes.c_int32), ("cams", ctypes.c_void_p),
                ("labels_dev", ctypes.c_void_p), ("T_wc", ctypes.c_void_p), ("pos_dev", ctypes.c_void_p),
                ("lab_dev", ctypes.c_void_p), ("edge_keys_dev", ctypes.c_void_p), ("cap_tris", ctypes.c_int64)]


class _Quality(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("cd", ctypes.c_double), ("rc", ctypes.c_double),
                ("miou", ctypes.c_double), ("acc", ctypes.c_double), ("n_eval", ctypes.c_int64)]


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("touched", "new_blocks", "updates", "votes", "mesh_blocks",
                                              "triangles", "allocated", "frames", "mesh_from_bitmap")]


_P, _I32, _I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
_sig = {
    "map_create": (ctypes.c_int, [ctypes.POINTER(_Params), _P, ctypes.POINTER(_P)]),
    "map_destroy": (None, [_P]),
    "map_integrate_lidar": (ctypes.c_int, [_P, ctypes.POINTER(_Lidar), _P, _P, _P]),
    "map_integrate_labels": (ctypes.c_int, [_P, ctypes.POINTER(_Camera), _P, _P, _P]),
    "map_integrate_labels_multi": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P]),
    "map_extract_mesh": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _I64, ctypes.POINTER(_I64), _P]),
    "map_query_sdf": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _P]),
    "map_integrate_labels_lidar": (ctypes.c_int, [_P, ctypes.POINTER(_Lidar), _P, _P, _P]),
    "map_range_image": (ctypes.c_int, [_P, ctypes.POINTER(_Lidar), _P, _I64, ctypes.c_float, ctypes.c_float, _P, _P,
                                       _P]),
    "map_sdf_pose_adjoint": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _P, _P, _P, _P]),
    "map_sdf_pose_adjoint_noalloc": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _P, _P, _P, _P]),
    "map_sync": (ctypes.c_int, [_P]),
    "map_stats": (ctypes.c_int, [_P, ctypes.POINTER(_Stats)]),
    "map_last_error": (ctypes.c_char_p, [_P]),
    "map_block_coords": (_I64, [_P, _P, _I64]),
    "map_touched_coords": (_I64, [_P, _P, _I64]),
    "map_download": (_I64, [_P, _I64, _P, _P, _P, _P, _P]),
    "map_read_block": (ctypes.c_int, [_P, _I32, _I32, _I32, _P, _P, _P, _P]),
    "map_profile": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "map_set_schedule": (ctypes.c_int, [_P, _I32, _I32, _I32]),
    "map_set_dirty_bitmap": (ctypes.c_int, [_P, _I64]),
    "map_batch_create": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_P)]),
    "map_batch_configure": (ctypes.c_int, [_P, _I32, _I32, _I32]),
    "map_batch_step": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "map_batch_destroy": (None, [_P]),
    "map_profile_read": (ctypes.c_int, [_P, _P, _P]),
    "map_set_distance": (ctypes.c_int, [_P, _I32, ctypes.c_float]),
    "map_set_label_fusion": (ctypes.c_int, [_P, _I32]),
    "map_integrate_logprobs": (ctypes.c_int, [_P, ctypes.POINTER(_Camera), _P, _P, _P]),
    "map_download_aux": (_I64, [_P, _I64, _P, _P]),
    "map_frame_normals": (_I64, [_P, _P, _I64]),
    "map_mesh_quality": (ctypes.c_int, [_P, _P, _I64, _P, _P, _I64, ctypes.c_float, _I32, _I32, _P, _P, _P, _P,
                                        ctypes.POINTER(_Quality), _P]),
}

KERNEL_NAMES = ["alloc", "tsdf", "labels", "mesh", "query", "adjoint", "batch", "range", "tsdf_labels"]
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class MapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mapcore error {code}: {msg}")
        self.code = code


@dataclass
class LidarModel:
    rows: int
    cols: int
    elev_rad: np.ndarray  # host float32 [rows], top row first
    r_max: float

    def _c(self):
        key = (self.rows, self.cols, self.r_max, id(self.elev_rad))
        cached = self.__dict__.get("_cstruct")
        if cached is not None and cached[0] == key:
            return cached[1]
        e = np.ascontiguousarray(self.elev_rad, dtype=np.float32)
        s = _Lidar(self.rows, self.cols, e.ctypes.data, self.r_max)
        s._keep = e
        if e is self.elev_rad:  # reusable: the struct points at the model's own array
            self.__dict__["_cstruct"] = (key, s)
        return s


@dataclass
class CameraModel:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def _c(self):
        return _Camera(self.width, self.height, self.fx, self.fy, self.cx, self.cy)


_raw_stream = None  # torch's getter of the current stream's raw handle (False: not available)


def _stream(stream):
    """The HIP stream handle of a call: the given one, or torch's current stream (read
    without building a Stream object when torch provides the raw getter: this runs on
    every call of a frame)."""
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    global _raw_stream
    import torch
    if _raw_stream is None:
        _raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None) or False
    if _raw_stream:
        return ctypes.c_void_p(_raw_stream(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name, shape_last=None):
    """Device pointer of a contiguous CUDA tensor of the given dtype (or None)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and t.shape[-1] != shape_last:
        raise ValueError(f"{name}: last dimension must be {shape_last}")
    return ctypes.c_void_p(t.data_ptr())


def _pose(T):
    a = np.ascontiguousarray(np.asarray(T, dtype=np.float32).reshape(16))
    return a, ctypes.c_void_p(a.ctypes.data)


# ----------------------------------------------------------------------------------------
# functions with the C ABI's names
# ----------------------------------------------------------------------------------------

def map_create(voxel_size, truncation, max_blocks, n_classes, device=0, stream=None):
    """Returns (status, handle)."""
    p = _Params(voxel_size, truncation, int(max_blocks), int(n_classes), int(device))
    h = _P()
    st = _lib.map_create(ctypes.byref(p), _stream(stream), ctypes.byref(h))
    return st, h


def map_destroy(handle):
    _lib.map_destroy(handle)


def map_integrate_lidar(handle, lidar: LidarModel, range_dev, T_wl, stream=None):
    import torch
    L = lidar._c()
    keep, T = _pose(T_wl)
    if range_dev.numel() != lidar.rows * lidar.cols:
        raise ValueError("range image size does not match the LiDAR model")
    return _lib.map_integrate_lidar(handle, ctypes.byref(L), _dev(range_dev, torch.float32, "range"), T,
                                    _stream(stream))


def map_integrate_labels(handle, cam: CameraModel, labels_dev, T_wc, stream=None):
    import torch
    if labels_dev.numel() != cam.width * cam.height:
        raise ValueError("label image size does not match the camera model")
    keep, T = _pose(T_wc)
    return _lib.map_integrate_labels(handle, ctypes.byref(cam._c()), _dev(labels_dev, torch.uint8, "labels"), T,
                                     _stream(stream))


def map_integrate_labels_lidar(handle, lidar: LidarModel, labels_dev, T_wl, stream=None):
    """Label range image (uint8 [rows, cols] device tensor, the scan's pixel layout) under
    the scan pose T_wl: the last scan's band voxels vote with the label at their pixel."""
    import torch
    if labels_dev.numel() != lidar.rows * lidar.cols:
        raise ValueError("label image size does not match the LiDAR model")
    L = lidar._c()
    keep, T = _pose(T_wl)
    return _lib.map_integrate_labels_lidar(handle, ctypes.byref(L), _dev(labels_dev, torch.uint8, "labels"), T,
                                           _stream(stream))


def map_integrate_labels_multi(handle, cams, labels_dev, T_wc, stream=None):
    """n cameras in one call: cams [n] CameraModel, labels_dev [n] uint8 device tensors,
    T_wc [n] 4x4 poses; equal to n single-camera calls in order."""
    import torch
    n = len(cams)
    if len(labels_dev) != n or len(T_wc) != n:
        raise ValueError("cams, labels and poses differ in length")
    carr = _cam_array(cams)
    ptrs = (ctypes.c_uint64 * n)()
    for i in range(n):
        c, l = cams[i], labels_dev[i]
        if l.numel() != c.width * c.height:
            raise ValueError("label image size does not match the camera model")
        ptrs[i] = _dev_ptr(l, torch.uint8, "labels")
    T = np.array(T_wc, dtype=np.float32).reshape(n, 16)
    return _lib.map_integrate_labels_multi(handle, n, ctypes.cast(carr, _P), ctypes.cast(ptrs, _P), T.ctypes.data,
                                           _stream(stream))


def map_extract_mesh(handle, mode, pos_dev, lab_dev, edge_keys_dev=None, stream=None):
    """Returns (status, n_tris).  Capacity is taken from pos_dev ([cap, 3, 3] float32).
    Returns once the count is known; the triangles are written on the stream after that,
    so later work on the same stream (or a stream synchronisation) sees them."""
    import torch
    cap = 0 if pos_dev is None else pos_dev.shape[0]
    if lab_dev is not None and lab_dev.shape[0] < cap:
        raise ValueError("label buffer smaller than the position buffer")
    if edge_keys_dev is not None and edge_keys_dev.shape[0] < cap:
        raise ValueError("edge-key buffer smaller than the position buffer")
    n = _I64(0)
    st = _lib.map_extract_mesh(handle, int(mode), _dev(pos_dev, torch.float32, "pos") if cap else None,
                               _dev(lab_dev, torch.uint8, "lab") if cap else None,
                               _dev(edge_keys_dev, torch.int64, "edge_keys") if cap else None,
                               cap, ctypes.byref(n), _stream(stream))
    return st, n.value


def map_range_image(handle, lidar: LidarModel, pts_dev, depth_dev, height_dev=None, F=1.0, O=0.0, stream=None):
    """Depth and height images (Eq. 3) of sensor-frame points pts_dev [n, 3] float32 into
    depth_dev (and height_dev, if given) [rows, cols] float32 device tensors."""
    import torch
    L = lidar._c()
    npix = lidar.rows * lidar.cols
    if depth_dev.numel() != npix or (height_dev is not None and height_dev.numel() != npix):
        raise ValueError("image size does not match the LiDAR model")
    n = pts_dev.shape[0]
    return _lib.map_range_image(handle, ctypes.byref(L), _dev(pts_dev, torch.float32, "pts", 3) if n else None, n,
                                float(F), float(O), _dev(depth_dev, torch.float32, "depth"),
                                _dev(height_dev, torch.float32, "height"), _stream(stream))


def map_query_sdf(handle, pts_dev, sdf_dev, grad_dev, valid_dev, stream=None):
    import torch
    n = pts_dev.shape[0]
    if sdf_dev.shape[0] != n or valid_dev.shape[0] != n or (grad_dev is not None and grad_dev.shape[0] != n):
        raise ValueError("query output sizes differ from the point count")
    return _lib.map_query_sdf(handle, _dev(pts_dev, torch.float32, "pts", 3), n, _dev(sdf_dev, torch.float32, "sdf"),
                              _dev(grad_dev, torch.float32, "grad", 3), _dev(valid_dev, torch.uint8, "valid"),
                              _stream(stream))


def map_sdf_pose_adjoint(handle, xi_dev, pts_dev, loss_dev, gxi_dev, gpts_dev=None, stream=None):
    import torch
    B, N = pts_dev.shape[0], pts_dev.shape[1]
    if tuple(xi_dev.shape) != (B, 6) or tuple(loss_dev.shape) != (B,) or tuple(gxi_dev.shape) != (B, 6):
        raise ValueError("adjoint argument shapes do not match B")
    if gpts_dev is not None and tuple(gpts_dev.shape) != tuple(pts_dev.shape):
        raise ValueError("gpts must have the points' shape")
    return _lib.map_sdf_pose_adjoint(handle, _dev(xi_dev, torch.float32, "xi"), _dev(pts_dev, torch.float32, "pts", 3),
                                     B, N, _dev(loss_dev, torch.float32, "loss"), _dev(gxi_dev, torch.float32, "gxi"),
                                     _dev(gpts_dev, torch.float32, "gpts", 3), _stream(stream))


def map_set_distance(handle, mode, max_incidence):
    """mode MAP_DIST_PROJECTIVE or MAP_DIST_NONPROJECTIVE; max_incidence in radians."""
    return _lib.map_set_distance(handle, int(mode), float(max_incidence))


def map_set_label_fusion(handle, mode):
    return _lib.map_set_label_fusion(handle, int(mode))


def map_integrate_logprobs(handle, cam: CameraModel, logp_dev, T_wc, n_classes, stream=None):
    """logp_dev: float32 [height, width, n_classes] device tensor of class log-probabilities."""
    import torch
    if tuple(logp_dev.shape) != (cam.height, cam.width, n_classes):
        raise ValueError("log-probability image shape does not match the camera model and class count")
    keep, T = _pose(T_wc)
    return _lib.map_integrate_logprobs(handle, ctypes.byref(cam._c()), _dev(logp_dev, torch.float32, "logp"), T,
                                       _stream(stream))


def map_download_aux(handle, n_classes, grad=True, logpost=True):
    """Per-voxel gradients [n, 3, 512] and log-posteriors [n, L, 512] in slot order."""
    n = _lib.map_download_aux(handle, 0, None, None)
    k = max(n, 1)
    G = np.zeros((k, 3, 512), np.float32) if grad else None
    LP = np.zeros((k, n_classes, 512), np.float32) if logpost else None
    _lib.map_download_aux(handle, n, G.ctypes.data if grad else None, LP.ctypes.data if logpost else None)
    return {"grad": G[:n] if grad else None, "logpost": LP[:n] if logpost else None}


def map_frame_normals(handle):
    """The last frame's normal image [n_pixels, 4] (world normal, kept range), or None."""
    n = _lib.map_frame_normals(handle, None, 0)
    if n <= 0:
        return None
    out = np.zeros((n, 4), np.float32)
    _lib.map_frame_normals(handle, out.ctypes.data, n)
    return out


def map_mesh_quality(mesh_pts, mesh_lab, gt_pts, gt_lab, voxel_size, n_classes, device=0, d_mesh=None, d_gt=None,
                     nn_gt=None, with_confusion=True, stream=None):
    """Map-quality metrics of mesh vertices (device float32 [n, 3], labels uint8 [n]) against
    a ground-truth cloud (float32 [m, 3], classes uint8 [m]).  Optional device outputs
    d_mesh, d_gt (float64) and nn_gt (int64).  Returns (status, dict)."""
    import torch
    nM, nG = mesh_pts.shape[0], gt_pts.shape[0]
    if mesh_lab.shape[0] != nM or gt_lab.shape[0] != nG:
        raise ValueError("label counts differ from the point counts")
    q = _Quality()
    conf = np.zeros(((n_classes + 1) * n_classes,), np.int64) if with_confusion else None
    st = _lib.map_mesh_quality(_dev(mesh_pts, torch.float32, "mesh_pts", 3) if nM else None,
                               _dev(mesh_lab, torch.uint8, "mesh_lab") if nM else None, nM,
                               _dev(gt_pts, torch.float32, "gt_pts", 3) if nG else None,
                               _dev(gt_lab, torch.uint8, "gt_lab") if nG else None, nG, float(voxel_size),
                               int(n_classes), int(device), _dev(d_mesh, torch.float64, "d_mesh"),
                               _dev(d_gt, torch.float64, "d_gt"), _dev(nn_gt, torch.int64, "nn_gt"),
                               conf.ctypes.data if with_confusion else None, ctypes.byref(q), _stream(stream))
    r = {f: getattr(q, f) for f, _ in _Quality._fields_}
    if with_confusion:
        r["confusion"] = conf.reshape(n_classes + 1, n_classes)
    return st, r


def map_sdf_pose_adjoint_noalloc(handle, xi_dev, pts_dev, loss_dev, gxi_dev, gpts_dev=None, stream=None):
    """map_sdf_pose_adjoint with the library's static scratch (no allocation)."""
    import torch
    B, N = pts_dev.shape[0], pts_dev.shape[1]
    if tuple(xi_dev.shape) != (B, 6) or tuple(loss_dev.shape) != (B,) or tuple(gxi_dev.shape) != (B, 6):
        raise ValueError("adjoint argument shapes do not match B")
    if gpts_dev is not None and tuple(gpts_dev.shape) != tuple(pts_dev.shape):
        raise ValueError("gpts must have the points' shape")
    return _lib.map_sdf_pose_adjoint_noalloc(handle, _dev(xi_dev, torch.float32, "xi"),
                                             _dev(pts_dev, torch.float32, "pts", 3), B, N,
                                             _dev(loss_dev, torch.float32, "loss"), _dev(gxi_dev, torch.float32, "gxi"),
                                             _dev(gpts_dev, torch.float32, "gpts", 3), _stream(stream))


def map_sync(handle):
    return _lib.map_sync(handle)


def map_stats(handle):
    s = _Stats()
    st = _lib.map_stats(handle, ctypes.byref(s))
    return st, {f: getattr(s, f) for f, _ in _Stats._fields_}


def map_last_error(handle):
    r = _lib.map_last_error(handle)
    return r.decode() if r else ""


def map_block_coords(handle):
    n = _lib.map_block_coords(handle, None, 0)
    out = np.zeros((max(n, 1), 3), np.int32)
    _lib.map_block_coords(handle, out.ctypes.data, n)
    return out[:n]


def map_touched_coords(handle):
    n = _lib.map_touched_coords(handle, None, 0)
    out = np.zeros((max(n, 1), 3), np.int32)
    _lib.map_touched_coords(handle, out.ctypes.data, n)
    return out[:n]


def map_download(handle, n_classes, with_counts=True):
    n = _lib.map_download(handle, 0, None, None, None, None, None)
    k = max(n, 1)
    coords = np.zeros((k, 3), np.int32)
    D = np.zeros((k, 512), np.float32)
    W = np.zeros((k, 512), np.float32)
    F = np.zeros((k, 512), np.uint8)
    C = np.zeros((k, n_classes, 512), np.uint16) if with_counts else None
    _lib.map_download(handle, n, coords.ctypes.data, D.ctypes.data, W.ctypes.data, F.ctypes.data,
                      C.ctypes.data if with_counts else None)
    return {"coords": coords[:n], "D": D[:n], "W": W[:n], "fused": F[:n],
            "counts": C[:n] if with_counts else None}


def map_profile(handle, mask):
    return _lib.map_profile(handle, int(mask))


def map_profile_read(handle):
    """{kernel name: (total ms, launches)} since the last read (synchronises)."""
    ms = np.zeros(len(KERNEL_NAMES), np.float64)
    n = np.zeros(len(KERNEL_NAMES), np.int64)
    st = _lib.map_profile_read(handle, ms.ctypes.data, n.ctypes.data)
    if st != MAP_OK:
        raise MapError(st, map_last_error(handle))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_NAMES)}


def map_read_block(handle, b, n_classes):
    D = np.zeros(512, np.float32)
    W = np.zeros(512, np.float32)
    F = np.zeros(512, np.uint8)
    C = np.zeros((n_classes, 512), np.uint16)
    ok = _lib.map_read_block(handle, int(b[0]), int(b[1]), int(b[2]), D.ctypes.data, W.ctypes.data,
                             F.ctypes.data, C.ctypes.data)
    return {"D": D, "W": W, "fused": F, "counts": C} if ok else None


# ----------------------------------------------------------------------------------------
# convenience wrapper
# ----------------------------------------------------------------------------------------

class Map:
    """One map on one device; raises MapError on a non-OK status."""

    def __init__(self, voxel_size, truncation, n_classes, max_blocks, device=0, stream=None):
        st, h = map_create(voxel_size, truncation, max_blocks, n_classes, device, stream)
        if st != MAP_OK:
            raise MapError(st, map_last_error(None))
        self.h = h
        self.n_classes = int(n_classes)
        self.voxel_size, self.truncation = float(voxel_size), float(truncation)

    def _check(self, st, ok=(MAP_OK,)):
        if st not in ok:
            raise MapError(st, map_last_error(self.h))
        return st

    def close(self):
        if getattr(self, "h", None):
            map_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def integrate_lidar(self, lidar, range_dev, T_wl, stream=None):
        return self._check(map_integrate_lidar(self.h, lidar, range_dev, T_wl, stream))

    def integrate_labels(self, cam, labels_dev, T_wc, stream=None):
        return self._check(map_integrate_labels(self.h, cam, labels_dev, T_wc, stream))

    def integrate_labels_lidar(self, lidar, labels_dev, T_wl, stream=None):
        return self._check(map_integrate_labels_lidar(self.h, lidar, labels_dev, T_wl, stream))

    def integrate_labels_multi(self, cams, labels_dev, T_wc, stream=None):
        return self._check(map_integrate_labels_multi(self.h, cams, labels_dev, T_wc, stream))

    def extract_mesh(self, mode, pos_dev, lab_dev, edge_keys_dev=None, stream=None, allow_small=False):
        st, n = map_extract_mesh(self.h, mode, pos_dev, lab_dev, edge_keys_dev, stream)
        self._check(st, (MAP_OK, MAP_ERR_BUFFER_TOO_SMALL) if allow_small else (MAP_OK,))
        return st, n

    def range_image(self, lidar, pts_dev, depth_dev, height_dev=None, F=1.0, O=0.0, stream=None):
        return self._check(map_range_image(self.h, lidar, pts_dev, depth_dev, height_dev, F, O, stream))

    def query_sdf(self, pts_dev, sdf_dev, grad_dev, valid_dev, stream=None):
        return self._check(map_query_sdf(self.h, pts_dev, sdf_dev, grad_dev, valid_dev, stream))

    def sdf_pose_adjoint(self, xi_dev, pts_dev, loss_dev, gxi_dev, gpts_dev=None, stream=None):
        return self._check(map_sdf_pose_adjoint(self.h, xi_dev, pts_dev, loss_dev, gxi_dev, gpts_dev, stream))

    def sync(self):
        return map_sync(self.h)

    def stats(self):
        st, s = map_stats(self.h)
        return st, s

    def block_coords(self):
        return map_block_coords(self.h)

    def touched_coords(self):
        return map_touched_coords(self.h)

    def download(self, with_counts=True):
        return map_download(self.h, self.n_classes, with_counts)

    def set_schedule(self, tsdf, labels, mesh):
        return self._check(_lib.map_set_schedule(self.h, int(tsdf), int(labels), int(mesh)))

    def set_dirty_bitmap(self, min_blocks):
        """Dirty meshing's candidates from the dirty bitmap above min_blocks allocated
        blocks (< 0: the default threshold); see map_set_dirty_bitmap."""
        return self._check(_lib.map_set_dirty_bitmap(self.h, int(min_blocks)))

    def profile(self, mask):
        return self._check(map_profile(self.h, mask))

    def profile_read(self):
        return map_profile_read(self.h)

    def read_block(self, b):
        return map_read_block(self.h, b, self.n_classes)

    def set_distance(self, mode, max_incidence):
        return self._check(map_set_distance(self.h, mode, max_incidence))

    def set_label_fusion(self, mode):
        return self._check(map_set_label_fusion(self.h, mode))

    def integrate_logprobs(self, cam, logp_dev, T_wc, stream=None):
        return self._check(map_integrate_logprobs(self.h, cam, logp_dev, T_wc, self.n_classes, stream))

    def download_aux(self, grad=True, logpost=True):
        return map_download_aux(self.h, self.n_classes, grad, logpost)

    def frame_normals(self):
        return map_frame_normals(self.h)


# ----------------------------------------------------------------------------------------
# batched steps
# ----------------------------------------------------------------------------------------

def map_batch_create(handles):
    """Returns (status, batch handle)."""
    n = len(handles)
    arr = (_P * n)(*[h.value if isinstance(h, _P) else h for h in handles])
    b = _P()
    st = _lib.map_batch_create(ctypes.cast(arr, _P), n, ctypes.byref(b))
    return st, b


def map_batch_configure(batch, schedule, grid, use_graph=True):
    return _lib.map_batch_configure(batch, int(schedule), int(grid), int(bool(use_graph)))


def map_batch_destroy(batch):
    _lib.map_batch_destroy(batch)


_ITEM_DTYPE = np.dtype({"names": ["map_index", "lidar", "range_dev", "T_wl", "n_cams", "cams", "labels_dev", "T_wc",
                                   "pos_dev", "lab_dev", "edge_keys_dev", "cap_tris"],
                         "formats": [np.int32, np.uint64, np.uint64, np.uint64, np.int32, np.uint64, np.uint64,
                                     np.uint64, np.uint64, np.uint64, np.uint64, np.int64],
                         "offsets": [_BatchItem.map_index.offset, _BatchItem.lidar.offset,
                                     _BatchItem.range_dev.offset, _BatchItem.T_wl.offset, _BatchItem.n_cams.offset,
                                     _BatchItem.cams.offset, _BatchItem.labels_dev.offset, _BatchItem.T_wc.offset,
                                     _BatchItem.pos_dev.offset, _BatchItem.lab_dev.offset,
                                     _BatchItem.edge_keys_dev.offset, _BatchItem.cap_tris.offset],
                         "itemsize": ctypes.sizeof(_BatchItem)})
_cam_cache = {}


def _cam_array(cams):
    """ctypes camera array for a list of CameraModel (cached by value)."""
    key = tuple((c.width, c.height, c.fx, c.fy, c.cx, c.cy) for c in cams)
    arr = _cam_cache.get(key)
    if arr is None:
        arr = (_Camera * max(len(cams), 1))(*[c._c() for c in cams])
        if len(_cam_cache) < 1024:
            _cam_cache[key] = arr
    return arr


def _dev_ptr(t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        _dev(t, dtype, name)  # raises the specific error
    return t.data_ptr()


def map_batch_step(batch, items, stream=None):
    """items: list of dicts with map_index, lidar (LidarModel), range (device tensor), T_wl,
    and optionally cams (CameraModel list), labels (device tensors), T_wc (poses), pos, lab,
    keys (mesh outputs).  Returns (status, [triangles per item]).  The descriptors are
    packed into one record array; poses and label pointers into one array each."""
    import torch
    n = len(items)
    rec = np.zeros(n, _ITEM_DTYPE)
    max_c = max((len(it.get("cams") or []) for it in items), default=0)
    poses = np.empty((n, 16), np.float32)
    cposes = np.zeros((n, max(max_c, 1), 16), np.float32)
    lptrs = np.zeros((n, max(max_c, 1)), np.uint64)
    keep = [rec, poses, cposes, lptrs]
    for i, it in enumerate(items):
        L = it["lidar"]._c()
        keep.append(L)
        poses[i] = np.asarray(it["T_wl"], np.float32).reshape(16)
        cams = it.get("cams") or []
        nc = len(cams)
        labels = it.get("labels") or []
        if len(labels) != nc or len(it.get("T_wc") or []) != nc:
            raise ValueError("cams, labels and poses differ in length")
        carr = _cam_array(cams)
        keep.append(carr)
        for c in range(nc):
            lptrs[i, c] = _dev_ptr(labels[c], torch.uint8, "labels")
            cposes[i, c] = np.asarray(it["T_wc"][c], np.float32).reshape(16)
        pos, lab, keys = it.get("pos"), it.get("lab"), it.get("keys")
        cap = 0 if pos is None else pos.shape[0]
        r = rec[i]
        r["map_index"] = int(it["map_index"])
        r["lidar"] = ctypes.addressof(L)
        r["range_dev"] = _dev_ptr(it["range"], torch.float32, "range")
        r["n_cams"] = nc
        r["cams"] = ctypes.addressof(carr)
        if cap:
            r["pos_dev"] = _dev_ptr(pos, torch.float32, "pos")
            r["lab_dev"] = _dev_ptr(lab, torch.uint8, "lab")
            if keys is not None:
                r["edge_keys_dev"] = _dev_ptr(keys, torch.int64, "keys")
        r["cap_tris"] = cap
    rec["T_wl"] = poses.ctypes.data + 64 * np.arange(n, dtype=np.uint64)
    rec["T_wc"] = cposes.ctypes.data + np.uint64(cposes.shape[1] * 64) * np.arange(n, dtype=np.uint64)
    rec["labels_dev"] = lptrs.ctypes.data + np.uint64(lptrs.shape[1] * 8) * np.arange(n, dtype=np.uint64)
    out = np.zeros(n, np.int64)
    st = _lib.map_batch_step(batch, rec.ctypes.data, n, out.ctypes.data, _stream(stream))
    del keep
    return st, out.tolist()


class Batch:
    """Maps stepped together; each keeps the state its own plain calls would give."""

    def __init__(self, maps, schedule=0, grid=2048, use_graph=True):
        self.maps = list(maps)
        st, self.h = map_batch_create([m.h for m in self.maps])
        if st != MAP_OK:
            raise MapError(st, map_last_error(None))
        self.configure(schedule, grid, use_graph)

    def configure(self, schedule, grid, use_graph=True):
        st = map_batch_configure(self.h, schedule, grid, use_graph)
        if st != MAP_OK:
            raise MapError(st, "bad batch configuration")
        self.schedule, self.grid, self.use_graph = schedule, grid, use_graph

    def step(self, items, stream=None, allow_small=False):
        st, n = map_batch_step(self.h, items, stream)
        if st not in ((MAP_OK, MAP_ERR_BUFFER_TOO_SMALL) if allow_small else (MAP_OK,)):
            raise MapError(st, "batched step failed")
        return st, n

    def close(self):
        if getattr(self, "h", None):
            map_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
