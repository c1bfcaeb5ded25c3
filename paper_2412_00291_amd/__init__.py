"""MI355X-native per-frame metric-semantic mapping (projective and non-projective TSDF,
label fusion, incremental marching cubes) behind the C ABI in ``include/mapcore.h``.

The Python layer only marshals arguments: every step of the path runs in the HIP
kernels of ``libmapcore.so``.  Importing fails loudly when the library is missing.
"""
from .mapcore import (  # noqa: F401
    MAP_OK, MAP_ERR_INVALID_ARG, MAP_ERR_CAPACITY, MAP_ERR_BUFFER_TOO_SMALL, MAP_ERR_NO_SCAN,
    MAP_ERR_DEVICE, MAP_MESH_DIRTY, MAP_MESH_ALL, MapError, Map, LidarModel, CameraModel, lib_path,
    MAP_DIST_PROJECTIVE, MAP_DIST_NONPROJECTIVE, MAP_LABELS_COUNTS, MAP_LABELS_LATEST, MAP_LABELS_BAYES,
    map_set_distance, map_set_label_fusion, map_integrate_logprobs, map_download_aux, map_frame_normals,
    map_mesh_quality, map_sdf_pose_adjoint_noalloc,
    map_create, map_destroy, map_integrate_lidar, map_integrate_labels, map_integrate_labels_multi,
    map_extract_mesh,
    map_query_sdf, map_range_image, map_integrate_labels_lidar, map_sdf_pose_adjoint, map_sync, map_stats, map_last_error, map_block_coords,
    map_touched_coords, map_download, map_read_block, map_profile, map_profile_read, KERNEL_NAMES,
    Batch, map_batch_create, map_batch_configure, map_batch_step, map_batch_destroy,
)
