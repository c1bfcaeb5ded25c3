/*
 * mapcore: per-frame metric-semantic mapping on one AMD Instinct MI355X (gfx950).
 *
 * The method is the TSDF-based volumetric mapping of "Real-Time Metric-Semantic Mapping
 * for Autonomous Navigation in Outdoor Environments" (Jiao et al.), Sec. IV-C, in its
 * projective-distance form: posed LiDAR range images allocate 8x8x8 voxel blocks in a
 * spatial hash and update a truncated signed distance and weight per voxel (Eq. 5);
 * camera label images update a per-voxel class distribution (Eq. 6); marching cubes
 * turns the distance field into a labelled triangle mesh (end of Sec. IV-C.3).
 *
 * Conventions (every call):
 *   - Voxel index v in Z^3 has its centre at x = voxel_size * v (Sec. IV-C.2); block
 *     b = floor(v / 8) per component; a voxel's local index is x + 8 y + 64 z.
 *   - Poses are host float[16], row-major 4x4 rigid transforms from the sensor frame to
 *     the map frame; the rotation must be orthonormal to 1e-5 with determinant > 0 and
 *     the last row (0, 0, 0, 1), otherwise MAP_ERR_INVALID_ARG.
 *   - Range images: device float, rows x cols, row-major.  Column c looks along azimuth
 *     pi - c * 2 pi / cols; row k along elevation elev_rad[k], top row first (Eq. 3).
 *     A return is valid if finite and 0 < r <= r_max; 0 marks a dropout.
 *   - Label images: device uint8, height x width, row-major; a value >= n_classes
 *     (e.g. 255) is "no label".  Cameras are undistorted pinholes, z forward.
 *   - Device buffers are borrowed: the library reads or writes them only from work
 *     enqueued on the given stream, so they must stay alive until that work completes.
 *     Outputs are caller-allocated.  `stream` is a hipStream_t (NULL = default stream).
 *   - A map is not thread-safe; order all calls on one map through one stream.
 *
 * Status codes: every call returns MAP_OK or a negative code; the text of the last
 * failure is available from map_last_error().
 */
#ifndef MAPCORE_H
#define MAPCORE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MAP_OK 0
#define MAP_ERR_INVALID_ARG -1
#define MAP_ERR_CAPACITY -2         /* a frame would exceed max_blocks: frame rejected */
#define MAP_ERR_BUFFER_TOO_SMALL -3 /* mesh output capacity too small */
#define MAP_ERR_NO_SCAN -4          /* labels before any accepted LiDAR frame */
#define MAP_ERR_DEVICE -5           /* HIP runtime error (see map_last_error) */

#define MAP_MESH_DIRTY 0 /* blocks changed since the last successful DIRTY extraction */
#define MAP_MESH_ALL 1   /* every allocated block; leaves the dirty set untouched */

typedef struct map_s map_t;

typedef struct {
    float voxel_size;   /* nu, metres (> 0) */
    float truncation;   /* tau, metres (0 < tau <= 64 nu) */
    int64_t max_blocks; /* capacity of the block pool (>= 1) */
    int32_t n_classes;  /* semantic classes L (1..254) */
    int32_t device;     /* HIP device ordinal */
} map_params;

typedef struct {
    int32_t rows, cols;    /* rows >= 2, cols >= 8 */
    const float *elev_rad; /* HOST pointer, rows entries, strictly decreasing, within
                              (-pi/2, pi/2) including half a row spacing beyond each end */
    float r_max;           /* metres */
} lidar_model;

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy; /* pixel (i, j) spans [i, i+1) x [j, j+1) */
} camera_model;

typedef struct {
    int64_t touched;     /* |T_k|: blocks met by the last frame's truncation bands */
    int64_t new_blocks;  /* blocks the last frame allocated */
    int64_t updates;     /* U_k: voxels whose distance and weight changed */
    int64_t votes;       /* V_k: label votes since the last LiDAR frame (all cameras) */
    int64_t mesh_blocks; /* blocks meshed by the last extraction */
    int64_t triangles;   /* triangles of the last extraction */
    int64_t allocated;   /* blocks in the map */
    int64_t frames;      /* accepted LiDAR frames */
    int64_t mesh_from_bitmap; /* 1 if the last extraction found its dirty blocks in the
                                 dirty bitmap, 0 if by a sweep of the slots */
} map_frame_stats;

/* Create an empty map on params->device: allocates and pre-initialises the block pool
 * (distance 0, weight 0 = unobserved, no votes, fused label 255), the block hash
 * (power of two >= 2 max_blocks slots) and the dirty set.  Work is enqueued on
 * `stream`; *out receives the map.  (Sec. IV-C.2: two-level voxel hashing.) */
int map_create(const map_params *params, void *stream, map_t **out);

/* Free every device and host resource of the map (NULL accepted).  Synchronises the
 * device first. */
void map_destroy(map_t *map);

/* Integrate one LiDAR range image taken at pose T_wl (Sec. IV-C.2, Eq. 5):
 *  1. allocation: every block met by the truncation band [max(r - tau, 0), r + tau]
 *     of a valid return (exact test in 2^-16-voxel fixed point, half-open blocks);
 *  2. projective TSDF: every voxel of those blocks takes the range of its nearest pixel
 *     (exact boundary predicates, ties to the higher index), psi = r - |p|; voxels with
 *     psi < -tau are skipped; w = min((psi + tau) / (2 tau), 1);
 *     D <- (W D + w min(psi, tau)) / (W + w), W <- W + w.
 * The touched blocks and their lower neighbours join the dirty set.
 * Asynchronous: returns after enqueueing the allocation pass, which also copies the range
 * image into the map.  The TSDF pass is enqueued by the map's next call, on this call's
 * stream: fused with the camera label fusion when that call is map_integrate_labels(_multi)
 * on the same stream (camera labels and counts or latest-label fusion), before anything
 * else otherwise; so range_dev need only stay valid until this call's work on `stream`
 * completes, as for any call.  If the frame would allocate more than max_blocks in total,
 * the frame is rejected on the device with the map unchanged (and later label calls are
 * no-ops until the next accepted frame); MAP_ERR_CAPACITY is then returned by the next
 * map_sync or map_stats. */
int map_integrate_lidar(map_t *map, const lidar_model *lidar, const float *range_dev,
                        const float T_wl[16], void *stream);

/* Fuse one camera label image taken at pose T_wc into the voxels updated by the last
 * accepted LiDAR frame whose |psi| <= tau (Sec. IV-C.3, Eq. 6 with hard labels): the
 * voxel centre is projected, pixel (floor u, floor v) is read, and if its label l is
 * below n_classes the voxel's count of l is incremented (saturating at 65535) and its
 * most probable label is updated (largest count, ties to the lowest id).  Call once per
 * camera.  Asynchronous.  MAP_ERR_NO_SCAN before the first LiDAR frame. */
int map_integrate_labels(map_t *map, const camera_model *cam, const uint8_t *labels_dev,
                         const float T_wc[16], void *stream);

/* The same for n cameras at once (host arrays: cams [n], labels_dev [n] device pointers,
 * T_wc [n][16]); the result equals n map_integrate_labels calls in array order. */
int map_integrate_labels_multi(map_t *map, int32_t n, const camera_model *cams,
                               const uint8_t *const *labels_dev, const float *T_wc, void *stream);

/* Marching cubes over blocks (end of Sec. IV-C.3): a cube whose eight corner voxels are
 * all observed (W > 0) emits triangles on its edges whose corners differ in D < 0;
 * each vertex lies at the linear zero crossing and carries the most probable label of
 * its endpoint with the smaller |D| (255 = none).  Triangles face D >= 0.
 * Outputs (device): pos [cap_tris][3][3] float, lab [cap_tris][3] uint8, and, if
 * non-NULL, edge_keys [cap_tris][3] int64 (the voxel v and axis of each vertex's edge:
 * ((vx + 2^19) << 42) | ((vy + 2^19) << 22) | ((vz + 2^19) << 2) | axis).
 * Writes the triangle count to the host *n_tris: the call returns as soon as the count
 * is known, while the triangles are still being written on `stream`, so order any use
 * of the outputs after it on that stream (or synchronise it).  If the count exceeds
 * cap_tris, only cap_tris triangles are written, MAP_ERR_BUFFER_TOO_SMALL is returned
 * and the dirty set is kept.  DIRTY mode clears the dirty set on success. */
int map_extract_mesh(map_t *map, int mode, float *pos_dev, uint8_t *lab_dev,
                     int64_t *edge_keys_dev, int64_t cap_tris, int64_t *n_tris, void *stream);

/* Work split of the per-map TSDF, label and meshing kernels (each 0 or 1): 0 = one
 * workgroup per block, 1 = one wavefront per block.  Results are identical either way;
 * only the speed differs.  Default 0, 0, 1.  The map's deferred TSDF launch, if any, is
 * enqueued first under the old schedule (its failure is returned).  MAP_ERR_INVALID_ARG
 * for a NULL map or a value other than 0 or 1 (the schedule is then unchanged). */
int map_set_schedule(map_t *map, int32_t tsdf, int32_t labels, int32_t mesh);

/* Candidates of DIRTY meshing (Sec. IV-C.3: only the blocks changed since the last
 * extraction are re-meshed).  The counting pass finds the dirty blocks either by a sweep of the
 * allocated slots (one coordinate read per slot) or, once the map holds more than
 * min_blocks blocks, from a dirty bitmap of one bit per slot that the TSDF pass keeps (one
 * bitmap read per slot, kept in the cache, and one coordinate read per dirty block).  An
 * extraction that follows a frame which ended at or below the threshold sweeps once more.
 * min_blocks < 0 (the default) takes the pool size one sweep round covers: 256 slots per
 * workgroup of the counting grid, 2^19 for a 2048-workgroup grid.  Results are identical
 * either way; only the speed differs.  The map's deferred TSDF launch, if any, is enqueued
 * first under the old threshold (its failure is returned).  MAP_ERR_INVALID_ARG for a
 * NULL map. */
int map_set_dirty_bitmap(map_t *map, int64_t min_blocks);

/* Label fusion from a label range image: the scan's points labelled by a point-cloud
 * segmentation network, the semantic measurements of the paper's LiDAR experiments
 * (Sec. V-A).  labels_dev: device uint8 [rows][cols] in the pixel layout of the scan model
 * L (as the range image); T_wl the scan's pose (host float row-major 4x4).  Every voxel
 * that the last accepted LiDAR frame updated within the truncation band (as for camera
 * labels) takes the label at its nearest pixel (the pixel rule of the projective update)
 * and votes as a camera label does (Eq. 6 with hard labels); labels >= n_classes (255 =
 * none) do not vote.  MAP_ERR_NO_SCAN before any LiDAR frame.  Asynchronous; a scan model
 * other than the one the map's tables were last built for rebuilds them after
 * synchronising the stream. */
int map_integrate_labels_lidar(map_t *map, const lidar_model *L, const uint8_t *labels_dev,
                               const float T_wl[16], void *stream);

/* Distance of the TSDF update (Sec. IV-C.2).  MAP_DIST_PROJECTIVE (the default): psi
 * along the ray, the paper's Ours-Proj baseline.  MAP_DIST_NONPROJECTIVE: the paper's own
 * distance (Eq. 4, "Ours"), with these readings of the paper:
 *   - each scan's normal image: pixel (k, c) back-projects to p = r d(k, c); its normal is
 *     the normalised cross product (p1 - p) x (p2 - p) with p1 from the pixel above (k-1, c)
 *     and p2 from the pixel to its left (k, c-1; columns wrap), turned to face the sensor;
 *     the top row and pixels next to an invalid return have none;
 *   - the point filter (Sec. V-C): a return is kept only if it has a normal and its ray
 *     meets it at no more than max_incidence radians; dropped returns take no part in the
 *     frame (allocation or update);
 *   - per-voxel unit gradients g (float [3] per voxel, pool allocated and zeroed by the
 *     first switch to this mode), the normalised weight-averaged normals of the voxel's
 *     pixels: g <- (W g + w n) / |W g + w n| at each update;
 *   - Eq. 4's second case lacks a length (the circle of Fig. 3b's radius, psi sin th / sin a
 *     by the sine rule); with the angles signed by the surface's bend both cases become
 *     d = -psi u.(e + n) / (1 + n.e), u the unit ray to the voxel, n its pixel's normal and
 *     e = g, or n where n.g <= 0 (no gradient yet);
 *   - Eq. 5 then averages min(max(d, -tau), tau) with the weight w of the projective psi
 *     (the same visibility, skip and band rules as the projective update).
 * Applies to later map_integrate_lidar calls; the batched step accepts only projective
 * maps.  MAP_ERR_INVALID_ARG for another mode or a non-finite or negative max_incidence.
 * Synchronises the map's last stream when it allocates the gradient pool
 * (max_blocks * 6 KiB). */
#define MAP_DIST_PROJECTIVE 0
#define MAP_DIST_NONPROJECTIVE 1
int map_set_distance(map_t *map, int32_t mode, float max_incidence);

/* Label fusion (Sec. IV-C.3).  MAP_LABELS_COUNTS (the default): vote counts with the most
 * probable label (Eq. 6 with hard labels; map_integrate_labels*).  MAP_LABELS_LATEST: a
 * visible voxel takes the label of its latest observation, counts untouched (the paper's
 * Ours-wo-Bay ablation, Sec. V-C; the same calls).  MAP_LABELS_BAYES: Eq. 6 on per-pixel
 * class log-probability images (map_integrate_logprobs only; the hard-label calls then
 * return MAP_ERR_INVALID_ARG), with L fp32 log-posteriors per voxel (pool of max_blocks *
 * L * 2 KiB, allocated and zeroed by the first switch to this mode, which synchronises the
 * map's last stream).  The batched step accepts only MAP_LABELS_COUNTS maps. */
#define MAP_LABELS_COUNTS 0
#define MAP_LABELS_LATEST 1
#define MAP_LABELS_BAYES 2
int map_set_label_fusion(map_t *map, int32_t mode);

/* Eq. 6 taken literally (Sec. IV-C.3): a camera's per-pixel class log-probabilities
 * logp_dev (device float [height][width][n_classes], e.g. a segmentation network's
 * log-softmax) at pose T_wc update every voxel the last accepted LiDAR frame updated with
 * |psi| <= tau that projects into the image (the visibility and pixel rule of
 * map_integrate_labels): its log-posteriors gain the pixel's log-probabilities, then the
 * largest sum is subtracted from all (the normaliser Z; the posterior's ratios, its argmax
 * and later updates are those Z gives), and its most probable label becomes the class at
 * 0 (the lowest on ties).  fp32, classes in increasing order.  Requires MAP_LABELS_BAYES
 * (else MAP_ERR_INVALID_ARG); MAP_ERR_NO_SCAN before any LiDAR frame.  Asynchronous. */
int map_integrate_logprobs(map_t *map, const camera_model *cam, const float *logp_dev, const float T_wc[16],
                           void *stream);

/* Measurement preprocessing (Eq. 3): depth image D = F r and height image H = F (z + O)
 * of n sensor-frame points (device float [n][3], undistorted), for the scan model L (the
 * same model map_integrate_lidar takes; D is then a range image it accepts when F = 1).
 * A point is valid when its coordinates are finite and 0 < r <= r_max, with r = |p|
 * rounded to fp32 as (x^2 + y^2) + z^2 then a correctly rounded square root; a valid
 * point goes to its nearest pixel (column c looks along azimuth pi - c 2pi/cols, row k
 * along elev_rad[k]; the exact boundary rule of the projective update).  A pixel keeps
 * its nearest point, the first in input order among equal ranges; pixels with no point
 * hold 0.  Outputs (device, row-major [rows][cols] float): depth (required), height
 * (nullable).  n <= 2^31 - 1.  The map contributes its device, look-up tables and a
 * per-pixel scratch image (8 bytes a pixel, grown on demand); the map's contents are not
 * read or changed.  Asynchronous, except that a scan model other than the one the map's
 * tables were last built for rebuilds them after synchronising the stream (as
 * map_integrate_lidar does); growing the scratch image synchronises the device. */
int map_range_image(map_t *map, const lidar_model *L, const float *pts_dev, int64_t n, float F, float O,
                    float *depth_dev, float *height_dev, void *stream);

/* Trilinear query of the distance field at n world points (device float [n][3]):
 * sdf [n] float, grad [n][3] float (nullable), valid [n] uint8.  A point is valid when
 * all eight voxels around it are observed; invalid points get 0.  Asynchronous. */
int map_query_sdf(map_t *map, const float *pts_dev, int64_t n, float *sdf_dev, float *grad_dev,
                  uint8_t *valid_dev, void *stream);

/* Loss and adjoint of B posed scans against the map: for pose b, xi_b = (t, w) (device
 * float [B][6]) maps the sensor-frame points p_bj (device float [B][N][3]) to
 * y = Exp(w) p + t; loss_b = sum_j valid * D(y)^2.  Writes loss [B], dL/dxi [B][6]
 * (translation part, then the rotation part through the SO(3) left Jacobian) and, if
 * non-NULL, dL/dp [B][N][3].  The reduction over points is in a fixed order (bitwise
 * reproducible).  Asynchronous. */
int map_sdf_pose_adjoint(map_t *map, const float *xi_dev, const float *pts_dev, int32_t B,
                         int64_t N, float *loss_dev, float *gxi_dev, float *gpts_dev, void *stream);

/* The same loss and adjoint for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the partial
 * sums go to a static device array of the library (4 MiB per device, held until the
 * process ends) instead of the map's scratch, and the call makes no allocation.  Limit:
 * B * ceil(N / 256) <= 131072 (MAP_ERR_INVALID_ARG beyond it).  Every call on one device
 * shares that array, so calls that overlap on one device (other streams, other maps, other
 * threads) race and must be ordered by the caller.  Results are bit-identical to
 * map_sdf_pose_adjoint.  Asynchronous. */
int map_sdf_pose_adjoint_noalloc(map_t *map, const float *xi_dev, const float *pts_dev, int32_t B,
                                 int64_t N, float *loss_dev, float *gxi_dev, float *gpts_dev, void *stream);

/* Batched integration (many maps of uneven size per step).  A batch holds up to 64 maps
 * created with map_create.  One map_batch_step integrates one frame into each listed map
 * (LiDAR scan, up to 8 camera label images, then DIRTY meshing into that map's output
 * buffers) with one launch per phase covering every map, replayed from a captured
 * hipGraph when enabled.  Each map ends in the state the same sequence of plain calls
 * (map_integrate_lidar, map_integrate_labels_multi, map_extract_mesh DIRTY) produces.
 * Items list distinct maps by index; the host pointers in an item are read during the
 * call.  n_tris [n_items] (host) receives each map's triangle count.  Returns MAP_OK,
 * MAP_ERR_BUFFER_TOO_SMALL if any map's output was too small (that map keeps its dirty
 * set), or an argument/device error; capacity rejections are reported per map by
 * map_sync.  Returns when every map's triangle count is known; the outputs are written
 * on `stream` after that, as with map_extract_mesh. */
typedef struct map_batch_s map_batch_t;
typedef struct {
    int32_t map_index;
    const lidar_model *lidar;
    const float *range_dev;
    const float *T_wl; /* host [16] */
    int32_t n_cams;    /* 0..8 */
    const camera_model *cams;
    const uint8_t *const *labels_dev;
    const float *T_wc; /* host [n_cams][16] */
    float *pos_dev;
    uint8_t *lab_dev;
    int64_t *edge_keys_dev; /* nullable */
    int64_t cap_tris;
} map_batch_item;

int map_batch_create(map_t *const *maps, int32_t n, map_batch_t **out);
/* schedule 0..3: one launch per phase for all maps; bit 0 for the TSDF phase, bit 1 for
 * the label phase, each 0 = one workgroup per touched block, 1 = one wavefront per touched
 * block; grid: workgroups of those phases (64..4096); use_graph: capture each step shape
 * once in a hipGraph and replay it.  schedule 4: each map's own kernels, as its plain calls
 * launch them (with its own schedules), the maps dealt over `grid` streams (1..16) of the
 * batch that run concurrently between the caller's stream's earlier and later work
 * (use_graph ignored).  Returns MAP_ERR_INVALID_ARG for values out of range. */
int map_batch_configure(map_batch_t *batch, int32_t schedule, int32_t grid, int32_t use_graph);
int map_batch_step(map_batch_t *batch, const map_batch_item *items, int32_t n_items, int64_t *n_tris,
                   void *stream);
void map_batch_destroy(map_batch_t *batch);

/* Synchronise the map's last stream and return (then clear) any deferred status. */
int map_sync(map_t *map);

/* Counters of the last frame, labels call and extraction (synchronises). */
int map_stats(map_t *map, map_frame_stats *out);

/* Message of the last failure on this map ("" if none).  With map == NULL: the last
 * failure of map_create. */
const char *map_last_error(const map_t *map);

/* Kernel timing with HIP events recorded on the launch stream around each launch of the
 * kernels selected by `mask` (bit i = kernel id i below; 0 disables).  map_profile_read
 * synchronises, writes per-kernel totals (ms) and launch counts since the last read into
 * arrays of MAP_KERNEL_COUNT entries, and clears them. */
#define MAP_K_ALLOC 0      /* band-segment walk, frame set, touched list */
#define MAP_K_TSDF 1       /* block commit, projective TSDF update, dirty marking */
#define MAP_K_LABELS 2     /* label vote fusion (one launch per up to 8 cameras) */
#define MAP_K_MESH 3       /* marching cubes */
#define MAP_K_QUERY 4      /* trilinear SDF query */
#define MAP_K_ADJOINT 5    /* pose / point adjoint (both of its launches) */
#define MAP_K_BATCH 6      /* batched multi-map step */
#define MAP_K_RANGE 7      /* point cloud to depth and height images (both launches) */
#define MAP_K_TSDF_LABELS 8 /* the TSDF launch with the frame's camera label fusion fused in */
#define MAP_KERNEL_COUNT 9
int map_profile(map_t *map, uint32_t mask);
int map_profile_read(map_t *map, double *total_ms, int64_t *launches);

/* Test and benchmark access (synchronous): copy the coordinates [n][3] int32 of all
 * allocated blocks in slot order, or the touched blocks of the last frame; returns the
 * count (entries beyond cap are not written). */
int64_t map_block_coords(map_t *map, int32_t *coords_host, int64_t cap);
int64_t map_touched_coords(map_t *map, int32_t *coords_host, int64_t cap);
/* Copy one block's voxels to host buffers (any may be NULL): D, W [512] float,
 * fused [512] uint8, counts [n_classes][512] uint16.  Returns 1, or 0 if absent. */
int map_read_block(map_t *map, int32_t bx, int32_t by, int32_t bz, float *D, float *W,
                   uint8_t *fused, uint16_t *counts);
/* Copy the first min(cap, allocated) blocks in slot order (any output may be NULL):
 * coords [cap][3] int32, D and W [cap][512] float, fused [cap][512] uint8, counts
 * [cap][n_classes][512] uint16.  Returns the number of allocated blocks, -1 on error. */
int64_t map_download(map_t *map, int64_t cap, int32_t *coords, float *D, float *W,
                     uint8_t *fused, uint16_t *counts);

/* Map-quality metrics (Sec. V-C): the vertices of a reconstructed mesh, M (device float
 * [n_mesh][3] with labels uint8 [n_mesh], 255 = unlabelled), against a ground-truth cloud
 * G (device float [n_gt][3] with classes uint8 [n_gt]), with cap = 2 voxel_size (computed
 * in double from the fp32 voxel size) and d(p, X) = min(cap, distance to the nearest point
 * of X), distances in fp64 from the fp32 coordinates, the nearest point the lowest index
 * among equidistant ones:
 *   re = sqrt(mean over M of d(p, G)^2)                             (Eq. 7)
 *   cd = mean over M of d(p, G) / 2 + mean over G of d(q, M) / 2     (Eq. 8)
 *   rc = fraction of G with a point of M within cap (completeness)
 *   every point of G within cap of M is evaluated with the label of its nearest vertex:
 *   confusion [pred (n_classes = none or unlabelled)][gt], per class IoU = TP / (TP + FP +
 *   FN) over the classes that occur, miou their mean, acc = correct / evaluated; points of
 *   G whose class is >= n_classes are not evaluated.
 * Optional outputs (NULL to skip): d_mesh_dev (device double [n_mesh], d(p, G)), d_gt_dev
 * (device double [n_gt], d(q, M)), nn_gt_dev (device int64 [n_gt], the nearest vertex of
 * each covered point, -1 otherwise), confusion_host (host int64 [(n_classes + 1)
 * n_classes]).  The library allocates its scratch (two cell grids) for the call and frees
 * it; synchronous.  Coordinates must lie within 2^20 cap of the origin.  Errors:
 * MAP_ERR_INVALID_ARG, MAP_ERR_DEVICE (text from map_last_error(NULL)). */
typedef struct {
    double re, cd, rc, miou, acc;
    int64_t n_eval; /* ground-truth points evaluated for the semantic scores */
} map_quality;
int map_mesh_quality(const float *mesh_pts_dev, const uint8_t *mesh_lab_dev, int64_t n_mesh,
                     const float *gt_pts_dev, const uint8_t *gt_lab_dev, int64_t n_gt, float voxel_size,
                     int32_t n_classes, int32_t device, double *d_mesh_dev, double *d_gt_dev, int64_t *nn_gt_dev,
                     int64_t *confusion_host, map_quality *out, void *stream);

/* Test access (synchronous): the per-voxel gradients [cap][3][512] float and
 * log-posteriors [cap][n_classes][512] float of the first min(cap, allocated) pool slots,
 * in the slot order of map_download (zeros while the mode's pool does not exist); either
 * may be NULL.  Returns the number of allocated blocks, -1 on error. */
int64_t map_download_aux(map_t *map, int64_t cap, float *grad, float *logpost);
/* Test access (synchronous): the last frame's normal image [rows * cols][4] float (world
 * normal xyz and kept range w, zeros where the point filter dropped the return) under the
 * non-projective distance; returns rows * cols, 0 in projective mode, -1 on error. */
int64_t map_frame_normals(map_t *map, float *out, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
