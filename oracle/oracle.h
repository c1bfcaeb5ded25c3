/*
 * CPU ORACLE for the metric-semantic mapping path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, scalar C that computes what the method computes, step by step, for
 * parity checks of the GPU library.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product never does.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * Method (paper Sec. IV-C): voxels of size nu with centres x = nu * v (Sec. IV-C.2),
 * grouped in 8x8x8 blocks held in a hash; projective signed distance psi along the
 * sensor ray, linear weight (psi + tau) / (2 tau), running weighted average with
 * truncation (Eq. 5); per-voxel class distribution updated by a recursive Bayes
 * filter (Eq. 6, taken here as per-class vote counts: see the label reading); marching
 * cubes with the most probable label per vertex (end of Sec. IV-C.3).
 */
#ifndef MAPPING_ORACLE_H
#define MAPPING_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OM_OK = 0, OM_INVALID = -1, OM_CAPACITY = -2, OM_BUFFER = -3, OM_NO_SCAN = -4 };
enum { OM_MESH_DIRTY = 0, OM_MESH_ALL = 1 };

typedef struct omap omap;

typedef struct {
    int64_t touched;     /* |T_k| */
    int64_t new_blocks;  /* |N_k| */
    int64_t updates;     /* U_k: voxels whose D, W changed */
    int64_t votes;       /* V_k: label votes since the last LiDAR frame */
    int64_t mesh_blocks; /* |M| meshed by the last extraction */
    int64_t triangles;   /* triangles of the last extraction */
    int64_t allocated;   /* blocks in the map */
} om_stats;

omap *om_create(float voxel, float trunc, int n_classes, int64_t max_blocks);
void om_destroy(omap *m);

/* range: rows*cols fp32 row-major; elev: rows fp32 radians, top row first; T_wl: 16 fp32
 * row-major.  Returns OM_OK, OM_INVALID or OM_CAPACITY (frame rejected, map unchanged). */
int om_integrate_lidar(omap *m, int rows, int cols, const float *elev, float r_max,
                       const float *range, const float *T_wl);
/* labels: height*width uint8 row-major; T_wc: 16 fp32.  Uses the last integrated scan. */
int om_integrate_labels(omap *m, int width, int height, float fx, float fy, float cx, float cy,
                        const uint8_t *labels, const float *T_wc);
/* Triangle soup: pos [3*cap][3] fp32, lab [3*cap], ekey [3*cap] (nullable).
 * *n_tris receives the count (also when the buffer is too small: OM_BUFFER). */
/* Label range image (rows x cols uint8, the scan model's pixel layout) under pose T:
 * each visible voxel of the last scan votes with the label at its nearest pixel. */
int om_integrate_labels_lidar(omap *m, int rows, int cols, const float *elev, const uint8_t *labels,
                              const float *T);
int om_extract_mesh(omap *m, int mode, int64_t cap_tris, float *pos, uint8_t *lab, int64_t *ekey,
                    int64_t *n_tris);

void om_get_stats(const omap *m, om_stats *s);
int64_t om_num_blocks(const omap *m);
/* block coordinates of all allocated blocks, [n][3] int32, in allocation order */
void om_block_coords(const omap *m, int32_t *out);
/* touched blocks of the last scan, [|T_k|][3] int32 (sorted by key) */
int64_t om_touched(const omap *m, int32_t *out, int64_t cap);
/* copy one block's voxels (x fastest); returns 0 if absent.  Any output may be NULL.
 * counts is [n_classes][512]. band is the last-scan band flag. */
int om_block_data(const omap *m, int bx, int by, int bz, float *D, float *W, uint8_t *fused,
                  uint16_t *counts, uint8_t *band);

/* Blocks met by the closed fixed-point segment [Q0, Q1] (2^-16 voxel units, offset so
 * voxel v spans [v, v+1) * 2^16): brute-force half-open slab test over the AABB. */
int64_t om_segment_blocks(const int64_t *Q0, const int64_t *Q1, int32_t *out, int64_t cap);
/* Fixed-point band segment of one return (for pins): writes Q0, Q1; 0 if invalid return */
int om_ray_segment(const omap *m, int rows, int cols, const float *elev, float r_max, int row,
                   int col, float r, const float *T_wl, int64_t *Q0, int64_t *Q1);
/* Pixel chosen for a sensor-frame point (for pins): returns 1 and row/col, or 0 if none. */
int om_pixel_of(int rows, int cols, const float *elev, const float *p, int *row, int *col);

/* Measurement preprocessing (Eq. 3): depth image D = F r and height image H = F (z + O)
 * of a sensor-frame point cloud pts[n][3].  Each valid point (finite, 0 < r <= r_max,
 * r = |p| in fp32) goes to its nearest pixel; a pixel keeps its nearest point, the lowest
 * index among equal ranges.  Pixels with no point hold 0 in D and H.  H may be NULL.
 * Returns the number of pixels written, or -1 for an invalid scan model. */
int64_t om_range_image(int rows, int cols, const float *elev, float r_max, const float *pts, int64_t n,
                       float F, float O, float *D, float *H);

/* Trilinear SDF query.  mode 0: fp64 points and decisions; mode 1: the points are fp32
 * values and the cell is chosen from the fp32 quotient x / nu.  grad nullable. */
void om_query_sdf(const omap *m, const double *pts, int64_t n, double *sdf, double *grad,
                  uint8_t *valid, int mode);
/* Pose adjoint in fp64: xi [B][6] = (t, omega); pts [B][N][3] fp32.
 * loss [B], gxi [B][6], gpts [B][N][3]; margin [B][N] (nullable): distance of x/nu
 * from the nearest integer plane (voxel units), for ill-conditioned-point masks. */
void om_pose_adjoint(const omap *m, const double *xi, const float *pts, int B, int64_t N,
                     double *loss, double *gxi, double *gpts, double *margin);

/* Test hooks: overwrite (creating if needed) one block's D, W, fused label and mark it
 * and its lower neighbours dirty; the rule's triangles (edge-id triples) for a mask. */
int om_set_block(omap *m, int bx, int by, int bz, const float *D, const float *W, const uint8_t *fused);
int om_cube_triangles(int inside_mask, int *out);

/* Distance of the TSDF update: mode 0 projective (the default; the paper's Ours-Proj),
 * mode 1 non-projective (the paper's Ours, Eq. 4): a normal image of each scan, a point
 * filter that keeps returns with a normal whose ray meets it at an angle of at most
 * max_incidence (radians), per-voxel unit gradients as the weighted average of normals,
 * and d = -psi u.(g + n) / (1 + n.g) truncated in place of psi (the weight stays the
 * linear weight of psi).  Returns OM_OK or OM_INVALID. */
int om_set_distance(omap *m, int mode, float max_incidence);
/* Normal image and point filter of one scan (for pins): range_out [rows*cols] holds the
 * kept returns (0 elsewhere), normals_out [rows*cols][3] their world-frame normals. */
int om_normal_image(int rows, int cols, const float *elev, float r_max, float max_incidence,
                    const float *range, const float *T_wl, float *range_out, float *normals_out);
/* The non-projective distance of Eq. 4 as read here (for pins): psi, ray u, gradient g,
 * normal n (g replaced by n when n.g <= 0). */
float om_nonproj_distance(float psi, const float *u, const float *g, const float *n);
/* A block's gradients [3][512] (zero in projective mode); returns 0 if absent. */
int om_block_gradient(const omap *m, int bx, int by, int bz, float *G);

/* Label fusion mode: 0 vote counts (the default; hard labels, Eq. 6 with a symmetric
 * likelihood), 1 latest label wins (the paper's Ours-wo-Bay: a visible voxel takes the
 * label of its latest observation; counts are untouched), 2 Eq. 6 on log-probability
 * images (om_integrate_logprobs; hard-label calls are then OM_INVALID).  Mode 2 keeps L
 * fp32 log-posteriors per voxel. */
int om_set_label_fusion(omap *m, int mode);
/* Eq. 6 with a camera's per-pixel class log-probabilities logp [height][width][L] (fp32):
 * each visible voxel of the last scan adds its pixel's log-probabilities to its
 * log-posterior and subtracts the largest (the normaliser); the most probable label is
 * the argmax, ties to the lowest class.  Returns OM_OK, OM_INVALID, OM_NO_SCAN. */
int om_integrate_logprobs(omap *m, int width, int height, float fx, float fy, float cx, float cy,
                          const float *logp, const float *T_wc);
/* A block's log-posteriors [L][512] (zero outside mode 2); returns 0 if absent. */
int om_block_logpost(const omap *m, int bx, int by, int bz, float *LP);

/* Threads this library uses: it is built twice from this one source, plain
 * (1 thread) and with OpenMP (loops over rows, touched blocks and meshed blocks run in
 * parallel; every result is identical, only the time differs). */
int om_threads(void);

#ifdef __cplusplus
}
#endif
#endif
