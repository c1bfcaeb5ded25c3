/*
 * CPU ORACLE for the metric-semantic mapping path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * this file's library.  It shares nothing with the GPU library: own types, own hash,
 * own look-up tables, and marching-cubes topology applied by rule per cube (no table).
 *
 * Written from the paper (Sec. IV-C) plus the readings listed with the design notes:
 *   - voxel centre x = nu * v, 8^3 blocks, block b = floor(v / 8)          (Sec. IV-C.2)
 *   - range-image geometry: column c looks along azimuth pi - c * 2 pi / C,
 *     row k along elevation elev[k]                                          (Eq. 3)
 *   - projective distance psi along the ray, D < 0 behind the surface       (Sec. IV-C.2)
 *   - linear weight w = (psi + tau) / (2 tau), running average, truncation  (Eq. 5)
 *   - recursive Bayes label filter (Eq. 6) with hard labels and a symmetric
 *     likelihood: the posterior's argmax equals the argmax of per-class vote counts
 *   - marching cubes, vertex label = the most probable label                (Sec. IV-C.3)
 *   - measurement preprocessing: depth and height images of a point cloud  (Eq. 3)
 *   - labels of the scan's points as a label range image                    (Sec. V-A)
 *
 * Arithmetic: every value that is stored in the map or decides which voxel, pixel or
 * block is touched is computed in IEEE binary32 with a fixed evaluation order and no
 * contraction (build with -ffp-contract=off), because the map stores fp32 distances
 * and weights and those decisions must be taken in the same precision on every side.
 * Sign decisions between a point and a pixel boundary are exact (fp64 products of fp32
 * operands).  The block walk is exact integer arithmetic.  The SDF query adjoint is fp64.
 *
 * Threads: the same source also builds with OpenMP (for the CPU timing baseline only).
 * Its parallel loops are over independent items (rows of a scan, touched blocks, meshed
 * blocks), each writing only its own item, with sums as reductions and per-block
 * outputs concatenated in order, so both builds compute identical results.
 *
 * Parity status: every function here is pinned by the CPU tests (closed forms, brute
 * force, invariants, textbook equivalences).  Two choices are fixed only by rule and
 * invariants, not by a value the paper prints: the label-visibility reading and the
 * marching-cubes triangulation rule.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BLOCK_VOXELS 512
#define DOMAIN_VOXELS ((1 << 19) - 64) /* |voxel index| stays below 2^19 */

typedef struct {
    int32_t b[3];
    float D[BLOCK_VOXELS];
    float W[BLOCK_VOXELS];
    uint8_t fused[BLOCK_VOXELS];
    uint8_t band[BLOCK_VOXELS];
    uint16_t *counts; /* [L][512] */
    float *G;         /* [3][512] unit gradient of the non-projective distance (all zero:
                         none yet); NULL while the map uses the projective distance */
    float *LP;        /* [L][512] log-posterior of each class relative to the most probable
                         one (Bayes label fusion); NULL in the other label modes */
    int dirty;
} oblock;

typedef struct {
    uint64_t *keys; /* 0 = empty; stored key is packed + 1 (unsigned: the packed key of
                       block (-1, -1, -1) is 2^63 - 1) */
    int64_t *vals;
    int64_t cap, n;
} ohash;

struct omap {
    float nu, tau;
    int L;
    int64_t max_blocks;
    ohash h;
    oblock **blocks;
    int64_t nblocks, cap_blocks;
    /* last scan */
    int has_scan;
    int64_t *touched;
    int64_t ntouched;
    om_stats st;
    /* distance: 0 projective (Ours-Proj), 1 non-projective (Ours, Eq. 4) */
    int nonproj;
    float cos_inc; /* returns whose ray meets their normal at a larger angle are dropped */
    /* label fusion: 0 vote counts (hard labels, Eq. 6 with a symmetric likelihood),
     * 1 latest label wins (the paper's Ours-wo-Bay), 2 Eq. 6 on log-probability images */
    int label_mode;
};

/* ------------------------------------------------------------------------------------ */
/* small helpers                                                                        */
/* ------------------------------------------------------------------------------------ */

static int64_t pack_key(int32_t x, int32_t y, int32_t z)
{
    return ((((int64_t)x) & 0x1FFFFF) << 42) | ((((int64_t)y) & 0x1FFFFF) << 21) |
           (((int64_t)z) & 0x1FFFFF);
}

static uint64_t mix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static void hash_init(ohash *h, int64_t cap)
{
    h->cap = cap;
    h->n = 0;
    h->keys = (uint64_t *)calloc(cap, sizeof(uint64_t));
    h->vals = (int64_t *)calloc(cap, sizeof(int64_t));
}

static void hash_free(ohash *h)
{
    free(h->keys);
    free(h->vals);
    h->keys = h->vals = NULL;
}

static int64_t hash_find(const ohash *h, int64_t key)
{
    uint64_t stored = (uint64_t)key + 1u;
    int64_t i = (int64_t)(mix64((uint64_t)key) & (uint64_t)(h->cap - 1));
    for (;;) {
        if (h->keys[i] == 0) return -1;
        if (h->keys[i] == stored) return h->vals[i];
        i = (i + 1) & (h->cap - 1);
    }
}

static void hash_put(ohash *h, int64_t key, int64_t val);

static void hash_grow(ohash *h)
{
    ohash nh;
    hash_init(&nh, h->cap * 2);
    for (int64_t i = 0; i < h->cap; ++i)
        if (h->keys[i]) hash_put(&nh, (int64_t)(h->keys[i] - 1u), h->vals[i]);
    hash_free(h);
    *h = nh;
}

static void hash_put(ohash *h, int64_t key, int64_t val)
{
    if (2 * (h->n + 1) > h->cap) hash_grow(h);
    uint64_t stored = (uint64_t)key + 1u;
    int64_t i = (int64_t)(mix64((uint64_t)key) & (uint64_t)(h->cap - 1));
    while (h->keys[i] != 0 && h->keys[i] != stored) i = (i + 1) & (h->cap - 1);
    if (h->keys[i] == 0) h->n++;
    h->keys[i] = stored;
    h->vals[i] = val;
}

static int64_t floor_div(int64_t a, int64_t d)
{
    int64_t q = a / d;
    if ((a % d != 0) && ((a < 0) != (d < 0))) q--;
    return q;
}

static oblock *find_block(const omap *m, int32_t x, int32_t y, int32_t z)
{
    int64_t i = hash_find(&m->h, pack_key(x, y, z));
    return i < 0 ? NULL : m->blocks[i];
}

/* voxel lookup: block pointer and local index of global voxel v */
static oblock *voxel_at(const omap *m, const int64_t v[3], int *local)
{
    int64_t b[3], l[3];
    for (int a = 0; a < 3; ++a) {
        b[a] = floor_div(v[a], 8);
        l[a] = v[a] - 8 * b[a];
    }
    *local = (int)(l[0] + 8 * l[1] + 64 * l[2]);
    return find_block(m, (int32_t)b[0], (int32_t)b[1], (int32_t)b[2]);
}

/* ------------------------------------------------------------------------------------ */
/* create / destroy                                                                     */
/* ------------------------------------------------------------------------------------ */

omap *om_create(float voxel, float trunc, int n_classes, int64_t max_blocks)
{
    if (!(voxel > 0.0f) || !(trunc > 0.0f) || !isfinite(voxel) || !isfinite(trunc)) return NULL;
    if (trunc > 64.0f * voxel) return NULL;
    if (n_classes < 1 || n_classes > 254 || max_blocks < 1) return NULL;
    omap *m = (omap *)calloc(1, sizeof(omap));
    m->nu = voxel;
    m->tau = trunc;
    m->L = n_classes;
    m->max_blocks = max_blocks;
    hash_init(&m->h, 1024);
    m->cap_blocks = 1024;
    m->blocks = (oblock **)calloc(m->cap_blocks, sizeof(oblock *));
    return m;
}

void om_destroy(omap *m)
{
    if (!m) return;
    for (int64_t i = 0; i < m->nblocks; ++i) {
        free(m->blocks[i]->counts);
        free(m->blocks[i]->G);
        free(m->blocks[i]->LP);
        free(m->blocks[i]);
    }
    free(m->blocks);
    hash_free(&m->h);
    free(m->touched);
    free(m);
}

static oblock *new_block(omap *m, int32_t x, int32_t y, int32_t z)
{
    if (m->nblocks == m->cap_blocks) {
        m->cap_blocks *= 2;
        m->blocks = (oblock **)realloc(m->blocks, m->cap_blocks * sizeof(oblock *));
    }
    oblock *b = (oblock *)calloc(1, sizeof(oblock));
    b->b[0] = x; b->b[1] = y; b->b[2] = z;
    /* initial state: D = 0, W = 0 (unobserved), no votes, fused label unknown (255) */
    memset(b->fused, 255, sizeof(b->fused));
    b->counts = (uint16_t *)calloc((size_t)m->L * BLOCK_VOXELS, sizeof(uint16_t));
    if (m->nonproj) b->G = (float *)calloc(3 * BLOCK_VOXELS, sizeof(float));
    if (m->label_mode == 2) b->LP = (float *)calloc((size_t)m->L * BLOCK_VOXELS, sizeof(float));
    m->blocks[m->nblocks] = b;
    hash_put(&m->h, pack_key(x, y, z), m->nblocks);
    m->nblocks++;
    return b;
}

/* ------------------------------------------------------------------------------------ */
/* argument checks shared by the calls                                                  */
/* ------------------------------------------------------------------------------------ */

static int check_pose(const float *T)
{
    for (int i = 0; i < 16; ++i)
        if (!isfinite(T[i])) return 0;
    if (T[12] != 0.0f || T[13] != 0.0f || T[14] != 0.0f || T[15] != 1.0f) return 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += (double)T[4 * k + i] * (double)T[4 * k + j];
            if (fabs(s - (i == j ? 1.0 : 0.0)) > 1e-5) return 0;
        }
    double det = (double)T[0] * ((double)T[5] * T[10] - (double)T[6] * T[9]) -
                 (double)T[1] * ((double)T[4] * T[10] - (double)T[6] * T[8]) +
                 (double)T[2] * ((double)T[4] * T[9] - (double)T[5] * T[8]);
    return det > 0.0;
}

/* ------------------------------------------------------------------------------------ */
/* sensor look-up tables (fp32 values computed once in double)                          */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int R, C;
    float *ce, *se;      /* ray elevation cos/sin per row */
    float *cp, *sp;      /* ray azimuth cos/sin per column */
    float *bcx, *bcy;    /* azimuth boundary j between columns j-1 and j, j in [0, C) */
    float *brc, *brs;    /* elevation boundary j, j in [0, R]: cos, sin */
} lut;

static int lut_build(lut *t, int R, int C, const float *elev)
{
    if (R < 2 || C < 8) return 0;
    for (int k = 0; k < R; ++k)
        if (!isfinite(elev[k])) return 0;
    for (int k = 1; k < R; ++k)
        if (!(elev[k] < elev[k - 1])) return 0;
    double e0 = elev[0], e1 = elev[1], en = elev[R - 1], en1 = elev[R - 2];
    double top = e0 + 0.5 * (e0 - e1), bot = en - 0.5 * (en1 - en);
    if (!(top < M_PI / 2) || !(bot > -M_PI / 2)) return 0;
    t->R = R;
    t->C = C;
    t->ce = (float *)malloc(R * sizeof(float));
    t->se = (float *)malloc(R * sizeof(float));
    t->cp = (float *)malloc(C * sizeof(float));
    t->sp = (float *)malloc(C * sizeof(float));
    t->bcx = (float *)malloc(C * sizeof(float));
    t->bcy = (float *)malloc(C * sizeof(float));
    t->brc = (float *)malloc((R + 1) * sizeof(float));
    t->brs = (float *)malloc((R + 1) * sizeof(float));
    for (int k = 0; k < R; ++k) {
        t->ce[k] = (float)cos((double)elev[k]);
        t->se[k] = (float)sin((double)elev[k]);
    }
    double dphi = 2.0 * M_PI / (double)C;
    for (int c = 0; c < C; ++c) {
        double phi = M_PI - (double)c * dphi;
        t->cp[c] = (float)cos(phi);
        t->sp[c] = (float)sin(phi);
        double pb = M_PI - ((double)c - 0.5) * dphi;
        t->bcx[c] = (float)cos(pb);
        t->bcy[c] = (float)sin(pb);
    }
    for (int j = 0; j <= R; ++j) {
        double eb;
        if (j == 0) eb = top;
        else if (j == R) eb = bot;
        else eb = 0.5 * ((double)elev[j - 1] + (double)elev[j]);
        t->brc[j] = (float)cos(eb);
        t->brs[j] = (float)sin(eb);
    }
    return 1;
}

static void lut_free(lut *t)
{
    free(t->ce); free(t->se); free(t->cp); free(t->sp);
    free(t->bcx); free(t->bcy); free(t->brc); free(t->brs);
}

/* exact sign of ax*qy - ay*qx for fp32 operands: both products are exact in fp64 */
static int cross_sign(float ax, float ay, float qx, float qy)
{
    double v = (double)ax * (double)qy - (double)ay * (double)qx;
    return (v > 0.0) - (v < 0.0);
}

/* Column c holds the points strictly counter-clockwise of boundary c+1 and clockwise of,
 * or on, boundary c: a point on a boundary goes to the higher column index. */
static int in_column(const lut *t, int c, float px, float py)
{
    int c1 = (c + 1 == t->C) ? 0 : c + 1;
    return cross_sign(t->bcx[c1], t->bcy[c1], px, py) > 0 &&
           cross_sign(t->bcx[c], t->bcy[c], px, py) <= 0;
}

/* Row k holds (rho, z) strictly above boundary k+1 and below or on boundary k. */
static int in_row(const lut *t, int k, float rho, float z)
{
    return cross_sign(t->brc[k + 1], t->brs[k + 1], rho, z) > 0 &&
           cross_sign(t->brc[k], t->brs[k], rho, z) <= 0;
}

/* nearest pixel of sensor-frame point p, chosen by the exact predicates */
static int pixel_of(const lut *t, float px, float py, float pz, int *row, int *col)
{
    if (px == 0.0f && py == 0.0f) return 0;
    /* column: initial guess from atan2, then the predicates decide */
    double dphi = 2.0 * M_PI / (double)t->C;
    double a = (M_PI - atan2((double)py, (double)px)) / dphi;
    long g = (long)floor(a + 0.5);
    g %= t->C;
    if (g < 0) g += t->C;
    int col_found = -1;
    for (int d = -1; d <= 1 && col_found < 0; ++d) {
        int c = (int)((g + d + t->C) % t->C);
        if (in_column(t, c, px, py)) col_found = c;
    }
    if (col_found < 0)
        for (int c = 0; c < t->C; ++c)
            if (in_column(t, c, px, py)) { col_found = c; break; }
    if (col_found < 0) return 0;
    /* row: rho in fp32, then a scan over the monotone boundaries */
    float rho = sqrtf(px * px + py * py);
    if (cross_sign(t->brc[0], t->brs[0], rho, pz) > 0) return 0;      /* above the top */
    if (cross_sign(t->brc[t->R], t->brs[t->R], rho, pz) <= 0) return 0; /* on/below the bottom */
    int row_found = -1;
    int lo = 0, hi = t->R - 1;
    /* boundaries decrease with index: find the last k with (rho, z) on/below boundary k */
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (cross_sign(t->brc[mid], t->brs[mid], rho, pz) <= 0) lo = mid;
        else hi = mid - 1;
    }
    if (in_row(t, lo, rho, pz)) row_found = lo;
    if (row_found < 0) return 0;
    *row = row_found;
    *col = col_found;
    return 1;
}

int om_pixel_of(int rows, int cols, const float *elev, const float *p, int *row, int *col)
{
    lut t;
    if (!lut_build(&t, rows, cols, elev)) return 0;
    int ok = pixel_of(&t, p[0], p[1], p[2], row, col);
    lut_free(&t);
    return ok;
}

/* Measurement preprocessing (Eq. 3): the point cloud's depth and height images.  The
 * paper gives the pixel as (pi - atan2(y, x)) / dphi and the elevation's offset over its
 * spacing; a point here goes to the nearest pixel centre by the same exact predicates as
 * the projective update, so a scan converted to points and back keeps every return at its
 * pixel.  Several points on one pixel: the nearest is kept (ties: the first in input
 * order), as a depth buffer does.  D = F r and H = F (z + O) with the scalars of Eq. 3. */
static int valid_return(float r, float r_max);

int64_t om_range_image(int rows, int cols, const float *elev, float r_max, const float *pts, int64_t n,
                       float F, float O, float *D, float *H)
{
    lut t;
    if (!lut_build(&t, rows, cols, elev)) return -1;
    const int64_t np = (int64_t)rows * cols;
    float *best = (float *)malloc(np * sizeof(float));
    int64_t *who = (int64_t *)malloc(np * sizeof(int64_t));
    for (int64_t q = 0; q < np; ++q) {
        best[q] = INFINITY;
        who[q] = -1;
    }
    for (int64_t i = 0; i < n; ++i) {
        const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) continue;
        const float r = sqrtf((x * x + y * y) + z * z);
        if (!valid_return(r, r_max)) continue;
        int row, col;
        if (!pixel_of(&t, x, y, z, &row, &col)) continue;
        const int64_t q = (int64_t)row * cols + col;
        if (r < best[q]) {
            best[q] = r;
            who[q] = i;
        }
    }
    int64_t written = 0;
    for (int64_t q = 0; q < np; ++q) {
        if (who[q] < 0) {
            D[q] = 0.0f;
            if (H) H[q] = 0.0f;
            continue;
        }
        D[q] = F * best[q];
        if (H) H[q] = F * (pts[3 * who[q] + 2] + O);
        ++written;
    }
    free(best);
    free(who);
    lut_free(&t);
    return written;
}

/* ------------------------------------------------------------------------------------ */
/* allocation: exact block set of a fixed-point band segment                            */
/* ------------------------------------------------------------------------------------ */

#define FX_SHIFT 16            /* 2^-16 voxel fixed point */
#define BLOCK_FX (8LL << FX_SHIFT)

typedef __int128 i128;

/* a rational bound n/d (d > 0) with an open/closed flag */
typedef struct { int64_t n, d; int open; } tbound;

static int rat_cmp(int64_t an, int64_t ad, int64_t bn, int64_t bd)
{
    i128 l = (i128)an * bd, r = (i128)bn * ad;
    return (l > r) - (l < r);
}

/* Does the closed segment Q0 + t (Q1 - Q0), t in [0, 1], meet the half-open cell
 * [lo, lo + BLOCK_FX)^3 of block b?  Liang-Barsky with exact rational comparisons. */
static int segment_meets_block(const int64_t *Q0, const int64_t *Q1, const int64_t *b)
{
    tbound lower = {0, 1, 0}, upper = {1, 1, 0};
    for (int a = 0; a < 3; ++a) {
        int64_t lo = b[a] * BLOCK_FX, hi = lo + BLOCK_FX;
        int64_t d = Q1[a] - Q0[a];
        if (d == 0) {
            if (!(lo <= Q0[a] && Q0[a] < hi)) return 0;
            continue;
        }
        tbound l, u;
        if (d > 0) {
            l.n = lo - Q0[a]; l.d = d; l.open = 0; /* t >= (lo - Q0) / d */
            u.n = hi - Q0[a]; u.d = d; u.open = 1; /* t <  (hi - Q0) / d */
        } else {
            u.n = Q0[a] - lo; u.d = -d; u.open = 0; /* t <= (Q0 - lo) / |d| */
            l.n = Q0[a] - hi; l.d = -d; l.open = 1; /* t >  (Q0 - hi) / |d| */
        }
        int c = rat_cmp(l.n, l.d, lower.n, lower.d);
        if (c > 0 || (c == 0 && l.open)) lower = l;
        c = rat_cmp(u.n, u.d, upper.n, upper.d);
        if (c < 0 || (c == 0 && u.open)) upper = u;
    }
    int c = rat_cmp(lower.n, lower.d, upper.n, upper.d);
    if (c < 0) return 1;
    if (c == 0 && !lower.open && !upper.open) return 1;
    return 0;
}

int64_t om_segment_blocks(const int64_t *Q0, const int64_t *Q1, int32_t *out, int64_t cap)
{
    int64_t lo[3], hi[3], n = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t mn = Q0[a] < Q1[a] ? Q0[a] : Q1[a], mx = Q0[a] < Q1[a] ? Q1[a] : Q0[a];
        lo[a] = floor_div(mn, BLOCK_FX);
        hi[a] = floor_div(mx, BLOCK_FX);
    }
    int64_t b[3];
    for (b[2] = lo[2]; b[2] <= hi[2]; ++b[2])
        for (b[1] = lo[1]; b[1] <= hi[1]; ++b[1])
            for (b[0] = lo[0]; b[0] <= hi[0]; ++b[0])
                if (segment_meets_block(Q0, Q1, b)) {
                    if (n < cap) {
                        out[3 * n] = (int32_t)b[0];
                        out[3 * n + 1] = (int32_t)b[1];
                        out[3 * n + 2] = (int32_t)b[2];
                    }
                    n++;
                }
    return n;
}

static int valid_return(float r, float r_max) { return isfinite(r) && r > 0.0f && r <= r_max; }

/* ------------------------------------------------------------------------------------ */
/* non-projective distance (Sec. IV-C.2, Eq. 4): normal image, point filter, distance    */
/* ------------------------------------------------------------------------------------ */

/* Normal image of a scan (Sec. IV-C.2).  Pixel (k, c) back-projects to p = r d(k, c); its
 * normal is the normalised cross product (p1 - p) x (p2 - p) with p1 from the pixel above
 * (k - 1, c) and p2 from the pixel to its left (k, c - 1), columns wrapping around (the
 * scan is a full turn).  Readings: the top row, and pixels whose own or neighbouring
 * return is invalid, have no normal; the normal is turned to face the sensor.  Point
 * filter (Sec. V-C): a return is kept only if it has a normal and the angle between its
 * ray and the normal is at most the incidence limit (cos >= cos_inc).  Outputs: the
 * filtered range image (0 where dropped) and, for kept returns, the normal rotated into
 * the world frame by T ([R*C][3], zero elsewhere).  fp32, fixed order. */
static void normal_image(const lut *t, const float *range, float r_max, float cos_inc, const float *T,
                         float *rng_out, float *nrm_out)
{
    const int R = t->R, C = t->C;
    for (int k = 0; k < R; ++k)
        for (int c = 0; c < C; ++c) {
            const int64_t q = (int64_t)k * C + c;
            rng_out[q] = 0.0f;
            nrm_out[3 * q] = nrm_out[3 * q + 1] = nrm_out[3 * q + 2] = 0.0f;
            const float r = range[q];
            if (k == 0 || !valid_return(r, r_max)) continue;
            const int cl = c == 0 ? C - 1 : c - 1;
            const float r1 = range[q - C], r2 = range[(int64_t)k * C + cl];
            if (!valid_return(r1, r_max) || !valid_return(r2, r_max)) continue;
            const float dx = t->ce[k] * t->cp[c], dy = t->ce[k] * t->sp[c], dz = t->se[k];
            const float px = r * dx, py = r * dy, pz = r * dz;
            const float p1x = r1 * (t->ce[k - 1] * t->cp[c]), p1y = r1 * (t->ce[k - 1] * t->sp[c]),
                        p1z = r1 * t->se[k - 1];
            const float p2x = r2 * (t->ce[k] * t->cp[cl]), p2y = r2 * (t->ce[k] * t->sp[cl]), p2z = r2 * t->se[k];
            const float ax = p1x - px, ay = p1y - py, az = p1z - pz;
            const float bx = p2x - px, by = p2y - py, bz = p2z - pz;
            float nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
            const float l2 = (nx * nx + ny * ny) + nz * nz;
            if (!(l2 > 0.0f) || !isfinite(l2)) continue;
            const float l = sqrtf(l2);
            nx = nx / l;
            ny = ny / l;
            nz = nz / l;
            float s = (nx * dx + ny * dy) + nz * dz;  /* cosine of the normal to the ray */
            if (s > 0.0f) {
                nx = -nx;
                ny = -ny;
                nz = -nz;
                s = -s;
            }
            if (!(-s >= cos_inc)) continue;
            rng_out[q] = r;
            for (int i = 0; i < 3; ++i)
                nrm_out[3 * q + i] = (T[4 * i] * nx + T[4 * i + 1] * ny) + T[4 * i + 2] * nz;
        }
}

int om_normal_image(int rows, int cols, const float *elev, float r_max, float max_incidence,
                    const float *range, const float *T_wl, float *range_out, float *normals_out)
{
    lut t;
    if (!range || !T_wl || !range_out || !normals_out) return OM_INVALID;
    if (!lut_build(&t, rows, cols, elev)) return OM_INVALID;
    normal_image(&t, range, r_max, (float)cos((double)max_incidence), T_wl, range_out, normals_out);
    lut_free(&t);
    return OM_OK;
}

/* Eq. 4 as read here.  The printed second case adds |(cos a - 1) sin th / sin a| to
 * |cos th| psi: a ratio without a length.  For a surface that is locally a circle (Fig.
 * 3b) through the measured point p with normal n there, and a voxel x = p - psi u on the
 * ray u whose distance gradient is g, the sine rule in the triangle (centre, p, x) gives
 * the radius as psi sin th / sin a, so the missing factor is psi and the term is the gap
 * (cos a - 1) r between that circle and the plane through p normal to g; its sign is
 * the surface's bend (negative when convex toward the voxel).  With the angles' signs
 * taken from the vectors, both cases of Eq. 4 collapse into
 *     d = -psi u.(g + n) / (1 + n.g),
 * which is |cos th| psi when g = n and the exact distance to a sphere or a cylinder
 * whatever the bend (the CPU tests pin both).  It needs n.g > -1; where the gradient and
 * the normal are 90 degrees or more apart (or there is no gradient yet) g is taken to be
 * n.  fp32 in this order. */
static float nonproj_distance(float psi, float ux, float uy, float uz, const float g[3], const float n[3])
{
    const float hx = g[0] + n[0], hy = g[1] + n[1], hz = g[2] + n[2];
    const float uh = (ux * hx + uy * hy) + uz * hz;
    const float ng = (n[0] * g[0] + n[1] * g[1]) + n[2] * g[2];
    const float f = uh / (1.0f + ng);
    return -(psi * f);
}

float om_nonproj_distance(float psi, const float *u, const float *g, const float *n)
{
    float ge[3] = {g[0], g[1], g[2]};
    const float ng = (n[0] * g[0] + n[1] * g[1]) + n[2] * g[2];
    if (!(ng > 0.0f)) ge[0] = n[0], ge[1] = n[1], ge[2] = n[2];
    return nonproj_distance(psi, u[0], u[1], u[2], ge, n);
}

int om_set_distance(omap *m, int mode, float max_incidence)
{
    if (!m || (mode != 0 && mode != 1) || !isfinite(max_incidence) || max_incidence < 0.0f) return OM_INVALID;
    m->nonproj = mode;
    m->cos_inc = (float)cos((double)max_incidence);
    if (mode)
        for (int64_t i = 0; i < m->nblocks; ++i)
            if (!m->blocks[i]->G) m->blocks[i]->G = (float *)calloc(3 * BLOCK_VOXELS, sizeof(float));
    return OM_OK;
}

int om_block_gradient(const omap *m, int bx, int by, int bz, float *G)
{
    oblock *b = find_block(m, bx, by, bz);
    if (!b) return 0;
    if (b->G) memcpy(G, b->G, 3 * BLOCK_VOXELS * sizeof(float));
    else memset(G, 0, 3 * BLOCK_VOXELS * sizeof(float));
    return 1;
}

/* band segment [max(r - tau, 0), r + tau] of one return in 2^-16 voxel fixed point */
static void ray_segment(const omap *m, const lut *t, int k, int c, float r, const float *T,
                        int64_t *Q0, int64_t *Q1)
{
    float dx = t->ce[k] * t->cp[c], dy = t->ce[k] * t->sp[c], dz = t->se[k];
    float w[3];
    for (int i = 0; i < 3; ++i) w[i] = (T[4 * i] * dx + T[4 * i + 1] * dy) + T[4 * i + 2] * dz;
    float s0 = r - m->tau;
    if (!(s0 > 0.0f)) s0 = 0.0f;
    float s1 = r + m->tau;
    for (int i = 0; i < 3; ++i) {
        float o = T[4 * i + 3];
        float p0 = o + s0 * w[i], p1 = o + s1 * w[i];
        float q0 = p0 / m->nu + 0.5f, q1 = p1 / m->nu + 0.5f;
        Q0[i] = (int64_t)rintf(q0 * 65536.0f);
        Q1[i] = (int64_t)rintf(q1 * 65536.0f);
    }
}

int om_ray_segment(const omap *m, int rows, int cols, const float *elev, float r_max, int row,
                   int col, float r, const float *T_wl, int64_t *Q0, int64_t *Q1)
{
    lut t;
    if (!lut_build(&t, rows, cols, elev)) return 0;
    int ok = valid_return(r, r_max);
    if (ok) ray_segment(m, &t, row, col, r, T_wl, Q0, Q1);
    lut_free(&t);
    return ok;
}

/* ------------------------------------------------------------------------------------ */
/* integrate one LiDAR scan: allocation, then the TSDF update (Eq. 5)                   */
/* ------------------------------------------------------------------------------------ */

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int om_integrate_lidar(omap *m, int rows, int cols, const float *elev, float r_max,
                       const float *range, const float *T)
{
    if (!m || !elev || !range || !T) return OM_INVALID;
    if (!(r_max > 0.0f) || !isfinite(r_max) || !check_pose(T)) return OM_INVALID;
    {
        double lim = (double)m->nu * DOMAIN_VOXELS;
        for (int i = 0; i < 3; ++i)
            if (fabs((double)T[4 * i + 3]) + (double)r_max + (double)m->tau >= lim) return OM_INVALID;
    }
    lut t;
    if (!lut_build(&t, rows, cols, elev)) return OM_INVALID;
    /* non-projective distance: the normal image and the point filter first; the kept
     * returns are the scan from here on (allocation and update) */
    float *nrm = NULL, *kept = NULL;
    if (m->nonproj) {
        kept = (float *)malloc((size_t)rows * cols * sizeof(float));
        nrm = (float *)malloc((size_t)rows * cols * 3 * sizeof(float));
        normal_image(&t, range, r_max, m->cos_inc, T, kept, nrm);
        range = kept;
    }

    /* T_k: every block met by the band segment of a valid return.  Each row's blocks
     * are listed on their own (rows are independent: the OpenMP build takes them in
     * parallel), then merged without repeats. */
    int64_t **rowkeys = (int64_t **)calloc((size_t)rows, sizeof(int64_t *));
    int64_t *rown = (int64_t *)calloc((size_t)rows, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < rows; ++k) {
        int32_t cand[3 * 256];
        int64_t cap = 256, n = 0;
        int64_t *keys = (int64_t *)malloc(cap * sizeof(int64_t));
        for (int c = 0; c < cols; ++c) {
            float r = range[(size_t)k * cols + c];
            if (!valid_return(r, r_max)) continue;
            int64_t Q0[3], Q1[3];
            ray_segment(m, &t, k, c, r, T, Q0, Q1);
            int64_t nb = om_segment_blocks(Q0, Q1, cand, 256);
            if (nb > 256) abort(); /* cannot happen for tau <= 64 nu */
            for (int64_t j = 0; j < nb; ++j) {
                if (n == cap) {
                    cap *= 2;
                    keys = (int64_t *)realloc(keys, cap * sizeof(int64_t));
                }
                keys[n++] = pack_key(cand[3 * j], cand[3 * j + 1], cand[3 * j + 2]);
            }
        }
        rowkeys[k] = keys;
        rown[k] = n;
    }
    ohash frame;
    hash_init(&frame, 1024);
    int64_t nlist = 0, caplist = 1024;
    int64_t *list = (int64_t *)malloc(caplist * sizeof(int64_t));
    for (int k = 0; k < rows; ++k) {
        for (int64_t j = 0; j < rown[k]; ++j) {
            int64_t key = rowkeys[k][j];
            if (hash_find(&frame, key) >= 0) continue;
            hash_put(&frame, key, nlist);
            if (nlist == caplist) {
                caplist *= 2;
                list = (int64_t *)realloc(list, caplist * sizeof(int64_t));
            }
            list[nlist++] = key;
        }
        free(rowkeys[k]);
    }
    free(rowkeys);
    free(rown);
    hash_free(&frame);
    /* N_k and the capacity check happen before any block is created */
    int64_t n_new = 0;
    for (int64_t i = 0; i < nlist; ++i)
        if (hash_find(&m->h, list[i]) < 0) n_new++;
    if (m->nblocks + n_new > m->max_blocks) {
        /* rejected: the map is unchanged, and the scan it leaves for label calls is
         * empty (a frame was submitted, so they are no-ops, not NO_SCAN) */
        free(list);
        free(kept);
        free(nrm);
        lut_free(&t);
        m->ntouched = 0;
        m->has_scan = 1;
        m->st.touched = 0;
        m->st.new_blocks = 0;
        m->st.updates = 0;
        m->st.votes = 0;
        return OM_CAPACITY;
    }
    qsort(list, nlist, sizeof(int64_t), cmp_i64);
    free(m->touched);
    m->touched = (int64_t *)malloc((nlist > 0 ? nlist : 1) * sizeof(int64_t));
    m->ntouched = nlist;
    for (int64_t i = 0; i < nlist; ++i) {
        int64_t key = list[i];
        int64_t idx = hash_find(&m->h, key);
        if (idx < 0) {
            /* unpack the 21-bit signed fields */
            int32_t x = (int32_t)((key >> 42) & 0x1FFFFF), y = (int32_t)((key >> 21) & 0x1FFFFF),
                    z = (int32_t)(key & 0x1FFFFF);
            if (x & 0x100000) x -= 0x200000;
            if (y & 0x100000) y -= 0x200000;
            if (z & 0x100000) z -= 0x200000;
            new_block(m, x, y, z);
            idx = m->nblocks - 1;
        }
        m->touched[i] = idx;
    }
    free(list);

    /* TSDF update over every voxel of every touched block */
    const float nu = m->nu, tau = m->tau, two_tau = m->tau + m->tau;
    const float tx = T[3], ty = T[7], tz = T[11];
    int64_t updates = 0;
    /* blocks are independent (one update per voxel per frame) */
#pragma omp parallel for reduction(+ : updates) schedule(dynamic, 4)
    for (int64_t i = 0; i < m->ntouched; ++i) {
        oblock *b = m->blocks[m->touched[i]];
        memset(b->band, 0, sizeof(b->band));
        for (int lz = 0; lz < 8; ++lz)
            for (int ly = 0; ly < 8; ++ly)
                for (int lx = 0; lx < 8; ++lx) {
                    int li = lx + 8 * ly + 64 * lz;
                    float x = (float)(8 * b->b[0] + lx) * nu;
                    float y = (float)(8 * b->b[1] + ly) * nu;
                    float z = (float)(8 * b->b[2] + lz) * nu;
                    float dx = x - tx, dy = y - ty, dz = z - tz;
                    /* p = R^T (x - t) */
                    float px = (T[0] * dx + T[4] * dy) + T[8] * dz;
                    float py = (T[1] * dx + T[5] * dy) + T[9] * dz;
                    float pz = (T[2] * dx + T[6] * dy) + T[10] * dz;
                    if (px == 0.0f && py == 0.0f && pz == 0.0f) continue;
                    int row, col;
                    if (!pixel_of(&t, px, py, pz, &row, &col)) continue;
                    float r = range[(size_t)row * cols + col];
                    if (!valid_return(r, r_max)) continue;
                    float dist = sqrtf((px * px + py * py) + pz * pz);
                    float psi = r - dist;
                    if (psi < -tau) continue;
                    float w = (psi + tau) / two_tau;
                    if (w > 1.0f) w = 1.0f;
                    if (w == 0.0f) continue;
                    float Wo = b->W[li], Do = b->D[li];
                    float gam;
                    if (nrm) {
                        /* Eq. 4 with the normal of the voxel's pixel and the voxel's
                         * gradient; the ray is the direction from the sensor to the voxel */
                        const float *n = nrm + 3 * ((size_t)row * cols + col);
                        float *G = b->G;
                        const float gs[3] = {G[li], G[BLOCK_VOXELS + li], G[2 * BLOCK_VOXELS + li]};
                        const float ng = (n[0] * gs[0] + n[1] * gs[1]) + n[2] * gs[2];
                        const float *ge = ng > 0.0f ? gs : n;
                        const float ux = dx / dist, uy = dy / dist, uz = dz / dist;
                        const float d = nonproj_distance(psi, ux, uy, uz, ge, n);
                        gam = d >= 0.0f ? (d < tau ? d : tau) : (d > -tau ? d : -tau);
                        /* gradient: the weighted average of the normals, normalised */
                        const float sx = Wo * gs[0] + w * n[0], sy = Wo * gs[1] + w * n[1],
                                    sz = Wo * gs[2] + w * n[2];
                        const float l2 = (sx * sx + sy * sy) + sz * sz;
                        if (l2 > 0.0f && isfinite(l2)) {
                            const float l = sqrtf(l2);
                            G[li] = sx / l;
                            G[BLOCK_VOXELS + li] = sy / l;
                            G[2 * BLOCK_VOXELS + li] = sz / l;
                        }
                    } else {
                        gam = psi < tau ? psi : tau;
                    }
                    float num = Wo * Do + w * gam;
                    float den = Wo + w;
                    b->D[li] = num / den;
                    b->W[li] = den;
                    b->band[li] = fabsf(psi) <= tau;
                    updates++;
                }
    }
    /* dirty set: every touched block and its lower neighbours b - e, e in {0,1}^3 */
    for (int64_t i = 0; i < m->ntouched; ++i) {
        oblock *b = m->blocks[m->touched[i]];
        for (int e = 0; e < 8; ++e) {
            oblock *n = find_block(m, b->b[0] - (e & 1), b->b[1] - ((e >> 1) & 1), b->b[2] - ((e >> 2) & 1));
            if (n) n->dirty = 1;
        }
    }
    free(kept);
    free(nrm);
    lut_free(&t);
    m->has_scan = 1;
    m->st.touched = m->ntouched;
    m->st.new_blocks = n_new;
    m->st.updates = updates;
    m->st.votes = 0;
    m->st.allocated = m->nblocks;
    return OM_OK;
}

/* ------------------------------------------------------------------------------------ */
/* label fusion (Eq. 6 as vote counts) against the last scan                            */
/* ------------------------------------------------------------------------------------ */

/* One vote for label l at voxel li (Eq. 6 with hard labels): the count saturates at
 * 65535 and the most probable label moves to l when l's count passes the current one's,
 * or equals it with a lower id. */
static void vote(oblock *b, int li, int l)
{
    uint16_t *cnt = b->counts;
    unsigned c = cnt[(size_t)l * BLOCK_VOXELS + li];
    if (c < 65535u) c++;
    cnt[(size_t)l * BLOCK_VOXELS + li] = (uint16_t)c;
    int f = b->fused[li];
    unsigned cf = (f == 255) ? 0u : cnt[(size_t)f * BLOCK_VOXELS + li];
    if (l != f && (c > cf || (c == cf && l < f))) b->fused[li] = (uint8_t)l;
}

/* The label of a voxel's latest observation (the paper's Ours-wo-Bay, Sec. V-C). */
static void vote_latest(oblock *b, int li, int l) { b->fused[li] = (uint8_t)l; }

int om_set_label_fusion(omap *m, int mode)
{
    if (!m || mode < 0 || mode > 2) return OM_INVALID;
    m->label_mode = mode;
    if (mode == 2)
        for (int64_t i = 0; i < m->nblocks; ++i)
            if (!m->blocks[i]->LP) m->blocks[i]->LP = (float *)calloc((size_t)m->L * BLOCK_VOXELS, sizeof(float));
    return OM_OK;
}

/* Visible voxels of the last scan for a pinhole camera (readings of the label update):
 * band voxels with W > 0 in front of the camera, the pixel the floor of the projection.
 * Returns the pixel index or -1. */
static int64_t camera_pixel(const omap *m, const oblock *b, int li, int width, int height, float fx, float fy,
                            float cx, float cy, const float *T)
{
    if (!b->band[li] || !(b->W[li] > 0.0f)) return -1;
    const float nu = m->nu;
    int lx = li & 7, ly = (li >> 3) & 7, lz = li >> 6;
    float x = (float)(8 * b->b[0] + lx) * nu;
    float y = (float)(8 * b->b[1] + ly) * nu;
    float z = (float)(8 * b->b[2] + lz) * nu;
    float dx = x - T[3], dy = y - T[7], dz = z - T[11];
    float px = (T[0] * dx + T[4] * dy) + T[8] * dz;
    float py = (T[1] * dx + T[5] * dy) + T[9] * dz;
    float pz = (T[2] * dx + T[6] * dy) + T[10] * dz;
    if (!(pz > 0.0f)) return -1;
    float u = fx * (px / pz) + cx;
    float v = fy * (py / pz) + cy;
    if (!(u >= 0.0f && u < (float)width && v >= 0.0f && v < (float)height)) return -1;
    return (int64_t)(int)v * width + (int)u; /* floor of non-negative values */
}

/* Eq. 6 taken literally: the recursive Bayes update of each visible voxel's class
 * distribution by the camera's per-pixel class probabilities, given as log-probabilities
 * logp [height][width][L] (a segmentation network's log-softmax output).  In log space
 * the update is an addition per class; the normaliser Z of Eq. 6 is applied by
 * subtracting the largest log-posterior (so the most probable class holds 0 and the others
 * their log-ratio to it), which leaves the posterior's ratios, its argmax and every later
 * update as Z would, with no transcendental function.  The most probable label is the
 * argmax, ties to the lowest class id.  fp32, classes in increasing order. */
int om_integrate_logprobs(omap *m, int width, int height, float fx, float fy, float cx, float cy,
                          const float *logp, const float *T)
{
    if (!m || !logp || !T || width < 1 || height < 1) return OM_INVALID;
    if (!isfinite(fx) || !isfinite(fy) || !isfinite(cx) || !isfinite(cy) || fx == 0.0f || fy == 0.0f)
        return OM_INVALID;
    if (!check_pose(T) || m->label_mode != 2) return OM_INVALID;
    if (!m->has_scan) return OM_NO_SCAN;
    const int L = m->L;
    int64_t votes = 0;
#pragma omp parallel for reduction(+ : votes) schedule(dynamic, 4)
    for (int64_t i = 0; i < m->ntouched; ++i) {
        oblock *b = m->blocks[m->touched[i]];
        for (int li = 0; li < BLOCK_VOXELS; ++li) {
            const int64_t q = camera_pixel(m, b, li, width, height, fx, fy, cx, cy, T);
            if (q < 0) continue;
            const float *o = logp + (size_t)q * L;
            float mx = -INFINITY;
            for (int l = 0; l < L; ++l) {
                const float v = b->LP[(size_t)l * BLOCK_VOXELS + li] + o[l];
                b->LP[(size_t)l * BLOCK_VOXELS + li] = v;
                if (v > mx) mx = v;
            }
            int best = -1;
            for (int l = 0; l < L; ++l) {
                const float v = b->LP[(size_t)l * BLOCK_VOXELS + li] - mx;
                b->LP[(size_t)l * BLOCK_VOXELS + li] = v;
                if (best < 0 && v == 0.0f) best = l;
            }
            b->fused[li] = (uint8_t)best;
            votes++;
        }
    }
    m->st.votes += votes;
    return OM_OK;
}

int om_block_logpost(const omap *m, int bx, int by, int bz, float *LP)
{
    oblock *b = find_block(m, bx, by, bz);
    if (!b) return 0;
    if (b->LP) memcpy(LP, b->LP, (size_t)m->L * BLOCK_VOXELS * sizeof(float));
    else memset(LP, 0, (size_t)m->L * BLOCK_VOXELS * sizeof(float));
    return 1;
}

int om_integrate_labels(omap *m, int width, int height, float fx, float fy, float cx, float cy,
                        const uint8_t *labels, const float *T)
{
    if (!m || !labels || !T || width < 1 || height < 1) return OM_INVALID;
    if (!isfinite(fx) || !isfinite(fy) || !isfinite(cx) || !isfinite(cy) || fx == 0.0f || fy == 0.0f)
        return OM_INVALID;
    if (!check_pose(T) || m->label_mode == 2) return OM_INVALID;
    if (!m->has_scan) return OM_NO_SCAN;
    const float nu = m->nu;
    const float tx = T[3], ty = T[7], tz = T[11];
    const float fw = (float)width, fh = (float)height;
    const int latest = m->label_mode == 1;
    int64_t votes = 0;
#pragma omp parallel for reduction(+ : votes) schedule(dynamic, 4)
    for (int64_t i = 0; i < m->ntouched; ++i) {
        oblock *b = m->blocks[m->touched[i]];
        for (int li = 0; li < BLOCK_VOXELS; ++li) {
            if (!b->band[li] || !(b->W[li] > 0.0f)) continue;
            int lx = li & 7, ly = (li >> 3) & 7, lz = li >> 6;
            float x = (float)(8 * b->b[0] + lx) * nu;
            float y = (float)(8 * b->b[1] + ly) * nu;
            float z = (float)(8 * b->b[2] + lz) * nu;
            float dx = x - tx, dy = y - ty, dz = z - tz;
            float px = (T[0] * dx + T[4] * dy) + T[8] * dz;
            float py = (T[1] * dx + T[5] * dy) + T[9] * dz;
            float pz = (T[2] * dx + T[6] * dy) + T[10] * dz;
            if (!(pz > 0.0f)) continue;
            float u = fx * (px / pz) + cx;
            float v = fy * (py / pz) + cy;
            if (!(u >= 0.0f && u < fw && v >= 0.0f && v < fh)) continue;
            int iu = (int)u, iv = (int)v; /* floor of a non-negative value */
            int l = labels[(size_t)iv * width + iu];
            if (l >= m->L) continue;
            if (latest) vote_latest(b, li, l);
            else vote(b, li, l);
            votes++;
        }
    }
    m->st.votes += votes;
    return OM_OK;
}

/* Labels of the scan's points as a label range image (the semantic measurements of the
 * paper's LiDAR-segmentation experiments, Sec. V-A): each visible voxel of the last scan
 * takes the label at its nearest pixel of the scan model under pose T (the pixel rule of
 * the projective update) and votes as a camera label does. */
int om_integrate_labels_lidar(omap *m, int rows, int cols, const float *elev, const uint8_t *labels,
                              const float *T)
{
    if (!m || !labels || !T || !elev) return OM_INVALID;
    if (!check_pose(T) || m->label_mode == 2) return OM_INVALID;
    lut t;
    if (!lut_build(&t, rows, cols, elev)) return OM_INVALID;
    if (!m->has_scan) {
        lut_free(&t);
        return OM_NO_SCAN;
    }
    const float nu = m->nu;
    const float tx = T[3], ty = T[7], tz = T[11];
    int64_t votes = 0;
#pragma omp parallel for reduction(+ : votes) schedule(dynamic, 4)
    for (int64_t i = 0; i < m->ntouched; ++i) {
        oblock *b = m->blocks[m->touched[i]];
        for (int li = 0; li < BLOCK_VOXELS; ++li) {
            if (!b->band[li] || !(b->W[li] > 0.0f)) continue;
            int lx = li & 7, ly = (li >> 3) & 7, lz = li >> 6;
            float x = (float)(8 * b->b[0] + lx) * nu;
            float y = (float)(8 * b->b[1] + ly) * nu;
            float z = (float)(8 * b->b[2] + lz) * nu;
            float dx = x - tx, dy = y - ty, dz = z - tz;
            float px = (T[0] * dx + T[4] * dy) + T[8] * dz;
            float py = (T[1] * dx + T[5] * dy) + T[9] * dz;
            float pz = (T[2] * dx + T[6] * dy) + T[10] * dz;
            int row, col;
            if (!pixel_of(&t, px, py, pz, &row, &col)) continue;
            int l = labels[(size_t)row * cols + col];
            if (l >= m->L) continue;
            if (m->label_mode == 1) vote_latest(b, li, l);
            else vote(b, li, l);
            votes++;
        }
    }
    lut_free(&t);
    m->st.votes += votes;
    return OM_OK;
}

/* ------------------------------------------------------------------------------------ */
/* marching cubes, topology by rule (no table)                                          */
/* ------------------------------------------------------------------------------------ */
/* corner n has offset (n & 1, (n >> 1) & 1, (n >> 2) & 1).
 * edge e: axis e / 4; base corner offset with the two other coordinates taken from
 * j = e % 4 (lower other axis first): x-edges (0, j&1, j>>1), y-edges (j&1, 0, j>>1),
 * z-edges (j&1, j>>1, 0). */

static void edge_base(int e, int off[3])
{
    int ax = e / 4, j = e % 4;
    int o1 = j & 1, o2 = j >> 1;
    if (ax == 0) { off[0] = 0; off[1] = o1; off[2] = o2; }
    else if (ax == 1) { off[0] = o1; off[1] = 0; off[2] = o2; }
    else { off[0] = o1; off[1] = o2; off[2] = 0; }
}

static int corner_of(const int off[3]) { return off[0] + 2 * off[1] + 4 * off[2]; }

static int edge_of(int axis, const int base[3])
{
    if (axis == 0) return 0 + base[1] + 2 * base[2];
    if (axis == 1) return 4 + base[0] + 2 * base[2];
    return 8 + base[0] + 2 * base[1];
}

/* do two cube edges lie on a common face? (an edge lies on the two faces fixing its
 * non-axis coordinates at its base values) */
static int edges_share_face(int e1, int e2)
{
    int o1[3], o2[3];
    edge_base(e1, o1);
    edge_base(e2, o2);
    for (int a = 0; a < 3; ++a)
        if (a != e1 / 4 && a != e2 / 4 && o1[a] == o2[a]) return 1;
    return 0;
}

/* Triangles (edge-id triples) of one cube for the given inside mask; returns the count.
 * On each face the crossing points are joined; on a face whose inside corners sit on a
 * diagonal the inside corners are kept apart.  Each face segment is directed so that,
 * seen against the face's outward normal, the inside corner lies to its right; the
 * segments then link into cycles.  Each cycle is fanned from its smallest edge id whose
 * diagonals never join two edges of one face. */
static int cube_triangles(int inside_mask, int tris[][3])
{
    int next[12];
    for (int e = 0; e < 12; ++e) next[e] = -1;
    int crossing[12];
    for (int e = 0; e < 12; ++e) {
        int b[3];
        edge_base(e, b);
        int a = corner_of(b);
        b[e / 4] = 1;
        int c = corner_of(b);
        crossing[e] = ((inside_mask >> a) & 1) != ((inside_mask >> c) & 1);
    }
    for (int f = 0; f < 3; ++f)
        for (int s = 0; s < 2; ++s) {
            int g = (f + 1) % 3, h = (f + 2) % 3;
            int fe[4], nfe = 0; /* crossing edges on this face */
            int ins[4], nins = 0; /* inside corners on this face */
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    int off[3];
                    off[f] = s; off[g] = i; off[h] = j;
                    if ((inside_mask >> corner_of(off)) & 1) ins[nins++] = corner_of(off);
                }
            for (int i = 0; i < 2; ++i) {
                int base[3];
                base[f] = s; base[g] = 0; base[h] = i; /* edges along g */
                int e = edge_of(g, base);
                if (crossing[e]) fe[nfe++] = e;
                base[f] = s; base[g] = i; base[h] = 0; /* edges along h */
                e = edge_of(h, base);
                if (crossing[e]) fe[nfe++] = e;
            }
            if (nfe == 0) continue;
            int segs[2][3], nseg = 0; /* (edge A, edge B, inside corner) */
            if (nfe == 2) {
                segs[0][0] = fe[0]; segs[0][1] = fe[1]; segs[0][2] = ins[0];
                nseg = 1;
            } else { /* 4 crossings: two diagonal inside corners, each cut off alone */
                for (int q = 0; q < nins; ++q) {
                    int c = ins[q], off[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
                    int bg[3] = {off[0], off[1], off[2]}, bh[3] = {off[0], off[1], off[2]};
                    bg[g] = 0; bh[h] = 0;
                    segs[nseg][0] = edge_of(g, bg);
                    segs[nseg][1] = edge_of(h, bh);
                    segs[nseg][2] = c;
                    nseg++;
                }
            }
            for (int q = 0; q < nseg; ++q) {
                int A = segs[q][0], B = segs[q][1], c = segs[q][2];
                int pa[3], pb[3], pc[3] = {2 * (c & 1), 2 * ((c >> 1) & 1), 2 * ((c >> 2) & 1)};
                edge_base(A, pa); edge_base(B, pb);
                for (int k = 0; k < 3; ++k) { pa[k] *= 2; pb[k] *= 2; }
                pa[A / 4] += 1; pb[B / 4] += 1; /* doubled edge midpoints */
                int u[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
                int v[3] = {pc[0] - pa[0], pc[1] - pa[1], pc[2] - pa[2]};
                int cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
                int dn = cr[f] * (s ? 1 : -1);
                if (dn == 0) abort();
                if (dn < 0) { if (next[A] != -1) abort(); next[A] = B; }
                else { if (next[B] != -1) abort(); next[B] = A; }
            }
        }
    int ntri = 0, seen[12] = {0};
    for (int e = 0; e < 12; ++e) {
        if (!crossing[e] || seen[e]) continue;
        int cyc[12], n = 0, x = e;
        do {
            if (x < 0 || seen[x]) abort();
            seen[x] = 1;
            cyc[n++] = x;
            x = next[x];
        } while (x != e);
        /* apex: the smallest edge id none of whose fan diagonals joins two edges of one
         * cube face (such a diagonal could coincide with the neighbour cube's) */
        int apex = -1;
        for (int cand = 0; cand < 12 && apex < 0; ++cand) {
            int pos = -1;
            for (int i = 0; i < n; ++i)
                if (cyc[i] == cand) pos = i;
            if (pos < 0) continue;
            int good = 1;
            for (int j = 2; j + 1 < n && good; ++j)
                if (edges_share_face(cand, cyc[(pos + j) % n])) good = 0;
            if (good) apex = pos;
        }
        if (apex < 0) abort();
        for (int i = 1; i + 1 < n; ++i) {
            tris[ntri][0] = cyc[apex];
            tris[ntri][1] = cyc[(apex + i) % n];
            tris[ntri][2] = cyc[(apex + i + 1) % n];
            ntri++;
        }
    }
    return ntri;
}

static int64_t edge_key(const int64_t a[3], int axis)
{
    const int64_t off = 1 << 19;
    return ((a[0] + off) << 42) | ((a[1] + off) << 22) | ((a[2] + off) << 2) | axis;
}

/* The triangles of one block's 512 cubes (cube order z, y, x), written to pos, lab and
 * (if non-NULL) ekey while fewer than cap are written; returns the block's count. */
static int64_t mesh_block(const omap *m, const oblock *blk, int64_t cap, float *pos, uint8_t *lab, int64_t *ekey)
{
    const float nu = m->nu;
    int64_t ntri = 0;
    for (int lz = 0; lz < 8; ++lz)
        for (int ly = 0; ly < 8; ++ly)
            for (int lx = 0; lx < 8; ++lx) {
                int64_t base[3] = {8LL * blk->b[0] + lx, 8LL * blk->b[1] + ly, 8LL * blk->b[2] + lz};
                float Dc[8];
                uint8_t Fc[8];
                int ok = 1, mask = 0;
                for (int n = 0; n < 8 && ok; ++n) {
                    int64_t v[3] = {base[0] + (n & 1), base[1] + ((n >> 1) & 1), base[2] + ((n >> 2) & 1)};
                    int li;
                    oblock *cb = voxel_at(m, v, &li);
                    if (!cb || !(cb->W[li] > 0.0f)) { ok = 0; break; }
                    Dc[n] = cb->D[li];
                    Fc[n] = cb->fused[li];
                    if (Dc[n] < 0.0f) mask |= 1 << n;
                }
                if (!ok || mask == 0 || mask == 255) continue;
                int tris[12][3];
                int nt = cube_triangles(mask, tris);
                for (int q = 0; q < nt; ++q) {
                    if (ntri < cap) {
                        for (int k = 0; k < 3; ++k) {
                            int e = tris[q][k], off[3];
                            edge_base(e, off);
                            int ax = e / 4;
                            int ca = corner_of(off);
                            int ob[3] = {off[0], off[1], off[2]};
                            ob[ax] = 1;
                            int cb = corner_of(ob);
                            int64_t va[3] = {base[0] + off[0], base[1] + off[1], base[2] + off[2]};
                            float Da = Dc[ca], Db = Dc[cb];
                            float tt = Da / (Da - Db);
                            float *P = pos + 9 * ntri + 3 * k;
                            for (int j = 0; j < 3; ++j) P[j] = (float)va[j] * nu;
                            P[ax] = P[ax] + tt * nu;
                            lab[3 * ntri + k] = fabsf(Da) <= fabsf(Db) ? Fc[ca] : Fc[cb];
                            if (ekey) ekey[3 * ntri + k] = edge_key(va, ax);
                        }
                    }
                    ntri++;
                }
            }
    return ntri;
}

int om_extract_mesh(omap *m, int mode, int64_t cap_tris, float *pos, uint8_t *lab, int64_t *ekey,
                    int64_t *n_tris)
{
    if (!m || !n_tris || cap_tris < 0 || (mode != OM_MESH_DIRTY && mode != OM_MESH_ALL)) return OM_INVALID;
    if (cap_tris > 0 && (!pos || !lab)) return OM_INVALID;
    /* the blocks to mesh, in slot order */
    int64_t nsel = 0;
    int64_t *sel = (int64_t *)malloc((size_t)(m->nblocks > 0 ? m->nblocks : 1) * sizeof(int64_t));
    for (int64_t bi = 0; bi < m->nblocks; ++bi)
        if (mode == OM_MESH_ALL || m->blocks[bi]->dirty) sel[nsel++] = bi;
    /* Blocks are independent: each is meshed into buffers of its own (in parallel in the
     * OpenMP build), and the buffers are concatenated in slot order. */
    const int64_t kMaxBlockTris = 12 * BLOCK_VOXELS; /* at most 12 triangles a cube */
    int64_t *cnt = (int64_t *)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(int64_t));
    float **bpos = (float **)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(float *));
    uint8_t **blab = (uint8_t **)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(uint8_t *));
    int64_t **bkey = (int64_t **)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(int64_t *));
#pragma omp parallel
    {
        float *sp = (float *)malloc((size_t)kMaxBlockTris * 9 * sizeof(float));
        uint8_t *sl = (uint8_t *)malloc((size_t)kMaxBlockTris * 3);
        int64_t *sk = ekey ? (int64_t *)malloc((size_t)kMaxBlockTris * 3 * sizeof(int64_t)) : NULL;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < nsel; ++i) {
            int64_t n = mesh_block(m, m->blocks[sel[i]], kMaxBlockTris, sp, sl, sk);
            cnt[i] = n;
            if (n > 0 && cap_tris > 0) {
                bpos[i] = (float *)malloc((size_t)n * 9 * sizeof(float));
                blab[i] = (uint8_t *)malloc((size_t)n * 3);
                memcpy(bpos[i], sp, (size_t)n * 9 * sizeof(float));
                memcpy(blab[i], sl, (size_t)n * 3);
                if (sk) {
                    bkey[i] = (int64_t *)malloc((size_t)n * 3 * sizeof(int64_t));
                    memcpy(bkey[i], sk, (size_t)n * 3 * sizeof(int64_t));
                }
            }
        }
        free(sp);
        free(sl);
        free(sk);
    }
    int64_t ntri = 0;
    for (int64_t i = 0; i < nsel; ++i) {
        int64_t k = cnt[i];
        if (ntri < cap_tris && k > 0) {
            int64_t c = k < cap_tris - ntri ? k : cap_tris - ntri;
            memcpy(pos + 9 * ntri, bpos[i], (size_t)c * 9 * sizeof(float));
            memcpy(lab + 3 * ntri, blab[i], (size_t)c * 3);
            if (ekey) memcpy(ekey + 3 * ntri, bkey[i], (size_t)c * 3 * sizeof(int64_t));
        }
        ntri += k;
        free(bpos[i]);
        free(blab[i]);
        free(bkey[i]);
    }
    free(bpos);
    free(blab);
    free(bkey);
    free(cnt);
    free(sel);
    *n_tris = ntri;
    if (ntri > cap_tris) return OM_BUFFER;
    if (mode == OM_MESH_DIRTY)
        for (int64_t bi = 0; bi < m->nblocks; ++bi) m->blocks[bi]->dirty = 0;
    m->st.mesh_blocks = nsel;
    m->st.triangles = ntri;
    return OM_OK;
}

/* Threads the OpenMP build of this file uses (1 without OpenMP). */
int om_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* accessors                                                                            */
/* ------------------------------------------------------------------------------------ */

void om_get_stats(const omap *m, om_stats *s) { *s = m->st; }
int64_t om_num_blocks(const omap *m) { return m->nblocks; }

void om_block_coords(const omap *m, int32_t *out)
{
    for (int64_t i = 0; i < m->nblocks; ++i)
        for (int a = 0; a < 3; ++a) out[3 * i + a] = m->blocks[i]->b[a];
}

int64_t om_touched(const omap *m, int32_t *out, int64_t cap)
{
    for (int64_t i = 0; i < m->ntouched && i < cap; ++i)
        for (int a = 0; a < 3; ++a) out[3 * i + a] = m->blocks[m->touched[i]]->b[a];
    return m->ntouched;
}

int om_block_data(const omap *m, int bx, int by, int bz, float *D, float *W, uint8_t *fused,
                  uint16_t *counts, uint8_t *band)
{
    oblock *b = find_block(m, bx, by, bz);
    if (!b) return 0;
    if (D) memcpy(D, b->D, sizeof(b->D));
    if (W) memcpy(W, b->W, sizeof(b->W));
    if (fused) memcpy(fused, b->fused, sizeof(b->fused));
    if (counts) memcpy(counts, b->counts, (size_t)m->L * BLOCK_VOXELS * sizeof(uint16_t));
    if (band) memcpy(band, b->band, sizeof(b->band));
    return 1;
}

/* ------------------------------------------------------------------------------------ */
/* trilinear SDF query and its pose adjoint (fp64)                                      */
/* ------------------------------------------------------------------------------------ */

/* corner values of the cell with lower corner v0; 0 if any corner is unobserved */
static int cell_values(const omap *m, const int64_t v0[3], double Dc[8])
{
    for (int n = 0; n < 8; ++n) {
        int64_t v[3] = {v0[0] + (n & 1), v0[1] + ((n >> 1) & 1), v0[2] + ((n >> 2) & 1)};
        int li;
        oblock *b = voxel_at(m, v, &li);
        if (!b || !(b->W[li] > 0.0f)) return 0;
        Dc[n] = (double)b->D[li];
    }
    return 1;
}

/* trilinear value and derivative w.r.t. the cell fraction f (lerp along x, then y, then z) */
static double trilinear(const double Dc[8], const double f[3], double dDdf[3])
{
    double fx = f[0], fy = f[1], fz = f[2];
    double c00 = Dc[0] + fx * (Dc[1] - Dc[0]), c10 = Dc[2] + fx * (Dc[3] - Dc[2]);
    double c01 = Dc[4] + fx * (Dc[5] - Dc[4]), c11 = Dc[6] + fx * (Dc[7] - Dc[6]);
    double c0 = c00 + fy * (c10 - c00), c1 = c01 + fy * (c11 - c01);
    double val = c0 + fz * (c1 - c0);
    if (dDdf) {
        double gx00 = Dc[1] - Dc[0], gx10 = Dc[3] - Dc[2], gx01 = Dc[5] - Dc[4], gx11 = Dc[7] - Dc[6];
        double gx0 = gx00 + fy * (gx10 - gx00), gx1 = gx01 + fy * (gx11 - gx01);
        dDdf[0] = gx0 + fz * (gx1 - gx0);
        dDdf[1] = (c10 - c00) + fz * ((c11 - c01) - (c10 - c00));
        dDdf[2] = c1 - c0;
    }
    return val;
}

static int query_one(const omap *m, const double x[3], int mode, double *sdf, double grad[3],
                     double *margin)
{
    double f[3];
    int64_t v0[3];
    double lim = (double)DOMAIN_VOXELS;
    for (int a = 0; a < 3; ++a) {
        double q;
        if (mode == 1) {
            float q32 = (float)x[a] / m->nu;
            q = (double)q32;
        } else {
            q = x[a] / (double)m->nu;
        }
        if (!(fabs(q) < lim)) return 0;
        double fl = floor(q);
        v0[a] = (int64_t)fl;
        f[a] = q - fl;
    }
    if (margin) {
        double mg = 1.0;
        for (int a = 0; a < 3; ++a) {
            double d = f[a] < 1.0 - f[a] ? f[a] : 1.0 - f[a];
            if (d < mg) mg = d;
        }
        *margin = mg;
    }
    double Dc[8], dDdf[3];
    if (!cell_values(m, v0, Dc)) return 0;
    *sdf = trilinear(Dc, f, dDdf);
    if (grad)
        for (int a = 0; a < 3; ++a) grad[a] = dDdf[a] / (double)m->nu;
    return 1;
}

void om_query_sdf(const omap *m, const double *pts, int64_t n, double *sdf, double *grad,
                  uint8_t *valid, int mode)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0, g[3] = {0, 0, 0};
        int ok = query_one(m, pts + 3 * i, mode, &s, g, NULL);
        if (!ok) { s = 0.0; g[0] = g[1] = g[2] = 0.0; }
        sdf[i] = s;
        if (grad) for (int a = 0; a < 3; ++a) grad[3 * i + a] = g[a];
        valid[i] = (uint8_t)ok;
    }
}

/* SO(3) exponential and left Jacobian, closed forms with series near zero */
static void so3_exp_jl(const double w[3], double R[9], double J[9])
{
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = sqrt(th2);
    double A, B, C; /* sin t / t, (1 - cos t) / t^2, (t - sin t) / t^3 */
    if (th < 0.1) {
        double t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        A = 1.0 - th2 / 6.0 + t4 / 120.0 - t6 / 5040.0 + t8 / 362880.0;
        B = 0.5 - th2 / 24.0 + t4 / 720.0 - t6 / 40320.0 + t8 / 3628800.0;
        C = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0 - t6 / 362880.0 + t8 / 39916800.0;
    } else {
        double sh = sin(0.5 * th);
        A = sin(th) / th;
        B = 2.0 * sh * sh / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += K[3 * i + k] * K[3 * k + j];
            K2[3 * i + j] = s;
        }
    for (int i = 0; i < 9; ++i) {
        double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * K[i] + B * K2[i];
        J[i] = I + B * K[i] + C * K2[i];
    }
}

void om_pose_adjoint(const omap *m, const double *xi, const float *pts, int B, int64_t N,
                     double *loss, double *gxi, double *gpts, double *margin)
{
    for (int b = 0; b < B; ++b) {
        const double *t = xi + 6 * b, *w = xi + 6 * b + 3;
        double R[9], J[9];
        so3_exp_jl(w, R, J);
        double L = 0.0, gt[3] = {0, 0, 0}, m3[3] = {0, 0, 0};
        for (int64_t j = 0; j < N; ++j) {
            const float *p = pts + 3 * ((size_t)b * N + j);
            double pd[3] = {p[0], p[1], p[2]};
            double Rp[3], y[3];
            for (int i = 0; i < 3; ++i) {
                Rp[i] = R[3 * i] * pd[0] + R[3 * i + 1] * pd[1] + R[3 * i + 2] * pd[2];
                y[i] = Rp[i] + t[i];
            }
            double s, g[3], mg = 0.0;
            int ok = query_one(m, y, 0, &s, g, &mg);
            if (margin) margin[(size_t)b * N + j] = mg;
            double gp[3] = {0, 0, 0};
            if (ok) {
                L += s * s;
                double gg[3] = {2.0 * s * g[0], 2.0 * s * g[1], 2.0 * s * g[2]};
                for (int i = 0; i < 3; ++i) gt[i] += gg[i];
                m3[0] += Rp[1] * gg[2] - Rp[2] * gg[1];
                m3[1] += Rp[2] * gg[0] - Rp[0] * gg[2];
                m3[2] += Rp[0] * gg[1] - Rp[1] * gg[0];
                for (int i = 0; i < 3; ++i) gp[i] = R[i] * gg[0] + R[3 + i] * gg[1] + R[6 + i] * gg[2];
            }
            if (gpts)
                for (int i = 0; i < 3; ++i) gpts[3 * ((size_t)b * N + j) + i] = gp[i];
        }
        loss[b] = L;
        for (int i = 0; i < 3; ++i) {
            gxi[6 * b + i] = gt[i];
            gxi[6 * b + 3 + i] = J[i] * m3[0] + J[3 + i] * m3[1] + J[6 + i] * m3[2];
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* test hooks                                                                           */
/* ------------------------------------------------------------------------------------ */

int om_set_block(omap *m, int bx, int by, int bz, const float *D, const float *W, const uint8_t *fused)
{
    oblock *b = find_block(m, bx, by, bz);
    if (!b) {
        if (m->nblocks >= m->max_blocks) return 0;
        b = new_block(m, bx, by, bz);
    }
    if (D) memcpy(b->D, D, sizeof(b->D));
    if (W) memcpy(b->W, W, sizeof(b->W));
    if (fused) memcpy(b->fused, fused, sizeof(b->fused));
    for (int e = 0; e < 8; ++e) {
        oblock *n = find_block(m, bx - (e & 1), by - ((e >> 1) & 1), bz - ((e >> 2) & 1));
        if (n) n->dirty = 1;
    }
    m->st.allocated = m->nblocks;
    return 1;
}

int om_cube_triangles(int inside_mask, int *out)
{
    int tris[12][3];
    int n = cube_triangles(inside_mask & 255, tris);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) out[3 * i + k] = tris[i][k];
    return n;
}
