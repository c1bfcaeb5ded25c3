/*
 * Seeded synthetic-scene ray caster.
 *
 * Test and benchmark input generator only: it intersects rays with primitive
 * shapes (axis-aligned boxes, vertical cylinders and cones, spheres, a ground
 * plane or a triangulated heightfield) and returns the first hit distance and
 * the class id of the object hit.  It holds none of the mapping method's
 * arithmetic; the oracle and the GPU library both consume what it produces.
 *
 * All geometry is in double precision.  An xy uniform grid accelerates the
 * object tests; the ground is intersected analytically (plane) or by a 2-D
 * walk over the lattice cells (heightfield).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OBJ_BOX = 0, OBJ_CYL = 1, OBJ_CONE = 2, OBJ_SPHERE = 3 };

typedef struct {
    int type;
    int cls;
    double a[6];
    double xmin, ymin, xmax, ymax; /* xy footprint bound */
} sobj;

typedef struct {
    int nobj;
    sobj *obj;
    /* ground */
    int ground_kind; /* 0 none, 1 plane, 2 heightfield */
    double ground_z;
    int n_bands;
    double band_y[16];
    int band_cls[16];
    int ground_default_cls;
    /* heightfield: z at lattice node (i, j) = hf_z[j * hf_nx + i], node (x0 + i h, y0 + j h) */
    double hf_x0, hf_y0, hf_h;
    int hf_nx, hf_ny;
    float *hf_z;
    double hf_zmax; /* highest lattice node: a ray above it and not descending hits no cell */
    /* grid */
    double gx0, gy0, gcell;
    int gnx, gny;
    int *cell_start; /* gnx*gny+1 */
    int *cell_items;
} scene;

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

void *synth_scene_new(int nobj, const int *types, const int *cls, const double *params,
                      int ground_kind, double ground_z, int n_bands, const double *band_y,
                      const int *band_cls, int ground_default_cls, double cell)
{
    scene *s = (scene *)calloc(1, sizeof(scene));
    s->nobj = nobj;
    s->obj = (sobj *)calloc(nobj > 0 ? nobj : 1, sizeof(sobj));
    double bx0 = 1e300, by0 = 1e300, bx1 = -1e300, by1 = -1e300;
    for (int i = 0; i < nobj; ++i) {
        sobj *o = &s->obj[i];
        o->type = types[i];
        o->cls = cls[i];
        memcpy(o->a, params + 6 * i, 6 * sizeof(double));
        switch (o->type) {
        case OBJ_BOX:
            o->xmin = o->a[0]; o->ymin = o->a[1]; o->xmax = o->a[3]; o->ymax = o->a[4];
            break;
        case OBJ_CYL:
        case OBJ_CONE:
            o->xmin = o->a[0] - o->a[2]; o->xmax = o->a[0] + o->a[2];
            o->ymin = o->a[1] - o->a[2]; o->ymax = o->a[1] + o->a[2];
            break;
        default: /* sphere */
            o->xmin = o->a[0] - o->a[3]; o->xmax = o->a[0] + o->a[3];
            o->ymin = o->a[1] - o->a[3]; o->ymax = o->a[1] + o->a[3];
            break;
        }
        bx0 = dmin(bx0, o->xmin); by0 = dmin(by0, o->ymin);
        bx1 = dmax(bx1, o->xmax); by1 = dmax(by1, o->ymax);
    }
    s->ground_kind = ground_kind;
    s->ground_z = ground_z;
    s->n_bands = n_bands > 16 ? 16 : n_bands;
    for (int i = 0; i < s->n_bands; ++i) {
        s->band_y[i] = band_y[i];
        s->band_cls[i] = band_cls[i];
    }
    s->ground_default_cls = ground_default_cls;

    if (nobj == 0) { bx0 = by0 = 0; bx1 = by1 = 1; }
    s->gcell = cell;
    s->gx0 = bx0 - 1e-6;
    s->gy0 = by0 - 1e-6;
    s->gnx = (int)ceil((bx1 - s->gx0) / cell) + 1;
    s->gny = (int)ceil((by1 - s->gy0) / cell) + 1;
    int ncell = s->gnx * s->gny;
    int *cnt = (int *)calloc(ncell + 1, sizeof(int));
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            int acc = 0;
            for (int c = 0; c < ncell; ++c) { int t = cnt[c]; cnt[c] = acc; acc += t; }
            cnt[ncell] = acc;
            s->cell_start = (int *)malloc((ncell + 1) * sizeof(int));
            memcpy(s->cell_start, cnt, (ncell + 1) * sizeof(int));
            s->cell_items = (int *)malloc((acc > 0 ? acc : 1) * sizeof(int));
        }
        for (int i = 0; i < nobj; ++i) {
            sobj *o = &s->obj[i];
            int i0 = (int)floor((o->xmin - s->gx0) / cell), i1 = (int)floor((o->xmax - s->gx0) / cell);
            int j0 = (int)floor((o->ymin - s->gy0) / cell), j1 = (int)floor((o->ymax - s->gy0) / cell);
            for (int j = j0; j <= j1; ++j)
                for (int ii = i0; ii <= i1; ++ii) {
                    int c = j * s->gnx + ii;
                    if (pass == 0) cnt[c]++;
                    else s->cell_items[cnt[c]++] = i;
                }
        }
    }
    free(cnt);
    return s;
}

void synth_scene_set_heightfield(void *sp, double x0, double y0, double h, int nx, int ny,
                                 const float *z)
{
    scene *s = (scene *)sp;
    s->hf_x0 = x0; s->hf_y0 = y0; s->hf_h = h; s->hf_nx = nx; s->hf_ny = ny;
    free(s->hf_z);
    s->hf_z = (float *)malloc((size_t)nx * ny * sizeof(float));
    memcpy(s->hf_z, z, (size_t)nx * ny * sizeof(float));
    s->hf_zmax = -INFINITY;
    for (size_t q = 0; q < (size_t)nx * ny; ++q) s->hf_zmax = dmax(s->hf_zmax, (double)z[q]);
    s->ground_kind = 2;
}

void synth_scene_free(void *sp)
{
    scene *s = (scene *)sp;
    if (!s) return;
    free(s->obj); free(s->cell_start); free(s->cell_items); free(s->hf_z);
    free(s);
}

/* smallest root of a t^2 + b t + c = 0 that is > tmin, or INFINITY; both roots returned */
static int quad_roots(double a, double b, double c, double *t0, double *t1)
{
    if (fabs(a) < 1e-300) {
        if (fabs(b) < 1e-300) return 0;
        *t0 = *t1 = -c / b;
        return 1;
    }
    double disc = b * b - 4 * a * c;
    if (disc < 0) return 0;
    double sq = sqrt(disc);
    double q = -0.5 * (b + (b >= 0 ? sq : -sq));
    double r0 = q / a, r1 = (q != 0) ? c / q : r0;
    if (r0 > r1) { double t = r0; r0 = r1; r1 = t; }
    *t0 = r0; *t1 = r1;
    return 2;
}

static const double TEPS = 1e-9;

static double hit_box(const sobj *o, const double *p, const double *d)
{
    double tn = -1e300, tf = 1e300;
    for (int k = 0; k < 3; ++k) {
        double lo = o->a[k], hi = o->a[3 + k];
        if (d[k] == 0.0) {
            if (p[k] < lo || p[k] > hi) return INFINITY;
        } else {
            double t0 = (lo - p[k]) / d[k], t1 = (hi - p[k]) / d[k];
            if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
            tn = dmax(tn, t0); tf = dmin(tf, t1);
        }
    }
    if (tn > tf) return INFINITY;
    if (tn > TEPS) return tn;
    if (tf > TEPS) return tf; /* origin inside: interior wall */
    return INFINITY;
}

static double hit_cyl(const sobj *o, const double *p, const double *d)
{
    double cx = o->a[0], cy = o->a[1], r = o->a[2], z0 = o->a[3], z1 = o->a[4];
    double best = INFINITY;
    double ox = p[0] - cx, oy = p[1] - cy;
    double a = d[0] * d[0] + d[1] * d[1], b = 2 * (ox * d[0] + oy * d[1]), c = ox * ox + oy * oy - r * r;
    double t0, t1;
    if (a > 0 && quad_roots(a, b, c, &t0, &t1)) {
        double ts[2] = {t0, t1};
        for (int i = 0; i < 2; ++i) {
            double t = ts[i];
            if (t > TEPS && t < best) {
                double z = p[2] + t * d[2];
                if (z >= z0 && z <= z1) best = t;
            }
        }
    }
    if (d[2] != 0.0) {
        double zc[2] = {z0, z1};
        for (int i = 0; i < 2; ++i) {
            double t = (zc[i] - p[2]) / d[2];
            if (t > TEPS && t < best) {
                double x = ox + t * d[0], y = oy + t * d[1];
                if (x * x + y * y <= r * r) best = t;
            }
        }
    }
    return best;
}

static double hit_cone(const sobj *o, const double *p, const double *d)
{
    /* base radius rb at z0, apex at z1 (z1 > z0) */
    double cx = o->a[0], cy = o->a[1], rb = o->a[2], z0 = o->a[3], z1 = o->a[4];
    double k = rb / (z1 - z0);
    double best = INFINITY;
    double ox = p[0] - cx, oy = p[1] - cy, oz = z1 - p[2];
    /* x^2 + y^2 = k^2 (z1 - z)^2, with z1 - z = oz - t dz */
    double k2 = k * k;
    double a = d[0] * d[0] + d[1] * d[1] - k2 * d[2] * d[2];
    double b = 2 * (ox * d[0] + oy * d[1]) + 2 * k2 * oz * d[2];
    double c = ox * ox + oy * oy - k2 * oz * oz;
    double t0, t1;
    int n = quad_roots(a, b, c, &t0, &t1);
    if (n) {
        double ts[2] = {t0, t1};
        for (int i = 0; i < 2; ++i) {
            double t = ts[i];
            if (t > TEPS && t < best) {
                double z = p[2] + t * d[2];
                if (z >= z0 && z <= z1) best = t;
            }
        }
    }
    if (d[2] != 0.0) {
        double t = (z0 - p[2]) / d[2];
        if (t > TEPS && t < best) {
            double x = ox + t * d[0], y = oy + t * d[1];
            if (x * x + y * y <= rb * rb) best = t;
        }
    }
    return best;
}

static double hit_sphere(const sobj *o, const double *p, const double *d)
{
    double ox = p[0] - o->a[0], oy = p[1] - o->a[1], oz = p[2] - o->a[2], r = o->a[3];
    double a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double b = 2 * (ox * d[0] + oy * d[1] + oz * d[2]);
    double c = ox * ox + oy * oy + oz * oz - r * r;
    double t0, t1;
    if (!quad_roots(a, b, c, &t0, &t1)) return INFINITY;
    if (t0 > TEPS) return t0;
    if (t1 > TEPS) return t1;
    return INFINITY;
}

static double hit_obj(const sobj *o, const double *p, const double *d)
{
    switch (o->type) {
    case OBJ_BOX: return hit_box(o, p, d);
    case OBJ_CYL: return hit_cyl(o, p, d);
    case OBJ_CONE: return hit_cone(o, p, d);
    default: return hit_sphere(o, p, d);
    }
}

static int ground_class(const scene *s, double y)
{
    double ay = fabs(y);
    for (int i = 0; i < s->n_bands; ++i)
        if (ay < s->band_y[i]) return s->band_cls[i];
    return s->ground_default_cls;
}

/* ray vs triangle (Moller-Trumbore), returns t or INFINITY */
static double hit_tri(const double *p, const double *d, const double *v0, const double *v1,
                      const double *v2)
{
    double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    double h[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    double a = e1[0] * h[0] + e1[1] * h[1] + e1[2] * h[2];
    if (fabs(a) < 1e-300) return INFINITY;
    double f = 1.0 / a;
    double sv[3] = {p[0] - v0[0], p[1] - v0[1], p[2] - v0[2]};
    double u = f * (sv[0] * h[0] + sv[1] * h[1] + sv[2] * h[2]);
    if (u < 0.0 || u > 1.0) return INFINITY;
    double q[3] = {sv[1] * e1[2] - sv[2] * e1[1], sv[2] * e1[0] - sv[0] * e1[2], sv[0] * e1[1] - sv[1] * e1[0]};
    double v = f * (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]);
    if (v < 0.0 || u + v > 1.0) return INFINITY;
    double t = f * (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]);
    return t > TEPS ? t : INFINITY;
}

static double hf_node(const scene *s, int i, int j, double *v)
{
    v[0] = s->hf_x0 + i * s->hf_h;
    v[1] = s->hf_y0 + j * s->hf_h;
    v[2] = s->hf_z[(size_t)j * s->hf_nx + i];
    return v[2];
}

static double hit_cell_tris(const scene *s, int i, int j, const double *p, const double *d)
{
    if (i < 0 || j < 0 || i >= s->hf_nx - 1 || j >= s->hf_ny - 1) return INFINITY;
    double a[3], b[3], c[3], e[3];
    hf_node(s, i, j, a); hf_node(s, i + 1, j, b); hf_node(s, i + 1, j + 1, c); hf_node(s, i, j + 1, e);
    double t0 = hit_tri(p, d, a, b, c), t1 = hit_tri(p, d, a, c, e);
    return dmin(t0, t1);
}

/* 2-D DDA over heightfield cells along the ray's xy projection, t in [0, tmax] */
static double hit_heightfield(const scene *s, const double *p, const double *d, double tmax)
{
    double h = s->hf_h;
    double gx = (p[0] - s->hf_x0) / h, gy = (p[1] - s->hf_y0) / h;
    int i = (int)floor(gx), j = (int)floor(gy);
    int si = d[0] > 0 ? 1 : -1, sj = d[1] > 0 ? 1 : -1;
    double tdx = d[0] != 0 ? fabs(h / d[0]) : INFINITY, tdy = d[1] != 0 ? fabs(h / d[1]) : INFINITY;
    double tx = d[0] != 0 ? ((si > 0 ? (i + 1 - gx) : (gx - i)) * h) / fabs(d[0]) : INFINITY;
    double ty = d[1] != 0 ? ((sj > 0 ? (j + 1 - gy) : (gy - j)) * h) / fabs(d[1]) : INFINITY;
    double t = 0;
    for (int it = 0; it < 1000000 && t <= tmax; ++it) {
        /* the triangles lie at or below hf_zmax; a ray that is above it at t and not
           descending stays above it, so it hits no further cell */
        if (d[2] >= 0.0 && p[2] + t * d[2] > s->hf_zmax) break;
        double th = hit_cell_tris(s, i, j, p, d);
        double texit = dmin(tx, ty);
        if (th <= texit + 1e-9) return th;
        if (tx < ty) { t = tx; tx += tdx; i += si; } else { t = ty; ty += tdy; j += sj; }
        if ((i < -1 && si < 0) || (j < -1 && sj < 0) || (i > s->hf_nx && si > 0) || (j > s->hf_ny && sj > 0))
            break;
    }
    return INFINITY;
}

static void cast_one(const scene *s, const double *p, const double *d, double tmax, double *t_out,
                     uint8_t *c_out)
{
    double best = INFINITY;
    int bcls = 255;
    /* ground */
    if (s->ground_kind == 1 && d[2] != 0.0) {
        double t = (s->ground_z - p[2]) / d[2];
        if (t > TEPS && t < best) { best = t; bcls = ground_class(s, p[1] + t * d[1]); }
    } else if (s->ground_kind == 2) {
        double t = hit_heightfield(s, p, d, dmin(tmax, best));
        if (t < best) { best = t; bcls = ground_class(s, p[1] + t * d[1]); }
    }
    /* objects: 2-D grid walk */
    if (s->nobj > 0) {
        double cell = s->gcell;
        double gx = (p[0] - s->gx0) / cell, gy = (p[1] - s->gy0) / cell;
        /* enter the grid */
        double tent = 0.0, texit_grid = INFINITY;
        {
            double lo[2] = {0, 0}, hi[2] = {(double)s->gnx, (double)s->gny}, g[2] = {gx, gy};
            double dd[2] = {d[0] / cell, d[1] / cell};
            for (int k = 0; k < 2; ++k) {
                if (dd[k] == 0.0) {
                    if (g[k] < lo[k] || g[k] >= hi[k]) { tent = INFINITY; break; }
                } else {
                    double t0 = (lo[k] - g[k]) / dd[k], t1 = (hi[k] - g[k]) / dd[k];
                    if (t0 > t1) { double tt = t0; t0 = t1; t1 = tt; }
                    tent = dmax(tent, t0); texit_grid = dmin(texit_grid, t1);
                }
            }
        }
        if (tent < texit_grid && tent <= dmin(tmax, best)) {
            double ex = gx + tent * d[0] / cell, ey = gy + tent * d[1] / cell;
            int i = (int)floor(ex), j = (int)floor(ey);
            if (i < 0) i = 0;
            if (j < 0) j = 0;
            if (i >= s->gnx) i = s->gnx - 1;
            if (j >= s->gny) j = s->gny - 1;
            int si = d[0] > 0 ? 1 : -1, sj = d[1] > 0 ? 1 : -1;
            double tdx = d[0] != 0 ? fabs(cell / d[0]) : INFINITY;
            double tdy = d[1] != 0 ? fabs(cell / d[1]) : INFINITY;
            double tx = d[0] != 0 ? ((si > 0 ? (i + 1 - gx) : (gx - i)) * cell) / fabs(d[0]) : INFINITY;
            double ty = d[1] != 0 ? ((sj > 0 ? (j + 1 - gy) : (gy - j)) * cell) / fabs(d[1]) : INFINITY;
            while (i >= 0 && j >= 0 && i < s->gnx && j < s->gny) {
                int c = j * s->gnx + i;
                for (int q = s->cell_start[c]; q < s->cell_start[c + 1]; ++q) {
                    const sobj *o = &s->obj[s->cell_items[q]];
                    double t = hit_obj(o, p, d);
                    if (t < best) { best = t; bcls = o->cls; }
                }
                double tcell_exit = dmin(tx, ty);
                if (best <= tcell_exit || tcell_exit > tmax) break;
                if (tx < ty) { tx += tdx; i += si; } else { ty += tdy; j += sj; }
            }
        }
    }
    if (best <= tmax) { *t_out = best; *c_out = (uint8_t)bcls; }
    else { *t_out = INFINITY; *c_out = 255; }
}

/* Cast n rays from one origin; dirs is n x 3 (need not be unit; t is in units of |d|). */
void synth_cast(const void *sp, int64_t n, const double *origin, const double *dirs, double tmax,
                double *t_out, uint8_t *cls_out)
{
    const scene *s = (const scene *)sp;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < n; ++r)
        cast_one(s, origin, dirs + 3 * r, tmax, t_out + r, cls_out + r);
}
