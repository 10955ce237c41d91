/*
 * FP64 brute-force closest-hit ray casting for the oracle (test infrastructure only).
 *
 * Sec. III-B renders depth, colour and segmentation views of triangle-mesh
 * scenes.  The oracle computes the defined result directly: every ray is tested
 * against every triangle with the Moller-Trumbore test (Moller & Trumbore 1997)
 * in IEEE double precision, no epsilon, closed triangles (u >= 0, v >= 0,
 * u + v <= 1), double-sided, det == 0 counted as a miss, and a hit accepted only
 * for near <= t <= far.  The closest hit is the minimum t; equal t goes to the
 * lower triangle index.
 *
 * Per ray it also reports the data that define the comparison mask:
 *   t2          second-smallest hit distance (INFINITY if fewer than two hits)
 *   edge_hit    lower bound on the 3-D distance from the ray to the boundary of
 *               the hit triangle, near the hit point: in-plane distance to the
 *               nearest edge line times |n.d|/|d|
 *   near_miss   lower bound on the 3-D distance from the ray to any triangle the
 *               ray misses while crossing its plane at near <= t <= t1*(1+1e-6)
 *               (or far): max over violated edge lines of the in-plane distance,
 *               times |n.d|/|d|
 *   boundary    1 if any triangle is hit inside its face at t within a relative
 *               1e-6 outside or inside [near, far]
 *
 * Compiled with -O2 -ffp-contract=off: no fused multiply-add, no reassociation.
 * One OpenMP loop over rays; the per-ray work is a plain loop over triangles.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double t, u, v;
    int hit;      /* inside the closed triangle */
    int valid;    /* det != 0 */
    double det;
} mt_result;

static void sub3(const double* a, const double* b, double* o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

static mt_result moller_trumbore(const double* o, const double* d, const double* v0, const double* v1, const double* v2) {
    mt_result r = {0.0, 0.0, 0.0, 0, 0, 0.0};
    double e1[3], e2[3], p[3], s[3], q[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    cross3(d, e2, p);
    double det = dot3(e1, p);
    r.det = det;
    if (det == 0.0) return r;
    r.valid = 1;
    sub3(o, v0, s);
    r.u = dot3(s, p) / det;
    cross3(s, e1, q);
    r.v = dot3(d, q) / det;
    r.t = dot3(e2, q) / det;
    r.hit = (r.u >= 0.0) && (r.v >= 0.0) && (r.u + r.v <= 1.0);
    return r;
}

/* in-plane heights h_k (distance from vertex k to the opposite edge line) and |n.d|/|d| */
static void tri_geometry(const double* d, const double* v0, const double* v1, const double* v2,
                         double det, double* h, double* cosang) {
    double e1[3], e2[3], e12[3], n[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    sub3(v2, v1, e12);
    cross3(e1, e2, n);
    double twice_area = norm3(n);
    h[0] = twice_area / norm3(e12);
    h[1] = twice_area / norm3(e2);
    h[2] = twice_area / norm3(e1);
    *cosang = fabs(det) / (twice_area * norm3(d));
}

void oracle_cast(int64_t n_rays, const double* orig, const double* dir,
                 int64_t n_tris, const double* v0, const double* v1, const double* v2,
                 double near_t, double far_t, int32_t with_mask,
                 double* t_out, int64_t* id_out, double* t2_out,
                 double* edge_hit_out, double* near_miss_out, int32_t* boundary_out,
                 int32_t* threads_used) {
    int nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        nthreads = omp_get_num_threads();
    }
#endif
    *threads_used = nthreads;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n_rays; ++r) {
        const double* o = orig + 3 * r;
        const double* d = dir + 3 * r;
        double t1 = INFINITY, t2 = INFINITY, u1 = 0.0, w1 = 0.0;
        int64_t id1 = -1;
        int boundary = 0;
        for (int64_t k = 0; k < n_tris; ++k) {
            mt_result m = moller_trumbore(o, d, v0 + 3 * k, v1 + 3 * k, v2 + 3 * k);
            if (!m.valid || !m.hit) continue;
            if (with_mask) {
                double lo = near_t * (1.0 - 1e-6), hi = near_t * (1.0 + 1e-6);
                double flo = far_t * (1.0 - 1e-6), fhi = far_t * (1.0 + 1e-6);
                if ((m.t >= lo && m.t <= hi) || (m.t >= flo && m.t <= fhi)) boundary = 1;
            }
            if (m.t < near_t || m.t > far_t) continue;
            if (m.t < t1 || (m.t == t1 && k < id1)) {
                t2 = t1;
                t1 = m.t;
                id1 = k;
                u1 = m.u;
                w1 = m.v;
            } else if (m.t < t2) {
                t2 = m.t;
            }
        }
        t_out[r] = t1;
        id_out[r] = id1;
        if (!with_mask) continue;
        t2_out[r] = t2;
        boundary_out[r] = boundary;
        double edge_hit = INFINITY;
        if (id1 >= 0) {
            double h[3], cosang;
            mt_result m = moller_trumbore(o, d, v0 + 3 * id1, v1 + 3 * id1, v2 + 3 * id1);
            tri_geometry(d, v0 + 3 * id1, v1 + 3 * id1, v2 + 3 * id1, m.det, h, &cosang);
            double b[3] = {1.0 - u1 - w1, u1, w1};
            double dmin = INFINITY;
            for (int e = 0; e < 3; ++e) {
                double de = b[e] * h[e];
                if (de < dmin) dmin = de;
            }
            edge_hit = dmin * cosang;
        }
        edge_hit_out[r] = edge_hit;
        double limit = (id1 >= 0) ? t1 * (1.0 + 1e-6) : far_t;
        double near_miss = INFINITY;
        for (int64_t k = 0; k < n_tris; ++k) {
            mt_result m = moller_trumbore(o, d, v0 + 3 * k, v1 + 3 * k, v2 + 3 * k);
            if (!m.valid || m.hit) continue;
            if (m.t < near_t || m.t > limit) continue;
            double h[3], cosang;
            tri_geometry(d, v0 + 3 * k, v1 + 3 * k, v2 + 3 * k, m.det, h, &cosang);
            double b[3] = {1.0 - m.u - m.v, m.u, m.v};
            double dv = 0.0;
            for (int e = 0; e < 3; ++e) {
                double viol = (b[e] < 0.0 ? -b[e] : 0.0) * h[e];
                if (viol > dv) dv = viol;
            }
            dv *= cosang;
            if (dv < near_miss) near_miss = dv;
        }
        near_miss_out[r] = near_miss;
    }
}

/* Exact-definition closest point on a triangle to a point: min over the face and its three edges.
 * Used by the nearest-obstacle query (Sec. III-B, spatial distance module). */
static double seg_closest(const double* p, const double* a, const double* b, double* out) {
    double ab[3], ap[3];
    sub3(b, a, ab);
    sub3(p, a, ap);
    double l2 = dot3(ab, ab);
    double s = l2 > 0.0 ? dot3(ap, ab) / l2 : 0.0;
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    for (int i = 0; i < 3; ++i) out[i] = a[i] + s * ab[i];
    double dd[3];
    sub3(p, out, dd);
    return dot3(dd, dd);
}

void oracle_closest_point(int64_t n_pts, const double* pts, int64_t n_tris,
                          const double* v0, const double* v1, const double* v2,
                          double* dist_out, double* point_out, int64_t* id_out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_pts; ++i) {
        const double* p = pts + 3 * i;
        double best = INFINITY, bp[3] = {0.0, 0.0, 0.0};
        int64_t bid = -1;
        for (int64_t k = 0; k < n_tris; ++k) {
            const double* a = v0 + 3 * k;
            const double* b = v1 + 3 * k;
            const double* c = v2 + 3 * k;
            double e1[3], e2[3], n[3], ap[3], cand[3];
            sub3(b, a, e1);
            sub3(c, a, e2);
            cross3(e1, e2, n);
            double nn = dot3(n, n);
            double d2 = INFINITY;
            if (nn > 0.0) {
                /* projection onto the plane; inside test by barycentric coordinates */
                sub3(p, a, ap);
                double dist = dot3(ap, n) / nn;
                double x[3] = {p[0] - dist * n[0], p[1] - dist * n[1], p[2] - dist * n[2]};
                double ax[3], c1[3], c2[3];
                sub3(x, a, ax);
                cross3(ax, e2, c1);
                cross3(e1, ax, c2);
                double bu = dot3(c1, n) / nn, bv = dot3(c2, n) / nn;
                if (bu >= 0.0 && bv >= 0.0 && bu + bv <= 1.0) {
                    double dd[3];
                    sub3(p, x, dd);
                    d2 = dot3(dd, dd);
                    for (int j = 0; j < 3; ++j) cand[j] = x[j];
                }
            }
            double tmp[3];
            double s;
            s = seg_closest(p, a, b, tmp);
            if (s < d2) { d2 = s; for (int j = 0; j < 3; ++j) cand[j] = tmp[j]; }
            s = seg_closest(p, b, c, tmp);
            if (s < d2) { d2 = s; for (int j = 0; j < 3; ++j) cand[j] = tmp[j]; }
            s = seg_closest(p, c, a, tmp);
            if (s < d2) { d2 = s; for (int j = 0; j < 3; ++j) cand[j] = tmp[j]; }
            if (d2 < best) {
                best = d2;
                bid = k;
                for (int j = 0; j < 3; ++j) bp[j] = cand[j];
            }
        }
        dist_out[i] = sqrt(best);
        id_out[i] = bid;
        for (int j = 0; j < 3; ++j) point_out[3 * i + j] = bp[j];
    }
}
