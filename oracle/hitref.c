/*
 * Brute-force FP64 ray/triangle queries for the oracle.
 *
 * TEST INFRASTRUCTURE ONLY: this file belongs to the CPU reference that the
 * GPU library is checked against.  It shares no code with the library.
 *
 * Every query tests every triangle; there is no acceleration structure.  The
 * intersection test is Moller-Trumbore (Moller & Trumbore, 1997), double
 * sided, with inclusive edges (u >= 0, v >= 0, u + v <= 1).  A triangle whose
 * face id equals the ray's excluded face id is skipped (a ray leaving a planar
 * reflector cannot meet the same plane again).  Closest hit: smallest t with
 * t > tmin; among equal t the smallest triangle index wins.
 *
 * The paper delegates intersection to its rendering back end (Sec. II:
 * "computation of ray intersections with scene primitives, i.e., triangles");
 * the rule above is the plain definition of the nearest ray/mesh crossing.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double v0[3], e1[3], e2[3];
    double inv_h[3]; /* 2A/|e2|, 2A/|e1|, 2A/|v2-v1|: barycentric -> distance to edge line */
} tri_t;

static void sub3(const double* a, const double* b, double* o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

static void make_tri(const double* V, const int32_t* F, int64_t k, tri_t* t) {
    const double* p0 = V + 3 * (int64_t)F[3 * k + 0];
    const double* p1 = V + 3 * (int64_t)F[3 * k + 1];
    const double* p2 = V + 3 * (int64_t)F[3 * k + 2];
    double n[3], e12[3];
    for (int i = 0; i < 3; ++i) t->v0[i] = p0[i];
    sub3(p1, p0, t->e1);
    sub3(p2, p0, t->e2);
    sub3(p2, p1, e12);
    cross3(t->e1, t->e2, n);
    double a2 = norm3(n);
    t->inv_h[0] = a2 / norm3(t->e2);
    t->inv_h[1] = a2 / norm3(t->e1);
    t->inv_h[2] = a2 / norm3(e12);
}

/* Moller-Trumbore.  Returns 1 and (t, u, v) if the ray's line crosses the
 * triangle's plane non-degenerately; *inside says whether the crossing lies in
 * the closed triangle. */
static int mt(const tri_t* tr, const double* o, const double* d, double* t, double* u, double* v, int* inside) {
    double P[3], T[3], Q[3];
    cross3(d, tr->e2, P);
    double det = dot3(tr->e1, P);
    if (fabs(det) < 1e-12 * norm3(tr->e1) * norm3(tr->e2)) return 0;
    double inv = 1.0 / det;
    sub3(o, tr->v0, T);
    *u = dot3(T, P) * inv;
    cross3(T, tr->e1, Q);
    *v = dot3(d, Q) * inv;
    *t = dot3(tr->e2, Q) * inv;
    *inside = (*u >= 0.0) && (*v >= 0.0) && (*u + *v <= 1.0);
    return 1;
}

/* Signed distance of the crossing point to the triangle's boundary measured
 * along the three edge lines (positive inside).  Its absolute value is a lower
 * bound of the distance to the boundary for points near the triangle. */
static double edge_margin(const tri_t* tr, double u, double v) {
    double a = u * tr->inv_h[0], b = v * tr->inv_h[1], c = (1.0 - u - v) * tr->inv_h[2];
    double m = a < b ? a : b;
    return m < c ? m : c;
}

/*
 * Closest hit for nr rays.
 *   O, D      [nr][3] ray origins and directions (D need not be unit; t is in units of |D|)
 *   excl      [nr] face id to skip (or -1)
 *   V, F      [nv][3] vertices, [nt][3] indices;  face [nt] face id per triangle
 *   out_tri   [nr] closest triangle index or -1;  out_t [nr] its t (or +inf)
 *   out_margin (nullable) [nr]: minimum over triangles whose plane the ray
 *             crosses within (tmin, t_hit] (all t > tmin on a miss) of
 *             |edge_margin|, i.e. how close the ray passes to any edge it
 *             could have hit first; 0 when another triangle ties with the
 *             hit (coincident geometry).
 */
void oracle_closest_hit(int64_t nr, const double* O, const double* D, const int32_t* excl, double tmin,
                        int64_t nv, const double* V, int64_t nt, const int32_t* F, const int32_t* face,
                        int32_t* out_tri, double* out_t, double* out_margin, int nthreads) {
    (void)nv;
    tri_t* tris = (tri_t*)malloc(sizeof(tri_t) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t k = 0; k < nt; ++k) make_tri(V, F, k, &tris[k]);

#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
    for (int64_t r = 0; r < nr; ++r) {
        const double* o = O + 3 * r;
        const double* d = D + 3 * r;
        int32_t best = -1;
        double tbest = INFINITY;
        for (int64_t k = 0; k < nt; ++k) {
            if (face[k] == excl[r]) continue;
            double t, u, v;
            int inside;
            if (!mt(&tris[k], o, d, &t, &u, &v, &inside)) continue;
            if (inside && t > tmin && t < tbest) { tbest = t; best = (int32_t)k; }
        }
        out_tri[r] = best;
        out_t[r] = tbest;
        if (out_margin) {
            double m = INFINITY;
            double tlim = best >= 0 ? tbest * (1.0 + 1e-9) + 1e-9 : INFINITY;
            for (int64_t k = 0; k < nt; ++k) {
                if (face[k] == excl[r]) continue;
                double t, u, v;
                int inside;
                if (!mt(&tris[k], o, d, &t, &u, &v, &inside)) continue;
                if (t > tmin && t <= tlim) {
                    double e = fabs(edge_margin(&tris[k], u, v));
                    /* a second triangle crossed inside at the hit distance is a tie
                       that only rounding decides (coincident geometry) */
                    if (inside && k != best && fabs(t - tbest) <= 1e-9 * (1.0 + tbest)) e = 0.0;
                    if (e < m) m = e;
                }
            }
            out_margin[r] = m;
        }
    }
    free(tris);
}

/*
 * Occlusion of segments A->B: occluded[s] = 1 if any triangle not in face
 * excl_a[s] or excl_b[s] is crossed, inside the closed triangle, at a
 * parameter t in (eps, 1 - eps) of the segment.
 */
void oracle_segments_occluded(int64_t ns, const double* A, const double* B, const int32_t* excl_a,
                              const int32_t* excl_b, double eps, int64_t nv, const double* V, int64_t nt,
                              const int32_t* F, const int32_t* face, uint8_t* occluded, int nthreads) {
    (void)nv;
    tri_t* tris = (tri_t*)malloc(sizeof(tri_t) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t k = 0; k < nt; ++k) make_tri(V, F, k, &tris[k]);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
    for (int64_t s = 0; s < ns; ++s) {
        double d[3];
        sub3(B + 3 * s, A + 3 * s, d);
        uint8_t occ = 0;
        for (int64_t k = 0; k < nt && !occ; ++k) {
            if (face[k] == excl_a[s] || face[k] == excl_b[s]) continue;
            double t, u, v;
            int inside;
            if (!mt(&tris[k], A + 3 * s, d, &t, &u, &v, &inside)) continue;
            if (inside && t > eps && t < 1.0 - eps) occ = 1;
        }
        occluded[s] = occ;
    }
    free(tris);
}
