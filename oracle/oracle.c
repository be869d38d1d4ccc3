/*
 * Plain FP64 CPU oracle for the overset direct cut and donor search.
 *
 * TEST INFRASTRUCTURE ONLY: it is called by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path, and shares no
 * source with the HIP library.
 *
 * What it computes (Crabill, Witherden & Jameson, "A Parallel Direct Cut
 * Algorithm for High-Order Overset Methods"):
 *
 *  Cut (Sec. 4.2 "Parallel Direct Cut Algorithm", Fig. quadsplit, Alg. cp2):
 *   every element face and every cut-surface face is taken as its node lattice
 *   split into 2x2 linear quads, each split into two triangles.  An element is
 *   hit by the surface when some pair of triangles is closer than the absolute
 *   tolerance 1e-7 used by the paper's distance passes (Alg. cp1/cp2), or when
 *   the surface lies inside it.  Whether a non-hit element is inside is the
 *   generalised winding number of the surface triangulation at the element's
 *   first node (> 1/2 means inside).  As a diagnostic the nearest-face side is
 *   also computed: the global nearest triangle pair, dotted with the outward
 *   normal of the surface triangle, with the tie rule of Sec. 4.1 (the pair of
 *   largest |dot| decides; normals are averaged only when equally visible
 *   pairs disagree in sign).
 *  Donor search (Sec. 4.3, eqs. reftophys, ref-update, Jac): Newton iterations
 *   on the isoparametric map from xi = 0, clamped to a small tolerance outside
 *   [-1, 1], at most ``maxit`` iterations; the lowest-id containing element is
 *   the donor.
 *
 * Accelerations (bounding volume hierarchies, box-distance pruning) only skip
 * pairs whose exact distance provably exceeds the bound in use, so they never
 * change a result; ``brute`` != 0 turns all of them off.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TOL_HIT 1e-7            /* Alg. cp1/cp2: tol = 1e-7 */
#define TIE_REL 1e-9            /* relative distance tie */
#define TIE_DOT 1e-9            /* |dot| tie */
#define CLAMP_EPS 0.01          /* Newton clamp: [-1-eps, 1+eps] */
#define CONTAIN_TOL 1e-10       /* contained if max|xi| <= 1 + tol */
#define STEP_TOL 1e-14
#define RES_TOL 1e-13

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                     */
/* ------------------------------------------------------------------------ */
static inline void v_sub(const double *a, const double *b, double *r) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static inline double v_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void v_cross(const double *a, const double *b, double *r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double v_dist2(const double *a, const double *b)
{
    double d[3];
    v_sub(a, b, d);
    return v_dot(d, d);
}
static inline void v_copy(double *d, const double *s) { d[0] = s[0]; d[1] = s[1]; d[2] = s[2]; }

/* closest point to p on segment [a, b] */
static void pt_seg(const double *p, const double *a, const double *b, double *q)
{
    double ab[3], ap[3];
    v_sub(b, a, ab);
    v_sub(p, a, ap);
    double L = v_dot(ab, ab);
    double t = (L > 0.0) ? v_dot(ap, ab) / L : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    for (int i = 0; i < 3; ++i) q[i] = a[i] + t * ab[i];
}

/* is x (in the plane of a,b,c with normal n) inside the closed triangle? */
static int in_tri(const double *x, const double *a, const double *b, const double *c, const double *n)
{
    const double *v[3] = {a, b, c};
    for (int k = 0; k < 3; ++k) {
        double e[3], w[3], cr[3];
        v_sub(v[(k + 1) % 3], v[k], e);
        v_sub(x, v[k], w);
        v_cross(e, w, cr);
        if (v_dot(cr, n) < 0.0) return 0;
    }
    return 1;
}

/* closest point to p on triangle (a, b, c): the projection if it falls in
 * the triangle, else the closest point of the three edges */
static void pt_tri(const double *p, const double *a, const double *b, const double *c, double *q)
{
    double ab[3], ac[3], n[3];
    v_sub(b, a, ab);
    v_sub(c, a, ac);
    v_cross(ab, ac, n);
    double nn = v_dot(n, n);
    if (nn > 0.0) {
        double ap[3];
        v_sub(p, a, ap);
        double t = v_dot(ap, n) / nn;
        double x[3] = {p[0] - t * n[0], p[1] - t * n[1], p[2] - t * n[2]};
        if (in_tri(x, a, b, c, n)) {
            v_copy(q, x);
            return;
        }
    }
    double best = INFINITY, cand[3];
    const double *v[3] = {a, b, c};
    for (int k = 0; k < 3; ++k) {
        pt_seg(p, v[k], v[(k + 1) % 3], cand);
        double d = v_dist2(p, cand);
        if (d < best) {
            best = d;
            v_copy(q, cand);
        }
    }
}

/* closest points of segments [p0,p1] and [q0,q1]: |P(s) - Q(t)|^2 is a convex
 * quadratic on [0,1]^2, so its minimum is the stationary point when that lies
 * in the square, else on one of the four sides (point-segment problems). */
static double seg_seg(const double *p0, const double *p1, const double *q0, const double *q1,
                      double *pc, double *qc)
{
    double d1[3], d2[3], r[3], c1[3], c2[3];
    v_sub(p1, p0, d1);
    v_sub(q1, q0, d2);
    v_sub(p0, q0, r);
    double best = INFINITY;
    double a = v_dot(d1, d1), b = v_dot(d1, d2), c = v_dot(d2, d2);
    double d = v_dot(d1, r), e = v_dot(d2, r);
    double den = a * c - b * b;
    if (den > 0.0) {
        double s = (b * e - c * d) / den;
        double t = (a * e - b * d) / den;
        if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
            for (int i = 0; i < 3; ++i) {
                c1[i] = p0[i] + s * d1[i];
                c2[i] = q0[i] + t * d2[i];
            }
            best = v_dist2(c1, c2);
            v_copy(pc, c1);
            v_copy(qc, c2);
        }
    }
    const double *ends[4] = {p0, p1, q0, q1};
    for (int k = 0; k < 4; ++k) {
        double x[3];
        double dd;
        if (k < 2) {
            pt_seg(ends[k], q0, q1, x);
            dd = v_dist2(ends[k], x);
            if (dd < best) { best = dd; v_copy(pc, ends[k]); v_copy(qc, x); }
        } else {
            pt_seg(ends[k], p0, p1, x);
            dd = v_dist2(ends[k], x);
            if (dd < best) { best = dd; v_copy(pc, x); v_copy(qc, ends[k]); }
        }
    }
    return best;
}

/* does segment [p0,p1] meet triangle (a,b,c) away from its plane's coplanar
 * case?  (Coplanar contacts are found by the vertex and edge distances.) */
static int seg_cross_tri(const double *p0, const double *p1, const double *a, const double *b,
                         const double *c, double *x)
{
    double ab[3], ac[3], n[3], w0[3], w1[3];
    v_sub(b, a, ab);
    v_sub(c, a, ac);
    v_cross(ab, ac, n);
    v_sub(p0, a, w0);
    v_sub(p1, a, w1);
    double s0 = v_dot(n, w0), s1 = v_dot(n, w1);
    if ((s0 > 0.0 && s1 > 0.0) || (s0 < 0.0 && s1 < 0.0)) return 0;
    if (s0 == 0.0 && s1 == 0.0) return 0;
    double t = s0 / (s0 - s1);
    for (int i = 0; i < 3; ++i) x[i] = p0[i] + t * (p1[i] - p0[i]);
    return in_tri(x, a, b, c, n);
}

double orc_tri_tri(const double *A, const double *B, double *pa, double *pb)
{
    const double *a[3] = {A, A + 3, A + 6};
    const double *b[3] = {B, B + 3, B + 6};
    double x[3], qa[3], qb[3];
    double dummy_a[3], dummy_b[3];
    if (!pa) pa = dummy_a;
    if (!pb) pb = dummy_b;
    /* intersecting triangles: some edge of one crosses the other */
    for (int k = 0; k < 3; ++k) {
        if (seg_cross_tri(a[k], a[(k + 1) % 3], b[0], b[1], b[2], x) ||
            seg_cross_tri(b[k], b[(k + 1) % 3], a[0], a[1], a[2], x)) {
            v_copy(pa, x);
            v_copy(pb, x);
            return 0.0;
        }
    }
    /* disjoint triangles: the distance is realised by a vertex-triangle or an
     * edge-edge pair */
    double best = INFINITY;
    for (int k = 0; k < 3; ++k) {
        pt_tri(a[k], b[0], b[1], b[2], x);
        double d = v_dist2(a[k], x);
        if (d < best) { best = d; v_copy(pa, a[k]); v_copy(pb, x); }
        pt_tri(b[k], a[0], a[1], a[2], x);
        d = v_dist2(b[k], x);
        if (d < best) { best = d; v_copy(pa, x); v_copy(pb, b[k]); }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double d = seg_seg(a[i], a[(i + 1) % 3], b[j], b[(j + 1) % 3], qa, qb);
            if (d < best) { best = d; v_copy(pa, qa); v_copy(pb, qb); }
        }
    return sqrt(best);
}

double orc_solid_angle(const double *p, const double *A, const double *B, const double *C)
{
    double a[3], b[3], c[3], bc[3];
    v_sub(A, p, a);
    v_sub(B, p, b);
    v_sub(C, p, c);
    double la = sqrt(v_dot(a, a)), lb = sqrt(v_dot(b, b)), lc = sqrt(v_dot(c, c));
    v_cross(b, c, bc);
    double num = v_dot(a, bc);
    double den = la * lb * lc + v_dot(a, b) * lc + v_dot(a, c) * lb + v_dot(b, c) * la;
    return 2.0 * atan2(num, den);
}

/* ------------------------------------------------------------------------ */
/* quadratic Lagrange map (eq. reftophys) and its Jacobian (eq. Jac)         */
/* ------------------------------------------------------------------------ */
static void lag2(double s, double *l, double *dl)
{
    l[0] = 0.5 * s * (s - 1.0);
    l[1] = 1.0 - s * s;
    l[2] = 0.5 * s * (s + 1.0);
    dl[0] = s - 0.5;
    dl[1] = -2.0 * s;
    dl[2] = s + 0.5;
}

void orc_q2_eval(const double *X, const double *xi, double *x, double *J)
{
    double l[3][3], dl[3][3];
    for (int d = 0; d < 3; ++d) lag2(xi[d], l[d], dl[d]);
    for (int i = 0; i < 3; ++i) x[i] = 0.0;
    if (J)
        for (int i = 0; i < 9; ++i) J[i] = 0.0;
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const double *p = X + 3 * (a + 3 * b + 9 * c);
                double N = l[0][a] * l[1][b] * l[2][c];
                double N0 = dl[0][a] * l[1][b] * l[2][c];
                double N1 = l[0][a] * dl[1][b] * l[2][c];
                double N2 = l[0][a] * l[1][b] * dl[2][c];
                for (int i = 0; i < 3; ++i) {
                    x[i] += p[i] * N;
                    if (J) {
                        J[i * 3 + 0] += p[i] * N0;
                        J[i * 3 + 1] += p[i] * N1;
                        J[i * 3 + 2] += p[i] * N2;
                    }
                }
            }
}

/* solve the 3x3 system M y = r by Gaussian elimination with partial pivoting */
static int solve3(const double *M, const double *r, double *y)
{
    double A[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) A[i][j] = M[i * 3 + j];
        A[i][3] = r[i];
    }
    for (int k = 0; k < 3; ++k) {
        int p = k;
        for (int i = k + 1; i < 3; ++i)
            if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
        if (A[p][k] == 0.0) return 0;
        if (p != k)
            for (int j = 0; j < 4; ++j) {
                double t = A[k][j];
                A[k][j] = A[p][j];
                A[p][j] = t;
            }
        for (int i = k + 1; i < 3; ++i) {
            double f = A[i][k] / A[k][k];
            for (int j = k; j < 4; ++j) A[i][j] -= f * A[k][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = A[i][3];
        for (int j = i + 1; j < 3; ++j) s -= A[i][j] * y[j];
        y[i] = s / A[i][i];
    }
    return 1;
}

static double node_diam(const double *X)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int n = 0; n < 27; ++n)
        for (int i = 0; i < 3; ++i) {
            if (X[3 * n + i] < lo[i]) lo[i] = X[3 * n + i];
            if (X[3 * n + i] > hi[i]) hi[i] = X[3 * n + i];
        }
    double s = 0.0;
    for (int i = 0; i < 3; ++i) s += (hi[i] - lo[i]) * (hi[i] - lo[i]);
    return sqrt(s);
}

/* Newton on x(xi) = xp (eq. ref-update): xi^0 = 0; stop when the residual is
 * below RES_TOL*diam (checked before each step) or the clamped step is below
 * STEP_TOL; contained if converged and max|xi| <= 1 + CONTAIN_TOL. */
int orc_newton(const double *X, const double *xp, int maxit, double *xi_out, int *iters_out)
{
    double xi[3] = {0.0, 0.0, 0.0};
    double diam = node_diam(X);
    int conv = 0, it;
    for (it = 1; it <= maxit; ++it) {
        double x[3], J[9], r[3], dxi[3];
        orc_q2_eval(X, xi, x, J);
        v_sub(xp, x, r);
        if (sqrt(v_dot(r, r)) <= RES_TOL * diam) {
            conv = 1;
            break;
        }
        if (!solve3(J, r, dxi)) break;
        double step = 0.0;
        for (int i = 0; i < 3; ++i) {
            double v = xi[i] + dxi[i];
            if (v < -1.0 - CLAMP_EPS) v = -1.0 - CLAMP_EPS;
            if (v > 1.0 + CLAMP_EPS) v = 1.0 + CLAMP_EPS;
            double s = fabs(v - xi[i]);
            if (s > step) step = s;
            xi[i] = v;
        }
        if (step <= STEP_TOL) {
            conv = 1;
            break;
        }
    }
    if (iters_out) *iters_out = it > maxit ? maxit : it;
    if (xi_out) v_copy(xi_out, xi);
    double m = fmax(fabs(xi[0]), fmax(fabs(xi[1]), fabs(xi[2])));
    return conv && m <= 1.0 + CONTAIN_TOL;
}

/* ------------------------------------------------------------------------ */
/* element boundary triangulation (Fig. quadsplit)                           */
/* ------------------------------------------------------------------------ */
/* node of face f's 3x3 lattice at (u, v); faces -xi,+xi,-eta,+eta,-zeta,+zeta */
static int face_node(int f, int u, int v)
{
    switch (f) {
    case 0: return 0 + 3 * u + 9 * v;
    case 1: return 2 + 3 * u + 9 * v;
    case 2: return u + 9 * v;
    case 3: return u + 6 + 9 * v;
    case 4: return u + 3 * v;
    default: return u + 3 * v + 18;
    }
}

/* two triangles of lattice quad (m, n) with corners p(m,n), p(m+1,n),
 * p(m+1,n+1), p(m,n+1), split along p(m,n)-p(m+1,n+1) */
static void quad_tris(int m, int n, int idx[6])
{
    int p00 = m + 3 * n, p10 = (m + 1) + 3 * n, p11 = (m + 1) + 3 * (n + 1), p01 = m + 3 * (n + 1);
    idx[0] = p00; idx[1] = p10; idx[2] = p11;
    idx[3] = p00; idx[4] = p11; idx[5] = p01;
}

static void elem_nodes(const double *nodes, const int32_t *conn, int64_t e, double *X)
{
    for (int n = 0; n < 27; ++n) {
        const double *p = nodes + 3 * (int64_t)conn[e * 27 + n];
        X[3 * n] = p[0];
        X[3 * n + 1] = p[1];
        X[3 * n + 2] = p[2];
    }
}

static void tris_from_elem(const double *X, double *tris)
{
    int t = 0;
    for (int f = 0; f < 6; ++f)
        for (int n = 0; n < 2; ++n)
            for (int m = 0; m < 2; ++m) {
                int q[6];
                quad_tris(m, n, q);
                for (int k = 0; k < 6; ++k) {
                    int u = q[k] % 3, v = q[k] / 3;
                    int node = face_node(f, u, v);
                    v_copy(tris + 9 * t + 3 * (k % 3), X + 3 * node);
                    if (k % 3 == 2) ++t;
                }
            }
}

void orc_element_tris(const double *nodes, const int32_t *conn, int64_t e, double *tris)
{
    double X[81];
    elem_nodes(nodes, conn, e, X);
    tris_from_elem(X, tris);
}

static void tris_from_face(const double *P /* 9 nodes */, double *tris /* 8*9 */)
{
    int t = 0;
    for (int n = 0; n < 2; ++n)
        for (int m = 0; m < 2; ++m) {
            int q[6];
            quad_tris(m, n, q);
            for (int k = 0; k < 6; ++k) {
                v_copy(tris + 9 * t + 3 * (k % 3), P + 3 * q[k]);
                if (k % 3 == 2) ++t;
            }
        }
}

static void box_of(const double *pts, int n, double *box /* lo3 hi3 */)
{
    for (int i = 0; i < 3; ++i) {
        box[i] = INFINITY;
        box[3 + i] = -INFINITY;
    }
    for (int k = 0; k < n; ++k)
        for (int i = 0; i < 3; ++i) {
            double v = pts[3 * k + i];
            if (v < box[i]) box[i] = v;
            if (v > box[3 + i]) box[3 + i] = v;
        }
}

/* Euclidean distance between two axis-aligned boxes (a lower bound on the
 * distance between anything they contain) */
static double box_dist(const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < 3; ++i) {
        double g = fmax(b[i] - a[3 + i], a[i] - b[3 + i]);
        if (g > 0.0) s += g * g;
    }
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* bounding volume hierarchy over boxes (oracle-only acceleration)           */
/* ------------------------------------------------------------------------ */
typedef struct {
    double box[6];
    int left, right;   /* children, -1 for a leaf */
    int start, count;  /* leaf item range in idx[] */
} bnode;

typedef struct {
    bnode *node;
    int n_node, cap;
    int *idx;
    const double *boxes; /* n x 6 */
} bvh;

static double ctr(const double *boxes, int i, int ax) { return boxes[6 * i + ax] + boxes[6 * i + 3 + ax]; }

/* partial sort of idx[lo..hi) so that idx[k] has the k-th centre along ax */
static void select_k(int *idx, int lo, int hi, int k, const double *boxes, int ax)
{
    while (hi - lo > 1) {
        double piv = ctr(boxes, idx[(lo + hi) / 2], ax);
        int i = lo, j = hi - 1;
        while (i <= j) {
            while (ctr(boxes, idx[i], ax) < piv) ++i;
            while (ctr(boxes, idx[j], ax) > piv) --j;
            if (i <= j) {
                int t = idx[i];
                idx[i] = idx[j];
                idx[j] = t;
                ++i;
                --j;
            }
        }
        if (k <= j) hi = j + 1;
        else if (k >= i) lo = i;
        else return;
    }
}

static int bvh_new_node(bvh *b)
{
    if (b->n_node == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->node = (bnode *)realloc(b->node, sizeof(bnode) * b->cap);
    }
    return b->n_node++;
}

static int bvh_build_rec(bvh *b, int lo, int hi)
{
    int id = bvh_new_node(b);
    double box[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int k = lo; k < hi; ++k) {
        const double *bx = b->boxes + 6 * b->idx[k];
        for (int i = 0; i < 3; ++i) {
            if (bx[i] < box[i]) box[i] = bx[i];
            if (bx[3 + i] > box[3 + i]) box[3 + i] = bx[3 + i];
        }
    }
    memcpy(b->node[id].box, box, sizeof box);
    if (hi - lo <= 4) {
        b->node[id].left = b->node[id].right = -1;
        b->node[id].start = lo;
        b->node[id].count = hi - lo;
        return id;
    }
    int ax = 0;
    double ext = box[3] - box[0];
    for (int i = 1; i < 3; ++i)
        if (box[3 + i] - box[i] > ext) {
            ext = box[3 + i] - box[i];
            ax = i;
        }
    int mid = (lo + hi) / 2;
    select_k(b->idx, lo, hi, mid, b->boxes, ax);
    int l = bvh_build_rec(b, lo, mid);
    int r = bvh_build_rec(b, mid, hi);
    b->node[id].left = l;
    b->node[id].right = r;
    b->node[id].start = 0;
    b->node[id].count = 0;
    return id;
}

static void bvh_build(bvh *b, const double *boxes, int n)
{
    memset(b, 0, sizeof *b);
    b->boxes = boxes;
    b->idx = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) b->idx[i] = i;
    if (n > 0) bvh_build_rec(b, 0, n);
}

static void bvh_free(bvh *b)
{
    free(b->node);
    free(b->idx);
}

typedef struct {
    int *v;
    int n, cap;
} ivec;

static void iv_push(ivec *a, int x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 256;
        a->v = (int *)realloc(a->v, sizeof(int) * a->cap);
    }
    a->v[a->n++] = x;
}

/* all items whose box is within distance r (<= r) of query box q */
static void bvh_near_box(const bvh *b, const double *q, double r, ivec *out, ivec *stack)
{
    out->n = 0;
    if (b->n_node == 0) return;
    stack->n = 0;
    iv_push(stack, 0);
    while (stack->n) {
        const bnode *nd = &b->node[stack->v[--stack->n]];
        if (box_dist(nd->box, q) > r) continue;
        if (nd->left < 0) {
            for (int k = 0; k < nd->count; ++k) {
                int it = b->idx[nd->start + k];
                if (box_dist(b->boxes + 6 * it, q) <= r) iv_push(out, it);
            }
        } else {
            iv_push(stack, nd->left);
            iv_push(stack, nd->right);
        }
    }
}

/* all items whose box contains point p */
static void bvh_contain(const bvh *b, const double *p, ivec *out, ivec *stack)
{
    out->n = 0;
    if (b->n_node == 0) return;
    stack->n = 0;
    iv_push(stack, 0);
    while (stack->n) {
        const bnode *nd = &b->node[stack->v[--stack->n]];
        const double *bx = nd->box;
        if (p[0] < bx[0] || p[1] < bx[1] || p[2] < bx[2] || p[0] > bx[3] || p[1] > bx[4] || p[2] > bx[5]) continue;
        if (nd->left < 0) {
            for (int k = 0; k < nd->count; ++k) {
                int it = b->idx[nd->start + k];
                const double *c = b->boxes + 6 * it;
                if (p[0] >= c[0] && p[1] >= c[1] && p[2] >= c[2] && p[0] <= c[3] && p[1] <= c[4] && p[2] <= c[5])
                    iv_push(out, it);
            }
        } else {
            iv_push(stack, nd->left);
            iv_push(stack, nd->right);
        }
    }
}

/* one leaf reached by always descending towards the nearer child */
static int bvh_greedy_leaf(const bvh *b, const double *q)
{
    int id = 0;
    while (b->node[id].left >= 0) {
        int l = b->node[id].left, r = b->node[id].right;
        id = box_dist(b->node[l].box, q) <= box_dist(b->node[r].box, q) ? l : r;
    }
    return id;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* face neighbours                                                          */
/* ------------------------------------------------------------------------ */
static const int FACE_CORNERS[6][4] = {
    {0, 6, 18, 24}, {2, 8, 20, 26}, {0, 2, 18, 20}, {6, 8, 24, 26}, {0, 2, 6, 8}, {18, 20, 24, 26}};

typedef struct {
    int32_t k[4];
    int64_t ef; /* e*6 + f */
} face_key;

static int cmp_face(const void *a, const void *b)
{
    const face_key *x = (const face_key *)a, *y = (const face_key *)b;
    for (int i = 0; i < 4; ++i)
        if (x->k[i] != y->k[i]) return x->k[i] < y->k[i] ? -1 : 1;
    return (x->ef > y->ef) - (x->ef < y->ef);
}

int orc_face_neighbors(const int32_t *conn, int64_t n_elem, int32_t *nbr)
{
    int64_t nf = n_elem * 6;
    face_key *fk = (face_key *)malloc(sizeof(face_key) * (nf > 0 ? nf : 1));
    if (!fk) return -1;
    for (int64_t e = 0; e < n_elem; ++e)
        for (int f = 0; f < 6; ++f) {
            face_key *k = &fk[e * 6 + f];
            for (int i = 0; i < 4; ++i) k->k[i] = conn[e * 27 + FACE_CORNERS[f][i]];
            qsort(k->k, 4, sizeof(int32_t), cmp_int);
            k->ef = e * 6 + f;
            nbr[e * 6 + f] = -1;
        }
    qsort(fk, nf, sizeof(face_key), cmp_face);
    for (int64_t i = 0; i + 1 < nf; ++i) {
        if (memcmp(fk[i].k, fk[i + 1].k, sizeof fk[i].k) == 0) {
            nbr[fk[i].ef] = (int32_t)(fk[i + 1].ef / 6);
            nbr[fk[i + 1].ef] = (int32_t)(fk[i].ef / 6);
        }
    }
    free(fk);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* direct cut                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_face;
    double *tris;    /* n_face * 8 * 9  (posed) */
    double *tbox;    /* n_face * 8 * 6 */
    double *fbox;    /* n_face * 6 */
    double *tnrm;    /* n_face * 8 * 3 unit outward normals */
    double sbox[6];  /* whole surface */
    double first[3]; /* first surface node (posed) */
    bvh tree;
} surf_t;

static void pose_point(const double *pose, const double *x, double *y)
{
    for (int i = 0; i < 3; ++i)
        y[i] = pose[3 * i] * x[0] + pose[3 * i + 1] * x[1] + pose[3 * i + 2] * x[2] + pose[9 + i];
}

static void surf_build(surf_t *S, const double *snodes, int64_t n_snodes, const int32_t *sconn,
                       int64_t n_face, const double *pose, int accel)
{
    S->n_face = n_face;
    S->tris = (double *)malloc(sizeof(double) * n_face * 72 + 8);
    S->tbox = (double *)malloc(sizeof(double) * n_face * 48 + 8);
    S->fbox = (double *)malloc(sizeof(double) * n_face * 6 + 8);
    S->tnrm = (double *)malloc(sizeof(double) * n_face * 24 + 8);
    for (int i = 0; i < 3; ++i) {
        S->sbox[i] = INFINITY;
        S->sbox[3 + i] = -INFINITY;
    }
    pose_point(pose, snodes, S->first);
    (void)n_snodes;
    for (int64_t f = 0; f < n_face; ++f) {
        double P[27];
        for (int k = 0; k < 9; ++k) pose_point(pose, snodes + 3 * (int64_t)sconn[f * 9 + k], P + 3 * k);
        tris_from_face(P, S->tris + 72 * f);
        box_of(P, 9, S->fbox + 6 * f);
        for (int i = 0; i < 3; ++i) {
            S->sbox[i] = fmin(S->sbox[i], S->fbox[6 * f + i]);
            S->sbox[3 + i] = fmax(S->sbox[3 + i], S->fbox[6 * f + 3 + i]);
        }
        for (int t = 0; t < 8; ++t) {
            const double *T = S->tris + 72 * f + 9 * t;
            box_of(T, 3, S->tbox + 48 * f + 6 * t);
            double ab[3], ac[3], n[3];
            v_sub(T + 3, T, ab);
            v_sub(T + 6, T, ac);
            v_cross(ab, ac, n);
            double L = sqrt(v_dot(n, n));
            for (int i = 0; i < 3; ++i) S->tnrm[24 * f + 3 * t + i] = L > 0.0 ? n[i] / L : 0.0;
        }
    }
    if (accel) bvh_build(&S->tree, S->fbox, (int)n_face);
    else memset(&S->tree, 0, sizeof S->tree);
}

static void surf_free(surf_t *S)
{
    free(S->tris);
    free(S->tbox);
    free(S->fbox);
    free(S->tnrm);
    bvh_free(&S->tree);
}

/* selection record for the nearest-face sign (tie rule) */
typedef struct {
    double absdot, dot;
    double v[3], n[3];
    int64_t f;
    int s, t;
    int valid;
} tie_rec;

/* ordering: larger |dot| first, then lower (face, face tri, element tri) */
static int tie_before(const tie_rec *a, const tie_rec *b)
{
    if (!b->valid) return 1;
    if (a->absdot != b->absdot) return a->absdot > b->absdot;
    if (a->f != b->f) return a->f < b->f;
    if (a->s != b->s) return a->s < b->s;
    return a->t < b->t;
}

static void tie_offer(tie_rec *b1, tie_rec *b2, const tie_rec *r)
{
    if (tie_before(r, b1)) {
        *b2 = *b1;
        *b1 = *r;
    } else if (tie_before(r, b2)) {
        *b2 = *r;
    }
}

/* exact element-face minimum distance over triangle pairs whose box distance
 * does not exceed ``bound`` (pairs farther than bound cannot lower a minimum
 * that is already <= bound).  stop_below: return as soon as a pair is closer
 * than it (used for the hit test). */
static double ef_min(const double *et, const double *ebox, const surf_t *S, int64_t f, double bound,
                     int prune, double stop_below)
{
    double best = INFINITY;
    for (int s = 0; s < 8; ++s) {
        const double *ft = S->tris + 72 * f + 9 * s;
        const double *fb = S->tbox + 48 * f + 6 * s;
        for (int t = 0; t < 48; ++t) {
            double lim = fmin(bound, best);
            if (prune && box_dist(ebox + 6 * t, fb) > lim) continue;
            double d = orc_tri_tri(et + 9 * t, ft, NULL, NULL);
            if (d < best) best = d;
            if (best < stop_below) return best;
        }
    }
    return best;
}

static void ef_ties(const double *et, const double *ebox, const surf_t *S, int64_t f, double thr,
                    int prune, tie_rec *b1, tie_rec *b2)
{
    for (int s = 0; s < 8; ++s) {
        const double *ft = S->tris + 72 * f + 9 * s;
        const double *fb = S->tbox + 48 * f + 6 * s;
        for (int t = 0; t < 48; ++t) {
            if (prune && box_dist(ebox + 6 * t, fb) > thr) continue;
            double pa[3], pb[3];
            double d = orc_tri_tri(et + 9 * t, ft, pa, pb);
            if (d > thr) continue;
            tie_rec r;
            v_sub(pa, pb, r.v);
            double L = sqrt(v_dot(r.v, r.v));
            v_copy(r.n, S->tnrm + 24 * f + 3 * s);
            r.dot = L > 0.0 ? v_dot(r.v, r.n) / L : 0.0;
            r.absdot = fabs(r.dot);
            r.f = f;
            r.s = s;
            r.t = t;
            r.valid = 1;
            tie_offer(b1, b2, &r);
        }
    }
}

static double winding(const surf_t *S, const double *p)
{
    double w = 0.0;
    for (int64_t f = 0; f < S->n_face; ++f)
        for (int t = 0; t < 8; ++t) {
            const double *T = S->tris + 72 * f + 9 * t;
            w += orc_solid_angle(p, T, T + 3, T + 6);
        }
    return w / (4.0 * M_PI);
}

/* Nearest-face side of a point (the rule of Sec. 4.1 applied to the
 * nearest surface point of one node): global nearest distance, then among
 * the triangles within best*(1+1e-9) the largest |dot| of the unit
 * point-to-surface vector with the outward normal decides; normals are
 * averaged only when the two most visible disagree in sign. */
static int point_side(const surf_t *S, const double *p, int brute, ivec *cand, ivec *stack, double *dout)
{
    double pb[6] = {p[0], p[1], p[2], p[0], p[1], p[2]};
    double best = INFINITY;
    if (brute) {
        for (int64_t f = 0; f < S->n_face; ++f)
            for (int t = 0; t < 8; ++t) {
                const double *T = S->tris + 72 * f + 9 * t;
                double q[3];
                pt_tri(p, T, T + 3, T + 6, q);
                best = fmin(best, sqrt(v_dist2(p, q)));
            }
    } else {
        int leaf = bvh_greedy_leaf(&S->tree, pb);
        const bnode *nd = &S->tree.node[leaf];
        for (int k = 0; k < nd->count; ++k) {
            int64_t f = S->tree.idx[nd->start + k];
            for (int t = 0; t < 8; ++t) {
                const double *T = S->tris + 72 * f + 9 * t;
                double q[3];
                pt_tri(p, T, T + 3, T + 6, q);
                best = fmin(best, sqrt(v_dist2(p, q)));
            }
        }
        bvh_near_box(&S->tree, pb, best, cand, stack);
        for (int k = 0; k < cand->n; ++k)
            for (int t = 0; t < 8; ++t) {
                const double *T = S->tris + 72 * (int64_t)cand->v[k] + 9 * t;
                if (box_dist(S->tbox + 48 * (int64_t)cand->v[k] + 6 * t, pb) > best) continue;
                double q[3];
                pt_tri(p, T, T + 3, T + 6, q);
                best = fmin(best, sqrt(v_dist2(p, q)));
            }
    }
    double thr = best * (1.0 + TIE_REL);
    tie_rec b1, b2;
    b1.valid = b2.valid = 0;
    if (!brute) bvh_near_box(&S->tree, pb, thr, cand, stack);
    int64_t nf = brute ? S->n_face : cand->n;
    for (int64_t k = 0; k < nf; ++k) {
        int64_t f = brute ? k : cand->v[k];
        for (int t = 0; t < 8; ++t) {
            const double *T = S->tris + 72 * f + 9 * t;
            double q[3];
            pt_tri(p, T, T + 3, T + 6, q);
            double d = sqrt(v_dist2(p, q));
            if (d > thr) continue;
            tie_rec r;
            v_sub(p, q, r.v);
            v_copy(r.n, S->tnrm + 24 * f + 3 * t);
            r.dot = d > 0.0 ? v_dot(r.v, r.n) / d : 0.0;
            r.absdot = fabs(r.dot);
            r.f = f;
            r.s = t;
            r.t = 0;
            r.valid = 1;
            tie_offer(&b1, &b2, &r);
        }
    }
    double sgn = b1.dot;
    if (b2.valid && b1.absdot - b2.absdot <= TIE_DOT && (b1.dot > 0.0) != (b2.dot > 0.0)) {
        double nn[3] = {b1.n[0] + b2.n[0], b1.n[1] + b2.n[1], b1.n[2] + b2.n[2]};
        sgn = v_dot(b1.v, nn);
    }
    if (dout) *dout = best;
    return sgn < 0.0 ? -1 : 1;
}

/* Winding number of an element's closed boundary at p.  The face lattices
 * of -xi, +eta and -zeta run clockwise seen from outside, so their
 * triangles count with the opposite sign. */
static double elem_winding(const double *et, const double *p)
{
    static const double face_sign[6] = {-1.0, 1.0, 1.0, -1.0, -1.0, 1.0};
    double w = 0.0;
    for (int t = 0; t < 48; ++t)
        w += face_sign[t / 8] * orc_solid_angle(p, et + 9 * t, et + 9 * t + 3, et + 9 * t + 6);
    return w / (4.0 * M_PI);
}

double orc_element_winding(const double *nodes, const int32_t *conn, int64_t e, const double *p)
{
    double X[81], et[48 * 9];
    elem_nodes(nodes, conn, e, X);
    tris_from_elem(X, et);
    return elem_winding(et, p);
}

static int in_box(const double *b, const double *p)
{
    return p[0] >= b[0] && p[1] >= b[1] && p[2] >= b[2] && p[0] <= b[3] && p[1] <= b[4] && p[2] <= b[5];
}

static void classify_one(const double *gnodes, const int32_t *gconn, int64_t e, const surf_t *S, int kind,
                         int brute, ivec *cand, ivec *stack, int8_t *status, int8_t *hit_out,
                         double *dstar_out, int8_t *nsign_out, double *wind_out, int8_t *psign_out)
{
    double X[81], et[48 * 9], ebox[48 * 6], box[6];
    elem_nodes(gnodes, gconn, e, X);
    tris_from_elem(X, et);
    box_of(X, 27, box);
    for (int t = 0; t < 48; ++t) box_of(et + 9 * t, 3, ebox + 6 * t);
    int prune = !brute;

    /* faces to consider for the hit test */
    if (brute) {
        cand->n = 0;
        for (int64_t f = 0; f < S->n_face; ++f) iv_push(cand, (int)f);
    } else {
        bvh_near_box(&S->tree, box, TOL_HIT, cand, stack);
    }
    int hit = 0;
    for (int k = 0; k < cand->n && !hit; ++k) {
        double d = ef_min(et, ebox, S, cand->v[k], TOL_HIT, prune, TOL_HIT);
        if (d < TOL_HIT) hit = 1;
    }
    /* surface enclosed by the element */
    if (!hit && (brute || in_box(box, S->first))) {
        if (fabs(elem_winding(et, S->first)) > 0.5) hit = 1;
    }
    /* winding number at the first node (zero outside the surface's box) */
    double w = 0.0;
    if (brute || in_box(S->sbox, X)) w = winding(S, X);
    int inside = w > 0.5;

    double dstar = 0.0;
    int nsign = 0;
    if (!hit && (dstar_out || nsign_out)) {
        /* global nearest pair */
        double best = INFINITY;
        if (brute) {
            for (int64_t f = 0; f < S->n_face; ++f) {
                double d = ef_min(et, ebox, S, f, INFINITY, 0, -1.0);
                if (d < best) best = d;
            }
        } else {
            int leaf = bvh_greedy_leaf(&S->tree, box);
            const bnode *nd = &S->tree.node[leaf];
            for (int k = 0; k < nd->count; ++k) {
                double d = ef_min(et, ebox, S, S->tree.idx[nd->start + k], INFINITY, 1, -1.0);
                if (d < best) best = d;
            }
            bvh_near_box(&S->tree, box, best, cand, stack);
            qsort(cand->v, cand->n, sizeof(int), cmp_int);
            for (int k = 0; k < cand->n; ++k) {
                if (box_dist(S->fbox + 6 * cand->v[k], box) > best) continue;
                double d = ef_min(et, ebox, S, cand->v[k], best, 1, -1.0);
                if (d < best) best = d;
            }
        }
        dstar = best;
        /* tie set and sign */
        double thr = best * (1.0 + TIE_REL);
        tie_rec b1, b2;
        b1.valid = b2.valid = 0;
        if (brute) {
            for (int64_t f = 0; f < S->n_face; ++f) ef_ties(et, ebox, S, f, thr, 0, &b1, &b2);
        } else {
            bvh_near_box(&S->tree, box, thr, cand, stack);
            for (int k = 0; k < cand->n; ++k) ef_ties(et, ebox, S, cand->v[k], thr, 1, &b1, &b2);
        }
        double sgn = b1.dot;
        if (b2.valid && b1.absdot - b2.absdot <= TIE_DOT && (b1.dot > 0.0) != (b2.dot > 0.0)) {
            double nn[3] = {b1.n[0] + b2.n[0], b1.n[1] + b2.n[1], b1.n[2] + b2.n[2]};
            sgn = v_dot(b1.v, nn);
        }
        nsign = sgn < 0.0 ? -1 : 1;
    }

    if (psign_out) *psign_out = hit ? 0 : (int8_t)point_side(S, X, brute, cand, stack, NULL);

    int hole;
    if (kind == 0) hole = hit || inside;  /* wall */
    else hole = inside && !hit;           /* overset */
    if (status) *status = hole ? 0 : 1;
    if (hit_out) *hit_out = (int8_t)hit;
    if (dstar_out) *dstar_out = dstar;
    if (nsign_out) *nsign_out = (int8_t)nsign;
    if (wind_out) *wind_out = w;
}

int orc_cut_surface(const double *gnodes, const int32_t *gconn, int64_t n_elem, const int64_t *sel,
                    int64_t n_sel, const double *snodes, int64_t n_snodes, const int32_t *sconn,
                    int64_t n_face, const double *pose, int kind, int brute, int n_threads, int8_t *status,
                    int8_t *hit, double *dstar, int8_t *nsign, double *wind, int8_t *psign)
{
    surf_t S;
    surf_build(&S, snodes, n_snodes, sconn, n_face, pose, !brute);
    int64_t n = sel ? n_sel : n_elem;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        ivec cand = {0, 0, 0}, stack = {0, 0, 0};
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < n; ++i) {
            int64_t e = sel ? sel[i] : i;
            classify_one(gnodes, gconn, e, &S, kind, brute, &cand, &stack, status ? status + i : NULL,
                         hit ? hit + i : NULL, dstar ? dstar + i : NULL, nsign ? nsign + i : NULL,
                         wind ? wind + i : NULL, psign ? psign + i : NULL);
        }
        free(cand.v);
        free(stack.v);
    }
    surf_free(&S);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* fringe points and donor search                                           */
/* ------------------------------------------------------------------------ */
int orc_fringe_points(const double *gnodes, const int32_t *gconn, const int64_t *elems, int64_t n,
                      const double *pose, double *pts)
{
    const double g[3] = {-sqrt(0.6), 0.0, sqrt(0.6)};
    for (int64_t i = 0; i < n; ++i) {
        double X[81];
        elem_nodes(gnodes, gconn, elems[i], X);
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    double xi[3] = {g[a], g[b], g[c]}, x[3];
                    orc_q2_eval(X, xi, x, NULL);
                    pose_point(pose, x, pts + 3 * (27 * i + a + 3 * b + 9 * c));
                }
    }
    return 0;
}

/* axis-aligned box of the element's Bernstein control net (the element lies
 * in its convex hull), inflated by 1e-10 of the node-box diagonal */
static void control_box(const double *X, double *box)
{
    double C[81];
    memcpy(C, X, sizeof C);
    /* along each reference axis, the middle Lagrange node becomes the
     * Bernstein control point 2 x1 - (x0 + x2)/2 */
    const int stride[3] = {1, 3, 9};
    for (int ax = 0; ax < 3; ++ax) {
        int s = stride[ax];
        for (int n = 0; n < 27; ++n) {
            int pos = (n / s) % 3;
            if (pos != 1) continue;
            for (int i = 0; i < 3; ++i)
                C[3 * n + i] = 2.0 * C[3 * n + i] - 0.5 * (C[3 * (n - s) + i] + C[3 * (n + s) + i]);
        }
    }
    box_of(C, 27, box);
    double infl = 1e-10 * node_diam(X);
    for (int i = 0; i < 3; ++i) {
        box[i] -= infl;
        box[3 + i] += infl;
    }
}

int orc_donor_search(const double *gnodes, const int32_t *gconn, int64_t n_elem, const double *pose,
                     const double *pts, int64_t n, int brute, int maxit, int n_threads, int32_t *donor,
                     double *xi, int32_t *iters, int32_t *n_cand)
{
    double *boxes = (double *)malloc(sizeof(double) * 6 * (n_elem > 0 ? n_elem : 1));
    for (int64_t e = 0; e < n_elem; ++e) {
        double X[81];
        elem_nodes(gnodes, gconn, e, X);
        control_box(X, boxes + 6 * e);
    }
    bvh tree;
    if (!brute) bvh_build(&tree, boxes, (int)n_elem);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        ivec cand = {0, 0, 0}, stack = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            /* into the grid's registration frame: x = R^T (x_world - t) */
            double q[3], p[3];
            for (int k = 0; k < 3; ++k) q[k] = pts[3 * i + k] - pose[9 + k];
            for (int k = 0; k < 3; ++k) p[k] = pose[k] * q[0] + pose[3 + k] * q[1] + pose[6 + k] * q[2];
            if (brute) {
                cand.n = 0;
                for (int64_t e = 0; e < n_elem; ++e) iv_push(&cand, (int)e);
            } else {
                bvh_contain(&tree, p, &cand, &stack);
                qsort(cand.v, cand.n, sizeof(int), cmp_int);
            }
            int32_t d = -1;
            double r[3] = {NAN, NAN, NAN};
            int used = 0;
            for (int k = 0; k < cand.n; ++k) {
                double X[81], x3[3];
                int it = 0;
                elem_nodes(gnodes, gconn, cand.v[k], X);
                int ok = orc_newton(X, p, maxit, x3, &it);
                if (ok) {
                    d = cand.v[k];
                    v_copy(r, x3);
                    used = it;
                    break;
                }
            }
            donor[i] = d;
            if (xi) v_copy(xi + 3 * i, r);
            if (iters) iters[i] = used;
            if (n_cand) n_cand[i] = cand.n;
        }
        free(cand.v);
        free(stack.v);
    }
    if (!brute) bvh_free(&tree);
    free(boxes);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* the paper's filtered cut (Sec. 4.2, Alg. cp0, bboxdix, cp1, cp2)          */
/* ------------------------------------------------------------------------ */
/* Element corners in the order i = ia + 2 ib + 4 ic (ia, ib, ic in {0, 1}),
 * i.e. lattice nodes a + 3b + 9c with a, b, c in {0, 2}. */
static const int hx_corner[8] = {0, 2, 6, 8, 18, 20, 24, 26};

/* Eigenvectors (columns of V) of the symmetric 3x3 matrix A by the cyclic
 * Jacobi method: 8 sweeps over the planes (0,1), (0,2), (1,2); each rotation
 * zeroes A[p][q] (Numerical Recipes' angle choice, the smaller rotation). */
static void hx_jacobi(double *A, double *V)
{
    static const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 8; ++sweep)
        for (int r = 0; r < 3; ++r) {
            const int p = P[r], q = Q[r];
            const double apq = A[3 * p + q];
            if (apq == 0.0) continue;
            const double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
            double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
            if (theta < 0.0) t = -t;
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            for (int k = 0; k < 3; ++k) {
                const double akp = A[3 * k + p], akq = A[3 * k + q];
                A[3 * k + p] = c * akp - s * akq;
                A[3 * k + q] = s * akp + c * akq;
            }
            for (int k = 0; k < 3; ++k) {
                const double apk = A[3 * p + k], aqk = A[3 * q + k];
                A[3 * p + k] = c * apk - s * aqk;
                A[3 * q + k] = s * apk + c * aqk;
            }
            for (int k = 0; k < 3; ++k) {
                const double vkp = V[3 * k + p], vkq = V[3 * k + q];
                V[3 * k + p] = c * vkp - s * vkq;
                V[3 * k + q] = s * vkp + c * vkq;
            }
        }
}

static double hx_rot(const double *R, int r, const double *x)
{
    return (R[3 * r] * x[0] + R[3 * r + 1] * x[1]) + R[3 * r + 2] * x[2];
}

/* Element OBB from its corner nodes: centroid, axes R (rows: eigenvectors of
 * the corner covariance), extents B = (lo0 lo1 lo2 hi0 hi1 hi2) of the
 * corners along R.  obb: cg[3], R[9], B[6]. */
static void hx_obb(const double *X /* 27 nodes xyz */, double *obb)
{
    double cg[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 8; ++i)
        for (int d = 0; d < 3; ++d) cg[d] += X[3 * hx_corner[i] + d];
    for (int d = 0; d < 3; ++d) cg[d] *= 0.125;
    double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, V[9];
    for (int i = 0; i < 8; ++i) {
        double dv[3];
        for (int d = 0; d < 3; ++d) dv[d] = X[3 * hx_corner[i] + d] - cg[d];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) A[3 * j + k] += dv[j] * dv[k];
    }
    for (int k = 0; k < 9; ++k) A[k] *= 0.125;
    hx_jacobi(A, V);
    double *R = obb + 3, *B = obb + 12;
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) R[3 * r + j] = V[3 * j + r];
    for (int r = 0; r < 3; ++r) {
        B[r] = INFINITY;
        B[3 + r] = -INFINITY;
    }
    for (int i = 0; i < 8; ++i)
        for (int r = 0; r < 3; ++r) {
            const double v = hx_rot(R, r, X + 3 * hx_corner[i]);
            B[r] = fmin(B[r], v);
            B[3 + r] = fmax(B[3 + r], v);
        }
    for (int d = 0; d < 3; ++d) obb[d] = cg[d];
}

void orc_hx_obb(const double *X, double *obb) { hx_obb(X, obb); }

/* Alg. bboxdix (its loop read as i = 0, 1, 2 over a 6-vector box) */
double orc_hx_bbox_dist(const double *B1, const double *B2)
{
    double D = 0.0;
    for (int i = 0; i < 3; ++i)
        if (B1[i + 3] < B2[i] || B2[i + 3] < B1[i]) {
            const double d = fmax(B2[i] - B1[i + 3], B1[i] - B2[i + 3]);
            D += d * d;
        }
    return sqrt(D);
}

/* centroid of a posed face's corner nodes 0, 2, 6, 8 */
static void hx_face_cg(const double *P /* 9 nodes */, double *cg)
{
    for (int d = 0; d < 3; ++d) cg[d] = (((P[d] + P[6 + d]) + P[18 + d]) + P[24 + d]) * 0.25;
}

/* Alg. cp0: approximate element-face distance */
static double hx_approx(const double *obb, const double *P)
{
    const double *cg = obb, *R = obb + 3, *Be = obb + 12;
    double Bf[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    static const int fc[4] = {0, 2, 6, 8};
    for (int k = 0; k < 4; ++k)
        for (int r = 0; r < 3; ++r) {
            const double v = hx_rot(R, r, P + 3 * fc[k]);
            Bf[r] = fmin(Bf[r], v);
            Bf[3 + r] = fmax(Bf[3 + r], v);
        }
    double fcg[3];
    hx_face_cg(P, fcg);
    const double dx = fcg[0] - cg[0], dy = fcg[1] - cg[1], dz = fcg[2] - cg[2];
    const double dxc = sqrt((dx * dx + dy * dy) + dz * dz);
    return 0.01 * dxc + orc_hx_bbox_dist(Bf, Be);
}

typedef struct {
    double d;
    int64_t f;
    int c;
} hx_cand;

/* keep the k smallest (d, f) of a list in ascending order */
static void hx_keep(hx_cand *list, int *n, int k, hx_cand x)
{
    if (*n == k && !(x.d < list[k - 1].d || (x.d == list[k - 1].d && x.f < list[k - 1].f))) return;
    int i = *n < k ? (*n)++ : k - 1;
    while (i > 0 && (x.d < list[i - 1].d || (x.d == list[i - 1].d && x.f < list[i - 1].f))) {
        list[i] = list[i - 1];
        --i;
    }
    list[i] = x;
}

/* faces of an element touching corner c, in the order xi, eta, zeta */
static void hx_corner_faces(int c, int *fl)
{
    fl[0] = (c & 1) ? 1 : 0;
    fl[1] = (c & 2) ? 3 : 2;
    fl[2] = (c & 4) ? 5 : 4;
}

/* Alg. cp1: nearest element corner to the face centroid, then the minimum
 * distance between the linear triangles of the 3 element faces at that
 * corner and of the face's corner quad. */
static double hx_pass1(const double *X, const double *P, int *corner)
{
    double fcg[3];
    hx_face_cg(P, fcg);
    double dmin = INFINITY;
    int c = 0;
    for (int i = 0; i < 8; ++i) {
        const double *x = X + 3 * hx_corner[i];
        const double dx = x[0] - fcg[0], dy = x[1] - fcg[1], dz = x[2] - fcg[2];
        const double D = sqrt((dx * dx + dy * dy) + dz * dz);
        if (D < dmin) {
            dmin = D;
            c = i;
        }
    }
    int fl[3];
    hx_corner_faces(c, fl);
    double TF[2][9];
    static const int ft[2][3] = {{0, 2, 8}, {0, 8, 6}};
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 3; ++k) v_copy(TF[j] + 3 * k, P + 3 * ft[j][k]);
    dmin = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const int q00 = face_node(fl[a], 0, 0), q20 = face_node(fl[a], 2, 0), q22 = face_node(fl[a], 2, 2),
                  q02 = face_node(fl[a], 0, 2);
        const int et[2][3] = {{q00, q20, q22}, {q00, q22, q02}};
        for (int i = 0; i < 2; ++i) {
            double TC[9];
            for (int k = 0; k < 3; ++k) v_copy(TC + 3 * k, X + 3 * et[i][k]);
            for (int j = 0; j < 2; ++j) {
                const double D = orc_tri_tri(TC, TF[j], NULL, NULL);
                if (D < dmin) dmin = D;
            }
        }
    }
    if (dmin < TOL_HIT) dmin = 0.0;
    *corner = c;
    return dmin;
}

/* One element through the filtered cut: returns 1 for a hole.  *hit_out: the
 * element was found intersected (a pass-2 distance below the tolerance). */
static int hx_classify(const double *X, const surf_t *S, const double *Pposed /* n_face x 27 */, int kind,
                       int nf1, int nf2, hx_cand *l1, hx_cand *l2, int8_t *hit_out)
{
    double obb[18];
    hx_obb(X, obb);
    int n1 = 0;
    for (int64_t f = 0; f < S->n_face; ++f) {
        hx_cand x = {hx_approx(obb, Pposed + 27 * f), f, 0};
        hx_keep(l1, &n1, nf1, x);
    }
    int n2 = 0;
    for (int k = 0; k < n1; ++k) {
        int c;
        const double D = hx_pass1(X, Pposed + 27 * l1[k].f, &c);
        hx_cand x = {D, l1[k].f, c};
        hx_keep(l2, &n2, nf2, x);
    }
    /* Alg. cp2 over the element's lattice triangles at the kept corner */
    double et[48 * 9];
    tris_from_elem(X, et);
    double best = INFINITY;
    int hit = 0;
    for (int k = 0; k < n2 && !hit; ++k) {
        int fl[3];
        hx_corner_faces(l2[k].c, fl);
        const int64_t f = l2[k].f;
        for (int a = 0; a < 3 && !hit; ++a)
            for (int tl = 0; tl < 8 && !hit; ++tl)
                for (int s = 0; s < 8; ++s) {
                    const double D = orc_tri_tri(et + 9 * (8 * fl[a] + tl), S->tris + 72 * f + 9 * s, NULL, NULL);
                    if (D < TOL_HIT) {
                        hit = 1;
                        break;
                    }
                    if (D < best) best = D;
                }
    }
    if (hit_out) *hit_out = (int8_t)hit;
    if (hit) return kind == 0;
    /* nearest pair and its tie set (reading of the normal averaging) */
    const double thr = best * (1.0 + TIE_REL);
    tie_rec b1, b2;
    b1.valid = b2.valid = 0;
    for (int k = 0; k < n2; ++k) {
        int fl[3];
        hx_corner_faces(l2[k].c, fl);
        const int64_t f = l2[k].f;
        for (int a = 0; a < 3; ++a)
            for (int tl = 0; tl < 8; ++tl)
                for (int s = 0; s < 8; ++s) {
                    double pa[3], pb[3];
                    const int t = 8 * fl[a] + tl;
                    const double D = orc_tri_tri(et + 9 * t, S->tris + 72 * f + 9 * s, pa, pb);
                    if (D > thr) continue;
                    tie_rec r;
                    v_sub(pa, pb, r.v);
                    const double L = sqrt(v_dot(r.v, r.v));
                    v_copy(r.n, S->tnrm + 24 * f + 3 * s);
                    r.dot = L > 0.0 ? v_dot(r.v, r.n) / L : 0.0;
                    r.absdot = fabs(r.dot);
                    r.f = f;
                    r.s = s;
                    r.t = t;
                    r.valid = 1;
                    tie_offer(&b1, &b2, &r);
                }
    }
    double sgn = b1.dot;
    if (b2.valid && b1.absdot - b2.absdot <= TIE_DOT && (b1.dot > 0.0) != (b2.dot > 0.0)) {
        const double nn[3] = {b1.n[0] + b2.n[0], b1.n[1] + b2.n[1], b1.n[2] + b2.n[2]};
        sgn = v_dot(b1.v, nn);
    }
    return sgn < 0.0;
}

int orc_cut_heuristic(const double *gnodes, const int32_t *gconn, int64_t n_elem, const double *snodes,
                      int64_t n_snodes, const int32_t *sconn, int64_t n_face, const double *pose, int kind, int nf1,
                      int nf2, int n_threads, int8_t *status, int8_t *hit)
{
    if (nf1 < 1 || nf2 < 1) return -1;
    if (nf1 > n_face) nf1 = (int)n_face;
    if (nf2 > nf1) nf2 = nf1;
    surf_t S;
    surf_build(&S, snodes, n_snodes, sconn, n_face, pose, 0);
    double *Pp = (double *)malloc(sizeof(double) * 27 * (size_t)n_face + 8);
    for (int64_t f = 0; f < n_face; ++f)
        for (int k = 0; k < 9; ++k) pose_point(pose, snodes + 3 * (int64_t)sconn[f * 9 + k], Pp + 27 * f + 3 * k);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        hx_cand *l1 = (hx_cand *)malloc(sizeof(hx_cand) * (size_t)nf1);
        hx_cand *l2 = (hx_cand *)malloc(sizeof(hx_cand) * (size_t)nf2);
#pragma omp for schedule(dynamic, 16)
        for (int64_t e = 0; e < n_elem; ++e) {
            double X[81], box[6];
            elem_nodes(gnodes, gconn, e, X);
            box_of(X, 27, box);
            /* filter: elements whose node box misses the surface's node box
             * (grown by the hit tolerance) lie outside the surface */
            int near = 1;
            for (int d = 0; d < 3; ++d)
                if (box[3 + d] < S.sbox[d] - TOL_HIT || box[d] > S.sbox[3 + d] + TOL_HIT) near = 0;
            int8_t h = 0;
            const int hole = near ? hx_classify(X, &S, Pp, kind, nf1, nf2, l1, l2, &h) : 0;
            status[e] = hole ? 0 : 1;
            if (hit) hit[e] = h;
        }
        free(l1);
        free(l2);
    }
    free(Pp);
    surf_free(&S);
    return 0;
}

/* The kept lists of one element (for the pins): the nf1 faces of smallest
 * approximate distance (l1, with their distances d1) and the nf2 of those
 * with the smallest first-pass distance (l2, d2, kept corner c2). */
int orc_hx_lists(const double *X, const double *snodes, const int32_t *sconn, int64_t n_face, const double *pose,
                 int nf1, int nf2, int64_t *l1, double *d1, int64_t *l2, double *d2, int32_t *c2)
{
    if (nf1 < 1 || nf2 < 1 || nf1 > n_face || nf2 > nf1) return -1;
    double *Pp = (double *)malloc(sizeof(double) * 27 * (size_t)n_face + 8);
    hx_cand *a = (hx_cand *)malloc(sizeof(hx_cand) * (size_t)nf1);
    hx_cand *b = (hx_cand *)malloc(sizeof(hx_cand) * (size_t)nf2);
    for (int64_t f = 0; f < n_face; ++f)
        for (int k = 0; k < 9; ++k) pose_point(pose, snodes + 3 * (int64_t)sconn[f * 9 + k], Pp + 27 * f + 3 * k);
    double obb[18];
    hx_obb(X, obb);
    int n1 = 0, n2 = 0;
    for (int64_t f = 0; f < n_face; ++f) {
        hx_cand x = {hx_approx(obb, Pp + 27 * f), f, 0};
        hx_keep(a, &n1, nf1, x);
    }
    for (int k = 0; k < n1; ++k) {
        int c;
        const double D = hx_pass1(X, Pp + 27 * a[k].f, &c);
        hx_cand x = {D, a[k].f, c};
        hx_keep(b, &n2, nf2, x);
        l1[k] = a[k].f;
        d1[k] = a[k].d;
    }
    for (int k = 0; k < n2; ++k) {
        l2[k] = b[k].f;
        d2[k] = b[k].d;
        c2[k] = b[k].c;
    }
    free(Pp);
    free(a);
    free(b);
    return 0;
}
