// FP64 device geometry on the linearised (triangulated) curved faces.
//
// * the lattice triangles of a surface face and of an element's boundary
//   (Fig. quadsplit: each 2x2 sub-quad split along its (m,n)-(m+1,n+1)
//   diagonal);
// * closest point of a triangle to a point (Voronoi-region classification of
//   the point against the triangle's vertices, edges and face);
// * squared distance of two segments (clamped stationary point);
// * the intersection predicate "two triangles are closer than tol", decided
//   by plane separation, edge/triangle crossing (signed volumes) and the
//   vertex-face / edge-edge distances that realise the distance of disjoint
//   triangles (Sec. 4.2, Alg. cp1/cp2: tol = 1e-7);
// * the distance of two triangles with a closest pair;
// * +x ray / triangle crossing with a symbolic perturbation of the ray
//   origin, so that a ray through shared vertices or edges of a watertight
//   triangulation is counted exactly once (parity classification).
#pragma once

#include "dev_common.h"

namespace oc {

// triangle s of a face stored x[9], y[9], z[9]
__device__ inline void face_tri(const double *P, int s, d3 *T)
{
    int uv[6];
    quad_tri_uv((s >> 1) & 1, s >> 2, s & 1, uv);
    for (int k = 0; k < 3; ++k) {
        int nd = uv[2 * k] + 3 * uv[2 * k + 1];
        T[k] = mk(P[nd], P[9 + nd], P[18 + nd]);
    }
}

// boundary triangle t (0..47) of an element stored x[27], y[27], z[27]
__device__ inline void elem_tri(const double *X, int t, d3 *T)
{
    int uv[6];
    quad_tri_uv((t >> 1) & 1, (t >> 2) & 1, t & 1, uv);
    for (int k = 0; k < 3; ++k) {
        int nd = elem_face_node(t >> 3, uv[2 * k], uv[2 * k + 1]);
        T[k] = mk(X[nd], X[27 + nd], X[54 + nd]);
    }
}

__device__ inline double clamp01(double v) { return fmin(fmax(v, 0.0), 1.0); }

// Closest point of triangle abc to p by Voronoi regions of the vertices,
// edges and face (the published method of C. Ericson, Real-Time Collision
// Detection, Morgan Kaufmann 2005, Sec. 5.1.5, written here in FP64).
__device__ inline d3 closest_on_tri(d3 p, d3 a, d3 b, d3 c)
{
    d3 ab = b - a, ac = c - a, ap = p - a;
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return a;
    d3 bp = p - b;
    double d3v = dot(ab, bp), d4 = dot(ac, bp);
    if (d3v >= 0.0 && d4 <= d3v) return b;
    double vc = d1 * d4 - d3v * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3v <= 0.0) return a + ab * (d1 / (d1 - d3v));
    d3 cp = p - c;
    double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) return c;
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return a + ac * (d2 / (d2 - d6));
    double va = d3v * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3v) >= 0.0 && (d5 - d6) >= 0.0) {
        double w = (d4 - d3v) / ((d4 - d3v) + (d5 - d6));
        return b + (c - b) * w;
    }
    double den = 1.0 / (va + vb + vc);
    return a + ab * (vb * den) + ac * (vc * den);
}

// Squared distance of segments [p1, q1] and [p2, q2]: the stationary point
// of the two-parameter distance, clamped to the unit square one parameter at
// a time (Ericson, Real-Time Collision Detection, Sec. 5.1.9).
__device__ inline double seg_seg_d2(d3 p1, d3 q1, d3 p2, d3 q2)
{
    d3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
    double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
    double s, t;
    if (a <= 0.0 && e <= 0.0) return dot(r, r);
    if (a <= 0.0) {
        s = 0.0;
        t = clamp01(f / e);
    } else {
        double c = dot(d1, r);
        if (e <= 0.0) {
            t = 0.0;
            s = clamp01(-c / a);
        } else {
            double b = dot(d1, d2), den = a * e - b * b;
            s = den > 0.0 ? clamp01((b * f - c * e) / den) : 0.0;
            t = (b * s + f) / e;
            if (t < 0.0) {
                t = 0.0;
                s = clamp01(-c / a);
            } else if (t > 1.0) {
                t = 1.0;
                s = clamp01((b - c) / a);
            }
        }
    }
    d3 w = (p1 + d1 * s) - (p2 + d2 * t);
    return dot(w, w);
}

__device__ inline double triple(d3 a, d3 b, d3 c) { return dot(a, cross(b, c)); }

// Segment pq meets triangle abc at a point off the triangle's plane-coplanar
// case: endpoints on opposite sides (or on) the plane and the line through
// them passing inside the triangle (three signed volumes of one sign).
__device__ inline bool seg_meets_tri(d3 p, d3 q, d3 a, d3 b, d3 c)
{
    d3 n = cross(b - a, c - a);
    double sp = dot(n, p - a), sq = dot(n, q - a);
    if ((sp > 0.0 && sq > 0.0) || (sp < 0.0 && sq < 0.0)) return false;
    if (sp == 0.0 && sq == 0.0) return false;
    d3 pq = q - p, pa = a - p, pb = b - p, pc = c - p;
    double u = triple(pq, pc, pb), v = triple(pq, pa, pc), w = triple(pq, pb, pa);
    bool pos = u >= 0.0 && v >= 0.0 && w >= 0.0;
    bool neg = u <= 0.0 && v <= 0.0 && w <= 0.0;
    return (pos || neg) && !(u == 0.0 && v == 0.0 && w == 0.0);
}

// True when some point of triangle A and some point of triangle B are
// closer than tol.
__device__ inline bool tri_tri_within(const d3 *A, const d3 *B, double tol)
{
    // a plane at distance >= tol from every vertex of the other triangle
    // separates them by at least tol
    d3 nb = cross(B[1] - B[0], B[2] - B[0]);
    double lb = sqrt(dot(nb, nb));
    if (lb > 0.0) {
        double s0 = dot(nb, A[0] - B[0]), s1 = dot(nb, A[1] - B[0]), s2 = dot(nb, A[2] - B[0]);
        double lim = tol * lb;
        if (fmin(s0, fmin(s1, s2)) >= lim || fmax(s0, fmax(s1, s2)) <= -lim) return false;
    }
    d3 na = cross(A[1] - A[0], A[2] - A[0]);
    double la = sqrt(dot(na, na));
    if (la > 0.0) {
        double s0 = dot(na, B[0] - A[0]), s1 = dot(na, B[1] - A[0]), s2 = dot(na, B[2] - A[0]);
        double lim = tol * la;
        if (fmin(s0, fmin(s1, s2)) >= lim || fmax(s0, fmax(s1, s2)) <= -lim) return false;
    }
    for (int k = 0; k < 3; ++k) {
        int k1 = k == 2 ? 0 : k + 1;
        if (seg_meets_tri(A[k], A[k1], B[0], B[1], B[2])) return true;
        if (seg_meets_tri(B[k], B[k1], A[0], A[1], A[2])) return true;
    }
    double tol2 = tol * tol;
    for (int k = 0; k < 3; ++k) {
        d3 q = closest_on_tri(A[k], B[0], B[1], B[2]);
        d3 w = A[k] - q;
        if (dot(w, w) < tol2) return true;
        q = closest_on_tri(B[k], A[0], A[1], A[2]);
        w = B[k] - q;
        if (dot(w, w) < tol2) return true;
    }
    for (int i = 0; i < 3; ++i) {
        int i1 = i == 2 ? 0 : i + 1;
        for (int j = 0; j < 3; ++j) {
            int j1 = j == 2 ? 0 : j + 1;
            if (seg_seg_d2(A[i], A[i1], B[j], B[j1]) < tol2) return true;
        }
    }
    return false;
}

// Closest points of segments [p1, q1] and [p2, q2] (clamped stationary
// point, Ericson, Real-Time Collision Detection, Sec. 5.1.9); returns the
// squared distance.
__device__ inline double seg_seg_cp(d3 p1, d3 q1, d3 p2, d3 q2, d3 &c1, d3 &c2)
{
    d3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
    double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
    double s = 0.0, t = 0.0;
    if (a <= 0.0 && e <= 0.0) {
        s = t = 0.0;
    } else if (a <= 0.0) {
        t = clamp01(f / e);
    } else {
        double c = dot(d1, r);
        if (e <= 0.0) {
            s = clamp01(-c / a);
        } else {
            double b = dot(d1, d2), den = a * e - b * b;
            s = den > 0.0 ? clamp01((b * f - c * e) / den) : 0.0;
            t = (b * s + f) / e;
            if (t < 0.0) {
                t = 0.0;
                s = clamp01(-c / a);
            } else if (t > 1.0) {
                t = 1.0;
                s = clamp01((b - c) / a);
            }
        }
    }
    c1 = p1 + d1 * s;
    c2 = p2 + d2 * t;
    d3 w = c1 - c2;
    return dot(w, w);
}

// Distance of triangles A and B with a closest pair (pa on A, pb on B): zero
// (at the crossing point) when an edge of one crosses the other, else the
// least of the six vertex-triangle and nine edge-edge distances, which
// realise the distance of disjoint triangles.
__device__ inline double tri_tri_dist(const d3 *A, const d3 *B, d3 &pa, d3 &pb)
{
    for (int pass = 0; pass < 2; ++pass) {
        const d3 *P = pass ? B : A, *Q = pass ? A : B;
        d3 n = cross(Q[1] - Q[0], Q[2] - Q[0]);
        for (int k = 0; k < 3; ++k) {
            const int k1 = k == 2 ? 0 : k + 1;
            if (seg_meets_tri(P[k], P[k1], Q[0], Q[1], Q[2])) {
                double sp = dot(n, P[k] - Q[0]), sq = dot(n, P[k1] - Q[0]);
                d3 x = P[k] + (P[k1] - P[k]) * (sp / (sp - sq));
                pa = x;
                pb = x;
                return 0.0;
            }
        }
    }
    double best = INFINITY;
    for (int k = 0; k < 3; ++k) {
        d3 q = closest_on_tri(A[k], B[0], B[1], B[2]);
        d3 w = A[k] - q;
        double d = dot(w, w);
        if (d < best) {
            best = d;
            pa = A[k];
            pb = q;
        }
        q = closest_on_tri(B[k], A[0], A[1], A[2]);
        w = B[k] - q;
        d = dot(w, w);
        if (d < best) {
            best = d;
            pa = q;
            pb = B[k];
        }
    }
    for (int i = 0; i < 3; ++i) {
        const int i1 = i == 2 ? 0 : i + 1;
        for (int j = 0; j < 3; ++j) {
            const int j1 = j == 2 ? 0 : j + 1;
            d3 c1, c2;
            const double d = seg_seg_cp(A[i], A[i1], B[j], B[j1], c1, c2);
            if (d < best) {
                best = d;
                pa = c1;
                pb = c2;
            }
        }
    }
    return sqrt(best);
}

// 2D edge function of directed edge (a, b) at q = (py, pz) in the (y, z)
// projection.  Evaluated with the same operation order for every triangle,
// without contraction, so the two triangles sharing an edge get exactly
// opposite values.
__device__ inline double edge_fn(double ay, double az, double by, double bz, double py, double pz)
{
#pragma clang fp contract(off)
    double p1 = (ay - py) * (bz - pz);
    double p2 = (az - pz) * (by - py);
    return p1 - p2;
}

// Sign of the edge function at the origin perturbed by (eps, eps^2):
// first order a.z - b.z, second order b.y - a.y.
__device__ inline int edge_sign(double e, double ay, double az, double by, double bz)
{
    if (e > 0.0) return 1;
    if (e < 0.0) return -1;
    if (az != bz) return az > bz ? 1 : -1;
    if (by != ay) return by > ay ? 1 : -1;
    return 0;
}

// Does the ray {p + s e_x, s > 0} (origin perturbed as above) cross triangle abc?
__device__ inline int ray_x_crosses(d3 p, d3 a, d3 b, d3 c)
{
    double e0 = edge_fn(a.y, a.z, b.y, b.z, p.y, p.z);
    double e1 = edge_fn(b.y, b.z, c.y, c.z, p.y, p.z);
    double e2 = edge_fn(c.y, c.z, a.y, a.z, p.y, p.z);
    int s0 = edge_sign(e0, a.y, a.z, b.y, b.z);
    int s1 = edge_sign(e1, b.y, b.z, c.y, c.z);
    int s2 = edge_sign(e2, c.y, c.z, a.y, a.z);
    if (s0 == 0 || s0 != s1 || s1 != s2) return 0;
    double S = e0 + e1 + e2;
    if (S == 0.0) return 0;
    double x = (e1 * a.x + e2 * b.x + e0 * c.x) / S;
    return x > p.x ? 1 : 0;
}

}  // namespace oc
