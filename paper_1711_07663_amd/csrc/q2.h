// The quadratic isoparametric map of eq. reftophys (K = 2): equispaced
// Lagrange basis on the nodes -1, 0, 1 per reference axis, node order
// a + 3b + 9c, element coordinates stored as x[27], y[27], z[27].
// Sum-factorised by node rows; shared by the donor search and the receptor
// point kernels.
#pragma once

#include "dev_common.h"

namespace oc {

__device__ inline void lag2(double s, double *l, double *dl)
{
    l[0] = 0.5 * s * (s - 1.0);
    l[1] = 1.0 - s * s;
    l[2] = 0.5 * s * (s + 1.0);
    dl[0] = s - 0.5;
    dl[1] = -2.0 * s;
    dl[2] = s + 0.5;
}

__device__ inline double pick3(int i, double a, double b, double c) { return i == 0 ? a : (i == 1 ? b : c); }

// One node row (fixed eta, zeta index r) of the sum-factorised map: adds its
// share of x(xi) and, with WITH_J, of J = dx/dxi.
template <bool WITH_J>
__device__ inline void q2_row(const double *__restrict__ X, int r, const double *la, const double *da,
                              const double *lb, const double *db, const double *lc, const double *dc, double *acc)
{
    const int b = r % 3, c = r / 3;
    const double wb = pick3(b, lb[0], lb[1], lb[2]), wc = pick3(c, lc[0], lc[1], lc[2]);
    const double w = wb * wc;
    const double *R = X + 3 * r;
    const double x0 = R[0], x1 = R[1], x2 = R[2];
    const double y0 = R[27], y1 = R[28], y2 = R[29];
    const double z0 = R[54], z1 = R[55], z2 = R[56];
    const double ux = x0 * la[0] + x1 * la[1] + x2 * la[2];
    const double uy = y0 * la[0] + y1 * la[1] + y2 * la[2];
    const double uz = z0 * la[0] + z1 * la[1] + z2 * la[2];
    acc[0] += ux * w;
    acc[1] += uy * w;
    acc[2] += uz * w;
    if (WITH_J) {
        const double wdb = pick3(b, db[0], db[1], db[2]) * wc;
        const double wdc = wb * pick3(c, dc[0], dc[1], dc[2]);
        const double vx = x0 * da[0] + x1 * da[1] + x2 * da[2];
        const double vy = y0 * da[0] + y1 * da[1] + y2 * da[2];
        const double vz = z0 * da[0] + z1 * da[1] + z2 * da[2];
        acc[3] += vx * w; acc[4] += ux * wdb; acc[5] += ux * wdc;
        acc[6] += vy * w; acc[7] += uy * wdb; acc[8] += uy * wdc;
        acc[9] += vz * w; acc[10] += uz * wdb; acc[11] += uz * wdc;
    }
}

// Component d of the same map: C = the element's 27 values of coordinate
// d; returns x_d(xi) and row d of J, contracting one reference axis at a
// time (xi, then eta, then zeta: 93 multiply-adds instead of the 117 of the
// row form; the rounding differs from q2_map in the last bits).
__device__ inline void q2_map_comp(const double *C, const double *xi, double &xd, double *Jd)
{
    double la[3], da[3], lb[3], db[3], lc[3], dc[3];
    lag2(xi[0], la, da);
    lag2(xi[1], lb, db);
    lag2(xi[2], lc, dc);
    // per zeta level c: along xi, the value and xi-derivative of its three
    // node rows, then along eta
    double U[3], Ue[3], V[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double u[3], v[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double *R = C + 9 * c + 3 * b;
            u[b] = R[0] * la[0] + R[1] * la[1] + R[2] * la[2];
            v[b] = R[0] * da[0] + R[1] * da[1] + R[2] * da[2];
        }
        U[c] = u[0] * lb[0] + u[1] * lb[1] + u[2] * lb[2];
        Ue[c] = u[0] * db[0] + u[1] * db[1] + u[2] * db[2];
        V[c] = v[0] * lb[0] + v[1] * lb[1] + v[2] * lb[2];
    }
    // along zeta
    xd = U[0] * lc[0] + U[1] * lc[1] + U[2] * lc[2];
    Jd[0] = V[0] * lc[0] + V[1] * lc[1] + V[2] * lc[2];
    Jd[1] = Ue[0] * lc[0] + Ue[1] * lc[1] + Ue[2] * lc[2];
    Jd[2] = U[0] * dc[0] + U[1] * dc[1] + U[2] * dc[2];
}

// The same polynomial in the monomial basis: one coordinate's 27 node values
// (order a + 3b + 9c) are replaced in place by the coefficients of
// xi^a eta^b zeta^c.  Per axis, the values v0, v1, v2 at -1, 0, 1 of a
// quadratic are v1 + s (v2 - v0) / 2 + s^2 ((v0 + v2) / 2 - v1).  The
// constant coefficient is the centre node itself.
__device__ inline void q2_mono(double *M)
{
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int S = ax == 0 ? 1 : (ax == 1 ? 3 : 9);
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            // the nine lines along axis ax: offsets over the other two axes
            const int u = l % 3, v = l / 3;
            const int o = ax == 0 ? 3 * u + 9 * v : (ax == 1 ? u + 9 * v : u + 3 * v);
            const double v0 = M[o], v1 = M[o + S], v2 = M[o + 2 * S];
            M[o] = v1;
            M[o + S] = 0.5 * (v2 - v0);
            M[o + 2 * S] = 0.5 * (v0 + v2) - v1;
        }
    }
}

// Value and gradient of one coordinate from its monomial coefficients M
// (q2_mono) by nested Horner steps along xi, eta, zeta: 49 fused
// multiply-adds; each derivative reuses the inner Horner term
// (p' = h + s m2 where p = m0 + s h, h = m1 + s m2).
__device__ inline void q2_mono_comp(const double *M, const double *xi, double &xd, double *Jd)
{
    const double s = xi[0], t = xi[1], u = xi[2];
    double Q[3], Qe[3], Sx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double P[3], D[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double *m = M + 3 * b + 9 * c;
            const double h = fma(s, m[2], m[1]);
            P[b] = fma(s, h, m[0]);
            D[b] = fma(s, m[2], h);
        }
        const double hq = fma(t, P[2], P[1]);
        Q[c] = fma(t, hq, P[0]);
        Qe[c] = fma(t, P[2], hq);
        Sx[c] = fma(t, fma(t, D[2], D[1]), D[0]);
    }
    const double hz = fma(u, Q[2], Q[1]);
    xd = fma(u, hz, Q[0]);
    Jd[0] = fma(u, fma(u, Sx[2], Sx[1]), Sx[0]);
    Jd[1] = fma(u, fma(u, Qe[2], Qe[1]), Qe[0]);
    Jd[2] = fma(u, Q[2], hz);
}

// x(xi) and J = dx/dxi of an element stored as x[27], y[27], z[27].  With
// STREAM the nine node rows are read one at a time (X in global memory, the
// 81 coordinates never resident together); otherwise X is a register copy
// and the rows are unrolled.  Both sum in the same order.
template <bool WITH_J, bool STREAM>
__device__ inline void q2_map(const double *__restrict__ X, const double *xi, double *x, double *J)
{
    double la[3], da[3], lb[3], db[3], lc[3], dc[3];
    lag2(xi[0], la, da);
    lag2(xi[1], lb, db);
    lag2(xi[2], lc, dc);
    double acc[12] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (STREAM) {
#pragma unroll 1
        for (int r = 0; r < 9; ++r) q2_row<WITH_J>(X, r, la, da, lb, db, lc, dc, acc);
    } else {
#pragma unroll
        for (int r = 0; r < 9; ++r) q2_row<WITH_J>(X, r, la, da, lb, db, lc, dc, acc);
    }
    x[0] = acc[0];
    x[1] = acc[1];
    x[2] = acc[2];
    if (WITH_J)
        for (int k = 0; k < 9; ++k) J[k] = acc[3 + k];
}

}  // namespace oc
