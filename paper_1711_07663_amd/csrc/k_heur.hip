// The paper's filtered cut (Sec. 4.2; Alg. cp0, bboxdix, cp1, cp2): the cut
// as the paper runs it, with its truncations N_F^1 (faces kept by
// approximate distance) and N_F^2 (faces kept by the linear first pass).
// It is an alternative to the exact cut, kept for comparison (speed, and
// the elements on which the truncations change the result).
//
//   k_hx_pose     posed face nodes (x[9], y[9], z[9] per face) and per-block
//                 surface boxes; k_hx_sbox reduces them
//   k_hx_filter   elements whose box meets the surface box (others lie
//                 outside the surface): wave-aggregated list
//   k_hx_obb      per listed element: corner centroid, corner covariance
//                 eigenvectors (cyclic Jacobi), extents along them
//   k_hx_approx   Alg. cp0 against every face, N_F^1 smallest per element:
//                 16 elements per block share LDS tiles of face corners;
//                 each of an element's 16 threads keeps a sorted register
//                 list, merged at the end; a face whose lower bound
//                 (centroid distance less both radii) exceeds the thread's
//                 current K-th distance is skipped, which changes nothing
//   k_hx_pass1    Alg. cp1 per (element, kept face): nearest corner, linear
//                 triangles of the three element faces at it
//   k_hx_keep2    N_F^2 smallest first-pass distances per element
//   k_hx_pass2    Alg. cp2 per element (one wavefront): lattice triangles at
//                 the kept corner; a pair within the tolerance is a hit,
//                 else the nearest pair's face normal decides the side, with
//                 the tie rule of the exact cut
//
// The approximate distances are evaluated without contraction in the
// operation order of the plain C implementation, so the N_F^1 selection is
// reproducible bit for bit.
#include <algorithm>
#include <string>
#include <vector>

#include "dev_common.h"
#include "dev_geom.h"

namespace oc {

constexpr int kHT = 256;
constexpr int kHxK1 = 32;          // largest N_F^1
constexpr int kHxK2 = 16;          // largest N_F^2
constexpr int kHxElems = 16;       // elements per k_hx_approx block
constexpr int kHxSub = kHT / kHxElems;
constexpr int kHxTile = 256;       // faces per LDS tile

__device__ inline d3 hx_pose(const Pose &p, double x, double y, double z)
{
#pragma clang fp contract(off)
    return d3{((p.r[0] * x + p.r[1] * y) + p.r[2] * z) + p.t[0], ((p.r[3] * x + p.r[4] * y) + p.r[5] * z) + p.t[1],
              ((p.r[6] * x + p.r[7] * y) + p.r[8] * z) + p.t[2]};
}

// posed face nodes, stored x[9], y[9], z[9] per face; partial box per block
__global__ __launch_bounds__(kHT) void k_hx_pose(const double *__restrict__ nodes, int64_t n_nodes,
                                                 const int32_t *__restrict__ conn, int64_t n_face,
                                                 const Pose *__restrict__ pose_dev, double *__restrict__ P,
                                                 double *__restrict__ part)
{
    const Pose pose = *pose_dev;
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (f < n_face) {
        for (int k = 0; k < 9; ++k) {
            const int id = conn[f * 9 + k];
            const d3 x = hx_pose(pose, nodes[id], nodes[n_nodes + id], nodes[2 * n_nodes + id]);
            P[f * 27 + k] = x.x;
            P[f * 27 + 9 + k] = x.y;
            P[f * 27 + 18 + k] = x.z;
            lo[0] = fmin(lo[0], x.x); hi[0] = fmax(hi[0], x.x);
            lo[1] = fmin(lo[1], x.y); hi[1] = fmax(hi[1], x.y);
            lo[2] = fmin(lo[2], x.z); hi[2] = fmax(hi[2], x.z);
        }
    }
    for (int d = 32; d >= 1; d >>= 1)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], d, 64));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], d, 64));
        }
    __shared__ double wb[kHT / 64][6];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            wb[w][a] = lo[a];
            wb[w][3 + a] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = wb[0][threadIdx.x];
        for (int k = 1; k < kHT / 64; ++k) v = threadIdx.x < 3 ? fmin(v, wb[k][threadIdx.x]) : fmax(v, wb[k][threadIdx.x]);
        part[blockIdx.x * 6 + threadIdx.x] = v;
    }
}

__global__ void k_hx_sbox(const double *__restrict__ part, int nb, double *__restrict__ sbox)
{
    const int a = threadIdx.x;
    if (a >= 6) return;
    double v = a < 3 ? INFINITY : -INFINITY;
    for (int b = 0; b < nb; ++b) v = a < 3 ? fmin(v, part[b * 6 + a]) : fmax(v, part[b * 6 + a]);
    sbox[a] = v;
}

// elements whose (outward FP32) box meets the surface box grown by the hit
// tolerance; the order of the list does not matter
__global__ __launch_bounds__(kHT) void k_hx_filter(const float *__restrict__ ebox, int64_t stride, int64_t n_elem,
                                                   const double *__restrict__ sbox, int32_t *__restrict__ list,
                                                   int32_t *__restrict__ count)
{
    const double t = kTolHit;
    const double s0 = sbox[0] - t, s1 = sbox[1] - t, s2 = sbox[2] - t, s3 = sbox[3] + t, s4 = sbox[4] + t,
                 s5 = sbox[5] + t;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n_elem; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = base + threadIdx.x;
        bool in = false;
        if (e < n_elem)
            in = (double)ebox[3 * stride + e] >= s0 && (double)ebox[e] <= s3 && (double)ebox[4 * stride + e] >= s1 &&
                 (double)ebox[stride + e] <= s4 && (double)ebox[5 * stride + e] >= s2 &&
                 (double)ebox[2 * stride + e] <= s5;
        const unsigned long long m = __ballot(in);
        const int lane = threadIdx.x & 63;
        int at = 0;
        if (m && lane == 0) at = atomicAdd(count, __popcll(m));
        at = __shfl(at, 0, 64);
        if (in) list[at + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)e;
    }
}

// corner node i = ia + 2 ib + 4 ic of an element stored x[27], y[27], z[27]
__device__ inline int hx_corner(int i) { return ((i & 1) ? 2 : 0) + ((i & 2) ? 6 : 0) + ((i & 4) ? 18 : 0); }

__device__ inline double hx_rot(const double *R, int r, double x, double y, double z)
{
#pragma clang fp contract(off)
    return (R[3 * r] * x + R[3 * r + 1] * y) + R[3 * r + 2] * z;
}

// Element OBB: centroid of the corners, eigenvectors of their covariance
// (cyclic Jacobi, 8 sweeps over the planes (0,1), (0,2), (1,2)) as the rows
// of R, extents of the corners along them.  Record: cg[3], R[9], B[6].
__global__ __launch_bounds__(kHT) void k_hx_obb(const double *__restrict__ enodes, const int32_t *__restrict__ list,
                                                const int32_t *__restrict__ count, double *__restrict__ obb)
{
#pragma clang fp contract(off)
    const int n = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double *X = enodes + (int64_t)list[i] * 81;
        double c[8][3];
        for (int k = 0; k < 8; ++k)
            for (int d = 0; d < 3; ++d) c[k][d] = X[27 * d + hx_corner(k)];
        double cg[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 8; ++k)
            for (int d = 0; d < 3; ++d) cg[d] += c[k][d];
        for (int d = 0; d < 3; ++d) cg[d] *= 0.125;
        double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        for (int k = 0; k < 8; ++k) {
            const double dv[3] = {c[k][0] - cg[0], c[k][1] - cg[1], c[k][2] - cg[2]};
            for (int j = 0; j < 3; ++j)
                for (int l = 0; l < 3; ++l) A[3 * j + l] += dv[j] * dv[l];
        }
        for (int k = 0; k < 9; ++k) A[k] *= 0.125;
        for (int sweep = 0; sweep < 8; ++sweep)
            for (int r = 0; r < 3; ++r) {
                const int p = r == 2 ? 1 : 0, q = r == 0 ? 1 : 2;
                const double apq = A[3 * p + q];
                if (apq == 0.0) continue;
                const double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[3 * k + p], akq = A[3 * k + q];
                    A[3 * k + p] = cs * akp - sn * akq;
                    A[3 * k + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[3 * p + k], aqk = A[3 * q + k];
                    A[3 * p + k] = cs * apk - sn * aqk;
                    A[3 * q + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[3 * k + p], vkq = V[3 * k + q];
                    V[3 * k + p] = cs * vkp - sn * vkq;
                    V[3 * k + q] = sn * vkp + cs * vkq;
                }
            }
        double *o = obb + (int64_t)i * 18;
        double R[9];
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < 3; ++j) R[3 * r + j] = V[3 * j + r];
        double B[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        for (int k = 0; k < 8; ++k)
            for (int r = 0; r < 3; ++r) {
                const double v = hx_rot(R, r, c[k][0], c[k][1], c[k][2]);
                B[r] = fmin(B[r], v);
                B[3 + r] = fmax(B[3 + r], v);
            }
        for (int d = 0; d < 3; ++d) o[d] = cg[d];
        for (int k = 0; k < 9; ++k) o[3 + k] = R[k];
        for (int k = 0; k < 6; ++k) o[12 + k] = B[k];
    }
}

// (d, f) before (e, g)
__device__ inline bool hx_less(double d, int f, double e, int g) { return d < e || (d == e && f < g); }

// Alg. cp0 for 16 elements per block: each element's 16 threads take every
// 16th face of each LDS tile and keep their K >= N_F^1 smallest (d, f),
// sorted; the element's N_F^1 smallest are merged from those lists.
template <int K>
__global__ __launch_bounds__(kHT) void k_hx_approx(const double *__restrict__ P, int64_t n_face,
                                                   const double *__restrict__ obb, const int32_t *__restrict__ count,
                                                   int nf1, int32_t *__restrict__ l1)
{
#pragma clang fp contract(off)
    __shared__ double sF[kHxTile][16];   // corners 0, 2, 6, 8 (x y z each), centroid, corner radius
    const int n = *count;
    const int j = threadIdx.x / kHxSub, sub = threadIdx.x % kHxSub;
    for (int base = blockIdx.x * kHxElems; base < n; base += gridDim.x * kHxElems) {
        const int i = base + j;
        const bool act = i < n;
        double o[18];
        for (int k = 0; k < 18; ++k) o[k] = act ? obb[(int64_t)i * 18 + k] : 0.0;
        // radius of the OBB about the rotated centroid: every point of the
        // box is within re of it
        double re = 0.0;
        for (int r = 0; r < 3; ++r) {
            const double c = hx_rot(o + 3, r, o[0], o[1], o[2]);
            const double h = fmax(fabs(o[12 + r] - c), fabs(o[15 + r] - c));
            re += h * h;
        }
        re = sqrt(re) * (1.0 + 1e-12);
        double Ld[K];
        int Lf[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            Ld[k] = INFINITY;
            Lf[k] = 0x7fffffff;
        }
        for (int64_t t0 = 0; t0 < n_face; t0 += kHxTile) {
            const int tn = (int)min((int64_t)kHxTile, n_face - t0);
            __syncthreads();
            for (int q = threadIdx.x; q < tn; q += blockDim.x) {
                const double *F = P + (t0 + q) * 27;
                const int cn[4] = {0, 2, 6, 8};
                for (int k = 0; k < 4; ++k) {
                    sF[q][3 * k] = F[cn[k]];
                    sF[q][3 * k + 1] = F[9 + cn[k]];
                    sF[q][3 * k + 2] = F[18 + cn[k]];
                }
                for (int d = 0; d < 3; ++d) sF[q][12 + d] = (((F[9 * d] + F[9 * d + 2]) + F[9 * d + 6]) + F[9 * d + 8]) * 0.25;
                double rf = 0.0;
                for (int k = 0; k < 4; ++k) {
                    const double ax = sF[q][3 * k] - sF[q][12], ay = sF[q][3 * k + 1] - sF[q][13],
                                 az = sF[q][3 * k + 2] - sF[q][14];
                    rf = fmax(rf, ax * ax + ay * ay + az * az);
                }
                sF[q][15] = sqrt(rf) * (1.0 + 1e-12);
            }
            __syncthreads();
            if (!act) continue;
            for (int q = sub; q < tn; q += kHxSub) {
                const double dx = sF[q][12] - o[0], dy = sF[q][13] - o[1], dz = sF[q][14] - o[2];
                const double dxc = sqrt((dx * dx + dy * dy) + dz * dz);
                // the rotated corner box lies within sqrt(3) rf of the rotated
                // face centroid, so the box distance is at least
                // dxc - re - sqrt(3) rf; a face whose bound exceeds this
                // thread's K-th distance cannot enter its list
                const double lb = 0.01 * dxc + fmax(0.0, dxc - re - 1.7320508075688774 * sF[q][15]);
                if (lb * (1.0 - 1e-12) > Ld[K - 1]) continue;
                double Bf[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
                for (int k = 0; k < 4; ++k)
                    for (int r = 0; r < 3; ++r) {
                        const double v = hx_rot(o + 3, r, sF[q][3 * k], sF[q][3 * k + 1], sF[q][3 * k + 2]);
                        Bf[r] = fmin(Bf[r], v);
                        Bf[3 + r] = fmax(Bf[3 + r], v);
                    }
                double D = 0.0;
                for (int a = 0; a < 3; ++a)
                    if (Bf[a + 3] < o[12 + a] || o[15 + a] < Bf[a]) {
                        const double g = fmax(o[12 + a] - Bf[a + 3], Bf[a] - o[15 + a]);
                        D += g * g;
                    }
                const double dist = 0.01 * dxc + sqrt(D);
                int cf = (int)(t0 + q);
                double cd = dist;
                if (hx_less(cd, cf, Ld[K - 1], Lf[K - 1])) {
                    // bubble the candidate through the sorted list
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const bool sw = hx_less(cd, cf, Ld[k], Lf[k]);
                        const double td = Ld[k];
                        const int tf = Lf[k];
                        Ld[k] = sw ? cd : td;
                        Lf[k] = sw ? cf : tf;
                        cd = sw ? td : cd;
                        cf = sw ? tf : cf;
                    }
                }
            }
        }
        // merge the element's 16 lists: nf1 rounds of a 16-lane minimum
        for (int r = 0; r < nf1; ++r) {
            double bd = Ld[0];
            int bf = Lf[0], bl = sub;
            for (int d = kHxSub / 2; d >= 1; d >>= 1) {
                const double od = __shfl_xor(bd, d, kHxSub);
                const int of = __shfl_xor(bf, d, kHxSub), ol = __shfl_xor(bl, d, kHxSub);
                if (hx_less(od, of, bd, bf)) {
                    bd = od;
                    bf = of;
                    bl = ol;
                }
            }
            if (bl == sub) {
#pragma unroll
                for (int k = 0; k < K - 1; ++k) {
                    Ld[k] = Ld[k + 1];
                    Lf[k] = Lf[k + 1];
                }
                Ld[K - 1] = INFINITY;
                Lf[K - 1] = 0x7fffffff;
            }
            if (act && sub == 0) l1[(int64_t)i * nf1 + r] = bf;
        }
    }
}

// faces of an element touching corner c (xi, eta, zeta order)
__device__ inline void hx_corner_faces(int c, int *fl)
{
    fl[0] = (c & 1) ? 1 : 0;
    fl[1] = (c & 2) ? 3 : 2;
    fl[2] = (c & 4) ? 5 : 4;
}

__device__ inline d3 hx_node(const double *X, int k) { return mk(X[k], X[27 + k], X[54 + k]); }
__device__ inline d3 hx_fnode(const double *F, int k) { return mk(F[k], F[9 + k], F[18 + k]); }

// Alg. cp1 for (element i, kept face k)
__global__ __launch_bounds__(kHT) void k_hx_pass1(const double *__restrict__ enodes, const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ count, const double *__restrict__ P,
                                                  int nf1, const int32_t *__restrict__ l1, double *__restrict__ d1,
                                                  int8_t *__restrict__ c1)
{
    const int64_t total = (int64_t)*count * nf1;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = w / nf1;
        const double *X = enodes + (int64_t)list[i] * 81;
        const double *F = P + (int64_t)l1[w] * 27;
        double cg[3];
        {
#pragma clang fp contract(off)
            for (int d = 0; d < 3; ++d) cg[d] = (((F[9 * d] + F[9 * d + 2]) + F[9 * d + 6]) + F[9 * d + 8]) * 0.25;
        }
        double dmin = INFINITY;
        int c = 0;
        for (int k = 0; k < 8; ++k) {
#pragma clang fp contract(off)
            const int nd = hx_corner(k);
            const double dx = X[nd] - cg[0], dy = X[27 + nd] - cg[1], dz = X[54 + nd] - cg[2];
            const double D = sqrt((dx * dx + dy * dy) + dz * dz);
            if (D < dmin) {
                dmin = D;
                c = k;
            }
        }
        int fl[3];
        hx_corner_faces(c, fl);
        const d3 TF[2][3] = {{hx_fnode(F, 0), hx_fnode(F, 2), hx_fnode(F, 8)},
                             {hx_fnode(F, 0), hx_fnode(F, 8), hx_fnode(F, 6)}};
        dmin = INFINITY;
        for (int a = 0; a < 3; ++a) {
            const d3 q00 = hx_node(X, elem_face_node(fl[a], 0, 0)), q20 = hx_node(X, elem_face_node(fl[a], 2, 0)),
                     q22 = hx_node(X, elem_face_node(fl[a], 2, 2)), q02 = hx_node(X, elem_face_node(fl[a], 0, 2));
            const d3 TC[2][3] = {{q00, q20, q22}, {q00, q22, q02}};
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) {
                    d3 pa, pb;
                    dmin = fmin(dmin, tri_tri_dist(TC[u], TF[v], pa, pb));
                }
        }
        if (dmin < kTolHit) dmin = 0.0;
        d1[w] = dmin;
        c1[w] = (int8_t)c;
    }
}

// N_F^2 smallest (d, face) of each element's first pass, ascending
__global__ __launch_bounds__(kHT) void k_hx_keep2(const int32_t *__restrict__ count, int nf1, int nf2,
                                                  const int32_t *__restrict__ l1, const double *__restrict__ d1,
                                                  const int8_t *__restrict__ c1, int32_t *__restrict__ l2,
                                                  int8_t *__restrict__ c2)
{
    const int n = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double Ld[kHxK2];
        int Lf[kHxK2], Lc[kHxK2];
#pragma unroll
        for (int k = 0; k < kHxK2; ++k) {
            Ld[k] = INFINITY;
            Lf[k] = 0x7fffffff;
            Lc[k] = 0;
        }
        for (int k = 0; k < nf1; ++k) {
            double cd = d1[(int64_t)i * nf1 + k];
            int cf = l1[(int64_t)i * nf1 + k], cc = c1[(int64_t)i * nf1 + k];
#pragma unroll
            for (int m = 0; m < kHxK2; ++m) {
                const bool sw = hx_less(cd, cf, Ld[m], Lf[m]);
                const double td = Ld[m];
                const int tf = Lf[m], tc = Lc[m];
                Ld[m] = sw ? cd : td;
                Lf[m] = sw ? cf : tf;
                Lc[m] = sw ? cc : tc;
                cd = sw ? td : cd;
                cf = sw ? tf : cf;
                cc = sw ? tc : cc;
            }
        }
#pragma unroll
        for (int m = 0; m < kHxK2; ++m)
            if (m < nf2) {
                l2[(int64_t)i * nf2 + m] = Lf[m];
                c2[(int64_t)i * nf2 + m] = (int8_t)Lc[m];
            }
    }
}

struct HxTie {
    double absdot, dot;
    double vx, vy, vz, nx, ny, nz;
    int f, s, t, valid;
};

// larger |dot| first, then lower (face, face triangle, element triangle)
__device__ inline bool hx_tie_before(const HxTie &a, const HxTie &b)
{
    if (!a.valid) return false;
    if (!b.valid) return true;
    if (a.absdot != b.absdot) return a.absdot > b.absdot;
    if (a.f != b.f) return a.f < b.f;
    if (a.s != b.s) return a.s < b.s;
    return a.t < b.t;
}

__device__ inline void hx_tie_offer(HxTie &b1, HxTie &b2, const HxTie &r)
{
    if (hx_tie_before(r, b1)) {
        b2 = b1;
        b1 = r;
    } else if (hx_tie_before(r, b2)) {
        b2 = r;
    }
}

__device__ inline HxTie hx_shfl(const HxTie &a, int d)
{
    HxTie r;
    r.absdot = __shfl_xor(a.absdot, d, 64);
    r.dot = __shfl_xor(a.dot, d, 64);
    r.vx = __shfl_xor(a.vx, d, 64);
    r.vy = __shfl_xor(a.vy, d, 64);
    r.vz = __shfl_xor(a.vz, d, 64);
    r.nx = __shfl_xor(a.nx, d, 64);
    r.ny = __shfl_xor(a.ny, d, 64);
    r.nz = __shfl_xor(a.nz, d, 64);
    r.f = __shfl_xor(a.f, d, 64);
    r.s = __shfl_xor(a.s, d, 64);
    r.t = __shfl_xor(a.t, d, 64);
    r.valid = __shfl_xor(a.valid, d, 64);
    return r;
}

// Alg. cp2, one wavefront per listed element: work item (kept face k,
// element triangle at the kept corner); every item runs over the face's 8
// lattice triangles.  A pair closer than the tolerance is a hit; the
// distances are kept in LDS so the tie pass recomputes closest points only
// for the pairs within the tie threshold.  Writes HOLE only (union over
// surfaces).
__global__ __launch_bounds__(64) void k_hx_pass2(const double *__restrict__ enodes, const int32_t *__restrict__ list,
                                                 const int32_t *__restrict__ count, const double *__restrict__ P,
                                                 int nf2, const int32_t *__restrict__ l2, const int8_t *__restrict__ c2,
                                                 int wall, int8_t *__restrict__ iblank)
{
    __shared__ double sD[kHxK2 * 24 * 8];
    const int n = *count;
    const int lane = threadIdx.x;
    const int n_items = nf2 * 24;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int e = list[i];
        const double *X = enodes + (int64_t)e * 81;
        bool hit = false;
        double best = INFINITY;
        for (int it = lane; it < n_items && !hit; it += 64) {
            const int k = it / 24, r = it - 24 * k;
            const int f = l2[(int64_t)i * nf2 + k];
            int fl[3];
            hx_corner_faces(c2[(int64_t)i * nf2 + k], fl);
            d3 T[3];
            elem_tri(X, 8 * fl[r >> 3] + (r & 7), T);
            const double *F = P + (int64_t)f * 27;
            for (int s = 0; s < 8; ++s) {
                d3 S[3], pa, pb;
                face_tri(F, s, S);
                const double d = tri_tri_dist(T, S, pa, pb);
                sD[8 * it + s] = d;
                if (d < kTolHit) {
                    hit = true;
                    break;
                }
                best = fmin(best, d);
            }
        }
        if (__ballot(hit)) {
            if (wall && lane == 0) iblank[e] = OC_HOLE;
            continue;
        }
        for (int d = 32; d >= 1; d >>= 1) best = fmin(best, __shfl_xor(best, d, 64));
        const double thr = best * (1.0 + 1e-9);
        HxTie b1, b2;
        b1.valid = b2.valid = 0;
        for (int it = lane; it < n_items; it += 64) {
            const int k = it / 24, r = it - 24 * k;
            const int f = l2[(int64_t)i * nf2 + k];
            int fl[3];
            hx_corner_faces(c2[(int64_t)i * nf2 + k], fl);
            const int t = 8 * fl[r >> 3] + (r & 7);
            for (int s = 0; s < 8; ++s) {
                if (sD[8 * it + s] > thr) continue;
                d3 T[3], S[3], pa, pb;
                elem_tri(X, t, T);
                face_tri(P + (int64_t)f * 27, s, S);
                tri_tri_dist(T, S, pa, pb);
                HxTie rec;
                const d3 v = pa - pb;
                const double L = sqrt(dot(v, v));
                d3 nn = cross(S[1] - S[0], S[2] - S[0]);
                const double ln = sqrt(dot(nn, nn));
                nn = ln > 0.0 ? nn * (1.0 / ln) : mk(0.0, 0.0, 0.0);
                rec.vx = v.x;
                rec.vy = v.y;
                rec.vz = v.z;
                rec.nx = nn.x;
                rec.ny = nn.y;
                rec.nz = nn.z;
                rec.dot = L > 0.0 ? dot(v, nn) / L : 0.0;
                rec.absdot = fabs(rec.dot);
                rec.f = f;
                rec.s = s;
                rec.t = t;
                rec.valid = 1;
                hx_tie_offer(b1, b2, rec);
            }
        }
        for (int d = 32; d >= 1; d >>= 1) {
            const HxTie o1 = hx_shfl(b1, d), o2 = hx_shfl(b2, d);
            hx_tie_offer(b1, b2, o1);
            hx_tie_offer(b1, b2, o2);
        }
        if (lane == 0 && b1.valid) {
            double sgn = b1.dot;
            if (b2.valid && b1.absdot - b2.absdot <= 1e-9 && (b1.dot > 0.0) != (b2.dot > 0.0))
                sgn = b1.vx * (b1.nx + b2.nx) + b1.vy * (b1.ny + b2.ny) + b1.vz * (b1.nz + b2.nz);
            if (sgn < 0.0) iblank[e] = OC_HOLE;
        }
    }
}

__global__ void k_hx_fill(int8_t *__restrict__ ib, int64_t n, int8_t v)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        ib[e] = v;
}

__global__ void k_hx_zero(int32_t *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

#define LAUNCH(name, grid, block, ...)                                                       \
    do {                                                                                     \
        size_t slot_;                                                                        \
        time_begin(ctx, st, #name, &slot_);                                                  \
        hipLaunchKernelGGL(name, grid, block, 0, st, __VA_ARGS__);                           \
        time_end(ctx, st, slot_);                                                            \
    } while (0)

static unsigned hx_blocks(int64_t n, int per)
{
    const int64_t b = (n + per - 1) / per;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}

// scratch carved from one slot-owned arena, grown on demand
static oc_status hx_reserve(oc_slot *sl, size_t bytes, char **base)
{
    if (bytes > sl->hx_cap) {
        OC_HIP(hipStreamSynchronize(sl->stream));
        OC_TRY(dev_alloc(sl->ctx, sl->owned, bytes, (void **)&sl->hx_buf));
        sl->hx_cap = bytes;
    }
    *base = reinterpret_cast<char *>(sl->hx_buf);
    return OC_OK;
}

static size_t hx_align(size_t v) { return (v + 255) / 256 * 256; }

oc_status filtered_cut_run(oc_slot *sl, Grid &g, Surf *const *surfs, const Pose *poses_dev, int n_surf, int nf1,
                           int nf2, int8_t *iblank, int64_t *n_listed)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    LAUNCH(k_hx_fill, dim3(hx_blocks(g.n_elem, kHT)), dim3(kHT), iblank, g.n_elem, (int8_t)OC_FIELD);
    int64_t listed = 0;
    for (int k = 0; k < n_surf; ++k) {
        const Surf &s = *surfs[k];
        const int k1 = (int)std::min<int64_t>(nf1, s.n_face), k2 = std::min(nf2, k1);
        const int nb = (int)((s.n_face + kHT - 1) / kHT);
        // surface part: posed faces, partial boxes, box, list, count
        const size_t o_P = 0, o_part = hx_align(o_P + sizeof(double) * 27 * (size_t)s.n_face);
        const size_t o_sbox = hx_align(o_part + sizeof(double) * 6 * (size_t)nb);
        const size_t o_cnt = hx_align(o_sbox + sizeof(double) * 6);
        const size_t o_list = hx_align(o_cnt + sizeof(int32_t));
        const size_t o_elem = hx_align(o_list + sizeof(int32_t) * (size_t)g.n_elem);
        char *base;
        OC_TRY(hx_reserve(sl, o_elem, &base));
        double *P = reinterpret_cast<double *>(base + o_P), *part = reinterpret_cast<double *>(base + o_part);
        double *sbox = reinterpret_cast<double *>(base + o_sbox);
        int32_t *cnt = reinterpret_cast<int32_t *>(base + o_cnt), *list = reinterpret_cast<int32_t *>(base + o_list);
        LAUNCH(k_hx_pose, dim3((unsigned)nb), dim3(kHT), s.nodes, s.n_nodes, s.conn, s.n_face, poses_dev + k, P, part);
        LAUNCH(k_hx_sbox, dim3(1), dim3(64), part, nb, sbox);
        LAUNCH(k_hx_zero, dim3(1), dim3(64), cnt);
        LAUNCH(k_hx_filter, dim3(hx_blocks(g.n_elem, kHT)), dim3(kHT), g.ebox, g.ebox_stride, g.n_elem, sbox, list,
               cnt);
        int32_t n = 0;
        OC_HIP(hipMemcpyAsync(&n, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        OC_HIP(hipStreamSynchronize(st));
        listed += n;
        if (n == 0) continue;
        // element part: OBBs, kept lists
        const size_t o_obb = o_elem, o_l1 = hx_align(o_obb + sizeof(double) * 18 * (size_t)n);
        const size_t o_d1 = hx_align(o_l1 + sizeof(int32_t) * (size_t)n * k1);
        const size_t o_c1 = hx_align(o_d1 + sizeof(double) * (size_t)n * k1);
        const size_t o_l2 = hx_align(o_c1 + (size_t)n * k1);
        const size_t o_c2 = hx_align(o_l2 + sizeof(int32_t) * (size_t)n * k2);
        const size_t o_end = hx_align(o_c2 + (size_t)n * k2);
        if (o_end > sl->hx_cap) {
            // keep the surface part: grow into a new arena and copy it over
            char *old = base;
            OC_TRY(hx_reserve(sl, o_end, &base));
            OC_HIP(hipMemcpyAsync(base, old, o_elem, hipMemcpyDeviceToDevice, st));
            P = reinterpret_cast<double *>(base + o_P);
            cnt = reinterpret_cast<int32_t *>(base + o_cnt);
            list = reinterpret_cast<int32_t *>(base + o_list);
        }
        double *obb = reinterpret_cast<double *>(base + o_obb), *d1 = reinterpret_cast<double *>(base + o_d1);
        int32_t *l1 = reinterpret_cast<int32_t *>(base + o_l1), *l2 = reinterpret_cast<int32_t *>(base + o_l2);
        int8_t *c1 = reinterpret_cast<int8_t *>(base + o_c1), *c2 = reinterpret_cast<int8_t *>(base + o_c2);
        LAUNCH(k_hx_obb, dim3(hx_blocks(n, kHT)), dim3(kHT), g.enodes, list, cnt, obb);
        if (k1 <= 4)
            LAUNCH(k_hx_approx<4>, dim3(hx_blocks(n, kHxElems)), dim3(kHT), P, s.n_face, obb, cnt, k1, l1);
        else if (k1 <= 8)
            LAUNCH(k_hx_approx<8>, dim3(hx_blocks(n, kHxElems)), dim3(kHT), P, s.n_face, obb, cnt, k1, l1);
        else if (k1 <= 16)
            LAUNCH(k_hx_approx<16>, dim3(hx_blocks(n, kHxElems)), dim3(kHT), P, s.n_face, obb, cnt, k1, l1);
        else
            LAUNCH(k_hx_approx<kHxK1>, dim3(hx_blocks(n, kHxElems)), dim3(kHT), P, s.n_face, obb, cnt, k1, l1);
        LAUNCH(k_hx_pass1, dim3(hx_blocks((int64_t)n * k1, kHT)), dim3(kHT), g.enodes, list, cnt, P, k1, l1, d1, c1);
        LAUNCH(k_hx_keep2, dim3(hx_blocks(n, kHT)), dim3(kHT), cnt, k1, k2, l1, d1, c1, l2, c2);
        LAUNCH(k_hx_pass2, dim3(hx_blocks(n, 1)), dim3(64), g.enodes, list, cnt, P, k2, l2, c2,
               s.kind == OC_SURF_WALL ? 1 : 0, iblank);
        OC_HIP(hipGetLastError());
    }
    OC_TRY(fringe_layer_run(sl, g, iblank));
    if (n_listed) *n_listed = listed;
    return OC_OK;
}

}  // namespace oc
