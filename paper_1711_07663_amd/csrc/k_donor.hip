// Receptor points and donor search (Sec. 4.3 "Donor/Receptor Point
// Connectivity on GPUs").
//
//   k_fr_count / scan / k_fr_write   ordered compaction of fringe elements
//   k_fringe_points                  27 Gauss points per fringe element mapped
//                                    by the quadratic isoparametric map
//                                    (eq. reftophys) and posed to world frame
//   k_dp_count / scan / k_dp_fill    per point: inverse pose into the donor
//                                    grid's registration frame (the rigid
//                                    motion trick of Sec. 4.3), one bin lookup
//                                    of control-net boxes, and the boxes that
//                                    contain it as (point, element) pairs
//   k_dp_newton                      Newton (eq. ref-update, eq. Jac) on every
//                                    pair; the lowest containing id wins
//   k_dp_final                       donor id and reference coordinates
// Registration-time kernels build the element node copies, the FP32 element
// boxes and the donor bins.
#include <cstring>
#include <mutex>

#include "dev_common.h"
#include "q2.h"

namespace oc {

constexpr int kT = 256;
// blocks of the kernels that loop over a device-side count: 16 waves per
// SIMD, twice what the device holds at once (dynamic balance) without a
// wave per possible item of the capacity
constexpr unsigned kLoopBlocks = 4096;

// Newton inversion: xi0 = 0; stop when |x_p - x(xi)| <= 1e-13 diam (checked
// before each step) or the clamped step is <= 1e-14; at most
// OC_NEWTON_MAXIT iterations; contained if converged and
// max|xi| <= 1 + OC_CONTAIN_TOL.  The 3x3 system is solved with the adjugate.
// Without STREAM the element's 81 coordinates are loaded once into registers
// (one round of independent loads) and reused by every iteration; with
// STREAM they are read row by row from memory each iteration (few registers,
// for rarely taken paths).  Both give the same bits; k_dp_newton's
// per-component map rounds differently in the last bits.
template <bool STREAM>
__device__ inline bool newton_q2(const double *__restrict__ Xg, d3 p, double diam, double *xi, int &iters)
{
    double Xr[STREAM ? 1 : 81];
    if (!STREAM) {
#pragma unroll
        for (int k = 0; k < 81; ++k) Xr[k] = Xg[k];
    }
    const double *X = STREAM ? Xg : Xr;
    xi[0] = xi[1] = xi[2] = 0.0;
    bool conv = false;
    // |r| <= 1e-13 diam, compared squared (no square root in the loop)
    const double rtol = 1e-13 * diam, rtol2 = rtol * rtol;
#pragma unroll 1
    for (int it = 0; it < OC_NEWTON_MAXIT; ++it) {
        ++iters;
        double x[3], J[9];
        if (it == 0) {
            // at xi = 0 the basis is l = (0, 1, 0), dl = (-1/2, 0, 1/2) on
            // every axis: x is the centre node 13 and the Jacobian columns
            // are half the differences of the opposite face-centre nodes
            // (14 - 12, 16 - 10, 22 - 4)
            for (int d = 0; d < 3; ++d) {
                const double *C = X + 27 * d;
                x[d] = C[13];
                J[3 * d] = 0.5 * (C[14] - C[12]);
                J[3 * d + 1] = 0.5 * (C[16] - C[10]);
                J[3 * d + 2] = 0.5 * (C[22] - C[4]);
            }
        } else {
            q2_map<true, STREAM>(X, xi, x, J);
        }
        const double r0 = p.x - x[0], r1 = p.y - x[1], r2 = p.z - x[2];
        if (r0 * r0 + r1 * r1 + r2 * r2 <= rtol2) {
            conv = true;
            break;
        }
        const double c00 = J[4] * J[8] - J[5] * J[7];
        const double c01 = J[5] * J[6] - J[3] * J[8];
        const double c02 = J[3] * J[7] - J[4] * J[6];
        const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
        if (det == 0.0) break;
        // 1 / det: hardware reciprocal and two Newton-Raphson corrections
        // (within an ulp; the quotients only steer the iteration)
        double id = __builtin_amdgcn_rcp(det);
        id = fma(id, fma(-det, id, 1.0), id);
        id = fma(id, fma(-det, id, 1.0), id);
        // inverse = adj / det, adj(i,j) = cofactor(j,i)
        const double d0 = (c00 * r0 + (J[2] * J[7] - J[1] * J[8]) * r1 + (J[1] * J[5] - J[2] * J[4]) * r2) * id;
        const double d1 = (c01 * r0 + (J[0] * J[8] - J[2] * J[6]) * r1 + (J[2] * J[3] - J[0] * J[5]) * r2) * id;
        const double d2 = (c02 * r0 + (J[1] * J[6] - J[0] * J[7]) * r1 + (J[0] * J[4] - J[1] * J[3]) * r2) * id;
        const double lim = 1.0 + OC_NEWTON_CLAMP;
        const double n0 = fmin(fmax(xi[0] + d0, -lim), lim);
        const double n1 = fmin(fmax(xi[1] + d1, -lim), lim);
        const double n2 = fmin(fmax(xi[2] + d2, -lim), lim);
        const double step = fmax(fabs(n0 - xi[0]), fmax(fabs(n1 - xi[1]), fabs(n2 - xi[2])));
        xi[0] = n0;
        xi[1] = n1;
        xi[2] = n2;
        if (step <= 1e-14) {
            conv = true;
            break;
        }
    }
    const double m = fmax(fabs(xi[0]), fmax(fabs(xi[1]), fabs(xi[2])));
    return conv && m <= 1.0 + OC_CONTAIN_TOL;
}

// ---------------------------------------------- registration kernels -----
// the union of the FP32 boxes of every 256 consecutive elements (one block of
// 64 lanes, four elements each): the element filter's wavefront skips its
// elements' boxes when this box misses the surface box
__global__ __launch_bounds__(64) void k_wave_boxes(const float *__restrict__ ebox, int64_t stride, int64_t n_elem,
                                                   float *__restrict__ wbox)
{
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t base = (int64_t)blockIdx.x * 256 + 4 * threadIdx.x;
    for (int k = 0; k < 4; ++k) {
        const int64_t e = base + k;
        if (e >= n_elem) break;
        for (int d = 0; d < 3; ++d) {
            lo[d] = fminf(lo[d], ebox[d * stride + e]);
            hi[d] = fmaxf(hi[d], ebox[(3 + d) * stride + e]);
        }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        for (int d = 0; d < 3; ++d) {
            lo[d] = fminf(lo[d], __shfl_xor(lo[d], s, 64));
            hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], s, 64));
        }
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) {
            wbox[blockIdx.x * 6 + d] = lo[d];
            wbox[blockIdx.x * 6 + 3 + d] = hi[d];
        }
}

// per (element, coordinate): the map's monomial coefficients (q2_mono), read
// by the Newton solves of the donor search
__global__ __launch_bounds__(kT) void k_elem_mono(const double *__restrict__ enodes, int64_t n_elem,
                                                  double *__restrict__ emono)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_elem * 3) return;
    double M[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) M[k] = enodes[i * 27 + k];
    q2_mono(M);
#pragma unroll
    for (int k = 0; k < 27; ++k) emono[i * 27 + k] = M[k];
}

__global__ __launch_bounds__(kT) void k_gather_nodes(const double *__restrict__ nodes,
                                                     const int32_t *__restrict__ conn, int64_t n_elem,
                                                     double *__restrict__ enodes)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_elem * 27) return;
    const int64_t e = i / 27;
    const int k = (int)(i - e * 27);
    const int64_t id = conn[i];
    enodes[e * 81 + k] = nodes[3 * id];
    enodes[e * 81 + 27 + k] = nodes[3 * id + 1];
    enodes[e * 81 + 54 + k] = nodes[3 * id + 2];
}

// FP32 node box (cut filter, SoA planes with padded stride), FP32
// control-net box (donor candidates, AoS) and node-box diagonal.  Also the
// Jacobian determinant at the element centre (validity check).
__global__ __launch_bounds__(kT) void k_elem_boxes(const double *__restrict__ enodes, int64_t n_elem,
                                                   int64_t stride, float *__restrict__ ebox,
                                                   float *__restrict__ cbox, double *__restrict__ ediam,
                                                   int *__restrict__ bad_jac)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elem) return;
    const double *X = enodes + e * 81;
    double lo[3], hi[3], clo[3], chi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
        clo[d] = INFINITY;
        chi[d] = -INFINITY;
        const double *C = X + 27 * d;
        for (int k = 0; k < 27; ++k) {
            lo[d] = fmin(lo[d], C[k]);
            hi[d] = fmax(hi[d], C[k]);
        }
        // Bernstein control net of the tensor-product quadratic: along each
        // reference axis the middle control point is 2 x1 - (x0 + x2) / 2
        double B[27];
        for (int k = 0; k < 27; ++k) B[k] = C[k];
        const int st[3] = {1, 3, 9};
        for (int ax = 0; ax < 3; ++ax)
            for (int k = 0; k < 27; ++k)
                if ((k / st[ax]) % 3 == 1) B[k] = 2.0 * B[k] - 0.5 * (B[k - st[ax]] + B[k + st[ax]]);
        for (int k = 0; k < 27; ++k) {
            clo[d] = fmin(clo[d], B[k]);
            chi[d] = fmax(chi[d], B[k]);
        }
    }
    const double diam = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                             (hi[2] - lo[2]) * (hi[2] - lo[2]));
    const double infl = 1e-10 * diam;
    for (int d = 0; d < 3; ++d) {
        ebox[d * stride + e] = f32_down(lo[d]);
        ebox[(3 + d) * stride + e] = f32_up(hi[d]);
        cbox[e * 6 + d] = f32_down(clo[d] - infl);
        cbox[e * 6 + 3 + d] = f32_up(chi[d] + infl);
    }
    ediam[e] = diam;
    double xi[3] = {0.0, 0.0, 0.0}, x[3], J[9];
    q2_map<true, true>(X, xi, x, J);
    const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                       J[2] * (J[3] * J[7] - J[4] * J[6]);
    if (!(det > 0.0)) atomicAdd(bad_jac, 1);
}

// Oriented box of the control net: a second, tighter candidate test for thin
// curved elements, whose axis-aligned boxes are loose.  Axes: the element's
// xi and eta centre chords (node 14 - node 12, node 16 - node 10),
// orthonormalised, and their cross product; centre: node 13.  Centre and
// axes are stored in FP32; the extents of the 27 control points along those
// same FP32 axes are computed in FP64, rounded outward and widened by 1e-7
// of the control-net box diagonal, which covers the containment tolerance
// (|xi| <= 1 + 1e-10 moves x by far less) and the rounding of the query.
// Record: c[3], u1[3], u2[3], u3[3], lo[3], hi[3].
__global__ __launch_bounds__(kT) void k_elem_obb(const double *__restrict__ enodes, int64_t n_elem,
                                                 const float *__restrict__ cbox, float *__restrict__ obox)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elem) return;
    const double *X = enodes + e * 81;
    double u[3][3];
    for (int d = 0; d < 3; ++d) {
        u[0][d] = X[27 * d + 14] - X[27 * d + 12];
        u[1][d] = X[27 * d + 16] - X[27 * d + 10];
    }
    double n0 = sqrt(u[0][0] * u[0][0] + u[0][1] * u[0][1] + u[0][2] * u[0][2]);
    bool ok = n0 > 0.0;
    if (ok)
        for (int d = 0; d < 3; ++d) u[0][d] /= n0;
    const double pr = u[1][0] * u[0][0] + u[1][1] * u[0][1] + u[1][2] * u[0][2];
    for (int d = 0; d < 3; ++d) u[1][d] -= pr * u[0][d];
    const double n1 = sqrt(u[1][0] * u[1][0] + u[1][1] * u[1][1] + u[1][2] * u[1][2]);
    ok = ok && n1 > 0.0;
    if (ok)
        for (int d = 0; d < 3; ++d) u[1][d] /= n1;
    u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
    u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
    u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    if (!ok)
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) u[k][d] = k == d ? 1.0 : 0.0;
    float fc[3], fu[3][3];
    for (int d = 0; d < 3; ++d) fc[d] = (float)X[27 * d + 13];
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) fu[k][d] = (float)u[k][d];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int st[3] = {1, 3, 9};
    for (int j = 0; j < 27; ++j) {
        // control point j: the tensor-product Bernstein net (middle point per
        // reference axis 2 x1 - (x0 + x2) / 2, applied axis by axis)
        double b[3];
        for (int d = 0; d < 3; ++d) {
            const double *C = X + 27 * d;
            const int ja = j % 3, jb = (j / 3) % 3, jc = j / 9;
            double v = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double wc = jc == 1 ? (c == 1 ? 2.0 : -0.5) : (c == jc ? 1.0 : 0.0);
                if (wc == 0.0) continue;
                for (int bb = 0; bb < 3; ++bb) {
                    const double wb = jb == 1 ? (bb == 1 ? 2.0 : -0.5) : (bb == jb ? 1.0 : 0.0);
                    if (wb == 0.0) continue;
                    for (int a = 0; a < 3; ++a) {
                        const double wa = ja == 1 ? (a == 1 ? 2.0 : -0.5) : (a == ja ? 1.0 : 0.0);
                        if (wa == 0.0) continue;
                        v += wa * wb * wc * C[a * st[0] + bb * st[1] + c * st[2]];
                    }
                }
            }
            b[d] = v;
        }
        for (int k = 0; k < 3; ++k) {
            const double sk = (b[0] - (double)fc[0]) * (double)fu[k][0] + (b[1] - (double)fc[1]) * (double)fu[k][1] +
                              (b[2] - (double)fc[2]) * (double)fu[k][2];
            lo[k] = fmin(lo[k], sk);
            hi[k] = fmax(hi[k], sk);
        }
    }
    const float *cb = cbox + e * 6;
    const double gx = (double)cb[3] - cb[0], gy = (double)cb[4] - cb[1], gz = (double)cb[5] - cb[2];
    const double m = 1e-7 * sqrt(gx * gx + gy * gy + gz * gz);
    float *o = obox + e * 18;
    for (int d = 0; d < 3; ++d) o[d] = fc[d];
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) o[3 + 3 * k + d] = fu[k][d];
    for (int k = 0; k < 3; ++k) {
        o[12 + k] = f32_down(lo[k] - m);
        o[15 + k] = f32_up(hi[k] + m);
    }
}

__global__ __launch_bounds__(kT) void k_dbin_count(const float *__restrict__ cbox, int64_t n_elem, BinGrid G,
                                                   int32_t *__restrict__ count)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elem) return;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = bin_of(cbox[e * 6 + a], G.o[a], G.inv[a], G.n[a]);
        hi[a] = bin_of(cbox[e * 6 + 3 + a], G.o[a], G.inv[a], G.n[a]);
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x)
                atomicAdd(&count[x + (int64_t)G.n[0] * (y + (int64_t)G.n[1] * z)], 1);
}

__global__ __launch_bounds__(kT) void k_dbin_fill(const float *__restrict__ cbox, int64_t n_elem, BinGrid G,
                                                  const int32_t *__restrict__ start, int32_t *cursor,
                                                  int32_t *__restrict__ items)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elem) return;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = bin_of(cbox[e * 6 + a], G.o[a], G.inv[a], G.n[a]);
        hi[a] = bin_of(cbox[e * 6 + 3 + a], G.o[a], G.inv[a], G.n[a]);
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                const int64_t b = x + (int64_t)G.n[0] * (y + (int64_t)G.n[1] * z);
                const int pos = atomicAdd(&cursor[b], 1);
                items[start[b] + pos] = (int32_t)e;
            }
}

// each bin's element ids in ascending order (insertion sort; bins are short)
__global__ __launch_bounds__(kT) void k_dbin_sort(const int32_t *__restrict__ start, int64_t n_bins,
                                                  int32_t *__restrict__ items)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_bins) return;
    const int j0 = start[b], j1 = start[b + 1];
    for (int i = j0 + 1; i < j1; ++i) {
        const int v = items[i];
        int k = i - 1;
        while (k >= j0 && items[k] > v) {
            items[k + 1] = items[k];
            --k;
        }
        items[k + 1] = v;
    }
}

// each bin entry as a 32-byte record: the element's control-net box and its
// id (lo xyz + id bits, hi xyz + 0), so a bin walk reads its entries'
// boxes contiguously instead of through the id
__global__ __launch_bounds__(kT) void k_dbin_records(const int32_t *__restrict__ items, int64_t n_items,
                                                    const float *__restrict__ cbox, float4 *__restrict__ rec)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_items) return;
    const int e = items[j];
    const float *c = cbox + (int64_t)e * 6;
    rec[2 * j] = make_float4(c[0], c[1], c[2], __int_as_float(e));
    rec[2 * j + 1] = make_float4(c[3], c[4], c[5], 0.f);
}

// ----------------------------------------------- fringe compaction --------
constexpr int kFrItems = 16;
constexpr int kFrTile = kT * kFrItems;

// element listed by an ordered compaction: a fringe element of iblank, or
// (prev given) a hole of prev that is not a hole of iblank (to unblank)
__device__ inline bool listed(const int8_t *__restrict__ ib, const int8_t *__restrict__ prev, int64_t i)
{
    return prev ? (prev[i] == OC_HOLE && ib[i] != OC_HOLE) : ib[i] == OC_FRINGE;
}

__global__ __launch_bounds__(kT) void k_fr_count(const int8_t *__restrict__ iblank, const int8_t *__restrict__ prev,
                                                 int64_t n_elem, int32_t *__restrict__ tcount)
{
    const int64_t base = (int64_t)blockIdx.x * kFrTile;
    int c = 0;
    for (int k = 0; k < kFrItems; ++k) {
        const int64_t i = base + (int64_t)k * kT + threadIdx.x;
        if (i < n_elem) c += listed(iblank, prev, i);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    __shared__ int ws[kT / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kT / 64; ++w) s += ws[w];
        tcount[blockIdx.x] = s;
    }
}

// count and tile-local write in one pass: tile t's fringe elements in
// ascending order at tl[t * kFrTile ...] and their number at tcount[t]; the
// tiles concatenated in order (after a scan of the counts) are the ordered
// list, read in place by k_fringe_points_t
__global__ __launch_bounds__(kT) void k_fr_tiles(const int8_t *__restrict__ iblank, int64_t n_elem,
                                                 int32_t *__restrict__ tcount, int32_t *__restrict__ tl)
{
    const int64_t my = (int64_t)blockIdx.x * kFrTile + (int64_t)threadIdx.x * kFrItems;
    int c = 0;
    for (int k = 0; k < kFrItems; ++k) {
        const int64_t i = my + k;
        if (i < n_elem) c += iblank[i] == OC_FRINGE;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    __shared__ int ws[kT / 64];
    if (lane == 63) ws[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < kT / 64; ++w) {
        if (w < wid) off += ws[w];
        tot += ws[w];
    }
    if (threadIdx.x == 0) tcount[blockIdx.x] = tot;
    int pos = (int)((int64_t)blockIdx.x * kFrTile) + off + inc - c;
    for (int k = 0; k < kFrItems; ++k) {
        const int64_t i = my + k;
        if (i < n_elem && iblank[i] == OC_FRINGE) tl[pos++] = (int32_t)i;
    }
}

// ordered write of the listed elements (at most cap)
__global__ __launch_bounds__(kT) void k_fr_write(const int8_t *__restrict__ iblank, const int8_t *__restrict__ prev,
                                                 int64_t n_elem, const int32_t *__restrict__ toff,
                                                 int32_t *__restrict__ list, int64_t cap)
{
    const int64_t my = (int64_t)blockIdx.x * kFrTile + (int64_t)threadIdx.x * kFrItems;
    int c = 0;
    for (int k = 0; k < kFrItems; ++k) {
        const int64_t i = my + k;
        if (i < n_elem) c += listed(iblank, prev, i);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    __shared__ int ws[kT / 64];
    if (lane == 63) ws[wid] = inc;
    __syncthreads();
    int off = toff[blockIdx.x];
    for (int w = 0; w < wid; ++w) off += ws[w];
    int pos = off + inc - c;
    for (int k = 0; k < kFrItems; ++k) {
        const int64_t i = my + k;
        if (i < n_elem && listed(iblank, prev, i)) {
            if (pos < cap) list[pos] = (int32_t)i;
            ++pos;
        }
    }
}

// a9: Gauss point k = a + 3b + 9c of fringe element list[i / 27], posed.
// The number of fringe elements is read from the device (nfr); at most cap
// points are written; n_out receives 27 * nfr.  An id outside [0, n_elem)
// gives NaN points and source -1.
// a9: 27 Gauss points per listed element.  A block takes 256 consecutive
// points (at most 11 elements): the elements' nodes are staged in LDS with
// coalesced loads, then every thread maps its point from LDS.  The list is
// either contiguous (list[q]) or tile-major as k_fr_tiles leaves it (the
// elements of tile t at tl[t * kFrTile ...], tile offsets toff[0..nt]).
constexpr int kPtElems = kT / 27 + 2;
constexpr int kToffLds = 2048;   // tile offsets staged in LDS up to this many tiles

// MODE 0: a contiguous list; 1: tile-major with the tile offsets toff[0..nt];
// 2: tile-major with the tile counts (nt <= kToffLds), each block forming the
// offsets itself in LDS (no scan launch)
template <int MODE>
__device__ inline void gauss_points(const double *__restrict__ enodes, int64_t n_elem,
                                    const int32_t *__restrict__ list, const int32_t *__restrict__ toff, int nt,
                                    const int32_t *__restrict__ nfr, int64_t cap, const Pose *__restrict__ pose_dev,
                                    double *__restrict__ pts, int32_t *__restrict__ src, int32_t *__restrict__ n_out)
{
    __shared__ double sN[kPtElems * 81];
    __shared__ int sE[kPtElems];
    __shared__ int sT[MODE ? kToffLds + 1 : 1];
    __shared__ int sW[kT / 64];
    const bool tl_lds = MODE == 2 || (MODE == 1 && nt + 1 <= kToffLds);
    int64_t total;
    if (MODE == 2) {
        // exclusive prefix of the tile counts: a contiguous run per thread,
        // then a block scan of the runs' sums
        const int per = (nt + kT - 1) / kT, lo = (int)threadIdx.x * per;
        int run = 0;
        for (int k = 0; k < per; ++k)
            if (lo + k < nt) run += toff[lo + k];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        int inc = run;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        if (lane == 63) sW[wid] = inc;
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < kT / 64; ++w) {
            if (w < wid) off += sW[w];
            tot += sW[w];
        }
        int p = off + inc - run;
        for (int k = 0; k < per; ++k)
            if (lo + k < nt) {
                const int v = toff[lo + k];
                sT[lo + k] = p;
                p += v;
            }
        if (threadIdx.x == 0) sT[nt] = tot;
        total = (int64_t)tot * 27;
    } else {
        if (tl_lds)
            for (int k = threadIdx.x; k <= nt; k += kT) sT[k] = toff[k];
        total = (int64_t)(*nfr) * 27;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_out) *n_out = (int32_t)total;
    const int64_t n = total < cap ? total : cap;
    const Pose pose = *pose_dev;
    for (int64_t i0 = (int64_t)blockIdx.x * kT; i0 < n; i0 += (int64_t)gridDim.x * kT) {
        const int64_t q0 = i0 / 27, q1 = (i0 + kT < n ? i0 + kT - 1 : n - 1) / 27;
        const int ne = (int)(q1 - q0 + 1);
        __syncthreads();   // the previous round's points are mapped (and the offsets staged)
        if ((int)threadIdx.x < ne) {
            const int q = (int)(q0 + threadIdx.x);
            if (MODE) {
                // the tile holding list position q: the last t with offset <= q
                int lo = 0, hi = nt - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((tl_lds ? sT[mid] : toff[mid]) <= q) lo = mid;
                    else hi = mid - 1;
                }
                sE[threadIdx.x] = list[(int64_t)lo * kFrTile + (q - (tl_lds ? sT[lo] : toff[lo]))];
            } else {
                sE[threadIdx.x] = list[q];
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < ne * 81; k += kT) {
            const int j = k / 81, e = sE[j];
            sN[k] = (e >= 0 && e < n_elem) ? enodes[(int64_t)e * 81 + (k - 81 * j)] : 0.0;
        }
        __syncthreads();
        const int64_t i = i0 + threadIdx.x;
        if (i >= n) continue;
        const int64_t q = i / 27;
        const int k = (int)(i - q * 27), j = (int)(q - q0);
        const int e = sE[j];
        if (e < 0 || e >= n_elem) {
            const double nan = __builtin_nan("");
            pts[3 * i] = nan;
            pts[3 * i + 1] = nan;
            pts[3 * i + 2] = nan;
            if (src) src[i] = -1;
            continue;
        }
        const double g = 0.7745966692414834;  // sqrt(3/5), 3-point Gauss-Legendre
        const double xi[3] = {(k % 3 - 1) * g, ((k / 3) % 3 - 1) * g, (k / 9 - 1) * g};
        double x[3];
        q2_map<false, true>(sN + 81 * j, xi, x, nullptr);
        const d3 w = pose_apply(pose, mk(x[0], x[1], x[2]));
        pts[3 * i] = w.x;
        pts[3 * i + 1] = w.y;
        pts[3 * i + 2] = w.z;
        if (src) src[i] = e;
    }
}

__global__ __launch_bounds__(kT) void k_fringe_points(const double *__restrict__ enodes, int64_t n_elem,
                                                      const int32_t *__restrict__ list, const int32_t *__restrict__ nfr,
                                                      int64_t cap, const Pose *__restrict__ pose_dev,
                                                      double *__restrict__ pts, int32_t *__restrict__ src,
                                                      int32_t *__restrict__ n_out)
{
    gauss_points<0>(enodes, n_elem, list, nullptr, 0, nfr, cap, pose_dev, pts, src, n_out);
}

// the same over the tile-major list of k_fr_tiles: MODE 1 with the tile
// offsets toff (nfr = toff + nt), MODE 2 with the tile counts themselves
// (nt <= kToffLds); one instance per mode keeps one mode's LDS per block
template <int MODE>
__global__ __launch_bounds__(kT) void k_fringe_points_t(const double *__restrict__ enodes, int64_t n_elem,
                                                        const int32_t *__restrict__ tl, const int32_t *__restrict__ toff,
                                                        int nt, int64_t cap, const Pose *__restrict__ pose_dev,
                                                        double *__restrict__ pts, int32_t *__restrict__ src,
                                                        int32_t *__restrict__ n_out)
{
    gauss_points<MODE>(enodes, n_elem, tl, toff, nt, MODE == 1 ? toff + nt : nullptr, cap, pose_dev, pts, src,
                       n_out);
}

__device__ inline bool box_has(const float *__restrict__ c, d3 p)
{
    return p.x >= (double)c[0] && p.y >= (double)c[1] && p.z >= (double)c[2] && p.x <= (double)c[3] &&
           p.y <= (double)c[4] && p.z <= (double)c[5];
}

// the oriented control-net box (k_elem_obb) holds p
__device__ inline bool obb_has(const float *__restrict__ o, d3 p)
{
    const double dx = p.x - (double)o[0], dy = p.y - (double)o[1], dz = p.z - (double)o[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double sk = dx * (double)o[3 + 3 * k] + dy * (double)o[4 + 3 * k] + dz * (double)o[5 + 3 * k];
        if (sk < (double)o[12 + k] || sk > (double)o[15 + k]) return false;
    }
    return true;
}

// candidate test of bin entry j (its record): the axis-aligned control-net
// box, then the oriented one; *e receives the entry's element
__device__ inline bool rec_has(const float4 *__restrict__ rec, const float *__restrict__ obox, int64_t j, d3 p,
                               int *e, int64_t n_elem, uint32_t *err)
{
    const float4 lo = rec[2 * j], hi = rec[2 * j + 1];
    *e = __float_as_int(lo.w);
    if (!chk(*e >= 0 && *e < n_elem, err, kChkDonorElem)) return false;
    return p.x >= (double)lo.x && p.y >= (double)lo.y && p.z >= (double)lo.z && p.x <= (double)hi.x &&
           p.y <= (double)hi.y && p.z <= (double)hi.z && obb_has(obox + (int64_t)*e * 18, p);
}

__device__ inline int64_t point_bin(const BinGrid &G, d3 p)
{
    const int bx = bin_of((float)p.x, G.o[0], G.inv[0], G.n[0]);
    const int by = bin_of((float)p.y, G.o[1], G.inv[1], G.n[1]);
    const int bz = bin_of((float)p.z, G.o[2], G.inv[2], G.n[2]);
    return bx + (int64_t)G.n[0] * (by + (int64_t)G.n[1] * bz);
}

struct DonorArgs {
    const double *enodes;
    const double *emono;   // monomial coefficients of the elements' maps (k_elem_mono)
    const float *cbox;
    const float *obox;
    const double *ediam;
    BinGrid G;
    const int32_t *bstart;
    const float4 *brec;    // bin entries as records (k_dbin_records)
    int64_t n_items;       // bin entries of the grid
    int64_t n_elem;        // elements of the grid
    uint32_t *err;         // the context's check word (checked builds)
    const Pose *pose;
    const double *pts;
    int64_t cap;           // point capacity
    const int32_t *n_dev;  // point count on the device (null: cap)
    int32_t *n_eff;        // min(*n_dev, cap), written by k_dp_count
    double *plocal;        // [cap][3] points in the grid's registration frame
    int32_t *cnt;          // [cap + 1] candidates per point
    int32_t *off;          // [cap + 1] exclusive scan of cnt
    int32_t *best;         // [cap] lowest containing element id
    int32_t *cache;        // [cap][kCandCache] first candidates of each point (ascending id)
    int32_t *pair_pt;      // [pair_cap]
    int32_t *pair_el;      // [pair_cap]
    double *pair_xi;       // [pair_cap][3] reference coordinates of contained pairs
    uint8_t *pair_it;      // [pair_cap] Newton iterations run per pair (statistics)
    int64_t pair_cap;
    int32_t *donor;
    double *ref;
    DonorCounters *dcnt;
    int lanes;             // lanes per point in the bin walks (power of two, <= 64)
    int pad;
};

constexpr int kCandCache = 4;   // candidates per point kept by k_dp_count for k_dp_fill

__device__ inline int64_t donor_points(const DonorArgs &a)
{
    return a.n_dev ? ((int64_t)*a.n_dev < a.cap ? (int64_t)*a.n_dev : a.cap) : a.cap;
}

// The bin walks give each point a group of L lanes of a wavefront (64 / L
// points per wavefront): the group's lanes take the bin's entries in turn,
// so a point whose bin holds many boxes is searched in parallel while points
// with small bins share a wavefront.  L starts at the grid's `lanes` and
// doubles while the launch has threads for it (a search far below its
// capacity then walks each bin in fewer dependent rounds); the candidates
// and their order do not depend on L.
__device__ inline int walk_lanes(const DonorArgs &a, int64_t n)
{
    const int64_t threads = (int64_t)gridDim.x * blockDim.x;
    int L = a.lanes;
    while (L < 64 && (int64_t)(2 * L) * n <= threads) L *= 2;
    return L;
}

//
// a10: per point, the registration-frame position (inverse pose, the rigid
// motion of Sec. 4.3), its bin, the number of elements of the bin whose
// control-net boxes contain it, and the first kCandCache of them.
__global__ __launch_bounds__(kT) void k_dp_count(DonorArgs a)
{
    const int64_t n = donor_points(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.n_eff = (int32_t)n;
        a.dcnt->n_points = (unsigned long long)n;
        a.dcnt->n_newton = a.dcnt->n_iter = a.dcnt->n_orphan = a.dcnt->n_overflow = 0ull;
    }
    const Pose pose = *a.pose;
    const int L = walk_lanes(a, n), lane = threadIdx.x & 63, sub = lane & (L - 1);
    const unsigned long long gmask = (L == 64 ? ~0ull : ((1ull << L) - 1ull)) << (lane & ~(L - 1));
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t ppw = 64 / L;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = wave * ppw; base < n; base += n_waves * ppw) {
        const int64_t i = base + lane / L;
        int c = 0;
        if (i < n) {
            const d3 p = pose_inverse(pose, mk(a.pts[3 * i], a.pts[3 * i + 1], a.pts[3 * i + 2]));
            if (sub == 0) {
                a.plocal[3 * i] = p.x;
                a.plocal[3 * i + 1] = p.y;
                a.plocal[3 * i + 2] = p.z;
            }
            const int64_t b = point_bin(a.G, p);
            const int j0 = a.bstart[b];
            int j1 = a.bstart[b + 1];
            if (!chk(0 <= j0 && j0 <= j1 && j1 <= a.n_items, a.err, kChkDonorBin)) j1 = j0;
            // the group takes the bin's entries L at a time, in order, and
            // keeps the first kCandCache candidates (ascending element id)
            for (int r = j0; r < j1; r += L) {
                const int j = r + sub;
                int e = -1;
                bool has = false;
                if (j < j1) has = rec_has(a.brec, a.obox, j, p, &e, a.n_elem, a.err);
                const unsigned long long m = __ballot(has) & gmask;
                const int at = c + __popcll(m & below);
                if (has && at < kCandCache) a.cache[i * kCandCache + at] = e;
                c += __popcll(m);
            }
        }
        if (i < n && sub == 0) {
            a.cnt[i] = c;
            a.best[i] = 0x7fffffff;
        }
    }
}

// a10: the candidates as (point, element) pairs in ascending element id per
// point (the containment tests are deferred to the next kernel, as in
// Sec. 4.3); pairs past the capacity are dropped and their points searched
// one by one in k_dp_final.
__global__ __launch_bounds__(kT) void k_dp_fill(DonorArgs a)
{
    const int64_t n = donor_points(a);
    const int L = walk_lanes(a, n), lane = threadIdx.x & 63, sub = lane & (L - 1);
    const unsigned long long gmask = (L == 64 ? ~0ull : ((1ull << L) - 1ull)) << (lane & ~(L - 1));
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t ppw = 64 / L;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = wave * ppw; base < n; base += n_waves * ppw) {
        const int64_t i = base + lane / L;
        if (i >= n) continue;
        int64_t q = a.off[i];
        const int nc = a.cnt[i];
        if (nc <= kCandCache) {
            // the candidates k_dp_count kept
            for (int k = sub; k < nc; k += L)
                if (q + k < a.pair_cap) {
                    a.pair_pt[q + k] = (int32_t)i;
                    a.pair_el[q + k] = a.cache[i * kCandCache + k];
                }
            continue;
        }
        const d3 p = mk(a.plocal[3 * i], a.plocal[3 * i + 1], a.plocal[3 * i + 2]);
        const int64_t b = point_bin(a.G, p);
        const int j0 = a.bstart[b];
        int j1 = a.bstart[b + 1];
        if (!chk(0 <= j0 && j0 <= j1 && j1 <= a.n_items, a.err, kChkDonorBin)) j1 = j0;
        for (int r = j0; r < j1; r += L) {
            const int j = r + sub;
            int e = -1;
            bool has = false;
            if (j < j1) has = rec_has(a.brec, a.obox, j, p, &e, a.n_elem, a.err);
            const unsigned long long m = __ballot(has) & gmask;
            const int64_t at = q + __popcll(m & below);
            if (has && at < a.pair_cap) {
                a.pair_pt[at] = (int32_t)i;
                a.pair_el[at] = e;
            }
            q += __popcll(m);
        }
    }
}

// a11: Newton on every pair, three lanes each: lane d of a group holds
// coordinate d of the element's map as 27 monomial coefficients and
// evaluates component d of the residual and row d of J (q2_mono_comp, nested
// Horner steps); the group shares them and every lane takes
// the same step (the steps of newton_q2), so the three stay in lock step and
// agree bit for bit.  21 groups per wavefront, lane 63
// idle.  A point keeps the lowest element id that contains it, and a
// contained pair keeps its xi.
constexpr int kNewtonGroups = 21;

__global__ __launch_bounds__(kT) void k_dp_newton(DonorArgs a)
{
    const int64_t n = *a.n_eff;
    const int64_t tot = a.off[n] < a.pair_cap ? (int64_t)a.off[n] : a.pair_cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.dcnt->n_newton, (unsigned long long)tot);
    const int lane = threadIdx.x & 63;
    if (lane >= 3 * kNewtonGroups) return;
    const int grp = lane / 3, d = lane - 3 * grp, base = 3 * grp;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t qstep = n_waves * kNewtonGroups;
    int64_t q = wave * kNewtonGroups + grp;
    // the next pair's ids are loaded while the current pair is solved, so a
    // pair's coefficient loads start without waiting for its ids
    int ni = 0, ne = 0;
    if (q < tot) {
        ni = a.pair_pt[q];
        ne = a.pair_el[q];
    }
    for (; q < tot; q += qstep) {
        const int i = ni, e = ne;
        if (q + qstep < tot) {
            ni = a.pair_pt[q + qstep];
            ne = a.pair_el[q + qstep];
        }
        if (!chk(e >= 0 && e < a.n_elem, a.err, kChkPairElem)) continue;   // the whole group (same pair)
        const double *Mg = a.emono + (int64_t)e * 81 + 27 * d;
        double M[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) M[k] = Mg[k];
        // this lane's coordinate taken relative to the centre node (the
        // constant coefficient): the point's offset from the centre is formed
        // once, and the map's value is a sum of small terms
        const double pd = a.plocal[3 * (int64_t)i + d] - M[0];
        M[0] = 0.0;
        const double rtol = 1e-13 * a.ediam[e], rtol2 = rtol * rtol;
        double xi[3] = {0.0, 0.0, 0.0};
        bool conv = false;
        int iters = 0;
#pragma unroll 1
        for (int it = 0; it < OC_NEWTON_MAXIT; ++it) {
            ++iters;
            double xd, jd[3];
            if (it == 0) {
                // xi = 0: the centre node and half the differences of the
                // opposite face-centre nodes (as in newton_q2)
                xd = 0.0;
                jd[0] = M[1];
                jd[1] = M[3];
                jd[2] = M[9];
            } else {
                q2_mono_comp(M, xi, xd, jd);
            }
            const double rd = pd - xd;
            double r[3], J[9];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                r[k] = __shfl(rd, base + k, 64);
                J[3 * k] = __shfl(jd[0], base + k, 64);
                J[3 * k + 1] = __shfl(jd[1], base + k, 64);
                J[3 * k + 2] = __shfl(jd[2], base + k, 64);
            }
            const double r0 = r[0], r1 = r[1], r2 = r[2];
            if (r0 * r0 + r1 * r1 + r2 * r2 <= rtol2) {
                conv = true;
                break;
            }
            const double c00 = J[4] * J[8] - J[5] * J[7];
            const double c01 = J[5] * J[6] - J[3] * J[8];
            const double c02 = J[3] * J[7] - J[4] * J[6];
            const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
            if (det == 0.0) break;
            double id = __builtin_amdgcn_rcp(det);
            id = fma(id, fma(-det, id, 1.0), id);
            id = fma(id, fma(-det, id, 1.0), id);
            const double d0 = (c00 * r0 + (J[2] * J[7] - J[1] * J[8]) * r1 + (J[1] * J[5] - J[2] * J[4]) * r2) * id;
            const double d1 = (c01 * r0 + (J[0] * J[8] - J[2] * J[6]) * r1 + (J[2] * J[3] - J[0] * J[5]) * r2) * id;
            const double d2 = (c02 * r0 + (J[1] * J[6] - J[0] * J[7]) * r1 + (J[0] * J[4] - J[1] * J[3]) * r2) * id;
            const double lim = 1.0 + OC_NEWTON_CLAMP;
            const double n0 = fmin(fmax(xi[0] + d0, -lim), lim);
            const double n1 = fmin(fmax(xi[1] + d1, -lim), lim);
            const double n2 = fmin(fmax(xi[2] + d2, -lim), lim);
            const double step = fmax(fabs(n0 - xi[0]), fmax(fabs(n1 - xi[1]), fabs(n2 - xi[2])));
            xi[0] = n0;
            xi[1] = n1;
            xi[2] = n2;
            if (step <= 1e-14) {
                conv = true;
                break;
            }
        }
        if (d == 0) {
            const double m = fmax(fabs(xi[0]), fmax(fabs(xi[1]), fabs(xi[2])));
            if (conv && m <= 1.0 + OC_CONTAIN_TOL) {
                a.pair_xi[3 * q] = xi[0];
                a.pair_xi[3 * q + 1] = xi[1];
                a.pair_xi[3 * q + 2] = xi[2];
                atomicMin(&a.best[i], e);
            }
            a.pair_it[q] = (uint8_t)iters;
        }
    }
}

// donor id and reference coordinates per point: the xi kept by the winning
// pair.  Points whose pairs did not all fit take their candidates one by one
// in ascending id order.
__global__ __launch_bounds__(kT) void k_dp_final(DonorArgs a)
{
    const int64_t n = *a.n_eff;
    int extra = 0, over = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t d = -1;
        double xi[3] = {NAN, NAN, NAN};
        int scratch = 0;
        if ((int64_t)a.off[i + 1] > a.pair_cap) {
            ++over;
            const d3 p = mk(a.plocal[3 * i], a.plocal[3 * i + 1], a.plocal[3 * i + 2]);
            const int64_t b = point_bin(a.G, p);
            const int j0 = a.bstart[b];
            int j1 = a.bstart[b + 1];
            if (!chk(0 <= j0 && j0 <= j1 && j1 <= a.n_items, a.err, kChkDonorBin)) j1 = j0;
            for (int j = j0; j < j1; ++j) {
                int e;
                if (!rec_has(a.brec, a.obox, j, p, &e, a.n_elem, a.err)) continue;
                ++extra;
                if (newton_q2<true>(a.enodes + (int64_t)e * 81, p, a.ediam[e], xi, scratch)) {
                    d = e;
                    break;
                }
                xi[0] = xi[1] = xi[2] = NAN;
            }
        } else if (a.best[i] != 0x7fffffff) {
            d = a.best[i];
            for (int64_t q = a.off[i]; q < (int64_t)a.off[i + 1]; ++q)
                if (a.pair_el[q] == d) {
                    xi[0] = a.pair_xi[3 * q];
                    xi[1] = a.pair_xi[3 * q + 1];
                    xi[2] = a.pair_xi[3 * q + 2];
                    break;
                }
        }
        a.donor[i] = d;
        a.ref[3 * i] = xi[0];
        a.ref[3 * i + 1] = xi[1];
        a.ref[3 * i + 2] = xi[2];
    }
    // solves and points of the overflow path (rare: only points whose pairs
    // did not fit)
    unsigned long long sx = extra, so = over;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        sx += __shfl_xor(sx, d, 64);
        so += __shfl_xor(so, d, 64);
    }
    if ((threadIdx.x & 63) == 0 && sx) atomicAdd(&a.dcnt->n_newton, sx);
    if ((threadIdx.x & 63) == 0 && so) atomicAdd(&a.dcnt->n_overflow, so);
}

// Statistics of the last search (only when asked for): Newton iterations
// over the pairs and orphan points.
__global__ __launch_bounds__(kT) void k_donor_stats(DonorArgs a)
{
    __shared__ unsigned long long acc[2];
    if (threadIdx.x < 2) acc[threadIdx.x] = 0ull;
    __syncthreads();
    const int64_t n = *a.n_eff;
    const int64_t tot = a.off[n] < a.pair_cap ? (int64_t)a.off[n] : a.pair_cap;
    unsigned long long it = 0, orph = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x)
        it += a.pair_it[q];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        orph += a.donor[i] < 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        it += __shfl_xor(it, d, 64);
        orph += __shfl_xor(orph, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&acc[0], it);
        atomicAdd(&acc[1], orph);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&a.dcnt->n_iter, acc[0]);
        atomicAdd(&a.dcnt->n_orphan, acc[1]);
    }
}

__global__ void k_donor_stats_reset(DonorCounters *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) c->n_iter = c->n_orphan = 0ull;
}

__global__ void k_donor_reset(DonorCounters *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->n_points = 0ull;
        c->n_newton = c->n_iter = c->n_orphan = c->n_overflow = 0ull;
    }
}

// ------------------------------------------------------------ host side --
#define LAUNCH(name, grid, block, ...)                                                       \
    do {                                                                                     \
        size_t slot_;                                                                        \
        time_begin(ctx, st, #name, &slot_);                                                  \
        hipLaunchKernelGGL(name, grid, block, 0, st, __VA_ARGS__);                           \
        time_end(ctx, st, slot_);                                                            \
    } while (0)

static unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per > 0 ? (n + per - 1) / per : 1); }

oc_status grid_build_device(oc_ctx *ctx, Grid &g, const int32_t *conn_dev, const double *nodes_dev)
{
    hipStream_t st = ctx->reg_stream;
    LAUNCH(k_gather_nodes, dim3(blocks(g.n_elem * 27, kT)), dim3(kT), nodes_dev, conn_dev, g.n_elem, g.enodes);
    int *bad = ctx->dev_scalar;
    OC_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    LAUNCH(k_elem_boxes, dim3(blocks(g.n_elem, kT)), dim3(kT), g.enodes, g.n_elem, g.ebox_stride, g.ebox, g.cbox,
           g.ediam, bad);
    LAUNCH(k_elem_obb, dim3(blocks(g.n_elem, kT)), dim3(kT), g.enodes, g.n_elem, g.cbox, g.obox);
    LAUNCH(k_wave_boxes, dim3(blocks(g.n_elem, 256)), dim3(64), g.ebox, g.ebox_stride, g.n_elem, g.wbox);
    LAUNCH(k_elem_mono, dim3(blocks(g.n_elem * 3, kT)), dim3(kT), g.enodes, g.n_elem, g.emono);
    int hbad = 0;
    OC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    OC_HIP(hipStreamSynchronize(st));
    if (hbad) {
        set_error(std::to_string(hbad) + " element(s) with a non-positive Jacobian at the centre");
        return OC_EGEOM;
    }
    return OC_OK;
}

oc_status grid_build_donor_bins(oc_ctx *ctx, Grid &g)
{
    hipStream_t st = ctx->reg_stream;
    // grid box from the control-net boxes (host reduction at registration)
    std::vector<float> cb((size_t)g.n_elem * 6);
    OC_HIP(hipMemcpy(cb.data(), g.cbox, cb.size() * sizeof(float), hipMemcpyDeviceToHost));
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t e = 0; e < g.n_elem; ++e)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], cb[e * 6 + a]);
            hi[a] = std::max(hi[a], cb[e * 6 + 3 + a]);
        }
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= std::max((double)hi[a] - lo[a], 1e-30);
    double edge = std::cbrt(vol / (double)g.n_elem) * ctx->donor_bin_scale;
    int64_t nb = 1;
    for (int a = 0; a < 3; ++a) {
        double ext = (double)hi[a] - lo[a];
        int n = (int)std::ceil(ext / edge);
        n = std::max(1, std::min(n, 1024));
        g.dgrid.o[a] = lo[a];
        g.dgrid.n[a] = n;
        g.dgrid.inv[a] = ext > 0 ? (float)(n / ext) : 0.f;
        nb *= n;
    }
    g.n_dbins = nb;
    int32_t *count = nullptr, *start = nullptr, *tmp = nullptr;
    OC_TRY(dev_alloc(ctx, g.owned, sizeof(int32_t) * (nb + 1), (void **)&count));
    OC_TRY(dev_alloc(ctx, g.owned, sizeof(int32_t) * (nb + 1), (void **)&start));
    OC_TRY(dev_alloc(ctx, g.owned, sizeof(int32_t) * scan_tmp_ints(nb), (void **)&tmp));
    OC_HIP(hipMemsetAsync(count, 0, sizeof(int32_t) * (nb + 1), st));
    LAUNCH(k_dbin_count, dim3(blocks(g.n_elem, kT)), dim3(kT), g.cbox, g.n_elem, g.dgrid, count);
    OC_TRY(scan_exclusive(ctx, st, count, start, nb, nullptr, tmp));
    int32_t total = 0;
    OC_HIP(hipMemcpyAsync(&total, start + nb, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    OC_HIP(hipStreamSynchronize(st));
    g.n_ditems = total;
    OC_TRY(dev_alloc(ctx, g.owned, sizeof(int32_t) * std::max<int64_t>(total, 1), (void **)&g.dbin_items));
    OC_HIP(hipMemsetAsync(count, 0, sizeof(int32_t) * (nb + 1), st));
    LAUNCH(k_dbin_fill, dim3(blocks(g.n_elem, kT)), dim3(kT), g.cbox, g.n_elem, g.dgrid, start, count, g.dbin_items);
    LAUNCH(k_dbin_sort, dim3(blocks(nb, kT)), dim3(kT), start, nb, g.dbin_items);
    OC_TRY(dev_alloc(ctx, g.owned, sizeof(float4) * 2 * (size_t)std::max<int64_t>(total, 1), (void **)&g.dbin_rec));
    LAUNCH(k_dbin_records, dim3(blocks(std::max<int64_t>(total, 1), kT)), dim3(kT), g.dbin_items, (int64_t)total,
           g.cbox, g.dbin_rec);
    g.dbin_start = start;
    // lanes per point in the donor bin walks: about four bin entries per
    // lane for the typical query (bins weighted by their entry count, since
    // points fall where elements are); on the dimpled case one or two
    // entries per lane run more, emptier waves and are slower, eight starts
    // to lengthen the per-point chains
    std::vector<int32_t> hs((size_t)nb + 1);
    OC_HIP(hipMemcpyAsync(hs.data(), start, sizeof(int32_t) * (nb + 1), hipMemcpyDeviceToHost, st));
    OC_HIP(hipStreamSynchronize(st));
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k = 0; k < nb; ++k) {
        const double c = hs[k + 1] - hs[k];
        s1 += c;
        s2 += c * c;
    }
    const double mean = s1 > 0 ? s2 / s1 : 1.0;
    g.dlanes = 1;
    while (g.dlanes < 64 && 4.0 * g.dlanes < mean) g.dlanes *= 2;
    OC_HIP(hipStreamSynchronize(st));
    OC_HIP(hipGetLastError());
    return OC_OK;
}

// Ordered compaction of the listed elements of g (see listed()) into list
// (at most cap; null: the slot's own list, taken after the slot's lists have
// been sized for g); the count stays on the device at *total.
oc_status list_elements_run(oc_slot *sl, const Grid &g, const int8_t *iblank, const int8_t *prev, int32_t *list,
                            int64_t cap, const int32_t **total)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    OC_TRY(slot_reserve_grid(sl, g));
    if (!list) {
        list = sl->list_fringe;
        cap = std::min<int64_t>(cap, sl->list_cap);
    }
    const int64_t nt = (g.n_elem + kFrTile - 1) / kFrTile;
    int32_t *tcount = sl->fr_tiles, *toff = sl->fr_tiles + (nt + 1);
    int32_t *tmp = sl->fr_tiles + 2 * (nt + 1);
    LAUNCH(k_fr_count, dim3((unsigned)std::max<int64_t>(nt, 1)), dim3(kT), iblank, prev, g.n_elem, tcount);
    OC_TRY(scan_exclusive(ctx, st, tcount, toff, nt, nullptr, tmp));
    LAUNCH(k_fr_write, dim3((unsigned)std::max<int64_t>(nt, 1)), dim3(kT), iblank, prev, g.n_elem, toff, list, cap);
    OC_HIP(hipGetLastError());
    *total = toff + nt;
    return OC_OK;
}

// 27 Gauss points of the first min(*count, cap / 27) listed elements;
// n_out (device, may be null) receives 27 * *count.
oc_status element_points_run(oc_slot *sl, const Grid &g, const Pose *pose_dev, const int32_t *list,
                             const int32_t *count, double *pts, int64_t cap, int32_t *n_out, int32_t *src)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    const int64_t cap_pts = std::min<int64_t>(cap, 27 * g.n_elem);
    LAUNCH(k_fringe_points, dim3(std::min<unsigned>(blocks(std::max<int64_t>(cap_pts, 1), kT), kLoopBlocks)), dim3(kT),
           g.enodes, g.n_elem, list, count, cap, pose_dev, pts, src, n_out);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status fringe_points_run(oc_slot *sl, Grid &g, const Pose *pose_dev, const int8_t *iblank, double *pts,
                            int64_t cap, int32_t *n_dev, int64_t *n_host, int32_t *src)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    OC_TRY(slot_reserve_grid(sl, g));
    // tile-local lists (one pass), a scan of the tile counts, and the points
    // read through the tile offsets: no separate ordered write
    const int64_t nt = std::max<int64_t>((g.n_elem + kFrTile - 1) / kFrTile, 1);
    int32_t *tcount = sl->fr_tiles, *toff = sl->fr_tiles + (nt + 1);
    int32_t *tmp = sl->fr_tiles + 2 * (nt + 1);
    LAUNCH(k_fr_tiles, dim3((unsigned)nt), dim3(kT), iblank, g.n_elem, tcount, sl->list_fringe);
    // up to point_tiles (<= kToffLds) tiles every block of the points kernel
    // forms the tile offsets from the counts itself (no scan launch)
    const bool counts_only = nt <= std::min(ctx->point_tiles, kToffLds);
    if (!counts_only) OC_TRY(scan_exclusive(ctx, st, tcount, toff, nt, nullptr, tmp));
    int32_t *cnt_out = n_dev ? n_dev : sl->scalar;
    const int64_t cap_pts = std::min<int64_t>(cap, 27 * g.n_elem);
    const dim3 grid_pts(std::min<unsigned>(blocks(std::max<int64_t>(cap_pts, 1), kT), kLoopBlocks));
    if (counts_only)
        LAUNCH(k_fringe_points_t<2>, grid_pts, dim3(kT), g.enodes, g.n_elem, sl->list_fringe, tcount, (int)nt, cap,
               pose_dev, pts, src, cnt_out);
    else
        LAUNCH(k_fringe_points_t<1>, grid_pts, dim3(kT), g.enodes, g.n_elem, sl->list_fringe, toff, (int)nt, cap,
               pose_dev, pts, src, cnt_out);
    OC_HIP(hipGetLastError());
    if (n_host) {
        int32_t n = 0;
        OC_HIP(hipMemcpyAsync(&n, cnt_out, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        OC_HIP(hipStreamSynchronize(st));
        *n_host = n;
        if (n > cap) {
            set_error("oc_fringe_points: capacity " + std::to_string(cap) + " < " + std::to_string(n) + " points");
            return OC_ECAPACITY;
        }
    }
    return OC_OK;
}

oc_status donor_run(oc_slot *sl, Grid &g, const Pose *pose_dev, const double *pts, int64_t cap, const int32_t *n_dev,
                    int32_t *donor, double *ref)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    sl->last_donor_args.clear();
    if (cap <= 0) {
        LAUNCH(k_donor_reset, dim3(1), dim3(64), sl->dcounters);
        return OC_OK;
    }
    OC_TRY(slot_reserve_points(sl, cap));
    DonorArgs a;
    a.enodes = g.enodes;
    a.emono = g.emono;
    a.cbox = g.cbox;
    a.obox = g.obox;
    a.ediam = g.ediam;
    a.G = g.dgrid;
    a.bstart = g.dbin_start;
    a.brec = g.dbin_rec;
    a.n_items = g.n_ditems;
    a.n_elem = g.n_elem;
    a.err = reinterpret_cast<uint32_t *>(ctx->dev_scalar) + 8;
    a.pose = pose_dev;
    a.pts = pts;
    a.cap = cap;
    a.n_dev = n_dev;
    a.n_eff = sl->scalar + 1;
    a.plocal = sl->dp_local;
    a.cnt = sl->dp_cnt;
    a.off = sl->dp_off;
    a.best = sl->dp_best;
    a.cache = sl->dp_cache;
    a.pair_pt = sl->dpair_pt;
    a.pair_el = sl->dpair_el;
    a.pair_xi = sl->dpair_xi;
    a.pair_it = sl->dpair_it;
    a.pair_cap = ctx->donor_pairs > 0 ? std::min<int64_t>(sl->dpair_cap, ctx->donor_pairs) : sl->dpair_cap;
    a.lanes = g.dlanes;
    a.pad = 0;
    a.donor = donor;
    a.ref = ref;
    a.dcnt = sl->dcounters;
    // every kernel loops over its work: grids are sized for the capacities
    // (the counts are on the device) but capped at kLoopBlocks, so a search
    // far below its capacity does not launch a wave per possible point or
    // pair; the tuning cap only lowers the search's share of the device
    const unsigned bcap = ctx->donor_waves > 0 ? (unsigned)std::max(1, ctx->donor_waves / (kT / 64)) : 1u << 30;
    const unsigned gp = std::min({blocks(cap, kT), kLoopBlocks, bcap});
    const unsigned gw = std::min({blocks(cap * g.dlanes, kT), kLoopBlocks, bcap});
    const unsigned gn = std::min({blocks(sl->dpair_cap, (kT / 64) * kNewtonGroups), kLoopBlocks, bcap});
    LAUNCH(k_dp_count, dim3(gw), dim3(kT), a);
    OC_TRY(scan_exclusive(ctx, st, sl->dp_cnt, sl->dp_off, cap, a.n_eff, sl->dp_scan_tmp));
    LAUNCH(k_dp_fill, dim3(gw), dim3(kT), a);
    LAUNCH(k_dp_newton, dim3(gn), dim3(kT), a);
    LAUNCH(k_dp_final, dim3(gp), dim3(kT), a);
    OC_HIP(hipGetLastError());
    sl->last_donor_args.assign(reinterpret_cast<const unsigned char *>(&a),
                               reinterpret_cast<const unsigned char *>(&a) + sizeof a);
    return OC_OK;
}

// Counters of the slot's last donor search (stream ordered).
oc_status donor_stats_run(oc_slot *sl)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    LAUNCH(k_donor_stats_reset, dim3(1), dim3(64), sl->dcounters);
    if (sl->last_donor_args.size() == sizeof(DonorArgs)) {
        DonorArgs a;
        memcpy(&a, sl->last_donor_args.data(), sizeof a);
        LAUNCH(k_donor_stats, dim3(256), dim3(kT), a);
    }
    OC_HIP(hipGetLastError());
    return OC_OK;
}

// ------------------------------------------------ allocation-free search --
// oc_donor_search_noalloc runs the same kernels as oc_donor_search on a
// fixed scratch array that the code object carries (one copy per device,
// held until the process ends), so the call allocates nothing.  Layout, each
// part 256-byte aligned: the pose, the counters and the effective point
// count, then the per-point and per-pair arrays of a search of up to
// kNaPoints points with kPairsPerPoint pairs per point.
constexpr int64_t kNaPoints = int64_t(1) << 17;
constexpr int64_t kNaPairs = kNaPoints * kPairsPerPoint;
constexpr size_t na_up(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kNaPose = 0;
constexpr size_t kNaCounters = kNaPose + na_up(sizeof(Pose));
constexpr size_t kNaNeff = kNaCounters + na_up(sizeof(DonorCounters));
constexpr size_t kNaLocal = kNaNeff + 256;
constexpr size_t kNaCnt = kNaLocal + na_up(sizeof(double) * 3 * kNaPoints);
constexpr size_t kNaOff = kNaCnt + na_up(sizeof(int32_t) * (kNaPoints + 1));
constexpr size_t kNaBest = kNaOff + na_up(sizeof(int32_t) * (kNaPoints + 1));
constexpr size_t kNaCache = kNaBest + na_up(sizeof(int32_t) * kNaPoints);
constexpr size_t kNaScan = kNaCache + na_up(sizeof(int32_t) * kCandCache * kNaPoints);
constexpr size_t kNaPairPt = kNaScan + na_up(sizeof(int32_t) * ((kNaPoints + 4095) / 4096 + 1));
constexpr size_t kNaPairEl = kNaPairPt + na_up(sizeof(int32_t) * kNaPairs);
constexpr size_t kNaPairXi = kNaPairEl + na_up(sizeof(int32_t) * kNaPairs);
constexpr size_t kNaPairIt = kNaPairXi + na_up(sizeof(double) * 3 * kNaPairs);
constexpr size_t kNaBytes = kNaPairIt + na_up(sizeof(uint8_t) * kNaPairs);
static_assert(kNaBytes < (size_t(48) << 20), "allocation-free scratch exceeds its stated 48 MiB bound");

// The scratch itself.  Host code never passes this name to a kernel (on the
// host it is only a stand-in for the symbol): it uses the device address
// taken by noalloc_init for the device at hand.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
static unsigned char *g_na_base[kNaMaxDevices];
static std::mutex g_na_mutex;

// device address of this device's scratch array (once per device; the
// device must be current)
oc_status noalloc_init(int device)
{
    if (device < 0 || device >= kNaMaxDevices) {
        set_error("device ordinal beyond the allocation-free scratch table");
        return OC_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_na_mutex);
    if (g_na_base[device]) return OC_OK;
    void *ptr = nullptr;
    OC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_na_base[device] = static_cast<unsigned char *>(ptr);
    return OC_OK;
}

int64_t noalloc_max_points() { return kNaPoints; }

__global__ void k_na_pose(Pose p, Pose *dst)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = p;
}

oc_status donor_noalloc_run(oc_ctx *ctx, Grid &g, const double *pose_host, const double *pts, int64_t n,
                            int32_t *donor, double *ref)
{
    if (n < 0 || n > kNaPoints) {
        set_error("oc_donor_search_noalloc: " + std::to_string(n) + " points; at most " + std::to_string(kNaPoints) +
                  " per call (split larger searches: every point is searched on its own)");
        return OC_EINVAL;
    }
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_na_mutex);
        if (ctx->device >= 0 && ctx->device < kNaMaxDevices) base = g_na_base[ctx->device];
    }
    if (!base) {
        set_error("oc_donor_search_noalloc: scratch of this device not initialised");
        return OC_EDEVICE;
    }
    if (n == 0) return OC_OK;
    hipStream_t st = ctx->dflt->stream;
    Pose P;
    for (int i = 0; i < 9; ++i) P.r[i] = pose_host[i];
    for (int i = 0; i < 3; ++i) P.t[i] = pose_host[9 + i];
    hipLaunchKernelGGL(k_na_pose, dim3(1), dim3(64), 0, st, P, reinterpret_cast<Pose *>(base + kNaPose));
    DonorArgs a;
    a.enodes = g.enodes;
    a.emono = g.emono;
    a.cbox = g.cbox;
    a.obox = g.obox;
    a.ediam = g.ediam;
    a.G = g.dgrid;
    a.bstart = g.dbin_start;
    a.brec = g.dbin_rec;
    a.n_items = g.n_ditems;
    a.n_elem = g.n_elem;
    a.err = reinterpret_cast<uint32_t *>(ctx->dev_scalar) + 8;
    a.pose = reinterpret_cast<const Pose *>(base + kNaPose);
    a.pts = pts;
    a.cap = n;
    a.n_dev = nullptr;
    a.n_eff = reinterpret_cast<int32_t *>(base + kNaNeff);
    a.plocal = reinterpret_cast<double *>(base + kNaLocal);
    a.cnt = reinterpret_cast<int32_t *>(base + kNaCnt);
    a.off = reinterpret_cast<int32_t *>(base + kNaOff);
    a.best = reinterpret_cast<int32_t *>(base + kNaBest);
    a.cache = reinterpret_cast<int32_t *>(base + kNaCache);
    a.pair_pt = reinterpret_cast<int32_t *>(base + kNaPairPt);
    a.pair_el = reinterpret_cast<int32_t *>(base + kNaPairEl);
    a.pair_xi = reinterpret_cast<double *>(base + kNaPairXi);
    a.pair_it = reinterpret_cast<uint8_t *>(base + kNaPairIt);
    a.pair_cap = ctx->donor_pairs > 0 ? std::min<int64_t>(kNaPairs, ctx->donor_pairs) : kNaPairs;
    a.lanes = g.dlanes;
    a.pad = 0;
    a.donor = donor;
    a.ref = ref;
    a.dcnt = reinterpret_cast<DonorCounters *>(base + kNaCounters);
    const unsigned bcap = ctx->donor_waves > 0 ? (unsigned)std::max(1, ctx->donor_waves / (kT / 64)) : 1u << 30;
    const unsigned gp = std::min({blocks(n, kT), kLoopBlocks, bcap});
    const unsigned gw = std::min({blocks(n * g.dlanes, kT), kLoopBlocks, bcap});
    const unsigned gn = std::min({blocks(kPairsPerPoint * n, (kT / 64) * kNewtonGroups), kLoopBlocks, bcap});
    // every array is written before it is read within the call (k_dp_count
    // sets the count, counters and per-point minima; the scan the offsets;
    // k_dp_fill the pairs), so nothing left by an earlier call is used
    hipLaunchKernelGGL(k_dp_count, dim3(gw), dim3(kT), 0, st, a);
    OC_TRY(scan_exclusive(nullptr, st, a.cnt, a.off, n, a.n_eff, reinterpret_cast<int32_t *>(base + kNaScan)));
    hipLaunchKernelGGL(k_dp_fill, dim3(gw), dim3(kT), 0, st, a);
    hipLaunchKernelGGL(k_dp_newton, dim3(gn), dim3(kT), 0, st, a);
    hipLaunchKernelGGL(k_dp_final, dim3(gp), dim3(kT), 0, st, a);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

}  // namespace oc
