// Receptor points and donor search (Sec. 4.3 "Donor/Receptor Point
// Connectivity on GPUs").
//
//   k_fr_count / scan / k_fr_write   ordered compaction of fringe elements
//   k_fringe_points                  27 Gauss points per fringe element mapped
//                                    by the quadratic isoparametric map
//                                    (eq. reftophys) and posed to world frame
//   k_donor                          per point: inverse pose into the donor
//                                    grid's registration frame (the rigid
//                                    motion trick of Sec. 4.3), one bin lookup
//                                    of control-net boxes, then Newton
//                                    (eq. ref-update, eq. Jac) on the boxes that
//                                    contain the point in ascending element id;
//                                    the first element that contains it wins.
// Registration-time kernels build the element node copies, the FP32 element
// boxes and the donor bins.
#include "dev_common.h"

namespace oc {

constexpr int kT = 256;

// ----------------------------------------------------- quadratic map ------
__device__ inline void lag2(double s, double *l, double *dl)
{
    l[0] = 0.5 * s * (s - 1.0);
    l[1] = 1.0 - s * s;
    l[2] = 0.5 * s * (s + 1.0);
    dl[0] = s - 0.5;
    dl[1] = -2.0 * s;
    dl[2] = s + 0.5;
}

// x(xi) and J = dx/dxi of an element stored as x[27], y[27], z[27]
// (sum factorisation: contract the xi index first, then eta, then zeta).
template <bool WITH_J>
__device__ inline void q2_map(const double *__restrict__ X, const double *xi, double *x, double *J)
{
    double la[3], da[3], lb[3], db[3], lc[3], dc[3];
    lag2(xi[0], la, da);
    lag2(xi[1], lb, db);
    lag2(xi[2], lc, dc);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *C = X + 27 * d;
        double s = 0.0, s_a = 0.0, s_b = 0.0, s_c = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double t = 0.0, t_a = 0.0, t_b = 0.0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double v0 = C[3 * b + 9 * c], v1 = C[1 + 3 * b + 9 * c], v2 = C[2 + 3 * b + 9 * c];
                const double u = v0 * la[0] + v1 * la[1] + v2 * la[2];
                t += u * lb[b];
                if (WITH_J) {
                    const double u_a = v0 * da[0] + v1 * da[1] + v2 * da[2];
                    t_a += u_a * lb[b];
                    t_b += u * db[b];
                }
            }
            s += t * lc[c];
            if (WITH_J) {
                s_a += t_a * lc[c];
                s_b += t_b * lc[c];
                s_c += t * dc[c];
            }
        }
        x[d] = s;
        if (WITH_J) {
            J[3 * d + 0] = s_a;
            J[3 * d + 1] = s_b;
            J[3 * d + 2] = s_c;
        }
    }
}

// Newton inversion: xi0 = 0; stop when |x_p - x(xi)| <= 1e-13 diam (checked
// before each step) or the clamped step is <= 1e-14; at most
// OC_NEWTON_MAXIT iterations; contained if converged and
// max|xi| <= 1 + OC_CONTAIN_TOL.  The 3x3 system is solved with the adjugate.
__device__ inline bool newton_q2(const double *__restrict__ X, d3 p, double diam, double *xi)
{
    xi[0] = xi[1] = xi[2] = 0.0;
    bool conv = false;
    for (int it = 0; it < OC_NEWTON_MAXIT; ++it) {
        double x[3], J[9];
        q2_map<true>(X, xi, x, J);
        const double r0 = p.x - x[0], r1 = p.y - x[1], r2 = p.z - x[2];
        if (sqrt(r0 * r0 + r1 * r1 + r2 * r2) <= 1e-13 * diam) {
            conv = true;
            break;
        }
        const double c00 = J[4] * J[8] - J[5] * J[7];
        const double c01 = J[5] * J[6] - J[3] * J[8];
        const double c02 = J[3] * J[7] - J[4] * J[6];
        const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
        if (det == 0.0) break;
        const double id = 1.0 / det;
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
    q2_map<true>(X, xi, x, J);
    const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                       J[2] * (J[3] * J[7] - J[4] * J[6]);
    if (!(det > 0.0)) atomicAdd(bad_jac, 1);
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

// ----------------------------------------------- fringe compaction --------
constexpr int kFrItems = 16;
constexpr int kFrTile = kT * kFrItems;

__global__ __launch_bounds__(kT) void k_fr_count(const int8_t *__restrict__ iblank, int64_t n_elem,
                                                 int32_t *__restrict__ tcount)
{
    const int64_t base = (int64_t)blockIdx.x * kFrTile;
    int c = 0;
    for (int k = 0; k < kFrItems; ++k) {
        const int64_t i = base + (int64_t)k * kT + threadIdx.x;
        if (i < n_elem) c += iblank[i] == OC_FRINGE;
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

__global__ __launch_bounds__(kT) void k_fr_write(const int8_t *__restrict__ iblank, int64_t n_elem,
                                                 const int32_t *__restrict__ toff, int32_t *__restrict__ list)
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
    int off = toff[blockIdx.x];
    for (int w = 0; w < wid; ++w) off += ws[w];
    int pos = off + inc - c;
    for (int k = 0; k < kFrItems; ++k) {
        const int64_t i = my + k;
        if (i < n_elem && iblank[i] == OC_FRINGE) list[pos++] = (int32_t)i;
    }
}

// a9: Gauss point k = a + 3b + 9c of fringe element list[i], posed
__global__ __launch_bounds__(kT) void k_fringe_points(const double *__restrict__ enodes,
                                                      const int32_t *__restrict__ list, int64_t n_pts, Pose pose,
                                                      double *__restrict__ pts, int32_t *__restrict__ src)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pts) return;
    const int64_t q = i / 27;
    const int k = (int)(i - q * 27);
    const int e = list[q];
    const double g = 0.7745966692414834;  // sqrt(3/5), 3-point Gauss-Legendre
    const double xi[3] = {(k % 3 - 1) * g, ((k / 3) % 3 - 1) * g, (k / 9 - 1) * g};
    double x[3];
    q2_map<false>(enodes + (int64_t)e * 81, xi, x, nullptr);
    const d3 w = pose_apply(pose, mk(x[0], x[1], x[2]));
    pts[3 * i] = w.x;
    pts[3 * i + 1] = w.y;
    pts[3 * i + 2] = w.z;
    if (src) src[i] = e;
}

// a10 + a11: donor search, one thread per point
__global__ __launch_bounds__(kT) void k_donor(const double *__restrict__ enodes, const float *__restrict__ cbox,
                                              const double *__restrict__ ediam, BinGrid G,
                                              const int32_t *__restrict__ bstart, const int32_t *__restrict__ bitems,
                                              Pose pose, const double *__restrict__ pts, int64_t n,
                                              int32_t *__restrict__ donor, double *__restrict__ ref)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const d3 p = pose_inverse(pose, mk(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]));
    const int bx = bin_of((float)p.x, G.o[0], G.inv[0], G.n[0]);
    const int by = bin_of((float)p.y, G.o[1], G.inv[1], G.n[1]);
    const int bz = bin_of((float)p.z, G.o[2], G.inv[2], G.n[2]);
    const int64_t b = bx + (int64_t)G.n[0] * (by + (int64_t)G.n[1] * bz);
    int32_t d = -1;
    double r[3] = {NAN, NAN, NAN};
    for (int j = bstart[b]; j < bstart[b + 1]; ++j) {
        const int e = bitems[j];
        const float *c = cbox + (int64_t)e * 6;
        if (p.x < (double)c[0] || p.y < (double)c[1] || p.z < (double)c[2] || p.x > (double)c[3] ||
            p.y > (double)c[4] || p.z > (double)c[5])
            continue;
        double xi[3];
        if (newton_q2(enodes + (int64_t)e * 81, p, ediam[e], xi)) {
            d = e;
            r[0] = xi[0];
            r[1] = xi[1];
            r[2] = xi[2];
            break;
        }
    }
    donor[i] = d;
    ref[3 * i] = r[0];
    ref[3 * i + 1] = r[1];
    ref[3 * i + 2] = r[2];
}

// ------------------------------------------------------------ host side --
#define LAUNCH(name, grid, block, ...)                                                       \
    do {                                                                                     \
        size_t slot_;                                                                        \
        time_begin(ctx, #name, &slot_);                                                      \
        hipLaunchKernelGGL(name, grid, block, 0, ctx->stream, __VA_ARGS__);                  \
        time_end(ctx, slot_);                                                                \
    } while (0)

static unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per > 0 ? (n + per - 1) / per : 1); }

oc_status grid_build_device(oc_ctx *ctx, Grid &g, const int32_t *conn_dev, const double *nodes_dev)
{
    LAUNCH(k_gather_nodes, dim3(blocks(g.n_elem * 27, kT)), dim3(kT), nodes_dev, conn_dev, g.n_elem, g.enodes);
    int *bad = ctx->dev_scalar;
    OC_HIP(hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    LAUNCH(k_elem_boxes, dim3(blocks(g.n_elem, kT)), dim3(kT), g.enodes, g.n_elem, g.ebox_stride, g.ebox, g.cbox,
           g.ediam, bad);
    int hbad = 0;
    OC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    OC_HIP(hipStreamSynchronize(ctx->stream));
    if (hbad) {
        set_error(std::to_string(hbad) + " element(s) with a non-positive Jacobian at the centre");
        return OC_EGEOM;
    }
    return OC_OK;
}

oc_status grid_build_donor_bins(oc_ctx *ctx, Grid &g)
{
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
    OC_HIP(hipMemsetAsync(count, 0, sizeof(int32_t) * (nb + 1), ctx->stream));
    LAUNCH(k_dbin_count, dim3(blocks(g.n_elem, kT)), dim3(kT), g.cbox, g.n_elem, g.dgrid, count);
    OC_TRY(scan_exclusive(ctx, count, start, nb, nullptr, tmp));
    int32_t total = 0;
    OC_HIP(hipMemcpyAsync(&total, start + nb, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    OC_HIP(hipStreamSynchronize(ctx->stream));
    g.n_ditems = total;
    OC_TRY(dev_alloc(ctx, g.owned, sizeof(int32_t) * std::max<int64_t>(total, 1), (void **)&g.dbin_items));
    OC_HIP(hipMemsetAsync(count, 0, sizeof(int32_t) * (nb + 1), ctx->stream));
    LAUNCH(k_dbin_fill, dim3(blocks(g.n_elem, kT)), dim3(kT), g.cbox, g.n_elem, g.dgrid, start, count, g.dbin_items);
    LAUNCH(k_dbin_sort, dim3(blocks(nb, kT)), dim3(kT), start, nb, g.dbin_items);
    g.dbin_start = start;
    OC_HIP(hipStreamSynchronize(ctx->stream));
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status fringe_points_run(oc_ctx *ctx, Grid &g, const Pose &pose, const int8_t *iblank, double *pts, int64_t cap,
                            int64_t *n_out, int32_t *src)
{
    const int64_t nt = (g.n_elem + kFrTile - 1) / kFrTile;
    int32_t *tcount = g.fr_blocksum, *toff = g.fr_blocksum + (nt + 1);
    int32_t *tmp = g.fr_blocksum + 2 * (nt + 1);
    LAUNCH(k_fr_count, dim3((unsigned)std::max<int64_t>(nt, 1)), dim3(kT), iblank, g.n_elem, tcount);
    OC_TRY(scan_exclusive(ctx, tcount, toff, nt, nullptr, tmp));
    LAUNCH(k_fr_write, dim3((unsigned)std::max<int64_t>(nt, 1)), dim3(kT), iblank, g.n_elem, toff, g.list_fringe);
    int32_t nfr = 0;
    OC_HIP(hipMemcpyAsync(&nfr, toff + nt, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    OC_HIP(hipStreamSynchronize(ctx->stream));
    const int64_t npts = (int64_t)nfr * 27;
    *n_out = npts;
    if (npts > cap) {
        set_error("oc_fringe_points: capacity " + std::to_string(cap) + " < " + std::to_string(npts) + " points");
        return OC_ECAPACITY;
    }
    if (npts > 0)
        LAUNCH(k_fringe_points, dim3(blocks(npts, kT)), dim3(kT), g.enodes, g.list_fringe, npts, pose, pts, src);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status donor_run(oc_ctx *ctx, Grid &g, const Pose &pose, const double *pts, int64_t n, int32_t *donor,
                    double *ref)
{
    if (n <= 0) return OC_OK;
    LAUNCH(k_donor, dim3(blocks(n, kT)), dim3(kT), g.enodes, g.cbox, g.ediam, g.dgrid, g.dbin_start, g.dbin_items,
           pose, pts, n, donor, ref);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

}  // namespace oc
