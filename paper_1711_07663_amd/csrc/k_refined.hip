// The refined cut: the exact predicate of the cut applied to the curved
// geometry on a finer lattice (the linearisation paragraph of Sec. 4.2).
// Every quadratic surface face is split into k x k quadratic sub-faces and
// every element near the surface into k^3 quadratic sub-elements, each the
// isoparametric map (eq. reftophys) restricted to a sub-square / sub-cube of
// the reference domain, so their nodes are the map evaluated on the
// sub-lattice.  An element is a hole when one of its sub-elements is: a
// closed surface that meets the element meets one of its pieces, and one
// that does not lies on the side of the element's first node, which is its
// first sub-element's first node.  Level 1 is the lattice cut; the
// triangulations of level k lie within O(1/k^2) of the curved faces.
//
// The run reuses the cut pipeline twice:
//   k_rf_surface   refined surface (sub-face nodes, edge points evaluated
//                  from the lower-id end of the edge so neighbours share them)
//   k_rf_cbox      the grid's control-net boxes as the filter's SoA planes
//   cut 1          the grid (its lattice, boxes holding the curved elements)
//                  against the refined surface: far elements are decided
//                  (not hit; ray parity of the first node), near ones listed
//   k_rf_near      near elements (hit or side items of cut 1)
//   k_rf_elements  their sub-elements: nodes and FP32 node boxes
//   cut 2          the sub-elements against the refined surface
//   k_rf_reduce    an element is a hole when any of its sub-elements is
//   k_rf_unfringe + fringe layer over the whole grid
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dev_common.h"

namespace oc {

constexpr int kRT = 256;
constexpr int kRfKeys = 12;   // sizing words per refined surface (11 used)

__device__ inline void lag2_rf(double s, double *l)
{
    l[0] = 0.5 * s * (s - 1.0);
    l[1] = 1.0 - s * s;
    l[2] = 0.5 * s * (s + 1.0);
}

// node q (a + 3b) of sub-face (f, bi, bj): parent lattice point (I, J) =
// (2 bi + a, 2 bj + b), reference coordinates -1 + I/k, -1 + J/k.  Points on
// the parent's boundary are evaluated from that edge's three nodes starting
// at the end with the lower node id.
__global__ __launch_bounds__(kRT) void k_rf_surface(const double *__restrict__ nodes, int64_t n_nodes,
                                                    const int32_t *__restrict__ conn, int64_t n_face, int k,
                                                    double *__restrict__ vnodes, int32_t *__restrict__ vconn)
{
    const int64_t n_sub = n_face * k * k, n_v = n_sub * 9;
    const int N = 2 * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_v; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sf = t / 9;
        const int q = (int)(t - 9 * sf), a = q % 3, b = q / 3;
        const int64_t f = sf / (k * k);
        const int r = (int)(sf - f * k * k), bi = r % k, bj = r / k;
        const int I = 2 * bi + a, J = 2 * bj + b;
        const int32_t *C = conn + 9 * f;
        double x[3];
        // edge of the parent face holding (I, J), if any: its nodes in
        // lattice order and the parameter along it
        int e0 = -1, e1 = -1, e2 = -1;
        double s = 0.0;
        if (J == 0) { e0 = C[0]; e1 = C[1]; e2 = C[2]; s = -1.0 + (double)I / k; }
        else if (J == N) { e0 = C[6]; e1 = C[7]; e2 = C[8]; s = -1.0 + (double)I / k; }
        else if (I == 0) { e0 = C[0]; e1 = C[3]; e2 = C[6]; s = -1.0 + (double)J / k; }
        else if (I == N) { e0 = C[2]; e1 = C[5]; e2 = C[8]; s = -1.0 + (double)J / k; }
        if (e0 >= 0) {
            if (e0 > e2) {
                const int tmp = e0;
                e0 = e2;
                e2 = tmp;
                s = -s;
            }
            double l[3];
            lag2_rf(s, l);
            for (int d = 0; d < 3; ++d) {
                const double *X = nodes + d * n_nodes;
                x[d] = (X[e0] * l[0] + X[e1] * l[1]) + X[e2] * l[2];
            }
        } else {
            double lu[3], lv[3];
            lag2_rf(-1.0 + (double)I / k, lu);
            lag2_rf(-1.0 + (double)J / k, lv);
            for (int d = 0; d < 3; ++d) {
                const double *X = nodes + d * n_nodes;
                double acc = 0.0;
                for (int jb = 0; jb < 3; ++jb)
                    for (int ia = 0; ia < 3; ++ia) acc += X[C[ia + 3 * jb]] * (lu[ia] * lv[jb]);
                x[d] = acc;
            }
        }
        for (int d = 0; d < 3; ++d) vnodes[d * n_v + t] = x[d];
        vconn[t] = (int32_t)t;
    }
}

// order-preserving 64-bit keys of doubles (for atomic min / max)
__device__ inline unsigned long long rf_key(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// sizing of a refined surface for its bins, as registration does it: the
// largest sub-face node-box diagonal, the node box, the largest node
// distance from the origin, and the first node.  out (keys, zeroed by the
// caller except the minima, set to all ones): [0] max diagonal, [1] max
// node norm, [2..4] box minima, [5..7] box maxima; [8..10] the first node
// (raw doubles)
__global__ __launch_bounds__(kRT) void k_rf_sizes(const double *__restrict__ vnodes, int64_t n_sub_f,
                                                  unsigned long long *__restrict__ out)
{
    __shared__ double red[8][kRT];
    const int64_t n_v = n_sub_f * 9;
    double acc[8] = {0.0, 0.0, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n_sub_f; f += (int64_t)gridDim.x * blockDim.x) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int q = 0; q < 9; ++q) {
            double r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double v = vnodes[d * n_v + 9 * f + q];
                lo[d] = fmin(lo[d], v);
                hi[d] = fmax(hi[d], v);
                r2 += v * v;
            }
            acc[1] = fmax(acc[1], sqrt(r2));
        }
        double g2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            g2 += (hi[d] - lo[d]) * (hi[d] - lo[d]);
            acc[2 + d] = fmin(acc[2 + d], lo[d]);
            acc[5 + d] = fmax(acc[5 + d], hi[d]);
        }
        acc[0] = fmax(acc[0], sqrt(g2));
    }
    for (int i = 0; i < 8; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int w = kRT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int i = 0; i < 8; ++i) {
                const double a = red[i][threadIdx.x], b = red[i][threadIdx.x + w];
                red[i][threadIdx.x] = (i >= 2 && i < 5) ? fmin(a, b) : fmax(a, b);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < 8; ++i) {
            if (i >= 2 && i < 5) atomicMin(out + i, rf_key(red[i][0]));
            else atomicMax(out + i, rf_key(red[i][0]));
        }
        if (blockIdx.x == 0)
            for (int d = 0; d < 3; ++d) out[8 + d] = (unsigned long long)__double_as_longlong(vnodes[d * n_v]);
    }
}

// control-net boxes (AoS, [e][6]) as the filter's SoA planes [6][stride]
__global__ __launch_bounds__(kRT) void k_rf_cbox(const float *__restrict__ cbox, int64_t n_elem, int64_t stride,
                                                 float *__restrict__ soa)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < stride; e += (int64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < 6; ++k)
            soa[k * stride + e] = e < n_elem ? cbox[6 * e + k] : (k < 3 ? INFINITY : -INFINITY);
}

// the near elements of cut 1 (items the exact stage decided: hit or side);
// order is free (each element's sub-elements are reduced on their own)
__global__ __launch_bounds__(kRT) void k_rf_near(const uint64_t *__restrict__ list_inbox,
                                                 const uint8_t *__restrict__ stat, const CutCounters *cnt,
                                                 int32_t *__restrict__ near, int32_t *__restrict__ n_near)
{
    const int n = cnt->n_inbox;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint8_t s = stat[i];
        if (s == ST_HIT || s == ST_SIDE) near[atomicAdd(n_near, 1)] = (int32_t)(uint32_t)list_inbox[i];
    }
}

// sub-element (j, s) of near element near[j], s = i + k j' + k^2 l; its node
// q = a + 3b + 9c is the element's map at lattice point (2i + a, 2j' + b,
// 2l + c); nodes stored x[27], y[27], z[27]; FP32 node box rounded outward
__global__ __launch_bounds__(kRT) void k_rf_elements(const double *__restrict__ enodes,
                                                     const int32_t *__restrict__ near, int64_t n_sub, int k,
                                                     double *__restrict__ vnodes, float *__restrict__ vbox,
                                                     int64_t stride)
{
    const int k3 = k * k * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_sub; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / k3;
        const int s = (int)(t - j * k3), si = s % k, sj = (s / k) % k, sl = s / (k * k);
        const double *X = enodes + (int64_t)near[j] * 81;
        double *V = vnodes + t * 81;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int q = 0; q < 27; ++q) {
            const int a = q % 3, b = (q / 3) % 3, c = q / 9;
            double lu[3], lv[3], lw[3];
            lag2_rf(-1.0 + (double)(2 * si + a) / k, lu);
            lag2_rf(-1.0 + (double)(2 * sj + b) / k, lv);
            lag2_rf(-1.0 + (double)(2 * sl + c) / k, lw);
            for (int d = 0; d < 3; ++d) {
                const double *C = X + 27 * d;
                double acc = 0.0;
                for (int ic = 0; ic < 3; ++ic)
                    for (int ib = 0; ib < 3; ++ib)
                        for (int ia = 0; ia < 3; ++ia) acc += C[ia + 3 * ib + 9 * ic] * ((lu[ia] * lv[ib]) * lw[ic]);
                V[27 * d + q] = acc;
                lo[d] = fmin(lo[d], acc);
                hi[d] = fmax(hi[d], acc);
            }
        }
        for (int d = 0; d < 3; ++d) {
            vbox[d * stride + t] = f32_down(lo[d]);
            vbox[(3 + d) * stride + t] = f32_up(hi[d]);
        }
    }
}

// padding of the sub-element box planes (never in a box test)
__global__ __launch_bounds__(kRT) void k_rf_pad(float *__restrict__ vbox, int64_t n_sub, int64_t stride)
{
    for (int64_t t = n_sub + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < stride; t += (int64_t)gridDim.x * blockDim.x)
        for (int d = 0; d < 3; ++d) {
            vbox[d * stride + t] = INFINITY;
            vbox[(3 + d) * stride + t] = -INFINITY;
        }
}

__global__ __launch_bounds__(kRT) void k_rf_reduce(const int32_t *__restrict__ near, const int32_t *__restrict__ n_near,
                                                   const int8_t *__restrict__ sub_ib, int k3, int8_t *__restrict__ iblank)
{
    const int n = *n_near;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        bool hole = false;
        for (int s = 0; s < k3; ++s) hole |= sub_ib[(int64_t)j * k3 + s] == OC_HOLE;
        iblank[near[j]] = hole ? OC_HOLE : OC_FIELD;
    }
}

__global__ __launch_bounds__(kRT) void k_rf_unfringe(int8_t *__restrict__ iblank, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        if (iblank[e] == OC_FRINGE) iblank[e] = OC_FIELD;
}

#define LAUNCH(name, grid, block, ...)                                                       \
    do {                                                                                     \
        size_t slot_;                                                                        \
        time_begin(ctx, st, #name, &slot_);                                                  \
        hipLaunchKernelGGL(name, grid, block, 0, st, __VA_ARGS__);                           \
        time_end(ctx, st, slot_);                                                            \
    } while (0)

static unsigned rblocks(int64_t n)
{
    const int64_t b = (n + kRT - 1) / kRT;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}

static size_t ralign(size_t v) { return (v + 255) / 256 * 256; }

// arena i of the slot's refined-cut scratch, grown on demand
static oc_status rf_reserve(oc_slot *sl, int i, size_t bytes, char **base)
{
    if (bytes > sl->rf_cap[i]) {
        OC_HIP(hipStreamSynchronize(sl->stream));
        OC_TRY(dev_alloc(sl->ctx, sl->owned, bytes, &sl->rf_buf[i]));
        sl->rf_cap[i] = bytes;
    }
    *base = reinterpret_cast<char *>(sl->rf_buf[i]);
    return OC_OK;
}

static double rf_unkey(unsigned long long k)
{
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double v;
    memcpy(&v, &b, sizeof v);
    return v;
}

// bins of a refined surface from its sizes (as registration sizes them:
// bins per axis about the surface radius over the largest face diagonal)
static void rf_surf_params(const unsigned long long *key, int surf_bins, Surf &sv)
{
    const double dmax = rf_unkey(key[0]);
    double rb = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double e = rf_unkey(key[5 + d]) - rf_unkey(key[2 + d]);
        rb += e * e;
    }
    rb = 0.5 * std::sqrt(rb);
    sv.dmax = f32_up(dmax);
    int nb = (int)std::ceil(rb / std::max(dmax, 1e-30)) + 1;
    nb = std::max(1, std::min(nb, 160));
    if (surf_bins > 0) nb = std::min(nb, surf_bins);
    sv.nb_max = sv.nb_auto = nb;
    for (int d = 0; d < 3; ++d) memcpy(&sv.first[d], key + 8 + d, sizeof(double));
    sv.rmax = rf_unkey(key[1]);
}

oc_status refined_cut_run(oc_slot *sl, Grid &g, Surf *const *surfs, const Pose *poses_dev, int n_surf, int k,
                          int8_t *iblank, int64_t *n_near_out)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    if (!sl->grow) {
        set_error("the refined cut runs on the context's own slot");
        return OC_EINVAL;
    }
    // arena 0: refined surfaces, the control-net planes, the near list
    std::vector<size_t> o_nodes(n_surf), o_conn(n_surf);
    std::vector<int64_t> n_v(n_surf);
    size_t o = 0;
    for (int i = 0; i < n_surf; ++i) {
        n_v[i] = surfs[i]->n_face * k * k * 9;
        if (n_v[i] >= INT32_MAX) {
            set_error("refined surface too large");
            return OC_EINVAL;
        }
        o_nodes[i] = o;
        o += ralign(sizeof(double) * 3 * (size_t)n_v[i]);
        o_conn[i] = o;
        o += ralign(sizeof(int32_t) * (size_t)n_v[i]);
    }
    const int64_t near_cap = std::max<int64_t>(g.n_elem * n_surf, 1);
    const size_t o_cbox = o, o_near = o_cbox + ralign(sizeof(float) * 6 * (size_t)g.ebox_stride);
    const size_t o_cnt = o_near + ralign(sizeof(int32_t) * (size_t)near_cap);
    const size_t o_keys = o_cnt + 256;
    char *A;
    OC_TRY(rf_reserve(sl, 0, o_keys + ralign(sizeof(unsigned long long) * kRfKeys * (size_t)n_surf), &A));
    float *cbox_soa = reinterpret_cast<float *>(A + o_cbox);
    int32_t *near = reinterpret_cast<int32_t *>(A + o_near);
    int32_t *n_near = reinterpret_cast<int32_t *>(A + o_cnt);
    std::vector<Surf> sv(n_surf);
    std::vector<Surf *> svp(n_surf);
    std::vector<unsigned long long> keys((size_t)n_surf * kRfKeys);
    for (int i = 0; i < n_surf; ++i) {
        const Surf &s = *surfs[i];
        double *vnodes = reinterpret_cast<double *>(A + o_nodes[i]);
        int32_t *vconn = reinterpret_cast<int32_t *>(A + o_conn[i]);
        unsigned long long *key = reinterpret_cast<unsigned long long *>(A + o_keys) + (size_t)i * kRfKeys;
        unsigned long long init[kRfKeys] = {0, 0, ~0ull, ~0ull, ~0ull, 0, 0, 0, 0, 0, 0, 0};
        OC_TRY(put_bytes(sl, key, init, sizeof init));
        LAUNCH(k_rf_surface, dim3(rblocks(n_v[i])), dim3(kRT), s.nodes, s.n_nodes, s.conn, s.n_face, k, vnodes, vconn);
        LAUNCH(k_rf_sizes, dim3(rblocks(s.n_face * k * k)), dim3(kRT), vnodes, s.n_face * k * k, key);
        sv[i].n_face = s.n_face * k * k;
        sv[i].n_nodes = n_v[i];
        sv[i].kind = s.kind;
        sv[i].nodes = vnodes;
        sv[i].conn = vconn;
        svp[i] = &sv[i];
    }
    OC_HIP(hipGetLastError());
    OC_HIP(hipMemcpyAsync(keys.data(), A + o_keys, sizeof(unsigned long long) * keys.size(), hipMemcpyDeviceToHost, st));
    OC_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n_surf; ++i) rf_surf_params(keys.data() + (size_t)i * kRfKeys, ctx->surf_bins, sv[i]);
    LAUNCH(k_rf_cbox, dim3(rblocks(g.ebox_stride)), dim3(kRT), g.cbox, g.n_elem, g.ebox_stride, cbox_soa);
    // cut 1: the grid, boxes that hold the curved elements
    Grid g1;
    g1.n_elem = g.n_elem;
    g1.enodes = g.enodes;
    g1.ebox = cbox_soa;
    g1.ebox_stride = g.ebox_stride;
    g1.nbr = g.nbr;
    g1.overset = g.overset;
    g1.n_overset = g.n_overset;
    CutReq q;
    q.g = &g1;
    q.n_surf = n_surf;
    q.surfs = svp.data();
    q.poses = poses_dev;
    q.iblank = iblank;
    OC_TRY(cut_batch_run(sl, &q, 1));
    static const int32_t zero = 0;
    OC_TRY(put_bytes(sl, n_near, &zero, sizeof zero));
    LAUNCH(k_rf_near, dim3(1024), dim3(kRT), sl->l_inbox, sl->l_stat, sl->counters, near, n_near);
    int32_t nn = 0;
    OC_HIP(hipMemcpyAsync(&nn, n_near, sizeof nn, hipMemcpyDeviceToHost, st));
    OC_HIP(hipStreamSynchronize(st));
    if (n_near_out) *n_near_out = nn;
    if (nn > 0) {
        const int64_t k3 = (int64_t)k * k * k, n_sub = (int64_t)nn * k3;
        if (n_sub >= INT32_MAX) {
            set_error("too many sub-elements for the refined cut");
            return OC_EINVAL;
        }
        const int64_t stride = (n_sub + 63) / 64 * 64;
        const size_t o_box = ralign(sizeof(double) * 81 * (size_t)n_sub);
        const size_t o_ib = o_box + ralign(sizeof(float) * 6 * (size_t)stride);
        char *B;
        OC_TRY(rf_reserve(sl, 1, o_ib + ralign((size_t)n_sub), &B));
        double *enodes_v = reinterpret_cast<double *>(B);
        float *ebox_v = reinterpret_cast<float *>(B + o_box);
        int8_t *sub_ib = reinterpret_cast<int8_t *>(B + o_ib);
        LAUNCH(k_rf_elements, dim3(rblocks(n_sub)), dim3(kRT), g.enodes, near, n_sub, k, enodes_v, ebox_v, stride);
        if (stride > n_sub) LAUNCH(k_rf_pad, dim3(1), dim3(kRT), ebox_v, n_sub, stride);
        // cut 2: the sub-elements (no neighbours: the fringe comes later)
        Grid gv;
        gv.n_elem = n_sub;
        gv.enodes = enodes_v;
        gv.ebox = ebox_v;
        gv.ebox_stride = stride;
        CutReq q2;
        q2.g = &gv;
        q2.n_surf = n_surf;
        q2.surfs = svp.data();
        q2.poses = poses_dev;
        q2.iblank = sub_ib;
        OC_TRY(cut_batch_run(sl, &q2, 1));
        LAUNCH(k_rf_reduce, dim3(rblocks(nn)), dim3(kRT), near, n_near, sub_ib, (int)k3, iblank);
    }
    LAUNCH(k_rf_unfringe, dim3(rblocks(g.n_elem)), dim3(kRT), iblank, g.n_elem);
    OC_TRY(fringe_layer_run(sl, g, iblank));
    OC_HIP(hipGetLastError());
    return OC_OK;
}

}  // namespace oc
