// Direct cut of a curved quadratic grid by closed cutting surfaces
// (Sec. 4.2 "Parallel Direct Cut Algorithm"): every element decides on its
// own whether it is intersected by, inside or outside the surface, so no
// paint-fill is needed.
//
// Pipeline per surface (all on the context stream):
//   k_surf_init / k_pose_faces      pose the surface nodes, FP32 face boxes
//                                   inflated by the hit tolerance, surface box
//   k_bins_setup / k_bin_count /    uniform bins over the surface box:
//   scan / k_bin_fill               count, exclusive scan, fill (CSR)
//   k_filter                        stream every element's FP32 box; boxes
//                                   meeting the surface box go to a list
//   k_candidates                    element box x binned face boxes: elements
//                                   with a candidate face are "near", others
//                                   "far"
//   k_exact                         one wavefront per near element: FP64
//                                   triangle-pair intersection (hit), else the
//                                   nearest-face side of the element's first
//                                   node (wavefront minimum + tie rule)
//   k_ray                           far elements: +x ray parity of the first
//                                   node against the surface triangles
// then once per cut:
//   k_fringe / k_overset_fringe     one fringe layer around holes, overset faces
#include "dev_geom.h"

namespace oc {

constexpr int kThreads = 256;

// ------------------------------------------------------------ wave utils --
__device__ inline int lane_id() { return threadIdx.x & 63; }

// Reserve c slots in a global list with one atomic per wavefront; returns
// this lane's first slot.  Must be called by every active lane of the wave.
__device__ inline int wave_append(int *counter, int c)
{
    const int lane = lane_id();
    int inc = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    int total = __shfl(inc, 63, 64);
    int base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(counter, total);
    base = __shfl(base, 63, 64);
    return base + inc - c;
}

__device__ inline long long wave_sum_ll(long long v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ inline double wave_min_d(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
    return v;
}

// ------------------------------------------------------- surface stage ----
__global__ void k_reset_counters(CutCounters *cnt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cnt->n_inbox = cnt->n_near = cnt->n_far = cnt->n_hit = cnt->n_hole = 0;
        cnt->n_cand_pairs = 0ull;
    }
}

__global__ void k_surf_init(SurfParams *sp, CutCounters *cnt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int k = 0; k < 3; ++k) {
            sp->sbox_ord[k] = f2ord(INFINITY);
            sp->sbox_ord[3 + k] = f2ord(-INFINITY);
        }
        cnt->n_inbox = cnt->n_near = cnt->n_far = 0;
    }
}

// a1 + a2 (face boxes): pose the 9 nodes of every face (x' = R x + t), store
// them face-major, and build the face's FP32 box rounded outward and inflated
// by tol_hit + 2^-20 * max|coordinate|.
__global__ __launch_bounds__(kThreads) void k_pose_faces(const double *__restrict__ nodes, int64_t n_nodes,
                                                         const int32_t *__restrict__ conn, int64_t n_face,
                                                         Pose pose, double *__restrict__ pnodes,
                                                         float *__restrict__ fbox, SurfParams *sp)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (f < n_face) {
        double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double L = 0.0;
        for (int k = 0; k < 9; ++k) {
            int id = conn[f * 9 + k];
            d3 x = pose_apply(pose, mk(nodes[id], nodes[n_nodes + id], nodes[2 * n_nodes + id]));
            pnodes[f * 27 + k] = x.x;
            pnodes[f * 27 + 9 + k] = x.y;
            pnodes[f * 27 + 18 + k] = x.z;
            blo[0] = fmin(blo[0], x.x); bhi[0] = fmax(bhi[0], x.x);
            blo[1] = fmin(blo[1], x.y); bhi[1] = fmax(bhi[1], x.y);
            blo[2] = fmin(blo[2], x.z); bhi[2] = fmax(bhi[2], x.z);
            L = fmax(L, fmax(fabs(x.x), fmax(fabs(x.y), fabs(x.z))));
        }
        const double delta = kTolHit + ldexp(L, -20);
        for (int a = 0; a < 3; ++a) {
            lo[a] = f32_down(blo[a] - delta);
            hi[a] = f32_up(bhi[a] + delta);
            fbox[f * 6 + a] = lo[a];
            fbox[f * 6 + 3 + a] = hi[a];
        }
    }
    // surface box: wavefront reduction, one atomic per wave and bound
    for (int a = 0; a < 3; ++a) {
        float l = lo[a], h = hi[a];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            l = fminf(l, __shfl_xor(l, d, 64));
            h = fmaxf(h, __shfl_xor(h, d, 64));
        }
        if (lane_id() == 0 && l <= h) {
            atomicMin(&sp->sbox_ord[a], f2ord(l));
            atomicMax(&sp->sbox_ord[3 + a], f2ord(h));
        }
    }
}

// Bin grid over the surface box.  The bin edge is at least the largest face
// box extent (dmax + 2 delta, pose invariant), so a face spans at most two
// bins per axis and at most 8 bins in total.
__global__ void k_bins_setup(SurfParams *sp, float dmax, int nb_max)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float L = 0.f;
    for (int k = 0; k < 6; ++k) {
        sp->sbox[k] = ord2f(sp->sbox_ord[k]);
        L = fmaxf(L, fabsf(sp->sbox[k]));
    }
    const float w = (dmax + 2.0f * (1e-7f + ldexpf(L, -20)) + ldexpf(L, -18)) * 1.001f;
    int nb = 1;
    for (int a = 0; a < 3; ++a) {
        float ext = sp->sbox[3 + a] - sp->sbox[a];
        int n = 1;
        if (ext > 0.f) {
            float q = fminf(floorf(ext / w), (float)nb_max);
            n = q < 1.f ? 1 : (int)q;
        }
        sp->grid.o[a] = sp->sbox[a];
        sp->grid.n[a] = n;
        sp->grid.inv[a] = ext > 0.f ? (float)n / ext : 0.f;
        nb *= n;
    }
    sp->n_bins = nb;
}

__global__ __launch_bounds__(kThreads) void k_zero_i32(int32_t *p, const int *n_dev, int64_t n_host)
{
    const int64_t n = n_dev ? (int64_t)*n_dev + 1 : n_host;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__device__ inline void box_bins(const BinGrid &G, const float *b, int *lo, int *hi)
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = bin_of(b[a], G.o[a], G.inv[a], G.n[a]);
        hi[a] = bin_of(b[3 + a], G.o[a], G.inv[a], G.n[a]);
    }
}

__global__ __launch_bounds__(kThreads) void k_bin_count(const float *__restrict__ fbox, int64_t n_face,
                                                        const SurfParams *__restrict__ sp,
                                                        int32_t *__restrict__ count)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_face) return;
    const BinGrid G = sp->grid;
    int lo[3], hi[3];
    box_bins(G, fbox + f * 6, lo, hi);
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) atomicAdd(&count[x + G.n[0] * (y + G.n[1] * z)], 1);
}

// fill: the count array doubles as the per-bin cursor and ends at zero
__global__ __launch_bounds__(kThreads) void k_bin_fill(const float *__restrict__ fbox, int64_t n_face,
                                                       const SurfParams *__restrict__ sp,
                                                       const int32_t *__restrict__ start, int32_t *count,
                                                       int32_t *__restrict__ items)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_face) return;
    const BinGrid G = sp->grid;
    int lo[3], hi[3];
    box_bins(G, fbox + f * 6, lo, hi);
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                int b = x + G.n[0] * (y + G.n[1] * z);
                int pos = atomicSub(&count[b], 1) - 1;
                items[start[b] + pos] = (int32_t)f;
            }
}

// ---------------------------------------------------------- element stage --
// a3, streaming part: every element's FP32 box (SoA planes, 4 elements per
// thread) is tested against the surface box.  Optionally initialises iblank
// to field.
__global__ __launch_bounds__(kThreads) void k_filter(const float *__restrict__ ebox, int64_t n_elem, int64_t stride_e,
                                                     const SurfParams *__restrict__ sp, int8_t *__restrict__ iblank,
                                                     int write_field, int32_t *__restrict__ list_inbox,
                                                     CutCounters *cnt)
{
    const float s0 = sp->sbox[0], s1 = sp->sbox[1], s2 = sp->sbox[2];
    const float s3 = sp->sbox[3], s4 = sp->sbox[4], s5 = sp->sbox[5];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
         e0 - (int64_t)lane_id() * 4 < n_elem; e0 += stride) {
        int flags = 0, c = 0;
        if (e0 + 3 < n_elem) {
            const float4 xl = *reinterpret_cast<const float4 *>(ebox + e0);
            const float4 yl = *reinterpret_cast<const float4 *>(ebox + stride_e + e0);
            const float4 zl = *reinterpret_cast<const float4 *>(ebox + 2 * stride_e + e0);
            const float4 xh = *reinterpret_cast<const float4 *>(ebox + 3 * stride_e + e0);
            const float4 yh = *reinterpret_cast<const float4 *>(ebox + 4 * stride_e + e0);
            const float4 zh = *reinterpret_cast<const float4 *>(ebox + 5 * stride_e + e0);
            const float L0[4] = {xl.x, xl.y, xl.z, xl.w}, L1[4] = {yl.x, yl.y, yl.z, yl.w};
            const float L2[4] = {zl.x, zl.y, zl.z, zl.w}, H0[4] = {xh.x, xh.y, xh.z, xh.w};
            const float H1[4] = {yh.x, yh.y, yh.z, yh.w}, H2[4] = {zh.x, zh.y, zh.z, zh.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                bool in = L0[k] <= s3 && H0[k] >= s0 && L1[k] <= s4 && H1[k] >= s1 && L2[k] <= s5 && H2[k] >= s2;
                flags |= (int)in << k;
                c += in;
            }
            if (write_field) *reinterpret_cast<uint32_t *>(iblank + e0) = 0x01010101u;
        } else {
            for (int k = 0; k < 4; ++k) {
                int64_t e = e0 + k;
                if (e >= n_elem) break;
                bool in = ebox[e] <= s3 && ebox[3 * stride_e + e] >= s0 && ebox[stride_e + e] <= s4 &&
                          ebox[4 * stride_e + e] >= s1 && ebox[2 * stride_e + e] <= s5 && ebox[5 * stride_e + e] >= s2;
                flags |= (int)in << k;
                c += in;
                if (write_field) iblank[e] = OC_FIELD;
            }
        }
        int pos = wave_append(&cnt->n_inbox, c);
        for (int k = 0; k < 4; ++k)
            if (flags >> k & 1) list_inbox[pos++] = (int32_t)(e0 + k);
    }
}

__device__ inline bool box_overlap(const float *a, const float *b)
{
    return a[0] <= b[3] && b[0] <= a[3] && a[1] <= b[4] && b[1] <= a[4] && a[2] <= b[5] && b[2] <= a[5];
}

// a3, bin part: count the candidate faces of each in-box element (element box
// overlapping an inflated face box).  A face found in several bins is
// counted only in the first bin (per axis) common to both bin ranges.
__global__ __launch_bounds__(kThreads) void k_candidates(const float *__restrict__ ebox, int64_t stride,
                                                         const float *__restrict__ fbox,
                                                         const SurfParams *__restrict__ sp,
                                                         const int32_t *__restrict__ bstart,
                                                         const int32_t *__restrict__ bitems,
                                                         const int32_t *__restrict__ list_inbox,
                                                         int32_t *__restrict__ list_near,
                                                         int32_t *__restrict__ list_far, CutCounters *cnt)
{
    const BinGrid G = sp->grid;
    const int n_in = cnt->n_inbox;
    const int gstride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < n_in; base += gstride) {
        const int i = base + threadIdx.x;
        int e = -1, nc = 0;
        if (i < n_in) {
            e = list_inbox[i];
            float eb[6];
            for (int k = 0; k < 6; ++k) eb[k] = ebox[(int64_t)k * stride + e];
            int lo[3], hi[3];
            box_bins(G, eb, lo, hi);
            for (int z = lo[2]; z <= hi[2]; ++z)
                for (int y = lo[1]; y <= hi[1]; ++y)
                    for (int x = lo[0]; x <= hi[0]; ++x) {
                        const int b = x + G.n[0] * (y + G.n[1] * z);
                        for (int j = bstart[b]; j < bstart[b + 1]; ++j) {
                            const float *fb = fbox + (int64_t)bitems[j] * 6;
                            int fl[3], fh[3];
                            box_bins(G, fb, fl, fh);
                            if (x != max(lo[0], fl[0]) || y != max(lo[1], fl[1]) || z != max(lo[2], fl[2])) continue;
                            nc += box_overlap(eb, fb);
                        }
                    }
        }
        const bool near = e >= 0 && nc > 0, far = e >= 0 && nc == 0;
        int pn = wave_append(&cnt->n_near, near ? 1 : 0);
        int pf = wave_append(&cnt->n_far, far ? 1 : 0);
        if (near) list_near[pn] = e;
        if (far) list_far[pf] = e;
        long long s = wave_sum_ll(nc);
        if (lane_id() == 0 && s) atomicAdd(&cnt->n_cand_pairs, (unsigned long long)s);
    }
}

// ------------------------------------------------------------ exact stage --
struct TieRec {
    double absdot, dot;
    double v[3], n[3];
    int f, s, valid, pad;
};

// order: larger |dot| first, then lower face id, then lower face triangle
__device__ inline bool tie_before(const TieRec &a, const TieRec &b)
{
    if (!a.valid) return false;
    if (!b.valid) return true;
    if (a.absdot != b.absdot) return a.absdot > b.absdot;
    if (a.f != b.f) return a.f < b.f;
    return a.s < b.s;
}
__device__ inline void tie_offer(TieRec &b1, TieRec &b2, const TieRec &r)
{
    if (tie_before(r, b1)) {
        b2 = b1;
        b1 = r;
    } else if (tie_before(r, b2)) {
        b2 = r;
    }
}

// triangle s of a posed face (face-major x[9], y[9], z[9])
__device__ inline void face_tri(const double *__restrict__ P, int s, d3 *T)
{
    int uv[6];
    quad_tri_uv((s >> 1) & 1, s >> 2, s & 1, uv);
    for (int k = 0; k < 3; ++k) {
        int nd = uv[2 * k] + 3 * uv[2 * k + 1];
        T[k] = mk(P[nd], P[9 + nd], P[18 + nd]);
    }
}

__device__ inline double point_box_dist(d3 p, const float *b)
{
    double gx = fmax(0.0, fmax((double)b[0] - p.x, p.x - (double)b[3]));
    double gy = fmax(0.0, fmax((double)b[1] - p.y, p.y - (double)b[4]));
    double gz = fmax(0.0, fmax((double)b[2] - p.z, p.z - (double)b[5]));
    return sqrt(gx * gx + gy * gy + gz * gz);
}

struct ExactArgs {
    const double *enodes;
    const float *ebox;
    int64_t stride;
    const double *pnodes;
    const float *fbox;
    const int32_t *bstart;
    const int32_t *bitems;
    const SurfParams *sp;
    const int32_t *list_near;
    CutCounters *cnt;
    int8_t *iblank;
    int32_t *list_hole;
    int kind;
    int pad;
    double sfirst[3];
};

// query box [p - r, p + r] rounded outward to FP32 and its bin range
__device__ inline void query_bins(const BinGrid &G, d3 p, double r, float *qb, int *lo, int *hi)
{
    qb[0] = f32_down(p.x - r);
    qb[1] = f32_down(p.y - r);
    qb[2] = f32_down(p.z - r);
    qb[3] = f32_up(p.x + r);
    qb[4] = f32_up(p.y + r);
    qb[5] = f32_up(p.z + r);
    box_bins(G, qb, lo, hi);
}

// a4 + a5: one wavefront per near element.
__global__ __launch_bounds__(64) void k_exact(ExactArgs a)
{
    __shared__ double sN[81];
    __shared__ TieRec rec[128];
    const int lane = threadIdx.x;
    const BinGrid G = a.sp->grid;
    const int n_near = a.cnt->n_near;
    const double tol = kTolHit;
    for (int item = blockIdx.x; item < n_near; item += gridDim.x) {
        const int e = a.list_near[item];
        __syncthreads();
        for (int k = lane; k < 81; k += 64) sN[k] = a.enodes[(int64_t)e * 81 + k];
        __syncthreads();

        // this lane's boundary triangle of the element (48 = 6 faces x 4 quads x 2)
        const bool tv = lane < 48;
        d3 T[3];
        double tlo[3], thi[3];
        {
            const int t = tv ? lane : 0;
            int uv[6];
            quad_tri_uv((t >> 1) & 1, (t >> 2) & 1, t & 1, uv);
            for (int k = 0; k < 3; ++k) {
                int nd = elem_face_node(t >> 3, uv[2 * k], uv[2 * k + 1]);
                T[k] = mk(sN[nd], sN[27 + nd], sN[54 + nd]);
            }
            tlo[0] = fmin(T[0].x, fmin(T[1].x, T[2].x)); thi[0] = fmax(T[0].x, fmax(T[1].x, T[2].x));
            tlo[1] = fmin(T[0].y, fmin(T[1].y, T[2].y)); thi[1] = fmax(T[0].y, fmax(T[1].y, T[2].y));
            tlo[2] = fmin(T[0].z, fmin(T[1].z, T[2].z)); thi[2] = fmax(T[0].z, fmax(T[1].z, T[2].z));
        }
        float eb[6];
        for (int k = 0; k < 6; ++k) eb[k] = a.ebox[(int64_t)k * a.stride + e];
        int lo[3], hi[3];
        box_bins(G, eb, lo, hi);

        // ---- hit test over the candidate faces (binned, deduplicated)
        bool hit = false;
        for (int z = lo[2]; z <= hi[2] && !hit; ++z)
            for (int y = lo[1]; y <= hi[1] && !hit; ++y)
                for (int x = lo[0]; x <= hi[0] && !hit; ++x) {
                    const int b = x + G.n[0] * (y + G.n[1] * z);
                    const int j0 = a.bstart[b], j1 = a.bstart[b + 1];
                    for (int base = j0; base < j1 && !hit; base += 64) {
                        const int j = base + lane;
                        int f = -1;
                        bool pass = false;
                        if (j < j1) {
                            f = a.bitems[j];
                            const float *fb = a.fbox + (int64_t)f * 6;
                            int fl[3], fh[3];
                            box_bins(G, fb, fl, fh);
                            pass = x == max(lo[0], fl[0]) && y == max(lo[1], fl[1]) && z == max(lo[2], fl[2]) &&
                                   box_overlap(eb, fb);
                        }
                        unsigned long long mask = __ballot(pass);
                        while (mask && !hit) {
                            const int l = __ffsll((long long)mask) - 1;
                            mask &= mask - 1;
                            const int fid = __shfl(f, l, 64);
                            const double *P = a.pnodes + (int64_t)fid * 27;
                            bool lh = false;
                            for (int s = 0; s < 8; ++s) {
                                d3 F[3];
                                face_tri(P, s, F);
                                double flo0 = fmin(F[0].x, fmin(F[1].x, F[2].x)), fhi0 = fmax(F[0].x, fmax(F[1].x, F[2].x));
                                double flo1 = fmin(F[0].y, fmin(F[1].y, F[2].y)), fhi1 = fmax(F[0].y, fmax(F[1].y, F[2].y));
                                double flo2 = fmin(F[0].z, fmin(F[1].z, F[2].z)), fhi2 = fmax(F[0].z, fmax(F[1].z, F[2].z));
                                bool nearb = tv && flo0 - thi[0] < tol && tlo[0] - fhi0 < tol && flo1 - thi[1] < tol &&
                                             tlo[1] - fhi1 < tol && flo2 - thi[2] < tol && tlo[2] - fhi2 < tol;
                                if (nearb && !lh) lh = tri_tri_within(T, F, tol);
                            }
                            if (__ballot(lh)) hit = true;
                        }
                    }
                }

        // ---- the whole surface inside the element (ray parity of its first node)
        const d3 sf = mk(a.sfirst[0], a.sfirst[1], a.sfirst[2]);
        if (!hit && sf.x >= eb[0] && sf.x <= eb[3] && sf.y >= eb[1] && sf.y <= eb[4] && sf.z >= eb[2] &&
            sf.z <= eb[5]) {
            int c = tv ? ray_x_crosses(sf, T[0], T[1], T[2]) : 0;
            if (__popcll(__ballot(c)) & 1) hit = true;
        }

        int hole;
        if (hit) {
            hole = a.kind == OC_SURF_WALL;
        } else {
            // ---- nearest-face side of the element's first node
            const d3 p = mk(sN[0], sN[27], sN[54]);
            // initial bound: distance to the nearest face box corner region of
            // the element's own box extent
            double r = 0.0;
            for (int k = 0; k < 3; ++k) r = fmax(r, fmax((double)eb[3 + k] - (double)eb[k], 0.0));
            r = r * 1.7320508075688772 + 1e-12;
            double best = INFINITY;
            bool found = false;
            // widen until some face is within the radius
            for (int grow = 0; grow < 40 && !found; ++grow) {
                float qb[6];
                int ql[3], qh[3];
                query_bins(G, p, r, qb, ql, qh);
                for (int z = ql[2]; z <= qh[2]; ++z)
                    for (int y = ql[1]; y <= qh[1]; ++y)
                        for (int x = ql[0]; x <= qh[0]; ++x) {
                            const int b = x + G.n[0] * (y + G.n[1] * z);
                            const int j0 = a.bstart[b], j1 = a.bstart[b + 1];
                            for (int base = j0; base < j1; base += 64) {
                                const int j = base + lane;
                                if (j < j1) {
                                    const int f = a.bitems[j];
                                    const float *fb = a.fbox + (int64_t)f * 6;
                                    int fl[3], fh[3];
                                    box_bins(G, fb, fl, fh);
                                    if (x == max(ql[0], fl[0]) && y == max(ql[1], fl[1]) && z == max(ql[2], fl[2]) &&
                                        point_box_dist(p, fb) <= fmin(r, best)) {
                                        const double *P = a.pnodes + (int64_t)f * 27;
                                        for (int s = 0; s < 8; ++s) {
                                            d3 F[3];
                                            face_tri(P, s, F);
                                            d3 q = closest_on_tri(p, F[0], F[1], F[2]);
                                            d3 w = p - q;
                                            best = fmin(best, sqrt(dot(w, w)));
                                        }
                                    }
                                }
                                best = wave_min_d(best);
                            }
                        }
                best = wave_min_d(best);
                found = best <= r;
                if (!found) r *= 2.0;
            }
            // ---- tie set within best*(1+1e-9): largest |dot| decides, normals
            // averaged only for equally visible pairs of opposite sign
            const double thr = best * (1.0 + 1e-9);
            TieRec b1, b2;
            b1.valid = b2.valid = 0;
            {
                float qb[6];
                int ql[3], qh[3];
                query_bins(G, p, thr, qb, ql, qh);
                for (int z = ql[2]; z <= qh[2]; ++z)
                    for (int y = ql[1]; y <= qh[1]; ++y)
                        for (int x = ql[0]; x <= qh[0]; ++x) {
                            const int b = x + G.n[0] * (y + G.n[1] * z);
                            const int j0 = a.bstart[b], j1 = a.bstart[b + 1];
                            for (int j = j0 + lane; j < j1; j += 64) {
                                const int f = a.bitems[j];
                                const float *fb = a.fbox + (int64_t)f * 6;
                                int fl[3], fh[3];
                                box_bins(G, fb, fl, fh);
                                if (x != max(ql[0], fl[0]) || y != max(ql[1], fl[1]) || z != max(ql[2], fl[2]) ||
                                    point_box_dist(p, fb) > thr)
                                    continue;
                                const double *P = a.pnodes + (int64_t)f * 27;
                                for (int s = 0; s < 8; ++s) {
                                    d3 F[3];
                                    face_tri(P, s, F);
                                    d3 q = closest_on_tri(p, F[0], F[1], F[2]);
                                    d3 v = p - q;
                                    double d = sqrt(dot(v, v));
                                    if (d > thr) continue;
                                    d3 n = cross(F[1] - F[0], F[2] - F[0]);
                                    double ln = sqrt(dot(n, n));
                                    TieRec rr;
                                    rr.v[0] = v.x; rr.v[1] = v.y; rr.v[2] = v.z;
                                    rr.n[0] = ln > 0 ? n.x / ln : 0.0;
                                    rr.n[1] = ln > 0 ? n.y / ln : 0.0;
                                    rr.n[2] = ln > 0 ? n.z / ln : 0.0;
                                    rr.dot = d > 0 ? (v.x * rr.n[0] + v.y * rr.n[1] + v.z * rr.n[2]) / d : 0.0;
                                    rr.absdot = fabs(rr.dot);
                                    rr.f = f;
                                    rr.s = s;
                                    rr.valid = 1;
                                    tie_offer(b1, b2, rr);
                                }
                            }
                        }
            }
            rec[2 * lane] = b1;
            rec[2 * lane + 1] = b2;
            __syncthreads();
            if (lane == 0) {
                TieRec c1, c2;
                c1.valid = c2.valid = 0;
                for (int k = 0; k < 128; ++k)
                    if (rec[k].valid) tie_offer(c1, c2, rec[k]);
                double sg = c1.dot;
                if (c2.valid && c1.absdot - c2.absdot <= 1e-9 && ((c1.dot > 0.0) != (c2.dot > 0.0))) {
                    sg = c1.v[0] * (c1.n[0] + c2.n[0]) + c1.v[1] * (c1.n[1] + c2.n[1]) +
                         c1.v[2] * (c1.n[2] + c2.n[2]);
                }
                rec[0].pad = (c1.valid && sg < 0.0) ? 1 : 0;
            }
            __syncthreads();
            hole = rec[0].pad;
        }
        if (lane == 0) {
            if (hit) atomicAdd(&a.cnt->n_hit, 1);
            if (hole && a.iblank[e] != OC_HOLE) {
                a.iblank[e] = OC_HOLE;
                a.list_hole[atomicAdd(&a.cnt->n_hole, 1)] = e;
            }
        }
    }
}

// a6: far elements (no candidate face): +x ray parity of the first node,
// walking the column of bins that contains the ray.
__global__ __launch_bounds__(kThreads) void k_ray(const double *__restrict__ enodes, const double *__restrict__ pnodes,
                                                  const float *__restrict__ fbox, const SurfParams *__restrict__ sp,
                                                  const int32_t *__restrict__ bstart,
                                                  const int32_t *__restrict__ bitems,
                                                  const int32_t *__restrict__ list_far, CutCounters *cnt,
                                                  int8_t *__restrict__ iblank, int32_t *__restrict__ list_hole)
{
    const BinGrid G = sp->grid;
    const int n_far = cnt->n_far;
    const float sb[6] = {sp->sbox[0], sp->sbox[1], sp->sbox[2], sp->sbox[3], sp->sbox[4], sp->sbox[5]};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_far; i += gridDim.x * blockDim.x) {
        const int e = list_far[i];
        const d3 p = mk(enodes[(int64_t)e * 81], enodes[(int64_t)e * 81 + 27], enodes[(int64_t)e * 81 + 54]);
        if (p.y < sb[1] || p.y > sb[4] || p.z < sb[2] || p.z > sb[5] || p.x > sb[3]) continue;
        const int iy = bin_of((float)p.y, G.o[1], G.inv[1], G.n[1]);
        const int iz = bin_of((float)p.z, G.o[2], G.inv[2], G.n[2]);
        const int ix0 = bin_of((float)p.x, G.o[0], G.inv[0], G.n[0]);
        int par = 0;
        for (int ix = ix0; ix < G.n[0]; ++ix) {
            const int b = ix + G.n[0] * (iy + G.n[1] * iz);
            for (int j = bstart[b]; j < bstart[b + 1]; ++j) {
                const int f = bitems[j];
                const float *fb = fbox + (int64_t)f * 6;
                if (ix != max(ix0, bin_of(fb[0], G.o[0], G.inv[0], G.n[0]))) continue;
                if ((double)fb[1] > p.y || (double)fb[4] < p.y || (double)fb[2] > p.z || (double)fb[5] < p.z ||
                    (double)fb[3] < p.x)
                    continue;
                const double *P = pnodes + (int64_t)f * 27;
                for (int s = 0; s < 8; ++s) {
                    d3 F[3];
                    face_tri(P, s, F);
                    par ^= ray_x_crosses(p, F[0], F[1], F[2]);
                }
            }
        }
        if (par && iblank[e] != OC_HOLE) {
            iblank[e] = OC_HOLE;
            list_hole[atomicAdd(&cnt->n_hole, 1)] = e;
        }
    }
}

// a8: fringe layer (field elements sharing a face with a hole)
__global__ __launch_bounds__(kThreads) void k_fringe(const int32_t *__restrict__ nbr,
                                                     const int32_t *__restrict__ list_hole,
                                                     const CutCounters *__restrict__ cnt, int8_t *iblank)
{
    const int n = cnt->n_hole;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int e = list_hole[i];
        for (int f = 0; f < 6; ++f) {
            const int q = nbr[(int64_t)e * 6 + f];
            if (q >= 0 && iblank[q] != OC_HOLE) iblank[q] = OC_FRINGE;
        }
    }
}

// elements carrying an overset-tagged face are fringe unless hole
__global__ __launch_bounds__(kThreads) void k_overset_fringe(const int32_t *__restrict__ list, int64_t n,
                                                             int8_t *iblank)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int e = list[i];
        if (iblank[e] != OC_HOLE) iblank[e] = OC_FRINGE;
    }
}

__global__ void k_fill_i8(int8_t *p, int64_t n, int8_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// -------------------------------------------------------------- host side --
static unsigned grid_for(int64_t n, int per_block, unsigned cap)
{
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

#define LAUNCH(name, grid, block, ...)                                                       \
    do {                                                                                     \
        size_t slot_;                                                                        \
        time_begin(ctx, #name, &slot_);                                                      \
        hipLaunchKernelGGL(name, grid, block, 0, ctx->stream, __VA_ARGS__);                  \
        time_end(ctx, slot_);                                                                \
    } while (0)

static oc_status cut_one_surface(oc_ctx *ctx, Grid &g, Surf &s, const Pose &pose, int8_t *iblank, bool first)
{
    const unsigned fb = grid_for(s.n_face, kThreads, 1u << 30);
    LAUNCH(k_surf_init, dim3(1), dim3(64), s.params, ctx->counters);
    LAUNCH(k_pose_faces, dim3(fb), dim3(kThreads), s.nodes, s.n_nodes, s.conn, s.n_face, pose, s.pnodes, s.fbox,
           s.params);
    LAUNCH(k_bins_setup, dim3(1), dim3(64), s.params, s.dmax, s.nb_max);
    const int64_t bcap = (int64_t)s.nb_max * s.nb_max * s.nb_max;
    LAUNCH(k_zero_i32, dim3(grid_for(bcap + 1, kThreads, 4096)), dim3(kThreads), s.bin_count, &s.params->n_bins,
           (int64_t)0);
    LAUNCH(k_bin_count, dim3(fb), dim3(kThreads), s.fbox, s.n_face, s.params, s.bin_count);
    OC_TRY(scan_exclusive(ctx, s.bin_count, s.bin_start, bcap, &s.params->n_bins, s.scan_tmp));
    LAUNCH(k_bin_fill, dim3(fb), dim3(kThreads), s.fbox, s.n_face, s.params, s.bin_start, s.bin_count, s.bin_items);

    LAUNCH(k_filter, dim3(grid_for(g.n_elem, kThreads * 4, 8192)), dim3(kThreads), g.ebox, g.n_elem, g.ebox_stride, s.params,
           iblank, first ? 1 : 0, g.list_inbox, ctx->counters);
    LAUNCH(k_candidates, dim3(1024), dim3(kThreads), g.ebox, g.ebox_stride, s.fbox, s.params, s.bin_start, s.bin_items,
           g.list_inbox, g.list_near, g.list_far, ctx->counters);
    ExactArgs ea;
    ea.enodes = g.enodes;
    ea.ebox = g.ebox;
    ea.stride = g.ebox_stride;
    ea.pnodes = s.pnodes;
    ea.fbox = s.fbox;
    ea.bstart = s.bin_start;
    ea.bitems = s.bin_items;
    ea.sp = s.params;
    ea.list_near = g.list_near;
    ea.cnt = ctx->counters;
    ea.iblank = iblank;
    ea.list_hole = g.list_hole;
    ea.kind = s.kind;
    ea.pad = 0;
    // first node of the surface, posed
    for (int i = 0; i < 3; ++i)
        ea.sfirst[i] = pose.r[3 * i] * s.first[0] + pose.r[3 * i + 1] * s.first[1] + pose.r[3 * i + 2] * s.first[2] +
                       pose.t[i];
    LAUNCH(k_exact, dim3(4096), dim3(64), ea);
    LAUNCH(k_ray, dim3(256), dim3(kThreads), g.enodes, s.pnodes, s.fbox, s.params, s.bin_start, s.bin_items,
           g.list_far, ctx->counters, iblank, g.list_hole);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status cut_run(oc_ctx *ctx, Grid &g, Surf **surfs, const Pose *poses, int n_surf, int8_t *iblank)
{
    LAUNCH(k_reset_counters, dim3(1), dim3(64), ctx->counters);
    if (n_surf == 0)
        LAUNCH(k_fill_i8, dim3(grid_for(g.n_elem, kThreads, 4096)), dim3(kThreads), iblank, g.n_elem,
               (int8_t)OC_FIELD);
    for (int k = 0; k < n_surf; ++k) OC_TRY(cut_one_surface(ctx, g, *surfs[k], poses[k], iblank, k == 0));
    LAUNCH(k_fringe, dim3(1024), dim3(kThreads), g.nbr, g.list_hole, ctx->counters, iblank);
    if (g.n_overset > 0)
        LAUNCH(k_overset_fringe, dim3(grid_for(g.n_overset, kThreads, 4096)), dim3(kThreads), g.overset, g.n_overset,
               iblank);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

}  // namespace oc
