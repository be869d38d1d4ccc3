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
        cnt->n_inbox = cnt->n_near = cnt->n_far = cnt->n_hit = cnt->n_hole = cnt->n_side = 0;
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
        cnt->n_inbox = cnt->n_near = cnt->n_far = cnt->n_side = 0;
    }
}

// a1 + a2 (face boxes): pose the 9 nodes of every face (x' = R x + t), store
// them face-major, and build the face's FP32 box rounded outward and inflated
// by tol_hit + 2^-20 * max|coordinate|.
__global__ __launch_bounds__(kThreads) void k_pose_faces(const double *__restrict__ nodes, int64_t n_nodes,
                                                         const int32_t *__restrict__ conn, int64_t n_face,
                                                         const Pose *__restrict__ pose_dev,
                                                         double *__restrict__ pnodes, float *__restrict__ fbox,
                                                         SurfParams *sp)
{
    const Pose pose = *pose_dev;
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

// Inclusive 3-D range of bins enumerated with a linear index, so that the
// 64 lanes of a wavefront can each take one bin per round.
struct BinRange {
    int lo[3], n[3], total;
};

__device__ inline BinRange make_range(const int *lo, const int *hi)
{
    BinRange R;
    for (int a = 0; a < 3; ++a) {
        R.lo[a] = lo[a];
        R.n[a] = hi[a] - lo[a] + 1;
    }
    R.total = R.n[0] * R.n[1] * R.n[2];
    return R;
}

__device__ inline int range_bin(const BinGrid &G, const BinRange &R, int idx, int *xyz)
{
    xyz[0] = R.lo[0] + idx % R.n[0];
    xyz[1] = R.lo[1] + (idx / R.n[0]) % R.n[1];
    xyz[2] = R.lo[2] + idx / (R.n[0] * R.n[1]);
    return xyz[0] + G.n[0] * (xyz[1] + G.n[1] * xyz[2]);
}

// a face found in bin xyz is taken only in the first bin (per axis) that its
// own range shares with the query range starting at qlo
__device__ inline bool first_common_bin(const BinGrid &G, const float *fb, const int *xyz, const int *qlo)
{
    for (int a = 0; a < 3; ++a) {
        int fl = bin_of(fb[a], G.o[a], G.inv[a], G.n[a]);
        if (xyz[a] != max(qlo[a], fl)) return false;
    }
    return true;
}

// LDS of one wavefront for walk_faces
struct WalkLds {
    int pre[64];
    int j0[64];
    int xyz[64];
};

// Visit every face stored in the bins of range R (a face stored in several
// bins is met once per bin; callers keep the first common bin).  A round
// loads the extents of 64 bins, one per lane, prefix-sums their lengths and
// then hands the stored faces out one per lane, so the dependent loads of a
// round are issued by the whole wavefront at once.  fn(face, xyz) is called
// with the same trip count on every lane (face < 0 on idle lanes) and may use
// wavefront operations; it returns true (wave-uniformly) to stop the walk.
// Requires a one-wavefront workgroup.
template <class Fn>
__device__ inline void walk_faces(const BinGrid &G, const BinRange &R, const int32_t *__restrict__ bstart,
                                  const int32_t *__restrict__ bitems, WalkLds &L, Fn &&fn)
{
    const int lane = threadIdx.x;
    for (int r = 0; r < R.total; r += 64) {
        const int idx = r + lane;
        int cnt = 0, j0 = 0, packed = 0;
        if (idx < R.total) {
            int xyz[3];
            const int b = range_bin(G, R, idx, xyz);
            j0 = bstart[b];
            cnt = bstart[b + 1] - j0;
            packed = xyz[0] | (xyz[1] << 10) | (xyz[2] << 20);
        }
        int inc = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        const int total = __shfl(inc, 63, 64);
        __syncthreads();
        L.pre[lane] = inc - cnt;
        L.j0[lane] = j0;
        L.xyz[lane] = packed;
        __syncthreads();
        for (int k0 = 0; k0 < total; k0 += 64) {
            const int k = k0 + lane;
            int face = -1, xyz[3] = {0, 0, 0};
            if (k < total) {
                int lo = 0, hi = 63;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.pre[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                face = bitems[L.j0[lo] + (k - L.pre[lo])];
                const int pk = L.xyz[lo];
                xyz[0] = pk & 1023;
                xyz[1] = (pk >> 10) & 1023;
                xyz[2] = pk >> 20;
            }
            if (fn(face, xyz)) return;
        }
    }
}

// a3, bin part: one wavefront per in-box element counts its candidate faces
// (element box overlapping an inflated face box).  Warm start (prev != null):
// the walk also counts faces whose box meets the element box grown by the
// sweep bound; an element meeting none keeps its previous side (the surface
// never came near it between the two poses) and skips the ray test.
__global__ __launch_bounds__(64) void k_candidates(const float *__restrict__ ebox, int64_t stride,
                                                   const float *__restrict__ fbox, const SurfParams *__restrict__ sp,
                                                   const int32_t *__restrict__ bstart,
                                                   const int32_t *__restrict__ bitems,
                                                   const int32_t *__restrict__ list_inbox,
                                                   int32_t *__restrict__ list_near, int32_t *__restrict__ list_far,
                                                   CutCounters *cnt, const int8_t *__restrict__ prev, double sweep,
                                                   int8_t *__restrict__ iblank, int32_t *__restrict__ list_hole)
{
    __shared__ WalkLds L;
    const BinGrid G = sp->grid;
    const int n_in = cnt->n_inbox;
    const int lane = threadIdx.x;
    for (int item = blockIdx.x; item < n_in; item += gridDim.x) {
        const int e = list_inbox[item];
        float eb[6], wb[6];
        for (int k = 0; k < 6; ++k) eb[k] = ebox[(int64_t)k * stride + e];
        for (int k = 0; k < 3; ++k) {
            wb[k] = prev ? f32_down((double)eb[k] - sweep) : eb[k];
            wb[3 + k] = prev ? f32_up((double)eb[3 + k] + sweep) : eb[3 + k];
        }
        int lo[3], hi[3];
        box_bins(G, wb, lo, hi);
        const BinRange R = make_range(lo, hi);
        int nc = 0, nw = 0;
        walk_faces(G, R, bstart, bitems, L, [&](int f, const int *xyz) {
            if (f >= 0) {
                const float *fb = fbox + (int64_t)f * 6;
                if (first_common_bin(G, fb, xyz, lo)) {
                    nc += box_overlap(eb, fb);
                    nw += box_overlap(wb, fb);
                }
            }
            return false;
        });
        const long long tot = wave_sum_ll(nc);
        const long long totw = prev ? wave_sum_ll(nw) : 1;
        if (lane == 0) {
            if (tot > 0) {
                list_near[atomicAdd(&cnt->n_near, 1)] = e;
                atomicAdd(&cnt->n_cand_pairs, (unsigned long long)tot);
            } else if (totw == 0) {
                if (prev[e] == OC_HOLE && iblank[e] != OC_HOLE) {
                    iblank[e] = OC_HOLE;
                    list_hole[atomicAdd(&cnt->n_hole, 1)] = e;
                }
            } else {
                list_far[atomicAdd(&cnt->n_far, 1)] = e;
            }
        }
    }
}

// ------------------------------------------------------------ exact stage --
struct TieRec {
    double absdot, dot;
    double vx, vy, vz, nx, ny, nz;
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
__device__ inline TieRec tie_sel(bool c, const TieRec &x, const TieRec &y)
{
    TieRec r;
    r.absdot = c ? x.absdot : y.absdot;
    r.dot = c ? x.dot : y.dot;
    r.vx = c ? x.vx : y.vx;
    r.vy = c ? x.vy : y.vy;
    r.vz = c ? x.vz : y.vz;
    r.nx = c ? x.nx : y.nx;
    r.ny = c ? x.ny : y.ny;
    r.nz = c ? x.nz : y.nz;
    r.f = c ? x.f : y.f;
    r.s = c ? x.s : y.s;
    r.valid = c ? x.valid : y.valid;
    r.pad = 0;
    return r;
}
// keep the two records that come first in tie order
__device__ inline void tie_offer(TieRec &b1, TieRec &b2, const TieRec &r)
{
    const bool before1 = tie_before(r, b1), before2 = tie_before(r, b2);
    const TieRec n2 = tie_sel(before1, b1, tie_sel(before2, r, b2));
    const TieRec n1 = tie_sel(before1, r, b1);
    b1 = n1;
    b2 = n2;
}

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

__device__ inline double point_box_dist(d3 p, const float *b)
{
    double gx = fmax(0.0, fmax((double)b[0] - p.x, p.x - (double)b[3]));
    double gy = fmax(0.0, fmax((double)b[1] - p.y, p.y - (double)b[4]));
    double gz = fmax(0.0, fmax((double)b[2] - p.z, p.z - (double)b[5]));
    return sqrt(gx * gx + gy * gy + gz * gz);
}

// distance from p to the 8 triangles of a posed face
__device__ inline double point_face_dist(d3 p, const double *__restrict__ P)
{
    double best = INFINITY;
    for (int s = 0; s < 8; ++s) {
        d3 F[3];
        face_tri(P, s, F);
        d3 w = p - closest_on_tri(p, F[0], F[1], F[2]);
        best = fmin(best, dot(w, w));
    }
    return sqrt(best);
}

// box gap test (FP64): closer than tol along every axis
__device__ inline bool boxes_within(const double *a, const double *b, double tol)
{
    return b[0] - a[3] < tol && a[0] - b[3] < tol && b[1] - a[4] < tol && a[1] - b[4] < tol && b[2] - a[5] < tol &&
           a[2] - b[5] < tol;
}

// closed boxes meet
__device__ inline bool boxes_meet(const double *a, const double *b)
{
    return b[0] <= a[3] && a[0] <= b[3] && b[1] <= a[4] && a[1] <= b[4] && b[2] <= a[5] && a[2] <= b[5];
}

// query box [p - r, p + r] rounded outward to FP32 and its bin range
__device__ inline void query_bins(const BinGrid &G, d3 p, double r, int *lo, int *hi)
{
    float qb[6];
    qb[0] = f32_down(p.x - r);
    qb[1] = f32_down(p.y - r);
    qb[2] = f32_down(p.z - r);
    qb[3] = f32_up(p.x + r);
    qb[4] = f32_up(p.y + r);
    qb[5] = f32_up(p.z + r);
    box_bins(G, qb, lo, hi);
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
    int32_t *list_side;
    CutCounters *cnt;
    int8_t *iblank;
    int32_t *list_hole;
    int kind;
    int pad;
    const Pose *pose;       // device pose of the surface
    double first[3];        // first surface node, registration frame
};

constexpr int kFaceCap = 256;

// a4: one wavefront per near element decides whether the surface intersects
// it: some element-boundary / surface triangle pair closer than tol_hit
// (Alg. cp2, with no truncation of the candidate faces), or the whole surface
// inside the element.  Candidate faces that come within the element's
// boundary-face boxes are collected in LDS; for each, the 384 triangle pairs
// are screened by FP64 boxes and only the survivors get the exact test, one
// pair per lane.
__global__ __launch_bounds__(64) void k_hit(ExactArgs a)
{
    __shared__ double sX[81];
    __shared__ double sTB[48 * 6];   // element triangle boxes
    __shared__ double sEF[6 * 6];    // element boundary-face boxes
    __shared__ double sF[27];        // current face nodes
    __shared__ double sFT[8 * 6];    // current face triangle boxes
    __shared__ int sList[kFaceCap];
    __shared__ short sPair[384];
    __shared__ WalkLds L;
    const int lane = threadIdx.x;
    const BinGrid G = a.sp->grid;
    const int n_near = a.cnt->n_near;
    const double tol = kTolHit;
    for (int item = blockIdx.x; item < n_near; item += gridDim.x) {
        const int e = a.list_near[item];
        __syncthreads();
        for (int k = lane; k < 81; k += 64) sX[k] = a.enodes[(int64_t)e * 81 + k];
        __syncthreads();
        if (lane < 48) {
            d3 T[3];
            elem_tri(sX, lane, T);
            double *b = sTB + 6 * lane;
            b[0] = fmin(T[0].x, fmin(T[1].x, T[2].x)); b[3] = fmax(T[0].x, fmax(T[1].x, T[2].x));
            b[1] = fmin(T[0].y, fmin(T[1].y, T[2].y)); b[4] = fmax(T[0].y, fmax(T[1].y, T[2].y));
            b[2] = fmin(T[0].z, fmin(T[1].z, T[2].z)); b[5] = fmax(T[0].z, fmax(T[1].z, T[2].z));
        } else if (lane < 54) {
            const int f = lane - 48;
            double *b = sEF + 6 * f;
            for (int k = 0; k < 3; ++k) {
                b[k] = INFINITY;
                b[3 + k] = -INFINITY;
            }
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v) {
                    const int nd = elem_face_node(f, u, v);
                    for (int k = 0; k < 3; ++k) {
                        b[k] = fmin(b[k], sX[27 * k + nd]);
                        b[3 + k] = fmax(b[3 + k], sX[27 * k + nd]);
                    }
                }
        }
        __syncthreads();
        float eb[6];
        for (int k = 0; k < 6; ++k) eb[k] = a.ebox[(int64_t)k * a.stride + e];
        int lo[3], hi[3];
        box_bins(G, eb, lo, hi);
        const BinRange R = make_range(lo, hi);
        bool hit = false;
        int nlist = 0;
        // exact test of the listed faces
        auto flush = [&]() {
            for (int i = 0; i < nlist && !hit; ++i) {
                const int fid = sList[i];
                if (lane < 27) sF[lane] = a.pnodes[(int64_t)fid * 27 + lane];
                __syncthreads();
                if (lane < 8) {
                    d3 F[3];
                    face_tri(sF, lane, F);
                    double *bb = sFT + 6 * lane;
                    bb[0] = fmin(F[0].x, fmin(F[1].x, F[2].x)); bb[3] = fmax(F[0].x, fmax(F[1].x, F[2].x));
                    bb[1] = fmin(F[0].y, fmin(F[1].y, F[2].y)); bb[4] = fmax(F[0].y, fmax(F[1].y, F[2].y));
                    bb[2] = fmin(F[0].z, fmin(F[1].z, F[2].z)); bb[5] = fmax(F[0].z, fmax(F[1].z, F[2].z));
                }
                __syncthreads();
                // screen the 384 pairs (pair p = 48 * face_tri + elem_tri)
                int np = 0;
                for (int kk = 0; kk < 6; ++kk) {
                    const int p = lane + 64 * kk;
                    const int s = p / 48, t = p - 48 * s;
                    const bool pass = boxes_within(sTB + 6 * t, sFT + 6 * s, tol);
                    const unsigned long long m = __ballot(pass);
                    if (pass) sPair[np + __popcll(m & ((1ull << lane) - 1ull))] = (short)p;
                    np += __popcll(m);
                }
                __syncthreads();
                bool lh = false;
                for (int q = lane; q < np && !lh; q += 64) {
                    const int p = sPair[q];
                    const int s = p / 48, t = p - 48 * s;
                    d3 T[3], F[3];
                    elem_tri(sX, t, T);
                    face_tri(sF, s, F);
                    lh = tri_tri_within(T, F, tol);
                }
                if (__ballot(lh)) hit = true;
                __syncthreads();
            }
            nlist = 0;
        };
        walk_faces(G, R, a.bstart, a.bitems, L, [&](int f, const int *xyz) {
            bool pass = false;
            if (f >= 0) {
                const float *fb = a.fbox + (int64_t)f * 6;
                if (first_common_bin(G, fb, xyz, lo) && box_overlap(eb, fb)) {
                    const double fd[6] = {fb[0], fb[1], fb[2], fb[3], fb[4], fb[5]};
                    for (int q = 0; q < 6; ++q) pass |= boxes_meet(sEF + 6 * q, fd);
                }
            }
            const unsigned long long m = __ballot(pass);
            if (pass) sList[nlist + __popcll(m & ((1ull << lane) - 1ull))] = f;
            nlist += __popcll(m);
            if (nlist > kFaceCap - 64) {
                __syncthreads();
                flush();
            }
            return hit;
        });
        if (!hit && nlist > 0) {
            __syncthreads();
            flush();
        }
        // the whole surface inside the element: ray parity of its first node
        // against the element's 48 boundary triangles
        const d3 sf = pose_apply(*a.pose, mk(a.first[0], a.first[1], a.first[2]));
        if (!hit && sf.x >= eb[0] && sf.x <= eb[3] && sf.y >= eb[1] && sf.y <= eb[4] && sf.z >= eb[2] &&
            sf.z <= eb[5]) {
            int c = 0;
            if (lane < 48) {
                d3 T[3];
                elem_tri(sX, lane, T);
                c = ray_x_crosses(sf, T[0], T[1], T[2]);
            }
            if (__popcll(__ballot(c)) & 1) hit = true;
        }
        if (lane == 0) {
            if (hit) {
                atomicAdd(&a.cnt->n_hit, 1);
                if (a.kind == OC_SURF_WALL && a.iblank[e] != OC_HOLE) {
                    a.iblank[e] = OC_HOLE;
                    a.list_hole[atomicAdd(&a.cnt->n_hole, 1)] = e;
                }
            } else {
                a.list_side[atomicAdd(&a.cnt->n_side, 1)] = e;
            }
        }
    }
}

// a5: near elements that the surface does not intersect lie on one side of
// it; that side is the nearest-face side of the element's first node:
// wavefront minimum of the point-to-triangle distance over the binned faces,
// then the tie rule (largest |dot| of the unit point-to-surface vector with
// the outward triangle normal; normals averaged only for equally visible
// triangles of opposite sign).
__global__ __launch_bounds__(64) void k_side(ExactArgs a)
{
    __shared__ TieRec rec[128];
    __shared__ WalkLds L;
    const int lane = threadIdx.x;
    const BinGrid G = a.sp->grid;
    const int n_side = a.cnt->n_side;
    for (int item = blockIdx.x; item < n_side; item += gridDim.x) {
        const int e = a.list_side[item];
        const double *X = a.enodes + (int64_t)e * 81;
        const d3 p = mk(X[0], X[27], X[54]);
        float eb[6];
        for (int k = 0; k < 6; ++k) eb[k] = a.ebox[(int64_t)k * a.stride + e];
        // upper bound: nearest of the element's candidate faces
        double u = INFINITY;
        {
            int lo[3], hi[3];
            box_bins(G, eb, lo, hi);
            const BinRange R = make_range(lo, hi);
            walk_faces(G, R, a.bstart, a.bitems, L, [&](int f, const int *xyz) {
                if (f >= 0) {
                    const float *fb = a.fbox + (int64_t)f * 6;
                    if (first_common_bin(G, fb, xyz, lo) && box_overlap(eb, fb) && point_box_dist(p, fb) < u)
                        u = fmin(u, point_face_dist(p, a.pnodes + (int64_t)f * 27));
                }
                return false;
            });
        }
        const double U = wave_min_d(u);
        // every face whose box is within U of the node
        double best = U;
        {
            int lo[3], hi[3];
            query_bins(G, p, U, lo, hi);
            const BinRange R = make_range(lo, hi);
            walk_faces(G, R, a.bstart, a.bitems, L, [&](int f, const int *xyz) {
                if (f >= 0) {
                    const float *fb = a.fbox + (int64_t)f * 6;
                    if (first_common_bin(G, fb, xyz, lo) && point_box_dist(p, fb) <= best)
                        best = fmin(best, point_face_dist(p, a.pnodes + (int64_t)f * 27));
                }
                return false;
            });
        }
        best = wave_min_d(best);
        // tie set within best * (1 + 1e-9)
        const double thr = best * (1.0 + 1e-9);
        TieRec b1, b2;
        b1.valid = b2.valid = 0;
        {
            int lo[3], hi[3];
            query_bins(G, p, thr, lo, hi);
            const BinRange R = make_range(lo, hi);
            walk_faces(G, R, a.bstart, a.bitems, L, [&](int f, const int *xyz) {
                if (f >= 0) {
                    const float *fb = a.fbox + (int64_t)f * 6;
                    if (first_common_bin(G, fb, xyz, lo) && point_box_dist(p, fb) <= thr) {
                        const double *P = a.pnodes + (int64_t)f * 27;
                        for (int s = 0; s < 8; ++s) {
                            d3 F[3];
                            face_tri(P, s, F);
                            const d3 v = p - closest_on_tri(p, F[0], F[1], F[2]);
                            const double d = sqrt(dot(v, v));
                            if (d > thr) continue;
                            const d3 n = cross(F[1] - F[0], F[2] - F[0]);
                            const double ln = sqrt(dot(n, n));
                            TieRec rr;
                            rr.vx = v.x;
                            rr.vy = v.y;
                            rr.vz = v.z;
                            rr.nx = ln > 0 ? n.x / ln : 0.0;
                            rr.ny = ln > 0 ? n.y / ln : 0.0;
                            rr.nz = ln > 0 ? n.z / ln : 0.0;
                            rr.dot = d > 0 ? (v.x * rr.nx + v.y * rr.ny + v.z * rr.nz) / d : 0.0;
                            rr.absdot = fabs(rr.dot);
                            rr.f = f;
                            rr.s = s;
                            rr.valid = 1;
                            rr.pad = 0;
                            tie_offer(b1, b2, rr);
                        }
                    }
                }
                return false;
            });
        }
        __syncthreads();
        rec[2 * lane] = b1;
        rec[2 * lane + 1] = b2;
        __syncthreads();
        if (lane == 0) {
            TieRec c1, c2;
            c1.valid = c2.valid = 0;
            for (int k = 0; k < 128; ++k)
                if (rec[k].valid) tie_offer(c1, c2, rec[k]);
            double sg = c1.dot;
            if (c2.valid && c1.absdot - c2.absdot <= 1e-9 && ((c1.dot > 0.0) != (c2.dot > 0.0)))
                sg = c1.vx * (c1.nx + c2.nx) + c1.vy * (c1.ny + c2.ny) + c1.vz * (c1.nz + c2.nz);
            if (c1.valid && sg < 0.0 && a.iblank[e] != OC_HOLE) {
                a.iblank[e] = OC_HOLE;
                a.list_hole[atomicAdd(&a.cnt->n_hole, 1)] = e;
            }
        }
    }
}

// a6: far elements (no candidate face): +x ray parity of the first node over
// the column of bins that holds the ray.
__global__ __launch_bounds__(64) void k_ray(const double *__restrict__ enodes, const double *__restrict__ pnodes,
                                            const float *__restrict__ fbox, const SurfParams *__restrict__ sp,
                                            const int32_t *__restrict__ bstart, const int32_t *__restrict__ bitems,
                                            const int32_t *__restrict__ list_far, CutCounters *cnt,
                                            int8_t *__restrict__ iblank, int32_t *__restrict__ list_hole)
{
    __shared__ WalkLds L;
    const BinGrid G = sp->grid;
    const int n_far = cnt->n_far;
    const int lane = threadIdx.x;
    const float sb[6] = {sp->sbox[0], sp->sbox[1], sp->sbox[2], sp->sbox[3], sp->sbox[4], sp->sbox[5]};
    for (int item = blockIdx.x; item < n_far; item += gridDim.x) {
        const int e = list_far[item];
        const double *X = enodes + (int64_t)e * 81;
        const d3 p = mk(X[0], X[27], X[54]);
        if (p.y < sb[1] || p.y > sb[4] || p.z < sb[2] || p.z > sb[5] || p.x > sb[3]) continue;
        int lo[3], hi[3];
        lo[0] = bin_of((float)p.x, G.o[0], G.inv[0], G.n[0]);
        lo[1] = hi[1] = bin_of((float)p.y, G.o[1], G.inv[1], G.n[1]);
        lo[2] = hi[2] = bin_of((float)p.z, G.o[2], G.inv[2], G.n[2]);
        hi[0] = G.n[0] - 1;
        const BinRange R = make_range(lo, hi);
        int par = 0;
        walk_faces(G, R, bstart, bitems, L, [&](int f, const int *xyz) {
            if (f >= 0) {
                const float *fb = fbox + (int64_t)f * 6;
                if (first_common_bin(G, fb, xyz, lo) && (double)fb[1] <= p.y && (double)fb[4] >= p.y &&
                    (double)fb[2] <= p.z && (double)fb[5] >= p.z && (double)fb[3] >= p.x) {
                    const double *P = pnodes + (int64_t)f * 27;
                    for (int s = 0; s < 8; ++s) {
                        d3 F[3];
                        face_tri(P, s, F);
                        par ^= ray_x_crosses(p, F[0], F[1], F[2]);
                    }
                }
            }
            return false;
        });
        const int odd = __popcll(__ballot(par)) & 1;
        if (lane == 0 && odd && iblank[e] != OC_HOLE) {
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
        time_begin(ctx, st, #name, &slot_);                                                  \
        hipLaunchKernelGGL(name, grid, block, 0, st, __VA_ARGS__);                           \
        time_end(ctx, st, slot_);                                                            \
    } while (0)

static oc_status cut_one_surface(oc_slot *sl, Grid &g, int surf_id, Surf &s, const Pose *pose_dev, int8_t *iblank,
                                 bool first, const int8_t *prev, double sweep)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    SurfWork &w = sl->sw.at(surf_id);
    const unsigned fb = grid_for(s.n_face, kThreads, 1u << 30);
    LAUNCH(k_surf_init, dim3(1), dim3(64), w.params, sl->counters);
    LAUNCH(k_pose_faces, dim3(fb), dim3(kThreads), s.nodes, s.n_nodes, s.conn, s.n_face, pose_dev, w.pnodes, w.fbox,
           w.params);
    LAUNCH(k_bins_setup, dim3(1), dim3(64), w.params, s.dmax, s.nb_max);
    const int64_t bcap = (int64_t)s.nb_max * s.nb_max * s.nb_max;
    LAUNCH(k_zero_i32, dim3(grid_for(bcap + 1, kThreads, 4096)), dim3(kThreads), w.bin_count, &w.params->n_bins,
           (int64_t)0);
    LAUNCH(k_bin_count, dim3(fb), dim3(kThreads), w.fbox, s.n_face, w.params, w.bin_count);
    OC_TRY(scan_exclusive(ctx, st, w.bin_count, w.bin_start, bcap, &w.params->n_bins, w.scan_tmp));
    LAUNCH(k_bin_fill, dim3(fb), dim3(kThreads), w.fbox, s.n_face, w.params, w.bin_start, w.bin_count, w.bin_items);

    LAUNCH(k_filter, dim3(grid_for(g.n_elem, kThreads * 4, 8192)), dim3(kThreads), g.ebox, g.n_elem, g.ebox_stride,
           w.params, iblank, first ? 1 : 0, sl->list_inbox, sl->counters);
    LAUNCH(k_candidates, dim3(8192), dim3(64), g.ebox, g.ebox_stride, w.fbox, w.params, w.bin_start, w.bin_items,
           sl->list_inbox, sl->list_near, sl->list_far, sl->counters, prev, sweep, iblank, sl->list_hole);
    ExactArgs ea;
    ea.enodes = g.enodes;
    ea.ebox = g.ebox;
    ea.stride = g.ebox_stride;
    ea.pnodes = w.pnodes;
    ea.fbox = w.fbox;
    ea.bstart = w.bin_start;
    ea.bitems = w.bin_items;
    ea.sp = w.params;
    ea.list_near = sl->list_near;
    ea.list_side = sl->list_side;
    ea.cnt = sl->counters;
    ea.iblank = iblank;
    ea.list_hole = sl->list_hole;
    ea.kind = s.kind;
    ea.pad = 0;
    ea.pose = pose_dev;
    for (int i = 0; i < 3; ++i) ea.first[i] = s.first[i];
    LAUNCH(k_hit, dim3(8192), dim3(64), ea);
    LAUNCH(k_side, dim3(8192), dim3(64), ea);
    LAUNCH(k_ray, dim3(8192), dim3(64), g.enodes, w.pnodes, w.fbox, w.params, w.bin_start, w.bin_items,
           sl->list_far, sl->counters, iblank, sl->list_hole);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

struct PosePack {
    Pose p[8];
    int n;
};

__global__ void k_set_poses(Pose *dst, PosePack pk)
{
    if (blockIdx.x == 0 && (int)threadIdx.x < pk.n) dst[threadIdx.x] = pk.p[threadIdx.x];
}

// Host poses into the slot's device pose slots, ordered on the slot stream
// (the values travel as kernel arguments, so the host array may be reused
// as soon as this returns).
oc_status set_poses(oc_slot *sl, int first, const double *host, int n)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    if (first < 0 || n < 0 || first + n > kPoseSlots) {
        set_error("too many poses");
        return OC_EINVAL;
    }
    for (int k0 = 0; k0 < n; k0 += 8) {
        PosePack pk;
        pk.n = std::min(8, n - k0);
        for (int k = 0; k < pk.n; ++k) {
            for (int i = 0; i < 9; ++i) pk.p[k].r[i] = host[12 * (k0 + k) + i];
            for (int i = 0; i < 3; ++i) pk.p[k].t[i] = host[12 * (k0 + k) + 9 + i];
        }
        LAUNCH(k_set_poses, dim3(1), dim3(64), sl->poses + first + k0, pk);
    }
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status cut_run(oc_slot *sl, Grid &g, const int *surf_ids, Surf **surfs, const Pose *poses_dev, int n_surf,
                  int8_t *iblank, const int8_t *prev, double sweep)
{
    if (prev && n_surf != 1) {
        set_error("warm start needs exactly one cutting surface");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    OC_TRY(slot_reserve_grid(sl, g));
    for (int k = 0; k < n_surf; ++k) OC_TRY(slot_reserve_surf(sl, surf_ids[k], *surfs[k]));
    sl->last_n_elem = g.n_elem;
    LAUNCH(k_reset_counters, dim3(1), dim3(64), sl->counters);
    if (n_surf == 0)
        LAUNCH(k_fill_i8, dim3(grid_for(g.n_elem, kThreads, 4096)), dim3(kThreads), iblank, g.n_elem,
               (int8_t)OC_FIELD);
    for (int k = 0; k < n_surf; ++k)
        OC_TRY(cut_one_surface(sl, g, surf_ids[k], *surfs[k], poses_dev + k, iblank, k == 0, prev, sweep));
    LAUNCH(k_fringe, dim3(1024), dim3(kThreads), g.nbr, sl->list_hole, sl->counters, iblank);
    if (g.n_overset > 0)
        LAUNCH(k_overset_fringe, dim3(grid_for(g.n_overset, kThreads, 4096)), dim3(kThreads), g.overset, g.n_overset,
               iblank);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

}  // namespace oc
