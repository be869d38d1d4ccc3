// Direct cut of curved quadratic grids by closed cutting surfaces
// (Sec. 4.2, parallel direct cut): every element decides on its own whether
// it is intersected by, inside or outside the surface, so no paint-fill is
// needed.
//
// A call cuts a batch: one or more requests, each a grid cut by one or more
// surfaces into its own iblank.  Each (grid, surface, pose) is a "cut" with
// a descriptor (CutInst); every stage is one launch for the whole batch:
//   k_pose_faces                    pose the surface nodes, FP32 face boxes
//                                   inflated by the hit tolerance, surface box
//   k_bin_count / scan /            uniform bins over each surface box (each
//   k_bin_fill                      cut's bins at a fixed offset, its caps
//                                   nb_max^3): count, scan, fill (CSR)
//   k_filter                        stream every element's FP32 box; boxes
//                                   meeting the surface box go to a list
//   k_candidates                    element box x binned face boxes: elements
//                                   with a candidate face are "near", others
//                                   "far" and decided at once by the +x ray
//                                   parity of the first node
//   k_hit                           one wavefront per near element: FP64
//                                   triangle-pair intersection
//   k_side                          near elements not hit: nearest-face side of
//                                   the first node (wavefront minimum + tie rule)
//   k_fringe / k_overset_fringe     one fringe layer around holes, overset faces
#include <algorithm>
#include <cstring>

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

// Owner of block b in a launch flattened over several entries: the number
// of entries k >= 1 whose first block is <= b (first blocks never decrease,
// entries with no block share their successor's first block).  Called by
// every thread of the block.
template <class F>
__device__ inline int block_owner(int n, int b, F first)
{
    int c = 0;
    for (int k0 = 1; k0 < n; k0 += blockDim.x) {
        const int k = k0 + (int)threadIdx.x;
        c += __syncthreads_count(k < n && first(k) <= b);
    }
    return c;
}

__device__ inline uint64_t pack_item(int cut, int e) { return ((uint64_t)(uint32_t)cut << 32) | (uint32_t)e; }
__device__ inline int item_cut(uint64_t v) { return (int)(v >> 32); }
__device__ inline int item_elem(uint64_t v) { return (int)(uint32_t)v; }

// ------------------------------------------------------- surface stage ----
// a1 + a2 (face boxes): pose the 9 nodes of every face (x' = R x + t), store
// them face-major, and build the face's FP32 box rounded outward and inflated
// by tol_hit + 2^-20 * max|coordinate|.  A face takes a group of 16 lanes,
// one node per lane (lanes 9..15 idle), so the gathers of a face's nodes are
// issued together; the face box is reduced within the group.  Blocks hold
// kPoseFaces faces and are flattened over the cuts (pblk0); each block writes
// the box of its faces to part[block] (ordered ints) and every block of
// k_bin_count reduces its cut's blocks (no contended atomics).
constexpr int kPoseFaces = kThreads / 16;

// A batch of one cut passes its descriptor by value (one, with dst the
// slot's descriptor array): block 0 stores it for the later stages, so no
// separate upload launch is needed.
__global__ __launch_bounds__(kThreads) void k_pose_faces(const CutInst *__restrict__ I, int n_cut,
                                                         int32_t *__restrict__ part, CutInst one, CutInst *dst)
{
    __shared__ float wb[kThreads / 64][6];
    const double *__restrict__ nodes;
    const int32_t *__restrict__ conn;
    int64_t n_nodes, n_face;
    double *__restrict__ pnodes;
    float *__restrict__ fbox;
    const Pose *pose_p;
    int pblk0;
    if (dst) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *dst = one;
        nodes = one.snodes;
        conn = one.conn;
        n_nodes = one.n_nodes;
        n_face = one.n_face;
        pnodes = one.pnodes;
        fbox = one.fbox;
        pose_p = one.pose;
        pblk0 = one.pblk0;
    } else {
        const CutInst &c = I[block_owner(n_cut, blockIdx.x, [&](int k) { return I[k].pblk0; })];
        nodes = c.snodes;
        conn = c.conn;
        n_nodes = c.n_nodes;
        n_face = c.n_face;
        pnodes = c.pnodes;
        fbox = c.fbox;
        pose_p = c.pose;
        pblk0 = c.pblk0;
    }
    const Pose pose = *pose_p;
    const int j = threadIdx.x & 15;
    const int64_t f = (int64_t)(blockIdx.x - pblk0) * kPoseFaces + (threadIdx.x >> 4);
    const bool on = f < n_face && j < 9;
    double xv[3] = {0.0, 0.0, 0.0};
    if (on) {
        const int id = conn[f * 9 + j];
        const d3 x = pose_apply(pose, mk(nodes[id], nodes[n_nodes + id], nodes[2 * n_nodes + id]));
        xv[0] = x.x;
        xv[1] = x.y;
        xv[2] = x.z;
        pnodes[f * 27 + j] = x.x;
        pnodes[f * 27 + 9 + j] = x.y;
        pnodes[f * 27 + 18 + j] = x.z;
    }
    double blo[3], bhi[3], L = on ? fmax(fabs(xv[0]), fmax(fabs(xv[1]), fabs(xv[2]))) : 0.0;
    for (int k = 0; k < 3; ++k) {
        blo[k] = on ? xv[k] : INFINITY;
        bhi[k] = on ? xv[k] : -INFINITY;
    }
#pragma unroll
    for (int d = 8; d >= 1; d >>= 1) {
        for (int k = 0; k < 3; ++k) {
            blo[k] = fmin(blo[k], __shfl_xor(blo[k], d, 64));
            bhi[k] = fmax(bhi[k], __shfl_xor(bhi[k], d, 64));
        }
        L = fmax(L, __shfl_xor(L, d, 64));
    }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (f < n_face && j == 0) {
        const double delta = kTolHit + ldexp(L, -20);
        for (int a = 0; a < 3; ++a) {
            lo[a] = f32_down(blo[a] - delta);
            hi[a] = f32_up(bhi[a] + delta);
            fbox[f * 6 + a] = lo[a];
            fbox[f * 6 + 3 + a] = hi[a];
        }
    }
    // surface box of the block: wavefront reduction, then across wavefronts
    for (int a = 0; a < 3; ++a) {
        float l = lo[a], h = hi[a];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            l = fminf(l, __shfl_xor(l, d, 64));
            h = fmaxf(h, __shfl_xor(h, d, 64));
        }
        if (lane_id() == 0) {
            wb[threadIdx.x >> 6][a] = l;
            wb[threadIdx.x >> 6][3 + a] = h;
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float v = wb[0][k];
        for (int w = 1; w < kThreads / 64; ++w) v = k < 3 ? fminf(v, wb[w][k]) : fmaxf(v, wb[w][k]);
        part[(int64_t)blockIdx.x * 6 + k] = f2ord(v);
    }
}

// exclusive scan over a block of kThreads (one value per thread)
__device__ inline int block_scan_excl(int v, int *total)
{
    __shared__ int wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Bin grid over a cut's surface box.  The bin edge is at least the largest
// face box extent (dmax + 2 delta, pose invariant), so a face spans at most
// two bins per axis and at most 8 bins in total; at most nb_max bins per
// axis.
__device__ inline void bin_grid(const float *sbox, float dmax, int nb_max, BinGrid &G, int *n_bins)
{
    float L = 0.f;
    for (int k = 0; k < 6; ++k) L = fmaxf(L, fabsf(sbox[k]));
    const float w = (dmax + 2.0f * (1e-7f + ldexpf(L, -20)) + ldexpf(L, -18)) * 1.001f;
    int nb = 1;
    for (int a = 0; a < 3; ++a) {
        float ext = sbox[3 + a] - sbox[a];
        int n = 1;
        if (ext > 0.f) {
            float q = fminf(floorf(ext / w), (float)nb_max);
            n = q < 1.f ? 1 : (int)q;
        }
        G.o[a] = sbox[a];
        G.n[a] = n;
        G.inv[a] = ext > 0.f ? (float)n / ext : 0.f;
        nb *= n;
    }
    *n_bins = nb;
}

__device__ inline void box_bins(const BinGrid &G, const float *b, int *lo, int *hi)
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = bin_of(b[a], G.o[a], G.inv[a], G.n[a]);
        hi[a] = bin_of(b[3 + a], G.o[a], G.inv[a], G.n[a]);
    }
}

// Bin counts of every face, after the cut's surface box and bin grid: each
// block folds its cut's per-pose-block partial boxes (no contended atomics;
// every block of a cut gets the same grid) and the cut's first block stores
// the box and grid for the later stages.  A cut's bins start at bin_off0, the
// sum of the bin caps nb_max^3 of the cuts before it (host side).  The
// first block also resets the batch's list counters.
__global__ __launch_bounds__(kThreads) void k_bin_count(const CutInst *__restrict__ I, int n_cut,
                                                        const int32_t *__restrict__ part, int32_t *__restrict__ count,
                                                        CutCounters *cnt)
{
    __shared__ int wb[kThreads / 64][6];
    __shared__ BinGrid sG;
    const int ci = block_owner(n_cut, blockIdx.x, [&](int k) { return I[k].fblk0; });
    const CutInst &c = I[ci];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cnt->n_inbox = 0;     // k_filter appends after this kernel
        cnt->n_sidelist = 0;  // k_hit appends after it
    }
    {
        const int b0 = c.pblk0, nblk = (int)((c.n_face + kPoseFaces - 1) / kPoseFaces);
        int ob[6] = {f2ord(INFINITY), f2ord(INFINITY), f2ord(INFINITY), f2ord(-INFINITY), f2ord(-INFINITY),
                     f2ord(-INFINITY)};
        for (int b = b0 + (int)threadIdx.x; b < b0 + nblk; b += kThreads)
            for (int k = 0; k < 6; ++k) {
                const int v = part[(int64_t)b * 6 + k];
                ob[k] = k < 3 ? min(ob[k], v) : max(ob[k], v);
            }
        for (int k = 0; k < 6; ++k)
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                const int o = __shfl_xor(ob[k], d, 64);
                ob[k] = k < 3 ? min(ob[k], o) : max(ob[k], o);
            }
        if (lane_id() == 0)
            for (int k = 0; k < 6; ++k) wb[threadIdx.x >> 6][k] = ob[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            float sbox[6];
            for (int k = 0; k < 6; ++k) {
                int v = wb[0][k];
                for (int w = 1; w < kThreads / 64; ++w) v = k < 3 ? min(v, wb[w][k]) : max(v, wb[w][k]);
                sbox[k] = ord2f(v);
            }
            BinGrid G;
            int nb;
            bin_grid(sbox, c.dmax, c.nb_max, G, &nb);
            sG = G;
            if ((int)blockIdx.x == c.fblk0) {
                SurfParams *sp = c.params;
                for (int k = 0; k < 6; ++k) sp->sbox[k] = sbox[k];
                sp->grid = G;
                sp->n_bins = nb;
                sp->bin_off = c.bin_off0;
            }
        }
        __syncthreads();
    }
    const int64_t f = (int64_t)(blockIdx.x - c.fblk0) * blockDim.x + threadIdx.x;
    if (f >= c.n_face) return;
    const BinGrid G = sG;
    int32_t *cb = count + c.bin_off0;
    int lo[3], hi[3];
    box_bins(G, c.fbox + f * 6, lo, hi);
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) atomicAdd(&cb[x + G.n[0] * (y + G.n[1] * z)], 1);
}

// fill: the count array doubles as the per-bin cursor and ends at zero;
// each entry is a 32-byte record of the face's FP32 box and its id local to
// its cut (lo xyz + id bits, hi xyz + 0), so bin walks read the boxes
// together with the ids
__global__ __launch_bounds__(kThreads) void k_bin_fill(const CutInst *__restrict__ I, int n_cut,
                                                       const int32_t *__restrict__ start, int32_t *count,
                                                       float4 *__restrict__ rec)
{
    const int ci = block_owner(n_cut, blockIdx.x, [&](int k) { return I[k].fblk0; });
    const CutInst &c = I[ci];
    const int64_t f = (int64_t)(blockIdx.x - c.fblk0) * blockDim.x + threadIdx.x;
    if (f >= c.n_face) return;
    const BinGrid G = c.params->grid;
    const int off = c.params->bin_off;
    const float *fb = c.fbox + f * 6;
    const float4 r0 = make_float4(fb[0], fb[1], fb[2], __int_as_float((int)f));
    const float4 r1 = make_float4(fb[3], fb[4], fb[5], 0.f);
    int lo[3], hi[3];
    box_bins(G, fb, lo, hi);
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                const int b = off + x + G.n[0] * (y + G.n[1] * z);
                const int64_t j = (int64_t)start[b] + (atomicSub(&count[b], 1) - 1);
                rec[2 * j] = r0;
                rec[2 * j + 1] = r1;
            }
}

// ---------------------------------------------------------- element stage --
// In-box bits of the four elements e0 .. e0 + 3 (their FP32 boxes in SoA
// planes) against the surface box sb.  The planes are read axis by axis, z
// first: once no element of the wavefront is left along an axis it reads no
// further planes (neighbouring elements share their slow coordinates).
__device__ inline int filter_quad(const float *__restrict__ ebox, int64_t stride, int64_t e0, const float *sb)
{
    int flags = 0;
#pragma unroll
    for (int ax = 2; ax >= 0; --ax) {
        if (ax < 2 && !__ballot(flags != 0)) return 0;
        const float4 l = *reinterpret_cast<const float4 *>(ebox + ax * stride + e0);
        const float4 h = *reinterpret_cast<const float4 *>(ebox + (3 + ax) * stride + e0);
        const float L[4] = {l.x, l.y, l.z, l.w}, H[4] = {h.x, h.y, h.z, h.w};
        int in = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) in |= (int)(L[k] <= sb[3 + ax] && H[k] >= sb[ax]) << k;
        flags = ax == 2 ? in : (flags & in);
    }
    return flags;
}

// a3, streaming part: every element's FP32 box (SoA planes, 4 elements per
// thread) is tested against its cut's surface box.  The first cut of an
// output also initialises its iblank to field.  Blocks are flattened over
// the cuts, 1024 elements per block.
__global__ __launch_bounds__(1024) void k_filter(const CutInst *__restrict__ I, int n_cut, CutInst one, int use_one,
                                                 uint64_t *__restrict__ list_inbox, CutCounters *cnt)
{
    // a batch of one cut passes its descriptor by value (no dependent load
    // of it before the element loads)
    int ci = 0;
    const float *__restrict__ ebox;
    const float *__restrict__ wbox;
    int64_t stride_e, n_elem;
    int8_t *__restrict__ iblank;
    int write_field, eblk0;
    const SurfParams *sp;
    if (use_one) {
        ebox = one.ebox;
        wbox = one.wbox;
        stride_e = one.stride;
        n_elem = one.n_elem;
        iblank = one.iblank;
        write_field = one.write_field;
        eblk0 = one.eblk0;
        sp = one.params;
    } else {
        ci = block_owner(n_cut, blockIdx.x, [&](int k) { return I[k].eblk0; });
        const CutInst &c = I[ci];
        ebox = c.ebox;
        wbox = c.wbox;
        stride_e = c.stride;
        n_elem = c.n_elem;
        iblank = c.iblank;
        write_field = c.write_field;
        eblk0 = c.eblk0;
        sp = c.params;
    }
    const int64_t e0 = ((int64_t)(blockIdx.x - eblk0) * blockDim.x + threadIdx.x) * 4;
    int flags = 0, cn = 0;
    if (e0 - (int64_t)lane_id() * 4 < n_elem) {   // the wavefront has elements
        const float s0 = sp->sbox[0], s1 = sp->sbox[1], s2 = sp->sbox[2];
        const float s3 = sp->sbox[3], s4 = sp->sbox[4], s5 = sp->sbox[5];
        // the wavefront's 256 elements (e0 of its first lane is a multiple
        // of 256) are skipped together when their union box misses the
        // surface box
        bool meets = true;
        if (wbox) {
            const float *wb = wbox + (e0 >> 8) * 6;
            meets = wb[0] <= s3 && wb[3] >= s0 && wb[1] <= s4 && wb[4] >= s1 && wb[2] <= s5 && wb[5] >= s2;
        }
        if (e0 + 3 < n_elem) {
            const float sb[6] = {s0, s1, s2, s3, s4, s5};
            if (meets) flags = filter_quad(ebox, stride_e, e0, sb);
            cn = __popc(flags);
            if (write_field) *reinterpret_cast<uint32_t *>(iblank + e0) = 0x01010101u;
        } else {
            for (int k = 0; k < 4; ++k) {
                int64_t e = e0 + k;
                if (e >= n_elem) break;
                bool in = meets && ebox[e] <= s3 && ebox[3 * stride_e + e] >= s0 && ebox[stride_e + e] <= s4 &&
                          ebox[4 * stride_e + e] >= s1 && ebox[2 * stride_e + e] <= s5 &&
                          ebox[5 * stride_e + e] >= s2;
                flags |= (int)in << k;
                cn += in;
                if (write_field) iblank[e] = OC_FIELD;
            }
        }
    }
    // one list reservation per block: the in-box elements cluster, and
    // appends to one counter from many wavefronts serialise
    __shared__ int s_tot[1024 / 64 + 1];
    const int lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc = cn;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) s_tot[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < nw; ++w) {
            const int t = s_tot[w];
            s_tot[w] = run;
            run += t;
        }
        s_tot[nw] = run > 0 ? atomicAdd(&cnt->n_inbox, run) : 0;
    }
    __syncthreads();
    int pos = s_tot[nw] + s_tot[wid] + inc - cn;
    for (int k = 0; k < 4; ++k)
        if (flags >> k & 1) list_inbox[pos++] = pack_item(ci, (int)(e0 + k));
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

// Orders LDS accesses between the lanes of a workgroup, or with kWave only
// between those of one wavefront (its LDS operations complete in order, so a
// wavefront-scope fence that the compiler keeps in place is enough).
template <bool kWave>
__device__ inline void group_sync()
{
    if constexpr (kWave) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
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
// round are issued by the whole wavefront at once.  fn(face, fb, xyz) gets
// the face's FP32 box fb from its bin record; it is called with the same
// trip count on every lane (face < 0 on idle lanes) and may use wavefront
// operations; it returns true (wave-uniformly) to stop the walk.
// The walk synchronises its workgroup: every wavefront of the workgroup must
// walk the same range R (each with its own WalkLds), and only a one-wavefront
// workgroup may stop early.  With kWave it synchronises only its own
// wavefront, which then walks alone (nparts = 1) whatever the others do.
// With nparts > 1 only the chunks of 64 stored faces whose running index is
// part (mod nparts) are visited, so nparts wavefronts can share one walk.
template <bool kWave = false, class Fn>
__device__ inline void walk_faces(const BinGrid &G, const BinRange &R, const int32_t *__restrict__ bstart,
                                  const float4 *__restrict__ brec, WalkLds &L, Fn &&fn, int part = 0,
                                  int nparts = 1, int64_t n_rec = INT64_MAX, int64_t n_face = INT64_MAX,
                                  uint32_t *err = nullptr)
{
    const int lane = threadIdx.x & 63;
    int chunk = 0;
    for (int r = 0; r < R.total; r += 64) {
        const int idx = r + lane;
        int cnt = 0, j0 = 0, packed = 0;
        if (idx < R.total) {
            int xyz[3];
            const int b = range_bin(G, R, idx, xyz);
            j0 = bstart[b];
            cnt = bstart[b + 1] - j0;
            if (!chk(j0 >= 0 && cnt >= 0 && (int64_t)j0 + cnt <= n_rec, err, kChkSurfBin)) cnt = 0;
            packed = xyz[0] | (xyz[1] << 10) | (xyz[2] << 20);
        }
        int inc = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        const int total = __shfl(inc, 63, 64);
        group_sync<kWave>();
        L.pre[lane] = inc - cnt;
        L.j0[lane] = j0;
        L.xyz[lane] = packed;
        group_sync<kWave>();
        for (int k0 = 0; k0 < total; k0 += 64, ++chunk) {
            if (chunk % nparts != part) continue;
            const int k = k0 + lane;
            int face = -1, xyz[3] = {0, 0, 0};
            float fb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (k < total) {
                int lo = 0, hi = 63;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.pre[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                const int64_t j = (int64_t)L.j0[lo] + (k - L.pre[lo]);
                const float4 r0 = brec[2 * j], r1 = brec[2 * j + 1];
                face = __float_as_int(r0.w);
                if (!chk(face >= 0 && face < n_face, err, kChkSurfFace)) face = -1;
                fb[0] = r0.x;
                fb[1] = r0.y;
                fb[2] = r0.z;
                fb[3] = r1.x;
                fb[4] = r1.y;
                fb[5] = r1.z;
                const int pk = L.xyz[lo];
                xyz[0] = pk & 1023;
                xyz[1] = (pk >> 10) & 1023;
                xyz[2] = pk >> 20;
            }
            if (fn(face, fb, xyz)) return;
        }
    }
}

// a6: a far element (no candidate face) lies on one side of the surface:
// +x ray parity of its first node over the column of bins that holds the
// ray (one wavefront).
__device__ inline void ray_item(const CutInst &c, const int32_t *__restrict__ bin_start,
                                const float4 *__restrict__ brec, int e, WalkLds &L, int64_t n_rec, uint32_t *err)
{
    const int lane = threadIdx.x & 63;
    const SurfParams *sp = c.params;
    const double *X = c.enodes + (int64_t)e * 81;
    const d3 p = mk(X[0], X[27], X[54]);
    if (p.y < sp->sbox[1] || p.y > sp->sbox[4] || p.z < sp->sbox[2] || p.z > sp->sbox[5] || p.x > sp->sbox[3])
        return;
    const BinGrid G = sp->grid;
    const int32_t *bstart = bin_start + sp->bin_off;
    const double *__restrict__ pnodes = c.pnodes;
    int lo[3], hi[3];
    lo[0] = bin_of((float)p.x, G.o[0], G.inv[0], G.n[0]);
    lo[1] = hi[1] = bin_of((float)p.y, G.o[1], G.inv[1], G.n[1]);
    lo[2] = hi[2] = bin_of((float)p.z, G.o[2], G.inv[2], G.n[2]);
    hi[0] = G.n[0] - 1;
    const BinRange R = make_range(lo, hi);
    int par = 0;
    walk_faces(G, R, bstart, brec, L, [&](int f, const float *fb, const int *xyz) {
        if (f >= 0) {
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
    }, 0, 1, n_rec, c.n_face, err);
    const int odd = __popcll(__ballot(par)) & 1;
    if (lane == 0 && odd) c.iblank[e] = OC_HOLE;
}

// a3, bin part: one wavefront per in-box element counts its candidate faces
// (element box overlapping an inflated face box) and marks the item near
// (some candidate) or far (none); a far element is then decided here by its
// ray parity (ray_item: far elements need no exact test, and this kernel
// holds more wavefronts per SIMD than the exact stage).  Warm start
// (prev != null): the walk also counts faces whose box meets the element
// box grown by the sweep bound; an element meeting none keeps its previous
// side (the surface never came near it between the two poses) and needs no
// further test.  k_hit takes the near items by status.
__global__ __launch_bounds__(64) void k_candidates(const CutInst *__restrict__ I, const int32_t *__restrict__ bin_start,
                                                   const float4 *__restrict__ brec,
                                                   const uint64_t *__restrict__ list_inbox, uint8_t *__restrict__ stat,
                                                   int32_t *__restrict__ ncand, const CutCounters *cnt,
                                                   int64_t bins_total, uint32_t *err)
{
    __shared__ WalkLds L;
    const int64_t n_rec = chk_size(bin_start + bins_total);
    const int n_in = cnt->n_inbox;
    const int lane = threadIdx.x;
    for (int item = blockIdx.x; item < n_in; item += gridDim.x) {
        const uint64_t it = list_inbox[item];
        const int ci = item_cut(it), e = item_elem(it);
        const CutInst &c = I[ci];
        const int8_t *prev = c.prev;
        const double sweep = c.sweep;
        const BinGrid G = c.params->grid;
        const int32_t *bstart = bin_start + c.params->bin_off;
        float eb[6], wb[6];
        for (int k = 0; k < 6; ++k) eb[k] = c.ebox[(int64_t)k * c.stride + e];
        for (int k = 0; k < 3; ++k) {
            wb[k] = prev ? f32_down((double)eb[k] - sweep) : eb[k];
            wb[3 + k] = prev ? f32_up((double)eb[3 + k] + sweep) : eb[3 + k];
        }
        int lo[3], hi[3];
        box_bins(G, wb, lo, hi);
        const BinRange R = make_range(lo, hi);
        int nc = 0, nw = 0;
        walk_faces(G, R, bstart, brec, L, [&](int f, const float *fb, const int *xyz) {
            if (f >= 0) {
                if (first_common_bin(G, fb, xyz, lo)) {
                    nc += box_overlap(eb, fb);
                    nw += box_overlap(wb, fb);
                }
            }
            return false;
        }, 0, 1, n_rec, c.n_face, err);
        const long long tot = wave_sum_ll(nc);
        const long long totw = prev ? wave_sum_ll(nw) : 1;
        if (lane == 0) {
            uint8_t st = ST_FAR;
            if (tot > 0) {
                st = ST_NEAR;
            } else if (totw == 0) {
                st = ST_NONE;
                if (prev[e] == OC_HOLE) c.iblank[e] = OC_HOLE;
            }
            stat[item] = st;
            ncand[item] = (int32_t)(tot < 0x7fffffff ? tot : 0x7fffffff);
        }
        if (tot == 0 && totw > 0) {
            __syncthreads();   // the ray walk reuses L
            ray_item(c, bin_start, brec, e, L, n_rec, err);
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
    const CutInst *insts;
    const int32_t *bin_start;
    const float4 *brec;         // bin records (k_bin_fill)
    const uint64_t *list_inbox;
    uint8_t *stat;              // k_hit takes ST_NEAR items and marks them ST_HIT or ST_SIDE
    CutCounters *cnt;
    int32_t *sidelist;          // the ST_SIDE items, appended by k_hit (count cnt->n_sidelist)
    double *side_u;             // per side-list entry: nearest node of the faces k_hit tested (bound U, or inf)
    int64_t bins_total;         // bins of the batch (bin_start[bins_total] = records)
    uint32_t *err;              // the context's check word (checked builds)
    int side_cap;               // faces a side-search wavefront lists (<= kSideList)
};

constexpr int kSideWaves = 8;        // wavefronts sharing one side item's walks (short lists)
constexpr int kSideGroups = 256;     // their workgroups: one per CU
constexpr int kSideGroupMax = 512;   // longest list taken that way (two rounds)
constexpr int kSideList = 64;        // faces a wavefront lists in the side search's second stage

// the faces (id and FP32 box) one wavefront of the side search finds within
// its item's bound, kept for the tie stage
struct SideList {
    int f[kSideList];
    float b[6][kSideList];
};

constexpr int kFaceCap = 64;    // one chunk of candidate faces
constexpr int kGroup = 8;   // candidate faces tested together by k_hit

// a4: one wavefront per near element decides whether the surface intersects
// it: some element-boundary / surface triangle pair closer than tol_hit
// (Alg. cp2, with no truncation of the candidate faces), or the whole surface
// inside the element.  Candidate faces that come within the element's
// boundary-face boxes are collected in LDS and taken in groups of 1, 2, 4,
// then kGroup faces (most intersected elements are decided by their first
// faces; the others must test them all): a group's nodes are loaded
// together, one lane builds each face triangle's box, the group's triangle
// pairs (384 per face) are screened by FP64 boxes and only the survivors get
// the exact test, one pair per lane; the element stops at the first group
// with a hit.
__global__ __launch_bounds__(64) void k_hit(ExactArgs a)
{
    __shared__ double sX[81];
    __shared__ double sTB[48 * 6];   // element triangle boxes
    __shared__ double sEF[6 * 6];    // element boundary-face boxes
    __shared__ double sF[kGroup * 27];       // nodes of the current group of faces
    __shared__ double sFT[kGroup * 8 * 6];   // their triangle boxes
    __shared__ int sList[kFaceCap];
    __shared__ short sPair[kGroup * 384];
    __shared__ WalkLds L;
    const int lane = threadIdx.x;
    const int n_in = a.cnt->n_inbox;
    const double tol = kTolHit;
    const int64_t n_rec = chk_size(a.bin_start + a.bins_total);
    for (int item = blockIdx.x; item < n_in; item += gridDim.x) {
        if (a.stat[item] != ST_NEAR) continue;
        const uint64_t it = a.list_inbox[item];
        const int ci = item_cut(it), e = item_elem(it);
        const CutInst &c = a.insts[ci];
        const BinGrid G = c.params->grid;
        const int32_t *bstart = a.bin_start + c.params->bin_off;
        const double *__restrict__ pnodes = c.pnodes;
        __syncthreads();
        for (int k = lane; k < 81; k += 64) sX[k] = c.enodes[(int64_t)e * 81 + k];
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
        for (int k = 0; k < 6; ++k) eb[k] = c.ebox[(int64_t)k * c.stride + e];
        int lo[3], hi[3];
        box_bins(G, eb, lo, hi);
        const BinRange R = make_range(lo, hi);
        bool hit = false;
        int nlist = 0;
        // nearest node of the faces tested to the element's first node: an
        // upper bound on its distance to the surface for the side search
        const double px = sX[0], py = sX[27], pz = sX[54];
        double u2 = INFINITY;
        // exact test of the listed faces
        int round = 0;   // group size 1, 2, 4 .. kGroup, kept across flushes
        auto flush = [&]() {
            int ng = 0;
            for (int i0 = 0; i0 < nlist && !hit; i0 += ng) {
                ng = min(1 << round, nlist - i0);
                if ((1 << round) < kGroup) ++round;
                for (int k = lane; k < 27 * ng; k += 64) {
                    const int g = k / 27;
                    sF[k] = pnodes[(int64_t)sList[i0 + g] * 27 + (k - 27 * g)];
                }
                __syncthreads();
                for (int k = lane; k < 9 * ng; k += 64) {
                    const double *F = sF + 27 * (k / 9);
                    const int q = k % 9;
                    const double dx = F[q] - px, dy = F[9 + q] - py, dz = F[18 + q] - pz;
                    u2 = fmin(u2, dx * dx + dy * dy + dz * dz);
                }
                if (lane < 8 * ng) {
                    d3 F[3];
                    face_tri(sF + 27 * (lane >> 3), lane & 7, F);
                    double *bb = sFT + 6 * lane;
                    bb[0] = fmin(F[0].x, fmin(F[1].x, F[2].x)); bb[3] = fmax(F[0].x, fmax(F[1].x, F[2].x));
                    bb[1] = fmin(F[0].y, fmin(F[1].y, F[2].y)); bb[4] = fmax(F[0].y, fmax(F[1].y, F[2].y));
                    bb[2] = fmin(F[0].z, fmin(F[1].z, F[2].z)); bb[5] = fmax(F[0].z, fmax(F[1].z, F[2].z));
                }
                __syncthreads();
                // screen the pairs p = 384 * group face + 48 * face triangle + element triangle
                int np = 0;
                for (int p0 = 0; p0 < 384 * ng; p0 += 64) {
                    const int p = p0 + lane;
                    bool pass = false;
                    if (p < 384 * ng) {
                        const int g = p / 384, r = p - 384 * g;
                        const int s = r / 48, t = r - 48 * s;
                        pass = boxes_within(sTB + 6 * t, sFT + 6 * (8 * g + s), tol);
                    }
                    const unsigned long long m = __ballot(pass);
                    if (pass) sPair[np + __popcll(m & ((1ull << lane) - 1ull))] = (short)p;
                    np += __popcll(m);
                }
                __syncthreads();
                bool lh = false;
                for (int q = lane; q < np && !lh; q += 64) {
                    const int p = sPair[q];
                    const int g = p / 384, r = p - 384 * g;
                    const int s = r / 48, t = r - 48 * s;
                    d3 T[3], F[3];
                    elem_tri(sX, t, T);
                    face_tri(sF + 27 * g, s, F);
                    lh = tri_tri_within(T, F, tol);
                }
                if (__ballot(lh)) hit = true;
                __syncthreads();
            }
            nlist = 0;
        };
        walk_faces(G, R, bstart, a.brec, L, [&](int f, const float *fb, const int *xyz) {
            bool pass = false;
            if (f >= 0) {
                if (first_common_bin(G, fb, xyz, lo) && box_overlap(eb, fb)) {
                    const double fd[6] = {fb[0], fb[1], fb[2], fb[3], fb[4], fb[5]};
                    for (int q = 0; q < 6; ++q) pass |= boxes_meet(sEF + 6 * q, fd);
                }
            }
            const unsigned long long m = __ballot(pass);
            if (pass) sList[nlist + __popcll(m & ((1ull << lane) - 1ull))] = f;
            nlist += __popcll(m);
            // test what this chunk found: an intersected element usually
            // stops here, before the rest of its bins are walked
            if (nlist > 0) {
                __syncthreads();
                flush();
            }
            return hit;
        }, 0, 1, n_rec, c.n_face, a.err);
        if (!hit && nlist > 0) {
            __syncthreads();
            flush();
        }
        // the whole surface inside the element: ray parity of its first node
        // against the element's 48 boundary triangles
        const d3 sf = pose_apply(*c.pose, mk(c.first[0], c.first[1], c.first[2]));
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
        if (!hit) u2 = wave_min_d(u2);
        if (lane == 0) {
            a.stat[item] = hit ? ST_HIT : ST_SIDE;
            if (hit && c.kind == OC_SURF_WALL) c.iblank[e] = OC_HOLE;
            if (!hit) {
                const int pos = atomicAdd(&a.cnt->n_sidelist, 1);
                a.sidelist[pos] = item;
                a.side_u[pos] = sqrt(u2);
            }
        }
    }
}

// a5: near elements that the surface does not intersect lie on one side of
// it; that side is the nearest-face side of the element's first node:
// minimum of the point-to-triangle distance over the binned faces, then the
// tie rule (largest |dot| of the unit point-to-surface vector with the
// outward triangle normal; normals averaged only for equally visible
// triangles of opposite sign).  Per element of the list k_hit leaves, three
// stages that meet in LDS: an upper bound U (the nearest node of the
// element's candidate faces), the nearest distance over the faces within U,
// and the two first records of the tie set in tie order, taken from the
// faces the second stage listed (a bin walk of its own only when a list
// overflowed).  In every walk each of the NW wavefronts takes every NW-th
// chunk of the stage's bins.  The stages compute a minimum over an exact set
// and the first two records of a total order, so neither the split among
// wavefronts nor the order of the listed faces changes any bit.
__device__ inline void side_item(const ExactArgs &a, int item, int &e, const CutInst *&cp, d3 &p)
{
    const uint64_t it = a.list_inbox[item];
    e = item_elem(it);
    cp = &a.insts[item_cut(it)];
    const double *X = cp->enodes + (int64_t)e * 81;
    p = mk(X[0], X[27], X[54]);
}

__device__ inline TieRec tie_shfl_xor(const TieRec &r, int d)
{
    TieRec o;
    o.absdot = __shfl_xor(r.absdot, d, 64);
    o.dot = __shfl_xor(r.dot, d, 64);
    o.vx = __shfl_xor(r.vx, d, 64);
    o.vy = __shfl_xor(r.vy, d, 64);
    o.vz = __shfl_xor(r.vz, d, 64);
    o.nx = __shfl_xor(r.nx, d, 64);
    o.ny = __shfl_xor(r.ny, d, 64);
    o.nz = __shfl_xor(r.nz, d, 64);
    o.f = __shfl_xor(r.f, d, 64);
    o.s = __shfl_xor(r.s, d, 64);
    o.valid = __shfl_xor(r.valid, d, 64);
    o.pad = 0;
    return o;
}

// the two first records of the wavefront in tie order, on every lane (the
// butterfly merges disjoint halves, so no record is offered twice)
__device__ inline void tie_wave_first2(TieRec &b1, TieRec &b2)
{
#pragma unroll 1
    for (int d = 32; d >= 1; d >>= 1) {
        const TieRec o1 = tie_shfl_xor(b1, d), o2 = tie_shfl_xor(b2, d);
        tie_offer(b1, b2, o1);
        tie_offer(b1, b2, o2);
    }
}

// The side items si0, si0 + sstep, ... of the list, NW wavefronts per item
// (kWave: one, synchronising only itself).  Wavefront `part` of the
// workgroup walks with WalkLds L[part], lists the faces of its share of the
// second stage in S[part] (over[part]: they did not fit) and reduces through
// red[part] and rec[2 part], rec[2 part + 1].
template <int NW, bool kWave>
__device__ inline void side_items(const ExactArgs &a, int n_side, WalkLds *L, double *red, TieRec *rec,
                                  SideList *S, int *over, int si0, int sstep)
{
    static_assert(!kWave || NW == 1, "a wavefront alone walks its item");
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int wp = kWave ? 0 : part;          // this wavefront's share of the item's walks
    const int r0 = kWave ? part : 0;          // first reduction slot of the item
    const int64_t n_rec = chk_size(a.bin_start + a.bins_total);
    for (int si = si0; si < n_side; si += sstep) {
        const int item = a.sidelist[si];
        int e;
        const CutInst *cp;
        d3 p;
        side_item(a, item, e, cp, p);
        const CutInst &c = *cp;
        const BinGrid G = c.params->grid;
        const int32_t *bstart = a.bin_start + c.params->bin_off;
        const double *__restrict__ pnodes = c.pnodes;
        // stage 1: upper bound, the nearest node of the element's candidate
        // faces (every face node lies on the surface; U only sizes stage 2).
        // k_hit leaves the nearest node of the faces it tested, a bound as
        // good for stage 2 (B, the minimum over every face within the bound,
        // does not depend on which bound); the walk runs only without it.
        const double u_hit = a.side_u[si];
        double u = u_hit;
        if (!(u_hit < INFINITY)) {
            float eb[6];
            for (int k = 0; k < 6; ++k) eb[k] = c.ebox[(int64_t)k * c.stride + e];
            int lo[3], hi[3];
            box_bins(G, eb, lo, hi);
            const BinRange R = make_range(lo, hi);
            walk_faces<kWave>(G, R, bstart, a.brec, L[part], [&](int f, const float *fb, const int *xyz) {
                if (f >= 0) {
                    if (first_common_bin(G, fb, xyz, lo) && box_overlap(eb, fb) && point_box_dist(p, fb) < u) {
                        const double *P = pnodes + (int64_t)f * 27;
                        double d2 = INFINITY;
                        for (int k = 0; k < 9; ++k) {
                            const double dx = P[k] - p.x, dy = P[9 + k] - p.y, dz = P[18 + k] - p.z;
                            d2 = fmin(d2, dx * dx + dy * dy + dz * dz);
                        }
                        u = fmin(u, sqrt(d2));
                    }
                }
                u = wave_min_d(u);
                return false;
            }, wp, NW, n_rec, c.n_face, a.err);
        }
        u = wave_min_d(u);
        if (lane == 0) red[part] = u;
        group_sync<kWave>();
        double U = red[r0];
        for (int k = 1; k < NW; ++k) U = fmin(U, red[r0 + k]);
        group_sync<kWave>();
        // stage 2: nearest distance over every face whose box is within U.
        // The walk covers the radius Uq a little beyond U, the largest radius
        // stage 3 can take, and each wavefront lists the faces whose boxes
        // are within Uq, so that stage 3 reads its faces from the lists
        // instead of walking the bins again (a face beyond U never lowers
        // the minimum, so the wider walk leaves B unchanged).
        const double Uq = U * (1.0 + 4e-9);
        double best = U;
        int nlist = 0;   // faces listed by this wavefront (the same on every lane)
        {
            int lo[3], hi[3];
            query_bins(G, p, Uq, lo, hi);
            const BinRange R = make_range(lo, hi);
            walk_faces<kWave>(G, R, bstart, a.brec, L[part], [&](int f, const float *fb, const int *xyz) {
                bool keep = false;
                if (f >= 0 && first_common_bin(G, fb, xyz, lo)) {
                    const double bd = point_box_dist(p, fb);
                    keep = bd <= Uq;
                    if (bd <= best) best = fmin(best, point_face_dist(p, pnodes + (int64_t)f * 27));
                }
                const unsigned long long m = __ballot(keep);
                if (keep) {
                    const int at = nlist + __popcll(m & ((1ull << lane) - 1ull));
                    if (at < a.side_cap) {
                        S[part].f[at] = f;
                        for (int k = 0; k < 6; ++k) S[part].b[k][at] = fb[k];
                    }
                }
                nlist += __popcll(m);
                best = wave_min_d(best);
                return false;
            }, wp, NW, n_rec, c.n_face, a.err);
        }
        best = wave_min_d(best);
        if (lane == 0) {
            red[part] = best;
            over[part] = nlist > a.side_cap;
        }
        group_sync<kWave>();
        double B = red[r0];
        bool from_lists = !over[r0];
        for (int k = 1; k < NW; ++k) {
            B = fmin(B, red[r0 + k]);
            from_lists = from_lists && !over[r0 + k];
        }
        // stage 3: tie set within B * (1 + 1e-9)
        const double thr = B * (1.0 + 1e-9);
        TieRec b1, b2;
        b1.valid = b2.valid = 0;
        auto tie_face = [&](int f) {
            const double *P = pnodes + (int64_t)f * 27;
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
        };
        if (from_lists) {
            if (lane < nlist) {
                float fb[6];
                for (int k = 0; k < 6; ++k) fb[k] = S[part].b[k][lane];
                if (point_box_dist(p, fb) <= thr) tie_face(S[part].f[lane]);
            }
        } else {
            int lo[3], hi[3];
            query_bins(G, p, thr, lo, hi);
            const BinRange R = make_range(lo, hi);
            walk_faces<kWave>(G, R, bstart, a.brec, L[part], [&](int f, const float *fb, const int *xyz) {
                if (f >= 0) {
                    if (first_common_bin(G, fb, xyz, lo) && point_box_dist(p, fb) <= thr) tie_face(f);
                }
                return false;
            }, wp, NW, n_rec, c.n_face, a.err);
        }
        tie_wave_first2(b1, b2);
        if (lane == 0) {
            rec[2 * part] = b1;
            rec[2 * part + 1] = b2;
        }
        group_sync<kWave>();
        if (lane == 0 && part == r0) {
            TieRec c1, c2;
            c1.valid = c2.valid = 0;
            for (int k = 0; k < 2 * NW; ++k) tie_offer(c1, c2, rec[2 * r0 + k]);
            double sg = c1.dot;
            if (c2.valid && c1.absdot - c2.absdot <= 1e-9 && ((c1.dot > 0.0) != (c2.dot > 0.0)))
                sg = c1.vx * (c1.nx + c2.nx) + c1.vy * (c1.ny + c2.ny) + c1.vz * (c1.nz + c2.nz);
            if (c1.valid && sg < 0.0) c.iblank[e] = OC_HOLE;
        }
        group_sync<kWave>();
    }
}

// a5: the side list, in one launch whatever its length (known only on the
// device): up to kSideGroupMax items the kSideWaves wavefronts of a
// workgroup share each item (the latency of a few items), beyond that each
// wavefront takes its own items (throughput when there are many).
__global__ __launch_bounds__(64 * kSideWaves) void k_side(ExactArgs a)
{
    __shared__ WalkLds L[kSideWaves];
    __shared__ double red[kSideWaves];
    __shared__ TieRec rec[2 * kSideWaves];
    __shared__ SideList S[kSideWaves];
    __shared__ int over[kSideWaves];
    const int n_side = a.cnt->n_sidelist;
    if (n_side <= kSideGroupMax)
        side_items<kSideWaves, false>(a, n_side, L, red, rec, S, over, blockIdx.x, gridDim.x);
    else
        side_items<1, true>(a, n_side, L, red, rec, S, over, blockIdx.x * kSideWaves + (threadIdx.x >> 6),
                            gridDim.x * kSideWaves);
}

// a8: fringe layer (field elements sharing a face with a hole).  Every hole
// is an in-box item of some cut of its output, so the scatter runs over the
// in-box items that ended up holes.
__global__ __launch_bounds__(kThreads) void k_fringe(const CutInst *__restrict__ I,
                                                     const uint64_t *__restrict__ list_inbox,
                                                     const CutCounters *__restrict__ cnt)
{
    const int n = cnt->n_inbox;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint64_t it = list_inbox[i];
        const int e = item_elem(it);
        const CutInst &c = I[item_cut(it)];
        int8_t *iblank = c.iblank;
        const int32_t *nbr = c.nbr;
        if (!nbr || iblank[e] != OC_HOLE) continue;   // no neighbours: loose elements
        for (int f = 0; f < 6; ++f) {
            const int q = nbr[(int64_t)e * 6 + f];
            if (q >= 0 && iblank[q] != OC_HOLE) iblank[q] = OC_FRINGE;
        }
    }
}

// Statistics of the last batch (only when asked for): item statuses,
// candidate pairs, and the holes of every output.
__global__ __launch_bounds__(kThreads) void k_cut_stats(const uint8_t *__restrict__ stat,
                                                        const int32_t *__restrict__ ncand, CutCounters *cnt)
{
    __shared__ unsigned long long acc[5];
    if (threadIdx.x < 5) acc[threadIdx.x] = 0ull;
    __syncthreads();
    const int n = cnt->n_inbox;
    unsigned long long h = 0, sd = 0, fr = 0, cp = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint8_t s = stat[i];
        h += s == ST_HIT;
        sd += s == ST_SIDE;
        fr += s == ST_FAR;
        if (s == ST_HIT || s == ST_SIDE) cp += (unsigned long long)ncand[i];
    }
    atomicAdd(&acc[0], h);
    atomicAdd(&acc[1], sd);
    atomicAdd(&acc[2], fr);
    atomicAdd(&acc[3], cp);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&cnt->n_hit, (int)acc[0]);
        atomicAdd(&cnt->n_side, (int)acc[1]);
        atomicAdd(&cnt->n_near, (int)(acc[0] + acc[1]));
        atomicAdd(&cnt->n_far, (int)acc[2]);
        atomicAdd(&cnt->n_cand_pairs, acc[3]);
    }
}

__global__ __launch_bounds__(kThreads) void k_count_holes(const CutOut *__restrict__ O, int n_out, CutCounters *cnt)
{
    const int oi = block_owner(n_out, blockIdx.x, [&](int k) { return O[k].cblk0; });
    const CutOut &o = O[oi];
    const int64_t e = (int64_t)(blockIdx.x - o.cblk0) * blockDim.x + threadIdx.x;
    const int h = __syncthreads_count(e < o.n_elem && o.iblank[e] == OC_HOLE);
    if (threadIdx.x == 0 && h) atomicAdd(&cnt->n_hole, h);
}

__global__ void k_stats_reset(CutCounters *cnt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cnt->n_near = cnt->n_far = cnt->n_hit = cnt->n_hole = cnt->n_side = 0;
        cnt->n_cand_pairs = 0ull;
    }
}

// outputs with no cutting surface: every element field (blocks flattened
// over those outputs, kThreads elements per block)
// (a batch of one output passes it by value: O null; block 0 stores it at
// dst for the later stages)
__global__ __launch_bounds__(kThreads) void k_fill_field(const CutOut *__restrict__ O, int n_out, CutOut one,
                                                         CutOut *dst)
{
    int8_t *iblank;
    int64_t n_elem;
    int fblk0;
    if (!O) {
        if (dst && blockIdx.x == 0 && threadIdx.x == 0) *dst = one;
        iblank = one.iblank;
        n_elem = one.n_elem;
        fblk0 = one.fblk0;
    } else {
        const CutOut &o = O[block_owner(n_out, blockIdx.x, [&](int k) { return O[k].fblk0; })];
        iblank = o.iblank;
        n_elem = o.n_elem;
        fblk0 = o.fblk0;
    }
    const int64_t e = (int64_t)(blockIdx.x - fblk0) * blockDim.x + threadIdx.x;
    if (e < n_elem) iblank[e] = OC_FIELD;
}

// elements carrying an overset-tagged face are fringe unless hole (blocks
// flattened over the outputs' overset lists)
__global__ __launch_bounds__(kThreads) void k_overset_fringe(const CutOut *__restrict__ O, int n_out, CutOut one)
{
    int8_t *iblank;
    const int32_t *overset;
    int64_t n_overset;
    int oblk0;
    if (!O) {
        iblank = one.iblank;
        overset = one.overset;
        n_overset = one.n_overset;
        oblk0 = one.oblk0;
    } else {
        const CutOut &o = O[block_owner(n_out, blockIdx.x, [&](int k) { return O[k].oblk0; })];
        iblank = o.iblank;
        overset = o.overset;
        n_overset = o.n_overset;
        oblk0 = o.oblk0;
    }
    const int64_t i = (int64_t)(blockIdx.x - oblk0) * blockDim.x + threadIdx.x;
    if (i < n_overset) {
        const int e = overset[i];
        if (iblank[e] != OC_HOLE) iblank[e] = OC_FRINGE;
    }
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

static int64_t blocks_of(int64_t n, int64_t per_block) { return (n + per_block - 1) / per_block; }

CutCaps cut_caps(const CutReq *reqs, int n)
{
    CutCaps c;
    for (int r = 0; r < n; ++r) {
        const CutReq &q = reqs[r];
        c.outs += 1;
        for (int k = 0; k < q.n_surf; ++k) {
            const Surf &s = *q.surfs[k];
            c.elem_inst += q.g->n_elem;
            c.faces += s.n_face;
            c.bins += (int64_t)s.nb_max * s.nb_max * s.nb_max;
            c.cuts += 1;
        }
    }
    return c;
}

// Host bytes travel to the device as kernel arguments, in stream order: the
// copy is captured by graph capture like any launch and the host array may
// be reused as soon as the call returns.
struct BytePack {
    unsigned char b[2048];
    int n;
    int pad;
};

__global__ void k_put_bytes(unsigned char *dst, BytePack pk)
{
    for (int i = threadIdx.x; i < pk.n; i += blockDim.x) dst[i] = pk.b[i];
}

oc_status put_bytes(oc_slot *sl, void *dst, const void *src, size_t n)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    const unsigned char *p = static_cast<const unsigned char *>(src);
    for (size_t k0 = 0; k0 < n; k0 += sizeof(BytePack::b)) {
        BytePack pk;
        pk.n = (int)std::min(sizeof pk.b, n - k0);
        pk.pad = 0;
        memcpy(pk.b, p + k0, (size_t)pk.n);
        LAUNCH(k_put_bytes, dim3(1), dim3(256), static_cast<unsigned char *>(dst) + k0, pk);
    }
    OC_HIP(hipGetLastError());
    return OC_OK;
}

// Device poses of surfaces in a grid's frame: out[k] = inverse(grid) after
// surfs[k] (R = Rg^T Rs, t = Rg^T ts - Rg^T tg), one thread per pose.
__global__ void k_compose_poses(const double *__restrict__ grid, const double *__restrict__ surfs, int n,
                                Pose *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double *G = grid, *S = surfs + 12 * k;
    Pose P;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) P.r[3 * i + j] = G[i] * S[j] + G[3 + i] * S[3 + j] + G[6 + i] * S[6 + j];
        const double a = G[i] * S[9] + G[3 + i] * S[10] + G[6 + i] * S[11];
        const double b = G[i] * G[9] + G[3 + i] * G[10] + G[6 + i] * G[11];
        P.t[i] = a - b;
    }
    out[k] = P;
}

oc_status compose_poses_run(oc_slot *sl, const double *grid_dev, const double *surfs_dev, int n, Pose *out)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    if (n <= 0) return OC_OK;
    LAUNCH(k_compose_poses, dim3((unsigned)((n + 63) / 64)), dim3(64), grid_dev, surfs_dev, n, out);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

// Host poses into the slot's device pose slots.
oc_status set_poses(oc_slot *sl, int first, const double *host, int n)
{
    if (first < 0 || n < 0 || first + n > kPoseSlots) {
        set_error("too many poses");
        return OC_EINVAL;
    }
    if (n == 0) return OC_OK;
    std::vector<Pose> P((size_t)n);
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < 9; ++i) P[k].r[i] = host[12 * k + i];
        for (int i = 0; i < 3; ++i) P[k].t[i] = host[12 * k + 9 + i];
    }
    return put_bytes(sl, sl->poses + first, P.data(), sizeof(Pose) * (size_t)n);
}

// Every request's cuts run together, one launch per stage: launches over
// faces or elements are flattened over the cuts (each block finds its cut
// from the cuts' first blocks), the later stages take (cut, element) items
// from batch-wide lists, so instances of very different sizes share the
// device without one launch sequence per instance.
oc_status cut_batch_run(oc_slot *sl, const CutReq *reqs, int n_req)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    const CutCaps need = cut_caps(reqs, n_req);
    // refused before anything is launched: a scan that failed after
    // k_bin_count would leave counts behind that the next cut would build on
    OC_TRY(cut_caps_check(need));
    OC_TRY(slot_reserve_cut(sl, need));
    for (int r = 0; r < n_req; ++r) {
        if (reqs[r].prev && reqs[r].n_surf != 1) {
            set_error("warm start needs exactly one cutting surface");
            return OC_EINVAL;
        }
        for (int q = 0; q < r; ++q)
            if (reqs[q].iblank == reqs[r].iblank) {
                set_error("two requests of one batch write the same iblank");
                return OC_EINVAL;
            }
    }
    std::vector<CutInst> I;
    std::vector<CutOut> O;
    int64_t fblk = 0, pblk = 0, eblk = 0, face_off = 0, fill_blk = 0, ov_blk = 0, cnt_blk = 0, n_elem_total = 0;
    int64_t bin_off = 0;
    for (int r = 0; r < n_req; ++r) {
        const CutReq &q = reqs[r];
        const Grid &g = *q.g;
        CutOut o{};
        o.iblank = q.iblank;
        o.overset = g.overset;
        o.n_elem = g.n_elem;
        o.n_overset = g.n_overset;
        o.fblk0 = (int)fill_blk;
        o.oblk0 = (int)ov_blk;
        o.cblk0 = (int)cnt_blk;
        o.pad = 0;
        cnt_blk += blocks_of(g.n_elem, kThreads);
        if (q.n_surf == 0) fill_blk += blocks_of(g.n_elem, kThreads);
        ov_blk += blocks_of(g.n_overset, kThreads);
        O.push_back(o);
        n_elem_total += g.n_elem;
        for (int k = 0; k < q.n_surf; ++k) {
            const Surf &s = *q.surfs[k];
            CutInst c{};
            c.enodes = g.enodes;
            c.ebox = g.ebox;
            c.wbox = g.wbox;
            c.nbr = g.nbr;
            c.snodes = s.nodes;
            c.conn = s.conn;
            c.pose = q.poses + k;
            c.pnodes = sl->pnodes + 27 * face_off;
            c.fbox = sl->fbox + 6 * face_off;
            c.params = sl->params + I.size();
            c.iblank = q.iblank;
            c.prev = q.prev;
            c.sweep = q.sweep;
            c.stride = g.ebox_stride;
            c.n_elem = g.n_elem;
            c.n_nodes = s.n_nodes;
            c.n_face = s.n_face;
            for (int d = 0; d < 3; ++d) c.first[d] = s.first[d];
            c.dmax = s.dmax;
            c.nb_max = s.nb_max;
            c.kind = s.kind;
            c.write_field = k == 0;
            c.fblk0 = (int)fblk;
            c.pblk0 = (int)pblk;
            c.bin_off0 = (int)bin_off;
            c.eblk0 = (int)eblk;
            bin_off += (int64_t)s.nb_max * s.nb_max * s.nb_max;
            fblk += blocks_of(s.n_face, kThreads);
            pblk += blocks_of(s.n_face, kPoseFaces);
            eblk += blocks_of(g.n_elem, (int64_t)ctx->filter_block * 4);
            face_off += s.n_face;
            I.push_back(c);
        }
    }
    if (fblk >= INT32_MAX || pblk >= INT32_MAX || eblk >= INT32_MAX || fill_blk >= INT32_MAX || ov_blk >= INT32_MAX ||
        need.elem_inst >= INT32_MAX || cnt_blk >= INT32_MAX) {
        set_error("cut batch too large");
        return OC_EINVAL;
    }
    sl->last_n_elem = n_elem_total;
    const int n_cut = (int)I.size(), n_out = (int)O.size();
    sl->last_n_cut = n_cut;
    sl->last_n_out = n_out;
    sl->last_cblk = (int)cnt_blk;
    sl->last_outs = O;
    // one cut / one output: the descriptor travels by value in the first
    // kernel that reads it (which stores it for the others)
    const bool one_cut = n_cut == 1, one_out = n_out == 1;
    if (n_cut && !one_cut) OC_TRY(put_bytes(sl, sl->insts, I.data(), sizeof(CutInst) * I.size()));
    if ((fill_blk || ov_blk) && !one_out) OC_TRY(put_bytes(sl, sl->outs, O.data(), sizeof(CutOut) * O.size()));
    const CutOut o1 = one_out ? O[0] : CutOut{};
    if (fill_blk)
        LAUNCH(k_fill_field, dim3((unsigned)fill_blk), dim3(kThreads), one_out ? nullptr : sl->outs, n_out, o1,
               one_out ? sl->outs : nullptr);
    if (n_cut) {
        LAUNCH(k_pose_faces, dim3((unsigned)pblk), dim3(kThreads), sl->insts, n_cut, sl->sbox_part,
               one_cut ? I[0] : CutInst{}, one_cut ? sl->insts : nullptr);
        // the bin counts are zero here: zeroed when the slot's arrays were
        // made, and k_bin_fill takes every count back to zero
        LAUNCH(k_bin_count, dim3((unsigned)fblk), dim3(kThreads), sl->insts, n_cut, sl->sbox_part, sl->bin_count,
               sl->counters);
        OC_TRY(scan_exclusive(ctx, st, sl->bin_count, sl->bin_start, bin_off, nullptr, sl->bin_scan_tmp));
        LAUNCH(k_bin_fill, dim3((unsigned)fblk), dim3(kThreads), sl->insts, n_cut, sl->bin_start, sl->bin_count,
               sl->bin_rec);
        LAUNCH(k_filter, dim3((unsigned)eblk), dim3((unsigned)ctx->filter_block), sl->insts, n_cut,
               one_cut ? I[0] : CutInst{}, (int)one_cut, sl->l_inbox,
               sl->counters);
        uint32_t *err = reinterpret_cast<uint32_t *>(ctx->dev_scalar) + 8;
        LAUNCH(k_candidates, dim3((unsigned)ctx->exact_waves), dim3(64), sl->insts, sl->bin_start, sl->bin_rec,
               sl->l_inbox, sl->l_stat, sl->l_ncand, sl->counters, bin_off, err);
        ExactArgs ea;
        ea.insts = sl->insts;
        ea.bin_start = sl->bin_start;
        ea.brec = sl->bin_rec;
        ea.list_inbox = sl->l_inbox;
        ea.stat = sl->l_stat;
        ea.cnt = sl->counters;
        ea.sidelist = sl->l_sidelist;
        ea.side_u = sl->l_sideu;
        ea.bins_total = bin_off;
        ea.err = err;
        ea.side_cap = std::min(ctx->side_list, kSideList);
        LAUNCH(k_hit, dim3((unsigned)ctx->exact_waves), dim3(64), ea);
        LAUNCH(k_side, dim3((unsigned)kSideGroups), dim3(64 * kSideWaves), ea);
        LAUNCH(k_fringe, dim3(1024), dim3(kThreads), sl->insts, sl->l_inbox, sl->counters);
    }
    if (ov_blk)
        LAUNCH(k_overset_fringe, dim3((unsigned)ov_blk), dim3(kThreads), one_out ? nullptr : sl->outs, n_out, o1);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

// Counters of the slot's last cut batch (on the slot stream; the caller
// reads them back).
oc_status cut_stats_run(oc_slot *sl)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    LAUNCH(k_stats_reset, dim3(1), dim3(64), sl->counters);
    if (sl->last_n_cut > 0)
        LAUNCH(k_cut_stats, dim3(256), dim3(kThreads), sl->l_stat, sl->l_ncand, sl->counters);
    if (sl->last_cblk > 0) {
        OC_TRY(put_bytes(sl, sl->outs, sl->last_outs.data(), sizeof(CutOut) * sl->last_outs.size()));
        LAUNCH(k_count_holes, dim3((unsigned)sl->last_cblk), dim3(kThreads), sl->outs, sl->last_n_out, sl->counters);
    }
    OC_HIP(hipGetLastError());
    return OC_OK;
}

}  // namespace oc
