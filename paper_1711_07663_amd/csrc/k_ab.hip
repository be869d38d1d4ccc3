// Artificial-boundary (AB) method of Sec. 2: the faces that separate kept
// cells from holes (plus the overset-tagged faces of a near-body grid), the
// flux points on them (the AB method's receptor points), and the Lagrange
// weights that query a donor's solution polynomial at each receptor's
// reference location.
//
//   k_ab_mark          every hole sets, in a per-element byte mask, the bit
//                      of its kept neighbours' face towards it (holes are
//                      few: the scatter reads their neighbour rows only)
//   k_ab_count / scan / k_ab_write
//                      ordered compaction of the set bits (and the overset
//                      bits of kept cells) into face ids 6 e + f; the write
//                      clears the mask, so it is zero between calls
//   k_face_points      m x m points per face mapped by eq. reftophys, posed
//   k_interp_weights   m^3 weights per receptor, one per thread (coalesced)
#include <algorithm>
#include <cmath>

#include "dev_common.h"
#include "q2.h"

namespace oc {

constexpr int kAT = 256;
constexpr int kAbItems = 16;
constexpr int kAbTile = kAT * kAbItems;
static_assert(kAbTile == 4096, "the slot's tile scratch is sized for 4096-element tiles");

__global__ __launch_bounds__(kAT) void k_ab_mark(const int8_t *__restrict__ ib, const int32_t *__restrict__ nbr,
                                                 int64_t n, uint32_t *__restrict__ mask)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (ib[e] != OC_HOLE) continue;
        for (int f = 0; f < 6; ++f) {
            const int q = nbr[e * 6 + f];
            if (q < 0 || ib[q] == OC_HOLE) continue;
            for (int g = 0; g < 6; ++g)
                if (nbr[(int64_t)q * 6 + g] == (int32_t)e) atomicOr(&mask[q >> 2], 1u << (8 * (q & 3) + g));
        }
    }
}

__device__ inline unsigned ab_bits(const uint8_t *__restrict__ m8, const int8_t *__restrict__ ib,
                                   const uint8_t *__restrict__ ov, int64_t e)
{
    unsigned b = m8[e];
    if (ov && ib[e] != OC_HOLE) b |= ov[e];
    return b;
}

__global__ __launch_bounds__(kAT) void k_ab_count(const uint8_t *__restrict__ m8, const int8_t *__restrict__ ib,
                                                  const uint8_t *__restrict__ ov, int64_t n,
                                                  int32_t *__restrict__ tcount)
{
    const int64_t base = (int64_t)blockIdx.x * kAbTile;
    int c = 0;
    for (int k = 0; k < kAbItems; ++k) {
        const int64_t e = base + (int64_t)k * kAT + threadIdx.x;
        if (e < n) c += __popc(ab_bits(m8, ib, ov, e));
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    __shared__ int ws[kAT / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kAT / 64; ++w) s += ws[w];
        tcount[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kAT) void k_ab_write(uint8_t *__restrict__ m8, const int8_t *__restrict__ ib,
                                                  const uint8_t *__restrict__ ov, int64_t n,
                                                  const int32_t *__restrict__ toff, int32_t *__restrict__ faces,
                                                  int64_t cap)
{
    const int64_t my = (int64_t)blockIdx.x * kAbTile + (int64_t)threadIdx.x * kAbItems;
    int c = 0;
    for (int k = 0; k < kAbItems; ++k)
        if (my + k < n) c += __popc(ab_bits(m8, ib, ov, my + k));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    __shared__ int ws[kAT / 64];
    if (lane == 63) ws[wid] = inc;
    __syncthreads();
    int pos = toff[blockIdx.x];
    for (int w = 0; w < wid; ++w) pos += ws[w];
    pos += inc - c;
    for (int k = 0; k < kAbItems; ++k) {
        const int64_t e = my + k;
        if (e >= n) break;
        const unsigned b = ab_bits(m8, ib, ov, e);
        for (int f = 0; f < 6; ++f)
            if (b & (1u << f)) {
                if (pos < cap) faces[pos] = (int32_t)(6 * e + f);
                ++pos;
            }
        if (m8[e]) m8[e] = 0;
    }
}

// Flux point q = a + m b of face id = 6 e + f: the face's own reference axis
// d = f / 2 at -1 (even f) or +1 (odd f); the other two axes, in increasing
// order, at z[a] and z[b].  An id outside [0, 6 n_elem) gives NaN, source -1.
__global__ __launch_bounds__(kAT) void k_face_points(const double *__restrict__ enodes, int64_t n_elem,
                                                     const int32_t *__restrict__ faces,
                                                     const int32_t *__restrict__ n_faces, int64_t faces_cap,
                                                     Nodes1D z, const Pose *__restrict__ pose_dev, int64_t cap,
                                                     double *__restrict__ pts, int32_t *__restrict__ src,
                                                     int32_t *__restrict__ n_out)
{
    const int m = z.m, mm = m * m;
    const int64_t nf = n_faces ? min((int64_t)*n_faces, faces_cap) : faces_cap;
    const int64_t total = nf * mm;
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_out) *n_out = (int32_t)total;
    const int64_t n = total < cap ? total : cap;
    const Pose pose = *pose_dev;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i / mm;
        const int q = (int)(i - j * mm);
        const int id = faces[j];
        if (id < 0 || (int64_t)id >= 6 * n_elem) {
            const double nan = __builtin_nan("");
            pts[3 * i] = nan;
            pts[3 * i + 1] = nan;
            pts[3 * i + 2] = nan;
            if (src) src[i] = -1;
            continue;
        }
        const int e = id / 6, f = id - 6 * e, d = f >> 1;
        const int u = d == 0 ? 1 : 0, v = d == 2 ? 1 : 2;
        double xi[3];
        xi[d] = (f & 1) ? 1.0 : -1.0;
        xi[u] = z.z[q % m];
        xi[v] = z.z[q / m];
        double x[3];
        q2_map<false, true>(enodes + (int64_t)e * 81, xi, x, nullptr);
        const d3 w = pose_apply(pose, mk(x[0], x[1], x[2]));
        pts[3 * i] = w.x;
        pts[3 * i + 1] = w.y;
        pts[3 * i + 2] = w.z;
        if (src) src[i] = id;
    }
}

// l_a(s) = prod_{j != a} (s - z_j) / (z_a - z_j), factors taken in j order
__device__ inline double lagrange(const Nodes1D &z, int a, double s)
{
    double l = 1.0;
    for (int j = 0; j < z.m; ++j)
        if (j != a) l *= (s - z.z[j]) / (z.z[a] - z.z[j]);
    return l;
}

// weight k = a + m b + m^2 c of receptor i: (l_a(xi) l_b(eta)) l_c(zeta).
// A block takes weight_receptors(m) receptors at a time: their 3m basis
// values go to LDS first (each computed once, two divisions at m = 3, not
// per weight), then the block writes their weights in order, one per
// thread.  The values and the products are those of the per-weight form.
constexpr int kWBasis = 3 * kAT;   // basis values staged per round (3m per receptor)
constexpr int kWRec = kAT;         // receptors per round, at most

// receptors per round: about four weights per thread, within the LDS
__host__ __device__ inline int weight_receptors(int m)
{
    const int m3 = m * m * m;
    int r = (4 * kAT) / m3;
    if (r > kWBasis / (3 * m)) r = kWBasis / (3 * m);
    if (r > kWRec) r = kWRec;
    return r < 1 ? 1 : r;
}

__global__ __launch_bounds__(kAT) void k_interp_weights(const int32_t *__restrict__ donors,
                                                        const double *__restrict__ ref,
                                                        const int32_t *__restrict__ n_dev, int64_t cap, Nodes1D z,
                                                        double *__restrict__ w)
{
    __shared__ double sb[kWBasis];
    __shared__ int sok[kWRec];
    const int m = z.m, m3 = m * m * m;
    const int rec = weight_receptors(m);
    const int64_t n = n_dev ? min((int64_t)*n_dev, cap) : cap;
    for (int64_t i0 = (int64_t)blockIdx.x * rec; i0 < n; i0 += (int64_t)gridDim.x * rec) {
        const int nr = (int)min((int64_t)rec, n - i0);
        for (int v = threadIdx.x; v < nr * 3 * m; v += blockDim.x) {
            const int r = v / (3 * m), q = v - r * 3 * m, d = q / m, a = q - d * m;
            sb[v] = lagrange(z, a, ref[3 * (i0 + r) + d]);
        }
        for (int r = threadIdx.x; r < nr; r += blockDim.x) sok[r] = donors[i0 + r] >= 0;
        __syncthreads();
        for (int t = threadIdx.x; t < nr * m3; t += blockDim.x) {
            const int r = t / m3, k = t - r * m3;
            const int a = k % m, b = (k / m) % m, c = k / (m * m);
            const double *L = sb + r * 3 * m;
            w[i0 * m3 + t] = sok[r] ? (L[a] * L[m + b]) * L[2 * m + c] : __builtin_nan("");
        }
        __syncthreads();
    }
}

#define LAUNCH(name, grid, block, ...)                                                       \
    do {                                                                                     \
        size_t slot_;                                                                        \
        time_begin(ctx, st, #name, &slot_);                                                  \
        hipLaunchKernelGGL(name, grid, block, 0, st, __VA_ARGS__);                           \
        time_end(ctx, st, slot_);                                                            \
    } while (0)

static unsigned ab_blocks(int64_t n)
{
    const int64_t b = (n + kAT - 1) / kAT;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

oc_status ab_faces_run(oc_slot *sl, const Grid &g, const int8_t *iblank, int32_t *faces, int64_t cap,
                       const int32_t **total)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    OC_TRY(slot_reserve_grid(sl, g));
    const int64_t nt = (g.n_elem + kAbTile - 1) / kAbTile;
    int32_t *tcount = sl->fr_tiles, *toff = sl->fr_tiles + (nt + 1);
    int32_t *tmp = sl->fr_tiles + 2 * (nt + 1);
    uint8_t *m8 = reinterpret_cast<uint8_t *>(sl->ab_mask);
    // sizes the scan refuses are refused before the mask is marked: k_ab_write
    // is what takes the mask back to zero, so nothing may fail in between
    if (nt > scan_max_items()) {
        set_error("ab faces: grid too large for the tile scan");
        return OC_EINVAL;
    }
    LAUNCH(k_ab_mark, dim3(ab_blocks(g.n_elem)), dim3(kAT), iblank, g.nbr, g.n_elem, sl->ab_mask);
    LAUNCH(k_ab_count, dim3((unsigned)std::max<int64_t>(nt, 1)), dim3(kAT), m8, iblank, g.ovmask, g.n_elem, tcount);
    OC_TRY(scan_exclusive(ctx, st, tcount, toff, nt, nullptr, tmp));
    LAUNCH(k_ab_write, dim3((unsigned)std::max<int64_t>(nt, 1)), dim3(kAT), m8, iblank, g.ovmask, g.n_elem, toff,
           faces, cap);
    OC_HIP(hipGetLastError());
    *total = toff + nt;
    return OC_OK;
}

oc_status face_points_run(oc_slot *sl, const Grid &g, const Pose *pose_dev, const int32_t *faces,
                          const int32_t *n_faces, int64_t faces_cap, const Nodes1D &z, double *pts, int64_t cap,
                          int32_t *n_out, int32_t *src)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    const int64_t work = std::min<int64_t>(cap, faces_cap * z.m * z.m);
    LAUNCH(k_face_points, dim3(ab_blocks(std::max<int64_t>(work, 1))), dim3(kAT), g.enodes, g.n_elem, faces, n_faces,
           faces_cap, z, pose_dev, cap, pts, src, n_out);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status weights_run(oc_slot *sl, const int32_t *donors, const double *ref, const int32_t *n_dev, int64_t cap,
                      const Nodes1D &z, double *w)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    const int64_t rec = weight_receptors(z.m);
    const int64_t blk = std::max<int64_t>(1, std::min<int64_t>((cap + rec - 1) / rec, 4096));
    LAUNCH(k_interp_weights, dim3((unsigned)blk), dim3(kAT), donors, ref, n_dev, cap, z, w);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

}  // namespace oc
