// Blanking of a moving grid's time step with unblanking (Sec. 3, Alg.
// unblank): the grid is cut at the poses of time t and of t + dt, the two
// hole sets are combined by the rule of the cutting surfaces' kind, one
// fringe layer is marked around the combined holes, and the holes of the
// previous blanking that are holes no more are listed (ascending) as the
// cells to unblank.  Their interior points and donors then come from the
// receptor-point and donor-search calls.
//
// Wall surfaces: a hole at t or at t + dt (a cell that becomes a hole is a
// hole now).  That union is what one cut by every surface at both poses
// computes (Sec. 4.2 takes the union over cutting surfaces), fringe layer
// and overset tags included, so the wall rule is that one cut.
// Overset surfaces: a hole at t and at t + dt (cells stay until known to be
// unneeded): two cuts in one batch, then
//   k_unblank_combine   hole where both cuts have one, else field
//   k_fringe_stencil    field cells with a hole face neighbour become fringe
//   k_overset_list      cells with an overset-tagged face are fringe unless hole
#include <algorithm>
#include <string>
#include <vector>

#include "dev_common.h"

namespace oc {

constexpr int kUT = 256;

__global__ __launch_bounds__(kUT) void k_unblank_combine(const int8_t *__restrict__ a, const int8_t *__restrict__ b,
                                                         int64_t n, int8_t *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (a[e] == OC_HOLE && b[e] == OC_HOLE) ? OC_HOLE : OC_FIELD;
}

// reads only hole marks, which no thread changes here
__global__ __launch_bounds__(kUT) void k_fringe_stencil(const int32_t *__restrict__ nbr, int64_t n, int8_t *out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (out[e] == OC_HOLE) continue;
        bool near = false;
        for (int f = 0; f < 6; ++f) {
            const int q = nbr[e * 6 + f];
            near |= q >= 0 && out[q] == OC_HOLE;
        }
        if (near) out[e] = OC_FRINGE;
    }
}

__global__ __launch_bounds__(kUT) void k_overset_list(const int32_t *__restrict__ list, int64_t n, int8_t *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int e = list[i];
        if (out[e] != OC_HOLE) out[e] = OC_FRINGE;
    }
}

__global__ void k_copy_i32(const int32_t *src, int32_t *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

#define LAUNCH(name, grid, block, ...)                                                       \
    do {                                                                                     \
        size_t slot_;                                                                        \
        time_begin(ctx, st, #name, &slot_);                                                  \
        hipLaunchKernelGGL(name, grid, block, 0, st, __VA_ARGS__);                           \
        time_end(ctx, st, slot_);                                                            \
    } while (0)

static unsigned ublocks(int64_t n)
{
    const int64_t b = (n + kUT - 1) / kUT;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

// overset rule: cuts at t and t + dt into the slot's two scratch arrays,
// holes where both agree, fringe layer, overset-tagged faces
static oc_status combine_overset(oc_slot *sl, Grid &g, Surf *const *surfs, int n_surf, const Pose *poses_t,
                                 const Pose *poses_tp, int8_t *out)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    if (g.n_elem > sl->ub_cap) {
        if (!sl->grow) {
            set_error("slot was not created for unblanking this grid");
            return OC_EINVAL;
        }
        OC_HIP(hipStreamSynchronize(st));
        OC_TRY(dev_alloc(ctx, sl->owned, (size_t)g.n_elem, (void **)&sl->ub_a));
        OC_TRY(dev_alloc(ctx, sl->owned, (size_t)g.n_elem, (void **)&sl->ub_b));
        sl->ub_cap = g.n_elem;
    }
    CutReq q[2];
    for (int r = 0; r < 2; ++r) {
        q[r].g = &g;
        q[r].n_surf = n_surf;
        q[r].surfs = surfs;
        q[r].poses = r == 0 ? poses_t : poses_tp;
        q[r].iblank = r == 0 ? sl->ub_a : sl->ub_b;
    }
    OC_TRY(cut_batch_run(sl, q, 2));
    LAUNCH(k_unblank_combine, dim3(ublocks(g.n_elem)), dim3(kUT), sl->ub_a, sl->ub_b, g.n_elem, out);
    LAUNCH(k_fringe_stencil, dim3(ublocks(g.n_elem)), dim3(kUT), g.nbr, g.n_elem, out);
    if (g.n_overset > 0) LAUNCH(k_overset_list, dim3(ublocks(g.n_overset)), dim3(kUT), g.overset, g.n_overset, out);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status fringe_layer_run(oc_slot *sl, const Grid &g, int8_t *out)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    LAUNCH(k_fringe_stencil, dim3(ublocks(g.n_elem)), dim3(kUT), g.nbr, g.n_elem, out);
    if (g.n_overset > 0) LAUNCH(k_overset_list, dim3(ublocks(g.n_overset)), dim3(kUT), g.overset, g.n_overset, out);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status copy_count_run(oc_slot *sl, const int32_t *src, int32_t *dst)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    LAUNCH(k_copy_i32, dim3(1), dim3(64), src, dst);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

oc_status unblank_run(oc_slot *sl, Grid &g, Surf *const *surfs, int n_surf, const Pose *poses_t,
                      const Pose *poses_tp, const int8_t *prev, int8_t *out, int32_t *ub_list, int64_t cap,
                      int32_t *n_dev, int64_t *n_host)
{
    oc_ctx *ctx = sl->ctx;
    hipStream_t st = sl->stream;
    int kind = OC_SURF_WALL;
    for (int k = 0; k < n_surf; ++k) {
        if (k > 0 && surfs[k]->kind != kind) {
            set_error("unblank: the cutting surfaces of one grid must be of one kind");
            return OC_EINVAL;
        }
        kind = surfs[k]->kind;
    }
    if (kind == OC_SURF_WALL) {
        // one cut by every surface at both poses; the pose table holds the
        // poses of t + dt right after those of t
        std::vector<Surf *> both(surfs, surfs + n_surf);
        both.insert(both.end(), surfs, surfs + n_surf);
        if (n_surf > 0 && poses_tp != poses_t + n_surf) {
            set_error("unblank: the poses of t + dt must follow those of t");
            return OC_EINVAL;
        }
        CutReq q;
        q.g = &g;
        q.n_surf = 2 * n_surf;
        q.surfs = both.data();
        q.poses = poses_t;
        q.iblank = out;
        OC_TRY(cut_batch_run(sl, &q, 1));
    } else {
        OC_TRY(combine_overset(sl, g, surfs, n_surf, poses_t, poses_tp, out));
    }
    const int32_t *total = nullptr;
    OC_TRY(list_elements_run(sl, g, out, prev, ub_list, cap, &total));
    int32_t *cnt = n_dev ? n_dev : sl->scalar;
    LAUNCH(k_copy_i32, dim3(1), dim3(64), total, cnt);
    OC_HIP(hipGetLastError());
    if (n_host) {
        int32_t n = 0;
        OC_HIP(hipMemcpyAsync(&n, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        OC_HIP(hipStreamSynchronize(st));
        *n_host = n;
        if (n > cap) {
            set_error("oc_unblank: capacity " + std::to_string(cap) + " < " + std::to_string(n) + " cells");
            return OC_ECAPACITY;
        }
    }
    return OC_OK;
}

}  // namespace oc
