// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/oc.h"

namespace oc {

// ---------------------------------------------------------------- errors --
void set_error(const std::string &msg);
#define OC_HIP(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            ::oc::set_error(std::string(#call) + ": " + hipGetErrorString(e_));                  \
            return OC_EDEVICE;                                                                   \
        }                                                                                        \
    } while (0)
#define OC_TRY(call)                                                                             \
    do {                                                                                         \
        oc_status s_ = (call);                                                                   \
        if (s_ != OC_OK) return s_;                                                              \
    } while (0)

// ------------------------------------------------------------- bin grids --
// Uniform bins over a box: bin index of coordinate v along an axis is
// clamp(floor((v - o) * inv), 0, n - 1), evaluated in FP32.  The function is
// monotone in v, so a box [lo, hi] inserted into bins [bin(lo), bin(hi)] is
// found from any query box that overlaps it.
struct BinGrid {
    float o[3];
    float inv[3];
    int n[3];
    int pad;
};

// Per-cut device state of a cutting surface.
struct SurfParams {
    float sbox[6];     // surface box (lo xyz, hi xyz), FP32, outward
    BinGrid grid;      // bins over the surface box
    int n_bins;        // grid.n[0]*n[1]*n[2]
    int bin_off;       // first bin of this cut in the batch's bin arrays
    int pad[2];
};

// Per-cut counters (device).
struct CutCounters {
    int n_inbox, n_near, n_far, n_hit, n_hole, n_side;
    unsigned long long n_cand_pairs;
    int n_sidelist, pad;   // entries of the side list (stream order, not statistics)
};

// Per-donor-search counters (device).
struct DonorCounters {
    unsigned long long n_points, n_newton, n_iter, n_orphan, n_overflow;
};

// -------------------------------------------------------- device buffers --
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Grid {
    int64_t n_elem = 0, n_nodes = 0;
    double *enodes = nullptr;   // [n_elem][81]: x[27], y[27], z[27]
    double *emono = nullptr;    // [n_elem][81]: the same map's monomial coefficients per coordinate
    float *ebox = nullptr;      // [6][ebox_stride] SoA: xlo ylo zlo xhi yhi zhi (outward FP32)
    int64_t ebox_stride = 0;    // plane stride, n_elem rounded up to 64
    float *wbox = nullptr;      // [ceil(n_elem / 256)][6] union of the FP32 boxes of 256 consecutive elements
    int32_t *nbr = nullptr;     // [n_elem][6], -1 = boundary
    int32_t *overset = nullptr; // elements with an OVERSET-tagged face (ascending)
    int64_t n_overset = 0;
    uint8_t *ovmask = nullptr;  // [n_elem] bit f: face f OVERSET-tagged (null without tags)
    // donor search structure (registration frame)
    float *cbox = nullptr;      // [n_elem][6] control-net boxes, outward FP32
    float *obox = nullptr;      // [n_elem][18] oriented control-net boxes (centre, axes, extents)
    double *ediam = nullptr;    // [n_elem] node-box diagonal
    BinGrid dgrid{};
    int32_t *dbin_start = nullptr; // [n_dbins + 1]
    int32_t *dbin_items = nullptr; // element ids, ascending within a bin
    float4 *dbin_rec = nullptr;    // the same entries as records: control-net box + id (2 x float4)
    int64_t n_dbins = 0, n_ditems = 0;
    int dlanes = 1;                // lanes per point in the donor bin walks
    std::vector<DevBuf> owned;
};

struct Surf {
    int64_t n_face = 0, n_nodes = 0;
    int kind = OC_SURF_WALL;
    int nb_max = 4;              // bins per axis cap in use
    int nb_auto = 4;             // cap chosen at registration
    float dmax = 0.f;            // largest face-box diagonal (pose invariant bound)
    double *nodes = nullptr;     // [3][n_nodes] SoA registration frame
    int32_t *conn = nullptr;     // [n_face][9]
    double first[3] = {0, 0, 0}; // first node (registration frame)
    double rmax = 0.0;           // largest node distance from the registration origin
    std::vector<DevBuf> owned;
};

// Pose passed to kernels through device memory.
struct Pose {
    double r[9];
    double t[3];
};

constexpr int kPoseSlots = 256;

// One cut of a batch, as the kernels read it: a grid, one cutting surface
// at a device pose, the iblank it writes (several cuts of one grid may
// write the same iblank: union of holes) and its share of the slot's work
// arrays.  Element lists of a batch hold (cut << 32 | element).
struct CutInst {
    const double *enodes;
    const float *ebox;
    const float *wbox;          // box of every 256 consecutive elements (null: none)
    const int32_t *nbr;
    const double *snodes;       // surface nodes, [3][n_nodes] registration frame
    const int32_t *conn;        // [n_face][9]
    const Pose *pose;
    double *pnodes;             // [n_face][27] posed: x[9], y[9], z[9]
    float *fbox;                // [n_face][6] inflated outward FP32 boxes
    SurfParams *params;
    int8_t *iblank;
    const int8_t *prev;         // warm start: previous iblank (or null)
    int64_t stride, n_elem, n_nodes, n_face;
    double first[3];            // first surface node, registration frame
    double sweep;               // warm start: sweep bound
    float dmax;
    int nb_max, kind, write_field;
    int fblk0, eblk0;           // first block in face / element flattened launches
    int pblk0;                  // first block of the pose launch (16 faces per block)
    int bin_off0;               // first bin of this cut: the bin caps nb_max^3 of the cuts before it
};

// One output of a batch: the iblank of a grid after all of its cuts.
struct CutOut {
    int8_t *iblank;
    const int32_t *overset;
    int64_t n_elem, n_overset;
    int fblk0;                  // first block of the field fill (no surface)
    int oblk0;                  // first block of the overset-face fringe
    int cblk0;                  // first block of the hole count (statistics)
    int pad;
};

// Status of an in-box item of a batch (one byte per item): set by
// k_candidates, refined by k_hit.
enum : uint8_t { ST_NONE = 0, ST_NEAR = 1, ST_FAR = 2, ST_HIT = 3, ST_SIDE = 4 };

// Capacity of a slot's cut scratch: summed over the cuts of one call.
struct CutCaps {
    int64_t elem_inst = 0;      // sum of the cut grids' element counts
    int64_t faces = 0;          // sum of the surfaces' face counts
    int64_t bins = 0;           // sum of nb_max^3
    int64_t cuts = 0;
    int64_t outs = 0;
};

}  // namespace oc

// A slot: the per-request device scratch of the cut / fringe / donor calls
// and the stream they are ordered on.  Everything is allocated when the
// slot is created, so the calls made through a slot never allocate.
struct oc_slot {
    oc_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    bool grow = false;                 // the context's default slot grows on demand
    int64_t list_cap = 0;              // fringe-point compaction capacity (elements)
    int32_t *list_fringe = nullptr;
    int32_t *fr_tiles = nullptr;       // fringe compaction: counts, offsets, scan scratch
    int64_t fr_tiles_cap = 0;
    uint32_t *ab_mask = nullptr;       // [list_cap] bytes: AB face bits per element, zero between calls
    void *hx_buf = nullptr;            // filtered-cut arena (grown on demand)
    size_t hx_cap = 0;
    void *rf_buf[2] = {nullptr, nullptr};   // refined-cut arenas (grown on demand)
    size_t rf_cap[2] = {0, 0};
    oc::CutCounters *counters = nullptr;
    oc::DonorCounters *dcounters = nullptr;
    oc::Pose *poses = nullptr;         // [kPoseSlots] device
    int32_t *scalar = nullptr;         // device scratch
    int64_t last_n_elem = 0;
    int8_t *ub_a = nullptr, *ub_b = nullptr;   // unblank: iblank at t and at t + dt
    int64_t ub_cap = 0;
    // donor search scratch: per point and per (point, candidate) pair
    int64_t dpt_cap = 0, dpair_cap = 0;
    double *dp_local = nullptr;
    int32_t *dp_cnt = nullptr, *dp_off = nullptr, *dp_best = nullptr, *dp_scan_tmp = nullptr;
    int32_t *dp_cache = nullptr;       // [cap][4] first candidates per point
    int32_t *dpair_pt = nullptr, *dpair_el = nullptr;
    double *dpair_xi = nullptr;
    uint8_t *dpair_it = nullptr;
    std::vector<unsigned char> last_donor_args;   // arguments of the last donor search (statistics)
    // cut scratch of a batch
    oc::CutCaps cc;
    uint64_t *l_inbox = nullptr;       // in-box items (cut << 32 | element)
    uint8_t *l_stat = nullptr;         // status per in-box item
    int32_t *l_ncand = nullptr;        // candidate faces per in-box item
    int32_t *l_sidelist = nullptr;     // in-box items left to the side search
    double *l_sideu = nullptr;         // per side-list entry: distance bound from k_hit
    int32_t *sbox_part = nullptr;      // per face block: partial surface box (ordered ints)
    int last_n_cut = 0, last_n_out = 0, last_cblk = 0;
    std::vector<oc::CutOut> last_outs;
    oc::CutInst *insts = nullptr;
    oc::CutOut *outs = nullptr;
    oc::SurfParams *params = nullptr;
    double *pnodes = nullptr;
    float *fbox = nullptr;
    int32_t *bin_count = nullptr, *bin_start = nullptr, *bin_scan_tmp = nullptr;
    float4 *bin_rec = nullptr;         // bin entries: face box + id (2 x float4 each)
    std::vector<oc::DevBuf> cut_owned;   // the cut scratch above (replaced when the default slot grows)
    std::vector<oc::DevBuf> owned;
};

namespace oc {

struct Service;   // cut service state (oc_submit / oc_wait)

struct TimingRec {
    hipEvent_t a, b;
    const char *name;
};

}  // namespace oc

struct oc_ctx {
    int device = 0;
    int surf_bins = 0;
    int exact_waves = 8192;                // persistent wavefronts of the exact-stage kernels
    int filter_block = 256;                // threads per block of the element-box filter
    int side_list = 64;                    // faces a side-search wavefront lists for the tie stage
    int point_tiles = 2048;                // most fringe tiles whose offsets the point kernel forms
    std::vector<std::pair<int, double>> bin_factor;   // tuned bins factor per face-count octave
    int donor_waves = 0;                   // cap on the donor-search wavefronts (0 = none)
    int64_t donor_pairs = 0;               // cap on the pairs one donor search keeps (0 = none)
    double donor_bin_scale = 0.5;
    int64_t budget = 0;
    int64_t used = 0;
    std::vector<std::unique_ptr<oc::Grid>> grids;
    std::vector<std::unique_ptr<oc::Surf>> surfs;
    oc_slot *dflt = nullptr;               // default slot of the simple calls
    std::vector<oc_slot *> slots;          // slots created by the caller
    int32_t *dev_scalar = nullptr;         // device scratch int (registration)
    hipStream_t reg_stream = nullptr;      // registration work
    // timing (default slot and slots alike, recorded on the launching stream)
    bool timing = false;
    std::vector<oc::TimingRec> trecs;
    std::vector<hipEvent_t> event_pool;
    size_t event_next = 0;
    // cut service (oc_submit / oc_wait)
    oc::Service *service = nullptr;
    int service_slots = 4;                 // most slots the service keeps
    // staging of host arrays given to the plain calls
    std::vector<oc::DevBuf> stage_owned;
    void *stage = nullptr;
    size_t stage_cap = 0;
};

namespace oc {

oc_status dev_alloc(oc_ctx *ctx, std::vector<DevBuf> &owner, size_t bytes, void **out);
void dev_free_all(oc_ctx *ctx, std::vector<DevBuf> &owner);

// Launch bracketing for per-kernel timing (events on the given stream).
void time_begin(oc_ctx *ctx, hipStream_t st, const char *name, size_t *slot);
void time_end(oc_ctx *ctx, hipStream_t st, size_t slot);

// exclusive scan of n (device count n_dev if non-null, else n_host) int32
// values; out[n] receives the total.  tmp must hold scan_tmp_ints(cap) ints.
int64_t scan_tmp_ints(int64_t cap);
// largest count scan_exclusive takes
int64_t scan_max_items();
oc_status scan_exclusive(oc_ctx *ctx, hipStream_t st, const int32_t *in, int32_t *out, int64_t cap,
                         const int *n_dev, int32_t *tmp);

// registration-time device work
oc_status grid_build_device(oc_ctx *ctx, Grid &g, const int32_t *conn_dev, const double *nodes_dev);
oc_status grid_build_donor_bins(oc_ctx *ctx, Grid &g);

// slot scratch sizing (grow-only for the default slot)
oc_status slot_reserve_grid(oc_slot *sl, const Grid &g);
oc_status slot_reserve_cut(oc_slot *sl, const CutCaps &need);
oc_status slot_reserve_points(oc_slot *sl, int64_t cap);
constexpr int kPairsPerPoint = 8;   // pair capacity per point capacity

oc_status set_poses(oc_slot *sl, int first, const double *host, int n);
// copy host bytes to device memory in stream order through kernel
// arguments (capturable; the host array may be reused on return)
oc_status put_bytes(oc_slot *sl, void *dst, const void *src, size_t n);
oc_status slot_init(oc_ctx *ctx, oc_slot *sl, bool grow);
void slot_free(oc_slot *sl);

// One request of a cut batch: a grid cut by n_surf surfaces (union of
// holes) at device poses, into its own iblank.  Warm start: prev = previous
// iblank of the same grid and single surface, sweep = bound on how far any
// surface point moved since (null / 0: cold).
struct CutReq {
    Grid *g = nullptr;
    int n_surf = 0;
    Surf *const *surfs = nullptr;
    const Pose *poses = nullptr;
    int8_t *iblank = nullptr;
    const int8_t *prev = nullptr;
    double sweep = 0.0;
};
CutCaps cut_caps(const CutReq *reqs, int n);
// OC_EINVAL (with a message) for cut capacities beyond what the scans and
// the int32 indices of the cut kernels take
oc_status cut_caps_check(const CutCaps &c);
// validate the public requests and resolve their grids and surfaces (poses
// are left null; with need_outputs the outputs and poses must be given)
oc_status collect_cut_reqs(oc_ctx *ctx, const oc_cut_req *reqs, int32_t n_req, std::vector<CutReq> &out,
                           std::vector<std::vector<Surf *>> &surfs, bool need_outputs);
// a slot with cut capacity cc, element lists for grids of up to ne
// elements and points_cap donor points, on the given stream (not entered in
// ctx->slots)
oc_status slot_make(oc_ctx *ctx, const CutCaps &cc, int64_t ne, int64_t points_cap, hipStream_t stream,
                    oc_slot **out);
int64_t slot_bytes(const oc_slot *sl);
bool pose_finite(const double *p);
// the cut service's slots and queue, released with the context
void service_destroy(oc_ctx *ctx);
// every request's cuts in one launch per stage
oc_status cut_batch_run(oc_slot *sl, const CutReq *reqs, int n);
// statistics of the slot's last cut batch into sl->counters (stream ordered)
oc_status cut_stats_run(oc_slot *sl);
// statistics of the slot's last donor search into sl->dcounters
oc_status donor_stats_run(oc_slot *sl);
// receptor points: the count stays on the device (n_dev, int32) and is also
// returned on the host when n_host is not null (synchronising)
oc_status fringe_points_run(oc_slot *sl, Grid &g, const Pose *pose_dev, const int8_t *iblank, double *pts,
                            int64_t cap, int32_t *n_dev, int64_t *n_host, int32_t *src);
// ordered compaction of the elements of g that are fringe in iblank (prev
// null) or holes of prev that are not holes of iblank; at most cap ids into
// list, the count left on the device at *total
oc_status list_elements_run(oc_slot *sl, const Grid &g, const int8_t *iblank, const int8_t *prev, int32_t *list,
                            int64_t cap, const int32_t **total);
// 27 Gauss points of the first min(*count, cap / 27) listed elements
oc_status element_points_run(oc_slot *sl, const Grid &g, const Pose *pose_dev, const int32_t *list,
                             const int32_t *count, double *pts, int64_t cap, int32_t *n_out, int32_t *src);
// 1-D reference nodes of the flux points and of the interpolation basis
constexpr int kMaxNodes1D = 8;
struct Nodes1D {
    double z[kMaxNodes1D];
    int m;
};
// artificial-boundary faces of iblank (ids 6 e + f, ascending, at most cap
// into faces); the count stays on the device at *total
oc_status ab_faces_run(oc_slot *sl, const Grid &g, const int8_t *iblank, int32_t *faces, int64_t cap,
                       const int32_t **total);
// m x m flux points of min(*n_faces, faces_cap) faces (n_faces null:
// faces_cap); at most cap points; n_out (device, may be null) receives the
// number of points
oc_status face_points_run(oc_slot *sl, const Grid &g, const Pose *pose_dev, const int32_t *faces,
                          const int32_t *n_faces, int64_t faces_cap, const Nodes1D &z, double *pts, int64_t cap,
                          int32_t *n_out, int32_t *src);
// one fringe layer around the holes of out (full-grid stencil) and the
// overset-tagged faces
oc_status fringe_layer_run(oc_slot *sl, const Grid &g, int8_t *out);
// the paper's filtered cut (N_F^1 = nf1 <= 32, N_F^2 = nf2 <= 16) of g by
// the surfaces at poses_dev; synchronises once per surface; *n_listed
// (may be null) receives the number of (surface, element) pairs examined
oc_status filtered_cut_run(oc_slot *sl, Grid &g, Surf *const *surfs, const Pose *poses_dev, int n_surf, int nf1,
                           int nf2, int8_t *iblank, int64_t *n_listed);
// *dst = *src on the slot stream (device counts)
oc_status copy_count_run(oc_slot *sl, const int32_t *src, int32_t *dst);
// m^3 interpolation weights of min(*n_dev, cap) points (n_dev null: cap)
oc_status weights_run(oc_slot *sl, const int32_t *donors, const double *ref, const int32_t *n_dev, int64_t cap,
                      const Nodes1D &z, double *w);
// blanking of a moving grid's time step with unblanking: cuts at poses_t
// and poses_tp (device), combined by the surfaces' kind, fringe layer, and
// the holes of prev that are holes no more (ascending, at most cap)
oc_status unblank_run(oc_slot *sl, Grid &g, Surf *const *surfs, int n_surf, const Pose *poses_t,
                      const Pose *poses_tp, const int8_t *prev, int8_t *out, int32_t *ub_list, int64_t cap,
                      int32_t *n_dev, int64_t *n_host);
// the allocation-free donor search: device address of this device's
// scratch array (once per device, device current), its point limit, and
// the search of n <= noalloc_max_points() points on the context stream
oc_status noalloc_init(int device);
int64_t noalloc_max_points();
oc_status donor_noalloc_run(oc_ctx *ctx, Grid &g, const double *pose_host, const double *pts, int64_t n,
                            int32_t *donor, double *ref);
// caller memory: device (or managed) memory, else host memory staged
bool device_memory(const void *p);
// the context's staging area, at least bytes (synchronises when it grows)
oc_status stage_reserve(oc_ctx *ctx, size_t bytes, char **base);
// rigid pose of a surface in a grid's frame (host)
void pose_relative(const double *grid, const double *surf, double *out);
// the same for device poses: out[k] = inverse(grid) after surfs[k]
oc_status compose_poses_run(oc_slot *sl, const double *grid_dev, const double *surfs_dev, int n, Pose *out);
// the refined cut of level k (the curved faces split k x k, the near
// elements k^3 times) of g by the surfaces at poses_dev into iblank;
// synchronises; *n_near (may be null) receives the number of near
// (surface, element) items refined
oc_status refined_cut_run(oc_slot *sl, Grid &g, Surf *const *surfs, const Pose *poses_dev, int n_surf, int k,
                          int8_t *iblank, int64_t *n_near);
// donor search of min(*n_dev, cap) points (n_dev may be null: cap points)
oc_status donor_run(oc_slot *sl, Grid &g, const Pose *pose_dev, const double *pts, int64_t cap, const int32_t *n_dev,
                    int32_t *donor, double *ref);

}  // namespace oc
