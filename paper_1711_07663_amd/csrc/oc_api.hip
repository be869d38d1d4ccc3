// C ABI entry points, context, validation and registration.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <unordered_map>

#include "dev_common.h"

namespace oc {

static thread_local std::string g_error;
void set_error(const std::string &msg) { g_error = msg; }

oc_status dev_alloc(oc_ctx *ctx, std::vector<DevBuf> &owner, size_t bytes, void **out)
{
    if (bytes == 0) bytes = 256;
    if (ctx->budget > 0 && ctx->used + (int64_t)bytes > ctx->budget) {
        set_error("HBM budget exceeded: " + std::to_string(ctx->used + bytes) + " > " + std::to_string(ctx->budget));
        return OC_EBUDGET;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
        (void)hipGetLastError();
        set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
        return OC_ENOMEM;
    }
    owner.push_back(DevBuf{p, bytes});
    ctx->used += (int64_t)bytes;
    *out = p;
    return OC_OK;
}

void dev_free_all(oc_ctx *ctx, std::vector<DevBuf> &owner)
{
    for (auto &b : owner) {
        (void)hipFree(b.p);
        ctx->used -= (int64_t)b.bytes;
    }
    owner.clear();
}

void time_begin(oc_ctx *ctx, hipStream_t st, const char *name, size_t *slot)
{
    *slot = std::numeric_limits<size_t>::max();
    if (!ctx || !ctx->timing) return;
    // no timing events inside a stream capture: the pooled events are
    // recorded again by later launches, and an event recorded more than once
    // within one capture is a form the captured steps never rely on
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    while (ctx->event_pool.size() < ctx->event_next + 2) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return;
        ctx->event_pool.push_back(ev);
    }
    TimingRec r{ctx->event_pool[ctx->event_next], ctx->event_pool[ctx->event_next + 1], name};
    ctx->event_next += 2;
    (void)hipEventRecord(r.a, st);
    *slot = ctx->trecs.size();
    ctx->trecs.push_back(r);
}

void time_end(oc_ctx *ctx, hipStream_t st, size_t slot)
{
    if (slot == std::numeric_limits<size_t>::max()) return;
    (void)hipEventRecord(ctx->trecs[slot].b, st);
}

// ------------------------------------------------ host or device memory --
// Caller arrays of the plain calls may be host or device memory (the
// pointer's attributes decide); host arrays pass through a staging area on
// the device, grown on demand and kept by the context.
bool device_memory(const void *p)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// a host copy of a caller array that may be device memory (read on the
// context stream, so work the caller ordered there before is seen)
template <class T>
static oc_status host_view(oc_ctx *ctx, const T *p, int64_t n, std::vector<T> &buf, const T **out)
{
    *out = p;
    if (!p || n <= 0 || !device_memory(p)) return OC_OK;
    buf.resize((size_t)n);
    OC_HIP(hipMemcpyAsync(buf.data(), p, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost, ctx->dflt->stream));
    OC_HIP(hipStreamSynchronize(ctx->dflt->stream));
    *out = buf.data();
    return OC_OK;
}

oc_status stage_reserve(oc_ctx *ctx, size_t bytes, char **base)
{
    bytes = (bytes + 255) / 256 * 256;
    if (bytes > ctx->stage_cap) {
        OC_HIP(hipStreamSynchronize(ctx->dflt->stream));
        dev_free_all(ctx, ctx->stage_owned);
        ctx->stage_cap = 0;
        OC_TRY(dev_alloc(ctx, ctx->stage_owned, bytes, &ctx->stage));
        ctx->stage_cap = bytes;
    }
    *base = reinterpret_cast<char *>(ctx->stage);
    return OC_OK;
}

// rigid pose of a surface in a grid's frame: inverse(grid) after surface,
// R = Rg^T Rs, t = Rg^T ts - Rg^T tg (poses: R row-major, then t)
void pose_relative(const double *grid, const double *surf, double *out)
{
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            out[3 * i + j] = grid[i] * surf[j] + grid[3 + i] * surf[3 + j] + grid[6 + i] * surf[6 + j];
        const double a = grid[i] * surf[9] + grid[3 + i] * surf[10] + grid[6 + i] * surf[11];
        const double b = grid[i] * grid[9] + grid[3 + i] * grid[10] + grid[6 + i] * grid[11];
        out[9 + i] = a - b;
    }
}

// ------------------------------------------------------------------ slots --
static oc_status slot_alloc_lists(oc_slot *sl, int64_t n_elem)
{
    oc_ctx *ctx = sl->ctx;
    const size_t ne = (size_t)std::max<int64_t>(n_elem, 1);
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * ne, (void **)&sl->list_fringe));
    const int64_t nt = (n_elem + 4095) / 4096;
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * (2 * (nt + 1) + scan_tmp_ints(nt) + 8), (void **)&sl->fr_tiles));
    OC_TRY(dev_alloc(ctx, sl->owned, (ne + 3) / 4 * 4, (void **)&sl->ab_mask));
    OC_HIP(hipMemset(sl->ab_mask, 0, (ne + 3) / 4 * 4));
    sl->list_cap = n_elem;
    sl->fr_tiles_cap = nt;
    return OC_OK;
}

// cut scratch for caps c (replaces any previous cut scratch of the slot)
oc_status cut_caps_check(const CutCaps &c)
{
    // bins are scanned in one device-wide scan and indexed by int32, element
    // lists hold int32 element ids per cut
    if (c.bins > scan_max_items() || c.bins >= INT32_MAX || c.elem_inst >= INT32_MAX || c.faces >= INT32_MAX / 27) {
        set_error("cut too large: " + std::to_string(c.bins) + " surface bins (at most " +
                  std::to_string(std::min<int64_t>(scan_max_items(), INT32_MAX - 1)) + "), " +
                  std::to_string(c.elem_inst) + " elements x surfaces, " + std::to_string(c.faces) + " faces");
        return OC_EINVAL;
    }
    return OC_OK;
}

static oc_status slot_alloc_cut(oc_slot *sl, CutCaps c)
{
    oc_ctx *ctx = sl->ctx;
    OC_TRY(cut_caps_check(c));
    dev_free_all(ctx, sl->cut_owned);
    sl->cc = CutCaps{};
    c.elem_inst = std::max<int64_t>(c.elem_inst, 1);
    c.faces = std::max<int64_t>(c.faces, 1);
    c.bins = std::max<int64_t>(c.bins, 1);
    c.cuts = std::max<int64_t>(c.cuts, 1);
    c.outs = std::max<int64_t>(c.outs, 1);
    auto &o = sl->cut_owned;
    OC_TRY(dev_alloc(ctx, o, sizeof(uint64_t) * (size_t)c.elem_inst, (void **)&sl->l_inbox));
    OC_TRY(dev_alloc(ctx, o, sizeof(uint8_t) * (size_t)c.elem_inst, (void **)&sl->l_stat));
    OC_TRY(dev_alloc(ctx, o, sizeof(int32_t) * (size_t)c.elem_inst, (void **)&sl->l_ncand));
    OC_TRY(dev_alloc(ctx, o, sizeof(int32_t) * (size_t)c.elem_inst, (void **)&sl->l_sidelist));
    OC_TRY(dev_alloc(ctx, o, sizeof(double) * (size_t)c.elem_inst, (void **)&sl->l_sideu));
    // partial boxes of the pose launch: blocks of 16 faces, plus one spare
    // block per cut
    OC_TRY(dev_alloc(ctx, o, sizeof(int32_t) * 6 * (size_t)(c.faces / 16 + 2 * c.cuts + 1),
                     (void **)&sl->sbox_part));
    OC_TRY(dev_alloc(ctx, o, sizeof(CutInst) * (size_t)c.cuts, (void **)&sl->insts));
    OC_TRY(dev_alloc(ctx, o, sizeof(CutOut) * (size_t)c.outs, (void **)&sl->outs));
    OC_TRY(dev_alloc(ctx, o, sizeof(SurfParams) * (size_t)c.cuts, (void **)&sl->params));
    OC_TRY(dev_alloc(ctx, o, sizeof(double) * 27 * (size_t)c.faces, (void **)&sl->pnodes));
    OC_TRY(dev_alloc(ctx, o, sizeof(float) * 6 * (size_t)c.faces, (void **)&sl->fbox));
    OC_TRY(dev_alloc(ctx, o, sizeof(int32_t) * (size_t)(c.bins + 1), (void **)&sl->bin_count));
    OC_TRY(dev_alloc(ctx, o, sizeof(int32_t) * (size_t)(c.bins + 1), (void **)&sl->bin_start));
    OC_TRY(dev_alloc(ctx, o, sizeof(float4) * 2 * 8 * (size_t)c.faces, (void **)&sl->bin_rec));
    OC_TRY(dev_alloc(ctx, o, sizeof(int32_t) * (size_t)scan_tmp_ints(c.bins + 1), (void **)&sl->bin_scan_tmp));
    // bin counts start at zero; every cut returns them to zero
    OC_HIP(hipMemset(sl->bin_count, 0, sizeof(int32_t) * (size_t)(c.bins + 1)));
    sl->cc = c;
    return OC_OK;
}

oc_status slot_init(oc_ctx *ctx, oc_slot *sl, bool grow)
{
    sl->ctx = ctx;
    sl->grow = grow;
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(CutCounters), (void **)&sl->counters));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(DonorCounters), (void **)&sl->dcounters));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(Pose) * kPoseSlots, (void **)&sl->poses));
    OC_TRY(dev_alloc(ctx, sl->owned, 256, (void **)&sl->scalar));
    OC_HIP(hipMemset(sl->counters, 0, sizeof(CutCounters)));
    OC_HIP(hipMemset(sl->dcounters, 0, sizeof(DonorCounters)));
    return OC_OK;
}

void slot_free(oc_slot *sl)
{
    if (!sl) return;
    (void)hipStreamSynchronize(sl->stream);
    dev_free_all(sl->ctx, sl->cut_owned);
    dev_free_all(sl->ctx, sl->owned);
}

// The default slot grows on demand (its calls may allocate); slots made by
// oc_slot_create are sized once and refuse larger work.
oc_status slot_reserve_grid(oc_slot *sl, const Grid &g)
{
    if (g.n_elem <= sl->list_cap) return OC_OK;
    if (!sl->grow) {
        set_error("slot was not created for a grid of " + std::to_string(g.n_elem) + " elements");
        return OC_EINVAL;
    }
    OC_HIP(hipStreamSynchronize(sl->stream));
    // the old lists stay allocated until the slot is freed (simple, rare)
    return slot_alloc_lists(sl, g.n_elem);
}

static oc_status slot_alloc_points(oc_slot *sl, int64_t cap)
{
    oc_ctx *ctx = sl->ctx;
    const int64_t pc = cap * kPairsPerPoint;
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(double) * 3 * cap, (void **)&sl->dp_local));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * (cap + 1), (void **)&sl->dp_cnt));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * (cap + 1), (void **)&sl->dp_off));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * cap, (void **)&sl->dp_best));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * 4 * cap, (void **)&sl->dp_cache));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * scan_tmp_ints(cap), (void **)&sl->dp_scan_tmp));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * pc, (void **)&sl->dpair_pt));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(int32_t) * pc, (void **)&sl->dpair_el));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(double) * 3 * pc, (void **)&sl->dpair_xi));
    OC_TRY(dev_alloc(ctx, sl->owned, sizeof(uint8_t) * pc, (void **)&sl->dpair_it));
    sl->dpt_cap = cap;
    sl->dpair_cap = pc;
    return OC_OK;
}

oc_status slot_reserve_points(oc_slot *sl, int64_t cap)
{
    if (cap <= sl->dpt_cap) return OC_OK;
    if (!sl->grow) {
        set_error("slot was not created for " + std::to_string(cap) + " points");
        return OC_EINVAL;
    }
    OC_HIP(hipStreamSynchronize(sl->stream));
    return slot_alloc_points(sl, cap);
}

static bool caps_fit(const CutCaps &have, const CutCaps &need)
{
    return need.elem_inst <= have.elem_inst && need.faces <= have.faces && need.bins <= have.bins &&
           need.cuts <= have.cuts && need.outs <= have.outs;
}

oc_status slot_reserve_cut(oc_slot *sl, const CutCaps &need)
{
    if (caps_fit(sl->cc, need)) return OC_OK;
    if (!sl->grow) {
        set_error("slot was not created for this cut (elements x surfaces " + std::to_string(need.elem_inst) +
                  ", faces " + std::to_string(need.faces) + ", cuts " + std::to_string(need.cuts) + ")");
        return OC_EINVAL;
    }
    OC_HIP(hipStreamSynchronize(sl->stream));
    CutCaps c = need;
    c.elem_inst = std::max(c.elem_inst, sl->cc.elem_inst);
    c.faces = std::max(c.faces, sl->cc.faces);
    c.bins = std::max(c.bins, sl->cc.bins);
    c.cuts = std::max(c.cuts, sl->cc.cuts);
    c.outs = std::max(c.outs, sl->cc.outs);
    return slot_alloc_cut(sl, c);
}

bool pose_finite(const double *p)
{
    if (!p) return false;
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// face corner local indices, order -xi,+xi,-eta,+eta,-zeta,+zeta
static const int kFaceCorners[6][4] = {{0, 6, 18, 24}, {2, 8, 20, 26}, {0, 2, 18, 20},
                                       {6, 8, 24, 26}, {0, 2, 6, 8},   {18, 20, 24, 26}};

// Face adjacency from shared corner ids: bucket every face by its smallest
// corner id (counting sort), then match the remaining three ids inside a
// bucket.  Returns false for a face shared by more than two elements.
static bool face_neighbors(const int32_t *conn, int64_t n_elem, int64_t n_nodes, std::vector<int32_t> &nbr)
{
    const int64_t nf = n_elem * 6;
    nbr.assign((size_t)nf, -1);
    std::vector<std::array<int32_t, 4>> key((size_t)nf);
    std::vector<int32_t> cnt((size_t)n_nodes + 1, 0);
    for (int64_t e = 0; e < n_elem; ++e)
        for (int f = 0; f < 6; ++f) {
            std::array<int32_t, 4> k;
            for (int i = 0; i < 4; ++i) k[i] = conn[e * 27 + kFaceCorners[f][i]];
            std::sort(k.begin(), k.end());
            key[(size_t)(e * 6 + f)] = k;
            cnt[(size_t)k[0] + 1]++;
        }
    for (int64_t i = 0; i < n_nodes; ++i) cnt[(size_t)i + 1] += cnt[(size_t)i];
    std::vector<int32_t> order((size_t)nf);
    {
        std::vector<int32_t> cur(cnt.begin(), cnt.end() - 1);
        for (int64_t i = 0; i < nf; ++i) order[(size_t)cur[(size_t)key[(size_t)i][0]]++] = (int32_t)i;
    }
    for (int64_t v = 0; v < n_nodes; ++v) {
        const int32_t b0 = cnt[(size_t)v], b1 = cnt[(size_t)v + 1];
        for (int32_t i = b0; i < b1; ++i) {
            const int32_t fi = order[(size_t)i];
            for (int32_t j = i + 1; j < b1; ++j) {
                const int32_t fj = order[(size_t)j];
                if (key[(size_t)fi] != key[(size_t)fj]) continue;
                if (nbr[(size_t)fi] >= 0 || nbr[(size_t)fj] >= 0) return false;
                nbr[(size_t)fi] = fj / 6;
                nbr[(size_t)fj] = fi / 6;
            }
        }
    }
    return true;
}

template <class T>
static oc_status upload(oc_ctx *ctx, std::vector<DevBuf> &owner, const T *src, size_t n, T **dst)
{
    OC_TRY(dev_alloc(ctx, owner, sizeof(T) * std::max<size_t>(n, 1), (void **)dst));
    if (n) OC_HIP(hipMemcpy(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice));
    return OC_OK;
}

}  // namespace oc

using namespace oc;

extern "C" {

const char *oc_last_error(void) { return g_error.c_str(); }

// The tuning file of oc_config.tune_cache: "key value" lines (see oc.h).
static oc_status read_tune_cache(oc_ctx *ctx, const char *path)
{
    FILE *f = fopen(path, "r");
    if (!f) {
        set_error(std::string("oc_create: cannot read tuning file ") + path);
        return OC_EINVAL;
    }
    char line[512];
    int ln = 0;
    oc_status st = OC_OK;
    while (st == OC_OK && fgets(line, sizeof line, f)) {
        ++ln;
        if (char *h = strchr(line, '#')) *h = 0;
        char key[64];
        long long a = 0;
        double b = 0.0;
        int n = sscanf(line, "%63s %lld %lf", key, &a, &b);
        if (n <= 0) continue;   // blank or comment
        bool ok = false;
        if (n == 2 && !strcmp(key, "exact_waves")) {
            ok = a >= 0 && a <= (1 << 20);
            if (ok) ctx->exact_waves = a == 0 ? 8192 : (int)a;
        } else if (n == 2 && !strcmp(key, "filter_block")) {
            ok = a == 0 || a == 64 || a == 128 || a == 256 || a == 512 || a == 1024;
            if (ok) ctx->filter_block = a == 0 ? 256 : (int)a;
        } else if (n == 2 && !strcmp(key, "donor_waves")) {
            ok = a >= 0 && a <= (1 << 22);
            if (ok) ctx->donor_waves = (int)a;
        } else if (n == 3 && !strcmp(key, "bin_factor")) {
            ok = a >= 0 && a < 63 && b > 0.0 && b <= 1.0;
            if (ok) ctx->bin_factor.emplace_back((int)a, b);
        }
        if (!ok) {
            set_error(std::string("oc_create: bad line ") + std::to_string(ln) + " in tuning file " + path);
            st = OC_EINVAL;
        }
    }
    fclose(f);
    return st;
}

oc_status oc_create(oc_ctx **out, const oc_config *cfg)
{
    if (!out) {
        set_error("oc_create: null output");
        return OC_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        set_error("oc_create: no HIP device");
        return OC_EDEVICE;
    }
    oc_ctx *ctx = new oc_ctx();
    if (cfg) {
        ctx->device = cfg->device;
        ctx->surf_bins = cfg->surf_bins;
        ctx->donor_bin_scale = cfg->donor_bin_scale > 0 ? cfg->donor_bin_scale : 0.5;
        ctx->budget = cfg->hbm_budget;
        if (cfg->tune_cache) {
            oc_status ts = read_tune_cache(ctx, cfg->tune_cache);
            if (ts != OC_OK) {
                delete ctx;
                return ts;
            }
        }
    }
    if (ctx->device < 0 || ctx->device >= ndev || hipSetDevice(ctx->device) != hipSuccess) {
        delete ctx;
        set_error("oc_create: invalid device");
        return OC_EINVAL;
    }
    // device address of the allocation-free search's scratch on this device
    if (noalloc_init(ctx->device) != OC_OK) {
        delete ctx;
        return OC_EDEVICE;
    }
    if (hipMalloc(&ctx->dev_scalar, 64) != hipSuccess) {
        delete ctx;
        set_error("oc_create: allocation failed");
        return OC_ENOMEM;
    }
    // registration flag and the check word of checked builds start at zero
    if (hipMemset(ctx->dev_scalar, 0, 64) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(ctx->dev_scalar);
        delete ctx;
        set_error("oc_create: device memset failed");
        return OC_EDEVICE;
    }
    ctx->dflt = new oc_slot();
    oc_status st = slot_init(ctx, ctx->dflt, true);
    if (st != OC_OK) {
        slot_free(ctx->dflt);
        delete ctx->dflt;
        (void)hipFree(ctx->dev_scalar);
        delete ctx;
        return st;
    }
    *out = ctx;
    return OC_OK;
}

oc_status oc_destroy(oc_ctx *ctx)
{
    if (!ctx) return OC_OK;
    (void)hipSetDevice(ctx->device);
    service_destroy(ctx);
    for (auto sl : ctx->slots) {
        slot_free(sl);
        delete sl;
    }
    ctx->slots.clear();
    slot_free(ctx->dflt);
    delete ctx->dflt;
    for (auto &g : ctx->grids)
        if (g) dev_free_all(ctx, g->owned);
    for (auto &s : ctx->surfs)
        if (s) dev_free_all(ctx, s->owned);
    dev_free_all(ctx, ctx->stage_owned);
    (void)hipFree(ctx->dev_scalar);
    for (auto ev : ctx->event_pool) (void)hipEventDestroy(ev);
    delete ctx;
    return OC_OK;
}

oc_status oc_set_stream(oc_ctx *ctx, void *stream)
{
    if (!ctx) {
        set_error("oc_set_stream: null context");
        return OC_EINVAL;
    }
    ctx->dflt->stream = (hipStream_t)stream;
    return OC_OK;
}

oc_status oc_register_grid(oc_ctx *ctx, const double *nodes, int64_t n_nodes, const int32_t *conn, int64_t n_elem,
                           const int8_t *face_tags, int32_t *grid_id)
{
    if (!ctx || !nodes || !conn || !grid_id || n_nodes <= 0 || n_elem <= 0 || n_elem > (1ll << 31) / 32 ||
        n_nodes >= (1ll << 31)) {
        set_error("oc_register_grid: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    // device arrays are read back first (registration validates on the host)
    std::vector<double> hn;
    std::vector<int32_t> hc;
    std::vector<int8_t> ht;
    OC_TRY(host_view(ctx, nodes, n_nodes * 3, hn, &nodes));
    OC_TRY(host_view(ctx, conn, n_elem * 27, hc, &conn));
    OC_TRY(host_view(ctx, face_tags, n_elem * 6, ht, &face_tags));
    for (int64_t i = 0; i < n_elem * 27; ++i)
        if (conn[i] < 0 || conn[i] >= n_nodes) {
            set_error("oc_register_grid: node id out of range at conn[" + std::to_string(i) + "]");
            return OC_EINVAL;
        }
    for (int64_t i = 0; i < n_nodes * 3; ++i)
        if (!std::isfinite(nodes[i])) {
            set_error("oc_register_grid: non-finite node coordinate");
            return OC_EINVAL;
        }
    std::vector<int32_t> nbr;
    if (!face_neighbors(conn, n_elem, n_nodes, nbr)) {
        set_error("oc_register_grid: a face is shared by more than two elements");
        return OC_EGEOM;
    }
    std::vector<int32_t> overset;
    if (face_tags)
        for (int64_t e = 0; e < n_elem; ++e)
            for (int f = 0; f < 6; ++f)
                if (face_tags[e * 6 + f] == OC_FACE_OVERSET) {
                    overset.push_back((int32_t)e);
                    break;
                }

    auto g = std::make_unique<Grid>();
    g->n_elem = n_elem;
    g->n_nodes = n_nodes;
    g->ebox_stride = (n_elem + 63) / 64 * 64;
    oc_status st = OC_OK;
    double *nodes_dev = nullptr;
    int32_t *conn_dev = nullptr;
    std::vector<DevBuf> tmp;
    auto fail = [&](oc_status s) {
        dev_free_all(ctx, tmp);
        dev_free_all(ctx, g->owned);
        return s;
    };
    if ((st = upload(ctx, tmp, nodes, (size_t)n_nodes * 3, &nodes_dev)) != OC_OK) return fail(st);
    if ((st = upload(ctx, tmp, conn, (size_t)n_elem * 27, &conn_dev)) != OC_OK) return fail(st);
    const size_t ne = (size_t)n_elem;
    if ((st = dev_alloc(ctx, g->owned, sizeof(double) * ne * 81, (void **)&g->enodes)) != OC_OK) return fail(st);
    if ((st = dev_alloc(ctx, g->owned, sizeof(double) * ne * 81, (void **)&g->emono)) != OC_OK) return fail(st);
    if ((st = dev_alloc(ctx, g->owned, sizeof(float) * 6 * (size_t)g->ebox_stride, (void **)&g->ebox)) != OC_OK)
        return fail(st);
    if ((st = dev_alloc(ctx, g->owned, sizeof(float) * 6 * ((ne + 255) / 256), (void **)&g->wbox)) != OC_OK)
        return fail(st);
    if ((st = dev_alloc(ctx, g->owned, sizeof(float) * 6 * ne, (void **)&g->cbox)) != OC_OK) return fail(st);
    if ((st = dev_alloc(ctx, g->owned, sizeof(float) * 18 * ne, (void **)&g->obox)) != OC_OK) return fail(st);
    if ((st = dev_alloc(ctx, g->owned, sizeof(double) * ne, (void **)&g->ediam)) != OC_OK) return fail(st);
    if ((st = upload(ctx, g->owned, nbr.data(), nbr.size(), &g->nbr)) != OC_OK) return fail(st);
    g->n_overset = (int64_t)overset.size();
    if ((st = upload(ctx, g->owned, overset.data(), overset.size(), &g->overset)) != OC_OK) return fail(st);
    if (!overset.empty()) {
        std::vector<uint8_t> ovm((size_t)n_elem, 0);
        for (int64_t e = 0; e < n_elem; ++e)
            for (int f = 0; f < 6; ++f)
                if (face_tags[e * 6 + f] == OC_FACE_OVERSET) ovm[(size_t)e] |= (uint8_t)(1u << f);
        if ((st = upload(ctx, g->owned, ovm.data(), ovm.size(), &g->ovmask)) != OC_OK) return fail(st);
    }
    if ((st = grid_build_device(ctx, *g, conn_dev, nodes_dev)) != OC_OK) return fail(st);
    dev_free_all(ctx, tmp);
    if ((st = grid_build_donor_bins(ctx, *g)) != OC_OK) return fail(st);
    ctx->grids.push_back(std::move(g));
    *grid_id = (int32_t)ctx->grids.size() - 1;
    return OC_OK;
}

oc_status oc_register_cut_surface(oc_ctx *ctx, const double *nodes, int64_t n_nodes, const int32_t *conn,
                                  int64_t n_face, int32_t kind, int32_t *surf_id)
{
    if (!ctx || !nodes || !conn || !surf_id || n_nodes <= 0 || n_face <= 0 || n_face > (1ll << 26) ||
        n_nodes >= (1ll << 31) || (kind != OC_SURF_WALL && kind != OC_SURF_OVERSET)) {
        set_error("oc_register_cut_surface: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    std::vector<double> hn;
    std::vector<int32_t> hc;
    OC_TRY(host_view(ctx, nodes, n_nodes * 3, hn, &nodes));
    OC_TRY(host_view(ctx, conn, n_face * 9, hc, &conn));
    for (int64_t i = 0; i < n_face * 9; ++i)
        if (conn[i] < 0 || conn[i] >= n_nodes) {
            set_error("oc_register_cut_surface: node id out of range");
            return OC_EINVAL;
        }
    for (int64_t i = 0; i < n_nodes * 3; ++i)
        if (!std::isfinite(nodes[i])) {
            set_error("oc_register_cut_surface: non-finite node coordinate");
            return OC_EINVAL;
        }
    // closed and consistently oriented: every directed boundary segment of a
    // face lattice appears once, and its reverse once
    static const int loop[9] = {0, 1, 2, 5, 8, 7, 6, 3, 0};
    std::unordered_map<uint64_t, int> seg;
    seg.reserve((size_t)n_face * 16);
    for (int64_t f = 0; f < n_face; ++f)
        for (int k = 0; k < 8; ++k) {
            uint32_t a = (uint32_t)conn[f * 9 + loop[k]], b = (uint32_t)conn[f * 9 + loop[k + 1]];
            if (a == b) {
                set_error("oc_register_cut_surface: degenerate face edge");
                return OC_EGEOM;
            }
            seg[((uint64_t)a << 32) | b]++;
        }
    for (auto &kv : seg) {
        uint64_t rev = (kv.first << 32) | (kv.first >> 32);
        auto it = seg.find(rev);
        if (kv.second != 1 || it == seg.end() || it->second != 1) {
            set_error("oc_register_cut_surface: surface is not closed and consistently oriented");
            return OC_EGEOM;
        }
    }
    // enclosed volume (divergence theorem on the triangulation) and face size
    double vol = 0.0, dmax = 0.0;
    double c[3] = {0, 0, 0};
    for (int64_t i = 0; i < n_nodes; ++i)
        for (int d = 0; d < 3; ++d) c[d] += nodes[3 * i + d] / (double)n_nodes;
    double rb = 0.0;
    for (int64_t i = 0; i < n_nodes; ++i) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += (nodes[3 * i + d] - c[d]) * (nodes[3 * i + d] - c[d]);
        rb = std::max(rb, std::sqrt(s));
    }
    static const int tri[8][3] = {{0, 1, 4}, {0, 4, 3}, {1, 2, 5}, {1, 5, 4}, {3, 4, 7}, {3, 7, 6}, {4, 5, 8}, {4, 8, 7}};
    for (int64_t f = 0; f < n_face; ++f) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = 0; k < 9; ++k)
            for (int d = 0; d < 3; ++d) {
                double v = nodes[3 * (int64_t)conn[f * 9 + k] + d];
                lo[d] = std::min(lo[d], v);
                hi[d] = std::max(hi[d], v);
            }
        dmax = std::max(dmax, std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                        (hi[2] - lo[2]) * (hi[2] - lo[2])));
        for (auto &t : tri) {
            const double *A = nodes + 3 * (int64_t)conn[f * 9 + t[0]];
            const double *B = nodes + 3 * (int64_t)conn[f * 9 + t[1]];
            const double *C = nodes + 3 * (int64_t)conn[f * 9 + t[2]];
            vol += (A[0] * (B[1] * C[2] - B[2] * C[1]) - A[1] * (B[0] * C[2] - B[2] * C[0]) +
                    A[2] * (B[0] * C[1] - B[1] * C[0])) / 6.0;
        }
    }
    if (!(vol > 0.0)) {
        set_error("oc_register_cut_surface: enclosed volume is not positive (inward orientation?)");
        return OC_EGEOM;
    }
    auto s = std::make_unique<Surf>();
    s->n_face = n_face;
    s->n_nodes = n_nodes;
    s->kind = kind;
    s->dmax = f32_up(dmax);
    // bins per axis: edge about twice the largest face box diagonal (a face
    // then meets at most 8 bins, mostly 1 or 2); finer bins measured slower
    // on the dimpled and batch workloads (more bins per element range)
    int nb = (int)std::ceil(rb / std::max(dmax, 1e-30)) + 1;
    nb = std::max(1, std::min(nb, 160));
    if (ctx->surf_bins > 0) nb = std::min(nb, ctx->surf_bins);
    s->nb_auto = nb;
    // a tuned factor for the surface's size class (face-count octave)
    int oct = 0;
    while (oct < 62 && (int64_t(2) << oct) <= n_face) ++oct;
    for (auto &bf : ctx->bin_factor)
        if (bf.first == oct) nb = std::max(1, (int)std::lround(nb * bf.second));
    s->nb_max = nb;
    for (int d = 0; d < 3; ++d) s->first[d] = nodes[d];
    for (int64_t i = 0; i < n_nodes; ++i)
        s->rmax = std::max(s->rmax, std::sqrt(nodes[3 * i] * nodes[3 * i] + nodes[3 * i + 1] * nodes[3 * i + 1] +
                                              nodes[3 * i + 2] * nodes[3 * i + 2]));
    std::vector<double> soa((size_t)n_nodes * 3);
    for (int64_t i = 0; i < n_nodes; ++i)
        for (int d = 0; d < 3; ++d) soa[(size_t)(d * n_nodes + i)] = nodes[3 * i + d];
    oc_status st = OC_OK;
    auto fail = [&](oc_status e) {
        dev_free_all(ctx, s->owned);
        return e;
    };
    if ((st = upload(ctx, s->owned, soa.data(), soa.size(), &s->nodes)) != OC_OK) return fail(st);
    if ((st = upload(ctx, s->owned, conn, (size_t)n_face * 9, &s->conn)) != OC_OK) return fail(st);
    ctx->surfs.push_back(std::move(s));
    *surf_id = (int32_t)ctx->surfs.size() - 1;
    return OC_OK;
}

static oc_status get_grid(oc_ctx *ctx, int32_t id, Grid **g)
{
    if (id < 0 || id >= (int32_t)ctx->grids.size() || !ctx->grids[id]) {
        set_error("unknown grid id " + std::to_string(id));
        return OC_ENOTFOUND;
    }
    *g = ctx->grids[id].get();
    return OC_OK;
}

static oc_status collect_surfs(oc_ctx *ctx, const int32_t *surf_ids, int32_t n_surf, std::vector<Surf *> &ss)
{
    for (int k = 0; k < n_surf; ++k) {
        if (surf_ids[k] < 0 || surf_ids[k] >= (int32_t)ctx->surfs.size() || !ctx->surfs[surf_ids[k]]) {
            set_error("unknown surface id " + std::to_string(surf_ids[k]));
            return OC_ENOTFOUND;
        }
        ss.push_back(ctx->surfs[surf_ids[k]].get());
    }
    return OC_OK;
}

static oc_status read_cut_info(oc_slot *sl, oc_cut_info *info)
{
    OC_TRY(cut_stats_run(sl));
    CutCounters c;
    OC_HIP(hipMemcpyAsync(&c, sl->counters, sizeof c, hipMemcpyDeviceToHost, sl->stream));
    OC_HIP(hipStreamSynchronize(sl->stream));
    info->n_elem = sl->last_n_elem;
    info->n_inbox = sl->last_n_cut > 0 ? c.n_inbox : 0;
    info->n_near = c.n_near;
    info->n_far = c.n_far;
    info->n_hit = c.n_hit;
    info->n_hole = c.n_hole;
    info->n_cand_pairs = (int64_t)c.n_cand_pairs;
    info->n_side = c.n_side;
    return OC_OK;
}

static oc_status read_donor_info(oc_slot *sl, oc_donor_info *info)
{
    OC_TRY(donor_stats_run(sl));
    DonorCounters c;
    OC_HIP(hipMemcpyAsync(&c, sl->dcounters, sizeof c, hipMemcpyDeviceToHost, sl->stream));
    OC_HIP(hipStreamSynchronize(sl->stream));
    info->n_points = (int64_t)c.n_points;
    info->n_newton = (int64_t)c.n_newton;
    info->n_iter = (int64_t)c.n_iter;
    info->n_orphan = (int64_t)c.n_orphan;
    info->n_overflow = (int64_t)c.n_overflow;
    return OC_OK;
}

static bool aligned4(const void *p) { return ((uintptr_t)p & 3) == 0; }

// The cut of oc_cut_multi / oc_cut_posed: surfaces at poses in the grid's
// frame, or (grid_pose given) both in the world frame, composed here as
// inverse(grid pose) after the surface pose.  A host iblank_out is written
// through the staging area.
static oc_status cut_multi_posed(oc_ctx *ctx, int32_t grid_id, const double *grid_pose, const int32_t *surf_ids,
                                 const double *poses, int32_t n_surf, int8_t *iblank_out)
{
    if (!ctx || !iblank_out || n_surf < 0 || n_surf > kPoseSlots - 2 || (n_surf > 0 && (!surf_ids || !poses))) {
        set_error("oc_cut: invalid arguments");
        return OC_EINVAL;
    }
    for (int k = 0; k < n_surf; ++k)
        if (!pose_finite(poses + 12 * k)) {
            set_error("oc_cut: non-finite pose");
            return OC_EINVAL;
        }
    if (grid_pose && !pose_finite(grid_pose)) {
        set_error("oc_cut_posed: non-finite grid pose");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    const bool host_out = !device_memory(iblank_out);
    if (!host_out && !aligned4(iblank_out)) {
        set_error("oc_cut: iblank_out must be 4-byte aligned");
        return OC_EINVAL;
    }
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, surf_ids, n_surf, ss));
    std::vector<double> rel;
    if (grid_pose && n_surf > 0) {
        rel.resize((size_t)n_surf * 12);
        for (int k = 0; k < n_surf; ++k) pose_relative(grid_pose, poses + 12 * k, rel.data() + 12 * k);
        poses = rel.data();
    }
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, 0, poses, n_surf));
    int8_t *dst = iblank_out;
    if (host_out) {
        char *base;
        OC_TRY(stage_reserve(ctx, (size_t)g->n_elem, &base));
        dst = reinterpret_cast<int8_t *>(base);
    }
    CutReq q;
    q.g = g;
    q.n_surf = n_surf;
    q.surfs = ss.data();
    q.poses = sl->poses;
    q.iblank = dst;
    OC_TRY(cut_batch_run(sl, &q, 1));
    if (host_out) {
        OC_HIP(hipMemcpyAsync(iblank_out, dst, (size_t)g->n_elem, hipMemcpyDeviceToHost, sl->stream));
        OC_HIP(hipStreamSynchronize(sl->stream));
    }
    return OC_OK;
}

oc_status oc_cut_multi(oc_ctx *ctx, int32_t grid_id, const int32_t *surf_ids, const double *poses, int32_t n_surf,
                       int8_t *iblank_out)
{
    return cut_multi_posed(ctx, grid_id, nullptr, surf_ids, poses, n_surf, iblank_out);
}

oc_status oc_cut_posed(oc_ctx *ctx, int32_t grid_id, const double grid_pose[12], const int32_t *surf_ids,
                       const double *poses, int32_t n_surf, int8_t *iblank_out)
{
    if (!grid_pose) {
        set_error("oc_cut_posed: null grid pose");
        return OC_EINVAL;
    }
    return cut_multi_posed(ctx, grid_id, grid_pose, surf_ids, poses, n_surf, iblank_out);
}

// Validates a batch and resolves its ids; poses of request r start at
// pose_base[r] (device).
}  // extern "C"

namespace oc {

oc_status collect_cut_reqs(oc_ctx *ctx, const oc_cut_req *reqs, int32_t n_req, std::vector<CutReq> &out,
                          std::vector<std::vector<Surf *>> &surfs, bool need_outputs)
{
    if (n_req < 0 || (n_req > 0 && !reqs)) {
        set_error("cut batch: invalid arguments");
        return OC_EINVAL;
    }
    out.assign((size_t)n_req, CutReq{});
    surfs.assign((size_t)n_req, {});
    for (int r = 0; r < n_req; ++r) {
        const oc_cut_req &q = reqs[r];
        if (q.n_surf < 0 || (q.n_surf > 0 && !q.surf_ids) ||
            (need_outputs && (!q.iblank_out || !aligned4(q.iblank_out) || (q.n_surf > 0 && !q.poses)))) {
            set_error("cut batch: invalid request " + std::to_string(r));
            return OC_EINVAL;
        }
        OC_TRY(get_grid(ctx, q.grid_id, &out[r].g));
        OC_TRY(collect_surfs(ctx, q.surf_ids, q.n_surf, surfs[r]));
        out[r].n_surf = q.n_surf;
        out[r].surfs = surfs[r].data();
        out[r].iblank = q.iblank_out;
    }
    return OC_OK;
}

}  // namespace oc

extern "C" {

oc_status oc_cut_batch(oc_ctx *ctx, const oc_cut_req *reqs, int32_t n_req)
{
    if (!ctx) {
        set_error("oc_cut_batch: null context");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    std::vector<CutReq> rq;
    std::vector<std::vector<Surf *>> ss;
    OC_TRY(collect_cut_reqs(ctx, reqs, n_req, rq, ss, true));
    int n_pose = 0;
    for (int r = 0; r < n_req; ++r) n_pose += reqs[r].n_surf;
    if (n_pose > kPoseSlots - 2) {
        set_error("oc_cut_batch: more than " + std::to_string(kPoseSlots - 2) + " poses");
        return OC_EINVAL;
    }
    std::vector<double> P;
    P.reserve((size_t)n_pose * 12);
    for (int r = 0; r < n_req; ++r)
        for (int k = 0; k < reqs[r].n_surf; ++k) {
            if (!pose_finite(reqs[r].poses + 12 * k)) {
                set_error("oc_cut_batch: non-finite pose");
                return OC_EINVAL;
            }
            P.insert(P.end(), reqs[r].poses + 12 * k, reqs[r].poses + 12 * k + 12);
        }
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, 0, P.data(), n_pose));
    int p0 = 0;
    for (int r = 0; r < n_req; ++r) {
        rq[r].poses = sl->poses + p0;
        p0 += reqs[r].n_surf;
    }
    return cut_batch_run(sl, rq.data(), n_req);
}

oc_status oc_cut(oc_ctx *ctx, int32_t grid_id, int32_t surf_id, const double pose[12], int8_t *iblank_out)
{
    return oc_cut_multi(ctx, grid_id, &surf_id, pose, 1, iblank_out);
}

oc_status oc_last_cut_info(oc_ctx *ctx, oc_cut_info *info)
{
    if (!ctx || !info) {
        set_error("oc_last_cut_info: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    return read_cut_info(ctx->dflt, info);
}

oc_status oc_last_donor_info(oc_ctx *ctx, oc_donor_info *info)
{
    if (!ctx || !info) {
        set_error("oc_last_donor_info: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    return read_donor_info(ctx->dflt, info);
}

oc_status oc_fringe_points(oc_ctx *ctx, int32_t grid_id, const double grid_pose[12], const int8_t *iblank,
                           double *points_out, int64_t cap, int64_t *n_out, int32_t *src_out)
{
    if (!ctx || !iblank || !n_out || cap < 0 || (cap > 0 && !points_out) || !grid_pose || !pose_finite(grid_pose)) {
        set_error("oc_fringe_points: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, kPoseSlots - 2, grid_pose, 1));
    // host arrays through the staging area: iblank in, points and sources out
    const bool h_ib = !device_memory(iblank), h_pts = cap > 0 && !device_memory(points_out),
               h_src = src_out && cap > 0 && !device_memory(src_out);
    const int8_t *ib = iblank;
    double *pts = points_out;
    int32_t *src = src_out;
    if (h_ib || h_pts || h_src) {
        const size_t o_pts = (size_t)(g->n_elem + 255) / 256 * 256, o_src = o_pts + sizeof(double) * 3 * (size_t)cap;
        char *base;
        OC_TRY(stage_reserve(ctx, o_src + sizeof(int32_t) * (size_t)cap, &base));
        if (h_ib) {
            OC_HIP(hipMemcpyAsync(base, iblank, (size_t)g->n_elem, hipMemcpyHostToDevice, sl->stream));
            ib = reinterpret_cast<const int8_t *>(base);
        }
        if (h_pts) pts = reinterpret_cast<double *>(base + o_pts);
        if (h_src) src = reinterpret_cast<int32_t *>(base + o_src);
    }
    const oc_status r = fringe_points_run(sl, *g, sl->poses + kPoseSlots - 2, ib, pts, cap, nullptr, n_out, src);
    if (r != OC_OK && r != OC_ECAPACITY) return r;
    const int64_t n = std::min(*n_out, cap);
    if (h_pts && n > 0)
        OC_HIP(hipMemcpyAsync(points_out, pts, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToHost, sl->stream));
    if (h_src && n > 0)
        OC_HIP(hipMemcpyAsync(src_out, src, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, sl->stream));
    if (h_ib || h_pts || h_src) OC_HIP(hipStreamSynchronize(sl->stream));
    if (r != OC_OK) set_error("oc_fringe_points: capacity " + std::to_string(cap) + " < " + std::to_string(*n_out) +
                              " points");
    return r;
}

oc_status oc_donor_search(oc_ctx *ctx, int32_t donor_grid_id, const double grid_pose[12], const double *points,
                          int64_t n, int32_t *donor_out, double *ref_out)
{
    if (!ctx || n < 0 || (n > 0 && (!points || !donor_out || !ref_out)) || !pose_finite(grid_pose)) {
        set_error("oc_donor_search: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, donor_grid_id, &g));
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, kPoseSlots - 1, grid_pose, 1));
    if (n == 0) return donor_run(sl, *g, sl->poses + kPoseSlots - 1, points, n, nullptr, donor_out, ref_out);
    // host arrays through the staging area: points in, donors and xi out
    const bool h_p = !device_memory(points), h_d = !device_memory(donor_out), h_r = !device_memory(ref_out);
    const double *P = points;
    int32_t *D = donor_out;
    double *X = ref_out;
    if (h_p || h_d || h_r) {
        const size_t b3 = sizeof(double) * 3 * (size_t)n, o_x = b3, o_d = 2 * b3;
        char *base;
        OC_TRY(stage_reserve(ctx, o_d + sizeof(int32_t) * (size_t)n, &base));
        if (h_p) {
            OC_HIP(hipMemcpyAsync(base, points, b3, hipMemcpyHostToDevice, sl->stream));
            P = reinterpret_cast<const double *>(base);
        }
        if (h_r) X = reinterpret_cast<double *>(base + o_x);
        if (h_d) D = reinterpret_cast<int32_t *>(base + o_d);
    }
    OC_TRY(donor_run(sl, *g, sl->poses + kPoseSlots - 1, P, n, nullptr, D, X));
    if (h_r) OC_HIP(hipMemcpyAsync(ref_out, X, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToHost, sl->stream));
    if (h_d) OC_HIP(hipMemcpyAsync(donor_out, D, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, sl->stream));
    if (h_p || h_d || h_r) OC_HIP(hipStreamSynchronize(sl->stream));
    return OC_OK;
}

oc_status oc_donor_search_noalloc(oc_ctx *ctx, int32_t donor_grid_id, const double grid_pose[12],
                                  const double *points, int64_t n, int32_t *donor_out, double *ref_out)
{
    if (!ctx || n < 0 || (n > 0 && (!points || !donor_out || !ref_out)) || !pose_finite(grid_pose)) {
        set_error("oc_donor_search_noalloc: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, donor_grid_id, &g));
    return donor_noalloc_run(ctx, *g, grid_pose, points, n, donor_out, ref_out);
}

oc_status oc_noalloc_max_points(int64_t *n)
{
    if (!n) {
        set_error("oc_noalloc_max_points: null output");
        return OC_EINVAL;
    }
    *n = noalloc_max_points();
    return OC_OK;
}

// Bound on the distance any point of surface s travels between two poses:
// rotation angle of R_b R_a^T times the largest node radius, plus the
// distance between the two offsets (a screw motion between the poses).
static double sweep_bound(const Surf &s, const double *a, const double *b)
{
    double tr = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) tr += b[3 * i + k] * a[3 * i + k];   // trace(R_b R_a^T)
    const double c = std::max(-1.0, std::min(1.0, 0.5 * (tr - 1.0)));
    const double th = std::acos(c);
    const double dt = std::sqrt((b[9] - a[9]) * (b[9] - a[9]) + (b[10] - a[10]) * (b[10] - a[10]) +
                                (b[11] - a[11]) * (b[11] - a[11]));
    return (th * s.rmax + dt) * (1.0 + 1e-9) + 1e-12;
}

oc_status oc_sweep_bound(oc_ctx *ctx, int32_t surf_id, const double pose_a[12], const double pose_b[12], double *out)
{
    if (!ctx || !out || !pose_finite(pose_a) || !pose_finite(pose_b)) {
        set_error("oc_sweep_bound: invalid arguments");
        return OC_EINVAL;
    }
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, &surf_id, 1, ss));
    *out = sweep_bound(*ss[0], pose_a, pose_b);
    return OC_OK;
}

oc_status oc_cut_warm(oc_ctx *ctx, int32_t grid_id, int32_t surf_id, const double pose[12], const double prev_pose[12],
                      const int8_t *prev_iblank, int8_t *iblank_out)
{
    if (!ctx || !iblank_out || !prev_iblank || !aligned4(iblank_out) || !pose_finite(pose) || !pose_finite(prev_pose) ||
        prev_iblank == iblank_out) {
        set_error("oc_cut_warm: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, &surf_id, 1, ss));
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, 0, pose, 1));
    CutReq q;
    q.g = g;
    q.n_surf = 1;
    q.surfs = ss.data();
    q.poses = sl->poses;
    q.iblank = iblank_out;
    q.prev = prev_iblank;
    q.sweep = sweep_bound(*ss[0], prev_pose, pose);
    return cut_batch_run(sl, &q, 1);
}

oc_status oc_unblank(oc_ctx *ctx, int32_t grid_id, const int32_t *surf_ids, int32_t n_surf, const double *poses_t,
                     const double *poses_tp, const int8_t *prev_iblank, int8_t *iblank_out, int32_t *unblank_out,
                     int64_t cap, int64_t *n_unblank)
{
    if (!ctx || !prev_iblank || !iblank_out || !n_unblank || cap < 0 || (cap > 0 && !unblank_out) || n_surf < 0 ||
        2 * n_surf > kPoseSlots - 2 || (n_surf > 0 && (!surf_ids || !poses_t || !poses_tp)) ||
        prev_iblank == iblank_out) {
        set_error("oc_unblank: invalid arguments");
        return OC_EINVAL;
    }
    for (int k = 0; k < n_surf; ++k)
        if (!pose_finite(poses_t + 12 * k) || !pose_finite(poses_tp + 12 * k)) {
            set_error("oc_unblank: non-finite pose");
            return OC_EINVAL;
        }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, surf_ids, n_surf, ss));
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, 0, poses_t, n_surf));
    OC_TRY(set_poses(sl, n_surf, poses_tp, n_surf));
    return unblank_run(sl, *g, ss.data(), n_surf, sl->poses, sl->poses + n_surf, prev_iblank, iblank_out,
                       unblank_out, cap, nullptr, n_unblank);
}

oc_status oc_element_points(oc_ctx *ctx, int32_t grid_id, const double grid_pose[12], const int32_t *elems, int64_t n,
                            double *points_out, int32_t *src_out)
{
    if (!ctx || n < 0 || (n > 0 && (!elems || !points_out)) || !pose_finite(grid_pose) || n > INT32_MAX / 27) {
        set_error("oc_element_points: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    if (n == 0) return OC_OK;
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, kPoseSlots - 2, grid_pose, 1));
    const int32_t n32 = (int32_t)n;
    OC_TRY(put_bytes(sl, sl->scalar + 2, &n32, sizeof n32));
    return element_points_run(sl, *g, sl->poses + kPoseSlots - 2, elems, sl->scalar + 2, points_out, 27 * n,
                              nullptr, src_out);
}

oc_status oc_cut_filtered(oc_ctx *ctx, int32_t grid_id, const int32_t *surf_ids, const double *poses, int32_t n_surf,
                          int32_t nf1, int32_t nf2, int8_t *iblank_out, int64_t *n_listed)
{
    if (!ctx || !iblank_out || n_surf < 0 || n_surf > kPoseSlots - 2 || (n_surf > 0 && (!surf_ids || !poses)) ||
        nf1 < 1 || nf1 > 32 || nf2 < 1 || nf2 > 16 || nf2 > nf1) {
        set_error("oc_cut_filtered: invalid arguments (1 <= nf2 <= nf1, nf1 <= 32, nf2 <= 16)");
        return OC_EINVAL;
    }
    for (int k = 0; k < n_surf; ++k)
        if (!pose_finite(poses + 12 * k)) {
            set_error("oc_cut_filtered: non-finite pose");
            return OC_EINVAL;
        }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, surf_ids, n_surf, ss));
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, 0, poses, n_surf));
    return filtered_cut_run(sl, *g, ss.data(), sl->poses, n_surf, nf1, nf2, iblank_out, n_listed);
}

oc_status oc_cut_refined(oc_ctx *ctx, int32_t grid_id, const int32_t *surf_ids, const double *poses, int32_t n_surf,
                         int32_t k, int8_t *iblank_out, int64_t *n_near)
{
    if (!ctx || !iblank_out || n_surf < 1 || n_surf > kPoseSlots - 2 || !surf_ids || !poses || k < 1 || k > 8) {
        set_error("oc_cut_refined: invalid arguments (1 <= k <= 8, at least one surface)");
        return OC_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(iblank_out) % 4) {
        set_error("oc_cut_refined: iblank_out must be 4-byte aligned");
        return OC_EINVAL;
    }
    for (int i = 0; i < n_surf; ++i)
        if (!pose_finite(poses + 12 * i)) {
            set_error("oc_cut_refined: non-finite pose");
            return OC_EINVAL;
        }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, surf_ids, n_surf, ss));
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, 0, poses, n_surf));
    return refined_cut_run(sl, *g, ss.data(), sl->poses, n_surf, k, iblank_out, n_near);
}

// ------------------------------------------------- artificial boundary --
static oc_status get_nodes1d(const double *z, int32_t m, Nodes1D *out, const char *who)
{
    if (!z || m < 1 || m > kMaxNodes1D) {
        set_error(std::string(who) + ": need 1 to " + std::to_string(kMaxNodes1D) + " one-dimensional nodes");
        return OC_EINVAL;
    }
    for (int i = 0; i < kMaxNodes1D; ++i) out->z[i] = 0.0;
    for (int i = 0; i < m; ++i) {
        if (!std::isfinite(z[i])) {
            set_error(std::string(who) + ": non-finite node");
            return OC_EINVAL;
        }
        for (int j = 0; j < i; ++j)
            if (z[j] == z[i]) {
                set_error(std::string(who) + ": repeated node");
                return OC_EINVAL;
            }
        out->z[i] = z[i];
    }
    out->m = m;
    return OC_OK;
}

oc_status oc_ab_faces(oc_ctx *ctx, int32_t grid_id, const int8_t *iblank, int32_t *faces_out, int64_t cap,
                      int64_t *n_out)
{
    if (!ctx || !iblank || !n_out || cap < 0 || (cap > 0 && !faces_out)) {
        set_error("oc_ab_faces: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    oc_slot *sl = ctx->dflt;
    const int32_t *total = nullptr;
    OC_TRY(ab_faces_run(sl, *g, iblank, faces_out, cap, &total));
    int32_t n = 0;
    OC_HIP(hipMemcpyAsync(&n, total, sizeof(int32_t), hipMemcpyDeviceToHost, sl->stream));
    OC_HIP(hipStreamSynchronize(sl->stream));
    *n_out = n;
    if (n > cap) {
        set_error("oc_ab_faces: capacity " + std::to_string(cap) + " < " + std::to_string(n) + " faces");
        return OC_ECAPACITY;
    }
    return OC_OK;
}

oc_status oc_face_points(oc_ctx *ctx, int32_t grid_id, const double grid_pose[12], const int32_t *faces, int64_t n,
                         const double *nodes1d, int32_t m, double *points_out, int32_t *src_out)
{
    Nodes1D z;
    OC_TRY(get_nodes1d(nodes1d, m, &z, "oc_face_points"));
    if (!ctx || n < 0 || (n > 0 && (!faces || !points_out)) || !pose_finite(grid_pose) || n > INT32_MAX / (m * m)) {
        set_error("oc_face_points: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    if (n == 0) return OC_OK;
    oc_slot *sl = ctx->dflt;
    OC_TRY(set_poses(sl, kPoseSlots - 2, grid_pose, 1));
    return face_points_run(sl, *g, sl->poses + kPoseSlots - 2, faces, nullptr, n, z, points_out, n * m * m, nullptr,
                           src_out);
}

oc_status oc_interp_weights(oc_ctx *ctx, const int32_t *donors, const double *ref, int64_t n, const double *nodes1d,
                            int32_t m, double *weights_out)
{
    Nodes1D z;
    OC_TRY(get_nodes1d(nodes1d, m, &z, "oc_interp_weights"));
    if (!ctx || n < 0 || (n > 0 && (!donors || !ref || !weights_out)) || n > ((int64_t)1 << 40) / (m * m * m)) {
        set_error("oc_interp_weights: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    if (n == 0) return OC_OK;
    return weights_run(ctx->dflt, donors, ref, nullptr, n, z, weights_out);
}

// ------------------------------------------------------------- slot API --
}  // extern "C"

namespace oc {

oc_status slot_make(oc_ctx *ctx, const CutCaps &cc, int64_t ne, int64_t points_cap, hipStream_t stream,
                    oc_slot **out)
{
    oc_slot *sl = new oc_slot();
    sl->stream = stream;
    oc_status st = slot_init(ctx, sl, false);
    if (st == OC_OK) st = slot_alloc_lists(sl, std::max<int64_t>(ne, 1));
    if (st == OC_OK) st = slot_alloc_cut(sl, cc);
    if (st == OC_OK && points_cap > 0) st = slot_alloc_points(sl, points_cap);
    if (st != OC_OK) {
        slot_free(sl);
        delete sl;
        return st;
    }
    *out = sl;
    return OC_OK;
}

}  // namespace oc

extern "C" {

oc_status oc_slot_create(oc_ctx *ctx, const int32_t *grid_ids, int32_t n_grids, const int32_t *surf_ids,
                         int32_t n_surfs, int64_t points_cap, oc_slot **out)
{
    if (!ctx || !out || n_grids < 0 || n_surfs < 0 || (n_grids && !grid_ids) || (n_surfs && !surf_ids) ||
        points_cap < 0) {
        set_error("oc_slot_create: invalid arguments");
        return OC_EINVAL;
    }
    *out = nullptr;
    OC_HIP(hipSetDevice(ctx->device));
    int64_t ne = 1;
    for (int k = 0; k < n_grids; ++k) {
        Grid *g;
        OC_TRY(get_grid(ctx, grid_ids[k], &g));
        ne = std::max(ne, g->n_elem);
    }
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, surf_ids, n_surfs, ss));
    // any cut of one listed grid by any of the listed surfaces
    CutCaps cc;
    cc.outs = 1;
    cc.cuts = n_surfs;
    cc.elem_inst = ne * n_surfs;
    for (auto s : ss) {
        cc.faces += s->n_face;
        cc.bins += (int64_t)s->nb_max * s->nb_max * s->nb_max;
    }
    oc_slot *sl = new oc_slot();
    oc_status st = slot_init(ctx, sl, false);
    if (st == OC_OK) st = slot_alloc_lists(sl, ne);
    if (st == OC_OK) st = slot_alloc_cut(sl, cc);
    if (st == OC_OK && points_cap > 0) st = slot_alloc_points(sl, points_cap);
    if (st != OC_OK) {
        slot_free(sl);
        delete sl;
        return st;
    }
    ctx->slots.push_back(sl);
    *out = sl;
    return OC_OK;
}

oc_status oc_slot_destroy(oc_slot *sl)
{
    if (!sl) return OC_OK;
    oc_ctx *ctx = sl->ctx;
    (void)hipSetDevice(ctx->device);
    for (size_t k = 0; k < ctx->slots.size(); ++k)
        if (ctx->slots[k] == sl) {
            ctx->slots.erase(ctx->slots.begin() + k);
            break;
        }
    slot_free(sl);
    delete sl;
    return OC_OK;
}

oc_status oc_slot_set_stream(oc_slot *sl, void *hip_stream)
{
    if (!sl) {
        set_error("oc_slot_set_stream: null slot");
        return OC_EINVAL;
    }
    sl->stream = (hipStream_t)hip_stream;
    return OC_OK;
}

}  // extern "C"

namespace oc {

int64_t slot_bytes(const oc_slot *sl)
{
    int64_t b = 0;
    for (auto &d : sl->owned) b += (int64_t)d.bytes;
    for (auto &d : sl->cut_owned) b += (int64_t)d.bytes;
    return b;
}

}  // namespace oc

extern "C" {

oc_status oc_slot_bytes(oc_slot *sl, int64_t *bytes)
{
    if (!sl || !bytes) {
        set_error("oc_slot_bytes: invalid arguments");
        return OC_EINVAL;
    }
    *bytes = slot_bytes(sl);
    return OC_OK;
}

oc_status oc_slot_cut(oc_slot *sl, int32_t grid_id, const int32_t *surf_ids, const double *poses_dev, int32_t n_surf,
                      int8_t *iblank_out)
{
    if (!sl || !iblank_out || n_surf < 0 || (n_surf > 0 && (!surf_ids || !poses_dev)) || !aligned4(iblank_out) ||
        ((uintptr_t)poses_dev & 7)) {
        set_error("oc_slot_cut: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, surf_ids, n_surf, ss));
    CutReq q;
    q.g = g;
    q.n_surf = n_surf;
    q.surfs = ss.data();
    q.poses = reinterpret_cast<const Pose *>(poses_dev);
    q.iblank = iblank_out;
    return cut_batch_run(sl, &q, 1);
}

oc_status oc_slot_cut_posed(oc_slot *sl, int32_t grid_id, const double *grid_pose_dev, const int32_t *surf_ids,
                            const double *poses_dev, int32_t n_surf, int8_t *iblank_out)
{
    if (!sl || !iblank_out || !grid_pose_dev || n_surf < 0 || n_surf > kPoseSlots ||
        (n_surf > 0 && (!surf_ids || !poses_dev)) || !aligned4(iblank_out) || ((uintptr_t)poses_dev & 7) ||
        ((uintptr_t)grid_pose_dev & 7)) {
        set_error("oc_slot_cut_posed: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, surf_ids, n_surf, ss));
    OC_TRY(compose_poses_run(sl, grid_pose_dev, poses_dev, n_surf, sl->poses));
    CutReq q;
    q.g = g;
    q.n_surf = n_surf;
    q.surfs = ss.data();
    q.poses = sl->poses;
    q.iblank = iblank_out;
    return cut_batch_run(sl, &q, 1);
}

oc_status oc_slot_cut_batch(oc_slot *sl, const oc_cut_req *reqs, int32_t n_req)
{
    if (!sl) {
        set_error("oc_slot_cut_batch: null slot");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    std::vector<CutReq> rq;
    std::vector<std::vector<Surf *>> ss;
    OC_TRY(collect_cut_reqs(ctx, reqs, n_req, rq, ss, true));
    for (int r = 0; r < n_req; ++r) {
        if ((uintptr_t)reqs[r].poses & 7) {
            set_error("oc_slot_cut_batch: poses must be 8-byte aligned");
            return OC_EINVAL;
        }
        rq[r].poses = reinterpret_cast<const Pose *>(reqs[r].poses);
    }
    return cut_batch_run(sl, rq.data(), n_req);
}

oc_status oc_slot_create_batch(oc_ctx *ctx, const oc_cut_req *reqs, int32_t n_req, int64_t points_cap,
                               oc_slot **out)
{
    if (!ctx || !out || points_cap < 0) {
        set_error("oc_slot_create_batch: invalid arguments");
        return OC_EINVAL;
    }
    *out = nullptr;
    OC_HIP(hipSetDevice(ctx->device));
    std::vector<CutReq> rq;
    std::vector<std::vector<Surf *>> ss;
    OC_TRY(collect_cut_reqs(ctx, reqs, n_req, rq, ss, false));
    oc_slot *sl;
    int64_t ne = 1;
    for (auto &q : rq) ne = std::max(ne, q.g->n_elem);
    OC_TRY(slot_make(ctx, cut_caps(rq.data(), n_req), ne, points_cap, nullptr, &sl));
    ctx->slots.push_back(sl);
    *out = sl;
    return OC_OK;
}

oc_status oc_slot_cut_warm(oc_slot *sl, int32_t grid_id, int32_t surf_id, const double *pose_dev, double sweep,
                           const int8_t *prev_iblank, int8_t *iblank_out)
{
    if (!sl || !pose_dev || !prev_iblank || !iblank_out || !aligned4(iblank_out) || ((uintptr_t)pose_dev & 7) ||
        !(sweep >= 0.0) || prev_iblank == iblank_out) {
        set_error("oc_slot_cut_warm: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, &surf_id, 1, ss));
    CutReq q;
    q.g = g;
    q.n_surf = 1;
    q.surfs = ss.data();
    q.poses = reinterpret_cast<const Pose *>(pose_dev);
    q.iblank = iblank_out;
    q.prev = prev_iblank;
    q.sweep = sweep;
    return cut_batch_run(sl, &q, 1);
}

oc_status oc_slot_fringe_points(oc_slot *sl, int32_t grid_id, const double *pose_dev, const int8_t *iblank,
                                double *points_out, int64_t cap, int32_t *n_dev, int32_t *src_out)
{
    if (!sl || !pose_dev || !iblank || !n_dev || cap < 0 || (cap > 0 && !points_out) || ((uintptr_t)pose_dev & 7)) {
        set_error("oc_slot_fringe_points: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    return fringe_points_run(sl, *g, reinterpret_cast<const Pose *>(pose_dev), iblank, points_out, cap, n_dev,
                             nullptr, src_out);
}

oc_status oc_slot_donor_search(oc_slot *sl, int32_t donor_grid_id, const double *pose_dev, const double *points,
                               int64_t cap, const int32_t *n_dev, int32_t *donor_out, double *ref_out)
{
    if (!sl || !pose_dev || cap < 0 || (cap > 0 && (!points || !donor_out || !ref_out)) ||
        ((uintptr_t)pose_dev & 7)) {
        set_error("oc_slot_donor_search: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, donor_grid_id, &g));
    return donor_run(sl, *g, reinterpret_cast<const Pose *>(pose_dev), points, cap, n_dev, donor_out, ref_out);
}

oc_status oc_slot_unblank(oc_slot *sl, int32_t grid_id, const int32_t *surf_ids, int32_t n_surf, const double *poses_dev,
                          const int8_t *prev_iblank, int8_t *iblank_out, int32_t *unblank_out, int64_t cap,
                          int32_t *n_dev)
{
    if (!sl || !prev_iblank || !iblank_out || !n_dev || cap < 0 || (cap > 0 && !unblank_out) || n_surf < 0 ||
        (n_surf > 0 && (!surf_ids || !poses_dev)) || ((uintptr_t)poses_dev & 7) || prev_iblank == iblank_out) {
        set_error("oc_slot_unblank: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    std::vector<Surf *> ss;
    OC_TRY(collect_surfs(ctx, surf_ids, n_surf, ss));
    const Pose *P = reinterpret_cast<const Pose *>(poses_dev);
    return unblank_run(sl, *g, ss.data(), n_surf, P, P + n_surf, prev_iblank, iblank_out, unblank_out, cap, n_dev,
                       nullptr);
}

oc_status oc_slot_element_points(oc_slot *sl, int32_t grid_id, const double *pose_dev, const int32_t *elems,
                                 const int32_t *n_dev, int64_t cap, double *points_out, int32_t *n_points_dev,
                                 int32_t *src_out)
{
    if (!sl || !pose_dev || ((uintptr_t)pose_dev & 7) || !n_dev || cap < 0 || (cap > 0 && (!elems || !points_out))) {
        set_error("oc_slot_element_points: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    return element_points_run(sl, *g, reinterpret_cast<const Pose *>(pose_dev), elems, n_dev, points_out, cap,
                              n_points_dev, src_out);
}

oc_status oc_slot_ab_faces(oc_slot *sl, int32_t grid_id, const int8_t *iblank, int32_t *faces_out, int64_t cap,
                           int32_t *n_dev)
{
    if (!sl || !iblank || !n_dev || cap < 0 || (cap > 0 && !faces_out)) {
        set_error("oc_slot_ab_faces: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    const int32_t *total = nullptr;
    OC_TRY(ab_faces_run(sl, *g, iblank, faces_out, cap, &total));
    return copy_count_run(sl, total, n_dev);
}

oc_status oc_slot_face_points(oc_slot *sl, int32_t grid_id, const double *pose_dev, const int32_t *faces,
                              const int32_t *n_faces_dev, int64_t faces_cap, const double *nodes1d, int32_t m,
                              double *points_out, int64_t cap, int32_t *n_points_dev, int32_t *src_out)
{
    Nodes1D z;
    OC_TRY(get_nodes1d(nodes1d, m, &z, "oc_slot_face_points"));
    if (!sl || !pose_dev || ((uintptr_t)pose_dev & 7) || faces_cap < 0 || cap < 0 ||
        (faces_cap > 0 && !faces) || (cap > 0 && !points_out) || faces_cap > INT32_MAX / (m * m)) {
        set_error("oc_slot_face_points: invalid arguments");
        return OC_EINVAL;
    }
    oc_ctx *ctx = sl->ctx;
    OC_HIP(hipSetDevice(ctx->device));
    Grid *g;
    OC_TRY(get_grid(ctx, grid_id, &g));
    return face_points_run(sl, *g, reinterpret_cast<const Pose *>(pose_dev), faces, n_faces_dev, faces_cap, z,
                           points_out, cap, n_points_dev, src_out);
}

oc_status oc_slot_interp_weights(oc_slot *sl, const int32_t *donors, const double *ref, const int32_t *n_dev,
                                 int64_t cap, const double *nodes1d, int32_t m, double *weights_out)
{
    Nodes1D z;
    OC_TRY(get_nodes1d(nodes1d, m, &z, "oc_slot_interp_weights"));
    if (!sl || cap < 0 || (cap > 0 && (!donors || !ref || !weights_out)) || cap > ((int64_t)1 << 40) / (m * m * m)) {
        set_error("oc_slot_interp_weights: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(sl->ctx->device));
    return weights_run(sl, donors, ref, n_dev, cap, z, weights_out);
}

oc_status oc_slot_cut_info(oc_slot *sl, oc_cut_info *info)
{
    if (!sl || !info) {
        set_error("oc_slot_cut_info: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(sl->ctx->device));
    return read_cut_info(sl, info);
}

oc_status oc_slot_donor_info(oc_slot *sl, oc_donor_info *info)
{
    if (!sl || !info) {
        set_error("oc_slot_donor_info: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(sl->ctx->device));
    return read_donor_info(sl, info);
}

oc_status oc_timing(oc_ctx *ctx, int32_t enable)
{
    if (!ctx) {
        set_error("oc_timing: null context");
        return OC_EINVAL;
    }
    OC_HIP(hipDeviceSynchronize());
    ctx->timing = enable != 0;
    ctx->trecs.clear();
    ctx->event_next = 0;
    return OC_OK;
}

oc_status oc_timing_report(oc_ctx *ctx, char *buf, int64_t buf_len)
{
    if (!ctx || !buf || buf_len <= 0) {
        set_error("oc_timing_report: invalid arguments");
        return OC_EINVAL;
    }
    OC_HIP(hipDeviceSynchronize());
    std::map<std::string, std::pair<double, int>> acc;
    for (auto &r : ctx->trecs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        auto &a = acc[r.name];
        a.first += ms;
        a.second += 1;
    }
    std::string js = "{";
    bool firstk = true;
    for (auto &kv : acc) {
        char tmp[256];
        snprintf(tmp, sizeof tmp, "%s\"%s\": [%.9g, %d]", firstk ? "" : ", ", kv.first.c_str(), kv.second.first,
                 kv.second.second);
        js += tmp;
        firstk = false;
    }
    js += "}";
    if ((int64_t)js.size() + 1 > buf_len) {
        set_error("oc_timing_report: buffer too small");
        return OC_ECAPACITY;
    }
    memcpy(buf, js.c_str(), js.size() + 1);
    ctx->trecs.clear();
    ctx->event_next = 0;
    return OC_OK;
}

oc_status oc_tune(oc_ctx *ctx, int32_t knob, int32_t arg, int64_t value, int64_t *applied)
{
    if (!ctx) {
        set_error("oc_tune: null context");
        return OC_EINVAL;
    }
    int64_t v = 0;
    if (value == -1) {   // query: the value in force, nothing changed
        if (knob == OC_TUNE_SURF_BINS) {
            std::vector<Surf *> ss;
            OC_TRY(collect_surfs(ctx, &arg, 1, ss));
            v = ss[0]->nb_max;
        } else if (knob == OC_TUNE_EXACT_WAVES) {
            v = ctx->exact_waves;
        } else if (knob == OC_TUNE_SERVICE_SLOTS) {
            v = ctx->service_slots;
        } else if (knob == OC_TUNE_DONOR_WAVES) {
            v = ctx->donor_waves;
        } else if (knob == OC_TUNE_DONOR_PAIRS) {
            v = ctx->donor_pairs;
        } else if (knob == OC_TUNE_FILTER_BLOCK) {
            v = ctx->filter_block;
        } else if (knob == OC_TUNE_POINT_TILES) {
            v = ctx->point_tiles;
        } else if (knob == OC_TUNE_SIDE_LIST) {
            v = ctx->side_list;
        } else if (knob == OC_TUNE_HBM_BUDGET) {
            v = ctx->budget;
        } else {
            set_error("oc_tune: unknown knob");
            return OC_EINVAL;
        }
        if (applied) *applied = v;
        return OC_OK;
    }
    if (knob == OC_TUNE_SURF_BINS) {
        std::vector<Surf *> ss;
        OC_TRY(collect_surfs(ctx, &arg, 1, ss));
        if (value < 0) {
            set_error("oc_tune: negative bin cap");
            return OC_EINVAL;
        }
        ss[0]->nb_max = value == 0 ? ss[0]->nb_auto : (int)std::max<int64_t>(1, std::min<int64_t>(value, ss[0]->nb_auto));
        v = ss[0]->nb_max;
    } else if (knob == OC_TUNE_EXACT_WAVES) {
        if (value < 0 || value > (1 << 20)) {
            set_error("oc_tune: exact waves out of range");
            return OC_EINVAL;
        }
        ctx->exact_waves = value == 0 ? 8192 : (int)value;
        v = ctx->exact_waves;
    } else if (knob == OC_TUNE_SERVICE_SLOTS) {
        if (value < 0 || value > 64) {
            set_error("oc_tune: service slots out of range");
            return OC_EINVAL;
        }
        ctx->service_slots = value == 0 ? 4 : (int)value;
        v = ctx->service_slots;
    } else if (knob == OC_TUNE_DONOR_WAVES) {
        if (value < 0 || value > (1 << 22)) {
            set_error("oc_tune: donor waves out of range");
            return OC_EINVAL;
        }
        ctx->donor_waves = (int)value;
        v = ctx->donor_waves;
    } else if (knob == OC_TUNE_DONOR_PAIRS) {
        if (value < 0) {
            set_error("oc_tune: negative pair cap");
            return OC_EINVAL;
        }
        ctx->donor_pairs = value;
        v = ctx->donor_pairs;
    } else if (knob == OC_TUNE_FILTER_BLOCK) {
        if (value != 0 && value != 64 && value != 128 && value != 256 && value != 512 && value != 1024) {
            set_error("oc_tune: filter block must be 64, 128, 256, 512 or 1024 threads");
            return OC_EINVAL;
        }
        ctx->filter_block = value == 0 ? 256 : (int)value;
        v = ctx->filter_block;
    } else if (knob == OC_TUNE_POINT_TILES) {
        if (value < 0 || value > 2048) {
            set_error("oc_tune: point tiles out of range (0 .. 2048)");
            return OC_EINVAL;
        }
        ctx->point_tiles = value == 0 ? 2048 : (int)value;
        v = ctx->point_tiles;
    } else if (knob == OC_TUNE_SIDE_LIST) {
        if (value < 0 || value > 64) {
            set_error("oc_tune: side list out of range (0 .. 64)");
            return OC_EINVAL;
        }
        ctx->side_list = value == 0 ? 64 : (int)value;
        v = ctx->side_list;
    } else if (knob == OC_TUNE_HBM_BUDGET) {
        if (value < 0) {
            set_error("oc_tune: negative budget");
            return OC_EINVAL;
        }
        ctx->budget = value;
        v = ctx->budget;
    } else {
        set_error("oc_tune: unknown knob");
        return OC_EINVAL;
    }
    if (applied) *applied = v;
    return OC_OK;
}

oc_status oc_check_word(oc_ctx *ctx, uint32_t *word, int32_t clear, int32_t *checked)
{
    if (!ctx || !word) {
        set_error("oc_check_word: invalid arguments");
        return OC_EINVAL;
    }
#ifdef OC_CHECKED
    if (checked) *checked = 1;
#else
    if (checked) *checked = 0;
#endif
    OC_HIP(hipSetDevice(ctx->device));
    OC_HIP(hipDeviceSynchronize());
    uint32_t *w = reinterpret_cast<uint32_t *>(ctx->dev_scalar) + 8;
    OC_HIP(hipMemcpy(word, w, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (clear) OC_HIP(hipMemset(w, 0, sizeof(uint32_t)));
    return OC_OK;
}

oc_status oc_memory_used(oc_ctx *ctx, int64_t *bytes)
{
    if (!ctx || !bytes) {
        set_error("oc_memory_used: invalid arguments");
        return OC_EINVAL;
    }
    *bytes = ctx->used;
    return OC_OK;
}

}  // extern "C"
