// Cut service: oc_submit queues a cut request and returns a ticket at once,
// oc_wait retires it.  Requests run on service slots (each with its own
// stream), so requests submitted while others are on the device run beside
// them.  A request is admitted when an idle slot covers it or a new slot
// fits in the context's HBM budget; idle slots that do not cover it are
// released first, oldest first.  New slots are sized for the largest
// request so far (componentwise), or for the request alone when that does
// not fit.  A request that
// cannot be admitted yet stays queued without holding back later requests.
#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <unordered_map>

#include "oc_internal.h"

namespace oc {

namespace {

struct SvcSlot {
    oc_slot *sl = nullptr;
    hipEvent_t done = nullptr;    // recorded after the request's last launch
    uint64_t ticket = 0;          // running request (0 = idle)
    int8_t *iblank = nullptr;     // its output
    uint64_t last_use = 0;        // admission count at its last request
    int64_t bytes = 0;
};

struct SvcReq {
    uint64_t ticket = 0;
    int32_t grid_id = 0;
    std::vector<int32_t> surf_ids;
    std::vector<double> poses;    // host copy [n_surf*12]
    int8_t *iblank = nullptr;
    hipEvent_t after = nullptr;   // the context stream when it was submitted
    bool blocked = false;         // admission failed for room since the last retirement
};

struct Done {
    oc_status st = OC_OK;
    std::string err;
    const int8_t *iblank = nullptr;
};

}  // namespace

struct Service {
    std::vector<SvcSlot> slots;
    std::deque<SvcReq> queue;
    std::unordered_map<uint64_t, Done> done;
    uint64_t next_ticket = 1;
    uint64_t admissions = 0;
    int peak_running = 0;
    CutCaps hwm;                  // componentwise largest request so far
    int64_t hwm_ne = 0;
};

namespace {

bool covers(const oc_slot *sl, const CutCaps &c, int64_t ne)
{
    return sl->cc.elem_inst >= c.elem_inst && sl->cc.faces >= c.faces && sl->cc.bins >= c.bins &&
           sl->cc.cuts >= c.cuts && sl->cc.outs >= c.outs && sl->list_cap >= ne;
}

void release(oc_ctx *ctx, SvcSlot &s)
{
    slot_free(s.sl);    // waits for the slot's stream
    (void)hipStreamDestroy(s.sl->stream);
    delete s.sl;
    (void)hipEventDestroy(s.done);
    s = SvcSlot{};
    (void)ctx;
}

oc_status new_slot(oc_ctx *ctx, const CutCaps &cc, int64_t ne, SvcSlot *out)
{
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string("cut service: ") + hipGetErrorString(e));
        if (st) (void)hipStreamDestroy(st);
        return OC_EDEVICE;
    }
    oc_slot *sl;
    oc_status r = slot_make(ctx, cc, ne, 0, st, &sl);
    if (r != OC_OK) {
        (void)hipStreamDestroy(st);
        (void)hipEventDestroy(ev);
        return r;
    }
    SvcSlot s;
    s.sl = sl;
    s.done = ev;
    s.bytes = slot_bytes(sl);
    *out = s;
    return OC_OK;
}

int n_running(const Service &sv)
{
    int n = 0;
    for (auto &s : sv.slots) n += s.ticket != 0;
    return n;
}

enum Admit { kAdmitted, kBlocked, kFailed };

// Launch q on slot s (the slot is idle and covers q).
oc_status launch(oc_ctx *ctx, SvcSlot &s, SvcReq &q, CutReq &rq)
{
    oc_slot *sl = s.sl;
    OC_HIP(hipStreamWaitEvent(sl->stream, q.after, 0));
    OC_TRY(set_poses(sl, 0, q.poses.data(), (int)q.surf_ids.size()));
    rq.poses = sl->poses;
    OC_TRY(cut_batch_run(sl, &rq, 1));
    OC_HIP(hipEventRecord(s.done, sl->stream));
    (void)ctx;
    return OC_OK;
}

Admit try_admit(oc_ctx *ctx, Service &sv, SvcReq &q, Done *fail)
{
    std::vector<CutReq> rq;
    std::vector<std::vector<Surf *>> ss;
    oc_cut_req pub{q.grid_id, (int32_t)q.surf_ids.size(), q.surf_ids.data(), q.poses.data(), q.iblank};
    oc_status st = collect_cut_reqs(ctx, &pub, 1, rq, ss, true);
    if (st != OC_OK) {
        *fail = Done{st, oc_last_error()};
        return kFailed;
    }
    const CutCaps need = cut_caps(rq.data(), 1);
    const int64_t ne = rq[0].g->n_elem;
    CutCaps big = sv.hwm;
    big.elem_inst = std::max(big.elem_inst, need.elem_inst);
    big.faces = std::max(big.faces, need.faces);
    big.bins = std::max(big.bins, need.bins);
    big.cuts = std::max(big.cuts, need.cuts);
    big.outs = std::max(big.outs, need.outs);
    const int64_t big_ne = std::max(sv.hwm_ne, ne);
    // the smallest idle slot that covers the request
    int pick = -1;
    for (int k = 0; k < (int)sv.slots.size(); ++k) {
        const SvcSlot &s = sv.slots[k];
        if (s.ticket == 0 && covers(s.sl, need, ne) && (pick < 0 || s.bytes < sv.slots[pick].bytes)) pick = k;
    }
    if (pick < 0) {
        // a new slot: release idle slots (oldest first) while the count or
        // the budget does not allow it
        for (;;) {
            int oldest = -1;
            for (int k = 0; k < (int)sv.slots.size(); ++k)
                if (sv.slots[k].ticket == 0 && (oldest < 0 || sv.slots[k].last_use < sv.slots[oldest].last_use))
                    oldest = k;
            // sized for the largest request so far, so that later requests
            // reuse it; sized for this one alone when that does not fit
            SvcSlot s;
            st = (int)sv.slots.size() >= ctx->service_slots ? OC_EBUDGET : new_slot(ctx, big, big_ne, &s);
            if (st == OC_EBUDGET && (int)sv.slots.size() < ctx->service_slots)
                st = new_slot(ctx, need, ne, &s);
            if (st == OC_OK) {
                sv.slots.push_back(s);
                pick = (int)sv.slots.size() - 1;
                break;
            }
            if (st != OC_EBUDGET && st != OC_ENOMEM) {
                *fail = Done{st, oc_last_error()};
                return kFailed;
            }
            if (oldest >= 0) {
                release(ctx, sv.slots[oldest]);
                sv.slots.erase(sv.slots.begin() + oldest);
                continue;
            }
            if (n_running(sv) > 0) return kBlocked;   // room comes back when a request ends
            *fail = Done{st, oc_last_error()};       // would not fit even alone
            return kFailed;
        }
    }
    SvcSlot &s = sv.slots[pick];
    st = launch(ctx, s, q, rq[0]);
    if (st != OC_OK) {
        *fail = Done{st, oc_last_error()};
        return kFailed;
    }
    s.ticket = q.ticket;
    s.iblank = q.iblank;
    s.last_use = ++sv.admissions;
    sv.hwm = big;
    sv.hwm_ne = big_ne;
    sv.peak_running = std::max(sv.peak_running, n_running(sv));
    return kAdmitted;
}

// Retire finished requests, then admit queued ones in submission order.  A
// request refused for room is tried again only after a request has ended
// (a failed attempt allocates and frees, and freeing waits for the device).
void pump(oc_ctx *ctx, Service &sv)
{
    bool ended = false;
    for (auto &s : sv.slots) {
        if (s.ticket == 0) continue;
        hipError_t e = hipEventQuery(s.done);
        if (e == hipErrorNotReady) continue;
        Done d;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            d = Done{OC_EDEVICE, std::string("cut service: ") + hipGetErrorString(e)};
        }
        d.iblank = s.iblank;
        sv.done[s.ticket] = d;
        s.ticket = 0;
        s.iblank = nullptr;
        ended = true;
    }
    for (auto it = sv.queue.begin(); it != sv.queue.end();) {
        if (it->blocked && !ended) {
            ++it;
            continue;
        }
        Done fail;
        Admit a = try_admit(ctx, sv, *it, &fail);
        if (a == kBlocked) {
            it->blocked = true;
            ++it;
            continue;
        }
        if (a == kFailed) sv.done[it->ticket] = fail;
        (void)hipEventDestroy(it->after);
        it = sv.queue.erase(it);
    }
}

bool in_flight(const Service &sv, const int8_t *iblank)
{
    for (auto &s : sv.slots)
        if (s.ticket && s.iblank == iblank) return true;
    for (auto &q : sv.queue)
        if (q.iblank == iblank) return true;
    for (auto &d : sv.done)
        if (d.second.st == OC_OK && d.second.iblank == iblank) return true;
    return false;
}

}  // namespace

void service_destroy(oc_ctx *ctx)
{
    Service *sv = ctx->service;
    if (!sv) return;
    for (auto &s : sv->slots) release(ctx, s);
    for (auto &q : sv->queue) (void)hipEventDestroy(q.after);
    delete sv;
    ctx->service = nullptr;
}

}  // namespace oc

using namespace oc;

extern "C" {

oc_status oc_submit(oc_ctx *ctx, const oc_request *req, uint64_t *ticket)
{
    if (!ctx || !req || !ticket) {
        set_error("oc_submit: invalid arguments");
        return OC_EINVAL;
    }
    *ticket = 0;
    OC_HIP(hipSetDevice(ctx->device));
    std::vector<CutReq> rq;
    std::vector<std::vector<Surf *>> ss;
    OC_TRY(collect_cut_reqs(ctx, req, 1, rq, ss, true));
    if (req->n_surf > kPoseSlots - 2) {
        set_error("oc_submit: more than " + std::to_string(kPoseSlots - 2) + " surfaces");
        return OC_EINVAL;
    }
    for (int k = 0; k < req->n_surf; ++k)
        if (!pose_finite(req->poses + 12 * k)) {
            set_error("oc_submit: non-finite pose");
            return OC_EINVAL;
        }
    if (!ctx->service) ctx->service = new Service();
    Service &sv = *ctx->service;
    if (in_flight(sv, req->iblank_out)) {
        set_error("oc_submit: iblank_out is the output of a request not yet waited for");
        return OC_EINVAL;
    }
    SvcReq q;
    q.ticket = sv.next_ticket;
    q.grid_id = req->grid_id;
    q.surf_ids.assign(req->surf_ids, req->surf_ids + req->n_surf);
    q.poses.assign(req->poses, req->poses + 12 * (size_t)req->n_surf);
    q.iblank = req->iblank_out;
    OC_HIP(hipEventCreateWithFlags(&q.after, hipEventDisableTiming));
    hipError_t e = hipEventRecord(q.after, ctx->dflt->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(q.after);
        set_error(std::string("oc_submit: ") + hipGetErrorString(e));
        return OC_EDEVICE;
    }
    const uint64_t t = sv.next_ticket++;
    sv.queue.push_back(std::move(q));
    pump(ctx, sv);
    auto it = sv.done.find(t);
    if (it != sv.done.end() && it->second.st != OC_OK) {
        // refused outright (would not fit even alone, or failed to launch)
        oc_status st = it->second.st;
        set_error(it->second.err);
        sv.done.erase(it);
        return st;
    }
    *ticket = t;
    return OC_OK;
}

oc_status oc_wait(oc_ctx *ctx, uint64_t ticket, int32_t timeout_ms)
{
    if (!ctx) {
        set_error("oc_wait: null context");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    if (!ctx->service) {
        set_error("oc_wait: unknown ticket " + std::to_string(ticket));
        return OC_ENOTFOUND;
    }
    Service &sv = *ctx->service;
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        pump(ctx, sv);
        auto it = sv.done.find(ticket);
        if (it != sv.done.end()) {
            oc_status st = it->second.st;
            if (st != OC_OK) set_error(it->second.err);
            sv.done.erase(it);
            return st;
        }
        bool pending = false;
        for (auto &s : sv.slots) pending |= s.ticket == ticket;
        for (auto &q : sv.queue) pending |= q.ticket == ticket;
        if (!pending) {
            set_error("oc_wait: unknown ticket " + std::to_string(ticket));
            return OC_ENOTFOUND;
        }
        if (timeout_ms >= 0 &&
            std::chrono::steady_clock::now() - t0 >= std::chrono::milliseconds(timeout_ms)) {
            set_error("oc_wait: ticket " + std::to_string(ticket) + " not finished");
            return OC_ETIMEDOUT;
        }
        std::this_thread::yield();
    }
}

oc_status oc_cancel(oc_ctx *ctx, uint64_t ticket)
{
    if (!ctx) {
        set_error("oc_cancel: null context");
        return OC_EINVAL;
    }
    OC_HIP(hipSetDevice(ctx->device));
    Service *sv = ctx->service;
    if (sv) {
        // a request still queued is dropped before anything is admitted
        for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
            if (it->ticket == ticket) {
                (void)hipEventDestroy(it->after);
                sv->queue.erase(it);
                pump(ctx, *sv);
                return OC_OK;
            }
        bool started = sv->done.count(ticket) > 0;
        for (auto &s : sv->slots) started |= s.ticket == ticket;
        if (started) {
            set_error("oc_cancel: ticket " + std::to_string(ticket) + " has started; retire it with oc_wait");
            return OC_ESTARTED;
        }
    }
    set_error("oc_cancel: unknown ticket " + std::to_string(ticket));
    return OC_ENOTFOUND;
}

oc_status oc_service_info(oc_ctx *ctx, oc_service_stats *info)
{
    if (!ctx || !info) {
        set_error("oc_service_info: invalid arguments");
        return OC_EINVAL;
    }
    *info = oc_service_stats{};
    Service *sv = ctx->service;
    if (!sv) return OC_OK;
    pump(ctx, *sv);
    info->slots = (int32_t)sv->slots.size();
    info->running = n_running(*sv);
    info->queued = (int32_t)sv->queue.size();
    info->finished = (int32_t)sv->done.size();
    info->peak_running = sv->peak_running;
    for (auto &s : sv->slots) info->slot_bytes += s.bytes;
    return OC_OK;
}

}  // extern "C"
