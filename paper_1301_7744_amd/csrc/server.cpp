// Continuous-batching sttsm server (declared in include/sttsm.h).
//
// One worker thread runs rounds.  A round (1) admits queued requests in
// arrival order while their footprint fits in the arena and the in-flight
// cap allows, (2) stages the inputs and index tables of newly admitted
// requests into their arena regions and builds their padded X panels, and
// (3) queues the next level of every active request in grouped persistent
// launches (one per kernel class present) whose workgroups take tiles of all
// requests from one shared queue.  Rounds are double buffered: round r + 1 is
// formed and queued on the stream while round r runs (the stream orders each
// request's levels), and the worker only then waits for round r.  Completion of the last level marks a
// request done; its A, X, temporaries and tables are released at once and
// its C when the caller fetches it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "abi_util.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace symt;

namespace {

// Kernel class of a stage in a server round: the compute form (generic
// grouped kernel), one (m, b, k) of the block-copy bf16 kernel, or one
// (m, k) of the X-resident bf16 kernel (b = 16).
constexpr int kXresClass0 = CMP_X3 + 1 + 2 * 2 * 4;
constexpr int kLaunchClasses = kXresClass0 + 2 * 4;
int launch_class(int m, int b, const StagePlan &St)
{
    if (!St.fast_bf16) return St.compute;
    if (St.tile.xres) return kXresClass0 + (m - 3) * 4 + St.k;
    return CMP_X3 + 1 + ((m - 3) * 2 + (b == 16 ? 1 : 0)) * 4 + St.k;
}

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

double now_us()
{
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, total) with coalescing frees.
struct ArenaAlloc {
    std::map<size_t, size_t> free_;   // offset -> size
    void init(size_t total)
    {
        free_.clear();
        if (total) free_[0] = total;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = round256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, o2 = it->first + n;
            free_.erase(it);
            if (rest) free_[o2] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round256(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Byte layout of a request's arena regions.
struct Footprint {
    size_t a = 0, x = 0, ws = 0, tables = 0, main = 0, c = 0;
    // offsets inside the main region
    size_t off_a = 0, off_x = 0, off_ws = 0, off_tab = 0;
    std::vector<size_t> off_groups, off_in;   // per level, inside the table area
};

// The plan a request runs.  bf16 requests take the plain path's tiles when
// every level is X-resident or has the bf16 block-copy kernel's default tile
// (the X-resident levels then run in the grouped X-resident kernel, the
// others in the grouped block-copy kernel, both with the plain path's
// arithmetic, so results are bit-identical to it); otherwise the plan is
// built with the grouped kernels' tiles throughout.
bool server_plan(PlanKey key, Plan *P, std::string *why)
{
    key.generic_only = false;
    key.grouped = false;
    key.xres_records = false;
    if (plan_build_host(key, P, why)) {
        bool ok = true;
        for (const StagePlan &St : P->stages) {
            int mt, nt, kt, pd;
            bf16_fast_tile(St.args.bA, &mt, &nt, &kt, &pd);
            ok = ok && St.fast_bf16 && (St.tile.xres || (St.tile.NT == nt && St.tile.KT == kt && St.tile.PD == pd));
        }
        if (ok) return true;
    }
    *P = Plan();
    key.grouped = true;
    return plan_build_host(key, P, why);
}

struct Req {
    uint64_t ticket = 0;
    int state = STTSM_QUEUED;
    sttsm_request r{};
    std::unique_ptr<Plan> plan;
    Footprint fp;
    size_t off_main = 0, off_c = 0;
    char *main = nullptr, *C = nullptr;
    int level = 0;             // next level to enqueue; m once the last is enqueued
    double t_submit = 0, t_done = 0;
};

int compute_footprint(const sttsm_request *q, const Plan &P, Footprint *fp)
{
    const int64_t na = bcss_num_elems(&q->A), nc = bcss_num_elems(&q->C);
    if (na < 0 || nc < 0) return STTSM_EINVAL;
    fp->a = round256((size_t)na * dtype_size(q->A.dtype));
    fp->x = round256((size_t)(q->C.n * q->A.n) * dtype_size(q->A.dtype));
    fp->ws = round256(P.ws_bytes);
    fp->tables = 0;
    fp->off_groups.clear();
    fp->off_in.clear();
    for (const StagePlan &S : P.stages) {
        fp->off_groups.push_back(fp->tables);
        fp->tables += round256(S.groups.size() * sizeof(GroupDesc));
        fp->off_in.push_back(fp->tables);
        fp->tables += round256(S.in_tab.size() * sizeof(InEntry));
    }
    fp->off_a = 0;
    fp->off_x = fp->a;
    fp->off_ws = fp->off_x + fp->x;
    fp->off_tab = fp->off_ws + fp->ws;
    fp->main = fp->off_tab + fp->tables;
    fp->c = round256((size_t)nc * 4);
    return STTSM_OK;
}

}  // namespace

struct sttsm_server {
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int max_inflight = 1;
    int device = 0;
    int grid = 512;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> arrival;
    std::vector<Req *> active;
    std::map<uint64_t, std::unique_ptr<Req>> all;
    ArenaAlloc alloc;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string fatal;
    // device side of the rounds: two slots, so that the next round is formed
    // and queued while the previous one runs
    hipStream_t stream = nullptr;
    // copies of finished results out of the arena (sttsm_fetch); its own
    // stream, so that a fetch never waits behind queued rounds
    hipStream_t fetch_stream = nullptr;
    struct Slot {
        hipEvent_t ev = nullptr;
        StageArgs *d_stages = nullptr;
        GroupedTask *d_tasks = nullptr;
        int *d_heads = nullptr;
        size_t cap_stages = 0, cap_tasks = 0;
        StageArgs *h_stages = nullptr;   // pinned staging
        GroupedTask *h_tasks = nullptr;
        bool pending = false;            // queued, not yet completed
        int launches = 0;
        std::vector<Req *> members;      // requests with a level in this round
        std::vector<Req *> finishing;    // ... whose last level it is
    } slot[2];
    // statistics
    double t_stage_us = 0, t_form_us = 0, t_queue_us = 0, t_wait_us = 0;   // worker host time by phase
    std::vector<double> lat_us;
    double t_first_submit = -1, t_last_done = 0;
    int64_t rounds = 0, launches = 0;
    std::thread worker;
};

namespace {

bool ensure_capacity(sttsm_server::Slot *S, size_t nstages, size_t ntasks, std::string *err)
{
    if (nstages > S->cap_stages) {
        const size_t cap = std::max(nstages, 2 * S->cap_stages);
        if (S->d_stages) (void)hipFree(S->d_stages);
        if (S->h_stages) (void)hipHostFree(S->h_stages);
        S->d_stages = nullptr;
        S->h_stages = nullptr;
        if (hipMalloc((void **)&S->d_stages, cap * sizeof(StageArgs)) != hipSuccess ||
            hipHostMalloc((void **)&S->h_stages, cap * sizeof(StageArgs), hipHostMallocDefault) != hipSuccess) {
            *err = "server: cannot allocate stage table";
            S->cap_stages = 0;
            return false;
        }
        S->cap_stages = cap;
    }
    if (ntasks > S->cap_tasks) {
        const size_t cap = std::max(ntasks, 2 * S->cap_tasks);
        if (S->d_tasks) (void)hipFree(S->d_tasks);
        if (S->h_tasks) (void)hipHostFree(S->h_tasks);
        S->d_tasks = nullptr;
        S->h_tasks = nullptr;
        if (hipMalloc((void **)&S->d_tasks, cap * sizeof(GroupedTask)) != hipSuccess ||
            hipHostMalloc((void **)&S->h_tasks, cap * sizeof(GroupedTask), hipHostMallocDefault) != hipSuccess) {
            *err = "server: cannot allocate task queue";
            S->cap_tasks = 0;
            return false;
        }
        S->cap_tasks = cap;
    }
    return true;
}

// Copies a newly admitted request's inputs and tables into its region and
// builds its X panels (all on the server stream).
bool stage_inputs(sttsm_server *S, Req *q, std::string *err)
{
    const sttsm_request &r = q->r;
    const Footprint &fp = q->fp;
    const hipMemcpyKind kin = r.src_is_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const int es = dtype_size(r.A.dtype);
    const int64_t na = bcss_num_elems(&r.A);
    if (hipMemcpyAsync(q->main + fp.off_a, r.A_bcss, (size_t)na * es, kin, S->stream) != hipSuccess) {
        *err = "server: copy of A failed";
        return false;
    }
    // X is repacked contiguous (rs = n, cs = 1)
    const int64_t p = r.C.n, n = r.A.n;
    if (hipMemcpy2DAsync(q->main + fp.off_x, (size_t)n * es, r.X, (size_t)r.rs_x * es, (size_t)n * es, (size_t)p,
                         kin, S->stream) != hipSuccess || r.cs_x != 1) {
        if (r.cs_x != 1) *err = "server: X must have unit column stride";
        else *err = "server: copy of X failed";
        return false;
    }
    for (size_t d = 0; d < q->plan->stages.size(); ++d) {
        const StagePlan &St = q->plan->stages[d];
        char *tab = q->main + fp.off_tab;
        if (!St.groups.empty() &&
            hipMemcpyAsync(tab + fp.off_groups[d], St.groups.data(), St.groups.size() * sizeof(GroupDesc),
                           hipMemcpyHostToDevice, S->stream) != hipSuccess) {
            *err = "server: copy of tables failed";
            return false;
        }
        if (!St.in_tab.empty() &&
            hipMemcpyAsync(tab + fp.off_in[d], St.in_tab.data(), St.in_tab.size() * sizeof(InEntry),
                           hipMemcpyHostToDevice, S->stream) != hipSuccess) {
            *err = "server: copy of tables failed";
            return false;
        }
    }
    const Plan &P = *q->plan;
    char *w = q->main + fp.off_ws;
    float *x32 = P.xp_off[0] >= 0 ? (float *)(w + P.xp_off[0]) : nullptr;
    uint16_t *xhi = P.xp_off[1] >= 0 ? (uint16_t *)(w + P.xp_off[1]) : nullptr;
    uint16_t *xlo = P.xp_off[2] >= 0 ? (uint16_t *)(w + P.xp_off[2]) : nullptr;
    if ((x32 || xhi || xlo) && launch_prep_x(es, q->main + fp.off_x, n, 1, p, n, P.Ppad, P.Kx, x32, xhi, xlo, S->stream)) {
        *err = "server: X panel launch failed";
        return false;
    }
    // The pageable host sources must be read before submit's caller may free
    // them; host copies are staged by the runtime before the call returns.
    return true;
}

StageArgs stage_args_for(const Req *q, int d)
{
    const Plan &P = *q->plan;
    const StagePlan &St = P.stages[d];
    const Footprint &fp = q->fp;
    StageArgs a = St.args;
    char *w = q->main + fp.off_ws;
    const void *slot[3] = {P.xp_off[0] >= 0 ? w + P.xp_off[0] : nullptr, P.xp_off[1] >= 0 ? w + P.xp_off[1] : nullptr,
                           P.xp_off[2] >= 0 ? w + P.xp_off[2] : nullptr};
    a.in = St.in_ws < 0 ? (const void *)(q->main + fp.off_a) : (const void *)(w + St.in_ws);
    a.out = St.out_ws < 0 ? (void *)q->C : (void *)(w + St.out_ws);
    a.xp = slot[St.xp_slot];
    a.xp_lo = St.xp_lo_slot >= 0 ? slot[St.xp_lo_slot] : nullptr;
    a.groups = (const GroupDesc *)(q->main + fp.off_tab + fp.off_groups[d]);
    a.in_tab = (const InEntry *)(q->main + fp.off_tab + fp.off_in[d]);
    a.xrec = nullptr;   // the grouped X-resident kernel assembles its records from the tables
    a.tasks = nullptr;
    return a;
}

void release_main(sttsm_server *S, Req *q)
{
    if (q->main) S->alloc.release(q->off_main, q->fp.main);
    q->main = nullptr;
}

void release_c(sttsm_server *S, Req *q)
{
    if (q->C) S->alloc.release(q->off_c, q->fp.c);
    q->C = nullptr;
}

void fail_active(sttsm_server *S, const std::string &why)
{
    for (Req *q : S->active) {
        q->state = STTSM_FAILED;
        release_main(S, q);
        release_c(S, q);
    }
    S->active.clear();
    for (auto &sl : S->slot) {
        for (Req *q : sl.finishing) {
            q->state = STTSM_FAILED;
            release_main(S, q);
            release_c(S, q);
        }
        sl.finishing.clear();
        sl.members.clear();
        sl.pending = false;
    }
    S->fatal = why;
    S->cv_done.notify_all();
}

// Waits for a queued round and retires it: requests whose last level ran in
// it are done (their inputs, temporaries and tables are released; C stays
// until fetched).  Called with the lock not held.
bool complete_round(sttsm_server *S, sttsm_server::Slot &sl, std::string *err)
{
    const double t0 = now_us();
    const hipError_t e = hipEventSynchronize(sl.ev);
    std::lock_guard<std::mutex> lk(S->mu);
    S->t_wait_us += now_us() - t0;
    sl.pending = false;
    if (e != hipSuccess) {
        *err = std::string("server: round failed: ") + hipGetErrorString(e);
        return false;
    }
    ++S->rounds;
    S->launches += sl.launches;
    const double t = now_us();
    for (Req *q : sl.finishing) {
        q->state = STTSM_DONE;
        q->t_done = t;
        release_main(S, q);
        S->lat_us.push_back(t - q->t_submit);
        S->t_last_done = t;
    }
    sl.finishing.clear();
    sl.members.clear();
    S->cv_done.notify_all();
    S->cv_work.notify_one();   // freed arena may admit waiting requests
    return true;
}

void worker_loop(sttsm_server *S)
{
    (void)hipSetDevice(S->device);
    std::string err;
    int cur = 0;   // slot of the round being formed; slot cur ^ 1 may be in flight
    for (;;) {
        std::vector<Req *> fresh, active;
        bool stopping = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] {
                return S->stop || !S->arrival.empty() || !S->active.empty() || S->slot[cur ^ 1].pending;
            });
            stopping = S->stop;
            if (!stopping) {
                // Admission: first come, first served, within the arena and the cap.
                while (!S->arrival.empty() && (int)S->active.size() < S->max_inflight) {
                    Req *q = S->arrival.front();
                    size_t om = 0, oc = 0;
                    if (!S->alloc.alloc(q->fp.main, &om)) break;
                    if (!S->alloc.alloc(q->fp.c, &oc)) {
                        S->alloc.release(om, q->fp.main);
                        break;
                    }
                    q->off_main = om;
                    q->off_c = oc;
                    q->main = S->arena + om;
                    q->C = S->arena + oc;
                    q->state = STTSM_ADMITTED;
                    S->arrival.pop_front();
                    S->active.push_back(q);
                    fresh.push_back(q);
                }
                active = S->active;
            }
        }
        if (stopping) {
            // let queued rounds finish before their memory is given back
            for (auto &sl : S->slot)
                if (sl.pending) (void)hipEventSynchronize(sl.ev);
            std::lock_guard<std::mutex> lk(S->mu);
            for (Req *q : S->arrival) q->state = STTSM_FAILED;
            S->arrival.clear();
            fail_active(S, "server stopped");
            return;
        }
        if (active.empty()) {
            if (S->slot[cur ^ 1].pending) {
                if (!complete_round(S, S->slot[cur ^ 1], &err)) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    fail_active(S, err);
                }
                continue;
            }
            // nothing fits yet although requests wait: a finished C is
            // holding the arena until fetched; sleep until something changes
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        sttsm_server::Slot &sl = S->slot[cur];
        bool ok = true;
        const double t_a = now_us();
        for (Req *q : fresh)
            if (!stage_inputs(S, q, &err)) { ok = false; break; }
        const double t_b = now_us();
        // Next level of every active request.  The stream orders it after the
        // request's previous level, which may still be running.
        size_t nst = active.size(), ntk = 0;
        for (Req *q : active) ntk += q->plan->stages[q->level].tasks.size();
        if (ok) ok = ensure_capacity(&sl, nst, ntk, &err);
        sl.launches = 0;
        if (ok) {
            // One launch per kernel class: the generic grouped kernel per
            // compute form, and the block-copy bf16 kernel per (m, b, k).
            size_t ti = 0;
            size_t cls_t0[kLaunchClasses] = {}, cls_cnt[kLaunchClasses] = {};
            int cls_m[kLaunchClasses] = {}, cls_b[kLaunchClasses] = {}, cls_k[kLaunchClasses] = {};
            int cls_nt[kLaunchClasses] = {}, cls_pd[kLaunchClasses] = {};
            for (int cls = 0; cls < kLaunchClasses; ++cls) {
                cls_t0[cls] = ti;
                for (size_t i = 0; i < active.size(); ++i) {
                    const Req *q = active[i];
                    const StagePlan &St = q->plan->stages[q->level];
                    if (launch_class(q->plan->m, q->plan->bA, St) != cls) continue;
                    sl.h_stages[i] = stage_args_for(q, q->level);
                    for (const Task &t : St.tasks) sl.h_tasks[ti++] = GroupedTask{(int32_t)i, t.group, t.mt, t.nt};
                    cls_m[cls] = q->plan->m;
                    cls_b[cls] = q->plan->bA;
                    cls_k[cls] = St.k;
                    cls_nt[cls] = St.tile.NT;
                    cls_pd[cls] = St.tile.PD;
                }
                cls_cnt[cls] = ti - cls_t0[cls];
            }
            S->t_form_us += now_us() - t_b;
            if (hipMemcpyAsync(sl.d_stages, sl.h_stages, nst * sizeof(StageArgs), hipMemcpyHostToDevice,
                               S->stream) != hipSuccess ||
                hipMemcpyAsync(sl.d_tasks, sl.h_tasks, ntk * sizeof(GroupedTask), hipMemcpyHostToDevice, S->stream) !=
                    hipSuccess ||
                hipMemsetAsync(sl.d_heads, 0, kLaunchClasses * sizeof(int), S->stream) != hipSuccess) {
                ok = false;
                err = "server: upload of the round failed";
            }
            for (int cls = 0; cls < kLaunchClasses && ok; ++cls) {
                if (!cls_cnt[cls]) continue;
                const int cnt = (int)cls_cnt[cls];
                const GroupedTask *tk = sl.d_tasks + cls_t0[cls];
                int *head = sl.d_heads + cls;
                const int rc = cls < CMP_X3 + 1
                                   ? launch_grouped(cls, sl.d_stages, tk, cnt, head, S->grid, S->stream)
                               : cls >= kXresClass0
                                   ? launch_grouped_xres(cls_m[cls], cls_k[cls], cls_nt[cls], cls_pd[cls], sl.d_stages,
                                                         tk, cnt, head, S->grid, S->stream)
                                   : launch_grouped_bf16(cls_m[cls], cls_b[cls], cls_k[cls], sl.d_stages, tk, cnt,
                                                         head, S->grid, S->stream);
                if (rc) {
                    ok = false;
                    err = "server: grouped launch failed";
                }
                ++sl.launches;
            }
        }
        if (ok && hipEventRecord(sl.ev, S->stream) != hipSuccess) {
            ok = false;
            err = std::string("server: event record failed: ") + hipGetErrorString(hipGetLastError());
        }
        S->t_stage_us += t_b - t_a;
        S->t_queue_us += now_us() - t_a - (t_b - t_a);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (!ok) {
                fail_active(S, err);
                continue;
            }
            sl.pending = true;
            sl.members = active;
            std::vector<Req *> still;
            for (Req *q : active) {
                q->state = STTSM_RUNNING;
                if (++q->level == q->r.A.m) sl.finishing.push_back(q);
                else still.push_back(q);
            }
            S->active.swap(still);
        }
        // The previous round completes while this one is queued behind it.
        sttsm_server::Slot &prev = S->slot[cur ^ 1];
        if (prev.pending && !complete_round(S, prev, &err)) {
            std::lock_guard<std::mutex> lk(S->mu);
            fail_active(S, err);
        }
        cur ^= 1;
    }
}

}  // namespace

extern "C" {

size_t sttsm_request_footprint(const sttsm_request *req)
{
    if (!req) return 0;
    PlanKey key;
    if (make_key(&req->A, &req->C, req->prec, &key) != STTSM_OK) return 0;
    Plan P;
    std::string why;
    if (!server_plan(key, &P, &why)) return 0;
    Footprint fp;
    if (compute_footprint(req, P, &fp) != STTSM_OK) return 0;
    return fp.main + fp.c;
}

int sttsm_server_create(void *arena, size_t arena_bytes, int32_t max_inflight, sttsm_server **out)
{
    if (!out) return fail(STTSM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!arena || arena_bytes < 256) return fail(STTSM_EINVAL, "arena must be non-null and hold >= 256 bytes");
    if (((uintptr_t)arena & 255) != 0) return fail(STTSM_EINVAL, "arena must be 256-byte aligned");
    if (max_inflight < 1) return fail(STTSM_EINVAL, "max_inflight must be >= 1");
    std::unique_ptr<sttsm_server> S(new sttsm_server);
    S->arena = (char *)arena;
    S->arena_bytes = arena_bytes / 256 * 256;
    S->max_inflight = max_inflight;
    S->alloc.init(S->arena_bytes);
    if (hipGetDevice(&S->device) != hipSuccess) return fail(STTSM_EHIP, "hipGetDevice failed");
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device) == hipSuccess && cus > 0)
        S->grid = 2 * cus;
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess)
        return fail(STTSM_EHIP, "hipStreamCreate failed");
    if (hipStreamCreateWithFlags(&S->fetch_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(S->stream);
        return fail(STTSM_EHIP, "hipStreamCreate failed");
    }
    for (auto &sl : S->slot)
        if (hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
            hipMalloc((void **)&sl.d_heads, kLaunchClasses * sizeof(int)) != hipSuccess) {
            for (auto &s2 : S->slot) {
                if (s2.ev) (void)hipEventDestroy(s2.ev);
                if (s2.d_heads) (void)hipFree(s2.d_heads);
            }
            (void)hipStreamDestroy(S->stream);
            (void)hipStreamDestroy(S->fetch_stream);
            return fail(STTSM_EHIP, "server: cannot create event or queue heads");
        }
    sttsm_server *raw = S.release();
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return STTSM_OK;
}

int sttsm_submit(sttsm_server *S, const sttsm_request *req, uint64_t *ticket)
{
    if (!S || !req || !ticket) return fail(STTSM_EINVAL, "null argument");
    if (!req->A_bcss || !req->X) return fail(STTSM_EINVAL, "null A or X");
    if (req->cs_x != 1 || req->rs_x < req->A.n) return fail(STTSM_EINVAL, "X must be row-major with unit column stride");
    PlanKey key;
    int rc = make_key(&req->A, &req->C, req->prec, &key);
    if (rc != STTSM_OK) return rc;
    std::unique_ptr<Req> q(new Req);
    q->r = *req;
    q->plan.reset(new Plan);
    std::string why;
    if (!server_plan(key, q->plan.get(), &why)) return fail(STTSM_EINVAL, why);
    if ((rc = compute_footprint(req, *q->plan, &q->fp)) != STTSM_OK) return fail(rc, "bad request layout");
    if (q->fp.main + q->fp.c > S->arena_bytes)
        return fail(STTSM_ENOMEM, "request footprint exceeds the whole arena");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(STTSM_EINVAL, "server is stopping");
    q->ticket = S->next_ticket++;
    q->t_submit = now_us();
    if (S->t_first_submit < 0) S->t_first_submit = q->t_submit;
    *ticket = q->ticket;
    S->arrival.push_back(q.get());
    S->all.emplace(q->ticket, std::move(q));
    S->cv_work.notify_one();
    return STTSM_OK;
}

int sttsm_poll(sttsm_server *S, uint64_t ticket, int32_t *state)
{
    if (!S || !state) return fail(STTSM_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(STTSM_ENOTFOUND, "unknown ticket");
    *state = it->second->state;
    return STTSM_OK;
}

int sttsm_wait(sttsm_server *S, uint64_t ticket, int64_t timeout_us, int32_t *state)
{
    if (!S || !state) return fail(STTSM_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(STTSM_ENOTFOUND, "unknown ticket");
    Req *q = it->second.get();
    auto done = [&] { return q->state == STTSM_DONE || q->state == STTSM_FAILED; };
    if (timeout_us < 0) S->cv_done.wait(lk, done);
    else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        *state = q->state;
        return fail(STTSM_EAGAIN, "not finished");
    }
    *state = q->state;
    return STTSM_OK;
}

int sttsm_fetch(sttsm_server *S, uint64_t ticket, void *C_dst, int32_t dst_is_host)
{
    if (!S || !C_dst) return fail(STTSM_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(STTSM_ENOTFOUND, "unknown or already fetched ticket");
    Req *q = it->second.get();
    if (q->state == STTSM_FAILED) {
        S->all.erase(it);
        return fail(STTSM_EHIP, "request failed: " + S->fatal);
    }
    if (q->state != STTSM_DONE) return fail(STTSM_EAGAIN, "not finished");
    // Take the request out of the table (a second fetch of the ticket now
    // finds nothing), copy without the lock, and give C's region back only
    // once the copy has completed: until then no admitted request can be
    // placed over it.
    std::unique_ptr<Req> own = std::move(it->second);
    S->all.erase(it);
    lk.unlock();
    const size_t bytes = (size_t)bcss_num_elems(&q->r.C) * 4;
    hipError_t e = hipMemcpyAsync(C_dst, q->C, bytes, dst_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                  S->fetch_stream);
    const hipError_t e2 = hipStreamSynchronize(S->fetch_stream);
    if (e == hipSuccess) e = e2;
    lk.lock();
    release_c(S, q);
    S->cv_work.notify_one();   // freed arena may admit waiting requests
    if (e != hipSuccess) return fail(STTSM_EHIP, std::string("copy of C failed: ") + hipGetErrorString(e));
    return STTSM_OK;
}

int sttsm_server_stats(sttsm_server *S, double *p50_us, double *p99_us, double *req_per_s, int64_t *completed,
                       int64_t *rounds, int64_t *launches)
{
    if (!S) return fail(STTSM_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    std::vector<double> v = S->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double f) {
        if (v.empty()) return 0.0;
        size_t i = (size_t)(f * (double)(v.size() - 1) + 0.5);
        return v[std::min(i, v.size() - 1)];
    };
    if (p50_us) *p50_us = pct(0.50);
    if (p99_us) *p99_us = pct(0.99);
    if (req_per_s)
        *req_per_s = v.empty() || S->t_last_done <= S->t_first_submit
                         ? 0.0
                         : (double)v.size() / ((S->t_last_done - S->t_first_submit) * 1e-6);
    if (completed) *completed = (int64_t)v.size();
    if (rounds) *rounds = S->rounds;
    if (launches) *launches = S->launches;
    return STTSM_OK;
}

int sttsm_server_destroy(sttsm_server *S)
{
    if (!S) return fail(STTSM_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    if (getenv("STTSM_SERVER_TIMING"))
        fprintf(stderr, "sttsm server: %lld rounds; worker ms: staging inputs %.1f, forming rounds %.1f, "
                        "forming+queueing %.1f, waiting %.1f\n", (long long)S->rounds, S->t_stage_us * 1e-3,
                S->t_form_us * 1e-3, S->t_queue_us * 1e-3, S->t_wait_us * 1e-3);
    (void)hipStreamSynchronize(S->stream);
    for (auto &sl : S->slot) {
        if (sl.d_stages) (void)hipFree(sl.d_stages);
        if (sl.d_tasks) (void)hipFree(sl.d_tasks);
        if (sl.d_heads) (void)hipFree(sl.d_heads);
        if (sl.h_stages) (void)hipHostFree(sl.h_stages);
        if (sl.h_tasks) (void)hipHostFree(sl.h_tasks);
        (void)hipEventDestroy(sl.ev);
    }
    (void)hipStreamSynchronize(S->fetch_stream);
    (void)hipStreamDestroy(S->stream);
    (void)hipStreamDestroy(S->fetch_stream);
    delete S;
    return STTSM_OK;
}

}  // extern "C"
