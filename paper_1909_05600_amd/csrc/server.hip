// Serving: a request loop over resident plans with HBM-budget admission and overlapping execution.
//
// Plans (trees, lists, operator tables) stay resident; a request is one apply of one plan.  A
// scheduler thread admits queued requests in arrival order as soon as a slot (a HIP stream) is free
// and the request's apply workspace fits in the device-memory budget still unclaimed; it then gives
// the request a workspace of its own, writes that request's level descriptors and launches the plan's
// stages on the slot's stream.  Requests in different slots run concurrently on the device, so a
// request that arrives while others run starts at once when resources allow instead of waiting for
// them.  Completion is observed by polling each running request's event; the workspace and the slot
// are then returned and the next queued request is admitted.  A request computes exactly what
// ffm_apply computes for its plan (same kernels, same work items, its own workspace), bitwise.
#include "common.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace ffm {

namespace {

typedef std::chrono::steady_clock Clock;

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Apply workspace of one request, carved from one device block.
struct ReqWork {
    DevBuf<char> block;
    WorkPtrs w;
};

}  // namespace

size_t apply_work_bytes(const Plan &P) {
    if (P.empty) return 0;
    return align256(sizeof(float2) * P.ny) + align256(sizeof(float2) * P.nx * P.ncomp()) + align256(sizeof(float4) * P.ws_src) +
           align256(sizeof(float4) * P.ws_tgt) + align256(sizeof(float2) * P.ws_z) +
           align256(sizeof(float4) * P.wpart.n) + align256(sizeof(float2) * P.wbpart.n) +
           align256(sizeof(float2) * P.wG.n) + align256(sizeof(float2) * P.wH.n) + align256(sizeof(float2) * P.wnsym.n) +
           align256(sizeof(float4) * P.wtgtx.n) + align256(sizeof(float2) * P.wtmp.n) +
           align256(sizeof(float2) * P.wucomp.n) + align256(sizeof(float4) * P.wsrcx.n) +
           (P.any_fp16 || P.any_grid ? 256 : 0);
}

WorkPtrs carve_work(const Plan &P, char *p) {
    WorkPtrs w;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += align256(bytes);
        return q;
    };
    w.u = reinterpret_cast<float2 *>(take(sizeof(float2) * P.ny));
    w.v = reinterpret_cast<float2 *>(take(sizeof(float2) * P.nx * P.ncomp()));
    w.lw.ut = reinterpret_cast<float4 *>(take(sizeof(float4) * P.ws_src));
    w.lw.vt = reinterpret_cast<float4 *>(take(sizeof(float4) * P.ws_tgt));
    w.lw.ut2 = reinterpret_cast<float2 *>(w.lw.ut);
    w.lw.Z = reinterpret_cast<float2 *>(take(sizeof(float2) * P.ws_z));
    w.lw.part = reinterpret_cast<float4 *>(take(sizeof(float4) * P.wpart.n));
    w.lw.bpart = reinterpret_cast<float2 *>(take(sizeof(float2) * P.wbpart.n));
    w.lw.G = reinterpret_cast<float2 *>(take(sizeof(float2) * P.wG.n));
    w.lw.H = reinterpret_cast<float2 *>(take(sizeof(float2) * P.wH.n));
    w.lw.nsym = reinterpret_cast<float2 *>(take(sizeof(float2) * P.wnsym.n));
    w.lw.vtx = reinterpret_cast<float4 *>(take(sizeof(float4) * P.wtgtx.n));
    w.lw.vtmp = P.wtmp.n ? reinterpret_cast<float2 *>(take(sizeof(float2) * P.wtmp.n)) : nullptr;
    w.lw.ucomp = P.wucomp.n ? reinterpret_cast<float2 *>(take(sizeof(float2) * P.wucomp.n)) : nullptr;
    w.lw.utx = P.wsrcx.n ? reinterpret_cast<float4 *>(take(sizeof(float4) * P.wsrcx.n)) : nullptr;
    w.amax = P.any_fp16 || P.any_grid ? reinterpret_cast<float *>(take(sizeof(float))) : nullptr;
    return w;
}

namespace {

void carve(const Plan &P, ReqWork &w) {
    const size_t b = apply_work_bytes(P);
    w.block.alloc(std::max<size_t>(b, 1));
    w.w = carve_work(P, w.block.p);
}

}  // namespace

struct Request {
    int64_t ticket = 0;
    Plan *plan = nullptr;
    IoEntry io{};
    size_t bytes = 0;
    Clock::time_point t_submit, t_start, t_done;
    int slot = -1;
    int status = FFM_OK;
    std::string msg;
    bool finished = false;
    // resources while running
    ReqWork work;
    DevBuf<LDesc> ddesc;
    DevBuf<IoEntry> dio;
    void *pinned = nullptr;            // descriptors + I/O entry staging
    hipEvent_t ev = nullptr;
    hipEvent_t ready = nullptr;        // recorded on the caller's stream at submission: wu is written
    ~Request() {
        if (ev) (void)hipEventDestroy(ev);
        if (ready) (void)hipEventDestroy(ready);
    }
};

struct Server {
    int nslots = 4;
    size_t budget = 0;
    std::vector<hipStream_t> streams;
    std::vector<Request *> slot_req;   // running request per slot (nullptr = free)
    std::mutex mx;
    std::condition_variable cv_sched, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
    int64_t next_ticket = 1;
    size_t in_use = 0, peak_in_use = 0;
    int running = 0, peak_running = 0;
    int64_t completed = 0, failed = 0;
    double points = 0;
    std::vector<double> lat_ms;        // submit -> observed completion of every finished request
    bool stop = false;
    int device = 0;
    std::thread th;

    void loop();
    void start_one(Request *r, int slot);
    void finish_one(Request *r);
};

void Server::start_one(Request *r, int slot) {
    Plan &P = *r->plan;
    hipStream_t st = streams[slot];
    r->slot = slot;
    r->t_start = Clock::now();
    FFM_HIP(hipEventCreateWithFlags(&r->ev, hipEventDisableTiming));
    if (P.empty) {
        if (r->ready) FFM_HIP(hipStreamWaitEvent(st, r->ready, 0));
        // no sources or no targets: the output is zero
        if (P.nx > 0) FFM_HIP(hipMemsetAsync(r->io.vout, 0, sizeof(float2) * P.nx * P.ncomp(), st));
        FFM_HIP(hipEventRecord(r->ev, st));
        return;
    }
    carve(P, r->work);
    const WorkPtrs &w = r->work.w;
    const int nd = plan_ndesc(P);
    const size_t db = sizeof(LDesc) * nd;
    r->pinned = pinned_alloc(db + sizeof(IoEntry));
    LDesc *hd = static_cast<LDesc *>(r->pinned);
    for (int k = 0; k < nd; ++k) hd[k] = plan_desc(P, k, 0, w.u, w.v, w.amax, w.lw);
    IoEntry *hio = reinterpret_cast<IoEntry *>(static_cast<char *>(r->pinned) + db);
    *hio = r->io;
    r->ddesc.alloc(nd);
    r->dio.alloc(1);
    if (r->ready) FFM_HIP(hipStreamWaitEvent(st, r->ready, 0));
    FFM_HIP(hipMemcpyAsync(r->ddesc.p, hd, db, hipMemcpyHostToDevice, st));
    FFM_HIP(hipMemcpyAsync(r->dio.p, hio, sizeof(IoEntry), hipMemcpyHostToDevice, st));
    for (const Stage &S : P.pre) run_stage(S, r->ddesc.p, r->dio.p, st);
    for (int l = 1; l <= P.leaf; ++l)
        for (const Stage &S : P.lev[l].stages) run_stage(S, r->ddesc.p, r->dio.p, st);
    for (const Stage &S : P.post) run_stage(S, r->ddesc.p, r->dio.p, st);
    FFM_HIP(hipEventRecord(r->ev, st));
}

// Called with the lock held, after the request's event has completed (or it failed to start).
void Server::finish_one(Request *r) {
    r->t_done = Clock::now();
    if (r->ev) (void)hipEventDestroy(r->ev);
    r->ev = nullptr;
    if (r->ready) (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
    r->work.block.release();
    r->ddesc.release();
    r->dio.release();
    if (r->pinned) pinned_free(r->pinned);
    r->pinned = nullptr;
    if (r->slot >= 0) slot_req[r->slot] = nullptr;
    in_use -= r->bytes;
    --running;
    --r->plan->server_refs;
    r->finished = true;
    if (r->status == FFM_OK) {
        ++completed;
        points += (double)r->plan->nx;
        lat_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
    } else {
        ++failed;
    }
}

void Server::loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mx);
    while (true) {
        // admit in arrival order while the head fits a free slot and the budget
        while (!queue.empty()) {
            Request *r = queue.front();
            int slot = -1;
            for (int s = 0; s < nslots; ++s)
                if (!slot_req[s]) {
                    slot = s;
                    break;
                }
            if (slot < 0 || in_use + r->bytes > budget) break;
            queue.pop_front();
            slot_req[slot] = r;
            in_use += r->bytes;
            peak_in_use = std::max(peak_in_use, in_use);
            ++running;
            peak_running = std::max(peak_running, running);
            try {
                start_one(r, slot);
            } catch (const Error &e) {
                r->status = e.code;
                r->msg = e.what();
            } catch (const std::exception &e) {
                r->status = FFM_EINTERNAL;
                r->msg = e.what();
            }
            if (r->status != FFM_OK) {
                // wait for whatever was enqueued before the failure, then release
                (void)hipStreamSynchronize(streams[slot]);
                finish_one(r);
                cv_done.notify_all();
            }
        }
        // observe completions
        bool any_running = false, progressed = false;
        for (int s = 0; s < nslots; ++s) {
            Request *r = slot_req[s];
            if (!r) continue;
            const hipError_t q = hipEventQuery(r->ev);
            if (q == hipErrorNotReady) {
                any_running = true;
                continue;
            }
            if (q != hipSuccess) {
                r->status = FFM_EDEVICE;
                r->msg = std::string("request failed on the device: ") + hipGetErrorString(q);
            }
            finish_one(r);
            progressed = true;
        }
        if (progressed) cv_done.notify_all();
        if (stop && queue.empty() && !any_running && running == 0) break;
        if (any_running) {
            // short polls while work is on the device
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else if (!progressed) {
            cv_sched.wait(lk, [&] { return stop || !queue.empty(); });
        }
    }
}

}  // namespace ffm

using namespace ffm;

struct ffm_server_s {
    Server S;
};

extern "C" {

ffm_status_t ffm_server_create(const ffm_server_options_t *opts, ffm_server_t *out) {
    if (!out) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_create: out is NULL");
    *out = nullptr;
    ffm_server_options_t o{};
    if (opts) o = *opts;
    if (o.slots < 0 || o.slots > 16 || o.reserved != 0 || !(o.budget_bytes >= 0.0))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_create: slots must be in [0, 16], budget >= 0");
    ffm_server_s *h = nullptr;
    int rc = Guard::run([&] {
        std::unique_ptr<ffm_server_s> s(new ffm_server_s());
        Server &S = s->S;
        FFM_HIP(hipGetDevice(&S.device));
        S.nslots = o.slots ? o.slots : 4;
        if (o.budget_bytes > 0) {
            S.budget = (size_t)o.budget_bytes;
        } else {
            size_t fr = 0, tot = 0;
            FFM_HIP(hipMemGetInfo(&fr, &tot));
            // 80% of the free device memory, counting the blocks the library has cached for reuse (the
            // workspaces are carved from them first, and the cache is released when the device runs out)
            S.budget = (fr + dev_bytes_cached()) / 10 * 8;
        }
        S.slot_req.assign(S.nslots, nullptr);
        for (int i = 0; i < S.nslots; ++i) {
            hipStream_t st;
            FFM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            S.streams.push_back(st);
        }
        S.th = std::thread([&S] { S.loop(); });
        h = s.release();
    });
    if (rc == FFM_OK) *out = h;
    return (ffm_status_t)rc;
}

ffm_status_t ffm_server_submit(ffm_server_t server, ffm_plan_t plan, const void *wu, ffm_dtype_t in_dtype, void *v,
                               void *hip_stream, int64_t *ticket) {
    if (!server || !plan || !ticket) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_submit: NULL argument");
    Plan &P = plan->P;
    if (P.nx > 0 && !v) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_submit: NULL output");
    if (P.ny > 0 && !wu) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_submit: NULL input");
    if (in_dtype < FFM_C64 || in_dtype > FFM_C128) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_submit: bad dtype");
    Server &S = server->S;
    const size_t bytes = apply_work_bytes(P);
    if (bytes > S.budget)
        return (ffm_status_t)set_err(FFM_ENOMEM, "ffm_server_submit: the request's workspace exceeds the whole budget");
    return (ffm_status_t)Guard::run([&] {
        plan_sync_ready(P);      // the server's streams then need no ordering after the planning stream
        std::unique_ptr<Request> r(new Request());
        r->plan = &P;
        r->io.wu = wu;
        r->io.vout = static_cast<float2 *>(v);
        r->io.dtype = (int)in_dtype;
        r->bytes = bytes;
        // the request starts only once the caller's stream has passed what it enqueued before submitting
        FFM_HIP(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
        FFM_HIP(hipEventRecord(r->ready, static_cast<hipStream_t>(hip_stream)));
        r->t_submit = Clock::now();
        std::lock_guard<std::mutex> lk(S.mx);
        FFM_CHECK(!S.stop, FFM_EINVAL, "ffm_server_submit: the server is shutting down");
        r->ticket = S.next_ticket++;
        *ticket = r->ticket;
        ++P.server_refs;
        S.queue.push_back(r.get());
        S.reqs[r->ticket] = std::move(r);
        S.cv_sched.notify_one();
    });
}

ffm_status_t ffm_server_wait(ffm_server_t server, int64_t ticket, double *latency_ms) {
    if (!server) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_wait: NULL server");
    Server &S = server->S;
    std::unique_lock<std::mutex> lk(S.mx);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_wait: unknown ticket");
    Request *r = it->second.get();
    S.cv_done.wait(lk, [&] { return r->finished; });
    const int st = r->status;
    const std::string msg = r->msg;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    S.reqs.erase(it);
    lk.unlock();
    if (st != FFM_OK) return (ffm_status_t)set_err(st, msg);
    return FFM_OK;
}

ffm_status_t ffm_server_poll(ffm_server_t server, int64_t ticket, int32_t *done) {
    if (!server || !done) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_poll: NULL argument");
    Server &S = server->S;
    std::lock_guard<std::mutex> lk(S.mx);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_poll: unknown ticket");
    *done = it->second->finished ? 1 : 0;
    return FFM_OK;
}

ffm_status_t ffm_server_stats(ffm_server_t server, ffm_server_stats_t *out) {
    if (!server || !out) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_server_stats: NULL argument");
    Server &S = server->S;
    std::lock_guard<std::mutex> lk(S.mx);
    std::memset(out, 0, sizeof(*out));
    out->slots = S.nslots;
    out->budget_bytes = (double)S.budget;
    out->completed = S.completed;
    out->failed = S.failed;
    out->queued = (int64_t)S.queue.size();
    out->running = S.running;
    out->peak_running = S.peak_running;
    out->in_use_bytes = (double)S.in_use;
    out->peak_in_use_bytes = (double)S.peak_in_use;
    out->points = S.points;
    if (!S.lat_ms.empty()) {
        std::vector<double> v = S.lat_ms;
        std::sort(v.begin(), v.end());
        auto q = [&](double f) {
            const double pos = f * (double)(v.size() - 1);
            const size_t i = (size_t)pos;
            const double t = pos - (double)i;
            return i + 1 < v.size() ? v[i] * (1.0 - t) + v[i + 1] * t : v[i];
        };
        out->p50_ms = q(0.50);
        out->p99_ms = q(0.99);
        out->max_ms = v.back();
    }
    return FFM_OK;
}

ffm_status_t ffm_server_destroy(ffm_server_t server) {
    if (!server) return FFM_OK;
    Server &S = server->S;
    {
        std::lock_guard<std::mutex> lk(S.mx);
        S.stop = true;
        S.cv_sched.notify_all();
    }
    if (S.th.joinable()) S.th.join();
    return (ffm_status_t)Guard::run([&] {
        for (hipStream_t st : S.streams) (void)hipStreamDestroy(st);
        delete server;
    });
}

}  // extern "C"
