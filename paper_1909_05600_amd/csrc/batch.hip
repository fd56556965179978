// Batches: many plans applied together, one launch per step kind for all of them.
//
// A batch borrows its plans (their trees, tables and workspaces) and merges their stages: every
// launch runs one kind of step (a source transform variant, a transfer, a target transform, the near
// field, a permutation) for every instance that has it, over the concatenated work items, whose .x
// names the instance's level descriptor.  Instances never share an output element, so a batch gives
// each instance bitwise the result of its own apply with the same tiles.  The merged launches can be
// captured once into a HIP graph; each apply then writes the per-instance input and output pointers
// into a device table (one copy) and replays the graph.
//
// The tile autotuner times the candidate tile choices of the plane-wave kernels on the batch itself
// and keeps the fastest; results are cached in a JSON file keyed by a signature of the batch's shapes.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

namespace ffm {

namespace {

constexpr int kThreadsB = 256;

template <class T>
void upload_b(DevBuf<T> &b, const std::vector<T> &h, hipStream_t st, Scratch &SC) {
    b.alloc(h.size());
    if (!h.empty()) FFM_HIP(hipMemcpyAsync(b.p, SC.stage(h), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// Order of a stage among its instance's stages of the same phase: stages of equal order from
// different instances are independent and run in one launch per kernel variant.
int stage_role(const Stage &S) {
    switch (S.kern) {
        case K_PERM_IN: return 0;
        case K_AMAX: return S.a ? 1 : 2;
        case K_FWD_PAIR: case K_FWD_RING: case K_ANTERP: case K_GSPREAD: case K_FWD_PAIR_DL: case K_ANTERP_DL: return 0;
        case K_SUM: case K_GZ: case K_DLCOMBINE: return 1;
        case K_GPHI: return 2;
        case K_TRANSFER: case K_MFMA32: case K_MFMA16: case K_ACA: case K_DIRSCALE: return 3;
        case K_BWD_PAIR: case K_BWD_RING: case K_INTERP: case K_GPHIT: case K_BWD_PAIR_DN: case K_INTERP_DN:
        case K_DNCOMBINE: return 4;
        case K_BSUM: case K_GZT: return 5;
        case K_GINTERP: return 6;
        // after the levels: the near fields of the early lists and the leaf in level order (they add into the same
        // outputs), the symmetric pairs' source-side sums, then the output permutation
        case K_ZERO_OUT: return 0;
        case K_NEAR: case K_NEAR_DN: case K_NEAR_DL: case K_NEAR_SYM: case K_NEAR_GRAD: return 1 + S.level;
        case K_NEAR_GATHER: return 1 + kMaxLev + 1;
        case K_PERM_OUT: return 1 + kMaxLev + 2;
        default: throw Error(FFM_EINTERNAL, "stage without a batch order");
    }
}

// FNV-1a over the shapes that decide the tile timings
struct Sig {
    uint64_t h = 1469598103934665603ull;
    void add(uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 255u;
            h *= 1099511628211ull;
        }
    }
};

}  // namespace

struct Batch {
    std::vector<Plan *> plans;           // borrowed; each holds a reference count
    std::vector<int> order;              // instances by decreasing size (work-item order)
    std::vector<LDesc> hdesc;
    DevBuf<LDesc> ddesc;
    DevBuf<IoEntry> dio;
    IoEntry *hio = nullptr;              // pinned
    std::vector<Stage> stages;           // merged launches in execution order
    DevBuf<int4> items;                  // their work items (one arena)
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool applied = false;
    Tune tune;
    float tuned_ms[4] = {0, 0, 0, 0};
    int tuned = 0;                       // 0: default tiles, 1: timed here, 2: from the cache
    ~Batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (done) (void)hipEventDestroy(done);
        if (hio) pinned_free(hio);
        for (Plan *p : plans) --p->batch_refs;
    }
};

namespace {

// Descriptors of every instance and the merged launches, from the plans' current stages.
void batch_build(Batch &B, hipStream_t st) {
    Scratch SC(st);
    const int n = (int)B.plans.size();
    std::vector<int> base(n, -1);
    B.hdesc.clear();
    for (int i : B.order) {
        Plan &P = *B.plans[i];
        base[i] = (int)B.hdesc.size();
        if (P.empty) {
            LDesc d;
            std::memset(&d, 0, sizeof(d));
            d.inst = i;
            d.nx = P.nx;
            d.ncomp = P.ncomp();
            B.hdesc.push_back(d);
            continue;
        }
        for (const LDesc &h : P.hdesc) {
            LDesc d = h;
            d.inst = i;
            B.hdesc.push_back(d);
        }
    }
    // (phase, level, role, kernel, a, b, shared memory) -> work items in instance order
    typedef std::tuple<int, int, int, int, int, int, size_t> Key;
    std::map<Key, std::vector<int4>> groups;
    auto add = [&](int phase, const Stage &S, int db) {
        std::vector<int4> &v =
            groups[Key(phase, phase == 1 ? S.level : 0, stage_role(S) + S.role_add, S.kern, S.a, S.b, S.shmem)];
        for (int4 it : S.items) {
            it.x += db;
            v.push_back(it);
        }
    };
    for (int i : B.order) {
        Plan &P = *B.plans[i];
        if (P.empty) {
            if (P.nx == 0) continue;
            Stage z;
            z.kern = K_ZERO_OUT;
            for (int64_t j = 0; j < P.nx * P.ncomp(); j += kThreadsB) z.items.push_back(make_int4(0, (int)j, 0, 0));
            add(2, z, base[i]);
            continue;
        }
        for (const Stage &S : P.pre) add(0, S, base[i]);
        for (int l = 1; l <= P.leaf; ++l)
            for (const Stage &S : P.lev[l].stages) add(1, S, base[i]);
        for (const Stage &S : P.post) add(2, S, base[i]);
    }
    B.stages.clear();
    for (auto &kv : groups) {
        Stage S;
        S.kern = std::get<3>(kv.first);
        S.a = std::get<4>(kv.first);
        S.b = std::get<5>(kv.first);
        S.shmem = std::get<6>(kv.first);
        S.level = std::get<1>(kv.first);
        S.items = std::move(kv.second);
        B.stages.push_back(std::move(S));
    }
    std::vector<Stage *> all;
    for (Stage &S : B.stages) all.push_back(&S);
    upload_stage_items(all, B.items, st, SC);
    upload_b(B.ddesc, B.hdesc, st, SC);
}

void batch_launch(const Batch &B, hipStream_t st) {
    for (const Stage &S : B.stages) run_stage(S, B.ddesc.p, B.dio.p, st);
}

void batch_capture(Batch &B) {
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    hipStream_t cs;
    FFM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    try {
        FFM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            batch_launch(B, cs);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        FFM_HIP(hipStreamEndCapture(cs, &B.graph));
        FFM_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    } catch (...) {
        (void)hipStreamDestroy(cs);
        throw;
    }
    FFM_HIP(hipStreamDestroy(cs));
}

uint64_t batch_signature(const Batch &B) {
    Sig s;
    s.add((uint64_t)B.plans.size());
    for (int i : B.order) {
        const Plan &P = *B.plans[i];
        s.add((uint64_t)P.kernel);
        s.add((uint64_t)P.nx);
        s.add((uint64_t)P.ny);
        s.add((uint64_t)P.leaf);
        for (int l = 1; l <= P.leaf; ++l) {
            const Level &LV = P.lev[l];
            s.add((uint64_t)LV.method);
            s.add((uint64_t)(LV.method == kGegenbauer ? LV.L : LV.r1));
            s.add((uint64_t)P.tx->lev[l].nbox);
            s.add((uint64_t)LV.phase64);
        }
    }
    return s.h;
}

// The cache file is one JSON object: {"<signature>": {"ring_g": G, "bwd_pt": PT, "ms": T}, ...}.
struct CacheEntry {
    int ring_g, bwd_pt;
    double ms;
};

std::map<std::string, CacheEntry> cache_read(const std::string &path) {
    std::map<std::string, CacheEntry> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while (true) {
        const size_t q0 = s.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = s.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
        const size_t ob = s.find('{', q1), cb = s.find('}', q1);
        if (ob == std::string::npos || cb == std::string::npos || cb < ob) break;
        const std::string body = s.substr(ob, cb - ob + 1);
        CacheEntry e{0, 0, 0.0};
        if (std::sscanf(body.c_str(), "{ \"ring_g\" : %d , \"bwd_pt\" : %d , \"ms\" : %lf", &e.ring_g, &e.bwd_pt, &e.ms) ==
                3 &&
            (e.ring_g == 2 || e.ring_g == 4) && (e.bwd_pt == 1 || e.bwd_pt == 2))
            m[key] = e;
        pos = cb + 1;
    }
    return m;
}

void cache_write(const std::string &path, const std::map<std::string, CacheEntry> &m) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        FFM_CHECK((bool)f, FFM_EINVAL, "ffm_batch_create: cannot write the tile cache " + path);
        f << "{\n";
        size_t i = 0;
        for (const auto &kv : m) {
            char line[256];
            std::snprintf(line, sizeof(line), "  \"%s\": {\"ring_g\": %d, \"bwd_pt\": %d, \"ms\": %.4f}%s\n",
                          kv.first.c_str(), kv.second.ring_g, kv.second.bwd_pt, kv.second.ms,
                          ++i < m.size() ? "," : "");
            f << line;
        }
        f << "}\n";
    }
    FFM_CHECK(std::rename(tmp.c_str(), path.c_str()) == 0, FFM_EINVAL, "ffm_batch_create: cannot replace " + path);
}

bool batch_has_rings(const Batch &B) {
    for (const Plan *P : B.plans)
        for (int l = 1; l <= P->leaf; ++l)
            if (P->lev[l].method == kGegenbauer && P->lev[l].L >= kRingMinL) return true;
    return false;
}

void set_all(Batch &B, const Tune &t, hipStream_t st) {
    for (Plan *P : B.plans)
        if (!P->empty) plan_set_tune(*P, t, st);
}

// Time every tile candidate on the batch (zero input, scratch output; one warm-up, best of three).
Tune autotune(Batch &B, hipStream_t st) {
    const Tune cand[4] = {{4, 2}, {4, 1}, {2, 2}, {2, 1}};
    int64_t maxny = 1, sumnx = 0;
    for (const Plan *P : B.plans) {
        maxny = std::max(maxny, P->ny);
        sumnx += P->nx * P->ncomp();
    }
    DevBuf<float2> in(maxny), out(std::max<int64_t>(sumnx, 1));
    FFM_HIP(hipMemsetAsync(in.p, 0, in.bytes(), st));
    int64_t off = 0;
    for (size_t i = 0; i < B.plans.size(); ++i) {
        B.hio[i].wu = in.p;
        B.hio[i].vout = out.p + off;
        B.hio[i].dtype = FFM_C64;
        off += B.plans[i]->nx * B.plans[i]->ncomp();
    }
    FFM_HIP(hipMemcpyAsync(B.dio.p, B.hio, B.plans.size() * sizeof(IoEntry), hipMemcpyHostToDevice, st));
    hipEvent_t e0, e1;
    FFM_HIP(hipEventCreate(&e0));
    FFM_HIP(hipEventCreate(&e1));
    int best = 0;
    try {
        for (int c = 0; c < 4; ++c) {
            set_all(B, cand[c], st);
            batch_build(B, st);
            batch_launch(B, st);
            float bestc = 1e30f;
            for (int r = 0; r < 3; ++r) {
                FFM_HIP(hipEventRecord(e0, st));
                batch_launch(B, st);
                FFM_HIP(hipEventRecord(e1, st));
                FFM_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                FFM_HIP(hipEventElapsedTime(&ms, e0, e1));
                bestc = std::min(bestc, ms);
            }
            B.tuned_ms[c] = bestc;
            if (bestc < B.tuned_ms[best]) best = c;
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FFM_HIP(hipStreamSynchronize(st));
    return cand[best];
}

}  // namespace

}  // namespace ffm

using namespace ffm;

struct ffm_batch_s {
    Batch B;
};

namespace ffm {
namespace {

int batch_create(const ffm_plan_t *plans, int32_t n, uint32_t flags, const char *tile_cache, void *hip_stream,
                 ffm_batch_t *out) {
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return set_err(FFM_EINVAL, "ffm_batch_create: a plan appears twice");
        if (plans[i]->P.batch_refs > 0) return set_err(FFM_EBUSY, "ffm_batch_create: a plan already belongs to a batch");
    }
    ffm_batch_s *h = nullptr;
    int rc = Guard::run([&] {
        std::unique_ptr<ffm_batch_s> b(new ffm_batch_s());
        Batch &B = b->B;
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        for (int32_t i = 0; i < n; ++i) {
            Plan &P = plans[i]->P;
            plan_sync_ready(P);
            if (P.applied) FFM_HIP(hipEventSynchronize(P.done));
            B.plans.push_back(&P);
            ++P.batch_refs;
        }
        B.order.resize(n);
        for (int i = 0; i < n; ++i) B.order[i] = i;
        std::stable_sort(B.order.begin(), B.order.end(), [&](int a, int c) {
            return B.plans[a]->nx + B.plans[a]->ny > B.plans[c]->nx + B.plans[c]->ny;
        });
        B.dio.alloc(n);
        B.hio = static_cast<IoEntry *>(pinned_alloc(sizeof(IoEntry) * n));
        std::memset(B.hio, 0, sizeof(IoEntry) * n);
        FFM_HIP(hipEventCreateWithFlags(&B.done, hipEventDisableTiming));
        if ((flags & FFM_BATCH_AUTOTUNE) && batch_has_rings(B)) {
            const std::string path = tile_cache ? tile_cache : "";
            char key[32];
            std::snprintf(key, sizeof(key), "%016llx", (unsigned long long)batch_signature(B));
            std::map<std::string, CacheEntry> m;
            if (!path.empty()) m = cache_read(path);
            auto it = m.find(key);
            if (it != m.end()) {
                B.tune.ring_g = it->second.ring_g;
                B.tune.bwd_pt = it->second.bwd_pt;
                B.tuned = 2;
            } else {
                B.tune = autotune(B, st);
                B.tuned = 1;
                if (!path.empty()) {
                    const int c = (B.tune.ring_g == 4 ? 0 : 2) + (B.tune.bwd_pt == 2 ? 0 : 1);
                    m[key] = CacheEntry{B.tune.ring_g, B.tune.bwd_pt, (double)B.tuned_ms[c]};
                    cache_write(path, m);
                }
            }
            set_all(B, B.tune, st);
        } else {
            B.tune = B.plans[0]->tune;
        }
        batch_build(B, st);
        FFM_HIP(hipStreamSynchronize(st));
        if (flags & FFM_BATCH_GRAPH) {
            B.use_graph = true;
            batch_capture(B);
        }
        h = b.release();
    });
    if (rc == FFM_OK) *out = h;
    return rc;
}

// The batch ffm_apply_batched builds for the plan set of its last call (graph-captured), kept for the next call
// with the same plans in the same order.  Its plans count it in batch_refs like any batch; destroying,
// retiling or batching one of them first releases it (implicit_batch_drop).
std::mutex g_imx;
ffm_batch_s *g_implicit = nullptr;
std::vector<ffm_plan_t> g_implicit_plans;

// with g_imx held: wait for the implicit batch's last apply and free it
void implicit_free_locked() {
    if (!g_implicit) return;
    if (g_implicit->B.applied) FFM_HIP(hipEventSynchronize(g_implicit->B.done));
    delete g_implicit;
    g_implicit = nullptr;
    g_implicit_plans.clear();
}

}  // namespace

int implicit_batch_drop(const Plan *P, bool wait) {
    std::lock_guard<std::mutex> lk(g_imx);
    if (!g_implicit) return FFM_OK;
    bool holds = false;
    for (Plan *q : g_implicit->B.plans) holds = holds || q == P;
    if (!holds) return FFM_OK;
    if (!wait && g_implicit->B.applied && hipEventQuery(g_implicit->B.done) == hipErrorNotReady)
        return set_err(FFM_EBUSY, "a batched apply of the plan is still in flight");
    return Guard::run([&] { implicit_free_locked(); });
}

}  // namespace ffm

extern "C" {

ffm_status_t ffm_plan_set_tiles(ffm_plan_t plan, const ffm_tiles_t *tiles, void *hip_stream) {
    if (!plan || !tiles) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_set_tiles: NULL argument");
    if ((tiles->ring_g != 2 && tiles->ring_g != 4) || (tiles->bwd_pt != 1 && tiles->bwd_pt != 2))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_set_tiles: ring_g must be 2 or 4, bwd_pt 1 or 2");
    Plan &P = plan->P;
    if (int rc = implicit_batch_drop(&P, true)) return (ffm_status_t)rc;
    if (P.batch_refs > 0) return (ffm_status_t)set_err(FFM_EBUSY, "ffm_plan_set_tiles: the plan belongs to a batch");
    if (P.server_refs > 0) return (ffm_status_t)set_err(FFM_EBUSY, "ffm_plan_set_tiles: server requests of the plan are pending");
    return (ffm_status_t)Guard::run([&] {
        plan_sync_ready(P);
        if (P.applied) FFM_HIP(hipEventSynchronize(P.done));
        Tune t;
        t.ring_g = tiles->ring_g;
        t.bwd_pt = tiles->bwd_pt;
        plan_set_tune(P, t, static_cast<hipStream_t>(hip_stream));
    });
}

ffm_status_t ffm_plan_get_tiles(ffm_plan_t plan, ffm_tiles_t *tiles) {
    if (!plan || !tiles) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_get_tiles: NULL argument");
    tiles->ring_g = plan->P.tune.ring_g;
    tiles->bwd_pt = plan->P.tune.bwd_pt;
    return FFM_OK;
}

ffm_status_t ffm_batch_create(const ffm_plan_t *plans, int32_t n, uint32_t flags, const char *tile_cache,
                              void *hip_stream, ffm_batch_t *out) {
    if (!out) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_batch_create: out is NULL");
    *out = nullptr;
    if (!plans || n <= 0) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_batch_create: need at least one plan");
    if (flags & ~(uint32_t)(FFM_BATCH_GRAPH | FFM_BATCH_AUTOTUNE))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_batch_create: unknown flags");
    for (int32_t i = 0; i < n; ++i)
        if (!plans[i]) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_batch_create: NULL plan");
    // a plan held only by the batch that ffm_apply_batched keeps is released from it
    for (int32_t i = 0; i < n; ++i) {
        int rc = implicit_batch_drop(&plans[i]->P, true);
        if (rc != FFM_OK) return (ffm_status_t)rc;
    }
    return (ffm_status_t)batch_create(plans, n, flags, tile_cache, hip_stream, out);
}

ffm_status_t ffm_batch_apply(ffm_batch_t batch, const void *const *wu, const ffm_dtype_t *in_dtype, void *const *v,
                             void *hip_stream) {
    if (!batch || !wu || !in_dtype || !v) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_batch_apply: NULL argument");
    Batch &B = batch->B;
    const size_t n = B.plans.size();
    for (size_t i = 0; i < n; ++i) {
        if (in_dtype[i] < FFM_C64 || in_dtype[i] > FFM_C128)
            return (ffm_status_t)set_err(FFM_EINVAL, "ffm_batch_apply: bad dtype");
        if ((B.plans[i]->ny > 0 && !wu[i]) || (B.plans[i]->nx > 0 && !v[i]))
            return (ffm_status_t)set_err(FFM_EINVAL, "ffm_batch_apply: NULL input or output");
    }
    return (ffm_status_t)Guard::run([&] {
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        // the pinned table is read by the previous apply's copy until that apply's event completes
        if (B.applied) FFM_HIP(hipEventSynchronize(B.done));
        for (size_t i = 0; i < n; ++i) {
            B.hio[i].wu = wu[i];
            B.hio[i].vout = static_cast<float2 *>(v[i]);
            B.hio[i].dtype = (int)in_dtype[i];
        }
        FFM_HIP(hipMemcpyAsync(B.dio.p, B.hio, n * sizeof(IoEntry), hipMemcpyHostToDevice, st));
        if (B.use_graph) {
            FFM_HIP(hipGraphLaunch(B.exec, st));
        } else {
            batch_launch(B, st);
        }
        FFM_HIP(hipEventRecord(B.done, st));
        B.applied = true;
    });
}

ffm_status_t ffm_batch_info(ffm_batch_t batch, ffm_batch_info_t *out) {
    if (!batch || !out) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_batch_info: NULL argument");
    const Batch &B = batch->B;
    out->n = (int32_t)B.plans.size();
    out->launches = (int32_t)B.stages.size();
    out->graph = B.use_graph ? 1 : 0;
    out->tuned = B.tuned;
    out->tiles.ring_g = B.tune.ring_g;
    out->tiles.bwd_pt = B.tune.bwd_pt;
    for (int c = 0; c < 4; ++c) out->tuned_ms[c] = B.tuned_ms[c];
    int64_t items = 0;
    for (const Stage &S : B.stages) items += (int64_t)S.items.size();
    out->work_items = items;
    return FFM_OK;
}

ffm_status_t ffm_batch_destroy(ffm_batch_t batch) {
    if (!batch) return FFM_OK;
    if (batch->B.applied) {
        hipError_t q = hipEventQuery(batch->B.done);
        if (q == hipErrorNotReady) return (ffm_status_t)set_err(FFM_EBUSY, "ffm_batch_destroy: an apply is still in flight");
    }
    return (ffm_status_t)Guard::run([&] { delete batch; });
}

ffm_status_t ffm_apply_batched(const ffm_plan_t *plans, const void *const *wu, void *const *v, int32_t n,
                               void *hip_stream) {
    if (!plans || !wu || !v || n <= 0) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply_batched: NULL argument or n <= 0");
    for (int32_t i = 0; i < n; ++i) {
        if (!plans[i]) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply_batched: NULL plan");
        if ((plans[i]->P.ny > 0 && !wu[i]) || (plans[i]->P.nx > 0 && !v[i]))
            return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply_batched: NULL input or output");
    }
    std::lock_guard<std::mutex> lk(g_imx);
    const bool same = g_implicit && (int32_t)g_implicit_plans.size() == n &&
                      std::equal(g_implicit_plans.begin(), g_implicit_plans.end(), plans);
    if (!same) {
        int rc = Guard::run([&] { implicit_free_locked(); });
        if (rc != FFM_OK) return (ffm_status_t)rc;
        ffm_batch_t b = nullptr;
        rc = batch_create(plans, n, FFM_BATCH_GRAPH, nullptr, hip_stream, &b);
        if (rc != FFM_OK) return (ffm_status_t)rc;
        g_implicit = b;
        g_implicit_plans.assign(plans, plans + n);
    }
    std::vector<ffm_dtype_t> dt((size_t)n, FFM_C64);
    return ffm_batch_apply(g_implicit, wu, dt.data(), v, hip_stream);
}

}  // extern "C"
