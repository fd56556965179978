// The C ABI of include/ffm.h: argument checks, error mapping, ownership.
#include <cstring>
#include "common.h"

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

namespace ffm {

namespace {
thread_local std::string g_err;
std::atomic<long long> g_alloc_count{0};
std::atomic<long long> g_live_bytes{0};

long long fail_after() {
    static long long v = [] {
        const char *e = std::getenv("FFM_TEST_FAIL_ALLOC_AFTER");
        return e ? std::atoll(e) : -1LL;
    }();
    return v;
}

}  // namespace

int set_err(int code, const std::string &msg) {
    g_err = msg;
    return code;
}
void clear_err() { g_err.clear(); }

// Device memory comes from a process-wide cache: a freed block goes back to a free list keyed by its
// rounded size and the next request of that size takes it without a hipMalloc.  Plans are rebuilt
// with the same shapes again and again (an iterative solve, a serving loop), so after the first plan
// no allocation reaches the runtime.  Every block is released to the free list only after the stream
// work that used it has completed (plan building synchronises; destroy refuses an in-flight plan).
namespace {
std::mutex g_mx;
std::unordered_map<void *, size_t> g_live;     // pointer -> rounded size
std::multimap<size_t, void *> g_free;          // rounded size -> cached block
size_t g_cached = 0;

size_t round_size(size_t b) {
    if (b <= ((size_t)1 << 20)) {
        size_t s = 256;
        while (s < b) s <<= 1;
        return s;
    }
    const size_t g = (size_t)2 << 20;
    return (b + g - 1) / g * g;
}

void release_cache_locked() {
    for (auto &kv : g_free) (void)hipFree(kv.second);
    g_free.clear();
    g_cached = 0;
}
}  // namespace

void *dev_alloc(size_t bytes) {
    const long long n = g_alloc_count.fetch_add(1);
    const long long lim = fail_after();
    if (lim >= 0 && n == lim) throw Error(FFM_ENOMEM, "device allocation refused by FFM_TEST_FAIL_ALLOC_AFTER");
    const size_t sz = round_size(bytes);
    std::lock_guard<std::mutex> lk(g_mx);
    auto it = g_free.find(sz);
    void *p = nullptr;
    if (it != g_free.end()) {
        p = it->second;
        g_free.erase(it);
        g_cached -= sz;
    } else {
        hipError_t e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            release_cache_locked();
            e = hipMalloc(&p, sz);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Error(FFM_ENOMEM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
            }
        }
    }
    g_live[p] = sz;
    g_live_bytes += (long long)sz;
    return p;
}

void dev_free(void *p) {
    std::lock_guard<std::mutex> lk(g_mx);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    const size_t sz = it->second;
    g_live.erase(it);
    g_live_bytes -= (long long)sz;
    g_free.emplace(sz, p);
    g_cached += sz;
}

namespace {
std::mutex g_pmx;
std::unordered_map<void *, size_t> g_plive;
std::multimap<size_t, void *> g_pfree;
}  // namespace

void *pinned_alloc(size_t bytes) {
    const size_t sz = round_size(bytes);
    std::lock_guard<std::mutex> lk(g_pmx);
    auto it = g_pfree.find(sz);
    void *p = nullptr;
    if (it != g_pfree.end()) {
        p = it->second;
        g_pfree.erase(it);
    } else {
        hipError_t e = hipHostMalloc(&p, sz, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(FFM_ENOMEM, std::string("hipHostMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
        }
    }
    g_plive[p] = sz;
    return p;
}

void pinned_free(void *p) {
    std::lock_guard<std::mutex> lk(g_pmx);
    auto it = g_plive.find(p);
    if (it == g_plive.end()) return;
    g_pfree.emplace(it->second, p);
    g_plive.erase(it);
}

size_t dev_bytes_live() { return (size_t)std::max<long long>(0, g_live_bytes.load()); }

size_t dev_bytes_cached() {
    std::lock_guard<std::mutex> lk(g_mx);
    return g_cached;
}

}  // namespace ffm

using namespace ffm;

extern "C" {

const char *ffm_last_error(void) { return g_err.c_str(); }

const char *ffm_version(void) { return "ffm-gfx950 0.1"; }

ffm_status_t ffm_plan(const double *X, int64_t n_x, const double *Y, int64_t n_y, ffm_kernel_t kernel, double k,
                      double eps, const ffm_options_t *opts, void *hip_stream, ffm_plan_t *out) {
    if (!out) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: out is NULL");
    if (n_x < 0 || n_y < 0 || n_x >= (int64_t(1) << 31) || n_y >= (int64_t(1) << 31))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: sizes must be in [0, 2^31)");
    if ((n_x > 0 && !X) || (n_y > 0 && !Y)) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: NULL coordinates");
    if (kernel != FFM_LAPLACE && kernel != FFM_HELMHOLTZ && kernel != FFM_LAPLACE_DN && kernel != FFM_HELMHOLTZ_DN &&
        kernel != FFM_LAPLACE_DL && kernel != FFM_HELMHOLTZ_DL && kernel != FFM_LAPLACE_GRAD &&
        kernel != FFM_HELMHOLTZ_GRAD)
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: unknown kernel");
    const bool grad = kernel == FFM_LAPLACE_GRAD || kernel == FFM_HELMHOLTZ_GRAD;
    const bool dn = kernel == FFM_LAPLACE_DN || kernel == FFM_HELMHOLTZ_DN;
    const bool dl = kernel == FFM_LAPLACE_DL || kernel == FFM_HELMHOLTZ_DL;
    if (dn && n_x > 0 && !(opts && opts->target_normals))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: normal-derivative kernels need options.target_normals");
    if (dl && n_y > 0 && !(opts && opts->source_normals))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: double-layer kernels need options.source_normals");
    if (!(eps >= 1e-7 && eps < 0.5)) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: eps must be in [1e-7, 0.5)");
    if (!(k >= 0.0) || !std::isfinite(k)) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: k must be finite and >= 0");
    ffm_options_t o{};
    if (opts) o = *opts;
    if (o.flags & ~(FFM_FLAG_TIMING | FFM_FLAG_DIRECT_TRANSFORMS | FFM_FLAG_GRID_TRANSFORMS | FFM_FLAG_NO_ACA | FFM_FLAG_ACA |
                    FFM_FLAG_ADAPTIVE_LEAVES))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: unknown options.flags bits");
    if ((o.flags & FFM_FLAG_DIRECT_TRANSFORMS) && (o.flags & FFM_FLAG_GRID_TRANSFORMS))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: direct and grid transforms both forced");
    if ((o.flags & FFM_FLAG_NO_ACA) && (o.flags & FFM_FLAG_ACA))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: ACA both forbidden and forced");
    if (o.n_leaf < 0 || o.max_level < 0 || o.max_level > kMaxLev || o.r1_override < 0 || o.r1_override > 8 ||
        !(o.kd_switch >= 0.0) || (o.precision != FFM_PREC_FP32 && o.precision != FFM_PREC_MIXED))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan: invalid options");
    if (o.n_leaf == 0) o.n_leaf = 64;
    if (o.max_level == 0) o.max_level = kMaxLev;
    if (o.kd_switch == 0.0) o.kd_switch = M_PI;
    *out = nullptr;
    ffm_plan_s *h = nullptr;
    int rc = Guard::run([&] {
        std::unique_ptr<ffm_plan_s> p(new ffm_plan_s());
        Plan &P = p->P;
        P.dn = dn;
        P.grad = grad;
        P.user_normals = dn ? o.target_normals : nullptr;
        P.dl = dl;
        P.user_snormals = dl ? o.source_normals : nullptr;
        P.kernel = (kernel == FFM_HELMHOLTZ || kernel == FFM_HELMHOLTZ_DN || kernel == FFM_HELMHOLTZ_DL ||
                    kernel == FFM_HELMHOLTZ_GRAD) ? FFM_HELMHOLTZ : FFM_LAPLACE;
        P.k = P.kernel == FFM_HELMHOLTZ ? k : 0.0;
        P.eps = eps;
        P.opt = o;
        P.nx = n_x;
        P.ny = n_y;
        P.same = (X == Y && n_x == n_y);
        P.empty = (n_x == 0 || n_y == 0);
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        plan_build(P, X, Y, st);
        P.user_normals = nullptr;
        P.user_snormals = nullptr;
        FFM_HIP(hipEventCreateWithFlags(&P.ready, hipEventDisableTiming));
        FFM_HIP(hipEventRecord(P.ready, st));
        FFM_HIP(hipEventCreateWithFlags(&P.done, hipEventDisableTiming));
        if (o.flags & FFM_FLAG_TIMING) {
            P.tev.resize(12 * kMaxLev + 16, nullptr);   // one event per launch (more are made as needed)
            P.tphase.assign(P.tev.size(), -1);
            P.tkern.assign(P.tev.size(), make_int4(-1, 0, 0, 0));
            P.tblocks.assign(P.tev.size(), 0);
            for (auto &e : P.tev) FFM_HIP(hipEventCreate(&e));
        }
        P.stats.plan_bytes = (double)plan_device_bytes(P);
        P.stats.workspace_bytes = (double)apply_work_bytes(P);
        h = p.release();
    });
    if (rc == FFM_OK) *out = h;
    return (ffm_status_t)rc;
}

ffm_status_t ffm_apply(ffm_plan_t plan, const void *wu, ffm_dtype_t in_dtype, void *v, void *hip_stream) {
    if (!plan) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply: NULL plan");
    Plan &P = plan->P;
    if (P.nx > 0 && !v) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply: NULL output");
    if (P.ny > 0 && !wu) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply: NULL input");
    if (in_dtype < FFM_C64 || in_dtype > FFM_C128) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply: bad dtype");
    return (ffm_status_t)Guard::run([&] {
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        plan_apply(P, wu, (int)in_dtype, static_cast<float2 *>(v), st);
        if (P.done) FFM_HIP(hipEventRecord(P.done, st));
        P.applied = true;
    });
}

ffm_status_t ffm_destroy(ffm_plan_t plan) {
    if (!plan) return FFM_OK;
    if (int rc = implicit_batch_drop(&plan->P, false)) return (ffm_status_t)rc;
    if (plan->P.batch_refs > 0) return (ffm_status_t)set_err(FFM_EBUSY, "ffm_destroy: the plan belongs to a batch");
    if (plan->P.server_refs > 0) return (ffm_status_t)set_err(FFM_EBUSY, "ffm_destroy: server requests of the plan are pending");
    if (plan->P.done && plan->P.applied) {
        hipError_t q = hipEventQuery(plan->P.done);
        if (q == hipErrorNotReady) return (ffm_status_t)set_err(FFM_EBUSY, "ffm_destroy: an apply is still in flight");
    }
    if (plan->P.sdone && plan->P.sapplied && hipEventQuery(plan->P.sdone) == hipErrorNotReady)
        return (ffm_status_t)set_err(FFM_EBUSY, "ffm_destroy: a static-workspace apply is still in flight");
    return (ffm_status_t)Guard::run([&] {
        plan_sync_ready(plan->P);
        if (plan->P.ready) (void)hipEventDestroy(plan->P.ready);
        if (plan->P.done) (void)hipEventDestroy(plan->P.done);
        if (plan->P.sdone) (void)hipEventDestroy(plan->P.sdone);
        if (plan->P.hio) pinned_free(plan->P.hio);
        if (plan->P.spin) pinned_free(plan->P.spin);
        for (auto e : plan->P.tev)
            if (e) (void)hipEventDestroy(e);
        delete plan;
    });
}

ffm_status_t ffm_plan_timing(ffm_plan_t plan, float *ms, int32_t n) {
    if (!plan || !ms || n < FFM_TIMING_SLOTS) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_timing: bad argument");
    Plan &P = plan->P;
    if (P.tev.empty()) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_timing: plan made without FFM_FLAG_TIMING");
    return (ffm_status_t)Guard::run([&] {
        for (int i = 0; i < n; ++i) ms[i] = 0.f;
        if (P.tused < 2) return;
        FFM_HIP(hipEventSynchronize(P.tev[P.tused - 1]));
        for (int i = 1; i < P.tused; ++i) {
            float t = 0.f;
            FFM_HIP(hipEventElapsedTime(&t, P.tev[i - 1], P.tev[i]));
            if (P.tphase[i] >= 0 && P.tphase[i] < n) ms[P.tphase[i]] += t;
        }
    });
}

ffm_status_t ffm_plan_launch_timing(ffm_plan_t plan, ffm_launch_t *out, int32_t n, int32_t *count) {
    if (!plan || !count || n < 0 || (n > 0 && !out))
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_launch_timing: bad argument");
    Plan &P = plan->P;
    if (P.tev.empty())
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_launch_timing: plan made without FFM_FLAG_TIMING");
    return (ffm_status_t)Guard::run([&] {
        *count = 0;
        if (P.tused < 2) return;
        FFM_HIP(hipEventSynchronize(P.tev[P.tused - 1]));
        int32_t k = 0;
        for (int i = 1; i < P.tused; ++i) {
            if (P.tkern[i].x < 0) continue;
            if (k < n) {
                float t = 0.f;
                FFM_HIP(hipEventElapsedTime(&t, P.tev[i - 1], P.tev[i]));
                ffm_launch_t &r = out[k];
                r.kernel = P.tkern[i].x;
                r.variant_a = P.tkern[i].y;
                r.variant_b = P.tkern[i].z;
                r.level = P.tkern[i].w;
                r.blocks = P.tblocks[i];
                r.ms = t;
                r.reserved = 0;
            }
            ++k;
        }
        *count = k;
    });
}

int32_t ffm_kernel_name(int32_t kernel, int32_t variant_a, int32_t variant_b, char *buf, int32_t n) {
    const std::string s = kernel_name(kernel, variant_a, variant_b);
    if (s.empty()) return -1;
    if (buf && n > 0) {
        const size_t m = std::min((size_t)n - 1, s.size());
        std::memcpy(buf, s.data(), m);
        buf[m] = 0;
    }
    return (int32_t)s.size();
}

ffm_status_t ffm_plan_stats(ffm_plan_t plan, ffm_stats_t *out) {
    if (!plan || !out) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_stats: NULL argument");
    *out = plan->P.stats;
    return FFM_OK;
}

ffm_status_t ffm_plan_export(ffm_plan_t plan, int32_t what, int32_t set, int32_t level, void *dst, int64_t *count) {
    if (!plan || !count) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_export: NULL argument");
    Plan &P = plan->P;
    if (set < 0 || set > 1) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_export: set must be 0 or 1");
    if (P.empty) {
        *count = 0;
        return FFM_OK;
    }
    if (level < 0 || level > P.leaf) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_plan_export: level out of range");
    return (ffm_status_t)Guard::run([&] {
        plan_sync_ready(P);
        const Tree &T = set == 0 ? *P.tx : *P.ty;
        const TreeLevel &TL = T.lev[level];
        const Level &LV = P.lev[level];
        auto copy = [&](const void *src, size_t bytes) {
            if (dst && bytes) FFM_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        };
        switch (what) {
            case FFM_EXPORT_KEYS:
                *count = T.n;
                copy(T.key.p, sizeof(uint64_t) * T.n);
                break;
            case FFM_EXPORT_PERM: {
                *count = T.n;
                if (dst) {
                    std::vector<int32_t> h(T.n);
                    FFM_HIP(hipMemcpy(h.data(), T.perm.p, sizeof(int32_t) * T.n, hipMemcpyDeviceToHost));
                    for (int64_t i = 0; i < T.n; ++i) static_cast<int64_t *>(dst)[i] = h[i];
                }
                break;
            }
            case FFM_EXPORT_BOX_START: {
                *count = TL.nbox + 1;
                if (dst) {
                    std::vector<int32_t> h(TL.nbox + 1);
                    FFM_HIP(hipMemcpy(h.data(), TL.start.p, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost));
                    for (size_t i = 0; i < h.size(); ++i) static_cast<int64_t *>(dst)[i] = h[i];
                }
                break;
            }
            case FFM_EXPORT_BOX_IJK:
                *count = 3 * (int64_t)TL.nbox;
                copy(TL.ijk.p, sizeof(int32_t) * 3 * TL.nbox);
                break;
            case FFM_EXPORT_BOX_CTR:
                *count = 3 * (int64_t)TL.nbox;
                copy(TL.ctr.p, sizeof(double) * 3 * TL.nbox);
                break;
            case FFM_EXPORT_FAR:
            case FFM_EXPORT_NEAR: {
                const bool far = what == FFM_EXPORT_FAR;
                const int64_t n = far ? LV.nfar : LV.nnear;
                const int w = far ? 5 : 2;
                *count = (int64_t)w * n;
                if (!dst || level == 0) {
                    if (level == 0) *count = far ? 0 : 2;
                    if (dst && level == 0 && !far) {
                        static_cast<int64_t *>(dst)[0] = 0;
                        static_cast<int64_t *>(dst)[1] = 0;
                    }
                    break;
                }
                const int32_t nbx = P.tx->lev[level].nbox;
                std::vector<int64_t> ptr(nbx + 1);
                std::vector<int32_t> src(n), cls;
                FFM_HIP(hipMemcpy(ptr.data(), far ? LV.far_ptr.p : LV.near_ptr.p, sizeof(int64_t) * (nbx + 1),
                                  hipMemcpyDeviceToHost));
                if (n)
                    FFM_HIP(hipMemcpy(src.data(), far ? LV.far_src.p : LV.near_src.p, sizeof(int32_t) * n,
                                      hipMemcpyDeviceToHost));
                if (far && n) {
                    cls.resize(n);
                    FFM_HIP(hipMemcpy(cls.data(), LV.far_cls.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
                }
                int64_t *o = static_cast<int64_t *>(dst);
                for (int32_t t = 0; t < nbx; ++t)
                    for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) {
                        o[0] = t;
                        o[1] = src[e];
                        if (far) {
                            o[2] = LV.cls_off[3 * cls[e]];
                            o[3] = LV.cls_off[3 * cls[e] + 1];
                            o[4] = LV.cls_off[3 * cls[e] + 2];
                        }
                        o += w;
                    }
                break;
            }
            case FFM_EXPORT_EARLY: {
                const int64_t n = level >= 1 && level < P.leaf ? LV.nearly : 0;
                *count = 2 * n;
                if (!dst || n == 0) break;
                const int32_t nbx = P.tx->lev[level].nbox;
                std::vector<int64_t> ptr(nbx + 1);
                std::vector<int32_t> src(n);
                FFM_HIP(hipMemcpy(ptr.data(), LV.early_ptr.p, sizeof(int64_t) * (nbx + 1), hipMemcpyDeviceToHost));
                FFM_HIP(hipMemcpy(src.data(), LV.early_src.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
                int64_t *o = static_cast<int64_t *>(dst);
                for (int32_t t = 0; t < nbx; ++t)
                    for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) {
                        o[0] = t;
                        o[1] = src[e];
                        o += 2;
                    }
                break;
            }
            case FFM_EXPORT_ACA_RANK: {
                const bool has = LV.method == kLagrange && LV.aca && level >= 1;
                *count = has ? 4 * (int64_t)LV.ncls : 0;
                if (dst && has) {
                    int64_t *o = static_cast<int64_t *>(dst);
                    for (int c = 0; c < LV.ncls; ++c) {
                        o[4 * c] = LV.cls_off[3 * c];
                        o[4 * c + 1] = LV.cls_off[3 * c + 1];
                        o[4 * c + 2] = LV.cls_off[3 * c + 2];
                        o[4 * c + 3] = LV.aca_ranks[c];
                    }
                }
                break;
            }
            default:
                throw Error(FFM_EINVAL, "ffm_plan_export: unknown array");
        }
    });
}

size_t ffm_plan_bytes(ffm_plan_t plan) { return plan ? plan_device_bytes(plan->P) : 0; }

size_t ffm_workspace_bytes(ffm_plan_t plan) { return plan ? apply_work_bytes(plan->P) : 0; }

size_t ffm_device_bytes_live(void) { return dev_bytes_live(); }

}  // extern "C"
