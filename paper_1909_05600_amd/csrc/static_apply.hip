// Apply over a workspace the library holds in static device memory, for callers that cannot allocate (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The workspace is one file-scope __device__ array of kScratchBytes: every device the library runs on holds its
// own copy until the process ends.  Host code never passes the array's name to a kernel (on the host it names a
// host-side stand-in, not device memory): the device address of each device's copy is taken once per device
// with hipGetSymbolAddress, with that device current, and kept.  A plan whose apply workspace fits gets, when it
// is built, level descriptors that point into that address (carved like a server request's workspace), so the
// apply itself only copies its I/O entry and launches the plan's stages: the same kernels, work items and
// arithmetic as ffm_apply, over another workspace.  Every apply over the array on a device shares it: the
// kernels clear what must start at zero (the sorted output and the maximum |u|) and write everything else
// before reading it, and applies that overlap on one device race.
#include "common.h"

#include <map>
#include <mutex>

namespace ffm {

namespace {

constexpr size_t kScratchBytes = FFM_STATIC_WORKSPACE_BYTES;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_smx;
std::map<int, char *> g_sptr;   // device -> address of its copy of the array

__global__ void __launch_bounds__(256) k_fill_zero(float2 *v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = make_float2(0.f, 0.f);
}

}  // namespace

char *static_work_base() {
    int dev = 0;
    FFM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_smx);
    auto it = g_sptr.find(dev);
    if (it != g_sptr.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        throw Error(FFM_EDEVICE, std::string("hipGetSymbolAddress(static workspace): ") + hipGetErrorString(e));
    }
    g_sptr[dev] = static_cast<char *>(ptr);
    return static_cast<char *>(ptr);
}

void plan_static_setup(Plan &P, hipStream_t st) {
    // rebuilt with the plan's launches (a new tile choice can change the workspace's layout): the last static
    // apply must be done with the old descriptors
    if (P.sapplied) FFM_HIP(hipEventSynchronize(P.sdone));
    P.sdesc.release();
    P.sdio.release();
    if (P.spin) pinned_free(P.spin);
    P.spin = nullptr;
    P.shio = nullptr;
    if (P.empty || apply_work_bytes(P) > kScratchBytes) return;
    char *base = static_work_base();
    const WorkPtrs w = carve_work(P, base);
    const int nd = plan_ndesc(P);
    // pinned host block held by the plan: the descriptors (copied once, here) and the I/O entry of each apply
    P.spin = pinned_alloc(sizeof(LDesc) * nd + sizeof(IoEntry));
    LDesc *hd = static_cast<LDesc *>(P.spin);
    for (int k = 0; k < nd; ++k) hd[k] = plan_desc(P, k, 0, w.u, w.v, w.amax, w.lw);
    P.shio = reinterpret_cast<IoEntry *>(hd + nd);
    std::memset(P.shio, 0, sizeof(IoEntry));
    P.sdesc.alloc((size_t)nd);
    P.sdio.alloc(1);
    FFM_HIP(hipMemcpyAsync(P.sdesc.p, hd, sizeof(LDesc) * nd, hipMemcpyHostToDevice, st));
    if (!P.sdone) FFM_HIP(hipEventCreateWithFlags(&P.sdone, hipEventDisableTiming));
    P.sapplied = false;
}

}  // namespace ffm

using namespace ffm;

extern "C" {

ffm_status_t ffm_apply_static(ffm_plan_t plan, const void *wu, ffm_dtype_t in_dtype, void *v, void *hip_stream) {
    if (!plan) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply_static: NULL plan");
    Plan &P = plan->P;
    if (P.nx > 0 && !v) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply_static: NULL output");
    if (P.ny > 0 && !wu) return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply_static: NULL input");
    if (in_dtype < FFM_C64 || in_dtype > FFM_C128)
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply_static: bad dtype");
    if (!P.empty && !P.sdesc.p)
        return (ffm_status_t)set_err(FFM_EINVAL, "ffm_apply_static: the plan's apply workspace (" +
                                                     std::to_string(apply_work_bytes(P)) +
                                                     " bytes) exceeds the static workspace (" +
                                                     std::to_string(kScratchBytes) + " bytes)");
    return (ffm_status_t)Guard::run([&] {
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        if (P.empty) {
            if (P.nx > 0)
                FFM_LAUNCH(k_fill_zero, (int)((P.nx * P.ncomp() + 255) / 256), 256, 0, st, static_cast<float2 *>(v),
                           P.nx * P.ncomp());
            return;
        }
        // the pinned I/O entry is read by the previous static apply's copy until that apply's event completes
        if (P.sapplied) FFM_HIP(hipEventSynchronize(P.sdone));
        // the plan's last tables, launch lists and these descriptors may still be copied on the planning stream
        if (P.ready) FFM_HIP(hipStreamWaitEvent(st, P.ready, 0));
        P.shio->wu = wu;
        P.shio->vout = static_cast<float2 *>(v);
        P.shio->dtype = (int)in_dtype;
        FFM_HIP(hipMemcpyAsync(P.sdio.p, P.shio, sizeof(IoEntry), hipMemcpyHostToDevice, st));
        for (const Stage &S : P.pre) run_stage(S, P.sdesc.p, P.sdio.p, st);
        for (int l = 1; l <= P.leaf; ++l)
            for (const Stage &S : P.lev[l].stages) run_stage(S, P.sdesc.p, P.sdio.p, st);
        for (const Stage &S : P.post) run_stage(S, P.sdesc.p, P.sdio.p, st);
        FFM_HIP(hipEventRecord(P.sdone, st));
        P.sapplied = true;
    });
}

}  // extern "C"
