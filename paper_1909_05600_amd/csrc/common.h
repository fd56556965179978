// Internal declarations of the gfx950 FFM library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "ffm.h"

namespace ffm {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define FFM_HIP(x)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess)                                                                       \
            throw ::ffm::Error(e_ == hipErrorOutOfMemory ? FFM_ENOMEM : FFM_EDEVICE,                \
                               std::string(#x) + ": " + hipGetErrorString(e_));                     \
    } while (0)

#define FFM_CHECK(cond, code, msg)                                                                  \
    do {                                                                                            \
        if (!(cond)) throw ::ffm::Error((code), (msg));                                             \
    } while (0)

// Kernel launches go through this so a bad configuration becomes an error, not a fault.
#define FFM_LAUNCH(kern, grid, block, shmem, stream, ...)                                           \
    do {                                                                                            \
        if ((grid) > 0) {                                                                           \
            hipLaunchKernelGGL(kern, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__);          \
            FFM_HIP(hipGetLastError());                                                             \
        }                                                                                           \
    } while (0)

// Test hook: FFM_TEST_FAIL_ALLOC_AFTER=n makes the (n+1)-th device allocation fail.
void *dev_alloc(size_t bytes);
void dev_free(void *p);
size_t dev_bytes_live();
// Pinned host staging memory (cached like device memory) for asynchronous uploads.
void *pinned_alloc(size_t bytes);
void pinned_free(void *p);

// ---------------------------------------------------------------- device buffer
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        p = count ? static_cast<T *>(dev_alloc(count * sizeof(T))) : nullptr;
    }
    void release() {
        if (p) dev_free(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// Temporaries that must outlive the stream work using them: device buffers and pinned host
// staging, released together when the scratch list goes out of scope, after its stream drains.
struct Scratch {
    hipStream_t stream = nullptr;
    std::vector<DevBuf<char>> bufs;
    std::vector<void *> pinned;
    explicit Scratch(hipStream_t st) : stream(st) {}
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    ~Scratch() {
        (void)hipStreamSynchronize(stream);
        for (void *p : pinned) pinned_free(p);
    }
    template <class T>
    T *get(size_t count) {
        bufs.emplace_back(count * sizeof(T));
        return reinterpret_cast<T *>(bufs.back().p);
    }
    // copy host data into pinned staging memory that stays valid until the scratch list is released
    template <class T>
    const T *stage(const std::vector<T> &h) {
        void *p = pinned_alloc(std::max<size_t>(h.size() * sizeof(T), 1));
        pinned.push_back(p);
        if (!h.empty()) std::memcpy(p, h.data(), h.size() * sizeof(T));
        return static_cast<const T *>(p);
    }
};

// ---------------------------------------------------------------- plan data
constexpr int kBits = 21;                 // Morton bits per axis
constexpr int kMaxLev = 20;               // deepest level
constexpr int kWin = 12;                  // translation window per axis
constexpr int kWin3 = kWin * kWin * kWin; // window cells per level

struct TreeLevel {
    int32_t nbox = 0;
    DevBuf<int32_t> start;    // [nbox + 1] sorted point ranges
    DevBuf<int32_t> ijk;      // [nbox][3] integer box coordinates
    DevBuf<double> ctr;       // [nbox][3] box centres (FP64)
    DevBuf<int32_t> parent;   // [nbox] box at level - 1
    DevBuf<int32_t> child;    // [nbox + 1] children at level + 1 (when that level exists)
};

struct Tree {
    int64_t n = 0;
    double corner[3] = {0, 0, 0};
    DevBuf<uint64_t> key;     // sorted Morton keys
    DevBuf<int32_t> perm;     // sorted position -> caller index
    DevBuf<double> xs, ys, zs;   // sorted coordinates, SoA FP64
    DevBuf<int32_t> boxid;    // scratch: point -> box at the level being built
    TreeLevel lev[kMaxLev + 1];
    int built = -1;
};

enum Method { kNone = 0, kLagrange = 1, kGegenbauer = 2 };

struct Level {
    // descent lists, CSR by target box of this level; sources ascending
    int64_t nfar = 0, nnear = 0;
    DevBuf<int64_t> far_ptr, near_ptr;   // [nbox_x + 1]
    DevBuf<int32_t> far_src, far_cls;    // [nfar]   (cls: compact translation class)
    DevBuf<int32_t> near_src;            // [nnear]
    int32_t win_base[3] = {0, 0, 0};     // integer offset of window cell 0
    std::vector<int32_t> cls_off;        // [ncls][3] integer offsets of the classes
    int32_t ncls = 0;

    int method = kNone;
    // Lagrange
    int r1 = 0, r = 0, rp = 0;           // nodes per axis, r1^3, r padded to a multiple of 32
    DevBuf<float> T;                     // [ncls][rp][rp] (x2 planes re/im for Helmholtz)
    DevBuf<int32_t> grp_pair;            // [ngrp][16] far pair index (-1 = empty), grouped by class
    DevBuf<int32_t> grp_cls;             // [ngrp]
    int32_t ngrp = 0;
    bool fp16 = false;                   // transfer on FP16 MFMA (mixed precision)
    DevBuf<_Float16> T16;                // [ncls][rp][rp] (x2 re/im), row-major by target index, times sT
    float sT = 1.f;                      // power-of-two scale of T16
    // Gegenbauer
    int L = 0;
    int64_t nq = 0, npair = 0;           // n_Q = 2L(L+1) directions, npair = n_Q / 2 antipodal pairs
    DevBuf<float4> dirs;                 // [npair] direction * k / (2 pi), FP32 (w unused)
    DevBuf<double> dirs64;               // [npair][3] direction * k / (2 pi), FP64
    DevBuf<float4> D;                    // [ncls][npair] (D(s_p), D(-s_p)) as two complex
    bool phase64 = false;                // FP64 phase reduction at this level
    // ring-pair form of the transforms: ring m and its antipodal ring share one in-plane phase
    int nrp = 0;                         // ring pairs: (L+1)/2 rounded up (the equator ring when L is even)
    DevBuf<double2> rings;               // [nrp] (sin theta_m, cos theta_m) * k / (2 pi)
    DevBuf<double2> phis;                // [L] (cos phi_n, sin phi_n), phi_n = pi n / L
    int qG = 0;                          // groups of 4 directions per thread (0: direction-pair kernels)
    int qSplit = 1;                      // point segments of the forward transform (partials summed in order)
    int bwd_tile = 256;                  // target points per backward block
    // Lagrange node tables (FP32): Chebyshev nodes and 1 / prod_{b != a}(t_a - t_b)
    DevBuf<float> lnodes, lden;
    // work lists, largest boxes first
    DevBuf<int32_t> fwd_boxes;           // source boxes in at least one far pair
    DevBuf<int32_t> tgt_boxes;           // target boxes with a non-empty far list
    DevBuf<int2> bwd_work;               // (target box, first point) tiles of 256 points
    DevBuf<int32_t> near_boxes;          // leaf: target boxes with a non-empty near list
    int32_t max_src_pts = 0, max_tgt_pts = 0;
    double pts_src = 0, pts_tgt = 0;     // points in the forward / backward work lists
};

struct Plan {
    int kernel = 0;
    double k = 0, eps = 0;
    ffm_options_t opt{};
    bool empty = false;
    bool same = false;
    bool aligned = false;
    int64_t nx = 0, ny = 0;
    double d0 = 1, S = 1;
    std::unique_ptr<Tree> tx, ty_own;
    Tree *ty = nullptr;                  // == tx.get() for one set
    int leaf = 0;
    Level lev[kMaxLev + 1];
    // apply workspace (reused level after level)
    DevBuf<float2> u_sorted, v_sorted;   // [ny], [nx]
    DevBuf<float4> wsrc, wtgt;           // Gegenbauer u~ / v~, or Lagrange (as float2) scratch
    DevBuf<float2> wz;                   // Lagrange per-pair products
    DevBuf<float4> wpart;                // forward-transform partial sums of point segments
    DevBuf<float> amax;                  // max |Re u|, |Im u| of the current apply (FP16 scaling)
    bool any_fp16 = false;
    size_t ws_src = 0, ws_tgt = 0, ws_z = 0, ws_part = 0;
    // stats
    ffm_stats_t stats{};
    hipEvent_t done = nullptr;           // recorded after every apply
    bool applied = false;
    // optional phase timing (FFM_FLAG_TIMING): events recorded at phase ends
    std::vector<hipEvent_t> tev;
    std::vector<int> tphase;             // phase slot of each recorded event (after the first)
    int tused = 0;
    void mark(int phase, hipStream_t st);
};

// ---------------------------------------------------------------- entry points
void plan_build(Plan &P, const double *X, const double *Y, hipStream_t st);
void plan_apply(Plan &P, const void *wu, int dtype, float2 *v, hipStream_t st);
size_t plan_device_bytes(const Plan &P);

// device primitives (scan_sort.hip)
// (temporaries come from the scratch list; nothing here synchronises the stream)
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t st, Scratch &S);  // out[n] = total
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t st, Scratch &S);  // out[n] = total
void radix_sort_u64_u32(uint64_t *keys, int32_t *vals, int64_t n, hipStream_t st, Scratch &S);      // stable

}  // namespace ffm
