// Internal declarations of the gfx950 FFM library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
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

// Error state of the C ABI: a thread-local message for ffm_last_error.  Every entry point runs its
// body inside Guard::run, which maps exceptions to status codes.
int set_err(int code, const std::string &msg);
void clear_err();
struct Guard {
    template <class F>
    static int run(F &&f) {
        try {
            clear_err();
            f();
            return FFM_OK;
        } catch (const Error &e) {
            return set_err(e.code, e.what());
        } catch (const std::bad_alloc &) {
            return set_err(FFM_ENOMEM, "host allocation failed");
        } catch (const std::exception &e) {
            return set_err(FFM_EINTERNAL, e.what());
        }
    }
};

// Kernel launches go through this so a bad configuration becomes an error, not a fault.
#define FFM_LAUNCH(kern, grid, block, shmem, stream, ...)                                           \
    do {                                                                                            \
        if ((grid) > 0) {                                                                           \
            hipLaunchKernelGGL(kern, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__);          \
            FFM_HIP(hipGetLastError());                                                             \
        }                                                                                           \
    } while (0)

// Test hook: FFM_TEST_FAIL_ALLOC_AFTER=n makes the (n+1)-th device allocation of the process fail (that one
// only: later allocations go through).
void *dev_alloc(size_t bytes);
void dev_free(void *p);
size_t dev_bytes_live();
size_t dev_bytes_cached();   // freed device blocks the library keeps for reuse
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
        if (bufs.empty() && pinned.empty()) return;
        (void)hipStreamSynchronize(stream);
        release();
    }
    // take over another list's temporaries (the other list is left empty and will not synchronise)
    void adopt(Scratch &o) {
        for (auto &b : o.bufs) bufs.push_back(std::move(b));
        pinned.insert(pinned.end(), o.pinned.begin(), o.pinned.end());
        o.bufs.clear();
        o.pinned.clear();
    }
    // free everything now; only once the work using it is known to be complete
    void release() {
        bufs.clear();
        for (void *p : pinned) pinned_free(p);
        pinned.clear();
    }
    template <class T>
    T *get(size_t count) {
        bufs.emplace_back(count * sizeof(T));
        return reinterpret_cast<T *>(bufs.back().p);
    }
    // pinned host memory for device-to-host copies, valid until the scratch list is released
    template <class T>
    T *pin(size_t count) {
        void *p = pinned_alloc(std::max<size_t>(count * sizeof(T), 1));
        pinned.push_back(p);
        return static_cast<T *>(p);
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
constexpr size_t kGridBatchBytes = (size_t)512 << 20;   // grid form: G and H of the boxes in flight at one level
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

// ---------------------------------------------------------------- execution descriptors
// Every apply kernel takes an array of level descriptors and a list of work items (int4, .x = descriptor
// index); a block reads everything it needs from its item's descriptor.  One plan's levels, or many
// plans' levels (a batch), run through the same kernels: a launch covers any mix of instances.
struct IoEntry {           // per-instance input and output of the current apply
    const void *wu;
    float2 *vout;
    int dtype;
    int pad;
};

struct LDesc {
    // instance
    int inst;                         // index into the I/O table
    int helm;                         // Helmholtz kernel
    const int32_t *perm_x, *perm_y;   // sorted position -> caller index
    int64_t nx, ny;
    float2 *u, *v;                    // sorted input, sorted output accumulator
    float *amax;                      // max |u| of the apply (FP16 scaling), or null
    float k_rev;                      // k / (2 pi)
    int same;                         // sources and targets are one set (one tree)
    // level
    const double *txs, *tys, *tzs, *tctr;
    const int32_t *tstart;
    const double *sxs, *sys, *szs, *sctr;
    const int32_t *sstart;
    const int64_t *far_ptr, *near_ptr;
    const int32_t *far_src, *far_cls, *near_src;
    const int64_t *near_off;               // leaf of one set: per near entry, the offset of the pair's
                                           // source-side sums in nsym (s > t), or of the reverse entry's (s < t
                                           // with a reverse entry), else -1
    float2 *nsym;                          // source-side sums of the symmetric near pairs
    int64_t nsymn;                         // entries of one component's plane of nsym (gradients: three planes)
    const int32_t *tr_tgt;                 // target boxes of the transfers, in Morton order
    int ntr, ncls;                         // their number; translation classes
    const int32_t *sib_tgt, *sib_src, *sib_cnt;   // transfers by sibling group (Level::sib_*)
    const uint2 *sib_cls;
    int nsibg;
    // Gegenbauer level
    const float4 *dirs;
    const double *dirs64;
    const double2 *rings, *phis;
    const float4 *D;
    float4 *ut, *vt, *part;           // u~ / v~ / point-segment partials of this level
    int64_t npair, part_stride;
    int L, nrp, Tr, R, nchunk, nsplit;
    int bsplit;                            // ring parts of the target transform (partials summed in order)
    float2 *bpart;                         // [bsplit][nx] target-transform partials
    // Lagrange level
    const float *T, *lnodes, *lden;
    const _Float16 *T16;
    const float4 *tn;                      // target normals in sorted order (normal-derivative kernels), or null
    const float4 *sn;                      // source normals in sorted order (double-layer kernels), or null
    float4 tnc;                            // the target normal of every point where tn is null (gradient plans:
                                           // the axis of the descriptor's component)
    int ncomp;                             // output components per target: 1, or 3 (gradient plans; component c
                                           // of sorted target i at v[c nx + i] of the level-0 descriptor's v)
    float4 *vtx;                           // gradient plans: v~ of components 1 and 2, vtstride apart
    int64_t vtstride;
    float2 *vtmp;                          // split normal derivative: the three axis planes (nx apart), or null
    float2 *ucomp;                         // split double layer: the densities u n_c (ny apart), or null
    float4 *utx;                           // split double layer: u~ of the densities u n_1, u n_2, utstride apart
    int64_t utstride;
    const float *acaA, *acaB;              // ACA factors: A [class][plane][kpm][rp], B^T [class][plane][rp][kpm]
    const int32_t *acaKp;                  // [class] rank padded to 32
    int kpm;                               // largest padded rank
    const int32_t *grp_pair, *grp_cls;
    float2 *ut2, *Z;
    double two_over_dl;
    int r1, rp, maxpts;
    float sT;
    // grid form of the plane-wave transforms (spread onto a uniform grid, separable sums to the
    // quadrature directions): p nodes per axis at spacing h, kernel width w, shape beta
    int gp, gw;
    float gbeta;                           // kernel shape
    double ginv_h;                         // 1 / h
    int64_t gnbox;                         // box slots in the grid arrays of this level
    const int32_t *gslot_s, *gslot_t;      // source / target box -> its slot in G and H (boxes go through the
                                           // grid stages in batches of at most gnbox, each batch reusing the slots)
    float2 *G, *H;                         // G [box][c][a][b] grid values, H [m][box][a][b] ring sums
    const float2 *Ez, *Ex, *Ey;            // [nrp][p], [nrp][p][L], [nrp][p][L]
    const float2 *ExT, *EyT;               // [nrp][L][p] (Ex, Ey transposed)
    const int32_t *gperm, *gzs;            // source points by z-plane: permutation, [box][p + 1] offsets
    const float4 *gxyz;                    // their grid coordinates (node units), in the same order
};

// Kernel variants (the template parameters travel with the stage).
enum Kern {
    K_PERM_IN = 0, K_AMAX, K_FWD_PAIR, K_FWD_RING, K_SUM, K_TRANSFER, K_BWD_PAIR, K_BWD_RING,
    K_ANTERP, K_MFMA32, K_MFMA16, K_INTERP, K_NEAR, K_PERM_OUT, K_ZERO_OUT, K_BSUM,
    K_GSPREAD, K_GZ, K_GPHI, K_GPHIT, K_GZT, K_GINTERP, K_ACA, K_NEAR_DN, K_BWD_PAIR_DN, K_INTERP_DN,
    K_NEAR_SYM, K_NEAR_GATHER, K_NEAR_DL, K_ANTERP_DL, K_FWD_PAIR_DL, K_DIRSCALE, K_DNCOMBINE, K_DLCOMBINE,
    K_NEAR_GRAD
};

struct Stage {
    int kern = 0, a = 0, b = 0;       // kernel and its template parameters
    int role_add = 0;                 // added to the stage's order among its level's stages in a batch (box batches
                                      // of the grid form follow one another)
    int slot = -1;                    // timing slot (FFM_TIMING layout) closed by this stage, or -1
    int tslot = -1;                   // timing slot the stage's time belongs to
    int level = 0;                    // level (ordering of target-side stages in batches)
    size_t shmem = 0;                 // dynamic LDS bytes
    std::vector<int4> items;          // work items (host copy, kept for batching)
    const int4 *ditems = nullptr;     // the items on the device: a slice of the owner's item arena
    size_t nitems = 0;
};

// Upload the work items of all the given stages into one device arena with one copy, and point each stage
// at its slice.
void upload_stage_items(const std::vector<Stage *> &stages, DevBuf<int4> &arena, hipStream_t st, Scratch &SC);


// Ring-pair blocks (16 ring pairs each) per work item of the grid form's sums over z: at most four per item,
// balanced over the items.
// Direction pairs per transfer tile: the tile of every class's D is staged in LDS (at most 48 KB).
// Gegenbauer levels of at least this order run the direct transforms in the ring-pair form (measured on the
// 1M-point sphere: L = 26 0.48 against 0.54 ms for both transforms in direction pairs; L = 16 0.59 against
// 0.24 ms)
constexpr int kRingMinL = 24;

__host__ __device__ inline int transfer_qt(int ncls) {
    return ncls * 4 * 16 <= 49152 ? 4 : (ncls * 2 * 16 <= 49152 ? 2 : 1);
}

__host__ __device__ inline void grid_z_groups(int nrp, int &ngroups, int &per) {
    const int nmb = (nrp + 15) / 16;
    ngroups = (nmb + 3) / 4;
    per = (nmb + ngroups - 1) / ngroups;
}

// Tile choices of the plane-wave kernels (the autotuner picks among them).
struct Tune {
    int ring_g = 4;                   // groups of 4 directions per thread in ring-pair forward kernels
    int bwd_pt = 2;                   // target points per thread in ring-pair backward kernels
};

struct Level {
    // descent lists, CSR by target box of this level; sources ascending
    int64_t nfar = 0, nnear = 0;
    DevBuf<int64_t> far_ptr, near_ptr;   // [nbox_x + 1]
    DevBuf<int64_t> near_off;            // leaf of one set: per near entry (LDesc::near_off)
    DevBuf<int32_t> far_src, far_cls;    // [nfar]   (cls: compact translation class)
    DevBuf<int32_t> near_src;            // [nnear]
    // per-pair leaf rule: the near pairs summed densely at this level (both boxes small), CSR by target box
    int64_t nearly = 0;
    DevBuf<int64_t> early_ptr;
    DevBuf<int32_t> early_src;
    std::vector<int32_t> h_early;        // target boxes with early pairs, largest first
    double early_pairs = 0;              // their point pairs
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
    // ACA factors of the transfer matrices (T is not kept): ranks, padded ranks, their maximum
    bool aca = false;
    double aca_rank = 0.0;               // mean rank over the classes (whenever ACA was evaluated)
    int kpm = 0;
    std::vector<int32_t> aca_ranks;
    DevBuf<float> acaA, acaB;
    DevBuf<int32_t> acaKp;
    // Gegenbauer
    int L = 0;
    int64_t nq = 0, npair = 0;           // n_Q = 2L(L+1) directions, npair = n_Q / 2 antipodal pairs
    DevBuf<float4> dirs;                 // [npair] direction * k / (2 pi), FP32 (w unused)
    DevBuf<double> dirs64;               // [npair][3] direction * k / (2 pi), FP64
    DevBuf<float4> D;                    // [ncls][npair] (D(s_p), D(-s_p)) as two complex
    DevBuf<int32_t> tr_tgt;              // target boxes with far work in Morton order (transfer slots)
    // transfers by sibling group (one tree): up to four targets of one parent box, [ngroup][4] (-1 past the
    // last); the sources of their far pairs, [ngroup][216] by position relative to the parent (compacted,
    // sib_cnt per group), with each sibling's class ([ngroup][216] x 4 int16, -1 where that pair is not far)
    int32_t nsibg = 0;
    DevBuf<int32_t> sib_tgt, sib_src, sib_cnt;
    DevBuf<uint2> sib_cls;
    std::vector<int32_t> h_par;          // parent of every target box (one tree, far levels)
    bool phase64 = false;                // FP64 phase reduction at this level
    // ring-pair form of the transforms: ring m and its antipodal ring share one in-plane phase
    int nrp = 0;                         // ring pairs: (L+1)/2 rounded up (the equator ring when L is even)
    DevBuf<double2> rings;               // [nrp] (sin theta_m, cos theta_m) * k / (2 pi)
    DevBuf<double2> phis;                // [L] (cos phi_n, sin phi_n), phi_n = pi n / L
    int qG = 0;                          // groups of 4 directions per thread (0: direction-pair kernels)
    int qSplit = 1;                      // point segments of the forward transform (partials summed in order)
    int bwd_tile = 256;                  // target points per backward block
    int Tr = 0, R = 0, nchunk = 0;       // ring-pair forward: threads per ring, rings per block, ring chunks
    int bSplit = 1;                      // ring parts of the target transform
    // grid form (tform 3): p nodes per axis, spacing h, kernel width w and shape beta
    bool grid = false;
    int gp = 0, gw = 0;
    double gh = 0, gbeta = 0;
    double galias = 0;                   // aliasing bound of one axis at the level's largest |k s_d h|
    DevBuf<float2> Ez, Ex, Ey;           // [nrp][p], [nrp][p][L], [nrp][p][L]
    DevBuf<float2> ExT, EyT;             // [nrp][L][p]
    DevBuf<int32_t> gperm, gzs;          // source points ordered by box and z-plane; [nbox_y][p + 1]
    int32_t gcap = 0;                    // box slots of the grid workspace (G, H) at this level
    DevBuf<int32_t> gslot_s, gslot_t;    // source / target box -> slot within its batch
    DevBuf<float4> gxyz;                 // grid coordinates of the source points, gperm order
    // Lagrange node tables (FP32): Chebyshev nodes and 1 / prod_{b != a}(t_a - t_b)
    DevBuf<float> lnodes, lden;
    // box lists on the host, largest boxes first, and the box point ranges
    std::vector<int32_t> h_fwd;          // source boxes in at least one far pair
    std::vector<int32_t> h_tgt;          // target boxes with a non-empty far list
    std::vector<int32_t> h_near;         // leaf: target boxes with a non-empty near list
    std::vector<int32_t> h_sx, h_sy;     // box start arrays of the two trees
    int32_t max_src_pts = 0, max_tgt_pts = 0;
    std::vector<Stage> stages;           // launches of this level, in order
    double pts_src = 0, pts_tgt = 0;     // points in the forward / backward work lists
};

struct Plan {
    int kernel = 0;                      // FFM_LAPLACE or FFM_HELMHOLTZ (the base kernel)
    bool dn = false;                     // normal derivative at the targets (adjoint double layer)
    const double *user_normals = nullptr;   // the caller's target normals, read while the plan is built
    DevBuf<float4> tnrm;                 // target normals in sorted order (FP32)
    bool grad = false;                   // gradient at the targets: target side once per axis
    DevBuf<float4> wtgtx;                // gradient plans, split normal derivative: v~ of components 1 and 2
    bool dnsplit = false;                // normal derivative with levels whose target side runs once per axis
    DevBuf<float2> wtmp;                 // their three axis planes of the sorted targets
    bool dlsplit = false;                // double layer with levels whose source side runs once per axis
    DevBuf<float2> wucomp;               // the densities u n_c of the sorted sources
    DevBuf<float4> wsrcx;                // u~ of the densities of axes 1 and 2
    int ncomp() const { return grad ? 3 : 1; }
    bool dl = false;                     // normal derivative at the sources (double layer)
    const double *user_snormals = nullptr;  // the caller's source normals, read while the plan is built
    DevBuf<float4> snrm;                 // source normals in sorted order (FP32)
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
    DevBuf<float2> wbpart;               // target-transform partial sums of ring parts
    DevBuf<float2> wG, wH;               // grid-form workspaces (grid values, ring sums)
    bool near_sym = false;               // leaf near field over unordered box pairs (one set, G symmetric)
    int64_t nsym = 0;                    // source-side sums of those pairs (points of the higher boxes)
    DevBuf<float2> wnsym;
    bool any_grid = false;
    DevBuf<float> amax;                  // max |Re u|, |Im u| of the current apply (FP16 scaling)
    bool any_fp16 = false;
    size_t ws_src = 0, ws_tgt = 0, ws_z = 0, ws_part = 0;
    // stats
    ffm_stats_t stats{};
    hipEvent_t done = nullptr;           // recorded after every apply
    bool applied = false;
    int batch_refs = 0;                  // batches that launch this plan's stages
    std::atomic<int> server_refs{0};     // server requests of this plan queued or running
    // execution: descriptors (index = level), I/O table, stages before and after the levels
    std::vector<LDesc> hdesc;
    DevBuf<LDesc> ddesc;
    DevBuf<int4> items;               // work items of every stage (one arena)
    // the plan's last GPU work (tables, launch lists) may still run on the planning stream when ffm_plan
    // returns: `ready` is recorded after it, and `pending` holds its temporaries until it is complete
    hipEvent_t ready = nullptr;
    std::unique_ptr<Scratch> pending;
    DevBuf<IoEntry> dio;
    IoEntry *hio = nullptr;              // pinned host copy of the I/O entry
    std::vector<Stage> pre, post;
    // applies over the library's static workspace (ffm_apply_static): descriptors pointing into it, built with
    // the plan when its workspace fits, the I/O entry, their pinned host block and the last such apply's event
    DevBuf<LDesc> sdesc;
    DevBuf<IoEntry> sdio;
    void *spin = nullptr;
    IoEntry *shio = nullptr;
    hipEvent_t sdone = nullptr;
    bool sapplied = false;
    Tune tune;
    // optional phase timing (FFM_FLAG_TIMING): events recorded at phase ends
    std::vector<hipEvent_t> tev;
    std::vector<int> tphase;             // phase slot of each recorded event (after the first)
    std::vector<int4> tkern;             // (kernel, a, b, level) of the launch each event closes
    std::vector<int64_t> tblocks;        // its thread blocks
    int tused = 0;
    void mark(int phase, hipStream_t st, const Stage *S = nullptr);
};

// ---------------------------------------------------------------- entry points
void plan_build(Plan &P, const double *X, const double *Y, hipStream_t st);
void plan_apply(Plan &P, const void *wu, int dtype, float2 *v, hipStream_t st);
size_t plan_device_bytes(const Plan &P);
// stages of a plan for a tile choice; descriptors of a plan over given workspaces
void plan_stages(Plan &P, const Tune &t, hipStream_t st, Scratch *keep = nullptr);
struct LevelWork {                     // apply workspace a descriptor points into
    float4 *ut = nullptr, *vt = nullptr, *part = nullptr;
    float2 *ut2 = nullptr, *Z = nullptr, *bpart = nullptr;
    float2 *G = nullptr, *H = nullptr;
    float2 *nsym = nullptr;
    float4 *vtx = nullptr;                // gradient plans: v~ of target components 1 and 2 (2 x ws_tgt)
    float2 *vtmp = nullptr;               // split normal derivative: three axis planes of the sorted targets
    float2 *ucomp = nullptr;              // split double layer: densities u n_c of the sorted sources
    float4 *utx = nullptr;                // split double layer: u~ of the densities of axes 1 and 2 (2 x ws_src)
};
// Apply workspace laid out in one block (requests of the server, the static-scratch apply): its size in bytes
// (every part aligned to 256 B; also what ffm_workspace_bytes and ffm_stats_t.workspace_bytes report), and the
// part pointers for a block at base.
struct WorkPtrs {
    float2 *u = nullptr, *v = nullptr;   // sorted input, sorted output accumulator
    float *amax = nullptr;
    LevelWork lw;
};
size_t apply_work_bytes(const Plan &P);
WorkPtrs carve_work(const Plan &P, char *base);
// The static workspace of ffm_apply_static: the device address of this device's copy (taken once per device),
// and the plan's descriptors over it (nothing if the plan's workspace does not fit).
char *static_work_base();
void plan_static_setup(Plan &P, hipStream_t st);
// Release the batch kept by ffm_apply_batched if it holds plan P; a status code.  With wait, its last apply is
// waited for; without, an apply still in flight gives FFM_EBUSY and nothing is released.
int implicit_batch_drop(const Plan *P, bool wait);
// concurrent blocks per CU of a kernel variant (occupancy) and the device's CU count
int stage_blocks_per_cu(int kern, int a, int b);
std::string kernel_name(int kern, int a, int b);
int device_cus();
LDesc make_desc(const Plan &P, int l, int inst, float2 *u, float2 *v, float *amax, const LevelWork &w);
// A plan's descriptors: one per level, and for gradient plans two more sets (components 1 and 2: descriptor
// k serves level k mod (leaf + 1), component k / (leaf + 1), with its own output plane and axis).
int plan_ndesc(const Plan &P);
LDesc plan_desc(const Plan &P, int k, int inst, float2 *u, float2 *v, float *amax, const LevelWork &w);
// rebuild the stages and descriptors of a built plan for a tile choice (the plan must be idle)
void plan_set_tune(Plan &P, const Tune &t, hipStream_t st, Scratch *keep = nullptr);
// Wait on the host until the plan's own GPU work is complete (plans return with their last tables and launch
// lists still being written on the planning stream) and free its temporaries.
void plan_sync_ready(Plan &P);
// one launch per stage
void run_stage(const Stage &S, const LDesc *ddesc, const IoEntry *dio, hipStream_t st);

// device primitives (scan_sort.hip)
// (temporaries come from the scratch list; nothing here synchronises the stream)
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t st, Scratch &S);  // out[n] = total
// Both scans at once (n <= 4096 tiles of 2048): oa and ob hold n + 1 elements, the totals going to oa[n] and
// ob[n] and also to host_tot[0..1] (host-visible memory, valid once the stream has passed the scan).
void exclusive_scan2_i64(const int64_t *a, int64_t *oa, const int64_t *b, int64_t *ob, int64_t n, int64_t *host_tot,
                         hipStream_t st, Scratch &S);
void radix_sort_u64_u32(uint64_t *keys, int32_t *vals, int64_t n, hipStream_t st, Scratch &S);      // stable

}  // namespace ffm

// the opaque handle of the C ABI
struct ffm_plan_s {
    ffm::Plan P;
};
