// Planner: root cubes, Morton-sorted octrees, descent lists and transfer tables.
//
// Paper: Sec. 2.2.1 (root cubes with a common edge d_0, d_l = d_0 / 2^l),
// Sec. 2.1 (two octrees whose boxes are translates of each other), Sec. 2.2.2
// (admissibility; Lagrange interpolation on Chebyshev nodes), Sec. 2.2.3
// (Gegenbauer series eq. gegenbauerSerie, rank eq. gegenbauerRank, quadrature
// eq. gegenbauerQuadrature), Sec. 2.2.4 (stopping rule), Sec. 3.2 proof of
// Prop. 1 (one transfer per translation class, descent-only lists).
//
// Geometry that must match an FP64 reference bit for bit (quantisation, box
// centres, the far test of shifted trees) is computed without FMA contraction.
#include "common.h"

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>

namespace ffm {

namespace {

constexpr int kThreads = 256;

inline int nblocks(int64_t n, int per = kThreads) { return (int)((n + per - 1) / per); }

// ------------------------------------------------------------------ bounding boxes
__global__ void __launch_bounds__(kThreads) k_bbox_partial(const double *P, int64_t n, double *part, int *bad) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nbad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            double v = P[3 * i + d];
            if (!isfinite(v)) nbad = 1;
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
        }
    }
    __shared__ double s[6][kThreads];
    for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = lo[d];
        s[3 + d][threadIdx.x] = hi[d];
    }
    if (nbad) atomicOr(bad, 1);
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int d = 0; d < 3; ++d) {
                s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + o]);
                s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(kThreads) k_bbox_final(const double *part, int nb, double *out) {
    __shared__ double s[6][kThreads];
    for (int d = 0; d < 6; ++d) {
        double v = d < 3 ? INFINITY : -INFINITY;
        for (int b = threadIdx.x; b < nb; b += kThreads) v = d < 3 ? fmin(v, part[6 * b + d]) : fmax(v, part[6 * b + d]);
        s[d][threadIdx.x] = v;
    }
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int d = 0; d < 6; ++d)
                s[d][threadIdx.x] = d < 3 ? fmin(s[d][threadIdx.x], s[d][threadIdx.x + o])
                                          : fmax(s[d][threadIdx.x], s[d][threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = s[threadIdx.x][0];
}

// ------------------------------------------------------------------ Morton keys
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ int32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (int32_t)v;
}

// q = clamp(floor((p - corner) * S), 0, 2^21 - 1): one rounded subtraction, one rounded product.
__device__ __forceinline__ uint64_t quantise(double p, double c, double S) {
#pragma clang fp contract(off)
    double t = (p - c) * S;
    double f = floor(t);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)((1 << kBits) - 1)) return (uint64_t)((1 << kBits) - 1);
    return (uint64_t)f;
}

__global__ void __launch_bounds__(kThreads)
k_morton(const double *P, int64_t n, double cx, double cy, double cz, double S, uint64_t *key, int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t qx = quantise(P[3 * i], cx, S), qy = quantise(P[3 * i + 1], cy, S), qz = quantise(P[3 * i + 2], cz, S);
    key[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    idx[i] = (int32_t)i;
}

__global__ void __launch_bounds__(kThreads)
k_gather(const double *P, int64_t n, const int32_t *perm, double *xs, double *ys, double *zs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    xs[i] = P[3 * j];
    ys[i] = P[3 * j + 1];
    zs[i] = P[3 * j + 2];
}

// Target (or source) normals in sorted order, FP32 (the normal-derivative kernels); w unused.
__global__ void __launch_bounds__(kThreads)
k_gather_normals(const double *N, int64_t n, const int32_t *perm, float4 *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    out[i] = make_float4((float)N[3 * j], (float)N[3 * j + 1], (float)N[3 * j + 2], 0.f);
}

// First level at which point i starts a box: boxes of level l are the runs of key >> 3(21 - l).
// 22 = never (equal keys).  Also a histogram of those levels (block-local, then one add per bin).
__global__ void __launch_bounds__(kThreads)
k_first_level(const uint64_t *key, int64_t n, int8_t *f, int32_t *hist) {
    __shared__ int32_t h[23];
    if (threadIdx.x < 23) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int lev;
        if (i == 0) {
            lev = 0;
        } else {
            const uint64_t x = key[i] ^ key[i - 1];
            if (x == 0) {
                lev = 22;
            } else {
                const int b = 63 - __clzll((long long)x);   // highest differing bit, 0..62
                lev = (63 - b + 2) / 3;                     // smallest l with b >= 3 (21 - l)
            }
        }
        f[i] = (int8_t)lev;
        atomicAdd(&h[lev], 1);
    }
    __syncthreads();
    if (threadIdx.x < 23 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// A level's boxes in two launches: k_lvl_count counts, per tile of kLvlTile points, the box starts
// (f[i] <= l); k_lvl_boxes numbers the starts (its tile's offset summed from the counts of the tiles before it,
// then a block scan) and writes every box's start, integer coordinates and centre and every point's box.
// Centres c = corner + (2i + 1) * (d_0 2^-(l+1)).
constexpr int kLvlItems = 8;
constexpr int kLvlTile = kThreads * kLvlItems;

__global__ void __launch_bounds__(kThreads) k_lvl_count(const int8_t *f, int64_t n, int l, int32_t *tcount) {
    __shared__ int32_t red[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kLvlTile;
    int32_t c = 0;
    for (int j = 0; j < kLvlItems; ++j) {
        const int64_t i = base + (int64_t)j * kThreads + threadIdx.x;
        if (i < n && f[i] <= l) ++c;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += red[w];
        tcount[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kThreads)
k_lvl_boxes(const uint64_t *key, const int8_t *f, int64_t n, int l, const int32_t *tcount, double cx, double cy,
            double cz, double h, int32_t *start, int32_t *ijk, double *ctr, int32_t *boxid, int32_t nbox) {
#pragma clang fp contract(off)
    __shared__ int32_t red[kThreads / 64];
    __shared__ int32_t wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // boxes started in the tiles before this one
    int32_t pre = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += kThreads) pre += tcount[j];
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if (lane == 0) red[wv] = pre;
    // this thread's kLvlItems consecutive points
    const int64_t base = (int64_t)blockIdx.x * kLvlTile + (int64_t)threadIdx.x * kLvlItems;
    bool stt[kLvlItems];
    int32_t c = 0;
    for (int j = 0; j < kLvlItems; ++j) {
        const int64_t i = base + j;
        stt[j] = i < n && f[i] <= l;
        c += stt[j];
    }
    // block exclusive scan of the per-thread counts
    int32_t v = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    int32_t off = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
        off += red[w];
        if (w < wv) off += wsum[w];
    }
    int32_t run = off + v - c;   // boxes started before this thread's first point
    for (int j = 0; j < kLvlItems; ++j) {
        const int64_t i = base + j;
        if (i >= n) break;
        if (stt[j]) ++run;
        const int32_t b = run - 1;
        boxid[i] = b;
        if (!stt[j]) continue;
        start[b] = (int32_t)i;
        const uint64_t pfx = key[i] >> (3 * (kBits - l));
        const int32_t a0 = compact3(pfx >> 2), a1 = compact3(pfx >> 1), a2 = compact3(pfx);
        ijk[3 * b] = a0;
        ijk[3 * b + 1] = a1;
        ijk[3 * b + 2] = a2;
        // product and sum rounded separately (no FMA)
        ctr[3 * b] = cx + (double)(2 * a0 + 1) * h;
        ctr[3 * b + 1] = cy + (double)(2 * a1 + 1) * h;
        ctr[3 * b + 2] = cz + (double)(2 * a2 + 1) * h;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[nbox] = (int32_t)n;
}

// parent of box b (level l) and children of box B (level l-1)
__global__ void __launch_bounds__(kThreads)
k_link(const int32_t *start_l, int32_t nb_l, const int32_t *boxid_prev, int32_t *parent_l,
       const int32_t *start_p, int32_t nb_p, const int32_t *boxid_cur, int32_t *child_p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb_l) parent_l[i] = boxid_prev[start_l[i]];
    if (i < nb_p) child_p[i] = boxid_cur[start_p[i]];
    if (i == 0) child_p[nb_p] = nb_l;
}

// ------------------------------------------------------------------ descent lists
struct FarTest {
    const int32_t *ijk_t, *ijk_s;
    const double *ctr_t, *ctr_s;
    double two_dl;
    int aligned;
    int32_t base[3];
};

// Admissibility (Sec. 2.2.2): max-norm centre distance >= 2 d_l.  Aligned trees use the
// integer box offsets (exact); shifted trees compare FP64 centre differences.
__device__ __forceinline__ bool is_far(const FarTest &ft, int32_t t, int32_t s) {
    if (ft.aligned) {
        int m = 0;
        for (int d = 0; d < 3; ++d) m = max(m, abs(ft.ijk_t[3 * t + d] - ft.ijk_s[3 * s + d]));
        return m >= 2;
    }
    double m = 0.0;
    for (int d = 0; d < 3; ++d) m = fmax(m, fabs(ft.ctr_t[3 * t + d] - ft.ctr_s[3 * s + d]));
    return m >= ft.two_dl;
}

// For every target box t of level l: the children of the near sources of its parent.  One wave per target
// box; a step takes 8 near entries with 8 children slots each (lane = 8 entry + child), in the order of the
// serial walk (near entries, then children), so ballots give each candidate's place in the lists.
__device__ __forceinline__ void list_candidate(int64_t e, int64_t e1, int j, const int32_t *pnear_src,
                                               const int32_t *child_y, bool &valid, int32_t &cs) {
    valid = false;
    cs = 0;
    if (e < e1) {
        const int32_t S = pnear_src[e];
        const int32_t c0 = child_y[S];
        if (j < child_y[S + 1] - c0) {
            valid = true;
            cs = c0 + j;
        }
    }
}

__global__ void __launch_bounds__(kThreads)
k_list_count(int32_t nbx, const int32_t *parent_x, const int64_t *pnear_ptr, const int32_t *pnear_src,
             const int32_t *child_y, FarTest ft, int64_t *nfar, int64_t *nnear, int32_t *win_used) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the translation windows the fill marks start cleared
    for (int64_t i = gid; i < kWin3; i += (int64_t)gridDim.x * blockDim.x) win_used[i] = 0;
    const int32_t t = (int32_t)(gid >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= nbx) return;
    const int32_t T = parent_x[t];
    const int64_t e0 = pnear_ptr[T], e1 = pnear_ptr[T + 1];
    int64_t cf = 0, cn = 0;
    for (int64_t eb = e0; eb < e1; eb += 8) {
        bool valid;
        int32_t cs;
        list_candidate(eb + (lane >> 3), e1, lane & 7, pnear_src, child_y, valid, cs);
        const bool far = valid && is_far(ft, t, cs);
        cf += __popcll(__ballot(far));
        cn += __popcll(__ballot(valid && !far));
    }
    if (lane == 0) {
        nfar[t] = cf;
        nnear[t] = cn;
    }
}

__global__ void __launch_bounds__(kThreads)
k_list_fill(int32_t nbx, const int32_t *parent_x, const int64_t *pnear_ptr, const int32_t *pnear_src,
            const int32_t *child_y, FarTest ft, const int64_t *far_ptr, const int64_t *near_ptr, int32_t *far_src,
            int32_t *far_win, int32_t *near_src, int32_t *win_used, int *bad) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t t = (int32_t)(gid >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= nbx) return;
    const int32_t T = parent_x[t];
    const int64_t e0 = pnear_ptr[T], e1 = pnear_ptr[T + 1];
    int64_t pf = far_ptr[t], pn = near_ptr[t];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int64_t eb = e0; eb < e1; eb += 8) {
        bool valid;
        int32_t cs;
        list_candidate(eb + (lane >> 3), e1, lane & 7, pnear_src, child_y, valid, cs);
        const bool far = valid && is_far(ft, t, cs), nr = valid && !far;
        const unsigned long long mf = __ballot(far), mn = __ballot(nr);
        if (far) {
            int w = 0;
            for (int d = 0; d < 3; ++d) {
                int o = ft.ijk_t[3 * t + d] - ft.ijk_s[3 * cs + d] - ft.base[d];
                if (o < 0 || o >= kWin) {
                    atomicOr(bad, 1);
                    o = 0;
                }
                w = w * kWin + o;
            }
            const int64_t at = pf + __popcll(mf & below);
            far_src[at] = cs;
            far_win[at] = w;
            win_used[w] = 1;
        }
        if (nr) near_src[pn + __popcll(mn & below)] = cs;
        pf += __popcll(mf);
        pn += __popcll(mn);
    }
}

// Per-pair leaf rule: the near pairs of target box t whose two boxes both hold at most n_leaf points (early, summed
// densely at this level) and the others (refined).  One thread per target box; order kept.
__global__ void __launch_bounds__(kThreads)
k_split_count(int32_t nbx, const int64_t *near_ptr, const int32_t *near_src, const int32_t *sx, const int32_t *sy,
              int32_t n_leaf, int64_t *cnt_e, int64_t *cnt_r) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nbx) return;
    const bool small_t = sx[t + 1] - sx[t] <= n_leaf;
    int64_t e = 0, r = 0;
    for (int64_t q = near_ptr[t]; q < near_ptr[t + 1]; ++q) {
        const int32_t s = near_src[q];
        if (small_t && sy[s + 1] - sy[s] <= n_leaf) ++e;
        else ++r;
    }
    cnt_e[t] = e;
    cnt_r[t] = r;
}

__global__ void __launch_bounds__(kThreads)
k_split_fill(int32_t nbx, const int64_t *near_ptr, const int32_t *near_src, const int32_t *sx, const int32_t *sy,
             int32_t n_leaf, const int64_t *early_ptr, const int64_t *ref_ptr, int32_t *early_src, int32_t *ref_src) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nbx) return;
    const bool small_t = sx[t + 1] - sx[t] <= n_leaf;
    int64_t e = early_ptr[t], r = ref_ptr[t];
    for (int64_t q = near_ptr[t]; q < near_ptr[t + 1]; ++q) {
        const int32_t s = near_src[q];
        if (small_t && sy[s + 1] - sy[s] <= n_leaf) early_src[e++] = s;
        else ref_src[r++] = s;
    }
}

__global__ void __launch_bounds__(kThreads) k_mark_sources(const int32_t *far_src, int64_t n, uint8_t *active) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) active[far_src[i]] = 1;
}

// number of point pairs of the near lists (exact: integer sum)
__global__ void __launch_bounds__(kThreads)
k_near_pairs(const int64_t *ptr, const int32_t *src, int32_t nbx, const int32_t *sx, const int32_t *sy,
             unsigned long long *out) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long acc = 0;
    if (t < nbx)
        for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e)
            acc += (unsigned long long)(sx[t + 1] - sx[t]) * (unsigned long long)(sy[src[e] + 1] - sy[src[e]]);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

// Symmetric near field of one set (leaf): per target box t, the points of its higher neighbours (the lengths of
// the source-side slices its block writes) ...
__global__ void __launch_bounds__(kThreads)
k_sym_box_count(const int64_t *ptr, const int32_t *src, int32_t nb, const int32_t *start, int64_t *cnt) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    int64_t c = 0;
    for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) {
        const int32_t s = src[e];
        if (s > t) c += start[s + 1] - start[s];
    }
    cnt[t] = c;
}

// ... the slice of each entry with s > t (in list order from the box's scanned offset), -1 for the others ...
__global__ void __launch_bounds__(kThreads)
k_sym_fill(const int64_t *ptr, const int32_t *src, int32_t nb, const int32_t *start, const int64_t *boff,
           int64_t *off) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    int64_t o = boff[t];
    for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) {
        const int32_t s = src[e];
        if (s > t) {
            off[e] = o;
            o += start[s + 1] - start[s];
        } else {
            off[e] = -1;
        }
    }
}

// ... and for an entry with s < t, the slice of the reverse entry (t in the list of s) if there is one.
__global__ void __launch_bounds__(kThreads)
k_sym_reverse(const int64_t *ptr, const int32_t *src, int32_t nb, int64_t *off) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) {
        const int32_t s = src[e];
        if (s >= t) continue;
        for (int64_t f = ptr[s]; f < ptr[s + 1]; ++f)
            if (src[f] == t) {
                off[e] = off[f];
                break;
            }
    }
}

// Grid-form workspace per level (G and H of the boxes in flight); test hook FFM_TEST_GRID_BATCH_BYTES lowers it so
// that the box batches can be tested on small problems.
size_t grid_batch_bytes() {
    static const size_t v = [] {
        const char *e = std::getenv("FFM_TEST_GRID_BATCH_BYTES");
        const long long x = e ? std::atoll(e) : 0;
        return x > 0 ? (size_t)x : kGridBatchBytes;
    }();
    return v;
}

// Sibling-group transfer tables (one tree): block g takes up to four targets of one parent box and places the
// sources of their far pairs by position relative to the parent (a far source's parent is adjacent to the
// targets' parent, so the position s_ijk - 2 P_ijk lies in [-2, 3]^3: 216 slots), with each sibling's class;
// then it compacts the slots in slot order.
__global__ void __launch_bounds__(64)
k_sib_fill(const int32_t *sib_tgt, const int64_t *far_ptr, const int32_t *far_src, const int32_t *far_cls,
           const int32_t *parent, const int32_t *ijk, const int32_t *ijk_up, int32_t *sib_src, uint2 *sib_cls,
           int32_t *sib_cnt) {
    __shared__ int32_t ssrc[216];
    __shared__ uint32_t scls[216][2];          // 4 int16 per slot
    const int g = blockIdx.x, lane = threadIdx.x;
    for (int k = lane; k < 216; k += 64) {
        ssrc[k] = -1;
        scls[k][0] = scls[k][1] = 0xFFFFFFFFu;
    }
    __syncthreads();
    const int32_t P = parent[sib_tgt[4 * g]];
    const int32_t px = 2 * ijk_up[3 * P], py = 2 * ijk_up[3 * P + 1], pz = 2 * ijk_up[3 * P + 2];
    for (int j = 0; j < 4; ++j) {
        const int32_t t = sib_tgt[4 * g + j];
        if (t < 0) break;
        for (int64_t e = far_ptr[t] + lane; e < far_ptr[t + 1]; e += 64) {
            const int32_t s = far_src[e];
            const int ax = ijk[3 * s] - px + 2, ay = ijk[3 * s + 1] - py + 2, az = ijk[3 * s + 2] - pz + 2;
            if (ax < 0 || ax > 5 || ay < 0 || ay > 5 || az < 0 || az > 5) continue;   // not for one tree
            const int k = ax + 6 * ay + 36 * az;
            ssrc[k] = s;                        // siblings sharing a source write the same value
            const uint32_t c = (uint32_t)far_cls[e] & 0xFFFFu;
            // one sibling per column: the 16-bit halves of a word belong to two siblings, so merge atomically
            const uint32_t sh = 16u * (uint32_t)(j & 1);
            atomicAnd(&scls[k][j >> 1], ~(0xFFFFu << sh) | (c << sh));
        }
    }
    __syncthreads();
    if (lane == 0) {
        int n = 0;
        for (int k = 0; k < 216; ++k)
            if (ssrc[k] >= 0) {
                sib_src[216 * (int64_t)g + n] = ssrc[k];
                sib_cls[216 * (int64_t)g + n] = make_uint2(scls[k][0], scls[k][1]);
                ++n;
            }
        sib_cnt[g] = n;
    }
}

// Far-list windows to class numbers: every block numbers the used windows itself (in window order, a block
// scan of the flags into LDS), then maps its entries.
__global__ void __launch_bounds__(kThreads) k_remap(int32_t *cls, int64_t n, const int32_t *used) {
    __shared__ int32_t map[kWin3];
    __shared__ int32_t part[kThreads];
    const int per = (kWin3 + kThreads - 1) / kThreads, w0 = threadIdx.x * per;
    int32_t c = 0;
    for (int w = w0; w < min(kWin3, w0 + per); ++w) c += used[w] != 0;
    part[threadIdx.x] = c;
    __syncthreads();
    int32_t off = 0;
    for (int q = 0; q < (int)threadIdx.x; ++q) off += part[q];
    for (int w = w0; w < min(kWin3, w0 + per); ++w) {
        map[w] = off;
        off += used[w] != 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cls[i] = map[cls[i]];
}

// ------------------------------------------------------------------ Lagrange tables
// FP16 copy of the FP32 transfer tables, row-major by target index (k contiguous for the MFMA A
// operand), times a power-of-two scale.
__global__ void __launch_bounds__(kThreads)
k_to_half(const float *T, int64_t nplanes, int rp, float scale, _Float16 *T16) {
    const int64_t per = (int64_t)rp * rp;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= per * nplanes) return;
    const int64_t pl = g / per, e = g % per;
    const int i = (int)(e / rp), j = (int)(e % rp);   // element (i, j); T is stored as [j][i]
    T16[g] = (_Float16)(T[pl * per + (int64_t)j * rp + i] * scale);
}

// T_c[i][j] = G(|r0_c + (d_l / 2)(xi_i - xi_j)|), xi on the tensor Chebyshev grid; stored transposed
// (column j contiguous over i) for the MFMA A operand; zero padding beyond r.
__global__ void __launch_bounds__(kThreads)
k_lagrange_T(int ncls, const double *r0, int r1, int rp, const double *nodes, double half_dl, int helm, double k,
             float *T) {
    const int64_t per = (int64_t)rp * rp;
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= per * ncls) return;
    const int c = (int)(g / per);
    const int64_t e = g % per;
    const int j = (int)(e / rp), i = (int)(e % rp);   // element (i, j) at [c][j][i]
    const int r = r1 * r1 * r1;
    float re = 0.f, im = 0.f;
    if (i < r && j < r) {
        const int ia[3] = {i / (r1 * r1), (i / r1) % r1, i % r1};
        const int ja[3] = {j / (r1 * r1), (j / r1) % r1, j % r1};
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            double dd = r0[3 * c + d] + half_dl * (nodes[ia[d]] - nodes[ja[d]]);
            d2 += dd * dd;
        }
        const double rr = sqrt(d2);
        const double inv = 1.0 / (4.0 * M_PI * rr);
        if (helm) {
            double sn, cs;
            sincos(k * rr, &sn, &cs);
            re = (float)(cs * inv);
            im = (float)(sn * inv);
        } else {
            re = (float)inv;
        }
    }
    if (helm) {
        T[(int64_t)c * 2 * per + e] = re;
        T[(int64_t)c * 2 * per + per + e] = im;
    } else {
        T[(int64_t)c * per + e] = re;
    }
}

__global__ void __launch_bounds__(kThreads)
k_count_cls(const int32_t *cls, int64_t n, int32_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&cnt[cls[i]], 1);
}

// Pairs of one class go to consecutive 16-slot groups (order inside a class is free: every
// pair's product is computed on its own and written to its own slot).
__global__ void __launch_bounds__(kThreads)
k_fill_groups(const int32_t *cls, int64_t n, const int32_t *gstart, int32_t *cursor, int32_t *grp_pair) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cls[i];
    const int slot = atomicAdd(&cursor[c], 1);
    grp_pair[(int64_t)gstart[c] * 16 + slot] = (int32_t)i;
}

// ------------------------------------------------------------------ Gegenbauer tables
// D_c(+-s_p) = (ik / 4pi) w_p T_{L,r0}(+-s_p),  T_{L,r0}(s) = sum_{p=0..L} coef_p P_p(s . r0 / |r0|),
// coef_p = (2p + 1) i^p h_p(k |r0|) / (4 pi).  P_p(-t) = (-1)^p P_p(t) gives the antipode.
__global__ void __launch_bounds__(kThreads)
k_gegen_D(int64_t npair, int L, const double *dirs /*[npair][3] unit*/, const double *wts, const double *rhat,
          const double2 *coef /*[ncls][L+1]*/, const int32_t *reps /*[2 nrep]: class, mirror class or -1*/,
          double k, float4 *D, const double *phat, int nphat, double dphat, double kh) {
    extern __shared__ double2 sm[];
    double2 *sc = sm;               // series coefficients of this class
    double2 *rc = sm + (L + 1);     // Bonnet recurrence: P_{p+1} = a_p t P_p - b_p P_{p-1}
    const int c = reps[2 * blockIdx.y], cm = reps[2 * blockIdx.y + 1];
    for (int p = threadIdx.x; p <= L; p += blockDim.x) {
        sc[p] = coef[(int64_t)c * (L + 1) + p];
        rc[p] = make_double2((2.0 * p + 1.0) / (p + 1.0), p / (p + 1.0));
    }
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npair) return;
    const double t = dirs[3 * q] * rhat[3 * c] + dirs[3 * q + 1] * rhat[3 * c + 1] + dirs[3 * q + 2] * rhat[3 * c + 2];
    double pm = 1.0, pc = t;                 // P_0, P_1
    double er = sc[0].x, ei = sc[0].y;       // even-p part of the series
    double orr = 0.0, oi = 0.0;              // odd-p part
    if (L >= 1) {
        orr = sc[1].x * pc;
        oi = sc[1].y * pc;
    }
    for (int p = 1; p < L; ++p) {
        const double pn = rc[p].x * t * pc - rc[p].y * pm;
        pm = pc;
        pc = pn;
        if (p & 1) {   // p + 1 even
            er += sc[p + 1].x * pc;
            ei += sc[p + 1].y * pc;
        } else {
            orr += sc[p + 1].x * pc;
            oi += sc[p + 1].y * pc;
        }
    }
    // T(t) = even + odd, T(-t) = even - odd;  (ik/4pi) w (a + ib) = (w k / 4pi) (-b + ia)
    double f = wts[q] * k / (4.0 * M_PI);
    if (phat) {
        // grid form: both transforms carry the kernel's Fourier transform Phi(q) = prod_d phi^(k s_d h);
        // divide it out twice here (Phi(-q) = Phi(q))
        double Phi = 1.0;
        for (int d = 0; d < 3; ++d) {
            const double x = fabs(k * dirs[3 * q + d] * kh) / dphat;
            const int i = min((int)x, nphat - 2);
            const double t = x - i;
            Phi *= phat[i] * (1.0 - t) + phat[i + 1] * t;
        }
        f /= Phi * Phi;
    }
    const float4 dq = make_float4((float)(-f * (ei + oi)), (float)(f * (er + orr)), (float)(-f * (ei - oi)),
                                  (float)(f * (er - orr)));
    D[(int64_t)c * npair + q] = dq;
    // the mirror translation -r0 (same norm, so the same series) sees every direction pair reversed
    if (cm >= 0) D[(int64_t)cm * npair + q] = make_float4(dq.z, dq.w, dq.x, dq.y);
}

// Quadrature directions of a Gegenbauer level in antipodal-pair order (ring pairs m < (L+1)/2 with all 2L
// azimuths, then the equator ring with L azimuths when L + 1 is odd) and their weights w_m pi / L: unit
// vectors in FP64, and scaled by k / 2pi in FP64 and FP32 for the transform kernels.
__global__ void __launch_bounds__(kThreads)
k_quad_dirs(int64_t npair, int L, const double *xm, const double *wm, double kr, double *unit, double *wts,
            double *dirs64, float4 *dirs32) {
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= npair) return;
    const int64_t full = (int64_t)((L + 1) / 2) * 2 * L;
    const int m = q < full ? (int)(q / (2 * L)) : (L + 1) / 2;
    const int n = q < full ? (int)(q % (2 * L)) : (int)(q - full);
    const double ct = xm[m], stt = sqrt(1.0 - ct * ct);
    double sp, cp;
    sincospi((double)n / (double)L, &sp, &cp);
    const double u[3] = {stt * cp, stt * sp, ct};
    for (int d = 0; d < 3; ++d) {
        unit[3 * q + d] = u[d];
        dirs64[3 * q + d] = u[d] * kr;
    }
    wts[q] = wm[m] * M_PI / L;
    dirs32[q] = make_float4((float)(u[0] * kr), (float)(u[1] * kr), (float)(u[2] * kr), 0.f);
}

// ------------------------------------------------------------------ grid form tables
// Ez[m][c] = e^{-ik cos(t_m) z_c}, Ex[m][a][n] = e^{-ik sin(t_m) cos(f_n) x_a}, Ey[m][b][n] =
// e^{-ik sin(t_m) sin(f_n) y_b} for ring pairs m < nrp, n < L, grid nodes x_a = (a - (p-1)/2) h; ExT and EyT
// hold Ex and Ey as [m][n][node].
// Phases in revolutions from the ring tables (k / 2pi folded in), reduced and evaluated in FP64.
__global__ void __launch_bounds__(kThreads)
k_grid_tables(int nrp, int L, int p, double h, const double2 *rings, const double2 *phis, float2 *Ez, float2 *Ex,
              float2 *Ey, float2 *ExT, float2 *EyT) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nxy = (int64_t)nrp * p * L;
    auto cis = [](double rev) {
        const double f = rev - floor(rev);
        double sn, cs;
        sincospi(2.0 * f, &sn, &cs);
        return make_float2((float)cs, (float)(-sn));
    };
    if (i < nxy) {
        const int n = (int)(i % L);
        const int64_t ma = i / L;
        const int a = (int)(ma % p), m = (int)(ma / p);
        const double x = (a - 0.5 * (p - 1)) * h;
        const float2 ex = cis(rings[m].x * phis[n].x * x), ey = cis(rings[m].x * phis[n].y * x);
        Ex[i] = ex;
        Ey[i] = ey;
        const int64_t it = ((int64_t)m * L + n) * p + a;
        ExT[it] = ex;
        EyT[it] = ey;
    }
    if (i < (int64_t)nrp * p) {
        const int c = (int)(i % p), m = (int)(i / p);
        Ez[i] = cis(rings[m].y * (c - 0.5 * (p - 1)) * h);
    }
}

// Grid coordinates of every source point of a level, in node units (x_a = a for the node at
// (a - (p-1)/2) h from the box centre), FP32 as the spreading kernels use them, and the z-plane floor(z_g)
// that orders the points for the spreading launches: count per (box, plane).  A block's 256 consecutive points
// lie in few boxes: their counts are gathered in LDS (bins from the block's first box on, 2 p of them) and
// added to the global counts once per bin; points beyond those bins count globally.
constexpr int kZBins = 512;

__device__ __forceinline__ int box_of(int64_t i, const int32_t *start, int nbox) {
    int lo = 0, hi = nbox;   // box b with start[b] <= i < start[b + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(kThreads)
k_grid_zcount(int64_t n, const int32_t *start, int nbox, const double *xs, const double *ys, const double *zs,
              const double *ctr, double inv_h, int p, float zshift, int32_t *cnt, int32_t *cell_of, float4 *gtmp) {
    __shared__ int32_t hist[kZBins];
    const int64_t i0 = (int64_t)blockIdx.x * kThreads, i = i0 + threadIdx.x;
    for (int k = threadIdx.x; k < kZBins; k += kThreads) hist[k] = 0;
    const int64_t base = (int64_t)box_of(i0, start, nbox) * p;
    __syncthreads();
    if (i < n) {
        const int b = box_of(i, start, nbox);
        const float half = 0.5f * (float)(p - 1);
        const float xg = (float)((xs[i] - ctr[3 * b]) * inv_h) + half;
        const float yg = (float)((ys[i] - ctr[3 * b + 1]) * inv_h) + half;
        const float zg = (float)((zs[i] - ctr[3 * b + 2]) * inv_h) + half;
        const int c = min(max((int)floorf(zg + zshift), 0), p - 1);
        const int64_t slot = (int64_t)b * p + c;
        cell_of[i] = (int32_t)slot;
        gtmp[i] = make_float4(xg, yg, zg, 0.f);
        if (slot - base < kZBins) atomicAdd(&hist[slot - base], 1);
        else atomicAdd(&cnt[slot], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kZBins; k += kThreads)
        if (hist[k]) atomicAdd(&cnt[base + k], hist[k]);
}

// Each point's position in the (box, plane) order: one global cursor addition per bin of the block, then the
// point's rank within its bin in the block.
__global__ void __launch_bounds__(kThreads)
k_grid_zscatter(int64_t n, int p, const int32_t *cell_of, int32_t *cursor, int32_t *perm, const float4 *gtmp,
                float4 *gxyz) {
    __shared__ int32_t hist[kZBins], bin0[kZBins];
    const int64_t i0 = (int64_t)blockIdx.x * kThreads, i = i0 + threadIdx.x;
    for (int k = threadIdx.x; k < kZBins; k += kThreads) hist[k] = 0;
    const int64_t base = (int64_t)(cell_of[i0] / p) * p;    // bins from plane 0 of the block's first box
    __syncthreads();
    int64_t slot = -1;
    int rank = 0;
    if (i < n) {
        slot = cell_of[i];
        if (slot >= base && slot - base < kZBins) rank = atomicAdd(&hist[slot - base], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kZBins; k += kThreads)
        if (hist[k]) bin0[k] = atomicAdd(&cursor[base + k], hist[k]);
    __syncthreads();
    if (i < n) {
        const int pos = (slot >= base && slot - base < kZBins) ? bin0[slot - base] + rank : atomicAdd(&cursor[slot], 1);
        perm[pos] = (int32_t)i;
        gxyz[pos] = gtmp[i];
    }
}

__global__ void k_copy_i32(const int32_t *a, int32_t *b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ------------------------------------------------------------------ host helpers
void gauss_legendre_host(int n, std::vector<double> &x, std::vector<double> &w);

// Fourier transform of the spreading kernel phi(x) = exp(beta (sqrt(1 - (2x/w)^2) - 1)), |x| < w/2
// (exponential of semicircle), on a uniform grid of frequencies [0, 2.1] (grid units; the transforms
// need |k s_d h| <= pi / 1.9): Gauss-Legendre quadrature on the support, kept per (w, beta) for the
// life of the process.
const std::vector<double> &phi_hat_table(int w, double beta, double &step) {
    static std::mutex mx;
    static std::map<std::tuple<int, double>, std::vector<double>> cache;
    constexpr int kTab = 4096;
    constexpr double wmax = 2.1;
    step = wmax / (kTab - 1);
    std::lock_guard<std::mutex> lk(mx);
    auto key = std::make_tuple(w, beta);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    std::vector<double> x, wt;
    gauss_legendre_host(256, x, wt);
    std::vector<double> f(x.size());
    for (size_t j = 0; j < x.size(); ++j) {
        const double t = x[j];   // 2 x / w
        f[j] = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - t * t)) - 1.0)) * wt[j] * 0.5 * w;
    }
    std::vector<double> tab(kTab);
    for (int i = 0; i < kTab; ++i) {
        const double om = i * step;
        double a = 0.0;
        for (size_t j = 0; j < x.size(); ++j) a += f[j] * std::cos(om * 0.5 * w * x[j]);
        tab[i] = a;
    }
    return cache.emplace(key, std::move(tab)).first->second;
}


// Bound on the relative aliasing error of spreading one frequency with the kernel above: by Poisson
// summation, sum_a phi(x - a) e^{i om (a - x)} = sum_m phi^(om + 2 pi m) e^{2 pi i m x} (grid units), so the
// error relative to phi^(om) is at most sum_{m != 0} |phi^(om + 2 pi m)| / phi^(om); maximised over
// |om| <= kh (33 samples).  phi^ by 128-point Gauss-Legendre quadrature; kept per (w, beta, kh to 1/64) for
// the process.
double spread_alias_bound(int w, double beta, double kh) {
    static std::mutex mx;
    static std::map<std::tuple<int, int, int>, double> cache;
    const int qkh = (int)std::ceil(kh * 64.0);
    const auto key = std::make_tuple(w, (int)std::lround(beta * 100.0), qkh);
    {
        std::lock_guard<std::mutex> lk(mx);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    std::vector<double> x, wt;
    gauss_legendre_host(128, x, wt);
    std::vector<double> f(x.size());
    for (size_t j = 0; j < x.size(); ++j)
        f[j] = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - x[j] * x[j])) - 1.0)) * wt[j] * 0.5 * w;
    auto ft = [&](double om) {
        double a = 0.0;
        for (size_t j = 0; j < x.size(); ++j) a += f[j] * std::cos(om * 0.5 * w * x[j]);
        return a;
    };
    const double khq = qkh / 64.0;
    double worst = 0.0;
    for (int i = 0; i <= 32; ++i) {
        const double om = khq * i / 32.0;
        double s = 0.0;
        for (int m = 1; m <= 4; ++m) s += std::fabs(ft(om + 2.0 * M_PI * m)) + std::fabs(ft(2.0 * M_PI * m - om));
        worst = std::max(worst, s / ft(om));
    }
    worst *= 1.1;   // the maximum between the sampled frequencies (within 10% of a 64-point scan)
    std::lock_guard<std::mutex> lk(mx);
    cache[key] = worst;
    return worst;
}

// Grid of a grid-form level: p nodes per axis (whole 16-row MFMA blocks) of spacing h = dl / (p - 1 - w), so that
// every point's support lies inside the grid, with |k s_d h| = kh <= kh_max.  For each p from the smallest
// such multiple of 16 up to two steps larger, the narrowest width w in 4 ... 8 (with the best shape beta among
// 2.0 w .. 2.3 w) whose aliasing bound at that kh is at most eps / 2 (the bound covers one axis of one transform
// in the worst direction; measured products err by well under a third of it), and of these (p, w) the one the
// cost function rates cheapest.  Returns false if none qualifies.
template <class Cost>
bool grid_choice(double eps, double k, double dl, double kh_max, const Cost &cost, int &w, double &beta, int &p,
                 double &h, double &alias) {
    double best_cost = 1e300;
    bool found = false;
    const int p0 = ((int)std::ceil(dl * k / kh_max) + 4 + 1 + 15) / 16 * 16;
    for (int pp = p0; pp <= p0 + 32; pp += 16) {
        for (int ww = 4; ww <= 8; ++ww) {
            if (pp - 1 - ww <= 0) continue;
            const double hh = dl / (double)(pp - 1 - ww);
            if (k * hh > kh_max) continue;
            double bnd = 1e300, bb = 2.3 * ww;
            for (int c = 0; c < 4; ++c) {
                const double b = (2.0 + 0.1 * c) * ww;
                const double e = spread_alias_bound(ww, b, k * hh);
                if (e < bnd) {
                    bnd = e;
                    bb = b;
                }
            }
            if (bnd > eps / 2.0) continue;
            const double c = cost(pp, ww);
            if (c < best_cost) {
                best_cost = c;
                found = true;
                w = ww;
                beta = bb;
                p = pp;
                h = hh;
                alias = bnd;
            }
            break;   // wider kernels on the same grid only cost more
        }
    }
    return found;
}

void gauss_legendre_host(int n, std::vector<double> &x, std::vector<double> &w) {
    // Newton iteration on P_n from the Chebyshev-like initial guesses; nodes x_m in descending
    // order with exact mirror symmetry x_{n-1-m} = -x_m.
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int m = 0; m < (n + 1) / 2; ++m) {
        double z = std::cos(M_PI * (m + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 200; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p0 = 1.0; p1 = z; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16) {
                p0 = 1.0; p1 = z;
                for (int j = 2; j <= n; ++j) {
                    double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                break;
            }
        }
        if (2 * m + 1 == n) z = 0.0;
        x[m] = z;
        x[n - 1 - m] = -z;
        w[m] = w[n - 1 - m] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// h_p^(1)(z), p = 0..L, upward recurrence from h_0 = -i e^{iz} / z, h_1 = -e^{iz}(z + i) / z^2.
void hankel_host(int L, double z, std::vector<std::complex<double>> &h) {
    using C = std::complex<double>;
    h.assign(L + 1, C(0, 0));
    const C I(0, 1), e = std::exp(I * z);
    h[0] = -I * e / z;
    if (L >= 1) h[1] = -e * (z + I) / (z * z);
    for (int p = 1; p < L; ++p) h[p + 1] = (2.0 * p + 1.0) / z * h[p] - h[p - 1];
}

// ---- ACA of the transfer matrices of a Lagrange level (Sec. 2.2.2, eq. ffmACAmatvec): T_c ~ A_c B_c^T by cross
// approximation with complete pivoting (Bebendorf), in FP64 on the host.  Step k takes the largest entry (i, j)
// of the residual R = T - sum of the terms so far, a_k = R(:, j), b_k = R(i, :) / R(i, j), and the rank is the
// first k with |R|_F <= tol |T|_F, so every class meets the tolerance exactly.  The pivot is the first entry in
// row-major order whose squared modulus is within a relative 2e-9 of the largest, so that entries equal up to
// rounding (the tensor grid is symmetric) pick the same pivot on every machine.
namespace {
typedef std::complex<double> cd;

cd transfer_entry(const double *r0, const double *nodes, double dl, int r1, int helm, double k, int i, int j) {
#pragma clang fp contract(off)
    const int ia[3] = {i / (r1 * r1), (i / r1) % r1, i % r1};
    const int ja[3] = {j / (r1 * r1), (j / r1) % r1, j % r1};
    double dd[3];
    for (int d = 0; d < 3; ++d) dd[d] = r0[d] + 0.5 * dl * (nodes[ia[d]] - nodes[ja[d]]);
    const double rr = std::sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
    if (!helm) return cd(1.0 / (4.0 * M_PI * rr), 0.0);
    return cd(std::cos(k * rr) / (4.0 * M_PI * rr), std::sin(k * rr) / (4.0 * M_PI * rr));
}

// Columns of A and B (r entries each, column after column); returns the rank.
int aca_class(const double *r0, const double *nodes, double dl, int r1, int helm, double k, double tol,
              std::vector<cd> &A, std::vector<cd> &B) {
#pragma clang fp contract(off)
    const int r = r1 * r1 * r1;
    const size_t rr = (size_t)r * r;
    A.clear();
    B.clear();
    std::vector<cd> R(rr);
    double T2 = 0.0;
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) {
            const cd t = transfer_entry(r0, nodes, dl, r1, helm, k, i, j);
            R[(size_t)i * r + j] = t;
            T2 += t.real() * t.real() + t.imag() * t.imag();
        }
    int rank = 0;
    while (rank < r) {
        double R2 = 0.0, m = 0.0;
        for (size_t e = 0; e < rr; ++e) {
            const double q = R[e].real() * R[e].real() + R[e].imag() * R[e].imag();
            R2 += q;
            m = std::max(m, q);
        }
        if (R2 <= tol * tol * T2 || m == 0.0) break;
        size_t piv = 0;
        for (size_t e = 0; e < rr; ++e)
            if (R[e].real() * R[e].real() + R[e].imag() * R[e].imag() >= (1.0 - 2e-9) * m) {
                piv = e;
                break;
            }
        const int pi = (int)(piv / r), pj = (int)(piv % r);
        const cd pv = R[piv];
        const size_t a0 = A.size();
        for (int q = 0; q < r; ++q) {
            A.push_back(R[(size_t)q * r + pj]);
            B.push_back(R[(size_t)pi * r + q] / pv);
        }
        for (int i = 0; i < r; ++i) {
            const cd ai = A[a0 + i];
            for (int j = 0; j < r; ++j) R[(size_t)i * r + j] -= ai * B[a0 + j];
        }
        ++rank;
    }
    return rank;
}
}  // namespace

int lagrange_r1(int kernel, double k, double dl, double eps, int override_r1) {
    if (override_r1 > 0) return override_r1;
    int r1 = (int)std::ceil(std::log(1.0 / eps) / std::log(3.0 + std::sqrt(8.0)));
    if (kernel == FFM_HELMHOLTZ) r1 += (int)std::ceil(k * dl / 2.0);
    return std::max(r1, 1);
}

int gegenbauer_L(double k, double dl, double eps) {
    int L = (int)std::floor(k * std::sqrt(3.0) * dl - std::log(eps));
    return std::max(L, 1);
}

template <class T>
void upload(DevBuf<T> &b, const std::vector<T> &h, hipStream_t st, Scratch &SC) {
    b.alloc(h.size());
    if (!h.empty()) FFM_HIP(hipMemcpyAsync(b.p, SC.stage(h), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// upload into a scratch-owned buffer (released with the scratch list, after the final sync)
template <class T>
T *keep(Scratch &SC, const std::vector<T> &h, hipStream_t st) {
    T *p = SC.get<T>(std::max<size_t>(h.size(), 1));
    if (!h.empty()) FFM_HIP(hipMemcpyAsync(p, SC.stage(h), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return p;
}

// ------------------------------------------------------------------ tree construction
void build_tree(Tree &T, const double *P, int64_t n, const double corner[3], double S, hipStream_t st,
                Scratch &SC) {
    T.n = n;
    std::memcpy(T.corner, corner, sizeof(double) * 3);
    T.key.alloc(n);
    T.perm.alloc(n);
    FFM_LAUNCH(k_morton, nblocks(n), kThreads, 0, st, P, n, corner[0], corner[1], corner[2], S, T.key.p, T.perm.p);
    radix_sort_u64_u32(T.key.p, T.perm.p, n, st, SC);
    T.xs.alloc(n);
    T.ys.alloc(n);
    T.zs.alloc(n);
    FFM_LAUNCH(k_gather, nblocks(n), kThreads, 0, st, P, n, T.perm.p, T.xs.p, T.ys.p, T.zs.p);
}

struct LevelScratch {
    DevBuf<int8_t> f;
    DevBuf<int32_t> boxid_prev;
    std::vector<int64_t> cum;   // boxes per level (cumulative start counts)
    Scratch *sc = nullptr;
};

void first_levels(Tree &T, LevelScratch &S, hipStream_t st) {
    const int64_t n = T.n;
    S.f.alloc(n);
    DevBuf<int32_t> hist(23);
    FFM_HIP(hipMemsetAsync(hist.p, 0, 23 * sizeof(int32_t), st));
    FFM_LAUNCH(k_first_level, nblocks(n), kThreads, 0, st, T.key.p, n, S.f.p, hist.p);
    std::vector<int32_t> h(23);
    FFM_HIP(hipMemcpyAsync(h.data(), hist.p, 23 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FFM_HIP(hipStreamSynchronize(st));
    S.cum.assign(23, 0);
    int64_t acc = 0;
    for (int l = 0; l < 23; ++l) {
        acc += h[l];
        S.cum[l] = acc;
    }
    T.boxid.alloc(n);
    S.boxid_prev.alloc(n);
}

void build_level(Tree &T, LevelScratch &S, int l, double d0, hipStream_t st) {
    const int64_t n = T.n;
    TreeLevel &L = T.lev[l];
    L.nbox = (int32_t)S.cum[l];
    const int64_t ntile = (n + kLvlTile - 1) / kLvlTile;
    int32_t *tcount = S.sc->get<int32_t>(std::max<int64_t>(ntile, 1));
    FFM_LAUNCH(k_lvl_count, ntile, kThreads, 0, st, S.f.p, n, l, tcount);
    L.start.alloc(L.nbox + 1);
    L.ijk.alloc((size_t)3 * L.nbox);
    L.ctr.alloc((size_t)3 * L.nbox);
    if (l > 0) std::swap(S.boxid_prev, T.boxid);
    const double h = std::ldexp(d0, -(l + 1));
    FFM_LAUNCH(k_lvl_boxes, ntile, kThreads, 0, st, T.key.p, S.f.p, n, l, (const int32_t *)tcount, T.corner[0],
               T.corner[1], T.corner[2], h, L.start.p, L.ijk.p, L.ctr.p, T.boxid.p, L.nbox);
    if (l > 0) {
        TreeLevel &Pl = T.lev[l - 1];
        L.parent.alloc(L.nbox);
        Pl.child.alloc(Pl.nbox + 1);
        FFM_LAUNCH(k_link, nblocks(std::max<int64_t>(L.nbox, Pl.nbox)), kThreads, 0, st, L.start.p, L.nbox,
                   S.boxid_prev.p, L.parent.p, Pl.start.p, Pl.nbox, T.boxid.p, Pl.child.p);
    }
    T.built = l;
}


// Work lists of a level, built on the host from the box sizes and list pointers: largest boxes
// first so that the longest blocks start early.
// What the work lists of a level need on the host (box ranges, the far or near pointer array, the marks of
// the source boxes with far work, the near pair count), copied into pinned memory in stream order, so that the
// lists of every level are read after one synchronisation.
struct WorkFetch {
    int32_t *par = nullptr;              // one tree, far levels: parent of every box
    int32_t *sx = nullptr, *sy = nullptr;
    int64_t *ptr = nullptr;
    uint8_t *act = nullptr;
    unsigned long long *near_pairs = nullptr;
    int64_t *sym_tot = nullptr;          // symmetric leaf near field: length of the source-side buffer
    int nbx = 0, nby = 0;
};

void fetch_work_lists(Level &LV, const TreeLevel &LX, const TreeLevel &LY, bool near, hipStream_t st, Scratch &SC,
                      WorkFetch &F, bool sym = false) {
    F.nbx = LX.nbox;
    F.nby = LY.nbox;
    F.sx = SC.pin<int32_t>(LX.nbox + 1);
    F.sy = SC.pin<int32_t>(LY.nbox + 1);
    F.ptr = SC.pin<int64_t>(LX.nbox + 1);
    FFM_HIP(hipMemcpyAsync(F.sx, LX.start.p, sizeof(int32_t) * (LX.nbox + 1), hipMemcpyDeviceToHost, st));
    FFM_HIP(hipMemcpyAsync(F.sy, LY.start.p, sizeof(int32_t) * (LY.nbox + 1), hipMemcpyDeviceToHost, st));
    const DevBuf<int64_t> &dptr = near ? LV.near_ptr : LV.far_ptr;
    FFM_HIP(hipMemcpyAsync(F.ptr, dptr.p, sizeof(int64_t) * (LX.nbox + 1), hipMemcpyDeviceToHost, st));
    if (near) {
        F.near_pairs = SC.pin<unsigned long long>(1);
        *F.near_pairs = 0;
        if (LV.nnear) {
            unsigned long long *dn = SC.get<unsigned long long>(1);
            FFM_HIP(hipMemsetAsync(dn, 0, sizeof(unsigned long long), st));
            FFM_LAUNCH(k_near_pairs, nblocks(LX.nbox), kThreads, 0, st, LV.near_ptr.p, LV.near_src.p, LX.nbox,
                       LX.start.p, LY.start.p, dn);
            FFM_HIP(hipMemcpyAsync(F.near_pairs, dn, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        }
        if (sym && LV.nnear) {
            // offsets of the symmetric pairs' source-side slices (one tree: LX is LY)
            // the scan writes its totals after the last element: outputs of nbox + 1
            int64_t *cnt = SC.get<int64_t>(LX.nbox), *boff = SC.get<int64_t>(LX.nbox + 1);
            int64_t *boff2 = SC.get<int64_t>(LX.nbox + 1);
            F.sym_tot = SC.pin<int64_t>(2);
            F.sym_tot[0] = F.sym_tot[1] = 0;
            FFM_LAUNCH(k_sym_box_count, nblocks(LX.nbox), kThreads, 0, st, LV.near_ptr.p, LV.near_src.p, LX.nbox,
                       LX.start.p, cnt);
            exclusive_scan2_i64(cnt, boff, cnt, boff2, LX.nbox, F.sym_tot, st, SC);
            LV.near_off.alloc((size_t)LV.nnear);
            FFM_LAUNCH(k_sym_fill, nblocks(LX.nbox), kThreads, 0, st, LV.near_ptr.p, LV.near_src.p, LX.nbox,
                       LX.start.p, boff, LV.near_off.p);
            FFM_LAUNCH(k_sym_reverse, nblocks(LX.nbox), kThreads, 0, st, LV.near_ptr.p, LV.near_src.p, LX.nbox,
                       LV.near_off.p);
        }
    } else {
        if (sym) {
            F.par = SC.pin<int32_t>(LX.nbox);
            FFM_HIP(hipMemcpyAsync(F.par, LX.parent.p, sizeof(int32_t) * LX.nbox, hipMemcpyDeviceToHost, st));
        }
        uint8_t *dact = SC.get<uint8_t>(std::max(LY.nbox, 1));
        FFM_HIP(hipMemsetAsync(dact, 0, LY.nbox, st));
        FFM_LAUNCH(k_mark_sources, nblocks(LV.nfar), kThreads, 0, st, LV.far_src.p, LV.nfar, dact);
        F.act = SC.pin<uint8_t>(LY.nbox);
        FFM_HIP(hipMemcpyAsync(F.act, dact, LY.nbox, hipMemcpyDeviceToHost, st));
    }
}

// The work lists of a level from its fetched data (after the stream has passed the fetch): boxes with work,
// largest first, and their point counts.
void build_work_lists(Plan &P, Level &LV, bool near, const WorkFetch &F) {
    std::vector<int32_t> sx(F.sx, F.sx + F.nbx + 1), sy(F.sy, F.sy + F.nby + 1);
    if (F.par) LV.h_par.assign(F.par, F.par + F.nbx);
    const int64_t *ptr = F.ptr;
    const uint8_t *act = F.act;
    const unsigned long long near_pairs = F.near_pairs ? *F.near_pairs : 0ull;
    struct {
        int32_t nbox;
    } LX{F.nbx}, LY{F.nby};
    // boxes by decreasing point count, ties in index order (counting sort over the counts)
    auto by_size = [](const std::vector<int32_t> &start, std::vector<int32_t> &boxes) {
        if (boxes.size() < 2) return;
        int32_t mx = 0;
        for (int32_t b : boxes) mx = std::max(mx, start[b + 1] - start[b]);
        if ((size_t)mx > 8 * boxes.size() + 4096) {
            std::stable_sort(boxes.begin(), boxes.end(), [&](int32_t a, int32_t b) {
                return start[a + 1] - start[a] > start[b + 1] - start[b];
            });
            return;
        }
        std::vector<int32_t> cnt((size_t)mx + 2, 0), out(boxes.size());
        for (int32_t b : boxes) ++cnt[(size_t)(mx - (start[b + 1] - start[b])) + 1];
        for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
        for (int32_t b : boxes) out[cnt[(size_t)(mx - (start[b + 1] - start[b]))]++] = b;
        boxes.swap(out);
    };
    std::vector<int32_t> tgt;
    for (int32_t t = 0; t < LX.nbox; ++t)
        if (ptr[t + 1] > ptr[t]) tgt.push_back(t);
    by_size(sx, tgt);
    LV.h_sx = sx;
    LV.h_sy = sy;
    if (near) {
        LV.h_near = std::move(tgt);
        P.stats.near_pairs = (double)near_pairs;
        return;
    }
    std::vector<int32_t> fwd;
    for (int32_t s = 0; s < LY.nbox; ++s)
        if (act[s]) {
            fwd.push_back(s);
            LV.max_src_pts = std::max(LV.max_src_pts, sy[s + 1] - sy[s]);
        }
    by_size(sy, fwd);
    double npts_src = 0, npts_tgt = 0;
    for (int32_t s : fwd) npts_src += sy[s + 1] - sy[s];
    for (int32_t t : tgt) {
        npts_tgt += sx[t + 1] - sx[t];
        LV.max_tgt_pts = std::max(LV.max_tgt_pts, sx[t + 1] - sx[t]);
    }
    LV.pts_src = npts_src;
    LV.pts_tgt = npts_tgt;
    LV.h_fwd = std::move(fwd);
    LV.h_tgt = std::move(tgt);
}

// The early lists of a level (per-pair leaf rule): target boxes with early pairs (host, after the fetch) and their
// point pairs.
void fetch_early_lists(Level &LV, const TreeLevel &LX, const TreeLevel &LY, hipStream_t st, Scratch &SC, WorkFetch &F) {
    F.nbx = LX.nbox;
    F.nby = LY.nbox;
    F.sx = SC.pin<int32_t>(LX.nbox + 1);
    F.ptr = SC.pin<int64_t>(LX.nbox + 1);
    FFM_HIP(hipMemcpyAsync(F.sx, LX.start.p, sizeof(int32_t) * (LX.nbox + 1), hipMemcpyDeviceToHost, st));
    FFM_HIP(hipMemcpyAsync(F.ptr, LV.early_ptr.p, sizeof(int64_t) * (LX.nbox + 1), hipMemcpyDeviceToHost, st));
    F.near_pairs = SC.pin<unsigned long long>(1);
    *F.near_pairs = 0;
    unsigned long long *dn = SC.get<unsigned long long>(1);
    FFM_HIP(hipMemsetAsync(dn, 0, sizeof(unsigned long long), st));
    FFM_LAUNCH(k_near_pairs, nblocks(LX.nbox), kThreads, 0, st, LV.early_ptr.p, LV.early_src.p, LX.nbox, LX.start.p,
               LY.start.p, dn);
    FFM_HIP(hipMemcpyAsync(F.near_pairs, dn, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
}

void build_early_lists(Level &LV, const WorkFetch &F) {
    std::vector<int32_t> tgt;
    for (int32_t t = 0; t < F.nbx; ++t)
        if (F.ptr[t + 1] > F.ptr[t]) tgt.push_back(t);
    // boxes by decreasing point count (ties in index order)
    std::stable_sort(tgt.begin(), tgt.end(), [&](int32_t a, int32_t b) {
        return F.sx[a + 1] - F.sx[a] > F.sx[b + 1] - F.sx[b];
    });
    LV.h_early = std::move(tgt);
    LV.early_pairs = (double)*F.near_pairs;
}

// FFM_LOG=1: host wall time of the plan phases on stderr (quiet by default)
struct PhaseLog {
    bool on = std::getenv("FFM_LOG") && std::getenv("FFM_LOG")[0] == '1';
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    std::string title = "ffm_plan ms:";
    std::string line;
    PhaseLog() = default;
    explicit PhaseLog(const char *what) : title(what) {}
    void mark(const char *what) {
        if (!on) return;
        auto now = std::chrono::steady_clock::now();
        char buf[64];
        std::snprintf(buf, sizeof(buf), " %s=%.3f", what, std::chrono::duration<double, std::milli>(now - t).count());
        line += buf;
        t = now;
    }
    ~PhaseLog() {
        if (on) std::fprintf(stderr, "%s%s\n", title.c_str(), line.c_str());
    }
};

}  // namespace

// =========================================================================== plan
void plan_build(Plan &P, const double *X, const double *Y, hipStream_t st) {
    PhaseLog plog;
    const int64_t nx = P.nx, ny = P.ny;
    if (P.empty) return;

    // --- root cubes (Sec. 2.2.1)
    double lo[2][3], hi[2][3];
    {
        const double *PS[2] = {X, Y};
        const int64_t NS[2] = {nx, ny};
        const int nsets = P.same ? 1 : 2;
        DevBuf<double> part(6 * 1024 * 2), out(12);
        DevBuf<int> bad(1);
        FFM_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
        for (int e = 0; e < nsets; ++e) {
            int nb = (int)std::min<int64_t>(1024, (NS[e] + kThreads - 1) / kThreads);
            FFM_LAUNCH(k_bbox_partial, nb, kThreads, 0, st, PS[e], NS[e], part.p + 6 * 1024 * e, bad.p);
            FFM_LAUNCH(k_bbox_final, 1, kThreads, 0, st, part.p + 6 * 1024 * e, nb, out.p + 6 * e);
        }
        double h6[12];
        int hbad = 0;
        FFM_HIP(hipMemcpyAsync(h6, out.p, sizeof(double) * 6 * nsets, hipMemcpyDeviceToHost, st));
        FFM_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
        FFM_HIP(hipStreamSynchronize(st));
        FFM_CHECK(!hbad, FFM_EINVAL, "ffm_plan: a coordinate is NaN or infinite");
        if (P.same) std::memcpy(h6 + 6, h6, sizeof(double) * 6);
        for (int e = 0; e < 2; ++e)
            for (int d = 0; d < 3; ++d) {
                lo[e][d] = h6[6 * e + d];
                hi[e][d] = h6[6 * e + 3 + d];
            }
    }
    double d0 = 0.0;
    for (int e = 0; e < 2; ++e)
        for (int d = 0; d < 3; ++d) d0 = std::max(d0, hi[e][d] - lo[e][d]);
    if (d0 == 0.0) d0 = 1.0;
    double corner[2][3];
    {
#pragma clang fp contract(off)
        for (int e = 0; e < 2; ++e)
            for (int d = 0; d < 3; ++d) corner[e][d] = (lo[e][d] + hi[e][d]) * 0.5 - d0 * 0.5;
    }
    P.d0 = d0;
    P.S = (double)(1 << kBits) / d0;
    P.aligned = std::memcmp(corner[0], corner[1], sizeof(double) * 3) == 0;

    plog.mark("bbox");
    // --- Morton-sorted trees (Sec. 2.1)
    Scratch SC(st);
    P.tx.reset(new Tree());
    build_tree(*P.tx, X, nx, corner[0], P.S, st, SC);
    if (P.dn) {
        // read before the plan's next host wait, so the caller may free the normals when ffm_plan returns
        P.tnrm.alloc(nx);
        FFM_LAUNCH(k_gather_normals, nblocks(nx), kThreads, 0, st, P.user_normals, nx, P.tx->perm.p, P.tnrm.p);
    }
    if (P.same) {
        P.ty = P.tx.get();
    } else {
        P.ty_own.reset(new Tree());
        build_tree(*P.ty_own, Y, ny, corner[1], P.S, st, SC);
        P.ty = P.ty_own.get();
    }
    if (P.dl) {
        P.snrm.alloc(ny);
        FFM_LAUNCH(k_gather_normals, nblocks(ny), kThreads, 0, st, P.user_snormals, ny, P.ty->perm.p, P.snrm.p);
    }
    Tree &TX = *P.tx, &TY = *P.ty;
    LevelScratch SX, SY;
    SX.sc = SY.sc = &SC;
    first_levels(TX, SX, st);
    if (!P.same) first_levels(TY, SY, st);
    plog.mark("trees");
    const int maxlev = P.opt.max_level;
    build_level(TX, SX, 0, d0, st);
    if (!P.same) build_level(TY, SY, 0, d0, st);

    // --- descent lists (Sec. 2.2.2, 2.2.4; Prop. 1): near_0 = {(root, root)}; the near lists of
    // level l - 1 (CSR by target) generate the candidates of level l.
    {
        Level &L0 = P.lev[0];
        const int64_t h_ptr[2] = {0, 1};
        const int32_t h_src[1] = {0};
        L0.near_ptr.alloc(2);
        L0.near_src.alloc(1);
        L0.nnear = 1;
        FFM_HIP(hipMemcpyAsync(L0.near_ptr.p, h_ptr, sizeof(h_ptr), hipMemcpyHostToDevice, st));
        FFM_HIP(hipMemcpyAsync(L0.near_src.p, h_src, sizeof(h_src), hipMemcpyHostToDevice, st));
    }
    int *bad = SC.get<int>(1);
    FFM_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    // translation windows in use per level: read back with the work lists, after the descent
    std::vector<int32_t *> win_used(maxlev + 1, nullptr);
    int64_t *tot_h = SC.pin<int64_t>(2);      // list totals, written by the scan kernel
    P.leaf = maxlev;
    for (int l = 1; l <= maxlev; ++l) {
        build_level(TX, SX, l, d0, st);
        if (!P.same) build_level(TY, SY, l, d0, st);
        const int32_t nbx = TX.lev[l].nbox;
        Level &LV = P.lev[l];
        const Level &LP = P.lev[l - 1];
        const double dl = std::ldexp(d0, -l);
        FarTest ft;
        ft.ijk_t = TX.lev[l].ijk.p;
        ft.ijk_s = TY.lev[l].ijk.p;
        ft.ctr_t = TX.lev[l].ctr.p;
        ft.ctr_s = TY.lev[l].ctr.p;
        ft.two_dl = 2.0 * dl;
        ft.aligned = P.aligned ? 1 : 0;
        for (int d = 0; d < 3; ++d) {
            // offsets of level-1 pairs lie in [-1, 1]; deeper ones within [f - 4, f + 5],
            // f = floor(-(corner_X - corner_Y) / d_l): window [f - 5, f + 6]
            ft.base[d] = (l == 1) ? -1 : (int32_t)std::floor(-(corner[0][d] - corner[1][d]) / dl) - 5;
            LV.win_base[d] = ft.base[d];
        }
        int64_t *cnt_f = SC.get<int64_t>(nbx + 1), *cnt_n = SC.get<int64_t>(nbx + 1);
        win_used[l] = SC.get<int32_t>(kWin3);
        FFM_LAUNCH(k_list_count, nblocks(std::max<int64_t>((int64_t)nbx * 64, kWin3)), kThreads, 0, st, nbx, TX.lev[l].parent.p,
                   LP.near_ptr.p, LP.near_src.p, TY.lev[l - 1].child.p, ft, cnt_f, cnt_n, win_used[l]);
        LV.far_ptr.alloc(nbx + 1);
        LV.near_ptr.alloc(nbx + 1);
        // both list offsets in one scan; the two totals arrive in host-visible memory (a total still negative
        // after the synchronisation, which never happens when the kernel's writes are visible, is read back
        // from the device instead: the list buffers are sized by it)
        tot_h[0] = tot_h[1] = -1;
        exclusive_scan2_i64(cnt_f, LV.far_ptr.p, cnt_n, LV.near_ptr.p, nbx, tot_h, st, SC);
        FFM_HIP(hipStreamSynchronize(st));
        if (tot_h[0] < 0 || tot_h[1] < 0) {
            FFM_HIP(hipMemcpy(&tot_h[0], LV.far_ptr.p + nbx, sizeof(int64_t), hipMemcpyDeviceToHost));
            FFM_HIP(hipMemcpy(&tot_h[1], LV.near_ptr.p + nbx, sizeof(int64_t), hipMemcpyDeviceToHost));
        }
        LV.nfar = tot_h[0];
        LV.nnear = tot_h[1];
        LV.far_src.alloc(LV.nfar);
        LV.far_cls.alloc(LV.nfar);
        LV.near_src.alloc(std::max<int64_t>(LV.nnear, 1));
        FFM_LAUNCH(k_list_fill, nblocks((int64_t)nbx * 64), kThreads, 0, st, nbx, TX.lev[l].parent.p, LP.near_ptr.p, LP.near_src.p,
                   TY.lev[l - 1].child.p, ft, LV.far_ptr.p, LV.near_ptr.p, LV.far_src.p, LV.far_cls.p,
                   LV.near_src.p, win_used[l], bad);
        // compact translation classes (numbered in window order) on the device
        if (LV.nfar) FFM_LAUNCH(k_remap, nblocks(LV.nfar), kThreads, 0, st, LV.far_cls.p, LV.nfar, win_used[l]);
        // stopping rule (Sec. 2.2.4)
        const int64_t nb = (int64_t)TX.lev[l].nbox + TY.lev[l].nbox;
        if (LV.nnear == 0 || nx + ny <= (int64_t)P.opt.n_leaf * nb || l == maxlev) {
            P.leaf = l;
            break;
        }
        // per-pair leaf rule (beyond the paper's global rule): near pairs whose two boxes both hold at most n_leaf
        // points are summed densely at this level (the early list) instead of refined; the level is the leaf if
        // nothing is left to refine
        if (P.opt.flags & FFM_FLAG_ADAPTIVE_LEAVES) {
            int64_t *cnt_e = SC.get<int64_t>(nbx + 1), *cnt_r = SC.get<int64_t>(nbx + 1);
            FFM_LAUNCH(k_split_count, nblocks(nbx), kThreads, 0, st, nbx, LV.near_ptr.p, LV.near_src.p,
                       TX.lev[l].start.p, TY.lev[l].start.p, P.opt.n_leaf, cnt_e, cnt_r);
            DevBuf<int64_t> eptr(nbx + 1), rptr(nbx + 1);
            tot_h[0] = tot_h[1] = -1;
            exclusive_scan2_i64(cnt_e, eptr.p, cnt_r, rptr.p, nbx, tot_h, st, SC);
            FFM_HIP(hipStreamSynchronize(st));
            if (tot_h[0] < 0 || tot_h[1] < 0) {
                FFM_HIP(hipMemcpy(&tot_h[0], eptr.p + nbx, sizeof(int64_t), hipMemcpyDeviceToHost));
                FFM_HIP(hipMemcpy(&tot_h[1], rptr.p + nbx, sizeof(int64_t), hipMemcpyDeviceToHost));
            }
            if (tot_h[1] == 0) {
                P.leaf = l;
                break;
            }
            if (tot_h[0] > 0) {
                DevBuf<int32_t> esrc(tot_h[0]), rsrc(tot_h[1]);
                FFM_LAUNCH(k_split_fill, nblocks(nbx), kThreads, 0, st, nbx, LV.near_ptr.p, LV.near_src.p,
                           TX.lev[l].start.p, TY.lev[l].start.p, P.opt.n_leaf, eptr.p, rptr.p, esrc.p, rsrc.p);
                LV.nearly = tot_h[0];
                LV.early_ptr = std::move(eptr);
                LV.early_src = std::move(esrc);
                LV.near_ptr = std::move(rptr);
                LV.near_src = std::move(rsrc);
                LV.nnear = tot_h[1];
            }
        }
    }

    plog.mark("lists");
    // the host side of every level's work lists, after one synchronisation
    std::vector<WorkFetch> wf(P.leaf + 1);
    WorkFetch wf_near;
    std::vector<WorkFetch> wf_early(P.leaf + 1);
    for (int l = 1; l <= P.leaf; ++l) {
        if (P.lev[l].nfar) fetch_work_lists(P.lev[l], TX.lev[l], TY.lev[l], false, st, SC, wf[l], P.same);
        if (l < P.leaf && P.lev[l].nearly) fetch_early_lists(P.lev[l], TX.lev[l], TY.lev[l], st, SC, wf_early[l]);
    }
    // one set: the leaf near field evaluates each unordered pair of distinct boxes once (G is symmetric; the
    // normal derivatives are not)
    P.near_sym = P.same;
    fetch_work_lists(P.lev[P.leaf], TX.lev[P.leaf], TY.lev[P.leaf], true, st, SC, wf_near, P.near_sym);
    int32_t *used_h = SC.pin<int32_t>((size_t)kWin3 * (P.leaf + 1) + 1);
    for (int l = 1; l <= P.leaf; ++l)
        FFM_HIP(hipMemcpyAsync(used_h + (size_t)kWin3 * l, win_used[l], sizeof(int32_t) * kWin3,
                               hipMemcpyDeviceToHost, st));
    FFM_HIP(hipMemcpyAsync(used_h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    FFM_HIP(hipStreamSynchronize(st));
    FFM_CHECK(!used_h[0], FFM_EINTERNAL, "ffm_plan: translation outside its window");
    // translation classes of every level on the host: the same window-order numbering as k_remap
    for (int l = 1; l <= P.leaf; ++l) {
        Level &LV = P.lev[l];
        const int32_t *used = used_h + (size_t)kWin3 * l;
        LV.cls_off.clear();
        LV.ncls = 0;
        for (int w = 0; w < kWin3; ++w)
            if (used[w]) {
                ++LV.ncls;
                LV.cls_off.push_back(w / (kWin * kWin) + LV.win_base[0]);
                LV.cls_off.push_back((w / kWin) % kWin + LV.win_base[1]);
                LV.cls_off.push_back(w % kWin + LV.win_base[2]);
            }
    }
    // --- compression form and tables per level (Sec. 2.2.2, 2.2.3)
    size_t ws_src = 0, ws_tgt = 0, ws_z = 0, ws_part = 0, ws_gG = 0, ws_gH = 0;
    for (int l = 1; l <= P.leaf; ++l) {
        Level &LV = P.lev[l];
        if (LV.nfar == 0) continue;
        const double dl = std::ldexp(d0, -l);
        std::vector<double> r0(3 * (size_t)LV.ncls);
        for (int c = 0; c < LV.ncls; ++c)
            for (int d = 0; d < 3; ++d)
                r0[3 * c + d] = (corner[0][d] - corner[1][d]) + (double)LV.cls_off[3 * c + d] * dl;
        const int32_t nby = TY.lev[l].nbox, nbx = TX.lev[l].nbox;
        plog.mark("tab.start");
        const bool geg = P.kernel == FFM_HELMHOLTZ && P.k * dl >= P.opt.kd_switch;
        if (geg) {
            LV.method = kGegenbauer;
            LV.L = gegenbauer_L(P.k, dl, P.eps);
            FFM_CHECK(LV.L <= 1000, FFM_EINVAL, "ffm_plan: k * d_0 too large (Gegenbauer rank above 1000)");
        }
        build_work_lists(P, LV, false, wf[l]);
        plog.mark("tab.work");
        if (geg) {
            const int L = LV.L, nth = L + 1;
            LV.nq = 2 * (int64_t)L * (L + 1);
            LV.npair = LV.nq / 2;
            std::vector<double> xm, wm;
            gauss_legendre_host(nth, xm, wm);
            std::vector<double> cph(L), sph(L);
            for (int n = 0; n < L; ++n) {
                cph[n] = std::cos(M_PI * n / L);
                sph[n] = std::sin(M_PI * n / L);
            }
            const double kr = P.k / (2.0 * M_PI);
            const double *dxm = keep(SC, xm, st), *dwm = keep(SC, wm, st);
            double *ddirs = SC.get<double>(3 * LV.npair), *dwts = SC.get<double>(LV.npair);
            LV.dirs.alloc((size_t)LV.npair);
            LV.dirs64.alloc((size_t)3 * LV.npair);
            FFM_LAUNCH(k_quad_dirs, nblocks(LV.npair), kThreads, 0, st, LV.npair, L, dxm, dwm, kr, ddirs, dwts,
                       LV.dirs64.p, LV.dirs.p);
            // ring-pair tables: (sin, cos) of every ring pair's polar angle, scaled by k / 2pi, and the
            // azimuths of one half turn
            LV.nrp = nth / 2 + (nth & 1);
            std::vector<double2> rings(LV.nrp), phis(L);
            for (int m = 0; m < LV.nrp; ++m)
                rings[m] = make_double2(std::sqrt(1.0 - xm[m] * xm[m]) * kr, xm[m] * kr);
            for (int n = 0; n < L; ++n) phis[n] = make_double2(cph[n], sph[n]);
            upload(LV.rings, rings, st, SC);
            upload(LV.phis, phis, st, SC);
            plog.mark("tab.quad");
            // FP64 phase reduction where the FP32 rounding of the largest phase (a few ulp of
            // k sqrt(3) d_l / 2 radians) would reach eps / 20; the per-(point, ring) factor e^{iC} of
            // the ring-pair form is always reduced in FP64
            const double max_rad = P.k * dl * std::sqrt(3.0) * 0.5;
            // FP32 phases go to the hardware sine unreduced, which needs |phase| <= 128 revolutions
            LV.phase64 = max_rad * std::ldexp(1.0, -22) > P.eps / 20.0 || max_rad / (2.0 * M_PI) > 128.0;
            // form of the transforms: the direct sums, or the grid form where it is cheaper (points spread
            // onto a uniform grid of spacing h <= pi / (1.9 k) with a kernel of width w, separable sums from
            // the grid to the directions, the kernel's Fourier transform divided out in the transfer)
            const double *dphat = nullptr;
            int nphat = 0;
            double dphat_step = 1.0;
            {
                // cost model in seconds, from measured MI355X rates: direct sums 9e-14 s per (point,
                // direction); grid form: spreading 0.29 ns per point plus 2.5 ns per (box, plane) launch item
                // and interpolation 0.12 ns per point (w = 6; w^3 nodes per point), and the four sums on FP32
                // MFMA (real multiply-adds as issued) at a fraction of the 78.6e12 per second peak that falls
                // with narrower grids (measured 0.5 at 64 nodes, 0.44 at 48, 0.37 at 32; 0.46 at 80 and 0.66 at
                // 128 with the plane sums' rows held in registers, linear between; 0.35 above 128)
                const double nbf = (double)LV.h_fwd.size(), nbt = (double)LV.h_tgt.size();
                auto grid_cost = [&](int pp, int ww) {
                    const double ws = (double)ww / 6.0, p2 = (double)pp * pp, p3 = p2 * pp;
                    const double rings16 = 16.0 * ((LV.nrp + 15) / 16), tiles64 = 64.0 * ((pp + 63) / 64);
                    const double macs = (nbf + nbt) * 4.0 * rings16 * p3 +                    // over z, both ways
                                        nbf * 4.0 * p2 * (L + 1.0) * 8.0 * ((L + 7) / 8) +    // plane to directions
                                        nbt * 4.0 * pp * tiles64 * (L + 1.0) * 2.0 * ((L + 1) / 2);   // and back
                    const double eff = pp > 128 ? 0.35
                                       : pp > 64 ? 0.46 + 0.2 * (pp - 80) / 48.0
                                                 : 0.5 * std::pow(pp / 64.0, 0.45);
                    return ws * ws * ws * (0.29e-9 * LV.pts_src + 0.12e-9 * LV.pts_tgt) + 2.5e-9 * nbf * pp +
                           macs / (eff * 78.6e12);
                };
                // grids down to 1.5 nodes per half wavelength: k s_d h <= pi / 1.5, where the kernel's Fourier
                // transform divided out stays above 0.3 per axis
                int w = 0, p = 0;
                double beta = 0.0, h = 0.0, alias = 0.0;
                const bool have = grid_choice(P.eps, P.k, dl, M_PI / 1.5, grid_cost, w, beta, p, h, alias);
                const double direct = (LV.pts_src + LV.pts_tgt) * (double)LV.nq * 9e-14;
                const double gridc = have ? grid_cost(p, w) : 1e300;
                const size_t gnb = (size_t)std::max(nbx, nby);
                const size_t gbytes = gnb * ((size_t)p * p * p + (size_t)(L + 1) * p * p) * sizeof(float2);
                const bool force_grid = (P.opt.flags & FFM_FLAG_GRID_TRANSFORMS) != 0;
                const bool force_direct = (P.opt.flags & FFM_FLAG_DIRECT_TRANSFORMS) != 0;
                LV.grid = have && !force_direct && L >= 8 && gbytes <= ((size_t)24 << 30) &&
                          (force_grid || gridc < direct);
                if (LV.grid) {
                    P.any_grid = true;
                    LV.gw = w;
                    LV.gp = p;
                    LV.gh = h;
                    LV.gbeta = beta;
                    LV.galias = alias;
                    const int64_t nxy = (int64_t)LV.nrp * p * L;
                    LV.Ez.alloc((size_t)LV.nrp * p);
                    LV.Ex.alloc((size_t)nxy);
                    LV.Ey.alloc((size_t)nxy);
                    LV.ExT.alloc((size_t)nxy);
                    LV.EyT.alloc((size_t)nxy);
                    FFM_LAUNCH(k_grid_tables, nblocks(std::max<int64_t>(nxy, (int64_t)LV.nrp * p)), kThreads, 0, st,
                               LV.nrp, L, p, h, LV.rings.p, LV.phis.p, LV.Ez.p, LV.Ex.p, LV.Ey.p, LV.ExT.p, LV.EyT.p);
                    // source points ordered by box and z-plane
                    const int64_t ncell = (int64_t)nby * p;
                    int32_t *cnt = SC.get<int32_t>(ncell + 1), *cell_of = SC.get<int32_t>(std::max<int64_t>(TY.n, 1));
                    float4 *gtmp = SC.get<float4>(std::max<int64_t>(TY.n, 1));
                    FFM_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (ncell + 1), st));
                    FFM_LAUNCH(k_grid_zcount, nblocks(TY.n), kThreads, 0, st, TY.n, TY.lev[l].start.p, nby, TY.xs.p,
                               TY.ys.p, TY.zs.p, TY.lev[l].ctr.p, 1.0 / h, p, (w & 1) ? 0.5f : 0.f, cnt, cell_of, gtmp);
                    LV.gzs.alloc((size_t)ncell + 1);
                    exclusive_scan_i32(cnt, LV.gzs.p, ncell, st, SC);
                    int32_t *cursor = SC.get<int32_t>(ncell + 1);
                    FFM_LAUNCH(k_copy_i32, nblocks(ncell + 1), kThreads, 0, st, LV.gzs.p, cursor, ncell + 1);
                    LV.gperm.alloc((size_t)std::max<int64_t>(TY.n, 1));
                    LV.gxyz.alloc((size_t)std::max<int64_t>(TY.n, 1));
                    FFM_LAUNCH(k_grid_zscatter, nblocks(TY.n), kThreads, 0, st, TY.n, p, cell_of, cursor, LV.gperm.p, gtmp,
                               LV.gxyz.p);
                    const std::vector<double> &tab = phi_hat_table(w, LV.gbeta, dphat_step);
                    dphat = keep(SC, tab, st);
                    nphat = (int)tab.size();
                    // boxes go through the grid stages in batches whose G and H fit kGridBatchBytes
                    const size_t per_box = ((size_t)p * p * p + (size_t)(L + 1) * p * p) * sizeof(float2);
                    LV.gcap = (int32_t)std::max<size_t>(1, std::min<size_t>(gnb, grid_batch_bytes() / per_box));
                    ws_gG = std::max(ws_gG, (size_t)LV.gcap * p * p * p);
                    ws_gH = std::max(ws_gH, (size_t)LV.gcap * (L + 1) * p * p);
                }
            }
            plog.mark("tab.grid");
            // per-class series coefficients (host FP64), unit directions r0/|r0|
            std::vector<double> rhat(3 * (size_t)LV.ncls);
            std::vector<double2> coef((size_t)LV.ncls * (L + 1));
            // the series coefficients depend on |r0| only: one Hankel recurrence per distinct norm
            std::vector<std::complex<double>> h;
            std::vector<std::pair<double, int>> seen;   // (|r0|, first class with that norm)
            for (int c = 0; c < LV.ncls; ++c) {
                const double rn = std::sqrt(r0[3 * c] * r0[3 * c] + r0[3 * c + 1] * r0[3 * c + 1] + r0[3 * c + 2] * r0[3 * c + 2]);
                for (int d = 0; d < 3; ++d) rhat[3 * c + d] = r0[3 * c + d] / rn;
                int same = -1;
                for (const auto &sn : seen)
                    if (sn.first == rn) same = sn.second;
                if (same >= 0) {
                    std::copy(coef.begin() + (size_t)same * (L + 1), coef.begin() + (size_t)(same + 1) * (L + 1),
                              coef.begin() + (size_t)c * (L + 1));
                    continue;
                }
                seen.emplace_back(rn, c);
                hankel_host(L, P.k * rn, h);
                std::complex<double> ip(1, 0);
                for (int p = 0; p <= L; ++p) {
                    std::complex<double> v = (2.0 * p + 1.0) * ip * h[p] / (4.0 * M_PI);
                    coef[(size_t)c * (L + 1) + p] = make_double2(v.real(), v.imag());
                    ip *= std::complex<double>(0, 1);
                }
            }
            plog.mark("tab.host");
            // classes evaluated: one of each pair of opposite translations (the other is written alongside)
            std::vector<int32_t> reps;
            {
                std::map<std::tuple<int, int, int>, int> by_off;
                for (int c = 0; c < LV.ncls; ++c)
                    by_off[std::make_tuple(LV.cls_off[3 * c], LV.cls_off[3 * c + 1], LV.cls_off[3 * c + 2])] = c;
                std::vector<char> done(LV.ncls, 0);
                for (int c = 0; c < LV.ncls; ++c) {
                    if (done[c]) continue;
                    int cm = -1;
                    bool opposite = true;   // r0(cm) = -r0(c) exactly
                    auto it = by_off.find(std::make_tuple(-LV.cls_off[3 * c], -LV.cls_off[3 * c + 1], -LV.cls_off[3 * c + 2]));
                    if (it != by_off.end() && it->second != c) {
                        for (int d = 0; d < 3; ++d) opposite = opposite && r0[3 * it->second + d] == -r0[3 * c + d];
                        if (opposite) cm = it->second;
                    }
                    reps.push_back(c);
                    reps.push_back(cm);
                    done[c] = 1;
                    if (cm >= 0) done[cm] = 1;
                }
            }
            const double *drhat = keep(SC, rhat, st);
            const double2 *dcoef = keep(SC, coef, st);
            const int32_t *dreps = keep(SC, reps, st);
            LV.D.alloc((size_t)LV.ncls * LV.npair);
            dim3 grid((unsigned)nblocks(LV.npair), (unsigned)(reps.size() / 2));
            hipLaunchKernelGGL(k_gegen_D, grid, dim3(kThreads), 2 * sizeof(double2) * (L + 1), st, LV.npair, L, ddirs,
                               dwts, drhat, dcoef, dreps, P.k, LV.D.p, dphat, nphat, dphat_step, LV.gh);
            FFM_HIP(hipGetLastError());
            plog.mark("tab.D");
            ws_src = std::max(ws_src, (size_t)nby * LV.npair);
            ws_tgt = std::max(ws_tgt, (size_t)nbx * LV.npair);
        } else {
            LV.method = kLagrange;
            LV.r1 = lagrange_r1(P.kernel, P.k, dl, P.eps, P.opt.r1_override);
            FFM_CHECK(LV.r1 <= 8, FFM_EINVAL, "ffm_plan: eps too small for the Lagrange levels (r1 > 8)");
            LV.r = LV.r1 * LV.r1 * LV.r1;
            LV.rp = (LV.r + 31) / 32 * 32;
            std::vector<double> nodes(LV.r1);
            for (int a = 1; a <= LV.r1; ++a) nodes[a - 1] = std::cos((2.0 * a - 1.0) * M_PI / (2.0 * LV.r1));
            std::vector<float> nf(LV.r1), df(LV.r1);
            for (int a = 0; a < LV.r1; ++a) {
                double den = 1.0;
                for (int b = 0; b < LV.r1; ++b)
                    if (b != a) den *= nodes[a] - nodes[b];
                nf[a] = (float)nodes[a];
                df[a] = (float)(1.0 / den);
            }
            upload(LV.lnodes, nf, st, SC);
            upload(LV.lden, df, st, SC);
            DevBuf<double> dnodes, dr0;
            upload(dnodes, nodes, st, SC);
            upload(dr0, r0, st, SC);
            const int helm = P.kernel == FFM_HELMHOLTZ ? 1 : 0;
            const int64_t per = (int64_t)LV.rp * LV.rp;
            // mixed precision: FP16 transfers where the FP16 rounding (2^-11 relative, twice that for the
            // oscillatory complex kernel) stays within eps; |T| <= 1 / (4 pi d_l) is scaled to <= 1
            const double cond = helm ? 2.0 : 1.0;
            // (the double layer's anterpolated u~ carries the factor 2 / d_l of the derivative, beyond the
            // range the FP16 scaling of the sources provides for: its transfers stay FP32)
            LV.fp16 = P.opt.precision == FFM_PREC_MIXED && !P.dl && std::ldexp(1.0, -11) * cond <= P.eps;
            // class groups of 16 pairs for the MFMA transfer
            DevBuf<int32_t> cnt(LV.ncls), cursor(LV.ncls);
            FFM_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * LV.ncls, st));
            FFM_LAUNCH(k_count_cls, nblocks(LV.nfar), kThreads, 0, st, LV.far_cls.p, LV.nfar, cnt.p);
            std::vector<int32_t> hc(LV.ncls), gstart(LV.ncls), gcls;
            FFM_HIP(hipMemcpyAsync(hc.data(), cnt.p, sizeof(int32_t) * LV.ncls, hipMemcpyDeviceToHost, st));
            FFM_HIP(hipStreamSynchronize(st));
            int32_t g = 0;
            for (int c = 0; c < LV.ncls; ++c) {
                gstart[c] = g;
                const int ng = (hc[c] + 15) / 16;
                for (int q = 0; q < ng; ++q) gcls.push_back(c);
                g += ng;
            }
            LV.ngrp = g;
            // ACA of the transfer matrices (eq. ffmACAmatvec, relative tolerance eps / 4) where it saves MFMA work:
            // each class's rank padded to whole 32-row tiles, at most one tile per wave of the transfer block; a
            // pair then costs 2 rp kp instead of rp^2 multiply-adds.  Not at FP16 levels (FP16 runs 16x the FP32
            // rate on full matrices) nor below r1 = 5 (r = 64: one 32-row tile already costs as much as T).
            LV.aca = false;
            const int nwv = std::min(4, LV.rp / 32);
            const bool force_aca = (P.opt.flags & FFM_FLAG_ACA) != 0;
            if (!LV.fp16 && !(P.opt.flags & FFM_FLAG_NO_ACA) && (LV.r1 >= 5 || force_aca)) {
                const double tol = P.eps / 4.0;
                std::vector<std::vector<cd>> Af(LV.ncls), Bf(LV.ncls);
                std::vector<int> rank(LV.ncls, 0);
                std::atomic<int> next{0};
                auto worker = [&] {
                    for (int c = next++; c < LV.ncls; c = next++)
                        rank[c] = aca_class(&r0[3 * (size_t)c], nodes.data(), dl, LV.r1, helm, P.k, tol, Af[c], Bf[c]);
                };
                const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
                std::vector<std::thread> pool;
                for (int t = 1; t < nth; ++t) pool.emplace_back(worker);
                worker();
                for (auto &t : pool) t.join();
                int kpm = 32;
                double cost_t = 0.0, cost_a = 0.0, rank_sum = 0.0;
                std::vector<int32_t> kp(LV.ncls);
                for (int c = 0; c < LV.ncls; ++c) {
                    kp[c] = std::max(32, (rank[c] + 31) / 32 * 32);
                    kpm = std::max(kpm, kp[c]);
                    const double ng = (hc[c] + 15) / 16;
                    cost_t += ng * (double)per;
                    cost_a += ng * 2.0 * LV.rp * kp[c];
                    rank_sum += rank[c];
                }
                LV.aca = kpm <= 32 * nwv && (force_aca || cost_a <= 0.75 * cost_t);
                LV.aca_rank = LV.ncls ? rank_sum / LV.ncls : 0.0;
                if (LV.aca) {
                    LV.kpm = kpm;
                    LV.aca_ranks.assign(rank.begin(), rank.end());
                    const int planes = helm ? 2 : 1;
                    std::vector<float> ha((size_t)LV.ncls * planes * kpm * LV.rp, 0.f);
                    std::vector<float> hb((size_t)LV.ncls * planes * LV.rp * kpm, 0.f);
                    const int r = LV.r;
                    for (int c = 0; c < LV.ncls; ++c)
                        for (int q = 0; q < rank[c]; ++q)
                            for (int i = 0; i < r; ++i) {
                                const cd a = Af[c][(size_t)q * r + i], b = Bf[c][(size_t)q * r + i];
                                // A: element (i, q) at [c][plane][q][i]; B^T: element (q, j = i) at [c][plane][j][q]
                                ha[(((size_t)c * planes) * kpm + q) * LV.rp + i] = (float)a.real();
                                hb[(((size_t)c * planes) * LV.rp + i) * kpm + q] = (float)b.real();
                                if (helm) {
                                    ha[(((size_t)c * planes + 1) * kpm + q) * LV.rp + i] = (float)a.imag();
                                    hb[(((size_t)c * planes + 1) * LV.rp + i) * kpm + q] = (float)b.imag();
                                }
                            }
                    upload(LV.acaA, ha, st, SC);
                    upload(LV.acaB, hb, st, SC);
                    upload(LV.acaKp, kp, st, SC);
                }
            }
            if (!LV.aca) {
                LV.T.alloc((size_t)per * LV.ncls * (helm ? 2 : 1));
                FFM_LAUNCH(k_lagrange_T, nblocks(per * LV.ncls), kThreads, 0, st, LV.ncls, dr0.p, LV.r1, LV.rp, dnodes.p,
                           0.5 * dl, helm, P.k, LV.T.p);
            }
            if (LV.fp16) {
                LV.sT = (float)std::ldexp(1.0, (int)std::floor(std::log2(4.0 * M_PI * dl)));
                const int64_t planes = (int64_t)LV.ncls * (helm ? 2 : 1);
                LV.T16.alloc((size_t)per * planes);
                FFM_LAUNCH(k_to_half, nblocks(per * planes), kThreads, 0, st, LV.T.p, planes, LV.rp, LV.sT,
                           LV.T16.p);
                P.any_fp16 = true;
            }
            DevBuf<int32_t> dgs;
            upload(dgs, gstart, st, SC);
            upload(LV.grp_cls, gcls, st, SC);
            LV.grp_pair.alloc((size_t)16 * std::max(g, 1));
            FFM_HIP(hipMemsetAsync(LV.grp_pair.p, 0xff, sizeof(int32_t) * 16 * std::max(g, 1), st));
            FFM_HIP(hipMemsetAsync(cursor.p, 0, sizeof(int32_t) * LV.ncls, st));
            FFM_LAUNCH(k_fill_groups, nblocks(LV.nfar), kThreads, 0, st, LV.far_cls.p, LV.nfar, dgs.p, cursor.p,
                       LV.grp_pair.p);
            FFM_HIP(hipStreamSynchronize(st));
            ws_src = std::max(ws_src, ((size_t)nby * LV.rp + 1) / 2);
            ws_z = std::max(ws_z, (size_t)LV.nfar * LV.rp);
        }
    }
    plog.mark("tables");
    build_work_lists(P, P.lev[P.leaf], true, wf_near);
    P.nsym = wf_near.sym_tot ? wf_near.sym_tot[0] : 0;
    if (!wf_near.sym_tot) P.near_sym = false;
    P.wnsym.alloc((size_t)std::max<int64_t>(P.nsym, 0) * P.ncomp());
    for (int l = 1; l < P.leaf; ++l)
        if (P.lev[l].nearly) build_early_lists(P.lev[l], wf_early[l]);
    (void)ws_part;
    P.ws_src = ws_src;
    P.ws_tgt = ws_tgt;
    P.ws_z = ws_z;
    P.u_sorted.alloc(ny);
    P.v_sorted.alloc(nx * P.ncomp());
    P.wsrc.alloc(ws_src);
    P.wtgt.alloc(ws_tgt);
    // the normal derivative at the targets splits, like the gradient, the levels whose target transform takes the
    // grid or the ring-pair form (k s . n = sum_c k s_c n_c: three plain target transforms, combined with n)
    P.dnsplit = false;
    if (P.dn)
        for (int l = 1; l <= P.leaf; ++l)
            if (P.lev[l].method == kGegenbauer && (P.lev[l].grid || P.lev[l].L >= kRingMinL)) P.dnsplit = true;
    if (P.grad || P.dnsplit) P.wtgtx.alloc(2 * ws_tgt);
    if (P.dnsplit) P.wtmp.alloc(3 * nx);
    // the double layer splits the levels whose source transform takes the grid or the ring-pair form: three plain
    // source transforms of the densities u n_c, combined with -ik s_c
    P.dlsplit = false;
    if (P.dl)
        for (int l = 1; l <= P.leaf; ++l)
            if (P.lev[l].method == kGegenbauer && (P.lev[l].grid || P.lev[l].L >= kRingMinL)) P.dlsplit = true;
    if (P.dlsplit) {
        P.wucomp.alloc(3 * ny);
        P.wsrcx.alloc(2 * ws_src);
    }
    P.wz.alloc(ws_z);
    P.wG.alloc(ws_gG);
    P.wH.alloc(ws_gH);
    if (P.any_fp16 || P.any_grid) P.amax.alloc(1);
    plog.mark("alloc");
    // launches and descriptors
    P.dio.alloc(1);
    P.hio = static_cast<IoEntry *>(pinned_alloc(sizeof(IoEntry)));
    std::memset(P.hio, 0, sizeof(IoEntry));
    // the last tables and the launch lists are left to run on the planning stream: their temporaries go to
    // P.pending, and applies wait for P.ready (recorded by the caller after this returns)
    P.pending = std::make_unique<Scratch>(st);
    plan_set_tune(P, P.tune, st, P.pending.get());
    plog.mark("stages");

    // --- statistics
    ffm_stats_t &s = P.stats;
    const double near_pairs = s.near_pairs;
    std::memset(&s, 0, sizeof(s));
    s.near_pairs = near_pairs;
    for (int l = 1; l < P.leaf; ++l) s.near_pairs += P.lev[l].early_pairs;
    s.leaf = P.leaf;
    s.same_set = P.same ? 1 : 0;
    s.d0 = d0;
    for (int d = 0; d < 3; ++d) {
        s.corner_x[d] = corner[0][d];
        s.corner_y[d] = corner[1][d];
    }
    for (int l = 0; l <= P.leaf; ++l) {
        s.nbox_x[l] = TX.lev[l].nbox;
        s.nbox_y[l] = TY.lev[l].nbox;
        const Level &LV = P.lev[l];
        s.nfar[l] = LV.nfar;
        s.nnear[l] = LV.nnear;
        s.method[l] = LV.method;
        s.order[l] = LV.method == kGegenbauer ? LV.L : LV.r1;
        s.nclass[l] = LV.ncls;
        s.nq[l] = LV.nq;
        s.fwd_points[l] = LV.pts_src;
        s.tform[l] = LV.method == kGegenbauer ? (LV.grid ? 3 : (LV.qG ? 2 : 1)) : 0;
        s.prec[l] = LV.fp16 ? 1 : 0;
        s.phase64[l] = LV.method == kGegenbauer && LV.phase64 ? 1 : 0;
        s.bwd_points[l] = LV.pts_tgt;
        s.grid_nodes[l] = LV.method == kGegenbauer && LV.grid ? LV.gp : 0;
        s.grid_width[l] = LV.method == kGegenbauer && LV.grid ? LV.gw : 0;
        s.grid_beta[l] = LV.method == kGegenbauer && LV.grid ? LV.gbeta : 0.0;
        s.aca[l] = LV.method == kLagrange && LV.aca ? 1 : 0;
        s.nearly[l] = LV.nearly;
        s.aca_rank[l] = LV.method == kLagrange ? LV.aca_rank : 0.0;
        s.grid_alias[l] = LV.method == kGegenbauer && LV.grid ? LV.galias : 0.0;
        s.fwd_boxes[l] = (int64_t)LV.h_fwd.size();
        s.bwd_boxes[l] = (int64_t)LV.h_tgt.size();
        if (LV.method == kGegenbauer) {
            s.transform_terms += (LV.pts_src + LV.pts_tgt) * (double)LV.nq;
            s.transfer_macs += (double)LV.nfar * (double)LV.nq;
        } else if (LV.method == kLagrange) {
            s.transfer_macs += (double)LV.nfar * (double)LV.r * (double)LV.r;
        }
    }
    (void)ws_tgt;
    P.pending->adopt(SC);
}

void plan_sync_ready(Plan &P) {
    if (!P.pending) return;
    if (P.ready) FFM_HIP(hipEventSynchronize(P.ready));
    else FFM_HIP(hipStreamSynchronize(P.pending->stream));
    P.pending->release();
    P.pending.reset();
}

// ---------------------------------------------------------------------------- launches
namespace {
Stage make_stage(int kern, int a, int b, int slot, int level, size_t shmem, std::vector<int4> &&items, hipStream_t st,
                 Scratch &SC) {
    Stage S;
    S.kern = kern;
    S.a = a;
    S.b = b;
    S.slot = slot;
    S.level = level;
    S.shmem = shmem;
    S.items = std::move(items);
    (void)st;
    (void)SC;
    return S;
}
}  // namespace

void upload_stage_items(const std::vector<Stage *> &stages, DevBuf<int4> &arena, hipStream_t st, Scratch &SC) {
    size_t total = 0;
    for (const Stage *S : stages) total += S->items.size();
    arena.alloc(total);
    if (total == 0) {
        for (Stage *S : stages) {
            S->ditems = nullptr;
            S->nitems = 0;
        }
        return;
    }
    int4 *h = SC.pin<int4>(total);
    size_t off = 0;
    for (Stage *S : stages) {
        if (!S->items.empty()) std::memcpy(h + off, S->items.data(), S->items.size() * sizeof(int4));
        S->ditems = arena.p + off;
        S->nitems = S->items.size();
        off += S->items.size();
    }
    FFM_HIP(hipMemcpyAsync(arena.p, h, total * sizeof(int4), hipMemcpyHostToDevice, st));
}

// Transfer work items, tile-major (the blocks running together share a tile of the class tables D): with the
// class tables staged in LDS (levels with many direction pairs), groups of 256 / qt consecutive target slots
// (targets with far work in Morton order) and tiles of qt pairs; otherwise one target box and a tile of
// bs ppt pairs per block.  Within a tile the groups (or targets, in Morton order) are cut into 8 contiguous
// ranges interleaved so that block b takes range b mod 8: workgroups are dealt to the 8 XCDs of the chip in
// turn, so each XCD works through one contiguous region, and neighbouring targets, which share most of their
// far sources, find u~ in that XCD's L2.
// Distinct box ids in increasing (Morton) order: flags over the id range instead of a comparison sort.
static std::vector<int32_t> morton_order(const std::vector<int32_t> &boxes) {
    int32_t hi = 0;
    for (int32_t t : boxes) hi = std::max(hi, t + 1);
    std::vector<char> on((size_t)hi, 0);
    for (int32_t t : boxes) on[(size_t)t] = 1;
    std::vector<int32_t> out;
    out.reserve(boxes.size());
    for (int32_t t = 0; t < hi; ++t)
        if (on[(size_t)t]) out.push_back(t);
    return out;
}

// tg: the targets with far work in Morton order
static std::vector<int4> transfer_items(int l, const std::vector<int32_t> &tg, int64_t npair, bool lds, int qt,
                                        int tile) {
    const int64_t n = lds ? ((int64_t)tg.size() + kThreads / qt - 1) / (kThreads / qt) : (int64_t)tg.size();
    const int64_t ntiles = (npair + tile - 1) / tile;
    constexpr int kXcd = 8;
    const int64_t per = (n + kXcd - 1) / kXcd;
    std::vector<int4> it;
    it.reserve((size_t)(n * ntiles));
    for (int64_t q = 0; q < ntiles; ++q)
        for (int64_t k = 0; k < per; ++k)
            for (int x = 0; x < kXcd; ++x) {
                const int64_t g = x * per + k;
                if (g < n) it.push_back(make_int4(l, lds ? (int)g : tg[(size_t)g], (int)q, 0));
            }
    return it;
}

// Parts s to split `blocks` equal blocks into, given `conc` blocks that run at once: the launch then runs
// in about blocks * s / conc rounds, and blocks of the last, partly filled round run with the chip partly
// idle.  Take the smallest s (up to smax, at most `cap`) that gives at least 8 rounds or a last round at
// least 90% full.
static int choose_split(int64_t blocks, int conc, int smax, int cap) {
    smax = std::max(1, std::min(smax, cap));
    for (int s = 1; s <= smax; ++s) {
        const double r = (double)blocks * s / conc;
        const double frac = r - std::floor(r);
        if (r >= 8.0 || frac == 0.0 || frac >= 0.9) return s;
    }
    return smax;
}

// Block size and pairs per thread of a direction-pair kernel over npair pairs: the variant among
// (64 threads, 1), (256, 1), (256, 2), (256, 4) (PPT at most ppt_max) whose tiles waste the fewest idle
// threads, the larger tile among near-equal ones.
static void pick_pair_tile(int64_t npair, int ppt_max, int &bs, int &ppt) {
    const int cand[4][2] = {{64, 1}, {256, 1}, {256, 2}, {256, 4}};
    double best = 1e30;
    bs = 256;
    ppt = 1;
    for (const auto &c : cand) {
        if (c[1] > ppt_max) continue;
        const int64_t T = (int64_t)c[0] * c[1];
        const double waste = (double)((npair + T - 1) / T * T) / (double)std::max<int64_t>(npair, 1);
        if (waste <= best * 1.05) {
            if (waste < best) best = waste;
            bs = c[0];
            ppt = c[1];
        }
    }
}

// The transfer stage of a Gegenbauer level: class tables in LDS where boxes have many direction pairs
// (measured faster from n_pair ~ 4096 on), one target per block otherwise.
// Gradient plans: v~ of the three components of a Gegenbauer level (k_dir_scale), over the level's target boxes.
static Stage dir_scale_stage(int l, const Level &LV, hipStream_t st, Scratch &SC) {
    std::vector<int4> it;
    const int nt = (int)((LV.npair + kThreads - 1) / kThreads);
    for (int32_t t : LV.h_tgt)
        for (int q = 0; q < nt; ++q) it.push_back(make_int4(l, t, q, 0));
    return make_stage(K_DIRSCALE, 0, 0, -1, l, 0, std::move(it), st, SC);
}

static Stage transfer_stage(const Plan &P, int l, Level &LV, const std::vector<int32_t> &tg, int slot,
                            hipStream_t st, Scratch &SC) {
    if (LV.npair >= 4096) {
        const int qt = transfer_qt(LV.ncls);
        return make_stage(K_TRANSFER, 1000 + qt, 0, slot, l, sizeof(float4) * LV.ncls * qt,
                          transfer_items(l, tg, LV.npair, true, qt, qt), st, SC);
    }
    int bs, ppt;
    pick_pair_tile(LV.npair, 2, bs, ppt);
    // 64-pair tiles: four consecutive targets per block (measured faster over a whole product than one target
    // per block, mostly through the plan's four times fewer work items)
    if (bs == 64 && P.same && LV.h_par.size() > 0) {
        // sibling groups: the targets of one parent share most far sources, so each source's u~ tile is read
        // once for up to four of them (3.5 to 3.8 times fewer reads at the levels of a 1M-point sphere)
        std::vector<int32_t> gt;
        for (size_t i = 0; i < tg.size();) {
            const int32_t par = LV.h_par[(size_t)tg[i]];
            size_t j = i;
            while (j < tg.size() && j - i < 4 && LV.h_par[(size_t)tg[j]] == par) gt.push_back(tg[j++]);
            while (gt.size() % 4) gt.push_back(-1);
            i = j;
        }
        LV.nsibg = (int32_t)(gt.size() / 4);
        upload(LV.sib_tgt, gt, st, SC);
        LV.sib_src.alloc((size_t)LV.nsibg * 216);
        LV.sib_cls.alloc((size_t)LV.nsibg * 216);
        LV.sib_cnt.alloc((size_t)LV.nsibg);
        const TreeLevel &TL = P.tx->lev[l], &TU = P.tx->lev[l - 1];
        FFM_LAUNCH(k_sib_fill, LV.nsibg, 64, 0, st, LV.sib_tgt.p, LV.far_ptr.p, LV.far_src.p, LV.far_cls.p,
                   TL.parent.p, TL.ijk.p, TU.ijk.p, LV.sib_src.p, LV.sib_cls.p, LV.sib_cnt.p);
        std::vector<int32_t> slots((size_t)LV.nsibg);     // only its size counts (four groups per block)
        return make_stage(K_TRANSFER, 301, 0, slot, l, 0, transfer_items(l, slots, LV.npair, true, 64, 64), st, SC);
    }
    if (bs == 64)
        return make_stage(K_TRANSFER, 201, 0, slot, l, 0, transfer_items(l, tg, LV.npair, true, 64, 64), st, SC);
    return make_stage(K_TRANSFER, ppt, 0, slot, l, 0, transfer_items(l, tg, LV.npair, false, 1, bs * ppt), st, SC);
}


// Choose the kernel form of every level for a tile choice and build its launches (work items).
void plan_stages(Plan &P, const Tune &tu, hipStream_t st, Scratch *keep) {
    PhaseLog plog("ffm_plan stages ms:");
    Scratch SC(st);
    P.pre.clear();
    P.post.clear();
    if (P.empty) return;
    const int64_t nmax = std::max(P.nx, P.ny);
    {
        std::vector<int4> it;
        for (int64_t i = 0; i < nmax; i += kThreads) it.push_back(make_int4(0, (int)i, 0, 0));
        P.pre.push_back(make_stage(K_PERM_IN, 0, 0, -1, 0, 0, std::move(it), st, SC));
        if (P.any_fp16 || P.any_grid) {
            std::vector<int4> z(1, make_int4(0, 0, 0, 0)), am;
            for (int64_t i = 0; i < P.ny; i += 16 * kThreads) am.push_back(make_int4(0, (int)i, 0, 0));
            P.pre.push_back(make_stage(K_AMAX, 1, 0, -1, 0, 0, std::move(z), st, SC));
            P.pre.push_back(make_stage(K_AMAX, 0, 0, -1, 0, 0, std::move(am), st, SC));
        }
    }
    size_t ws_part = 0, ws_bpart = 0;
    // concurrent blocks of the ring-pair kernels on this device: [G == 4 / PT == 2][FP64 phase]
    const int cus = device_cus();
    int conc_fwd[2][2], conc_bwd[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            conc_fwd[i][j] = cus * stage_blocks_per_cu(K_FWD_RING, i ? 4 : 2, j);
            conc_bwd[i][j] = cus * stage_blocks_per_cu(K_BWD_RING, i ? 2 : 1, j);
        }
    for (int l = 1; l <= P.leaf; ++l) {
        plog.mark("l");
        Level &LV = P.lev[l];
        LV.stages.clear();
        if (LV.method == kNone) continue;
        const int s1 = 1 + 3 * (l - 1), s2 = s1 + 1, s3 = s1 + 2;
        const std::vector<int32_t> &sx = LV.h_sx;
        // transfer slots: the targets with far work in Morton order
        std::vector<int32_t> tg;
        if (LV.method == kGegenbauer) {
            tg = morton_order(LV.h_tgt);
            upload(LV.tr_tgt, tg, st, SC);
        }
        if (LV.method == kGegenbauer && LV.grid) {
            // grid form: spread (per z-plane and 64 x 64 tile), sums over z (64 grid columns and up to 64
            // ring pairs per block), sums over the plane to the directions (one ring per block); the transfer;
            // the mirror stages (one ring and 64 x 64 tile, then 64 columns x 64 planes per block)
            const int L = LV.L, p = LV.gp, nta = (p + 63) / 64;
            LV.qG = 0;
            LV.qSplit = 1;
            LV.bSplit = 1;
            const int ncol = (p * p + 63) / 64;
            int zng, zper;
            grid_z_groups(LV.nrp, zng, zper);
            zng = ((LV.nrp + 15) / 16 + zper - 1) / zper;
            std::vector<int4> a1, a2, a3, b1, b2, b3;
            // the plane sums go ring by ring, rings m and L - m (which share their tables) together, so that
            // the blocks running at once read the same few tables
            std::vector<int> ring_order;
            for (int mt = 0; mt < LV.nrp; ++mt) {
                ring_order.push_back(mt);
                if (L - mt != mt) ring_order.push_back(L - mt);
            }
            // boxes in batches of gcap: each batch's grids and ring sums reuse the same slots of G and H, so a batch's
            // stages run after the previous batch's (stage order; in merged batches, by role_add)
            const int cap = std::max(1, LV.gcap);
            const int nbf = (int)((LV.h_fwd.size() + cap - 1) / cap), nbt = (int)((LV.h_tgt.size() + cap - 1) / cap);
            {
                std::vector<int32_t> slot((size_t)P.ty->lev[l].nbox, 0);
                for (size_t i = 0; i < LV.h_fwd.size(); ++i) slot[(size_t)LV.h_fwd[i]] = (int32_t)(i % cap);
                upload(LV.gslot_s, slot, st, SC);
                std::vector<int32_t> tslot((size_t)P.tx->lev[l].nbox, 0);
                for (size_t i = 0; i < LV.h_tgt.size(); ++i) tslot[(size_t)LV.h_tgt[i]] = (int32_t)(i % cap);
                upload(LV.gslot_t, tslot, st, SC);
            }
            for (int bi = 0; bi < nbf; ++bi) {
                const size_t i0 = (size_t)bi * cap, i1 = std::min(LV.h_fwd.size(), i0 + cap);
                for (size_t i = i0; i < i1; ++i) {
                    const int32_t b = LV.h_fwd[i];
                    for (int c = 0; c < p; ++c)
                        for (int t = 0; t < nta * nta; ++t) a1.push_back(make_int4(l, b, c, t));
                    for (int t = 0; t < ncol; ++t)
                        for (int g = 0; g < zng; ++g) a2.push_back(make_int4(l, b, t, g));
                }
                for (int m : ring_order)
                    for (size_t i = i0; i < i1; ++i) a3.push_back(make_int4(l, LV.h_fwd[i], m, 0));
                Stage S1 = make_stage(K_GSPREAD, LV.gw, 0, -1, l, 2 * sizeof(uint64_t) * std::min(p, 64) * std::min(p, 64),
                                      std::move(a1), st, SC);
                Stage S2 = make_stage(K_GZ, 0, 0, -1, l, 0, std::move(a2), st, SC);
                Stage S3 = make_stage(K_GPHI, p <= 128 ? p / 16 : 0, 0, bi + 1 == nbf ? s1 : -1, l, 0, std::move(a3), st, SC);
                S1.role_add = S2.role_add = S3.role_add = 16 * bi;
                LV.stages.push_back(std::move(S1));
                LV.stages.push_back(std::move(S2));
                LV.stages.push_back(std::move(S3));
                a1.clear();
                a2.clear();
                a3.clear();
            }
            {
                Stage S = transfer_stage(P, l, LV, tg, s2, st, SC);
                S.role_add = 16 * (nbf - 1);
                LV.stages.push_back(std::move(S));
                if (P.grad || P.dn) {
                    Stage D = dir_scale_stage(l, LV, st, SC);
                    D.role_add = 16 * (nbf - 1);
                    LV.stages.push_back(std::move(D));
                }
            }
            // mirror plane sums: 64 x 64 tiles, or 64 rows by the whole plane for grids of 80, 96 and 112 nodes,
            // whose 64 x 64 tiles would leave slivers (measured 18.3 -> 13.7 ms at 80 nodes; 128 nodes keep full
            // 64 x 64 tiles, 14.6 against 15.1 ms wide)
            const bool phit_wide = p > 64 && p < 128;
            // grids of at most 32 nodes: rings m and L - m in one block (they share their tables)
            const bool phit_pair = p <= 32;
            const int phit_tiles = phit_wide ? nta : nta * nta;
            for (int bi = 0; bi < nbt; ++bi) {
                const size_t i0 = (size_t)bi * cap, i1 = std::min(LV.h_tgt.size(), i0 + cap);
                if (phit_pair) {
                    for (int mt = 0; mt < LV.nrp; ++mt)
                        for (size_t i = i0; i < i1; ++i) b1.push_back(make_int4(l, LV.h_tgt[i], mt, 0));
                } else {
                    for (int m : ring_order)
                        for (size_t i = i0; i < i1; ++i)
                            for (int q = 0; q < phit_tiles; ++q) b1.push_back(make_int4(l, LV.h_tgt[i], m, q));
                }
                for (size_t i = i0; i < i1; ++i) {
                    const int32_t t = LV.h_tgt[i];
                    for (int q = 0; q < ncol; ++q)
                        for (int cc = 0; cc < nta; ++cc) b2.push_back(make_int4(l, t, q, cc));
                    for (int32_t j = sx[t]; j < sx[t + 1]; j += kThreads) b3.push_back(make_int4(l, t, j, 0));
                }
                Stage T1 = make_stage(K_GPHIT, phit_wide ? 1 : (phit_pair ? 2 : 0), 0, -1, l, 0, std::move(b1), st, SC);
                Stage T2 = make_stage(K_GZT, 0, 0, -1, l, 0, std::move(b2), st, SC);
                Stage T3 = make_stage(K_GINTERP, LV.gw, 0, bi + 1 == nbt ? s3 : -1, l, 0, std::move(b3), st, SC);
                T1.role_add = T2.role_add = T3.role_add = 16 * (nbf - 1) + 16 * bi;
                LV.stages.push_back(std::move(T1));
                LV.stages.push_back(std::move(T2));
                LV.stages.push_back(std::move(T3));
                b1.clear();
                b2.clear();
                b3.clear();
            }
        } else if (LV.method == kGegenbauer) {
            const int L = LV.L;
            LV.qG = L >= 64 ? tu.ring_g : (L >= kRingMinL ? 2 : 0);
            if (LV.qG && (L + LV.qG - 1) / LV.qG > kThreads) LV.qG = 4;   // one ring must fit one block
            // the normal derivative at the targets multiplies every direction by its own ik (s . n): the target
            // transform runs in the direction-pair form
            const bool ring_bwd = LV.qG != 0;
            // two target points per thread in blocks of kThreads where the target boxes hold more than a block's
            // worth on average, else (bpt = 102) in blocks of 128 threads, so that a box's points fill one block
            // while each staged azimuth entry still serves two points
            const bool big_tgt = LV.pts_tgt > (double)kThreads * (double)std::max<size_t>(1, LV.h_tgt.size());
            const int bpt = big_tgt ? tu.bwd_pt : (tu.bwd_pt == 2 ? 102 : 1);
            LV.bwd_tile = ring_bwd ? (bpt == 102 ? 256 : kThreads * bpt) : kThreads;
            std::vector<int4> fw;
            // (the double layer splits its ring-pair source transform by axis, like the grid form's)
            if (LV.qG) {
                // ring-pair form; split each box's points into segments when boxes are too few to fill the chip
                LV.Tr = (L + LV.qG - 1) / LV.qG;
                LV.R = std::max(1, std::min({16, kThreads / LV.Tr, LV.nrp}));
                LV.nchunk = (LV.nrp + LV.R - 1) / LV.R;
                const int64_t blocks = (int64_t)LV.h_fwd.size() * LV.nchunk;
                const double avg = LV.pts_src / std::max<double>(1.0, (double)LV.h_fwd.size());
                const int split = choose_split(blocks, conc_fwd[LV.qG == 4][LV.phase64], 16,
                                               (int)std::max(1.0, avg / 256.0));
                LV.qSplit = split;
                if (split > 1) ws_part = std::max(ws_part, (size_t)split * P.ty->lev[l].nbox * LV.npair);
                fw.reserve((size_t)(LV.h_fwd.size() * LV.nchunk * split));
                for (int32_t b : LV.h_fwd)
                    for (int c = 0; c < LV.nchunk; ++c)
                        for (int g = 0; g < split; ++g) fw.push_back(make_int4(l, b, c, g));
                LV.stages.push_back(make_stage(K_FWD_RING, LV.qG, LV.phase64, split > 1 ? -1 : s1, l, 0, std::move(fw), st, SC));
                if (split > 1) {
                    std::vector<int4> sm;
                    for (int32_t b : LV.h_fwd) sm.push_back(make_int4(l, b, 0, 0));
                    LV.stages.push_back(make_stage(K_SUM, 0, 0, s1, l, 0, std::move(sm), st, SC));
                }
            } else {
                LV.qSplit = 1;
                int bs, ppt;
                pick_pair_tile(LV.npair, 4, bs, ppt);
                const int64_t nt = (LV.npair + bs * ppt - 1) / (bs * ppt);
                fw.reserve((size_t)(LV.h_fwd.size() * nt));
                for (int32_t b : LV.h_fwd)
                    for (int64_t t = 0; t < nt; ++t) fw.push_back(make_int4(l, b, (int)t, 0));
                LV.stages.push_back(make_stage(P.dl ? K_FWD_PAIR_DL : K_FWD_PAIR, ppt + (bs == 64 ? 100 : 0),
                                               LV.phase64, s1, l, 0, std::move(fw), st, SC));
            }
            std::vector<int4> bw;
            LV.stages.push_back(transfer_stage(P, l, LV, tg, s2, st, SC));
            if (P.grad || (P.dn && ring_bwd)) LV.stages.push_back(dir_scale_stage(l, LV, st, SC));
            // direction-pair target transform: 64-point blocks where target boxes are small
            const bool small = !ring_bwd && LV.pts_tgt <= 96.0 * (double)std::max<size_t>(1, LV.h_tgt.size());
            if (small) LV.bwd_tile = 64;
            int64_t tiles = 0;
            for (int32_t t : LV.h_tgt) tiles += (sx[t + 1] - sx[t] + LV.bwd_tile - 1) / LV.bwd_tile;
            // ring parts of the target transform: enough blocks for several rounds of the chip
            const int conc_b = bpt == 102 ? cus * stage_blocks_per_cu(K_BWD_RING, 102, LV.phase64)
                                          : conc_bwd[bpt == 2][LV.phase64];
            LV.bSplit = ring_bwd ? choose_split(tiles, conc_b, 8, LV.nrp) : 1;
            if (LV.bSplit > 1) ws_bpart = std::max(ws_bpart, (size_t)LV.bSplit * P.nx);
            bw.reserve((size_t)(tiles * LV.bSplit));
            for (int g = 0; g < LV.bSplit; ++g)
                for (int32_t t : LV.h_tgt)
                    for (int32_t i = sx[t]; i < sx[t + 1]; i += LV.bwd_tile) bw.push_back(make_int4(l, t, i, g));
            if (ring_bwd)
                LV.stages.push_back(make_stage(K_BWD_RING, bpt, LV.phase64, LV.bSplit > 1 ? -1 : s3, l, 0,
                                               std::move(bw), st, SC));
            else
                LV.stages.push_back(make_stage(P.dn ? K_BWD_PAIR_DN : K_BWD_PAIR, small ? 100 : 0, LV.phase64, s3, l, 0,
                                               std::move(bw), st, SC));
            if (LV.bSplit > 1) {
                std::vector<int4> bs;
                for (int32_t t : LV.h_tgt)
                    for (int32_t i = sx[t]; i < sx[t + 1]; i += kThreads) bs.push_back(make_int4(l, t, i, 0));
                LV.stages.push_back(make_stage(K_BSUM, 0, 0, s3, l, 0, std::move(bs), st, SC));
            }
        } else {
            std::vector<int4> an, mf, ip;
            for (int32_t b : LV.h_fwd) an.push_back(make_int4(l, b, 0, 0));
            // class groups are numbered class by class; blocks are dealt to the 8 XCDs in turn, so block b takes
            // group (b mod 8) per + b / 8 and each XCD works through a contiguous range of classes, reading
            // each class's T into its own L2 once
            {
                constexpr int kXcd = 8;
                const int32_t per = (LV.ngrp + kXcd - 1) / kXcd;
                for (int32_t k = 0; k < per; ++k)
                    for (int x = 0; x < kXcd; ++x) {
                        const int32_t g = x * per + k;
                        if (g < LV.ngrp) mf.push_back(make_int4(l, g, 0, 0));
                    }
            }
            for (int32_t t : LV.h_tgt) ip.push_back(make_int4(l, t, 0, 0));
            LV.stages.push_back(make_stage(P.dl ? K_ANTERP_DL : K_ANTERP, 0, 0, s1, l, 0, std::move(an), st, SC));
            if (LV.aca)
                LV.stages.push_back(make_stage(K_ACA, std::min(4, LV.rp / 32), 0, s2, l, (size_t)LV.rp * 32 * 4,
                                               std::move(mf), st, SC));
            else
                LV.stages.push_back(make_stage(LV.fp16 ? K_MFMA16 : K_MFMA32, LV.fp16 ? 1 : std::min(4, LV.rp / 32), 0,
                                               s2, l, (size_t)LV.rp * 32 * (LV.fp16 ? 2 : 4), std::move(mf), st, SC));
            LV.stages.push_back(make_stage(P.dn || P.grad ? K_INTERP_DN : K_INTERP, 0, 0, s3, l, sizeof(float2) * LV.r,
                                           std::move(ip), st, SC));
        }
    }
    plog.mark("lev");
    if (ws_part > P.wpart.n) P.wpart.alloc(ws_part);
    if (ws_bpart > P.wbpart.n) P.wbpart.alloc(ws_bpart);
    {
        const Level &LL = P.lev[P.leaf];
        std::vector<int4> nr, po;
        for (int32_t t : LL.h_near) nr.push_back(make_int4(P.leaf, t, 0, 0));
        for (int64_t i = 0; i < P.nx; i += kThreads) po.push_back(make_int4(0, (int)i, 0, 0));
        // Helmholtz near field (k > 0; k = 0 is the Laplace kernel): phases k r / 2 pi of a level's near pairs
        // stay below 4 sqrt(3) k d_l / 2 pi revolutions (adjacent boxes, either tree); beyond 128 revolutions
        // they are reduced to [0, 1) before the hardware sine and cosine
        const bool nhelm = P.kernel == FFM_HELMHOLTZ && P.k > 0.0;
        auto big = [&](int l) {
            return nhelm && P.k / (2.0 * M_PI) * 4.0 * std::sqrt(3.0) * std::ldexp(P.d0, -l) > 128.0 ? 1 : 0;
        };
        const int near_kern = P.grad ? K_NEAR_GRAD : (P.dn ? K_NEAR_DN : (P.dl ? K_NEAR_DL : K_NEAR));
        // near pairs the per-pair rule stopped above the leaf: the same kernel over each level's early list
        for (int l = 1; l < P.leaf; ++l) {
            if (P.lev[l].h_early.empty()) continue;
            std::vector<int4> er;
            for (int32_t t : P.lev[l].h_early) er.push_back(make_int4(l, t, 0, 0));
            P.post.push_back(make_stage(near_kern, big(l), nhelm, -1, l, 0, std::move(er), st, SC));
        }
        if (P.near_sym) {
            std::vector<int4> ga = nr;
            const int nrm = P.grad ? 3 : (P.dn ? 1 : (P.dl ? 2 : 0));
            P.post.push_back(make_stage(K_NEAR_SYM, big(P.leaf) + 2 * nrm, nhelm, -1, P.leaf, 0, std::move(nr), st, SC));
            P.post.push_back(make_stage(K_NEAR_GATHER, 0, 0, 61, P.leaf, 0, std::move(ga), st, SC));
        } else {
            P.post.push_back(make_stage(near_kern, big(P.leaf), nhelm, 61, P.leaf, 0, std::move(nr), st, SC));
        }
        P.post.push_back(make_stage(K_PERM_OUT, 0, 0, 62, 0, 0, std::move(po), st, SC));
    }
    // gradient plans: each level's target side (from its first target-transform stage on) once more for components
    // 1 and 2, over their own descriptors (items pointing at descriptor k + c (leaf + 1)) and after component 0's
    // (a batch orders them by role: they share the level's target workspace); component 2's copies close the
    // original timing slots.  The near field (k_near_grad) writes all three components in one pass.
    // Split normal derivative: at the levels with a k_dir_scale stage, the target side three times over the axis
    // descriptors (sets 1 to 3, into the axis planes), then k_dn_combine, which closes the original slot.
    constexpr int kRoleComp = 4096;
    auto copy = [&](Stage S, int set, bool keep_slot) {
        for (int4 &x : S.items) x.x += set * (P.leaf + 1);
        S.role_add += set * kRoleComp;
        if (!keep_slot) S.slot = -1;
        return S;
    };
    auto tgt_kind = [](int k) {
        return k == K_BWD_PAIR || k == K_BWD_RING || k == K_GPHIT || k == K_INTERP_DN;
    };
    if (P.grad) {
        for (int l = 1; l <= P.leaf; ++l) {
            std::vector<Stage> &v = P.lev[l].stages;
            size_t k0 = 0;
            while (k0 < v.size() && !tgt_kind(v[k0].kern)) ++k0;
            const std::vector<Stage> tail(v.begin() + (std::ptrdiff_t)k0, v.end());
            v.resize(k0);
            for (int c = 0; c < 3; ++c)
                for (const Stage &S : tail) v.push_back(copy(S, c, c == 2));
        }
    }
    if (P.dlsplit) {
        // split double layer: at the levels whose source side is the grid or the ring-pair form, the source stages
        // (everything before the transfer) three times over the axis descriptors (sets 1 to 3: density u n_c
        // into u~_c), then k_dl_combine into u~; a batch orders the rest of the level after them
        for (int l = 1; l <= P.leaf; ++l) {
            std::vector<Stage> &v = P.lev[l].stages;
            if (P.lev[l].method != kGegenbauer || !(P.lev[l].grid || P.lev[l].qG)) continue;
            size_t k1 = 0;
            while (k1 < v.size() && v[k1].kern != K_TRANSFER) ++k1;
            const std::vector<Stage> head(v.begin(), v.begin() + (std::ptrdiff_t)k1);
            std::vector<Stage> rest(v.begin() + (std::ptrdiff_t)k1, v.end());
            int slot = -1, role = 0;
            for (const Stage &S : head) {
                if (S.slot >= 0) slot = S.slot;
                role = std::max(role, S.role_add);
            }
            v.clear();
            for (int c = 0; c < 3; ++c)
                for (const Stage &S : head) v.push_back(copy(S, 1 + c, false));
            std::vector<int4> it;
            const int nt = (int)((P.lev[l].npair + kThreads - 1) / kThreads);
            for (int32_t b : P.lev[l].h_fwd)
                for (int q = 0; q < nt; ++q) it.push_back(make_int4(l, b, q, 0));
            Stage C = make_stage(K_DLCOMBINE, 0, 0, slot, l, 0, std::move(it), st, SC);
            C.role_add = role + 4 * kRoleComp;
            v.push_back(std::move(C));
            for (Stage &S : rest) {
                S.role_add += 5 * kRoleComp;
                v.push_back(std::move(S));
            }
        }
    }
    if (P.dnsplit) {
        for (int l = 1; l <= P.leaf; ++l) {
            std::vector<Stage> &v = P.lev[l].stages;
            bool split = false;
            for (const Stage &S : v) split = split || S.kern == K_DIRSCALE;
            if (!split) continue;
            size_t k0 = 0;
            while (k0 < v.size() && !tgt_kind(v[k0].kern)) ++k0;
            const std::vector<Stage> tail(v.begin() + (std::ptrdiff_t)k0, v.end());
            int slot = -1, role = 0;
            for (const Stage &S : tail) {
                if (S.slot >= 0) slot = S.slot;
                role = std::max(role, S.role_add);
            }
            v.resize(k0);
            for (int c = 0; c < 3; ++c)
                for (const Stage &S : tail) v.push_back(copy(S, 1 + c, false));
            std::vector<int4> it;
            const std::vector<int32_t> &sx = P.lev[l].h_sx;
            for (int32_t t : P.lev[l].h_tgt)
                for (int32_t i = sx[t]; i < sx[t + 1]; i += kThreads) it.push_back(make_int4(l, t, i, 0));
            Stage C = make_stage(K_DNCOMBINE, 0, 0, slot, l, 0, std::move(it), st, SC);
            C.role_add = role + 4 * kRoleComp;
            v.push_back(std::move(C));
        }
    }
    // timing slot of every stage: a stage that closes no phase belongs to the next one that does
    auto fill = [](std::vector<Stage> &v) {
        int next = -1;
        for (int i = (int)v.size() - 1; i >= 0; --i) {
            if (v[i].slot >= 0) next = v[i].slot;
            v[i].tslot = next;
        }
    };
    fill(P.post);
    for (int l = 1; l <= P.leaf; ++l) fill(P.lev[l].stages);
    plog.mark("levels");
    std::vector<Stage *> all;
    for (Stage &S : P.pre) all.push_back(&S);
    for (int l = 1; l <= P.leaf; ++l)
        for (Stage &S : P.lev[l].stages) all.push_back(&S);
    for (Stage &S : P.post) all.push_back(&S);
    upload_stage_items(all, P.items, st, SC);
    plog.mark("upload");
    if (keep) keep->adopt(SC);
}

// The descriptor of level l of a plan, over the given instance buffers and level workspace.
LDesc make_desc(const Plan &P, int l, int inst, float2 *u, float2 *v, float *amax, const LevelWork &w) {
    LDesc d;
    std::memset(&d, 0, sizeof(d));
    d.inst = inst;
    d.helm = P.kernel == FFM_HELMHOLTZ ? 1 : 0;
    d.perm_x = P.tx->perm.p;
    d.perm_y = P.ty->perm.p;
    d.nx = P.nx;
    d.ny = P.ny;
    d.u = u;
    d.v = v;
    d.amax = amax;
    d.k_rev = (float)(P.k / (2.0 * M_PI));
    d.same = P.same ? 1 : 0;
    const TreeLevel &LX = P.tx->lev[l], &LY = P.ty->lev[l];
    d.txs = P.tx->xs.p;
    d.tys = P.tx->ys.p;
    d.tzs = P.tx->zs.p;
    d.tctr = LX.ctr.p;
    d.tstart = LX.start.p;
    d.sxs = P.ty->xs.p;
    d.sys = P.ty->ys.p;
    d.szs = P.ty->zs.p;
    d.sctr = LY.ctr.p;
    d.sstart = LY.start.p;
    const Level &LV = P.lev[l];
    d.far_ptr = LV.far_ptr.p;
    d.far_src = LV.far_src.p;
    d.far_cls = LV.far_cls.p;
    d.tr_tgt = LV.tr_tgt.p;
    d.ntr = (int)LV.h_tgt.size();
    d.sib_tgt = LV.sib_tgt.p;
    d.sib_src = LV.sib_src.p;
    d.sib_cnt = LV.sib_cnt.p;
    d.sib_cls = LV.sib_cls.p;
    d.nsibg = LV.nsibg;
    d.ncls = LV.ncls;
    // the near field of a level above the leaf sums that level's early pairs (per-pair leaf rule)
    const bool early = l < P.leaf && LV.nearly > 0;
    d.near_ptr = early ? LV.early_ptr.p : LV.near_ptr.p;
    d.near_src = early ? LV.early_src.p : LV.near_src.p;
    d.near_off = l == P.leaf && P.near_sym ? LV.near_off.p : nullptr;
    d.nsym = l == P.leaf && P.near_sym ? w.nsym : nullptr;
    d.nsymn = P.nsym;
    d.dirs = LV.dirs.p;
    d.dirs64 = LV.dirs64.p;
    d.rings = LV.rings.p;
    d.phis = LV.phis.p;
    d.D = LV.D.p;
    d.ut = w.ut;
    d.vt = w.vt;
    d.vtx = w.vtx;
    d.vtstride = (int64_t)P.ws_tgt;
    d.vtmp = w.vtmp;
    d.ucomp = w.ucomp;
    d.utx = w.utx;
    d.utstride = (int64_t)P.ws_src;
    d.part = w.part;
    d.npair = LV.npair;
    d.part_stride = (int64_t)LY.nbox * LV.npair;
    d.L = LV.L;
    d.nrp = LV.nrp;
    d.Tr = LV.Tr;
    d.R = LV.R;
    d.nchunk = LV.nchunk;
    d.nsplit = LV.qSplit;
    d.bsplit = LV.bSplit;
    d.bpart = w.bpart;
    d.T = LV.T.p;
    d.lnodes = LV.lnodes.p;
    d.lden = LV.lden.p;
    d.T16 = LV.T16.p;
    d.tn = P.tnrm.p;
    d.sn = P.snrm.p;
    d.tnc = make_float4(1.f, 0.f, 0.f, 0.f);
    d.ncomp = P.ncomp();
    d.acaA = LV.acaA.p;
    d.acaB = LV.acaB.p;
    d.acaKp = LV.acaKp.p;
    d.kpm = LV.kpm;
    d.grp_pair = LV.grp_pair.p;
    d.grp_cls = LV.grp_cls.p;
    d.ut2 = w.ut2;
    d.Z = w.Z;
    d.two_over_dl = 2.0 / std::ldexp(P.d0, -l);
    d.r1 = LV.r1;
    d.rp = LV.rp;
    d.maxpts = LV.max_src_pts;
    d.sT = LV.sT;
    d.gp = LV.gp;
    d.gw = LV.gw;
    d.gbeta = (float)LV.gbeta;
    d.ginv_h = LV.grid ? 1.0 / LV.gh : 0.0;
    d.gnbox = LV.gcap;
    d.gslot_s = LV.gslot_s.p;
    d.gslot_t = LV.gslot_t.p;
    d.G = w.G;
    d.H = w.H;
    d.Ez = LV.Ez.p;
    d.Ex = LV.Ex.p;
    d.Ey = LV.Ey.p;
    d.ExT = LV.ExT.p;
    d.EyT = LV.EyT.p;
    d.gperm = LV.gperm.p;
    d.gzs = LV.gzs.p;
    d.gxyz = LV.gxyz.p;
    return d;
}

int plan_ndesc(const Plan &P) { return (P.leaf + 1) * (P.grad ? 3 : (P.dnsplit || P.dlsplit ? 4 : 1)); }

LDesc plan_desc(const Plan &P, int k, int inst, float2 *u, float2 *v, float *amax, const LevelWork &w) {
    const int l = k % (P.leaf + 1), set = k / (P.leaf + 1);
    if (!P.grad && set == 0) return make_desc(P, l, inst, u, v, amax, w);
    if (P.dlsplit) {
        // split double layer: set 1 + c is the density u n_c into u~_c
        const int c = set - 1;
        LDesc d = make_desc(P, l, inst, w.ucomp + (int64_t)c * P.ny, v, amax, w);
        d.ucomp = nullptr;
        if (c > 0) {
            d.ut = w.utx + (int64_t)(c - 1) * P.ws_src;
            d.ut2 = reinterpret_cast<float2 *>(d.ut);
        }
        return d;
    }
    // gradient: set c is axis c into output plane c; split normal derivative: set 1 + c is axis c into the
    // combine's plane c
    const int c = P.grad ? set : set - 1;
    LDesc d = make_desc(P, l, inst, u, P.grad ? v + (int64_t)c * P.nx : w.vtmp + (int64_t)c * P.nx, amax, w);
    d.tnc = make_float4(c == 0 ? 1.f : 0.f, c == 1 ? 1.f : 0.f, c == 2 ? 1.f : 0.f, 0.f);
    if (c > 0 && w.vtx) d.vt = w.vtx + (int64_t)(c - 1) * P.ws_tgt;   // v~ of this axis (Gegenbauer levels)
    return d;
}

void plan_set_tune(Plan &P, const Tune &tu, hipStream_t st, Scratch *keep) {
    plan_stages(P, tu, st, keep);
    P.tune = tu;
    if (P.empty) return;
    LevelWork w;
    w.ut = P.wsrc.p;
    w.vt = P.wtgt.p;
    w.part = P.wpart.p;
    w.ut2 = reinterpret_cast<float2 *>(P.wsrc.p);
    w.Z = P.wz.p;
    w.bpart = P.wbpart.p;
    w.G = P.wG.p;
    w.H = P.wH.p;
    w.nsym = P.wnsym.p;
    w.vtx = P.wtgtx.p;
    w.vtmp = P.wtmp.p;
    w.ucomp = P.wucomp.p;
    w.utx = P.wsrcx.p;
    P.hdesc.clear();
    for (int k = 0; k < plan_ndesc(P); ++k) P.hdesc.push_back(plan_desc(P, k, 0, P.u_sorted.p, P.v_sorted.p, P.amax.p, w));
    Scratch SC(st);
    upload(P.ddesc, P.hdesc, st, SC);
    if (keep) keep->adopt(SC);
    P.stats.workspace_bytes = (double)apply_work_bytes(P);
    plan_static_setup(P, st);
}

size_t plan_device_bytes(const Plan &P) {
    size_t b = 0;
    auto tree = [&](const Tree &T) {
        b += T.key.bytes() + T.perm.bytes() + T.xs.bytes() + T.ys.bytes() + T.zs.bytes() + T.boxid.bytes();
        for (int l = 0; l <= T.built; ++l) {
            const TreeLevel &L = T.lev[l];
            b += L.start.bytes() + L.ijk.bytes() + L.ctr.bytes() + L.parent.bytes() + L.child.bytes();
        }
    };
    if (P.tx) tree(*P.tx);
    if (P.ty_own) tree(*P.ty_own);
    for (int l = 0; l <= kMaxLev; ++l) {
        const Level &L = P.lev[l];
        b += L.far_ptr.bytes() + L.near_ptr.bytes() + L.far_src.bytes() + L.far_cls.bytes() + L.near_src.bytes() +
             L.T.bytes() + L.grp_pair.bytes() + L.grp_cls.bytes() + L.dirs.bytes() + L.dirs64.bytes() + L.D.bytes() +
             L.lnodes.bytes() + L.lden.bytes() + L.rings.bytes() + L.phis.bytes() + L.T16.bytes() + L.acaA.bytes() +
             L.acaB.bytes() + L.acaKp.bytes() + L.Ez.bytes() +
             L.Ex.bytes() + L.Ey.bytes() + L.ExT.bytes() + L.EyT.bytes() + L.gperm.bytes() + L.gzs.bytes() + L.gxyz.bytes() +
             L.tr_tgt.bytes() + L.gslot_s.bytes() + L.gslot_t.bytes() + L.near_off.bytes() + L.sib_tgt.bytes() + L.sib_src.bytes() + L.sib_cnt.bytes() +
             L.sib_cls.bytes();
    }
    b += P.u_sorted.bytes() + P.v_sorted.bytes() + P.wsrc.bytes() + P.wtgt.bytes() + P.wz.bytes() + P.wpart.bytes() +
         P.wbpart.bytes() + P.wG.bytes() + P.wH.bytes() + P.wnsym.bytes();
    b += P.tnrm.bytes() + P.snrm.bytes() + P.wtgtx.bytes() + P.wtmp.bytes() + P.wucomp.bytes() + P.wsrcx.bytes();
    b += P.ddesc.bytes() + P.dio.bytes();
    b += P.items.bytes();
    return b;
}

}  // namespace ffm
