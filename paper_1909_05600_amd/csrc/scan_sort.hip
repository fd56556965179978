// Device scans and the stable LSD radix sort of Morton keys (plan time).
//
// The sort orders (key, index) pairs by the full 63-bit key with ties kept in
// index order: eight 8-bit passes, each a histogram, a digit-major scan and a
// stable scatter.  Stability inside a tile comes from ranking a wavefront's
// lanes by ballot matching of their digits, round by round in element order,
// so equal keys leave in the order they came in.
#include "common.h"

namespace ffm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__device__ T block_inclusive_sum(T v, T *lds_wave, T &block_total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    if (lane == 63) lds_wave[wave] = v;
    __syncthreads();
    T off = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        T s = lds_wave[w];
        if (w < wave) off += s;
        tot += s;
    }
    __syncthreads();
    block_total = tot;
    return v + off;
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const T *in, int64_t n, T *bsum) {
    __shared__ T lw[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    T tot;
    block_inclusive_sum(s, lw, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// out[i] = boff[block] + exclusive prefix within the tile; the last block writes out[n].
template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const T *in, T *out, int64_t n, const T *boff) {
    __shared__ T lw[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T loc[kScanItems];
    T s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        loc[j] = (i < n) ? in[i] : T(0);
        s += loc[j];
    }
    T tot;
    T incl = block_inclusive_sum(s, lw, tot);
    T run = (boff ? boff[blockIdx.x] : T(0)) + incl - s;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        if (i < n) out[i] = run;
        run += loc[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (boff ? boff[blockIdx.x] : T(0)) + tot;
}

// The same with the block offset summed from the per-block totals by the block itself (a short block
// reduction over bsum[0 .. block - 1]), so that a two-level scan takes two launches.
template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply_sum(const T *in, T *out, int64_t n, const T *bsum) {
    __shared__ T lw[kScanThreads / 64];
    __shared__ T red[kScanThreads / 64];
    T pre = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += kScanThreads) pre += bsum[j];
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pre;
    __syncthreads();
    T boff = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) boff += red[w];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T loc[kScanItems];
    T s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        loc[j] = (i < n) ? in[i] : T(0);
        s += loc[j];
    }
    T tot;
    T incl = block_inclusive_sum(s, lw, tot);
    T run = boff + incl - s;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        if (i < n) out[i] = run;
        run += loc[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = boff + tot;
}

template <class T>
void exclusive_scan(const T *in, T *out, int64_t n, hipStream_t st, Scratch &S) {
    if (n <= 0) {
        FFM_HIP(hipMemsetAsync(out, 0, sizeof(T), st));
        return;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        FFM_LAUNCH(k_scan_apply<T>, 1, kScanThreads, 0, st, in, out, n, (const T *)nullptr);
        return;
    }
    T *bsum = S.get<T>(nb + 1);
    FFM_LAUNCH(k_scan_reduce<T>, nb, kScanThreads, 0, st, in, n, bsum);
    if (nb <= 4096) {
        FFM_LAUNCH(k_scan_apply_sum<T>, nb, kScanThreads, 0, st, in, out, n, (const T *)bsum);
        return;
    }
    T *boff = S.get<T>(nb + 1);
    exclusive_scan<T>(bsum, boff, nb, st, S);
    FFM_LAUNCH(k_scan_apply<T>, nb, kScanThreads, 0, st, in, out, n, (const T *)boff);
}

// ------------------------------------------------------------------ radix sort
// A block takes a tile of 4096 keys.  In the scatter, wave w of the block takes the tile's items
// w 1024 ... w 1024 + 1023, 64 consecutive items per round, so the tile's element order is (wave, round,
// lane).  Every lane loads its 16 items first; the lanes of one round that share a digit find each other by
// ballots over the digit's bits, and the lowest of them adds their number to the wave's count of that digit.
constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRsWaveTile = 64 * kRsItems;

// the lanes of the wave holding a valid item whose digit is d
__device__ __forceinline__ uint64_t rs_peers(int d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

__global__ void __launch_bounds__(kRsThreads)
k_rs_hist(const uint64_t *keys, int64_t n, int shift, int32_t *counts, int nblk) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int j = 0; j < kRsItems; ++j) {
        const int64_t i = base + (int64_t)j * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & 255u)], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: each item's place within its digit's run of the tile is the number of items of
// that digit before it in element order (earlier waves, then earlier rounds of its wave, then lower lanes of its
// round); offs[d nblk + b] is where block b's run of digit d starts.  Items go from registers straight to their
// places: the kernel holds only the per-wave digit counts in LDS, so that its blocks fit beside other work on
// a busy device.
__global__ void __launch_bounds__(kRsThreads)
k_rs_scatter(const uint64_t *kin, const int32_t *vin, uint64_t *kout, int32_t *vout, int64_t n, int shift,
             const int32_t *offs, int nblk) {
    __shared__ int wcnt[kRsWaves][256];     // the wave's count of each digit, then the place of its first item
    __shared__ int gstart[256];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
#pragma unroll
    for (int ww = 0; ww < kRsWaves; ++ww) wcnt[ww][t] = 0;
    gstart[t] = offs[(int64_t)t * nblk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)w * kRsWaveTile + lane;
    uint64_t key[kRsItems];
    int32_t val[kRsItems];
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t i = base + r * 64;
        key[r] = i < n ? kin[i] : 0ull;
        val[r] = i < n ? vin[i] : 0;
    }
    __syncthreads();
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int pos[kRsItems];                       // digit << 16 | place among the wave's items of that digit; -1: none
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const bool valid = base + r * 64 < n;
        const int d = (int)((key[r] >> shift) & 255u);
        const uint64_t m = rs_peers(d, valid);
        const int rank = __popcll(m & lt);
        // every lane reads the count before the lowest lane of its digit writes it: one wave, in program order
        const int before = wcnt[w][d];
        if (valid && rank == 0) wcnt[w][d] = before + __popcll(m);
        pos[r] = valid ? (d << 16) | (before + rank) : -1;
    }
    __syncthreads();
    int tot = gstart[t];
#pragma unroll
    for (int ww = 0; ww < kRsWaves; ++ww) {
        const int c = wcnt[ww][t];
        wcnt[ww][t] = tot;
        tot += c;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        if (pos[r] < 0) continue;
        const int d = pos[r] >> 16;
        const int dst = wcnt[w][d] + (pos[r] & 0xffff);
        kout[dst] = key[r];
        vout[dst] = val[r];
    }
}

// Two arrays of the same length in one pass: per-block totals of both, then both scans with the block
// offsets summed in the block; the last block also stores both totals to host-visible memory.
template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce2(const T *a, const T *b, int64_t n, T *bsum, int nb) {
    __shared__ T lw[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T sa = 0, sb = 0;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
        if (i < n) {
            sa += a[i];
            sb += b[i];
        }
    }
    T ta, tb;
    block_inclusive_sum(sa, lw, ta);
    block_inclusive_sum(sb, lw, tb);
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = ta;
        bsum[nb + blockIdx.x] = tb;
    }
}

template <class T>
__device__ T block_prefix_of(const T *bsum, T *red) {
    T pre = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += kScanThreads) pre += bsum[j];
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pre;
    __syncthreads();
    T r = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) r += red[w];
    return r;
}

template <class T>
__global__ void __launch_bounds__(kScanThreads)
k_scan_apply2(const T *a, T *oa, const T *b, T *ob, int64_t n, const T *bsum, int nb, T *host_tot) {
    __shared__ T lw[kScanThreads / 64];
    __shared__ T red[kScanThreads / 64];
    const T offa = block_prefix_of(bsum, red);
    const T offb = block_prefix_of(bsum + nb, red);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T la[kScanItems], lb[kScanItems];
    T sa = 0, sb = 0;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        la[j] = i < n ? a[i] : T(0);
        lb[j] = i < n ? b[i] : T(0);
        sa += la[j];
        sb += lb[j];
    }
    T ta, tb;
    const T ia = block_inclusive_sum(sa, lw, ta);
    const T ib = block_inclusive_sum(sb, lw, tb);
    T ra = offa + ia - sa, rb = offb + ib - sb;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j;
        if (i < n) {
            oa[i] = ra;
            ob[i] = rb;
        }
        ra += la[j];
        rb += lb[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        oa[n] = offa + ta;
        ob[n] = offb + tb;
        // host-visible memory: the caller reads it after synchronising the stream, and the kernel's
        // completion makes its writes visible to the host (no fence here: a system-scope fence writes back
        // the whole L2)
        host_tot[0] = offa + ta;
        host_tot[1] = offb + tb;
    }
}

}  // namespace

void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t st, Scratch &S) {
    exclusive_scan<int32_t>(in, out, n, st, S);
}

void exclusive_scan2_i64(const int64_t *a, int64_t *oa, const int64_t *b, int64_t *ob, int64_t n, int64_t *host_tot,
                         hipStream_t st, Scratch &S) {
    FFM_CHECK(n > 0, FFM_EINTERNAL, "two-array scan of an empty range");
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    FFM_CHECK(nb <= 4096, FFM_EINTERNAL, "two-array scan: too many tiles");
    int64_t *bsum = S.get<int64_t>(2 * nb);
    FFM_LAUNCH(k_scan_reduce2<int64_t>, nb, kScanThreads, 0, st, a, b, n, bsum, (int)nb);
    FFM_LAUNCH(k_scan_apply2<int64_t>, nb, kScanThreads, 0, st, a, oa, b, ob, n, (const int64_t *)bsum, (int)nb,
               host_tot);
}

void radix_sort_u64_u32(uint64_t *keys, int32_t *vals, int64_t n, hipStream_t st, Scratch &S) {
    if (n <= 1) return;
    FFM_CHECK(n < (int64_t(1) << 31), FFM_EINVAL, "radix sort: too many keys");
    const int nblk = (int)((n + kRsTile - 1) / kRsTile);
    uint64_t *k2 = S.get<uint64_t>(n);
    int32_t *v2 = S.get<int32_t>(n);
    int32_t *counts = S.get<int32_t>((size_t)256 * nblk + 1), *offs = S.get<int32_t>((size_t)256 * nblk + 1);
    uint64_t *ka = keys, *kb = k2;
    int32_t *va = vals, *vb = v2;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        FFM_LAUNCH(k_rs_hist, nblk, kRsThreads, 0, st, ka, n, shift, counts, nblk);
        exclusive_scan<int32_t>(counts, offs, (int64_t)256 * nblk, st, S);
        FFM_LAUNCH(k_rs_scatter, nblk, kRsThreads, 0, st, ka, va, kb, vb, n, shift, offs, nblk);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // eight passes: the result is back in (keys, vals)
}

}  // namespace ffm
