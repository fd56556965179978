// Apply: v = FFM(w u), one descent over the plan's levels, then the leaf near field.
//
// Paper: Sec. 2.2.2 (v ~ L_X^T (T (L_Y u)), Lagrange levels), Sec. 2.2.3 (v ~ F_{s->X} (T_L (F_{Y->s} u)),
// Gegenbauer levels, eqs. gegenbauerQuadrature and the three products that follow it), Sec. 2.2.4 (dense
// remainder), remark closing Sec. 2.2.3 (transforms evaluated on the fly at every level, no upward pass).
//
// Every kernel reads its parameters from the level descriptor named by its work item (int4, .x =
// descriptor), so one launch serves one level of one plan or the same step of many plans (a batch).
// Every output element is owned by exactly one thread of each kernel and accumulated in a fixed order,
// so results are bitwise reproducible and independent of how work items are grouped into launches.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

namespace ffm {

namespace {

constexpr int kThreads = 256;

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
using gch4 = const __attribute__((address_space(1))) half4_t *;
using gch8 = const __attribute__((address_space(1))) half8_t *;

// sin(2 pi x), cos(2 pi x) for x in revolutions.  The hardware reduces its argument itself over
// |x| <= 256 revolutions; against an exact reduction to [0, 1) first it differs by at most 2.4e-7
// (measured over 1.6e7 arguments), below the FP32 rounding of a phase of even one revolution.  FP32
// phases are passed unreduced where the planner bounds them by 128 revolutions (FP64 phases are
// reduced exactly in FP64 before rounding to FP32).
__device__ __forceinline__ void sincos_rev(float x, float &s, float &c) {
    s = __builtin_amdgcn_sinf(x);
    c = __builtin_amdgcn_cosf(x);
}

// ------------------------------------------------------------------ permutations and scaling
// item (desc, first index): u[i] = wu[perm_y[i]] for i < ny, v[i] = 0 for i < nx (256 per block)
__global__ void __launch_bounds__(kThreads)
k_perm_in(const LDesc *__restrict__ descs, const IoEntry *__restrict__ io, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const IoEntry e = io[d.inst];
    const int64_t i = (int64_t)wk.y + threadIdx.x;
    if (i < d.ny) {
        const int64_t j = d.perm_y[i];
        float2 r;
        switch (e.dtype) {
            case FFM_C64: r = static_cast<const float2 *>(e.wu)[j]; break;
            case FFM_F32: r = make_float2(static_cast<const float *>(e.wu)[j], 0.f); break;
            case FFM_F64: r = make_float2((float)static_cast<const double *>(e.wu)[j], 0.f); break;
            default: {
                const double2 w = static_cast<const double2 *>(e.wu)[j];
                r = make_float2((float)w.x, (float)w.y);
            }
        }
        d.u[i] = r;
        if (d.ucomp) {
            // split double layer: the densities u n_c
            const float4 n = d.sn[i];
            d.ucomp[i] = make_float2(r.x * n.x, r.y * n.x);
            d.ucomp[d.ny + i] = make_float2(r.x * n.y, r.y * n.y);
            d.ucomp[2 * d.ny + i] = make_float2(r.x * n.z, r.y * n.z);
        }
    }
    if (i < d.nx) {
        for (int c = 0; c < d.ncomp; ++c) d.v[(int64_t)c * d.nx + i] = make_float2(0.f, 0.f);
        if (d.vtmp)
            for (int c = 0; c < 3; ++c) d.vtmp[(int64_t)c * d.nx + i] = make_float2(0.f, 0.f);
    }
}

// max over |Re u|, |Im u| (non-negative floats compare as their bit patterns); item (desc, first index),
// 4096 entries per block.  The maximum is zeroed by the stage before (k_zero_amax).
__global__ void __launch_bounds__(kThreads)
k_amax(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    float m = 0.f;
    const int64_t end = min<int64_t>(d.ny, (int64_t)wk.y + 16 * kThreads);
    for (int64_t i = (int64_t)wk.y + threadIdx.x; i < end; i += kThreads)
        m = fmaxf(m, fmaxf(fabsf(d.u[i].x), fabsf(d.u[i].y)));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.f) atomicMax(reinterpret_cast<unsigned int *>(d.amax), __float_as_uint(m));
}

// item (desc, 0): zero the instance's max |u| (a kernel, not a memset, so the apply can be captured)
__global__ void k_zero_amax(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    if (threadIdx.x == 0) *descs[wk.x].amax = 0.f;
}

// v[i] = 0 (empty plans: no sources or no targets)
__global__ void __launch_bounds__(kThreads) k_zero_out(float2 *v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) v[i] = make_float2(0.f, 0.f);
}

// item (desc, first index): vout[i] = 0 for i < nx ncomp (an instance without sources inside a batch)
__global__ void __launch_bounds__(kThreads)
k_zero_io(const LDesc *__restrict__ descs, const IoEntry *__restrict__ io, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int64_t i = (int64_t)wk.y + threadIdx.x;
    if (i < d.nx * d.ncomp) io[d.inst].vout[i] = make_float2(0.f, 0.f);
}

// item (desc, first index): vout[perm_x[i]] = v[i]; gradient plans: vout[3 perm_x[i] + c] = v[c nx + i]
__global__ void __launch_bounds__(kThreads)
k_perm_out(const LDesc *__restrict__ descs, const IoEntry *__restrict__ io, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int64_t i = (int64_t)wk.y + threadIdx.x;
    if (i >= d.nx) return;
    if (d.ncomp == 1) {
        io[d.inst].vout[d.perm_x[i]] = d.v[i];
        return;
    }
    const int64_t o = 3 * (int64_t)d.perm_x[i];
    for (int c = 0; c < 3; ++c) io[d.inst].vout[o + c] = d.v[(int64_t)c * d.nx + i];
}

// ------------------------------------------------------------------ Gegenbauer levels, direction pairs
// Forward transform u~_s(q) = sum_{j in s} e^{-ik s_q.(y_j - c_s)} u_j for an antipodal pair (q, -q): with
// S = sum cos(th) u, T = sum sin(th) u, u~(q) = S - iT and u~(-q) = S + iT.
// Item (desc, source box, tile of 256 PPT pairs); the box's points stream through LDS.
// With DL (the normal derivative at the sources), every direction's term is multiplied by -ik (s . n_j): with
// a_j = k (s_q . n_j) u_j and S, T now the sums of cos(th) a and sin(th) a, u~(q) = -i (S - iT) and
// u~(-q) = i (S + iT).
template <int PPT, int BS, bool P64, bool DL>
__device__ __forceinline__ void pw_forward_body(const LDesc &d, const int4 wk) {
    const int b = wk.y;
    const int tid = threadIdx.x;
    const int64_t npair = d.npair;
    const int64_t p0 = (int64_t)wk.z * BS * PPT + tid;
    typedef typename std::conditional<P64, double, float>::type real;
    real sx[PPT], sy[PPT], sz[PPT];
    float Sre[PPT], Sim[PPT], Tre[PPT], Tim[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = p0 + (int64_t)j * BS;
        const int64_t pc = p < npair ? p : npair - 1;
        if (P64) {
            sx[j] = d.dirs64[3 * pc]; sy[j] = d.dirs64[3 * pc + 1]; sz[j] = d.dirs64[3 * pc + 2];
        } else {
            const float4 q = d.dirs[pc];
            sx[j] = q.x; sy[j] = q.y; sz[j] = q.z;
        }
        Sre[j] = Sim[j] = Tre[j] = Tim[j] = 0.f;
    }
    const double cx = d.sctr[3 * b], cy = d.sctr[3 * b + 1], cz = d.sctr[3 * b + 2];
    __shared__ real px[BS], py[BS], pz[BS];
    __shared__ float2 us[BS];
    __shared__ float4 ns[DL ? BS : 1];
    const int i0 = d.sstart[b], i1 = d.sstart[b + 1];
    for (int s0 = i0; s0 < i1; s0 += BS) {
        const int cnt = min(BS, i1 - s0);
        __syncthreads();
        if (tid < cnt) {
            const int i = s0 + tid;
            px[tid] = (real)(d.sxs[i] - cx);
            py[tid] = (real)(d.sys[i] - cy);
            pz[tid] = (real)(d.szs[i] - cz);
            us[tid] = d.u[i];
            if (DL) ns[tid] = d.sn[i];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const real x = px[jj], y = py[jj], z = pz[jj];
            const float2 uu = us[jj];
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                float f;
                if (P64) {
                    const double ph = fma((double)sx[j], (double)x, fma((double)sy[j], (double)y, (double)sz[j] * z));
                    f = (float)__builtin_amdgcn_fract(ph);
                } else {
                    const float ph = fmaf((float)sx[j], (float)x, fmaf((float)sy[j], (float)y, (float)sz[j] * (float)z));
                    f = ph;
                }
                float sn, cs;
                sincos_rev(f, sn, cs);
                float ax = uu.x, ay = uu.y;
                if (DL) {
                    // k (s . n) = 2 pi (s k / 2 pi) . n
                    const float4 n = ns[jj];
                    const float D = 6.2831853f * fmaf((float)sx[j], n.x, fmaf((float)sy[j], n.y, (float)sz[j] * n.z));
                    ax *= D;
                    ay *= D;
                }
                Sre[j] = fmaf(cs, ax, Sre[j]);
                Sim[j] = fmaf(cs, ay, Sim[j]);
                Tre[j] = fmaf(sn, ax, Tre[j]);
                Tim[j] = fmaf(sn, ay, Tim[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = p0 + (int64_t)j * BS;
        if (p < npair) {
            d.ut[(int64_t)b * npair + p] =
                DL ? make_float4(Sim[j] - Tre[j], -(Sre[j] + Tim[j]), -(Sim[j] + Tre[j]), Sre[j] - Tim[j])
                   : make_float4(Sre[j] + Tim[j], Sim[j] - Tre[j], Sre[j] - Tim[j], Sim[j] + Tre[j]);
        }
    }
}

template <int PPT, int BS, bool P64>
__global__ void __launch_bounds__(BS)
k_pw_forward(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    pw_forward_body<PPT, BS, P64, false>(descs[wk.x], wk);
}

template <int PPT, int BS, bool P64>
__global__ void __launch_bounds__(BS)
k_pw_forward_dl(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    pw_forward_body<PPT, BS, P64, true>(descs[wk.x], wk);
}

// Diagonal transfer v~_t(q) = sum_{s in far(t)} D_{c(t,s)}(q) u~_s(q) (both directions of a pair), for
// target t and the pairs p0 + j BS, j < PPT (t the same across the wave).
template <int PPT, int BS>
__device__ __forceinline__ void transfer_target(const LDesc &d, int t, int64_t p0) {
    const int64_t npair = d.npair;
    float4 acc[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) acc[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int e0 = __builtin_amdgcn_readfirstlane((int)d.far_ptr[t]);
    const int e1 = __builtin_amdgcn_readfirstlane((int)d.far_ptr[t + 1]);
    const float4 *__restrict__ D = d.D;
    const float4 *__restrict__ ut = d.ut;
    // the far list in chunks of 64 entries, one per lane (a single load and wait per chunk), then four far
    // pairs per step taken from the lanes' registers, their data loads issued together
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    for (int c0 = e0; c0 < e1; c0 += 64) {
        const int nch = min(64, e1 - c0);
        int src_l = 0, cls_l = 0;
        if (lane < nch) {
            src_l = d.far_src[c0 + lane];
            cls_l = d.far_cls[c0 + lane];
        }
        int k0 = 0;
        for (; k0 + U <= nch; k0 += U) {
            int64_t sv[U], cv[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                sv[k] = __builtin_amdgcn_readlane(src_l, k0 + k);
                cv[k] = __builtin_amdgcn_readlane(cls_l, k0 + k);
            }
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int64_t p = p0 + (int64_t)j * BS;
                if (p < npair) {
                    float4 q[U], w[U];
#pragma unroll
                    for (int k = 0; k < U; ++k) {
                        q[k] = D[cv[k] * npair + p];
                        w[k] = ut[sv[k] * npair + p];
                    }
#pragma unroll
                    for (int k = 0; k < U; ++k) {
                        acc[j].x = fmaf(q[k].x, w[k].x, fmaf(-q[k].y, w[k].y, acc[j].x));
                        acc[j].y = fmaf(q[k].x, w[k].y, fmaf(q[k].y, w[k].x, acc[j].y));
                        acc[j].z = fmaf(q[k].z, w[k].z, fmaf(-q[k].w, w[k].w, acc[j].z));
                        acc[j].w = fmaf(q[k].z, w[k].w, fmaf(q[k].w, w[k].z, acc[j].w));
                    }
                }
            }
        }
        for (; k0 < nch; ++k0) {
            const int64_t s = __builtin_amdgcn_readlane(src_l, k0), c = __builtin_amdgcn_readlane(cls_l, k0);
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int64_t p = p0 + (int64_t)j * BS;
                if (p < npair) {
                    const float4 q = D[c * npair + p];
                    const float4 w = ut[s * npair + p];
                    acc[j].x = fmaf(q.x, w.x, fmaf(-q.y, w.y, acc[j].x));
                    acc[j].y = fmaf(q.x, w.y, fmaf(q.y, w.x, acc[j].y));
                    acc[j].z = fmaf(q.z, w.z, fmaf(-q.w, w.w, acc[j].z));
                    acc[j].w = fmaf(q.z, w.w, fmaf(q.w, w.z, acc[j].w));
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = p0 + (int64_t)j * BS;
        if (p < npair) d.vt[(int64_t)t * npair + p] = acc[j];
    }
}

// Item (desc, target box, tile of BS PPT pairs).
template <int PPT, int BS>
__global__ void __launch_bounds__(BS)
k_pw_transfer(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    transfer_target<PPT, BS>(descs[wk.x], wk.y, (int64_t)wk.z * BS * PPT + threadIdx.x);
}

// Four consecutive target slots (Morton order) per block, one per wave, on the same tile of 64 pairs: a
// quarter of the blocks and work items of one target per block, for the same work per wave.  Item (desc,
// group of four slots, tile).
__global__ void __launch_bounds__(kThreads)
k_pw_transfer_grp(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int ti = __builtin_amdgcn_readfirstlane(wk.y * 4 + (int)(threadIdx.x >> 6));
    if (ti >= d.ntr) return;
    transfer_target<1, 64>(d, __builtin_amdgcn_readfirstlane(d.tr_tgt[ti]), (int64_t)wk.z * 64 + (threadIdx.x & 63));
}

// The transfer by sibling group (one tree): wave w of a block takes group 4 item.y + w, up to four targets of one
// parent box, on a tile of 64 pairs.  The group's far sources are visited once each (in position order): u~_s is read
// once and applied to every sibling whose far list holds s, with that pair's D.  Item (desc, block of four
// groups, tile).
__global__ void __launch_bounds__(kThreads)
k_pw_transfer_sib(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int g = __builtin_amdgcn_readfirstlane(wk.y * 4 + (int)(threadIdx.x >> 6));
    if (g >= d.nsibg) return;
    const int64_t npair = d.npair;
    const int64_t p0 = (int64_t)wk.z * 64 + (threadIdx.x & 63);
    const bool active = p0 < npair;
    const int64_t p = active ? p0 : npair - 1;       // idle lanes read a valid pair and store nothing
    const float4 *__restrict__ D = d.D;
    const float4 *__restrict__ ut = d.ut;
    float4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int n = __builtin_amdgcn_readfirstlane(d.sib_cnt[g]);
    const int32_t *src = d.sib_src + (int64_t)216 * g;
    const uint2 *cls = d.sib_cls + (int64_t)216 * g;
    const int lane = threadIdx.x & 63;
    // the group's slots in chunks of 64, one per lane (one load and wait per chunk), then taken from the lanes'
    // registers slot by slot
    for (int c0 = 0; c0 < n; c0 += 64) {
        const int nch = min(64, n - c0);
        int src_l = 0;
        uint2 cls_l = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
        if (lane < nch) {
            src_l = src[c0 + lane];
            cls_l = cls[c0 + lane];
        }
        for (int k = 0; k < nch; ++k) {
            const int64_t sv = __builtin_amdgcn_readlane(src_l, k);
            const uint32_t wds[2] = {(uint32_t)__builtin_amdgcn_readlane((int)cls_l.x, k),
                                     (uint32_t)__builtin_amdgcn_readlane((int)cls_l.y, k)};
            const float4 w = ut[sv * npair + p];
            float4 q[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = (int)(int16_t)(wds[j >> 1] >> (16 * (j & 1)));
                if (c >= 0) q[j] = D[(int64_t)c * npair + p];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = (int)(int16_t)(wds[j >> 1] >> (16 * (j & 1)));
                if (c >= 0) {
                    acc[j].x = fmaf(q[j].x, w.x, fmaf(-q[j].y, w.y, acc[j].x));
                    acc[j].y = fmaf(q[j].x, w.y, fmaf(q[j].y, w.x, acc[j].y));
                    acc[j].z = fmaf(q[j].z, w.z, fmaf(-q[j].w, w.w, acc[j].z));
                    acc[j].w = fmaf(q[j].z, w.w, fmaf(q[j].w, w.z, acc[j].w));
                }
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int t = __builtin_amdgcn_readfirstlane(d.sib_tgt[4 * g + j]);
        if (t >= 0) d.vt[(int64_t)t * npair + p0] = acc[j];
    }
}

// The same transfer for levels with many direction pairs per box.  Block: a
// tile of QT direction pairs for 256 / QT target boxes (consecutive in Morton order); the tile of every class's
// D is staged in LDS once per block, so each far pair reads D from LDS and only u~ from memory.  Four far pairs
// per step, their loads issued together.  Item (desc, group of target slots, tile).
template <int QT>
__global__ void __launch_bounds__(kThreads)
k_pw_transfer_lds(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    extern __shared__ float4 Ds[];            // [ncls][QT]
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int64_t npair = d.npair, q0 = (int64_t)wk.z * QT;
    const int ncls = d.ncls;
    for (int k = threadIdx.x; k < ncls * QT; k += kThreads) {
        const int c = k / QT, ql = k % QT;
        Ds[k] = q0 + ql < npair ? d.D[(int64_t)c * npair + q0 + ql] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    const int slot = threadIdx.x / QT, ql = threadIdx.x % QT;
    const int ti = wk.y * (kThreads / QT) + slot;
    const int64_t q = q0 + ql;
    if (ti >= d.ntr || q >= npair) return;
    const int t = d.tr_tgt[ti];
    const float4 *__restrict__ ut = d.ut;
    const float4 *Dq = Ds + ql;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    auto step = [&](const float4 &dq, const float4 &w) {
        acc.x = fmaf(dq.x, w.x, fmaf(-dq.y, w.y, acc.x));
        acc.y = fmaf(dq.x, w.y, fmaf(dq.y, w.x, acc.y));
        acc.z = fmaf(dq.z, w.z, fmaf(-dq.w, w.w, acc.z));
        acc.w = fmaf(dq.z, w.w, fmaf(dq.w, w.z, acc.w));
    };
    const int64_t e0 = d.far_ptr[t], e1 = d.far_ptr[t + 1];
    int64_t e = e0;
    // groups of four far pairs; the list entries of the next group are loaded while this group's u~ loads
    // are in flight
    int sn[4], cn[4];
    if (e + 4 <= e1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sn[k] = d.far_src[e + k];
            cn[k] = d.far_cls[e + k];
        }
    }
    for (; e + 4 <= e1; e += 4) {
        int64_t sv[4];
        int cv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sv[k] = sn[k];
            cv[k] = cn[k];
        }
        float4 w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = ut[sv[k] * npair + q];
        if (e + 8 <= e1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sn[k] = d.far_src[e + 4 + k];
                cn[k] = d.far_cls[e + 4 + k];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) step(Dq[cv[k] * QT], w[k]);
    }
    for (; e < e1; ++e) step(Dq[d.far_cls[e] * QT], ut[(int64_t)d.far_src[e] * npair + q]);
    d.vt[(int64_t)t * npair + q] = acc;
}

// Gradient plans: the target transform of component c is that of ik s_c v~, so the plain transforms (direct,
// ring or grid form) give the derivative along axis c.  For the pair (q, -q) (s(-q) = -s(q)):
// ik s_c v~(q) = f (-Im, Re) and -ik s_c v~(-q) = f (Im, -Re), f = k s_c = 2 pi (k s / 2 pi)_c.  Components 1 and 2
// go to the descriptor's vtx planes, component 0 replaces v~.  Item (desc, target box, tile of 256 pairs).
__global__ void __launch_bounds__(kThreads)
k_dir_scale(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int64_t p = (int64_t)wk.z * kThreads + threadIdx.x;
    if (p >= d.npair) return;
    const int64_t o = (int64_t)wk.y * d.npair + p;
    const float4 w = d.vt[o];
    const float4 s = d.dirs[p];
    auto sc = [&](float f) { return make_float4(-f * w.y, f * w.x, f * w.w, -f * w.z); };
    d.vtx[o] = sc(6.2831853f * s.y);
    d.vtx[d.vtstride + o] = sc(6.2831853f * s.z);
    d.vt[o] = sc(6.2831853f * s.x);
}

// Split double layer: u~(q) = -ik sum_c s_c u~_c(q) from the source transforms u~_c of the densities u n_c (in
// place of u~_0); for the pair (q, -q), with f_c = k s_c(q) = 2 pi (k s / 2 pi)_c:
// u~(q) = sum_c f_c (Im, -Re) u~_c(q) and u~(-q) = sum_c f_c (-Im, Re) u~_c(-q).  Item (desc, source box, tile of
// 256 pairs).
__global__ void __launch_bounds__(kThreads)
k_dl_combine(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int64_t p = (int64_t)wk.z * kThreads + threadIdx.x;
    if (p >= d.npair) return;
    const int64_t o = (int64_t)wk.y * d.npair + p;
    const float4 a = d.ut[o], b = d.utx[o], c = d.utx[d.utstride + o];
    const float4 s = d.dirs[p];
    const float fx = 6.2831853f * s.x, fy = 6.2831853f * s.y, fz = 6.2831853f * s.z;
    d.ut[o] = make_float4(fmaf(fx, a.y, fmaf(fy, b.y, fz * c.y)), -fmaf(fx, a.x, fmaf(fy, b.x, fz * c.x)),
                          -fmaf(fx, a.w, fmaf(fy, b.w, fz * c.w)), fmaf(fx, a.z, fmaf(fy, b.z, fz * c.z)));
}

// Split normal derivative at the targets: v_i += n_i . (T_0, T_1, T_2)_i over the axis planes of a level's
// target transforms, which are cleared for the next level.  Item (desc, target box, first point), 256 points.
__global__ void __launch_bounds__(kThreads)
k_dn_combine(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int i = wk.z + threadIdx.x;
    if (i >= d.tstart[wk.y + 1]) return;
    const float4 n = d.tn[i];
    float2 *t0 = d.vtmp + i, *t1 = t0 + d.nx, *t2 = t1 + d.nx;
    const float2 a = *t0, b = *t1, c = *t2;
    float2 o = d.v[i];
    o.x = fmaf(n.x, a.x, fmaf(n.y, b.x, fmaf(n.z, c.x, o.x)));
    o.y = fmaf(n.x, a.y, fmaf(n.y, b.y, fmaf(n.z, c.y, o.y)));
    d.v[i] = o;
    *t0 = *t1 = *t2 = make_float2(0.f, 0.f);
}

// Backward transform v_i += sum_q e^{ik s_q.(x_i - c_t)} v~_t(q): per pair, with A = v~(q) + v~(-q) and
// B = v~(q) - v~(-q), the pair contributes cos(th) A + i sin(th) B.  Item (desc, target box, first point);
// BS points per block (64 for levels of small boxes).
// With DN (the normal derivative at the target), every direction's term is multiplied by ik (s . n_i): the pair
// (q, -q) contributes ik (s_q . n) (e^{iP} v~(q) - e^{-iP} v~(-q)), with k s_q . n from the scaled directions.
template <int BS, bool P64, bool DN>
__device__ __forceinline__ void pw_backward_body(const LDesc &d, const int4 wk) {
    const int t = wk.y;
    const int tid = threadIdx.x;
    const int i = wk.z + tid;
    const bool valid = i < d.tstart[t + 1];
    const int64_t npair = d.npair;
    typedef typename std::conditional<P64, double, float>::type real;
    real x = 0, y = 0, z = 0;
    float nx = 0.f, ny = 0.f, nz = 0.f;
    if (valid) {
        x = (real)(d.txs[i] - d.tctr[3 * t]);
        y = (real)(d.tys[i] - d.tctr[3 * t + 1]);
        z = (real)(d.tzs[i] - d.tctr[3 * t + 2]);
        if (DN) {
            const float4 n = d.tn ? d.tn[i] : d.tnc;
            nx = n.x;
            ny = n.y;
            nz = n.z;
        }
    }
    float are = 0.f, aim = 0.f;
    __shared__ real sdx[BS], sdy[BS], sdz[BS];
    __shared__ float4 ab[BS];
    const float4 *vb = d.vt + (int64_t)t * npair;
    for (int64_t q0 = 0; q0 < npair; q0 += BS) {
        const int cnt = (int)min<int64_t>(BS, npair - q0);
        __syncthreads();
        if (tid < cnt) {
            const int64_t q = q0 + tid;
            if (P64) {
                sdx[tid] = d.dirs64[3 * q]; sdy[tid] = d.dirs64[3 * q + 1]; sdz[tid] = d.dirs64[3 * q + 2];
            } else {
                const float4 w = d.dirs[q];
                sdx[tid] = w.x; sdy[tid] = w.y; sdz[tid] = w.z;
            }
            const float4 w = vb[q];
            ab[tid] = DN ? make_float4(w.x - w.z, w.y - w.w, w.x + w.z, w.y + w.w)
                         : make_float4(w.x + w.z, w.y + w.w, w.x - w.z, w.y - w.w);
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            float f;
            if (P64) {
                const double ph = fma((double)sdx[jj], (double)x, fma((double)sdy[jj], (double)y, (double)sdz[jj] * z));
                f = (float)__builtin_amdgcn_fract(ph);
            } else {
                const float ph = fmaf((float)sdx[jj], (float)x, fmaf((float)sdy[jj], (float)y, (float)sdz[jj] * (float)z));
                f = ph;
            }
            float sn, cs;
            sincos_rev(f, sn, cs);
            const float4 w = ab[jj];
            if (DN) {
                // k (s . n) = 2 pi (s k / 2 pi) . n; X + iY = e^{iP} v~(q) - e^{-iP} v~(-q); adds i k (s . n) (X + iY)
                const float D = 6.2831853f * fmaf((float)sdx[jj], nx, fmaf((float)sdy[jj], ny, (float)sdz[jj] * nz));
                const float X = fmaf(cs, w.x, -sn * w.w), Y = fmaf(cs, w.y, sn * w.z);
                are = fmaf(-D, Y, are);
                aim = fmaf(D, X, aim);
            } else {
                are = fmaf(cs, w.x, fmaf(-sn, w.w, are));
                aim = fmaf(cs, w.y, fmaf(sn, w.z, aim));
            }
        }
    }
    if (valid) {
        float2 o = d.v[i];
        o.x += are;
        o.y += aim;
        d.v[i] = o;
    }
}

template <int BS, bool P64>
__global__ void __launch_bounds__(BS)
k_pw_backward(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    pw_backward_body<BS, P64, false>(descs[wk.x], wk);
}

template <int BS, bool P64>
__global__ void __launch_bounds__(BS)
k_pw_backward_dn(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    pw_backward_body<BS, P64, true>(descs[wk.x], wk);
}

// ------------------------------------------------------------------ Gegenbauer levels, ring-pair form
// The quadrature's directions (sin t_m cos f_n, sin t_m sin f_n, cos t_m) of ring m and its antipodal
// ring L - m (cos t_{L-m} = -cos t_m) with f_n and f_n + pi give four directions whose phases against
// a box-centred point y are +-P +- C, P = (k/2pi) sin t_m (y_1 cos f_n + y_2 sin f_n) and
// C = (k/2pi) cos t_m y_3.  One sin/cos of P and the per-(point, ring) factors e^{-+iC} serve all four:
//   u~(m, n)        = sum e^{-iP} u',    u~(m, n+L)     = sum e^{+iP} u',    u' = u e^{-iC}
//   u~(L-m, n)      = sum e^{-iP} u'',   u~(L-m, n+L)   = sum e^{+iP} u'',   u'' = u e^{+iC}
// Storage keeps the direction-pair layout: pair (m, n) = (u~(m,n), u~(L-m,n+L)), pair (m, n+L) =
// (u~(m,n+L), u~(L-m,n)); the equator ring (m = L/2, L even) holds pair (m, n) = (u~(m,n), u~(m,n+L)).
// C is reduced in FP64 once per (point, ring); P is evaluated in FP32 or FP64 (P64).
constexpr int kRingChunk = 64;
constexpr int kMaxRings = 16;

// Item (desc, source box, ring chunk, point segment); Tr threads per ring, R rings per block.
template <int G, bool P64>
__global__ void __launch_bounds__(kThreads)
k_pw_forward_rings(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    typedef typename std::conditional<P64, double, float>::type real;
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int b = wk.y;
    const int L = d.L, nrp = d.nrp, Tr = d.Tr, R = d.R, nsplit = d.nsplit, seg = wk.w;
    const int64_t npair = d.npair;
    const int m0 = wk.z * R;
    const int tid = threadIdx.x;
    const int rl = tid / Tr, nloc = tid % Tr;
    const int m = m0 + rl;
    const int nr = min(R, nrp - m0);
    const bool active = rl < nr;
    real cf[G], sf[G];
    float acc[G][8];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const int n = min(nloc + j * Tr, L - 1);
        cf[j] = (real)d.phis[n].x;
        sf[j] = (real)d.phis[n].y;
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[j][q] = 0.f;
    }
    const double cx = d.sctr[3 * b], cy = d.sctr[3 * b + 1], cz = d.sctr[3 * b + 2];
    __shared__ real sA[kMaxRings][kRingChunk], sB[kMaxRings][kRingChunk];
    __shared__ float4 sU[kMaxRings][kRingChunk];
    // this block's segment of the box's points
    const int b0 = d.sstart[b], b1 = d.sstart[b + 1];
    const int per = (b1 - b0 + nsplit - 1) / nsplit;
    const int i0 = b0 + seg * per, i1 = min(b1, i0 + per);
    for (int s0 = i0; s0 < i1; s0 += kRingChunk) {
        const int cnt = min(kRingChunk, i1 - s0);
        __syncthreads();
        for (int it = tid; it < nr * cnt; it += kThreads) {
            const int r = it / cnt, j = it % cnt, i = s0 + j;
            const double2 rg = d.rings[m0 + r];
            const double xr = d.sxs[i] - cx, yr = d.sys[i] - cy, zr = d.szs[i] - cz;
            sA[r][j] = (real)(rg.x * xr);
            sB[r][j] = (real)(rg.x * yr);
            const double C = rg.y * zr;
            float sn, cs;
            sincos_rev((float)(C - floor(C)), sn, cs);
            const float2 uu = d.u[i];
            // explicit fused forms: the rounding must not depend on how the compiler contracts
            sU[r][j] = make_float4(fmaf(uu.x, cs, uu.y * sn), fmaf(uu.y, cs, -(uu.x * sn)),
                                   fmaf(uu.x, cs, -(uu.y * sn)), fmaf(uu.y, cs, uu.x * sn));
        }
        __syncthreads();
        if (active) {
            for (int jj = 0; jj < cnt; ++jj) {
                const real A = sA[rl][jj], B = sB[rl][jj];
                const float4 w = sU[rl][jj];
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    float f;
                    if (P64) {
                        const double P = fma((double)A, (double)cf[j], (double)B * (double)sf[j]);
                        f = (float)__builtin_amdgcn_fract(P);
                    } else {
                        const float P = fmaf((float)A, (float)cf[j], (float)B * (float)sf[j]);
                        f = P;
                    }
                    float sn, cs;
                    sincos_rev(f, sn, cs);
                    acc[j][0] = fmaf(cs, w.x, acc[j][0]);
                    acc[j][1] = fmaf(cs, w.y, acc[j][1]);
                    acc[j][2] = fmaf(sn, w.x, acc[j][2]);
                    acc[j][3] = fmaf(sn, w.y, acc[j][3]);
                    acc[j][4] = fmaf(cs, w.z, acc[j][4]);
                    acc[j][5] = fmaf(cs, w.w, acc[j][5]);
                    acc[j][6] = fmaf(sn, w.z, acc[j][6]);
                    acc[j][7] = fmaf(sn, w.w, acc[j][7]);
                }
            }
        }
    }
    if (!active) return;
    const bool equator = 2 * m == L;
    float4 *o = (nsplit > 1 ? d.part + (int64_t)seg * d.part_stride : d.ut) + (int64_t)b * npair + (int64_t)m * 2 * L;
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const int n = nloc + j * Tr;
        if (n >= L) continue;
        // S' = (0,1), T' = (2,3), S'' = (4,5), T'' = (6,7); S -+ iT
        const float2 k0 = make_float2(acc[j][0] + acc[j][3], acc[j][1] - acc[j][2]);
        const float2 k1 = make_float2(acc[j][0] - acc[j][3], acc[j][1] + acc[j][2]);
        const float2 k2 = make_float2(acc[j][4] + acc[j][7], acc[j][5] - acc[j][6]);
        const float2 k3 = make_float2(acc[j][4] - acc[j][7], acc[j][5] + acc[j][6]);
        if (equator) {
            o[n] = make_float4(k0.x, k0.y, k1.x, k1.y);
        } else {
            o[n] = make_float4(k0.x, k0.y, k3.x, k3.y);
            o[n + L] = make_float4(k1.x, k1.y, k2.x, k2.y);
        }
    }
}

// Sum the point-segment partials of the forward transform in segment order.  Item (desc, source box).
__global__ void __launch_bounds__(kThreads)
k_sum_segments(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int64_t npair = d.npair;
    for (int64_t p = threadIdx.x; p < npair; p += kThreads) {
        const int64_t o = (int64_t)wk.y * npair + p;
        float4 a = d.part[o];
        for (int s = 1; s < d.nsplit; ++s) {
            const float4 w = d.part[(int64_t)s * d.part_stride + o];
            a.x += w.x; a.y += w.y; a.z += w.z; a.w += w.w;
        }
        d.ut[o] = a;
    }
}

// Backward transform in ring-pair form: per target point and ring pair m,
//   v += e^{iC} sum_n [e^{iP} v~(m,n) + e^{-iP} v~(m,n+L)] + e^{-iC} sum_n [e^{iP} v~(L-m,n) + e^{-iP} v~(L-m,n+L)]
// PT target points per thread, BS threads per block; item (desc, target box, first point).  The staged entries of a ring pair are
// padded with zeros to a multiple of U (a zero term leaves every sum unchanged), so the inner loop runs in
// unrolled steps of U with immediate LDS offsets.  Where a ring's padded azimuths fit one block's worth, the
// entries of as many ring pairs as fit kBkStage go to LDS at once (one load round and one barrier pair for
// all of them); otherwise ring pair by ring pair in chunks of kThreads azimuths.  Either way each ring pair's
// sums run over the same terms in the same order.
constexpr int kBkStage = 512;

// entries of ring pair m, azimuth n: (v~(m,n) + v~(m,n+L), i-free difference) pairs as the inner sums use them
__device__ __forceinline__ void bk_stage_entry(const float4 *vb, int L, int m, int n, float4 &e01, float4 &e23) {
    const float4 p1 = vb[(int64_t)m * 2 * L + n];
    if (2 * m == L) {
        e01 = make_float4(p1.x + p1.z, p1.y + p1.w, p1.x - p1.z, p1.y - p1.w);
        e23 = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        const float4 p2 = vb[(int64_t)m * 2 * L + n + L];
        e01 = make_float4(p1.x + p2.x, p1.y + p2.y, p1.x - p2.x, p1.y - p2.y);
        e23 = make_float4(p2.z + p1.z, p2.w + p1.w, p2.z - p1.z, p2.w - p1.w);
    }
}

template <int PT, int U, bool P64, typename real>
__device__ __forceinline__ void bk_ring_terms(const float4 *s01, const float4 *s23, const real *scf, const real *ssf,
                                              int cnt4, const real *A, const real *B, float *xre, float *xim,
                                              float *yre, float *yim) {
    for (int j0 = 0; j0 < cnt4; j0 += U) {
#pragma unroll
        for (int ju = 0; ju < U; ++ju) {
            const int jj = j0 + ju;
            const real cfn = scf[jj], sfn = ssf[jj];
            const float4 a = s01[jj], c = s23[jj];
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                float f;
                if (P64) {
                    const double P = fma((double)A[q], (double)cfn, (double)B[q] * (double)sfn);
                    f = (float)__builtin_amdgcn_fract(P);
                } else {
                    const float P = fmaf((float)A[q], (float)cfn, (float)B[q] * (float)sfn);
                    f = P;
                }
                float sn, cs;
                sincos_rev(f, sn, cs);
                xre[q] = fmaf(cs, a.x, fmaf(-sn, a.w, xre[q]));
                xim[q] = fmaf(cs, a.y, fmaf(sn, a.z, xim[q]));
                yre[q] = fmaf(cs, c.x, fmaf(-sn, c.w, yre[q]));
                yim[q] = fmaf(cs, c.y, fmaf(sn, c.z, yim[q]));
            }
        }
    }
}

template <int PT, int U, bool P64, int BS = kThreads>
__global__ void __launch_bounds__(BS)
k_pw_backward_rings(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    typedef typename std::conditional<P64, double, float>::type real;
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int tid = threadIdx.x;
    const int L = d.L, nrp = d.nrp;
    const int64_t npair = d.npair;
    const int iend = d.tstart[t + 1];
    double xr[PT], yr[PT], zr[PT];
    bool valid[PT];
    float vr[PT], vi[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        const int i = wk.z + tid + q * BS;
        valid[q] = i < iend;
        xr[q] = valid[q] ? d.txs[i] - d.tctr[3 * t] : 0.0;
        yr[q] = valid[q] ? d.tys[i] - d.tctr[3 * t + 1] : 0.0;
        zr[q] = valid[q] ? d.tzs[i] - d.tctr[3 * t + 2] : 0.0;
        vr[q] = vi[q] = 0.f;
    }
    __shared__ float4 s01[kBkStage], s23[kBkStage];
    __shared__ real scf[kThreads], ssf[kThreads];
    const float4 *vb = d.vt + (int64_t)t * npair;
    // this block's ring pairs (part wk.w of bsplit)
    const int mper = (nrp + d.bsplit - 1) / d.bsplit;
    const int mb = wk.w * mper, me = min(nrp, mb + mper);
    const int Lp = (L + U - 1) / U * U;
    // per ring pair: the point factors, then the sums over its azimuths (staged at e01, e23), then the
    // ring's contribution to v
    auto ring = [&](int m, const float4 *e01, const float4 *e23, int n0, int cnt4, bool first, bool last,
                    float *xre, float *xim, float *yre, float *yim, float *ecs, float *esn, real *A, real *B) {
        if (first) {
            const double2 rg = d.rings[m];
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                A[q] = (real)(rg.x * xr[q]);
                B[q] = (real)(rg.x * yr[q]);
                const double C = rg.y * zr[q];
                sincos_rev((float)(C - floor(C)), esn[q], ecs[q]);
                xre[q] = xim[q] = yre[q] = yim[q] = 0.f;
            }
        }
        bk_ring_terms<PT, U, P64, real>(e01, e23, scf + n0, ssf + n0, cnt4, A, B, xre, xim, yre, yim);
        if (last) {
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                // explicit fused forms, so every points-per-thread variant rounds identically
                vr[q] = fmaf(ecs[q], xre[q] + yre[q], fmaf(-esn[q], xim[q] - yim[q], vr[q]));
                vi[q] = fmaf(ecs[q], xim[q] + yim[q], fmaf(esn[q], xre[q] - yre[q], vi[q]));
            }
        }
    };
    real A[PT], B[PT];
    float ecs[PT], esn[PT], xre[PT], xim[PT], yre[PT], yim[PT];
    if (Lp <= kThreads) {
        // whole rings: the azimuth tables once, then groups of ring pairs
        for (int e = tid; e < Lp; e += BS) {
            scf[e] = e < L ? (real)d.phis[e].x : (real)0;
            ssf[e] = e < L ? (real)d.phis[e].y : (real)0;
        }
        const int rps = kBkStage / Lp;
        for (int g0 = mb; g0 < me; g0 += rps) {
            const int ng = min(rps, me - g0);
            __syncthreads();
            for (int e = tid; e < ng * Lp; e += BS) {
                const int r = e / Lp, n = e - r * Lp;
                if (n >= L) {
                    s01[e] = make_float4(0.f, 0.f, 0.f, 0.f);
                    s23[e] = make_float4(0.f, 0.f, 0.f, 0.f);
                } else {
                    bk_stage_entry(vb, L, g0 + r, n, s01[e], s23[e]);
                }
            }
            __syncthreads();
            for (int r = 0; r < ng; ++r)
                ring(g0 + r, s01 + r * Lp, s23 + r * Lp, 0, Lp, true, true, xre, xim, yre, yim, ecs, esn, A, B);
        }
    } else {
        for (int m = mb; m < me; ++m) {
            for (int n0 = 0; n0 < L; n0 += BS) {
                const int cnt = min(BS, L - n0);
                const int cnt4 = (cnt + U - 1) / U * U;
                __syncthreads();
                if (tid < cnt4) {
                    const int n = n0 + tid;
                    if (tid >= cnt) {
                        s01[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                        s23[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                        scf[tid] = (real)0;
                        ssf[tid] = (real)0;
                    } else {
                        bk_stage_entry(vb, L, m, n, s01[tid], s23[tid]);
                        scf[tid] = (real)d.phis[n].x;
                        ssf[tid] = (real)d.phis[n].y;
                    }
                }
                __syncthreads();
                ring(m, s01, s23, 0, cnt4, n0 == 0, n0 + BS >= L, xre, xim, yre, yim, ecs, esn, A, B);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        if (!valid[q]) continue;
        const int i = wk.z + tid + q * BS;
        if (d.bsplit > 1) {
            d.bpart[(int64_t)wk.w * d.nx + i] = make_float2(vr[q], vi[q]);
        } else {
            float2 o = d.v[i];
            o.x += vr[q];
            o.y += vi[q];
            d.v[i] = o;
        }
    }
}

// v_i += sum over ring parts of the target-transform partials, in part order.  Item (desc, target box,
// first point), 256 points per block.
__global__ void __launch_bounds__(kThreads)
k_sum_parts(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int i = wk.z + threadIdx.x;
    if (i >= d.tstart[wk.y + 1]) return;
    float2 a = d.bpart[i];
    for (int s = 1; s < d.bsplit; ++s) {
        const float2 w = d.bpart[(int64_t)s * d.nx + i];
        a.x += w.x;
        a.y += w.y;
    }
    float2 o = d.v[i];
    o.x += a.x;
    o.y += a.y;
    d.v[i] = o;
}

// ------------------------------------------------------------------ Gegenbauer levels, grid form
// The transforms as sums over a uniform grid: with a smooth kernel phi of width w (grid units) and its
// Fourier transform phi^, e^{-ik s.y} ~ (1/Phi(s)) sum_g phi((x_g - y)/h) e^{-ik s.x_g} (per axis, aliasing
// negligible for kh <= pi / 1.9), Phi(s) = prod_d phi^(k s_d h).  Forward: spread u onto the grid, sum
// over z for every ring (cos t_m), then over the plane for every direction; backward: the mirror sums
// and an interpolation at the targets.  Phi is divided out (twice) in the transfer diagonal.  Grid nodes
// x_a = (a - (p-1)/2) h about the box centre; G [box][c][a][b] (c: z), H [ring][box][a][b].
// Rings m and L - m (cos t opposite) share Ex, Ey; azimuths n and n + L give the conjugate tables.

// phi(x) = exp(beta (sqrt(1 - (2x/w)^2) - 1)) for |x| < w/2, 0 outside (exponential of semicircle), with
// k1 = 2 / w and k2 = beta log2(e): the hardware square root and base-2 exponential (exponents in
// [-27, 0]), about 1e-7 relative.
__device__ __forceinline__ float es_phi(float x, float k1, float k2) {
    const float t = x * k1;
    const float s = fmaf(-t, t, 1.f);
    return s > 0.f ? __builtin_amdgcn_exp2f(k2 * (__builtin_amdgcn_sqrtf(s) - 1.f)) : 0.f;
}

constexpr int kGT = 64;      // spreading tile edge (grid nodes)

// A contribution t (|t| < 2^62) as 64-bit fixed point: hi = floor(t 2^-32) and lo = t - hi 2^32 in [0, 2^32),
// th = t 2^-32 given.  lo is rounded to FP32 and truncated (at most 2^32 - 256), so the value is within a few
// hundred units of t, far below the FP32 rounding of the sums; each contribution is converted once, which keeps the integer sums order-independent.
__device__ __forceinline__ unsigned long long fixed64(float t, float th) {
    const float hi = floorf(th);
    const float lo = fmaf(-hi, 4294967296.f, t);
    return ((unsigned long long)(unsigned)(int)hi << 32) | (unsigned long long)(unsigned)fminf(lo, 4294967040.f);
}

// Spread the source points of a box onto one z-plane of its grid (one tile of at most 64 x 64 nodes), kernel
// width W.  The points come ordered by z-plane floor(z_g) with their grid coordinates: the W planes below and
// at c + W/2 - 1 hold exactly the points whose support reaches plane c.  Every contribution is rounded once
// to 64-bit fixed point (u scaled by 2^(61-e), 2^e >= (points of the box) x max |Re u|, |Im u| >= any partial
// sum) and summed with integer LDS atomics: the sums are exact, so the result does not depend on the order of
// the points.  Lane l of a wave takes every R-th point from l R on, so that the lanes of one atomic
// instruction fall on distinct, distant nodes (points are in Morton order within a plane).  Item (desc, box,
// plane, tile).
template <int W>
__global__ void __launch_bounds__(kThreads)
k_grid_spread(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int sb = wk.y, c = wk.z;
    const int p = d.gp;
    const int nta = (p + kGT - 1) / kGT;
    const int a0 = (wk.w / nta) * kGT, b0 = (wk.w % nta) * kGT;
    const int na = min(kGT, p - a0), nb = min(kGT, p - b0), ncell = na * nb;
    extern __shared__ unsigned long long accs[];           // [part][(a - a0) nb + b - b0], dynamic: 2 ncell
    unsigned long long *acc0 = accs, *acc1 = accs + ncell;
    for (int i = threadIdx.x; i < ncell; i += kThreads) {
        acc0[i] = 0ull;
        acc1[i] = 0ull;
    }
    __syncthreads();
    const double bound = (double)(d.sstart[sb + 1] - d.sstart[sb]) * (double)(*d.amax);
    int e = 0;
    if (bound > 0.0) frexp(bound, &e);
    constexpr float hw = 0.5f * W, k1 = 2.f / W;
    const float k2 = d.gbeta * 1.44269504f;
    const int64_t zoff = (int64_t)sb * p;
    // points binned by plane (even W: floor(z), odd W: nearest plane) whose support reaches plane c
    constexpr int zlo = W / 2, zhi = (W - 1) / 2;
    const int j0 = d.gzs[zoff + max(0, c - zlo)], j1 = d.gzs[zoff + min(p - 1, c + zhi) + 1];
    const int R = (j1 - j0 + 63) / 64, lane = threadIdx.x & 63;
    for (int r = threadIdx.x >> 6; r < R; r += kThreads / 64) {
        const int j = j0 + lane * R + r;
        if (j >= j1) continue;
        const float4 g = d.gxyz[j];
        const int alo = min(max((int)floorf(g.x - hw) + 1, 0), p - W);
        const int blo = min(max((int)floorf(g.y - hw) + 1, 0), p - W);
        if (alo + W <= a0 || alo >= a0 + na || blo + W <= b0 || blo >= b0 + nb) continue;
        const float wz = es_phi((float)c - g.z, k1, k2);
        const float2 uu = d.u[d.gperm[j]];
        const float ur = ldexpf(uu.x * wz, 61 - e), ui = ldexpf(uu.y * wz, 61 - e);
        float wx[W], ry[W], iy[W], rh[W], ih[W];
        int col[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int a = alo + k, b = blo + k;
            wx[k] = (a >= a0 && a < a0 + na) ? es_phi((float)a - g.x, k1, k2) : 0.f;
            const float wy = (b >= b0 && b < b0 + nb) ? es_phi((float)b - g.y, k1, k2) : 0.f;
            ry[k] = ur * wy;
            iy[k] = ui * wy;
            rh[k] = ry[k] * 2.3283064e-10f;    // 2^-32
            ih[k] = iy[k] * 2.3283064e-10f;
            col[k] = min(max(b - b0, 0), nb - 1);
        }
#pragma unroll
        for (int ka = 0; ka < W; ++ka) {
            const int row = min(max(alo + ka - a0, 0), na - 1) * nb;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                atomicAdd(&acc0[row + col[q]], fixed64(ry[q] * wx[ka], rh[q] * wx[ka]));
                atomicAdd(&acc1[row + col[q]], fixed64(iy[q] * wx[ka], ih[q] * wx[ka]));
            }
        }
    }
    __syncthreads();
    const double inv_scale = ldexp(1.0, e - 61);
    float2 *G = d.G + ((int64_t)d.gslot_s[sb] * p + c) * p * p;
    for (int kk = threadIdx.x; kk < ncell; kk += kThreads) {
        const int al = kk / nb, bl = kk % nb;
        G[(int64_t)(a0 + al) * p + b0 + bl] = make_float2((float)((double)(long long)acc0[kk] * inv_scale),
                                                          (float)((double)(long long)acc1[kk] * inv_scale));
    }
}

// v_mfma_f32_16x16x4f32: A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k, D[4 (lane / 16) + r][lane % 16]
// in register r.  The four grid sums below are real products with the real and imaginary parts of each
// operand as separate rows or columns; LDS operand rows are padded (80 floats for 64 columns, 144 for 128) so
// that the four 16-lane groups of a wave, which read four consecutive rows, hit distinct banks.  Steps run in
// groups of four without per-step conditions, so that the LDS reads of a group are issued together.
__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
constexpr int kRow64 = 80;
constexpr int kRow128 = 144;

// Global-memory views of device pointers: accesses through them compile to global instructions, which the
// LDS wait counter does not track (flat accesses are counted by both the memory and the LDS counters).
// Complex values are accessed as two-float vectors.
typedef float v2f __attribute__((ext_vector_type(2)));
using gc2 = const __attribute__((address_space(1))) v2f *;
using gm2 = __attribute__((address_space(1))) v2f *;
__device__ __forceinline__ gc2 gl(const float2 *p) { return (gc2)p; }
__device__ __forceinline__ gm2 gw(float2 *p) { return (gm2)p; }
using gcf = const __attribute__((address_space(1))) float *;
__device__ __forceinline__ gcf gfl(const float *p) { return (gcf)p; }
// Read-only views in the constant address space: wave-uniform loads through them are scalar loads.
using kc2 = const __attribute__((address_space(4))) v2f *;
__device__ __forceinline__ kc2 kcv(const float2 *p) { return (kc2)p; }

// Sums over z: C[(m, pe)][(ab, pg)] = sum_c Ez_pe[m][c] G_pg[c][ab]; H[m] = C_rr - C_ii + i (C_ri + C_ir) and
// H[L-m] = C_rr + C_ii + i (C_ri - C_ir) (rings m and L - m have conjugate z tables).  Block: 64 grid columns
// (16 per wave, held in registers) and a group of up to four 16-ring-pair blocks (grid_z_groups, their z
// tables staged through LDS); planes 64 at a time, MFMA step s and lane group g taking plane c0 + S g + s.
// Item (desc, box, column chunk, group).
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_grid_z(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int sb = wk.y, p = d.gp, L = d.L, nrp = d.nrp, p2 = p * p;
    const int ab0 = wk.z * 64;
    int ngr, gsz;
    grid_z_groups(nrp, ngr, gsz);
    const int nmb = (nrp + 15) / 16, mb0 = wk.w * gsz, nmbg = min(gsz, nmb - mb0);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    __shared__ float As[64 * kRow128];       // [step s, group g][ring block, part, ring]
    floatx4 acc[4][2][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 2; ++k) acc[i][j][k] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int ab = ab0 + wv * 16 + li;
    const gc2 G = gl(d.G) + (int64_t)d.gslot_s[sb] * p * p2 + min(ab, p2 - 1);
    const gc2 Ez = gl(d.Ez);
    const float gkeep = ab < p2 ? 1.f : 0.f;
    for (int c0 = 0; c0 < p; c0 += 64) {
        const int nc = min(64, p - c0), S = nc / 4;
        float gr[16], gi[16];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
            if (4 * s4 < S) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const v2f g = G[(int64_t)(c0 + S * lg + 4 * s4 + u) * p2];
                    gr[4 * s4 + u] = g.x * gkeep;
                    gi[4 * s4 + u] = g.y * gkeep;
                }
            }
        __syncthreads();
        for (int k = threadIdx.x; k < nc * 16 * nmbg; k += kThreads) {
            const int cl = k % nc, mr = k / nc, m = mb0 * 16 + mr;
            v2f e = {0.f, 0.f};
            if (m < nrp) e = Ez[(int64_t)m * p + c0 + cl];
            float *r = As + (4 * (cl % S) + cl / S) * kRow128 + (mr >> 4) * 32 + (mr & 15);
            r[0] = e.x;
            r[16] = e.y;
        }
        __syncthreads();
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            if (mi < nmbg) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
                    if (4 * s4 < S) {
                        float er[4], ei[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const float *ar = As + (4 * (4 * s4 + u) + lg) * kRow128 + mi * 32 + li;
                            er[u] = ar[0];
                            ei[u] = ar[16];
                        }
                        __builtin_amdgcn_sched_barrier(0);   // the group's LDS reads are issued together
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int s = 4 * s4 + u;
                            acc[mi][0][0] = mfma16(er[u], gr[s], acc[mi][0][0]);
                            acc[mi][0][1] = mfma16(er[u], gi[s], acc[mi][0][1]);
                            acc[mi][1][0] = mfma16(ei[u], gr[s], acc[mi][1][0]);
                            acc[mi][1][1] = mfma16(ei[u], gi[s], acc[mi][1][1]);
                        }
                    }
            }
        }
    }
    if (ab >= p2) return;
    const gm2 H = gw(d.H);
    const int hslot = d.gslot_s[sb];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        if (mi >= nmbg) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = (mb0 + mi) * 16 + 4 * lg + r;
            if (m >= nrp) continue;
            const float q1 = acc[mi][0][0][r], q3 = acc[mi][0][1][r], q4 = acc[mi][1][0][r], q2 = acc[mi][1][1][r];
            H[((int64_t)m * d.gnbox + hslot) * p2 + ab] = v2f{q1 - q2, q3 + q4};
            if (L - m != m) H[((int64_t)(L - m) * d.gnbox + hslot) * p2 + ab] = v2f{q1 + q2, q3 - q4};
        }
    }
}

// The MFMA steps of k_grid_phi: 4 S4 steps over the staged rows, NT column tiles, in groups of four steps
// whose LDS operands are read together before their products.
template <int S4, int NT>
__device__ __forceinline__ void phi_steps(const float *bl, const float (&hr)[16], const float (&hi)[16],
                                          floatx4 (&acc)[2][4]) {
#pragma unroll
    for (int g = 0; g < S4; ++g) {
        float bv[4][NT];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) bv[u][t] = bl[4 * (4 * g + u) * kRow64 + t * 16];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                acc[0][t] = mfma16(hr[4 * g + u], bv[u][t], acc[0][t]);
                acc[1][t] = mfma16(hi[4 * g + u], bv[u][t], acc[1][t]);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int S4>
__device__ __forceinline__ void phi_steps_nt(int ntile, const float *bl, const float (&hr)[16], const float (&hi)[16],
                                             floatx4 (&acc)[2][4]) {
    switch (ntile) {
        case 1: phi_steps<S4, 1>(bl, hr, hi, acc); break;
        case 2: phi_steps<S4, 2>(bl, hr, hi, acc); break;
        case 3: phi_steps<S4, 3>(bl, hr, hi, acc); break;
        default: phi_steps<S4, 4>(bl, hr, hi, acc); break;
    }
}

// Sums over the plane to the directions of ring m: C[(a, pa)][(n, pe)] = sum_b H_pa[a][b] Ey_pe[b][n], whose
// four real products give z0 = C_rr + i C_ir and z1 = C_ri + i C_ii per (a, n); then u~(m, n) = sum_a Ex[a][n]
// (z0 + i z1) and u~(m, n + L) = sum_a conj(Ex[a][n]) (z0 - i z1) (azimuths n and n + L have conjugate
// in-plane tables).  Block: one ring of one box; waves take 16-row blocks of a (held in registers when the
// grid has at most 64 rows); azimuths in chunks of 32 (four column tiles of 8 azimuths, real parts in columns
// 0-7 and imaginary parts in 8-15), b staged through LDS 64 at a time (step s, lane group g: b = b0 + S g + s)
// with Ex beside it.  Each lane sums its four rows, the two parts are added across lanes, and the partial
// sums of the 16 row groups are added in order.  Item (desc, box, ring, 0).
__global__ void __launch_bounds__(kThreads)
k_grid_phi(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int sb = wk.y, m = wk.z;
    const int p = d.gp, L = d.L, mt = min(m, L - m);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    constexpr int kExRow = 68;               // 32 complex azimuths + pad, in floats
    __shared__ float Bs[64 * kRow64];
    __shared__ float Exs[64 * kExRow];
    __shared__ float4 red[4][4][32];         // [wave][lane group][azimuth]
    const gc2 H = gl(d.H) + ((int64_t)m * d.gnbox + d.gslot_s[sb]) * p * p;
    const gc2 Ey = gl(d.Ey) + (int64_t)mt * p * L;
    const gc2 Ex = gl(d.Ex) + (int64_t)mt * p * L;
    const int nab = p / 16, rounds = (nab + 3) / 4;
    const bool one = p <= 64;                // one round of row blocks and one chunk of b
    const gm2 ut = gw(reinterpret_cast<float2 *>(d.ut)) + (int64_t)sb * d.npair * 2;
    const int64_t twoL = 2 * (int64_t)L;
    float hr[16], hi[16];
    auto load_rows = [&](int blk, int b0, int S) {
        const gc2 hrow = H + (int64_t)(blk * 16 + li) * p + b0 + S * lg;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
            if (4 * s4 < S) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const v2f h = hrow[4 * s4 + u];
                    hr[4 * s4 + u] = h.x;
                    hi[4 * s4 + u] = h.y;
                }
            }
    };
    if (one && wv < nab) load_rows(wv, 0, p / 4);
    const float *bl = Bs + lg * kRow64 + li;
    for (int n0 = 0; n0 < L; n0 += 32) {
        const int ntile = min(4, (L - n0 + 7) / 8);
        float4 tot[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) tot[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int rd = 0; rd < rounds; ++rd) {
            const int blk = rd * 4 + wv;
            const bool act = blk < nab;
            floatx4 acc[2][4];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[i][t] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int b0 = 0; b0 < p; b0 += 64) {
                const int nb = min(64, p - b0), S = nb / 4;
                __syncthreads();
                {
                    // all loads of the chunk in flight at once: 8 per thread for Ey, 8 for Ex
                    const int nl = threadIdx.x % 32, n = n0 + nl, q0 = threadIdx.x / 32;
                    const int na = b0 == 0 ? min(64, p - rd * 64) : 0;
                    v2f ey[8], ex[8];
#pragma unroll
                    for (int it = 0; it < 8; ++it) {
                        const int q = q0 + 8 * it;
                        ey[it] = v2f{0.f, 0.f};
                        ex[it] = v2f{0.f, 0.f};
                        if (q < nb && n < L) ey[it] = Ey[(int64_t)(b0 + q) * L + n];
                        if (q < na && n < L) ex[it] = Ex[(int64_t)(rd * 64 + q) * L + n];
                    }
#pragma unroll
                    for (int it = 0; it < 8; ++it) {
                        const int q = q0 + 8 * it;
                        if (q < nb) {
                            float *r = Bs + (4 * (q % S) + q / S) * kRow64 + (nl >> 3) * 16 + (nl & 7);
                            r[0] = ey[it].x;
                            r[8] = ey[it].y;
                        }
                        if (q < na) reinterpret_cast<float2 *>(Exs + q * kExRow)[nl] = make_float2(ex[it].x, ex[it].y);
                    }
                }
                __syncthreads();
                if (act) {
                    if (!one) load_rows(blk, b0, S);
                    switch (S / 4) {
                        case 1: phi_steps_nt<1>(ntile, bl, hr, hi, acc); break;
                        case 2: phi_steps_nt<2>(ntile, bl, hr, hi, acc); break;
                        case 3: phi_steps_nt<3>(ntile, bl, hr, hi, acc); break;
                        default: phi_steps_nt<4>(ntile, bl, hr, hi, acc); break;
                    }
                }
            }
            if (act) {
                const bool im = li >= 8;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (t >= ntile) continue;
                    const int nl = 8 * t + (li & 7);
                    float fr = 0.f, fi = 0.f, gr = 0.f, gi = 0.f;   // sum Ex z, sum conj(Ex) z over this lane's rows
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float2 ex = reinterpret_cast<const float2 *>(Exs + (wv * 16 + 4 * lg + r) * kExRow)[nl];
                        const float x = acc[0][t][r], y = acc[1][t][r];
                        fr = fmaf(ex.x, x, fmaf(-ex.y, y, fr));
                        fi = fmaf(ex.x, y, fmaf(ex.y, x, fi));
                        gr = fmaf(ex.x, x, fmaf(ex.y, y, gr));
                        gi = fmaf(ex.x, y, fmaf(-ex.y, x, gi));
                    }
                    // the imaginary-part columns hold z1: contribute i F and -i G
                    float t0 = im ? -fi : fr, t1 = im ? fr : fi, t2 = im ? gi : gr, t3 = im ? -gr : gi;
                    t0 += __shfl_xor(t0, 8, 64);
                    t1 += __shfl_xor(t1, 8, 64);
                    t2 += __shfl_xor(t2, 8, 64);
                    t3 += __shfl_xor(t3, 8, 64);
                    tot[t].x += t0;
                    tot[t].y += t1;
                    tot[t].z += t2;
                    tot[t].w += t3;
                }
            }
        }
        if (li < 8) {
#pragma unroll
            for (int t = 0; t < 4; ++t) red[wv][lg][8 * t + li] = tot[t];
        }
        __syncthreads();
        const int nl = threadIdx.x, n = n0 + nl;
        if (nl < 32 && n < L) {
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int w = 0; w < min(4, nab); ++w)
                for (int g = 0; g < 4; ++g) {
                    const float4 b = red[w][g][nl];
                    a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
                }
            // a.xy = u~(m, n), a.zw = u~(m, n + L), into the antipodal-pair layout
            if (2 * m < L) {
                ut[(m * twoL + n) * 2] = v2f{a.x, a.y};
                ut[(m * twoL + n + L) * 2] = v2f{a.z, a.w};
            } else if (2 * m > L) {
                const int64_t m2 = L - m;
                ut[(m2 * twoL + n) * 2 + 1] = v2f{a.z, a.w};
                ut[(m2 * twoL + n + L) * 2 + 1] = v2f{a.x, a.y};
            } else {
                ut[(m * twoL + n) * 2] = v2f{a.x, a.y};
                ut[(m * twoL + n) * 2 + 1] = v2f{a.z, a.w};
            }
        }
    }
}

// The MFMA steps of k_grid_phi_r: 16 P16 steps over all staged rows (groups of four whose LDS operands are read
// together before their products), NT column tiles, the A operand (H rows) in registers.
template <int P16, int NT>
__device__ __forceinline__ void phi_steps_r(const float *bl, const float (&hr)[4 * P16], const float (&hi)[4 * P16],
                                            floatx4 (&acc)[2][4]) {
#pragma unroll
    for (int g = 0; g < P16; ++g) {
        float bv[4][NT];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) bv[u][t] = bl[4 * (4 * g + u) * kRow64 + t * 16];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                acc[0][t] = mfma16(hr[4 * g + u], bv[u][t], acc[0][t]);
                acc[1][t] = mfma16(hi[4 * g + u], bv[u][t], acc[1][t]);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The sums of k_grid_phi for grids of P = 16 P16 nodes, 64 < P <= 128: rounds of four 16-row blocks of a on
// the outside, each wave's H rows over the whole of b loaded once per round into registers (4 P16 values per
// lane and part), and every chunk of 32 azimuths staged with all of Ey's P rows.  The partial sums of a round
// (over its rows, the two parts and the four lane groups, in that order) are added to u~ in round order by the
// thread that owns the azimuth.  Item (desc, box, ring, 0).
template <int P16>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_grid_phi_r(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    constexpr int P = 16 * P16, S = 4 * P16;        // nodes; MFMA steps (b = S g + s for lane group g, step s)
    constexpr int kExRow = 68;                       // 32 complex azimuths + pad, in floats
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int sb = wk.y, m = wk.z;
    const int L = d.L, mt = min(m, L - m);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    __shared__ float Bs[P * kRow64];
    __shared__ float Exs[64 * kExRow];
    __shared__ float4 red[4][4][32];                 // [wave][lane group][azimuth]
    const gc2 H = gl(d.H) + ((int64_t)m * d.gnbox + d.gslot_s[sb]) * P * P;
    const gc2 Ey = gl(d.Ey) + (int64_t)mt * P * L;
    const gc2 Ex = gl(d.Ex) + (int64_t)mt * P * L;
    const gm2 ut = gw(reinterpret_cast<float2 *>(d.ut)) + (int64_t)sb * d.npair * 2;
    const int64_t twoL = 2 * (int64_t)L;
    const float *bl = Bs + lg * kRow64 + li;
    for (int rd = 0; rd < (P16 + 3) / 4; ++rd) {
        const int blk = rd * 4 + wv, nact = min(4, P16 - rd * 4), na = min(64, P - rd * 64);
        const bool act = blk < P16;
        float hr[S], hi[S];
        if (act) {
            const gc2 hrow = H + (int64_t)(blk * 16 + li) * P + S * lg;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const v2f h = hrow[s];
                hr[s] = h.x;
                hi[s] = h.y;
            }
        }
        for (int n0 = 0; n0 < L; n0 += 32) {
            const int ntile = min(4, (L - n0 + 7) / 8);
            __syncthreads();
            {
                // Ey rows q < P and Ex rows q < na of this round, azimuth n0 + nl; loads in flight together
                const int nl = threadIdx.x % 32, n = n0 + nl, q0 = threadIdx.x / 32;
                v2f ey[P / 8], ex[8];
#pragma unroll
                for (int it = 0; it < P / 8; ++it) {
                    const int q = q0 + 8 * it;
                    ey[it] = n < L ? Ey[(int64_t)q * L + n] : v2f{0.f, 0.f};
                }
#pragma unroll
                for (int it = 0; it < 8; ++it) {
                    const int q = q0 + 8 * it;
                    ex[it] = (q < na && n < L) ? Ex[(int64_t)(rd * 64 + q) * L + n] : v2f{0.f, 0.f};
                }
#pragma unroll
                for (int it = 0; it < P / 8; ++it) {
                    const int q = q0 + 8 * it;
                    float *r = Bs + (4 * (q % S) + q / S) * kRow64 + (nl >> 3) * 16 + (nl & 7);
                    r[0] = ey[it].x;
                    r[8] = ey[it].y;
                }
#pragma unroll
                for (int it = 0; it < 8; ++it)
                    reinterpret_cast<float2 *>(Exs + (q0 + 8 * it) * kExRow)[nl] = make_float2(ex[it].x, ex[it].y);
            }
            __syncthreads();
            float4 tot[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) tot[t] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (act) {
                floatx4 acc[2][4];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[i][t] = floatx4{0.f, 0.f, 0.f, 0.f};
                switch (ntile) {
                    case 1: phi_steps_r<P16, 1>(bl, hr, hi, acc); break;
                    case 2: phi_steps_r<P16, 2>(bl, hr, hi, acc); break;
                    case 3: phi_steps_r<P16, 3>(bl, hr, hi, acc); break;
                    default: phi_steps_r<P16, 4>(bl, hr, hi, acc); break;
                }
                const bool im = li >= 8;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (t >= ntile) continue;
                    const int nl = 8 * t + (li & 7);
                    float fr = 0.f, fi = 0.f, gr = 0.f, gi = 0.f;   // sum Ex z, sum conj(Ex) z over this lane's rows
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float2 ex = reinterpret_cast<const float2 *>(Exs + (wv * 16 + 4 * lg + r) * kExRow)[nl];
                        const float x = acc[0][t][r], y = acc[1][t][r];
                        fr = fmaf(ex.x, x, fmaf(-ex.y, y, fr));
                        fi = fmaf(ex.x, y, fmaf(ex.y, x, fi));
                        gr = fmaf(ex.x, x, fmaf(ex.y, y, gr));
                        gi = fmaf(ex.x, y, fmaf(-ex.y, x, gi));
                    }
                    // the imaginary-part columns hold z1: contribute i F and -i G
                    float t0 = im ? -fi : fr, t1 = im ? fr : fi, t2 = im ? gi : gr, t3 = im ? -gr : gi;
                    t0 += __shfl_xor(t0, 8, 64);
                    t1 += __shfl_xor(t1, 8, 64);
                    t2 += __shfl_xor(t2, 8, 64);
                    t3 += __shfl_xor(t3, 8, 64);
                    tot[t] = make_float4(t0, t1, t2, t3);
                }
            }
            if (li < 8) {
#pragma unroll
                for (int t = 0; t < 4; ++t) red[wv][lg][8 * t + li] = tot[t];
            }
            __syncthreads();
            const int nl = threadIdx.x, n = n0 + nl;
            if (nl < 32 && n < L) {
                float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
                for (int w = 0; w < nact; ++w)
                    for (int g = 0; g < 4; ++g) {
                        const float4 b = red[w][g][nl];
                        a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
                    }
                // a.xy: u~(m, n), a.zw: u~(m, n + L), added to the earlier rounds' sums in the antipodal-pair layout
                int64_t i1, i2;
                if (2 * m < L) {
                    i1 = (m * twoL + n) * 2;
                    i2 = (m * twoL + n + L) * 2;
                } else if (2 * m > L) {
                    const int64_t m2 = L - m;
                    i1 = (m2 * twoL + n + L) * 2 + 1;
                    i2 = (m2 * twoL + n) * 2 + 1;
                } else {
                    i1 = (m * twoL + n) * 2;
                    i2 = (m * twoL + n) * 2 + 1;
                }
                if (rd > 0) {
                    const v2f o1 = ut[i1], o2 = ut[i2];
                    a.x = o1.x + a.x;
                    a.y = o1.y + a.y;
                    a.z = o2.x + a.z;
                    a.w = o2.y + a.w;
                }
                ut[i1] = v2f{a.x, a.y};
                ut[i2] = v2f{a.z, a.w};
            }
        }
    }
}

// Sums over the plane to the directions for grids of P = 16 P16 <= 64 nodes per axis: the products of
// k_grid_phi with H staged once in LDS as the A operand ([b][a block, part, a % 16], b = 4 s + g for step s and
// lane group g); each wave then runs on its own over its 8-azimuth column tiles (tiles w, w + 4, ...): the Ey
// values a lane needs come from memory straight into registers one tile ahead, Ex goes through a
// wave-private LDS slice, and the sums over a are completed inside the wave (its 4 rows per lane, then across
// the two parts and the four lane groups).  Steps go in groups of two (their LDS reads issued together), and
// the kernel keeps to 53 KB of LDS and the registers of three waves per SIMD, so that three blocks share a CU
// (64 nodes: 0.58 -> 0.53 ms on the 1M-point sphere's level 2 against groups of four steps at two blocks per
// CU).  Item (desc, box, ring, 0).
template <int P16>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
k_grid_phi_s(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    constexpr int P = 16 * P16, S = 4 * P16, NX = P / 8;   // nodes, MFMA steps, Ex values per lane and tile
    constexpr int kExR = 16;                                // floats per Ex row: 8 complex azimuths
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int sb = wk.y, m = wk.z, L = d.L, mt = min(m, L - m);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    __shared__ float As[P * kRow128];
    __shared__ float Exw[4][P * kExR];
    {
        const gc2 H = gl(d.H) + ((int64_t)m * d.gnbox + d.gslot_s[sb]) * P * P;
        v2f hv[P16 * P16];
#pragma unroll
        for (int it = 0; it < P16 * P16; ++it) hv[it] = H[threadIdx.x + it * kThreads];
#pragma unroll
        for (int it = 0; it < P16 * P16; ++it) {
            const int idx = threadIdx.x + it * kThreads, a = idx / P, b = idx % P;
            float *r = As + b * kRow128 + (a >> 4) * 32 + (a & 15);
            r[0] = hv[it].x;
            r[16] = hv[it].y;
        }
    }
    __syncthreads();
    using gcf = const __attribute__((address_space(1))) float *;
    const gcf Eyf = (gcf)(d.Ey + (int64_t)mt * P * L);
    const gc2 Ex = gl(d.Ex) + (int64_t)mt * P * L;
    const int pe = li >> 3, ntiles = (L + 7) / 8;
    float *exw = Exw[wv];
    const gm2 ut = gw(reinterpret_cast<float2 *>(d.ut)) + (int64_t)sb * d.npair * 2;
    const int64_t twoL = 2 * (int64_t)L;
    float bnx[S];
    v2f xnx[NX];
    auto prefetch = [&](int t) {
        const int n = 8 * t + (li & 7);
        const bool ok = n < L;
        const int nc = ok ? n : 0;
#pragma unroll
        for (int s = 0; s < S; ++s) bnx[s] = ok ? Eyf[2 * ((int64_t)(4 * s + lg) * L + nc) + pe] : 0.f;
        const int nx = 8 * t + (lane & 7);
        const bool okx = nx < L;
#pragma unroll
        for (int j = 0; j < NX; ++j) xnx[j] = okx ? Ex[(int64_t)(lane / 8 + 8 * j) * L + nx] : v2f{0.f, 0.f};
    };
    if (wv < ntiles) prefetch(wv);
    for (int t = wv; t < ntiles; t += 4) {
        float bv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) bv[s] = bnx[s];
#pragma unroll
        for (int j = 0; j < NX; ++j)
            reinterpret_cast<float2 *>(exw + (lane / 8 + 8 * j) * kExR)[lane & 7] = make_float2(xnx[j].x, xnx[j].y);
        if (t + 4 < ntiles) prefetch(t + 4);
        floatx4 acc[P16][2];
#pragma unroll
        for (int q = 0; q < P16; ++q) acc[q][0] = acc[q][1] = floatx4{0.f, 0.f, 0.f, 0.f};
        const float *al = As + lg * kRow128 + li;
#pragma unroll
        for (int g = 0; g < 2 * P16; ++g) {
            float av[2][P16][2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < P16; ++q) {
                    av[u][q][0] = al[4 * (2 * g + u) * kRow128 + q * 32];
                    av[u][q][1] = al[4 * (2 * g + u) * kRow128 + q * 32 + 16];
                }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < P16; ++q) {
                    acc[q][0] = mfma16(av[u][q][0], bv[2 * g + u], acc[q][0]);
                    acc[q][1] = mfma16(av[u][q][1], bv[2 * g + u], acc[q][1]);
                }
            __builtin_amdgcn_sched_barrier(0);
        }
        // sums over this lane's rows: F = sum Ex z, G = sum conj(Ex) z, z = (row of H_r, row of H_i) products
        float fr = 0.f, fi = 0.f, gr = 0.f, gi = 0.f;
#pragma unroll
        for (int q = 0; q < P16; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float2 ex = reinterpret_cast<const float2 *>(exw + (q * 16 + 4 * lg + r) * kExR)[li & 7];
                const float x = acc[q][0][r], y = acc[q][1][r];
                fr = fmaf(ex.x, x, fmaf(-ex.y, y, fr));
                fi = fmaf(ex.x, y, fmaf(ex.y, x, fi));
                gr = fmaf(ex.x, x, fmaf(ex.y, y, gr));
                gi = fmaf(ex.x, y, fmaf(-ex.y, x, gi));
            }
        // the imaginary-part columns hold z1: contribute i F and -i G
        float t0 = pe ? -fi : fr, t1 = pe ? fr : fi, t2 = pe ? gi : gr, t3 = pe ? -gr : gi;
#pragma unroll
        for (int o = 8; o < 64; o <<= 1) {
            t0 += __shfl_xor(t0, o, 64);
            t1 += __shfl_xor(t1, o, 64);
            t2 += __shfl_xor(t2, o, 64);
            t3 += __shfl_xor(t3, o, 64);
        }
        const int n = 8 * t + li;
        if (lane < 8 && n < L) {
            // (t0, t1) = u~(m, n), (t2, t3) = u~(m, n + L), into the antipodal-pair layout
            if (2 * m < L) {
                ut[(m * twoL + n) * 2] = v2f{t0, t1};
                ut[(m * twoL + n + L) * 2] = v2f{t2, t3};
            } else if (2 * m > L) {
                const int64_t m2 = L - m;
                ut[(m2 * twoL + n) * 2 + 1] = v2f{t2, t3};
                ut[(m2 * twoL + n + L) * 2 + 1] = v2f{t0, t1};
            } else {
                ut[(m * twoL + n) * 2] = v2f{t0, t1};
                ut[(m * twoL + n) * 2 + 1] = v2f{t2, t3};
            }
        }
    }
}

// The products of steps s_lo .. s_hi - 1 of one staged chunk of k_grid_phit for the 16-row block ab of a: QN
// column tiles of 16, in groups of four steps where the range allows (a group's LDS reads are all issued before
// its products; rows past the staged azimuths of a partial chunk are zero), with no conditions inside a step.
template <int QN, int RB, int QB>
__device__ __forceinline__ void phit_mma(const float *Ar, const float *Ai, const float *Bs, int ab, int li, int lg,
                                         int s_lo, int s_hi, floatx4 (&acc)[2][QB]) {
    int s0 = s_lo;
#pragma unroll 1
    for (; s0 + 4 <= s_hi; s0 += 4) {
        float ar[4], ai[4], bv[4][QN];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int row = (4 * (s0 + u) + lg) * kRow64;
            ar[u] = Ar[row + ab * 16 + li];
            ai[u] = Ai[row + ab * 16 + li];
#pragma unroll
            for (int q = 0; q < QN; ++q) bv[u][q] = Bs[(4 * (s0 + u) + lg) * RB + q * 16 + li];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                acc[0][q] = mfma16(ar[u], bv[u][q], acc[0][q]);
                acc[1][q] = mfma16(ai[u], bv[u][q], acc[1][q]);
            }
    }
    {
        for (int s = s0; s < s_hi; ++s) {
            const int row = (4 * s + lg) * kRow64;
            const float ar = Ar[row + ab * 16 + li], ai = Ai[row + ab * 16 + li];
            float bv[QN];
#pragma unroll
            for (int q = 0; q < QN; ++q) bv[q] = Bs[(4 * s + lg) * RB + q * 16 + li];
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                acc[0][q] = mfma16(ar, bv[q], acc[0][q]);
                acc[1][q] = mfma16(ai, bv[q], acc[1][q]);
            }
        }
    }
}

// v~ of ring m back to its plane: H'_pa[a][b] = sum over (n, pe) of A[(a, pa)][(n, pe)] E_pe[b][n] with
// A = (S_r, -D_i | S_i, D_r), S = conj(Ex) v~(n) + Ex v~(n + L), D = Ex v~(n + L) - conj(Ex) v~(n).  Block: one
// ring and a 64 x 64 tile of the plane; waves take 16-row blocks of a and all four 16-column blocks of b;
// azimuths staged through LDS 16 at a time from the transposed tables ([n][node]), step s and lane group g
// taking azimuth 2 s + g / 2 and part g % 2.  Where the tile has only one or two 16-row blocks of a (grids of
// 16 or 32 nodes, edge tiles), the otherwise idle waves take a share of each chunk's steps, and their partial
// sums are added to the first share's through LDS, in the order of the shares.  The next chunk's table values
// and v~ are loaded into registers while the current chunk's products run.  Grids of 80, 96 and 112 nodes take
// tiles of 64 rows of a by the whole of b (k_grid_phit_wide: up to eight 16-column blocks per wave), so that
// no tile is a sliver and each chunk's A operand is staged once per 64 rows.  Item (desc, box, ring, tile).
template <int BW>
__device__ __forceinline__ void grid_phit_body(const int4 wk, const LDesc &d) {
    constexpr int QB = BW / 16;                              // column blocks of 16 in a tile
    constexpr int RB = BW == 64 ? kRow64 : kRow128;          // floats per staged row of B
    constexpr int kStage = 2 * 32 * kRow64 + 32 * RB;        // A (two parts) and B
    constexpr int kRed = 3 * 2 * QB * 4 * 64;                // at most three shares of partial sums
    const int tb = wk.y, m = wk.z;
    const int p = d.gp, L = d.L, mt = min(m, L - m);
    const int nta = (p + 63) / 64;
    const int a0 = BW == 64 ? (wk.w / nta) * 64 : wk.w * 64, b0 = BW == 64 ? (wk.w % nta) * 64 : 0;
    const int qn = min(QB, (p - b0 + 15) / 16);   // column tiles of 16 inside the grid
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    __shared__ float lds[kStage > kRed ? kStage : kRed];
    float *const Ar = lds, *const Ai = lds + 32 * kRow64, *const Bs = lds + 2 * 32 * kRow64;
    floatx4 acc[2][QB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < QB; ++q) acc[i][q] = floatx4{0.f, 0.f, 0.f, 0.f};
    // row blocks of a in the tile, shares of the steps, this wave's row block and share
    const int nab = min(4, (p - a0 + 15) / 16);
    const int ks = nab == 1 ? 4 : (nab == 2 ? 2 : 1);
    const int ab = wv % nab, kp = wv / nab;
    const bool act = kp < ks;
    constexpr int kStepsPerChunk = 8;
    const int64_t twoL = 2 * (int64_t)L;
    const gc2 ExT = gl(d.ExT) + (int64_t)mt * L * p, EyT = gl(d.EyT) + (int64_t)mt * L * p;
    // v~(m, n) and v~(m, n + L) in the antipodal-pair layout
    int64_t o1, o2, dn;   // v1 at vt[o1 + dn n], v2 at vt[o2 + dn n]
    if (2 * m < L) {
        o1 = (int64_t)m * twoL * 2;
        o2 = ((int64_t)m * twoL + L) * 2;
    } else if (2 * m > L) {
        o1 = ((int64_t)(L - m) * twoL + L) * 2 + 1;
        o2 = (int64_t)(L - m) * twoL * 2 + 1;
    } else {
        o1 = (int64_t)m * twoL * 2;
        o2 = (int64_t)m * twoL * 2 + 1;
    }
    dn = 2;
    const int x = threadIdx.x % 64, nq = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    // v~ depends on the azimuth only, one per wave and step: scalar loads into scalar registers
    const kc2 vts = kcv(reinterpret_cast<const float2 *>(d.vt)) + (int64_t)tb * d.npair * 2;
    v2f exv[4], eyv[4], eyw[4], v1v[4], v2v[4];   // eyw: columns 64 .. 127 of wide tiles
    auto fetch = [&](int n0) {
        const int cnt = min(16, L - n0);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int nl = nq + 4 * it, n = n0 + nl;
            const bool ok = nl < cnt;
            exv[it] = eyv[it] = eyw[it] = v1v[it] = v2v[it] = v2f{0.f, 0.f};
            if (ok) {
                v1v[it] = vts[o1 + dn * n];
                v2v[it] = vts[o2 + dn * n];
            }
            if (ok && a0 + x < p) exv[it] = ExT[(int64_t)n * p + a0 + x];
            if (ok && b0 + x < p) eyv[it] = EyT[(int64_t)n * p + b0 + x];
            if (BW > 64 && ok && b0 + 64 + x < p) eyw[it] = EyT[(int64_t)n * p + b0 + 64 + x];
        }
    };
    fetch(0);
    for (int n0 = 0; n0 < L; n0 += 16) {
        const int cnt = min(16, L - n0);
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int nl = nq + 4 * it;
            const v2f ex = exv[it], v1 = v1v[it], v2 = v2v[it];
            const float y1r = fmaf(ex.x, v1.x, ex.y * v1.y), y1i = fmaf(ex.x, v1.y, -(ex.y * v1.x));   // conj(ex) v1
            const float y2r = fmaf(ex.x, v2.x, -(ex.y * v2.y)), y2i = fmaf(ex.x, v2.y, ex.y * v2.x);   // ex v2
            Ar[(2 * nl) * kRow64 + x] = y1r + y2r;          // S_r
            Ar[(2 * nl + 1) * kRow64 + x] = y1i - y2i;      // -D_i
            Ai[(2 * nl) * kRow64 + x] = y1i + y2i;          // S_i
            Ai[(2 * nl + 1) * kRow64 + x] = y2r - y1r;      // D_r
            Bs[(2 * nl) * RB + x] = eyv[it].x;
            Bs[(2 * nl + 1) * RB + x] = eyv[it].y;
            if (BW > 64) {
                Bs[(2 * nl) * RB + 64 + x] = eyw[it].x;
                Bs[(2 * nl + 1) * RB + 64 + x] = eyw[it].y;
            }
        }
        if (n0 + 16 < L) fetch(n0 + 16);
        __syncthreads();
        if (act) {
            // branch-free bodies for the common shapes, so that the LDS reads of later steps are issued
            // ahead of the products (rows past the chunk hold zeros in the partial last chunk)
            const int steps = (2 * cnt + 3) / 4;
            const int s_lo = kp * (kStepsPerChunk / ks), s_hi = min(steps, s_lo + kStepsPerChunk / ks);
            if (BW == 64) {
                switch (qn) {
                    case 4: phit_mma<4, RB, QB>(Ar, Ai, Bs, ab, li, lg, s_lo, s_hi, acc); break;
                    case 3: phit_mma<3, RB, QB>(Ar, Ai, Bs, ab, li, lg, s_lo, s_hi, acc); break;
                    case 2: phit_mma<2, RB, QB>(Ar, Ai, Bs, ab, li, lg, s_lo, s_hi, acc); break;
                    default: phit_mma<1, RB, QB>(Ar, Ai, Bs, ab, li, lg, s_lo, s_hi, acc); break;
                }
            } else {
                switch (qn) {   // wide tiles cover grids of 80 .. 128 nodes: 5 .. 8 column blocks
                    case 8: phit_mma<(QB < 8 ? QB : 8), RB, QB>(Ar, Ai, Bs, ab, li, lg, s_lo, s_hi, acc); break;
                    case 7: phit_mma<(QB < 7 ? QB : 7), RB, QB>(Ar, Ai, Bs, ab, li, lg, s_lo, s_hi, acc); break;
                    case 6: phit_mma<(QB < 6 ? QB : 6), RB, QB>(Ar, Ai, Bs, ab, li, lg, s_lo, s_hi, acc); break;
                    default: phit_mma<(QB < 5 ? QB : 5), RB, QB>(Ar, Ai, Bs, ab, li, lg, s_lo, s_hi, acc); break;
                }
            }
        }
    }
    if (ks > 1) {
        // shares 1 .. ks-1 through LDS (8 QB floats per lane and share: [part][column tile][row]), added to share
        // 0 in share order; (ks - 1) nab <= 3 shares, within the array
        constexpr int kShare = 2 * QB * 4 * 64;
        __syncthreads();
        if (act && kp > 0) {
            float *red = lds + ((kp - 1) * nab + ab) * kShare + lane;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int q = 0; q < QB; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) red[((i * QB + q) * 4 + r) * 64] = acc[i][q][r];
        }
        __syncthreads();
        if (act && kp == 0)
            for (int k = 1; k < ks; ++k) {
                const float *red = lds + ((k - 1) * nab + ab) * kShare + lane;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int q = 0; q < QB; ++q)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[i][q][r] += red[((i * QB + q) * 4 + r) * 64];
            }
    }
    if (!act || kp > 0) return;
    const gm2 Hb = gw(d.H) + ((int64_t)m * d.gnbox + d.gslot_t[tb]) * p * p;
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        const int b = b0 + q * 16 + li;
        if (b >= p) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = a0 + ab * 16 + 4 * lg + r;
            Hb[(int64_t)a * p + b] = v2f{acc[0][q][r], acc[1][q][r]};
        }
    }
}

// The mirror plane sums for grids of at most 32 nodes, rings m and L - m together (they share the tables ExT and
// EyT; only v~ differs): the staged A operand holds both rings' 32 rows of a side by side (64 columns), B the
// shared 32 columns of Ey, and wave w takes ring w / 2 and row block w % 2, so every wave has two full column
// blocks of products.  Item (desc, box, ring m <= L / 2, 0).
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_grid_phit_pair(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int tb = wk.y, m = wk.z;
    const int p = d.gp, L = d.L;                   // p <= 32, m <= L - m
    const int mr[2] = {m, L - m};
    const bool two = L - m != m;
    const int qn = (p + 15) / 16;                  // column blocks of b (1 or 2)
    const int nab = (p + 15) / 16;                 // row blocks of a per ring
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    const int rr = wv >> 1, ab = wv & 1;
    const bool act = ab < nab && (rr == 0 || two);
    __shared__ float Ar[32 * kRow64], Ai[32 * kRow64], Bs[32 * kRow64];
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[i][q] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int64_t twoL = 2 * (int64_t)L;
    const gc2 ExT = gl(d.ExT) + (int64_t)m * L * p, EyT = gl(d.EyT) + (int64_t)m * L * p;
    // v~(m', n) and v~(m', n + L) of both rings in the antipodal-pair layout: v1 at vt[o1 + 2 n], v2 at vt[o2 + 2 n]
    int64_t o1[2], o2[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int mm = mr[k];
        if (2 * mm < L) {
            o1[k] = (int64_t)mm * twoL * 2;
            o2[k] = ((int64_t)mm * twoL + L) * 2;
        } else if (2 * mm > L) {
            o1[k] = ((int64_t)(L - mm) * twoL + L) * 2 + 1;
            o2[k] = (int64_t)(L - mm) * twoL * 2 + 1;
        } else {
            o1[k] = (int64_t)mm * twoL * 2;
            o2[k] = (int64_t)mm * twoL * 2 + 1;
        }
    }
    // staging thread: column x of A is ring x / 32, row a = x % 32; columns x < 32 of B are b = x
    const int x = threadIdx.x % 64, xr = x >> 5, xa = x & 31, nq = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const kc2 vts = kcv(reinterpret_cast<const float2 *>(d.vt)) + (int64_t)tb * d.npair * 2;
    v2f exv[4], eyv[4], v1v[4], v2v[4];
    auto fetch = [&](int n0) {
        const int cnt = min(16, L - n0);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int nl = nq + 4 * it, n = n0 + nl;
            const bool ok = nl < cnt;
            exv[it] = eyv[it] = v1v[it] = v2v[it] = v2f{0.f, 0.f};
            if (ok) {
                // both rings' values by scalar loads, each lane keeping its own ring's
                const v2f a1 = vts[o1[0] + 2 * n], a2 = vts[o2[0] + 2 * n];
                v2f b1 = a1, b2 = a2;
                if (two) {
                    b1 = vts[o1[1] + 2 * n];
                    b2 = vts[o2[1] + 2 * n];
                }
                v1v[it] = xr ? b1 : a1;
                v2v[it] = xr ? b2 : a2;
            }
            if (ok && xa < p) exv[it] = ExT[(int64_t)n * p + xa];
            if (ok && x < p) eyv[it] = EyT[(int64_t)n * p + x];
        }
    };
    fetch(0);
    for (int n0 = 0; n0 < L; n0 += 16) {
        const int cnt = min(16, L - n0);
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int nl = nq + 4 * it;
            const v2f ex = exv[it], v1 = v1v[it], v2 = v2v[it];
            const float y1r = fmaf(ex.x, v1.x, ex.y * v1.y), y1i = fmaf(ex.x, v1.y, -(ex.y * v1.x));   // conj(ex) v1
            const float y2r = fmaf(ex.x, v2.x, -(ex.y * v2.y)), y2i = fmaf(ex.x, v2.y, ex.y * v2.x);   // ex v2
            Ar[(2 * nl) * kRow64 + x] = y1r + y2r;          // S_r
            Ar[(2 * nl + 1) * kRow64 + x] = y1i - y2i;      // -D_i
            Ai[(2 * nl) * kRow64 + x] = y1i + y2i;          // S_i
            Ai[(2 * nl + 1) * kRow64 + x] = y2r - y1r;      // D_r
            Bs[(2 * nl) * kRow64 + x] = eyv[it].x;
            Bs[(2 * nl + 1) * kRow64 + x] = eyv[it].y;
        }
        if (n0 + 16 < L) fetch(n0 + 16);
        __syncthreads();
        if (act) {
            const int steps = (2 * cnt + 3) / 4;
            // A's row block for this wave: ring rr's rows start at column 32 rr
            if (qn == 2)
                phit_mma<2, kRow64, 2>(Ar, Ai, Bs, 2 * rr + ab, li, lg, 0, steps, acc);
            else
                phit_mma<1, kRow64, 2>(Ar, Ai, Bs, 2 * rr + ab, li, lg, 0, steps, acc);
        }
    }
    if (!act) return;
    const gm2 Hb = gw(d.H) + ((int64_t)mr[rr] * d.gnbox + d.gslot_t[tb]) * p * p;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int b = q * 16 + li;
        if (q >= qn || b >= p) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = ab * 16 + 4 * lg + r;
            Hb[(int64_t)a * p + b] = v2f{acc[0][q][r], acc[1][q][r]};
        }
    }
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_grid_phit(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    grid_phit_body<64>(wk, descs[wk.x]);
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_grid_phit_wide(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    grid_phit_body<128>(wk, descs[wk.x]);
}

// Back over z: G'_pg[c][ab] = sum over (ring pair m, part pe) of A[c][(m, pe)] B[(m, pe)][(ab, pg)] with
// A = (Re Ez, Im Ez) and B = (S_r, S_i | -D_i, D_r), S = H'[m] + H'[L-m], D = H'[L-m] - H'[m].  Block: 64 grid
// columns and 64 planes (16 per wave); ring pairs staged through LDS 16 at a time, step s and lane group g
// taking ring pair 2 s + g / 2 and part g % 2.  Item (desc, box, column chunk, plane chunk).
__global__ void __launch_bounds__(kThreads)
k_grid_zt(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int tb = wk.y, p = d.gp, L = d.L, nrp = d.nrp, p2 = p * p;
    const int ab0 = wk.z * 64, c0 = wk.w * 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    __shared__ float As[32 * kRow64];
    __shared__ float Bs[32 * kRow128];
    floatx4 acc[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bool act = c0 + wv * 16 < p;
    const gc2 H = gl(d.H), Ez = gl(d.Ez);
    const int hslot = d.gslot_t[tb];
    for (int mp0 = 0; mp0 < nrp; mp0 += 16) {
        const int mc = min(16, nrp - mp0);
        __syncthreads();
        {
            const int x = threadIdx.x % 64, mq = threadIdx.x / 64, ab = ab0 + x;
            v2f ev[4], h1v[4], h2v[4];
#pragma unroll
            for (int it = 0; it < 4; ++it) {     // all loads of the chunk in flight at once
                const int ml = mq + 4 * it, mp = mp0 + ml, m2 = L - mp;
                ev[it] = h1v[it] = h2v[it] = v2f{0.f, 0.f};
                if (ml < mc) {
                    if (c0 + x < p) ev[it] = Ez[(int64_t)mp * p + c0 + x];
                    if (ab < p2) {
                        h1v[it] = H[((int64_t)mp * d.gnbox + hslot) * p2 + ab];
                        if (m2 != mp) h2v[it] = H[((int64_t)m2 * d.gnbox + hslot) * p2 + ab];
                    }
                }
            }
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int ml = mq + 4 * it;
                const v2f h1 = h1v[it], h2 = h2v[it];
                const float Sx = h1.x + h2.x, Sy = h1.y + h2.y, Dx = h2.x - h1.x, Dy = h2.y - h1.y;
                As[(2 * ml) * kRow64 + x] = ev[it].x;
                As[(2 * ml + 1) * kRow64 + x] = ev[it].y;
                float *r0 = Bs + (2 * ml) * kRow128 + (x >> 4) * 32 + (x & 15);
                float *r1 = r0 + kRow128;
                r0[0] = Sx;
                r0[16] = Sy;
                r1[0] = -Dy;
                r1[16] = Dx;
            }
        }
        __syncthreads();
        if (act) {
            const int steps = (2 * mc + 3) / 4;
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                if (4 * g >= steps) break;
                float av[4], bv[4][8];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int s = 4 * g + u;
                    av[u] = As[(4 * s + lg) * kRow64 + wv * 16 + li];
                    const float *br = Bs + (4 * s + lg) * kRow128 + li;
#pragma unroll
                    for (int q = 0; q < 8; ++q) bv[u][q] = br[q * 16];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        acc[q][0] = mfma16(av[u], bv[u][2 * q], acc[q][0]);
                        acc[q][1] = mfma16(av[u], bv[u][2 * q + 1], acc[q][1]);
                    }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (!act) return;
    const gm2 G = gw(d.G) + (int64_t)hslot * p * p2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ab = ab0 + q * 16 + li;
        if (ab >= p2) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = c0 + wv * 16 + 4 * lg + r;
            if (c < p) G[(int64_t)c * p2 + ab] = v2f{acc[q][0][r], acc[q][1][r]};
        }
    }
}

// v_i += sum over the W^3 grid nodes around x_i of phi phi phi G'.  Item (desc, target box, first point).
template <int W>
__global__ void __launch_bounds__(kThreads)
k_grid_interp(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int i = wk.z + threadIdx.x;
    if (i >= d.tstart[t + 1]) return;
    const int p = d.gp;
    constexpr float hw = 0.5f * W, k1 = 2.f / W;
    const float half = 0.5f * (float)(p - 1), k2 = d.gbeta * 1.44269504f;
    const double ih = d.ginv_h;
    const float xg = (float)((d.txs[i] - d.tctr[3 * t]) * ih) + half;
    const float yg = (float)((d.tys[i] - d.tctr[3 * t + 1]) * ih) + half;
    const float zg = (float)((d.tzs[i] - d.tctr[3 * t + 2]) * ih) + half;
    const int alo = min(max((int)floorf(xg - hw) + 1, 0), p - W);
    const int blo = min(max((int)floorf(yg - hw) + 1, 0), p - W);
    const int clo = min(max((int)floorf(zg - hw) + 1, 0), p - W);
    float wx[W], wy[W], wz[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        wx[k] = es_phi((float)(alo + k) - xg, k1, k2);
        wy[k] = es_phi((float)(blo + k) - yg, k1, k2);
        wz[k] = es_phi((float)(clo + k) - zg, k1, k2);
    }
    const gc2 G = gl(d.G) + (int64_t)d.gslot_t[t] * p * p * p + ((int64_t)clo * p + alo) * p + blo;
    float sr = 0.f, si = 0.f;
#pragma unroll
    for (int kc = 0; kc < W; ++kc) {
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int ka = 0; ka < W; ++ka) {
            const gc2 row = G + ((int64_t)kc * p + ka) * p;
            float rr = 0.f, ri = 0.f;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const v2f g = row[q];
                rr = fmaf(wy[q], g.x, rr);
                ri = fmaf(wy[q], g.y, ri);
            }
            pr = fmaf(wx[ka], rr, pr);
            pi = fmaf(wx[ka], ri, pi);
        }
        sr = fmaf(wz[kc], pr, sr);
        si = fmaf(wz[kc], pi, si);
    }
    float2 o = d.v[i];
    o.x += sr;
    o.y += si;
    d.v[i] = o;
}

// ------------------------------------------------------------------ Lagrange levels
constexpr int kMaxR1 = 8;
constexpr int kAnterpChunk = 64;

// One-dimensional Lagrange polynomials on the Chebyshev nodes at t (denominators precomputed).
__device__ __forceinline__ void lagrange_1d(float t, int r1, const float *nodes, const float *inv_den, float *ell) {
    for (int a = 0; a < r1; ++a) {
        float v = inv_den[a];
        for (int b = 0; b < r1; ++b)
            if (b != a) v *= (t - nodes[b]);
        ell[a] = v;
    }
}

// Their derivatives: l_a'(t) = inv_den_a sum_{m != a} prod_{b != a, m} (t - t_b).
__device__ __forceinline__ void lagrange_1d_deriv(float t, int r1, const float *nodes, const float *inv_den, float *dell) {
    for (int a = 0; a < r1; ++a) {
        float sum = 0.f;
        for (int m = 0; m < r1; ++m) {
            if (m == a) continue;
            float pr = 1.f;
            for (int b = 0; b < r1; ++b)
                if (b != a && b != m) pr *= (t - nodes[b]);
            sum += pr;
        }
        dell[a] = sum * inv_den[a];
    }
}

// u~_s = L_Y u_s: u~_s[(a r1 + b) r1 + c] = sum_j l_a(t_x) l_b(t_y) l_c(t_z) u_j, t = 2 (y - c_s) / d_l.
// With DL (the normal derivative at the sources) the weight of node (a, b, c) is n_j . grad_y of its polynomial:
// (2 / d_l) (n_x l'_a l_b l_c + n_y l_a l'_b l_c + n_z l_a l_b l'_c); the staged derivative tables carry the
// factors (2 / d_l) n.  Item (desc, source box).
template <bool DL, int R1>
__device__ __forceinline__ void lag_anterp_r1(const LDesc &d, const int4 wk, float (*ell)[(DL ? 6 : 3) * kMaxR1],
                                              float2 *us, float *nodes, float *den) {
    const int b = wk.y;
    const int tid = threadIdx.x;
    constexpr int r1 = R1, r = R1 * R1 * R1;
    const int rp = d.rp;
    const double two_over_dl = d.two_over_dl;
    if (tid < r1) {
        nodes[tid] = d.lnodes[tid];
        den[tid] = d.lden[tid];
    }
    constexpr int kOut = (r + kThreads - 1) / kThreads;
    float2 acc[kOut];
    int ia[kOut], ib[kOut], ic[kOut];
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
        const int i = tid + o * kThreads;
        acc[o] = make_float2(0.f, 0.f);
        const int ii = i < r ? i : 0;
        ia[o] = ii / (r1 * r1);
        ib[o] = (ii / r1) % r1;
        ic[o] = ii % r1;
    }
    constexpr int nout = kOut;
    const double cx = d.sctr[3 * b], cy = d.sctr[3 * b + 1], cz = d.sctr[3 * b + 2];
    const int i0 = d.sstart[b], i1 = d.sstart[b + 1];
    for (int s0 = i0; s0 < i1; s0 += kAnterpChunk) {
        const int cnt = min(kAnterpChunk, i1 - s0);
        __syncthreads();
        if (tid < cnt) {
            const int j = s0 + tid;
            lagrange_1d((float)((d.sxs[j] - cx) * two_over_dl), r1, nodes, den, &ell[tid][0]);
            lagrange_1d((float)((d.sys[j] - cy) * two_over_dl), r1, nodes, den, &ell[tid][r1]);
            lagrange_1d((float)((d.szs[j] - cz) * two_over_dl), r1, nodes, den, &ell[tid][2 * r1]);
            if (DL) {
                const float4 n = d.sn[j];
                const float f = (float)two_over_dl;
                float *g = &ell[tid][3 * r1];
                lagrange_1d_deriv((float)((d.sxs[j] - cx) * two_over_dl), r1, nodes, den, g);
                lagrange_1d_deriv((float)((d.sys[j] - cy) * two_over_dl), r1, nodes, den, g + r1);
                lagrange_1d_deriv((float)((d.szs[j] - cz) * two_over_dl), r1, nodes, den, g + 2 * r1);
                for (int a = 0; a < r1; ++a) {
                    g[a] *= f * n.x;
                    g[r1 + a] *= f * n.y;
                    g[2 * r1 + a] *= f * n.z;
                }
            }
            us[tid] = d.u[j];
        }
        __syncthreads();
#pragma unroll 4
        for (int jj = 0; jj < cnt; ++jj) {
            const float2 uu = us[jj];
#pragma unroll
            for (int o = 0; o < kOut; ++o) {
                if (o < nout) {
                    const float *e = ell[jj];
                    float w;
                    if (DL) {
                        const float ex = e[ia[o]], ey = e[r1 + ib[o]], ez = e[2 * r1 + ic[o]];
                        w = fmaf(e[3 * r1 + ia[o]], ey * ez, fmaf(ex, e[4 * r1 + ib[o]] * ez, ex * ey * e[5 * r1 + ic[o]]));
                    } else {
                        w = e[ia[o]] * e[r1 + ib[o]] * e[2 * r1 + ic[o]];
                    }
                    acc[o].x = fmaf(w, uu.x, acc[o].x);
                    acc[o].y = fmaf(w, uu.y, acc[o].y);
                }
            }
        }
    }
    float2 *ut = d.ut2 + (int64_t)b * rp;
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
        const int i = tid + o * kThreads;
        if (o < nout && i < rp) ut[i] = (i < r) ? acc[o] : make_float2(0.f, 0.f);
    }
    for (int i = r + tid; i < rp; i += kThreads) ut[i] = make_float2(0.f, 0.f);
}

template <bool DL>
__device__ __forceinline__ void lag_anterp_body(const LDesc &d, const int4 wk) {
    __shared__ float ell[kAnterpChunk][(DL ? 6 : 3) * kMaxR1];
    __shared__ float2 us[kAnterpChunk];
    __shared__ float nodes[kMaxR1], den[kMaxR1];
    // the node count as a compile-time constant: the basis loops unroll and the outputs per thread are fixed
    switch (d.r1) {
        case 1: lag_anterp_r1<DL, 1>(d, wk, ell, us, nodes, den); break;
        case 2: lag_anterp_r1<DL, 2>(d, wk, ell, us, nodes, den); break;
        case 3: lag_anterp_r1<DL, 3>(d, wk, ell, us, nodes, den); break;
        case 4: lag_anterp_r1<DL, 4>(d, wk, ell, us, nodes, den); break;
        case 5: lag_anterp_r1<DL, 5>(d, wk, ell, us, nodes, den); break;
        case 6: lag_anterp_r1<DL, 6>(d, wk, ell, us, nodes, den); break;
        case 7: lag_anterp_r1<DL, 7>(d, wk, ell, us, nodes, den); break;
        default: lag_anterp_r1<DL, 8>(d, wk, ell, us, nodes, den); break;
    }
}

__global__ void __launch_bounds__(kThreads)
k_lag_anterp(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    lag_anterp_body<false>(descs[wk.x], wk);
}

__global__ void __launch_bounds__(kThreads)
k_lag_anterp_dl(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    lag_anterp_body<true>(descs[wk.x], wk);
}

// U[k][2m + part] = part of u~_{s_m}[k] for the 16 pairs m of a class group (zero where the slot is empty): both
// parts of an entry come from one 8-byte load, and each thread issues eight loads before it writes them to LDS.
__device__ __forceinline__ void stage_group_sources(const float2 *ut2, const int *ps, int rp, float *U) {
    const int nel = rp * 16, nth = blockDim.x, tid = threadIdx.x;
    const gc2 src = gl(ut2);
    for (int base = 0; base < nel; base += 8 * nth) {
        v2f w[8];
        int sm[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sm[u] = ps[(base + u * nth + tid) & 15];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * nth + tid, k = idx >> 4;
            w[u] = v2f{0.f, 0.f};
            if (idx < nel && sm[u] >= 0) w[u] = src[(int64_t)sm[u] * rp + k];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * nth + tid;
            if (idx < nel) {
                U[2 * idx] = w[u].x;
                U[2 * idx + 1] = w[u].y;
            }
        }
    }
}

// Transfer products of one class group on MFMA: Z_e = T_c u~_{s(e)} for up to 16 pairs e.
// C (rp x 32) = T_c (rp x rp) x U (rp x 32), U[k][2m + part] = part of u~_{s(e_m)}[k].
// v_mfma_f32_32x32x2f32 operands: A[i][k] from lane i + 32 k, B[k][j] from lane j + 32 k,
// D[i][j] in lane j + 32 ((i / 4) % 2), register (i % 4) + 4 (i / 8).  Item (desc, group).
__global__ void __launch_bounds__(256)
k_lag_mfma(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    extern __shared__ float U[];   // [rp][32]
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int g = wk.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
    const int rp = d.rp, helm = d.helm;
    const int c = d.grp_cls[g];
    __shared__ int pe[16], ps[16];
    if (tid < 16) {
        const int e = d.grp_pair[(int64_t)g * 16 + tid];
        pe[tid] = e;
        ps[tid] = e >= 0 ? d.far_src[e] : -1;
    }
    __syncthreads();
    stage_group_sources(d.ut2, ps, rp, U);
    __syncthreads();
    const int64_t per = (int64_t)rp * rp;
    const float *Tre = d.T + (int64_t)c * (helm ? 2 : 1) * per;
    const float *Tim = Tre + per;
    const int col = lane & 31, kh = lane >> 5;
    const int e = pe[col >> 1];
    for (int mt = wv; mt < rp / 32; mt += nwv) {   // the waves share the staged sources, one row tile each
        floatx16 acc1, acc2;
        for (int v = 0; v < 16; ++v) {
            acc1[v] = 0.f;
            acc2[v] = 0.f;
        }
        // groups of four steps (rp / 2 is a multiple of 16): the group's operands are loaded before its
        // products, through global-address-space views of T
        const gcf TreG = gfl(Tre) + mt * 32 + col, TimG = gfl(Tim) + mt * 32 + col;
        // groups of four steps, double-buffered: the next group's T loads are issued before this group's
        // products (rp / 2 is a multiple of 16)
        float a1n[4], a2n[4];
        auto load = [&](int kk0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 2 * (kk0 + u) + kh;
                a1n[u] = TreG[(int64_t)k * rp];
                a2n[u] = 0.f;
                if (helm) a2n[u] = TimG[(int64_t)k * rp];   // Laplace tables have no imaginary part
            }
        };
        load(0);
        for (int kk0 = 0; kk0 < rp / 2; kk0 += 4) {
            float bv[4], a1[4], a2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bv[u] = U[(2 * (kk0 + u) + kh) * 32 + col];
                a1[u] = a1n[u];
                a2[u] = a2n[u];
            }
            if (kk0 + 4 < rp / 2) load(kk0 + 4);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[u], bv[u], acc1, 0, 0, 0);
                if (helm) acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[u], bv[u], acc2, 0, 0, 0);
            }
        }
        for (int v = 0; v < 16; ++v) {
            const int i = mt * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            float val = acc1[v];
            if (helm) {
                const float sw = __shfl_xor(acc2[v], 1, 64);
                val = (col & 1) ? val + sw : val - sw;
            }
            if (e >= 0) reinterpret_cast<float *>(d.Z + (int64_t)e * rp + i)[col & 1] = val;
        }
    }
}

// Transfer of one class group through the ACA factors of its class (Sec. 2.2.2, eq. ffmACAmatvec): Z_e =
// A_c (B_c^T u~_{s(e)}) for up to 16 pairs e, two products on MFMA with the operand layouts of k_lag_mfma.
// Phase 1: Y (kp x 32) = B_c^T (kp x rp) U (rp x 32): the class's padded rank kp is at most one 32-row tile per
// wave (the planner keeps kp <= 32 x waves), and each tile's K steps are split over the waves left, their
// partial tiles added in LDS in a fixed order; phase 2, once every wave has read U: Y is written over U in LDS
// and C (rp x 32) = A_c (rp x kp) Y.  Complex factors are two planes, and the complex products are formed from the
// real and imaginary columns as in k_lag_mfma.  Item (desc, group).
__global__ void __launch_bounds__(256)
k_lag_aca(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    extern __shared__ float U[];   // [rp][32], then Y [kp][32]
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int g = wk.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
    const int rp = d.rp, helm = d.helm, kpm = d.kpm;
    const int c = d.grp_cls[g];
    const int kp = d.acaKp[c];
    __shared__ int pe[16], ps[16];
    if (tid < 16) {
        const int e = d.grp_pair[(int64_t)g * 16 + tid];
        pe[tid] = e;
        ps[tid] = e >= 0 ? d.far_src[e] : -1;
    }
    __syncthreads();
    stage_group_sources(d.ut2, ps, rp, U);
    __syncthreads();
    const int planes = helm ? 2 : 1;
    const int col = lane & 31, kh = lane >> 5;
    // phase 1: B^T U.  The kp / 32 rank tiles times nparts ranges of the K steps go to the waves (every wave
    // busy when kp is one or two tiles); each range is a multiple of four steps, the last takes the rest
    const int ntile = kp / 32, nparts = nwv / ntile, steps = rp / 2;
    const int mt1 = wv % ntile, part = wv / ntile;
    const bool active = part < nparts;
    const int chunk = (steps / nparts) / 4 * 4;
    const int k0 = part * chunk, k1 = part == nparts - 1 ? steps : k0 + chunk;
    floatx16 y;
    if (active) {
        const float *Bre = d.acaB + (int64_t)c * planes * rp * kpm;
        const float *Bim = Bre + (int64_t)rp * kpm;
        const gcf BreG = gfl(Bre) + mt1 * 32 + col, BimG = gfl(Bim) + mt1 * 32 + col;
        floatx16 acc1, acc2;
        for (int v = 0; v < 16; ++v) {
            acc1[v] = 0.f;
            acc2[v] = 0.f;
        }
        float a1n[4], a2n[4];
        auto load = [&](int kk0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 2 * (kk0 + u) + kh;
                a1n[u] = BreG[(int64_t)k * kpm];
                a2n[u] = 0.f;
                if (helm) a2n[u] = BimG[(int64_t)k * kpm];
            }
        };
        load(k0);
        for (int kk0 = k0; kk0 < k1; kk0 += 4) {
            float bv[4], a1[4], a2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bv[u] = U[(2 * (kk0 + u) + kh) * 32 + col];
                a1[u] = a1n[u];
                a2[u] = a2n[u];
            }
            if (kk0 + 4 < k1) load(kk0 + 4);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[u], bv[u], acc1, 0, 0, 0);
                if (helm) acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[u], bv[u], acc2, 0, 0, 0);
            }
        }
        for (int v = 0; v < 16; ++v) {
            float val = acc1[v];
            if (helm) {
                const float sw = __shfl_xor(acc2[v], 1, 64);
                val = (col & 1) ? val + sw : val - sw;
            }
            y[v] = val;
        }
    }
    __syncthreads();              // every wave is done with U: its space holds the partial tiles, then Y
    if (active)
        for (int v = 0; v < 16; ++v)
            U[(part * ntile + mt1) * 1024 + (8 * (v >> 2) + 4 * kh + (v & 3)) * 32 + col] = y[v];
    __syncthreads();
    float ys[16];                 // kp x 32 entries of Y, at most 16 per thread; partial tiles added in order
    int ny = 0;
    for (int e = tid; e < kp * 32; e += blockDim.x, ++ny) {
        const int tile = e >> 10, within = e & 1023;
        float acc = 0.f;
        for (int q = 0; q < nparts; ++q) acc += U[(q * ntile + tile) * 1024 + within];
        ys[ny] = acc;
    }
    __syncthreads();
    ny = 0;
    for (int e = tid; e < kp * 32; e += blockDim.x, ++ny) U[e] = ys[ny];
    __syncthreads();
    // phase 2: A Y
    const float *Are = d.acaA + (int64_t)c * planes * kpm * rp;
    const float *Aim = Are + (int64_t)kpm * rp;
    const int e = pe[col >> 1];
    for (int mt = wv; mt < rp / 32; mt += nwv) {
        floatx16 acc1, acc2;
        for (int v = 0; v < 16; ++v) {
            acc1[v] = 0.f;
            acc2[v] = 0.f;
        }
        const gcf AreG = gfl(Are) + mt * 32 + col, AimG = gfl(Aim) + mt * 32 + col;
        float a1n[4], a2n[4];
        auto load = [&](int kk0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 2 * (kk0 + u) + kh;
                a1n[u] = AreG[(int64_t)k * rp];
                a2n[u] = 0.f;
                if (helm) a2n[u] = AimG[(int64_t)k * rp];
            }
        };
        load(0);
        for (int kk0 = 0; kk0 < kp / 2; kk0 += 4) {
            float bv[4], a1[4], a2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bv[u] = U[(2 * (kk0 + u) + kh) * 32 + col];
                a1[u] = a1n[u];
                a2[u] = a2n[u];
            }
            if (kk0 + 4 < kp / 2) load(kk0 + 4);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[u], bv[u], acc1, 0, 0, 0);
                if (helm) acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[u], bv[u], acc2, 0, 0, 0);
            }
        }
        for (int v = 0; v < 16; ++v) {
            const int i = mt * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            float val = acc1[v];
            if (helm) {
                const float sw = __shfl_xor(acc2[v], 1, 64);
                val = (col & 1) ? val + sw : val - sw;
            }
            if (e >= 0) reinterpret_cast<float *>(d.Z + (int64_t)e * rp + i)[col & 1] = val;
        }
    }
}

// Mixed precision: the same class-group products on FP16 MFMA (v_mfma_f32_32x32x16_f16, K = 16 per
// instruction) with FP32 accumulation.  A[i][k] comes from lane i + 32 (k / 8) (element k % 8 of a half8),
// B[k][j] from lane j + 32 (k / 8); D as for the FP32 instruction.  T16 = T * sT (plan time); the sources are scaled by a
// power of two s_u derived on the device from max |u| so that |u~ s_u| < 6e4; Z = C / (sT s_u).
__device__ __forceinline__ float u_scale(float amax, int maxpts) {
    // |u~| <= (Lebesgue constant of the tensor grid, <= 8) * points * max|u|
    const float bound = 8.f * (float)maxpts * fmaxf(amax, 1e-30f);
    return exp2f(floorf(log2f(6.0e4f / bound)));
}

__global__ void __launch_bounds__(256)
k_lag_mfma16(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    extern __shared__ _Float16 U16[];   // [32][rp]: column-major tile, k contiguous
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int g = wk.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
    const int rp = d.rp, helm = d.helm;
    const int c = d.grp_cls[g];
    const float su = u_scale(*d.amax, d.maxpts);
    __shared__ int pe[16], ps[16];
    if (tid < 16) {
        const int e = d.grp_pair[(int64_t)g * 16 + tid];
        pe[tid] = e;
        ps[tid] = e >= 0 ? d.far_src[e] : -1;
    }
    __syncthreads();
    {
        // entry (m, k): both parts of u~_{s_m}[k] from one 8-byte load (consecutive threads, consecutive k), eight
        // loads in flight per thread before the LDS writes
        const int nel = rp * 16, nth = blockDim.x;
        const gc2 src = gl(d.ut2);
        for (int base = 0; base < nel; base += 8 * nth) {
            v2f w[8];
            int sm[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * nth + tid;
                sm[u] = idx < nel ? ps[idx / rp] : -1;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * nth + tid, m = idx / rp, k = idx - m * rp;
                w[u] = v2f{0.f, 0.f};
                if (sm[u] >= 0) w[u] = src[(int64_t)sm[u] * rp + k];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * nth + tid, m = idx / rp, k = idx - m * rp;
                if (idx < nel) {
                    U16[(2 * m) * rp + k] = (_Float16)(w[u].x * su);
                    U16[(2 * m + 1) * rp + k] = (_Float16)(w[u].y * su);
                }
            }
        }
    }
    __syncthreads();
    const int64_t per = (int64_t)rp * rp;
    const _Float16 *Tre = d.T16 + (int64_t)c * (helm ? 2 : 1) * per;
    const _Float16 *Tim = Tre + per;
    const int col = lane & 31, kh = lane >> 5;
    const int e = pe[col >> 1];
    const float inv = 1.f / (d.sT * su);
    for (int mt = wv; mt < rp / 32; mt += nwv) {   // the waves share the staged sources, one row tile each
        floatx16 acc1, acc2;
        for (int v = 0; v < 16; ++v) {
            acc1[v] = 0.f;
            acc2[v] = 0.f;
        }
        const int i = mt * 32 + col;
        // groups of two steps of 16 (rp is a multiple of 32), operands loaded before the group's products
        const gch8 TreG = (gch8) reinterpret_cast<const half8_t *>(Tre + (int64_t)i * rp + 8 * kh);
        const gch8 TimG = (gch8) reinterpret_cast<const half8_t *>(Tim + (int64_t)i * rp + 8 * kh);
        // double-buffered as in the FP32 kernel
        half8_t a1n[2], a2n[2];
        auto load = [&](int k00) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k0 = k00 + 16 * u;
                a1n[u] = TreG[k0 / 8];
                a2n[u] = a1n[u];
                if (helm) a2n[u] = TimG[k0 / 8];   // Laplace tables have no imaginary part
            }
        };
        load(0);
        for (int k00 = 0; k00 < rp; k00 += 32) {
            half8_t bv[2], a1[2], a2[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                bv[u] = *reinterpret_cast<const half8_t *>(U16 + col * rp + k00 + 16 * u + 8 * kh);
                a1[u] = a1n[u];
                a2[u] = a2n[u];
            }
            if (k00 + 32 < rp) load(k00 + 32);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[u], bv[u], acc1, 0, 0, 0);
                if (helm) acc2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a2[u], bv[u], acc2, 0, 0, 0);
            }
        }
        for (int v = 0; v < 16; ++v) {
            const int row = mt * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            float val = acc1[v];
            if (helm) {
                const float sw = __shfl_xor(acc2[v], 1, 64);
                val = (col & 1) ? val + sw : val - sw;
            }
            if (e >= 0) reinterpret_cast<float *>(d.Z + (int64_t)e * rp + row)[col & 1] = val * inv;
        }
    }
}

// R1 nodes per axis (a compile-time constant, so the basis arrays stay in registers with constant indices).
// v~_t = sum_{e in far(t)} Z_e in list order; the loads of eight entries are issued before their additions.
template <bool DN, int R1>
__device__ __forceinline__ void lag_interp_r1(const LDesc &d, const int4 wk, float2 *vt, const float *nodes,
                                              const float *den) {
    constexpr int r = R1 * R1 * R1;
    const int t = wk.y;
    const int tid = threadIdx.x;
    const int rp = d.rp;
    const double two_over_dl = d.two_over_dl;
    const int64_t e0 = d.far_ptr[t], e1 = d.far_ptr[t + 1];
    const gc2 Z = gl(d.Z);
    for (int i = tid; i < r; i += kThreads) {
        float ax = 0.f, ay = 0.f;
        int64_t e = e0;
        for (; e + 8 <= e1; e += 8) {
            v2f z[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) z[u] = Z[(e + u) * rp + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                ax += z[u].x;
                ay += z[u].y;
            }
        }
        for (; e < e1; ++e) {
            const v2f z = Z[e * rp + i];
            ax += z.x;
            ay += z.y;
        }
        vt[i] = make_float2(ax, ay);
    }
    __syncthreads();
    const double cx = d.tctr[3 * t], cy = d.tctr[3 * t + 1], cz = d.tctr[3 * t + 2];
    for (int i = d.tstart[t] + tid; i < d.tstart[t + 1]; i += kThreads) {
        float lx[R1], ly[R1], lz[R1];
        const float tx = (float)((d.txs[i] - cx) * two_over_dl), ty = (float)((d.tys[i] - cy) * two_over_dl);
        const float tz = (float)((d.tzs[i] - cz) * two_over_dl);
        lagrange_1d(tx, R1, nodes, den, lx);
        lagrange_1d(ty, R1, nodes, den, ly);
        lagrange_1d(tz, R1, nodes, den, lz);
        float sre = 0.f, sim = 0.f;
        if (DN) {
            // n . grad of the interpolant: (2 / d_l) (n_x l'_a l_b l_c + n_y l_a l'_b l_c + n_z l_a l_b l'_c) v~
            float dx[R1], dy[R1], dz[R1];
            lagrange_1d_deriv(tx, R1, nodes, den, dx);
            lagrange_1d_deriv(ty, R1, nodes, den, dy);
            lagrange_1d_deriv(tz, R1, nodes, den, dz);
            const float4 n = d.tn ? d.tn[i] : d.tnc;
#pragma unroll
            for (int a = 0; a < R1; ++a) {
                float b0r = 0.f, b0i = 0.f, b1r = 0.f, b1i = 0.f;
#pragma unroll
                for (int bb = 0; bb < R1; ++bb) {
                    float c0r = 0.f, c0i = 0.f, c1r = 0.f, c1i = 0.f;
                    const float2 *row = vt + (a * R1 + bb) * R1;
#pragma unroll
                    for (int c = 0; c < R1; ++c) {
                        c0r = fmaf(lz[c], row[c].x, c0r);
                        c0i = fmaf(lz[c], row[c].y, c0i);
                        c1r = fmaf(dz[c], row[c].x, c1r);
                        c1i = fmaf(dz[c], row[c].y, c1i);
                    }
                    b0r = fmaf(ly[bb], c0r, b0r);      // l_b l_c
                    b0i = fmaf(ly[bb], c0i, b0i);
                    b1r = fmaf(n.y * dy[bb], c0r, fmaf(n.z * ly[bb], c1r, b1r));   // n_y l'_b l_c + n_z l_b l'_c
                    b1i = fmaf(n.y * dy[bb], c0i, fmaf(n.z * ly[bb], c1i, b1i));
                }
                sre = fmaf(n.x * dx[a], b0r, fmaf(lx[a], b1r, sre));
                sim = fmaf(n.x * dx[a], b0i, fmaf(lx[a], b1i, sim));
            }
            const float f = (float)two_over_dl;
            sre *= f;
            sim *= f;
        } else {
#pragma unroll
            for (int a = 0; a < R1; ++a) {
                float bre = 0.f, bim = 0.f;
#pragma unroll
                for (int bb = 0; bb < R1; ++bb) {
                    float cre = 0.f, cim = 0.f;
                    const float2 *row = vt + (a * R1 + bb) * R1;
#pragma unroll
                    for (int c = 0; c < R1; ++c) {
                        cre = fmaf(lz[c], row[c].x, cre);
                        cim = fmaf(lz[c], row[c].y, cim);
                    }
                    bre = fmaf(ly[bb], cre, bre);
                    bim = fmaf(ly[bb], cim, bim);
                }
                sre = fmaf(lx[a], bre, sre);
                sim = fmaf(lx[a], bim, sim);
            }
        }
        float2 o = d.v[i];
        o.x += sre;
        o.y += sim;
        d.v[i] = o;
    }
}

template <bool DN>
__device__ __forceinline__ void lag_interp_body(const LDesc &d, const int4 wk) {
    extern __shared__ float2 vt[];   // [r]
    __shared__ float nodes[kMaxR1], den[kMaxR1];
    const int tid = threadIdx.x;
    if (tid < d.r1) {
        nodes[tid] = d.lnodes[tid];
        den[tid] = d.lden[tid];
    }
    // (the reduction into vt below does not read nodes or den; the barrier after it orders their writes)
    switch (d.r1) {
        case 1: lag_interp_r1<DN, 1>(d, wk, vt, nodes, den); break;
        case 2: lag_interp_r1<DN, 2>(d, wk, vt, nodes, den); break;
        case 3: lag_interp_r1<DN, 3>(d, wk, vt, nodes, den); break;
        case 4: lag_interp_r1<DN, 4>(d, wk, vt, nodes, den); break;
        case 5: lag_interp_r1<DN, 5>(d, wk, vt, nodes, den); break;
        case 6: lag_interp_r1<DN, 6>(d, wk, vt, nodes, den); break;
        case 7: lag_interp_r1<DN, 7>(d, wk, vt, nodes, den); break;
        default: lag_interp_r1<DN, 8>(d, wk, vt, nodes, den); break;
    }
}

// v_i += L_X^T v~_t (or its normal derivative at x_i, k_lag_interp_dn) with v~_t = sum_{e in far(t)} Z_e (fixed
// order), t = 2 (x - c_t) / d_l.  Item (desc, target box).
__global__ void __launch_bounds__(kThreads)
k_lag_interp(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    lag_interp_body<false>(descs[wk.x], wk);
}

__global__ void __launch_bounds__(kThreads)
k_lag_interp_dn(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    lag_interp_body<true>(descs[wk.x], wk);
}

// ------------------------------------------------------------------ near field (leaf)
// v_i += sum_{s in near(t)} sum_{j in s, r_ij > 0} G(r_ij) u_j.  One 64-lane block per target box.  Source points
// are staged through LDS in chunks of 64, in FP64 relative to the target centre, and every pair's difference is
// formed in FP64 and rounded once to FP32, so close pairs keep the full FP32 relative accuracy of r.  Helmholtz
// coordinates are scaled by k / 2 pi when staged (r then reads in revolutions, the phase of e^{ikr}), and the
// factors that scaling takes out of 1/r (and of the derivative's 1/r^3) go into the staged u.
//
// Targets go through the lanes in passes.  A pass of nt targets gives each lane T of them (T = 1, 2 or 4: g =
// ceil(nt / T) target groups, group gi holding targets gi, gi + g, ...) and gives each group R = 64 / g lanes;
// lane r of a group takes the contiguous range r * steps ... r * steps + steps - 1 of the chunk's staged sources
// (steps = ceil(cnt / R); staged slots past the chunk hold zero sources).  A lane evaluates every staged source
// against its T targets, so one set of LDS reads serves T pairs.  The R partial sums of a target are added in
// order of r.  The pass sizes come from the box's target count alone, so the summation order is fixed.
// Ranges of consecutive lanes start an odd number of 8-byte slots apart (slot r * (steps | 1) + q), so the R
// distinct addresses of one read fall in distinct banks.  The r > 0 test runs only where coincident points can
// occur: a box against itself when sources and targets are one set, every pair otherwise.
constexpr int kNearSlots = 128;

struct NearPass {
    int nt, T;
};

// Pass sizes for rem remaining targets: a full pass (64 m targets, m = 1, 2, 4, four per lane on 4 / m lanes
// each) is taken while it beats a single partial pass over everything left; cost = pairs per lane per staged
// source.  Equal costs go to four targets per lane, whose LDS reads serve four pairs.
__device__ __forceinline__ float near_pass_cost(int n, int T) {
    const int g = (n + T - 1) / T;
    return g > 64 ? 1e30f : (float)T / (float)(64 / g);
}

__device__ __forceinline__ NearPass near_next_pass(int rem) {
    float best = 1e30f;
    int bt = 1;
    for (int T = 1; T <= 4; T *= 2) {
        const float c = near_pass_cost(rem, T);
        if (c <= best) {
            best = c;
            bt = T;
        }
    }
    NearPass out{rem, bt};
    for (int m = 4; m >= 1; m /= 2) {
        const int full = 64 * m;
        if (rem <= full) continue;
        float rest = 1e30f;
        for (int T2 = 1; T2 <= 4; T2 *= 2) rest = fminf(rest, near_pass_cost(rem - full, T2));
        if (rest > 1e29f) rest = (float)((rem - full + 255) / 256) * 4.f;   // more full passes follow
        if ((float)m + rest < best) {
            best = (float)m + rest;
            out = NearPass{full, 4};
        }
    }
    return out;
}

struct NearSmem {
    double x[kNearSlots], y[kNearSlots], z[kNearSlots];   // part[] reuses x and y after the last chunk
    float2 u[kNearSlots];
    float2 sp[kNearSlots];                                 // source-side sums of a chunk (symmetric pairs)
};

// Stage the chunk's sources c0 ... c0 + cnt - 1 (relative to the target centre, scaled) for R lane rows of
// `steps` sources each: source jj at slot (jj / steps) * so + jj % steps, zero sources in the slots of
// cnt <= jj < R * steps (at most 127).  d.two_over_dl is 2 / d_l of the descriptor's level.  With snm, the
// source normals nsrc[j] times nsign go to snm[slot] (the double layer stages the negated source normals:
// n_y . grad_y G(x - y) = (-n_y) . grad_x G(x - y)).
__device__ __forceinline__ void near_stage_chunk(const LDesc &d, NearSmem &sm, int c0, int cnt, int R, int steps,
                                                 int so, double cx, double cy, double cz, double scale,
                                                 float uscale, float4 *snm, const float4 *nsrc = nullptr,
                                                 float nsign = -1.f) {
    const int lane = threadIdx.x;
    // zero sources sit at (2, 2, 2) d_l from the target centre: no target is there (each lies within d_l / 2 of
    // its centre on every axis), so every pair with them has r > 0 and adds exactly zero, and their phases stay
    // within the bound of the level's near pairs
    const double pad = 4.0 / d.two_over_dl * scale;
    const uint32_t mul = (65536u + (uint32_t)steps - 1u) / (uint32_t)steps;   // jj / steps for jj < 128
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int jj = lane + 64 * h;
        if (jj < R * steps) {
            const int qd = (int)(((uint32_t)jj * mul) >> 16);
            const int slot = qd * so + (jj - qd * steps);
            if (jj < cnt) {
                const int j = c0 + jj;
                sm.x[slot] = (d.sxs[j] - cx) * scale;
                sm.y[slot] = (d.sys[j] - cy) * scale;
                sm.z[slot] = (d.szs[j] - cz) * scale;
                const float2 uu = d.u[j];
                sm.u[slot] = make_float2(uu.x * uscale, uu.y * uscale);
                if (snm) {
                    const float4 n = nsrc[j];
                    snm[slot] = make_float4(nsign * n.x, nsign * n.y, nsign * n.z, 0.f);
                }
            } else {
                sm.x[slot] = sm.y[slot] = sm.z[slot] = pad;   // padding: zero sources
                sm.u[slot] = make_float2(0.f, 0.f);
                if (snm) snm[slot] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    }
    __syncthreads();
}

template <bool HELM, bool DN, bool BIG, bool CHK>
__device__ __forceinline__ void near_pair(double x, double y, double z, float nx, float ny, float nz, double sx,
                                          double sy, double sz, float2 uu, float &are, float &aim) {
    const float dx = (float)(x - sx), dy = (float)(y - sy), dz = (float)(z - sz);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float inv = __builtin_amdgcn_rsqf(r2);
    if (CHK) inv = r2 > 0.f ? inv : 0.f;
    if (DN) {
        // n . grad_x G: (n . d) G'(r) / r with G' = -1 / r^2 (Laplace), (ikr - 1) e^{ikr} / r^2 (Helmholtz)
        const float i3 = inv * inv * inv * fmaf(nx, dx, fmaf(ny, dy, nz * dz));
        if (HELM) {
            const float rr = r2 * inv;
            float sn, cs;
            sincos_rev(BIG ? __builtin_amdgcn_fractf(rr) : rr, sn, cs);
            const float kr = 6.2831853f * rr;
            const float gr = i3 * fmaf(-kr, sn, -cs), gi = i3 * fmaf(kr, cs, -sn);
            are = fmaf(gr, uu.x, fmaf(-gi, uu.y, are));
            aim = fmaf(gr, uu.y, fmaf(gi, uu.x, aim));
        } else {
            are = fmaf(-i3, uu.x, are);
            aim = fmaf(-i3, uu.y, aim);
        }
    } else if (HELM) {
        const float rr = r2 * inv;
        float sn, cs;
        sincos_rev(BIG ? __builtin_amdgcn_fractf(rr) : rr, sn, cs);
        const float gr = cs * inv, gi = sn * inv;
        are = fmaf(gr, uu.x, fmaf(-gi, uu.y, are));
        aim = fmaf(gr, uu.y, fmaf(gi, uu.x, aim));
    } else {
        are = fmaf(inv, uu.x, are);
        aim = fmaf(inv, uu.y, aim);
    }
}

// One staged source against the lane's T targets.  NRM: 0 the kernel itself, 1 the normal derivative at the
// targets (their normals in nx, ny, nz), 2 at the sources (the staged negated normal of slot s).
template <bool HELM, int NRM, bool BIG, bool CHK, int T>
__device__ __forceinline__ void near_source(const NearSmem &sm, const float4 *snm, int s, const double (&x)[T],
                                            const double (&y)[T], const double (&z)[T], const float (&nx)[T],
                                            const float (&ny)[T], const float (&nz)[T], float (&are)[T],
                                            float (&aim)[T]) {
    const double sx = sm.x[s], sy = sm.y[s], sz = sm.z[s];
    const float2 uu = sm.u[s];
    if (NRM == 2) {
        const float4 n = snm[s];
#pragma unroll
        for (int t = 0; t < T; ++t)
            near_pair<HELM, true, BIG, CHK>(x[t], y[t], z[t], n.x, n.y, n.z, sx, sy, sz, uu, are[t], aim[t]);
    } else {
#pragma unroll
        for (int t = 0; t < T; ++t)
            near_pair<HELM, NRM == 1, BIG, CHK>(x[t], y[t], z[t], nx[t], ny[t], nz[t], sx, sy, sz, uu, are[t], aim[t]);
    }
}

// steps staged sources from slot base against the lane's T targets
template <bool HELM, int NRM, bool BIG, bool CHK, int T>
__device__ __forceinline__ void near_range(const NearSmem &sm, const float4 *snm, int base, int steps,
                                           const double (&x)[T], const double (&y)[T], const double (&z)[T],
                                           const float (&nx)[T], const float (&ny)[T], const float (&nz)[T],
                                           float (&are)[T], float (&aim)[T]) {
    constexpr int U = T >= 4 ? 1 : 4 / T;
    int q = 0;
    for (; q + U <= steps; q += U) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            near_source<HELM, NRM, BIG, CHK, T>(sm, snm, base + q + u, x, y, z, nx, ny, nz, are, aim);
    }
    for (; q < steps; ++q) near_source<HELM, NRM, BIG, CHK, T>(sm, snm, base + q, x, y, z, nx, ny, nz, are, aim);
}

// One pass: targets i0 ... i0 + nt - 1 of box t, T per lane.
template <bool HELM, int NRM, bool BIG, int T>
__device__ __forceinline__ void near_pass(const LDesc &d, NearSmem &sm, float4 *snm, int t, int i0, int nt,
                                          double scale, float uscale) {
    const int lane = threadIdx.x;
    const int g = __builtin_amdgcn_readfirstlane((nt + T - 1) / T), R = __builtin_amdgcn_readfirstlane(64 / g);
    const int r = lane / g, gi = lane - r * g;
    const bool valid = r < R;
    const double cx = d.tctr[3 * t], cy = d.tctr[3 * t + 1], cz = d.tctr[3 * t + 2];
    double x[T], y[T], z[T];
    float nx[T], ny[T], nz[T], are[T], aim[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int ti = gi + g * k;
        x[k] = y[k] = z[k] = 0.0;
        nx[k] = ny[k] = nz[k] = 0.f;
        are[k] = aim[k] = 0.f;
        if (valid && ti < nt) {
            const int i = i0 + ti;
            x[k] = (d.txs[i] - cx) * scale;
            y[k] = (d.tys[i] - cy) * scale;
            z[k] = (d.tzs[i] - cz) * scale;
            if (NRM == 1) {
                const float4 n = d.tn ? d.tn[i] : d.tnc;
                nx[k] = n.x;
                ny[k] = n.y;
                nz[k] = n.z;
            }
        }
    }
    const int64_t e0 = d.near_ptr[t], e1 = d.near_ptr[t + 1];
    const bool same = d.same != 0;
    for (int64_t e = e0; e < e1; ++e) {
        const int s = __builtin_amdgcn_readfirstlane(d.near_src[e]);
        const int j0 = __builtin_amdgcn_readfirstlane(d.sstart[s]), j1 = __builtin_amdgcn_readfirstlane(d.sstart[s + 1]);
        const bool chk = !same || s == t;
        for (int c0 = j0; c0 < j1; c0 += 64) {
            const int cnt = min(64, j1 - c0);
            const int steps = __builtin_amdgcn_readfirstlane((cnt + R - 1) / R), so = steps | 1;
            near_stage_chunk(d, sm, c0, cnt, R, steps, so, cx, cy, cz, scale, uscale, NRM == 2 ? snm : nullptr, d.sn);
            const int base = valid ? r * so : 0;     // idle lanes read staged slots and discard their sums
            if (chk)
                near_range<HELM, NRM, BIG, true, T>(sm, snm, base, steps, x, y, z, nx, ny, nz, are, aim);
            else
                near_range<HELM, NRM, BIG, false, T>(sm, snm, base, steps, x, y, z, nx, ny, nz, are, aim);
        }
    }
    // the R partial sums of each target, added in order of r
    float2 *part = reinterpret_cast<float2 *>(sm.x);   // [T][64], over x and y
    __syncthreads();
#pragma unroll
    for (int k = 0; k < T; ++k) part[k * 64 + lane] = make_float2(are[k], aim[k]);
    __syncthreads();
    if (lane < g) {
#pragma unroll
        for (int k = 0; k < T; ++k) {
            const int ti = lane + g * k;
            if (ti >= nt) break;
            float2 a = part[k * 64 + lane];
            for (int rr = 1; rr < R; ++rr) {
                const float2 b = part[k * 64 + lane + rr * g];
                a.x += b.x;
                a.y += b.y;
            }
            float2 o = d.v[i0 + ti];
            o.x += a.x;
            o.y += a.y;
            d.v[i0 + ti] = o;
        }
    }
}

template <bool HELM, int NRM, bool BIG>
__device__ __forceinline__ void near_body(const LDesc &d, const int4 wk) {
    __shared__ NearSmem sm;
    __shared__ float4 snm[NRM == 2 ? kNearSlots : 1];   // staged source normals (double layer)
    const int t = wk.y;
    const int ta = d.tstart[t], tz = d.tstart[t + 1];
    // Helmholtz: coordinates in units of 2 pi / k; 1/r = (k / 2 pi) / r', 1/r^3 = (k / 2 pi)^3 / r'^3 and
    // n . d = (2 pi / k) n . d'
    const double kr = (double)d.k_rev;
    const double scale = HELM ? kr : 1.0;
    const float uscale = (float)((1.0 / (4.0 * M_PI)) * (HELM ? (NRM ? kr * kr : kr) : 1.0));
    for (int i0 = ta; i0 < tz;) {
        const NearPass ps = near_next_pass(tz - i0);
        if (ps.T == 1)
            near_pass<HELM, NRM, BIG, 1>(d, sm, snm, t, i0, ps.nt, scale, uscale);
        else if (ps.T == 2)
            near_pass<HELM, NRM, BIG, 2>(d, sm, snm, t, i0, ps.nt, scale, uscale);
        else
            near_pass<HELM, NRM, BIG, 4>(d, sm, snm, t, i0, ps.nt, scale, uscale);
        i0 += ps.nt;
    }
}

template <bool HELM, bool BIG>
__global__ void __launch_bounds__(64)
k_near(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    near_body<HELM, 0, BIG>(descs[wk.x], wk);
}

// The normal derivative at the target (the adjoint double-layer kernel), same blocks and lanes.
template <bool HELM, bool BIG>
__global__ void __launch_bounds__(64)
k_near_dn(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    near_body<HELM, 1, BIG>(descs[wk.x], wk);
}

// The normal derivative at the source (the double-layer kernel), same blocks and lanes.
template <bool HELM, bool BIG>
__global__ void __launch_bounds__(64)
k_near_dl(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    near_body<HELM, 2, BIG>(descs[wk.x], wk);
}

// The gradient at the targets: grad_x G(x - y) = d G'(r) / r, d = x - y.  The three components share r, 1/r^3
// and the phase; each component is formed as the normal derivative along its axis would form it (the same
// operations in the same order), so component c equals that pass with n = e_c.
template <bool HELM, bool BIG, bool CHK>
__device__ __forceinline__ void near_pair_grad(double x, double y, double z, double sx, double sy, double sz,
                                               float2 uu, float &ar0, float &ai0, float &ar1, float &ai1,
                                               float &ar2, float &ai2) {
    const float dx = (float)(x - sx), dy = (float)(y - sy), dz = (float)(z - sz);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float inv = __builtin_amdgcn_rsqf(r2);
    if (CHK) inv = r2 > 0.f ? inv : 0.f;
    const float i3 = inv * inv * inv;
    const float f0 = i3 * dx, f1 = i3 * dy, f2 = i3 * dz;
    if (HELM) {
        const float rr = r2 * inv;
        float sn, cs;
        sincos_rev(BIG ? __builtin_amdgcn_fractf(rr) : rr, sn, cs);
        const float kr = 6.2831853f * rr;
        const float hr = fmaf(-kr, sn, -cs), hi = fmaf(kr, cs, -sn);
        float gr = f0 * hr, gi = f0 * hi;
        ar0 = fmaf(gr, uu.x, fmaf(-gi, uu.y, ar0));
        ai0 = fmaf(gr, uu.y, fmaf(gi, uu.x, ai0));
        gr = f1 * hr;
        gi = f1 * hi;
        ar1 = fmaf(gr, uu.x, fmaf(-gi, uu.y, ar1));
        ai1 = fmaf(gr, uu.y, fmaf(gi, uu.x, ai1));
        gr = f2 * hr;
        gi = f2 * hi;
        ar2 = fmaf(gr, uu.x, fmaf(-gi, uu.y, ar2));
        ai2 = fmaf(gr, uu.y, fmaf(gi, uu.x, ai2));
    } else {
        ar0 = fmaf(-f0, uu.x, ar0);
        ai0 = fmaf(-f0, uu.y, ai0);
        ar1 = fmaf(-f1, uu.x, ar1);
        ai1 = fmaf(-f1, uu.y, ai1);
        ar2 = fmaf(-f2, uu.x, ar2);
        ai2 = fmaf(-f2, uu.y, ai2);
    }
}

// steps staged sources from slot base against the lane's T targets, three components each
template <bool HELM, bool BIG, bool CHK, int T>
__device__ __forceinline__ void near_range_grad(const NearSmem &sm, int base, int steps, const double (&x)[T],
                                                const double (&y)[T], const double (&z)[T], float (&ar)[3][T],
                                                float (&ai)[3][T]) {
    for (int q = 0; q < steps; ++q) {
        const int s = base + q;
        const double sx = sm.x[s], sy = sm.y[s], sz = sm.z[s];
        const float2 uu = sm.u[s];
#pragma unroll
        for (int t = 0; t < T; ++t)
            near_pair_grad<HELM, BIG, CHK>(x[t], y[t], z[t], sx, sy, sz, uu, ar[0][t], ai[0][t], ar[1][t], ai[1][t],
                                           ar[2][t], ai[2][t]);
    }
}

// One pass of the gradient near field: the lanes and sources of near_pass; component c of target i is added
// to output plane c (d.v + c n_x).
template <bool HELM, bool BIG, int T>
__device__ __forceinline__ void near_pass_grad(const LDesc &d, NearSmem &sm, int t, int i0, int nt, double scale,
                                               float uscale) {
    const int lane = threadIdx.x;
    const int g = __builtin_amdgcn_readfirstlane((nt + T - 1) / T), R = __builtin_amdgcn_readfirstlane(64 / g);
    const int r = lane / g, gi = lane - r * g;
    const bool valid = r < R;
    const double cx = d.tctr[3 * t], cy = d.tctr[3 * t + 1], cz = d.tctr[3 * t + 2];
    double x[T], y[T], z[T];
    float ar[3][T], ai[3][T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int ti = gi + g * k;
        x[k] = y[k] = z[k] = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) ar[c][k] = ai[c][k] = 0.f;
        if (valid && ti < nt) {
            const int i = i0 + ti;
            x[k] = (d.txs[i] - cx) * scale;
            y[k] = (d.tys[i] - cy) * scale;
            z[k] = (d.tzs[i] - cz) * scale;
        }
    }
    const int64_t e0 = d.near_ptr[t], e1 = d.near_ptr[t + 1];
    const bool same = d.same != 0;
    for (int64_t e = e0; e < e1; ++e) {
        const int s = __builtin_amdgcn_readfirstlane(d.near_src[e]);
        const int j0 = __builtin_amdgcn_readfirstlane(d.sstart[s]), j1 = __builtin_amdgcn_readfirstlane(d.sstart[s + 1]);
        const bool chk = !same || s == t;
        for (int c0 = j0; c0 < j1; c0 += 64) {
            const int cnt = min(64, j1 - c0);
            const int steps = __builtin_amdgcn_readfirstlane((cnt + R - 1) / R), so = steps | 1;
            near_stage_chunk(d, sm, c0, cnt, R, steps, so, cx, cy, cz, scale, uscale, nullptr);
            const int base = valid ? r * so : 0;     // idle lanes read staged slots and discard their sums
            if (chk)
                near_range_grad<HELM, BIG, true, T>(sm, base, steps, x, y, z, ar, ai);
            else
                near_range_grad<HELM, BIG, false, T>(sm, base, steps, x, y, z, ar, ai);
        }
    }
    // per component: the R partial sums of each target, added in order of r
    float2 *part = reinterpret_cast<float2 *>(sm.x);   // [T][64], over x and y
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < T; ++k) part[k * 64 + lane] = make_float2(ar[c][k], ai[c][k]);
        __syncthreads();
        if (lane < g) {
            float2 *vc = d.v + (int64_t)c * d.nx;
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const int ti = lane + g * k;
                if (ti >= nt) break;
                float2 a = part[k * 64 + lane];
                for (int rr = 1; rr < R; ++rr) {
                    const float2 b = part[k * 64 + lane + rr * g];
                    a.x += b.x;
                    a.y += b.y;
                }
                float2 o = vc[i0 + ti];
                o.x += a.x;
                o.y += a.y;
                vc[i0 + ti] = o;
            }
        }
    }
}

// The gradient at the targets, all three components in one pass over the near pairs.  Item (desc, target box).
template <bool HELM, bool BIG>
__global__ void __launch_bounds__(64)
k_near_grad(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    __shared__ NearSmem sm;
    const int t = wk.y;
    const int ta = d.tstart[t], tz = d.tstart[t + 1];
    const double kr = (double)d.k_rev;
    const double scale = HELM ? kr : 1.0;
    const float uscale = (float)((1.0 / (4.0 * M_PI)) * (HELM ? kr * kr : 1.0));
    for (int i0 = ta; i0 < tz;) {
        const NearPass ps = near_next_pass(tz - i0);
        if (ps.T == 1)
            near_pass_grad<HELM, BIG, 1>(d, sm, t, i0, ps.nt, scale, uscale);
        else if (ps.T == 2)
            near_pass_grad<HELM, BIG, 2>(d, sm, t, i0, ps.nt, scale, uscale);
        else
            near_pass_grad<HELM, BIG, 4>(d, sm, t, i0, ps.nt, scale, uscale);
        i0 += ps.nt;
    }
}

// ------------------------------------------------------------------ near field, one set (symmetric pairs)
// Sources and targets one set: G(x, y) = G(y, x), so an unordered pair of distinct neighbour boxes {t, s} is
// evaluated once, by the block of the lower box index: each pair's kernel value gives both v_i += G u_j (target
// side, in the lane's registers as above) and w_j += G u_i (source side).  The lanes form 4 rows of 16; a row
// holds 16 T targets (T = 1 ... 8 per lane, target slot gi + 16 k) and takes a contiguous range of the staged
// sources.  The source-side sums of a staged source over the row's 16 lanes are added in a fixed tree
// (data-parallel shifts within the row), and the chunk's sums are written, in order, to the entry's slice of a
// buffer (offset near_off[e]); passes after the first add to it.  The box itself (ordered, with the r > 0
// test) and lower neighbours without a reverse entry are evaluated as in k_near; lower neighbours with one are
// skipped here and added afterwards from the buffer by k_near_gather, in list order.  Passes hold up to 80
// targets (T <= 5: more targets per lane would cost registers, hence resident waves, more than they save).
template <int N>
__device__ __forceinline__ float dpp_row_shr(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 | N, 0xF, 0xF,
                                                                  true));
}

// inclusive sum over each 16-lane row: the row's total in its last lane
__device__ __forceinline__ float row_sum16(float v) {
    v += dpp_row_shr<1>(v);
    v += dpp_row_shr<2>(v);
    v += dpp_row_shr<4>(v);
    v += dpp_row_shr<8>(v);
    return v;
}

// nuy = -us.y and nty = -ut.y keep every product an FMA without a negation
template <bool HELM, bool BIG>
__device__ __forceinline__ void near_pair_sym(double x, double y, double z, float2 ut, float nty, double sx, double sy,
                                              double sz, float2 us, float nuy, float &are, float &aim, float &sre,
                                              float &sim) {
    const float dx = (float)(x - sx), dy = (float)(y - sy), dz = (float)(z - sz);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float inv = __builtin_amdgcn_rsqf(r2);   // distinct boxes of one set, padding far away: r > 0
    if (HELM) {
        const float rr = r2 * inv;
        float sn, cs;
        sincos_rev(BIG ? __builtin_amdgcn_fractf(rr) : rr, sn, cs);
        const float gr = cs * inv, gi = sn * inv;
        are = fmaf(gi, nuy, fmaf(gr, us.x, are));
        aim = fmaf(gi, us.x, fmaf(gr, us.y, aim));
        sre = fmaf(gi, nty, fmaf(gr, ut.x, sre));
        sim = fmaf(gi, ut.x, fmaf(gr, ut.y, sim));
    } else {
        are = fmaf(inv, us.x, are);
        aim = fmaf(inv, us.y, aim);
        sre = fmaf(inv, ut.x, sre);
        sim = fmaf(inv, ut.y, sim);
    }
}

template <bool HELM, bool BIG, int T>
__device__ __forceinline__ void near_pass_sym(const LDesc &d, NearSmem &sm, int t, int i0, int nt, bool first,
                                              double scale, float uscale) {
    constexpr int g = 16, R = 4;
    const int lane = threadIdx.x;
    const int r = lane >> 4, gi = lane & 15;
    const bool last = gi == g - 1;
    const double cx = d.tctr[3 * t], cy = d.tctr[3 * t + 1], cz = d.tctr[3 * t + 2];
    double x[T], y[T], z[T];
    float nx[T], ny[T], nz[T], are[T], aim[T], nty[T];
    float2 ut[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        // a slot past nt repeats target 0 with zero input: its source-side terms are zero, its own sums discarded
        const int ti = gi + g * k;
        const int i = i0 + (ti < nt ? ti : 0);
        x[k] = (d.txs[i] - cx) * scale;
        y[k] = (d.tys[i] - cy) * scale;
        z[k] = (d.tzs[i] - cz) * scale;
        nx[k] = ny[k] = nz[k] = 0.f;
        are[k] = aim[k] = 0.f;
        const float2 uu = d.u[i];
        ut[k] = ti < nt ? make_float2(uu.x * uscale, uu.y * uscale) : make_float2(0.f, 0.f);
        nty[k] = -ut[k].y;
    }
    const int64_t e0 = d.near_ptr[t], e1 = d.near_ptr[t + 1];
    for (int64_t e = e0; e < e1; ++e) {
        const int s = __builtin_amdgcn_readfirstlane(d.near_src[e]);
        const int64_t off = d.near_off[e];
        if (s < t && off >= 0) continue;          // the block of box s evaluates this pair of boxes
        const int j0 = __builtin_amdgcn_readfirstlane(d.sstart[s]), j1 = __builtin_amdgcn_readfirstlane(d.sstart[s + 1]);
        for (int c0 = j0; c0 < j1; c0 += 64) {
            const int cnt = min(64, j1 - c0);
            const int steps = __builtin_amdgcn_readfirstlane((cnt + R - 1) / R), so = steps | 1;
            near_stage_chunk(d, sm, c0, cnt, R, steps, so, cx, cy, cz, scale, uscale, nullptr);
            const int base = r * so;
            if (s == t) {
                near_range<HELM, 0, BIG, true, T>(sm, nullptr, base, steps, x, y, z, nx, ny, nz, are, aim);
            } else if (s < t) {
                near_range<HELM, 0, BIG, false, T>(sm, nullptr, base, steps, x, y, z, nx, ny, nz, are, aim);
            } else {
                const int jb = r * steps;
                for (int q = 0; q < steps; ++q) {
                    const int sl = base + q;
                    const double sx = sm.x[sl], sy = sm.y[sl], sz = sm.z[sl];
                    const float2 us = sm.u[sl];
                    const float nuy = -us.y;
                    float sre = 0.f, sim = 0.f;
#pragma unroll
                    for (int k = 0; k < T; ++k)
                        near_pair_sym<HELM, BIG>(x[k], y[k], z[k], ut[k], nty[k], sx, sy, sz, us, nuy, are[k], aim[k],
                                                 sre, sim);
                    sre = row_sum16(sre);
                    sim = row_sum16(sim);
                    if (last) sm.sp[jb + q] = make_float2(sre, sim);   // slots past cnt are never read
                }
                __syncthreads();
                if (lane < cnt) {
                    float2 *o = d.nsym + off + (c0 - j0) + lane;
                    float2 a = sm.sp[lane];
                    if (!first) {
                        const float2 b = *o;
                        a.x += b.x;
                        a.y += b.y;
                    }
                    *o = a;
                }
            }
        }
    }
    float2 *part = reinterpret_cast<float2 *>(sm.x);   // [T][64] over x, y, z and u (T <= 5)
    __syncthreads();
#pragma unroll
    for (int k = 0; k < T; ++k) part[k * 64 + lane] = make_float2(are[k], aim[k]);
    __syncthreads();
    if (lane < g) {
#pragma unroll
        for (int k = 0; k < T; ++k) {
            const int ti = lane + g * k;
            if (ti >= nt) break;
            float2 a = part[k * 64 + lane];
#pragma unroll
            for (int rr = 1; rr < R; ++rr) {
                const float2 b = part[k * 64 + lane + rr * g];
                a.x += b.x;
                a.y += b.y;
            }
            float2 o = d.v[i0 + ti];
            o.x += a.x;
            o.y += a.y;
            d.v[i0 + ti] = o;
        }
    }
}

template <bool HELM, bool BIG>
__global__ void __launch_bounds__(64)
k_near_sym(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    __shared__ NearSmem sm;
    static_assert(sizeof(NearSmem) >= 5 * 64 * sizeof(float2) + sizeof(float2) * kNearSlots, "part[] must fit");
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int ta = d.tstart[t], tz = d.tstart[t + 1];
    const double kr = (double)d.k_rev;
    const double scale = HELM ? kr : 1.0;
    const float uscale = (float)((1.0 / (4.0 * M_PI)) * (HELM ? kr : 1.0));
    for (int i0 = ta; i0 < tz;) {
        const int nt = min(80, tz - i0);
        const int T = (nt + 15) >> 4;
        const bool first = i0 == ta;
        switch (T) {
            case 1: near_pass_sym<HELM, BIG, 1>(d, sm, t, i0, nt, first, scale, uscale); break;
            case 2: near_pass_sym<HELM, BIG, 2>(d, sm, t, i0, nt, first, scale, uscale); break;
            case 3: near_pass_sym<HELM, BIG, 3>(d, sm, t, i0, nt, first, scale, uscale); break;
            case 4: near_pass_sym<HELM, BIG, 4>(d, sm, t, i0, nt, first, scale, uscale); break;
            default: near_pass_sym<HELM, BIG, 5>(d, sm, t, i0, nt, first, scale, uscale); break;
        }
        i0 += nt;
    }
}

// The symmetric pairs of the derivative kernels (one set), NRM 1: the normal derivative at the targets, 2: at the
// sources, 3: the gradient.  With d = x_i - x_j, grad_x G(x_i - x_j) = d h(r) and grad_x G(x_j - x_i) = -d h(r):
//   NRM 1: target i gets (n_i . d) h u_j, source j gets -(n_j . d) h u_i;
//   NRM 2: target i gets -(n_j . d) h u_j, source j gets (n_i . d) h u_i (the staged normals are -n_j);
//   NRM 3: target i gets d h u_j, source j gets -d h u_i (three components).
// h = -1 / r^3 (Laplace), (ikr - 1) e^{ikr} / r^3 (Helmholtz), in the scaled units of the ordered kernels.
template <bool HELM, bool BIG, int NRM, int NC>
__device__ __forceinline__ void near_pair_symd(double x, double y, double z, float tnx, float tny, float tnz,
                                               float2 ut, double sx, double sy, double sz, float4 sn, float2 us,
                                               float (&are)[NC], float (&aim)[NC], float (&sre)[NC],
                                               float (&sim)[NC]) {
    const float dx = (float)(x - sx), dy = (float)(y - sy), dz = (float)(z - sz);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float inv = __builtin_amdgcn_rsqf(r2);   // distinct boxes of one set, padding far away: r > 0
    const float i3 = inv * inv * inv;
    float hr = -1.f, hi = 0.f;
    if (HELM) {
        const float rr = r2 * inv;
        float sn_, cs;
        sincos_rev(BIG ? __builtin_amdgcn_fractf(rr) : rr, sn_, cs);
        const float kr = 6.2831853f * rr;
        hr = fmaf(-kr, sn_, -cs);
        hi = fmaf(kr, cs, -sn_);
    }
    if (NRM == 3) {
        const float dd[3] = {dx, dy, dz};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const float f = i3 * dd[c];
            if (HELM) {
                const float gr = f * hr, gi = f * hi;
                are[c] = fmaf(gr, us.x, fmaf(-gi, us.y, are[c]));
                aim[c] = fmaf(gr, us.y, fmaf(gi, us.x, aim[c]));
                sre[c] = fmaf(-gr, ut.x, fmaf(gi, ut.y, sre[c]));
                sim[c] = fmaf(-gr, ut.y, fmaf(-gi, ut.x, sim[c]));
            } else {
                are[c] = fmaf(-f, us.x, are[c]);
                aim[c] = fmaf(-f, us.y, aim[c]);
                sre[c] = fmaf(f, ut.x, sre[c]);
                sim[c] = fmaf(f, ut.y, sim[c]);
            }
        }
    } else {
        const float a = fmaf(tnx, dx, fmaf(tny, dy, tnz * dz));       // n_i . d
        const float b = fmaf(sn.x, dx, fmaf(sn.y, dy, sn.z * dz));      // staged normal . d
        const float ft = NRM == 1 ? i3 * a : i3 * b, fs = NRM == 1 ? -(i3 * b) : i3 * a;
        if (HELM) {
            float gr = ft * hr, gi = ft * hi;
            are[0] = fmaf(gr, us.x, fmaf(-gi, us.y, are[0]));
            aim[0] = fmaf(gr, us.y, fmaf(gi, us.x, aim[0]));
            gr = fs * hr;
            gi = fs * hi;
            sre[0] = fmaf(gr, ut.x, fmaf(-gi, ut.y, sre[0]));
            sim[0] = fmaf(gr, ut.y, fmaf(gi, ut.x, sim[0]));
        } else {
            are[0] = fmaf(-ft, us.x, are[0]);
            aim[0] = fmaf(-ft, us.y, aim[0]);
            sre[0] = fmaf(-fs, ut.x, sre[0]);
            sim[0] = fmaf(-fs, ut.y, sim[0]);
        }
    }
}

// One pass of the symmetric derivative near field: the lanes, rows, lists and buffer of near_pass_sym; the
// sources' normals are staged beside them (NRM 1: n_j, NRM 2: -n_j), and a gradient's three components have
// their own accumulators, source-side sums, buffer planes (nsym + c nsymn) and output planes (v + c n_x).
template <bool HELM, bool BIG, int NRM, int T>
__device__ __forceinline__ void near_pass_symd(const LDesc &d, NearSmem &sm, float4 *snm, float2 (*sp12)[kNearSlots],
                                               int t, int i0, int nt, bool first, double scale, float uscale) {
    constexpr int g = 16, R = 4, NC = NRM == 3 ? 3 : 1;
    const int lane = threadIdx.x;
    const int r = lane >> 4, gi = lane & 15;
    const bool last = gi == g - 1;
    const double cx = d.tctr[3 * t], cy = d.tctr[3 * t + 1], cz = d.tctr[3 * t + 2];
    const float4 *nrm = NRM == 1 ? d.tn : d.sn;   // one set: a target's normal is its source normal
    double x[T], y[T], z[T];
    float nx[T], ny[T], nz[T];
    float are[NC][T], aim[NC][T];
    float2 ut[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        // a slot past nt repeats target 0 with zero input: its source-side terms are zero, its own sums discarded
        const int ti = gi + g * k;
        const int i = i0 + (ti < nt ? ti : 0);
        x[k] = (d.txs[i] - cx) * scale;
        y[k] = (d.tys[i] - cy) * scale;
        z[k] = (d.tzs[i] - cz) * scale;
        nx[k] = ny[k] = nz[k] = 0.f;
        if (NRM != 3) {
            const float4 n = nrm[i];
            nx[k] = n.x;
            ny[k] = n.y;
            nz[k] = n.z;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) are[c][k] = aim[c][k] = 0.f;
        const float2 uu = d.u[i];
        ut[k] = ti < nt ? make_float2(uu.x * uscale, uu.y * uscale) : make_float2(0.f, 0.f);
    }
    const int64_t e0 = d.near_ptr[t], e1 = d.near_ptr[t + 1];
    for (int64_t e = e0; e < e1; ++e) {
        const int s = __builtin_amdgcn_readfirstlane(d.near_src[e]);
        const int64_t off = d.near_off[e];
        if (s < t && off >= 0) continue;          // the block of box s evaluates this pair of boxes
        const int j0 = __builtin_amdgcn_readfirstlane(d.sstart[s]), j1 = __builtin_amdgcn_readfirstlane(d.sstart[s + 1]);
        for (int c0 = j0; c0 < j1; c0 += 64) {
            const int cnt = min(64, j1 - c0);
            const int steps = __builtin_amdgcn_readfirstlane((cnt + R - 1) / R), so = steps | 1;
            near_stage_chunk(d, sm, c0, cnt, R, steps, so, cx, cy, cz, scale, uscale, NRM == 3 ? nullptr : snm,
                             nrm, NRM == 1 ? 1.f : -1.f);
            const int base = r * so;
            if (s <= t) {
                // the box itself (r > 0 test) and lower neighbours without a reverse entry: ordered pairs
                if constexpr (NRM == 3) {
                    if (s == t)
                        near_range_grad<HELM, BIG, true, T>(sm, base, steps, x, y, z, are, aim);
                    else
                        near_range_grad<HELM, BIG, false, T>(sm, base, steps, x, y, z, are, aim);
                } else {
                    if (s == t)
                        near_range<HELM, NRM, BIG, true, T>(sm, snm, base, steps, x, y, z, nx, ny, nz, are[0], aim[0]);
                    else
                        near_range<HELM, NRM, BIG, false, T>(sm, snm, base, steps, x, y, z, nx, ny, nz, are[0], aim[0]);
                }
            } else {
                const int jb = r * steps;
                for (int q = 0; q < steps; ++q) {
                    const int sl = base + q;
                    const double sx = sm.x[sl], sy = sm.y[sl], sz = sm.z[sl];
                    const float2 us = sm.u[sl];
                    const float4 sn = NRM == 3 ? make_float4(0.f, 0.f, 0.f, 0.f) : snm[sl];
                    float sre[NC], sim[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) sre[c] = sim[c] = 0.f;
#pragma unroll
                    for (int k = 0; k < T; ++k) {
                        float ar[NC], ai[NC];
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            ar[c] = are[c][k];
                            ai[c] = aim[c][k];
                        }
                        near_pair_symd<HELM, BIG, NRM, NC>(x[k], y[k], z[k], nx[k], ny[k], nz[k], ut[k], sx, sy, sz,
                                                           sn, us, ar, ai, sre, sim);
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            are[c][k] = ar[c];
                            aim[c][k] = ai[c];
                        }
                    }
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const float a = row_sum16(sre[c]), b = row_sum16(sim[c]);
                        if (last) (c == 0 ? sm.sp : sp12[c - 1])[jb + q] = make_float2(a, b);
                    }
                }
                __syncthreads();
                if (lane < cnt) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        float2 *o = d.nsym + (int64_t)c * d.nsymn + off + (c0 - j0) + lane;
                        float2 a = (c == 0 ? sm.sp : sp12[c - 1])[lane];
                        if (!first) {
                            const float2 b = *o;
                            a.x += b.x;
                            a.y += b.y;
                        }
                        *o = a;
                    }
                }
            }
        }
    }
    float2 *part = reinterpret_cast<float2 *>(sm.x);   // [T][64] over x, y, z and u (T <= 5)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < T; ++k) part[k * 64 + lane] = make_float2(are[c][k], aim[c][k]);
        __syncthreads();
        if (lane < g) {
            float2 *vc = d.v + (int64_t)c * d.nx;
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const int ti = lane + g * k;
                if (ti >= nt) break;
                float2 a = part[k * 64 + lane];
#pragma unroll
                for (int rr = 1; rr < R; ++rr) {
                    const float2 b = part[k * 64 + lane + rr * g];
                    a.x += b.x;
                    a.y += b.y;
                }
                float2 o = vc[i0 + ti];
                o.x += a.x;
                o.y += a.y;
                vc[i0 + ti] = o;
            }
        }
    }
}

template <bool HELM, bool BIG, int NRM>
__global__ void __launch_bounds__(64)
k_near_sym_d(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    __shared__ NearSmem sm;
    __shared__ float4 snm[NRM == 3 ? 1 : kNearSlots];
    __shared__ float2 sp12[NRM == 3 ? 2 : 1][kNearSlots];
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int ta = d.tstart[t], tz = d.tstart[t + 1];
    const double kr = (double)d.k_rev;
    const double scale = HELM ? kr : 1.0;
    const float uscale = (float)((1.0 / (4.0 * M_PI)) * (HELM ? kr * kr : 1.0));
    for (int i0 = ta; i0 < tz;) {
        const int nt = min(80, tz - i0);
        const int T = (nt + 15) >> 4;
        const bool first = i0 == ta;
        switch (T) {
            case 1: near_pass_symd<HELM, BIG, NRM, 1>(d, sm, snm, sp12, t, i0, nt, first, scale, uscale); break;
            case 2: near_pass_symd<HELM, BIG, NRM, 2>(d, sm, snm, sp12, t, i0, nt, first, scale, uscale); break;
            case 3: near_pass_symd<HELM, BIG, NRM, 3>(d, sm, snm, sp12, t, i0, nt, first, scale, uscale); break;
            case 4: near_pass_symd<HELM, BIG, NRM, 4>(d, sm, snm, sp12, t, i0, nt, first, scale, uscale); break;
            default: near_pass_symd<HELM, BIG, NRM, 5>(d, sm, snm, sp12, t, i0, nt, first, scale, uscale); break;
        }
        i0 += nt;
    }
}

// v_i += the source-side sums that lower neighbour boxes computed for box b's points (list order).  Item
// (desc, box b).
__global__ void __launch_bounds__(64)
k_near_gather(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int b = wk.y;
    const int ta = d.tstart[b], tz = d.tstart[b + 1];
    const int64_t e0 = d.near_ptr[b], e1 = d.near_ptr[b + 1];
    for (int c = 0; c < d.ncomp; ++c) {
        const float2 *ns = d.nsym + (int64_t)c * d.nsymn;
        float2 *vc = d.v + (int64_t)c * d.nx;
        for (int i = ta + (int)threadIdx.x; i < tz; i += 64) {
            float2 a = make_float2(0.f, 0.f);
            for (int64_t e = e0; e < e1; ++e) {
                const int s = __builtin_amdgcn_readfirstlane(d.near_src[e]);
                const int64_t off = d.near_off[e];
                if (s < b && off >= 0) {
                    const float2 w = ns[off + (i - ta)];
                    a.x += w.x;
                    a.y += w.y;
                }
            }
            float2 o = vc[i];
            o.x += a.x;
            o.y += a.y;
            vc[i] = o;
        }
    }
}

typedef void (*KernelFn)(const LDesc *, const IoEntry *, const int4 *);

KernelFn kernel_of(const Stage &S, int &threads) {
    threads = kThreads;
    switch (S.kern) {
        case K_PERM_IN: return k_perm_in;
        case K_AMAX: return S.a ? k_zero_amax : k_amax;
        case K_PERM_OUT: return k_perm_out;
        case K_FWD_PAIR:
            // a = PPT (+100: 64-thread blocks)
            if (S.a == 101) {
                threads = 64;
                return S.b ? k_pw_forward<1, 64, true> : k_pw_forward<1, 64, false>;
            }
            if (S.a == 4) return S.b ? k_pw_forward<4, kThreads, true> : k_pw_forward<4, kThreads, false>;
            if (S.a == 2) return S.b ? k_pw_forward<2, kThreads, true> : k_pw_forward<2, kThreads, false>;
            return S.b ? k_pw_forward<1, kThreads, true> : k_pw_forward<1, kThreads, false>;
        case K_FWD_PAIR_DL:
            if (S.a == 101) {
                threads = 64;
                return S.b ? k_pw_forward_dl<1, 64, true> : k_pw_forward_dl<1, 64, false>;
            }
            if (S.a == 4) return S.b ? k_pw_forward_dl<4, kThreads, true> : k_pw_forward_dl<4, kThreads, false>;
            if (S.a == 2) return S.b ? k_pw_forward_dl<2, kThreads, true> : k_pw_forward_dl<2, kThreads, false>;
            return S.b ? k_pw_forward_dl<1, kThreads, true> : k_pw_forward_dl<1, kThreads, false>;
        case K_FWD_RING:
            if (S.a == 4) return S.b ? k_pw_forward_rings<4, true> : k_pw_forward_rings<4, false>;
            return S.b ? k_pw_forward_rings<2, true> : k_pw_forward_rings<2, false>;
        case K_SUM: return k_sum_segments;
        case K_TRANSFER:
            // a = 1000 + direction pairs per tile (transfer_qt): class tables staged in LDS; else
            // a = PPT (+100: 64-thread blocks)
            switch (S.a) {
                case 1004: return k_pw_transfer_lds<4>;
                case 1002: return k_pw_transfer_lds<2>;
                case 1001: return k_pw_transfer_lds<1>;
                case 101: threads = 64; return k_pw_transfer<1, 64>;
                case 201: return k_pw_transfer_grp;
                case 301: return k_pw_transfer_sib;
                case 2: return k_pw_transfer<2, kThreads>;
                default: return k_pw_transfer<1, kThreads>;
            }
        case K_BWD_PAIR:
            // a = 100: 64-thread blocks
            if (S.a == 100) {
                threads = 64;
                return S.b ? k_pw_backward<64, true> : k_pw_backward<64, false>;
            }
            return S.b ? k_pw_backward<kThreads, true> : k_pw_backward<kThreads, false>;
        case K_BWD_RING:
            // inner loop unrolled by 4 (one point per thread) or 2 (two points per thread)
            // (a = 102: two points per thread in 128-thread blocks)
            if (S.a == 102) {
                threads = 128;
                return S.b ? k_pw_backward_rings<2, 2, true, 128> : k_pw_backward_rings<2, 2, false, 128>;
            }
            if (S.a == 2) return S.b ? k_pw_backward_rings<2, 2, true> : k_pw_backward_rings<2, 2, false>;
            return S.b ? k_pw_backward_rings<1, 4, true> : k_pw_backward_rings<1, 4, false>;
        case K_BSUM: return k_sum_parts;
        case K_ANTERP: return k_lag_anterp;
        case K_ANTERP_DL: return k_lag_anterp_dl;
        case K_DIRSCALE: return k_dir_scale;
        case K_DNCOMBINE: return k_dn_combine;
        case K_DLCOMBINE: return k_dl_combine;
        // a = waves per block (each takes its own 32-row tiles of T over the block's staged sources)
        case K_MFMA32: threads = 64 * std::max(1, S.a); return k_lag_mfma;
        case K_MFMA16: threads = 64 * std::max(1, S.a); return k_lag_mfma16;
        case K_ACA: threads = 64 * std::max(1, S.a); return k_lag_aca;
        case K_INTERP: return k_lag_interp;
        case K_NEAR: threads = 64; return S.b ? (S.a ? k_near<true, true> : k_near<true, false>) : k_near<false, false>;
        case K_NEAR_SYM:
            // a = BIG + 2 NRM (NRM 0: the kernel itself, 1: normal derivative at the targets, 2: at the sources,
            // 3: the gradient)
            threads = 64;
            switch (S.a >> 1) {
                case 1:
                    return S.b ? ((S.a & 1) ? k_near_sym_d<true, true, 1> : k_near_sym_d<true, false, 1>)
                               : k_near_sym_d<false, false, 1>;
                case 2:
                    return S.b ? ((S.a & 1) ? k_near_sym_d<true, true, 2> : k_near_sym_d<true, false, 2>)
                               : k_near_sym_d<false, false, 2>;
                case 3:
                    return S.b ? ((S.a & 1) ? k_near_sym_d<true, true, 3> : k_near_sym_d<true, false, 3>)
                               : k_near_sym_d<false, false, 3>;
                default:
                    return S.b ? ((S.a & 1) ? k_near_sym<true, true> : k_near_sym<true, false>) : k_near_sym<false, false>;
            }
        case K_NEAR_GATHER: threads = 64; return k_near_gather;
        case K_NEAR_DL:
            threads = 64;
            return S.b ? (S.a ? k_near_dl<true, true> : k_near_dl<true, false>) : k_near_dl<false, false>;
        case K_NEAR_DN:
            threads = 64;
            return S.b ? (S.a ? k_near_dn<true, true> : k_near_dn<true, false>) : k_near_dn<false, false>;
        case K_NEAR_GRAD:
            threads = 64;
            return S.b ? (S.a ? k_near_grad<true, true> : k_near_grad<true, false>) : k_near_grad<false, false>;
        case K_INTERP_DN: return k_lag_interp_dn;
        case K_BWD_PAIR_DN:
            if (S.a == 100) {
                threads = 64;
                return S.b ? k_pw_backward_dn<64, true> : k_pw_backward_dn<64, false>;
            }
            return S.b ? k_pw_backward_dn<kThreads, true> : k_pw_backward_dn<kThreads, false>;
        case K_ZERO_OUT: return k_zero_io;
        case K_GSPREAD:
            switch (S.a) {
                case 4: return k_grid_spread<4>;
                case 5: return k_grid_spread<5>;
                case 6: return k_grid_spread<6>;
                case 7: return k_grid_spread<7>;
                case 8: return k_grid_spread<8>;
                default: throw Error(FFM_EINTERNAL, "unknown spreading width");
            }
        case K_GZ: return k_grid_z;
        case K_GPHI:
            // a = p / 16 for grids of at most 128 nodes per axis, 0 otherwise
            switch (S.a) {
                case 1: return k_grid_phi_s<1>;
                case 2: return k_grid_phi_s<2>;
                case 3: return k_grid_phi_s<3>;
                case 4: return k_grid_phi_s<4>;
                case 5: return k_grid_phi_r<5>;
                case 6: return k_grid_phi_r<6>;
                case 7: return k_grid_phi_r<7>;
                case 8: return k_grid_phi_r<8>;
                default: return k_grid_phi;
            }
        case K_GPHIT: return S.a == 1 ? k_grid_phit_wide : (S.a == 2 ? k_grid_phit_pair : k_grid_phit);
        case K_GZT: return k_grid_zt;
        case K_GINTERP:
            switch (S.a) {
                case 4: return k_grid_interp<4>;
                case 5: return k_grid_interp<5>;
                case 6: return k_grid_interp<6>;
                case 7: return k_grid_interp<7>;
                case 8: return k_grid_interp<8>;
                default: throw Error(FFM_EINTERNAL, "unknown spreading width");
            }
        default: throw Error(FFM_EINTERNAL, "unknown kernel variant");
    }
}

}  // namespace

int stage_blocks_per_cu(int kern, int a, int b) {
    // a property of the compiled kernel and the device: queried once per (device, variant)
    static std::mutex mx;
    static std::map<std::tuple<int, int, int, int>, int> cache;
    int dev = 0;
    FFM_HIP(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, kern, a, b);
    {
        std::lock_guard<std::mutex> lk(mx);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    Stage S;
    S.kern = kern;
    S.a = a;
    S.b = b;
    int threads = kThreads;
    KernelFn fn = kernel_of(S, threads);
    int nb = 0;
    FFM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, 0));
    nb = std::max(nb, 1);
    std::lock_guard<std::mutex> lk(mx);
    cache[key] = nb;
    return nb;
}

int device_cus() {
    static std::mutex mx;
    static std::map<int, int> cache;
    int dev = 0, n = 0;
    FFM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mx);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    FFM_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    return cache[dev] = std::max(n, 1);
}

void run_stage(const Stage &S, const LDesc *ddesc, const IoEntry *dio, hipStream_t st) {
    if (S.nitems == 0) return;
    FFM_CHECK(S.nitems < ((size_t)1 << 31), FFM_EINTERNAL, "stage grid too large");
    int threads = kThreads;
    KernelFn fn = kernel_of(S, threads);
    hipLaunchKernelGGL(fn, dim3((unsigned)S.nitems), dim3(threads), S.shmem, st, ddesc, dio, S.ditems);
    FFM_HIP(hipGetLastError());
}

// Record the end of a phase (timing plans only): the first call opens the apply.
void Plan::mark(int phase, hipStream_t st, const Stage *S) {
    if (tev.empty()) return;
    if (tused == (int)tev.size()) {
        // more launches than the events made with the plan (box batches, per-axis passes): one more event
        hipEvent_t e = nullptr;
        FFM_HIP(hipEventCreate(&e));
        tev.push_back(e);
        tphase.push_back(-1);
        tkern.push_back(make_int4(-1, 0, 0, 0));
        tblocks.push_back(0);
    }
    FFM_HIP(hipEventRecord(tev[tused], st));
    tphase[tused] = phase;
    tkern[tused] = S ? make_int4(S->kern, S->a, S->b, S->level) : make_int4(-1, 0, 0, 0);
    tblocks[tused] = S ? (int64_t)S->nitems : 0;
    ++tused;
}

void plan_apply(Plan &P, const void *wu, int dtype, float2 *v, hipStream_t st) {
    P.tused = 0;
    if (P.empty) {
        P.mark(-1, st);
        const int64_t nv = P.nx * P.ncomp();
        if (nv > 0) FFM_LAUNCH(k_zero_out, (int)((nv + kThreads - 1) / kThreads), kThreads, 0, st, v, nv);
        return;
    }
    // this apply's input and output go to the plan's I/O entry (pinned, copied in stream order); the
    // previous apply's copy has completed once its completion event has
    if (P.applied) FFM_HIP(hipEventSynchronize(P.done));
    if (P.pending) {
        // the plan's last GPU work runs on its planning stream: order this apply after it, and free its
        // temporaries once it is complete
        FFM_HIP(hipStreamWaitEvent(st, P.ready, 0));
        if (hipEventQuery(P.ready) == hipSuccess) {
            P.pending->release();
            P.pending.reset();
        }
    }
    P.hio->wu = wu;
    P.hio->vout = v;
    P.hio->dtype = dtype;
    FFM_HIP(hipMemcpyAsync(P.dio.p, P.hio, sizeof(IoEntry), hipMemcpyHostToDevice, st));
    P.mark(-1, st);
    for (const Stage &S : P.pre) {
        run_stage(S, P.ddesc.p, P.dio.p, st);
        P.mark(0, st, &S);
    }
    for (int l = 1; l <= P.leaf; ++l)
        for (const Stage &S : P.lev[l].stages) {
            run_stage(S, P.ddesc.p, P.dio.p, st);
            P.mark(S.tslot, st, &S);
        }
    for (const Stage &S : P.post) {
        run_stage(S, P.ddesc.p, P.dio.p, st);
        P.mark(S.tslot, st, &S);
    }
}

// The symbol of a stage's kernel as profilers print it (see kernel_of for the variants).
std::string kernel_name(int kern, int a, int b) {
    auto tf = [](int v) { return std::string(v ? "true" : "false"); };
    switch (kern) {
        case K_PERM_IN: return "k_perm_in";
        case K_AMAX: return a ? "k_zero_amax" : "k_amax";
        case K_PERM_OUT: return "k_perm_out";
        case K_FWD_PAIR:
            if (a == 101) return "k_pw_forward<1, 64, " + tf(b) + ">";
            return "k_pw_forward<" + std::to_string(a == 4 || a == 2 ? a : 1) + ", 256, " + tf(b) + ">";
        case K_FWD_PAIR_DL:
            if (a == 101) return "k_pw_forward_dl<1, 64, " + tf(b) + ">";
            return "k_pw_forward_dl<" + std::to_string(a == 4 || a == 2 ? a : 1) + ", 256, " + tf(b) + ">";
        case K_FWD_RING: return "k_pw_forward_rings<" + std::to_string(a == 4 ? 4 : 2) + ", " + tf(b) + ">";
        case K_SUM: return "k_sum_segments";
        case K_TRANSFER:
            if (a > 1000) return "k_pw_transfer_lds<" + std::to_string(a - 1000) + ">";
            if (a == 101) return "k_pw_transfer<1, 64>";
            if (a == 201) return "k_pw_transfer_grp";
            if (a == 301) return "k_pw_transfer_sib";
            return "k_pw_transfer<" + std::to_string(a == 2 ? 2 : 1) + ", 256>";
        case K_BWD_PAIR: return "k_pw_backward<" + std::to_string(a == 100 ? 64 : 256) + ", " + tf(b) + ">";
        case K_BWD_RING:
            if (a == 102) return "k_pw_backward_rings<2, 2, " + tf(b) + ", 128>";
            return a == 2 ? "k_pw_backward_rings<2, 2, " + tf(b) + ", 256>" : "k_pw_backward_rings<1, 4, " + tf(b) + ", 256>";
        case K_BSUM: return "k_sum_parts";
        case K_ANTERP: return "k_lag_anterp";
        case K_ANTERP_DL: return "k_lag_anterp_dl";
        case K_DIRSCALE: return "k_dir_scale";
        case K_DNCOMBINE: return "k_dn_combine";
        case K_DLCOMBINE: return "k_dl_combine";
        case K_MFMA32: return "k_lag_mfma";
        case K_MFMA16: return "k_lag_mfma16";
        case K_ACA: return "k_lag_aca";
        case K_INTERP: return "k_lag_interp";
        case K_NEAR: return "k_near<" + tf(b) + ", " + tf(b && a) + ">";
        case K_NEAR_SYM:
            if (a >> 1)
                return "k_near_sym_d<" + tf(b) + ", " + tf(b && (a & 1)) + ", " + std::to_string(a >> 1) + ">";
            return "k_near_sym<" + tf(b) + ", " + tf(b && a) + ">";
        case K_NEAR_GATHER: return "k_near_gather";
        case K_NEAR_DN: return "k_near_dn<" + tf(b) + ", " + tf(b && a) + ">";
        case K_NEAR_GRAD: return "k_near_grad<" + tf(b) + ", " + tf(b && a) + ">";
        case K_NEAR_DL: return "k_near_dl<" + tf(b) + ", " + tf(b && a) + ">";
        case K_INTERP_DN: return "k_lag_interp_dn";
        case K_BWD_PAIR_DN: return "k_pw_backward_dn<" + std::to_string(a == 100 ? 64 : 256) + ", " + tf(b) + ">";
        case K_ZERO_OUT: return "k_zero_io";
        case K_GSPREAD: return a >= 4 && a <= 8 ? "k_grid_spread<" + std::to_string(a) + ">" : "";
        case K_GZ: return "k_grid_z";
        case K_GPHI:
            if (a >= 1 && a <= 4) return "k_grid_phi_s<" + std::to_string(a) + ">";
            return a >= 5 && a <= 8 ? "k_grid_phi_r<" + std::to_string(a) + ">" : "k_grid_phi";
        case K_GPHIT: return a == 1 ? "k_grid_phit_wide" : (a == 2 ? "k_grid_phit_pair" : "k_grid_phit");
        case K_GZT: return "k_grid_zt";
        case K_GINTERP: return a >= 4 && a <= 8 ? "k_grid_interp<" + std::to_string(a) + ">" : "";
        default: return "";
    }
}

}  // namespace ffm
