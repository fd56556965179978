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
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

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
    }
    if (i < d.nx) d.v[i] = make_float2(0.f, 0.f);
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

// item (desc, first index): vout[i] = 0 for i < nx (an instance without sources inside a batch)
__global__ void __launch_bounds__(kThreads)
k_zero_io(const LDesc *__restrict__ descs, const IoEntry *__restrict__ io, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int64_t i = (int64_t)wk.y + threadIdx.x;
    if (i < d.nx) io[d.inst].vout[i] = make_float2(0.f, 0.f);
}

// item (desc, first index): vout[perm_x[i]] = v[i]
__global__ void __launch_bounds__(kThreads)
k_perm_out(const LDesc *__restrict__ descs, const IoEntry *__restrict__ io, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int64_t i = (int64_t)wk.y + threadIdx.x;
    if (i < d.nx) io[d.inst].vout[d.perm_x[i]] = d.v[i];
}

// ------------------------------------------------------------------ Gegenbauer levels, direction pairs
// Forward transform u~_s(q) = sum_{j in s} e^{-ik s_q.(y_j - c_s)} u_j for an antipodal pair (q, -q): with
// S = sum cos(th) u, T = sum sin(th) u, u~(q) = S - iT and u~(-q) = S + iT.
// Item (desc, source box, tile of 256 PPT pairs); the box's points stream through LDS.
template <int PPT, int BS, bool P64>
__global__ void __launch_bounds__(BS)
k_pw_forward(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
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
                Sre[j] = fmaf(cs, uu.x, Sre[j]);
                Sim[j] = fmaf(cs, uu.y, Sim[j]);
                Tre[j] = fmaf(sn, uu.x, Tre[j]);
                Tim[j] = fmaf(sn, uu.y, Tim[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = p0 + (int64_t)j * BS;
        if (p < npair)
            d.ut[(int64_t)b * npair + p] = make_float4(Sre[j] + Tim[j], Sim[j] - Tre[j], Sre[j] - Tim[j], Sim[j] + Tre[j]);
    }
}

// Diagonal transfer v~_t(q) = sum_{s in far(t)} D_{c(t,s)}(q) u~_s(q) (both directions of a pair).
// Item (desc, target box, tile of 256 PPT pairs).
template <int PPT, int BS>
__global__ void __launch_bounds__(BS)
k_pw_transfer(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int64_t npair = d.npair;
    const int64_t p0 = (int64_t)wk.z * BS * PPT + threadIdx.x;
    float4 acc[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) acc[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t e0 = d.far_ptr[t], e1 = d.far_ptr[t + 1];
    const float4 *__restrict__ D = d.D;
    const float4 *__restrict__ ut = d.ut;
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t s = d.far_src[e], c = d.far_cls[e];
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
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = p0 + (int64_t)j * BS;
        if (p < npair) d.vt[(int64_t)t * npair + p] = acc[j];
    }
}

// Backward transform v_i += sum_q e^{ik s_q.(x_i - c_t)} v~_t(q): per pair, with A = v~(q) + v~(-q) and
// B = v~(q) - v~(-q), the pair contributes cos(th) A + i sin(th) B.  Item (desc, target box, first point);
// BS points per block (64 for levels of small boxes).
template <int BS, bool P64>
__global__ void __launch_bounds__(BS)
k_pw_backward(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int tid = threadIdx.x;
    const int i = wk.z + tid;
    const bool valid = i < d.tstart[t + 1];
    const int64_t npair = d.npair;
    typedef typename std::conditional<P64, double, float>::type real;
    real x = 0, y = 0, z = 0;
    if (valid) {
        x = (real)(d.txs[i] - d.tctr[3 * t]);
        y = (real)(d.tys[i] - d.tctr[3 * t + 1]);
        z = (real)(d.tzs[i] - d.tctr[3 * t + 2]);
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
            ab[tid] = make_float4(w.x + w.z, w.y + w.w, w.x - w.z, w.y - w.w);
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
            are = fmaf(cs, w.x, fmaf(-sn, w.w, are));
            aim = fmaf(cs, w.y, fmaf(sn, w.z, aim));
        }
    }
    if (valid) {
        float2 o = d.v[i];
        o.x += are;
        o.y += aim;
        d.v[i] = o;
    }
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
// PT target points per thread; item (desc, target box, first point).
template <int PT, int U, bool P64>
__global__ void __launch_bounds__(kThreads)
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
        const int i = wk.z + tid + q * kThreads;
        valid[q] = i < iend;
        xr[q] = valid[q] ? d.txs[i] - d.tctr[3 * t] : 0.0;
        yr[q] = valid[q] ? d.tys[i] - d.tctr[3 * t + 1] : 0.0;
        zr[q] = valid[q] ? d.tzs[i] - d.tctr[3 * t + 2] : 0.0;
        vr[q] = vi[q] = 0.f;
    }
    __shared__ float4 s01[kThreads], s23[kThreads];
    __shared__ real scf[kThreads], ssf[kThreads];
    const float4 *vb = d.vt + (int64_t)t * npair;
    // this block's ring pairs (part wk.w of bsplit)
    const int mper = (nrp + d.bsplit - 1) / d.bsplit;
    const int mb = wk.w * mper, me = min(nrp, mb + mper);
    for (int m = mb; m < me; ++m) {
        const double2 rg = d.rings[m];
        const bool eq = 2 * m == L;
        real A[PT], B[PT];
        float ecs[PT], esn[PT], xre[PT], xim[PT], yre[PT], yim[PT];
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            A[q] = (real)(rg.x * xr[q]);
            B[q] = (real)(rg.x * yr[q]);
            const double C = rg.y * zr[q];
            sincos_rev((float)(C - floor(C)), esn[q], ecs[q]);
            xre[q] = xim[q] = yre[q] = yim[q] = 0.f;
        }
        for (int n0 = 0; n0 < L; n0 += kThreads) {
            const int cnt = min(kThreads, L - n0);
            // staged entries padded with zeros to a multiple of U (a zero term leaves every sum unchanged),
            // so the inner loop runs in unrolled steps of U with immediate LDS offsets
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
                    const float4 p1 = vb[(int64_t)m * 2 * L + n];
                    if (eq) {
                        s01[tid] = make_float4(p1.x + p1.z, p1.y + p1.w, p1.x - p1.z, p1.y - p1.w);
                        s23[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                    } else {
                        const float4 p2 = vb[(int64_t)m * 2 * L + n + L];
                        s01[tid] = make_float4(p1.x + p2.x, p1.y + p2.y, p1.x - p2.x, p1.y - p2.y);
                        s23[tid] = make_float4(p2.z + p1.z, p2.w + p1.w, p2.z - p1.z, p2.w - p1.w);
                    }
                    scf[tid] = (real)d.phis[n].x;
                    ssf[tid] = (real)d.phis[n].y;
                }
            }
            __syncthreads();
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
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            // explicit fused forms, so every points-per-thread variant rounds identically
            vr[q] = fmaf(ecs[q], xre[q] + yre[q], fmaf(-esn[q], xim[q] - yim[q], vr[q]));
            vi[q] = fmaf(ecs[q], xim[q] + yim[q], fmaf(esn[q], xre[q] - yre[q], vi[q]));
        }
    }
#pragma unroll
    for (int q = 0; q < PT; ++q) {
        if (!valid[q]) continue;
        const int i = wk.z + tid + q * kThreads;
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

// phi(x) = exp(beta (sqrt(1 - (2x/w)^2) - 1)) for |x| < w/2, 0 outside (exponential of semicircle)
__device__ __forceinline__ float es_phi(float x, float w, float beta) {
    const float t = 2.f * x / w;
    const float s = 1.f - t * t;
    return s > 0.f ? expf(beta * (sqrtf(s) - 1.f)) : 0.f;
}

constexpr int kGT = 64;      // spreading tile edge (grid nodes)
constexpr int kGW = 9;       // most grid nodes a point touches per axis (w <= 8)

// Spread the source points of a box onto one z-plane of its grid (one 64 x 64 tile of it).  Every
// contribution is rounded once to 64-bit fixed point and summed with integer LDS atomics: the sums are
// exact, so the result does not depend on the order of the points.  Item (desc, box, plane, tile).
__global__ void __launch_bounds__(kThreads)
k_grid_spread(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int sb = wk.y, c = wk.z;
    const int p = d.gp, w = d.gw;
    const int nta = (p + kGT - 1) / kGT;
    const int a0 = (wk.w / nta) * kGT, b0 = (wk.w % nta) * kGT;
    const int na = min(kGT, p - a0), nb = min(kGT, p - b0);
    __shared__ unsigned long long acc[2][kGT * kGT];
    for (int i = threadIdx.x; i < kGT * kGT; i += kThreads) {
        acc[0][i] = 0ull;
        acc[1][i] = 0ull;
    }
    __syncthreads();
    // fixed point: |sum| <= (points of the box) x max |Re u|, |Im u| (phi <= 1)
    const double bound = (double)(d.sstart[sb + 1] - d.sstart[sb]) * (double)(*d.amax);
    int e = 0;
    if (bound > 0.0) frexp(bound, &e);
    e = max(e, -900);
    const double scale = ldexp(1.0, 61 - e), inv_scale = ldexp(1.0, e - 61);
    const float half = 0.5f * (float)(p - 1), hw = 0.5f * (float)w, fw = (float)w, beta = d.gbeta;
    const double ih = (double)d.ginv_h;
    const double cx = d.sctr[3 * sb], cy = d.sctr[3 * sb + 1], cz = d.sctr[3 * sb + 2];
    const int clo = max(0, c - w / 2 - 1), chi = min(p - 1, c + w / 2 + 1);
    const int64_t zoff = (int64_t)sb * p;
    const int j0 = d.gzs[zoff + clo], j1 = d.gzs[zoff + chi + 1];
    for (int j = j0 + (int)threadIdx.x; j < j1; j += kThreads) {
        const int i = d.gperm[j];
        const float zg = (float)((d.szs[i] - cz) * ih) + half;
        const float wz = es_phi((float)c - zg, fw, beta);
        if (wz == 0.f) continue;
        const float xg = (float)((d.sxs[i] - cx) * ih) + half;
        const float yg = (float)((d.sys[i] - cy) * ih) + half;
        const int alo = max(a0, (int)ceilf(xg - hw)), ahi = min(a0 + na - 1, (int)floorf(xg + hw));
        const int blo = max(b0, (int)ceilf(yg - hw)), bhi = min(b0 + nb - 1, (int)floorf(yg + hw));
        const float2 uu = d.u[i];
        const float ur = uu.x * wz, ui = uu.y * wz;
        float wy[kGW];
#pragma unroll
        for (int q = 0; q < kGW; ++q) wy[q] = (blo + q <= bhi) ? es_phi((float)(blo + q) - yg, fw, beta) : 0.f;
        for (int a = alo; a <= ahi; ++a) {
            const float wx = es_phi((float)a - xg, fw, beta);
            const int row = (a - a0) * kGT - b0;
#pragma unroll
            for (int q = 0; q < kGW; ++q) {
                if (blo + q <= bhi) {
                    const float wxy = wx * wy[q];
                    const int kk = row + blo + q;
                    atomicAdd(&acc[0][kk], (unsigned long long)__double2ll_rn((double)(ur * wxy) * scale));
                    atomicAdd(&acc[1][kk], (unsigned long long)__double2ll_rn((double)(ui * wxy) * scale));
                }
            }
        }
    }
    __syncthreads();
    float2 *G = d.G + ((int64_t)sb * p + c) * p * p;
    for (int kk = threadIdx.x; kk < kGT * kGT; kk += kThreads) {
        const int al = kk / kGT, bl = kk % kGT;
        if (al < na && bl < nb)
            G[(int64_t)(a0 + al) * p + b0 + bl] = make_float2((float)((double)(long long)acc[0][kk] * inv_scale),
                                                              (float)((double)(long long)acc[1][kk] * inv_scale));
    }
}

// Sums over z: H[m][a][b] = sum_c Ez[m][c] G[c][a][b] and H[L-m] with conj(Ez[m]) (four real products
// serve both), as a tiled product: 32 ring pairs x 128 grid columns per block, 4 x 4 per thread, the
// planes c staged through LDS 32 at a time.  Item (desc, box, column tile, ring-pair tile).
__global__ void __launch_bounds__(kThreads)
k_grid_z(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int sb = wk.y, p = d.gp, L = d.L, nrp = d.nrp;
    const int p2 = p * p;
    const int ab0 = wk.z * 128, m0 = wk.w * 32;
    const int tid = threadIdx.x, tm = tid / 32, tab = tid % 32;   // 8 x 32 threads
    __shared__ float4 Es[32][16];    // [c][ring pairs m0 .. m0+31] (two complex per float4)
    __shared__ float4 Gs[32][64];    // [c][columns ab0 .. ab0+127]
    float q1[4][4], q2[4][4], q3[4][4], q4[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) q1[i][j] = q2[i][j] = q3[i][j] = q4[i][j] = 0.f;
    const float2 *G = d.G + (int64_t)sb * p * p2;
    for (int c0 = 0; c0 < p; c0 += 32) {
        const int cc = min(32, p - c0);
        __syncthreads();
        for (int k = tid; k < 32 * 32; k += kThreads) {
            const int c = k / 32, m = k % 32;
            reinterpret_cast<float2 *>(&Es[c][0])[m] =
                (c < cc && m0 + m < nrp) ? d.Ez[(int64_t)(m0 + m) * p + c0 + c] : make_float2(0.f, 0.f);
        }
        for (int k = tid; k < 32 * 128; k += kThreads) {
            const int c = k / 128, j = k % 128;
            reinterpret_cast<float2 *>(&Gs[c][0])[j] =
                (c < cc && ab0 + j < p2) ? G[(int64_t)(c0 + c) * p2 + ab0 + j] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        for (int c = 0; c < cc; ++c) {
            const float4 e01 = Es[c][2 * tm], e23 = Es[c][2 * tm + 1];
            const float4 g01 = Gs[c][2 * tab], g23 = Gs[c][2 * tab + 1];
            const float er[4] = {e01.x, e01.z, e23.x, e23.z}, ei[4] = {e01.y, e01.w, e23.y, e23.w};
            const float gr[4] = {g01.x, g01.z, g23.x, g23.z}, gi[4] = {g01.y, g01.w, g23.y, g23.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    q1[i][j] = fmaf(er[i], gr[j], q1[i][j]);
                    q2[i][j] = fmaf(ei[i], gi[j], q2[i][j]);
                    q3[i][j] = fmaf(er[i], gi[j], q3[i][j]);
                    q4[i][j] = fmaf(ei[i], gr[j], q4[i][j]);
                }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + tm * 4 + i;
        if (m >= nrp) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ab = ab0 + tab * 4 + j;
            if (ab >= p2) continue;
            d.H[((int64_t)m * d.gnbox + sb) * p2 + ab] = make_float2(q1[i][j] - q2[i][j], q3[i][j] + q4[i][j]);
            if (L - m != m)
                d.H[((int64_t)(L - m) * d.gnbox + sb) * p2 + ab] = make_float2(q1[i][j] + q2[i][j], q3[i][j] - q4[i][j]);
        }
    }
}

// Sums over the plane to the directions: u~(m, n) = sum_a Ex[a][n] X[a][n], X = H_m Ey (sum over b), and
// u~(m, n+L) with the conjugate tables (the same four real products).  A tiled product: 4 rows x 4 azimuths
// per thread; the rows of a 64-row pass are split over TA = ceil(rows / 4) thread rows and the azimuths over
// TN = min(32, 256 / TA) thread columns (grid_phi_tile); b is staged through LDS 32 at a time.  Each thread's
// sums over its rows are then added over the thread rows in order.  Item (desc, box, ring, azimuth tile).
__global__ void __launch_bounds__(kThreads)
k_grid_phi(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int sb = wk.y, m = wk.z;
    const int p = d.gp, L = d.L, mt = min(m, L - m);
    int TA, TN;
    grid_phi_tile(p, TA, TN);
    const int NT = 4 * TN, n0 = wk.w * NT;
    const int tid = threadIdx.x, ta = tid / TN, tn = tid % TN;
    const bool act = tid < TA * TN;
    __shared__ float4 smem[3072];            // 48 KB
    float4 *Hs = smem;                       // [32 b][32]: 64 complex rows a
    float4 *Es = smem + 32 * 32;             // [32 b][64]: 128 complex azimuths n
    const float2 *H = d.H + ((int64_t)m * d.gnbox + sb) * p * p;
    const float2 *Ey = d.Ey + (int64_t)mt * p * L;
    const float2 *Ex = d.Ex + (int64_t)mt * p * L;
    float tr[4], ti[4], ur[4], ui[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) tr[j] = ti[j] = ur[j] = ui[j] = 0.f;
    for (int a0 = 0; a0 < p; a0 += 64) {
        float P1[4][4], P2[4][4], P3[4][4], P4[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) P1[i][j] = P2[i][j] = P3[i][j] = P4[i][j] = 0.f;
        for (int b0 = 0; b0 < p; b0 += 32) {
            const int nbb = min(32, p - b0);
            __syncthreads();
            for (int k = tid; k < 32 * 64; k += kThreads) {
                const int b = k / 64, r = k % 64;
                reinterpret_cast<float2 *>(Hs + b * 32)[r] =
                    (b < nbb && a0 + r < p) ? H[(int64_t)(a0 + r) * p + b0 + b] : make_float2(0.f, 0.f);
            }
            for (int k = tid; k < 32 * NT; k += kThreads) {
                const int b = k / NT, r = k % NT;
                reinterpret_cast<float2 *>(Es + b * 64)[r] =
                    (b < nbb && n0 + r < L) ? Ey[(int64_t)(b0 + b) * L + n0 + r] : make_float2(0.f, 0.f);
            }
            __syncthreads();
            if (act) {
                for (int b = 0; b < nbb; ++b) {
                    const float4 h01 = Hs[b * 32 + 2 * ta], h23 = Hs[b * 32 + 2 * ta + 1];
                    const float4 e01 = Es[b * 64 + 2 * tn], e23 = Es[b * 64 + 2 * tn + 1];
                    const float hr[4] = {h01.x, h01.z, h23.x, h23.z}, hi[4] = {h01.y, h01.w, h23.y, h23.w};
                    const float er[4] = {e01.x, e01.z, e23.x, e23.z}, ei[4] = {e01.y, e01.w, e23.y, e23.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            P1[i][j] = fmaf(er[j], hr[i], P1[i][j]);
                            P2[i][j] = fmaf(ei[j], hi[i], P2[i][j]);
                            P3[i][j] = fmaf(er[j], hi[i], P3[i][j]);
                            P4[i][j] = fmaf(ei[j], hr[i], P4[i][j]);
                        }
                }
            }
        }
        if (act) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int a = a0 + ta * 4 + i;
                if (a >= p) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int n = n0 + tn * 4 + j;
                    if (n >= L) continue;
                    const float2 ex = Ex[(int64_t)a * L + n];
                    const float xr = P1[i][j] - P2[i][j], xi = P3[i][j] + P4[i][j];     // sum_b Ey H
                    const float yr = P1[i][j] + P2[i][j], yi = P3[i][j] - P4[i][j];     // sum_b conj(Ey) H
                    tr[j] = fmaf(ex.x, xr, fmaf(-ex.y, xi, tr[j]));
                    ti[j] = fmaf(ex.x, xi, fmaf(ex.y, xr, ti[j]));
                    ur[j] = fmaf(ex.x, yr, fmaf(ex.y, yi, ur[j]));
                    ui[j] = fmaf(ex.x, yi, fmaf(-ex.y, yr, ui[j]));
                }
            }
        }
    }
    __syncthreads();
    float4 *red = smem;                      // [16 thread rows][128 azimuths]
    if (act) {
#pragma unroll
        for (int j = 0; j < 4; ++j) red[ta * 128 + tn * 4 + j] = make_float4(tr[j], ti[j], ur[j], ui[j]);
    }
    __syncthreads();
    if (tid >= NT) return;
    const int n = n0 + tid;
    if (n >= L) return;
    float4 a = red[tid];
    for (int q = 1; q < TA; ++q) {
        const float4 b = red[q * 128 + tid];
        a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
    }
    // a.xy = u~(m, n), a.zw = u~(m, n + L), into the antipodal-pair layout
    float2 *ut = reinterpret_cast<float2 *>(d.ut) + (int64_t)sb * d.npair * 2;
    const int64_t twoL = 2 * (int64_t)L;
    if (2 * m < L) {
        ut[(m * twoL + n) * 2] = make_float2(a.x, a.y);
        ut[(m * twoL + n + L) * 2] = make_float2(a.z, a.w);
    } else if (2 * m > L) {
        const int64_t m2 = L - m;
        ut[(m2 * twoL + n) * 2 + 1] = make_float2(a.z, a.w);
        ut[(m2 * twoL + n + L) * 2 + 1] = make_float2(a.x, a.y);
    } else {
        ut[(m * twoL + n) * 2] = make_float2(a.x, a.y);
        ut[(m * twoL + n) * 2 + 1] = make_float2(a.z, a.w);
    }
}

// v~ of ring m back to the plane: H'[a][b] = sum_{n < L} conj(Ex) conj(Ey) v~(m, n) + Ex Ey v~(m, n + L)
// = sum_n S Re(Ey) + i D Im(Ey) with S = conj(Ex) v~(n) + Ex v~(n+L), D = Ex v~(n+L) - conj(Ex) v~(n).
// 4 x 4 (a, b) per thread over a 64 x 64 tile; when the grid is smaller, R = grid_phit_rings rings share a
// block (each its own tables and v~), n staged through LDS 32 / R at a time.  Item (desc, box, first ring,
// tile).
__global__ void __launch_bounds__(kThreads)
k_grid_phit(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int tb_ = wk.y;
    const int p = d.gp, L = d.L;
    const int R = grid_phit_rings(p), NC = 32 / R;
    const int TC = p > 64 ? 16 : (p + 3) / 4, TAB = TC * TC;     // thread tiles per ring
    const int nta = (p + 63) / 64;
    const int a0 = (wk.w / nta) * 64, b0 = (wk.w % nta) * 64;
    const int tid = threadIdx.x, rr = tid / TAB, tt = tid % TAB, ta = tt / TC, tb = tt % TC;
    const int m = wk.z + rr;
    const bool act = rr < R && m <= L;
    const int mt = act ? min(m, L - m) : 0;
    __shared__ float4 sS[32][32], sD[32][32], sE[32][32];   // [ring r x NC + n][64 complex]
    float2 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_float2(0.f, 0.f);
    const float2 *vt = reinterpret_cast<const float2 *>(d.vt) + (int64_t)tb_ * d.npair * 2;
    const int64_t twoL = 2 * (int64_t)L;
    for (int n0 = 0; n0 < L; n0 += NC) {
        const int cnt = min(NC, L - n0);
        __syncthreads();
        for (int k = tid; k < R * NC * 64; k += kThreads) {
            const int r = k / (NC * 64), nn = (k / 64) % NC, idx = k % 64, n = n0 + nn;
            const int mr = wk.z + r;
            float2 S = make_float2(0.f, 0.f), Dd = S, E = S;
            if (nn < cnt && mr <= L) {
                const int mtr = min(mr, L - mr);
                float2 v1, v2;   // v~(mr, n), v~(mr, n + L)
                if (2 * mr < L) {
                    v1 = vt[(mr * twoL + n) * 2];
                    v2 = vt[(mr * twoL + n + L) * 2];
                } else if (2 * mr > L) {
                    const int64_t m2 = L - mr;
                    v1 = vt[(m2 * twoL + n + L) * 2 + 1];
                    v2 = vt[(m2 * twoL + n) * 2 + 1];
                } else {
                    v1 = vt[(mr * twoL + n) * 2];
                    v2 = vt[(mr * twoL + n) * 2 + 1];
                }
                const int a = a0 + idx;
                if (a < p) {
                    const float2 ex = d.Ex[((int64_t)mtr * p + a) * L + n];
                    const float y1r = fmaf(ex.x, v1.x, ex.y * v1.y), y1i = fmaf(ex.x, v1.y, -(ex.y * v1.x));   // conj(ex) v1
                    const float y2r = fmaf(ex.x, v2.x, -(ex.y * v2.y)), y2i = fmaf(ex.x, v2.y, ex.y * v2.x);   // ex v2
                    S = make_float2(y1r + y2r, y1i + y2i);
                    Dd = make_float2(y2r - y1r, y2i - y1i);
                }
                const int b = b0 + idx;
                if (b < p) E = d.Ey[((int64_t)mtr * p + b) * L + n];
            }
            reinterpret_cast<float2 *>(&sS[r * NC + nn][0])[idx] = S;
            reinterpret_cast<float2 *>(&sD[r * NC + nn][0])[idx] = Dd;
            reinterpret_cast<float2 *>(&sE[r * NC + nn][0])[idx] = E;
        }
        __syncthreads();
        if (act) {
            for (int nn = 0; nn < cnt; ++nn) {
                const int row = rr * NC + nn;
                const float4 s01 = sS[row][2 * ta], s23 = sS[row][2 * ta + 1];
                const float4 d01 = sD[row][2 * ta], d23 = sD[row][2 * ta + 1];
                const float4 e01 = sE[row][2 * tb], e23 = sE[row][2 * tb + 1];
                const float2 sv[4] = {make_float2(s01.x, s01.y), make_float2(s01.z, s01.w), make_float2(s23.x, s23.y),
                                      make_float2(s23.z, s23.w)};
                const float2 dv[4] = {make_float2(d01.x, d01.y), make_float2(d01.z, d01.w), make_float2(d23.x, d23.y),
                                      make_float2(d23.z, d23.w)};
                const float2 ev[4] = {make_float2(e01.x, e01.y), make_float2(e01.z, e01.w), make_float2(e23.x, e23.y),
                                      make_float2(e23.z, e23.w)};
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[i][j].x = fmaf(sv[i].x, ev[j].x, fmaf(-dv[i].y, ev[j].y, acc[i][j].x));
                        acc[i][j].y = fmaf(sv[i].y, ev[j].x, fmaf(dv[i].x, ev[j].y, acc[i][j].y));
                    }
            }
        }
    }
    if (!act) return;
    (void)mt;
    float2 *Hb = d.H + ((int64_t)m * d.gnbox + tb_) * p * p;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int a = a0 + ta * 4 + i;
        if (a >= p) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + tb * 4 + j;
            if (b < p) Hb[(int64_t)a * p + b] = acc[i][j];
        }
    }
}

// Back over z: G'[c][a][b] = sum over ring pairs of conj(Ez[m][c]) H'[m][a][b] + Ez[m][c] H'[L-m][a][b]
// = Re(Ez) (H'[m] + H'[L-m]) + i Im(Ez) (H'[L-m] - H'[m]), as a tiled product: 32 planes x 128 columns per
// block, 4 x 4 per thread, ring pairs staged through LDS 16 at a time.  Item (desc, box, column tile,
// plane tile).
__global__ void __launch_bounds__(kThreads)
k_grid_zt(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int tb_ = wk.y, p = d.gp, L = d.L, nrp = d.nrp;
    const int p2 = p * p;
    const int ab0 = wk.z * 128, c0 = wk.w * 32;
    const int tid = threadIdx.x, tc = tid / 32, tab = tid % 32;
    __shared__ float4 Es[16][16];    // [ring pair][planes c0 .. c0+31]
    __shared__ float4 Ss[16][64];    // [ring pair][columns]: H'[m] + H'[L-m]
    __shared__ float4 Ds[16][64];    //                       H'[L-m] - H'[m]
    float2 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_float2(0.f, 0.f);
    for (int mp0 = 0; mp0 < nrp; mp0 += 16) {
        const int mc = min(16, nrp - mp0);
        __syncthreads();
        for (int k = tid; k < 16 * 32; k += kThreads) {
            const int mm = k / 32, c = k % 32;
            reinterpret_cast<float2 *>(&Es[mm][0])[c] =
                (mm < mc && c0 + c < p) ? d.Ez[(int64_t)(mp0 + mm) * p + c0 + c] : make_float2(0.f, 0.f);
        }
        for (int k = tid; k < 16 * 128; k += kThreads) {
            const int mm = k / 128, j = k % 128, mp = mp0 + mm, ab = ab0 + j;
            float2 S = make_float2(0.f, 0.f), Dd = S;
            if (mm < mc && ab < p2) {
                const int m2 = L - mp;
                const float2 h1 = d.H[((int64_t)mp * d.gnbox + tb_) * p2 + ab];
                const float2 h2 = (m2 != mp) ? d.H[((int64_t)m2 * d.gnbox + tb_) * p2 + ab] : make_float2(0.f, 0.f);
                S = make_float2(h1.x + h2.x, h1.y + h2.y);
                Dd = make_float2(h2.x - h1.x, h2.y - h1.y);
            }
            reinterpret_cast<float2 *>(&Ss[mm][0])[j] = S;
            reinterpret_cast<float2 *>(&Ds[mm][0])[j] = Dd;
        }
        __syncthreads();
        for (int mm = 0; mm < mc; ++mm) {
            const float4 e01 = Es[mm][2 * tc], e23 = Es[mm][2 * tc + 1];
            const float4 s01 = Ss[mm][2 * tab], s23 = Ss[mm][2 * tab + 1];
            const float4 d01 = Ds[mm][2 * tab], d23 = Ds[mm][2 * tab + 1];
            const float er[4] = {e01.x, e01.z, e23.x, e23.z}, ei[4] = {e01.y, e01.w, e23.y, e23.w};
            const float sr[4] = {s01.x, s01.z, s23.x, s23.z}, si[4] = {s01.y, s01.w, s23.y, s23.w};
            const float dr[4] = {d01.x, d01.z, d23.x, d23.z}, di[4] = {d01.y, d01.w, d23.y, d23.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j].x = fmaf(er[i], sr[j], fmaf(-ei[i], di[j], acc[i][j].x));
                    acc[i][j].y = fmaf(er[i], si[j], fmaf(ei[i], dr[j], acc[i][j].y));
                }
        }
    }
    float2 *G = d.G + (int64_t)tb_ * p * p2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = c0 + tc * 4 + i;
        if (c >= p) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ab = ab0 + tab * 4 + j;
            if (ab < p2) G[(int64_t)c * p2 + ab] = acc[i][j];
        }
    }
}

// v_i += sum over the grid nodes around x_i of phi phi phi G'.  Item (desc, target box, first point).
__global__ void __launch_bounds__(kThreads)
k_grid_interp(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int i = wk.z + threadIdx.x;
    if (i >= d.tstart[t + 1]) return;
    const int p = d.gp;
    const float half = 0.5f * (float)(p - 1), hw = 0.5f * (float)d.gw, fw = (float)d.gw, beta = d.gbeta;
    const double ih = (double)d.ginv_h;
    const float xg = (float)((d.txs[i] - d.tctr[3 * t]) * ih) + half;
    const float yg = (float)((d.tys[i] - d.tctr[3 * t + 1]) * ih) + half;
    const float zg = (float)((d.tzs[i] - d.tctr[3 * t + 2]) * ih) + half;
    const int alo = max(0, (int)ceilf(xg - hw)), ahi = min(p - 1, (int)floorf(xg + hw));
    const int blo = max(0, (int)ceilf(yg - hw)), bhi = min(p - 1, (int)floorf(yg + hw));
    const int clo = max(0, (int)ceilf(zg - hw)), chi = min(p - 1, (int)floorf(zg + hw));
    float wy[kGW];
#pragma unroll
    for (int q = 0; q < kGW; ++q) wy[q] = (blo + q <= bhi) ? es_phi((float)(blo + q) - yg, fw, beta) : 0.f;
    const float2 *G = d.G + (int64_t)t * p * p * p;
    float sr = 0.f, si = 0.f;
    for (int c = clo; c <= chi; ++c) {
        const float wz = es_phi((float)c - zg, fw, beta);
        float pr = 0.f, pi = 0.f;
        for (int a = alo; a <= ahi; ++a) {
            const float wx = es_phi((float)a - xg, fw, beta);
            const float2 *row = G + ((int64_t)c * p + a) * p;
            float rr = 0.f, ri = 0.f;
#pragma unroll
            for (int q = 0; q < kGW; ++q) {
                if (blo + q <= bhi) {
                    const float2 g = row[blo + q];
                    rr = fmaf(wy[q], g.x, rr);
                    ri = fmaf(wy[q], g.y, ri);
                }
            }
            pr = fmaf(wx, rr, pr);
            pi = fmaf(wx, ri, pi);
        }
        sr = fmaf(wz, pr, sr);
        si = fmaf(wz, pi, si);
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

// u~_s = L_Y u_s: u~_s[(a r1 + b) r1 + c] = sum_j l_a(t_x) l_b(t_y) l_c(t_z) u_j, t = 2 (y - c_s) / d_l.
// Item (desc, source box).
__global__ void __launch_bounds__(kThreads)
k_lag_anterp(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int b = wk.y;
    const int tid = threadIdx.x;
    const int r1 = d.r1, rp = d.rp, r = r1 * r1 * r1;
    const double two_over_dl = d.two_over_dl;
    __shared__ float ell[kAnterpChunk][3 * kMaxR1];
    __shared__ float2 us[kAnterpChunk];
    __shared__ float nodes[kMaxR1], den[kMaxR1];
    if (tid < r1) {
        nodes[tid] = d.lnodes[tid];
        den[tid] = d.lden[tid];
    }
    constexpr int kOut = (kMaxR1 * kMaxR1 * kMaxR1 + kThreads - 1) / kThreads;
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
    const int nout = (r + kThreads - 1) / kThreads;
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
            us[tid] = d.u[j];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const float2 uu = us[jj];
#pragma unroll
            for (int o = 0; o < kOut; ++o) {
                if (o < nout) {
                    const float w = ell[jj][ia[o]] * ell[jj][r1 + ib[o]] * ell[jj][2 * r1 + ic[o]];
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

// Transfer products of one class group on MFMA: Z_e = T_c u~_{s(e)} for up to 16 pairs e.
// C (rp x 32) = T_c (rp x rp) x U (rp x 32), U[k][2m + part] = part of u~_{s(e_m)}[k].
// v_mfma_f32_32x32x2f32 operands: A[i][k] from lane i + 32 k, B[k][j] from lane j + 32 k,
// D[i][j] in lane j + 32 ((i / 4) % 2), register (i % 4) + 4 (i / 8).  Item (desc, group).
__global__ void __launch_bounds__(64)
k_lag_mfma(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    extern __shared__ float U[];   // [rp][32]
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int g = wk.y;
    const int lane = threadIdx.x;
    const int rp = d.rp, helm = d.helm;
    const int c = d.grp_cls[g];
    __shared__ int pe[16], ps[16];
    if (lane < 16) {
        const int e = d.grp_pair[(int64_t)g * 16 + lane];
        pe[lane] = e;
        ps[lane] = e >= 0 ? d.far_src[e] : -1;
    }
    __syncthreads();
    for (int idx = lane; idx < rp * 32; idx += 64) {
        const int k = idx >> 5, col = idx & 31, m = col >> 1;
        float val = 0.f;
        if (ps[m] >= 0) {
            const float2 w = d.ut2[(int64_t)ps[m] * rp + k];
            val = (col & 1) ? w.y : w.x;
        }
        U[idx] = val;
    }
    __syncthreads();
    const int64_t per = (int64_t)rp * rp;
    const float *Tre = d.T + (int64_t)c * (helm ? 2 : 1) * per;
    const float *Tim = Tre + per;
    const int col = lane & 31, kh = lane >> 5;
    const int e = pe[col >> 1];
    for (int mt = 0; mt < rp / 32; ++mt) {
        floatx16 acc1, acc2;
        for (int v = 0; v < 16; ++v) {
            acc1[v] = 0.f;
            acc2[v] = 0.f;
        }
        for (int kk = 0; kk < rp / 2; ++kk) {
            const int k = 2 * kk + kh;
            const float bval = U[k * 32 + col];
            const float a1 = Tre[(int64_t)k * rp + mt * 32 + col];
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bval, acc1, 0, 0, 0);
            if (helm) {
                const float a2 = Tim[(int64_t)k * rp + mt * 32 + col];
                acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, bval, acc2, 0, 0, 0);
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

// Mixed precision: the same class-group products on FP16 MFMA (v_mfma_f32_32x32x8f16) with FP32
// accumulation.  A[i][k] comes from lane i + 32 (k / 4) (element k % 4 of a half4), B[k][j] from lane
// j + 32 (k / 4); D as for the FP32 instruction.  T16 = T * sT (plan time); the sources are scaled by a
// power of two s_u derived on the device from max |u| so that |u~ s_u| < 6e4; Z = C / (sT s_u).
__device__ __forceinline__ float u_scale(float amax, int maxpts) {
    // |u~| <= (Lebesgue constant of the tensor grid, <= 8) * points * max|u|
    const float bound = 8.f * (float)maxpts * fmaxf(amax, 1e-30f);
    return exp2f(floorf(log2f(6.0e4f / bound)));
}

__global__ void __launch_bounds__(64)
k_lag_mfma16(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    extern __shared__ _Float16 U16[];   // [32][rp]: column-major tile, k contiguous
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int g = wk.y;
    const int lane = threadIdx.x;
    const int rp = d.rp, helm = d.helm;
    const int c = d.grp_cls[g];
    const float su = u_scale(*d.amax, d.maxpts);
    __shared__ int pe[16], ps[16];
    if (lane < 16) {
        const int e = d.grp_pair[(int64_t)g * 16 + lane];
        pe[lane] = e;
        ps[lane] = e >= 0 ? d.far_src[e] : -1;
    }
    __syncthreads();
    for (int idx = lane; idx < rp * 32; idx += 64) {
        const int col = idx / rp, k = idx % rp, m = col >> 1;
        float val = 0.f;
        if (ps[m] >= 0) {
            const float2 w = d.ut2[(int64_t)ps[m] * rp + k];
            val = ((col & 1) ? w.y : w.x) * su;
        }
        U16[idx] = (_Float16)val;
    }
    __syncthreads();
    const int64_t per = (int64_t)rp * rp;
    const _Float16 *Tre = d.T16 + (int64_t)c * (helm ? 2 : 1) * per;
    const _Float16 *Tim = Tre + per;
    const int col = lane & 31, kh = lane >> 5;
    const int e = pe[col >> 1];
    const float inv = 1.f / (d.sT * su);
    for (int mt = 0; mt < rp / 32; ++mt) {
        floatx16 acc1, acc2;
        for (int v = 0; v < 16; ++v) {
            acc1[v] = 0.f;
            acc2[v] = 0.f;
        }
        const int i = mt * 32 + col;
        for (int k0 = 0; k0 < rp; k0 += 8) {
            const int k = k0 + 4 * kh;
            const half4_t b = *reinterpret_cast<const half4_t *>(U16 + col * rp + k);
            const half4_t a1 = *reinterpret_cast<const half4_t *>(Tre + (int64_t)i * rp + k);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x8f16(a1, b, acc1, 0, 0, 0);
            if (helm) {
                const half4_t a2 = *reinterpret_cast<const half4_t *>(Tim + (int64_t)i * rp + k);
                acc2 = __builtin_amdgcn_mfma_f32_32x32x8f16(a2, b, acc2, 0, 0, 0);
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

// v_i += L_X^T v~_t with v~_t = sum_{e in far(t)} Z_e (fixed order), t = 2 (x - c_t) / d_l.
// Item (desc, target box).
__global__ void __launch_bounds__(kThreads)
k_lag_interp(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    extern __shared__ float2 vt[];   // [r]
    __shared__ float nodes[kMaxR1], den[kMaxR1];
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int tid = threadIdx.x;
    const int r1 = d.r1, rp = d.rp, r = r1 * r1 * r1;
    const double two_over_dl = d.two_over_dl;
    if (tid < r1) {
        nodes[tid] = d.lnodes[tid];
        den[tid] = d.lden[tid];
    }
    const int64_t e0 = d.far_ptr[t], e1 = d.far_ptr[t + 1];
    for (int i = tid; i < r; i += kThreads) {
        float2 a = make_float2(0.f, 0.f);
        for (int64_t e = e0; e < e1; ++e) {
            const float2 z = d.Z[e * rp + i];
            a.x += z.x;
            a.y += z.y;
        }
        vt[i] = a;
    }
    __syncthreads();
    const double cx = d.tctr[3 * t], cy = d.tctr[3 * t + 1], cz = d.tctr[3 * t + 2];
    for (int i = d.tstart[t] + tid; i < d.tstart[t + 1]; i += kThreads) {
        float lx[kMaxR1], ly[kMaxR1], lz[kMaxR1];
        lagrange_1d((float)((d.txs[i] - cx) * two_over_dl), r1, nodes, den, lx);
        lagrange_1d((float)((d.tys[i] - cy) * two_over_dl), r1, nodes, den, ly);
        lagrange_1d((float)((d.tzs[i] - cz) * two_over_dl), r1, nodes, den, lz);
        float sre = 0.f, sim = 0.f;
        for (int a = 0; a < r1; ++a) {
            float bre = 0.f, bim = 0.f;
            for (int bb = 0; bb < r1; ++bb) {
                float cre = 0.f, cim = 0.f;
                const float2 *row = vt + (a * r1 + bb) * r1;
                for (int c = 0; c < r1; ++c) {
                    cre = fmaf(lz[c], row[c].x, cre);
                    cim = fmaf(lz[c], row[c].y, cim);
                }
                bre = fmaf(ly[bb], cre, bre);
                bim = fmaf(ly[bb], cim, bim);
            }
            sre = fmaf(lx[a], bre, sre);
            sim = fmaf(lx[a], bim, sim);
        }
        float2 o = d.v[i];
        o.x += sre;
        o.y += sim;
        d.v[i] = o;
    }
}

// ------------------------------------------------------------------ near field (leaf)
// v_i += sum_{s in near(t)} sum_{j in s, r_ij > 0} G(r_ij) u_j.  One 64-lane block per target box; source
// points are staged through LDS in FP64 relative to the target centre, and every pair's difference is
// formed in FP64 and rounded once to FP32, so close pairs keep the full FP32 relative accuracy of r.
// Item (desc, target box).
template <bool HELM>
__global__ void __launch_bounds__(64)
k_near(const LDesc *__restrict__ descs, const IoEntry *__restrict__, const int4 *__restrict__ work) {
    const int4 wk = work[blockIdx.x];
    const LDesc &d = descs[wk.x];
    const int t = wk.y;
    const int lane = threadIdx.x;
    const float k_rev = d.k_rev;
    const double cx = d.tctr[3 * t], cy = d.tctr[3 * t + 1], cz = d.tctr[3 * t + 2];
    __shared__ double spx[64], spy[64], spz[64];   // sources relative to c_t
    __shared__ float2 su[64];                      // u / (4 pi)
    const float inv4pi = (float)(1.0 / (4.0 * M_PI));
    const int64_t e0 = d.near_ptr[t], e1 = d.near_ptr[t + 1];
    for (int i0 = d.tstart[t]; i0 < d.tstart[t + 1]; i0 += 64) {
        const int i = i0 + lane;
        const bool valid = i < d.tstart[t + 1];
        double x = 0.0, y = 0.0, z = 0.0;
        if (valid) {
            x = d.txs[i] - cx;
            y = d.tys[i] - cy;
            z = d.tzs[i] - cz;
        }
        float are = 0.f, aim = 0.f;
        for (int64_t e = e0; e < e1; ++e) {
            const int s = d.near_src[e];
            const int j0 = d.sstart[s], j1 = d.sstart[s + 1];
            for (int c0 = j0; c0 < j1; c0 += 64) {
                const int cnt = min(64, j1 - c0);
                __syncthreads();
                if (lane < cnt) {
                    const int j = c0 + lane;
                    spx[lane] = d.sxs[j] - cx;
                    spy[lane] = d.sys[j] - cy;
                    spz[lane] = d.szs[j] - cz;
                    const float2 uu = d.u[j];
                    su[lane] = make_float2(uu.x * inv4pi, uu.y * inv4pi);
                }
                __syncthreads();
                for (int jj = 0; jj < cnt; ++jj) {
                    const float dx = (float)(x - spx[jj]), dy = (float)(y - spy[jj]), dz = (float)(z - spz[jj]);
                    const float2 uu = su[jj];
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float inv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
                    if (HELM) {
                        const float ph = r2 * inv * k_rev;
                        float sn, cs;
                        sincos_rev(__builtin_amdgcn_fractf(ph), sn, cs);
                        const float gr = cs * inv, gi = sn * inv;
                        are = fmaf(gr, uu.x, fmaf(-gi, uu.y, are));
                        aim = fmaf(gr, uu.y, fmaf(gi, uu.x, aim));
                    } else {
                        are = fmaf(inv, uu.x, are);
                        aim = fmaf(inv, uu.y, aim);
                    }
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
        case K_FWD_RING:
            if (S.a == 4) return S.b ? k_pw_forward_rings<4, true> : k_pw_forward_rings<4, false>;
            return S.b ? k_pw_forward_rings<2, true> : k_pw_forward_rings<2, false>;
        case K_SUM: return k_sum_segments;
        case K_TRANSFER:
            if (S.a == 101) {
                threads = 64;
                return k_pw_transfer<1, 64>;
            }
            return S.a == 2 ? k_pw_transfer<2, kThreads> : k_pw_transfer<1, kThreads>;
        case K_BWD_PAIR:
            // a = 100: 64-thread blocks
            if (S.a == 100) {
                threads = 64;
                return S.b ? k_pw_backward<64, true> : k_pw_backward<64, false>;
            }
            return S.b ? k_pw_backward<kThreads, true> : k_pw_backward<kThreads, false>;
        case K_BWD_RING:
            // inner loop unrolled by 4 (one point per thread) or 2 (two points per thread)
            if (S.a == 2) return S.b ? k_pw_backward_rings<2, 2, true> : k_pw_backward_rings<2, 2, false>;
            return S.b ? k_pw_backward_rings<1, 4, true> : k_pw_backward_rings<1, 4, false>;
        case K_BSUM: return k_sum_parts;
        case K_ANTERP: return k_lag_anterp;
        case K_MFMA32: threads = 64; return k_lag_mfma;
        case K_MFMA16: threads = 64; return k_lag_mfma16;
        case K_INTERP: return k_lag_interp;
        case K_NEAR: threads = 64; return S.b ? k_near<true> : k_near<false>;
        case K_ZERO_OUT: return k_zero_io;
        case K_GSPREAD: return k_grid_spread;
        case K_GZ: return k_grid_z;
        case K_GPHI: return k_grid_phi;
        case K_GPHIT: return k_grid_phit;
        case K_GZT: return k_grid_zt;
        case K_GINTERP: return k_grid_interp;
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
    if (S.ditems.n == 0) return;
    FFM_CHECK(S.ditems.n < ((size_t)1 << 31), FFM_EINTERNAL, "stage grid too large");
    int threads = kThreads;
    KernelFn fn = kernel_of(S, threads);
    hipLaunchKernelGGL(fn, dim3((unsigned)S.ditems.n), dim3(threads), S.shmem, st, ddesc, dio, S.ditems.p);
    FFM_HIP(hipGetLastError());
}

// Record the end of a phase (timing plans only): the first call opens the apply.
void Plan::mark(int phase, hipStream_t st) {
    if (tev.empty()) return;
    FFM_CHECK(tused < (int)tev.size(), FFM_EINTERNAL, "timing events exhausted");
    FFM_HIP(hipEventRecord(tev[tused], st));
    tphase[tused] = phase;
    ++tused;
}

void plan_apply(Plan &P, const void *wu, int dtype, float2 *v, hipStream_t st) {
    P.tused = 0;
    if (P.empty) {
        P.mark(-1, st);
        if (P.nx > 0) FFM_LAUNCH(k_zero_out, (int)((P.nx + kThreads - 1) / kThreads), kThreads, 0, st, v, P.nx);
        return;
    }
    // this apply's input and output go to the plan's I/O entry (pinned, copied in stream order); the
    // previous apply's copy has completed once its completion event has
    if (P.applied) FFM_HIP(hipEventSynchronize(P.done));
    P.hio->wu = wu;
    P.hio->vout = v;
    P.hio->dtype = dtype;
    FFM_HIP(hipMemcpyAsync(P.dio.p, P.hio, sizeof(IoEntry), hipMemcpyHostToDevice, st));
    P.mark(-1, st);
    for (const Stage &S : P.pre) run_stage(S, P.ddesc.p, P.dio.p, st);
    P.mark(0, st);
    for (int l = 1; l <= P.leaf; ++l)
        for (const Stage &S : P.lev[l].stages) {
            run_stage(S, P.ddesc.p, P.dio.p, st);
            if (S.slot >= 0) P.mark(S.slot, st);
        }
    for (const Stage &S : P.post) {
        run_stage(S, P.ddesc.p, P.dio.p, st);
        if (S.slot >= 0) P.mark(S.slot, st);
    }
}

}  // namespace ffm
