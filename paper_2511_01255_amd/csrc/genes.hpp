// genes.hpp -- per-gene-quad arithmetic of the optimiser steps (paper Sec.
// 2.2.1 DE rand/1 + binomial crossover, Sec. 2.2.2 grey-wolf update), and
// the row / bit-word helpers, shared by the single-design and batched
// kernels. Binary32 arithmetic is spelled out with explicit fmaf and the
// library is built with -ffp-contract=off, so trial and candidate genes are
// bit-for-bit what these formulas state.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "philox.hpp"

namespace qpm {

__device__ __forceinline__ const float *row_of(const PopView &pv, int64_t r)
{
    const bool second = pv.flags != nullptr && pv.flags[r] != 0u;
    return (second ? pv.x1 : pv.x0) + r * pv.ldx;
}

__device__ __forceinline__ float *out_row_of(const PopView &pv, int64_t r)
{
    const bool second = pv.flags != nullptr && pv.flags[r] != 0u;
    return (second ? pv.out0 : pv.out1) + r * pv.ldx;
}

__device__ __forceinline__ float clamp1(float v) { return fminf(fmaxf(v, -1.0f), 1.0f); }

// x / 3 correctly rounded, without a division: q0 = x RN(1/3), the exact
// remainder r = x - 3 q0 by FMA, one FMA correction, and the sign of x
// restored (only -0 would otherwise come out as +0). Checked against IEEE
// division for every finite binary32 input.
__device__ __forceinline__ float div3(float x)
{
    const float c = 0x1.555556p-2f;  // RN(1/3)
    const float q0 = x * c;
    const float r = fmaf(-q0, 3.0f, x);
    return copysignf(fmaf(r, c, q0), x);
}

// div3 for x != 0: the same three steps without the sign restore (checked
// against IEEE division for every nonzero finite binary32 input)
__device__ __forceinline__ float div3_nonzero(float x)
{
    const float c = 0x1.555556p-2f;
    const float q0 = x * c;
    const float r = fmaf(-q0, 3.0f, x);
    return fmaf(r, c, q0);
}

// n / d correctly rounded for d in [2^-60, 2^60] and |n| in [2^-60, 2^60]:
// the IEEE single-precision division sequence (reciprocal, one Newton step,
// quotient, two FMA remainder corrections) without its scaling and fix-up
// steps, which leave every operand and result unchanged in this range (no
// operand or quotient near the subnormal or overflow range, exponent gap
// far below 96, no special value), so the result is that of n / d.
__device__ __forceinline__ float div_in_range(float n, float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    const float e = fmaf(-d, r, 1.0f);
    const float r1 = fmaf(e, r, r);
    const float q = n * r1;
    const float rem = fmaf(-d, q, n);
    const float q1 = fmaf(rem, r1, q);
    const float rem2 = fmaf(-d, q1, n);
    return fmaf(rem2, r1, q1);
}

__device__ __forceinline__ void store_quad(float *dst, int64_t j0, int64_t D, float4 v)
{
    if (j0 + 3 < D) {
        *reinterpret_cast<float4 *>(dst + j0) = v;
    } else {
        dst[j0] = v.x;
        if (j0 + 1 < D) dst[j0 + 1] = v.y;
        if (j0 + 2 < D) dst[j0 + 2] = v.z;
    }
}

// store_quad with non-temporal full-quad stores: trial and candidate rows
// are not read again before the next step, so they should not displace the
// rows the donor reads are served from
__device__ __forceinline__ void store_quad_nt(float *dst, int64_t j0, int64_t D, float4 v)
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    if (j0 + 3 < D) {
        const v4f w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<v4f *>(dst + j0));
    } else {
        dst[j0] = v.x;
        if (j0 + 1 < D) dst[j0 + 1] = v.y;
        if (j0 + 2 < D) dst[j0 + 2] = v.z;
    }
}

__device__ __forceinline__ uint32_t quad_nibble(float4 v, int64_t j0, int64_t D)
{
    uint32_t n = 0;
    n |= (v.x < 0.0f) ? 1u : 0u;
    n |= (j0 + 1 < D && v.y < 0.0f) ? 2u : 0u;
    n |= (j0 + 2 < D && v.z < 0.0f) ? 4u : 0u;
    n |= (j0 + 3 < D && v.w < 0.0f) ? 8u : 0u;
    return n;
}

// OR of the values of lanes l - 7 .. l, valid in lanes l = 7 (mod 8): three
// DPP row shifts (1, 2, 4) within the 16-lane row, no LDS traffic.
__device__ __forceinline__ uint32_t or8_into_last(uint32_t w)
{
    w |= static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(w), 0x111, 0xF, 0xF, true));
    w |= static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(w), 0x112, 0xF, 0xF, true));
    w |= static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(w), 0x114, 0xF, 0xF, true));
    return w;
}

// Merge the nibbles of 8 neighbouring lanes (gene quads 8w .. 8w+7) into
// word w and store it from the last lane of the group when the word holds
// genes (4 (8w) < D). Every lane of the wave must call this.
__device__ __forceinline__ void store_word(uint32_t nib, int64_t q, int64_t D, uint32_t *bits, int64_t ld, int64_t i)
{
    const uint32_t w = or8_into_last(nib << (4 * (threadIdx.x & 7)));
    if ((threadIdx.x & 7) == 7 && 4 * (q & ~int64_t(7)) < D) bits[(q >> 3) * ld + i] = w;
}

// DE for genes j0..j0+3 of individual i: v = clamp(fmaf(F, b - c, a)),
// u_j = v_j where ((w_j >> 8) 2^-24 <= CR) or j == jrand, else x_j, with
// the words w of Philox counter (j0 / 4, i, g, inst << 8 | DE_CR). The
// crossover test is taken on the raw word: w <= cr_max = cr_threshold(CR)
// holds exactly when (w >> 8) 2^-24 <= CR.
__device__ __forceinline__ float4 de_quad(float4 xv, float4 a, float4 b, float4 c, int64_t j0, int jrand, uint32_t i,
                                          uint32_t g, uint32_t inst, uint32_t k0, uint32_t k1, float F,
                                          uint32_t cr_max)
{
    const U4 r = philox10(static_cast<uint32_t>(j0 >> 2), i, g, (inst << 8) | kTagDeCr, k0, k1);
    const int rel = jrand - static_cast<int>(j0);  // D <= 2^30
    const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
    const float as[4] = {a.x, a.y, a.z, a.w};
    const float bs[4] = {b.x, b.y, b.z, b.w};
    const float cs[4] = {c.x, c.y, c.z, c.w};
    const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
    float us[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const bool take = (rw[e] <= cr_max) || (rel == e);
        const float v = clamp1(fmaf(F, bs[e] - cs[e], as[e]));
        us[e] = take ? v : xs[e];
    }
    return make_float4(us[0], us[1], us[2], us[3]);
}

// Grey-wolf update of gene quad q of a non-leader: per gene e and leader k,
// word t = 3e + k of the counters (3q + t / 4, i, g, inst << 8 | GWO) gives
// r1 = lo16 2^-16 and C = 2 r2 = hi16 2^-15; A = fmaf(2a, r1, -a),
// D_k = |fmaf(C, X_k, -x)|, Y_k = fmaf(-A, D_k, X_k); then the weighted
// combination (variant 0) or the mean (variant 1), divided by 3, clamped.
template <int VARIANT>
__device__ __forceinline__ float4 gwo_quad(float4 xv, float4 X0, float4 X1, float4 X2, uint32_t q, uint32_t i,
                                           uint32_t g, uint32_t inst, uint32_t k0, uint32_t k1, float a, float two_a)
{
    const uint32_t c3 = (inst << 8) | kTagGwo;
    const uint32_t cq = 3u * q;
    const float two_a_s = two_a * 0x1p-16f;
    const U4 wa = philox10(cq, i, g, c3, k0, k1);
    const U4 wb = philox10(cq + 1u, i, g, c3, k0, k1);
    const U4 wc = philox10(cq + 2u, i, g, c3, k0, k1);
    const uint32_t wrd[12] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w, wc.x, wc.y, wc.z, wc.w};
    const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
    const float Xs[3][4] = {{X0.x, X0.y, X0.z, X0.w}, {X1.x, X1.y, X1.z, X1.w}, {X2.x, X2.y, X2.z, X2.w}};
    float ys[4], ss[4], ns[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float Y[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t o = wrd[3 * e + k];
            // A = fmaf(2a, lo16 2^-16, -a) with the power of two moved onto
            // 2a: the product is the same real number (both scalings are
            // exact for a = 0 or a >= 2^-100), so A is the same float
            const float A = fmaf(two_a_s, static_cast<float>(o & 0xFFFFu), -a);
            const float Cc = static_cast<float>(o >> 16) * 0x1p-15f;  // = 2 r2, exactly
            const float Dk = fabsf(fmaf(Cc, Xs[k][e], -xs[e]));
            Y[k] = fmaf(-A, Dk, Xs[k][e]);
        }
        if constexpr (VARIANT == 1) {
            ys[e] = clamp1(div3((Y[0] + Y[1]) + Y[2]));
        } else {
            ss[e] = (fabsf(Y[0]) + fabsf(Y[1])) + fabsf(Y[2]);
            ns[e] = fmaf(fabsf(Y[2]), Y[2], fmaf(fabsf(Y[1]), Y[1], fabsf(Y[0]) * Y[0]));
        }
    }
    if constexpr (VARIANT == 0) {
        // |Y| <= 7, so s <= 21 and |num| <= 147: when every s and |num| of
        // the wave's quads is >= 2^-60, the division takes its short form
        // and, the quotient being nonzero, x / 3 needs no sign restore and
        // s == 0 cannot occur. Otherwise (tiny or zero weights) the full
        // IEEE division and the s == 0 case.
        const float lo = fminf(fminf(fminf(ss[0], fabsf(ns[0])), fminf(ss[1], fabsf(ns[1]))),
                               fminf(fminf(ss[2], fabsf(ns[2])), fminf(ss[3], fabsf(ns[3]))));
        if (__all(lo >= 0x1p-60f)) {
#pragma unroll
            for (int e = 0; e < 4; ++e) ys[e] = clamp1(div3_nonzero(div_in_range(ns[e], ss[e])));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // evaluated unconditionally (no divergent branch); the 0/0
                // of s == 0 is selected away
                const float qv = div3(ns[e] / ss[e]);
                ys[e] = clamp1(ss[e] == 0.0f ? 0.0f : qv);
            }
        }
    }
    return make_float4(ys[0], ys[1], ys[2], ys[3]);
}

// Improved discrete four-leader step (paper Sec. 3.1.2, as read here: the
// paper gives no formula) for the 4 genes of quad q of wolf i: one Philox
// word per gene (counter (q, i, g, inst << 8 | 5), word e); X0..X3 the
// leaders' genes (state +1 when >= 0); par = {t, 1 - 2 eps, eps, lambda}.
//   n = leaders in state +1; dist = n / 4; maj = 1, 0, 1/2 for n > 2, < 2, = 2;
//   p = fmaf(t, maj - dist, dist); p' = fmaf(1 - 2 eps, p, eps);
//   social learning when (w >> 16 & 0x3FFF) 2^-14 < lambda: the state of
//   leader w >> 30; else +1 when (w & 0xFFFF) 2^-16 < p', else -1.
__device__ __forceinline__ float4 dgwo_quad(float4 X0, float4 X1, float4 X2, float4 X3, uint32_t q, uint32_t i,
                                            uint32_t g, uint32_t inst, uint32_t k0, uint32_t k1, float4 par)
{
    const U4 w4 = philox10(q, i, g, (inst << 8) | kTagDgwo, k0, k1);
    const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
    const float Xs[4][4] = {{X0.x, X0.y, X0.z, X0.w}, {X1.x, X1.y, X1.z, X1.w}, {X2.x, X2.y, X2.z, X2.w},
                            {X3.x, X3.y, X3.z, X3.w}};
    float ys[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint32_t w = ws[e];
        uint32_t plus = 0;  // bit k: leader k in state +1
        int n = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t pk = Xs[k][e] < 0.0f ? 0u : 1u;
            plus |= pk << k;
            n += static_cast<int>(pk);
        }
        const float dist = static_cast<float>(n) * 0.25f;
        const float maj = n > 2 ? 1.0f : (n < 2 ? 0.0f : 0.5f);
        const float p = fmaf(par.x, maj - dist, dist);
        const float p2 = fmaf(par.y, p, par.z);
        const float us = static_cast<float>((w >> 16) & 0x3FFFu) * 0x1p-14f;
        const float up = static_cast<float>(w & 0xFFFFu) * 0x1p-16f;
        const bool st = us < par.w ? ((plus >> (w >> 30)) & 1u) != 0u : up < p2;
        ys[e] = st ? 1.0f : -1.0f;
    }
    return make_float4(ys[0], ys[1], ys[2], ys[3]);
}

}  // namespace qpm
