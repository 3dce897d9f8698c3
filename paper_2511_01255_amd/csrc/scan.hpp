// scan.hpp -- the per-domain walk of the d_eff double integral over one
// bit word of a genome, shared by the single-design and batched fitness
// kernels.
//
// Per genome, d_eff = sum_n d_n b_n P_{n-1} + C with P_n = sum_{m<=n} d_m a_m;
// a stretch of domains reduces to the triple (A, B, Q) = (sum d a, sum d b,
// sum d_n b_n (A before n)), and triples combine associatively:
// (A1,B1,Q1) + (A2,B2,Q2) = (A1+A2, B1+B2, Q1+Q2+A1 B2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace qpm {

// +-1.0 from bit k of w (bit set -> -1), as a double and as a float
__device__ __forceinline__ double sign64(uint32_t w, int k)
{
    const uint32_t hi = ((w << (31 - k)) & 0x80000000u) | 0x3ff00000u;
    return __hiloint2double(static_cast<int>(hi), 0);
}
__device__ __forceinline__ float sign32(uint32_t w, int k)
{
    return __uint_as_float(((w << (31 - k)) & 0x80000000u) | 0x3f800000u);
}

struct Tri {
    double ar, ai, br, bi, qr, qi;
};

// t <- t (+) u   (t covers the domains before u)
__device__ __forceinline__ void tri_append(Tri &t, const Tri &u)
{
    t.qr = fma(t.ar, u.br, fma(-t.ai, u.bi, t.qr + u.qr));
    t.qi = fma(t.ar, u.bi, fma(t.ai, u.br, t.qi + u.qi));
    t.ar += u.ar;
    t.ai += u.ai;
    t.br += u.br;
    t.bi += u.bi;
}

// Segment triples of genome i are stored as part[s][6][ld] (A, B, Q real
// and imaginary parts). The gy segments are split into NW contiguous
// ranges, range w = [gy w / NW, gy (w+1) / NW) folded in order by wave w of
// the workgroup (lane = genome); wave 0 then folds the NW range triples in
// order. Every caller uses this one association, so a genome's fitness has
// the same bits whichever kernel combines it. Call from every lane (the
// workgroup synchronises); the result is valid in wave 0.
template <int NW>
__device__ __forceinline__ Tri combine_segments_in(const double *__restrict__ part, int gy, int64_t ld, int64_t i,
                                                   bool valid, int wave, int lane, double *sh)
{
    const int s0 = static_cast<int>((static_cast<int64_t>(gy) * wave) / NW);
    const int s1 = static_cast<int>((static_cast<int64_t>(gy) * (wave + 1)) / NW);
    Tri t{0, 0, 0, 0, 0, 0};
    if (valid && s0 < s1) {
        const double *p = part + static_cast<int64_t>(s0) * 6 * ld + i;
        t = Tri{p[0], p[ld], p[2 * ld], p[3 * ld], p[4 * ld], p[5 * ld]};
#pragma unroll 4
        for (int sg = s0 + 1; sg < s1; ++sg) {
            const double *q = part + static_cast<int64_t>(sg) * 6 * ld + i;
            tri_append(t, Tri{q[0], q[ld], q[2 * ld], q[3 * ld], q[4 * ld], q[5 * ld]});
        }
    }
    if constexpr (NW > 1) {
        // sh: [6][NW][64] doubles of this group
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double v = c == 0 ? t.ar : c == 1 ? t.ai : c == 2 ? t.br : c == 3 ? t.bi : c == 4 ? t.qr : t.qi;
            sh[(c * NW + wave) * 64 + lane] = v;
        }
        __syncthreads();
        if (wave == 0) {
            for (int w = 1; w < NW; ++w) {
                const int a = static_cast<int>((static_cast<int64_t>(gy) * w) / NW);
                const int b = static_cast<int>((static_cast<int64_t>(gy) * (w + 1)) / NW);
                if (a < b)
                    tri_append(t, Tri{sh[(0 * NW + w) * 64 + lane], sh[(1 * NW + w) * 64 + lane],
                                      sh[(2 * NW + w) * 64 + lane], sh[(3 * NW + w) * 64 + lane],
                                      sh[(4 * NW + w) * 64 + lane], sh[(5 * NW + w) * 64 + lane]});
            }
        }
    }
    return t;
}

// combine_segments_in for a workgroup of NW waves over one group of 64
// genomes (wave = threadIdx.x / 64)
template <int NW>
__device__ __forceinline__ Tri combine_segments(const double *__restrict__ part, int gy, int64_t ld, int64_t i,
                                                bool valid)
{
    __shared__ double sh[6 * NW * 64];
    return combine_segments_in<NW>(part, gy, ld, i, valid, static_cast<int>(threadIdx.x >> 6),
                                   static_cast<int>(threadIdx.x & 63), sh);
}

__device__ __forceinline__ void store_fitness(void *fit, int out_f64, int64_t i, const Tri &t,
                                              const double *__restrict__ C)
{
    const double sr = t.qr + C[0], si = t.qi + C[1];
    const double f = fma(sr, sr, si * si);
    if (out_f64)
        static_cast<double *>(fit)[i] = f;
    else
        static_cast<float *>(fit)[i] = static_cast<float>(f);
}

// One word (32 domains) in FP64.
__device__ __forceinline__ void scan_word_f64(Tri &t, uint32_t word, const double4 *__restrict__ p)
{
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const double4 c = p[k];  // {a.re, a.im, b.re, b.im}, wave-uniform
        const double s = sign64(word, k);
        const double tr = fma(c.z, t.ar, -(c.w * t.ai));
        const double ti = fma(c.z, t.ai, c.w * t.ar);
        t.qr = fma(s, tr, t.qr);
        t.qi = fma(s, ti, t.qi);
        t.ar = fma(s, c.x, t.ar);
        t.ai = fma(s, c.y, t.ai);
        t.br = fma(s, c.z, t.br);
        t.bi = fma(s, c.w, t.bi);
    }
}

// One word in the FP32 form of the per-domain walk: the word's sums A and B
// in FP64 (they multiply, and are carried into, the long prefix of the
// design, where FP32 rounding would accumulate coherently over periodic
// sign patterns), its own Q in FP32 from a float copy of the running A and
// the float b; the word's triple is folded into t in FP64.
__device__ __forceinline__ void scan_word_f32(Tri &t, uint32_t word, const double4 *__restrict__ p64,
                                              const float4 *__restrict__ p32)
{
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
    float qr = 0.f, qi = 0.f;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const double4 c = p64[k];
        const float4 cf = p32[k];
        const double sd = sign64(word, k);
        const float s = sign32(word, k);
        const float fr = static_cast<float>(ar), fi = static_cast<float>(ai);
        const float tr = fmaf(cf.z, fr, -(cf.w * fi));
        const float ti = fmaf(cf.z, fi, cf.w * fr);
        qr = fmaf(s, tr, qr);
        qi = fmaf(s, ti, qi);
        ar = fma(sd, c.x, ar);
        ai = fma(sd, c.y, ai);
        br = fma(sd, c.z, br);
        bi = fma(sd, c.w, bi);
    }
    tri_append(t, Tri{ar, ai, br, bi, qr, qi});
}

// One word of the FP32 table walk. tb: the word's 8 blocks x R table rows x
// 16 patterns (row 0 A, then B and Q when R = 3): A and B are fixed-point
// integers at the word's scale 2^e and Q holds the float bits of Q 2^(2e);
// sc = 2^-e. A and B are summed exactly in 32-bit integers (the word scale
// keeps every partial sum below 2^31), the word's Q in FP32 from float
// copies of the running A and of B; the triple (only A when R = 1) is
// scaled back exactly and folded into t in FP64.
template <int R>
__device__ __forceinline__ void word_tab_q(Tri &t, uint32_t word, const int2 *__restrict__ tb, double sc)
{
    const uint32_t p0 = word & 15u;
    const int2 A0 = tb[p0];
    int ar = A0.x, ai = A0.y;
    if constexpr (R == 1) {
#pragma unroll
        for (int h = 1; h < 8; ++h) {
            const int2 A = tb[h * 16 + ((word >> (4 * h)) & 15u)];
            ar += A.x;
            ai += A.y;
        }
        t.ar += static_cast<double>(ar) * sc;
        t.ai += static_cast<double>(ai) * sc;
    } else {
        const int2 B0 = tb[16 + p0], Q0 = tb[32 + p0];
        int br = B0.x, bi = B0.y;
        float qr = __int_as_float(Q0.x), qi = __int_as_float(Q0.y);
#pragma unroll
        for (int h = 1; h < 8; ++h) {
            const uint32_t pt = (word >> (4 * h)) & 15u;
            const int2 A = tb[h * R * 16 + pt], B = tb[(h * R + 1) * 16 + pt], Q = tb[(h * R + 2) * 16 + pt];
            const float fr = static_cast<float>(ar), fi = static_cast<float>(ai);
            const float bx = static_cast<float>(B.x), by = static_cast<float>(B.y);
            qr = fmaf(-fi, by, fmaf(fr, bx, qr + __int_as_float(Q.x)));
            qi = fmaf(fi, bx, fmaf(fr, by, qi + __int_as_float(Q.y)));
            ar += A.x;
            ai += A.y;
            br += B.x;
            bi += B.y;
        }
        const double sc2 = sc * sc;
        tri_append(t, Tri{static_cast<double>(ar) * sc, static_cast<double>(ai) * sc, static_cast<double>(br) * sc,
                          static_cast<double>(bi) * sc, static_cast<double>(qr) * sc2, static_cast<double>(qi) * sc2});
    }
}

// One workgroup of the table kernels (GW genome groups of 64 x 4 segment
// waves, lane = genome) over the words [wbase, wbase + 4 wpw) of a design
// of W words: `bits` and the tables point at the design's word 0; the
// workgroup copies the tables of its words to `lds` (table_lds_bytes), each
// wave walks wpw words of its segment, and the 4 segment triples of each
// genome are folded in order. Returns true (with the workgroup's triple in
// t) in the first segment wave of each group for genomes i < np, where
// i = (blockIdx.x GW + group) 64 + lane. Every lane of the workgroup must
// call it (it synchronises the workgroup). FP32 walks the fixed-point
// tables tabq at the word scales wsc (word_tab_q), FP64 the tables tab64.
template <bool F32, int GW>
__device__ __forceinline__ bool tab_segment(Tri &t, const uint32_t *__restrict__ bits, int64_t ld, int W, int wbase,
                                            const double2 *__restrict__ tab64, const int2 *__restrict__ tabq,
                                            const double *__restrict__ wsc, int wpw, int64_t np, unsigned char *lds)
{
    constexpr int SW = 4;
    constexpr int NT = GW * 256;
    constexpr int MAXW = table_max_wpw(F32);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int gsub = wave / SW, ssub = wave % SW;
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * GW + gsub) * 64 + lane;
    const int nw = min(W - wbase, SW * wpw);  // >= 1 by the grid
    // the tables of words [wbase, wbase + nw) go straight to LDS (16 bytes
    // per lane per load, no registers, no wait between loads)
    {
        const int n16 = nw * 8 * 48 * (F32 ? 8 : 16) / 16;
        const uint4 *src = F32 ? reinterpret_cast<const uint4 *>(tabq + static_cast<int64_t>(wbase) * 8 * 48)
                               : reinterpret_cast<const uint4 *>(tab64 + static_cast<int64_t>(wbase) * 8 * 48);
        for (int k = 0; k * NT < n16; ++k) {
            const int idx = k * NT + static_cast<int>(threadIdx.x);
            if (idx < n16)
                __builtin_amdgcn_global_load_lds(
                    src + idx, reinterpret_cast<__attribute__((address_space(3))) void *>(
                                   reinterpret_cast<uintptr_t>(lds + static_cast<size_t>(k * NT + wave * 64) * 16)),
                    16, 0, 0);
        }
    }
    // this wave's bit words, loaded while the tables arrive (clamped
    // addresses, so every load is in bounds and none is branched around)
    const bool live = i < np;
    const int w0 = ssub * wpw, w1 = min(nw, w0 + wpw);
    const int64_t ic = i < ld ? i : ld - 1;
    uint32_t wv[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) wv[k] = bits[static_cast<int64_t>(min(wbase + w0 + k, W - 1)) * ld + ic];
    // keep the loads here, issued together with the table copies (the
    // compiler would otherwise sink each one to its first use, one memory
    // latency per word)
#pragma unroll
    for (int k = 0; k < MAXW; ++k) asm volatile("" ::"v"(wv[k]));
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    t = Tri{0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
        const int wr = w0 + k;
        if (wr >= w1) break;
        const uint32_t word = live ? wv[k] : 0u;
        if constexpr (F32) {
            word_tab_q<3>(t, word, reinterpret_cast<const int2 *>(lds) + wr * 8 * 48, wsc[wbase + wr]);
        } else {
            const double2 *tb = reinterpret_cast<const double2 *>(lds) + wr * 8 * 48;
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const uint32_t pt = (word >> (4 * h)) & 15u;
                const double2 A = tb[h * 48 + pt], B = tb[h * 48 + 16 + pt], Q = tb[h * 48 + 32 + pt];
                t.qr = fma(-t.ai, B.y, fma(t.ar, B.x, t.qr + Q.x));
                t.qi = fma(t.ai, B.x, fma(t.ar, B.y, t.qi + Q.y));
                t.ar += A.x;
                t.ai += A.y;
                t.br += B.x;
                t.bi += B.y;
            }
        }
    }
    // the 4 segment triples of each genome group, in order, through LDS
    // (the tables are no longer read)
    __syncthreads();
    double *sh = reinterpret_cast<double *>(lds);  // [6][GW * SW][64]
    constexpr int NWV = GW * SW;
    sh[(0 * NWV + wave) * 64 + lane] = t.ar;
    sh[(1 * NWV + wave) * 64 + lane] = t.ai;
    sh[(2 * NWV + wave) * 64 + lane] = t.br;
    sh[(3 * NWV + wave) * 64 + lane] = t.bi;
    sh[(4 * NWV + wave) * 64 + lane] = t.qr;
    sh[(5 * NWV + wave) * 64 + lane] = t.qi;
    __syncthreads();
    if (ssub != 0 || !live) return false;
#pragma unroll 1
    for (int s2 = 1; s2 < SW; ++s2) {
        if (s2 * wpw >= nw) break;
        const int v = gsub * SW + s2;
        tri_append(t, Tri{sh[(0 * NWV + v) * 64 + lane], sh[(1 * NWV + v) * 64 + lane], sh[(2 * NWV + v) * 64 + lane],
                          sh[(3 * NWV + v) * 64 + lane], sh[(4 * NWV + v) * 64 + lane],
                          sh[(5 * NWV + v) * 64 + lane]});
    }
    return true;
}

}  // namespace qpm
