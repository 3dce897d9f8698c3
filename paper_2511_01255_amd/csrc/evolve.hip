// evolve.hip -- the optimiser steps around the fitness: initialisation, DE
// rand/1 mutation + binomial crossover (paper Sec. 2.2.1), the grey-wolf
// update of the omega wolves (paper Sec. 2.2.2), greedy selection and the
// leader (top-3) reduction (paper Sec. 3.2 steps 2-5).
//
// Layout: genes are float rows (row stride ldx, a multiple of 4) so that a
// lane moves one float4 (a gene quad) per row; a workgroup of 256 lanes
// covers 1024 genes of one individual, so the individual index -- and with
// it the donor / leader rows and the per-individual Philox draws -- is
// uniform across the workgroup and lives in scalar registers. The +-1 bits
// of a quad (4 bits) are merged across 8 neighbouring lanes with xor
// shuffles into one 32-gene word of the population-major layout.
//
// Binary32 arithmetic here is spelled out with explicit fmaf and the
// library is built with -ffp-contract=off, so trial and candidate genes are
// bit-for-bit what these formulas state.
#include <cfloat>
#include <climits>
#include <vector>

#include "common.hpp"
#include "device_common.hpp"
#include "genes.hpp"

namespace qpm {

// ------------------------------------------------------------ initialisation

__global__ __launch_bounds__(256) void init_kernel(int64_t D, int64_t ldx, uint32_t k0, uint32_t k1, uint32_t inst,
                                                   float *__restrict__ x, uint32_t *__restrict__ bits, int64_t ld)
{
    const int64_t i = blockIdx.x;
    const int64_t q = static_cast<int64_t>(blockIdx.y) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) {
        const U4 r = philox10(static_cast<uint32_t>(q), static_cast<uint32_t>(i), 0u, (inst << 8) | kTagInit, k0, k1);
        const float4 v = make_float4(sym24(r.x), sym24(r.y), sym24(r.z), sym24(r.w));
        store_quad(x + i * ldx, j0, D, v);
        nib = quad_nibble(v, j0, D);
    }
    store_word(nib, q, D, bits, ld, i);
}

// ------------------------------------------------------------ DE rand/1 + binomial crossover

// One draw per individual and generation, shared by every gene chunk.
__global__ __launch_bounds__(256) void de_draws_kernel(int64_t np, int64_t D, uint32_t k0, uint32_t k1,
                                                       const uint32_t *__restrict__ gen_dev, uint32_t gen_c,
                                                       uint32_t inst, int4 *__restrict__ draws)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= np) return;
    const uint32_t g = gen_dev ? gen_dev[0] : gen_c;
    draws[i] = de_draw(i, np, D, g, inst, k0, k1);
}

// Work split: a lane moves one gene quad (float4). A chunk is CW = 256 /
// IPW genes; one wave covers IPW individuals of a chunk (64 / IPW lanes
// each) and a 256-lane workgroup covers IPG = 4 IPW consecutive
// individuals per pass, R passes over R IPG consecutive individuals. The
// rows of pass r + 1 are loaded before the trials of pass r are stored, so
// two passes' reads are in flight per wave. Chunks are dealt to the eight
// XCDs round-robin (workgroup id mod 8 = XCD) and every XCD walks its
// chunks in order over all individuals, so while it works on a chunk that
// slice of the whole population (np x CW x 4 bytes, chosen <= 2 MB) stays in
// the XCD's L2 and the random donor rows hit it.
//
// Each row's buffer is named by its flag. PACKED (a run's population: the
// two buffers are one allocation, x1 = x0 + np ldx, out0 = x0, out1 = x1,
// np <= 65536, ldx < 2^24): the workgroup first copies the flags, packed one
// bit per individual, to LDS; row r of buffer b is then row r + b np of one
// array, addressed with 24-bit multiplies, so a donor address costs an LDS
// read and a few ALU operations instead of a second dependent global load.
// Otherwise the flags (if any) are read from global memory.
template <int IPW, int R, bool PACKED>
__global__ __launch_bounds__(256) void de_kernel(PopView pv, const int4 *__restrict__ draws,
                                                 const uint32_t *__restrict__ fbits, float F,
                                                 const float *__restrict__ F_tab, uint32_t cr_max,
                                                 uint32_t k0, uint32_t k1, const uint32_t *__restrict__ gen_dev,
                                                 uint32_t gen_c, uint32_t inst, uint32_t *__restrict__ bits,
                                                 int64_t ld, int groups, int chunks, int store_genes,
                                                 uint32_t *__restrict__ reset_cnt)
{
    constexpr int LPI = 64 / IPW;  // lanes per individual
    constexpr int CW = 4 * LPI;    // genes per chunk
    constexpr int WPC = CW / 32;   // bit words per chunk and individual
    constexpr int IPG = 4 * IPW;   // individuals per workgroup pass
    constexpr int IPB = R * IPG;   // individuals per workgroup
    static_assert(IPB * WPC <= 256, "one bit word per thread at the end");
    const uint32_t b = blockIdx.x;
    const int xcd = static_cast<int>(b & 7u);
    const int k = static_cast<int>(b >> 3);
    const int gi = k % groups;
    const int c = xcd + 8 * (k / groups);
    if (c >= chunks) return;
    const int t = threadIdx.x;
    const int local = t / LPI;  // individual within a pass
    const int li = t % LPI;     // lane within the individual
    const int64_t D = pv.D, np = pv.np;
    const int64_t i0 = static_cast<int64_t>(gi) * IPB + local;
    const int64_t j0 = static_cast<int64_t>(c) * CW + 4 * li;
    const uint32_t g = gen_dev ? gen_dev[0] : gen_c;
    const float Fg = F_tab ? F_tab[g] : F;  // a run's per-generation F
    // a run without stored trials: the list counter of the accepted trials
    // starts at 0 for this generation (the finish step appends to it)
    if (reset_cnt != nullptr && b == 0 && threadIdx.x == 0) reset_cnt[0] = 0u;
    __shared__ uint32_t wsh[IPB][WPC];
    extern __shared__ uint32_t sfb[];  // PACKED: (np + 31) / 32 flag words
    // PACKED: per individual of the workgroup, the float offsets from x0 of
    // its target row, its three donor rows and its output row, and jrand,
    // worked out once by one lane instead of by every lane of every pass
    __shared__ uint64_t soff[PACKED ? IPB : 1][5];
    __shared__ int sjr[PACKED ? IPB : 1];
    int4 dr[PACKED ? 1 : R];
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r) act[r] = i0 + r * IPG < np && j0 < D;
    const uint32_t np32 = static_cast<uint32_t>(np), ldx24 = static_cast<uint32_t>(pv.ldx) & 0xFFFFFFu;
    // PACKED: float offset of row r of buffer (flag of r) ^ flip from x0
    auto packed_row = [&](int64_t r, uint32_t flip) -> uint64_t {
        const uint32_t rr = static_cast<uint32_t>(r);
        const uint32_t b = ((sfb[rr >> 5] >> (rr & 31u)) & 1u) ^ flip;
        const uint32_t row = (rr + b * np32) & 0xFFFFFFu;
        return static_cast<uint64_t>(row) * ldx24;
    };
    if constexpr (PACKED) {
        // lane t < IPB loads the draws of individual gi IPB + t; the load is
        // in flight while the flags are staged
        const int64_t ip = static_cast<int64_t>(gi) * IPB + t;
        int4 d4 = make_int4(0, 0, 0, 0);
        if (t < IPB) d4 = draws[ip < np ? ip : np - 1];
        for (int k = t; k < static_cast<int>((np + 31) / 32); k += 256) sfb[k] = fbits[k];
        __syncthreads();
        if (t < IPB && ip < np) {
            soff[t][0] = packed_row(ip, 0u);
            soff[t][1] = packed_row(d4.x, 0u);
            soff[t][2] = packed_row(d4.y, 0u);
            soff[t][3] = packed_row(d4.z, 0u);
            soff[t][4] = packed_row(ip, 1u);
            sjr[t] = d4.w;
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = i0 + r * IPG;
            dr[r] = draws[i < np ? i : np - 1];
        }
    }
    auto second = [&](int64_t r) -> bool { return pv.flags != nullptr && pv.flags[r] != 0u; };
    auto src = [&](int64_t r) -> const float * { return (second(r) ? pv.x1 : pv.x0) + r * pv.ldx; };
    // two row buffers used alternately by the passes (the pass loop is
    // unrolled, so each pass names its buffers statically and the next
    // pass's rows load without a register copy)
    float4 buf0[4], buf1[4];
    auto load = [&](int r, float4 *v) {
        if (act[r]) {
            if constexpr (PACKED) {
                const uint64_t *o = soff[r * IPG + local];
#pragma unroll
                for (int m = 0; m < 4; ++m) v[m] = *reinterpret_cast<const float4 *>(pv.x0 + o[m] + j0);
            } else {
                const int64_t i = i0 + r * IPG;
                v[0] = *reinterpret_cast<const float4 *>(src(i) + j0);
                v[1] = *reinterpret_cast<const float4 *>(src(dr[r].x) + j0);
                v[2] = *reinterpret_cast<const float4 *>(src(dr[r].y) + j0);
                v[3] = *reinterpret_cast<const float4 *>(src(dr[r].z) + j0);
            }
        }
    };
    load(0, buf0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float4 *cur = (r & 1) ? buf1 : buf0;
        if (r + 1 < R) load(r + 1, (r & 1) ? buf0 : buf1);
        uint32_t nib = 0;
        if (act[r]) {
            const int64_t i = i0 + r * IPG;
            int jrand;
            if constexpr (PACKED)
                jrand = sjr[r * IPG + local];
            else
                jrand = dr[r].w;
            const float4 uv = de_quad(cur[0], cur[1], cur[2], cur[3], j0, jrand, static_cast<uint32_t>(i), g, inst, k0,
                                      k1, Fg, cr_max);
            if (store_genes) {
                float *dst;
                if constexpr (PACKED)
                    dst = pv.out0 + soff[r * IPG + local][4];
                else
                    dst = (second(i) ? pv.out0 : pv.out1) + i * pv.ldx;
                store_quad_nt(dst, j0, D, uv);
            }
            nib = quad_nibble(uv, j0, D);
        }
        // merge the nibbles of 8 neighbouring lanes (32 genes) into one word
        const uint32_t w = or8_into_last(nib << (4 * (t & 7)));
        if ((t & 7) == 7) wsh[r * IPG + local][li >> 3] = w;
    }
    __syncthreads();
    // the IPB consecutive individuals of this workgroup share each bit row:
    // one contiguous store of IPB words per chunk word
    if (t < IPB * WPC) {
        const int wd = t / IPB, ii = t % IPB;
        const int64_t row = static_cast<int64_t>(gi) * IPB + ii;
        const int64_t wg = static_cast<int64_t>(c) * WPC + wd;
        if (row < np && wg * 32 < D) bits[wg * ld + row] = wsh[ii][wd];
    }
}

// The accepted trials of a run whose DE step stored only their bits: the
// trial genes of every individual in list[0 .. cnt) are computed again,
// exactly as the DE kernel computed them (same draws, words and de_quad),
// from the population before the selection (fb_old: its packed flags), and
// written to the buffer that the selection made current. A work item is
// (chunk of 256 genes, listed individual) for one wave. Chunk c belongs to
// XCD c mod 8 (workgroup x runs on XCD x mod 8), and each XCD walks its
// items chunk by chunk, so the waves running together on an XCD read the
// same chunk of many rows and donor rows shared between accepted trials
// come from its L2. The grid is fixed; every wave loops until its XCD's
// items run out. With top3_out, workgroup 0 first merges the finish step's
// leader candidates (3 per group of 64) into the leaders, which saves the
// finish step a one-workgroup kernel (the grey-wolf step after this kernel
// reads them).
__global__ __launch_bounds__(256) void materialize_kernel(PopView pv, const int4 *__restrict__ draws,
                                                          const uint32_t *__restrict__ fb_old, float F,
                                                          const float *__restrict__ F_tab, uint32_t cr_max,
                                                          uint32_t k0, uint32_t k1, const uint32_t *__restrict__ gen,
                                                          uint32_t inst, const int32_t *__restrict__ list,
                                                          const uint32_t *__restrict__ cnt, const void *cand,
                                                          int64_t ngroups, int cand_f64, int32_t *top3_out)
{
    extern __shared__ uint32_t sfb[];  // (np + 31) / 32 old flag words
    if (top3_out != nullptr && blockIdx.x == 0) {
        // cand: 3 values per group (T) followed by 3 slots per group
        if (cand_f64) {
            const double *cv = static_cast<const double *>(cand);
            block_top3<double, 256>(cv, 3 * ngroups, top3_out, reinterpret_cast<const int32_t *>(cv + 3 * ngroups));
        } else {
            const float *cv = static_cast<const float *>(cand);
            block_top3<float, 256>(cv, 3 * ngroups, top3_out, reinterpret_cast<const int32_t *>(cv + 3 * ngroups));
        }
    }
    const int64_t np = pv.np, D = pv.D;
    for (int k = threadIdx.x; k < static_cast<int>((np + 31) / 32); k += 256) sfb[k] = fb_old[k];
    __syncthreads();
    const uint32_t g = gen[0];
    const float Fg = F_tab ? F_tab[g] : F;
    // np <= 65536 and D < 2^24 (checked by the launcher), so the item
    // counts fit 32 bits
    const uint32_t n_acc = static_cast<uint32_t>(min(static_cast<int64_t>(cnt[0]), np));
    const uint32_t chunks = static_cast<uint32_t>((D + 255) / 256);
    const uint32_t xcd = blockIdx.x & 7u;
    const uint32_t stride = (gridDim.x / 8) * 4;  // the waves of one XCD (the grid is a multiple of 8)
    const uint32_t my_chunks = chunks > xcd ? (chunks - xcd + 7) / 8 : 0;
    const int lane = threadIdx.x & 63;
    // the wave index is the same in all lanes: the item walk below is
    // scalar, and so are an item's individual, draws and row offsets
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t np32 = static_cast<uint32_t>(np), ldx24 = static_cast<uint32_t>(pv.ldx) & 0xFFFFFFu;
    auto row = [&](uint32_t rr, uint32_t flip) -> const float * {
        const uint32_t b = __builtin_amdgcn_readfirstlane((sfb[rr >> 5] >> (rr & 31u)) & 1u) ^ flip;
        return pv.x0 + static_cast<uint64_t>((rr + b * np32) & 0xFFFFFFu) * ldx24;
    };
    if (n_acc == 0 || my_chunks == 0) return;
    // item it = (chunk slot cq, list entry ir) with it = cq n_acc + ir,
    // stepped by `stride` without a division
    uint32_t it = (blockIdx.x >> 3) * 4 + wave;
    uint32_t cq = it / n_acc, ir = it - cq * n_acc;
    const uint32_t sq = stride / n_acc, sr = stride - sq * n_acc;
    for (; cq < my_chunks; cq += sq, ir += sr) {
        if (ir >= n_acc) {
            ir -= n_acc;
            ++cq;
            if (cq >= my_chunks) break;
        }
        const int64_t j0 = static_cast<int64_t>(xcd + 8 * cq) * 256 + 4 * lane;
        const int32_t iv = list[ir];
        if (iv < 0 || iv >= np || j0 >= D) continue;
        const uint32_t i = static_cast<uint32_t>(iv);
        const int4 dr = draws[i];
        const float4 xv = *reinterpret_cast<const float4 *>(row(i, 0u) + j0);
        const float4 a = *reinterpret_cast<const float4 *>(row(static_cast<uint32_t>(dr.x), 0u) + j0);
        const float4 bq = *reinterpret_cast<const float4 *>(row(static_cast<uint32_t>(dr.y), 0u) + j0);
        const float4 cv = *reinterpret_cast<const float4 *>(row(static_cast<uint32_t>(dr.z), 0u) + j0);
        const float4 uv = de_quad(xv, a, bq, cv, j0, dr.w, i, g, inst, k0, k1, Fg, cr_max);
        store_quad_nt(const_cast<float *>(row(i, 1u)), j0, D, uv);
    }
}

qpm_status launch_materialize(const PopView &pv, const int4 *draws, const uint32_t *fb_old, float F,
                              const float *F_tab, float CR, uint64_t seed, const uint32_t *gen, uint32_t inst,
                              const int32_t *list, const uint32_t *cnt, hipStream_t s, const void *cand,
                              int64_t ngroups, bool f64, int32_t *top3_out)
{
    QPM_REQUIRE(top3_out == nullptr || cand != nullptr, QPM_EINVAL, "merging leaders needs the candidates");
    QPM_REQUIRE(pv.np <= 65536 && pv.ldx < (int64_t(1) << 24) && pv.x1 == pv.x0 + pv.np * pv.ldx &&
                    pv.out0 == pv.x0 && pv.out1 == pv.x1,
                QPM_EINVAL, "materialising trials needs one allocation for both gene buffers");
    const size_t lds = sizeof(uint32_t) * static_cast<size_t>((pv.np + 31) / 32);
    materialize_kernel<<<2048, 256, lds, s>>>(pv, draws, fb_old, F, F_tab, cr_threshold(CR),
                                              static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), gen,
                                              inst, list, cnt, cand, ngroups, f64 ? 1 : 0, top3_out);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

// ------------------------------------------------------------ grey-wolf update

// Grid x = 8 ceil(np / 8): workgroup x runs on XCD x mod 8 (gridDim.x is a
// multiple of 8, so this holds for every y) and takes individual
// (x mod 8) ceil(np / 8) + x / 8. Each XCD thus owns a contiguous range of
// individuals and the 32-bit bit words of neighbouring individuals, which
// share cache lines, are written from one L2 instead of eight.
template <int VARIANT>
__global__ __launch_bounds__(256) void gwo_kernel(PopView pv, const int32_t *__restrict__ leaders, int4 lead_c,
                                                  const float *__restrict__ a_tab, float a_c, uint32_t k0, uint32_t k1,
                                                  const uint32_t *__restrict__ gen_dev, uint32_t gen_c, uint32_t inst,
                                                  uint32_t *__restrict__ bits, int64_t ld, int64_t per_xcd)
{
    const int64_t np = pv.np, D = pv.D;
    const int64_t i = static_cast<int64_t>(blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
    if (i >= np) return;
    // leaders from the device (runs) or by value (the entry point)
    const int64_t L0 = leaders ? leaders[0] : lead_c.x, L1 = leaders ? leaders[1] : lead_c.y,
                  L2 = leaders ? leaders[2] : lead_c.z;
    // leaders keep their positions; indices outside the population make
    // the launch a no-op instead of an out-of-bounds read
    if (i == L0 || i == L1 || i == L2) return;
    if (L0 < 0 || L0 >= np || L1 < 0 || L1 >= np || L2 < 0 || L2 >= np) return;
    const uint32_t g = gen_dev ? gen_dev[0] : gen_c;
    const float a = a_tab ? a_tab[g] : a_c;
    const float two_a = 2.0f * a;

    const int64_t q = static_cast<int64_t>(blockIdx.y) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) {
        const float4 xv = *reinterpret_cast<const float4 *>(row_of(pv, i) + j0);
        const float4 X0 = *reinterpret_cast<const float4 *>(row_of(pv, L0) + j0);
        const float4 X1 = *reinterpret_cast<const float4 *>(row_of(pv, L1) + j0);
        const float4 X2 = *reinterpret_cast<const float4 *>(row_of(pv, L2) + j0);
        const float4 yv4 = gwo_quad<VARIANT>(xv, X0, X1, X2, static_cast<uint32_t>(q), static_cast<uint32_t>(i), g,
                                             inst, k0, k1, a, two_a);
        store_quad_nt(out_row_of(pv, i), j0, D, yv4);
        nib = quad_nibble(yv4, j0, D);
    }
    store_word(nib, q, D, bits, ld, i);
}

// Improved discrete four-leader step (dgwo_quad), same grid as gwo_kernel.
// The new genes depend on the leaders' genes only, so the wolf's own row is
// not read. leaders: alpha, beta, delta (kept), then the fourth.
__global__ __launch_bounds__(256) void dgwo_kernel(PopView pv, const int32_t *__restrict__ leaders, int4 lead_c,
                                                   const float4 *__restrict__ par_tab, float4 par_c, uint32_t k0,
                                                   uint32_t k1, const uint32_t *__restrict__ gen_dev, uint32_t gen_c,
                                                   uint32_t inst, uint32_t *__restrict__ bits, int64_t ld,
                                                   int64_t per_xcd)
{
    const int64_t np = pv.np, D = pv.D;
    const int64_t i = static_cast<int64_t>(blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
    if (i >= np) return;
    const int64_t L0 = leaders ? leaders[0] : lead_c.x, L1 = leaders ? leaders[1] : lead_c.y,
                  L2 = leaders ? leaders[2] : lead_c.z, L3 = leaders ? leaders[3] : lead_c.w;
    if (i == L0 || i == L1 || i == L2) return;
    if (L0 < 0 || L0 >= np || L1 < 0 || L1 >= np || L2 < 0 || L2 >= np || L3 < 0 || L3 >= np) return;
    const uint32_t g = gen_dev ? gen_dev[0] : gen_c;
    const float4 par = par_tab ? par_tab[g] : par_c;
    const int64_t q = static_cast<int64_t>(blockIdx.y) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) {
        const float4 X0 = *reinterpret_cast<const float4 *>(row_of(pv, L0) + j0);
        const float4 X1 = *reinterpret_cast<const float4 *>(row_of(pv, L1) + j0);
        const float4 X2 = *reinterpret_cast<const float4 *>(row_of(pv, L2) + j0);
        const float4 X3 = *reinterpret_cast<const float4 *>(row_of(pv, L3) + j0);
        const float4 yv4 = dgwo_quad(X0, X1, X2, X3, static_cast<uint32_t>(q), static_cast<uint32_t>(i), g, inst, k0,
                                     k1, par);
        store_quad_nt(out_row_of(pv, i), j0, D, yv4);
        nib = quad_nibble(yv4, j0, D);
    }
    store_word(nib, q, D, bits, ld, i);
}

// The fourth leader: the best genome (f descending, slot ascending) other
// than leaders[0..2], into leaders[3]. One workgroup; the order is total,
// so the result does not depend on the reduction order.
template <typename T>
__global__ __launch_bounds__(1024) void fourth_kernel(const T *__restrict__ f, int64_t np, int32_t *__restrict__ leaders)
{
    __shared__ T sv[16];
    __shared__ int si[16];
    const int64_t L0 = leaders[0], L1 = leaders[1], L2 = leaders[2];
    T bv = static_cast<T>(-INFINITY);
    int bi = INT_MAX;
    for (int64_t k = threadIdx.x; k < np; k += 1024) {
        if (k == L0 || k == L1 || k == L2) continue;
        const T v = f[k];
        if (v > bv || (v == bv && static_cast<int>(k) < bi)) {
            bv = v;
            bi = static_cast<int>(k);
        }
    }
    for (int o = 1; o < 64; o <<= 1) {
        const T ov = __shfl_xor(bv, o);
        const int oi = __shfl_xor(bi, o);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = bv;
        si[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w)
            if (sv[w] > bv || (sv[w] == bv && si[w] < bi)) {
                bv = sv[w];
                bi = si[w];
            }
        leaders[3] = bi;
    }
}

// ------------------------------------------------------------ top-3

template <typename T>
__global__ __launch_bounds__(1024) void top3_kernel(const T *__restrict__ f, int64_t np, int32_t *__restrict__ out)
{
    block_top3<T, 1024>(f, np, out);
}

// ------------------------------------------------------------ gather / pack

__global__ __launch_bounds__(256) void gather_kernel(PopView pv, const int32_t *__restrict__ rows,
                                                     float *__restrict__ out, int64_t ldo)
{
    const int64_t r = blockIdx.y;
    const int64_t src = rows ? rows[r] : r;
    const float *x = row_of(pv, src);
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; j < pv.D; j += 256 * gridDim.x)
        out[r * ldo + j] = x[j];
}

__global__ __launch_bounds__(256) void pack_pop_kernel(const float *__restrict__ x, int64_t D, int64_t ldx,
                                                       uint32_t *__restrict__ bits, int64_t ld)
{
    const int64_t i = blockIdx.x;
    const int64_t q = static_cast<int64_t>(blockIdx.y) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) nib = quad_nibble(*reinterpret_cast<const float4 *>(x + i * ldx + j0), j0, D);
    store_word(nib, q, D, bits, ld, i);
}

__global__ __launch_bounds__(256) void pack_row_kernel(const float *__restrict__ x, int64_t D,
                                                       uint32_t *__restrict__ bits)
{
    const int64_t w = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (32 * w >= D) return;
    uint32_t v = 0;
    for (int k = 0; k < 32; ++k) {
        const int64_t j = 32 * w + k;
        if (j < D && x[j] < 0.0f) v |= 1u << k;
    }
    bits[w] = v;
}

// ------------------------------------------------------------ launchers

// x = individual (fastest in dispatch order), y = 1024-gene chunk: all
// individuals of one chunk run before the next chunk, so the random donor
// rows of DE hit the caches (one chunk of the whole population is
// np x 4 KB) instead of streaming the population from HBM three times.
static dim3 quad_grid(int64_t D, int64_t rows)
{
    const int64_t quads = (D + 3) / 4;
    return dim3(static_cast<unsigned>(rows), static_cast<unsigned>((quads + 255) / 256));
}

// grid.x holds rows (< 2^31) and grid.y the 1024-gene chunks (<= 65535)
static qpm_status check_quad_grid(int64_t D, int64_t rows)
{
    QPM_REQUIRE(rows < (int64_t(1) << 31), QPM_ERANGE, "too many rows for one launch (%lld)", (long long)rows);
    QPM_REQUIRE((D + 1023) / 1024 <= 65535, QPM_ERANGE, "D = %lld exceeds 65535 chunks of 1024 genes",
                (long long)D);
    return QPM_OK;
}

qpm_status launch_init(int64_t np, int64_t D, int64_t ldx, uint64_t seed, uint32_t inst, float *x, uint32_t *bits,
                       int64_t ld, hipStream_t s)
{
    const qpm_status st = check_quad_grid(D, np);
    if (st != QPM_OK) return st;
    init_kernel<<<quad_grid(D, np), 256, 0, s>>>(D, ldx, static_cast<uint32_t>(seed),
                                                 static_cast<uint32_t>(seed >> 32), inst, x, bits, ld);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_de(const PopView &pv, float F, float CR, uint64_t seed, const uint32_t *gen_dev, uint32_t gen,
                     uint32_t inst, uint32_t *bits, int64_t ld, int4 *draws, bool compute_draws, hipStream_t s,
                     int ipw_req, int passes, const uint32_t *fbits, const float *F_tab, bool store_genes,
                     uint32_t *reset_cnt)
{
    QPM_REQUIRE(F_tab == nullptr || gen_dev != nullptr, QPM_EINVAL, "an F table needs the device generation");
    QPM_REQUIRE(store_genes || fbits != nullptr, QPM_EINVAL, "trials that are not stored need the packed flags");
    // the packed-flag path: one allocation for both buffers, flags staged
    // in LDS (at most 65536 individuals, 8 KB), 24-bit row arithmetic
    const bool packed = fbits != nullptr && pv.np <= 65536 && pv.ldx < (int64_t(1) << 24) &&
                        pv.x1 == pv.x0 + pv.np * pv.ldx && pv.out0 == pv.x0 && pv.out1 == pv.x1;
    const size_t lds = packed ? sizeof(uint32_t) * static_cast<size_t>((pv.np + 31) / 32) : 0;
    const uint32_t cr_max = cr_threshold(CR);
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    if (compute_draws)
        de_draws_kernel<<<static_cast<unsigned>((pv.np + 255) / 256), 256, 0, s>>>(pv.np, pv.D, k0, k1, gen_dev,
                                                                                   gen, inst, draws);
    // individuals per wave so that one chunk of the population fits in 2 MB
    const int64_t row_bytes = 2 * 1024 * 1024 / pv.np;
    const int ipw_auto = row_bytes >= 1024 ? 1 : (row_bytes >= 512 ? 2 : 4);
    const int ipw = (ipw_req == 1 || ipw_req == 2 || ipw_req == 4) ? ipw_req : ipw_auto;
    const int R = (passes == 2 || passes == 4) ? passes : 1;
    const int64_t cw = 256 / ipw;
    const int64_t chunks = (pv.D + cw - 1) / cw;
    const int64_t groups = (pv.np + 4 * ipw * R - 1) / (4 * ipw * R);
    const int64_t blocks = 8 * ((chunks + 7) / 8) * groups;
    QPM_REQUIRE(blocks < (int64_t(1) << 31), QPM_ERANGE, "population too large for one DE launch");
    const int gr = static_cast<int>(groups), ch = static_cast<int>(chunks);
    const unsigned nb = static_cast<unsigned>(blocks);
#define QPM_DE(I, P)                                                                                            \
    if (packed)                                                                                                 \
        de_kernel<I, P, true><<<nb, 256, lds, s>>>(pv, draws, fbits, F, F_tab, cr_max, k0, k1, gen_dev, gen,     \
                                                   inst, bits, ld, gr, ch, store_genes ? 1 : 0, reset_cnt);     \
    else                                                                                                        \
        de_kernel<I, P, false><<<nb, 256, 0, s>>>(pv, draws, nullptr, F, F_tab, cr_max, k0, k1, gen_dev, gen,    \
                                                  inst, bits, ld, gr, ch, store_genes ? 1 : 0, reset_cnt);
    if (ipw == 1) {
        if (R == 1) { QPM_DE(1, 1) } else if (R == 2) { QPM_DE(1, 2) } else { QPM_DE(1, 4) }
    } else if (ipw == 2) {
        if (R == 1) { QPM_DE(2, 1) } else if (R == 2) { QPM_DE(2, 2) } else { QPM_DE(2, 4) }
    } else {
        if (R == 1) { QPM_DE(4, 1) } else if (R == 2) { QPM_DE(4, 2) } else { QPM_DE(4, 4) }
    }
#undef QPM_DE
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_dgwo(const PopView &pv, const int32_t *leaders, const float4 *par_tab, float4 par,
                       uint64_t seed, const uint32_t *gen_dev, uint32_t gen, uint32_t inst, uint32_t *bits,
                       int64_t ld, hipStream_t s, int4 lead_c)
{
    const int64_t per_xcd = (pv.np + 7) / 8;
    const qpm_status st = check_quad_grid(pv.D, 8 * per_xcd);
    if (st != QPM_OK) return st;
    const dim3 grid(static_cast<unsigned>(8 * per_xcd), quad_grid(pv.D, pv.np).y);
    dgwo_kernel<<<grid, 256, 0, s>>>(pv, leaders, lead_c, par_tab, par, static_cast<uint32_t>(seed),
                                     static_cast<uint32_t>(seed >> 32), gen_dev, gen, inst, bits, ld, per_xcd);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_fourth(const void *f, int64_t np, bool f64, int32_t *leaders, hipStream_t s)
{
    if (f64)
        fourth_kernel<double><<<1, 1024, 0, s>>>(static_cast<const double *>(f), np, leaders);
    else
        fourth_kernel<float><<<1, 1024, 0, s>>>(static_cast<const float *>(f), np, leaders);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_gwo(const PopView &pv, const int32_t *leaders, const float *a_tab, float a, uint64_t seed,
                      const uint32_t *gen_dev, uint32_t gen, uint32_t inst, int variant, uint32_t *bits, int64_t ld,
                      hipStream_t s, int4 lead_c)
{
    const int64_t per_xcd = (pv.np + 7) / 8;
    const qpm_status st = check_quad_grid(pv.D, 8 * per_xcd);
    if (st != QPM_OK) return st;
    const dim3 grid(static_cast<unsigned>(8 * per_xcd), quad_grid(pv.D, pv.np).y);
    if (variant == 1)
        gwo_kernel<1><<<grid, 256, 0, s>>>(pv, leaders, lead_c, a_tab, a, static_cast<uint32_t>(seed),
                                           static_cast<uint32_t>(seed >> 32), gen_dev, gen, inst, bits, ld, per_xcd);
    else
        gwo_kernel<0><<<grid, 256, 0, s>>>(pv, leaders, lead_c, a_tab, a, static_cast<uint32_t>(seed),
                                           static_cast<uint32_t>(seed >> 32), gen_dev, gen, inst, bits, ld, per_xcd);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_top3(const void *f, int64_t np, bool f64, int32_t *out3, hipStream_t s)
{
    if (f64)
        top3_kernel<double><<<1, 1024, 0, s>>>(static_cast<const double *>(f), np, out3);
    else
        top3_kernel<float><<<1, 1024, 0, s>>>(static_cast<const float *>(f), np, out3);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_gather(const PopView &pv, const int32_t *rows, int64_t nrows, float *out, int64_t ldo,
                         hipStream_t s)
{
    const int64_t blocks = (pv.D + 255) / 256;
    gather_kernel<<<dim3(static_cast<unsigned>(blocks < 64 ? blocks : 64), static_cast<unsigned>(nrows)), 256, 0,
                    s>>>(pv, rows, out, ldo);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_pack_pop(const float *x, int64_t np, int64_t D, int64_t ldx, uint32_t *bits, int64_t ld,
                           hipStream_t s)
{
    const qpm_status st = check_quad_grid(D, np);
    if (st != QPM_OK) return st;
    pack_pop_kernel<<<quad_grid(D, np), 256, 0, s>>>(x, D, ldx, bits, ld);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_draws(int64_t np, int64_t D, uint64_t seed, const uint32_t *gen_dev, uint32_t inst, int4 *draws,
                        hipStream_t s)
{
    de_draws_kernel<<<static_cast<unsigned>((np + 255) / 256), 256, 0, s>>>(
        np, D, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), gen_dev, 0u, inst, draws);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_pack_row(const float *x, int64_t D, uint32_t *bits, hipStream_t s)
{
    const int64_t W = words_for(D);
    pack_row_kernel<<<static_cast<unsigned>((W + 255) / 256), 256, 0, s>>>(x, D, bits);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

}  // namespace qpm

using namespace qpm;

static qpm_status check_rows(const void *p, int64_t np, int64_t D, int64_t ldx, const char *name)
{
    QPM_REQUIRE(p != nullptr, QPM_EINVAL, "%s must not be NULL", name);
    QPM_REQUIRE(aligned16(p), QPM_EINVAL, "%s must be 16-byte aligned", name);
    QPM_REQUIRE(D >= 1 && D <= (int64_t(1) << 30), QPM_EINVAL, "D must be in [1, 2^30] (got %lld)", (long long)D);
    QPM_REQUIRE(ldx % 4 == 0 && ldx >= ((D + 3) / 4) * 4, QPM_EINVAL,
                "ldx (%lld) must be a multiple of 4 and >= D rounded up to 4", (long long)ldx);
    QPM_REQUIRE(np >= 1 && np <= (int64_t(1) << 31) - 1, QPM_EINVAL, "np out of range (%lld)", (long long)np);
    return QPM_OK;
}

static qpm_status check_bits(const uint32_t *bits, int64_t np, int64_t ld)
{
    QPM_REQUIRE(bits != nullptr, QPM_EINVAL, "bits must not be NULL");
    QPM_REQUIRE(ld >= np && ld % 64 == 0, QPM_EINVAL, "ld (%lld) must be >= np (%lld) and a multiple of 64",
                (long long)ld, (long long)np);
    return QPM_OK;
}

static bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + nb && pb < pa + na;
}

QPM_API qpm_status qpm_init_population(int64_t np, int64_t D, int64_t ldx, uint64_t seed, uint32_t inst, float *x,
                                       uint32_t *bits, int64_t ld, qpm_stream sv)
{
    clear_error();
    qpm_status st = check_rows(x, np, D, ldx, "x");
    if (st != QPM_OK) return st;
    st = check_bits(bits, np, ld);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(inst < (1u << 24), QPM_EINVAL, "inst must be < 2^24");
    return launch_init(np, D, ldx, seed, inst, x, bits, ld, static_cast<hipStream_t>(sv));
}

static qpm_status de_step(const float *x, int64_t np, int64_t D, int64_t ldx, float F, float CR, uint64_t seed,
                          uint32_t generation, uint32_t inst, float *u, uint32_t *u_bits, int64_t ld, int ipw,
                          int passes, qpm_stream sv)
{
    qpm_status st = check_rows(x, np, D, ldx, "x");
    if (st != QPM_OK) return st;
    st = check_rows(u, np, D, ldx, "u");
    if (st != QPM_OK) return st;
    st = check_bits(u_bits, np, ld);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(np >= 4, QPM_EINVAL, "DE rand/1 needs np >= 4 (got %lld)", (long long)np);
    QPM_REQUIRE(F >= 0.0f && F <= 2.0f, QPM_EINVAL, "F must be in [0, 2] (got %g)", (double)F);
    QPM_REQUIRE(CR >= 0.0f && CR <= 1.0f, QPM_EINVAL, "CR must be in [0, 1] (got %g)", (double)CR);
    QPM_REQUIRE(inst < (1u << 24), QPM_EINVAL, "inst must be < 2^24");
    const size_t bytes = sizeof(float) * static_cast<size_t>(np) * static_cast<size_t>(ldx);
    QPM_REQUIRE(!overlaps(x, bytes, u, bytes), QPM_EINVAL, "x and u must not overlap");
    const PopView pv{x, x, nullptr, u, u, np, D, ldx};
    hipStream_t s = static_cast<hipStream_t>(sv);
    int4 *draws = nullptr;
    QPM_TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&draws), sizeof(int4) * np, s));
    qpm_status st2 = launch_de(pv, F, CR, seed, nullptr, generation, inst, u_bits, ld, draws, true, s, ipw, passes);
    (void)hipFreeAsync(draws, s);
    return st2;
}

QPM_API qpm_status qpm_de_step(const float *x, int64_t np, int64_t D, int64_t ldx, float F, float CR,
                               uint64_t seed, uint32_t generation, uint32_t inst, float *u, uint32_t *u_bits,
                               int64_t ld, qpm_stream sv)
{
    clear_error();
    return de_step(x, np, D, ldx, F, CR, seed, generation, inst, u, u_bits, ld, 0, 1, sv);
}

QPM_API qpm_status qpm_de_step_shape(const float *x, int64_t np, int64_t D, int64_t ldx, float F, float CR,
                                     uint64_t seed, uint32_t generation, uint32_t inst, float *u, uint32_t *u_bits,
                                     int64_t ld, int32_t individuals_per_wave, int32_t passes, qpm_stream sv)
{
    clear_error();
    QPM_REQUIRE(individuals_per_wave == 0 || individuals_per_wave == 1 || individuals_per_wave == 2 ||
                    individuals_per_wave == 4,
                QPM_EINVAL, "individuals_per_wave must be 0, 1, 2 or 4 (got %d)", (int)individuals_per_wave);
    QPM_REQUIRE(passes == 1 || passes == 2 || passes == 4, QPM_EINVAL, "passes must be 1, 2 or 4 (got %d)",
                (int)passes);
    return de_step(x, np, D, ldx, F, CR, seed, generation, inst, u, u_bits, ld, individuals_per_wave, passes, sv);
}

QPM_API qpm_status qpm_gwo_step(const float *x, int64_t np, int64_t D, int64_t ldx, const int32_t *leaders, float a,
                                uint64_t seed, uint32_t generation, uint32_t inst, int32_t variant, float *y,
                                uint32_t *y_bits, int64_t ld, qpm_stream sv)
{
    clear_error();
    qpm_status st = check_rows(x, np, D, ldx, "x");
    if (st != QPM_OK) return st;
    st = check_rows(y, np, D, ldx, "y");
    if (st != QPM_OK) return st;
    st = check_bits(y_bits, np, ld);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(leaders != nullptr, QPM_EINVAL, "leaders must not be NULL");
    QPM_REQUIRE(np >= 4, QPM_EINVAL, "the grey-wolf step needs np >= 4 (got %lld)", (long long)np);
    QPM_REQUIRE(a == 0.0f || (a >= 0x1p-100f && a <= 1e30f), QPM_EINVAL,
                "a must be 0 or in [2^-100, 1e30] (got %g)", (double)a);
    QPM_REQUIRE(variant == 0 || variant == 1, QPM_EINVAL, "variant must be 0 or 1");
    QPM_REQUIRE(inst < (1u << 24), QPM_EINVAL, "inst must be < 2^24");
    const size_t bytes = sizeof(float) * static_cast<size_t>(np) * static_cast<size_t>(ldx);
    QPM_REQUIRE(!overlaps(x, bytes, y, bytes), QPM_EINVAL, "x and y must not overlap");
    hipStream_t s = static_cast<hipStream_t>(sv);
    const int32_t *L = leaders;  // host memory: validated here, passed by value
    for (int k = 0; k < 3; ++k)
        QPM_REQUIRE(L[k] >= 0 && L[k] < np, QPM_EINVAL, "leader %d (%d) is outside [0, np)", k, (int)L[k]);
    QPM_REQUIRE(L[0] != L[1] && L[0] != L[2] && L[1] != L[2], QPM_EINVAL, "leaders must be distinct");
    const PopView pv{x, x, nullptr, y, y, np, D, ldx};
    return launch_gwo(pv, nullptr, nullptr, a, seed, nullptr, generation, inst, variant, y_bits, ld, s,
                      make_int4(L[0], L[1], L[2], 0));
}

QPM_API qpm_status qpm_dgwo_step(const float *x, int64_t np, int64_t D, int64_t ldx, const int32_t *leaders,
                                 const float *params, uint64_t seed, uint32_t generation, uint32_t inst, float *y,
                                 uint32_t *y_bits, int64_t ld, qpm_stream sv)
{
    clear_error();
    qpm_status st = check_rows(x, np, D, ldx, "x");
    if (st != QPM_OK) return st;
    st = check_rows(y, np, D, ldx, "y");
    if (st != QPM_OK) return st;
    st = check_bits(y_bits, np, ld);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(leaders != nullptr && params != nullptr, QPM_EINVAL, "leaders and params must not be NULL");
    QPM_REQUIRE(np >= 4, QPM_EINVAL, "the four-leader step needs np >= 4 (got %lld)", (long long)np);
    QPM_REQUIRE(inst < (1u << 24), QPM_EINVAL, "inst must be < 2^24");
    for (int k = 0; k < 4; ++k)
        QPM_REQUIRE(std::isfinite(params[k]), QPM_EINVAL, "params[%d] is not finite", k);
    const size_t bytes = sizeof(float) * static_cast<size_t>(np) * static_cast<size_t>(ldx);
    QPM_REQUIRE(!overlaps(x, bytes, y, bytes), QPM_EINVAL, "x and y must not overlap");
    hipStream_t s = static_cast<hipStream_t>(sv);
    const int32_t *L = leaders;  // host memory: validated here, passed by value
    for (int k = 0; k < 4; ++k)
        QPM_REQUIRE(L[k] >= 0 && L[k] < np, QPM_EINVAL, "leader %d (%d) is outside [0, np)", k, (int)L[k]);
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) QPM_REQUIRE(L[a] != L[b], QPM_EINVAL, "leaders must be distinct");
    const PopView pv{x, x, nullptr, y, y, np, D, ldx};
    const float4 par = make_float4(params[0], params[1], params[2], params[3]);
    return launch_dgwo(pv, nullptr, nullptr, par, seed, nullptr, generation, inst, y_bits, ld, s,
                       make_int4(L[0], L[1], L[2], L[3]));
}
