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

__device__ __forceinline__ uint32_t quad_nibble(float4 v, int64_t j0, int64_t D)
{
    uint32_t n = 0;
    n |= (v.x < 0.0f) ? 1u : 0u;
    n |= (j0 + 1 < D && v.y < 0.0f) ? 2u : 0u;
    n |= (j0 + 2 < D && v.z < 0.0f) ? 4u : 0u;
    n |= (j0 + 3 < D && v.w < 0.0f) ? 8u : 0u;
    return n;
}

// Merge the nibbles of 8 neighbouring lanes (gene quads 8w .. 8w+7) into
// word w and store it from the first lane of the group. Every lane of the
// wave must call this (it shuffles).
__device__ __forceinline__ void store_word(uint32_t nib, int64_t q, bool valid, uint32_t *bits, int64_t ld,
                                           int64_t i)
{
    uint32_t w = nib << (4 * (threadIdx.x & 7));
    w |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(w), 1));
    w |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(w), 2));
    w |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(w), 4));
    if (valid && (threadIdx.x & 7) == 0) bits[(q >> 3) * ld + i] = w;
}

// ------------------------------------------------------------ initialisation

__global__ __launch_bounds__(256) void init_kernel(int64_t D, int64_t ldx, uint32_t k0, uint32_t k1, uint32_t inst,
                                                   float *__restrict__ x, uint32_t *__restrict__ bits, int64_t ld)
{
    const int64_t i = blockIdx.y;
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) {
        const U4 r = philox10(static_cast<uint32_t>(q), static_cast<uint32_t>(i), 0u, (inst << 8) | kTagInit, k0, k1);
        const float4 v = make_float4(sym24(r.x), sym24(r.y), sym24(r.z), sym24(r.w));
        store_quad(x + i * ldx, j0, D, v);
        nib = quad_nibble(v, j0, D);
    }
    store_word(nib, q, valid, bits, ld, i);
}

// ------------------------------------------------------------ DE rand/1 + binomial crossover

__global__ __launch_bounds__(256) void de_kernel(PopView pv, float F, float CR, uint32_t k0, uint32_t k1,
                                                 const uint32_t *__restrict__ gen_dev, uint32_t gen_c, uint32_t inst,
                                                 uint32_t *__restrict__ bits, int64_t ld)
{
    const int64_t i = blockIdx.y;
    const uint32_t g = gen_dev ? gen_dev[0] : gen_c;
    const uint32_t c3 = inst << 8;
    const int64_t np = pv.np, D = pv.D;

    // donors: three distinct indices != i, each the k-th index not yet
    // excluded (exclusions applied in ascending order), and jrand
    const U4 o = philox10(0u, static_cast<uint32_t>(i), g, c3 | kTagDeIdx, k0, k1);
    int64_t r1 = bounded(o.x, static_cast<uint32_t>(np - 1));
    if (r1 >= i) ++r1;
    int64_t r2 = bounded(o.y, static_cast<uint32_t>(np - 2));
    {
        const int64_t lo = i < r1 ? i : r1, hi = i < r1 ? r1 : i;
        if (r2 >= lo) ++r2;
        if (r2 >= hi) ++r2;
    }
    int64_t r3 = bounded(o.z, static_cast<uint32_t>(np - 3));
    {
        int64_t e0 = i, e1 = r1, e2 = r2, t;
        if (e0 > e1) { t = e0; e0 = e1; e1 = t; }
        if (e1 > e2) { t = e1; e1 = e2; e2 = t; }
        if (e0 > e1) { t = e0; e0 = e1; e1 = t; }
        if (r3 >= e0) ++r3;
        if (r3 >= e1) ++r3;
        if (r3 >= e2) ++r3;
    }
    const int64_t jrand = bounded(o.w, static_cast<uint32_t>(D));

    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) {
        const float4 xv = *reinterpret_cast<const float4 *>(row_of(pv, i) + j0);
        const float4 a = *reinterpret_cast<const float4 *>(row_of(pv, r1) + j0);
        const float4 b = *reinterpret_cast<const float4 *>(row_of(pv, r2) + j0);
        const float4 c = *reinterpret_cast<const float4 *>(row_of(pv, r3) + j0);
        const U4 r = philox10(static_cast<uint32_t>(q), static_cast<uint32_t>(i), g, c3 | kTagDeCr, k0, k1);
        const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
        const float as[4] = {a.x, a.y, a.z, a.w};
        const float bs[4] = {b.x, b.y, b.z, b.w};
        const float cs[4] = {c.x, c.y, c.z, c.w};
        const uint32_t rs[4] = {r.x, r.y, r.z, r.w};
        float us[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool take = (unit24(rs[e]) <= CR) || (j0 + e == jrand);
            const float v = clamp1(fmaf(F, bs[e] - cs[e], as[e]));
            us[e] = take ? v : xs[e];
        }
        const float4 uv = make_float4(us[0], us[1], us[2], us[3]);
        store_quad(out_row_of(pv, i), j0, D, uv);
        nib = quad_nibble(uv, j0, D);
    }
    store_word(nib, q, valid, bits, ld, i);
}

// ------------------------------------------------------------ grey-wolf update

__global__ __launch_bounds__(256) void gwo_kernel(PopView pv, const int32_t *__restrict__ leaders,
                                                  const float *__restrict__ a_tab, float a_c, uint32_t k0, uint32_t k1,
                                                  const uint32_t *__restrict__ gen_dev, uint32_t gen_c, uint32_t inst,
                                                  int variant, uint32_t *__restrict__ bits, int64_t ld)
{
    const int64_t i = blockIdx.y;
    const int64_t L0 = leaders[0], L1 = leaders[1], L2 = leaders[2];
    const int64_t np = pv.np, D = pv.D;
    // leaders keep their positions; indices outside the population make
    // the launch a no-op instead of an out-of-bounds read
    if (i == L0 || i == L1 || i == L2) return;
    if (L0 < 0 || L0 >= np || L1 < 0 || L1 >= np || L2 < 0 || L2 >= np) return;
    const uint32_t g = gen_dev ? gen_dev[0] : gen_c;
    const float a = a_tab ? a_tab[g] : a_c;
    const float two_a = 2.0f * a;
    const uint32_t c3 = (inst << 8) | kTagGwo;

    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) {
        const float4 xv = *reinterpret_cast<const float4 *>(row_of(pv, i) + j0);
        const float4 X0 = *reinterpret_cast<const float4 *>(row_of(pv, L0) + j0);
        const float4 X1 = *reinterpret_cast<const float4 *>(row_of(pv, L1) + j0);
        const float4 X2 = *reinterpret_cast<const float4 *>(row_of(pv, L2) + j0);
        const uint32_t cq = static_cast<uint32_t>(3 * q);
        const U4 wa = philox10(cq, static_cast<uint32_t>(i), g, c3, k0, k1);
        const U4 wb = philox10(cq + 1u, static_cast<uint32_t>(i), g, c3, k0, k1);
        const U4 wc = philox10(cq + 2u, static_cast<uint32_t>(i), g, c3, k0, k1);
        // word t of the quad: gene e = t / 3, leader k = t % 3
        const uint32_t wrd[12] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w, wc.x, wc.y, wc.z, wc.w};
        const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
        const float Xs[3][4] = {{X0.x, X0.y, X0.z, X0.w}, {X1.x, X1.y, X1.z, X1.w}, {X2.x, X2.y, X2.z, X2.w}};
        float ys[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float Y[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint32_t o = wrd[3 * e + k];
                const float r1 = static_cast<float>(o & 0xFFFFu) * 0x1p-16f;
                const float r2 = static_cast<float>(o >> 16) * 0x1p-16f;
                const float A = fmaf(two_a, r1, -a);
                const float Cc = 2.0f * r2;
                const float Dk = fabsf(fmaf(Cc, Xs[k][e], -xs[e]));
                Y[k] = fmaf(-A, Dk, Xs[k][e]);
            }
            float yv;
            if (variant == 1) {
                yv = ((Y[0] + Y[1]) + Y[2]) / 3.0f;
            } else {
                const float s = (fabsf(Y[0]) + fabsf(Y[1])) + fabsf(Y[2]);
                const float num = fmaf(fabsf(Y[2]), Y[2], fmaf(fabsf(Y[1]), Y[1], fabsf(Y[0]) * Y[0]));
                yv = (s == 0.0f) ? 0.0f : (num / s) / 3.0f;
            }
            ys[e] = clamp1(yv);
        }
        const float4 yv4 = make_float4(ys[0], ys[1], ys[2], ys[3]);
        store_quad(out_row_of(pv, i), j0, D, yv4);
        nib = quad_nibble(yv4, j0, D);
    }
    store_word(nib, q, valid, bits, ld, i);
}

// ------------------------------------------------------------ selection

template <typename T>
__global__ __launch_bounds__(256) void select_kernel(T *__restrict__ f, const T *__restrict__ fnew,
                                                     uint32_t *__restrict__ flags, int64_t np,
                                                     const int32_t *__restrict__ leaders)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= np) return;
    if (leaders && (i == leaders[0] || i == leaders[1] || i == leaders[2])) return;
    const T v = fnew[i];
    if (v > f[i]) {
        f[i] = v;
        flags[i] ^= 1u;
    }
}

// ------------------------------------------------------------ top-3

template <typename T>
struct Top3 {
    T v[3];
    int i[3];
};

template <typename T>
__device__ __forceinline__ bool ahead(T va, int ia, T vb, int ib)
{
    return va > vb || (va == vb && ia < ib);
}

template <typename T>
__device__ __forceinline__ void top3_insert(Top3<T> &t, T v, int idx)
{
    if (ahead(v, idx, t.v[0], t.i[0])) {
        t.v[2] = t.v[1]; t.i[2] = t.i[1];
        t.v[1] = t.v[0]; t.i[1] = t.i[0];
        t.v[0] = v; t.i[0] = idx;
    } else if (ahead(v, idx, t.v[1], t.i[1])) {
        t.v[2] = t.v[1]; t.i[2] = t.i[1];
        t.v[1] = v; t.i[1] = idx;
    } else if (ahead(v, idx, t.v[2], t.i[2])) {
        t.v[2] = v; t.i[2] = idx;
    }
}

// One workgroup of 1024 lanes. (f descending, slot ascending) is a strict
// total order, so the three best are unique whatever the merge order.
template <typename T>
__global__ __launch_bounds__(1024) void top3_kernel(const T *__restrict__ f, int64_t np, int32_t *__restrict__ out)
{
    Top3<T> t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        t.v[k] = -INFINITY;
        t.i[k] = INT_MAX;
    }
    for (int64_t i = threadIdx.x; i < np; i += 1024) top3_insert(t, f[i], static_cast<int>(i));
    for (int off = 32; off >= 1; off >>= 1) {
        T ov[3];
        int oi[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ov[k] = __shfl_xor(t.v[k], off);
            oi[k] = __shfl_xor(t.i[k], off);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) top3_insert(t, ov[k], oi[k]);
    }
    __shared__ T sv[16][3];
    __shared__ int si[16][3];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            sv[wave][k] = t.v[k];
            si[wave][k] = t.i[k];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Top3<T> r = t;
        for (int w = 1; w < 16; ++w)
            for (int k = 0; k < 3; ++k) top3_insert(r, sv[w][k], si[w][k]);
        out[0] = r.i[0];
        out[1] = r.i[1];
        out[2] = r.i[2];
    }
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
    const int64_t i = blockIdx.y;
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) nib = quad_nibble(*reinterpret_cast<const float4 *>(x + i * ldx + j0), j0, D);
    store_word(nib, q, valid, bits, ld, i);
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

static dim3 quad_grid(int64_t D, int64_t rows)
{
    const int64_t quads = (D + 3) / 4;
    return dim3(static_cast<unsigned>((quads + 255) / 256), static_cast<unsigned>(rows));
}

qpm_status launch_init(int64_t np, int64_t D, int64_t ldx, uint64_t seed, uint32_t inst, float *x, uint32_t *bits,
                       int64_t ld, hipStream_t s)
{
    init_kernel<<<quad_grid(D, np), 256, 0, s>>>(D, ldx, static_cast<uint32_t>(seed),
                                                 static_cast<uint32_t>(seed >> 32), inst, x, bits, ld);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_de(const PopView &pv, float F, float CR, uint64_t seed, const uint32_t *gen_dev, uint32_t gen,
                     uint32_t inst, uint32_t *bits, int64_t ld, hipStream_t s)
{
    de_kernel<<<quad_grid(pv.D, pv.np), 256, 0, s>>>(pv, F, CR, static_cast<uint32_t>(seed),
                                                     static_cast<uint32_t>(seed >> 32), gen_dev, gen, inst, bits, ld);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_gwo(const PopView &pv, const int32_t *leaders, const float *a_tab, float a, uint64_t seed,
                      const uint32_t *gen_dev, uint32_t gen, uint32_t inst, int variant, uint32_t *bits, int64_t ld,
                      hipStream_t s)
{
    gwo_kernel<<<quad_grid(pv.D, pv.np), 256, 0, s>>>(pv, leaders, a_tab, a, static_cast<uint32_t>(seed),
                                                      static_cast<uint32_t>(seed >> 32), gen_dev, gen, inst, variant,
                                                      bits, ld);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_select(void *f, const void *fnew, uint32_t *flags, int64_t np, const int32_t *leaders, bool f64,
                         hipStream_t s)
{
    const unsigned blocks = static_cast<unsigned>((np + 255) / 256);
    if (f64)
        select_kernel<double><<<blocks, 256, 0, s>>>(static_cast<double *>(f), static_cast<const double *>(fnew),
                                                     flags, np, leaders);
    else
        select_kernel<float><<<blocks, 256, 0, s>>>(static_cast<float *>(f), static_cast<const float *>(fnew), flags,
                                                    np, leaders);
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
    pack_pop_kernel<<<quad_grid(D, np), 256, 0, s>>>(x, D, ldx, bits, ld);
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

QPM_API qpm_status qpm_de_step(const float *x, int64_t np, int64_t D, int64_t ldx, float F, float CR,
                               uint64_t seed, uint32_t generation, uint32_t inst, float *u, uint32_t *u_bits,
                               int64_t ld, qpm_stream sv)
{
    clear_error();
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
    return launch_de(pv, F, CR, seed, nullptr, generation, inst, u_bits, ld, static_cast<hipStream_t>(sv));
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
    QPM_REQUIRE(a >= 0.0f && a <= 1e30f, QPM_EINVAL, "a must be finite and >= 0 (got %g)", (double)a);
    QPM_REQUIRE(variant == 0 || variant == 1, QPM_EINVAL, "variant must be 0 or 1");
    QPM_REQUIRE(inst < (1u << 24), QPM_EINVAL, "inst must be < 2^24");
    const size_t bytes = sizeof(float) * static_cast<size_t>(np) * static_cast<size_t>(ldx);
    QPM_REQUIRE(!overlaps(x, bytes, y, bytes), QPM_EINVAL, "x and y must not overlap");
    hipStream_t s = static_cast<hipStream_t>(sv);
    int32_t L[3];
    QPM_TRY_HIP(hipMemcpyAsync(L, leaders, sizeof(L), hipMemcpyDeviceToHost, s));
    QPM_TRY_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < 3; ++k)
        QPM_REQUIRE(L[k] >= 0 && L[k] < np, QPM_EINVAL, "leader %d (%d) is outside [0, np)", k, (int)L[k]);
    QPM_REQUIRE(L[0] != L[1] && L[0] != L[2] && L[1] != L[2], QPM_EINVAL, "leaders must be distinct");
    const PopView pv{x, x, nullptr, y, y, np, D, ldx};
    return launch_gwo(pv, leaders, nullptr, a, seed, nullptr, generation, inst, variant, y_bits, ld, s);
}
