// device_common.hpp -- device helpers shared by the optimiser kernels:
// the per-individual DE draws and the (f descending, slot ascending) top-3.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "philox.hpp"

namespace qpm {

// Donors r1, r2, r3 (distinct, != i) and jrand of individual i in
// generation g: one Philox call; word m < 3 gives k = floor(u (np-1-m) /
// 2^32) and r is the k-th index not yet excluded (exclusions applied in
// ascending order); word 3 gives jrand = floor(u D / 2^32).
__device__ __forceinline__ int4 de_draw(int64_t i, int64_t np, int64_t D, uint32_t g, uint32_t inst, uint32_t k0,
                                        uint32_t k1)
{
    const U4 o = philox10(0u, static_cast<uint32_t>(i), g, (inst << 8) | kTagDeIdx, k0, k1);
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
    return make_int4(static_cast<int>(r1), static_cast<int>(r2), static_cast<int>(r3), static_cast<int>(jrand));
}

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

template <typename T>
__device__ __forceinline__ Top3<T> top3_empty()
{
    Top3<T> t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        t.v[k] = -INFINITY;
        t.i[k] = INT_MAX;
    }
    return t;
}

// merge the lists of the 64 lanes of a wave (every lane ends with the
// wave's three best)
template <typename T>
__device__ __forceinline__ void wave_top3(Top3<T> &t)
{
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
}

// The three best of the n candidates (f[j], idx ? idx[j] : j) over one
// workgroup of NT lanes (NT a multiple of 64, <= 1024). (f descending,
// slot ascending) is a strict total order, so the result is unique
// whatever the merge order. Loads are issued four at a time. Written by
// lane 0.
template <typename T, int NT>
__device__ void block_top3(const T *__restrict__ f, int64_t n, int32_t *__restrict__ out,
                           const int32_t *__restrict__ idx = nullptr)
{
    Top3<T> t = top3_empty<T>();
    for (int64_t base = threadIdx.x; base < n; base += 4 * NT) {
        T v[4];
        int ix[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = base + static_cast<int64_t>(u) * NT;
            const int64_t jj = j < n ? j : 0;
            const T fv = f[jj];
            const int iv = idx ? idx[jj] : static_cast<int>(jj);
            v[u] = j < n ? fv : static_cast<T>(-INFINITY);
            ix[u] = j < n ? iv : INT_MAX;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) top3_insert(t, v[u], ix[u]);
    }
    wave_top3(t);
    __shared__ T sv[NT / 64][3];
    __shared__ int si[NT / 64][3];
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
        for (int w = 1; w < NT / 64; ++w)
            for (int k = 0; k < 3; ++k) top3_insert(r, sv[w][k], si[w][k]);
        out[0] = r.i[0];
        out[1] = r.i[1];
        out[2] = r.i[2];
    }
}

}  // namespace qpm
