// objective.hip -- the multi-wavelength objective (the paper's
// multi-wavelength second-harmonic and coupled third-harmonic designs, its
// last section): K designs on one set of boundaries, one per wavelength,
// G_k = |sum d a| / L (SHG) or |d_eff| / L^2 (THG), and the paper's
// objective h = sum_k |G0 - G_k| + beta (max G - min G), maximised as -h.
//
// One bit stream serves the K designs: a workgroup (4 segment waves over
// one group of 64 genomes) loads its genomes' bit words into registers once,
// then for each design copies that design's sign-pattern tables of the
// workgroup's words to LDS and walks the words again from registers. SHG
// needs only the A row of each table (sum d a of a 4-domain block), THG
// the whole (A, B, Q) triple.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "device_common.hpp"
#include "scan.hpp"
#include "select.hpp"

namespace qpm {

namespace {

// table rows per 4-domain block (A only, or A, B, Q) and components of a
// segment partial
template <bool THG>
struct ObjShape {
    static constexpr int R = THG ? 3 : 1;
    static constexpr int NC = THG ? 6 : 2;
};

constexpr int kSegWaves = 4;

template <bool F32, bool THG>
size_t obj_lds_bytes(int wpw)
{
    const size_t tables = static_cast<size_t>(kSegWaves) * wpw * 8 * ObjShape<THG>::R * 16 * (F32 ? 8 : 16);
    const size_t fold = static_cast<size_t>(ObjShape<THG>::NC) * kSegWaves * 64 * sizeof(double);
    return tables > fold ? tables : fold;
}

}  // namespace

// Grid: x = genome groups of 64, y = workgroup segments of 4 wpw words.
// part[(k gy + y) NC + c][ld] + i: the segment's (A, B, Q) (THG) or A (SHG)
// of design k for genome i, the 4 segment waves folded in order.
template <bool F32, bool THG>
__global__ __launch_bounds__(256) void obj_partials_kernel(ObjTabs tabs, int K, const uint32_t *__restrict__ bits,
                                                           int64_t ld, int W, int wpw, int gy, int64_t np,
                                                           double *__restrict__ part, uint32_t *__restrict__ advance)
{
    if (advance != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) advance[0] += 1u;
    constexpr int R = ObjShape<THG>::R;
    constexpr int NC = ObjShape<THG>::NC;
    constexpr int ES = F32 ? 8 : 16;        // bytes per table entry (complex)
    constexpr int PPR = 16 * ES / 16;       // 16-byte pieces per block row of 16 entries
    constexpr int MAXW = table_max_wpw(F32);
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const int wbase = static_cast<int>(blockIdx.y) * kSegWaves * wpw;
    const int nw = min(W - wbase, kSegWaves * wpw);  // >= 1 by the grid
    const bool live = i < np;
    const int w0 = wave * wpw, w1 = min(nw, w0 + wpw);
    const int64_t ic = i < ld ? i : ld - 1;
    // the bit words of this wave's segment, loaded once for all K designs
    uint32_t wv[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) wv[k] = bits[static_cast<int64_t>(min(wbase + w0 + k, W - 1)) * ld + ic];
    const int n16 = nw * 8 * R * PPR;
    for (int kd = 0; kd < K; ++kd) {
        // design kd's table rows of words [wbase, wbase + nw) into LDS:
        // piece idx = ((word 8 + block) R + row) PPR + q
        const unsigned char *src = F32 ? reinterpret_cast<const unsigned char *>(tabs.tq[kd])
                                       : reinterpret_cast<const unsigned char *>(tabs.t64[kd]);
        for (int r0 = 0; r0 * 256 < n16; ++r0) {
            const int idx = r0 * 256 + static_cast<int>(threadIdx.x);
            if (idx < n16) {
                const int q = idx % PPR, row = (idx / PPR) % R, blk = idx / (PPR * R);  // blk = word 8 + block
                const int64_t off =
                    ((static_cast<int64_t>(wbase) * 8 + blk) * 48 + row * 16) * ES + static_cast<int64_t>(q) * 16;
                __builtin_amdgcn_global_load_lds(
                    reinterpret_cast<const uint4 *>(src + off),
                    reinterpret_cast<__attribute__((address_space(3))) void *>(
                        reinterpret_cast<uintptr_t>(lds + static_cast<size_t>(r0 * 256 + wave * 64) * 16)),
                    16, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        Tri t{0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            const int wr = w0 + k;
            if (wr >= w1) break;
            const uint32_t word = live ? wv[k] : 0u;
            if constexpr (F32) {
                word_tab_q<R>(t, word, reinterpret_cast<const int2 *>(lds) + wr * 8 * R * 16,
                              tabs.wsc[kd][wbase + wr]);
            } else {
                const double2 *tb = reinterpret_cast<const double2 *>(lds) + wr * 8 * R * 16;
#pragma unroll
                for (int h = 0; h < 8; ++h) {
                    const uint32_t pt = (word >> (4 * h)) & 15u;
                    const double2 A = tb[(h * R) * 16 + pt];
                    if constexpr (THG) {
                        const double2 B = tb[(h * R + 1) * 16 + pt], Q = tb[(h * R + 2) * 16 + pt];
                        t.qr = fma(-t.ai, B.y, fma(t.ar, B.x, t.qr + Q.x));
                        t.qi = fma(t.ai, B.x, fma(t.ar, B.y, t.qi + Q.y));
                        t.br += B.x;
                        t.bi += B.y;
                    }
                    t.ar += A.x;
                    t.ai += A.y;
                }
            }
        }
        // fold the 4 segment waves in order through LDS (tables done)
        __syncthreads();
        double *sh = reinterpret_cast<double *>(lds);  // [NC][4][64]
        const double comp[6] = {t.ar, t.ai, t.br, t.bi, t.qr, t.qi};
#pragma unroll
        for (int c = 0; c < NC; ++c) sh[(c * kSegWaves + wave) * 64 + lane] = comp[c];
        __syncthreads();
        if (wave == 0 && live) {
            for (int s2 = 1; s2 < kSegWaves; ++s2) {
                if (s2 * wpw >= nw) break;
                if constexpr (THG) {
                    tri_append(t, Tri{sh[(0 * kSegWaves + s2) * 64 + lane], sh[(1 * kSegWaves + s2) * 64 + lane],
                                      sh[(2 * kSegWaves + s2) * 64 + lane], sh[(3 * kSegWaves + s2) * 64 + lane],
                                      sh[(4 * kSegWaves + s2) * 64 + lane], sh[(5 * kSegWaves + s2) * 64 + lane]});
                } else {
                    t.ar += sh[(0 * kSegWaves + s2) * 64 + lane];
                    t.ai += sh[(1 * kSegWaves + s2) * 64 + lane];
                }
            }
            double *p = part + ((static_cast<int64_t>(kd) * gy + blockIdx.y) * NC) * ld + i;
            const double out[6] = {t.ar, t.ai, t.br, t.bi, t.qr, t.qi};
#pragma unroll
            for (int c = 0; c < NC; ++c) p[c * ld] = out[c];
        }
        __syncthreads();  // LDS is refilled for the next design
    }
}

// A of genome i over the gy segments of one design (part: [gy][2][ld]),
// split in NW ranges folded in order as combine_segments_in does for
// triples; valid in wave 0.
template <int NW>
__device__ __forceinline__ void combine_a_in(const double *__restrict__ part, int gy, int64_t ld, int64_t i,
                                             bool valid, int wave, int lane, double *sh, double &ar, double &ai)
{
    const int s0 = static_cast<int>((static_cast<int64_t>(gy) * wave) / NW);
    const int s1 = static_cast<int>((static_cast<int64_t>(gy) * (wave + 1)) / NW);
    ar = 0.0;
    ai = 0.0;
    if (valid)
        for (int sg = s0; sg < s1; ++sg) {
            const double *q = part + static_cast<int64_t>(sg) * 2 * ld + i;
            ar += q[0];
            ai += q[ld];
        }
    sh[(0 * NW + wave) * 64 + lane] = ar;
    sh[(1 * NW + wave) * 64 + lane] = ai;
    __syncthreads();
    if (wave == 0)
        for (int w = 1; w < NW; ++w) {
            ar += sh[(0 * NW + w) * 64 + lane];
            ai += sh[(1 * NW + w) * 64 + lane];
        }
}

// -h of genome i from the K designs' segment partials; valid in wave 0
// (every thread of the 4-wave workgroup calls it). G (optional): G_k at
// G[k ldG + i].
template <bool THG>
__device__ double obj_value(const ObjTabs &tabs, int K, double scale, double G0, double beta,
                            const double *__restrict__ part, int gy, int64_t ld, int64_t i, bool valid, double *G,
                            int64_t ldG, double *sh)
{
    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    double sum = 0.0, gmax = 0.0, gmin = 0.0;
    for (int k = 0; k < K; ++k) {
        double re, im;
        if constexpr (THG) {
            const Tri t = combine_segments_in<4>(part + static_cast<int64_t>(k) * gy * 6 * ld, gy, ld, i, valid,
                                                 wave, lane, sh);
            re = t.qr + tabs.C[k][0];
            im = t.qi + tabs.C[k][1];
        } else {
            combine_a_in<4>(part + static_cast<int64_t>(k) * gy * 2 * ld, gy, ld, i, valid, wave, lane, sh, re, im);
        }
        __syncthreads();  // sh is reused by the next design
        const double Gk = sqrt(fma(re, re, im * im)) * scale;
        if (G && wave == 0 && valid) G[k * ldG + i] = Gk;
        sum += fabs(G0 - Gk);
        gmax = k == 0 ? Gk : fmax(gmax, Gk);
        gmin = k == 0 ? Gk : fmin(gmin, Gk);
    }
    return -(sum + beta * (gmax - gmin));
}

template <typename T, bool THG>
__global__ __launch_bounds__(256) void obj_values_kernel(ObjTabs tabs, int K, double scale, double G0, double beta,
                                                         const double *__restrict__ part, int gy, int64_t ld,
                                                         int64_t np, T *__restrict__ fit, double *__restrict__ G,
                                                         int64_t ldG)
{
    __shared__ double sh[6 * 4 * 64];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + (threadIdx.x & 63);
    const bool valid = i < np;
    const double v = obj_value<THG>(tabs, K, scale, G0, beta, part, gy, ld, i, valid, G, ldG, sh);
    if (threadIdx.x < 64 && valid) fit[i] = static_cast<T>(v);
}

// the run's finish step on the objective: as finish_kernel, with the
// fitness -h
template <typename T, bool THG>
__global__ __launch_bounds__(256) void obj_finish_kernel(ObjTabs tabs, int K, double scale, double G0, double beta,
                                                         const double *__restrict__ part, int gy, int64_t ld,
                                                         int64_t np, T *__restrict__ f_cur,
                                                         uint32_t *__restrict__ flags, uint32_t *__restrict__ fbits,
                                                         const int32_t *__restrict__ skip3, T *__restrict__ cand_v,
                                                         int32_t *__restrict__ cand_i, int4 *__restrict__ draws_next,
                                                         const uint32_t *__restrict__ gen, int64_t D, uint32_t k0,
                                                         uint32_t k1, uint32_t inst, AcceptOut acc, uint32_t next_off,
                                                         int replace_all)
{
    __shared__ double sh[6 * 4 * 64];
    const int lane = threadIdx.x & 63;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const double v = obj_value<THG>(tabs, K, scale, G0, beta, part, gy, ld, i, i < np, nullptr, 0, sh);
    if (threadIdx.x < 64)
        select_group<T>(v, blockIdx.x, lane, np, f_cur, flags, fbits, skip3, cand_v, cand_i, draws_next, gen, D, k0,
                        k1, inst, acc, next_off, replace_all != 0);
}

ObjPlan plan_objective_shape(const Objective &o, int wpw)
{
    ObjPlan pl;
    pl.wpw = wpw;
    pl.gy = static_cast<int>((o.words + 4 * pl.wpw - 1) / (4 * pl.wpw));
    return pl;
}

ObjPlan plan_objective(const Objective &o, qpm_prec p, int64_t np)
{
    // the most words per wave (fewest partials) that still gives about
    // 2048 workgroups (8 per CU, so staging and walking overlap across
    // workgroups), at most the register limit of the word cache
    const bool f32 = p == QPM_PREC_F32;
    const int64_t groups = (np + 63) / 64;
    int wpw = table_max_wpw(f32);
    while (wpw > 1 && groups * ((o.words + 4 * wpw - 1) / (4 * wpw)) < 2048) --wpw;
    while (wpw < table_max_wpw(f32) && (o.words + 4 * wpw - 1) / (4 * wpw) > 65535) ++wpw;
    return plan_objective_shape(o, wpw);
}

size_t objective_partials_bytes(const Objective &o, const ObjPlan &pl, int64_t ld)
{
    const int nc = o.kind == QPM_OBJ_THG ? 6 : 2;
    return sizeof(double) * static_cast<size_t>(o.K) * pl.gy * nc * static_cast<size_t>(ld);
}

qpm_status launch_objective_partials(const Objective &o, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                     const ObjPlan &pl, double *part, hipStream_t s, uint32_t *advance)
{
    QPM_REQUIRE(pl.gy <= 65535, QPM_ERANGE, "too many workgroup segments (%d)", pl.gy);
    const dim3 grid(static_cast<unsigned>((np + 63) / 64), static_cast<unsigned>(pl.gy));
    const int W = static_cast<int>(o.words);
    const bool f32 = p == QPM_PREC_F32, thg = o.kind == QPM_OBJ_THG;
    if (f32 && thg)
        obj_partials_kernel<true, true><<<grid, 256, obj_lds_bytes<true, true>(pl.wpw), s>>>(o.tabs, o.K, bits, ld, W,
                                                                                          pl.wpw, pl.gy, np, part,
                                                                                          advance);
    else if (f32)
        obj_partials_kernel<true, false><<<grid, 256, obj_lds_bytes<true, false>(pl.wpw), s>>>(
            o.tabs, o.K, bits, ld, W, pl.wpw, pl.gy, np, part, advance);
    else if (thg)
        obj_partials_kernel<false, true><<<grid, 256, obj_lds_bytes<false, true>(pl.wpw), s>>>(
            o.tabs, o.K, bits, ld, W, pl.wpw, pl.gy, np, part, advance);
    else
        obj_partials_kernel<false, false><<<grid, 256, obj_lds_bytes<false, false>(pl.wpw), s>>>(
            o.tabs, o.K, bits, ld, W, pl.wpw, pl.gy, np, part, advance);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_objective_values(const Objective &o, const ObjPlan &pl, const double *part, int64_t ld, int64_t np,
                                   void *fitness, bool f64, double *G, int64_t ldG, hipStream_t s)
{
    const unsigned blocks = static_cast<unsigned>((np + 63) / 64);
    const bool thg = o.kind == QPM_OBJ_THG;
#define QPM_OV(T, H)                                                                                             \
    obj_values_kernel<T, H><<<blocks, 256, 0, s>>>(o.tabs, o.K, o.scale, o.G0, o.beta, part, pl.gy, ld, np,     \
                                                   static_cast<T *>(fitness), G, ldG)
    if (f64) {
        if (thg) QPM_OV(double, true); else QPM_OV(double, false);
    } else {
        if (thg) QPM_OV(float, true); else QPM_OV(float, false);
    }
#undef QPM_OV
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_objective_finish(const Objective &o, const ObjPlan &pl, const double *part, int64_t ld, int64_t np,
                                   void *f_cur, bool f64, uint32_t *flags, uint32_t *fbits, const int32_t *skip3,
                                   int32_t *top3_out, void *cand, int4 *draws_next, uint32_t *gen, int64_t D,
                                   uint64_t seed, uint32_t inst, hipStream_t s, AcceptOut acc, FinishMode mode)
{
    const unsigned blocks = static_cast<unsigned>((np + 63) / 64);
    QPM_REQUIRE(top3_out == nullptr || cand != nullptr, QPM_EINVAL, "leader candidates need a buffer");
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    const int advance = draws_next != nullptr && !mode.gen_advanced;
    const uint32_t next_off = mode.gen_advanced ? 0u : 1u;
    const bool tail = (top3_out != nullptr && !mode.defer_leaders) || advance;
    int32_t *tail_top3 = mode.defer_leaders ? nullptr : top3_out;
    const bool thg = o.kind == QPM_OBJ_THG;
    // cand: 3 values per workgroup (T) followed by 3 slots per workgroup
#define QPM_OF(T, H)                                                                                              \
    {                                                                                                             \
        T *cv = top3_out ? static_cast<T *>(cand) : nullptr;                                                      \
        int32_t *ci = cv ? reinterpret_cast<int32_t *>(cv + 3 * static_cast<size_t>(blocks)) : nullptr;          \
        obj_finish_kernel<T, H><<<blocks, 256, 0, s>>>(o.tabs, o.K, o.scale, o.G0, o.beta, part, pl.gy, ld, np,  \
                                                       static_cast<T *>(f_cur), flags, fbits, skip3, cv, ci,     \
                                                       draws_next, gen, D, k0, k1, inst, acc, next_off,          \
                                                       mode.replace_all ? 1 : 0);                                 \
        if (tail) finish_tail_kernel<T><<<1, 256, 0, s>>>(cv, ci, blocks, tail_top3, gen, advance);               \
    }
    if (f64) {
        if (thg) QPM_OF(double, true) else QPM_OF(double, false)
    } else {
        if (thg) QPM_OF(float, true) else QPM_OF(float, false)
    }
#undef QPM_OF
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

}  // namespace qpm

using namespace qpm;

QPM_API qpm_status qpm_objective_create(const qpm_design *designs, int32_t K, int32_t kind, double G0, double beta,
                                        qpm_objective *out)
{
    clear_error();
    QPM_REQUIRE(designs != nullptr && out != nullptr, QPM_EINVAL, "designs and out must not be NULL");
    QPM_REQUIRE(K >= 1 && K <= kMaxObjectiveDesigns, QPM_EINVAL, "K must be in [1, %d] (got %d)",
                kMaxObjectiveDesigns, (int)K);
    QPM_REQUIRE(kind == QPM_OBJ_SHG || kind == QPM_OBJ_THG, QPM_EINVAL, "unknown objective kind %d", (int)kind);
    QPM_REQUIRE(std::isfinite(G0) && std::isfinite(beta), QPM_EINVAL, "G0 and beta must be finite");
    for (int k = 0; k < K; ++k) QPM_REQUIRE(designs[k] != nullptr, QPM_EINVAL, "design %d is NULL", k);
    const Design *d0 = designs[0];
    for (int k = 1; k < K; ++k) {
        const Design *dk = designs[k];
        QPM_REQUIRE(dk->n == d0->n && dk->z0 == d0->z0 && dk->zN == d0->zN && dk->zhash == d0->zhash, QPM_EINVAL,
                    "design %d has other boundaries than design 0", k);
        QPM_REQUIRE(dk->device == d0->device, QPM_EINVAL, "design %d lives on another device", k);
    }
    const double L = d0->zN - d0->z0;
    auto *o = new qpm_objective_s();
    o->K = K;
    o->kind = kind;
    o->G0 = G0;
    o->beta = beta;
    o->scale = kind == QPM_OBJ_SHG ? 1.0 / L : 1.0 / (L * L);
    o->n = d0->n;
    o->words = d0->words;
    for (int k = 0; k < K; ++k) {
        o->d[k] = designs[k];
        o->tabs.tq[k] = designs[k]->tabq;
        o->tabs.wsc[k] = designs[k]->wsc;
        o->tabs.t64[k] = designs[k]->tab64;
        o->tabs.C[k][0] = designs[k]->C[0];
        o->tabs.C[k][1] = designs[k]->C[1];
    }
    o->scratch = scratch_cache_create();
    *out = o;
    return QPM_OK;
}

QPM_API qpm_status qpm_objective_free(qpm_objective o)
{
    clear_error();
    if (o) scratch_cache_destroy(o->scratch);
    delete o;
    return QPM_OK;
}

static qpm_status eval_with_plan(qpm_objective o, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                 void *fitness, double *G, int64_t ldG, const ObjPlan &pl, hipStream_t s);

static qpm_status check_objective_args(qpm_objective o, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                       void *fitness, double *G, int64_t ldG)
{
    QPM_REQUIRE(o && bits && fitness, QPM_EINVAL, "objective, bits and fitness must not be NULL");
    QPM_REQUIRE(p == QPM_PREC_F32 || p == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", (int)p);
    QPM_REQUIRE(np >= 1, QPM_EINVAL, "np must be >= 1 (got %lld)", (long long)np);
    QPM_REQUIRE(ld >= np && ld % 64 == 0, QPM_EINVAL, "ld (%lld) must be >= np (%lld) and a multiple of 64",
                (long long)ld, (long long)np);
    QPM_REQUIRE((reinterpret_cast<uintptr_t>(bits) & 3u) == 0, QPM_EINVAL, "bits must be 4-byte aligned");
    QPM_REQUIRE(G == nullptr || ldG >= np, QPM_EINVAL, "ldG (%lld) must be >= np (%lld)", (long long)ldG,
                (long long)np);
    QPM_REQUIRE(np <= (int64_t(1) << 31) && o->words * ld <= (int64_t(1) << 40), QPM_ERANGE, "population too large");
    return QPM_OK;
}

QPM_API qpm_status qpm_eval_objective(qpm_objective o, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                      void *fitness, double *G, int64_t ldG, qpm_stream sv)
{
    clear_error();
    qpm_status st = check_objective_args(o, p, bits, np, ld, fitness, G, ldG);
    if (st != QPM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(sv);
    const ObjPlan pl = plan_objective(*o, p, np);
    return eval_with_plan(o, p, bits, np, ld, fitness, G, ldG, pl, s);
}

QPM_API qpm_status qpm_eval_objective_shape(qpm_objective o, qpm_prec p, const uint32_t *bits, int64_t np,
                                            int64_t ld, void *fitness, double *G, int64_t ldG, int32_t wpw,
                                            qpm_stream sv)
{
    clear_error();
    qpm_status st = check_objective_args(o, p, bits, np, ld, fitness, G, ldG);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(wpw >= 1 && wpw <= table_max_wpw(p == QPM_PREC_F32), QPM_EINVAL,
                "words_per_wave must be in [1, %d] (got %d)", table_max_wpw(p == QPM_PREC_F32), (int)wpw);
    const ObjPlan pl = plan_objective_shape(*o, wpw);
    QPM_REQUIRE(pl.gy <= 65535, QPM_ERANGE, "too many workgroup segments (%d)", pl.gy);
    return eval_with_plan(o, p, bits, np, ld, fitness, G, ldG, pl, static_cast<hipStream_t>(sv));
}

static qpm_status eval_with_plan(qpm_objective o, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                 void *fitness, double *G, int64_t ldG, const ObjPlan &pl, hipStream_t s)
{
    ScratchLease lease(o->scratch, s);
    void *ws = nullptr;
    qpm_status st = lease.begin(objective_partials_bytes(*o, pl, ld), &ws);
    if (st != QPM_OK) return st;
    double *part = static_cast<double *>(ws);
    st = launch_objective_partials(*o, p, bits, np, ld, pl, part, s);
    if (st == QPM_OK) st = launch_objective_values(*o, pl, part, ld, np, fitness, p == QPM_PREC_F64, G, ldG, s);
    const qpm_status se = lease.end();
    return st != QPM_OK ? st : se;
}
