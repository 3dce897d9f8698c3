// fused.hip -- whole HWSDA generations (paper Sec. 3.2, steps 2-6) in one
// workgroup for populations small enough to live in LDS (the plain
// configuration: N = 256 domains, NP = 32). A run's generation is otherwise
// six or seven launches of a few microseconds each; here one launch runs
// any number of generations with workgroup barriers between the steps.
//
// LDS holds both gene buffers (a per-row flag names the one holding the
// current row, as in the multi-kernel path), the fitness (as doubles), the
// trial / candidate bits, the DE draws, the leaders and, when they fit, the
// design's FP64 sign-pattern tables. The arithmetic of every step is the
// multi-kernel path's (de_draw, de_quad, gwo_quad; the FP64 table walk),
// so in FP64 trials, candidates and decisions are those of the oracle. An
// FP32 run takes the same FP64 walk and rounds each fitness to binary32,
// the precision its fitness is held and compared in (on one CU the FP64
// walk costs what an FP32 one would).
//
// Thread mapping: the optimiser steps walk (individual, gene quad) pairs,
// each individual padded to a whole number of 32-gene words, so eight
// neighbouring lanes always hold one bit word; the fitness gives each
// genome one 16-lane DPP row whose lanes walk consecutive 4-domain blocks
// and fold their triples in order with row shifts; the leaders come from
// each individual's rank, counted by its 16 lanes. The DE draws of the next
// generation depend on its number only, so they are drawn during the last
// evaluation of a generation by the highest threads (idle in the evaluation
// when np <= 32). Each genome's selection is taken by the first lane of its
// evaluation row right after the fold, so an evaluation and its selection
// need one barrier.
#include <algorithm>

#include "common.hpp"
#include "device_common.hpp"
#include "genes.hpp"
#include "scan.hpp"

namespace qpm {

namespace {

constexpr int kFusedThreads = 1024;

struct FusedArgs {
    float *x0;              // run buffer 0 (rows written back here)
    const float *x1;        // run buffer 1
    uint32_t *flags;        // per-row buffer flags (cleared on exit)
    uint32_t *fbits;        // packed flags (cleared on exit), nfb words
    void *f_cur;            // current fitness, double or float (read, written back)
    int f32;                // the run's fitness is binary32
    int32_t *leaders;       // leaders of the last generation (written)
    uint32_t *gen;          // generation counter (advanced by gens)
    const float *a_tab;     // a_g
    const float *F_tab;     // F_g
    const double2 *tab64;   // the design's FP64 sign-pattern tables
    const double *C;        // C (re, im)
    int64_t np, D, ldx;
    int W;                  // bit words per genome
    int nfb;                // packed flag words
    int gens;               // generations to run
    int algo;               // qpm_algo
    uint32_t cr_max, k0, k1, inst;
};

// LDS layout (bytes), shared by the kernel and the launcher
struct FusedLayout {
    int64_t D4, Q, Qpad;    // gene stride, quads, quads padded to whole words
    size_t buf, fs, fl, bw, dr, sl, tab, total;
};

__host__ __device__ inline FusedLayout fused_layout(int64_t np, int64_t D, int W, bool tab_lds)
{
    FusedLayout L;
    L.D4 = (D + 3) / 4 * 4;
    L.Q = (D + 3) / 4;
    L.Qpad = static_cast<int64_t>(W) * 8;
    size_t o = 0;
    L.buf = o;
    o += 2 * static_cast<size_t>(np) * L.D4 * sizeof(float);
    L.fs = o;
    o += static_cast<size_t>(np) * sizeof(double);
    L.dr = o;
    o += static_cast<size_t>(np) * sizeof(int4);
    L.fl = o;
    o += static_cast<size_t>(np) * sizeof(uint32_t);
    L.bw = o;
    o += static_cast<size_t>(np) * W * sizeof(uint32_t);
    L.sl = o;
    o += 4 * sizeof(int32_t);
    o = (o + 15) / 16 * 16;
    L.tab = o;
    if (tab_lds) o += static_cast<size_t>(W) * 8 * 48 * sizeof(double2);
    L.total = o;
    return L;
}

// lanes per genome of the fitness walk (np <= 64, so np T <= 1024); 16
// lanes keep the fold within one DPP row
constexpr int kFusedLanes = 16;

// the value of lane l + off (off in {1, 2, 4, 8}) of the same 16-lane row,
// by DPP row shifts (lanes past the row's end read 0; they are not used)
__device__ __forceinline__ double row_down(double v, int off)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int rl = 0, rh = 0;
    switch (off) {
    case 1:
        rl = __builtin_amdgcn_update_dpp(0, lo, 0x101, 0xF, 0xF, false);
        rh = __builtin_amdgcn_update_dpp(0, hi, 0x101, 0xF, 0xF, false);
        break;
    case 2:
        rl = __builtin_amdgcn_update_dpp(0, lo, 0x102, 0xF, 0xF, false);
        rh = __builtin_amdgcn_update_dpp(0, hi, 0x102, 0xF, 0xF, false);
        break;
    case 4:
        rl = __builtin_amdgcn_update_dpp(0, lo, 0x104, 0xF, 0xF, false);
        rh = __builtin_amdgcn_update_dpp(0, hi, 0x104, 0xF, 0xF, false);
        break;
    default:
        rl = __builtin_amdgcn_update_dpp(0, lo, 0x108, 0xF, 0xF, false);
        rh = __builtin_amdgcn_update_dpp(0, hi, 0x108, 0xF, 0xF, false);
        break;
    }
    return __hiloint2double(rh, rl);
}

// How the evaluated genomes replace the current ones (paper Sec. 3.2 steps 4
// and 5): SEL_GREEDY keeps a genome whose fitness is strictly higher;
// SEL_GREEDY_OMEGA does so for every genome but the three leaders; SEL_MOVE
// (the grey-wolf optimiser alone) moves every genome but the leaders.
enum { SEL_GREEDY = 0, SEL_GREEDY_OMEGA = 1, SEL_MOVE = 2 };

// The fitness of every genome of the bit words, then its selection, by the
// genome's first lane once its triples are folded (no other thread reads
// fs or fl meanwhile).
template <bool TAB_LDS>
__device__ __forceinline__ void fused_fitness(const FusedArgs &a, const FusedLayout &L, unsigned char *lds,
                                              const double2 *__restrict__ tabs, int sel, int4 lead)
{
    const uint32_t *bw = reinterpret_cast<const uint32_t *>(lds + L.bw);
    double *fs = reinterpret_cast<double *>(lds + L.fs);
    uint32_t *fl = reinterpret_cast<uint32_t *>(lds + L.fl);
    constexpr int T = kFusedLanes;
    const int tid = static_cast<int>(threadIdx.x);
    const int64_t i = tid / T;
    const int s = tid % T;
    const int NB = 8 * a.W;
    const int bpt = (NB + T - 1) / T;
    Tri t{0, 0, 0, 0, 0, 0};
    if (i < a.np) {
        const int b0 = s * bpt, b1 = min(NB, b0 + bpt);
        for (int b = b0; b < b1; ++b) {
            const uint32_t p = (bw[i * a.W + (b >> 3)] >> (4 * (b & 7))) & 15u;
            const double2 *e = tabs + static_cast<int64_t>(b) * 48 + p;
            const double2 A = e[0], B = e[16], Q = e[32];
            t.qr = fma(-t.ai, B.y, fma(t.ar, B.x, t.qr + Q.x));
            t.qi = fma(t.ai, B.x, fma(t.ar, B.y, t.qi + Q.y));
            t.ar += A.x;
            t.ai += A.y;
            t.br += B.x;
            t.bi += B.y;
        }
    }
    // fold the T triples of each genome in block order: after the round with
    // offset o, lane s (s a multiple of 2 o) holds blocks of lanes [s, s + 2 o)
#pragma unroll
    for (int off = 1; off < T; off <<= 1) {
        Tri u;
        u.ar = row_down(t.ar, off);
        u.ai = row_down(t.ai, off);
        u.br = row_down(t.br, off);
        u.bi = row_down(t.bi, off);
        u.qr = row_down(t.qr, off);
        u.qi = row_down(t.qi, off);
        if ((s & (2 * off - 1)) == 0) tri_append(t, u);
    }
    if (i < a.np && s == 0) {
        const double sr = t.qr + a.C[0], si = t.qi + a.C[1];
        double fnew = fma(sr, sr, si * si);
        // an FP32 run holds its fitness in binary32 (compared as such)
        if (a.f32) fnew = static_cast<double>(static_cast<float>(fnew));
        const bool leader = i == lead.x || i == lead.y || i == lead.z;
        const bool take = sel == SEL_GREEDY ? fnew > fs[i] : (!leader && (sel == SEL_MOVE || fnew > fs[i]));
        if (take) {
            fs[i] = fnew;
            fl[i] ^= 1u;
        }
    }
}

// The three best of fs[0..np) (f descending, slot ascending) into sl: 16
// lanes per individual count the individuals ahead of it over a quarter of
// the population each (np <= 64), the counts are summed across the DPP row,
// and the individuals of rank 0, 1, 2 write themselves. The order is strict
// and total, so the ranks are distinct. Called by every thread; ends with a
// barrier.
__device__ __forceinline__ void fused_leaders(const double *fs, int64_t np, int32_t *sl)
{
    const int tid = static_cast<int>(threadIdx.x);
    const int i = tid >> 4, part = tid & 15;
    int ahead = 0;
    if (i < np) {
        const double fi = fs[i];
        for (int j = part; j < np; j += 16) {
            const double fj = fs[j];
            ahead += (fj > fi || (fj == fi && j < i)) ? 1 : 0;
        }
    }
    ahead += __builtin_amdgcn_update_dpp(0, ahead, 0x101, 0xF, 0xF, false);
    ahead += __builtin_amdgcn_update_dpp(0, ahead, 0x102, 0xF, 0xF, false);
    ahead += __builtin_amdgcn_update_dpp(0, ahead, 0x104, 0xF, 0xF, false);
    ahead += __builtin_amdgcn_update_dpp(0, ahead, 0x108, 0xF, 0xF, false);
    if (i < np && part == 0 && ahead < 3) sl[ahead] = i;
    __syncthreads();
}

template <int VARIANT, bool TAB_LDS>
__global__ __launch_bounds__(kFusedThreads) void fused_gen_kernel(FusedArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const FusedLayout L = fused_layout(a.np, a.D, a.W, TAB_LDS);
    float *xb = reinterpret_cast<float *>(lds + L.buf);  // [2][np][D4]
    double *fs = reinterpret_cast<double *>(lds + L.fs);
    int4 *dr = reinterpret_cast<int4 *>(lds + L.dr);
    uint32_t *fl = reinterpret_cast<uint32_t *>(lds + L.fl);
    uint32_t *bw = reinterpret_cast<uint32_t *>(lds + L.bw);
    int32_t *sl = reinterpret_cast<int32_t *>(lds + L.sl);
    const double2 *tabs = TAB_LDS ? reinterpret_cast<const double2 *>(lds + L.tab) : a.tab64;
    const int tid = static_cast<int>(threadIdx.x);
    const int64_t np = a.np, D = a.D, D4 = L.D4, Q = L.Q, Qpad = L.Qpad;
    const size_t bufsz = static_cast<size_t>(np) * D4;  // floats per buffer
    auto row = [&](int64_t r, uint32_t b) -> float * { return xb + b * bufsz + r * D4; };

    // load the population (current rows through the run's flags) into
    // buffer 0, the fitness, and the tables
    for (int64_t k = tid; k < np * Q; k += kFusedThreads) {
        const int64_t r = k / Q, q = k % Q;
        const float *src = (a.flags[r] ? a.x1 : a.x0) + r * a.ldx;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (4 * q + 3 < D) {
            v = *reinterpret_cast<const float4 *>(src + 4 * q);
        } else {
            v.x = src[4 * q];
            if (4 * q + 1 < D) v.y = src[4 * q + 1];
            if (4 * q + 2 < D) v.z = src[4 * q + 2];
        }
        *reinterpret_cast<float4 *>(row(r, 0) + 4 * q) = v;
    }
    for (int64_t r = tid; r < np; r += kFusedThreads) {
        fs[r] = a.f32 ? static_cast<double>(static_cast<const float *>(a.f_cur)[r])
                      : static_cast<const double *>(a.f_cur)[r];
        fl[r] = 0u;
    }
    if constexpr (TAB_LDS) {
        double2 *dst = reinterpret_cast<double2 *>(lds + L.tab);
        for (int64_t k = tid; k < static_cast<int64_t>(a.W) * 8 * 48; k += kFusedThreads) dst[k] = a.tab64[k];
    }
    uint32_t g = a.gen[0];
    if (a.algo != QPM_ALGO_GWO && tid < np) dr[tid] = de_draw(tid, np, D, g, a.inst, a.k0, a.k1);
    __syncthreads();

    // one optimiser step over every (individual, quad) pair: fn(i, q) gives
    // the quad (and whether it exists); results go to the other buffer and
    // the bit words. All threads run the same number of rounds.
    const int64_t pairs = np * Qpad;
    const int rounds = static_cast<int>((pairs + kFusedThreads - 1) / kFusedThreads);

    for (int it = 0; it < a.gens; ++it, ++g) {
        const float Fg = a.F_tab[g];
        const float ag = a.a_tab[g];
        if (a.algo != QPM_ALGO_GWO) {
            // DE trials (draws of generation g ready), evaluation, greedy
            // selection
            for (int rd = 0; rd < rounds; ++rd) {
                const int64_t k = static_cast<int64_t>(rd) * kFusedThreads + tid;
                const int64_t i = k / Qpad, q = k % Qpad;
                uint32_t nib = 0;
                if (i < np && q < Q) {
                    const int4 d4 = dr[i];
                    const int64_t j0 = 4 * q;
                    const float4 xv = *reinterpret_cast<const float4 *>(row(i, fl[i]) + j0);
                    const float4 r1 = *reinterpret_cast<const float4 *>(row(d4.x, fl[d4.x]) + j0);
                    const float4 r2 = *reinterpret_cast<const float4 *>(row(d4.y, fl[d4.y]) + j0);
                    const float4 r3 = *reinterpret_cast<const float4 *>(row(d4.z, fl[d4.z]) + j0);
                    const float4 uv = de_quad(xv, r1, r2, r3, j0, d4.w, static_cast<uint32_t>(i), g, a.inst, a.k0,
                                              a.k1, Fg, a.cr_max);
                    *reinterpret_cast<float4 *>(row(i, fl[i] ^ 1u) + j0) = uv;
                    nib = quad_nibble(uv, j0, D);
                }
                const uint32_t w = or8_into_last(nib << (4 * (tid & 7)));
                if ((tid & 7) == 7 && i < np) bw[i * a.W + (q >> 3)] = w;
            }
            __syncthreads();
            // evaluation and greedy selection; DE alone: the draws of the
            // next generation (read by its DE step only)
            fused_fitness<TAB_LDS>(a, L, lds, tabs, SEL_GREEDY, make_int4(-1, -1, -1, -1));
            if (a.algo == QPM_ALGO_DE && tid >= kFusedThreads - np)
                dr[tid - (kFusedThreads - np)] =
                    de_draw(tid - (kFusedThreads - np), np, D, g + 1, a.inst, a.k0, a.k1);
            __syncthreads();
        }
        // leaders: the three best (f descending, slot ascending)
        fused_leaders(fs, np, sl);
        if (a.algo != QPM_ALGO_DE) {
            // grey-wolf candidates of the omega wolves, evaluation, selection
            const int32_t L0 = sl[0], L1 = sl[1], L2 = sl[2];
            const float two_a = 2.0f * ag;
            for (int rd = 0; rd < rounds; ++rd) {
                const int64_t k = static_cast<int64_t>(rd) * kFusedThreads + tid;
                const int64_t i = k / Qpad, q = k % Qpad;
                uint32_t nib = 0;
                if (i < np && q < Q && i != L0 && i != L1 && i != L2) {
                    const int64_t j0 = 4 * q;
                    const float4 xv = *reinterpret_cast<const float4 *>(row(i, fl[i]) + j0);
                    const float4 X0 = *reinterpret_cast<const float4 *>(row(L0, fl[L0]) + j0);
                    const float4 X1 = *reinterpret_cast<const float4 *>(row(L1, fl[L1]) + j0);
                    const float4 X2 = *reinterpret_cast<const float4 *>(row(L2, fl[L2]) + j0);
                    const float4 yv = gwo_quad<VARIANT>(xv, X0, X1, X2, static_cast<uint32_t>(q),
                                                        static_cast<uint32_t>(i), g, a.inst, a.k0, a.k1, ag, two_a);
                    *reinterpret_cast<float4 *>(row(i, fl[i] ^ 1u) + j0) = yv;
                    nib = quad_nibble(yv, j0, D);
                }
                const uint32_t w = or8_into_last(nib << (4 * (tid & 7)));
                if ((tid & 7) == 7 && i < np) bw[i * a.W + (q >> 3)] = w;
            }
            __syncthreads();
            // evaluation and selection (leaders kept); the DE draws of the
            // next generation (they depend on its number only)
            fused_fitness<TAB_LDS>(a, L, lds, tabs, a.algo == QPM_ALGO_GWO ? SEL_MOVE : SEL_GREEDY_OMEGA,
                                   make_int4(L0, L1, L2, -1));
            if (a.algo == QPM_ALGO_HWSDA && tid >= kFusedThreads - np)
                dr[tid - (kFusedThreads - np)] =
                    de_draw(tid - (kFusedThreads - np), np, D, g + 1, a.inst, a.k0, a.k1);
            __syncthreads();
            // the leaders of the next generation (and those reported)
            if (a.algo == QPM_ALGO_GWO) fused_leaders(fs, np, sl);
        }
    }

    // write back: every row to buffer 0 with its flag cleared
    for (int64_t k = tid; k < np * Q; k += kFusedThreads) {
        const int64_t r = k / Q, q = k % Q;
        const float4 v = *reinterpret_cast<const float4 *>(row(r, fl[r]) + 4 * q);
        float *dst = a.x0 + r * a.ldx + 4 * q;
        if (4 * q + 3 < D) {
            *reinterpret_cast<float4 *>(dst) = v;
        } else {
            dst[0] = v.x;
            if (4 * q + 1 < D) dst[1] = v.y;
            if (4 * q + 2 < D) dst[2] = v.z;
        }
    }
    for (int64_t r = tid; r < np; r += kFusedThreads) {
        if (a.f32)
            static_cast<float *>(a.f_cur)[r] = static_cast<float>(fs[r]);  // (exact: fs holds binary32 values)
        else
            static_cast<double *>(a.f_cur)[r] = fs[r];
        a.flags[r] = 0u;
    }
    for (int k = tid; k < a.nfb; k += kFusedThreads) a.fbits[k] = 0u;
    if (tid < 3) a.leaders[tid] = sl[tid];
    if (tid == 0) a.gen[0] = g;
}

}  // namespace

bool fused_eligible(int64_t np, int64_t D)
{
    if (np < 4 || np > 64 || D < 1) return false;
    const int W = static_cast<int>((D + 31) / 32);
    return fused_layout(np, D, W, false).total <= kFusedMaxLds;
}

qpm_status launch_fused_generations(const FusedRun &fr, int gens, hipStream_t s)
{
    QPM_REQUIRE(fused_eligible(fr.np, fr.D), QPM_EINVAL, "population does not fit the fused generation kernel");
    QPM_REQUIRE(fr.variant == 0 || fr.variant == 1, QPM_EINVAL, "fused generations take gwo_variant 0 or 1");
    FusedArgs a;
    a.x0 = fr.x0;
    a.x1 = fr.x1;
    a.flags = fr.flags;
    a.fbits = fr.fbits;
    a.f_cur = fr.f_cur;
    a.f32 = fr.f32;
    a.leaders = fr.leaders;
    a.gen = fr.gen;
    a.a_tab = fr.a_tab;
    a.F_tab = fr.F_tab;
    a.tab64 = fr.tab64;
    a.C = fr.C;
    a.np = fr.np;
    a.D = fr.D;
    a.ldx = fr.ldx;
    a.W = static_cast<int>((fr.D + 31) / 32);
    a.nfb = static_cast<int>(2 * ((fr.np + 63) / 64));
    a.gens = gens;
    a.algo = fr.algo;
    a.cr_max = cr_threshold(fr.CR);
    a.k0 = static_cast<uint32_t>(fr.seed);
    a.k1 = static_cast<uint32_t>(fr.seed >> 32);
    a.inst = fr.inst;
    const bool tab_lds = fused_layout(fr.np, fr.D, a.W, true).total <= kFusedMaxLds;
    const size_t lds = fused_layout(fr.np, fr.D, a.W, tab_lds).total;
#define QPM_FUSED(V, T)                                                                                          \
    {                                                                                                            \
        QPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&fused_gen_kernel<V, T>),                 \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));     \
        fused_gen_kernel<V, T><<<1, kFusedThreads, lds, s>>>(a);                                                 \
    }
    if (fr.variant == 1) {
        if (tab_lds) QPM_FUSED(1, true) else QPM_FUSED(1, false)
    } else {
        if (tab_lds) QPM_FUSED(0, true) else QPM_FUSED(0, false)
    }
#undef QPM_FUSED
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

}  // namespace qpm
