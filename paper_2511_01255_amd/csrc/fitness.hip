// fitness.hip -- f = |d_eff|^2 over bit-packed +-1 genomes (paper Sec. 2.1).
//
// Per genome the double integral splits domain by domain into
//   d_eff = sum_n d_n b_n P_{n-1} + C,   P_n = sum_{m<=n} d_m a_m,
// and a stretch of domains reduces to the triple (A, B, Q) =
// (sum d a, sum d b, sum d_n b_n (A before n)). Triples combine
// associatively: (A1,B1,Q1) + (A2,B2,Q2) = (A1+A2, B1+B2, Q1+Q2+A1 B2).
//
// Mapping on gfx950: one lane per genome (a wave = 64 consecutive genomes,
// so each bit word load is one 256-byte coalesced row of the
// population-major layout). The domain axis is cut into segments of `wpw`
// words; each wave scans one segment, reading the per-domain coefficients
// with scalar loads (they are the same for every lane), the waves of a
// workgroup combine their triples in LDS in segment order, and a second
// small pass combines workgroup segments in order. No float atomics: the
// result depends only on the launch plan, never on timing.
#include "common.hpp"
#include "scan.hpp"

namespace qpm {

template <bool F32, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void fit_seg_kernel(const uint32_t *__restrict__ bits, int64_t ld, int W,
                                                             const double4 *__restrict__ ph64,
                                                             const float4 *__restrict__ ph32, int wpw, int64_t np,
                                                             double *__restrict__ part,
                                                             const double *__restrict__ C, void *__restrict__ fit,
                                                             int direct, int out_f64, uint32_t *__restrict__ advance)
{
    if (advance != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) advance[0] += 1u;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const int seg = static_cast<int>(blockIdx.y) * WAVES + wave;
    const int w0 = seg * wpw;
    const int w1 = min(W, w0 + wpw);
    Tri t{0, 0, 0, 0, 0, 0};
    const uint32_t *bp = bits + i;
    if (w0 < w1) {
        uint32_t next = bp[static_cast<int64_t>(w0) * ld];
        for (int wd = w0; wd < w1; ++wd) {
            const uint32_t word = next;
            if (wd + 1 < w1) next = bp[static_cast<int64_t>(wd + 1) * ld];
            if constexpr (F32)
                scan_word_f32(t, word, ph64 + static_cast<int64_t>(wd) * 32, ph32 + static_cast<int64_t>(wd) * 32);
            else
                scan_word_f64(t, word, ph64 + static_cast<int64_t>(wd) * 32);
        }
    }
    if constexpr (WAVES > 1) {
        __shared__ double sh[6][WAVES][64];
        sh[0][wave][lane] = t.ar;
        sh[1][wave][lane] = t.ai;
        sh[2][wave][lane] = t.br;
        sh[3][wave][lane] = t.bi;
        sh[4][wave][lane] = t.qr;
        sh[5][wave][lane] = t.qi;
        __syncthreads();
        if (wave != 0) return;
#pragma unroll 1
        for (int w = 1; w < WAVES; ++w) {
            const Tri u{sh[0][w][lane], sh[1][w][lane], sh[2][w][lane],
                        sh[3][w][lane], sh[4][w][lane], sh[5][w][lane]};
            tri_append(t, u);
        }
    }
    if (direct) {
        if (i < np) store_fitness(fit, out_f64, i, t, C);
    } else {
        double *o = part + static_cast<int64_t>(blockIdx.y) * 6 * ld + i;
        o[0 * ld] = t.ar;
        o[1 * ld] = t.ai;
        o[2 * ld] = t.br;
        o[3 * ld] = t.bi;
        o[4 * ld] = t.qr;
        o[5 * ld] = t.qi;
    }
}

// 64 genomes per workgroup of 4 waves (see combine_segments)
__global__ __launch_bounds__(256) void fit_combine_kernel(const double *__restrict__ part, int gy, int64_t ld,
                                                          int64_t np, const double *__restrict__ C,
                                                          void *__restrict__ fit, int out_f64)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + (threadIdx.x & 63);
    const Tri t = combine_segments<4>(part, gy, ld, i, i < np);
    if (threadIdx.x < 64 && i < np) store_fitness(fit, out_f64, i, t, C);
}

// The per-individual scheme: one lane walks its whole genome; no segment
// triples, so B is not tracked. With `part` the result is written as the
// single segment triple (A, 0, Q) instead of a fitness value.
__global__ __launch_bounds__(128) void fit_per_genome_kernel(const uint32_t *__restrict__ bits, int64_t ld, int W,
                                                             const double4 *__restrict__ ph64, int64_t np,
                                                             const double *__restrict__ C, double *__restrict__ fit,
                                                             double *__restrict__ part, uint32_t *__restrict__ advance)
{
    if (advance != nullptr && blockIdx.x == 0 && threadIdx.x == 0) advance[0] += 1u;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 128 + threadIdx.x;
    if (i >= np) return;
    double ar = 0, ai = 0, qr = 0, qi = 0;
    for (int wd = 0; wd < W; ++wd) {
        const uint32_t word = bits[static_cast<int64_t>(wd) * ld + i];
        const double4 *p = ph64 + static_cast<int64_t>(wd) * 32;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const double4 c = p[k];
            const double s = sign64(word, k);
            const double tr = fma(c.z, ar, -(c.w * ai));
            const double ti = fma(c.z, ai, c.w * ar);
            qr = fma(s, tr, qr);
            qi = fma(s, ti, qi);
            ar = fma(s, c.x, ar);
            ai = fma(s, c.y, ai);
        }
    }
    if (part) {
        double *o = part + i;
        o[0] = ar;
        o[ld] = ai;
        o[2 * ld] = 0.0;
        o[3 * ld] = 0.0;
        o[4 * ld] = qr;
        o[5 * ld] = qi;
        return;
    }
    const double sr = qr + C[0], si = qi + C[1];
    fit[i] = fma(sr, sr, si * si);
}

// The table kernel: each 4-domain block contributes the precomputed triple
// of its sign pattern (16 patterns per block, Design::tabq / tab64), so a
// domain evaluation costs a quarter of a pattern lookup plus one triple
// append, instead of a complex multiply-add per domain:
//   Q += A Bp + Qp,  A += Ap,  B += Bp   (complex; p = 4 bits of the word).
// Workgroup = GW genome groups x 4 segment waves (wave = 64 genomes, lane =
// genome). The workgroup copies the tables of its 4 wpw words to LDS (one
// component row of 16 patterns is 128 bytes in FP32, so a wave's lookups
// of one component hit distinct banks), each wave walks wpw words of its
// segment, and the 4 segment triples of each genome are combined in LDS in
// order. FP32: the word's A and B summed exactly in fixed point, its Q in
// binary32, each word's triple folded into FP64 (word_tab_q); FP64:
// binary64 throughout.
template <bool F32, int GW>
__global__ __launch_bounds__(GW * 256) void fit_tab_kernel(const uint32_t *__restrict__ bits, int64_t ld, int W,
                                                           const double2 *__restrict__ tab64,
                                                           const int2 *__restrict__ tabq,
                                                           const double *__restrict__ wsc, int wpw, int64_t np,
                                                           double *__restrict__ part, const double *__restrict__ C,
                                                           void *__restrict__ fit, int direct, int out_f64,
                                                           uint32_t *__restrict__ advance)
{
    extern __shared__ __align__(16) unsigned char lds[];
    // a run's generation advance, taken here because this kernel does not
    // read the counter (the finish step after it reads the new value)
    if (advance != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) advance[0] += 1u;
    const int wbase = static_cast<int>(blockIdx.y) * 4 * wpw;
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * GW + (threadIdx.x >> 8)) * 64 + (threadIdx.x & 63);
    Tri t;
    if (!tab_segment<F32, GW>(t, bits, ld, W, wbase, tab64, tabq, wsc, wpw, np, lds)) return;
    if (direct) {
        store_fitness(fit, out_f64, i, t, C);
    } else {
        double *o = part + static_cast<int64_t>(blockIdx.y) * 6 * ld + i;
        o[0 * ld] = t.ar;
        o[1 * ld] = t.ai;
        o[2 * ld] = t.br;
        o[3 * ld] = t.bi;
        o[4 * ld] = t.qr;
        o[5 * ld] = t.qi;
    }
}

size_t table_lds_bytes(int64_t W, bool f32, int gw, int wpw)
{
    const int64_t words = std::min<int64_t>(W, 4 * static_cast<int64_t>(wpw));
    const size_t tab = static_cast<size_t>(words) * 8 * 48 * (f32 ? 8 : 16);
    const size_t comb = static_cast<size_t>(gw) * 4 * 64 * 6 * 8;
    return std::max(tab, comb);
}

template <bool F32>
static qpm_status launch_tab(const Design &d, const FitPlan &pl, const uint32_t *bits, int64_t np, int64_t ld,
                             double *part, void *fit, int out_f64, bool direct_ok, hipStream_t s,
                             uint32_t *advance = nullptr)
{
    const int gw = pl.waves;
    const dim3 grid(static_cast<unsigned>((np + 64 * gw - 1) / (64 * gw)), static_cast<unsigned>(pl.gy));
    const int direct = direct_ok && pl.gy == 1;
    const int W = static_cast<int>(d.words);
    const size_t lds = table_lds_bytes(d.words, F32, gw, pl.wpw);
#define QPM_TAB_CASE(G)                                                                                       \
    case G:                                                                                                   \
        fit_tab_kernel<F32, G><<<grid, dim3(G * 256), lds, s>>>(bits, ld, W, d.tab64, d.tabq, d.wsc, pl.wpw, np,  \
                                                                part,                                         \
                                                                d.Cdev, fit, direct, out_f64, advance);      \
        break;
    switch (gw) {
        QPM_TAB_CASE(1)
        QPM_TAB_CASE(2)
        QPM_TAB_CASE(4)
    default: QPM_REQUIRE(false, QPM_EINVAL, "unsupported genome groups per workgroup %d", gw);
    }
#undef QPM_TAB_CASE
    return QPM_OK;
}

template <bool F32>
static qpm_status launch_seg(const Design &d, const FitPlan &pl, const uint32_t *bits, int64_t np, int64_t ld,
                             double *part, void *fit, int out_f64, bool direct_ok, hipStream_t s,
                             uint32_t *advance = nullptr)
{
    const dim3 grid(static_cast<unsigned>((np + 63) / 64), static_cast<unsigned>(pl.gy));
    const int direct = direct_ok && pl.gy == 1;
    const int W = static_cast<int>(d.words);
#define QPM_SEG_CASE(NW)                                                                                       \
    case NW:                                                                                                   \
        fit_seg_kernel<F32, NW><<<grid, dim3(NW * 64), 0, s>>>(bits, ld, W, d.ph64, d.ph32, pl.wpw, np, part, \
                                                              d.Cdev, fit, direct, out_f64, advance);         \
        break;
    switch (pl.waves) {
        QPM_SEG_CASE(1)
        QPM_SEG_CASE(2)
        QPM_SEG_CASE(4)
        QPM_SEG_CASE(8)
        QPM_SEG_CASE(16)
    default: QPM_REQUIRE(false, QPM_EINVAL, "unsupported waves per workgroup %d", pl.waves);
    }
#undef QPM_SEG_CASE
    return QPM_OK;
}

FitPlan plan_fitness_table(const Design &d, qpm_prec p, int gw, int wpw)
{
    (void)p;
    FitPlan pl;
    pl.kind = QPM_FIT_TABLE;
    pl.waves = gw;
    pl.wpw = wpw;
    pl.gy = static_cast<int>((d.words + 4 * static_cast<int64_t>(wpw) - 1) / (4 * static_cast<int64_t>(wpw)));
    return pl;
}

FitPlan plan_fitness(const Design &d, qpm_prec p, int64_t np, int kernel)
{
    FitPlan pl;
    if (kernel == QPM_FIT_PER_GENOME) {
        pl.kind = QPM_FIT_PER_GENOME;
        pl.gy = 1;
        return pl;
    }
    if (kernel == QPM_FIT_AUTO || kernel == QPM_FIT_TABLE) {
        // 48 KB of tables per workgroup: 4 wpw words of 3 KB (FP32) or 6 KB
        const int wpw = p == QPM_PREC_F32 ? 4 : 2;
        const int gw = np >= 1024 ? 4 : (np >= 256 ? 2 : 1);
        return plan_fitness_table(d, p, gw, wpw);
    }
    pl.kind = QPM_FIT_SEGMENTED;
    const int64_t groups = (np + 63) / 64;
    const int64_t W = d.words;
    // aim for ~8 waves per SIMD on 256 CUs x 4 SIMDs
    const int64_t target_waves = 8192;
    int64_t segs = (target_waves + groups - 1) / groups;
    if (segs < 1) segs = 1;
    int64_t wpw = (W + segs - 1) / segs;
    if (wpw < 1) wpw = 1;
    const int64_t nseg = (W + wpw - 1) / wpw;
    int waves = 1;
    while (waves < 16 && waves < nseg) waves *= 2;
    pl.waves = waves;
    pl.wpw = static_cast<int>(wpw);
    pl.gy = static_cast<int>((nseg + waves - 1) / waves);
    return pl;
}

FitPlan plan_fitness_shape(const Design &d, int waves, int wpw)
{
    FitPlan pl;
    pl.kind = QPM_FIT_SEGMENTED;
    pl.waves = waves;
    pl.wpw = wpw;
    const int64_t nseg = (d.words + wpw - 1) / wpw;
    pl.gy = static_cast<int>((nseg + waves - 1) / waves);
    return pl;
}

size_t fitness_workspace_bytes(const FitPlan &pl, int64_t ld)
{
    if (pl.kind == QPM_FIT_PER_GENOME || pl.gy <= 1) return 0;
    return sizeof(double) * 6 * static_cast<size_t>(pl.gy) * static_cast<size_t>(ld);
}

size_t fitness_partials_bytes(const FitPlan &pl, int64_t ld)
{
    const size_t gy = pl.kind == QPM_FIT_PER_GENOME ? 1 : static_cast<size_t>(pl.gy);
    return sizeof(double) * 6 * gy * static_cast<size_t>(ld);
}

qpm_status launch_fitness(const Design &d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld, void *fit,
                          const FitPlan &pl, double *part, hipStream_t s)
{
    const int out_f64 = (p == QPM_PREC_F64);
    if (pl.kind == QPM_FIT_PER_GENOME) {
        const unsigned blocks = static_cast<unsigned>((np + 127) / 128);
        fit_per_genome_kernel<<<blocks, 128, 0, s>>>(bits, ld, static_cast<int>(d.words), d.ph64, np, d.Cdev,
                                                     static_cast<double *>(fit), nullptr, nullptr);
    } else {
        qpm_status st;
        if (pl.kind == QPM_FIT_TABLE)
            st = p == QPM_PREC_F32 ? launch_tab<true>(d, pl, bits, np, ld, part, fit, out_f64, true, s)
                                   : launch_tab<false>(d, pl, bits, np, ld, part, fit, out_f64, true, s);
        else
            st = p == QPM_PREC_F32 ? launch_seg<true>(d, pl, bits, np, ld, part, fit, out_f64, true, s)
                                   : launch_seg<false>(d, pl, bits, np, ld, part, fit, out_f64, true, s);
        if (st != QPM_OK) return st;
        if (pl.gy > 1) {
            const unsigned blocks = static_cast<unsigned>((np + 63) / 64);
            fit_combine_kernel<<<blocks, 256, 0, s>>>(part, pl.gy, ld, np, d.Cdev, fit, out_f64);
        }
    }
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_fitness_partials(const Design &d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                   const FitPlan &pl, double *part, hipStream_t s, uint32_t *advance)
{
    if (pl.kind == QPM_FIT_PER_GENOME) {
        const unsigned blocks = static_cast<unsigned>((np + 127) / 128);
        fit_per_genome_kernel<<<blocks, 128, 0, s>>>(bits, ld, static_cast<int>(d.words), d.ph64, np, d.Cdev,
                                                     nullptr, part, advance);
    } else {
        qpm_status st;
        if (pl.kind == QPM_FIT_TABLE)
            st = p == QPM_PREC_F32 ? launch_tab<true>(d, pl, bits, np, ld, part, nullptr, 0, false, s, advance)
                                   : launch_tab<false>(d, pl, bits, np, ld, part, nullptr, 1, false, s, advance);
        else
            st = p == QPM_PREC_F32 ? launch_seg<true>(d, pl, bits, np, ld, part, nullptr, 0, false, s, advance)
                                   : launch_seg<false>(d, pl, bits, np, ld, part, nullptr, 1, false, s, advance);
        if (st != QPM_OK) return st;
    }
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

}  // namespace qpm

using namespace qpm;

static qpm_status check_fitness_args(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                     void *fitness)
{
    QPM_REQUIRE(d && bits && fitness, QPM_EINVAL, "design, bits and fitness must not be NULL");
    QPM_REQUIRE(p == QPM_PREC_F32 || p == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", (int)p);
    QPM_REQUIRE(np >= 1, QPM_EINVAL, "np must be >= 1 (got %lld)", (long long)np);
    QPM_REQUIRE(ld >= np && ld % 64 == 0, QPM_EINVAL, "ld (%lld) must be >= np (%lld) and a multiple of 64",
                (long long)ld, (long long)np);
    QPM_REQUIRE((reinterpret_cast<uintptr_t>(bits) & 3u) == 0, QPM_EINVAL, "bits must be 4-byte aligned");
    QPM_REQUIRE(np <= (int64_t(1) << 31) && d->words * ld <= (int64_t(1) << 40), QPM_ERANGE,
                "population too large");
    return QPM_OK;
}

static qpm_status run_plan(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld, void *fitness,
                           const FitPlan &pl, hipStream_t s)
{
    ScratchLease lease(d->scratch, s);
    void *ws = nullptr;
    qpm_status st = lease.begin(fitness_workspace_bytes(pl, ld), &ws);
    if (st != QPM_OK) return st;
    st = launch_fitness(*d, p, bits, np, ld, fitness, pl, static_cast<double *>(ws), s);
    const qpm_status se = lease.end();
    return st != QPM_OK ? st : se;
}

QPM_API qpm_status qpm_eval_fitness(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                    void *fitness, int32_t kernel, qpm_stream sv)
{
    clear_error();
    QPM_REQUIRE(kernel == QPM_FIT_AUTO || kernel == QPM_FIT_SEGMENTED || kernel == QPM_FIT_PER_GENOME ||
                    kernel == QPM_FIT_TABLE,
                QPM_EINVAL, "unknown fitness kernel %d", (int)kernel);
    QPM_REQUIRE(!(kernel == QPM_FIT_PER_GENOME && p != QPM_PREC_F64), QPM_EINVAL,
                "the per-genome kernel computes in FP64 only");
    qpm_status st = check_fitness_args(d, p, bits, np, ld, fitness);
    if (st != QPM_OK) return st;
    return run_plan(d, p, bits, np, ld, fitness, plan_fitness(*d, p, np, kernel), static_cast<hipStream_t>(sv));
}

QPM_API qpm_status qpm_eval_fitness_shape(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                          void *fitness, int32_t waves, int32_t wpw, qpm_stream sv)
{
    clear_error();
    QPM_REQUIRE(waves == 1 || waves == 2 || waves == 4 || waves == 8 || waves == 16, QPM_EINVAL,
                "waves_per_group must be 1, 2, 4, 8 or 16 (got %d)", (int)waves);
    QPM_REQUIRE(wpw >= 1, QPM_EINVAL, "words_per_wave must be >= 1 (got %d)", (int)wpw);
    qpm_status st = check_fitness_args(d, p, bits, np, ld, fitness);
    if (st != QPM_OK) return st;
    const FitPlan pl = plan_fitness_shape(*d, waves, wpw);
    QPM_REQUIRE(pl.gy <= 65535, QPM_ERANGE, "too many workgroup segments (%d)", pl.gy);
    return run_plan(d, p, bits, np, ld, fitness, pl, static_cast<hipStream_t>(sv));
}

QPM_API qpm_status qpm_eval_fitness_table_shape(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np,
                                                int64_t ld, void *fitness, int32_t groups, int32_t wpw,
                                                qpm_stream sv)
{
    clear_error();
    QPM_REQUIRE(groups == 1 || groups == 2 || groups == 4, QPM_EINVAL,
                "groups_per_workgroup must be 1, 2 or 4 (got %d)", (int)groups);
    QPM_REQUIRE(wpw >= 1, QPM_EINVAL, "words_per_wave must be >= 1 (got %d)", (int)wpw);
    qpm_status st = check_fitness_args(d, p, bits, np, ld, fitness);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(wpw <= table_max_wpw(p == QPM_PREC_F32), QPM_EINVAL,
                "words_per_wave %d exceeds %d (the tables of 4 words_per_wave words must fit in 64 KB of LDS)",
                (int)wpw, table_max_wpw(p == QPM_PREC_F32));
    const FitPlan pl = plan_fitness_table(*d, p, groups, wpw);
    QPM_REQUIRE(pl.gy <= 65535, QPM_ERANGE, "too many workgroup segments (%d)", pl.gy);
    return run_plan(d, p, bits, np, ld, fitness, pl, static_cast<hipStream_t>(sv));
}
