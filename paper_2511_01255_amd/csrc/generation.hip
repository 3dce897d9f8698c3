// generation.hip -- the end of each evaluation in a run: combine the
// segment triples into f = |d_eff|^2, greedy one-to-one selection (paper
// Sec. 2.2.1 step 4; Sec. 3.2 steps 2 and 5), then the global steps in a
// one-workgroup kernel: the three leaders after DE selection (Sec. 3.2
// step 3) or the advance to the next generation (whose DE draws the
// selection kernel writes).
#include "common.hpp"
#include "device_common.hpp"
#include "scan.hpp"
#include "select.hpp"

namespace qpm {

// Workgroup = 4 waves over 64 consecutive individuals (lane = individual):
// the waves fold the segment triples (combine_segments), wave 0 selects,
// keeps the packed copy of the buffer flags (bit i % 32 of word i / 32)
// that the DE kernel stages in LDS, and, when leaders are wanted, leaves
// its own three best in cand (3 per workgroup). The global steps (merging
// the candidates into the leaders, advancing the generation) run in
// finish_tail_kernel after it: a kernel boundary orders them, which costs
// less here than an agent-scope release (an L2 write-back) in every
// workgroup.
template <typename T>
__global__ __launch_bounds__(256) void finish_kernel(const double *__restrict__ part, int gy, int64_t ld, int64_t np,
                                                     const double *__restrict__ C, T *__restrict__ f_cur,
                                                     uint32_t *__restrict__ flags, uint32_t *__restrict__ fbits,
                                                     const int32_t *__restrict__ skip3, T *__restrict__ cand_v,
                                                     int32_t *__restrict__ cand_i, int4 *__restrict__ draws_next,
                                                     const uint32_t *__restrict__ gen, int64_t D, uint32_t k0,
                                                     uint32_t k1, uint32_t inst, AcceptOut acc, uint32_t next_off,
                                                     int32_t *__restrict__ top3_direct, int replace_all)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const Tri t = combine_segments<4>(part, gy, ld, i, i < np);
    if (threadIdx.x < 64) {
        const double sr = t.qr + C[0], si = t.qi + C[1];
        select_group<T>(fma(sr, sr, si * si), blockIdx.x, lane, np, f_cur, flags, fbits, skip3, cand_v, cand_i,
                        draws_next, gen, D, k0, k1, inst, acc, next_off, replace_all != 0);
    }
    // a one-workgroup population (np <= 64): the leaders from its own three
    // candidates, as the tail kernel would take them, without that launch
    if (top3_direct != nullptr) {
        __syncthreads();
        block_top3<T, 256>(cand_v, 3, top3_direct, cand_i);
    }
}

// Sum, maximum and minimum over the 1024 threads of the workgroup in a
// fixed order (butterfly within each wave, then the 16 wave results in
// order by every thread), so the result does not depend on timing.
__device__ __forceinline__ void block_sum_max_min(double &s, double &mx, double &mn, double *sh)
{
    for (int o = 1; o < 64; o <<= 1) {
        s += __shfl_xor(s, o);
        mx = fmax(mx, __shfl_xor(mx, o));
        mn = fmin(mn, __shfl_xor(mn, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[3 * w] = s;
        sh[3 * w + 1] = mx;
        sh[3 * w + 2] = mn;
    }
    __syncthreads();
    s = sh[0];
    mx = sh[1];
    mn = sh[2];
    for (int k = 1; k < 16; ++k) {
        s += sh[3 * k];
        mx = fmax(mx, sh[3 * k + 1]);
        mn = fmin(mn, sh[3 * k + 2]);
    }
    __syncthreads();
}

// The adaptive scale factor of paper Sec. 3.1.1 for generation g from the
// fitness of the population entering it: relative spread s = std / mean,
// kappa = (max - mean) / max (how far the mean trails the best), range =
// max - min. Low diversity (s < 0.1 or kappa < 0.1) raises F by 1.2; too
// much spread or a narrow range (s > 0.5 or range < 1e3) lowers it by 0.8;
// the factor scales the decay law F_base[g] and the result is kept in
// [0.01, 0.1]. Two passes (mean, then squared deviations) in FP64.
template <typename T>
__global__ __launch_bounds__(1024) void adapt_F_kernel(const T *__restrict__ f, int64_t np,
                                                       const uint32_t *__restrict__ gen, int64_t G,
                                                       const double *__restrict__ F_base, float *__restrict__ F_tab)
{
    __shared__ double sh[48];
    const int64_t g = gen[0];
    if (g >= G) return;
    double s = 0.0, mx = -INFINITY, mn = INFINITY;
    for (int64_t i = threadIdx.x; i < np; i += 1024) {
        const double v = static_cast<double>(f[i]);
        s += v;
        mx = fmax(mx, v);
        mn = fmin(mn, v);
    }
    block_sum_max_min(s, mx, mn, sh);
    const double mean = s / static_cast<double>(np);
    double ss = 0.0, d0 = 0.0, d1 = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 1024) {
        const double d = static_cast<double>(f[i]) - mean;
        ss += d * d;
    }
    block_sum_max_min(ss, d0, d1, sh);
    if (threadIdx.x == 0) {
        const double sd = sqrt(ss / static_cast<double>(np));
        const double rel = mean > 0.0 ? sd / mean : 0.0;
        const double kappa = mx > 0.0 ? (mx - mean) / mx : 0.0;
        double m = 1.0;
        if (rel < 0.1 || kappa < 0.1)
            m = 1.2;
        else if (rel > 0.5 || mx - mn < 1e3)
            m = 0.8;
        const double F = fmin(fmax(F_base[g] * m, 0.01), 0.1);
        F_tab[g] = static_cast<float>(F);
    }
}

qpm_status launch_adapt_F(const void *f, bool f64, int64_t np, const uint32_t *gen, int64_t G, const double *F_base,
                          float *F_tab, hipStream_t s)
{
    if (f64)
        adapt_F_kernel<double><<<1, 1024, 0, s>>>(static_cast<const double *>(f), np, gen, G, F_base, F_tab);
    else
        adapt_F_kernel<float><<<1, 1024, 0, s>>>(static_cast<const float *>(f), np, gen, G, F_base, F_tab);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_finish(const double *part, int gy, int64_t ld, int64_t np, const double *C, void *f_cur, bool f64,
                         uint32_t *flags, uint32_t *fbits, const int32_t *skip3, int32_t *top3_out, void *cand,
                         int4 *draws_next, uint32_t *gen, int64_t D, uint64_t seed, uint32_t inst, hipStream_t s,
                         AcceptOut acc, FinishMode mode)
{
    QPM_REQUIRE((acc.list == nullptr) == (acc.cnt == nullptr) && (acc.list == nullptr) == (acc.fbits_prev == nullptr),
                QPM_EINVAL, "the accepted list, its counter and the previous flags go together");
    const unsigned blocks = static_cast<unsigned>((np + 63) / 64);
    QPM_REQUIRE(top3_out == nullptr || cand != nullptr, QPM_EINVAL, "leader candidates need a buffer");
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    const int advance = draws_next != nullptr && !mode.gen_advanced;
    const uint32_t next_off = mode.gen_advanced ? 0u : 1u;
    // one workgroup: it merges its own candidates into the leaders
    int32_t *direct = blocks == 1 && !mode.defer_leaders ? top3_out : nullptr;
    const bool tail = (top3_out != nullptr && !mode.defer_leaders && direct == nullptr) || advance;
    int32_t *tail_top3 = mode.defer_leaders || direct != nullptr ? nullptr : top3_out;
    // cand: 3 values per workgroup (T) followed by 3 slots per workgroup (int32)
    if (f64) {
        double *cv = top3_out ? static_cast<double *>(cand) : nullptr;
        int32_t *ci = cv ? reinterpret_cast<int32_t *>(cv + 3 * static_cast<size_t>(blocks)) : nullptr;
        finish_kernel<double><<<blocks, 256, 0, s>>>(part, gy, ld, np, C, static_cast<double *>(f_cur), flags, fbits,
                                                     skip3, cv, ci, draws_next, gen, D, k0, k1, inst, acc, next_off,
                                                     direct, mode.replace_all ? 1 : 0);
        if (tail) finish_tail_kernel<double><<<1, 256, 0, s>>>(cv, ci, blocks, tail_top3, gen, advance);
    } else {
        float *cv = top3_out ? static_cast<float *>(cand) : nullptr;
        int32_t *ci = cv ? reinterpret_cast<int32_t *>(cv + 3 * static_cast<size_t>(blocks)) : nullptr;
        finish_kernel<float><<<blocks, 256, 0, s>>>(part, gy, ld, np, C, static_cast<float *>(f_cur), flags, fbits,
                                                    skip3, cv, ci, draws_next, gen, D, k0, k1, inst, acc, next_off,
                                                    direct, mode.replace_all ? 1 : 0);
        if (tail) finish_tail_kernel<float><<<1, 256, 0, s>>>(cv, ci, blocks, tail_top3, gen, advance);
    }
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

}  // namespace qpm
