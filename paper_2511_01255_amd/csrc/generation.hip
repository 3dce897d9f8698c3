// generation.hip -- the end of each evaluation in a run: combine the
// segment triples into f = |d_eff|^2, greedy one-to-one selection (paper
// Sec. 2.2.1 step 4; Sec. 3.2 steps 2 and 5), then the global steps in a
// one-workgroup kernel: the three leaders after DE selection (Sec. 3.2
// step 3) or the advance to the next generation (whose DE draws the
// selection kernel writes).
#include "common.hpp"
#include "device_common.hpp"
#include "scan.hpp"

namespace qpm {

// Selection for the 64 genomes of group grp (i = 64 grp + lane), from their
// combined triple t; called by one whole wave. Writes f_cur, flags, the
// group's two packed flag words, the DE draws of generation gen + 1 (with
// draws_next) and the group's three best (with cand_v).
template <typename T>
__device__ __forceinline__ void select_group(const Tri &t, int64_t grp, int lane, int64_t np,
                                             const double *__restrict__ C, T *__restrict__ f_cur,
                                             uint32_t *__restrict__ flags, uint32_t *__restrict__ fbits,
                                             const int32_t *__restrict__ skip3, T *__restrict__ cand_v,
                                             int32_t *__restrict__ cand_i, int4 *__restrict__ draws_next,
                                             const uint32_t *__restrict__ gen, int64_t D, uint32_t k0, uint32_t k1,
                                             uint32_t inst)
{
    const int64_t i = grp * 64 + lane;
    const bool valid = i < np;
    uint32_t fl = 0;
    T fv = static_cast<T>(-INFINITY);
    if (valid) {
        const double sr = t.qr + C[0], si = t.qi + C[1];
        const T v = static_cast<T>(fma(sr, sr, si * si));
        const bool skip = skip3 != nullptr && (i == skip3[0] || i == skip3[1] || i == skip3[2]);
        fl = flags[i];
        fv = f_cur[i];
        if (!skip && v > fv) {
            fv = v;
            f_cur[i] = v;
            fl ^= 1u;
            flags[i] = fl;
        }
        if (draws_next) draws_next[i] = de_draw(i, np, D, gen[0] + 1u, inst, k0, k1);
    }
    const uint64_t m = __ballot(fl != 0u);
    if (fbits != nullptr && lane == 0) {
        fbits[2 * grp] = static_cast<uint32_t>(m);
        fbits[2 * grp + 1] = static_cast<uint32_t>(m >> 32);
    }
    if (cand_v) {
        Top3<T> tp = top3_empty<T>();
        tp.v[0] = fv;
        tp.i[0] = valid ? static_cast<int>(i) : INT_MAX;
        wave_top3(tp);
        if (lane < 3) {
            cand_v[3 * grp + lane] = lane == 0 ? tp.v[0] : (lane == 1 ? tp.v[1] : tp.v[2]);
            cand_i[3 * grp + lane] = lane == 0 ? tp.i[0] : (lane == 1 ? tp.i[1] : tp.i[2]);
        }
    }
}

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
                                                     uint32_t k1, uint32_t inst)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const Tri t = combine_segments<4>(part, gy, ld, i, i < np);
    if (threadIdx.x < 64)
        select_group<T>(t, blockIdx.x, lane, np, C, f_cur, flags, fbits, skip3, cand_v, cand_i, draws_next, gen, D,
                        k0, k1, inst);
}

// One workgroup: the leaders from the 3 candidates of each of the ngroups
// groups (top3_out), and/or the advance of the generation counter.
template <typename T>
__global__ __launch_bounds__(256) void finish_tail_kernel(const T *__restrict__ cand_v,
                                                          const int32_t *__restrict__ cand_i, int64_t ngroups,
                                                          int32_t *__restrict__ top3_out, uint32_t *__restrict__ gen,
                                                          int advance)
{
    if (top3_out) block_top3<T, 256>(cand_v, 3 * ngroups, top3_out, cand_i);
    if (advance && threadIdx.x == 0) gen[0] += 1u;
}

qpm_status launch_finish(const double *part, int gy, int64_t ld, int64_t np, const double *C, void *f_cur, bool f64,
                         uint32_t *flags, uint32_t *fbits, const int32_t *skip3, int32_t *top3_out, void *cand,
                         int4 *draws_next, uint32_t *gen, int64_t D, uint64_t seed, uint32_t inst, hipStream_t s)
{
    const unsigned blocks = static_cast<unsigned>((np + 63) / 64);
    QPM_REQUIRE(top3_out == nullptr || cand != nullptr, QPM_EINVAL, "leader candidates need a buffer");
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    const int advance = draws_next != nullptr;
    // cand: 3 values per workgroup (T) followed by 3 slots per workgroup (int32)
    if (f64) {
        double *cv = top3_out ? static_cast<double *>(cand) : nullptr;
        int32_t *ci = cv ? reinterpret_cast<int32_t *>(cv + 3 * static_cast<size_t>(blocks)) : nullptr;
        finish_kernel<double><<<blocks, 256, 0, s>>>(part, gy, ld, np, C, static_cast<double *>(f_cur), flags, fbits,
                                                     skip3, cv, ci, draws_next, gen, D, k0, k1, inst);
        if (top3_out || advance) finish_tail_kernel<double><<<1, 256, 0, s>>>(cv, ci, blocks, top3_out, gen, advance);
    } else {
        float *cv = top3_out ? static_cast<float *>(cand) : nullptr;
        int32_t *ci = cv ? reinterpret_cast<int32_t *>(cv + 3 * static_cast<size_t>(blocks)) : nullptr;
        finish_kernel<float><<<blocks, 256, 0, s>>>(part, gy, ld, np, C, static_cast<float *>(f_cur), flags, fbits,
                                                    skip3, cv, ci, draws_next, gen, D, k0, k1, inst);
        if (top3_out || advance) finish_tail_kernel<float><<<1, 256, 0, s>>>(cv, ci, blocks, top3_out, gen, advance);
    }
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

}  // namespace qpm
