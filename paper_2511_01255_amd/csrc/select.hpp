// select.hpp -- greedy one-to-one selection of a group of 64 genomes
// (paper Sec. 2.2.1 step 4; Sec. 3.2 steps 2 and 5) and the one-workgroup
// tail of an evaluation (leaders, Sec. 3.2 step 3, or the generation
// advance), shared by the |d_eff|^2 fitness and the multi-wavelength
// objective.
#pragma once

#include "common.hpp"
#include "device_common.hpp"

namespace qpm {

// Selection for the 64 genomes of group grp (i = 64 grp + lane), from their
// fitness `value` (rounded to T here); called by one whole wave. Writes
// f_cur, flags, the group's two packed flag words, the DE draws of
// generation gen + next_off (with draws_next; next_off = 0 when the
// counter was already advanced), the group's three best (with
// cand_v) and, with acc.list, the accepted slots (appended in any order)
// and the packed flags from before the selection. With replace_all every
// genome outside skip3 takes its new value whatever its fitness (the move
// of the basic grey-wolf optimiser, which has no greedy selection).
template <typename T>
__device__ __forceinline__ void select_group(double value, int64_t grp, int lane, int64_t np, T *__restrict__ f_cur,
                                             uint32_t *__restrict__ flags, uint32_t *__restrict__ fbits,
                                             const int32_t *__restrict__ skip3, T *__restrict__ cand_v,
                                             int32_t *__restrict__ cand_i, int4 *__restrict__ draws_next,
                                             const uint32_t *__restrict__ gen, int64_t D, uint32_t k0, uint32_t k1,
                                             uint32_t inst, AcceptOut acc = AcceptOut{}, uint32_t next_off = 1u,
                                             bool replace_all = false)
{
    const int64_t i = grp * 64 + lane;
    const bool valid = i < np;
    uint32_t fl = 0, fl_old = 0;
    bool accepted = false;
    T fv = static_cast<T>(-INFINITY);
    if (valid) {
        const T v = static_cast<T>(value);
        const bool skip = skip3 != nullptr && (i == skip3[0] || i == skip3[1] || i == skip3[2]);
        fl = flags[i];
        fl_old = fl;
        fv = f_cur[i];
        if (!skip && (replace_all || v > fv)) {
            accepted = true;
            fv = v;
            f_cur[i] = v;
            fl ^= 1u;
            flags[i] = fl;
        }
        if (draws_next) draws_next[i] = de_draw(i, np, D, gen[0] + next_off, inst, k0, k1);
    }
    const uint64_t m = __ballot(fl != 0u);
    if (fbits != nullptr && lane == 0) {
        fbits[2 * grp] = static_cast<uint32_t>(m);
        fbits[2 * grp + 1] = static_cast<uint32_t>(m >> 32);
    }
    if (acc.list != nullptr) {
        const uint64_t mo = __ballot(fl_old != 0u);
        const uint64_t am = __ballot(accepted);
        if (lane == 0) {
            acc.fbits_prev[2 * grp] = static_cast<uint32_t>(mo);
            acc.fbits_prev[2 * grp + 1] = static_cast<uint32_t>(mo >> 32);
        }
        uint32_t base = 0;
        if (lane == 0 && am != 0) base = atomicAdd(acc.cnt, static_cast<uint32_t>(__popcll(am)));
        base = static_cast<uint32_t>(__shfl(static_cast<int>(base), 0));
        if (accepted)
            acc.list[base + static_cast<uint32_t>(__popcll(am & ((uint64_t(1) << lane) - 1)))] = static_cast<int32_t>(i);
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

}  // namespace qpm
