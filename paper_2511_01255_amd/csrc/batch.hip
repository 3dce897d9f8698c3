// batch.hip -- many independent designs of uneven length and phase
// mismatch optimised together: every step of a generation is one launch over
// all instances (an addition to the paper, whose runs optimise one crystal
// at a time).
//
// Layout: the per-domain tables of all instances are concatenated by whole
// 32-domain words (instance b starts at word row wofs_b), and so are the
// population-major bit rows; gene rows of instance b start at float offset
// xofs_b (row stride ldx_b). Per-individual arrays (fitness, flags, DE
// draws) are instance-major, np per instance. Small device tables map a
// workgroup to its (instance, segment) for the fitness and (instance,
// chunk) for DE, GWO and initialisation. Every instance uses the Philox
// instance number inst0 + b, so its random streams are those of a
// single-design run with that instance number.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "device_common.hpp"
#include "genes.hpp"
#include "scan.hpp"

namespace qpm {

struct InstDesc {
    int64_t n;     // domains (= genes)
    int64_t words; // W
    int64_t wofs;  // first word row of the instance
    int64_t xofs;  // float offset of row 0 in a gene buffer
    int64_t ldx;   // gene row stride
    double C[2];
};

struct FitSeg {
    int inst;  // instance
    int w0;    // first word (within the instance) of the workgroup
    int slot;  // partial slot
    int pad;
};

struct Tile {
    int inst;
    int chunk;
};

// ---------------------------------------------------------------- fitness

template <bool F32, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void batch_fit_kernel(const uint32_t *__restrict__ bits, int64_t ld,
                                                               const double4 *__restrict__ ph64,
                                                               const float4 *__restrict__ ph32, int wpw,
                                                               const InstDesc *__restrict__ inst,
                                                               const FitSeg *__restrict__ tab,
                                                               double *__restrict__ part, uint32_t *__restrict__ advance)
{
    if (advance != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) advance[0] += 1u;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const FitSeg fs = tab[blockIdx.y];
    const InstDesc id = inst[fs.inst];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const int w0 = fs.w0 + wave * wpw;
    const int w1 = min(static_cast<int>(id.words), w0 + wpw);
    Tri t{0, 0, 0, 0, 0, 0};
    const uint32_t *bp = bits + id.wofs * ld + i;
    if (w0 < w1) {
        uint32_t next = bp[static_cast<int64_t>(w0) * ld];
        for (int wd = w0; wd < w1; ++wd) {
            const uint32_t word = next;
            if (wd + 1 < w1) next = bp[static_cast<int64_t>(wd + 1) * ld];
            const int64_t dom = (id.wofs + wd) * 32;
            if constexpr (F32)
                scan_word_f32(t, word, ph64 + dom, ph32 + dom);
            else
                scan_word_f64(t, word, ph64 + dom);
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
    double *o = part + static_cast<int64_t>(fs.slot) * 6 * ld + i;
    o[0] = t.ar;
    o[ld] = t.ai;
    o[2 * ld] = t.br;
    o[3 * ld] = t.bi;
    o[4 * ld] = t.qr;
    o[5 * ld] = t.qi;
}

// The table kernel over (instance, segment) tiles: the sign-pattern tables
// and bit rows of instance b start at its word row wofs_b.
template <bool F32, int GW>
__global__ __launch_bounds__(GW * 256) void batch_fit_tab_kernel(const uint32_t *__restrict__ bits, int64_t ld,
                                                                 const double2 *__restrict__ tab64,
                                                                 const int2 *__restrict__ tabq,
                                                                 const double *__restrict__ wsc, int wpw,
                                                                 int64_t np, const InstDesc *__restrict__ inst,
                                                                 const FitSeg *__restrict__ tab,
                                                                 double *__restrict__ part,
                                                                 uint32_t *__restrict__ advance)
{
    extern __shared__ __align__(16) unsigned char lds[];
    // a run's generation advance (this kernel does not read the counter)
    if (advance != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) advance[0] += 1u;
    const FitSeg fs = tab[blockIdx.y];
    const InstDesc id = inst[fs.inst];
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * GW + (threadIdx.x >> 8)) * 64 + (threadIdx.x & 63);
    Tri t;
    if (!tab_segment<F32, GW>(t, bits + id.wofs * ld, ld, static_cast<int>(id.words), fs.w0,
                              tab64 + id.wofs * 8 * 48, tabq + id.wofs * 8 * 48, wsc + id.wofs, wpw, np, lds))
        return;
    double *o = part + static_cast<int64_t>(fs.slot) * 6 * ld + i;
    o[0] = t.ar;
    o[ld] = t.ai;
    o[2 * ld] = t.br;
    o[3 * ld] = t.bi;
    o[4 * ld] = t.qr;
    o[5 * ld] = t.qi;
}

// One workgroup of 1024 threads per instance: four threads per genome fold
// a quarter of the instance's slots each (in order), the first folds the
// four quarters in order, then
//   mode 0 (evaluation only): f_out[b][i] = f;
//   mode 1 (initial): f_cur = f, leaders, DE draws of generation gen;
//   mode 2 (after DE): select, leaders;
//   mode 3 (after GWO): select with the leaders excluded, DE draws of the
//     next generation (gen, which the evaluation kernel before this one
//     advanced: it does not read the counter, so no cross-workgroup
//     ordering is needed here).
template <typename T>
__global__ __launch_bounds__(1024) void batch_finish_kernel(int mode, const double *__restrict__ part,
                                                           const int *__restrict__ slot_ofs, int64_t ld, int64_t np,
                                                           const InstDesc *__restrict__ inst, T *__restrict__ f_cur,
                                                           uint32_t *__restrict__ flags, int32_t *__restrict__ leaders,
                                                           int4 *__restrict__ draws, uint32_t *__restrict__ gen,
                                                           uint32_t k0, uint32_t k1, uint32_t inst0,
                                                           uint32_t *__restrict__ fbits,
                                                           AcceptOut acc)
{
    const int b = blockIdx.x;
    const InstDesc id = inst[b];
    const int s0 = slot_ofs[b], s1 = slot_ofs[b + 1];
    T *fb = f_cur + static_cast<int64_t>(b) * np;
    uint32_t *flb = flags ? flags + static_cast<int64_t>(b) * np : nullptr;
    int32_t *Lb = leaders ? leaders + 3 * b : nullptr;
    const uint32_t g = gen ? gen[0] : 0u;
    int32_t L0 = -1, L1 = -1, L2 = -1;
    if (mode == 3) {
        L0 = Lb[0];
        L1 = Lb[1];
        L2 = Lb[2];
    }
    const int64_t fw = (np + 31) / 32;  // packed flag words per instance
    const int quarter = static_cast<int>(threadIdx.x >> 8);
    const int q0 = s0 + (s1 - s0) * quarter / 4, q1 = s0 + (s1 - s0) * (quarter + 1) / 4;
    __shared__ double sq[3][6][256];
    for (int64_t base = 0; base < np; base += 256) {
        const int64_t i = base + (threadIdx.x & 255);
        const bool valid = i < np;
        Tri t{0, 0, 0, 0, 0, 0};
        if (valid && q0 < q1) {
            const double *p = part + static_cast<int64_t>(q0) * 6 * ld + i;
            t = Tri{p[0], p[ld], p[2 * ld], p[3 * ld], p[4 * ld], p[5 * ld]};
            for (int sg = q0 + 1; sg < q1; ++sg) {
                const double *q = part + static_cast<int64_t>(sg) * 6 * ld + i;
                tri_append(t, Tri{q[0], q[ld], q[2 * ld], q[3 * ld], q[4 * ld], q[5 * ld]});
            }
        }
        if (quarter > 0) {
            sq[quarter - 1][0][threadIdx.x & 255] = t.ar;
            sq[quarter - 1][1][threadIdx.x & 255] = t.ai;
            sq[quarter - 1][2][threadIdx.x & 255] = t.br;
            sq[quarter - 1][3][threadIdx.x & 255] = t.bi;
            sq[quarter - 1][4][threadIdx.x & 255] = t.qr;
            sq[quarter - 1][5][threadIdx.x & 255] = t.qi;
        }
        __syncthreads();
        uint32_t fl = 0, fl_old = 0;
        bool accepted = false;
        if (quarter == 0 && valid) {
        for (int u = 0; u < 3; ++u) {
            const int lo = s0 + (s1 - s0) * (u + 1) / 4, hi = s0 + (s1 - s0) * (u + 2) / 4;
            if (lo < hi)
                tri_append(t, Tri{sq[u][0][threadIdx.x], sq[u][1][threadIdx.x], sq[u][2][threadIdx.x],
                                  sq[u][3][threadIdx.x], sq[u][4][threadIdx.x], sq[u][5][threadIdx.x]});
        }
        const double sr = t.qr + id.C[0], si = t.qi + id.C[1];
        const T v = static_cast<T>(fma(sr, sr, si * si));
        if (mode <= 1) {
            fb[i] = v;
        } else {
            const bool skip = (mode == 3) && (i == L0 || i == L1 || i == L2);
            fl = flb[i];
            fl_old = fl;
            if (!skip && v > fb[i]) {
                accepted = true;
                fb[i] = v;
                fl ^= 1u;
                flb[i] = fl;
            }
        }
        if (mode == 1 || mode == 3)  // mode 3: the evaluation kernel already advanced gen
            draws[static_cast<int64_t>(b) * np + i] = de_draw(i, np, id.n, g, inst0 + static_cast<uint32_t>(b), k0, k1);
        }
        // the packed copy of this wave's 64 flags (words (base + 64 w) / 32 and + 1)
        if (quarter == 0 && mode >= 2 && fbits) {
            const uint64_t m = __ballot(fl != 0u);
            const int64_t w0 = (base + 64 * (threadIdx.x >> 6)) / 32;
            if ((threadIdx.x & 63) == 0) {
                if (w0 < fw) fbits[b * fw + w0] = static_cast<uint32_t>(m);
                if (w0 + 1 < fw) fbits[b * fw + w0 + 1] = static_cast<uint32_t>(m >> 32);
            }
        }
        // accepted trials listed (as instance * np + slot) for
        // batch_materialize_kernel, with the flags from before the selection
        if (quarter == 0 && mode == 2 && acc.list != nullptr) {
            const int lane = threadIdx.x & 63;
            const uint64_t mo = __ballot(fl_old != 0u);
            const uint64_t am = __ballot(accepted);
            const int64_t w0 = (base + 64 * (threadIdx.x >> 6)) / 32;
            if (lane == 0) {
                if (w0 < fw) acc.fbits_prev[b * fw + w0] = static_cast<uint32_t>(mo);
                if (w0 + 1 < fw) acc.fbits_prev[b * fw + w0 + 1] = static_cast<uint32_t>(mo >> 32);
            }
            uint32_t basec = 0;
            if (lane == 0 && am != 0) basec = atomicAdd(acc.cnt, static_cast<uint32_t>(__popcll(am)));
            basec = static_cast<uint32_t>(__shfl(static_cast<int>(basec), 0));
            if (accepted)
                acc.list[basec + static_cast<uint32_t>(__popcll(am & ((uint64_t(1) << lane) - 1)))] =
                    static_cast<int32_t>(static_cast<int64_t>(b) * np + i);
        }
        __syncthreads();  // sq is refilled for the next 256 genomes
    }
    if (mode == 1 || mode == 2) {
        __syncthreads();
        block_top3<T, 1024>(fb, np, Lb);
    }
}

// ---------------------------------------------------------------- evolution

struct BatchPop {
    const float *x0, *x1;
    float *out0, *out1;
    const uint32_t *flags;  // instance-major, np per instance
    int64_t np;
};

__device__ __forceinline__ PopView view_of(const BatchPop &bp, const InstDesc &id, int b)
{
    return PopView{bp.x0 + id.xofs, bp.x1 + id.xofs, bp.flags + static_cast<int64_t>(b) * bp.np,
                   bp.out0 + id.xofs, bp.out1 + id.xofs, bp.np, id.n, id.ldx};
}

// initialisation: grid x = individual, y = tile (instance, 1024-gene chunk)
__global__ __launch_bounds__(256) void batch_init_kernel(int64_t np, const InstDesc *__restrict__ inst,
                                                         const Tile *__restrict__ tiles, uint32_t k0, uint32_t k1,
                                                         uint32_t inst0, float *__restrict__ x,
                                                         uint32_t *__restrict__ bits, int64_t ld)
{
    const Tile tl = tiles[blockIdx.y];
    const InstDesc id = inst[tl.inst];
    const int64_t i = blockIdx.x;
    const int64_t q = static_cast<int64_t>(tl.chunk) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < id.n;
    uint32_t nib = 0;
    if (valid) {
        const U4 r = philox10(static_cast<uint32_t>(q), static_cast<uint32_t>(i), 0u,
                              ((inst0 + static_cast<uint32_t>(tl.inst)) << 8) | kTagInit, k0, k1);
        const float4 v = make_float4(sym24(r.x), sym24(r.y), sym24(r.z), sym24(r.w));
        store_quad(x + id.xofs + i * id.ldx, j0, id.n, v);
        nib = quad_nibble(v, j0, id.n);
    }
    store_word(nib, q, id.n, bits + id.wofs * ld, ld, i);
}

// DE: tiles (instance, chunk of CW = 256 / IPW genes) dealt round-robin to
// the XCDs (workgroup id mod 8); a workgroup makes R passes over groups of
// 4 IPW consecutive individuals of one tile, loading the rows of pass r + 1
// before storing the trials of pass r. Each row's buffer flag comes from
// the instance's packed flags (np / 32 words, np <= 4096), copied to LDS
// first, instead of a dependent global load after the draw.
template <int IPW, int R>
__global__ __launch_bounds__(256) void batch_de_kernel(BatchPop bp, const InstDesc *__restrict__ inst,
                                                       const Tile *__restrict__ tiles, int ntiles, int groups,
                                                       const int4 *__restrict__ draws, float F, uint32_t cr_max,
                                                       uint32_t k0, uint32_t k1, const uint32_t *__restrict__ gen,
                                                       uint32_t inst0, uint32_t *__restrict__ bits, int64_t ld,
                                                       const uint32_t *__restrict__ fbits, int store_genes,
                                                       uint32_t *__restrict__ reset_cnt)
{
    constexpr int LPI = 64 / IPW;
    if (reset_cnt != nullptr && blockIdx.x == 0 && threadIdx.x == 0) reset_cnt[0] = 0u;
    constexpr int CW = 4 * LPI;
    constexpr int WPC = CW / 32;
    constexpr int IPG = 4 * IPW;
    constexpr int IPB = R * IPG;
    static_assert(IPB * WPC <= 256, "one bit word per thread at the end");
    const uint32_t blk = blockIdx.x;
    const int xcd = static_cast<int>(blk & 7u);
    const int k = static_cast<int>(blk >> 3);
    const int gi = k % groups;
    const int ti = xcd + 8 * (k / groups);
    if (ti >= ntiles) return;
    const Tile tl = tiles[ti];
    const InstDesc id = inst[tl.inst];
    const PopView pv = view_of(bp, id, tl.inst);
    const int t = threadIdx.x;
    const int local = t / LPI, li = t % LPI;
    const int64_t np = bp.np, D = id.n;
    const int64_t i0 = static_cast<int64_t>(gi) * IPB + local;
    const int64_t j0 = static_cast<int64_t>(tl.chunk) * CW + 4 * li;
    const uint32_t g = gen[0];
    const uint32_t instb = inst0 + static_cast<uint32_t>(tl.inst);
    __shared__ uint32_t wsh[IPB][WPC];
    __shared__ uint32_t sfb[128];
    // per individual of the workgroup: its target row, three donor rows and
    // output row, and jrand, worked out once by one lane (lane t < IPB
    // takes individual gi IPB + t) instead of by every lane of every pass
    __shared__ const float *srow[IPB][4];
    __shared__ float *sout[IPB];
    __shared__ int sjr[IPB];
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r) act[r] = i0 + r * IPG < np && j0 < D;
    const int64_t ip = static_cast<int64_t>(gi) * IPB + t;
    int4 d4 = make_int4(0, 0, 0, 0);
    if (t < IPB) d4 = draws[static_cast<int64_t>(tl.inst) * np + (ip < np ? ip : np - 1)];
    const int fw = static_cast<int>((np + 31) / 32);
    if (t < fw) sfb[t] = fbits[static_cast<int64_t>(tl.inst) * fw + t];
    __syncthreads();
    auto second = [&](int64_t r) -> bool { return ((sfb[r >> 5] >> (r & 31)) & 1u) != 0u; };
    auto src = [&](int64_t r) -> const float * { return (second(r) ? pv.x1 : pv.x0) + r * pv.ldx; };
    if (t < IPB && ip < np) {
        srow[t][0] = src(ip);
        srow[t][1] = src(d4.x);
        srow[t][2] = src(d4.y);
        srow[t][3] = src(d4.z);
        sout[t] = (second(ip) ? pv.out0 : pv.out1) + ip * pv.ldx;
        sjr[t] = d4.w;
    }
    __syncthreads();
    // two row buffers used alternately by the unrolled passes (no register
    // copy between passes)
    float4 buf0[4], buf1[4];
    auto load = [&](int r, float4 *v) {
        if (act[r]) {
            const float *const *rw = srow[r * IPG + local];
#pragma unroll
            for (int m = 0; m < 4; ++m) v[m] = *reinterpret_cast<const float4 *>(rw[m] + j0);
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
            const float4 uv = de_quad(cur[0], cur[1], cur[2], cur[3], j0, sjr[r * IPG + local], static_cast<uint32_t>(i),
                                      g, instb, k0, k1, F, cr_max);
            if (store_genes) store_quad_nt(sout[r * IPG + local], j0, D, uv);
            nib = quad_nibble(uv, j0, D);
        }
        const uint32_t w = or8_into_last(nib << (4 * (t & 7)));
        if ((t & 7) == 7) wsh[r * IPG + local][li >> 3] = w;
    }
    __syncthreads();
    if (t < IPB * WPC) {
        const int wd = t / IPB, ii = t % IPB;
        const int64_t row = static_cast<int64_t>(gi) * IPB + ii;
        const int64_t wg = static_cast<int64_t>(tl.chunk) * WPC + wd;
        if (row < np && wg * 32 < D) bits[(id.wofs + wg) * ld + row] = wsh[ii][wd];
    }
}

// The accepted trials of a batched run whose DE step stored only bits:
// entry e = b np + i of list[0 .. cnt) is slot i of instance b; its trial
// genes are computed again exactly as batch_de_kernel computed them, from
// the rows before the selection (fb_old: the instance's packed flags before
// it), and written to the buffer the selection made current. Work items
// (chunk of 256 genes, entry), chunk c on XCD c mod 8, walked chunk by
// chunk; chunks past an instance's genes are skipped.
__global__ __launch_bounds__(256) void batch_materialize_kernel(BatchPop bp, const InstDesc *__restrict__ inst,
                                                                const int4 *__restrict__ draws,
                                                                const uint32_t *__restrict__ fb_old, float F,
                                                                uint32_t cr_max, uint32_t k0, uint32_t k1,
                                                                const uint32_t *__restrict__ gen, uint32_t inst0,
                                                                const int32_t *__restrict__ list,
                                                                const uint32_t *__restrict__ cnt, int64_t n_inst,
                                                                int64_t max_chunks)
{
    const int64_t np = bp.np;
    const int64_t n_acc = min(static_cast<int64_t>(cnt[0]), n_inst * np);
    const uint32_t g = gen[0];
    const int xcd = static_cast<int>(blockIdx.x & 7u);
    const int64_t wg_per_xcd = gridDim.x / 8;  // the grid is a multiple of 8
    const int64_t my_chunks = max_chunks > xcd ? (max_chunks - xcd + 7) / 8 : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t fw = (np + 31) / 32;
    for (int64_t it = static_cast<int64_t>(blockIdx.x >> 3) * 4 + wave; it < n_acc * my_chunks;
         it += wg_per_xcd * 4) {
        const int64_t c = xcd + 8 * (it / n_acc);
        const int64_t e = list[it % n_acc];
        if (e < 0 || e >= n_inst * np) continue;
        const int b = static_cast<int>(e / np);
        const int64_t i = e % np;
        const InstDesc id = inst[b];
        const int64_t j0 = c * 256 + 4 * lane;
        if (j0 >= id.n) continue;
        const uint32_t *fo = fb_old + b * fw;
        auto old = [&](int64_t r) -> bool { return ((fo[r >> 5] >> (r & 31)) & 1u) != 0u; };
        auto src = [&](int64_t r) -> const float * { return (old(r) ? bp.x1 : bp.x0) + id.xofs + r * id.ldx; };
        const int4 dr = draws[e];
        const float4 xv = *reinterpret_cast<const float4 *>(src(i) + j0);
        const float4 a = *reinterpret_cast<const float4 *>(src(dr.x) + j0);
        const float4 bq = *reinterpret_cast<const float4 *>(src(dr.y) + j0);
        const float4 cq = *reinterpret_cast<const float4 *>(src(dr.z) + j0);
        const float4 uv = de_quad(xv, a, bq, cq, j0, dr.w, static_cast<uint32_t>(i), g,
                                  inst0 + static_cast<uint32_t>(b), k0, k1, F, cr_max);
        store_quad_nt((old(i) ? bp.out0 : bp.out1) + id.xofs + i * id.ldx, j0, id.n, uv);
    }
}

// GWO: grid x = 8 ceil(np / 8) (individuals in contiguous ranges per XCD,
// as in the single-design kernel), y = tile (instance, 1024-gene chunk)
template <int VARIANT>
__global__ __launch_bounds__(256) void batch_gwo_kernel(BatchPop bp, const InstDesc *__restrict__ inst,
                                                        const Tile *__restrict__ tiles,
                                                        const int32_t *__restrict__ leaders,
                                                        const float *__restrict__ a_tab, uint32_t k0, uint32_t k1,
                                                        const uint32_t *__restrict__ gen, uint32_t inst0,
                                                        uint32_t *__restrict__ bits, int64_t ld, int64_t per_xcd)
{
    const int64_t np = bp.np;
    const int64_t i = static_cast<int64_t>(blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
    if (i >= np) return;
    const Tile tl = tiles[blockIdx.y];
    const InstDesc id = inst[tl.inst];
    const int64_t D = id.n;
    const int64_t L0 = leaders[3 * tl.inst], L1 = leaders[3 * tl.inst + 1], L2 = leaders[3 * tl.inst + 2];
    if (i == L0 || i == L1 || i == L2) return;
    if (L0 < 0 || L0 >= np || L1 < 0 || L1 >= np || L2 < 0 || L2 >= np) return;
    const PopView pv = view_of(bp, id, tl.inst);
    const uint32_t g = gen[0];
    const float a = a_tab[g];
    const float two_a = 2.0f * a;
    const int64_t q = static_cast<int64_t>(tl.chunk) * 256 + threadIdx.x;
    const int64_t j0 = 4 * q;
    const bool valid = j0 < D;
    uint32_t nib = 0;
    if (valid) {
        const float4 xv = *reinterpret_cast<const float4 *>(row_of(pv, i) + j0);
        const float4 X0 = *reinterpret_cast<const float4 *>(row_of(pv, L0) + j0);
        const float4 X1 = *reinterpret_cast<const float4 *>(row_of(pv, L1) + j0);
        const float4 X2 = *reinterpret_cast<const float4 *>(row_of(pv, L2) + j0);
        const float4 yv = gwo_quad<VARIANT>(xv, X0, X1, X2, static_cast<uint32_t>(q), static_cast<uint32_t>(i), g,
                                            inst0 + static_cast<uint32_t>(tl.inst), k0, k1, a, two_a);
        store_quad_nt(out_row_of(pv, i), j0, D, yv);
        nib = quad_nibble(yv, j0, D);
    }
    store_word(nib, q, id.n, bits + id.wofs * ld, ld, i);
}

// rows of instance b's current population -> dense out[np][ldo]
__global__ __launch_bounds__(256) void batch_gather_kernel(BatchPop bp, const InstDesc *__restrict__ inst, int b,
                                                           float *__restrict__ out, int64_t ldo)
{
    const InstDesc id = inst[b];
    const PopView pv = view_of(bp, id, b);
    const int64_t r = blockIdx.y;
    const float *x = row_of(pv, r);
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; j < id.n; j += 256 * gridDim.x)
        out[r * ldo + j] = x[j];
}

// ---------------------------------------------------------------- plans

struct BatchFitPlan {
    int waves = 16;  // per-domain kernel: waves per workgroup; table kernel: 4 segment waves
    int wpw = 8;
    int gw = 0;      // table kernel: genome groups of 64 per workgroup (0 = per-domain kernel)
    std::vector<FitSeg> segs;
    std::vector<int> slot_ofs;  // n_inst + 1
};

static BatchFitPlan make_fit_plan(const std::vector<InstDesc> &h, int waves, int wpw)
{
    BatchFitPlan p;
    p.waves = waves;
    p.wpw = wpw;
    p.slot_ofs.push_back(0);
    int slot = 0;
    const int per_wg = waves * wpw;
    for (size_t b = 0; b < h.size(); ++b) {
        for (int w0 = 0; w0 < h[b].words; w0 += per_wg) p.segs.push_back(FitSeg{static_cast<int>(b), w0, slot++, 0});
        p.slot_ofs.push_back(slot);
    }
    return p;
}

// the table plan: tiles of 4 wpw words, gw genome groups per workgroup
static BatchFitPlan make_tab_plan(const std::vector<InstDesc> &h, int gw, int wpw)
{
    BatchFitPlan p = make_fit_plan(h, 4, wpw);
    p.gw = gw;
    return p;
}

static void default_tab_shape(int64_t np, bool f32, int *gw, int *wpw)
{
    *gw = np >= 256 ? 4 : (np >= 128 ? 2 : 1);
    *wpw = f32 ? 4 : 2;
}

static void default_fit_shape(const std::vector<InstDesc> &h, int64_t np, int *waves, int *wpw)
{
    int64_t words = 0;
    for (const auto &d : h) words += d.words;
    const int64_t groups = (np + 63) / 64;
    // aim for ~8 waves per SIMD (8192 waves) over 256 CUs x 4 SIMDs
    int64_t w = (groups * words + 8191) / 8192;
    if (w < 1) w = 1;
    *waves = 16;
    *wpw = static_cast<int>(w);
}

}  // namespace qpm

using namespace qpm;

// ---------------------------------------------------------------- the batch design

struct qpm_batch_s {
    int32_t n_inst = 0;
    int64_t total_words = 0;
    int64_t total_genes_stride = 0;  // sum over instances of ldx
    std::vector<InstDesc> host;
    InstDesc *dev = nullptr;
    double4 *ph64 = nullptr;
    float4 *ph32 = nullptr;
    double2 *c64 = nullptr;
    double *Cdev = nullptr;
    double2 *tab64 = nullptr;  // sign-pattern tables, [8 total_words][3][16]
    int2 *tabq = nullptr;      // their fixed-point form at the word scales
    double *wsc = nullptr;     // [total_words] word scales (word_scales per instance)
};

static void free_batch(qpm_batch_s *b)
{
    if (!b) return;
    (void)hipFree(b->dev);
    (void)hipFree(b->ph64);
    (void)hipFree(b->ph32);
    (void)hipFree(b->c64);
    (void)hipFree(b->Cdev);
    (void)hipFree(b->tab64);
    (void)hipFree(b->tabq);
    (void)hipFree(b->wsc);
    delete b;
}

QPM_API qpm_status qpm_precompute_phases_batched(const double *z, const int64_t *offsets, int32_t n_inst,
                                                 const double *dk1, const double *dk2, qpm_stream sv,
                                                 qpm_batch *out)
{
    clear_error();
    QPM_REQUIRE(z && offsets && dk1 && dk2 && out, QPM_EINVAL, "z, offsets, dk1, dk2 and out must not be NULL");
    QPM_REQUIRE(n_inst >= 1 && n_inst <= 65535, QPM_EINVAL, "n_inst must be in [1, 65535] (got %d)", (int)n_inst);
    QPM_REQUIRE(offsets[0] == 0, QPM_EINVAL, "offsets[0] must be 0");
    int64_t words = 0, genes = 0;
    for (int32_t b = 0; b < n_inst; ++b) {
        const int64_t n = offsets[b + 1] - offsets[b] - 1;
        QPM_REQUIRE(n >= 1 && n <= (int64_t(1) << 27), QPM_EINVAL,
                    "instance %d: needs 2 .. 2^27 + 1 boundaries (offsets must increase by >= 2)", (int)b);
        QPM_REQUIRE(std::isfinite(dk1[b]) && std::isfinite(dk2[b]), QPM_EINVAL, "instance %d: dk not finite",
                    (int)b);
        for (int64_t k = offsets[b]; k < offsets[b + 1]; ++k)
            QPM_REQUIRE(std::isfinite(z[k]), QPM_EINVAL, "instance %d: z[%lld] not finite", (int)b, (long long)k);
        for (int64_t k = offsets[b]; k + 1 < offsets[b + 1]; ++k)
            QPM_REQUIRE(z[k + 1] > z[k], QPM_EINVAL, "instance %d: z must be strictly increasing", (int)b);
        QPM_REQUIRE(z[offsets[b + 1] - 1] - z[offsets[b]] <= 1e100, QPM_EINVAL,
                    "instance %d: the crystal length must be at most 1e100", (int)b);
        words += words_for(n);
        genes += ((n + 63) / 64) * 64;
    }
    QPM_REQUIRE(words <= (int64_t(1) << 28), QPM_ERANGE, "batch too large (%lld words)", (long long)words);
    qpm_status st = check_device();
    if (st != QPM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(sv);
    auto *bt = new qpm_batch_s();
    bt->n_inst = n_inst;
    bt->total_words = words;
    bt->total_genes_stride = genes;
    int64_t wofs = 0, xofs = 0;
    for (int32_t b = 0; b < n_inst; ++b) {
        InstDesc d{};
        d.n = offsets[b + 1] - offsets[b] - 1;
        d.words = words_for(d.n);
        d.wofs = wofs;
        d.ldx = ((d.n + 63) / 64) * 64;
        d.xofs = xofs;  // in units of rows x ldx: scaled by np at run creation
        wofs += d.words;
        xofs += d.ldx;
        bt->host.push_back(d);
    }
    double *zdev = nullptr;
    hipError_t e = hipMalloc(&bt->ph64, sizeof(double4) * 32 * words);
    if (e == hipSuccess) e = hipMalloc(&bt->ph32, sizeof(float4) * 32 * words);
    if (e == hipSuccess) e = hipMalloc(&bt->c64, sizeof(double2) * 32 * words);
    if (e == hipSuccess) e = hipMalloc(&bt->Cdev, sizeof(double) * 2 * n_inst);
    if (e == hipSuccess) e = hipMalloc(&bt->tab64, sizeof(double2) * 48 * 8 * words);
    if (e == hipSuccess) e = hipMalloc(&bt->tabq, sizeof(int2) * 48 * 8 * words);
    if (e == hipSuccess) e = hipMalloc(&bt->wsc, sizeof(double) * words);
    std::vector<double> wsc(words);
    for (int32_t b = 0; b < n_inst; ++b) word_scales(z + offsets[b], bt->host[b].n, wsc.data() + bt->host[b].wofs);
    if (e == hipSuccess) e = hipMemcpyAsync(bt->wsc, wsc.data(), sizeof(double) * words, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMalloc(&bt->dev, sizeof(InstDesc) * n_inst);
    if (e == hipSuccess) e = hipMalloc(&zdev, sizeof(double) * offsets[n_inst]);
    if (e == hipSuccess) e = hipMemcpyAsync(zdev, z, sizeof(double) * offsets[n_inst], hipMemcpyHostToDevice, s);
    for (int32_t b = 0; b < n_inst && e == hipSuccess; ++b) {
        const InstDesc &d = bt->host[b];
        if (launch_phases(zdev + offsets[b], d.n, dk1[b], dk2[b], bt->ph64 + 32 * d.wofs, bt->ph32 + 32 * d.wofs,
                          bt->c64 + 32 * d.wofs, bt->Cdev + 2 * b, s) != QPM_OK)
            e = hipErrorLaunchFailure;
    }
    if (e == hipSuccess && launch_pattern_tables(bt->ph64, words, bt->wsc, bt->tab64, bt->tabq, s) != QPM_OK)
        e = hipErrorLaunchFailure;
    std::vector<double> C(2 * n_inst);
    if (e == hipSuccess) e = hipMemcpyAsync(C.data(), bt->Cdev, sizeof(double) * 2 * n_inst, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(zdev);
    if (e == hipSuccess) {
        for (int32_t b = 0; b < n_inst; ++b) {
            bt->host[b].C[0] = C[2 * b];
            bt->host[b].C[1] = C[2 * b + 1];
        }
        e = hipMemcpy(bt->dev, bt->host.data(), sizeof(InstDesc) * n_inst, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        set_error("batched phase precompute failed: %s", hipGetErrorString(e));
        free_batch(bt);
        return e == hipErrorOutOfMemory ? QPM_ENOMEM : QPM_EHIP;
    }
    *out = bt;
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_free(qpm_batch b)
{
    clear_error();
    if (!b) return QPM_OK;
    (void)hipDeviceSynchronize();
    free_batch(b);
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_info(qpm_batch b, int32_t *n_inst, int64_t *n_domains, double *C)
{
    clear_error();
    QPM_REQUIRE(b != nullptr, QPM_EINVAL, "batch is NULL");
    if (n_inst) *n_inst = b->n_inst;
    for (int32_t i = 0; i < b->n_inst; ++i) {
        if (n_domains) n_domains[i] = b->host[i].n;
        if (C) {
            C[2 * i] = b->host[i].C[0];
            C[2 * i + 1] = b->host[i].C[1];
        }
    }
    return QPM_OK;
}

// ---------------------------------------------------------------- batched fitness

static qpm_status launch_batch_fit(const qpm_batch_s &bt, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                   const BatchFitPlan &pl, const FitSeg *segs_dev, double *part, hipStream_t s,
                                   uint32_t *advance = nullptr)
{
    if (pl.gw > 0) {
        const dim3 grid(static_cast<unsigned>((np + 64 * pl.gw - 1) / (64 * pl.gw)),
                        static_cast<unsigned>(pl.segs.size()));
        const size_t lds = table_lds_bytes(4 * pl.wpw, p == QPM_PREC_F32, pl.gw, pl.wpw);
#define QPM_BT_CASE(G)                                                                                             \
    case G:                                                                                                        \
        if (p == QPM_PREC_F32)                                                                                     \
            batch_fit_tab_kernel<true, G><<<grid, G * 256, lds, s>>>(bits, ld, bt.tab64, bt.tabq, bt.wsc, pl.wpw, np,   \
                                                                     bt.dev,                                      \
                                                                    segs_dev, part, advance);                      \
        else                                                                                                       \
            batch_fit_tab_kernel<false, G><<<grid, G * 256, lds, s>>>(bits, ld, bt.tab64, bt.tabq, bt.wsc, pl.wpw, np, \
                                                                     bt.dev, segs_dev, part, advance);             \
        break;
        switch (pl.gw) {
            QPM_BT_CASE(1)
            QPM_BT_CASE(2)
            QPM_BT_CASE(4)
        default: QPM_REQUIRE(false, QPM_EINVAL, "unsupported genome groups per workgroup %d", pl.gw);
        }
#undef QPM_BT_CASE
        QPM_TRY_HIP(hipGetLastError());
        return QPM_OK;
    }
    const dim3 grid(static_cast<unsigned>((np + 63) / 64), static_cast<unsigned>(pl.segs.size()));
#define QPM_BF_CASE(NW)                                                                                           \
    case NW:                                                                                                      \
        if (p == QPM_PREC_F32)                                                                                    \
            batch_fit_kernel<true, NW><<<grid, NW * 64, 0, s>>>(bits, ld, bt.ph64, bt.ph32, pl.wpw, bt.dev,       \
                                                                segs_dev, part, advance);                         \
        else                                                                                                      \
            batch_fit_kernel<false, NW><<<grid, NW * 64, 0, s>>>(bits, ld, bt.ph64, bt.ph32, pl.wpw, bt.dev,      \
                                                                 segs_dev, part, advance);                        \
        break;
    switch (pl.waves) {
        QPM_BF_CASE(4)
        QPM_BF_CASE(8)
        QPM_BF_CASE(16)
    default: QPM_REQUIRE(false, QPM_EINVAL, "unsupported waves per group %d", pl.waves);
    }
#undef QPM_BF_CASE
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

// device copies of a fitness plan's tables
struct FitPlanDev {
    FitSeg *segs = nullptr;
    int *slot_ofs = nullptr;
    double *part = nullptr;
};

static qpm_status upload_fit_plan(const BatchFitPlan &pl, int64_t ld, hipStream_t s, FitPlanDev *out)
{
    FitPlanDev d;
    hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&d.segs), sizeof(FitSeg) * pl.segs.size(), s);
    if (e == hipSuccess)
        e = hipMallocAsync(reinterpret_cast<void **>(&d.slot_ofs), sizeof(int) * pl.slot_ofs.size(), s);
    if (e == hipSuccess)
        e = hipMallocAsync(reinterpret_cast<void **>(&d.part), sizeof(double) * 6 * pl.segs.size() * ld, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d.segs, pl.segs.data(), sizeof(FitSeg) * pl.segs.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d.slot_ofs, pl.slot_ofs.data(), sizeof(int) * pl.slot_ofs.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors must outlive the copies
    if (e != hipSuccess) {
        (void)hipFreeAsync(d.segs, s);
        (void)hipFreeAsync(d.slot_ofs, s);
        (void)hipFreeAsync(d.part, s);
        set_error("fitness plan upload failed: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? QPM_ENOMEM : QPM_EHIP;
    }
    *out = d;
    return QPM_OK;
}

static void free_fit_plan(FitPlanDev &d, hipStream_t s)
{
    (void)hipFreeAsync(d.segs, s);
    (void)hipFreeAsync(d.slot_ofs, s);
    (void)hipFreeAsync(d.part, s);
    d = FitPlanDev{};
}

static qpm_status launch_batch_finish(int mode, const qpm_batch_s &bt, qpm_prec p, const FitPlanDev &fp, int64_t ld,
                                      int64_t np, void *f, uint32_t *flags, int32_t *leaders, int4 *draws,
                                      uint32_t *gen, uint64_t seed, uint32_t inst0, hipStream_t s,
                                      uint32_t *fbits = nullptr, AcceptOut acc = AcceptOut{})
{
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    if (p == QPM_PREC_F64)
        batch_finish_kernel<double><<<bt.n_inst, 1024, 0, s>>>(mode, fp.part, fp.slot_ofs, ld, np, bt.dev,
                                                             static_cast<double *>(f), flags, leaders, draws, gen, k0,
                                                             k1, inst0, fbits, acc);
    else
        batch_finish_kernel<float><<<bt.n_inst, 1024, 0, s>>>(mode, fp.part, fp.slot_ofs, ld, np, bt.dev,
                                                            static_cast<float *>(f), flags, leaders, draws, gen, k0,
                                                            k1, inst0, fbits, acc);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

static qpm_status batch_eval_plan(qpm_batch b, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                  void *fitness, const BatchFitPlan &pl, hipStream_t s);

QPM_API qpm_status qpm_batch_eval_fitness(qpm_batch b, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                          void *fitness, int32_t waves_per_group, int32_t words_per_wave,
                                          qpm_stream sv)
{
    clear_error();
    QPM_REQUIRE(b && bits && fitness, QPM_EINVAL, "batch, bits and fitness must not be NULL");
    QPM_REQUIRE(p == QPM_PREC_F32 || p == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", (int)p);
    QPM_REQUIRE(np >= 1 && np <= (int64_t(1) << 24), QPM_EINVAL, "np out of range (%lld)", (long long)np);
    QPM_REQUIRE(ld >= np && ld % 64 == 0, QPM_EINVAL, "ld (%lld) must be >= np and a multiple of 64", (long long)ld);
    QPM_REQUIRE(waves_per_group == 0 || waves_per_group == 4 || waves_per_group == 8 || waves_per_group == 16,
                QPM_EINVAL, "waves_per_group must be 0 (default), 4, 8 or 16");
    QPM_REQUIRE(words_per_wave >= 0, QPM_EINVAL, "words_per_wave must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(sv);
    BatchFitPlan pl;
    if (waves_per_group == 0 && words_per_wave == 0) {
        int gw, wpw;
        default_tab_shape(np, p == QPM_PREC_F32, &gw, &wpw);
        pl = make_tab_plan(b->host, gw, wpw);
    } else {
        int waves, wpw;
        default_fit_shape(b->host, np, &waves, &wpw);
        if (waves_per_group) waves = waves_per_group;
        if (words_per_wave) wpw = words_per_wave;
        pl = make_fit_plan(b->host, waves, wpw);
    }
    return batch_eval_plan(b, p, bits, np, ld, fitness, pl, s);
}

QPM_API qpm_status qpm_batch_eval_fitness_table(qpm_batch b, qpm_prec p, const uint32_t *bits, int64_t np,
                                                int64_t ld, void *fitness, int32_t groups, int32_t wpw,
                                                qpm_stream sv)
{
    clear_error();
    QPM_REQUIRE(b && bits && fitness, QPM_EINVAL, "batch, bits and fitness must not be NULL");
    QPM_REQUIRE(p == QPM_PREC_F32 || p == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", (int)p);
    QPM_REQUIRE(np >= 1 && np <= (int64_t(1) << 24), QPM_EINVAL, "np out of range (%lld)", (long long)np);
    QPM_REQUIRE(ld >= np && ld % 64 == 0, QPM_EINVAL, "ld (%lld) must be >= np and a multiple of 64", (long long)ld);
    QPM_REQUIRE(groups == 1 || groups == 2 || groups == 4, QPM_EINVAL,
                "groups_per_workgroup must be 1, 2 or 4 (got %d)", (int)groups);
    QPM_REQUIRE(wpw >= 1 && wpw <= table_max_wpw(p == QPM_PREC_F32), QPM_EINVAL,
                "words_per_wave must be in [1, %d] (got %d)", table_max_wpw(p == QPM_PREC_F32), (int)wpw);
    return batch_eval_plan(b, p, bits, np, ld, fitness, make_tab_plan(b->host, groups, wpw),
                           static_cast<hipStream_t>(sv));
}

static qpm_status batch_eval_plan(qpm_batch b, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                  void *fitness, const BatchFitPlan &pl, hipStream_t s)
{
    QPM_REQUIRE(pl.segs.size() <= 65535, QPM_ERANGE, "too many fitness segments (%zu)", pl.segs.size());
    FitPlanDev fp;
    qpm_status st = upload_fit_plan(pl, ld, s, &fp);
    if (st != QPM_OK) return st;
    st = launch_batch_fit(*b, p, bits, np, ld, pl, fp.segs, fp.part, s);
    if (st == QPM_OK)
        st = launch_batch_finish(0, *b, p, fp, ld, np, fitness, nullptr, nullptr, nullptr, nullptr, 0, 0, s);
    free_fit_plan(fp, s);
    return st;
}

// ---------------------------------------------------------------- the batched run

struct qpm_batch_run_s {
    const qpm_batch_s *bt = nullptr;
    qpm_run_config cfg{};
    hipStream_t st = nullptr;
    int64_t ld = 0;
    float *buf[2] = {nullptr, nullptr};
    uint32_t *flags = nullptr;
    uint32_t *fbits = nullptr;  // flags packed one bit per individual, ceil(np / 32) words per instance
    void *f_cur = nullptr;
    uint32_t *bits = nullptr;
    int32_t *leaders = nullptr;
    int4 *draws = nullptr;
    uint32_t *gen = nullptr;
    float *a_tab = nullptr;
    InstDesc *inst = nullptr;  // instance table with xofs scaled by np
    Tile *gtiles = nullptr;    // (instance, 1024-gene chunk)
    int n_gtiles = 0;
    Tile *dtiles[3] = {nullptr, nullptr, nullptr};  // (instance, DE chunk) for 1, 2, 4 individuals per wave
    int n_dtiles[3] = {0, 0, 0};
    int de_ipw = 1, de_passes = 1;
    // accepted-only trials (as in a single-design run): the DE step writes
    // bits only, the finish lists accepted slots, a kernel recomputes them
    bool lazy = false;
    int32_t *acc_list = nullptr;   // n_inst np entries
    uint32_t *acc_cnt = nullptr;
    uint32_t *fbits_prev = nullptr;
    int64_t max_chunks = 0;        // 256-gene chunks of the largest instance
    BatchFitPlan fplan;
    FitPlanDev fdev;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t done = 0;
    bool timing = false;
    hipEvent_t ev[QPM_K_COUNT + 1] = {};
    double ms[QPM_K_COUNT] = {};
    int64_t timed = 0;
    double tune_us = 0.0;

    bool f64() const { return cfg.prec == QPM_PREC_F64; }
    BatchPop pop() const { return BatchPop{buf[0], buf[1], buf[0], buf[1], flags, cfg.np}; }
};

static void release_batch_run(qpm_batch_run_s *r)
{
    if (!r) return;
    if (r->st) (void)hipStreamSynchronize(r->st);
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    (void)hipFree(r->buf[0]);
    (void)hipFree(r->buf[1]);
    (void)hipFree(r->fbits);
    (void)hipFree(r->flags);
    (void)hipFree(r->f_cur);
    (void)hipFree(r->bits);
    (void)hipFree(r->leaders);
    (void)hipFree(r->draws);
    (void)hipFree(r->acc_list);
    (void)hipFree(r->acc_cnt);
    (void)hipFree(r->fbits_prev);
    (void)hipFree(r->gen);
    (void)hipFree(r->a_tab);
    (void)hipFree(r->inst);
    (void)hipFree(r->gtiles);
    for (auto *t : r->dtiles) (void)hipFree(t);
    if (r->st && r->fdev.segs) {
        free_fit_plan(r->fdev, r->st);
        (void)hipStreamSynchronize(r->st);
    }
    for (auto &e : r->ev)
        if (e) (void)hipEventDestroy(e);
    if (r->st) (void)hipStreamDestroy(r->st);
    delete r;
}

static qpm_status launch_batch_de(qpm_batch_run_s *r, int ipw, int passes)
{
    const qpm_run_config &c = r->cfg;
    const uint32_t k0 = static_cast<uint32_t>(c.seed), k1 = static_cast<uint32_t>(c.seed >> 32);
    const int64_t groups = (c.np + 4 * ipw * passes - 1) / (4 * ipw * passes);
    const Tile *tiles = ipw == 1 ? r->dtiles[0] : (ipw == 2 ? r->dtiles[1] : r->dtiles[2]);
    const int ntiles = ipw == 1 ? r->n_dtiles[0] : (ipw == 2 ? r->n_dtiles[1] : r->n_dtiles[2]);
    const int64_t blocks = 8 * ((ntiles + 7) / 8) * groups;
    QPM_REQUIRE(blocks < (int64_t(1) << 31), QPM_ERANGE, "batch too large for one DE launch");
    const unsigned nb = static_cast<unsigned>(blocks);
    const BatchPop bp = r->pop();
    const int gr = static_cast<int>(groups);
#define QPM_BDE(I, P)                                                                                       \
    batch_de_kernel<I, P><<<nb, 256, 0, r->st>>>(bp, r->inst, tiles, ntiles, gr, r->draws, c.F,             \
                                                 cr_threshold(c.CR), k0, k1, r->gen, c.inst, r->bits, r->ld, \
                                                 r->fbits, r->lazy ? 0 : 1, r->lazy ? r->acc_cnt : nullptr)
    if (ipw == 1) {
        if (passes == 1) { QPM_BDE(1, 1); } else if (passes == 2) { QPM_BDE(1, 2); } else { QPM_BDE(1, 4); }
    } else if (ipw == 2) {
        if (passes == 1) { QPM_BDE(2, 1); } else if (passes == 2) { QPM_BDE(2, 2); } else { QPM_BDE(2, 4); }
    } else {
        if (passes == 1) { QPM_BDE(4, 1); } else if (passes == 2) { QPM_BDE(4, 2); } else { QPM_BDE(4, 4); }
    }
#undef QPM_BDE
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

static qpm_status launch_batch_gwo(qpm_batch_run_s *r)
{
    const qpm_run_config &c = r->cfg;
    const int64_t per_xcd = (c.np + 7) / 8;
    const dim3 grid(static_cast<unsigned>(8 * per_xcd), static_cast<unsigned>(r->n_gtiles));
    if (c.gwo_variant == 1)
        batch_gwo_kernel<1><<<grid, 256, 0, r->st>>>(r->pop(), r->inst, r->gtiles, r->leaders, r->a_tab,
                                                    static_cast<uint32_t>(c.seed), static_cast<uint32_t>(c.seed >> 32),
                                                    r->gen, c.inst, r->bits, r->ld, per_xcd);
    else
        batch_gwo_kernel<0><<<grid, 256, 0, r->st>>>(r->pop(), r->inst, r->gtiles, r->leaders, r->a_tab,
                                                    static_cast<uint32_t>(c.seed), static_cast<uint32_t>(c.seed >> 32),
                                                    r->gen, c.inst, r->bits, r->ld, per_xcd);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

static qpm_status batch_generation(qpm_batch_run_s *r, hipEvent_t *ev = nullptr)
{
    const qpm_run_config &c = r->cfg;
    const qpm_prec p = static_cast<qpm_prec>(c.prec);
    auto mark = [&](int k) -> qpm_status {
        if (ev) QPM_TRY_HIP(hipEventRecord(ev[k], r->st));
        return QPM_OK;
    };
    qpm_status st;
#define QPM_STEP(k, call)                    \
    if ((st = mark(k)) != QPM_OK) return st; \
    if ((st = (call)) != QPM_OK) return st;
    QPM_STEP(QPM_K_DE, launch_batch_de(r, r->de_ipw, r->de_passes))
    QPM_STEP(QPM_K_FIT_DE, launch_batch_fit(*r->bt, p, r->bits, c.np, r->ld, r->fplan, r->fdev.segs, r->fdev.part,
                                            r->st))
    QPM_STEP(QPM_K_FINISH_DE, launch_batch_finish(2, *r->bt, p, r->fdev, r->ld, c.np, r->f_cur, r->flags, r->leaders,
                                                  r->draws, r->gen, c.seed, c.inst, r->st, r->fbits,
                                                  r->lazy ? AcceptOut{r->acc_list, r->acc_cnt, r->fbits_prev}
                                                          : AcceptOut{}))
    if (r->lazy) {  // the accepted trials' genes (timed with the finish)
        const uint32_t k0 = static_cast<uint32_t>(c.seed), k1 = static_cast<uint32_t>(c.seed >> 32);
        batch_materialize_kernel<<<2048, 256, 0, r->st>>>(r->pop(), r->inst, r->draws, r->fbits_prev, c.F,
                                                          cr_threshold(c.CR), k0, k1, r->gen, c.inst, r->acc_list,
                                                          r->acc_cnt, r->bt->n_inst, r->max_chunks);
        QPM_TRY_HIP(hipGetLastError());
    }
    QPM_STEP(QPM_K_GWO, launch_batch_gwo(r))
    QPM_STEP(QPM_K_FIT_GWO, launch_batch_fit(*r->bt, p, r->bits, c.np, r->ld, r->fplan, r->fdev.segs, r->fdev.part,
                                             r->st, r->gen))
    QPM_STEP(QPM_K_FINISH_GWO, launch_batch_finish(3, *r->bt, p, r->fdev, r->ld, c.np, r->f_cur, r->flags,
                                                   r->leaders, r->draws, r->gen, c.seed, c.inst, r->st,
                                                   r->fbits))
#undef QPM_STEP
    return mark(QPM_K_COUNT);
}

// time the batched table fitness for a few launch shapes on the current
// bits and keep the fastest (results are equal up to the summation order)
static qpm_status tune_fitness(qpm_batch_run_s *r)
{
    const qpm_run_config &c = r->cfg;
    const qpm_prec p = static_cast<qpm_prec>(c.prec);
    const std::string key = tune_key("batchtab", r->bt->total_words, c.np, c.prec, r->bt->n_inst);
    {
        int v0, v1;
        const int maxw = table_max_wpw(p == QPM_PREC_F32);
        if (tune_lookup(key, &v0, &v1, [&](int g, int w) { return (g == 1 || g == 2 || g == 4) && w >= 1 && w <= maxw; })) {
            r->fplan = make_tab_plan(r->bt->host, v0, v1);
            return QPM_OK;
        }
    }
    std::vector<std::pair<int, int>> cands;
    for (int g : {1, 2, 4})
        for (int w = 1; w <= table_max_wpw(p == QPM_PREC_F32); ++w) cands.push_back({g, w});
    hipEvent_t e0, e1;
    QPM_TRY_HIP(hipEventCreate(&e0));
    QPM_TRY_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    std::pair<int, int> pick{1, 1};
    default_tab_shape(c.np, p == QPM_PREC_F32, &pick.first, &pick.second);
    for (auto cand : cands) {
        BatchFitPlan pl = make_tab_plan(r->bt->host, cand.first, cand.second);
        if (pl.segs.size() > 65535) continue;
        FitPlanDev fp;
        qpm_status st = upload_fit_plan(pl, r->ld, r->st, &fp);
        if (st != QPM_OK) return st;
        st = launch_batch_fit(*r->bt, p, r->bits, c.np, r->ld, pl, fp.segs, fp.part, r->st);  // warm-up
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && st == QPM_OK; ++rep) {
            QPM_TRY_HIP(hipEventRecord(e0, r->st));
            st = launch_batch_fit(*r->bt, p, r->bits, c.np, r->ld, pl, fp.segs, fp.part, r->st);
            QPM_TRY_HIP(hipEventRecord(e1, r->st));
            QPM_TRY_HIP(hipEventSynchronize(e1));
            float t = 0.0f;
            QPM_TRY_HIP(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t);
        }
        free_fit_plan(fp, r->st);
        if (st != QPM_OK) return st;
        if (ms < best) {
            best = ms;
            pick = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    QPM_TRY_HIP(hipStreamSynchronize(r->st));
    r->tune_us = best * 1000.0;
    r->fplan = make_tab_plan(r->bt->host, pick.first, pick.second);
    tune_store(key, pick.first, pick.second);
    return QPM_OK;
}

// one generation captured into r->graph / r->exec
static qpm_status capture_batch_generation(qpm_batch_run_s *r)
{
    hipError_t e = hipStreamBeginCapture(r->st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        set_error("hipStreamBeginCapture failed: %s", hipGetErrorString(e));
        return QPM_EHIP;
    }
    qpm_status st = batch_generation(r);
    e = hipStreamEndCapture(r->st, &r->graph);
    if (st == QPM_OK && e != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
        st = QPM_EHIP;
    }
    if (st == QPM_OK && hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error("hipGraphInstantiate failed");
        st = QPM_EHIP;
    }
    return st;
}

// time the batched DE for every (individuals per wave, passes) shape on the
// initial population and keep the fastest (the shape never changes results)
static qpm_status tune_de(qpm_batch_run_s *r)
{
    const qpm_run_config &c = r->cfg;
    const std::string key = tune_key("batchde", r->bt->total_words, c.np, 0, r->bt->n_inst);
    int ipw = 0, passes = 0;
    const auto de_ok = [](int w, int pc) { return (w == 1 || w == 2 || w == 4) && (pc == 1 || pc == 2 || pc == 4); };
    if (!tune_lookup(key, &ipw, &passes, de_ok)) {
        hipEvent_t e0, e1;
        QPM_TRY_HIP(hipEventCreate(&e0));
        QPM_TRY_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        qpm_status st = QPM_OK;
        for (int cand : {1, 2, 4})
            for (int pc : {1, 2, 4}) {
                st = launch_batch_de(r, cand, pc);  // warm-up
                float ms = 1e30f;
                for (int rep = 0; rep < 3 && st == QPM_OK; ++rep) {
                    QPM_TRY_HIP(hipEventRecord(e0, r->st));
                    st = launch_batch_de(r, cand, pc);
                    QPM_TRY_HIP(hipEventRecord(e1, r->st));
                    QPM_TRY_HIP(hipEventSynchronize(e1));
                    float t = 0.0f;
                    QPM_TRY_HIP(hipEventElapsedTime(&t, e0, e1));
                    ms = std::min(ms, t);
                }
                if (st != QPM_OK) break;
                if (ms < best) {
                    best = ms;
                    ipw = cand;
                    passes = pc;
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != QPM_OK) return st;
        tune_store(key, ipw, passes);
    }
    r->de_ipw = ipw;
    r->de_passes = passes;
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_run_create(qpm_batch b, const qpm_run_config *cfg, int32_t tune, qpm_stream sv,
                                        qpm_batch_run_handle *out)
{
    clear_error();
    QPM_REQUIRE(b && cfg && out, QPM_EINVAL, "batch, cfg and out must not be NULL");
    const qpm_run_config c = *cfg;
    QPM_REQUIRE(c.np >= 4 && c.np <= 4096, QPM_EINVAL, "batched runs need 4 <= np <= 4096 (got %lld)",
                (long long)c.np);
    QPM_REQUIRE(c.generations >= 1 && c.generations <= (int64_t(1) << 31) - 2, QPM_EINVAL, "generations out of range");
    QPM_REQUIRE(c.F >= 0.0f && c.F <= 2.0f, QPM_EINVAL, "F must be in [0, 2]");
    QPM_REQUIRE(c.CR >= 0.0f && c.CR <= 1.0f, QPM_EINVAL, "CR must be in [0, 1]");
    QPM_REQUIRE(c.prec == QPM_PREC_F32 || c.prec == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", c.prec);
    QPM_REQUIRE(c.gwo_variant == 0 || c.gwo_variant == 1, c.gwo_variant == 2 ? QPM_ENOTSUP : QPM_EINVAL,
                "batched runs take gwo_variant 0 or 1 (got %d)", (int)c.gwo_variant);
    QPM_REQUIRE(c.control == QPM_CONTROL_FIXED, QPM_ENOTSUP, "batched runs use the fixed parameter control only");
    QPM_REQUIRE(c.algo == QPM_ALGO_HWSDA, c.algo == QPM_ALGO_DE || c.algo == QPM_ALGO_GWO ? QPM_ENOTSUP : QPM_EINVAL,
                "batched runs apply the hybrid optimiser only (algo %d)", (int)c.algo);
    QPM_REQUIRE(c.fused == 0 || c.fused == -1, c.fused == 1 ? QPM_ENOTSUP : QPM_EINVAL,
                "batched runs have no fused single-workgroup generations (fused %d)", (int)c.fused);
    QPM_REQUIRE(c.trials == QPM_TRIALS_AUTO || c.trials == QPM_TRIALS_STORE || c.trials == QPM_TRIALS_ACCEPTED,
                QPM_EINVAL, "unknown trial storage %d", c.trials);
    QPM_REQUIRE(static_cast<int64_t>(c.inst) + b->n_inst <= (int64_t(1) << 24), QPM_EINVAL,
                "inst + n_inst must be <= 2^24");
    qpm_status st = check_device();
    if (st != QPM_OK) return st;
    auto *r = new qpm_batch_run_s();
    r->bt = b;
    r->cfg = c;
    r->ld = ((c.np + 63) / 64) * 64;
    const int64_t n_inst = b->n_inst;
    // instance table with gene offsets for np rows per instance
    std::vector<InstDesc> h = b->host;
    int64_t xofs = 0;
    for (auto &d : h) {
        d.xofs = xofs;
        xofs += c.np * d.ldx;
    }
    const size_t gene_bytes = sizeof(float) * static_cast<size_t>(xofs);
    // tiles: GWO / init chunks of 1024 genes; DE chunks of 256 / ipw genes
    // for ipw = 1, 2, 4 (the shape is chosen by the default or the tuner)
    std::vector<Tile> gt, dt[3];
    const int64_t row_bytes = 2 * 1024 * 1024 / c.np;
    r->de_ipw = row_bytes >= 1024 ? 1 : (row_bytes >= 512 ? 2 : 4);
    for (int32_t i = 0; i < b->n_inst; ++i) {
        for (int64_t ch = 0; ch * 1024 < h[i].n; ++ch) gt.push_back(Tile{i, static_cast<int>(ch)});
        for (int v = 0; v < 3; ++v) {
            const int64_t cw = 256 >> v;
            for (int64_t ch = 0; ch * cw < h[i].n; ++ch) dt[v].push_back(Tile{i, static_cast<int>(ch)});
        }
    }
    // accepted-only trials: recomputing an accepted trial reads 20 B per
    // gene against 4 B per gene for storing every trial, so they pay below
    // about 20 % acceptance and for large populations; chosen automatically,
    // as for single runs, above 64 MB for both gene buffers (the 64-design
    // workload, NP = 256, 1.7 GB: a whole 500-generation run 0.909 s against
    // 0.946 s storing every trial)
    int64_t total_n = 0;
    for (const auto &d : h) total_n += d.n;
    r->lazy = c.trials == QPM_TRIALS_ACCEPTED ||
              (c.trials == QPM_TRIALS_AUTO && 2 * static_cast<int64_t>(sizeof(float)) * c.np * total_n >
                                                  (int64_t(64) << 20));
    if (r->lazy && n_inst * c.np >= (int64_t(1) << 31)) {  // list entries are int32 instance * np + slot
        if (c.trials == QPM_TRIALS_ACCEPTED) {
            set_error("accepted-only trials need n_inst * np < 2^31");
            release_batch_run(r);
            return QPM_EINVAL;
        }
        r->lazy = false;
    }
    for (const auto &d : h) r->max_chunks = std::max<int64_t>(r->max_chunks, (d.n + 255) / 256);
    if (gt.size() > 65535) {  // the GWO and init grids put these chunks on gridDim.y
        set_error("too many 1024-gene chunks over the batch (%zu > 65535)", gt.size());
        release_batch_run(r);
        return QPM_ERANGE;
    }
    r->n_gtiles = static_cast<int>(gt.size());
    for (int v = 0; v < 3; ++v) r->n_dtiles[v] = static_cast<int>(dt[v].size());
    hipError_t e = hipStreamCreateWithFlags(&r->st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&r->buf[0], gene_bytes);
    if (e == hipSuccess) e = hipMalloc(&r->buf[1], gene_bytes);
    if (e == hipSuccess) e = hipMalloc(&r->flags, sizeof(uint32_t) * n_inst * c.np);
    if (e == hipSuccess) e = hipMalloc(&r->fbits, sizeof(uint32_t) * n_inst * ((c.np + 31) / 32));
    if (e == hipSuccess) e = hipMalloc(&r->f_cur, (r->f64() ? 8 : 4) * n_inst * c.np);
    if (e == hipSuccess) e = hipMalloc(&r->bits, sizeof(uint32_t) * b->total_words * r->ld);
    if (e == hipSuccess) e = hipMalloc(&r->leaders, sizeof(int32_t) * 3 * n_inst);
    if (e == hipSuccess) e = hipMalloc(&r->draws, sizeof(int4) * n_inst * c.np);
    if (e == hipSuccess && r->lazy) e = hipMalloc(&r->acc_list, sizeof(int32_t) * n_inst * c.np);
    if (e == hipSuccess && r->lazy) e = hipMalloc(&r->acc_cnt, sizeof(uint32_t));
    if (e == hipSuccess && r->lazy) e = hipMalloc(&r->fbits_prev, sizeof(uint32_t) * n_inst * ((c.np + 31) / 32));
    if (e == hipSuccess) e = hipMalloc(&r->gen, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&r->a_tab, sizeof(float) * c.generations);
    if (e == hipSuccess) e = hipMalloc(&r->inst, sizeof(InstDesc) * n_inst);
    if (e == hipSuccess) e = hipMalloc(&r->gtiles, sizeof(Tile) * gt.size());
    for (int v = 0; v < 3; ++v)
        if (e == hipSuccess) e = hipMalloc(&r->dtiles[v], sizeof(Tile) * dt[v].size());
    if (e != hipSuccess) {
        set_error("batched run allocation failed: %s", hipGetErrorString(e));
        release_batch_run(r);
        return e == hipErrorOutOfMemory ? QPM_ENOMEM : QPM_EHIP;
    }
    std::vector<float> a(c.generations);
    for (int64_t g = 0; g < c.generations; ++g)
        a[g] = static_cast<float>(2.0 * (1.0 - static_cast<double>(g) / static_cast<double>(c.generations)));
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, static_cast<hipStream_t>(sv));
    if (e == hipSuccess) e = hipStreamWaitEvent(r->st, ev, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->a_tab, a.data(), sizeof(float) * c.generations, hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(r->inst, h.data(), sizeof(InstDesc) * n_inst, hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->gtiles, gt.data(), sizeof(Tile) * gt.size(), hipMemcpyHostToDevice, r->st);
    for (int v = 0; v < 3; ++v)
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->dtiles[v], dt[v].data(), sizeof(Tile) * dt[v].size(), hipMemcpyHostToDevice,
                               r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->flags, 0, sizeof(uint32_t) * n_inst * c.np, r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->fbits, 0, sizeof(uint32_t) * n_inst * ((c.np + 31) / 32), r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->gen, 0, sizeof(uint32_t), r->st);
    if (e == hipSuccess && r->lazy) e = hipMemsetAsync(r->acc_cnt, 0, sizeof(uint32_t), r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->bits, 0, sizeof(uint32_t) * b->total_words * r->ld, r->st);
    if (e == hipSuccess) e = hipStreamSynchronize(r->st);
    if (ev) (void)hipEventDestroy(ev);
    if (e != hipSuccess) {
        set_error("batched run set-up failed: %s", hipGetErrorString(e));
        release_batch_run(r);
        return QPM_EHIP;
    }
    // step 1: initialise every instance
    {
        const dim3 grid(static_cast<unsigned>(c.np), static_cast<unsigned>(r->n_gtiles));
        batch_init_kernel<<<grid, 256, 0, r->st>>>(c.np, r->inst, r->gtiles, static_cast<uint32_t>(c.seed),
                                                  static_cast<uint32_t>(c.seed >> 32), c.inst, r->buf[0], r->bits,
                                                  r->ld);
        e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("batched init launch failed: %s", hipGetErrorString(e));
            release_batch_run(r);
            return QPM_EHIP;
        }
    }
    if (tune) {
        st = tune_fitness(r);
    } else {
        int gw, wpw;
        default_tab_shape(c.np, c.prec == QPM_PREC_F32, &gw, &wpw);
        r->fplan = make_tab_plan(b->host, gw, wpw);
    }
    if (st == QPM_OK && r->fplan.segs.size() > 65535) {
        set_error("too many fitness segments (%zu)", r->fplan.segs.size());
        st = QPM_ERANGE;
    }
    if (st == QPM_OK) st = upload_fit_plan(r->fplan, r->ld, r->st, &r->fdev);
    const qpm_prec p = static_cast<qpm_prec>(c.prec);
    if (st == QPM_OK) st = launch_batch_fit(*b, p, r->bits, c.np, r->ld, r->fplan, r->fdev.segs, r->fdev.part, r->st);
    if (st == QPM_OK)
        st = launch_batch_finish(1, *b, p, r->fdev, r->ld, c.np, r->f_cur, r->flags, r->leaders, r->draws, r->gen,
                                 c.seed, c.inst, r->st);
    // the DE shape: the trial launches of the tuner write only the other
    // gene buffer and the bit rows, which the first generation overwrites
    if (st == QPM_OK && tune) st = tune_de(r);
    if (st == QPM_OK && c.use_graph) st = capture_batch_generation(r);
    if (st != QPM_OK) {
        release_batch_run(r);
        return st;
    }
    *out = r;
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_run_set_de_shape(qpm_batch_run_handle r, int32_t individuals_per_wave, int32_t passes)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    QPM_REQUIRE(individuals_per_wave == 1 || individuals_per_wave == 2 || individuals_per_wave == 4, QPM_EINVAL,
                "individuals_per_wave must be 1, 2 or 4 (got %d)", (int)individuals_per_wave);
    QPM_REQUIRE(passes == 1 || passes == 2 || passes == 4, QPM_EINVAL, "passes must be 1, 2 or 4 (got %d)",
                (int)passes);
    QPM_TRY_HIP(hipStreamSynchronize(r->st));
    r->de_ipw = individuals_per_wave;
    r->de_passes = passes;
    if (r->exec) {
        (void)hipGraphExecDestroy(r->exec);
        (void)hipGraphDestroy(r->graph);
        r->exec = nullptr;
        r->graph = nullptr;
        return capture_batch_generation(r);
    }
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_run_advance(qpm_batch_run_handle r, int64_t generations)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    QPM_REQUIRE(generations >= 0 && r->done + generations <= r->cfg.generations, QPM_EINVAL,
                "advancing %lld generations would pass the configured %lld (done %lld)", (long long)generations,
                (long long)r->cfg.generations, (long long)r->done);
    for (int64_t g = 0; g < generations; ++g) {
        if (r->timing) {
            qpm_status st = batch_generation(r, r->ev);
            if (st != QPM_OK) return st;
            QPM_TRY_HIP(hipEventSynchronize(r->ev[QPM_K_COUNT]));
            for (int k = 0; k < QPM_K_COUNT; ++k) {
                float t = 0.0f;
                QPM_TRY_HIP(hipEventElapsedTime(&t, r->ev[k], r->ev[k + 1]));
                r->ms[k] += t;
            }
            ++r->timed;
        } else if (r->exec) {
            QPM_TRY_HIP(hipGraphLaunch(r->exec, r->st));
        } else {
            qpm_status st = batch_generation(r);
            if (st != QPM_OK) return st;
        }
        ++r->done;
    }
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_run_set_timing(qpm_batch_run_handle r, int32_t enable)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    if (enable && !r->ev[0])
        for (auto &e : r->ev) QPM_TRY_HIP(hipEventCreate(&e));
    r->timing = enable != 0;
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_run_timing(qpm_batch_run_handle r, double *ms, int64_t *generations, int32_t reset)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    if (ms)
        for (int k = 0; k < QPM_K_COUNT; ++k) ms[k] = r->ms[k];
    if (generations) *generations = r->timed;
    if (reset) {
        for (double &v : r->ms) v = 0.0;
        r->timed = 0;
    }
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_run_read(qpm_batch_run_handle r, int32_t inst, float *x, int64_t ldx, void *fitness,
                                      int32_t *leaders, int32_t *fit_shape)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    QPM_REQUIRE(inst >= 0 && inst < r->bt->n_inst, QPM_EINVAL, "instance %d out of range", (int)inst);
    const InstDesc &d = r->bt->host[inst];
    if (x) {
        QPM_REQUIRE(ldx >= d.n, QPM_EINVAL, "ldx (%lld) must be >= the instance's N (%lld)", (long long)ldx,
                    (long long)d.n);
        const int64_t blocks = (d.n + 255) / 256;
        batch_gather_kernel<<<dim3(static_cast<unsigned>(blocks < 64 ? blocks : 64),
                                   static_cast<unsigned>(r->cfg.np)),
                              256, 0, r->st>>>(r->pop(), r->inst, inst, x, ldx);
        QPM_TRY_HIP(hipGetLastError());
    }
    const size_t es = r->f64() ? sizeof(double) : sizeof(float);
    if (fitness)
        QPM_TRY_HIP(hipMemcpyAsync(fitness, static_cast<char *>(r->f_cur) + es * r->cfg.np * inst, es * r->cfg.np,
                                   hipMemcpyDeviceToDevice, r->st));
    if (leaders)
        QPM_TRY_HIP(hipMemcpyAsync(leaders, r->leaders + 3 * inst, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, r->st));
    QPM_TRY_HIP(hipStreamSynchronize(r->st));
    if (fit_shape) {
        fit_shape[0] = r->fplan.waves;
        fit_shape[1] = r->fplan.wpw;
    }
    return QPM_OK;
}

QPM_API qpm_status qpm_batch_run_destroy(qpm_batch_run_handle r)
{
    clear_error();
    release_batch_run(r);
    return QPM_OK;
}
