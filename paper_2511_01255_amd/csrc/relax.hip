// relax.hip -- the differentiable relaxation d = tanh(theta) of the +-1
// design (an addition to the paper's discrete search): for real d the
// double integral of paper Sec. 2.1 is
//   S = sum_{m<n} d_m d_n a_m b_n + sum_n d_n^2 c_n,   f = |S|^2,
// and its adjoint is
//   dS/dd_k = b_k P_{k-1} + a_k R_{k+1} + 2 c_k d_k,
//   P_{k-1} = sum_{m<k} d_m a_m,  R_{k+1} = sum_{n>k} d_n b_n,
//   df/dtheta_k = 2 Re(conj(S) dS/dd_k) (1 - d_k^2).
//
// Mapping: a wave owns a tile of 64 consecutive rows x one sub-segment of 32
// consecutive domains, lane = row; the 4 waves of a workgroup take the 4
// consecutive sub-segments of one 128-domain segment (short sub-segments:
// about 6 waves per SIMD at 256 rows x 5 x 10^4 domains). The rows' theta of
// a 16-domain chunk is loaded coalesced (four lanes per row, 16 bytes each),
// transposed through LDS, and each lane walks its row's domains in order;
// the coefficients of a domain are the same for every lane (LDS
// broadcasts).
// A lane's sub-segment reduces to (A, B, Q, Dg) = (sum d a, sum d b,
// sum_n d_n b_n (A before n), sum c d^2) with no exchange between lanes; the
// workgroup folds its 4 sub-segments per row in order through LDS, the
// segments of a row combine in order in a small per-row pass that also
// forms, for the adjoint, the prefix A before and the sum of B from every
// segment on, and the forward pass keeps each sub-segment's A and B. The
// adjoint walks the same tiles from those edges and stores the gradient
// back through LDS, coalesced. Precision: FP32 evaluates tanh in binary32
// (hardware exp2 and reciprocal); the sums, products and the adjoint are
// FP64 in both precisions (FP64 costs what FP32 does on this chip without
// packed FP32 instructions).
#include "common.hpp"

namespace qpm {

struct RelaxPlan {
    int nseg;        // segments of kRelaxSeg domains per row
    int nsub;        // sub-segments of kRelaxSub domains per row (4 nseg)
    int64_t groups;  // row groups of 64
};

constexpr int kRelaxSub = 32;                 // domains per wave tile
constexpr int kRelaxSeg = 4 * kRelaxSub;      // domains per workgroup (4 waves)
constexpr int kRelaxChunk = 16;               // domains per transposed chunk

static RelaxPlan plan_relax(int64_t n, int64_t B, bool f32)
{
    (void)f32;
    RelaxPlan p;
    p.nseg = static_cast<int>((n + kRelaxSeg - 1) / kRelaxSeg);
    p.nsub = 4 * p.nseg;
    p.groups = (B + 63) / 64;
    return p;
}

// doubles of the edges: per row, 4 per segment (A before it, B from it on,
// as doubles) and 4 values per sub-segment (its own A and B, in the
// precision of the walk: binary32 for FP32, 2 doubles' worth)
static int64_t relax_edges_count(const RelaxPlan &p, int64_t rows, bool f32)
{
    return (4 * static_cast<int64_t>(p.nseg) + (f32 ? 2 : 4) * static_cast<int64_t>(p.nsub)) * rows;
}

// The work item (seg groups + rg) of a workgroup. Workgroups go to the 8
// XCDs in turn; each XCD takes a contiguous range of items (the row groups
// of a segment, then the next segment), so a segment's coefficients are
// fetched into one XCD's L2 rather than several. -1: past the last item.
__device__ __forceinline__ int64_t relax_item(int64_t per_xcd, int64_t items)
{
    const int64_t it = static_cast<int64_t>(blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
    return it < items ? it : -1;
}

static int64_t relax_per_xcd(const RelaxPlan &p) { return (static_cast<int64_t>(p.nseg) * p.groups + 7) / 8; }

template <typename T>
__device__ __forceinline__ T tanh_t(T x);
// FP32: tanh x = 1 - 2 / (1 + e^{2x}) from the hardware exp2 and
// reciprocal (a few ulp; exact +-1 once e^{2x} overflows or underflows),
// and x (1 - x^2 / 3) for |x| < 2^-6, where the first form loses relative
// accuracy (the next term, 2 x^5 / 15, is below 1e-8 relative there). The
// FP32 path's tolerance (1e-5) is far above either error.
template <>
__device__ __forceinline__ float tanh_t<float>(float x)
{
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 log2(e) x
    const float big = fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
    const float x2 = x * x;
    const float small = fmaf(-x2 * (1.0f / 3.0f), x, x);
    return fabsf(x) < 0.015625f ? small : big;
}
template <>
__device__ __forceinline__ double tanh_t<double>(double x) { return tanh(x); }

// the triple of a stretch of domains plus its diagonal sum
struct RTri {
    double ar, ai, br, bi, qr, qi, gr, gi;
};

// t <- t (+) u (t covers the domains before u)
__device__ __forceinline__ void rtri_append(RTri &t, const RTri &u)
{
    t.qr = fma(t.ar, u.br, fma(-t.ai, u.bi, t.qr + u.qr));
    t.qi = fma(t.ar, u.bi, fma(t.ai, u.br, t.qi + u.qi));
    t.ar += u.ar;
    t.ai += u.ai;
    t.br += u.br;
    t.bi += u.bi;
    t.gr += u.gr;
    t.gi += u.gi;
}

__device__ __forceinline__ RTri rtri_shfl_down(const RTri &t, int off)
{
    return RTri{__shfl_down(t.ar, off), __shfl_down(t.ai, off), __shfl_down(t.br, off), __shfl_down(t.bi, off),
                __shfl_down(t.qr, off), __shfl_down(t.qi, off), __shfl_down(t.gr, off), __shfl_down(t.gi, off)};
}

// The loads of one 16-domain chunk [kc, kc + 16) of rows rg 64 .. + 63:
// four instructions of 16 rows each, four lanes per row, 16 bytes per lane
// (0 past n or B). Issued ahead of use: every chunk of a tile is in flight
// before the first is consumed.
template <bool VEC>
__device__ __forceinline__ void load_chunk_regs(float4 (&v)[4], const float *__restrict__ theta, int64_t ldt,
                                                int64_t B, int64_t n, int64_t rg, int64_t kc, int lane)
{
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        const int rt = step * 16 + (lane >> 2), col = (lane & 3) * 4;
        const int64_t row = rg * 64 + rt, k = kc + col;
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < B) {
            const float *src = theta + row * ldt + k;
            if (VEC && k + 3 < n) {
                q = *reinterpret_cast<const float4 *>(src);
            } else {
                if (k < n) q.x = src[0];
                if (k + 1 < n) q.y = src[1];
                if (k + 2 < n) q.z = src[2];
                if (k + 3 < n) q.w = src[3];
            }
        }
        v[step] = q;
    }
}

// The chunk's loaded values into the wave's LDS tile, row-major with a
// padded stride (kRelaxST floats: the column reads of lane = row are free
// of bank conflicts). Lane l then reads its row's values at
// tile[l kRelaxST + e]; only the wave that staged a tile reads it, so no
// workgroup barrier is needed (a wave's LDS accesses complete in order) and
// the waves of a workgroup run their chunks independently.
constexpr int kRelaxST = kRelaxChunk + 1;
__device__ __forceinline__ void stage_chunk(const float4 (&v)[4], float *tile, int lane)
{
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        const int rt = step * 16 + (lane >> 2), col = (lane & 3) * 4;
        float *t = tile + rt * kRelaxST + col;
        t[0] = v[step].x;
        t[1] = v[step].y;
        t[2] = v[step].z;
        t[3] = v[step].w;
    }
    // (the wave reads only its own tile: its LDS accesses complete in order)
    __builtin_amdgcn_wave_barrier();
}

// domains per step of the walks
constexpr int kRelaxStep = 4;

// The coefficients of the workgroup's segment [seg S, seg S + S) (S =
// kRelaxSeg) into LDS: co[3 j] = (a.re, a.im), co[3 j + 1] = (b.re, b.im),
// co[3 j + 2] = c of domain seg S + j (0 past n), staged by lane j % Sub of
// wave j / Sub (Sub = kRelaxSub), so every wave stages exactly the
// coefficients of its own sub-segment; read back as broadcasts (every lane
// the same address).
__device__ __forceinline__ void stage_coef(double2 *co, const double4 *__restrict__ ph64,
                                           const double2 *__restrict__ c64, int64_t seg, int64_t n)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l < kRelaxSub) {
        const int j = w * kRelaxSub + l;  // lane l of wave w: domain l of the wave's sub-segment
        const int64_t k = seg * kRelaxSeg + j;
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
        double2 c = make_double2(0.0, 0.0);
        if (k < n) {
            v = ph64[k];
            c = c64[k];
        }
        co[3 * j] = make_double2(v.x, v.y);
        co[3 * j + 1] = make_double2(v.z, v.w);
        co[3 * j + 2] = c;
    }
    // (each wave stages and reads only its own sub-segment's coefficients)
    __builtin_amdgcn_wave_barrier();
}

// Segment partials: part[(row * nseg + seg) * 8 + c], c = A.re, A.im,
// B.re, B.im, Q.re, Q.im, Dg.re, Dg.im (doubles, a row's segments
// contiguous for the per-row combine); with sub, also each
// sub-segment's A and B: sub[(ss * 4 + c) * lds + row], c = A.re, A.im,
// B.re, B.im, in T (binary32 for FP32: the adjoint adds them to FP64
// edges, so their rounding stays far below the FP32 tolerance and the
// pass pair moves half the bytes for them). Workgroup item (seg, rg) = item / groups, % groups; wave w
// walks sub-segment 4 seg + w of the rows rg 64 + lane.
// (FP32: at most about 80 VGPRs, so the 6 waves per SIMD the grid gives at
// 256 rows x 5 x 10^4 domains fit; the FP64 tanh needs more registers)
template <typename T, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1))) void
relax_fwd_kernel(const float *__restrict__ theta, int64_t ldt, int64_t B,
                 int64_t n, const double4 *__restrict__ ph64,
                 const double2 *__restrict__ c64, int64_t groups, int nseg,
                 int64_t per_xcd, double *__restrict__ part,
                 T *__restrict__ sub, int64_t lds)
{
    __shared__ float tiles[4][64 * kRelaxST];
    // the segment's coefficients
    __shared__ double2 co[3 * kRelaxSeg];
    // after the walk, the fold of the waves (in the tiles)
    double(*fold)[8][64] = reinterpret_cast<double(*)[8][64]>(&tiles[0][0]);
    static_assert(sizeof(tiles) >= 3 * 8 * 64 * sizeof(double), "the fold reuses the tiles");
    // the wave index as a wave-uniform value: the segment and domain indices
    // below stay scalar, so the coefficients are scalar loads
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t item = relax_item(per_xcd, nseg * groups);
    if (item < 0) return;  // the whole workgroup
    const int64_t seg = item / groups, rg = item % groups;
    const int64_t ss = 4 * seg + wave;
    const int64_t row = rg * 64 + lane;
    double ar = 0, ai = 0, br = 0, bi = 0, qr = 0, qi = 0, gr = 0, gi = 0;
    constexpr int NCH = kRelaxSub / kRelaxChunk;
    // a chunk is staged, then the next chunk's loads go out into the same
    // registers while the chunk is walked
    float4 buf[4];
    load_chunk_regs<VEC>(buf, theta, ldt, B, n, rg, ss * kRelaxSub, lane);
    stage_coef(co, ph64, c64, seg, n);
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
        const int64_t kc = ss * kRelaxSub + ch * kRelaxChunk;
        float *tl = tiles[wave];
        stage_chunk(buf, tl, lane);
        if (ch + 1 < NCH) load_chunk_regs<VEC>(buf, theta, ldt, B, n, rg, kc + kRelaxChunk, lane);
#pragma unroll 1
        for (int e0 = 0; e0 < kRelaxChunk; e0 += kRelaxStep) {
#pragma unroll
            for (int e1 = 0; e1 < kRelaxStep; ++e1) {
                // past the row's end theta and the coefficients are 0, so
                // d = tanh 0 = 0 and the domain adds nothing
                const int e = e0 + e1;
                const int jl = wave * kRelaxSub + ch * kRelaxChunk + e;  // domain within the segment
                const double2 ca = co[3 * jl], cb = co[3 * jl + 1], cc = co[3 * jl + 2];
                const double4 c = make_double4(ca.x, ca.y, cb.x, cb.y);
                const float th = tl[lane * kRelaxST + e];
                const double d = static_cast<double>(tanh_t<T>(static_cast<T>(th)));
                const double yr = d * c.z, yi = d * c.w;
                qr = fma(yr, ar, fma(-yi, ai, qr));
                qi = fma(yr, ai, fma(yi, ar, qi));
                ar = fma(d, c.x, ar);
                ai = fma(d, c.y, ai);
                br += yr;
                bi += yi;
                const double d2 = d * d;
                gr = fma(d2, cc.x, gr);
                gi = fma(d2, cc.y, gi);
            }
        }
        __builtin_amdgcn_wave_barrier();  // the tile is refilled by the next chunk
    }
    if (sub != nullptr && row < B) {
        T *o = sub + ss * 4 * lds + row;
        o[0] = static_cast<T>(ar);
        o[lds] = static_cast<T>(ai);
        o[2 * lds] = static_cast<T>(br);
        o[3 * lds] = static_cast<T>(bi);
    }
    // the 4 sub-segments of each row in order: waves 1-3 through LDS into
    // wave 0 (fold reuses the tiles: every wave must be done with its own)
    __syncthreads();
    if (wave > 0) {
        const double v[8] = {ar, ai, br, bi, qr, qi, gr, gi};
#pragma unroll
        for (int c = 0; c < 8; ++c) fold[wave - 1][c][lane] = v[c];
    }
    __syncthreads();
    if (wave == 0 && row < B) {
        RTri t{ar, ai, br, bi, qr, qi, gr, gi};
#pragma unroll
        for (int w = 0; w < 3; ++w)
            rtri_append(t, RTri{fold[w][0][lane], fold[w][1][lane], fold[w][2][lane], fold[w][3][lane],
                                fold[w][4][lane], fold[w][5][lane], fold[w][6][lane], fold[w][7][lane]});
        double *o = part + (row * nseg + seg) * 8;
        o[0] = t.ar;
        o[1] = t.ai;
        o[2] = t.br;
        o[3] = t.bi;
        o[4] = t.qr;
        o[5] = t.qi;
        o[6] = t.gr;
        o[7] = t.gi;
    }
}

// The partial triple of segment sg of a row (zero past the row's segments:
// the identity of rtri_append).
__device__ __forceinline__ RTri load_part(const double *__restrict__ pr, int sg, int nseg)
{
    if (sg >= nseg) return RTri{0, 0, 0, 0, 0, 0, 0, 0};
    const double2 *p = reinterpret_cast<const double2 *>(pr + static_cast<int64_t>(sg) * 8);
    const double2 a = p[0], b = p[1], q = p[2], g = p[3];
    return RTri{a.x, a.y, b.x, b.y, q.x, q.y, g.x, g.y};
}

// DPP moves within 16-lane rows (double as two 32-bit moves): lane l reads
// lane l + k (row_shl k) or l - k (row_shr k) of its own row; a lane whose
// source lies outside its row reads 0.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int K>
__device__ __forceinline__ double row_from_above(double v) { return dpp_d<0x100 + K>(v); }  // lane l + K
template <int K>
__device__ __forceinline__ double row_from_below(double v) { return dpp_d<0x110 + K>(v); }  // lane l - K

__device__ __forceinline__ double lane_value(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

template <int K>
__device__ __forceinline__ void rtri_tree_level(RTri &u, int lane)
{
    const RTri o{row_from_above<K>(u.ar), row_from_above<K>(u.ai), row_from_above<K>(u.br),
                 row_from_above<K>(u.bi), row_from_above<K>(u.qr), row_from_above<K>(u.qi),
                 row_from_above<K>(u.gr), row_from_above<K>(u.gi)};
    if ((lane & (2 * K - 1)) == 0) rtri_append(u, o);
}

__device__ __forceinline__ RTri rtri_lane(const RTri &u, int l)
{
    return RTri{lane_value(u.ar, l), lane_value(u.ai, l), lane_value(u.br, l), lane_value(u.bi, l),
                lane_value(u.qr, l), lane_value(u.qi, l), lane_value(u.gr, l), lane_value(u.gi, l)};
}

// inclusive scan of v within each 16-lane row
__device__ __forceinline__ double row_scan(double v)
{
    v += row_from_below<1>(v);
    v += row_from_below<2>(v);
    v += row_from_below<4>(v);
    v += row_from_below<8>(v);
    return v;
}

// rounds of 64 segments whose loads are issued together
constexpr int kCombineBatch = 4;
// waves per row of the combine, each taking a contiguous share of the rounds
constexpr int kCombineWaves = 8;

// Per row (a workgroup of kCombineWaves waves): S = (combined Q) + sum Dg and
// f = |S|^2; with `edges`, also the prefix A before every segment and the
// sum of B from the segment on: edges[(row * nseg + seg) * 4 + c],
// c = Apre.re, Apre.im, Bfrom.re, Bfrom.im.
// The row's segments go in rounds of 64, lane l taking segment 64 t + l (a
// row's partials are contiguous, so a round's loads are coalesced), and
// wave w takes a contiguous share of the rounds (the loads of up to four
// rounds in flight together). A round folds in order: within each 16-lane
// row by a DPP tree, then the four row heads; the waves' folds combine in
// order through LDS. For the edges each wave rereads its A and B and scans
// them (DPP within rows, then the rows' totals) from the A and B of the
// waves before it: A before the segment, and B from it on as the row's B
// less the B before the segment.
__global__ __launch_bounds__(64 * kCombineWaves) void relax_combine_kernel(const double *__restrict__ part,
                                                                          int nseg, int64_t B,
                                                                          double *__restrict__ S,
                                                                          float *__restrict__ f,
                                                                          double *__restrict__ edges)
{
    __shared__ double folds[kCombineWaves][8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row = blockIdx.x;
    if (row >= B) return;  // the whole workgroup (the grid is B workgroups)
    const double *pr = part + row * nseg * 8;
    const int rounds = (nseg + 63) / 64;
    const int t_beg = wave * rounds / kCombineWaves, t_end = (wave + 1) * rounds / kCombineWaves;
    RTri mine{0, 0, 0, 0, 0, 0, 0, 0};
    for (int t0 = t_beg; t0 < t_end; t0 += kCombineBatch) {
        RTri u[kCombineBatch];  // every round of the batch in flight at once
#pragma unroll
        for (int b = 0; b < kCombineBatch; ++b)
            u[b] = t0 + b < t_end ? load_part(pr, 64 * (t0 + b) + lane, nseg) : RTri{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < kCombineBatch; ++b) {
            if (t0 + b < t_end) {
                rtri_tree_level<1>(u[b], lane);
                rtri_tree_level<2>(u[b], lane);
                rtri_tree_level<4>(u[b], lane);
                rtri_tree_level<8>(u[b], lane);
#pragma unroll
                for (int h = 0; h < 64; h += 16) rtri_append(mine, rtri_lane(u[b], h));
            }
        }
    }
    if (lane == 0) {
        const double v[8] = {mine.ar, mine.ai, mine.br, mine.bi, mine.qr, mine.qi, mine.gr, mine.gi};
#pragma unroll
        for (int c = 0; c < 8; ++c) folds[wave][c] = v[c];
    }
    __syncthreads();
    // the row's fold (the same order in every wave) and the A and B of the
    // waves before this one
    RTri tot{0, 0, 0, 0, 0, 0, 0, 0};
    double carry[4] = {0, 0, 0, 0};  // A.re, A.im, B.re, B.im before the wave's next round
#pragma unroll
    for (int w = 0; w < kCombineWaves; ++w) {
        const RTri tw{folds[w][0], folds[w][1], folds[w][2], folds[w][3],
                      folds[w][4], folds[w][5], folds[w][6], folds[w][7]};
        if (w < wave) {
            carry[0] += tw.ar;
            carry[1] += tw.ai;
            carry[2] += tw.br;
            carry[3] += tw.bi;
        }
        rtri_append(tot, tw);
    }
    if (edges) {
        double *er = edges + row * nseg * 4;
        const int rid = lane >> 4;
        for (int t0 = t_beg; t0 < t_end; t0 += kCombineBatch) {
            double4 vb[kCombineBatch];
#pragma unroll
            for (int b = 0; b < kCombineBatch; ++b) {
                const int sg = 64 * (t0 + b) + lane;
                vb[b] = make_double4(0.0, 0.0, 0.0, 0.0);
                if (t0 + b < t_end && sg < nseg) {
                    const double2 *p = reinterpret_cast<const double2 *>(pr + static_cast<int64_t>(sg) * 8);
                    const double2 a = p[0], bb = p[1];
                    vb[b] = make_double4(a.x, a.y, bb.x, bb.y);
                }
            }
#pragma unroll
            for (int b = 0; b < kCombineBatch; ++b) {
                if (t0 + b >= t_end) break;
                const int sg = 64 * (t0 + b) + lane;
                const double in[4] = {row_scan(vb[b].x), row_scan(vb[b].y), row_scan(vb[b].z), row_scan(vb[b].w)};
                double ex[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    // the rows' totals; the sum of the rows before this lane's
                    const double r0 = lane_value(in[c], 15), r1 = lane_value(in[c], 31),
                                 r2 = lane_value(in[c], 47), r3 = lane_value(in[c], 63);
                    const double before = rid == 0 ? 0.0 : rid == 1 ? r0 : rid == 2 ? r0 + r1 : (r0 + r1) + r2;
                    ex[c] = (before + row_from_below<1>(in[c])) + carry[c];  // lane 16 k reads 0
                    carry[c] += ((r0 + r1) + r2) + r3;
                }
                if (sg < nseg) {
                    double *e = er + static_cast<int64_t>(sg) * 4;  // (only 8-byte aligned)
                    e[0] = ex[0];
                    e[1] = ex[1];
                    e[2] = tot.br - ex[2];
                    e[3] = tot.bi - ex[3];
                }
            }
        }
    }
    if (threadIdx.x != 0) return;
    const double Sr = tot.qr + tot.gr, Si = tot.qi + tot.gi;
    if (S) {
        S[2 * row] = Sr;
        S[2 * row + 1] = Si;
    }
    if (f) f[row] = static_cast<float>(fma(Sr, Sr, Si * Si));
}

// The adjoint over the tiles of the forward pass: per lane (row), walking
// its sub-segment's domains in order from P = A before the sub-segment and
// R = B from the sub-segment on (the segment's edges, less the earlier
// sub-segments of the segment),
//   R_{k+1} = R - (B of the sub-segment up to k),  P_{k-1} = P + (A before k),
//   grad_k = grad_f 2 Re(conj(S) (b_k P_{k-1} + a_k R_{k+1} + 2 c_k d_k)) (1 - d_k^2);
// each chunk's gradients go back through the wave's LDS tile and are stored
// coalesced (four lanes per row, 16 bytes each).
// (no register cap: held to 6 waves per SIMD, the FP32 adjoint spills and
// measured slower than at its natural 82 VGPRs)
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void
relax_bwd_kernel(const float *__restrict__ theta, int64_t ldt, int64_t B,
                 int64_t n, const double4 *__restrict__ ph64,
                 const double2 *__restrict__ c64, int64_t groups, int nseg,
                 int64_t per_xcd, const double *__restrict__ edges,
                 const T *__restrict__ sub, int64_t lde,
                 const double *__restrict__ S,
                 const float *__restrict__ grad_f,
                 float *__restrict__ grad_theta, int64_t ldg)
{
    __shared__ float tiles[4][64 * kRelaxST];
    __shared__ double2 co[3 * kRelaxSeg];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t item = relax_item(per_xcd, nseg * groups);
    if (item < 0) return;  // the whole workgroup
    const int64_t seg = item / groups, rg = item % groups;
    const int64_t ss = 4 * seg + wave;
    const int64_t row = rg * 64 + lane;
    const bool rv = row < B;
    double pr = 0, pi = 0, rr = 0, ri = 0, Sr = 0, Si = 0, gs = 0;
    if (rv) {
        const double *e = edges + (row * nseg + seg) * 4;
        pr = e[0];
        pi = e[1];
        rr = e[2];
        ri = e[3];
        for (int w = 0; w < wave; ++w) {
            const T *u = sub + (4 * seg + w) * 4 * lde + row;
            pr += u[0];
            pi += u[lde];
            rr -= u[2 * lde];
            ri -= u[3 * lde];
        }
        Sr = S[2 * row];
        Si = S[2 * row + 1];
        gs = 2.0 * static_cast<double>(grad_f[row]);
    }
    float *tl = tiles[wave];
    constexpr int NCH = kRelaxSub / kRelaxChunk;
    // a chunk is staged, then the next chunk's loads go out into the same
    // registers while the chunk is walked
    float4 buf[4];
    load_chunk_regs<VEC>(buf, theta, ldt, B, n, rg, ss * kRelaxSub, lane);
    stage_coef(co, ph64, c64, seg, n);
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
        const int64_t kc = ss * kRelaxSub + ch * kRelaxChunk;
        stage_chunk(buf, tl, lane);
        if (ch + 1 < NCH) load_chunk_regs<VEC>(buf, theta, ldt, B, n, rg, kc + kRelaxChunk, lane);
#pragma unroll 1
        for (int e0 = 0; e0 < kRelaxChunk; e0 += kRelaxStep) {
#pragma unroll
            for (int e1 = 0; e1 < kRelaxStep; ++e1) {
                // past the row's end theta and the coefficients are 0: d = 0
                // and the domain adds nothing (its gradient is not stored)
                const int e = e0 + e1;
                const int jl = wave * kRelaxSub + ch * kRelaxChunk + e;  // domain within the segment
                const double2 ca = co[3 * jl], cb = co[3 * jl + 1], cc = co[3 * jl + 2];
                const double4 c = make_double4(ca.x, ca.y, cb.x, cb.y);
                float *slot = tl + lane * kRelaxST + e;  // theta in, the gradient out
                const double d = static_cast<double>(tanh_t<T>(static_cast<T>(*slot)));
                // R_{k+1}: B from k + 1 on
                rr = fma(-d, c.z, rr);
                ri = fma(-d, c.w, ri);
                const double two_d = d + d;
                const double dsr =
                    fma(c.z, pr, fma(-c.w, pi, fma(c.x, rr, fma(-c.y, ri, two_d * cc.x))));
                const double dsi = fma(c.z, pi, fma(c.w, pr, fma(c.x, ri, fma(c.y, rr, two_d * cc.y))));
                const double re = fma(Sr, dsr, Si * dsi);
                *slot = static_cast<float>(gs * re * fma(-d, d, 1.0));
                pr = fma(d, c.x, pr);
                pi = fma(d, c.y, pi);
            }
        }
        __builtin_amdgcn_wave_barrier();
        // the chunk's gradients, coalesced (rows of this wave's tile)
#pragma unroll
        for (int step = 0; step < 4; ++step) {
            const int rt = step * 16 + (lane >> 2), col = (lane & 3) * 4;
            const int64_t r = rg * 64 + rt, k = kc + col;
            if (r < B && k < n) {
                float *dst = grad_theta + r * ldg + k;
                const float *v = tl + rt * kRelaxST + col;
                if (VEC && k + 3 < n) {
                    *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (k + e < n) dst[e] = v[e];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <typename T>
static void launch_relax_fwd(const Design &d, const RelaxPlan &pl, bool vec, const float *theta, int64_t B,
                             int64_t ldt, double *part, T *sub, int64_t lds, hipStream_t s)
{
    const int64_t per_xcd = relax_per_xcd(pl);
    const unsigned blocks = static_cast<unsigned>(8 * per_xcd);
    if (vec)
        relax_fwd_kernel<T, true><<<blocks, 256, 0, s>>>(theta, ldt, B, d.n, d.ph64, d.c64, pl.groups, pl.nseg,
                                                         per_xcd, part, sub, lds);
    else
        relax_fwd_kernel<T, false><<<blocks, 256, 0, s>>>(theta, ldt, B, d.n, d.ph64, d.c64, pl.groups, pl.nseg,
                                                          per_xcd, part, sub, lds);
}

template <typename T>
static void launch_relax_bwd(const Design &d, const RelaxPlan &pl, bool vec, const float *theta, int64_t B,
                             int64_t ldt, const double *edges, const T *sub, int64_t lde, const double *S,
                             const float *grad_f, float *grad_theta, int64_t ldg, hipStream_t s)
{
    const int64_t per_xcd = relax_per_xcd(pl);
    const unsigned blocks = static_cast<unsigned>(8 * per_xcd);
    if (vec)
        relax_bwd_kernel<T, true><<<blocks, 256, 0, s>>>(theta, ldt, B, d.n, d.ph64, d.c64, pl.groups, pl.nseg,
                                                         per_xcd, edges, sub, lde, S, grad_f, grad_theta, ldg);
    else
        relax_bwd_kernel<T, false><<<blocks, 256, 0, s>>>(theta, ldt, B, d.n, d.ph64, d.c64, pl.groups, pl.nseg,
                                                          per_xcd, edges, sub, lde, S, grad_f, grad_theta, ldg);
}

// segment partials part (8 nseg B doubles) and, with sub, the
// sub-segments' A and B (4 nsub lds doubles)
static qpm_status relax_partials(const Design &d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                                 const RelaxPlan &pl, double *part, void *sub, int64_t lds, hipStream_t s)
{
    const bool vec = (reinterpret_cast<uintptr_t>(theta) & 15u) == 0 && ldt % 4 == 0;
    if (p == QPM_PREC_F32)
        launch_relax_fwd<float>(d, pl, vec, theta, B, ldt, part, static_cast<float *>(sub), lds, s);
    else
        launch_relax_fwd<double>(d, pl, vec, theta, B, ldt, part, static_cast<double *>(sub), lds, s);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

// ---------------------------------------------------------------- polish

// theta_r += eta g_r / max_k |g_rk| for each row r (one workgroup per row)
__global__ __launch_bounds__(256) void polish_step_kernel(float *__restrict__ theta, const float *__restrict__ grad,
                                                          int64_t n, int64_t ld, float eta)
{
    const int64_t r = blockIdx.x;
    float *th = theta + r * ld;
    const float *g = grad + r * ld;
    float m = 0.0f;
    for (int64_t k = threadIdx.x; k < n; k += 256) m = fmaxf(m, fabsf(g[k]));
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    __shared__ float sm[4];
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
    if (m == 0.0f) return;
    const float sc = eta / m;
    for (int64_t k = threadIdx.x; k < n; k += 256) th[k] = fmaf(sc, g[k], th[k]);
}

// y = clamp(theta, -1, 1): the +-1 projection keeps the sign of theta and
// is a valid gene row
__global__ __launch_bounds__(256) void polish_project_kernel(const float *__restrict__ theta, float *__restrict__ y,
                                                             int64_t n, int64_t ld)
{
    const int64_t r = blockIdx.y;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < n; k += 256 * gridDim.x)
        y[r * ld + k] = fminf(fmaxf(theta[r * ld + k], -1.0f), 1.0f);
}

// For each of the three leaders: keep the projected row when its exact +-1
// fitness beats the leader's. One workgroup per leader.
template <typename T>
__global__ __launch_bounds__(256) void polish_accept_kernel(const float *__restrict__ y, int64_t n, int64_t ldy,
                                                            const T *__restrict__ fcand, const int32_t *__restrict__ L,
                                                            float *__restrict__ x0, float *__restrict__ x1,
                                                            const uint32_t *__restrict__ flags, int64_t ldx,
                                                            T *__restrict__ f_cur, uint32_t *__restrict__ accepted)
{
    const int k = blockIdx.x;
    const int64_t row = L[k];
    const T fc = fcand[k];
    if (!(fc > f_cur[row])) return;
    float *dst = (flags[row] ? x1 : x0) + row * ldx;
    for (int64_t j = threadIdx.x; j < n; j += 256) dst[j] = y[k * ldy + j];
    __syncthreads();
    if (threadIdx.x == 0) {
        f_cur[row] = fc;
        atomicAdd(accepted, 1u);
    }
}

qpm_status launch_polish_step(float *theta, const float *grad, int64_t rows, int64_t n, int64_t ld, float eta,
                              hipStream_t s)
{
    polish_step_kernel<<<static_cast<unsigned>(rows), 256, 0, s>>>(theta, grad, n, ld, eta);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_polish_project(const float *theta, float *y, int64_t rows, int64_t n, int64_t ld, hipStream_t s)
{
    const int64_t bx = (n + 255) / 256;
    polish_project_kernel<<<dim3(static_cast<unsigned>(bx < 64 ? bx : 64), static_cast<unsigned>(rows)), 256, 0, s>>>(
        theta, y, n, ld);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

qpm_status launch_polish_accept(const float *y, int64_t n, int64_t ldy, const void *fcand, bool f64, const int32_t *L,
                                const PopView &pv, void *f_cur, uint32_t *accepted, hipStream_t s)
{
    float *x0 = const_cast<float *>(pv.x0), *x1 = const_cast<float *>(pv.x1);
    if (f64)
        polish_accept_kernel<double><<<3, 256, 0, s>>>(y, n, ldy, static_cast<const double *>(fcand), L, x0, x1,
                                                       pv.flags, pv.ldx, static_cast<double *>(f_cur), accepted);
    else
        polish_accept_kernel<float><<<3, 256, 0, s>>>(y, n, ldy, static_cast<const float *>(fcand), L, x0, x1,
                                                      pv.flags, pv.ldx, static_cast<float *>(f_cur), accepted);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

}  // namespace qpm

using namespace qpm;

static qpm_status check_relax(qpm_design d, qpm_prec p, const float *theta, int64_t B, int64_t ldt)
{
    QPM_REQUIRE(d != nullptr && theta != nullptr, QPM_EINVAL, "design and theta must not be NULL");
    QPM_REQUIRE(p == QPM_PREC_F32 || p == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", (int)p);
    QPM_REQUIRE(B >= 1 && B <= (int64_t(1) << 24), QPM_EINVAL, "batch must be in [1, 2^24] (got %lld)",
                (long long)B);
    QPM_REQUIRE(ldt >= d->n, QPM_EINVAL, "ldt (%lld) must be >= n_domains (%lld)", (long long)ldt,
                (long long)d->n);
    return QPM_OK;
}

static qpm_status launch_combine(const double *part, int nseg, int64_t B, double *S, float *f, double *edges,
                                 hipStream_t s)
{
    relax_combine_kernel<<<static_cast<unsigned>(B), 64 * kCombineWaves, 0, s>>>(part, nseg, B, S, f, edges);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

QPM_API qpm_status qpm_relax_edges_size(qpm_design d, qpm_prec p, int64_t B, int64_t *count)
{
    clear_error();
    QPM_REQUIRE(d != nullptr && count != nullptr, QPM_EINVAL, "design and count must not be NULL");
    QPM_REQUIRE(p == QPM_PREC_F32 || p == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", (int)p);
    QPM_REQUIRE(B >= 1 && B <= (int64_t(1) << 24), QPM_EINVAL, "batch must be in [1, 2^24] (got %lld)",
                (long long)B);
    *count = relax_edges_count(plan_relax(d->n, B, p == QPM_PREC_F32), B, p == QPM_PREC_F32);
    return QPM_OK;
}

QPM_API qpm_status qpm_relax_forward(qpm_design d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                                     float *f, double *S, double *edges, qpm_stream sv)
{
    clear_error();
    qpm_status st = check_relax(d, p, theta, B, ldt);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(f != nullptr || S != nullptr, QPM_EINVAL, "at least one of f and S must be given");
    hipStream_t s = static_cast<hipStream_t>(sv);
    const RelaxPlan pl = plan_relax(d->n, B, p == QPM_PREC_F32);
    QPM_REQUIRE(static_cast<int64_t>(pl.nseg) * pl.groups < (int64_t(1) << 31) - 8, QPM_ERANGE,
                "batch x segments too large for one launch");
    ScratchLease lease(d->scratch, s);
    void *ws = nullptr;
    st = lease.begin(sizeof(double) * 8 * pl.nseg * B, &ws);
    if (st != QPM_OK) return st;
    double *part = static_cast<double *>(ws);
    // edges: the segments' (A before, B from) then the sub-segments' (A, B)
    void *sub = edges ? edges + 4 * static_cast<int64_t>(pl.nseg) * B : nullptr;
    st = relax_partials(*d, p, theta, B, ldt, pl, part, sub, B, s);
    if (st == QPM_OK) st = launch_combine(part, pl.nseg, B, S, f, edges, s);
    const qpm_status se = lease.end();
    return st != QPM_OK ? st : se;
}

QPM_API qpm_status qpm_relax_backward(qpm_design d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                                      const double *S, const double *edges, const float *grad_f, float *grad_theta,
                                      int64_t ldg, qpm_stream sv)
{
    clear_error();
    qpm_status st = check_relax(d, p, theta, B, ldt);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(S != nullptr && grad_f != nullptr && grad_theta != nullptr, QPM_EINVAL,
                "S, grad_f and grad_theta must not be NULL");
    QPM_REQUIRE(ldg >= d->n, QPM_EINVAL, "ldg (%lld) must be >= n_domains", (long long)ldg);
    hipStream_t s = static_cast<hipStream_t>(sv);
    const RelaxPlan pl = plan_relax(d->n, B, p == QPM_PREC_F32);
    QPM_REQUIRE(static_cast<int64_t>(pl.nseg) * pl.groups < (int64_t(1) << 31) - 8, QPM_ERANGE,
                "batch x segments too large for one launch");
    ScratchLease lease(d->scratch, s);
    const double *e = edges;
    const void *sub = edges ? edges + 4 * static_cast<int64_t>(pl.nseg) * B : nullptr;
    const int64_t lde = B;
    if (!edges) {
        // no saved edges: recompute the segment partials and their edges
        void *ws = nullptr;
        st = lease.begin(sizeof(double) * (12 * static_cast<int64_t>(pl.nseg) + 4 * pl.nsub) * B, &ws);
        if (st != QPM_OK) return st;
        double *work = static_cast<double *>(ws);
        double *ework = work + static_cast<int64_t>(8) * pl.nseg * B;
        double *swork = ework + static_cast<int64_t>(4) * pl.nseg * B;
        st = relax_partials(*d, p, theta, B, ldt, pl, work, swork, B, s);
        if (st == QPM_OK) st = launch_combine(work, pl.nseg, B, nullptr, nullptr, ework, s);
        e = ework;
        sub = swork;
    }
    if (st == QPM_OK) {
        const bool vec = (reinterpret_cast<uintptr_t>(theta) & 15u) == 0 && ldt % 4 == 0 &&
                         (reinterpret_cast<uintptr_t>(grad_theta) & 15u) == 0 && ldg % 4 == 0;
        if (p == QPM_PREC_F32)
            launch_relax_bwd<float>(*d, pl, vec, theta, B, ldt, e, static_cast<const float *>(sub), lde, S, grad_f,
                                    grad_theta, ldg, s);
        else
            launch_relax_bwd<double>(*d, pl, vec, theta, B, ldt, e, static_cast<const double *>(sub), lde, S, grad_f,
                                     grad_theta, ldg, s);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) {
            set_error("relax adjoint launch failed: %s", hipGetErrorString(err));
            st = QPM_EHIP;
        }
    }
    const qpm_status se = lease.end();
    return st != QPM_OK ? st : se;
}
