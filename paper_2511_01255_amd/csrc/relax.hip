// relax.hip -- the differentiable relaxation d = tanh(theta) of the +-1
// design (an addition to the paper's discrete search): for real d the
// double integral of paper Sec. 2.1 is
//   S = sum_{m<n} d_m d_n a_m b_n + sum_n d_n^2 c_n,   f = |S|^2,
// and its adjoint is
//   dS/dd_k = b_k P_{k-1} + a_k R_{k+1} + 2 c_k d_k,
//   P_{k-1} = sum_{m<k} d_m a_m,  R_{k+1} = sum_{n>k} d_n b_n,
//   df/dtheta_k = 2 Re(conj(S) dS/dd_k) (1 - d_k^2).
//
// Mapping: a workgroup of 256 lanes covers one segment of L = 256 M
// consecutive domains for R consecutive rows; lane t owns the M domains
// [seg L + t M, seg L + (t + 1) M), so the loads of theta and the stores of
// the gradient are coalesced along the row, and it keeps its M domains'
// coefficients in registers while it walks the R rows. A lane's chunk
// reduces to (A, B, Q, Dg) = (sum d a, sum d b, sum_n d_n b_n (A before n),
// sum c d^2); the 256 chunk triples of a segment combine in order (a
// shuffle tree in each wave, then the 4 waves through LDS, in FP64), and
// the segments of a row combine in order in a small per-row pass that also
// forms, for the adjoint, the prefix A before and the suffix B after every
// segment. The adjoint takes a lane's prefix of A and suffix of B from
// ordered scans over the lanes and walks its chunk from them.
#include "common.hpp"

namespace qpm {

struct RelaxPlan {
    int M;     // domains per lane
    int R;     // rows per workgroup
    int L;     // domains per segment (256 M)
    int nseg;  // segments per row
};

static RelaxPlan plan_relax(int64_t n, int64_t B, bool f32)
{
    RelaxPlan p;
    p.M = f32 ? 8 : 4;
    p.R = B >= 64 ? 4 : 1;
    p.L = 256 * p.M;
    p.nseg = static_cast<int>((n + p.L - 1) / p.L);
    return p;
}

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

// coefficients of lane-owned domains (0 past n)
template <typename T, int M>
struct Coef {
    T ar[M], ai[M], br[M], bi[M], cr[M], ci[M];
};

template <typename T, int M>
__device__ __forceinline__ void load_coef(Coef<T, M> &c, int64_t k0, int64_t n, const double4 *__restrict__ ph64,
                                          const float4 *__restrict__ ph32, const double2 *__restrict__ c64)
{
#pragma unroll
    for (int e = 0; e < M; ++e) {
        const int64_t k = k0 + e;
        const bool in = k < n;
        const int64_t kc = in ? k : 0;
        if constexpr (sizeof(T) == 4) {
            const float4 v = ph32[kc];
            c.ar[e] = in ? v.x : 0.f;
            c.ai[e] = in ? v.y : 0.f;
            c.br[e] = in ? v.z : 0.f;
            c.bi[e] = in ? v.w : 0.f;
        } else {
            const double4 v = ph64[kc];
            c.ar[e] = in ? v.x : 0.0;
            c.ai[e] = in ? v.y : 0.0;
            c.br[e] = in ? v.z : 0.0;
            c.bi[e] = in ? v.w : 0.0;
        }
        const double2 cc = c64[kc];
        c.cr[e] = in ? static_cast<T>(cc.x) : T(0);
        c.ci[e] = in ? static_cast<T>(cc.y) : T(0);
    }
}

// theta[row][k0 .. k0 + M) (0 past n); VEC: 16-byte aligned rows
template <int M, bool VEC>
__device__ __forceinline__ void load_theta(float (&th)[M], const float *__restrict__ rowp, int64_t k0, int64_t n)
{
    if (VEC && k0 + M <= n) {
#pragma unroll
        for (int e = 0; e < M; e += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(rowp + k0 + e);
            th[e] = v.x;
            th[e + 1] = v.y;
            th[e + 2] = v.z;
            th[e + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < M; ++e) th[e] = k0 + e < n ? rowp[k0 + e] : 0.f;
    }
}

// Lane value of lane l - OFF in the lane's row of 16 lanes (row_shr, CTRL
// 0x110 + OFF), or of the last lane of the previous row (row_bcast:15, CTRL
// 0x142, rows 1 and 3) or of lane 31 (row_bcast:31, CTRL 0x143, rows 2 and
// 3); undefined where there is none (no lane reads those). DPP moves: no
// LDS traffic, unlike a shuffle.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_from(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROWS, 0xF, true);
    return __hiloint2double(hi, lo);
}

// one level of the ordered tree: the lanes that `take` prepend the triple
// of the lanes before them (u <- o (+) u)
template <int CTRL, int ROWS>
__device__ __forceinline__ void tree_level(RTri &u, bool take)
{
    RTri o{dpp_from<CTRL, ROWS>(u.ar), dpp_from<CTRL, ROWS>(u.ai), dpp_from<CTRL, ROWS>(u.br),
           dpp_from<CTRL, ROWS>(u.bi), dpp_from<CTRL, ROWS>(u.qr), dpp_from<CTRL, ROWS>(u.qi),
           dpp_from<CTRL, ROWS>(u.gr), dpp_from<CTRL, ROWS>(u.gi)};
    if (take) {
        rtri_append(o, u);
        u = o;
    }
}

// The 64 chunk triples of a wave combined in order into lane 63: pairs of
// neighbours, then groups of 4, 8, 16, 32 and 64 lanes, each the left group
// followed by the right one.
__device__ __forceinline__ void wave_fold_rtri(RTri &u, int lane)
{
    tree_level<0x111, 0xF>(u, (lane & 1) == 1);
    tree_level<0x112, 0xF>(u, (lane & 3) == 3);
    tree_level<0x114, 0xF>(u, (lane & 7) == 7);
    tree_level<0x118, 0xF>(u, (lane & 15) == 15);
    tree_level<0x142, 0xA>(u, (lane & 31) == 31);
    tree_level<0x143, 0xC>(u, lane == 63);
}

// Inclusive prefix sums of four values over the 64 lanes of a wave with DPP
// moves: within rows of 16 lanes (shifts 1, 2, 4, 8), then the last lane of
// row 0 / 2 into rows 1 / 3, then lane 31 into rows 2 and 3.
template <int CTRL, int ROWS>
__device__ __forceinline__ void scan_step(double &a, double &b, double &c, double &d, bool take)
{
    const double oa = dpp_from<CTRL, ROWS>(a), ob = dpp_from<CTRL, ROWS>(b);
    const double oc = dpp_from<CTRL, ROWS>(c), od = dpp_from<CTRL, ROWS>(d);
    if (take) {
        a += oa;
        b += ob;
        c += oc;
        d += od;
    }
}

__device__ __forceinline__ void wave_scan4(double &a, double &b, double &c, double &d, int lane)
{
    scan_step<0x111, 0xF>(a, b, c, d, (lane & 15) >= 1);
    scan_step<0x112, 0xF>(a, b, c, d, (lane & 15) >= 2);
    scan_step<0x114, 0xF>(a, b, c, d, (lane & 15) >= 4);
    scan_step<0x118, 0xF>(a, b, c, d, (lane & 15) >= 8);
    scan_step<0x142, 0xA>(a, b, c, d, (lane & 16) != 0);
    scan_step<0x143, 0xC>(a, b, c, d, lane >= 32);
}

// Segment partials: part[(seg * 8 + c) * ldb + row], c = A.re, A.im,
// B.re, B.im, Q.re, Q.im, Dg.re, Dg.im (doubles).
template <typename T, int M, int R, bool VEC>
__global__ __launch_bounds__(256) void relax_fwd_kernel(const float *__restrict__ theta, int64_t ldt, int64_t B,
                                                        int64_t n, const double4 *__restrict__ ph64,
                                                        const float4 *__restrict__ ph32,
                                                        const double2 *__restrict__ c64, int nseg, int64_t ldb,
                                                        double *__restrict__ part)
{
    __shared__ RTri sh[4];
    const int seg = static_cast<int>(blockIdx.x % static_cast<unsigned>(nseg));
    const int64_t row0 = static_cast<int64_t>(blockIdx.x / static_cast<unsigned>(nseg)) * R;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t k0 = static_cast<int64_t>(seg) * 256 * M + static_cast<int64_t>(t) * M;
    Coef<T, M> c;
    load_coef<T, M>(c, k0, n, ph64, ph32, c64);
    for (int r = 0; r < R; ++r) {
        const int64_t row = row0 + r;
        if (row >= B) break;
        float th[M];
        load_theta<M, VEC>(th, theta + row * ldt, k0, n);
        T ar = 0, ai = 0, br = 0, bi = 0, qr = 0, qi = 0, gr = 0, gi = 0;
#pragma unroll
        for (int e = 0; e < M; ++e) {
            const T d = tanh_t<T>(static_cast<T>(th[e]));
            const T yr = d * c.br[e], yi = d * c.bi[e];
            qr = fma(yr, ar, fma(-yi, ai, qr));
            qi = fma(yr, ai, fma(yi, ar, qi));
            ar = fma(d, c.ar[e], ar);
            ai = fma(d, c.ai[e], ai);
            br += yr;
            bi += yi;
            const T d2 = d * d;
            gr = fma(d2, c.cr[e], gr);
            gi = fma(d2, c.ci[e], gi);
        }
        RTri u{ar, ai, br, bi, qr, qi, gr, gi};
        wave_fold_rtri(u, lane);
        if (lane == 63) sh[wave] = u;
        __syncthreads();
        if (t == 0) {
            RTri s0 = sh[0];
            rtri_append(s0, sh[1]);
            rtri_append(s0, sh[2]);
            rtri_append(s0, sh[3]);
            double *o = part + static_cast<int64_t>(seg) * 8 * ldb + row;
            o[0] = s0.ar;
            o[ldb] = s0.ai;
            o[2 * ldb] = s0.br;
            o[3 * ldb] = s0.bi;
            o[4 * ldb] = s0.qr;
            o[5 * ldb] = s0.qi;
            o[6 * ldb] = s0.gr;
            o[7 * ldb] = s0.gi;
        }
        __syncthreads();
    }
}

// Per row (one wave): S = (combined Q) + sum Dg and f = |S|^2; with `edges`,
// also the prefix A before and the suffix B after every segment:
// edges[(seg * 4 + c) * lde + row], c = Apre.re, Apre.im, Bsuf.re, Bsuf.im.
// Lane l folds the segments [l m, (l + 1) m), m = ceil(nseg / 64), in
// order; an ordered shuffle tree combines the lanes, and lane scans give
// each lane's prefix of A and suffix of B for the edges.
__global__ __launch_bounds__(256) void relax_combine_kernel(const double *__restrict__ part, int nseg, int64_t ldb,
                                                            int64_t B, double *__restrict__ S,
                                                            float *__restrict__ f, double *__restrict__ edges,
                                                            int64_t lde)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (row >= B) return;  // a whole wave: no barriers below
    const int m = (nseg + 63) / 64;
    const int s0 = min(nseg, lane * m), s1 = min(nseg, s0 + m);
    RTri t{0, 0, 0, 0, 0, 0, 0, 0};
    for (int sg = s0; sg < s1; ++sg) {
        const double *p = part + static_cast<int64_t>(sg) * 8 * ldb + row;
        rtri_append(t, RTri{p[0], p[ldb], p[2 * ldb], p[3 * ldb], p[4 * ldb], p[5 * ldb], p[6 * ldb], p[7 * ldb]});
    }
    if (edges) {
        double par = t.ar, pai = t.ai, sbr = t.br, sbi = t.bi;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double ur = __shfl_up(par, off), ui = __shfl_up(pai, off);
            const double vr = __shfl_down(sbr, off), vi = __shfl_down(sbi, off);
            if (lane >= off) {
                par += ur;
                pai += ui;
            }
            if (lane + off < 64) {
                sbr += vr;
                sbi += vi;
            }
        }
        double ar = par - t.ar, ai = pai - t.ai;  // A before this lane's segments
        for (int sg = s0; sg < s1; ++sg) {
            const double *p = part + static_cast<int64_t>(sg) * 8 * ldb + row;
            double *e = edges + static_cast<int64_t>(sg) * 4 * lde + row;
            e[0] = ar;
            e[lde] = ai;
            ar += p[0];
            ai += p[ldb];
        }
        double br = sbr - t.br, bi = sbi - t.bi;  // B after this lane's segments
        for (int sg = s1 - 1; sg >= s0; --sg) {
            const double *p = part + static_cast<int64_t>(sg) * 8 * ldb + row;
            double *e = edges + static_cast<int64_t>(sg) * 4 * lde + row;
            e[2 * lde] = br;
            e[3 * lde] = bi;
            br += p[2 * ldb];
            bi += p[3 * ldb];
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const RTri o = rtri_shfl_down(t, off);
        if ((lane & (2 * off - 1)) == 0) rtri_append(t, o);
    }
    if (lane != 0) return;
    const double Sr = t.qr + t.gr, Si = t.qi + t.gi;
    if (S) {
        S[2 * row] = Sr;
        S[2 * row + 1] = Si;
    }
    if (f) f[row] = static_cast<float>(fma(Sr, Sr, Si * Si));
}

// The adjoint over one segment for R rows: lane prefix of A and suffix of
// B by ordered scans (FP64), then each lane walks its chunk.
template <typename T, int M, int R, bool VEC>
__global__ __launch_bounds__(256) void relax_bwd_kernel(const float *__restrict__ theta, int64_t ldt, int64_t B,
                                                        int64_t n, const double4 *__restrict__ ph64,
                                                        const float4 *__restrict__ ph32,
                                                        const double2 *__restrict__ c64, int nseg,
                                                        const double *__restrict__ edges, int64_t lde,
                                                        const double *__restrict__ S,
                                                        const float *__restrict__ grad_f,
                                                        float *__restrict__ grad_theta, int64_t ldg)
{
    __shared__ double swa[4][2], swb[4][2];
    const int seg = static_cast<int>(blockIdx.x % static_cast<unsigned>(nseg));
    const int64_t row0 = static_cast<int64_t>(blockIdx.x / static_cast<unsigned>(nseg)) * R;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t k0 = static_cast<int64_t>(seg) * 256 * M + static_cast<int64_t>(t) * M;
    Coef<T, M> c;
    load_coef<T, M>(c, k0, n, ph64, ph32, c64);
    for (int r = 0; r < R; ++r) {
        const int64_t row = row0 + r;
        if (row >= B) break;
        float th[M];
        load_theta<M, VEC>(th, theta + row * ldt, k0, n);
        T d[M];
        T alr = 0, ali = 0, blr = 0, bli = 0;
#pragma unroll
        for (int e = 0; e < M; ++e) {
            d[e] = tanh_t<T>(static_cast<T>(th[e]));
            alr = fma(d[e], c.ar[e], alr);
            ali = fma(d[e], c.ai[e], ali);
            blr = fma(d[e], c.br[e], blr);
            bli = fma(d[e], c.bi[e], bli);
        }
        // inclusive prefix scans of A and B over the wave (DPP moves); B
        // after a lane's chunk is the wave's total less that prefix
        double par = alr, pai = ali, pbr = blr, pbi = bli;
        wave_scan4(par, pai, pbr, pbi, lane);
        const double tbr = __shfl(pbr, 63), tbi = __shfl(pbi, 63);
        if (lane == 63) {
            swa[wave][0] = par;
            swa[wave][1] = pai;
            swb[wave][0] = tbr;
            swb[wave][1] = tbi;
        }
        __syncthreads();
        const double *e = edges + static_cast<int64_t>(seg) * 4 * lde + row;
        // A before this lane's chunk, B after it
        double Pr = e[0] + (par - alr), Pi = e[lde] + (pai - ali);
        double Rr = e[2 * lde] + (tbr - pbr), Ri = e[3 * lde] + (tbi - pbi);
        for (int w = 0; w < wave; ++w) {
            Pr += swa[w][0];
            Pi += swa[w][1];
        }
        for (int w = 3; w > wave; --w) {
            Rr += swb[w][0];
            Ri += swb[w][1];
        }
        __syncthreads();
        const T Sr = static_cast<T>(S[2 * row]), Si = static_cast<T>(S[2 * row + 1]);
        const T gscale = static_cast<T>(2.0f * grad_f[row]);
        // R_{k+1} = (B after the chunk) + (chunk B) - (chunk B up to k)
        const T rr0 = static_cast<T>(Rr) + blr, ri0 = static_cast<T>(Ri) + bli;
        T pr = static_cast<T>(Pr), pi = static_cast<T>(Pi), cbr = 0, cbi = 0;
        float g[M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const T dq = d[q];
            cbr = fma(dq, c.br[q], cbr);
            cbi = fma(dq, c.bi[q], cbi);
            const T rr = rr0 - cbr, ri = ri0 - cbi;
            // dS/dd = b P + a R + 2 c d
            const T two_d = dq + dq;
            const T dsr = fma(c.br[q], pr, fma(-c.bi[q], pi, fma(c.ar[q], rr, fma(-c.ai[q], ri, two_d * c.cr[q]))));
            const T dsi = fma(c.br[q], pi, fma(c.bi[q], pr, fma(c.ar[q], ri, fma(c.ai[q], rr, two_d * c.ci[q]))));
            const T re = fma(Sr, dsr, Si * dsi);
            g[q] = static_cast<float>(gscale * re * (1 - dq * dq));
            pr = fma(dq, c.ar[q], pr);
            pi = fma(dq, c.ai[q], pi);
        }
        float *go = grad_theta + row * ldg;
        if (VEC && k0 + M <= n) {
#pragma unroll
            for (int q = 0; q < M; q += 4)
                *reinterpret_cast<float4 *>(go + k0 + q) = make_float4(g[q], g[q + 1], g[q + 2], g[q + 3]);
        } else {
#pragma unroll
            for (int q = 0; q < M; ++q)
                if (k0 + q < n) go[k0 + q] = g[q];
        }
    }
}

template <typename T, int M>
static void launch_relax_fwd(const Design &d, const RelaxPlan &pl, bool vec, const float *theta, int64_t B,
                             int64_t ldt, int64_t ldb, double *part, hipStream_t s)
{
    const unsigned blocks = static_cast<unsigned>(((B + pl.R - 1) / pl.R) * pl.nseg);
#define QPM_RF(RR, V)                                                                                          \
    relax_fwd_kernel<T, M, RR, V><<<blocks, 256, 0, s>>>(theta, ldt, B, d.n, d.ph64, d.ph32, d.c64, pl.nseg, ldb, \
                                                         part)
    if (pl.R == 4) {
        if (vec) QPM_RF(4, true); else QPM_RF(4, false);
    } else {
        if (vec) QPM_RF(1, true); else QPM_RF(1, false);
    }
#undef QPM_RF
}

template <typename T, int M>
static void launch_relax_bwd(const Design &d, const RelaxPlan &pl, bool vec, const float *theta, int64_t B,
                             int64_t ldt, const double *edges, int64_t lde, const double *S, const float *grad_f,
                             float *grad_theta, int64_t ldg, hipStream_t s)
{
    const unsigned blocks = static_cast<unsigned>(((B + pl.R - 1) / pl.R) * pl.nseg);
#define QPM_RB(RR, V)                                                                                              \
    relax_bwd_kernel<T, M, RR, V><<<blocks, 256, 0, s>>>(theta, ldt, B, d.n, d.ph64, d.ph32, d.c64, pl.nseg, edges, \
                                                         lde, S, grad_f, grad_theta, ldg)
    if (pl.R == 4) {
        if (vec) QPM_RB(4, true); else QPM_RB(4, false);
    } else {
        if (vec) QPM_RB(1, true); else QPM_RB(1, false);
    }
#undef QPM_RB
}

static qpm_status relax_partials(const Design &d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                                 const RelaxPlan &pl, int64_t ldb, double *part, hipStream_t s)
{
    const bool vec = (reinterpret_cast<uintptr_t>(theta) & 15u) == 0 && ldt % 4 == 0;
    if (p == QPM_PREC_F32)
        launch_relax_fwd<float, 8>(d, pl, vec, theta, B, ldt, ldb, part, s);
    else
        launch_relax_fwd<double, 4>(d, pl, vec, theta, B, ldt, ldb, part, s);
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

static qpm_status launch_combine(const double *part, int nseg, int64_t ldb, int64_t B, double *S, float *f,
                                 double *edges, int64_t lde, hipStream_t s)
{
    relax_combine_kernel<<<static_cast<unsigned>((B + 3) / 4), 256, 0, s>>>(part, nseg, ldb, B, S, f, edges, lde);
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
    *count = 4 * static_cast<int64_t>(plan_relax(d->n, B, p == QPM_PREC_F32).nseg) * B;
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
    QPM_REQUIRE(((B + pl.R - 1) / pl.R) * pl.nseg < (int64_t(1) << 31), QPM_ERANGE,
                "batch x segments too large for one launch");
    const int64_t ldb = ((B + 63) / 64) * 64;
    ScratchLease lease(d->scratch, s);
    void *ws = nullptr;
    st = lease.begin(sizeof(double) * 8 * pl.nseg * ldb, &ws);
    if (st != QPM_OK) return st;
    double *part = static_cast<double *>(ws);
    st = relax_partials(*d, p, theta, B, ldt, pl, ldb, part, s);
    if (st == QPM_OK) st = launch_combine(part, pl.nseg, ldb, B, S, f, edges, B, s);
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
    QPM_REQUIRE(((B + pl.R - 1) / pl.R) * pl.nseg < (int64_t(1) << 31), QPM_ERANGE,
                "batch x segments too large for one launch");
    ScratchLease lease(d->scratch, s);
    const double *e = edges;
    int64_t lde = B;
    if (!edges) {
        // no saved edges: recompute the segment partials and their edges
        const int64_t ldb = ((B + 63) / 64) * 64;
        void *ws = nullptr;
        st = lease.begin(sizeof(double) * 12 * pl.nseg * ldb, &ws);
        if (st != QPM_OK) return st;
        double *work = static_cast<double *>(ws);
        double *ework = work + static_cast<int64_t>(8) * pl.nseg * ldb;
        st = relax_partials(*d, p, theta, B, ldt, pl, ldb, work, s);
        if (st == QPM_OK) st = launch_combine(work, pl.nseg, ldb, B, nullptr, nullptr, ework, ldb, s);
        e = ework;
        lde = ldb;
    }
    if (st == QPM_OK) {
        const bool vec = (reinterpret_cast<uintptr_t>(theta) & 15u) == 0 && ldt % 4 == 0 &&
                         (reinterpret_cast<uintptr_t>(grad_theta) & 15u) == 0 && ldg % 4 == 0;
        if (p == QPM_PREC_F32)
            launch_relax_bwd<float, 8>(*d, pl, vec, theta, B, ldt, e, lde, S, grad_f, grad_theta, ldg, s);
        else
            launch_relax_bwd<double, 4>(*d, pl, vec, theta, B, ldt, e, lde, S, grad_f, grad_theta, ldg, s);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) {
            set_error("relax adjoint launch failed: %s", hipGetErrorString(err));
            st = QPM_EHIP;
        }
    }
    const qpm_status se = lease.end();
    return st != QPM_OK ? st : se;
}
