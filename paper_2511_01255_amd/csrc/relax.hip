// relax.hip -- the differentiable relaxation d = tanh(theta) of the +-1
// design (an addition to the paper's discrete search): for real d the
// double integral of paper Sec. 2.1 is
//   S = sum_{m<n} d_m d_n a_m b_n + sum_n d_n^2 c_n,   f = |S|^2,
// and its adjoint is
//   dS/dd_k = b_k P_{k-1} + a_k R_{k+1} + 2 c_k d_k,
//   P_{k-1} = sum_{m<k} d_m a_m,  R_{k+1} = sum_{n>k} d_n b_n,
//   df/dtheta_k = 2 Re(conj(S) dS/dd_k) (1 - d_k^2).
//
// Mapping: one lane per batch row (64 rows per wave); the domain axis is cut
// into segments, one per wave, scanned in order with the per-domain
// coefficients in scalar registers. A segment reduces to (A, B, Q, Dg) =
// (sum d a, sum d b, sum_n d_n b_n (A before n), sum c d^2); segments are
// combined in order by a small per-row pass that also forms, for the
// adjoint, the prefix A before and the suffix B after every segment. The
// adjoint then re-walks each segment from those two values.
#include "common.hpp"

namespace qpm {

struct RelaxPlan {
    int seg_len;  // domains per segment (multiple of 4)
    int nseg;     // segments
    int waves;    // waves per workgroup
};

static RelaxPlan plan_relax(int64_t n, int64_t B)
{
    const int64_t groups = (B + 63) / 64;
    const int64_t target = 4096;  // waves in flight
    int64_t segs = (target + groups - 1) / groups;
    int64_t len = (n + segs - 1) / segs;
    len = ((len + 3) / 4) * 4;
    if (len < 16) len = 16;
    RelaxPlan p;
    p.seg_len = static_cast<int>(len);
    p.nseg = static_cast<int>((n + len - 1) / len);
    p.waves = 4;
    return p;
}

template <typename T>
__device__ __forceinline__ T tanh_t(T x);
template <>
__device__ __forceinline__ float tanh_t<float>(float x) { return tanhf(x); }
template <>
__device__ __forceinline__ double tanh_t<double>(double x) { return tanh(x); }

// Segment partials: part[(seg * 8 + c) * ldb + row], c = A.re, A.im,
// B.re, B.im, Q.re, Q.im, Dg.re, Dg.im (doubles).
template <typename T>
__global__ __launch_bounds__(256) void relax_seg_kernel(const float *__restrict__ theta, int64_t ldt, int64_t B,
                                                        int64_t n, const double4 *__restrict__ ph64,
                                                        const float4 *__restrict__ ph32,
                                                        const double2 *__restrict__ c64, int seg_len, int nseg,
                                                        int64_t ldb, double *__restrict__ part)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int seg = static_cast<int>(blockIdx.y) * 4 + wave;
    if (seg >= nseg) return;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const bool live = row < B;
    const int64_t n0 = static_cast<int64_t>(seg) * seg_len;
    const int64_t n1 = n0 + seg_len < n ? n0 + seg_len : n;
    T ar = 0, ai = 0, br = 0, bi = 0, qr = 0, qi = 0, gr = 0, gi = 0;
    const float *th = theta + (live ? row : 0) * ldt;
    for (int64_t k = n0; k < n1; k += 4) {
        float4 t4 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (live) {
            if (k + 3 < n1) {
                t4 = make_float4(th[k], th[k + 1], th[k + 2], th[k + 3]);
            } else {
                t4.x = th[k];
                if (k + 1 < n1) t4.y = th[k + 1];
                if (k + 2 < n1) t4.z = th[k + 2];
            }
        }
        const float tv[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (k + e >= n1) break;
            T pa_r, pa_i, pb_r, pb_i;
            if constexpr (sizeof(T) == 4) {
                const float4 c = ph32[k + e];
                pa_r = c.x; pa_i = c.y; pb_r = c.z; pb_i = c.w;
            } else {
                const double4 c = ph64[k + e];
                pa_r = c.x; pa_i = c.y; pb_r = c.z; pb_i = c.w;
            }
            const double2 cc = c64[k + e];
            const T d = tanh_t<T>(static_cast<T>(tv[e]));
            const T yr = d * pb_r, yi = d * pb_i;
            // Q += y * A (A before this domain)
            qr = fma(yr, ar, fma(-yi, ai, qr));
            qi = fma(yr, ai, fma(yi, ar, qi));
            ar = fma(d, pa_r, ar);
            ai = fma(d, pa_i, ai);
            br += yr;
            bi += yi;
            const T d2 = d * d;
            gr = fma(d2, static_cast<T>(cc.x), gr);
            gi = fma(d2, static_cast<T>(cc.y), gi);
        }
    }
    if (!live) return;
    double *o = part + static_cast<int64_t>(seg) * 8 * ldb + row;
    o[0] = ar; o[ldb] = ai; o[2 * ldb] = br; o[3 * ldb] = bi;
    o[4 * ldb] = qr; o[5 * ldb] = qi; o[6 * ldb] = gr; o[7 * ldb] = gi;
}

// Per row: S = (combined Q) + sum Dg and f = |S|^2; with `edges`, also the
// prefix A before and the suffix B after every segment:
// edges[(seg * 4 + c) * ldb + row], c = Apre.re, Apre.im, Bsuf.re, Bsuf.im.
__global__ __launch_bounds__(256) void relax_combine_kernel(const double *__restrict__ part, int nseg, int64_t ldb,
                                                            int64_t B, double *__restrict__ S,
                                                            float *__restrict__ f, double *__restrict__ edges)
{
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (row >= B) return;
    double ar = 0, ai = 0, qr = 0, qi = 0, gr = 0, gi = 0;
    for (int s = 0; s < nseg; ++s) {
        const double *p = part + static_cast<int64_t>(s) * 8 * ldb + row;
        if (edges) {
            double *e = edges + static_cast<int64_t>(s) * 4 * ldb + row;
            e[0] = ar;
            e[ldb] = ai;
        }
        const double vr = p[2 * ldb], vi = p[3 * ldb];
        qr = fma(ar, vr, fma(-ai, vi, qr + p[4 * ldb]));
        qi = fma(ar, vi, fma(ai, vr, qi + p[5 * ldb]));
        ar += p[0];
        ai += p[ldb];
        gr += p[6 * ldb];
        gi += p[7 * ldb];
    }
    if (edges) {
        double sr = 0, si = 0;
        for (int s = nseg - 1; s >= 0; --s) {
            double *e = edges + static_cast<int64_t>(s) * 4 * ldb + row;
            e[2 * ldb] = sr;
            e[3 * ldb] = si;
            const double *p = part + static_cast<int64_t>(s) * 8 * ldb + row;
            sr += p[2 * ldb];
            si += p[3 * ldb];
        }
    }
    const double Sr = qr + gr, Si = qi + gi;
    if (S) {
        S[2 * row] = Sr;
        S[2 * row + 1] = Si;
    }
    if (f) f[row] = static_cast<float>(fma(Sr, Sr, Si * Si));
}

// The adjoint walk of one segment.
template <typename T>
__global__ __launch_bounds__(256) void relax_grad_kernel(const float *__restrict__ theta, int64_t ldt, int64_t B,
                                                         int64_t n, const double4 *__restrict__ ph64,
                                                         const float4 *__restrict__ ph32,
                                                         const double2 *__restrict__ c64, int seg_len, int nseg,
                                                         int64_t ldb, const double *__restrict__ part,
                                                         const double *__restrict__ edges,
                                                         const double *__restrict__ S,
                                                         const float *__restrict__ grad_f,
                                                         float *__restrict__ grad_theta, int64_t ldg)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int seg = static_cast<int>(blockIdx.y) * 4 + wave;
    if (seg >= nseg) return;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    if (row >= B) return;
    const int64_t n0 = static_cast<int64_t>(seg) * seg_len;
    const int64_t n1 = n0 + seg_len < n ? n0 + seg_len : n;
    const double *e = edges + static_cast<int64_t>(seg) * 4 * ldb + row;
    const double *p = part + static_cast<int64_t>(seg) * 8 * ldb + row;
    T pr = static_cast<T>(e[0]), pi = static_cast<T>(e[ldb]);  // P_{k-1}
    // R_{k+1} = (suffix after the segment) + (segment B) - (B up to k)
    const T rr0 = static_cast<T>(e[2 * ldb] + p[2 * ldb]), ri0 = static_cast<T>(e[3 * ldb] + p[3 * ldb]);
    T cbr = 0, cbi = 0;
    const T Sr = static_cast<T>(S[2 * row]), Si = static_cast<T>(S[2 * row + 1]);
    const T gscale = static_cast<T>(2.0f * grad_f[row]);
    const float *th = theta + row * ldt;
    float *go = grad_theta + row * ldg;
    for (int64_t k = n0; k < n1; ++k) {
        T pa_r, pa_i, pb_r, pb_i;
        if constexpr (sizeof(T) == 4) {
            const float4 c = ph32[k];
            pa_r = c.x; pa_i = c.y; pb_r = c.z; pb_i = c.w;
        } else {
            const double4 c = ph64[k];
            pa_r = c.x; pa_i = c.y; pb_r = c.z; pb_i = c.w;
        }
        const double2 cc = c64[k];
        const T d = tanh_t<T>(static_cast<T>(th[k]));
        const T yr = d * pb_r, yi = d * pb_i;
        cbr += yr;
        cbi += yi;
        const T rr = rr0 - cbr, ri = ri0 - cbi;
        // dS/dd = b P + a R + 2 c d
        const T two_d = d + d;
        const T dsr = fma(pb_r, pr, fma(-pb_i, pi, fma(pa_r, rr, fma(-pa_i, ri, two_d * static_cast<T>(cc.x)))));
        const T dsi = fma(pb_r, pi, fma(pb_i, pr, fma(pa_r, ri, fma(pa_i, rr, two_d * static_cast<T>(cc.y)))));
        const T re = fma(Sr, dsr, Si * dsi);
        go[k] = static_cast<float>(gscale * re * (1 - d * d));
        pr = fma(d, pa_r, pr);
        pi = fma(d, pa_i, pi);
    }
}

static qpm_status relax_partials(const Design &d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                                 const RelaxPlan &pl, int64_t ldb, double *part, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>((B + 63) / 64), static_cast<unsigned>((pl.nseg + 3) / 4));
    if (p == QPM_PREC_F32)
        relax_seg_kernel<float><<<grid, 256, 0, s>>>(theta, ldt, B, d.n, d.ph64, d.ph32, d.c64, pl.seg_len, pl.nseg,
                                                     ldb, part);
    else
        relax_seg_kernel<double><<<grid, 256, 0, s>>>(theta, ldt, B, d.n, d.ph64, d.ph32, d.c64, pl.seg_len,
                                                      pl.nseg, ldb, part);
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

QPM_API qpm_status qpm_relax_forward(qpm_design d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                                     float *f, double *S, qpm_stream sv)
{
    clear_error();
    qpm_status st = check_relax(d, p, theta, B, ldt);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(f != nullptr || S != nullptr, QPM_EINVAL, "at least one of f and S must be given");
    hipStream_t s = static_cast<hipStream_t>(sv);
    const RelaxPlan pl = plan_relax(d->n, B);
    const int64_t ldb = ((B + 63) / 64) * 64;
    double *part = nullptr;
    QPM_TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&part), sizeof(double) * 8 * pl.nseg * ldb, s));
    st = relax_partials(*d, p, theta, B, ldt, pl, ldb, part, s);
    if (st == QPM_OK) {
        relax_combine_kernel<<<static_cast<unsigned>((B + 255) / 256), 256, 0, s>>>(part, pl.nseg, ldb, B, S, f,
                                                                                    nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("relax combine launch failed: %s", hipGetErrorString(e));
            st = QPM_EHIP;
        }
    }
    (void)hipFreeAsync(part, s);
    return st;
}

QPM_API qpm_status qpm_relax_backward(qpm_design d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                                      const double *S, const float *grad_f, float *grad_theta, int64_t ldg,
                                      qpm_stream sv)
{
    clear_error();
    qpm_status st = check_relax(d, p, theta, B, ldt);
    if (st != QPM_OK) return st;
    QPM_REQUIRE(S != nullptr && grad_f != nullptr && grad_theta != nullptr, QPM_EINVAL,
                "S, grad_f and grad_theta must not be NULL");
    QPM_REQUIRE(ldg >= d->n, QPM_EINVAL, "ldg (%lld) must be >= n_domains", (long long)ldg);
    hipStream_t s = static_cast<hipStream_t>(sv);
    const RelaxPlan pl = plan_relax(d->n, B);
    const int64_t ldb = ((B + 63) / 64) * 64;
    double *part = nullptr, *edges = nullptr;
    QPM_TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&part), sizeof(double) * 12 * pl.nseg * ldb, s));
    edges = part + static_cast<int64_t>(8) * pl.nseg * ldb;
    st = relax_partials(*d, p, theta, B, ldt, pl, ldb, part, s);
    if (st == QPM_OK) {
        relax_combine_kernel<<<static_cast<unsigned>((B + 255) / 256), 256, 0, s>>>(part, pl.nseg, ldb, B, nullptr,
                                                                                    nullptr, edges);
        const dim3 grid(static_cast<unsigned>((B + 63) / 64), static_cast<unsigned>((pl.nseg + 3) / 4));
        if (p == QPM_PREC_F32)
            relax_grad_kernel<float><<<grid, 256, 0, s>>>(theta, ldt, B, d->n, d->ph64, d->ph32, d->c64, pl.seg_len,
                                                          pl.nseg, ldb, part, edges, S, grad_f, grad_theta, ldg);
        else
            relax_grad_kernel<double><<<grid, 256, 0, s>>>(theta, ldt, B, d->n, d->ph64, d->ph32, d->c64,
                                                           pl.seg_len, pl.nseg, ldb, part, edges, S, grad_f,
                                                           grad_theta, ldg);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("relax adjoint launch failed: %s", hipGetErrorString(e));
            st = QPM_EHIP;
        }
    }
    (void)hipFreeAsync(part, s);
    return st;
}
