// phases.hip -- qpm_precompute_phases: per-domain integrals of the d_eff
// double integral (paper Sec. 2.1) in FP64 on the GPU.
//
// For domain n on [z_{n-1}, z_n), width w:
//   a_n = e^{-i dk1 z_{n-1}} E(dk1, w),  b_n = e^{-i dk2 z_{n-1}} E(dk2, w),
//   c_n = e^{-i (dk1 + dk2) z_{n-1}} G(dk1, dk2, w),
// with E(k, w) = int_0^w e^{-i k t} dt = w sinc(k w / 2) e^{-i k w / 2} and
// G(k1, k2, w) = int_0^w e^{-i k2 t} E(k1, t) dt
//              = (E(k2, w) - E(k1 + k2, w)) / (i k1)      for |k1 w| >= 1/8,
// and by 16-point Gauss-Legendre panels of the same integrand otherwise
// (where the closed form cancels).
//
// Argument reduction: dk z reaches ~1e5 rad, where one ulp of the rounded
// product is ~1e-11 rad. The product is carried exactly as p + e (e from an
// FMA) and the unit phasor of p is rotated by the small e to first order.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace qpm {

struct GLRule16 {
    double x[16];
    double w[16];
};

// 16-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_16.
static GLRule16 make_gl16()
{
    GLRule16 r;
    const int n = 16;
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double deriv = 0.0;
        for (int it = 0; it < 64; ++it) {
            double pm1 = 1.0, p = t;
            for (int k = 2; k <= n; ++k) {
                double pn = ((2.0 * k - 1.0) * t * p - (k - 1.0) * pm1) / k;
                pm1 = p;
                p = pn;
            }
            deriv = n * (t * p - pm1) / (t * t - 1.0);
            double step = p / deriv;
            t -= step;
            if (std::fabs(step) < 1e-17) break;
        }
        double pm1 = 1.0, p = t;
        for (int k = 2; k <= n; ++k) {
            double pn = ((2.0 * k - 1.0) * t * p - (k - 1.0) * pm1) / k;
            pm1 = p;
            p = pn;
        }
        deriv = n * (t * p - pm1) / (t * t - 1.0);
        r.x[i] = t;
        r.w[i] = 2.0 / ((1.0 - t * t) * deriv * deriv);
    }
    return r;
}

struct Cx {
    double re, im;
};

__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return Cx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// e^{-i k z} with k z carried exactly (p + e)
__device__ __forceinline__ Cx phasor(double k, double z)
{
    const double p = k * z;
    const double e = fma(k, z, -p);
    double sp, cp;
    sincos(p, &sp, &cp);
    const double c = fma(-e, sp, cp);  // cos(p + e)
    const double s = fma(e, cp, sp);   // sin(p + e)
    return Cx{c, -s};
}

__device__ __forceinline__ double sinc(double x)
{
    if (fabs(x) < 1e-4) {
        const double x2 = x * x;
        return 1.0 - x2 * (1.0 / 6.0) + x2 * x2 * (1.0 / 120.0);
    }
    return sin(x) / x;
}

// E(k, w) = w sinc(k w / 2) e^{-i k w / 2}
__device__ __forceinline__ Cx Efun(double k, double w)
{
    const double h = 0.5 * k * w;
    double sh, ch;
    sincos(h, &sh, &ch);
    const double m = w * sinc(h);
    return Cx{m * ch, -m * sh};
}

__device__ Cx Gfun(double k1, double k2, double w, const GLRule16 &gl)
{
    if (fabs(k1 * w) >= 0.125) {
        const Cx e2 = Efun(k2, w), e12 = Efun(k1 + k2, w);
        const double dre = e2.re - e12.re, dim = e2.im - e12.im;
        // (dre + i dim) / (i k1) = (dim - i dre) / k1
        return Cx{dim / k1, -dre / k1};
    }
    const double rate = fabs(k1) + fabs(k2);
    int panels = 1 + static_cast<int>(fmin(rate * w / 0.5, 1.0e6));
    const double h = w / panels;
    Cx acc{0.0, 0.0};
    for (int p = 0; p < panels; ++p) {
        const double mid = (p + 0.5) * h, half = 0.5 * h;
        for (int q = 0; q < 16; ++q) {
            const double t = fma(half, gl.x[q], mid);
            double s2, c2;
            sincos(k2 * t, &s2, &c2);
            const Cx v = cmul(Cx{c2, -s2}, Efun(k1, t));
            acc.re = fma(half * gl.w[q], v.re, acc.re);
            acc.im = fma(half * gl.w[q], v.im, acc.im);
        }
    }
    return acc;
}

__global__ __launch_bounds__(256) void phases_kernel(const double *__restrict__ z, int64_t n, int64_t npad,
                                                     double dk1, double dk2, GLRule16 gl,
                                                     double4 *__restrict__ ph64, float4 *__restrict__ ph32,
                                                     double2 *__restrict__ c64)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i >= n) {
        ph64[i] = make_double4(0.0, 0.0, 0.0, 0.0);
        ph32[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const double lo = z[i], hi = z[i + 1];
    const double w = hi - lo;
    const Cx p1 = phasor(dk1, lo), p2 = phasor(dk2, lo);
    const Cx a = cmul(p1, Efun(dk1, w));
    const Cx b = cmul(p2, Efun(dk2, w));
    const Cx c = cmul(cmul(p1, p2), Gfun(dk1, dk2, w, gl));
    ph64[i] = make_double4(a.re, a.im, b.re, b.im);
    ph32[i] = make_float4(static_cast<float>(a.re), static_cast<float>(a.im), static_cast<float>(b.re),
                          static_cast<float>(b.im));
    c64[i] = make_double2(c.re, c.im);
}

// C = sum_n c_n, one workgroup, fixed order: strided partial sums, then a
// pairwise tree over the 256 partials.
__global__ __launch_bounds__(256) void sum_c_kernel(const double2 *__restrict__ c, int64_t n, double *__restrict__ out)
{
    __shared__ double sre[256], sim[256];
    double re = 0.0, im = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        re += c[i].x;
        im += c[i].y;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(s)) {
            sre[threadIdx.x] += sre[threadIdx.x + s];
            sim[threadIdx.x] += sim[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sre[0];
        out[1] = sim[0];
    }
}

// The 16 sign patterns of each block of 4 domains, reduced to their triple:
// for block q and pattern p (bit k set -> d = -1 for domain 4q + k),
//   A = sum_k d_k a_k,  B = sum_k d_k b_k,  Q = sum_k d_k b_k sum_{m<k} d_m a_m,
// in FP64 from the FP64 integrals (padding domains have a = b = 0). Layout
// [q][A, B, Q][p], one complex value per entry, so the 16 patterns of one
// component are one contiguous row. The fixed-point copy for the FP32
// kernels holds A 2^e and B 2^e rounded to integers and Q 2^(2e) rounded to
// float, e the scale exponent of the block's word (wsc = 2^-e).
__global__ __launch_bounds__(256) void pattern_table_kernel(const double4 *__restrict__ ph64, int64_t nblocks,
                                                            const double *__restrict__ wsc,
                                                            double2 *__restrict__ tab64, int2 *__restrict__ tabq)
{
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (tid >= nblocks * 16) return;
    const int64_t q = tid >> 4;
    const int p = static_cast<int>(tid & 15);
    double ar = 0, ai = 0, br = 0, bi = 0, qr = 0, qi = 0;
    for (int k = 0; k < 4; ++k) {
        const double4 c = ph64[4 * q + k];
        const double sg = ((p >> k) & 1) ? -1.0 : 1.0;
        qr = fma(sg, fma(c.z, ar, -(c.w * ai)), qr);
        qi = fma(sg, fma(c.z, ai, c.w * ar), qi);
        ar = fma(sg, c.x, ar);
        ai = fma(sg, c.y, ai);
        br = fma(sg, c.z, br);
        bi = fma(sg, c.w, bi);
    }
    double2 *o = tab64 + q * 48 + p;
    o[0] = make_double2(ar, ai);
    o[16] = make_double2(br, bi);
    o[32] = make_double2(qr, qi);
    const double up = 1.0 / wsc[q >> 3];  // 2^e, exact
    const double up2 = up * up;
    int2 *f = tabq + q * 48 + p;
    f[0] = make_int2(__double2int_rn(ar * up), __double2int_rn(ai * up));
    f[16] = make_int2(__double2int_rn(br * up), __double2int_rn(bi * up));
    f[32] = make_int2(__float_as_int(static_cast<float>(qr * up2)), __float_as_int(static_cast<float>(qi * up2)));
}

qpm_status launch_pattern_tables(const double4 *ph64, int64_t words, const double *wsc, double2 *tab64, int2 *tabq,
                                 hipStream_t s)
{
    const int64_t nblocks = words * 8;
    pattern_table_kernel<<<static_cast<unsigned>((nblocks * 16 + 255) / 256), 256, 0, s>>>(ph64, nblocks, wsc, tab64,
                                                                                           tabq);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

void word_scales(const double *z, int64_t n, double *sc)
{
    const double lim = 2147483648.0 - 64.0;  // 2^31 - 64
    const int64_t W = words_for(n);
    for (int64_t w = 0; w < W; ++w) {
        const double M = z[std::min<int64_t>(32 * w + 32, n)] - z[32 * w];
        int e = 30 - std::ilogb(M);  // M 2^e < 2^31
        if (std::ldexp(M, e) > lim) --e;
        e = std::min(e, 60);
        sc[w] = std::ldexp(1.0, -e);
    }
}

qpm_status launch_phases(const double *zdev, int64_t n, double dk1, double dk2, double4 *ph64, float4 *ph32,
                         double2 *c64, double *Cdev, hipStream_t s)
{
    static const GLRule16 gl = make_gl16();
    const int64_t npad = words_for(n) * 32;
    const int64_t blocks = (npad + 255) / 256;
    phases_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(zdev, n, npad, dk1, dk2, gl, ph64, ph32,
                                                                           c64);
    QPM_TRY_HIP(hipGetLastError());
    sum_c_kernel<<<1, 256, 0, s>>>(c64, n, Cdev);
    QPM_TRY_HIP(hipGetLastError());
    return QPM_OK;
}

static void free_design(Design *d)
{
    if (!d) return;
    (void)hipFree(d->ph64);
    (void)hipFree(d->ph32);
    (void)hipFree(d->c64);
    (void)hipFree(d->Cdev);
    (void)hipFree(d->tab64);
    (void)hipFree(d->tabq);
    (void)hipFree(d->wsc);
    scratch_cache_destroy(d->scratch);
    delete static_cast<qpm_design_s *>(d);
}

}  // namespace qpm

using namespace qpm;

QPM_API qpm_status qpm_precompute_phases(const double *z, int64_t n, double dk1, double dk2, qpm_stream sv,
                                         qpm_design *out)
{
    clear_error();
    QPM_REQUIRE(z != nullptr && out != nullptr, QPM_EINVAL, "z and out must not be NULL");
    QPM_REQUIRE(n >= 1, QPM_EINVAL, "n_domains must be >= 1 (got %lld)", (long long)n);
    QPM_REQUIRE(n <= (int64_t(1) << 27), QPM_ERANGE, "n_domains %lld exceeds 2^27", (long long)n);
    QPM_REQUIRE(std::isfinite(dk1) && std::isfinite(dk2), QPM_EINVAL, "dk1 and dk2 must be finite");
    for (int64_t i = 0; i <= n; ++i)
        QPM_REQUIRE(std::isfinite(z[i]), QPM_EINVAL, "z[%lld] is not finite", (long long)i);
    for (int64_t i = 0; i < n; ++i)
        QPM_REQUIRE(z[i + 1] > z[i], QPM_EINVAL, "z must be strictly increasing (z[%lld] >= z[%lld])",
                    (long long)i, (long long)(i + 1));
    QPM_REQUIRE(z[n] - z[0] <= 1e100, QPM_EINVAL, "the crystal length z[n] - z[0] must be at most 1e100");
    qpm_status st = check_device();
    if (st != QPM_OK) return st;

    hipStream_t s = static_cast<hipStream_t>(sv);
    auto *d = new qpm_design_s();
    d->n = n;
    d->words = words_for(n);
    d->dk1 = dk1;
    d->dk2 = dk2;
    d->z0 = z[0];
    d->zN = z[n];
    {
        uint64_t h = 1469598103934665603ull;  // FNV-1a, 64 bit
        const unsigned char *bytes = reinterpret_cast<const unsigned char *>(z);
        for (size_t k = 0; k < sizeof(double) * static_cast<size_t>(n + 1); ++k) h = (h ^ bytes[k]) * 1099511628211ull;
        d->zhash = h;
    }
    QPM_TRY_HIP(hipGetDevice(&d->device));
    const int64_t npad = d->words * 32;
    double *zdev = nullptr;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&d->ph64, sizeof(double4) * npad);
    if (e == hipSuccess) e = hipMalloc(&d->ph32, sizeof(float4) * npad);
    if (e == hipSuccess) e = hipMalloc(&d->c64, sizeof(double2) * n);
    if (e == hipSuccess) e = hipMalloc(&d->Cdev, sizeof(double) * 2);
    if (e == hipSuccess) e = hipMalloc(&d->tab64, sizeof(double2) * 48 * 8 * d->words);
    if (e == hipSuccess) e = hipMalloc(&d->tabq, sizeof(int2) * 48 * 8 * d->words);
    if (e == hipSuccess) e = hipMalloc(&d->wsc, sizeof(double) * d->words);
    if (e == hipSuccess) e = hipMalloc(&zdev, sizeof(double) * (n + 1));
    if (e != hipSuccess) {
        (void)hipFree(zdev);
        free_design(d);
        set_error("device allocation for a design of %lld domains failed: %s", (long long)n, hipGetErrorString(e));
        return QPM_ENOMEM;
    }
    std::vector<double> wsc(d->words);
    word_scales(z, n, wsc.data());
    e = hipMemcpyAsync(zdev, z, sizeof(double) * (n + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d->wsc, wsc.data(), sizeof(double) * d->words, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && launch_phases(zdev, n, dk1, dk2, d->ph64, d->ph32, d->c64, d->Cdev, s) != QPM_OK)
        e = hipErrorLaunchFailure;
    if (e == hipSuccess && launch_pattern_tables(d->ph64, d->words, d->wsc, d->tab64, d->tabq, s) != QPM_OK)
        e = hipErrorLaunchFailure;
    if (e == hipSuccess) e = hipMemcpyAsync(d->C, d->Cdev, sizeof(double) * 2, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(zdev);
    if (e != hipSuccess) {
        free_design(d);
        set_error("phase precompute failed: %s", hipGetErrorString(e));
        return QPM_EHIP;
    }
    // the per-call scratch cache (without it every call allocates its own)
    d->scratch = scratch_cache_create();
    *out = d;
    return QPM_OK;
}

QPM_API qpm_status qpm_design_free(qpm_design d)
{
    clear_error();
    if (!d) return QPM_OK;
    (void)hipDeviceSynchronize();
    free_design(d);
    return QPM_OK;
}

QPM_API qpm_status qpm_design_info(qpm_design d, int64_t *n, double *C)
{
    clear_error();
    QPM_REQUIRE(d != nullptr, QPM_EINVAL, "design is NULL");
    if (n) *n = d->n;
    if (C) {
        C[0] = d->C[0];
        C[1] = d->C[1];
    }
    return QPM_OK;
}

QPM_API qpm_status qpm_design_read_phases(qpm_design d, double *a, double *b, double *c)
{
    clear_error();
    QPM_REQUIRE(d != nullptr, QPM_EINVAL, "design is NULL");
    const int64_t n = d->n;
    if (a || b) {
        std::vector<double4> h(n);
        QPM_TRY_HIP(hipMemcpy(h.data(), d->ph64, sizeof(double4) * n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            if (a) { a[2 * i] = h[i].x; a[2 * i + 1] = h[i].y; }
            if (b) { b[2 * i] = h[i].z; b[2 * i + 1] = h[i].w; }
        }
    }
    if (c) QPM_TRY_HIP(hipMemcpy(c, d->c64, sizeof(double2) * n, hipMemcpyDeviceToHost));
    return QPM_OK;
}
