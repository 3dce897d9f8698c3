/* Exhaustive check of the division-free x / 3 used by the grey-wolf kernel:
 * for every finite binary32 x, copysign(fma(fma(-q0, 3, x), c, q0), x) with
 * q0 = x * c and c = RN(1/3) equals the IEEE quotient x / 3 bit for bit,
 * and so does fma(fma(-q0, 3, x), c, q0) without the copysign for every
 * x != 0. Prints the number of mismatches. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

int main(void)
{
    const float c = 0x1.555556p-2f;
    unsigned long long bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static)
    for (long long b = 0; b < (1LL << 32); ++b) {
        uint32_t u = (uint32_t)b;
        float x;
        memcpy(&x, &u, 4);
        if (!isfinite(x)) continue;
        float ref = x / 3.0f;
        float q0 = x * c;
        float r = fmaf(-q0, 3.0f, x);
        float q = copysignf(fmaf(r, c, q0), x);
        float q2 = fmaf(r, c, q0);
        uint32_t a, d, d2;
        memcpy(&a, &ref, 4);
        memcpy(&d, &q, 4);
        memcpy(&d2, &q2, 4);
        if (a != d) ++bad;
        if (x != 0.0f && a != d2) ++bad;
    }
    printf("%llu\n", bad);
    return 0;
}
