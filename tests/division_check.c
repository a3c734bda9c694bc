/* The pivot-row quotient of the block-tile kernel, on the CPU: with
 * y = 1.0 / b (IEEE), q = x * y, r = fma(-b, q, x), p = fma(r, y, q) must equal
 * x / b whenever |x| and |b| lie in [2^-500, 2^500] (Markstein's theorem);
 * x = 0 takes the product q.  Prints the number of mismatches. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static uint64_t st[2] = {0x243f6a8885a308d3ULL, 0x13198a2e03707344ULL};
static uint64_t next(void) {
    uint64_t s1 = st[0];
    const uint64_t s0 = st[1];
    st[0] = s0;
    s1 ^= s1 << 23;
    st[1] = s1 ^ s0 ^ (s1 >> 17) ^ (s0 >> 26);
    return st[1] + s0;
}
static double mk(uint64_t mant, int e, int sign) {
    uint64_t b = ((uint64_t)sign << 63) | ((uint64_t)(e + 1023) << 52) | (mant & ((1ULL << 52) - 1));
    double d;
    memcpy(&d, &b, 8);
    return d;
}
static double quot(double x, double b) {
    const double y = 1.0 / b, q = x * y;
    if (x == 0.0) return q;
    return fma(fma(-b, q, x), y, q);
}
static int differs(double x, double b) {
    const double p = quot(x, b), t = x / b;
    return memcmp(&p, &t, 8) != 0;
}
int main(int argc, char** argv) {
    const long n = argc > 1 ? atol(argv[1]) : 20000000L;
    long bad = 0, cnt = 0;
    for (long i = 0; i < n; ++i) {
        const uint64_t u = next(), v = next(), w = next();
        const int ex = (int)(w % 1000) - 500, eb = (int)((w >> 16) % 1000) - 500;
        double x = mk(u, ex, (int)(v & 1)), b = mk(v >> 1, eb, (int)(u >> 63));
        switch ((w >> 40) % 8) {
            case 0: b = mk((1ULL << 52) - 1, eb, 0); break;              /* all-ones significand */
            case 1: b = mk(0, eb, 1); break;                              /* power of two */
            case 2: x = mk((1ULL << 52) - 1 - (w >> 60), ex, 0); break;
            case 3: x = b * (double)(w % 1000 + 1); break;                /* exact quotients */
            case 4: x = nextafter(b * (double)(w % 97 + 1), 0.0); break;  /* one ulp off */
            default: break;
        }
        if (fabs(b) < 0x1p-500 || fabs(b) > 0x1p500 || fabs(x) > 0x1p500 || (x != 0.0 && fabs(x) < 0x1p-500)) continue;
        bad += differs(x, b);
        ++cnt;
    }
    /* small integer and rational data like the workloads' tableaux, and zeros of both signs */
    for (int a = -2000; a <= 2000; ++a)
        for (int c = -200; c <= 200; ++c)
            if (c) {
                bad += differs((double)a, (double)c) + differs(a / 7.0, c / 3.0) + differs(-0.0, c / 3.0);
                cnt += 3;
            }
    printf("%ld %ld\n", cnt, bad);
    return 0;
}
