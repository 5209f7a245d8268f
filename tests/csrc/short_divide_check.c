/*
 * Exhaustive check of the interpreter's short divide over every numerator
 * significand, for a given list of divisor significands.
 *
 * The short form computes, in IEEE binary32 with round to nearest even:
 *   y  = the correctly rounded 1/b
 *   q  = a * y
 *   r  = fma(-b, q, a)
 *   q1 = fma(r, y, q)
 * and must equal the correctly rounded a / b.  Markstein's theorem covers the
 * case where q is within one ulp of a/b; q = RN(a * RN(1/b)) can be up to 1.5
 * ulp away, so this check runs every numerator significand A in [1, 2)
 * (2^23 values) against each divisor significand B in [1, 2).  Scaling a or
 * b by a power of two scales q, r and q1 exactly while no step leaves the
 * normal range (which the interpreter's range checks guarantee), so the
 * pairs (A, B) cover every numerator for these divisors.
 *
 * Input: divisor bit patterns (one decimal uint32 per line, b in [1, 2)) on
 * stdin.  Output: one line "divisors N pairs P beyond_one_ulp U mismatches M"
 * and, for the first mismatches, the pair.  Exit status 1 on any mismatch.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -mfma (no FMA contraction of
 * a * y: every operation rounds once, as on the GPU).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

static float from_bits(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

static uint32_t to_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

int main(void)
{
    uint32_t bb;
    long long divisors = 0, pairs = 0, beyond = 0, bad = 0;
    while (scanf("%u", &bb) == 1) {
        const float b = from_bits(bb);
        if (!(b >= 1.0f && b < 2.0f)) {
            fprintf(stderr, "divisor %u not in [1, 2)\n", bb);
            return 2;
        }
        const float y = 1.0f / b;
        ++divisors;
        for (uint32_t m = 0; m < (1u << 23); ++m) {
            const float a = from_bits(0x3f800000u | m);
            const float q = a * y;
            const float r = fmaf(-b, q, a);
            const float q1 = fmaf(r, y, q);
            const float want = a / b;
            /* more than one ulp of the quotient between q and the exact a/b:
               |q - a/b| > ulp  <=>  |b*q - a| > ulp * b, exact in double */
            const double ulp = ldexp(1.0, ilogb(want) - 23);
            if (fabs((double)b * (double)q - (double)a) > ulp * (double)b) ++beyond;
            ++pairs;
            if (to_bits(q1) != to_bits(want)) {
                if (bad < 10) printf("mismatch a=%08x b=%08x q1=%08x want=%08x\n", to_bits(a), bb, to_bits(q1),
                                     to_bits(want));
                ++bad;
            }
        }
    }
    printf("divisors %lld pairs %lld beyond_one_ulp %lld mismatches %lld\n", divisors, pairs, beyond, bad);
    return bad ? 1 : 0;
}
