// Host check of the kernels' division by host-computed multipliers (DivM, fdiv): for every
// divisor given and a spread of dividends, fdiv(n, div_magic(d)) must equal n / d. Prints the
// number of (n, d) pairs checked, or the first mismatch (exit status 1).
#include <stdio.h>
#include <stdlib.h>

#include "pgm_internal.h"

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32()
{   // xorshift64*: any spread of 32-bit values will do
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (uint32_t)((state * 0x2545F4914F6CDD1Dull) >> 32);
}

static int check(uint32_t d, long long& n_checked)
{
    const pgm::DivM m = pgm::div_magic(d);
    uint32_t ns[64] = {0u, 1u, d - 1u, d, d + 1u, 2u * d - 1u, 2u * d, 0xFFFFFFFFu, 0xFFFFFFFEu,
                       0xFFFFFFFFu / d * d, 0xFFFFFFFFu / d * d - 1u};
    int k = 11;
    while (k < 40) ns[k++] = next_u32();
    while (k < 64) ns[k++] = next_u32() >> (next_u32() & 31);
    for (int i = 0; i < 64; i++) {
        const uint32_t n = ns[i];
        if (pgm::fdiv(n, m) != n / d) {
            printf("mismatch: n=%u d=%u got %u want %u\n", n, d, pgm::fdiv(n, m), n / d);
            return 1;
        }
        n_checked++;
    }
    return 0;
}

int main()
{
    long long n_checked = 0;
    for (uint32_t d = 1; d <= 70000; d++)
        if (check(d, n_checked)) return 1;
    for (int b = 1; b < 32; b++)
        for (int e = -2; e <= 2; e++) {
            const uint32_t d = (uint32_t)((1ull << b) + e);
            if (d >= 1 && check(d, n_checked)) return 1;
        }
    for (int i = 0; i < 200000; i++) {
        const uint32_t d = next_u32();
        if (d >= 1 && check(d, n_checked)) return 1;
    }
    if (check(0xFFFFFFFFu, n_checked) || check(0xFFFFFFFEu, n_checked)) return 1;
    printf("%lld\n", n_checked);
    return 0;
}
