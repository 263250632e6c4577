/*
 * Memory-safety check of the oracle (test infrastructure): built with
 * -fsanitize=address,undefined by tests/test_oracle_sanitize.py and run as a
 * child process.  It round-trips seeded inputs over dtypes, parameters and
 * policies (with and without an XOR base), then decodes containers with
 * flipped bytes and truncations: every call must return normally (an error
 * code or some output), and the sanitizers must report nothing.  Prints
 * "ok <count>" at the end.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "zipnn_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{
    /* xorshift64* (Vigna, 2016) */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 2685821657736338717ull) >> 32);
}

static void fill(uint8_t* x, uint64_t nb, int kind)
{
    for (uint64_t i = 0; i < nb; i++) {
        uint32_t r = rnd();
        if (kind == 0) x[i] = (uint8_t)r;                                  /* uniform */
        else if (kind == 1) x[i] = (r % 20 == 0) ? (uint8_t)(r >> 8) : 0;  /* sparse */
        else x[i] = (uint8_t)(0x38 + (r % 7));                             /* few values */
    }
}

int main(void)
{
    const int dtypes[] = {ORC_BF16, ORC_FP16, ORC_FP32, ORC_FP8_E4M3, ORC_U8};
    const int widths[] = {2, 2, 4, 1, 1};
    int count = 0;
    for (int it = 0; it < 160; it++) {
        const int di = (int)(rnd() % 5);
        const int dtype = dtypes[di], B = widths[di];
        const uint32_t chunk = 256u << (rnd() % 4);
        const uint32_t E = chunk / (uint32_t)B;
        const uint32_t g = 2u << (rnd() % 3);
        uint32_t S = g << (rnd() % 5);
        while (E / S > 4096) S <<= 1;
        const uint32_t L = 8 + rnd() % 4;
        const uint64_t n = (uint64_t)(rnd() % 4) * E + (rnd() % 5);
        uint8_t policy[4];
        for (int k = 0; k < 4; k++) policy[k] = (uint8_t)(rnd() % 4);
        const uint64_t nb = n * (uint64_t)B;
        uint8_t* x = (uint8_t*)malloc(nb + 1);
        uint8_t* base = (rnd() & 1) ? (uint8_t*)malloc(nb + 1) : NULL;
        fill(x, nb, (int)(rnd() % 3));
        if (base) fill(base, nb, 0);
        const uint64_t cap = orc_compress_bound(dtype, n, chunk, S);
        uint8_t* c = (uint8_t*)malloc(cap + 1);
        uint64_t clen = 0;
        const uint32_t skip = rnd() % 4;
        const int exp = (dtype == ORC_BF16 || dtype == ORC_FP32) ? (int)(rnd() & 1) : 0;
        if (orc_compress(x, dtype, n, base, chunk, S, g, L, policy, skip, exp, c, cap, &clen, 2) != ORC_OK) {
            printf("compress failed at %d\n", it);
            return 1;
        }
        uint8_t* y = (uint8_t*)malloc(nb + 1);
        if (orc_decompress(c, clen, base, y, nb, 2) != ORC_OK || (nb && memcmp(x, y, nb) != 0)) {
            printf("round trip failed at %d\n", it);
            return 1;
        }
        /* damaged copies: flipped bytes anywhere, then truncations */
        uint8_t* d = (uint8_t*)malloc(clen + 1);
        for (int f = 0; f < 24; f++) {
            memcpy(d, c, clen);
            const uint64_t pos = rnd() % clen;
            d[pos] ^= (uint8_t)(1u << (rnd() % 8));
            (void)orc_decompress(d, clen, base, y, nb, 1);
            count++;
        }
        for (int f = 0; f < 4; f++) {
            const uint64_t len = rnd() % clen;
            (void)orc_decompress(c, len, base, y, nb, 1);
            count++;
        }
        (void)orc_decompress(c, clen, base, y, nb ? nb - 1 : 0, 1);   /* output too small */
        free(d);
        free(y);
        free(c);
        free(base);
        free(x);
        count++;
    }
    printf("ok %d\n", count);
    return 0;
}
