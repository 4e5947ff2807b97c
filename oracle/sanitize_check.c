/*
 * Sanitizer run of the CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Built together with oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitized.py, this driver
 * exercises every oracle entry point on small inputs: both products (O1
 * and O2) on random and all-(10^19 - 1) operands of many sizes including
 * empty ones and every forced k, the prime search, the transform against
 * the O(N^2) DFT definition, and the error paths.  It exits non-zero on
 * any disagreement; the sanitizers abort on any memory or UB error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

typedef struct {
    int k;
    uint64_t n, m, N, p1, p2;
} oracle_info;

int oracle_schoolbook(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out);
int oracle_mul_ntt(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out,
                   int force_k, oracle_info *info);
int oracle_find_primes(int w, int n_min, int l, uint64_t *out);
int oracle_primes(uint64_t *p, uint64_t *g);
int oracle_transform(uint64_t *A, size_t len, uint64_t p, uint64_t omega);

static uint64_t rng_state = 0x243F6A8885A308D3ULL;
static uint64_t next_u64(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

static uint64_t powm(uint64_t x, uint64_t e, uint64_t p)
{
    uint64_t r = 1;
    x %= p;
    while (e) {
        if (e & 1) r = (uint64_t)((u128)r * x % p);
        x = (uint64_t)((u128)x * x % p);
        e >>= 1;
    }
    return r;
}

static int check_products(size_t na, size_t nb, int nines)
{
    uint64_t *a = malloc((na + 1) * 8), *b = malloc((nb + 1) * 8);
    uint64_t *z1 = malloc((na + nb + 1) * 8), *z2 = malloc((na + nb + 1) * 8);
    size_t i;
    int k, bad = 0;
    for (i = 0; i < na; i++) a[i] = nines ? 9999999999999999999ULL : next_u64() % 10000000000000000000ULL;
    for (i = 0; i < nb; i++) b[i] = nines ? 9999999999999999999ULL : next_u64() % 10000000000000000000ULL;
    if (oracle_schoolbook(a, na, b, nb, z1) != 0) bad = 1;
    if (!bad && oracle_mul_ntt(a, na, b, nb, z2, 0, NULL) != 0) bad = 2;
    if (!bad && memcmp(z1, z2, (na + nb) * 8) != 0) bad = 3;
    for (k = 13; k <= 18 && !bad && na && nb && na < 64 && nb < 64; k++) {
        oracle_info info;
        const int rc = oracle_mul_ntt(a, na, b, nb, z2, k, &info);
        if (rc == 0 && memcmp(z1, z2, (na + nb) * 8) != 0) bad = 4;
    }
    if (bad) fprintf(stderr, "products %zu x %zu (nines %d): failure %d\n", na, nb, nines, bad);
    free(a); free(b); free(z1); free(z2);
    return bad;
}

int main(void)
{
    static const size_t sizes[][2] = {{0, 0}, {0, 3}, {3, 0}, {1, 1}, {1, 2}, {2, 1}, {7, 7}, {17, 31},
                                      {80, 80}, {81, 81}, {100, 1}, {255, 257}, {600, 450}};
    uint64_t p[2], g[2], q[2], A[64], B[64];
    size_t i, j, s;
    int fails = 0;
    for (s = 0; s < sizeof sizes / sizeof sizes[0]; s++) {
        fails += check_products(sizes[s][0], sizes[s][1], 0) != 0;
        fails += check_products(sizes[s][0], sizes[s][1], 1) != 0;
    }
    if (oracle_primes(p, g) != 0 || oracle_find_primes(64, 32, 2, q) != 2 || q[0] != p[0] || q[1] != p[1]) {
        fprintf(stderr, "primes\n");
        fails++;
    }
    if (oracle_find_primes(63, 32, 2, q) != 2 || q[0] >= q[1] || q[1] >= (1ULL << 62)) {
        fprintf(stderr, "primes below 2^62\n");
        fails++;
    }
    for (i = 0; i < 2; i++) {
        const uint64_t w = powm(g[i], (p[i] - 1) / 64, p[i]);
        for (j = 0; j < 64; j++) A[j] = next_u64() % p[i];
        memcpy(B, A, sizeof A);
        if (oracle_transform(B, 64, p[i], w) != 0) fails++;
        for (j = 0; j < 64; j++) {
            uint64_t acc = 0;
            size_t t;
            for (t = 0; t < 64; t++)
                acc = (uint64_t)(((u128)acc + (u128)A[t] * powm(w, (t * j) % 64, p[i])) % p[i]);
            if (acc != B[j]) {
                fprintf(stderr, "transform prime %zu point %zu\n", i, j);
                fails++;
                break;
            }
        }
    }
    {
        uint64_t bad[2] = {10000000000000000000ULL, 1}, z[4];
        if (oracle_schoolbook(bad, 2, bad, 2, z) == 0 || oracle_mul_ntt(bad, 2, bad, 2, z, 0, NULL) == 0 ||
            oracle_transform(A, 48, p[0], 1) == 0) {
            fprintf(stderr, "error paths\n");
            fails++;
        }
    }
    printf("oracle sanitizer run: %d failure(s)\n", fails);
    return fails ? 1 : 0;
}
