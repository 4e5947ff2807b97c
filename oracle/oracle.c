/*
 * CPU oracle for the exact product of two decimal integers held as
 * little-endian base-10^19 limbs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU library.
 *
 * Two independent implementations of the same exact result:
 *
 *   O1  oracle_schoolbook  -- the plain definition of the product
 *       (Section 3.2: z = x*y for x = <<x_0..x_{n-1}>>, y = <<y_0..y_{m-1}>>),
 *       computed row by row in base 10^19 with 128-bit intermediates.
 *
 *   O2  oracle_mul_ntt     -- the paper's method taken step by step in its
 *       plainest form: split into base 10^k digit groups (Section 3.2 and the
 *       base choice of Section 4.3), zero-pad to a power of two N >= n+m,
 *       for each of two primes found by FindPrimes (Section 4.5) compute
 *       the transform tau(A, omega) of eq. dft by the recursive radix-2
 *       split into even- and odd-indexed terms (Section 5), multiply
 *       pointwise, transform back with omega^-1 and scale by N^-1
 *       (Section 3.3, eqs. dft/idft and the convolution theorem), recover
 *       each coefficient with the two-prime CRT formula (Section 8.2.2),
 *       then run the carry recurrence sigma/z (Section 3.2, eq.
 *       sigmai_and_zi) and regroup into base 10^19.
 *       Modular products use the naive reduction of Section 4.4.1 (a
 *       128-bit product followed by '%'); no Montgomery arithmetic here.
 *
 * Helpers exported for the pin tests: Miller-Rabin with the first 12 primes
 * as bases (Section 4.5), FindPrimesForN / FindPrimes (Section 4.5), the
 * smallest generator of F_p^*, the transform tau(A, omega) itself, and the
 * digit-group choice.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - primes: FindPrimes(w=64, n_min=32, l=2); p1 < p2.
 *   - root of unity: xi_N = g^((p-1)/N) with g the smallest generator.
 *   - digit-group size k: the largest k in [1,18] with
 *       (10^k - 1)^2 * min(n_k, m_k) < p1*p2            (strict),
 *     where n_k = ceil(19*na / k), m_k = ceil(19*nb / k) count every limb as
 *     19 digits (leading zero digits included).  This is eq. ci_bound used
 *     as the CRT range condition of eq. product_inequality.
 *   - N = the smallest power of two >= n_k + m_k (Section 3.2, padding).
 *   - output: exactly na+nb limbs, leading zero limbs kept.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_EDIGIT (-2)
#define ORACLE_ERANGE (-3)
#define ORACLE_ENOMEM (-4)
#define ORACLE_EINTERNAL (-5)

static const uint64_t LIMB_BASE = 10000000000000000000ULL; /* 10^19 */

/* ------------------------------------------------------------------ */
/* O1: schoolbook product, the plain definition.                        */
/* ------------------------------------------------------------------ */

int oracle_schoolbook(const uint64_t *a, size_t na, const uint64_t *b,
                      size_t nb, uint64_t *out)
{
    size_t i, j;
    for (i = 0; i < na; i++)
        if (a[i] >= LIMB_BASE) return ORACLE_EDIGIT;
    for (j = 0; j < nb; j++)
        if (b[j] >= LIMB_BASE) return ORACLE_EDIGIT;
    memset(out, 0, (na + nb) * sizeof(uint64_t));
    for (i = 0; i < na; i++) {
        uint64_t carry = 0;
        for (j = 0; j < nb; j++) {
            /* out[i+j] + a[i]*b[j] + carry < 10^19 + (10^19-1)^2 + 10^19 < 2^127 */
            u128 t = (u128)a[i] * b[j] + out[i + j] + carry;
            out[i + j] = (uint64_t)(t % LIMB_BASE);
            carry = (uint64_t)(t / LIMB_BASE);
        }
        out[i + nb] = carry;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* Field arithmetic in F_p by naive reduction (Section 4.4.1).          */
/* ------------------------------------------------------------------ */

static uint64_t mulmod(uint64_t x, uint64_t y, uint64_t p)
{
    return (uint64_t)(((u128)x * y) % p);
}

static uint64_t addmod(uint64_t x, uint64_t y, uint64_t p)
{
    u128 s = (u128)x + y;
    return (uint64_t)(s % p);
}

static uint64_t submod(uint64_t x, uint64_t y, uint64_t p)
{
    return x >= y ? x - y : (uint64_t)((u128)x + p - y);
}

static uint64_t powmod(uint64_t x, uint64_t e, uint64_t p)
{
    uint64_t r = 1 % p;
    x %= p;
    while (e) {
        if (e & 1) r = mulmod(r, x, p);
        x = mulmod(x, x, p);
        e >>= 1;
    }
    return r;
}

/* ------------------------------------------------------------------ */
/* Prime search (Section 4.5).                                          */
/* ------------------------------------------------------------------ */

/* Miller-Rabin with the first twelve primes as bases; the paper notes this
 * is a deterministic test below 2^64. */
int oracle_is_prime(uint64_t n)
{
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    uint64_t d;
    int s = 0, i, r;
    if (n < 2) return 0;
    for (i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    d = n - 1;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (i = 0; i < 12; i++) {
        uint64_t x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        for (r = 1; r < s; r++) {
            x = mulmod(x, x, n);
            if (x == n - 1) break;
        }
        if (r == s) return 0;
    }
    return 1;
}

/* FindPrimesForN(n, p_max, l) (Section 4.5): up to l largest primes of the
 * form c*3*2^n + 1 <= p_max with c odd, in decreasing order.  The odd
 * multipliers c are scanned from the largest one allowed downward.
 * Returns how many were written. */
int oracle_find_primes_for_n(int n, uint64_t p_max, int l, uint64_t *res)
{
    int count = 0;
    uint64_t step, c;
    if (n < 0 || n > 62 || p_max < 2) return 0;   /* 3 * 2^62 still fits a word */
    step = 3ULL << n;                          /* p = c * step + 1 */
    c = (p_max - 1) / step;                    /* largest c with p <= p_max */
    if (c % 2 == 0) {
        if (c == 0) return 0;
        c -= 1;                                /* c must be odd */
    }
    for (; count < l; c -= 2) {
        uint64_t p = c * step + 1;
        if (oracle_is_prime(p)) res[count++] = p;
        if (c < 3) break;                      /* c = 1 was the last odd multiplier */
    }
    return count;
}

/* FindPrimes(w, n_min, l): the l largest primes c*3*2^n+1 < 2^(w-1) with
 * n >= n_min and c odd, written in increasing order (p1 < p2 < ...).
 * Returns l on success, ORACLE_ERANGE if fewer exist. */
int oracle_find_primes(int w, int n_min, int l, uint64_t *out)
{
    uint64_t p_max, cand[64 * 8];
    int total = 0, n, i, j;
    if (w < 4 || w > 64 || l < 1 || l > 8) return ORACLE_EINVAL;
    p_max = (w == 64) ? 0x7fffffffffffffffULL : ((1ULL << (w - 1)) - 1);
    for (n = n_min; n <= w - 2; n++)
        total += oracle_find_primes_for_n(n, p_max, l, cand + total);
    if (total < l) return ORACLE_ERANGE;
    /* The same prime cannot appear for two values of n: c odd makes the
     * representation unique.  Sort descending and keep the l largest. */
    for (i = 0; i < total; i++)
        for (j = i + 1; j < total; j++)
            if (cand[j] > cand[i]) { uint64_t t = cand[i]; cand[i] = cand[j]; cand[j] = t; }
    for (i = 0; i < l; i++) out[i] = cand[l - 1 - i];
    return l;
}

/* Smallest generator of the multiplicative group F_p^*: the least g with
 * g^((p-1)/q) != 1 for every prime q dividing p-1.  The factorisation of
 * p-1 is found by trial division. */
uint64_t oracle_generator(uint64_t p)
{
    uint64_t q[64], m = p - 1, d, g;
    int nq = 0, i;
    for (d = 2; d * d <= m; d += (d == 2 ? 1 : 2)) {
        if (m % d == 0) {
            q[nq++] = d;
            while (m % d == 0) m /= d;
        }
    }
    if (m > 1) q[nq++] = m;
    for (g = 2; g < p; g++) {
        int ok = 1;
        for (i = 0; i < nq; i++)
            if (powmod(g, (p - 1) / q[i], p) == 1) { ok = 0; break; }
        if (ok) return g;
    }
    return 0;
}

/* The two primes of the method, computed once. */
static uint64_t g_p[2], g_gen[2];
static int g_init = 0;

static int init_primes(void)
{
    if (g_init) return ORACLE_OK;
    if (oracle_find_primes(64, 32, 2, g_p) != 2) return ORACLE_EINTERNAL;
    g_gen[0] = oracle_generator(g_p[0]);
    g_gen[1] = oracle_generator(g_p[1]);
    if (!g_gen[0] || !g_gen[1]) return ORACLE_EINTERNAL;
    g_init = 1;
    return ORACLE_OK;
}

int oracle_primes(uint64_t *p, uint64_t *g)
{
    int rc = init_primes();
    if (rc) return rc;
    p[0] = g_p[0]; p[1] = g_p[1];
    g[0] = g_gen[0]; g[1] = g_gen[1];
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* The transform tau(A, omega) (Section 5, eq. dft): A'[k] =            */
/* sum_i A[i] omega^(ik), by the radix-2 split of the sum into its      */
/* even- and odd-indexed terms.                                         */
/* ------------------------------------------------------------------ */

/* out[k], k < len, = sum_t in[t*stride] * w^(t*k), w a primitive len-th
 * root of unity, len a power of two.  With E and O the transforms of the
 * even and odd terms (length len/2, root w^2):
 *   out[k] = E[k] + w^k O[k],  out[k + len/2] = E[k] - w^k O[k]. */
static void dft_split(const uint64_t *in, size_t stride, uint64_t *out, size_t len,
                      uint64_t w, uint64_t p)
{
    size_t h = len / 2, k;
    uint64_t wk = 1, w2;
    if (len == 1) {
        out[0] = in[0];
        return;
    }
    w2 = mulmod(w, w, p);
    dft_split(in, 2 * stride, out, h, w2, p);              /* E in out[0, h)   */
    dft_split(in + stride, 2 * stride, out + h, h, w2, p); /* O in out[h, len) */
    for (k = 0; k < h; k++) {
        uint64_t e = out[k];
        uint64_t o = mulmod(wk, out[k + h], p);
        out[k] = addmod(e, o, p);
        out[k + h] = submod(e, o, p);
        wk = mulmod(wk, w, p);
    }
}

/* A'[k] = sum_i A[i] omega^(ik) for len a power of two and omega a
 * primitive len-th root of unity mod p; in place (through a copy). */
int oracle_transform(uint64_t *A, size_t len, uint64_t p, uint64_t omega)
{
    uint64_t *copy;
    if (len == 0 || (len & (len - 1))) return ORACLE_EINVAL;
    copy = malloc(len * sizeof(uint64_t));
    if (!copy) return ORACLE_ENOMEM;
    memcpy(copy, A, len * sizeof(uint64_t));
    dft_split(copy, 1, A, len, omega, p);
    free(copy);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* Decimal digit handling: limbs <-> digits <-> base-10^k groups.       */
/* ------------------------------------------------------------------ */

static void limbs_to_digits(const uint64_t *x, size_t n, uint8_t *d)
{
    size_t i;
    int t;
    for (i = 0; i < n; i++) {
        uint64_t v = x[i];
        for (t = 0; t < 19; t++) { d[19 * i + t] = (uint8_t)(v % 10); v /= 10; }
    }
}

static void digits_to_groups(const uint8_t *d, size_t nd, int k, uint64_t *g, size_t ng)
{
    size_t i;
    int t;
    for (i = 0; i < ng; i++) {
        uint64_t v = 0;
        for (t = k - 1; t >= 0; t--) {
            size_t pos = i * (size_t)k + (size_t)t;
            v = v * 10 + (pos < nd ? d[pos] : 0);
        }
        g[i] = v;
    }
}

static uint64_t pow10u(int e)
{
    uint64_t r = 1;
    while (e-- > 0) r *= 10;
    return r;
}

/* The product of the two primes as a 128-bit integer. */
static u128 prime_product(void)
{
    return (u128)g_p[0] * g_p[1];
}

/* Digit-group size for operands of na and nb limbs: the largest k in
 * [1,18] with (10^k-1)^2 * min(n_k, m_k) < p1*p2, or 0 if none fits.
 * If force_k is nonzero only that k is tried. */
int oracle_choose_k(size_t na, size_t nb, int force_k)
{
    int k;
    u128 P;
    if (init_primes()) return 0;
    P = prime_product();
    for (k = 18; k >= 1; k--) {
        size_t nk, mk, mn;
        u128 L;
        if (force_k && k != force_k) continue;
        nk = (19 * na + (size_t)k - 1) / (size_t)k;
        mk = (19 * nb + (size_t)k - 1) / (size_t)k;
        mn = nk < mk ? nk : mk;
        L = (u128)(pow10u(k) - 1) * (pow10u(k) - 1);
        /* L * mn < P  <=>  L <= (P-1) / mn, avoiding 128-bit overflow. */
        if (mn == 0 || L <= (P - 1) / mn) return k;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* O2: the product by the two-prime NTT.                                */
/* ------------------------------------------------------------------ */

typedef struct {
    int k;            /* digit-group size used */
    uint64_t n;       /* groups in a */
    uint64_t m;       /* groups in b */
    uint64_t N;       /* transform length */
    uint64_t p1, p2;  /* primes */
} oracle_info;

int oracle_mul_ntt(const uint64_t *a, size_t na, const uint64_t *b, size_t nb,
                   uint64_t *out, int force_k, oracle_info *info)
{
    int rc = init_primes(), k, j, bits;
    size_t n, m, N, i, nd_a, nd_b, nd_out, ng_out;
    uint8_t *da = NULL, *db = NULL, *dz = NULL;
    uint64_t *x[2] = {NULL, NULL}, *y[2] = {NULL, NULL}, *z = NULL;
    u128 sigma;
    uint64_t B, r;

    if (rc) return rc;
    if ((na && !a) || (nb && !b) || !out) return ORACLE_EINVAL;
    for (i = 0; i < na; i++) if (a[i] >= LIMB_BASE) return ORACLE_EDIGIT;
    for (i = 0; i < nb; i++) if (b[i] >= LIMB_BASE) return ORACLE_EDIGIT;
    if (force_k < 0 || force_k > 18) return ORACLE_EINVAL;
    if (na == 0 || nb == 0) {
        memset(out, 0, (na + nb) * sizeof(uint64_t));
        if (info) memset(info, 0, sizeof(*info));
        return ORACLE_OK;
    }
    k = oracle_choose_k(na, nb, force_k);
    if (k == 0) return ORACLE_ERANGE;
    B = pow10u(k);
    nd_a = 19 * na;
    nd_b = 19 * nb;
    n = (nd_a + (size_t)k - 1) / (size_t)k;
    m = (nd_b + (size_t)k - 1) / (size_t)k;
    N = 1;
    bits = 0;
    while (N < n + m) { N <<= 1; bits++; }
    if (bits > 32) return ORACLE_ERANGE;   /* 2^32 divides p-1 for both primes */
    if (info) {
        info->k = k; info->n = n; info->m = m; info->N = N;
        info->p1 = g_p[0]; info->p2 = g_p[1];
    }

    da = malloc(nd_a);
    db = malloc(nd_b);
    for (j = 0; j < 2; j++) {
        x[j] = calloc(N, sizeof(uint64_t));
        y[j] = calloc(N, sizeof(uint64_t));
    }
    z = malloc((n + m) * sizeof(uint64_t));
    if (!da || !db || !x[0] || !x[1] || !y[0] || !y[1] || !z) { rc = ORACLE_ENOMEM; goto done; }

    /* Split into base-10^k groups; zero padding up to N (Section 3.2). */
    limbs_to_digits(a, na, da);
    limbs_to_digits(b, nb, db);
    digits_to_groups(da, nd_a, k, x[0], n);
    digits_to_groups(db, nd_b, k, y[0], m);
    memcpy(x[1], x[0], n * sizeof(uint64_t));
    memcpy(y[1], y[0], m * sizeof(uint64_t));

    /* Cyclic convolution modulo each prime by the convolution theorem. */
    for (j = 0; j < 2; j++) {
        uint64_t p = g_p[j];
        uint64_t xi = powmod(g_gen[j], (p - 1) / N, p);   /* primitive N-th root */
        uint64_t xi_inv = powmod(xi, p - 2, p);
        uint64_t n_inv = powmod(N % p, p - 2, p);
        if (oracle_transform(x[j], N, p, xi) || oracle_transform(y[j], N, p, xi)) {
            rc = ORACLE_ENOMEM;
            goto done;
        }
        for (i = 0; i < N; i++) x[j][i] = mulmod(x[j][i], y[j][i], p);
        if (oracle_transform(x[j], N, p, xi_inv)) { rc = ORACLE_ENOMEM; goto done; }
        for (i = 0; i < N; i++) x[j][i] = mulmod(x[j][i], n_inv, p);
    }

    /* CRT (Section 8.2.2): c = a1 + p1 * ((r * (a2 - a1)) mod p2),
     * r = p1^-1 mod p2; then the carry recurrence (Section 3.2). */
    r = powmod(g_p[0] % g_p[1], g_p[1] - 2, g_p[1]);
    sigma = 0;
    for (i = 0; i < n + m; i++) {
        uint64_t a1 = x[0][i], a2 = x[1][i];
        uint64_t a1m = a1 % g_p[1];
        uint64_t t = mulmod(r, submod(a2, a1m, g_p[1]), g_p[1]);
        u128 c = (u128)a1 + (u128)g_p[0] * t;
        u128 s = sigma + c;
        z[i] = (uint64_t)(s % B);
        sigma = s / B;
    }
    /* The coefficients past n+m must vanish and the final carry must be 0:
     * otherwise the convolution bound was violated. */
    for (i = n + m; i < N; i++)
        if (x[0][i] != 0 || x[1][i] != 0) { rc = ORACLE_EINTERNAL; goto done; }
    if (sigma != 0) { rc = ORACLE_EINTERNAL; goto done; }

    /* Regroup base-10^k digits into base-10^19 limbs. */
    nd_out = 19 * (na + nb);
    ng_out = n + m;
    dz = calloc(ng_out * (size_t)k > nd_out ? ng_out * (size_t)k : nd_out, 1);
    if (!dz) { rc = ORACLE_ENOMEM; goto done; }
    for (i = 0; i < ng_out; i++) {
        uint64_t v = z[i];
        int t;
        for (t = 0; t < k; t++) { dz[i * (size_t)k + (size_t)t] = (uint8_t)(v % 10); v /= 10; }
    }
    for (i = nd_out; i < ng_out * (size_t)k; i++)
        if (dz[i] != 0) { rc = ORACLE_EINTERNAL; goto done; }
    for (i = 0; i < na + nb; i++) {
        uint64_t v = 0;
        int t;
        for (t = 18; t >= 0; t--) v = v * 10 + dz[19 * i + (size_t)t];
        out[i] = v;
    }
    rc = ORACLE_OK;
done:
    free(da); free(db); free(dz); free(z);
    for (j = 0; j < 2; j++) { free(x[j]); free(y[j]); }
    return rc;
}

/* Cyclic convolution (eq. star) over Z of two length-n sequences with
 * 128-bit results split into (lo, hi) words -- the O(n^2) definition used
 * to pin the transform-based convolution on small inputs. */
void oracle_cyclic_convolution(const uint64_t *x, const uint64_t *y, size_t n,
                               uint64_t *lo, uint64_t *hi)
{
    size_t k, i;
    for (k = 0; k < n; k++) {
        u128 s = 0;
        for (i = 0; i < n; i++) s += (u128)x[i] * y[(k + n - i) % n];
        lo[k] = (uint64_t)s;
        hi[k] = (uint64_t)(s >> 64);
    }
}
