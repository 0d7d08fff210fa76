/*
 * CPU oracle for the exact Catalan-number method of arXiv 2601.11621
 * ("Exact Computation of the Catalan Number C(2,050,572,903)").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * It is deliberately plain and slow:
 *   - primes by trial division (the paper sieves; a different route on purpose),
 *   - exponents by the literal Legendre sums (Sec. 2, Legendre's formula and the
 *     valuation v_p(C(n)) = v_p((2n)!) - 2 v_p(n!) - v_p(n+1)),
 *   - n+1 factored by trial division (Alg. 1, factorisation step),
 *   - groups G_e with primes ascending (Sec. 3.1),
 *   - Q_e by a balanced product tree, P_e = Q_e^e by square-and-multiply and
 *     C(n) = prod_e P_e by a balanced product tree over the P_e (Sec. 3.2, Alg. 2),
 *   - big integers as little-endian uint32 limb vectors, multiplied by
 *     schoolbook below 32 limbs and Karatsuba above.
 * Threads: an optional OpenMP pragma over the independent pairs of one tree level.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-2)
#define ORC_ENOMEM (-3)
#define ORC_EINTERNAL (-5)

#define KARATSUBA_MIN 32

/* Planted-mistake switch, used only by the test that shows the pins catch a
 * wrong oracle: 0 = correct; 1 = drop the v_p(n+1) term; 2 = drop the carry
 * out of each schoolbook row; 3 = use v_p(n!) once instead of twice; 4 = drop
 * the leading zeros of the inner nine-digit groups of the decimal text. */
static int g_fault = 0;
void orc_set_fault(int f) { g_fault = f; }

/* ---------------------------------------------------------------------------
 * Primes <= limit by trial division (Phase 1 input set: all primes p <= 2n).
 * Returns the count; writes at most cap primes.  limit < 2^32.
 * ------------------------------------------------------------------------- */
size_t orc_primes(uint64_t limit, uint32_t *out, size_t cap)
{
    size_t cnt = 0;
    if (!out || cap == 0) return limit >= 2 ? (size_t)-1 : 0;
    if (limit >= 2) {
        out[cnt++] = 2;
    }
    /* trial division of each odd m by the primes q <= sqrt(m) already found */
    for (uint64_t m = 3; m <= limit; m += 2) {
        int is_prime = 1;
        for (size_t k = 1; k < cnt; k++) {
            uint64_t q = out[k];
            if (q * q > m) break;
            if (m % q == 0) { is_prime = 0; break; }
        }
        if (is_prime) {
            if (cnt >= cap) return (size_t)-1; /* caller must size by a bound */
            out[cnt++] = (uint32_t)m;
        }
    }
    return cnt;
}

/* Legendre: v_p(m!) = sum_{k>=1} floor(m / p^k), by repeated division so that
 * no power of p is formed (p may exceed 2^32 / p). */
uint64_t orc_legendre(uint64_t m, uint64_t p)
{
    uint64_t s = 0;
    while (m) { m /= p; s += m; }
    return s;
}

/* Factor n+1 by trial division with the primes q <= sqrt(n+1) (Alg. 1,
 * factorisation step).  A cofactor > 1 left after that is itself a prime of
 * multiplicity one.  Writes (prime, multiplicity) pairs; returns their number. */
static int factor_np1(uint64_t n, const uint32_t *primes, size_t np,
                      uint64_t *fp, uint64_t *fe)
{
    uint64_t m = n + 1;
    int k = 0;
    for (size_t i = 0; i < np; i++) {
        uint64_t q = primes[i];
        if (q * q > m) break;
        if (m % q == 0) {
            uint64_t c = 0;
            while (m % q == 0) { m /= q; c++; }
            fp[k] = q; fe[k] = c; k++;
        }
    }
    if (m > 1) { fp[k] = m; fe[k] = 1; k++; }
    return k;
}

/* Exponent e_p = v_p((2n)!) - 2 v_p(n!) - v_p(n+1) for every prime in the
 * list (Sec. 2, Catalan valuation; Alg. 1, exponent loop).  Returns ORC_EINTERNAL
 * if any exponent is negative (C(n) is an integer, so none may be). */
int orc_exponents(uint64_t n, const uint32_t *primes, size_t np, int32_t *e_out)
{
    uint64_t fp[64], fe[64];
    int nf = factor_np1(n, primes, np, fp, fe);
    for (size_t i = 0; i < np; i++) {
        uint64_t p = primes[i];
        int64_t a = (int64_t)orc_legendre(2 * n, p);
        int64_t b = (int64_t)orc_legendre(n, p);
        int64_t c = 0;
        for (int k = 0; k < nf; k++)
            if (fp[k] == p) c = (int64_t)fe[k];
        int64_t e = (g_fault == 3) ? a - b - c : a - 2 * b - c;
        if (g_fault == 1) e = a - 2 * b;
        if (e < 0) return ORC_EINTERNAL;
        e_out[i] = (int32_t)e;
    }
    return ORC_OK;
}

/* Upper bound on pi(x) (Rosser-Schoenfeld style, generous) for buffer sizing */
size_t orc_pi_bound(uint64_t x)
{
    if (x < 100) return 30;
    double t = (double)x;
    return (size_t)(1.3 * t / log(t)) + 64;  /* pi(x) < 1.25506 x / ln x */
}

/* Groups G_e, e >= 1, exponent ascending, primes ascending inside a group
 * (Sec. 3.1, grouping by exponent).  primes_out needs pi(2n) capacity.
 * exps[g], off[g..g+1] describe group g; at most 64 groups. */
int orc_factor(uint64_t n, uint32_t *primes_out, size_t cap,
               uint32_t *exps, uint64_t *off, uint32_t *n_groups, size_t *n_primes)
{
    if (n > 2147483647ull) return ORC_EINVAL;
    size_t bound = orc_pi_bound(2 * n);
    uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * (bound ? bound : 1));
    int32_t *ex = (int32_t *)malloc(sizeof(int32_t) * (bound ? bound : 1));
    if (!pr || !ex) { free(pr); free(ex); return ORC_ENOMEM; }
    size_t np = orc_primes(2 * n, pr, bound);
    if (np == (size_t)-1) { free(pr); free(ex); return ORC_EINTERNAL; }
    int st = orc_exponents(n, pr, np, ex);
    if (st) { free(pr); free(ex); return st; }
    int32_t emax = 0;
    for (size_t i = 0; i < np; i++) if (ex[i] > emax) emax = ex[i];
    size_t total = 0;
    uint32_t g = 0;
    off[0] = 0;
    for (int32_t e = 1; e <= emax; e++) {
        size_t cnt = 0;
        for (size_t i = 0; i < np; i++) {
            if (ex[i] != e) continue;
            if (total + cnt < cap && primes_out) primes_out[total + cnt] = pr[i];
            cnt++;
        }
        if (cnt == 0) continue;
        exps[g] = (uint32_t)e;
        total += cnt;
        off[g + 1] = total;
        g++;
    }
    free(pr); free(ex);
    *n_groups = g;
    *n_primes = total;
    if (total > cap) return ORC_ERANGE;
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Multiprecision multiply: c[0..la+lb) = a[0..la) * b[0..lb), little-endian
 * uint32 limbs.  c must not alias a or b.
 * ------------------------------------------------------------------------- */
static void schoolbook(const uint32_t *a, size_t la, const uint32_t *b, size_t lb, uint32_t *c)
{
    memset(c, 0, sizeof(uint32_t) * (la + lb));
    for (size_t i = 0; i < la; i++) {
        uint64_t carry = 0;
        for (size_t j = 0; j < lb; j++) {
            uint64_t t = (uint64_t)a[i] * b[j] + c[i + j] + carry;
            c[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        if (g_fault == 2) carry = 0;
        c[i + lb] = (uint32_t)carry;
    }
}

/* r[0..n) += x[0..m), m <= n; returns the carry out of r[n-1] */
static uint32_t add_into(uint32_t *r, size_t n, const uint32_t *x, size_t m)
{
    uint64_t carry = 0;
    size_t i = 0;
    for (; i < m; i++) {
        uint64_t t = (uint64_t)r[i] + x[i] + carry;
        r[i] = (uint32_t)t; carry = t >> 32;
    }
    for (; carry && i < n; i++) {
        uint64_t t = (uint64_t)r[i] + carry;
        r[i] = (uint32_t)t; carry = t >> 32;
    }
    return (uint32_t)carry;
}

/* r[0..n) -= x[0..m), m <= n; the result must be non-negative */
static void sub_from(uint32_t *r, size_t n, const uint32_t *x, size_t m)
{
    int64_t borrow = 0;
    size_t i = 0;
    for (; i < m; i++) {
        int64_t t = (int64_t)r[i] - x[i] - borrow;
        borrow = t < 0; r[i] = (uint32_t)t;
    }
    for (; borrow && i < n; i++) {
        int64_t t = (int64_t)r[i] - borrow;
        borrow = t < 0; r[i] = (uint32_t)t;
    }
}

void orc_mul(const uint32_t *a, size_t la, const uint32_t *b, size_t lb, uint32_t *c);

/* Karatsuba on equal lengths n (>= KARATSUBA_MIN): with a = a0 + a1 B^h,
 * b = b0 + b1 B^h, a*b = z0 + (z1 - z0 - z2) B^h + z2 B^{2h},
 * z0 = a0 b0, z2 = a1 b1, z1 = (a0+a1)(b0+b1).  c has 2n limbs. */
static void karatsuba(const uint32_t *a, const uint32_t *b, size_t n, uint32_t *c)
{
    size_t h = n / 2;          /* low half length */
    size_t hh = n - h;         /* high half length, hh >= h */
    uint32_t *sa = (uint32_t *)calloc(hh + 1, 4);
    uint32_t *sb = (uint32_t *)calloc(hh + 1, 4);
    uint32_t *z1 = (uint32_t *)calloc(2 * hh + 2, 4);
    uint32_t *z0 = (uint32_t *)calloc(2 * h, 4);
    uint32_t *z2 = (uint32_t *)calloc(2 * hh, 4);
    /* sa = a0 + a1, sb = b0 + b1 */
    memcpy(sa, a + h, hh * 4);
    sa[hh] = add_into(sa, hh, a, h);
    memcpy(sb, b + h, hh * 4);
    sb[hh] = add_into(sb, hh, b, h);
    orc_mul(a, h, b, h, z0);
    orc_mul(a + h, hh, b + h, hh, z2);
    orc_mul(sa, hh + 1, sb, hh + 1, z1);
    sub_from(z1, 2 * hh + 2, z0, 2 * h);
    sub_from(z1, 2 * hh + 2, z2, 2 * hh);
    memset(c, 0, 2 * n * 4);
    memcpy(c, z0, 2 * h * 4);
    memcpy(c + 2 * h, z2, 2 * hh * 4);
    /* z1 fits in 2*hh+1 limbs at most and c has room above offset h */
    size_t zl = 2 * hh + 2;
    while (zl > 0 && z1[zl - 1] == 0) zl--;
    add_into(c + h, 2 * n - h, z1, zl);
    free(sa); free(sb); free(z0); free(z1); free(z2);
}

void orc_mul(const uint32_t *a, size_t la, const uint32_t *b, size_t lb, uint32_t *c)
{
    if (la < lb) { const uint32_t *t = a; a = b; b = t; size_t tl = la; la = lb; lb = tl; }
    if (lb == 0) { memset(c, 0, la * 4); return; }
    if (lb < KARATSUBA_MIN) { schoolbook(a, la, b, lb, c); return; }
    if (la == lb) { karatsuba(a, b, la, c); return; }
    /* la > lb: cut a into lb-limb blocks, multiply each by b, add at its offset */
    memset(c, 0, (la + lb) * 4);
    uint32_t *t = (uint32_t *)malloc((2 * lb) * 4);
    for (size_t s = 0; s < la; s += lb) {
        size_t blk = (la - s < lb) ? la - s : lb;
        orc_mul(a + s, blk, b, lb, t);
        add_into(c + s, la + lb - s, t, blk + lb);
    }
    free(t);
}

/* ---------------------------------------------------------------------------
 * Big integers for the tree: owned limb vectors, normalised (no zero top limb,
 * except the value 0 which has length 0).
 * ------------------------------------------------------------------------- */
typedef struct { uint32_t *d; size_t n; } big_t;

static void big_norm(big_t *x) { while (x->n > 0 && x->d[x->n - 1] == 0) x->n--; }

static big_t big_mul(const big_t *x, const big_t *y)
{
    big_t r;
    r.n = x->n + y->n;
    r.d = (uint32_t *)malloc((r.n ? r.n : 1) * 4);
    orc_mul(x->d, x->n, y->d, y->n, r.d);
    big_norm(&r);
    return r;
}

/* Balanced product tree: adjacent pairs (x0 x1, x2 x3, ...), an odd last
 * element carried up unchanged, repeated until one value remains (Sec. 3.2,
 * "operands are recursively paired and multiplied").  Consumes the items. */
static big_t product_tree(big_t *items, size_t cnt)
{
    if (cnt == 0) {
        big_t one; one.d = (uint32_t *)malloc(4); one.d[0] = 1; one.n = 1;
        return one;
    }
    while (cnt > 1) {
        size_t half = cnt / 2;
#pragma omp parallel for schedule(dynamic, 1)
        for (size_t i = 0; i < half; i++) {
            big_t r = big_mul(&items[2 * i], &items[2 * i + 1]);
            free(items[2 * i].d); free(items[2 * i + 1].d);
            items[2 * i] = r;
        }
        for (size_t i = 0; i < half; i++) items[i] = items[2 * i];
        if (cnt & 1) { items[half] = items[cnt - 1]; cnt = half + 1; }
        else cnt = half;
    }
    return items[0];
}

/* Left-to-right binary square-and-multiply: x^e, e >= 1 (Alg. 2, P_e = Q_e^e) */
static big_t big_pow(const big_t *x, uint32_t e)
{
    int top = 31;
    while (top > 0 && !((e >> top) & 1)) top--;
    big_t r; r.n = x->n; r.d = (uint32_t *)malloc((x->n ? x->n : 1) * 4);
    memcpy(r.d, x->d, x->n * 4);
    for (int bit = top - 1; bit >= 0; bit--) {
        big_t s = big_mul(&r, &r);
        free(r.d); r = s;
        if ((e >> bit) & 1) {
            big_t t = big_mul(&r, x);
            free(r.d); r = t;
        }
    }
    return r;
}

/* Reconstruction (Alg. 2): for each exponent group G_e, Q_e = tree(G_e),
 * P_e = Q_e^e; C(n) = tree(P_e in exponent order). */
static int reconstruct(const uint32_t *primes, const uint32_t *exps, const uint64_t *off,
                       uint32_t ng, big_t *out)
{
    big_t *pe = (big_t *)malloc(sizeof(big_t) * (ng ? ng : 1));
    if (!pe) return ORC_ENOMEM;
    for (uint32_t g = 0; g < ng; g++) {
        size_t cnt = (size_t)(off[g + 1] - off[g]);
        big_t *leaves = (big_t *)malloc(sizeof(big_t) * (cnt ? cnt : 1));
        for (size_t i = 0; i < cnt; i++) {
            leaves[i].d = (uint32_t *)malloc(4);
            leaves[i].d[0] = primes[off[g] + i];
            leaves[i].n = 1;
        }
        big_t q = product_tree(leaves, cnt);
        free(leaves);
        if (exps[g] == 1) pe[g] = q;
        else { pe[g] = big_pow(&q, exps[g]); free(q.d); }
    }
    *out = product_tree(pe, ng);
    free(pe);
    return ORC_OK;
}

/* Upper bound on the limb count of C(n): C(n) <= 4^n, so <= 2n+1 bits */
size_t orc_catalan_limbs_bound(uint64_t n) { return (size_t)((2 * n + 1) / 32 + 2); }

/* C(n) = (2n)!/(n!(n+1)!) (Sec. 1) as normalised little-endian uint32 limbs;
 * C(0) = C(1) = {1}.  out == NULL is a size query. */
int orc_catalan(uint64_t n, uint32_t *out, size_t cap, size_t *len)
{
    if (n > 2147483647ull) return ORC_EINVAL;
    size_t bound = orc_pi_bound(2 * n);
    uint32_t *pr = (uint32_t *)malloc(4 * bound);
    uint32_t exps[64];
    uint64_t off[65];
    uint32_t ng = 0;
    size_t np = 0;
    if (!pr) return ORC_ENOMEM;
    int st = orc_factor(n, pr, bound, exps, off, &ng, &np);
    if (st) { free(pr); return st; }
    big_t c;
    st = reconstruct(pr, exps, off, ng, &c);
    free(pr);
    if (st) return st;
    *len = c.n;
    if (out) {
        if (cap < c.n) { free(c.d); return ORC_ERANGE; }
        memcpy(out, c.d, c.n * 4);
    }
    free(c.d);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Factorial ratios N = prod_i a_i! / prod_j b_j! (Sec. 6.3).  The exponent of
 * p is sum_i v_p(a_i!) - sum_j v_p(b_j!) with Legendre's sums; N is the product
 * over the primes p <= max(a_i, b_j) of p^{v_p(N)}, rebuilt as in Alg. 2:
 * groups of equal exponent, Q_e by the balanced tree, P_e = Q_e^e, and the
 * balanced tree over the P_e in exponent order.
 * ------------------------------------------------------------------------- */

/* (p, v_p(N)) for every prime with v_p(N) > 0, p ascending.  ORC_EINVAL for a
 * negative exponent (N not an integer), ORC_ERANGE for an exponent >= 2^32 or
 * more than cap primes.  primes_out == NULL: count only. */
int orc_ratio_factor(const uint64_t *a, size_t k, const uint64_t *b, size_t m,
                     uint32_t *primes_out, uint64_t *exp_out, size_t cap, size_t *np_out)
{
    uint64_t A = 0;
    for (size_t i = 0; i < k; i++) { if (a[i] > 0xFFFFFFFFull) return ORC_EINVAL; if (a[i] > A) A = a[i]; }
    for (size_t j = 0; j < m; j++) { if (b[j] > 0xFFFFFFFFull) return ORC_EINVAL; if (b[j] > A) A = b[j]; }
    size_t bound = orc_pi_bound(A);
    uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * (bound ? bound : 1));
    if (!pr) return ORC_ENOMEM;
    size_t np = A >= 2 ? orc_primes(A, pr, bound) : 0;
    if (np == (size_t)-1) { free(pr); return ORC_EINTERNAL; }
    size_t cnt = 0;
    int st = ORC_OK;
    for (size_t i = 0; i < np; i++) {
        int64_t e = 0;
        for (size_t t = 0; t < k; t++) e += (int64_t)orc_legendre(a[t], pr[i]);
        for (size_t t = 0; t < m; t++) e -= (int64_t)orc_legendre(b[t], pr[i]);
        if (e < 0) { st = ORC_EINVAL; break; }
        if (e >= ((int64_t)1 << 32)) { st = ORC_ERANGE; break; }
        if (e == 0) continue;
        if (primes_out) {
            if (cnt >= cap) { st = ORC_ERANGE; break; }
            primes_out[cnt] = pr[i];
            exp_out[cnt] = (uint64_t)e;
        }
        cnt++;
    }
    free(pr);
    *np_out = cnt;
    return st;
}

static int cmp_pe(const void *x, const void *y)
{
    const uint64_t *u = (const uint64_t *)x, *v = (const uint64_t *)y;   /* (e, p) pairs */
    if (u[0] != v[0]) return u[0] < v[0] ? -1 : 1;
    if (u[1] != v[1]) return u[1] < v[1] ? -1 : 1;
    return 0;
}

/* N as normalised limbs; out == NULL is a size query. */
int orc_ratio(const uint64_t *a, size_t k, const uint64_t *b, size_t m, uint32_t *out, size_t cap, size_t *len)
{
    size_t np = 0;
    int st = orc_ratio_factor(a, k, b, m, NULL, NULL, 0, &np);
    if (st) return st;
    uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * (np ? np : 1));
    uint64_t *ex = (uint64_t *)malloc(sizeof(uint64_t) * (np ? np : 1));
    uint64_t *pe = (uint64_t *)malloc(2 * sizeof(uint64_t) * (np ? np : 1));
    if (!pr || !ex || !pe) { free(pr); free(ex); free(pe); return ORC_ENOMEM; }
    st = orc_ratio_factor(a, k, b, m, pr, ex, np, &np);
    if (st) { free(pr); free(ex); free(pe); return st; }
    /* groups G_e: exponent ascending, primes ascending inside a group */
    for (size_t i = 0; i < np; i++) { pe[2 * i] = ex[i]; pe[2 * i + 1] = pr[i]; }
    qsort(pe, np, 2 * sizeof(uint64_t), cmp_pe);
    uint32_t *gp = (uint32_t *)malloc(sizeof(uint32_t) * (np ? np : 1));
    uint32_t *gexp = (uint32_t *)malloc(sizeof(uint32_t) * (np ? np : 1));
    uint64_t *goff = (uint64_t *)malloc(sizeof(uint64_t) * (np + 1));
    uint32_t ng = 0;
    goff[0] = 0;
    for (size_t i = 0; i < np; i++) {
        gp[i] = (uint32_t)pe[2 * i + 1];
        if (i == 0 || pe[2 * i] != pe[2 * (i - 1)]) { gexp[ng] = (uint32_t)pe[2 * i]; ng++; }
        goff[ng] = i + 1;
    }
    big_t c;
    st = reconstruct(gp, gexp, goff, ng, &c);
    free(pr); free(ex); free(pe); free(gp); free(gexp); free(goff);
    if (st) return st;
    *len = c.n;
    if (out) {
        if (cap < c.n) { free(c.d); return ORC_ERANGE; }
        memcpy(out, c.d, c.n * 4);
    }
    free(c.d);
    return ORC_OK;
}

/* Product of an arbitrary list of big integers by the same balanced tree;
 * items are given as one flat limb array with offsets (n_items+1 entries).
 * Result normalised; out == NULL is a size query. */
int orc_product(const uint32_t *limbs, const uint64_t *offs, size_t n_items,
                uint32_t *out, size_t cap, size_t *len)
{
    big_t *it = (big_t *)malloc(sizeof(big_t) * (n_items ? n_items : 1));
    for (size_t i = 0; i < n_items; i++) {
        it[i].n = (size_t)(offs[i + 1] - offs[i]);
        it[i].d = (uint32_t *)malloc((it[i].n ? it[i].n : 1) * 4);
        memcpy(it[i].d, limbs + offs[i], it[i].n * 4);
        big_norm(&it[i]);
    }
    big_t r = product_tree(it, n_items);
    free(it);
    *len = r.n;
    if (out) {
        if (cap < r.n) { free(r.d); return ORC_ERANGE; }
        memcpy(out, r.d, r.n * 4);
    }
    free(r.d);
    return ORC_OK;
}

/* Batched exact products c_i = a_i * b_i (the operation the batched GPU
 * multiply performs), each c_i exactly la_i + lb_i limbs, not normalised. */
void orc_mul_batched(size_t batch, const uint32_t *a, const uint64_t *a_off,
                     const uint32_t *b, const uint64_t *b_off,
                     uint32_t *c, const uint64_t *c_off)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (size_t i = 0; i < batch; i++) {
        size_t la = (size_t)(a_off[i + 1] - a_off[i]);
        size_t lb = (size_t)(b_off[i + 1] - b_off[i]);
        orc_mul(a + a_off[i], la, b + b_off[i], lb, c + c_off[i]);
    }
}

/* Threads of the parallel loops: t >= 1 sets them, t <= 0 restores the
 * count the OpenMP runtime chose at start-up. */
static int g_default_threads = 0;
void orc_set_threads(int t)
{
#ifdef _OPENMP
    if (g_default_threads == 0) g_default_threads = omp_get_max_threads();
    omp_set_num_threads(t >= 1 ? t : g_default_threads);
#else
    (void)t;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Residues of C(n) straight from the definition C(n) = (2n)!/(n!(n+1)!)
 * (Sec. 1), in O(n) word operations: used to check results at sizes where a
 * full product on the CPU would take hours.
 * ------------------------------------------------------------------------- */
static uint64_t mulmod_u64(uint64_t a, uint64_t b, uint64_t q)
{
    return (uint64_t)((unsigned __int128)a * b % q);
}
static uint64_t powmod_u64(uint64_t b, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q;
    b %= q;
    while (e) { if (e & 1) r = mulmod_u64(r, b, q); b = mulmod_u64(b, b, q); e >>= 1; }
    return r;
}

/* C(n) mod q for a prime q > 2n: (prod_{k=n+2}^{2n} k) / n! mod q. */
uint64_t orc_catalan_mod_prime(uint64_t n, uint64_t q)
{
    uint64_t num = 1 % q, den = 1 % q;
    for (uint64_t k = n + 2; k <= 2 * n; k++) num = mulmod_u64(num, k, q);
    for (uint64_t k = 2; k <= n; k++) den = mulmod_u64(den, k, q);
    return mulmod_u64(num, powmod_u64(den, q - 2, q), q);
}

/* C(n) mod 2^64: the power of two is 2^{v}, v = popcount(n+1) - 1 (Kummer);
 * the odd part is (odd parts of k = n+2..2n) * (odd parts of k = 2..n)^-1. */
uint64_t orc_catalan_low64(uint64_t n)
{
    uint64_t num = 1, den = 1;
    for (uint64_t k = n + 2; k <= 2 * n; k++) { uint64_t t = k; while (!(t & 1)) t >>= 1; num *= t; }
    for (uint64_t k = 2; k <= n; k++) { uint64_t t = k; while (!(t & 1)) t >>= 1; den *= t; }
    /* inverse of an odd number mod 2^64 by Newton's iteration */
    uint64_t inv = den;
    for (int i = 0; i < 6; i++) inv *= 2 - den * inv;
    int v = __builtin_popcountll(n + 1) - 1;
    return (num * inv) << v;
}

/* ---------------------------------------------------------------------------
 * Decimal text of a limb vector (the optional decimal output of Sec. 3.2), by
 * the textbook route: divide the whole number by 10^9 again and again
 * (schoolbook long division, most significant limb first), each remainder
 * giving the next nine digits from the bottom; O(L^2).  Writes the digits
 * most significant first, no leading zeros ("0" for zero), no terminator, and
 * returns their count; returns it without writing when cap is too small.
 * ------------------------------------------------------------------------- */
size_t orc_to_decimal(const uint32_t *x, size_t L, char *out, size_t cap)
{
    size_t n = L;
    while (n > 0 && x[n - 1] == 0) n--;
    if (n == 0) {
        if (out && cap >= 1) out[0] = '0';
        return 1;
    }
    uint32_t *q = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint32_t *grp = (uint32_t *)malloc((n * 32 / 29 + 2) * sizeof(uint32_t));   /* 10^9 > 2^29 */
    if (!q || !grp) { free(q); free(grp); return 0; }
    memcpy(q, x, n * sizeof(uint32_t));
    size_t ng = 0;
    while (n > 0) {
        uint64_t r = 0;
        for (size_t i = n; i-- > 0;) {
            uint64_t cur = (r << 32) | q[i];
            q[i] = (uint32_t)(cur / 1000000000u);
            r = cur % 1000000000u;
        }
        grp[ng++] = (uint32_t)r;
        while (n > 0 && q[n - 1] == 0) n--;
    }
    /* groups least significant first; the top one without leading zeros */
    char buf[16];
    size_t top = 0;
    for (uint32_t v = grp[ng - 1]; ; v /= 10) { buf[top++] = (char)('0' + v % 10); if (v < 10) break; }
    size_t len = top;
    for (size_t k = 0; k + 1 < ng; k++) {
        if (g_fault == 4) { uint32_t v = grp[k]; do { len++; v /= 10; } while (v); }
        else len += 9;
    }
    if (out && cap >= len) {
        size_t o = 0;
        while (top > 0) out[o++] = buf[--top];
        for (size_t k = ng - 1; k-- > 0;) {
            uint32_t v = grp[k];
            int w = 9;
            if (g_fault == 4) { w = 0; uint32_t t = v; do { w++; t /= 10; } while (t); }
            for (int i = w - 1; i >= 0; i--) { out[o + i] = (char)('0' + v % 10); v /= 10; }
            o += (size_t)w;
        }
    }
    free(q);
    free(grp);
    return len;
}
