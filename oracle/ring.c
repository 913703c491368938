/*
 * Oracle ring helpers: exact arithmetic in Z_q and Z_q[X]/(X^n+1), plain C.
 *
 * TEST INFRASTRUCTURE ONLY. This file is part of the CPU oracle that the
 * tests, the smoke check and the benchmark's CPU-baseline leg use to decide
 * what the right answer is. The library never links it.
 *
 * Every product is formed as an exact 128-bit integer and reduced with the
 * C '%' operator: no Montgomery, Barrett, Shoup or lazy-reduction tricks, so
 * each line can be checked by eye. Moduli are below 2^62.
 *
 * The negacyclic transform is the textbook one: twist by powers of psi (a
 * primitive 2n-th root of unity mod q), then a cyclic radix-2 DFT with
 * omega = psi^2 in natural order (bit-reversal permutation up front). After
 * o_ntt, entry i holds a(psi^(2i+1)). It serves only to multiply ring
 * elements; nothing outside the oracle sees this ordering.
 */
#include <stdint.h>
#include <stdlib.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * b) % q);
}

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

/* bit reversal of i over 'bits' bits */
static uint64_t brv(uint64_t i, int bits) {
    uint64_t r = 0;
    for (int k = 0; k < bits; k++) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

static int log2u(uint64_t n) {
    int l = 0;
    while ((1ull << l) < n) l++;
    return l;
}

/* in-place cyclic DFT: A_i = sum_j a_j w^(i j), natural order in and out */
static void cyclic_dft(uint64_t* a, uint64_t n, uint64_t q, uint64_t w) {
    int logn = log2u(n);
    for (uint64_t i = 0; i < n; i++) {
        uint64_t j = brv(i, logn);
        if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (uint64_t len = 2; len <= n; len <<= 1) {
        uint64_t wl = powmod(w, n / len, q);  /* primitive len-th root */
        for (uint64_t st = 0; st < n; st += len) {
            uint64_t wk = 1;
            for (uint64_t k = 0; k < len / 2; k++) {
                uint64_t u = a[st + k];
                uint64_t v = mulmod(a[st + k + len / 2], wk, q);
                a[st + k] = (u + v) % q;
                a[st + k + len / 2] = (u + q - v) % q;
                wk = mulmod(wk, wl, q);
            }
        }
    }
}

/* a <- (a(psi^1), a(psi^3), ..., a(psi^(2n-1))) */
void o_ntt(uint64_t* a, uint64_t n, uint64_t q, uint64_t psi) {
    uint64_t pj = 1;
    for (uint64_t j = 0; j < n; j++) {  /* twist: a_j psi^j */
        a[j] = mulmod(a[j], pj, q);
        pj = mulmod(pj, psi, q);
    }
    cyclic_dft(a, n, q, mulmod(psi, psi, q));
}

/* inverse of o_ntt */
void o_intt(uint64_t* a, uint64_t n, uint64_t q, uint64_t psi) {
    uint64_t psi_inv = powmod(psi, q - 2, q);
    cyclic_dft(a, n, q, mulmod(psi_inv, psi_inv, q));
    uint64_t n_inv = powmod(n % q, q - 2, q);
    uint64_t pj = n_inv;
    for (uint64_t j = 0; j < n; j++) {  /* untwist and scale: a_j psi^-j / n */
        a[j] = mulmod(a[j], pj, q);
        pj = mulmod(pj, psi_inv, q);
    }
}

/* out = a * b in Z_q[X]/(X^n+1); out may alias neither a nor b */
void o_negacyclic_mul(uint64_t* out, const uint64_t* a, const uint64_t* b,
                      uint64_t n, uint64_t q, uint64_t psi) {
    uint64_t* ta = (uint64_t*)malloc(n * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++) { ta[i] = a[i] % q; out[i] = b[i] % q; }
    o_ntt(ta, n, q, psi);
    o_ntt(out, n, q, psi);
    for (uint64_t i = 0; i < n; i++) out[i] = mulmod(ta[i], out[i], q);
    o_intt(out, n, q, psi);
    free(ta);
}

/* element-wise: out_i = a_i * b_i mod q */
void o_vec_mul(uint64_t* out, const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t q) {
    for (uint64_t i = 0; i < n; i++) out[i] = mulmod(a[i], b[i], q);
}

/* element-wise: out_i = a_i * c mod q */
void o_vec_scale(uint64_t* out, const uint64_t* a, uint64_t c, uint64_t n, uint64_t q) {
    for (uint64_t i = 0; i < n; i++) out[i] = mulmod(a[i], c, q);
}
