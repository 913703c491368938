// Modular arithmetic for primes below 2^62 on gfx950 (and the host, for tables).
//
// Residues are uint64_t. CDNA has no 64x64 multiplier; the compiler builds
// lo/hi products from 32-bit v_mad_u64_u32 / v_mul_hi_u32. Three forms:
//  * Shoup: multiply by a constant w with precomputed w' = floor(w 2^64 / q);
//    one high and two low products, result in [0, 2q) (lazy).
//  * Montgomery: REDC(T) = T 2^-64 mod q for T < q 2^64; multiplying by an
//    operand stored as w 2^64 mod q ("Montgomery form") gives the plain
//    product, and a sum of several 128-bit products can be reduced once.
//  * additions kept below 2^64 by conditional subtraction.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#define HC_HD __host__ __device__ __forceinline__

struct u128p { uint64_t lo, hi; };

HC_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

HC_HD u128p mul128(uint64_t a, uint64_t b) {
    u128p r;
    r.lo = a * b;
    r.hi = mulhi64(a, b);
    return r;
}

HC_HD void add128(u128p& acc, u128p x) {
    uint64_t lo = acc.lo + x.lo;
    acc.hi += x.hi + (lo < x.lo ? 1 : 0);
    acc.lo = lo;
}

HC_HD uint64_t csub(uint64_t x, uint64_t q) { return x >= q ? x - q : x; }

HC_HD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) { return csub(a + b, q); }

HC_HD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

// x * w mod q, lazily in [0, 2q); x any 64-bit value, w < q, wp = floor(w 2^64 / q).
HC_HD uint64_t shoup_lazy(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t qh = mulhi64(x, wp);
    return x * w - qh * q;
}

HC_HD uint64_t shoup(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
    return csub(shoup_lazy(x, w, wp, q), q);
}

// Montgomery reduction of T = (hi, lo) < q 2^64: returns T 2^-64 mod q in [0, q).
// qinv = -q^-1 mod 2^64.
HC_HD uint64_t redc(u128p T, uint64_t q, uint64_t qinv) {
    uint64_t m = T.lo * qinv;
    uint64_t mqh = mulhi64(m, q);
    uint64_t t = T.hi + mqh + (T.lo != 0 ? 1 : 0);
    return csub(t, q);
}

// a * bm 2^-64 mod q: with bm = b 2^64 mod q this is a b mod q.
HC_HD uint64_t mont_mul(uint64_t a, uint64_t bm, uint64_t q, uint64_t qinv) {
    return redc(mul128(a, bm), q, qinv);
}

// ---------------------------------------------------------------- host-side helpers

static inline uint64_t h_mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((unsigned __int128)a * b) % q);
}

static inline uint64_t h_powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = h_mulmod(r, a, q);
        a = h_mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

static inline uint64_t h_invmod(uint64_t a, uint64_t q) { return h_powmod(a, q - 2, q); }  // q prime

static inline uint64_t h_shoup_const(uint64_t w, uint64_t q) {
    return (uint64_t)(((unsigned __int128)w << 64) / q);
}

// -q^-1 mod 2^64 by Newton iteration (q odd).
static inline uint64_t h_mont_qinv(uint64_t q) {
    uint64_t x = q;  // correct to 3 bits
    for (int i = 0; i < 6; i++) x *= 2 - q * x;
    return (uint64_t)0 - x;
}

// w 2^64 mod q.
static inline uint64_t h_to_mont(uint64_t w, uint64_t q) {
    return (uint64_t)(((unsigned __int128)w << 64) % q);
}
