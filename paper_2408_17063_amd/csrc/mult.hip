// Ciphertext products and what is built on them: Power (Alg. 5's Power_{p-1}), Match
// (Alg. 7 step 1, exact-match predicate) and the generic Comp of Alg. 5.
//
// A product of (a0, a1) and (b0, b1) at the full modulus Q is the exact rounding
// z = round(p/Q e) mod Q of the integer tensor e = (a0 b0, a0 b1 + a1 b0, a1 b1) of
// the centred lifts (representatives in (-Q/2, Q/2)), followed by relinearisation
// of z2. Everything is exact integer arithmetic in RNS:
//  1. each centred lift is extended from Q to an auxiliary basis B of L + 1 primes
//     below 2^61 (prod B > n Q, so |e| < Q prod B / 2 and e is determined by its
//     residues over Q and B) by mixed-radix conversion (MRC): the digits y_i of the
//     lift in radix (q_0, q_0 q_1, ...) are exact, their comparison with the digits of
//     (Q - 1)/2 decides the sign, and the value is re-evaluated mod each b_j;
//  2. forward NTTs over Q and B, the three pointwise products, inverse NTTs;
//  3. scale and round per coefficient: r = (p e + (Q-1)/2) mod Q is recovered exactly by
//     MRC over Q, z = (p e + (Q-1)/2 - r) / Q is then an exact division mod each b_j,
//     and z (|z| < prod B / 2) is brought back to Q by MRC over B with its sign;
//  4. relinearisation: (z0, z2) is key-switched like a rotation with k = 1 by the key
//     for s^2 (ModUp, inner product over PQ, ModDown) and z1 is added to the second
//     component (in the coefficient domain: z1 is never transformed).
// One thread handles one coefficient of one polynomial, its digits in registers. The
// products of several ciphertexts (Power and Match) run as one batch per step.
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "compress.h"

namespace hc {

// Device constants of the exact conversions (one allocation, word offsets below).
// The MRC multipliers are Shoup pairs (w, floor(w 2^64 / q)); the base-conversion
// multipliers are in Montgomery form mod the prime they multiply under and split into
// 31-bit limbs, low limb in the low word (see conv_sum). The kernels hold a
// coefficient's digits in registers, in arrays of compile-time length:
// CQ = L rounded up to a multiple of 8 over Q, CB = CQ + 1 over B (nb = L + 1). The
// tables are laid out at those lengths; the rows past L (past nb) are padding whose
// multipliers are 0 and whose modulus is the basis's first prime, so their digits stay
// exactly 0 and add nothing to any sum or comparison.
struct MultTab {
    const uint64_t* modq;   // [CQ]      q_i (padding: q_0)
    const uint64_t* qiq;    // [CQ]      -q_i^-1 mod 2^64
    const uint64_t* modb;   // [CB]      b_j (padding: b_0)
    const uint64_t* qib;    // [CB]      -b_j^-1 mod 2^64
    const uint64_t* invq;   // [CQ][CQ][2] [k][i]: q_k^-1 mod q_i (k < i < L), Shoup pair mod q_i
    const uint64_t* hq;     // [CQ]      digits of (Q-1)/2 in the radix of Q
    const uint64_t* mqb;    // [nb][CQ]  prod_{k<i} q_k mod b_j, Montgomery mod b_j, limbs
    const uint64_t* qmodb;  // [nb]      Q mod b_j
    const uint64_t* qinvb;  // [nb]      Q^-1 mod b_j, Montgomery mod b_j
    const uint64_t* hmodq;  // [CQ]      (Q-1)/2 mod q_i
    const uint64_t* pmontq; // [CQ]      p in Montgomery form mod q_i
    const uint64_t* hmodb;  // [nb]      (Q-1)/2 mod b_j
    const uint64_t* pmontb; // [nb]      p in Montgomery form mod b_j
    const uint64_t* invb;   // [CB][CB][2] [k][j]: b_k^-1 mod b_j (k < j < nb), Shoup pair mod b_j
    const uint64_t* hb;     // [CB]      digits of (prod B - 1)/2 in the radix of B
    const uint64_t* mbq;    // [L][CB]   prod_{k<j} b_k mod q_i, Montgomery mod q_i, limbs
    const uint64_t* bmodq;  // [L]       prod B mod q_i
};
constexpr int MAX_DIG = 48;  // limit on L + 1 (context creation keeps L + K <= 64; products need L <= 47)

// Digit capacity over Q for L primes: L rounded up to a multiple of 8.
static int mult_cq(int L) { return (L + 7) / 8 * 8; }

static MultTab mult_tab(const Ctx& c) {
    const int L = c.L, nb = c.nb, CQ = mult_cq(L), CB = CQ + 1;
    const uint64_t* d = c.d_mult;
    MultTab t;
    size_t o = 0;
    t.modq = d + o; o += CQ;
    t.qiq = d + o; o += CQ;
    t.modb = d + o; o += CB;
    t.qib = d + o; o += CB;
    t.invq = d + o; o += (size_t)2 * CQ * CQ;
    t.hq = d + o; o += CQ;
    t.mqb = d + o; o += (size_t)nb * CQ;
    t.qmodb = d + o; o += nb;
    t.qinvb = d + o; o += nb;
    t.hmodq = d + o; o += CQ;
    t.pmontq = d + o; o += CQ;
    t.hmodb = d + o; o += nb;
    t.pmontb = d + o; o += nb;
    t.invb = d + o; o += (size_t)2 * CB * CB;
    t.hb = d + o; o += CB;
    t.mbq = d + o; o += (size_t)L * CB;
    t.bmodq = d + o;
    return t;
}

// host: mixed-radix digits of the integer with residues `res` over `mods`
static std::vector<uint64_t> h_mrc(const std::vector<uint64_t>& res, const std::vector<uint64_t>& mods) {
    const size_t m = mods.size();
    std::vector<uint64_t> y(m);
    for (size_t i = 0; i < m; i++) {
        uint64_t t = res[i] % mods[i];
        for (size_t k = 0; k < i; k++) {
            const uint64_t yk = y[k] % mods[i];
            t = (t + mods[i] - yk) % mods[i];
            t = h_mulmod(t, h_invmod(mods[k] % mods[i], mods[i]), mods[i]);
        }
        y[i] = t;
    }
    return y;
}

// v < 2^62 as two 31-bit limbs: v mod 2^31 in the low word, v >> 31 in the high word
__host__ __device__ __forceinline__ uint64_t limbs31(uint64_t v) {
    return (v & 0x7fffffffull) | ((v >> 31) << 32);
}

hc_status build_mult_tables(Ctx& c) {
    const int L = c.L, nb = c.nb, nq = c.nq;
    if (L + 1 > MAX_DIG || nb != L + 1) return HC_OK;  // products unavailable (context limit)
    const int CQ = mult_cq(L), CB = CQ + 1;
    std::vector<uint64_t> Qp(c.primes.begin(), c.primes.begin() + L),
        Bp(c.primes.begin() + nq, c.primes.begin() + nq + nb);
    std::vector<uint64_t> all;
    auto pad = [&](size_t count) { all.insert(all.end(), count, 0); };
    // moduli and Montgomery constants, padded with the basis's first prime
    for (int i = 0; i < CQ; i++) all.push_back(Qp[i < L ? i : 0]);
    for (int i = 0; i < CQ; i++) all.push_back(h_mont_qinv(Qp[i < L ? i : 0]));
    for (int j = 0; j < CB; j++) all.push_back(Bp[j < nb ? j : 0]);
    for (int j = 0; j < CB; j++) all.push_back(h_mont_qinv(Bp[j < nb ? j : 0]));
    // invq [k][i]: Shoup pairs
    for (int k = 0; k < CQ; k++)
        for (int i = 0; i < CQ; i++) {
            const uint64_t w = k < i && i < L ? h_invmod(Qp[k] % Qp[i], Qp[i]) : 0;
            all.push_back(w);
            all.push_back(w ? h_shoup_const(w, Qp[i]) : 0);
        }
    // hq: (Q-1)/2 = (q_i - 1)/2 mod q_i
    std::vector<uint64_t> hres(L);
    for (int i = 0; i < L; i++) hres[i] = (Qp[i] - 1) / 2;
    for (uint64_t x : h_mrc(hres, Qp)) all.push_back(x);
    pad(CQ - L);
    // mqb [j][i]
    for (int j = 0; j < nb; j++) {
        uint64_t pr = 1;
        for (int i = 0; i < L; i++) {
            all.push_back(limbs31(h_to_mont(pr, Bp[j])));
            pr = h_mulmod(pr, Qp[i] % Bp[j], Bp[j]);
        }
        pad(CQ - L);
    }
    // qmodb, qinvb
    std::vector<uint64_t> qmb(nb);
    for (int j = 0; j < nb; j++) {
        uint64_t pr = 1;
        for (int i = 0; i < L; i++) pr = h_mulmod(pr, Qp[i] % Bp[j], Bp[j]);
        qmb[j] = pr;
        all.push_back(pr);
    }
    for (int j = 0; j < nb; j++) all.push_back(h_to_mont(h_invmod(qmb[j], Bp[j]), Bp[j]));
    // (Q-1)/2 and p over Q (padded), then over B: (Q-1)/2 mod b = (Q mod b - 1) 2^-1 mod b
    for (int i = 0; i < L; i++) all.push_back((Qp[i] - 1) / 2);
    pad(CQ - L);
    for (int i = 0; i < L; i++) all.push_back(h_to_mont(c.p % Qp[i], Qp[i]));
    pad(CQ - L);
    for (int j = 0; j < nb; j++)
        all.push_back(h_mulmod((qmb[j] + Bp[j] - 1) % Bp[j], h_invmod(2, Bp[j]), Bp[j]));
    for (int j = 0; j < nb; j++) all.push_back(h_to_mont(c.p % Bp[j], Bp[j]));
    // invb [k][j]: Shoup pairs
    for (int k = 0; k < CB; k++)
        for (int j = 0; j < CB; j++) {
            const uint64_t w = k < j && j < nb ? h_invmod(Bp[k] % Bp[j], Bp[j]) : 0;
            all.push_back(w);
            all.push_back(w ? h_shoup_const(w, Bp[j]) : 0);
        }
    // hb: (prod B - 1)/2 = (b_j - 1)/2 mod b_j
    std::vector<uint64_t> hbres(nb);
    for (int j = 0; j < nb; j++) hbres[j] = (Bp[j] - 1) / 2;
    for (uint64_t x : h_mrc(hbres, Bp)) all.push_back(x);
    pad(CB - nb);
    // mbq [i][j], bmodq
    for (int i = 0; i < L; i++) {
        uint64_t pr = 1;
        for (int j = 0; j < nb; j++) {
            all.push_back(limbs31(h_to_mont(pr, Qp[i])));
            pr = h_mulmod(pr, Bp[j] % Qp[i], Qp[i]);
        }
        pad(CB - nb);
    }
    for (int i = 0; i < L; i++) {
        uint64_t pr = 1;
        for (int j = 0; j < nb; j++) pr = h_mulmod(pr, Bp[j] % Qp[i], Qp[i]);
        all.push_back(pr);
    }
    HC_CHECK(hipMalloc((void**)&c.d_mult, sizeof(uint64_t) * all.size()));
    c.owned.push_back(c.d_mult);
    HC_CHECK(hipMemcpy(c.d_mult, all.data(), sizeof(uint64_t) * all.size(), hipMemcpyHostToDevice));
    return HC_OK;
}

// The digit arrays of one coefficient live in registers, indexed only at compile time:
// loops over digits are unrolled (the padding rows compute exact zeros), and where a
// loop runs over a runtime index (the MRC step, the output prime) the element it needs
// is picked by selects.

// MRC digits in place: t[i] (residues over the M primes of mods) become the digits
// y_i < m_i. Step k takes digit k off every later residue and divides by m_k; the rows
// of a step are independent, updated in chunks of 4 (chunks wholly at or before k are
// skipped, and only the chunk holding k needs selects). Digit k lies below 2 m_i (every
// prime of a basis lies in [2^(t-1), 2^t) for one t), so t_i + 2 m_i - y_k lies in
// (0, 4 m_i) for a row kept lazily in [0, 2 m_i), and one Shoup product by m_k^-1 (inv:
// [k][i] pairs) brings it back to [0, 2 m_i). A row is reduced to [0, m_i) when it
// becomes a digit (for the next step) and once more at the end.
template <int M>
__device__ __forceinline__ void mrc(uint64_t (&t)[M], const uint64_t* __restrict__ mods,
                                    const uint64_t* __restrict__ inv) {
    constexpr int W = 4;
    uint64_t yk = t[0];
    for (int k = 0; k + 1 < M; k++) {
        const uint64_t* ik = inv + (size_t)2 * k * M;
        uint64_t next = 0;
        #pragma unroll
        for (int c = 0; c < M; c += W) {
            const int ce = c + W < M ? c + W : M;
            if (c > k) {
                #pragma unroll
                for (int i = c; i < ce; i++) {
                    const uint64_t q = mods[i];
                    t[i] = shoup_lazy(t[i] + 2 * q - yk, ik[2 * i], ik[2 * i + 1], q);
                }
                next = c == k + 1 ? t[c] : next;
            } else if (ce > k + 1) {
                #pragma unroll
                for (int i = c; i < ce; i++) {
                    const uint64_t q = mods[i];
                    const uint64_t v = shoup_lazy(t[i] + 2 * q - yk, ik[2 * i], ik[2 * i + 1], q);
                    t[i] = i > k ? v : t[i];
                    next = i == k + 1 ? v : next;
                }
            }
        }
        yk = csub(next, mods[k + 1]);
    }
    #pragma unroll
    for (int i = 1; i < M; i++) t[i] = csub(t[i], mods[i]);
}

// y > h for digit vectors (most significant digit last)
template <int M>
__device__ __forceinline__ bool digits_gt(const uint64_t (&y)[M], const uint64_t* __restrict__ h) {
    bool gt = false, decided = false;
    #pragma unroll
    for (int i = M - 1; i >= 0; i--) {
        const uint64_t hv = h[i];
        gt = decided ? gt : y[i] > hv;
        decided = decided || y[i] != hv;
    }
    return gt;
}

// Digits to 31-bit limb form (see limbs31), for conv_sum.
template <int M>
__device__ __forceinline__ void to_limbs(uint64_t (&y)[M]) {
    #pragma unroll
    for (int i = 0; i < M; i++) y[i] = limbs31(y[i]);
}

// sum_i y_i c_i mod q for y_i < 2^61 and c_i < q in Montgomery form, both as 31-bit
// limbs (y = y0 + y1 2^31): each term is four 32x32-bit multiply-adds into the column
// sums of a batch of 8 terms: y0 c0 alternately into a0e and a0o (4 terms each below
// 2^64), y0 c1 into a1x and y1 c0 into a1y (each below 2^61 a term), y1 c1 into a2. The
// batch's T = a0e + a0o + (a1x + a1y) 2^31 + a2 2^62 lies below 2^64 q: one REDC.
template <int M>
__device__ __forceinline__ uint64_t conv_sum(const uint64_t (&y)[M], const uint64_t* __restrict__ c, uint64_t q,
                                             uint64_t qi) {
    uint64_t v = 0;
    #pragma unroll
    for (int i8 = 0; i8 < M; i8 += 8) {
        uint64_t a0e = 0, a0o = 0, a1x = 0, a1y = 0, a2 = 0;
        #pragma unroll
        for (int i = i8; i < (i8 + 8 < M ? i8 + 8 : M); i++) {
            const uint32_t y0 = (uint32_t)y[i], y1 = (uint32_t)(y[i] >> 32);
            const uint32_t c0 = (uint32_t)c[i], c1 = (uint32_t)(c[i] >> 32);
            if ((i - i8) & 1) a0o += (uint64_t)y0 * c0;
            else a0e += (uint64_t)y0 * c0;
            a1x += (uint64_t)y0 * c1;
            a1y += (uint64_t)y1 * c0;
            a2 += (uint64_t)y1 * c1;
        }
        const uint64_t s1 = a1x + a1y, carry = s1 < a1x ? 1 : 0;  // a1x + a1y = s1 + carry 2^64
        u128p T{a0e, 0};
        add128(T, u128p{a0o, 0});
        add128(T, u128p{s1 << 31, (s1 >> 33) | (carry << 31)});
        add128(T, u128p{a2 << 62, a2 >> 2});
        v = add_mod(v, redc(T, q, qi), q);
    }
    return v;
}

// out[t][j] = centred lift of in[t] (over Q, coefficient domain) mod b_j, t < count
template <int CQ>
__global__ void __launch_bounds__(256) bext_kernel(uint64_t* __restrict__ out, const uint64_t* __restrict__ in, MultTab tb,
                                                   int n, int L, int nb) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int t = blockIdx.z;
    const uint64_t* a = in + (size_t)t * L * n + x;
    uint64_t y[CQ];
    #pragma unroll
    for (int i = 0; i < CQ; i++) y[i] = i < L ? a[(size_t)i * n] : 0;
    mrc<CQ>(y, tb.modq, tb.invq);
    const bool neg = digits_gt<CQ>(y, tb.hq);
    to_limbs<CQ>(y);
    uint64_t* o = out + (size_t)t * nb * n + x;
    for (int j = 0; j < nb; j++) {
        const uint64_t b = tb.modb[j], bi = tb.qib[j];
        uint64_t v = conv_sum<CQ>(y, tb.mqb + (size_t)j * CQ, b, bi);
        if (neg) v = sub_mod(v, tb.qmodb[j], b);
        o[(size_t)j * n] = v;
    }
}

// e = (a0 b0, a0 b1 + a1 b0, a1 b1) pointwise (NTT domain) on R rows of prime indices
// prime0 + row, for ciphertext blockIdx.z; a, b: [count][2][R][n]; e: [count][3][R][n]
__global__ void tensor_kernel(uint64_t* __restrict__ e, const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                              const uint64_t* __restrict__ mods, const uint64_t* __restrict__ qinv,
                              const uint64_t* __restrict__ r2, int n, int R, int prime0) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int row = blockIdx.y, pi = prime0 + row;
    const uint64_t q = mods[pi], qi = qinv[pi], rr = r2[pi];
    const size_t P = (size_t)R * n, o = (size_t)row * n + x, ct = blockIdx.z;
    a += ct * 2 * P;
    b += ct * 2 * P;
    e += ct * 3 * P;
    // b to Montgomery form: mont_mul(b, 2^128 mod q) = b 2^64 mod q
    const uint64_t b0 = mont_mul(b[o], rr, q, qi), b1 = mont_mul(b[P + o], rr, q, qi);
    const uint64_t a0 = a[o], a1 = a[P + o];
    e[o] = mont_mul(a0, b0, q, qi);
    e[P + o] = add_mod(mont_mul(a0, b1, q, qi), mont_mul(a1, b0, q, qi), q);
    e[2 * P + o] = mont_mul(a1, b1, q, qi);
}

// round(p e_t / Q) mod Q (over Q, coefficient domain) from e_t over Q (eq,
// [count][3][L][n]) and over B (eb, [count][3][nb][n]), coefficient domain; blockIdx.z =
// 3 ct + t. t = 0 and 2 go to zc[ct] = (z0, z2) ([count][2][L][n], the ciphertext to
// relinearise), t = 1 to z1[ct] ([count][L][n]).
template <int CQ>
__global__ void __launch_bounds__(256) scale_round_kernel(uint64_t* __restrict__ zc, uint64_t* __restrict__ z1,
                                                          const uint64_t* __restrict__ eq,
                                                          const uint64_t* __restrict__ eb, MultTab tb, int n, int L,
                                                          int nb) {
    constexpr int CB = CQ + 1;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int t = blockIdx.z % 3;
    const size_t ct = blockIdx.z / 3, Ln = (size_t)L * n;
    eq += ct * 3 * Ln;
    eb += ct * 3 * nb * n;
    uint64_t* z = t == 1 ? z1 + ct * Ln : zc + ct * 2 * Ln + (t == 2 ? Ln : 0);
    uint64_t r[CQ], y[CB];
    // r = (p e + H) mod Q, exactly, as MRC digits over Q
    #pragma unroll
    for (int i = 0; i < CQ; i++) r[i] = i < L ? eq[((size_t)t * L + i) * n + x] : 0;
    #pragma unroll
    for (int i = 0; i < CQ; i++) {
        const uint64_t q = tb.modq[i];
        r[i] = add_mod(mont_mul(r[i], tb.pmontq[i], q, tb.qiq[i]), tb.hmodq[i], q);
    }
    mrc<CQ>(r, tb.modq, tb.invq);
    to_limbs<CQ>(r);
    // z mod b_j = (p e + H - r) Q^-1 mod b_j (the division is exact)
    #pragma unroll
    for (int j = 0; j < CB; j++) y[j] = 0;
    for (int j = 0; j < nb; j++) {
        const uint64_t b = tb.modb[j], bi = tb.qib[j];
        const uint64_t ev = eb[((size_t)t * nb + j) * n + x];
        const uint64_t rv = conv_sum<CQ>(r, tb.mqb + (size_t)j * CQ, b, bi);
        const uint64_t v = add_mod(mont_mul(ev, tb.pmontb[j], b, bi), tb.hmodb[j], b);
        const uint64_t zj = mont_mul(sub_mod(v, rv, b), tb.qinvb[j], b, bi);
        #pragma unroll
        for (int jj = 0; jj < CB; jj++) y[jj] = jj == j ? zj : y[jj];
    }
    // z (|z| < prod B / 2) from its residues over B, back to Q
    mrc<CB>(y, tb.modb, tb.invb);
    const bool neg = digits_gt<CB>(y, tb.hb);
    to_limbs<CB>(y);
    for (int i = 0; i < L; i++) {
        const uint64_t q = tb.modq[i];
        uint64_t v = conv_sum<CB>(y, tb.mbq + (size_t)i * CB, q, tb.qiq[i]);
        if (neg) v = sub_mod(v, tb.bmodq[i], q);
        z[(size_t)i * n + x] = v;
    }
}

// out[ct][1] += z1[ct] over the first L primes (ciphertext ct = blockIdx.z; out:
// [count][2][L][n], z1: [count][L][n])
__global__ void add_z1_kernel(uint64_t* __restrict__ out, const uint64_t* __restrict__ z,
                              const uint64_t* __restrict__ mods, int n, int L) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int r = blockIdx.y;
    const size_t ct = blockIdx.z, Ln = (size_t)L * n, o = (size_t)r * n + x;
    uint64_t* d = out + ct * 2 * Ln + Ln + o;
    *d = add_mod(*d, z[ct * Ln + o], mods[r]);
}

// Calls f(integral_constant<int, CQ>) with the digit capacity over Q for L primes.
template <typename F>
static void with_cap(int L, F&& f) {
    switch (mult_cq(L)) {
        case 8: f(std::integral_constant<int, 8>{}); break;
        case 16: f(std::integral_constant<int, 16>{}); break;
        case 24: f(std::integral_constant<int, 24>{}); break;
        case 32: f(std::integral_constant<int, 32>{}); break;
        case 40: f(std::integral_constant<int, 40>{}); break;
        default: f(std::integral_constant<int, 48>{}); break;
    }
}

// c0 = c0 - Delta m over the first L primes (coefficient domain; m canonical in [0, p))
__global__ void sub_delta_m_kernel(uint64_t* ct, const uint32_t* m, const uint64_t* mods, const uint64_t* delta,
                                   int n) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int r = blockIdx.y;
    const uint64_t q = mods[r];
    const size_t o = (size_t)r * n + x;
    ct[o] = sub_mod(ct[o], shoup((uint64_t)m[x], delta[2 * r], delta[2 * r + 1], q), q);
}

// ct = 1 - ct: (Delta - c0, -c1), Delta on the constant coefficient (coefficient domain)
__global__ void one_minus_kernel(uint64_t* ct, const uint64_t* mods, const uint64_t* delta, int n, int L) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int r = blockIdx.y, comp = blockIdx.z;
    const uint64_t q = mods[r];
    const size_t o = ((size_t)comp * L + r) * n + x;
    const uint64_t d = (comp == 0 && x == 0) ? delta[2 * r] : 0;
    ct[o] = sub_mod(d, ct[o], q);
}

// Products of `count` pairs at the full level, all in one pass per step: out[i] =
// relin(round(p/Q (a[i] x b[i]))). a, b, out: [count][2][L][n] coefficient domain (out
// may alias a or b; b == a squares). a_scratch: a may be overwritten (it is then
// transformed in place; otherwise the transform reads a and writes the workspace). Every launch covers the whole batch, and the
// relinearisations are one key-switching pass whose jobs share the key and write out.
static hc_status mul_ct(Ctx& c, Lane& l, KsScratch& ks, const uint64_t* rk, uint64_t* a, const uint64_t* b,
                        uint64_t* out, int count, bool a_scratch, uint64_t* const* buf, hipStream_t st) {
    const size_t n = c.n;
    const int L = c.L, nb = c.nb, nq = c.nq;
    const size_t QW = (size_t)L * n, BW = (size_t)nb * n;
    uint64_t *aN = a_scratch ? a : buf[0], *bN = buf[1], *aB = buf[2], *bB = buf[3], *eQ = buf[4], *eB = buf[5],
             *z = buf[6];
    const MultTab tb = mult_tab(c);
    const bool sq = a == b;
    const unsigned gx = (unsigned)((n + 255) / 256), cnt = (unsigned)count;
    // 1. the centred lifts over B
    with_cap(L, [&](auto cap) {
        constexpr int C = decltype(cap)::value;
        hipLaunchKernelGGL(bext_kernel<C>, dim3(gx, 1, 2 * cnt), dim3(256), 0, st, aB, a, tb, (int)n, L, nb);
        if (!sq) hipLaunchKernelGGL(bext_kernel<C>, dim3(gx, 1, 2 * cnt), dim3(256), 0, st, bB, b, tb, (int)n, L, nb);
    });
    // 2. NTT domain over Q and B, the tensor, back
    ntt64(c, aN, QW, 2 * count, 0, L, false, st, a_scratch ? nullptr : a);
    ntt64(c, aB, BW, 2 * count, nq, nb, false, st);
    if (!sq) {
        ntt64(c, bN, QW, 2 * count, 0, L, false, st, b);
        ntt64(c, bB, BW, 2 * count, nq, nb, false, st);
    }
    hipLaunchKernelGGL(tensor_kernel, dim3(gx, L, cnt), dim3(256), 0, st, eQ, aN, sq ? aN : bN, c.d_mods, c.d_qinv,
                       c.d_r2, (int)n, L, 0);
    hipLaunchKernelGGL(tensor_kernel, dim3(gx, nb, cnt), dim3(256), 0, st, eB, aB, sq ? aB : bB, c.d_mods, c.d_qinv,
                       c.d_r2, (int)n, nb, nq);
    ntt64(c, eQ, QW, 3 * count, 0, L, true, st);
    ntt64(c, eB, BW, 3 * count, nq, nb, true, st);
    // 3. z = round(p e / Q): (z0, z2) in z, a ciphertext to key-switch; z1 apart (buf[0],
    //    free once the tensor is formed, holds it). a and b are not read after the tensor.
    uint64_t* z1 = buf[0];
    with_cap(L, [&](auto cap) {
        constexpr int C = decltype(cap)::value;
        hipLaunchKernelGGL(scale_round_kernel<C>, dim3(gx, 1, 3 * cnt), dim3(256), 0, st, z, z1, eQ, eB, tb, (int)n,
                           L, nb);
    });
    // 4. relinearisation: (z0 + KS(z2)_0, z1 + KS(z2)_1), z1 added in the coefficient domain
    ntt64(c, z, QW, 2 * count, 0, L, false, st);
    std::vector<KsJob> jobs;
    for (int i = 0; i < count; i++) jobs.push_back(KsJob{z + (size_t)i * 2 * QW, out + (size_t)i * 2 * QW, rk, 1u, 0});
    hc_status s = ks_run(c, l, ks, jobs, nullptr, L, st);
    if (s != HC_OK) return s;
    ntt64(c, out, QW, 2 * count, 0, L, true, st);
    hipLaunchKernelGGL(add_z1_kernel, dim3(gx, L, cnt), dim3(256), 0, st, out, z1, c.d_mods, (int)n, L);
    return HC_OK;
}

// Ciphertexts a product pass takes at once (the workspace grows with it: about 0.4 GB
// per ciphertext at 24 primes and ring 2^16).
constexpr int MUL_BATCH = 16;

// Workspace of products for up to `count` ciphertexts: 7 buffers, two spare ciphertext
// arrays and key-switching scratch for `count` jobs at level L.
struct MulWs {
    KsScratch ks;
    uint64_t* buf[7];
    uint64_t* t0;  // [count][2][L][n] spare ciphertexts
    uint64_t* t1;
};

static void mul_ws_sizes(const Ctx& c, int count, size_t (&sizes)[9]) {
    const size_t QW = (size_t)c.L * c.n, BW = (size_t)c.nb * c.n, k = (size_t)count;
    const size_t sz[9] = {2 * QW, 2 * QW, 2 * BW, 2 * BW, 3 * QW, 3 * BW, 2 * QW, 2 * QW, 2 * QW};
    for (int i = 0; i < 9; i++) sizes[i] = k * sz[i];
}

static size_t mul_ws_bytes(const Ctx& c, int count) {
    size_t sizes[9], b = 0;
    mul_ws_sizes(c, count, sizes);
    for (size_t v : sizes) b += 8 * v + 256;
    return b + ks_scratch_bytes(c, c.L, count) + 16 * 256;
}

static hc_status mul_ws(Ctx& c, Arena& a, int count, MulWs& w) {
    size_t sizes[9];
    mul_ws_sizes(c, count, sizes);
    w.ks = ks_scratch(c, a, c.L, count);
    for (int i = 0; i < 7; i++) {
        w.buf[i] = a.take<uint64_t>(sizes[i]);
        if (!w.buf[i]) return HC_ENOMEM;
    }
    w.t0 = a.take<uint64_t>(sizes[7]);
    w.t1 = a.take<uint64_t>(sizes[8]);
    if (!w.t0 || !w.t1 || !w.ks.tmpC) return HC_ENOMEM;
    return HC_OK;
}

// out[i] = in[i]^e for i < count by left-to-right binary exponentiation, the count
// ciphertexts in lockstep (coefficient domain, [count][2][L][n]; out may alias in)
static hc_status power_ct(Ctx& c, Lane& l, MulWs& w, const uint64_t* rk, const uint64_t* in, uint32_t e,
                          uint64_t* out, int count, hipStream_t st) {
    const size_t CW = 2 * (size_t)c.L * c.n * count;
    int top = 31;
    while (top > 0 && !((e >> top) & 1u)) top--;
    // acc in t0, the inputs kept in t1 (out may alias in)
    HC_CHECK(hipMemcpyAsync(w.t1, in, sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
    HC_CHECK(hipMemcpyAsync(w.t0, in, sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
    for (int bit = top - 1; bit >= 0; bit--) {
        hc_status s = mul_ct(c, l, w.ks, rk, w.t0, w.t0, w.t0, count, true, w.buf, st);
        if (s != HC_OK) return s;
        if ((e >> bit) & 1u) {
            s = mul_ct(c, l, w.ks, rk, w.t0, w.t1, w.t0, count, true, w.buf, st);
            if (s != HC_OK) return s;
        }
    }
    HC_CHECK(hipMemcpyAsync(out, w.t0, sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
    return HC_OK;
}

static hc_status rk_of(const hc_gk* rk, const uint64_t** key) {
    *key = rk ? find_key(rk, 1u) : nullptr;
    return *key ? HC_OK : HC_ENOKEY;
}

// Power_{p-1} of n_ct ciphertexts (device [n_ct][2][L][n]) into out (same layout)
hc_status power_many(Ctx& c, const hc_gk* rk, const uint64_t* in, uint32_t n_ct, uint32_t e, uint64_t* out,
                     hipStream_t st) {
    const uint64_t* key = nullptr;
    hc_status s = rk_of(rk, &key);
    if (s != HC_OK) return s;
    if (!c.d_mult) return HC_EINVAL;
    stage_reset(c.lane, st);
    // the largest batch whose workspace fits (halved until it does)
    int batch = (int)std::min<uint32_t>(n_ct, MUL_BATCH);
    while (c.lane.ws.reserve(mul_ws_bytes(c, batch)) != HC_OK) {
        if (batch == 1) return HC_ENOMEM;
        batch = (batch + 1) / 2;
    }
    MulWs w;
    if ((s = mul_ws(c, c.lane.ws, batch, w)) != HC_OK) return s;
    const size_t CW = 2 * (size_t)c.L * c.n;
    for (uint32_t i = 0; i < n_ct; i += batch) {
        const int cnt = (int)std::min<uint32_t>(batch, n_ct - i);
        if ((s = power_ct(c, c.lane, w, key, in + i * CW, e, out + i * CW, cnt, st)) != HC_OK) return s;
    }
    return HC_OK;
}

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_relin_keygen(hc_context* cp, const hc_sk* sk, const uint8_t seed[32], hc_gk** rk) {
    if (!cp || !sk || !seed || !rk) return HC_EINVAL;
    return ks_keygen(*cp, sk, nullptr, 0, seed, true, rk);
}

extern "C" hc_status hc_mul(hc_context* cp, const hc_gk* rk, const uint64_t* ct_a, const uint64_t* ct_b,
                            uint64_t* ct_out, hipStream_t st) {
    if (!cp || !ct_a || !ct_b || !ct_out) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    const uint64_t* key = nullptr;
    hc_status s = rk_of(rk, &key);
    if (s != HC_OK) return s;
    if (!c.d_mult) return HC_EINVAL;
    stage_reset(c.lane, st);
    if (c.lane.ws.reserve(mul_ws_bytes(c, 1)) != HC_OK) return HC_ENOMEM;
    MulWs w;
    if ((s = mul_ws(c, c.lane.ws, 1, w)) != HC_OK) return s;
    if ((s = mul_ct(c, c.lane, w.ks, key, const_cast<uint64_t*>(ct_a), ct_b, ct_out, 1, false, w.buf, st)) != HC_OK)
        return s;
    HC_CHECK(hipGetLastError());
    HC_CHECK(hipStreamSynchronize(st));
    return HC_OK;
}

extern "C" hc_status hc_power(hc_context* cp, const hc_gk* rk, const uint64_t* ct_in, uint32_t exponent,
                              uint64_t* ct_out, hipStream_t st) {
    if (!cp || !ct_in || !ct_out || exponent == 0) return HC_EINVAL;
    HC_CHECK(hipSetDevice(cp->device));
    hc_status s = power_many(*cp, rk, ct_in, 1, exponent, ct_out, st);
    if (s != HC_OK) return s;
    HC_CHECK(hipGetLastError());
    HC_CHECK(hipStreamSynchronize(st));
    return HC_OK;
}

extern "C" hc_status hc_match(hc_context* cp, const hc_gk* rk, const hc_db* keys, const uint64_t* ct_x, uint64_t N,
                              uint64_t* ct_v, hipStream_t st) {
    if (!cp || !keys || !ct_x || !ct_v || N == 0 || keys->ncol < 1 || keys->N < N || !keys->d_raw) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    const uint64_t* key = nullptr;
    hc_status s = rk_of(rk, &key);
    if (s != HC_OK) return s;
    if (!c.d_mult) return HC_EINVAL;
    const size_t n = c.n, L = c.L, CW = 2 * L * n;
    const uint32_t n_ct = (uint32_t)((N + n - 1) / n);
    // per ciphertext: the keys' plaintext m (coefficients mod p), the query minus it
    uint32_t *slots = nullptr, *m = nullptr;
    HC_CHECK(hipMalloc((void**)&slots, sizeof(uint32_t) * n));
    HC_CHECK(hipMalloc((void**)&m, sizeof(uint32_t) * n));
    for (uint32_t i = 0; i < n_ct; i++) {
        const uint64_t r0 = (uint64_t)i * n, cnt = std::min<uint64_t>(n, N - r0);
        k_zero(c, reinterpret_cast<uint64_t*>(slots), n / 2, st);
        HC_CHECK(hipMemcpyAsync(slots, keys->d_raw + r0, sizeof(uint32_t) * cnt, hipMemcpyDeviceToDevice, st));
        k_slots_to_eval(c, m, slots, 1, st);
        ntt32(c, m, 1, true, st);
        uint64_t* v = ct_v + i * CW;
        HC_CHECK(hipMemcpyAsync(v, ct_x, sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(sub_delta_m_kernel, dim3((unsigned)((n + 255) / 256), L), dim3(256), 0, st, v, m, c.d_mods,
                           c.d_delta, (int)n);
    }
    // Power_{p-1}, then 1 - v
    s = power_many(c, rk, ct_v, n_ct, (uint32_t)(c.p - 1), ct_v, st);
    if (s == HC_OK)
        for (uint32_t i = 0; i < n_ct; i++)
            hipLaunchKernelGGL(one_minus_kernel, dim3((unsigned)((n + 255) / 256), L, 2), dim3(256), 0, st,
                               ct_v + i * CW, c.d_mods, c.d_delta, (int)n, (int)L);
    // slots past the last record: multiplied by the 0/1 mask of the records present
    if (s == HC_OK && N % n) {
        std::vector<uint32_t> valid(n, 0);
        for (uint64_t r = 0; r < N % n; r++) valid[r] = 1;
        uint64_t *pt = nullptr, *tmp = nullptr;
        HC_CHECK(hipMalloc((void**)&pt, sizeof(uint64_t) * L * n));
        HC_CHECK(hipMalloc((void**)&tmp, sizeof(uint64_t) * CW));
        s = encode_plain(c, pt, valid.data(), 1, true, st);
        if (s == HC_OK) {
            uint64_t* last = ct_v + (size_t)(n_ct - 1) * CW;
            HC_CHECK(hipMemcpyAsync(tmp, last, sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
            ntt64(c, tmp, L * n, 2, 0, (int)L, false, st);
            k_mul_plain(c, tmp, tmp, pt, (int)L, st);
            ntt64(c, tmp, L * n, 2, 0, (int)L, true, st);
            HC_CHECK(hipMemcpyAsync(last, tmp, sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
        }
        HC_CHECK(hipStreamSynchronize(st));
        HC_CHECK(hipFree(pt));
        HC_CHECK(hipFree(tmp));
    }
    HC_CHECK(hipStreamSynchronize(st));
    HC_CHECK(hipFree(slots));
    HC_CHECK(hipFree(m));
    if (s != HC_OK) return s;
    HC_CHECK(hipGetLastError());
    return HC_OK;
}

extern "C" hc_status hc_compress_generic(hc_context* cp, const hc_gk* gk, const hc_gk* rk, const uint64_t* ct_d,
                                         uint64_t N, uint32_t t_bound, uint32_t comp_level, uint32_t out_level,
                                         uint64_t* ct_out, hc_compress_info* info, hipStream_t st) {
    if (!cp || !gk || !ct_d || !ct_out) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    std::vector<QueryRun> qs(1);
    hc_status s = make_plan(c, N, 1, t_bound, comp_level, out_level, qs[0].pl);
    if (s != HC_OK) return s;
    // v = Power_{p-1}(d) at the full level, the ciphertexts in lockstep
    const size_t CW = 2 * (size_t)c.L * c.n;
    uint64_t* v = nullptr;
    HC_CHECK(hipMalloc((void**)&v, sizeof(uint64_t) * CW * qs[0].pl.n_ct));
    s = power_many(c, rk, ct_d, qs[0].pl.n_ct, (uint32_t)(c.p - 1), v, st);
    if (s == HC_OK) {
        qs[0].ct_v = v;
        qs[0].ct_d = ct_d;
        qs[0].ct_out = ct_out;
        s = compress_many(c, c.lane, gk, nullptr, qs, st);
    }
    const hipError_t e = hipStreamSynchronize(st);
    (void)hipFree(v);
    if (s != HC_OK) return s;
    if (e != hipSuccess) return fail_hip(e, "hc_compress_generic", __FILE__, __LINE__);
    fill_info(qs[0], info);
    return HC_OK;
}
