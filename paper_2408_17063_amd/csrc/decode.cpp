// Client side on the host: decryption and decompression.
//
// Decryption: x = [c0 + c1 s]_Q (ring product by a host NTT per prime), then
// m = round(p x / Q) mod p computed exactly in RNS: with y_i = [x_i (Q/q_i)^-1]_{q_i},
// x = sum_i y_i (Q/q_i) - v Q for an integer v, so p x / Q = sum_i y_i p / q_i - v p
// and, modulo p, m = sum_i floor(y_i p / q_i) + round(sum_i frac(y_i p / q_i)).
// The fractional parts are summed in 64.64 fixed point (error < L 2^-64); a sum
// within 2^-50 of one half is reported as HC_ENOISE instead of guessed.
//
// Decompression (Alg. 6 with Alg. 1 and Alg. 4): Newton's identities give the
// polynomial whose roots are the matched indices padded with zeros; the X
// factors are stripped; the roots are found with Cantor-Zassenhaus equal-degree
// splitting over F_p (after checking the polynomial divides X^p - X); the
// values come from the l x l transposed-Vandermonde system of the first l
// power sums, solved with the Lagrange basis in O(l^2), and the remaining
// s - l equations are verified.
#include <string.h>

#include <algorithm>
#include <random>

#include "hc_internal.h"

namespace hc {

// ------------------------------------------------------------------ host NTT (same ordering as the device)

// tw: (w, w') pairs, forward direction
static void host_ntt(uint64_t* a, int n, int logn, const uint64_t* tw, uint64_t q) {
    int t = n;
    for (int m = 1; m < n; m <<= 1) {
        t >>= 1;
        for (int i = 0; i < m; i++) {
            uint64_t w = tw[2 * (m + i)], wp = tw[2 * (m + i) + 1];
            int j1 = 2 * i * t;
            for (int j = j1; j < j1 + t; j++) {
                uint64_t U = a[j], V = shoup(a[j + t], w, wp, q);
                a[j] = add_mod(U, V, q);
                a[j + t] = sub_mod(U, V, q);
            }
        }
    }
    (void)logn;
}

// tw: (w, w') pairs, inverse direction
static void host_intt(uint64_t* a, int n, const uint64_t* tw, uint64_t q, uint64_t ninv, uint64_t ninvp) {
    int t = 1;
    for (int m = n >> 1; m >= 1; m >>= 1) {
        for (int i = 0; i < m; i++) {
            uint64_t w = tw[2 * (m + i)], wp = tw[2 * (m + i) + 1];
            int j1 = 2 * i * t;
            for (int j = j1; j < j1 + t; j++) {
                uint64_t U = a[j], V = a[j + t];
                a[j] = add_mod(U, V, q);
                a[j + t] = shoup(sub_mod(U, V, q), w, wp, q);
            }
        }
        t <<= 1;
    }
    for (int j = 0; j < n; j++) a[j] = shoup(a[j], ninv, ninvp, q);
}

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_decrypt(hc_context* cp, const hc_sk* sk, const uint64_t* ct, uint32_t level,
                                uint32_t* slots_out) {
    if (!cp || !sk || !ct || !slots_out) return HC_EINVAL;
    Ctx& c = *cp;
    if (level < 1 || (int)level > c.L) return HC_EINVAL;
    const int n = c.n, L = (int)level;
    const uint64_t p = c.p;
    std::vector<uint64_t> x((size_t)L * n), s(n), t(n);
    for (int i = 0; i < L; i++) {
        const uint64_t q = c.primes[i];
        const uint64_t* tw = c.h_tw.data() + (size_t)i * 4 * n;
        const uint64_t* c0 = ct + (size_t)i * n;
        const uint64_t* c1 = ct + (size_t)(L + i) * n;
        for (int j = 0; j < n; j++) {
            if (c0[j] >= q || c1[j] >= q) return HC_EINVAL;
            s[j] = sk->s[j] < 0 ? q - 1 : (uint64_t)sk->s[j];
            t[j] = c1[j];
        }
        host_ntt(s.data(), n, c.logn, tw, q);
        host_ntt(t.data(), n, c.logn, tw, q);
        for (int j = 0; j < n; j++) t[j] = h_mulmod(t[j], s[j], q);
        uint64_t ninv = h_invmod((uint64_t)n % q, q);
        host_intt(t.data(), n, tw + 2 * n, q, ninv, h_shoup_const(ninv, q));
        for (int j = 0; j < n; j++) x[(size_t)i * n + j] = add_mod(c0[j], t[j], q);
    }
    // y_i multipliers (Q/q_i)^-1 mod q_i
    std::vector<uint64_t> qhat_inv(L);
    for (int i = 0; i < L; i++) {
        uint64_t q = c.primes[i], h = 1;
        for (int k = 0; k < L; k++)
            if (k != i) h = h_mulmod(h, c.primes[k] % q, q);
        qhat_inv[i] = h_invmod(h, q);
    }
    std::vector<uint64_t> m(n);
    for (int j = 0; j < n; j++) {
        uint64_t ip = 0;                  // integer part mod p
        unsigned __int128 frac = 0;       // 64.64 fixed point
        for (int i = 0; i < L; i++) {
            uint64_t q = c.primes[i];
            uint64_t yi = h_mulmod(x[(size_t)i * n + j], qhat_inv[i], q);
            unsigned __int128 v = (unsigned __int128)yi * p;
            uint64_t quo = (uint64_t)(v / q), rem = (uint64_t)(v % q);
            ip = (ip + quo % p) % p;
            frac += (unsigned __int128)(((unsigned __int128)rem << 64) / q);
        }
        uint64_t fint = (uint64_t)(frac >> 64), ffrac = (uint64_t)frac;
        const uint64_t half = 1ull << 63, tol = 1ull << 14;  // 2^-50 in 2^-64 units
        if (ffrac > half - tol && ffrac < half + tol) return HC_ENOISE;
        uint64_t rnd = fint + (ffrac >= half ? 1 : 0);
        m[j] = (ip + rnd % p) % p;
    }
    // decode: forward transform mod p, slot (r, col) at its evaluation position
    std::vector<uint64_t> W(2 * (size_t)n);
    for (int k = 0; k < n; k++) { W[2 * k] = c.h_twp[2 * k]; W[2 * k + 1] = h_shoup_const(W[2 * k], p); }
    host_ntt(m.data(), n, c.logn, W.data(), p);
    for (int i = 0; i < n; i++) slots_out[i] = (uint32_t)m[c.h_slotpos[i]];
    return HC_OK;
}

// ------------------------------------------------------------------ decompression

namespace {

typedef std::vector<uint64_t> Pol;  // coefficients, lowest degree first, mod p

struct Fp {
    uint64_t p;
    uint64_t mul(uint64_t a, uint64_t b) const { return a * b % p; }
    uint64_t add(uint64_t a, uint64_t b) const { return (a + b) % p; }
    uint64_t sub(uint64_t a, uint64_t b) const { return (a + p - b) % p; }
    uint64_t pw(uint64_t a, uint64_t e) const {
        uint64_t r = 1;
        a %= p;
        while (e) {
            if (e & 1) r = mul(r, a);
            a = mul(a, a);
            e >>= 1;
        }
        return r;
    }
    uint64_t inv(uint64_t a) const { return pw(a, p - 2); }

    void trim(Pol& a) const {
        while (!a.empty() && a.back() == 0) a.pop_back();
    }
    Pol mulp(const Pol& a, const Pol& b) const {
        if (a.empty() || b.empty()) return {};
        std::vector<unsigned __int128> acc(a.size() + b.size() - 1, 0);
        for (size_t i = 0; i < a.size(); i++)
            if (a[i])
                for (size_t j = 0; j < b.size(); j++) acc[i + j] += (unsigned __int128)a[i] * b[j];
        Pol r(acc.size());
        for (size_t i = 0; i < acc.size(); i++) r[i] = (uint64_t)(acc[i] % p);
        trim(r);
        return r;
    }
    // a mod m (m monic or not), returns remainder
    Pol modp(Pol a, const Pol& m) const {
        trim(a);
        if (m.empty()) return a;
        uint64_t li = inv(m.back());
        size_t dm = m.size() - 1;
        while (a.size() > dm && !a.empty()) {
            uint64_t coef = mul(a.back(), li);
            size_t shift = a.size() - 1 - dm;
            for (size_t i = 0; i <= dm; i++) a[shift + i] = sub(a[shift + i], mul(coef, m[i]));
            a.pop_back();
            trim(a);
        }
        return a;
    }
    Pol divp(Pol a, const Pol& m) const {  // exact quotient a / m
        trim(a);
        size_t dm = m.size() - 1;
        if (a.size() <= dm) return {};
        Pol q(a.size() - dm, 0);
        uint64_t li = inv(m.back());
        while (a.size() > dm) {
            uint64_t coef = mul(a.back(), li);
            size_t shift = a.size() - 1 - dm;
            q[shift] = coef;
            for (size_t i = 0; i <= dm; i++) a[shift + i] = sub(a[shift + i], mul(coef, m[i]));
            a.pop_back();
        }
        return q;
    }
    Pol gcd(Pol a, Pol b) const {
        trim(a);
        trim(b);
        while (!b.empty()) {
            Pol r = modp(a, b);
            a = b;
            b = r;
        }
        if (!a.empty()) {  // monic
            uint64_t li = inv(a.back());
            for (auto& v : a) v = mul(v, li);
        }
        return a;
    }
    // base^e mod m
    Pol powmod(Pol base, uint64_t e, const Pol& m) const {
        Pol r = {1};
        base = modp(base, m);
        while (e) {
            if (e & 1) r = modp(mulp(r, base), m);
            base = modp(mulp(base, base), m);
            e >>= 1;
        }
        return r;
    }
};

// roots of a squarefree g that splits into distinct linear factors over F_p
static void split_roots(const Fp& F, const Pol& g, std::mt19937_64& rng, std::vector<uint64_t>& out) {
    size_t d = g.size() - 1;
    if (d == 0) return;
    if (d == 1) {  // g = g1 X + g0
        out.push_back(F.mul(F.sub(0, g[0]), F.inv(g[1])));
        return;
    }
    for (int attempt = 0; attempt < 200; attempt++) {
        uint64_t a = rng() % F.p;
        Pol h = F.powmod(Pol{a, 1}, (F.p - 1) / 2, g);  // (X + a)^((p-1)/2) mod g
        if (h.empty()) h = {0};
        h[0] = F.sub(h[0], 1);
        F.trim(h);
        Pol f = F.gcd(h, g);
        size_t df = f.empty() ? 0 : f.size() - 1;
        if (df > 0 && df < d) {
            split_roots(F, f, rng, out);
            split_roots(F, F.divp(g, f), rng, out);
            return;
        }
    }
}

}  // namespace

extern "C" hc_status hc_decompress(uint64_t p, uint64_t N_group, uint32_t s, uint32_t ncols,
                                   const uint32_t* w, const uint32_t* e, uint64_t* idx_out,
                                   uint32_t* val_out, uint32_t* count_out) {
    if (!w || !idx_out || !count_out || (ncols && (!e || !val_out))) return HC_EINVAL;
    if (p < 3 || p >= (1ull << 31) || N_group == 0 || N_group >= p || s == 0 || s >= p) return HC_EINVAL;
    Fp F{p};
    // Alg. 1 step 1: a_0 = 1, a_k = k^-1 sum_{i=1..k} (-1)^(i-1) a_{k-i} w_i
    std::vector<uint64_t> a(s + 1, 0);
    a[0] = 1;
    for (uint32_t k = 1; k <= s; k++) {
        uint64_t acc = 0;
        for (uint32_t i = 1; i <= k; i++) {
            uint64_t t = F.mul(a[k - i], w[i - 1] % p);
            acc = (i % 2 == 1) ? F.add(acc, t) : F.sub(acc, t);
        }
        a[k] = F.mul(acc, F.inv(k));
    }
    // f = sum_k (-1)^k a_k X^(s-k); lowest degree first: coefficient of X^j is (-1)^(s-j) a_{s-j}
    Pol f(s + 1);
    for (uint32_t j = 0; j <= s; j++) {
        uint64_t v = a[s - j];
        f[j] = ((s - j) % 2 == 0) ? v : F.sub(0, v);
    }
    // strip factors X (the zero padding of the multiset)
    size_t z = 0;
    while (z < f.size() - 1 && f[z] == 0) z++;
    Pol g(f.begin() + z, f.end());
    const size_t deg = g.size() - 1;
    std::vector<uint64_t> roots;
    if (deg > 0) {
        // all roots in F_p and distinct  <=>  g | X^p - X
        Pol xp = F.powmod(Pol{0, 1}, p, g);
        if (xp.size() < 2) xp.resize(2, 0);
        xp[1] = F.sub(xp[1], 1);
        xp = F.modp(xp, g);  // X itself is not reduced when deg g = 1
        if (!xp.empty()) return HC_EDECODE;
        std::mt19937_64 rng(0x9E3779B97F4A7C15ull ^ p ^ ((uint64_t)s << 32));
        split_roots(F, g, rng, roots);
        if (roots.size() != deg) return HC_EDECODE;
    }
    std::sort(roots.begin(), roots.end());
    for (size_t i = 0; i < roots.size(); i++) {
        if (roots[i] == 0 || roots[i] > N_group) return HC_EDECODE;
        if (i && roots[i] == roots[i - 1]) return HC_EDECODE;
    }
    {   // the power sums of the roots must reproduce every w_j (Lemma 2)
        std::vector<uint64_t> pw(roots);
        for (uint32_t j = 0; j < s; j++) {
            uint64_t acc = 0;
            for (size_t k = 0; k < roots.size(); k++) {
                acc = F.add(acc, pw[k]);
                pw[k] = F.mul(pw[k], roots[k]);
            }
            if (acc != w[j] % p) return HC_EDECODE;
        }
    }
    const size_t l = roots.size();
    // Alg. 4: sum_k d_k x_k^(j+1) = e_j. With z_k = d_k x_k this is the transposed
    // Vandermonde system sum_k z_k x_k^j = e_j (j < l), solved by the Lagrange basis:
    // z_k = sum_j [X^j] (M(X) / (X - x_k)) e_j / M'(x_k), M = prod (X - x_m).
    Pol M = {1};
    for (uint64_t r : roots) M = F.mulp(M, Pol{F.sub(0, r), 1});
    if (M.size() < l + 1) M.resize(l + 1, 0);
    std::vector<std::vector<uint64_t>> basis(l);  // quotient coefficients, and 1/M'(x_k)
    std::vector<uint64_t> dinv(l);
    for (size_t k = 0; k < l; k++) {
        std::vector<uint64_t> qk(l, 0);  // M / (X - x_k) by synthetic division
        uint64_t carry = 0;
        for (size_t j = l; j-- > 0;) {
            carry = F.add(M[j + 1], F.mul(carry, roots[k]));
            qk[j] = carry;
        }
        uint64_t val = 0;  // qk(x_k) = M'(x_k)
        for (size_t j = l; j-- > 0;) val = F.add(F.mul(val, roots[k]), qk[j]);
        dinv[k] = F.inv(val);
        basis[k] = std::move(qk);
    }
    for (uint32_t col = 0; col < ncols; col++) {
        const uint32_t* ec = e + (size_t)col * s;
        std::vector<uint64_t> d(l);
        for (size_t k = 0; k < l; k++) {
            uint64_t acc = 0;
            for (size_t j = 0; j < l; j++) acc = F.add(acc, F.mul(basis[k][j], ec[j] % p));
            uint64_t zk = F.mul(acc, dinv[k]);
            d[k] = F.mul(zk, F.inv(roots[k]));
        }
        // verify every equation j = 1..s
        std::vector<uint64_t> pw(l);
        for (size_t k = 0; k < l; k++) pw[k] = roots[k];
        for (uint32_t j = 0; j < s; j++) {
            uint64_t acc = 0;
            for (size_t k = 0; k < l; k++) {
                acc = F.add(acc, F.mul(d[k], pw[k]));
                pw[k] = F.mul(pw[k], roots[k]);
            }
            if (acc != ec[j] % p) return HC_EDECODE;
        }
        for (size_t k = 0; k < l; k++) val_out[(size_t)col * s + k] = (uint32_t)d[k];
    }
    for (size_t k = 0; k < l; k++) idx_out[k] = roots[k];
    *count_out = (uint32_t)l;
    return HC_OK;
}
