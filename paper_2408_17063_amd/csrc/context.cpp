// Context creation: parameter derivation and the constant tables every kernel uses.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "hc_internal.h"

namespace hc {

hc_status upload_keccak_constants(const uint64_t rc[24], const uint32_t rho[25], const uint32_t cdt[20]);

hc_status fail_hip(hipError_t e, const char* what, const char* file, int line) {
    fprintf(stderr, "libhc: %s failed at %s:%d: %s\n", what, file, line, hipGetErrorString(e));
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? HC_ENOMEM : HC_EDEVICE;
}

// Device scratch of the allocation-free entry points (hc_rotate_level_noalloc): one
// copy per GPU, loaded with the code object and held until the process ends. Host
// code reaches it only through the address hipGetSymbolAddress returns for the
// current device (kept per context); the symbol itself is not a device address.
static __device__ __align__(256) uint64_t scratch[HC_NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)];

hc_status Arena::reserve(size_t bytes) {
    if (bytes <= cap) { used = 0; return HC_OK; }
    release();
    hipError_t e = hipMalloc((void**)&base, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // an allocation that did not fit leaves no error behind
        base = nullptr;
        cap = 0;
        return HC_ENOMEM;
    }
    cap = bytes;
    used = 0;
    return HC_OK;
}

void Arena::release() {
    if (base) (void)hipFree(base);
    base = nullptr;
    cap = 0;
    used = 0;
}

hc_status Lane::init(size_t stage_bytes) {
    stage_cap = stage_bytes;
    if (hipHostMalloc((void**)&stage_host, stage_cap, hipHostMallocDefault) != hipSuccess) {
        stage_host = nullptr;
        return HC_ENOMEM;
    }
    if (hipMalloc((void**)&stage_dev, stage_cap) != hipSuccess) {
        stage_dev = nullptr;
        return HC_ENOMEM;
    }
    if (hipEventCreateWithFlags(&copied, hipEventDisableTiming) != hipSuccess) {
        copied = nullptr;
        return HC_EDEVICE;
    }
    return HC_OK;
}

void Lane::release() {
    if (stage_host) (void)hipHostFree(stage_host);
    if (stage_dev) (void)hipFree(stage_dev);
    if (copied) (void)hipEventDestroy(copied);
    stage_host = nullptr;
    stage_dev = nullptr;
    copied = nullptr;
    ws.release();
}

// ------------------------------------------------------------------ number theory (host)

static bool is_prime_u64(uint64_t x) {
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (x < 2) return false;
    for (uint64_t b : bases) {
        if (x % b == 0) return x == b;
    }
    uint64_t d = x - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (uint64_t a : bases) {
        uint64_t y = h_powmod(a, d, x);
        if (y == 1 || y == x - 1) continue;
        bool comp = true;
        for (int i = 1; i < r; i++) {
            y = h_mulmod(y, y, x);
            if (y == x - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

static bool ntt_primes(int bits, int count, uint64_t two_n, const std::vector<uint64_t>& skip,
                       std::vector<uint64_t>& out) {
    uint64_t top = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
    uint64_t x = top / two_n * two_n + 1;
    if (x > top) x -= two_n;
    while ((int)out.size() < count) {
        if (x <= two_n) return false;
        if (std::find(skip.begin(), skip.end(), x) == skip.end() && is_prime_u64(x)) out.push_back(x);
        x -= two_n;
    }
    return true;
}

static uint32_t brv(uint32_t i, int bits) {
    uint32_t r = 0;
    for (int k = 0; k < bits; k++) { r = (r << 1) | (i & 1); i >>= 1; }
    return r;
}

// a primitive 2n-th root of unity mod q: g^((q-1)/2n) for the least g whose power has order 2n
static uint64_t root_2n(uint64_t q, uint64_t n) {
    for (uint64_t g = 2;; g++) {
        uint64_t x = h_powmod(g, (q - 1) / (2 * n), q);
        if (h_powmod(x, n, q) == q - 1) return x;
    }
}

// Keccak-f[1600] constants from their FIPS 202 definitions.
static void keccak_constants(uint64_t rc[24], uint32_t rho[25]) {
    // rc(t): LFSR x^8 + x^6 + x^5 + x^4 + 1 (FIPS 202 Alg. 5)
    auto rcbit = [](int t) -> int {
        if (t % 255 == 0) return 1;
        uint32_t R = 1;  // R[0] = 1, bits 0..7
        for (int i = 1; i <= t % 255; i++) {
            R <<= 1;     // R = 0 || R
            uint32_t r8 = (R >> 8) & 1;
            R ^= r8 << 0;
            R ^= r8 << 4;
            R ^= r8 << 5;
            R ^= r8 << 6;
            R &= 0xff;
        }
        return R & 1;
    };
    for (int ir = 0; ir < 24; ir++) {
        uint64_t c = 0;
        for (int j = 0; j <= 6; j++)
            if (rcbit(j + 7 * ir)) c |= 1ull << ((1 << j) - 1);
        rc[ir] = c;
    }
    // rho offsets: walk (x, y) <- (y, 2x + 3y) from (1, 0)
    for (int i = 0; i < 25; i++) rho[i] = 0;
    int x = 1, y = 0;
    for (int t = 0; t < 24; t++) {
        rho[x + 5 * y] = (uint32_t)(((t + 1) * (t + 2) / 2) % 64);
        int nx = y, ny = (2 * x + 3 * y) % 5;
        x = nx;
        y = ny;
    }
}

// CDF of |X| for P(X = x) ~ exp(-x^2 / (2 sigma^2)) on -19..19, scaled to 2^32.
static void gaussian_cdt(double sigma, uint32_t T[20]) {
    double rho[20], total;
    for (int x = 0; x < 20; x++) rho[x] = exp(-(double)(x * x) / (2.0 * sigma * sigma));
    total = rho[0];
    for (int x = 1; x < 20; x++) total += 2 * rho[x];
    double acc = 0;
    for (int k = 0; k < 20; k++) {
        acc += (k == 0) ? rho[0] : 2 * rho[k];
        double v = floor(acc / total * 4294967296.0 + 0.5);
        T[k] = (k == 19 || v >= 4294967295.0) ? 0xffffffffu : (uint32_t)v;
    }
}

template <typename T>
static hc_status upload(Ctx& c, T** dst, const std::vector<T>& src) {
    HC_CHECK(hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1)));
    c.owned.push_back(*dst);
    if (!src.empty()) HC_CHECK(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return HC_OK;
}

hc_status encode_plain(Ctx& c, uint64_t* out, const uint32_t* host_slots, int count, bool mont,
                       hipStream_t st);
hc_status build_ms_tables(Ctx& c);
hc_status build_mult_tables(Ctx& c);

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_context_create(const hc_params* prm, int device, hc_context** out) {
    if (!prm || !out) return HC_EINVAL;
    *out = nullptr;
    if (prm->log_n < 10 || prm->log_n > 16) return HC_EINVAL;
    if (prm->K < 1 || prm->K > 4 || prm->L < 1 || prm->L % prm->K) return HC_EINVAL;
    if (prm->q_bits < 30 || prm->q_bits > 60 || prm->p_bits < 30 || prm->p_bits > 61) return HC_EINVAL;
    const uint64_t n = 1ull << prm->log_n;
    if (prm->p >= (1ull << 26) || (prm->p - 1) % (2 * n) != 0 || !is_prime_u64(prm->p)) return HC_EINVAL;
    if (prm->L + prm->K > 64) return HC_EINVAL;

    int ndev = 0;
    HC_CHECK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return HC_EINVAL;
    HC_CHECK(hipSetDevice(device));
    int cus = 0;
    HC_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));

    Ctx* cp = new Ctx();
    Ctx& c = *cp;
    c.device = device;
    c.cus = cus;
    c.logn = prm->log_n;
    c.n = (int)n;
    c.nh = c.n / 2;
    c.L = prm->L;
    c.K = prm->K;
    c.alpha = prm->K;
    c.dnum = prm->L / prm->K;
    c.nq = c.L + c.K;
    c.p = prm->p;

    std::vector<uint64_t> qs, sps;
    if (!ntt_primes(prm->q_bits, c.L, 2 * n, {}, qs) || !ntt_primes(prm->p_bits, c.K, 2 * n, qs, sps)) {
        delete cp;
        return HC_EINVAL;
    }
    c.primes = qs;
    c.primes.insert(c.primes.end(), sps.begin(), sps.end());
    // the key inner product reduces a sum of dnum products below q^2 with one
    // Montgomery reduction, which needs dnum q < 2^64
    for (uint64_t q : c.primes)
        if ((unsigned __int128)c.dnum * q >= ((unsigned __int128)1 << 64)) {
            delete cp;
            return HC_EINVAL;
        }
    // the auxiliary basis B of ciphertext products (L + 1 primes below 2^61, distinct from
    // every q_i and p_k): the tensor of two centred ciphertexts is exact over Q and B
    {
        std::vector<uint64_t> skip = c.primes, bs;
        if (!ntt_primes(61, c.L + 1, 2 * n, skip, bs)) {
            delete cp;
            return HC_EINVAL;
        }
        c.nb = (int)bs.size();
        c.primes.insert(c.primes.end(), bs.begin(), bs.end());
    }
    c.ntab = c.nq + c.nb;
    const int nq = c.nq, L = c.L, K = c.K, logn = c.logn, ntab = c.ntab;

    // ---- NTT tables for every prime (Q, P and B)
    c.h_tw.assign((size_t)ntab * 4 * n, 0);
    std::vector<uint64_t> ninv(4 * ntab), qinv(ntab), r2(ntab);
    for (int i = 0; i < ntab; i++) {
        uint64_t q = c.primes[i];
        uint64_t psi = root_2n(q, n), psii = h_invmod(psi, q);
        uint64_t* t = c.h_tw.data() + (size_t)i * 4 * n;
        std::vector<uint64_t> pw(n), pwi(n);
        pw[0] = pwi[0] = 1;
        for (uint32_t k = 1; k < n; k++) {
            pw[k] = h_mulmod(pw[k - 1], psi, q);
            pwi[k] = h_mulmod(pwi[k - 1], psii, q);
        }
        // layout [direction][k][(w, w')]
        for (uint32_t k = 0; k < n; k++) {
            uint32_t e = brv(k, logn);
            t[2 * k] = pw[e];
            t[2 * k + 1] = h_shoup_const(pw[e], q);
            t[2 * n + 2 * k] = pwi[e];
            t[2 * n + 2 * k + 1] = h_shoup_const(pwi[e], q);
        }
        // n^-1 and, for the inverse transform's last stage, its one twiddle times n^-1
        ninv[4 * i] = h_invmod(n % q, q);
        ninv[4 * i + 1] = h_shoup_const(ninv[4 * i], q);
        ninv[4 * i + 2] = h_mulmod(t[2 * n + 2], ninv[4 * i], q);
        ninv[4 * i + 3] = h_shoup_const(ninv[4 * i + 2], q);
        qinv[i] = h_mont_qinv(q);
        r2[i] = h_mulmod(h_to_mont(1, q), h_to_mont(1, q), q);  // 2^128 mod q
    }
    c.h_qinv = qinv;
    c.h_r2 = r2;

    // ---- slot transform mod p: zeta = least x >= 2 with x^n = -1
    uint32_t p = (uint32_t)c.p;
    uint32_t zeta = 2;
    while (h_powmod(zeta, n, p) != p - 1) zeta++;
    c.zeta = zeta;
    c.h_twp.assign((size_t)4 * n, 0);
    uint32_t zinv = (uint32_t)h_invmod(zeta, p);
    std::vector<uint32_t> zp(n), zpi(n);
    zp[0] = zpi[0] = 1;
    for (uint32_t k = 1; k < n; k++) {
        zp[k] = (uint32_t)((uint64_t)zp[k - 1] * zeta % p);
        zpi[k] = (uint32_t)((uint64_t)zpi[k - 1] * zinv % p);
    }
    for (uint32_t k = 0; k < n; k++) {
        uint32_t e = brv(k, logn);
        uint32_t w = zp[e], wi = zpi[e];
        c.h_twp[2 * k] = w;
        c.h_twp[2 * k + 1] = (uint32_t)(((uint64_t)w << 32) / p);
        c.h_twp[2 * n + 2 * k] = wi;
        c.h_twp[2 * n + 2 * k + 1] = (uint32_t)(((uint64_t)wi << 32) / p);
    }
    uint32_t ninvp = (uint32_t)h_invmod(n % p, p);
    const uint32_t w1ninv = (uint32_t)(((uint64_t)c.h_twp[2 * n + 2] * ninvp) % p);
    std::vector<uint32_t> ninvp_v = {ninvp, (uint32_t)(((uint64_t)ninvp << 32) / p), w1ninv,
                                     (uint32_t)(((uint64_t)w1ninv << 32) / p)};
    // slot (r, c) <-> evaluation at zeta^e, e = (-1)^r 3^c mod 2n; forward NTT entry i
    // holds the evaluation at zeta^(2 brv(i) + 1)
    c.h_slotpos.assign(n, 0);
    std::vector<uint32_t> posslot(n);
    uint64_t e = 1;
    for (int col = 0; col < c.nh; col++) {
        uint64_t e0 = e, e1 = (2 * n - e) % (2 * n);
        c.h_slotpos[col] = brv((uint32_t)((e0 - 1) / 2), logn);
        c.h_slotpos[c.nh + col] = brv((uint32_t)((e1 - 1) / 2), logn);
        e = e * 3 % (2 * n);
    }
    for (uint32_t i = 0; i < n; i++) posslot[c.h_slotpos[i]] = i;

    // ---- basis conversion constants
    const int alpha = c.alpha, dnum = c.dnum;
    std::vector<uint64_t> modup_inv((size_t)dnum * alpha * 2), modup_c((size_t)dnum * alpha * nq);
    for (int j = 0; j < dnum; j++) {
        for (int a = 0; a < alpha; a++) {
            int i = j * alpha + a;
            uint64_t qi = c.primes[i];
            // (D_j / q_i) mod q_i and mod every r
            uint64_t hat_qi = 1;
            for (int a2 = 0; a2 < alpha; a2++)
                if (a2 != a) hat_qi = h_mulmod(hat_qi, c.primes[j * alpha + a2] % qi, qi);
            uint64_t iv = h_invmod(hat_qi, qi);
            modup_inv[((size_t)j * alpha + a) * 2] = iv;
            modup_inv[((size_t)j * alpha + a) * 2 + 1] = h_shoup_const(iv, qi);
            for (int r = 0; r < nq; r++) {
                uint64_t m = c.primes[r], h = 1;
                for (int a2 = 0; a2 < alpha; a2++)
                    if (a2 != a) h = h_mulmod(h, c.primes[j * alpha + a2] % m, m);
                modup_c[((size_t)j * alpha + a) * nq + r] = h_to_mont(h, m);
            }
        }
    }
    std::vector<uint64_t> moddown_inv((size_t)K * 2), moddown_c((size_t)K * L), pinv((size_t)L * 2),
        pmodq(L), delta((size_t)L * 2);
    for (int k = 0; k < K; k++) {
        uint64_t pk = c.primes[L + k];
        uint64_t h = 1;
        for (int k2 = 0; k2 < K; k2++)
            if (k2 != k) h = h_mulmod(h, c.primes[L + k2] % pk, pk);
        moddown_inv[2 * k] = h_invmod(h, pk);
        moddown_inv[2 * k + 1] = h_shoup_const(moddown_inv[2 * k], pk);
        for (int i = 0; i < L; i++) {
            uint64_t qi = c.primes[i], hq = 1;
            for (int k2 = 0; k2 < K; k2++)
                if (k2 != k) hq = h_mulmod(hq, c.primes[L + k2] % qi, qi);
            moddown_c[(size_t)k * L + i] = h_to_mont(hq, qi);
        }
    }
    uint64_t Qmodp = 1;
    for (int i = 0; i < L; i++) Qmodp = h_mulmod(Qmodp, c.primes[i] % c.p, c.p);
    for (int i = 0; i < L; i++) {
        uint64_t qi = c.primes[i], P = 1;
        for (int k = 0; k < K; k++) P = h_mulmod(P, c.primes[L + k] % qi, qi);
        pmodq[i] = P;
        pinv[2 * i] = h_invmod(P, qi);
        pinv[2 * i + 1] = h_shoup_const(pinv[2 * i], qi);
        // Delta = (Q - (Q mod p)) / p, and Q = 0 mod q_i
        uint64_t d = h_mulmod((qi - Qmodp % qi) % qi, h_invmod(c.p % qi, qi), qi);
        delta[2 * i] = d;
        delta[2 * i + 1] = h_shoup_const(d, qi);
    }

    // ---- samplers
    uint64_t rc[24];
    uint32_t rho[25];
    keccak_constants(rc, rho);
    c.h_cdt.assign(20, 0);
    gaussian_cdt(3.2, c.h_cdt.data());

    hc_status st = HC_OK;
#define UP(dst, src) if ((st = upload(c, &dst, src)) != HC_OK) { hc_context_destroy(cp); return st; }
    UP(c.d_mods, c.primes);
    UP(c.d_qinv, qinv);
    UP(c.d_r2, r2);
    UP(c.d_tw, c.h_tw);
    UP(c.d_ninv, ninv);
    UP(c.d_modp, std::vector<uint32_t>{p});
    UP(c.d_twp, c.h_twp);
    UP(c.d_ninvp, ninvp_v);
    UP(c.d_slotpos, c.h_slotpos);
    UP(c.d_posslot, posslot);
    UP(c.d_modup_inv, modup_inv);
    UP(c.d_modup_c, modup_c);
    UP(c.d_moddown_inv, moddown_inv);
    UP(c.d_moddown_c, moddown_c);
    UP(c.d_pinv, pinv);
    UP(c.d_pmodq, pmodq);
    UP(c.d_delta, delta);
    {
        // n^-1 (and W^-1[1] n^-1) times the factor the base conversion of key switching
        // multiplies a coefficient by before its sum, (D_j/q_i)^-1 mod q_i for a ciphertext
        // prime of digit j and (P/p_k)^-1 mod p_k for a special prime: an inverse transform
        // with these final constants yields the factored residues directly
        std::vector<uint64_t> nconv(4 * (size_t)nq);
        for (int i = 0; i < nq; i++) {
            const uint64_t q = c.primes[i];
            const uint64_t f = i < L ? modup_inv[2 * (size_t)i] : moddown_inv[2 * (size_t)(i - L)];
            nconv[4 * i] = h_mulmod(ninv[4 * i], f, q);
            nconv[4 * i + 1] = h_shoup_const(nconv[4 * i], q);
            nconv[4 * i + 2] = h_mulmod(ninv[4 * i + 2], f, q);
            nconv[4 * i + 3] = h_shoup_const(nconv[4 * i + 2], q);
        }
        UP(c.d_ninv_conv, nconv);
    }
    {
        // digit weights of the matrix-core multiply-accumulate: 256^s 2^64 mod q_i
        std::vector<uint64_t> mfw((size_t)L * 16, 0);
        for (int i = 0; i < L; i++)
            for (int s = 0; s < 13; s++) mfw[(size_t)i * 16 + s] = h_to_mont(h_powmod(256, (uint64_t)s, c.primes[i]), c.primes[i]);
        UP(c.d_mfw, mfw);
    }
#undef UP
    // the allocation-free scratch of this device (the device is current here)
    {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fprintf(stderr, "libhc: no allocation-free scratch on device %d: %s\n", device, hipGetErrorString(e));
            ptr = nullptr;
        }
        c.d_scratch = (uint64_t*)ptr;
    }
    if ((st = ntt_build_tw2(c)) != HC_OK) { hc_context_destroy(cp); return st; }
    if ((st = build_ms_tables(c)) != HC_OK) { hc_context_destroy(cp); return st; }
    if ((st = build_mult_tables(c)) != HC_OK) { hc_context_destroy(cp); return st; }
    if ((st = upload_keccak_constants(rc, rho, c.h_cdt.data())) != HC_OK) { hc_context_destroy(cp); return st; }

    // ---- row masks [1;0] and [0;1] as plaintext multipliers
    std::vector<uint32_t> rows((size_t)2 * n, 0);
    for (int col = 0; col < c.nh; col++) { rows[col] = 1; rows[(size_t)n + c.nh + col] = 1; }
    for (int r = 0; r < 2; r++) {
        if (hipMalloc((void**)&c.d_rowmask[r], sizeof(uint64_t) * (size_t)L * n) != hipSuccess) {
            hc_context_destroy(cp);
            return HC_ENOMEM;
        }
        c.owned.push_back(c.d_rowmask[r]);
    }
    if ((st = encode_plain(c, c.d_rowmask[0], rows.data(), 1, true, 0)) != HC_OK ||
        (st = encode_plain(c, c.d_rowmask[1], rows.data() + n, 1, true, 0)) != HC_OK) {
        hc_context_destroy(cp);
        return st;
    }
    // staging for per-call tables
    if (c.lane.init((size_t)8 << 20) != HC_OK) {
        hc_context_destroy(cp);
        return HC_ENOMEM;
    }
    if (hipDeviceSynchronize() != hipSuccess) { hc_context_destroy(cp); return HC_EDEVICE; }
    *out = cp;
    return HC_OK;
}

extern "C" void hc_context_destroy(hc_context* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (void* p : c->owned) (void)hipFree(p);
    for (auto& kv : c->prefix_masks) (void)hipFree(kv.second);
    for (auto& kv : c->diag_tabs) (void)hipFree(kv.second.d);
    c->lane.release();
    for (auto& t : c->tlaunches) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    delete c;
}

extern "C" void hc_context_trim(hc_context* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->lane.ws.release();
}

extern "C" hc_status hc_context_primes(const hc_context* c, uint64_t* out) {
    if (!c || !out) return HC_EINVAL;
    for (int i = 0; i < c->nq; i++) out[i] = c->primes[i];
    return HC_OK;
}

extern "C" const char* hc_status_str(hc_status s) {
    switch (s) {
        case HC_OK: return "ok";
        case HC_EINVAL: return "invalid argument";
        case HC_ENOMEM: return "out of memory";
        case HC_EDEVICE: return "device error";
        case HC_ENOKEY: return "missing Galois key";
        case HC_EDECODE: return "decoding failed";
        case HC_ENOISE: return "noise at the decryption budget";
        case HC_ESCRATCH: return "call exceeds the fixed allocation-free scratch";
    }
    return "unknown status";
}

// ------------------------------------------------------------------ kernel timing

namespace hc {

static hipEvent_t pool_get(const hc_context& c) {
    std::lock_guard<std::mutex> g(c.timing_mu);
    if (!c.event_pool.empty()) {
        hipEvent_t e = c.event_pool.back();
        c.event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

TimeScope*& TimeScope::current() {
    static thread_local TimeScope* cur = nullptr;
    return cur;
}

TimeScope::TimeScope(const hc_context& c_, int kind_, hipStream_t st_, double bytes_, double ops_)
    : c(c_), kind(kind_), st(st_), bytes(bytes_), ops(ops_) {
    if (!c.timing) return;
    a = pool_get(c);
    b = pool_get(c);
    if (!a || !b) {
        std::lock_guard<std::mutex> g(c.timing_mu);
        if (a) c.event_pool.push_back(a);
        if (b) c.event_pool.push_back(b);
        a = b = nullptr;
        return;
    }
    prev = current();
    current() = this;
}

TimeScope::~TimeScope() {
    if (!c.timing || !a || !b) return;
    current() = prev;
    if (!used) {  // no kernel launched through hc_launch: nothing to time
        std::lock_guard<std::mutex> g(c.timing_mu);
        c.event_pool.push_back(a);
        c.event_pool.push_back(b);
        return;
    }
    std::lock_guard<std::mutex> g(c.timing_mu);
    c.tlaunches.push_back({kind, a, b, bytes, ops});
}

}  // namespace hc

extern "C" hc_status hc_timing_enable(hc_context* c, int enable) {
    if (!c) return HC_EINVAL;
    HC_CHECK(hipSetDevice(c->device));
    HC_CHECK(hipDeviceSynchronize());
    // An event a kernel launch carried stays bound to that launch, which holds on to the
    // device memory the kernel used (memory freed since stays allocated): such events are
    // destroyed here, never reused.
    std::lock_guard<std::mutex> g(c->timing_mu);
    for (auto& t : c->tlaunches) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    c->tlaunches.clear();
    c->timing = enable != 0;
    return HC_OK;
}

extern "C" hc_status hc_timing_read(hc_context* c, int kind, double* total_ms, uint64_t* launches,
                                    double* work_bytes, double* work_ops) {
    if (!c || kind < 0 || kind >= HC_KT_COUNT) return HC_EINVAL;
    HC_CHECK(hipSetDevice(c->device));
    HC_CHECK(hipDeviceSynchronize());
    double ms = 0, by = 0, op = 0;
    uint64_t cnt = 0;
    std::lock_guard<std::mutex> g(c->timing_mu);
    for (auto& t : c->tlaunches) {
        if (t.kind != kind) continue;
        float e = 0;
        HC_CHECK(hipEventElapsedTime(&e, t.a, t.b));
        ms += e;
        by += t.bytes;
        op += t.ops;
        cnt++;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = cnt;
    if (work_bytes) *work_bytes = by;
    if (work_ops) *work_ops = op;
    return HC_OK;
}
