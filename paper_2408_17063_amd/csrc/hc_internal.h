// Internal declarations of libhc: the context, key and database objects and
// the device launchers the host orchestration calls.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hc.h"
#include "../../include/hc_kernels.h"
#include "modarith.h"

#define HC_CHECK(x)                                            \
    do {                                                       \
        hipError_t e_ = (x);                                   \
        if (e_ != hipSuccess) return hc::fail_hip(e_, #x, __FILE__, __LINE__); \
    } while (0)

namespace hc {

hc_status fail_hip(hipError_t e, const char* what, const char* file, int line);

// A grow-only device arena for per-call temporaries.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    hc_status reserve(size_t bytes);   // (re)allocates; invalidates earlier pointers
    void reset() { used = 0; }
    template <typename T> T* take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
        if (used + bytes > cap) return nullptr;
        T* p = reinterpret_cast<T*>(base + used);
        used += bytes;
        return p;
    }
    void release();
};

// The per-call device workspace and pinned staging area of one stream of work. The
// context owns one (for its entry points); a server owns one per concurrent batch.
struct Lane {
    Arena ws;
    uint8_t* stage_host = nullptr;   // pinned host staging for per-call tables
    uint8_t* stage_dev = nullptr;    // its device mirror
    size_t stage_cap = 0, stage_used = 0;
    hipStream_t stage_stream = nullptr;
    hipEvent_t copied = nullptr;     // recorded after the last copy out of the staging area
    // set while a graph's device work is being captured with this lane (which the graph
    // owns): the staging area then only grows during the call and is never reused, so the
    // graph's host-to-device copies of its tables re-read unchanged memory at every launch
    bool capture = false;
    hc_status init(size_t stage_bytes);
    void release();
};

}  // namespace hc

struct hc_context {
    int device = 0;
    int cus = 0;  // compute units of the device
    int logn = 0, n = 0, nh = 0;
    int L = 0, K = 0, dnum = 0, alpha = 0, nq = 0;
    int nb = 0;    // primes of the auxiliary basis B of ciphertext products (prime indices nq..nq+nb-1)
    int ntab = 0;  // primes with NTT tables: nq + nb
    uint64_t p = 0;
    uint32_t zeta = 0;
    std::vector<uint64_t> primes;          // q_1..q_L, p_1..p_K, then the product basis b_1..b_nb
    std::vector<uint64_t> h_qinv, h_r2;    // Montgomery constants per prime
    std::vector<uint64_t> h_tw;            // host copy of the NTT tables [nq][2][n][2]
    std::vector<uint32_t> h_twp;           // mod-p tables [2][n][2]
    std::vector<uint32_t> h_slotpos;       // NTT-mod-p position of slot r*nh + c
    std::vector<uint32_t> h_cdt;           // Gaussian CDT (20 entries)

    // device tables
    uint64_t* d_mods = nullptr;     // [nq]
    uint64_t* d_qinv = nullptr;     // [nq] -q^-1 mod 2^64
    uint64_t* d_r2 = nullptr;       // [nq] 2^128 mod q
    uint64_t* d_tw = nullptr;       // [nq][2][n][2]: (w, w') forward then inverse
    uint64_t* d_tw2 = nullptr;      // low-bit NTT pass twiddles in thread order (rings above 2^12)
    uint64_t* d_ninv = nullptr;     // [nq][4]: n^-1, Shoup; W^-1[1] n^-1, Shoup
    uint64_t* d_ninv_conv = nullptr;  // [nq][4]: as d_ninv, times the key-switching conversion factor
    uint32_t* d_modp = nullptr;     // [1] p
    uint32_t* d_twp = nullptr;      // [2][n][2] mod p
    uint32_t* d_ninvp = nullptr;    // [4]: as d_ninv, mod p
    uint32_t* d_slotpos = nullptr;  // [n]
    uint32_t* d_posslot = nullptr;  // [n] inverse of slotpos
    uint64_t* d_modup_inv = nullptr;  // [dnum][alpha][2]  (D_j/q_i)^-1 mod q_i and Shoup
    uint64_t* d_modup_c = nullptr;    // [dnum][alpha][nq] (D_j/q_i) mod r, Montgomery form mod r
    uint64_t* d_moddown_inv = nullptr;  // [K][2] (P/p_k)^-1 mod p_k and Shoup
    uint64_t* d_moddown_c = nullptr;    // [K][L] (P/p_k) mod q_i, Montgomery form
    uint64_t* d_pinv = nullptr;         // [L][2] P^-1 mod q_i and Shoup
    uint64_t* d_pmodq = nullptr;        // [L] P mod q_i
    uint64_t* d_delta = nullptr;        // [L][2] Delta mod q_i and Shoup
    uint32_t* d_cdt = nullptr;          // [20]
    uint64_t* d_keccak_rc = nullptr;    // [24]

    // modulus-switching constants for dropping the primes Lc..Lin-1 of a ciphertext at
    // level Lin, for every 1 <= Lc < Lin <= L (built at creation, so no call allocates
    // them): inv [Lin-Lc][2], cst [Lin-Lc][Lc], dinv [Lc][2]; keyed by Lin * 256 + Lc.
    // For Lin = L also ninv [L][4]: an inverse transform's final constants (as d_ninv)
    // times inv's factor on the dropped rows, so that the transform yields the
    // multiplied residues [x (D/q_j)^-1]_{q_j} directly (nullptr for Lin < L).
    struct MsTab { uint64_t* inv; uint64_t* cst; uint64_t* dinv; uint64_t* ninv; };
    std::map<int, MsTab> ms_tabs;

    // plaintext multipliers owned by the context (NTT domain, Montgomery form, [L][n])
    uint64_t* d_rowmask[2] = {nullptr, nullptr};
    std::map<uint32_t, uint64_t*> prefix_masks;  // keyed by s

    // resident diagonal tables keyed by (s, B, level): [kb][s/B][B][level][n], NTT domain,
    // Montgomery form
    // mfma: the table is in the digit layout of the int8 matrix-core multiply-accumulate
    // (mfma_mac.hip) instead of the split-word layout
    struct DiagTab { uint32_t kb = 0; uint64_t* d = nullptr; size_t bytes = 0; bool mfma = false; };
    std::map<std::tuple<uint32_t, uint32_t, int>, DiagTab> diag_tabs;
    int diag_layout = HC_DIAG_LAYOUT_AUTO;  // layout of tables built next (hc_diag_layout)

    // digit weights of the int8 matrix-core multiply-accumulate: 256^s 2^64 mod q_i,
    // [L][16] (s < 13)
    uint64_t* d_mfw = nullptr;

    uint64_t* d_scratch = nullptr;  // this device's fixed allocation-free scratch (context.cpp)

    // exact base conversion constants of ciphertext products (mult.hip), device, one block:
    // see MultTab there
    uint64_t* d_mult = nullptr;

    // kernel variants picked by hc_autotune / hc_tune_set (bit-neutral): the diagonal
    // multiply-accumulate's (terms per stage, stages in flight) and the 64-bit NTT
    // passes' occupancy or persistent grid
    int tune_mac = 0, tune_ntt = 0;

    hc::Lane lane;     // workspace and staging of the context's own entry points
    std::mutex lazy_mu;  // guards the lazily built tables (prefix masks, switch tables)
    std::vector<void*> owned;  // device allocations freed at destroy

    // kernel timing (measurement only)
    struct TimedLaunch { int kind; hipEvent_t a, b; double bytes, ops; };
    bool timing = false;
    mutable std::mutex timing_mu;
    mutable std::vector<TimedLaunch> tlaunches;
    mutable std::vector<hipEvent_t> event_pool;
};

struct hc_sk {
    std::vector<int8_t> s;        // host copy of the ternary secret
    uint64_t* d_s_mont = nullptr; // NTT domain over PQ, Montgomery form [nq][n]
};

struct hc_pk {
    uint64_t* d_b = nullptr;  // NTT domain, normal form, [L][n]
    uint64_t* d_a = nullptr;
};

struct hc_gk {
    int dnum = 0, nq = 0, n = 0;
    std::map<uint32_t, uint64_t*> keys;  // element -> [dnum][2][nq][n], NTT domain, Montgomery form
};

struct hc_db {
    uint32_t ncol = 0;
    uint64_t N = 0;
    uint32_t n_ct = 0;
    uint64_t* d_pt = nullptr;  // [ncol][n_ct][L][n] NTT domain, Montgomery form
    uint32_t* d_raw = nullptr; // [ncol][N] the values mod p (the unencrypted-database form)
};

namespace hc {

using Ctx = hc_context;

// One key-switching job: out = Rot_k(in) with `key` ([dnum][2][L+K][n], Montgomery
// form); xidx selects the raised digits (its own for plain jobs, the shared
// source's for hoisted jobs). in/out: [2][Lc][n] NTT domain, out != in.
struct KsJob {
    const uint64_t* in;
    uint64_t* out;
    const uint64_t* key;
    uint32_t k;
    uint32_t xidx;
    // nonzero: out points into the multiply-accumulate's gathered layout (see
    // kb_final), words between consecutive (prime, 64-coefficient tile) blocks
    uint64_t tstride = 0;
};

// Jobs [j0, j1) of a key-switching pass that belong to sum group g (indices into a
// member list).
struct KsGroupRange { uint32_t g, j0, j1, pad; };
// Jobs [j0, j0 + cnt) of a pass that share one key (cnt <= KS_RUN).
constexpr int KS_RUN = 8;
struct KsRun { uint32_t j0, cnt; };

// One element-wise job over a ciphertext [2][Lc][n]: out = a (*|+) b.
struct EwJob {
    uint64_t* out;
    const uint64_t* a;
    const uint64_t* b;
};

// Products of one ciphertext a ([2][L][n]) with ncol plaintexts ([L][n] each, Montgomery
// form): out + c out_step = a * (b + c b_step), c < ncol.
struct MaskJob {
    const uint64_t* a;
    uint64_t* out;
    const uint64_t* b;
    uint64_t out_step, b_step;
    uint32_t ncol, pad;
};

// Times the kernel launches made through hc_launch on stream st while it lives, when
// timing is enabled: the first such launch carries the start event and every one the stop
// event (hipExtLaunchKernel takes them from the dispatch itself, with no marker packets
// between the kernels).
struct TimeScope {
    const hc_context& c;
    int kind;
    hipStream_t st;
    double bytes, ops;
    hipEvent_t a = nullptr, b = nullptr;
    bool used = false;
    TimeScope* prev = nullptr;
    TimeScope(const hc_context& c_, int kind_, hipStream_t st_, double bytes_, double ops_);
    ~TimeScope();
    static TimeScope*& current();  // the calling thread's innermost active scope
};

template <typename... F, typename... A, size_t... I>
inline void launch_args(std::tuple<F...>& f, void** args, std::index_sequence<I...>) {
    ((args[I] = (void*)&std::get<I>(f)), ...);
}

// Launches kernel(actuals...) like hipLaunchKernelGGL; inside a TimeScope of this stream,
// with that scope's events.
template <typename... Formals, typename... Actuals>
inline void hc_launch(void (*kernel)(Formals...), dim3 grid, dim3 block, uint32_t shm, hipStream_t st,
                      Actuals... actuals) {
    static_assert(sizeof...(Formals) == sizeof...(Actuals) && sizeof...(Formals) > 0, "kernel arguments");
    std::tuple<Formals...> f{std::tuple<Actuals...>{actuals...}};
    void* args[sizeof...(Formals)];
    launch_args(f, args, std::index_sequence_for<Formals...>{});
    TimeScope* ts = TimeScope::current();
    if (ts && ts->st == st) {
        (void)hipExtLaunchKernel((const void*)kernel, grid, block, args, shm, st, ts->used ? nullptr : ts->a, ts->b, 0);
        ts->used = true;
    } else {
        (void)hipLaunchKernel((const void*)kernel, grid, block, args, shm, st);
    }
}

// ------------------------------------------------------------------ NTT (ntt.hip)
// data: `count` polynomials spaced poly_stride elements apart; data points at
// the first transformed row, whose prime index is limb_first. src (optional): the input,
// laid out as data and left unchanged; the result goes to data (no copy first).
void ntt64(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
           bool inverse, hipStream_t stream, const uint64_t* src = nullptr);
// mod-p transforms of `count` contiguous length-n rows.
void ntt32(const Ctx& c, uint32_t* data, int count, bool inverse, hipStream_t stream);
// builds d_tw2 from d_tw (context creation; synchronises the device)
hc_status ntt_build_tw2(Ctx& c);
// Ring 2^16 (two NTT passes of 8 stages): key switching's conversions run fused with the
// forward transform's high-bit pass (k_modup_fused, k_moddown_fused); its low-bit pass
// alone runs through ntt64_low_pass (inverse: the first pass; forward: the last).
bool conv_fused_ring(const Ctx& c);
void ntt64_low_pass(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                    bool inverse, hipStream_t stream);
// ModUp's forward low-bit pass (ring 2^16) over the ciphertext rows of every raised digit
// in one launch: X holds `count` = sources x dn polynomials spaced poly_stride apart
// (digit y % dn of source y / dn), rows 0..Lc-1; a digit's own rows are left as they are.
// Nothing is launched for dn < 2.
void ntt64_low_raise(const Ctx& c, uint64_t* X, size_t poly_stride, int count, int Lc, int dn, hipStream_t st);
// The inverse transform of rows limb_first.. (ciphertext primes of whole digits, or special
// primes) scaled by the base conversion's factor: [x (D_j/q_i)^-1]_{q_i} or
// [x (P/p_k)^-1]_{p_k} per coefficient, canonical (one multiplication folded into n^-1).
void ntt64_inverse_conv(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                        hipStream_t stream);
// ModUp's inputs at ring 2^16 straight from the jobs' ciphertexts: row r of tmpC[u] gets c1
// (row Lc + r) of jobs[u].in rotated by sigma_{k_u}, through the inverse transform's first
// pass, and the rotated words also go to the digit's own row of X (ModUp leaves those
// unchanged); then ntt64_inverse_high_conv finishes the transform. Together: kb_take_c1
// followed by ntt64_inverse_conv.
void ntt_take_c1_low(const Ctx& c, const KsJob* jobs, uint64_t* tmpC, uint64_t* X, int U, int Lc, hipStream_t st);
void ntt64_inverse_high_conv(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                             hipStream_t stream);
// ModDown of the M jobs of a pass at ring 2^16: the special rows of their key products
// T[m][comp][Lc..R-1] computed inside the inverse transform's first pass (the words
// kb_inner writes there); ntt64_inverse_high_conv then finishes the transform.
void ntt_inner_low(const Ctx& c, const KsJob* jobs, const uint64_t* X, uint64_t* T, int M, int Lc, bool hoisted,
                   hipStream_t st);
// ModUp of U sources at level Lc: tmpC [U][Lc][n] (from ntt64_inverse_conv) -> every row
// of X[U][dn][R][n] outside each digit, after the forward high-bit pass (its low-bit pass
// follows); the words equal kb_modup's followed by the full transform.
void k_modup_fused(const Ctx& c, uint64_t* X, const uint64_t* tmpC, int U, int Lc, hipStream_t st);
// ModDown's P -> Q conversion of M jobs at level Lc: T [M][2][R][n] special rows (from
// ntt64_inverse_conv) -> conv [M][2][Lc][n] after the forward high-bit pass.
void k_moddown_fused(const Ctx& c, uint64_t* conv, const uint64_t* T, int M, int Lc, hipStream_t st);

// ------------------------------------------------------------------ kernels (ops.hip)
// All arrays are [rows][n] per polynomial; "nl" rows starting at prime index lf.

// out = in permuted by sigma_k in the NTT domain (k = 1: copy), for nl rows.
void k_permute(const Ctx& c, uint64_t* out, const uint64_t* in, int nl, uint32_t k, int count,
               size_t stride, hipStream_t st);
// out = a + b (mod), nl rows starting at prime lf, `count` polynomials of stride.
void k_add(const Ctx& c, uint64_t* out, const uint64_t* a, const uint64_t* b, int lf, int nl,
           int count, size_t stride, hipStream_t st);
// out[c] = ct[c] * pt (Montgomery pt) for c = 0, 1 over the first Lc ciphertext primes
// (ct and out at level Lc: [2][Lc][n]; pt rows 0..Lc-1).
void k_mul_plain(const Ctx& c, uint64_t* out, const uint64_t* ct, const uint64_t* pt_mont, int Lc,
                 hipStream_t st);
// ModUp of all digits: X [dnum][nq][n] (coefficient domain) from x [L][n] (coefficient domain).
// ---- batched key switching (compact rows: Lc ciphertext primes, then K special primes)
// tmpC[m] = c1 of job m's input (permuted by sigma_k unless k = 1), [M][Lc][n], NTT
// domain; the same rows also into the digits' own rows of X [M][dn][Lc+K][n]
void kb_take_c1(const Ctx& c, uint64_t* tmpC, uint64_t* X, const KsJob* jobs, int M, int Lc, hipStream_t st);
// X [U][dn][Lc+K][n] raised digits of the coefficient-domain tmpC [U][Lc][n]
// ModUp of U sources [Lc][n] (coefficient domain) into digits X[U][dn][Lc+K][n]; a
// digit's own rows are written only if own_rows.
void kb_modup(const Ctx& c, uint64_t* X, const uint64_t* tmpC, int U, int Lc, bool own_rows, hipStream_t st);
// T [M][2][Lc+K][n] = sum_j X[xidx_m][j] (rotated by k_m if hoisted) * key_m[j], rows row0..
void kb_inner(const Ctx& c, uint64_t* T, const uint64_t* X, const KsJob* jobs, const KsRun* runs, int nruns, int M,
              int Lc, bool hoisted, hipStream_t st, int row0 = 0);
// kb_final for the jobs of a pass in key runs, the ciphertext rows of T computed in place
// from X and the keys (kb_inner need only have computed the special rows). maxrun: the
// longest run's job count (1 selects the kernel built for runs of one job).
void kb_final_inner(const Ctx& c, const KsJob* jobs, const KsRun* runs, int nruns, const uint64_t* X,
                    const uint64_t* conv, int M, int Lc, bool hoisted, hipStream_t st, int maxrun);
// conv [M][2][Lc][n] = Conv_{P->Q} of the special rows of T (coefficient domain)
void kb_conv(const Ctx& c, uint64_t* conv, const uint64_t* T, int M, int Lc, hipStream_t st);
// out_m = (sigma_k(c0_m) + (T0 - conv0) P^-1, (T1 - conv1) P^-1), NTT domain
void kb_final(const Ctx& c, const KsJob* jobs, const uint64_t* T, const uint64_t* conv, int M, int Lc,
              hipStream_t st);
// y[g] = sum of `cnt` consecutive ciphertexts of src group g (level Lc, contiguous)
void k_sum_cts(const Ctx& c, uint64_t* y, const uint64_t* src, int groups, int cnt, int Lc, hipStream_t st);
// element-wise jobs at level Lc: out = a * b (b a Montgomery plaintext [Lc rows]) or out = a + b
void k_ew_jobs(const Ctx& c, const EwJob* jobs, int M, int Lc, bool mul, hipStream_t st);
// MaskJob products at rows 0..rows-1 of ciphertexts with L rows: a thread reads its
// coefficient of both components once and each plaintext once
void k_mask_jobs(const Ctx& c, const MaskJob* jobs, int M, int rows, int L, hipStream_t st);
// The MaskJob products at the rows Lc..L-1 (ring 2^16), computed while loading the inverse
// transform's first pass: every column's output rows hold the pass's result there (the
// words k_mask_jobs writes, after ntt64_low_pass(inverse)). cmax: the most columns of a
// job; nprod: the jobs' columns in all.
void ntt_mask_low(const Ctx& c, const MaskJob* jobs, int M, int cmax, int nprod, int Lc, hipStream_t st);
// The inverse transform's second pass (ring 2^16) with the final constants `ninv`
// ([prime][4], the layout of d_ninv) in place of n^-1.
void ntt64_inverse_high_tab(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                            const uint64_t* ninv, hipStream_t stream);
// modulus switching of `count` contiguous ciphertexts from Lin to Lc primes:
// conv [count][2][Lc][n] from the dropped rows of ct [count][2][Lin][n] (coefficient domain;
// with inv == nullptr already multiplied by their factors (D/q_j)^-1);
// out [count][2][Lc][n] = (ct - conv) D^-1 (element-wise: conv in ct's domain)
void k_ms_conv(const Ctx& c, uint64_t* conv, const uint64_t* ct, const uint64_t* inv, const uint64_t* cst,
               int Lin, int Lc, int count, hipStream_t st);
void k_ms_final(const Ctx& c, uint64_t* out, const uint64_t* ct, const uint64_t* conv, const uint64_t* dinv,
                int Lin, int Lc, int count, hipStream_t st);
// slots (device u32 [count][2][nh]) -> NTT-mod-p positions [count][n]
void k_slots_to_eval(const Ctx& c, uint32_t* out, const uint32_t* slots, int count, hipStream_t st);
// centred lift of mod-p coefficients [count][n] into [count][L][n]; Montgomery form if mont
void k_lift(const Ctx& c, uint64_t* out, const uint32_t* in, int count, bool mont, int Lc,
            hipStream_t st);
// compression diagonals in NTT-mod-p positions: out [count][n], params [count][3] (beta, gi, b)
// diagonals of the unencrypted-database form in NTT-mod-p positions: out [count][n], params
// [count][7] (beta_0, beta_1, gi, b, col_0, col_1, rec_start): row r for record block beta_r
// of matrix col_r (0: C; c >= 1: C diag(DB_c) with raw [ncol][Ndb]; 0xffffffff: zero row)
void k_diag_gen_db(const Ctx& c, uint32_t* out, const uint32_t* params, int count, uint32_t s, uint32_t B,
                   const uint32_t* raw, uint64_t Ndb, hipStream_t st);
void k_diag_gen(const Ctx& c, uint32_t* out, const uint32_t* params, int count, uint32_t s,
                uint32_t B, hipStream_t st);
// samplers: uniform residues for rows lf..lf+nl-1 (stream limb index = row prime index)
void k_sample_uniform(const Ctx& c, uint64_t* out, const uint8_t* seed_dev, uint64_t tag,
                      uint64_t obj, int lf, int nl, hipStream_t st);
// small samplers (kind 1 ternary, 2 Gaussian): residues over rows lf..lf+nl-1 and,
// if raw != nullptr, the signed values.
void k_sample_small(const Ctx& c, uint64_t* out, int64_t* raw, const uint8_t* seed_dev,
                    uint64_t tag, uint64_t obj, int kind, int lf, int nl, hipStream_t st);
// pointwise multiply-add helpers for key generation (NTT domain):
// out = e - a * s_mont + g * rot_s_mont (g per row, may be null), rows lf..lf+nl-1
void k_keyrow(const Ctx& c, uint64_t* out, const uint64_t* e, const uint64_t* a,
              const uint64_t* s_mont, const uint64_t* rot_s_mont, const uint64_t* grow, int lf,
              int nl, hipStream_t st);
// x -> x * 2^64 mod q (to Montgomery form), rows lf..lf+nl-1, count polys of stride
void k_to_mont(const Ctx& c, uint64_t* x, int lf, int nl, int count, size_t stride, hipStream_t st);
// x -> x * 2^-64 mod q (from Montgomery form)
void k_from_mont(const Ctx& c, uint64_t* x, int lf, int nl, int count, size_t stride, hipStream_t st);
// out = a * bm (Montgomery bm), rows lf..lf+nl-1
void k_mul_mont(const Ctx& c, uint64_t* out, const uint64_t* a, const uint64_t* bm, int lf, int nl,
                hipStream_t st);
// encryption finish (coefficient domain): c0 += e0 + Delta m ; c1 += e1
void k_enc_finish(const Ctx& c, uint64_t* ct, const uint64_t* e0, const uint64_t* e1,
                  const uint32_t* m, hipStream_t st);
// Device memory reached through a pointer held in a job table, as a global (not a
// generic) pointer: loads through a generic pointer might read LDS, so they cannot move
// past a kernel's LDS stores, and every load of a loop that also fills LDS then waits
// for the one before it.
typedef __attribute__((address_space(1))) const uint64_t gl_cu64;
typedef __attribute__((address_space(1))) uint64_t gl_mu64;
__device__ __forceinline__ gl_cu64* gl(const uint64_t* p) { return (gl_cu64*)p; }
__device__ __forceinline__ gl_mu64* gl(uint64_t* p) { return (gl_mu64*)p; }

// NTT-domain index that sigma_k pulls from: entry i holds a(psi^(2 brv(i)+1)),
// so sigma_k(a) at i equals a at the entry whose exponent is (2 brv(i)+1) k.
__device__ __forceinline__ uint32_t galois_src(uint32_t i, uint32_t k, int logn) {
    uint32_t e = (__brev(i) >> (32 - logn)) * 2u + 1u;
    uint32_t e2 = (e * k) & ((2u << logn) - 1u);
    return __brev((e2 - 1u) >> 1) >> (32 - logn);
}
// diagonal multiply-accumulate:
//   A[pp][g] (+)= sum_{beta < kb, b < B} D[beta][g][b] * R[pp][beta][b]
// R, A given as device arrays of ciphertext pointers; D contiguous
// [kb][G][B][L][n] (Montgomery). accumulate: add to the existing A.
// Giant indices per wave of the diagonal multiply-accumulate (and per chunk of the
// resident tables' layout), and terms per LDS stage.
constexpr int DIAG_GC = 8;
constexpr int DIAG_T = 4;
// Word strides of a diagonal table (split words, see k_diag_split): D(beta, g, b) of
// limb r at coefficient 64 tile + lane, term j = beta B + b, giant g = DIAG_GC c + i, is
// D[r sr + tile st + c sgc + j sj + i sg + lane].
struct DiagLayout { size_t sr, st, sgc, sj, sg; };
// one [Lc][n] polynomial per diagonal, index (beta B + b) gc + g (gc giants per chunk)
DiagLayout diag_layout_natural(const Ctx& c, int Lc, uint32_t gc);
// resident tables: [Lc][n/64][ceil(dG/DIAG_GC)][Jt][DIAG_GC][64], Jt = kbt B terms
DiagLayout diag_layout_tiled(const Ctx& c, uint32_t Jt, uint32_t dG);
// words of a resident table of Jt terms and dG giants
size_t diag_table_words(const Ctx& c, int Lc, uint32_t Jt, uint32_t dG);
// natural order (beta dG + g) B + b -> tiled and split, for `count` diagonals from index i0
void k_diag_tile(const Ctx& c, uint64_t* out, const uint64_t* in, size_t i0, int count, uint32_t kbt,
                 uint32_t B, uint32_t dG, int Lc, hipStream_t st);
// words v -> (v >> h) 2^32 + (v mod 2^h), h = ceil(bits of the largest of the first Lc primes / 2)
void k_diag_split(const Ctx& c, uint64_t* d, size_t words, int Lc, hipStream_t st);
// TA[g] += sum of the jobs' key products (raised digits X times their keys, over PQ),
// C0A[g] += sum of their rotated c0, per group range of a pass of M jobs with nkeys
// distinct keys
void kb_inner_sum(const Ctx& c, uint64_t* TA, uint64_t* C0A, const uint64_t* X, const KsJob* jobs,
                  const KsGroupRange* ranges, const uint32_t* members, int nranges, int M, int nkeys, int Lc,
                  hipStream_t st);
// p[0..words) = 0 (a kernel, so it can sit in a captured graph)
void k_zero(const Ctx& c, uint64_t* p, size_t words, hipStream_t st);
// terms of the gathered rotated ciphertexts per pair: J rounded up to whole rounds of
// the multiply-accumulate (DIAG_NS stages of DIAG_T terms: the stages in flight at once)
constexpr int DIAG_NS = 4;
// split position h of the first Lc primes (ceil(bits of the largest / 2))
int diag_split_h(const Ctx& c, int Lc);
inline int diag_terms_padded(int J) {
    return (J + DIAG_NS * DIAG_T - 1) / (DIAG_NS * DIAG_T) * (DIAG_NS * DIAG_T);
}
// Rt[r][tile][pp][j][64][2] (split) from the pointer table R[pp][j] (j < J; nullptr and
// J <= j < diag_terms_padded(J): zeros; kRtInPlace: already written there). Only the
// entries pp * diag_terms_padded(J) + j listed in work[0..nwork) are written; the
// list holds every entry that is not kRtInPlace (diag_gather_list builds it).
static const uint64_t* const kRtInPlace = reinterpret_cast<const uint64_t*>(uintptr_t(1));
std::vector<uint32_t> diag_gather_list(const std::vector<const uint64_t*>& R, int npairs, int J);
void k_diag_gather(const Ctx& c, uint64_t* Rt, const uint64_t* const* R, const uint32_t* work, int nwork, int npairs,
                   int J, int Lc, hipStream_t st);
// A[pp][g] (=|+=) sum_{j<J} D(j, g) R[pp][j], g < ga, for npairs pairs: A pointers
// [npairs][ga], R gathered by k_diag_gather, D split and in Montgomery form.
// HC_EINVAL if one term's diagonal words for DIAG_GC giants span 2^31 bytes or more
hc_status k_diag_mac(const Ctx& c, uint64_t* const* A, const uint64_t* Rt, const uint64_t* D,
                     const DiagLayout& lay, int npairs, int J, int ga, bool accumulate, int Lc, hipStream_t st);
// The same product (A written, not accumulated) on the matrix cores (int8 MFMA over
// balanced base-256 digits) from a resident table in the digit layout, Jt terms
// (J <= Jt <= 128 used: J) by ga giants:
// diag_mfma_fits says whether a table of Jt terms and G giants at level Lc takes that
// layout (every prime below 2^55, Jt <= 128, padding at most doubling the bytes),
// k_diag_digits writes its giant tile t / term block jb from ng x nj natural-layout
// diagonals [(gl nj + jl)][Lc][n] (plain residues, NTT domain). HC_EINVAL outside.
bool diag_mfma_fits(const Ctx& c, int Lc, uint32_t Jt, uint32_t G);
size_t diag_mfma_table_bytes(const Ctx& c, int Lc, uint32_t Jt, uint32_t G);
void k_diag_digits(const Ctx& c, void* table, const uint64_t* in, uint32_t Jt, uint32_t G, uint32_t t, uint32_t jb,
                   int Lc, hipStream_t st);
hc_status k_diag_mac_mfma(const Ctx& c, uint64_t* const* A, const uint64_t* Rt, const void* D, uint32_t Jt, int npairs,
                          int J, int ga, int Lc, hipStream_t st);

}  // namespace hc
