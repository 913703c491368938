// Device kernels of libhc other than the NTT.
//
// Layout: a ring element over a set of primes is rows of n uint64_t residues
// ([row][coefficient]); a ciphertext is [2][L][n]. Every kernel below is
// element-wise over (row, coefficient) -- one thread per coefficient, rows
// along grid.y -- so all accesses are unit-stride across a wavefront, except
// the automorphism gathers (a fixed permutation within a row).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "hc_internal.h"

namespace hc {

constexpr int EW_THREADS = 256;

static inline dim3 ew_grid(int n, int rows, int count = 1) {
    return dim3((n + EW_THREADS - 1) / EW_THREADS, rows, count);
}

// A residue v < 2^(2h) stored split for the multiply-accumulate: (v >> h) 2^32 + (v mod 2^h).
__device__ __forceinline__ uint64_t split_word(uint64_t v, int h) {
    return ((v >> h) << 32) | (v & ((1ull << h) - 1));
}


// ------------------------------------------------------------------ basic element-wise

__global__ void permute_kernel(uint64_t* __restrict__ out, const uint64_t* __restrict__ in, int n,
                               int logn, uint32_t k, size_t stride) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    size_t off = (size_t)blockIdx.z * stride + (size_t)blockIdx.y * n;
    uint32_t src = (k == 1) ? x : galois_src(x, k, logn);
    out[off + x] = in[off + src];
}

void k_permute(const Ctx& c, uint64_t* out, const uint64_t* in, int nl, uint32_t k, int count,
               size_t stride, hipStream_t st) {
    hipLaunchKernelGGL(permute_kernel, ew_grid(c.n, nl, count), dim3(EW_THREADS), 0, st, out, in,
                       c.n, c.logn, k, stride);
}

__global__ void add_kernel(uint64_t* out, const uint64_t* a, const uint64_t* b, const uint64_t* mods,
                           int n, int lf, size_t stride) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    size_t off = (size_t)blockIdx.z * stride + (size_t)blockIdx.y * n + x;
    out[off] = add_mod(a[off], b[off], mods[lf + blockIdx.y]);
}

void k_add(const Ctx& c, uint64_t* out, const uint64_t* a, const uint64_t* b, int lf, int nl,
           int count, size_t stride, hipStream_t st) {
    hipLaunchKernelGGL(add_kernel, ew_grid(c.n, nl, count), dim3(EW_THREADS), 0, st, out, a, b,
                       c.d_mods, c.n, lf, stride);
}

__global__ void mul_plain_kernel(uint64_t* out, const uint64_t* ct, const uint64_t* pt,
                                 const uint64_t* mods, const uint64_t* qinv, int n, int L) {
    // L: ciphertext primes of this ciphertext (its component stride is L n)
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int r = blockIdx.y;
    uint64_t q = mods[r], qi = qinv[r];
    uint64_t m = pt[(size_t)r * n + x];
    size_t o0 = (size_t)r * n + x, o1 = o0 + (size_t)L * n;
    uint64_t v0 = ct[o0], v1 = ct[o1];
    out[o0] = mont_mul(v0, m, q, qi);
    out[o1] = mont_mul(v1, m, q, qi);
}

void k_mul_plain(const Ctx& c, uint64_t* out, const uint64_t* ct, const uint64_t* pt_mont, int Lc,
                 hipStream_t st) {
    hipLaunchKernelGGL(mul_plain_kernel, ew_grid(c.n, Lc), dim3(EW_THREADS), 0, st, out, ct,
                       pt_mont, c.d_mods, c.d_qinv, c.n, Lc);
}

__global__ void mul_mont_kernel(uint64_t* out, const uint64_t* a, const uint64_t* bm,
                                const uint64_t* mods, const uint64_t* qinv, int n, int lf) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int r = blockIdx.y;
    size_t o = (size_t)r * n + x;
    out[o] = mont_mul(a[o], bm[o], mods[lf + r], qinv[lf + r]);
}

void k_mul_mont(const Ctx& c, uint64_t* out, const uint64_t* a, const uint64_t* bm, int lf, int nl,
                hipStream_t st) {
    hipLaunchKernelGGL(mul_mont_kernel, ew_grid(c.n, nl), dim3(EW_THREADS), 0, st, out, a, bm,
                       c.d_mods, c.d_qinv, c.n, lf);
}

__global__ void to_mont_kernel(uint64_t* x, const uint64_t* mods, const uint64_t* qinv,
                               const uint64_t* r2, int n, int lf, size_t stride, int inverse) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = lf + blockIdx.y;
    size_t o = (size_t)blockIdx.z * stride + (size_t)blockIdx.y * n + i;
    uint64_t q = mods[r];
    // x * 2^128 * 2^-64 = x 2^64 ; or x * 1 * 2^-64
    x[o] = inverse ? redc(u128p{x[o], 0}, q, qinv[r]) : mont_mul(x[o], r2[r], q, qinv[r]);
}

void k_to_mont(const Ctx& c, uint64_t* x, int lf, int nl, int count, size_t stride, hipStream_t st) {
    hipLaunchKernelGGL(to_mont_kernel, ew_grid(c.n, nl, count), dim3(EW_THREADS), 0, st, x,
                       c.d_mods, c.d_qinv, c.d_r2, c.n, lf, stride, 0);
}

void k_from_mont(const Ctx& c, uint64_t* x, int lf, int nl, int count, size_t stride, hipStream_t st) {
    hipLaunchKernelGGL(to_mont_kernel, ew_grid(c.n, nl, count), dim3(EW_THREADS), 0, st, x,
                       c.d_mods, c.d_qinv, c.d_r2, c.n, lf, stride, 1);
}

// ------------------------------------------------------------------ key switching (batched)
//
// Intermediates of key switching at level Lc use a compact row layout: rows
// 0..Lc-1 are the first Lc ciphertext primes, rows Lc..Lc+K-1 the special primes
// (prime index L + row - Lc). A pass handles M jobs (rotations); job m reads
// the raised digits X[xidx_m] and its own key, and writes out_m.

__device__ __forceinline__ int row_prime(int row, int Lc, int L) { return row < Lc ? row : L + row - Lc; }

// tmpC[m] = c1 of job m's input, permuted by sigma_{k_m} (k = 1: plain copy)
__global__ void kb_take_c1_kernel(uint64_t* __restrict__ tmpC, uint64_t* __restrict__ X,
                                  const KsJob* __restrict__ jobs, int n, int logn, int Lc, int alpha, int R,
                                  int dn) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const KsJob jb = jobs[blockIdx.z];
    const uint32_t src = (jb.k == 1) ? x : galois_src(x, jb.k, logn);
    const int r = blockIdx.y, u = blockIdx.z;
    const uint64_t v = jb.in[((size_t)Lc + r) * n + src];
    tmpC[((size_t)u * Lc + r) * n + x] = v;
    X[(((size_t)u * dn + r / alpha) * R + r) * n + x] = v;
}

// tmpC[u] = c1 of job u (rotated by its element), NTT domain, and the same rows into
// X[u][j] for the digit j they belong to: ModUp leaves a digit's own residues unchanged,
// so their transform is the input's.
void kb_take_c1(const Ctx& c, uint64_t* tmpC, uint64_t* X, const KsJob* jobs, int M, int Lc, hipStream_t st) {
    hipLaunchKernelGGL(kb_take_c1_kernel, ew_grid(c.n, Lc, M), dim3(EW_THREADS), 0, st, tmpC, X, jobs, c.n,
                       c.logn, Lc, c.alpha, Lc + c.K, Lc / c.alpha);
}

// X[u][j] (compact rows) from the coefficient-domain tmpC[u]: the digit's own rows
// are copied; row r outside the digit gets sum_a [x_a (D_j/q_a)^-1]_{q_a} (D_j/q_a) mod r.
__global__ void kb_modup_kernel(uint64_t* __restrict__ X, const uint64_t* __restrict__ tmpC,
                                const uint64_t* __restrict__ mods, const uint64_t* __restrict__ qinv,
                                const uint64_t* __restrict__ inv, const uint64_t* __restrict__ cst,
                                int n, int nq, int alpha, int L, int Lc, int K, int dn, int own) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int j = blockIdx.y, u = blockIdx.z, R = Lc + K;
    const uint64_t* src = tmpC + (size_t)u * Lc * n;
    uint64_t* out = X + ((size_t)u * dn + j) * R * n;
    // alpha <= 4 (the context's limit): fixed-trip loops, so the loads issue together
    uint64_t v[4], y[4];
    #pragma unroll
    for (int a = 0; a < 4; a++)
        if (a < alpha) v[a] = src[(size_t)(j * alpha + a) * n + x];
    #pragma unroll
    for (int a = 0; a < 4; a++)
        if (a < alpha) {
            const int r = j * alpha + a;
            if (own) out[(size_t)r * n + x] = v[a];
            const uint64_t* iv = inv + ((size_t)j * alpha + a) * 2;
            y[a] = shoup(v[a], iv[0], iv[1], mods[r]);
        }
    const uint64_t* cj = cst + (size_t)j * alpha * nq;
    for (int row = 0; row < R; row++) {
        if (row >= j * alpha && row < (j + 1) * alpha) continue;
        const int pr = row_prime(row, Lc, L);
        u128p acc{0, 0};
        #pragma unroll
        for (int a = 0; a < 4; a++)
            if (a < alpha) add128(acc, mul128(y[a], cj[(size_t)a * nq + pr]));
        out[(size_t)row * n + x] = redc(acc, mods[pr], qinv[pr]);
    }
}

void kb_modup(const Ctx& c, uint64_t* X, const uint64_t* tmpC, int U, int Lc, bool own_rows, hipStream_t st) {
    const int dn = Lc / c.alpha, R = Lc + c.K;
    const double n = c.n;
    TimeScope ts(c, HC_KT_MODUP, st,
                 8.0 * n * U * ((double)Lc + (double)dn * (R - (own_rows ? 0 : c.alpha))),
                 n * U * dn * (double)(R - c.alpha) * c.alpha);
    hc_launch(kb_modup_kernel, ew_grid(c.n, dn, U), dim3(EW_THREADS), 0, st, X, tmpC, c.d_mods,
                       c.d_qinv, c.d_modup_inv, c.d_modup_c, c.n, c.nq, c.alpha, c.L, Lc, c.K, dn,
                       own_rows ? 1 : 0);
}

// T[m][comp][row][x] = sum_j X[xidx][j][row][src(x)] * key_m[j][comp][prime(row)][x]; the key is
// in Montgomery form, so one reduction of the 128-bit sum gives the plain sum (dnum q^2 < q 2^64).
// Key inner product of a pass, one run of up to KS_RUN jobs that share one key per
// block (jobs sorted by key): each key word is read once per run, and each job's
// raised digit (rotated on the fly for hoisted jobs) is multiplied into its own
// 128-bit sums, reduced once.
__global__ __launch_bounds__(EW_THREADS) void kb_inner_kernel(uint64_t* __restrict__ T, const uint64_t* __restrict__ X,
                                const KsJob* __restrict__ jobs, const KsRun* __restrict__ runs,
                                const uint64_t* __restrict__ mods, const uint64_t* __restrict__ qinv, int n,
                                int logn, int nq, int L, int Lc, int K, int dn, int hoisted, int row0) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int row = row0 + (int)blockIdx.y, R = Lc + K;
    const KsRun run = runs[blockIdx.z];
    const int pr = row_prime(row, Lc, L);
    const size_t keyrow = (size_t)nq * n;
    const int cnt = (int)run.cnt;
    gl_cu64* kp = gl(jobs[run.j0].key) + (size_t)pr * n + x;
    u128p a0[KS_RUN], a1[KS_RUN];
    #pragma unroll
    for (int i = 0; i < KS_RUN; i++) { a0[i] = u128p{0, 0}; a1[i] = u128p{0, 0}; }
    for (int j = 0; j < dn; j++) {
        const uint64_t k0 = kp[(size_t)j * 2 * keyrow], k1 = kp[(size_t)j * 2 * keyrow + keyrow];
        // the run's words loaded together and unconditionally (a slot past the run rereads
        // its first job and is not stored)
        uint64_t xv[KS_RUN];
        #pragma unroll
        for (int i = 0; i < KS_RUN; i++) {
            const KsJob jb = jobs[run.j0 + (i < cnt ? i : 0)];
            // plain jobs raised their already-rotated c1; hoisted jobs rotate the shared raised digits
            const uint32_t src = (!hoisted || jb.k == 1) ? x : galois_src(x, jb.k, logn);
            xv[i] = X[((size_t)jb.xidx * dn + j) * R * n + (size_t)row * n + src];
        }
        #pragma unroll
        for (int i = 0; i < KS_RUN; i++) {
            add128(a0[i], mul128(xv[i], k0));
            add128(a1[i], mul128(xv[i], k1));
        }
    }
    const uint64_t q = mods[pr], qi = qinv[pr];
    #pragma unroll
    for (int i = 0; i < KS_RUN; i++) {
        if (i < (int)run.cnt) {
            uint64_t* t = T + (size_t)(run.j0 + i) * 2 * R * n + (size_t)row * n + x;
            t[0] = redc(a0[i], q, qi);
            t[(size_t)R * n] = redc(a1[i], q, qi);
        }
    }
}
void kb_inner(const Ctx& c, uint64_t* T, const uint64_t* X, const KsJob* jobs, const KsRun* runs, int nruns, int M,
              int Lc, bool hoisted, hipStream_t st, int row0) {
    const int dn = Lc / c.alpha, R = Lc + c.K;
    // per run and row: the key (2 dn words) once; per job: its raised digits and T
    const double rows = (double)(R - row0) * c.n;
    TimeScope ts(c, HC_KT_KS_INNER, st, 8.0 * rows * (2.0 * dn * nruns + (dn + 2.0) * M), 2.0 * dn * rows * M);
    hc_launch(kb_inner_kernel, ew_grid(c.n, R - row0, nruns), dim3(EW_THREADS), 0, st, T, X, jobs, runs,
                       c.d_mods, c.d_qinv, c.n, c.logn, c.nq, c.L, Lc, c.K, dn, hoisted ? 1 : 0, row0);
}

// kb_final with the ciphertext rows of T computed in place, for the jobs of a pass in key
// runs (as kb_inner): T0, T1 = sum_j X[xidx][j] (rotated if hoisted) * key[j] (one REDC of
// the 128-bit sums, the words kb_inner writes), then out as kb_final. kb_inner then only
// computes the special rows, so the ciphertext rows of T never go through device memory.
// RUN: the longest run of the launch (KS_RUN, or 1 when no two jobs share a key).
template <int RUN>
__global__ __launch_bounds__(EW_THREADS) void kb_final_inner_kernel(const KsJob* __restrict__ jobs, const KsRun* __restrict__ runs,
                                      const uint64_t* __restrict__ X, const uint64_t* __restrict__ conv,
                                      const uint64_t* __restrict__ mods, const uint64_t* __restrict__ qinv,
                                      const uint64_t* __restrict__ pinv, int n, int logn, int nq, int Lc, int K,
                                      int dn, int hoisted, int sh) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int i = blockIdx.y, R = Lc + K;
    const KsRun run = runs[blockIdx.z];
    const int cnt = (int)run.cnt;
    const size_t keyrow = (size_t)nq * n;
    gl_cu64* kp = gl(jobs[run.j0].key) + (size_t)i * n + x;
    // The run's loads are issued together and unconditionally (a job slot past the run
    // reads the run's first job again and is not used): one conditional load per job
    // would wait for each before the next.
    u128p a0[RUN], a1[RUN];
    #pragma unroll
    for (int u = 0; u < RUN; u++) { a0[u] = u128p{0, 0}; a1[u] = u128p{0, 0}; }
    for (int j = 0; j < dn; j++) {
        const uint64_t k0 = kp[(size_t)j * 2 * keyrow], k1 = kp[(size_t)j * 2 * keyrow + keyrow];
        uint64_t xv[RUN];
        #pragma unroll
        for (int u = 0; u < RUN; u++) {
            const KsJob jb = jobs[run.j0 + (u < cnt ? u : 0)];
            const uint32_t src = (!hoisted || jb.k == 1) ? x : galois_src(x, jb.k, logn);
            xv[u] = X[((size_t)jb.xidx * dn + j) * R * n + (size_t)i * n + src];
        }
        #pragma unroll
        for (int u = 0; u < RUN; u++) {
            add128(a0[u], mul128(xv[u], k0));
            add128(a1[u], mul128(xv[u], k1));
        }
    }
    const uint64_t q = mods[i], qi = qinv[i], pi = pinv[2 * i], pis = pinv[2 * i + 1];
    // the outputs in two halves of the run (all of a half's loads first)
    constexpr int HALF = RUN > 1 ? RUN / 2 : 1;
    #pragma unroll
    for (int h = 0; h < RUN; h += HALF) {
        uint64_t cv0[HALF], cv1[HALF], c0v[HALF];
        #pragma unroll
        for (int v = 0; v < HALF; v++) {
            const int m = (int)run.j0 + (h + v < cnt ? h + v : 0);
            const KsJob jb = jobs[m];
            const uint64_t* Cm = conv + (size_t)m * 2 * Lc * n + (size_t)i * n + x;
            cv0[v] = Cm[0];
            cv1[v] = Cm[(size_t)Lc * n];
            c0v[v] = gl(jb.in)[(size_t)i * n + ((jb.k == 1) ? x : galois_src(x, jb.k, logn))];
        }
        #pragma unroll
        for (int v = 0; v < HALF; v++) {
            const int u = h + v;
            if (u >= cnt) continue;
            const KsJob jb = jobs[run.j0 + u];
            const uint64_t d0 = shoup(sub_mod(redc(a0[u], q, qi), cv0[v], q), pi, pis, q);
            const uint64_t d1 = shoup(sub_mod(redc(a1[u], q, qi), cv1[v], q), pi, pis, q);
            gl_mu64* out = gl(jb.out);
            if (jb.tstride) {
                const size_t o = ((size_t)i * (n >> 6) + (x >> 6)) * jb.tstride + 2 * (x & 63);
                typedef unsigned long long w2 __attribute__((ext_vector_type(2)));
                *reinterpret_cast<__attribute__((address_space(1))) w2*>(out + o) =
                    w2{split_word(add_mod(d0, c0v[v], q), sh), split_word(d1, sh)};
            } else {
                out[(size_t)i * n + x] = add_mod(d0, c0v[v], q);
                out[((size_t)Lc + i) * n + x] = d1;
            }
        }
    }
}

void kb_final_inner(const Ctx& c, const KsJob* jobs, const KsRun* runs, int nruns, const uint64_t* X,
                    const uint64_t* conv, int M, int Lc, bool hoisted, hipStream_t st, int maxrun) {
    const int dn = Lc / c.alpha;
    // per run and row the key (2 dn words) once; per job its digits (dn), the two
    // conversions, the rotated c0 and the two outputs
    const double rows = (double)Lc * c.n;
    TimeScope ts(c, HC_KT_KS_INNER, st, 8.0 * rows * (2.0 * dn * nruns + (dn + 5.0) * M), 2.0 * dn * rows * M);
    if (maxrun == 1)
        hc_launch(kb_final_inner_kernel<1>, ew_grid(c.n, Lc, nruns), dim3(EW_THREADS), 0, st, jobs, runs, X, conv,
                  c.d_mods, c.d_qinv, c.d_pinv, c.n, c.logn, c.nq, Lc, c.K, dn, hoisted ? 1 : 0,
                  diag_split_h(c, Lc));
    else
        hc_launch(kb_final_inner_kernel<KS_RUN>, ew_grid(c.n, Lc, nruns), dim3(EW_THREADS), 0, st, jobs, runs, X,
                  conv, c.d_mods, c.d_qinv, c.d_pinv, c.n, c.logn, c.nq, Lc, c.K, dn, hoisted ? 1 : 0,
                  diag_split_h(c, Lc));
}

// conv[m][comp][i][x] = sum_k [T_{p_k}(x) (P/p_k)^-1]_{p_k} (P/p_k) mod q_i (coefficient domain).
// A thread converts one coefficient to CONV_ROWS consecutive output primes, so each
// [T_{p_k}(x) (P/p_k)^-1] is read and computed once for all of them.
constexpr int CONV_ROWS = 8;
__global__ void kb_conv_kernel(uint64_t* __restrict__ conv, const uint64_t* __restrict__ T,
                               const uint64_t* __restrict__ mods, const uint64_t* __restrict__ qinv,
                               const uint64_t* __restrict__ inv, const uint64_t* __restrict__ cst,
                               int n, int L, int Lc, int K) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int i0 = blockIdx.y * CONV_ROWS, mc = blockIdx.z, R = Lc + K;  // mc = m * 2 + comp
    const uint64_t* Tc = T + (size_t)mc * R * n;
    // K <= 4 (the context's limit): fixed-trip loops, so the loads issue together
    uint64_t v[4], y[4];
    #pragma unroll
    for (int k = 0; k < 4; k++)
        if (k < K) v[k] = Tc[(size_t)(Lc + k) * n + x];
    #pragma unroll
    for (int k = 0; k < 4; k++)
        if (k < K) y[k] = shoup(v[k], inv[2 * k], inv[2 * k + 1], mods[L + k]);
    const int i1 = (i0 + CONV_ROWS) < Lc ? (i0 + CONV_ROWS) : Lc;
    for (int i = i0; i < i1; i++) {
        u128p acc{0, 0};
        #pragma unroll
        for (int k = 0; k < 4; k++)
            if (k < K) add128(acc, mul128(y[k], cst[(size_t)k * L + i]));
        conv[((size_t)mc * Lc + i) * n + x] = redc(acc, mods[i], qinv[i]);
    }
}

void kb_conv(const Ctx& c, uint64_t* conv, const uint64_t* T, int M, int Lc, hipStream_t st) {
    hipLaunchKernelGGL(kb_conv_kernel, ew_grid(c.n, (Lc + CONV_ROWS - 1) / CONV_ROWS, 2 * M), dim3(EW_THREADS), 0,
                       st, conv, T, c.d_mods, c.d_qinv, c.d_moddown_inv, c.d_moddown_c, c.n, c.L, Lc, c.K);
}

// out_m = (sigma_k(c0_m) + (T0 - conv0) P^-1, (T1 - conv1) P^-1)   (NTT domain, level Lc).
// A job with a tile stride writes into the multiply-accumulate's gathered layout
// instead: word (comp, i, x) at out[(i (n/64) + x/64) tstride + 2 (x mod 64) + comp], split.
__global__ void kb_final_kernel(const KsJob* __restrict__ jobs, const uint64_t* __restrict__ T,
                                const uint64_t* __restrict__ conv, const uint64_t* __restrict__ mods,
                                const uint64_t* __restrict__ pinv, int n, int logn, int Lc, int K, int h) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int i = blockIdx.y, m = blockIdx.z, R = Lc + K;
    const KsJob jb = jobs[m];
    const uint64_t q = mods[i], pi = pinv[2 * i], pis = pinv[2 * i + 1];
    const uint64_t* Tm = T + (size_t)m * 2 * R * n + (size_t)i * n + x;
    const uint64_t* Cm = conv + (size_t)m * 2 * Lc * n + (size_t)i * n + x;
    uint64_t d0 = shoup(sub_mod(Tm[0], Cm[0], q), pi, pis, q);
    uint64_t d1 = shoup(sub_mod(Tm[(size_t)R * n], Cm[(size_t)Lc * n], q), pi, pis, q);
    const uint32_t src = (jb.k == 1) ? x : galois_src(x, jb.k, logn);
    const uint64_t c0 = jb.in[(size_t)i * n + src];
    if (jb.tstride) {
        const size_t o = ((size_t)i * (n >> 6) + (x >> 6)) * jb.tstride + 2 * (x & 63);
        *reinterpret_cast<ulonglong2*>(jb.out + o) = ulonglong2{split_word(add_mod(d0, c0, q), h), split_word(d1, h)};
    } else {
        jb.out[(size_t)i * n + x] = add_mod(d0, c0, q);
        jb.out[((size_t)Lc + i) * n + x] = d1;
    }
}

void kb_final(const Ctx& c, const KsJob* jobs, const uint64_t* T, const uint64_t* conv, int M, int Lc,
              hipStream_t st) {
    hipLaunchKernelGGL(kb_final_kernel, ew_grid(c.n, Lc, M), dim3(EW_THREADS), 0, st, jobs, T, conv,
                       c.d_mods, c.d_pinv, c.n, c.logn, Lc, c.K, diag_split_h(c, Lc));
}

// Key products of rotations summed per group before the group's single ModDown:
// TA[g][comp][row] += sum over the group's jobs m of X_m[row] * key_m[comp][row] (all
// digits; X_m is job m's raised, already rotated c1) and C0A[g][i] += sum of the jobs'
// rotated c0 (rows R..R+Lc-1 of the grid). Per-job products are never written out.
// Work item (range, tile, row) with the range fastest. Blocks go to the XCDs round robin,
// so block b takes item (b mod 8) per_xcd + b / 8: consecutive items run on one XCD, the
// blocks of all groups at one (tile, row) run together there, and the
// jobs of a pass that share a key (one rotation, different groups) read its words
// through that XCD's L2 at the same time. The key is in Montgomery form, so a
// reduction of a 128-bit sum of at most `fold` products (fold q < 2^64) is the plain
// sum of those products.
__global__ void kb_inner_sum_kernel(uint64_t* __restrict__ TA, uint64_t* __restrict__ C0A,
                                    const uint64_t* __restrict__ X, const KsJob* __restrict__ jobs,
                                    const KsGroupRange* __restrict__ ranges, const uint32_t* __restrict__ members,
                                    const uint64_t* __restrict__ mods, const uint64_t* __restrict__ qinv, int n,
                                    int logn, int nq, int L, int Lc, int K, int dn, int fold, uint32_t nranges,
                                    uint32_t ntiles, uint32_t work, uint32_t per_xcd) {
    const uint32_t bid = blockIdx.x;
    const uint32_t wk = (bid & 7u) * per_xcd + (bid >> 3);
    if (wk >= work) return;  // uniform over the block
    const uint32_t tr = wk / nranges;
    const int x = (int)(tr % ntiles) * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int row = (int)(tr / ntiles), R = Lc + K;
    const KsGroupRange gr = ranges[wk % nranges];
    if (row < R) {
        const int pr = row_prime(row, Lc, L);
        const uint64_t q = mods[pr], qi = qinv[pr];
        const size_t keyrow = (size_t)nq * n;
        u128p a0{0, 0}, a1{0, 0};
        uint64_t s0 = 0, s1 = 0;
        int terms = 0;
        for (uint32_t u = gr.j0; u < gr.j1; u++) {
            const KsJob jb = jobs[members[u]];
            gl_cu64* kp = gl(jb.key) + (size_t)pr * n + x;
            const uint64_t* xp = X + ((size_t)jb.xidx * dn * R + row) * n + x;
            for (int j = 0; j < dn; j++) {
                const uint64_t xv = xp[(size_t)j * R * n];
                add128(a0, mul128(xv, kp[(size_t)j * 2 * keyrow]));
                add128(a1, mul128(xv, kp[(size_t)j * 2 * keyrow + keyrow]));
                if (++terms == fold) {
                    s0 = add_mod(s0, redc(a0, q, qi), q);
                    s1 = add_mod(s1, redc(a1, q, qi), q);
                    a0 = u128p{0, 0};
                    a1 = u128p{0, 0};
                    terms = 0;
                }
            }
        }
        s0 = add_mod(s0, redc(a0, q, qi), q);
        s1 = add_mod(s1, redc(a1, q, qi), q);
        uint64_t* ta = TA + ((size_t)gr.g * 2 * R + row) * n + x;
        ta[0] = add_mod(ta[0], s0, q);
        ta[(size_t)R * n] = add_mod(ta[(size_t)R * n], s1, q);
    } else {
        const int i = row - R;
        const uint64_t q = mods[i];
        uint64_t* ca = C0A + ((size_t)gr.g * Lc + i) * n + x;
        uint64_t acc = *ca;
        for (uint32_t u = gr.j0; u < gr.j1; u++) {
            const KsJob jb = jobs[members[u]];
            const uint32_t src = (jb.k == 1) ? x : galois_src(x, jb.k, logn);
            acc = add_mod(acc, gl(jb.in)[(size_t)i * n + src], q);
        }
        *ca = acc;
    }
}

void kb_inner_sum(const Ctx& c, uint64_t* TA, uint64_t* C0A, const uint64_t* X, const KsJob* jobs,
                  const KsGroupRange* ranges, const uint32_t* members, int nranges, int M, int nkeys, int Lc,
                  hipStream_t st) {
    const int R = Lc + c.K, dn = Lc / c.alpha;
    uint64_t qmax = 0;
    for (int i = 0; i < c.nq; i++) qmax = qmax > c.primes[i] ? qmax : c.primes[i];
    const int fold = (int)std::min<uint64_t>(1024, (~0ull) / qmax);
    // the distinct keys once, each job's raised digits and rotated c0 once, the sums read and written
    const double n = c.n;
    TimeScope ts(c, HC_KT_KS_INNER, st,
                 8.0 * n * ((double)nkeys * 2 * dn * R + (double)M * (dn * R + Lc) + (double)nranges * 2 * (2 * R + Lc)),
                 2.0 * dn * R * n * M);
    const uint32_t ntiles = (uint32_t)((c.n + EW_THREADS - 1) / EW_THREADS);
    const uint64_t work = (uint64_t)nranges * ntiles * (uint32_t)(R + Lc);
    const uint32_t per_xcd = (uint32_t)((work + 7) / 8);
    hc_launch(kb_inner_sum_kernel, dim3(per_xcd * 8), dim3(EW_THREADS), 0, st, TA, C0A, X, jobs, ranges,
                       members, c.d_mods, c.d_qinv, c.n, c.logn, c.nq, c.L, Lc, c.K, dn, fold < 1 ? 1 : fold,
                       (uint32_t)nranges, ntiles, (uint32_t)work, per_xcd);
}

__global__ void zero_words_kernel(uint64_t* __restrict__ p, size_t words) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) p[i] = 0;
}

void k_zero(const Ctx& c, uint64_t* p, size_t words, hipStream_t st) {
    (void)c;
    if (words) hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, p, words);
}

// y[g] = sum_{t < cnt} src[g][t] for `groups` groups of `cnt` ciphertexts (stride CW words
// between ciphertexts, cnt*CW between groups); rows: 2 Lc per ciphertext.
__global__ void sum_cts_kernel(uint64_t* __restrict__ y, const uint64_t* __restrict__ src,
                               const uint64_t* __restrict__ mods, int n, int Lc, int cnt, size_t CW) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int rr = blockIdx.y, g = blockIdx.z;  // rr = comp * Lc + row
    const uint64_t q = mods[rr % Lc];
    const uint64_t* s = src + (size_t)g * cnt * CW + (size_t)rr * n + x;
    uint64_t acc = 0;
    for (int t = 0; t < cnt; t++) acc = add_mod(acc, s[(size_t)t * CW], q);
    y[(size_t)g * CW + (size_t)rr * n + x] = acc;
}

void k_sum_cts(const Ctx& c, uint64_t* y, const uint64_t* src, int groups, int cnt, int Lc, hipStream_t st) {
    const size_t CW = 2 * (size_t)Lc * c.n;
    hipLaunchKernelGGL(sum_cts_kernel, ew_grid(c.n, 2 * Lc, groups), dim3(EW_THREADS), 0, st, y, src,
                       c.d_mods, c.n, Lc, cnt, CW);
}

// ------------------------------------------------------------------ modulus switching

// conv[c][i][x] = sum_{j dropped} [ct_j(x) (D/q_j)^-1]_{q_j} (D/q_j) mod q_i  for kept i < Lc;
// ct [count][2][L][n] (L = the source level) with the dropped rows Lc..L-1 in the
// coefficient domain; blockIdx.z = t*2+comp.
// A thread covers CONV_ROWS consecutive kept primes: each dropped residue is read and
// scaled once (PRE: the rows already hold [ct_j (D/q_j)^-1]_{q_j}).
template <int NI, bool PRE>
__global__ void ms_conv_kernel(uint64_t* __restrict__ conv, const uint64_t* __restrict__ ct,
                               const uint64_t* __restrict__ mods, const uint64_t* __restrict__ qinv,
                               const uint64_t* __restrict__ inv, const uint64_t* __restrict__ cst,
                               int n, int L, int Lc, int i0) {
    // two adjacent coefficients per thread: each row is read in 16-byte pieces
    const int x = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    if (x >= n) return;
    const int tc = blockIdx.z, nd = L - Lc;
    const uint64_t* cc = ct + (size_t)tc * L * n;
    u128p acc[NI][2];
    uint64_t sum[NI][2];
    #pragma unroll
    for (int u = 0; u < NI; u++) sum[u][0] = sum[u][1] = 0;
    // the dropped residues in batches of 8 whose loads issue together; each batch's
    // 128-bit sums (8 products below 2^60 q_i) are reduced before the next
    constexpr int MS_BATCH = 8;
    for (int j0 = 0; j0 < nd; j0 += MS_BATCH) {
        ulonglong2 v[MS_BATCH];
        #pragma unroll
        for (int b = 0; b < MS_BATCH; b++)
            if (j0 + b < nd) v[b] = *reinterpret_cast<const ulonglong2*>(cc + (size_t)(Lc + j0 + b) * n + x);
        #pragma unroll
        for (int u = 0; u < NI; u++) acc[u][0] = acc[u][1] = u128p{0, 0};
        #pragma unroll
        for (int b = 0; b < MS_BATCH; b++) {
            const int j = j0 + b;
            if (j < nd) {
                uint64_t y0 = v[b].x, y1 = v[b].y;
                if (!PRE) {
                    const uint64_t qj = mods[Lc + j], w = inv[2 * j], wp = inv[2 * j + 1];
                    y0 = shoup(y0, w, wp, qj);
                    y1 = shoup(y1, w, wp, qj);
                }
                const uint64_t* cj = cst + (size_t)j * Lc + i0;
                #pragma unroll
                for (int u = 0; u < NI; u++) {
                    add128(acc[u][0], mul128(y0, cj[u]));
                    add128(acc[u][1], mul128(y1, cj[u]));
                }
            }
        }
        #pragma unroll
        for (int u = 0; u < NI; u++) {
            const uint64_t q = mods[i0 + u], qi = qinv[i0 + u];
            sum[u][0] = add_mod(sum[u][0], redc(acc[u][0], q, qi), q);
            sum[u][1] = add_mod(sum[u][1], redc(acc[u][1], q, qi), q);
        }
    }
    #pragma unroll
    for (int u = 0; u < NI; u++)
        *reinterpret_cast<ulonglong2*>(conv + ((size_t)tc * Lc + i0 + u) * n + x) = ulonglong2{sum[u][0], sum[u][1]};
}

// out[t][c][i] = (ct[t][c][i] - conv[t][c][i]) D^-1 mod q_i, out at level Lc (element-wise:
// ct and conv in the same domain, NTT or coefficient)
__global__ void ms_final_kernel(uint64_t* __restrict__ out, const uint64_t* __restrict__ ct,
                                const uint64_t* __restrict__ conv, const uint64_t* __restrict__ mods,
                                const uint64_t* __restrict__ dinv, int n, int L, int Lc) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int tc = blockIdx.z, i = blockIdx.y;
    const uint64_t q = mods[i];
    uint64_t d = sub_mod(ct[((size_t)tc * L + i) * n + x], conv[((size_t)tc * Lc + i) * n + x], q);
    out[((size_t)tc * Lc + i) * n + x] = shoup(d, dinv[2 * i], dinv[2 * i + 1], q);
}

// Calls f(integral_constant<int, v>) for a runtime v in 1..8.
template <typename F>
static void with_rows(int v, F&& f) {
    switch (v) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        case 7: f(std::integral_constant<int, 7>{}); break;
        default: f(std::integral_constant<int, 8>{}); break;
    }
}

void k_ms_conv(const Ctx& c, uint64_t* conv, const uint64_t* ct, const uint64_t* inv, const uint64_t* cst,
               int Lin, int Lc, int count, hipStream_t st) {
    if (count <= 0) return;
    // the kept primes in chunks of up to CONV_ROWS per thread (primes below 2^60, so a
    // batch of 8 products stays below q 2^64)
    for (int i0 = 0; i0 < Lc; i0 += CONV_ROWS)
        with_rows(std::min(CONV_ROWS, Lc - i0), [&](auto ni_c) {
            constexpr int NI = decltype(ni_c)::value;
            if (inv)
                hipLaunchKernelGGL((ms_conv_kernel<NI, false>), ew_grid(c.n / 2, 1, 2 * count), dim3(EW_THREADS), 0, st,
                                   conv, ct, c.d_mods, c.d_qinv, inv, cst, c.n, Lin, Lc, i0);
            else
                hipLaunchKernelGGL((ms_conv_kernel<NI, true>), ew_grid(c.n / 2, 1, 2 * count), dim3(EW_THREADS), 0, st,
                                   conv, ct, c.d_mods, c.d_qinv, inv, cst, c.n, Lin, Lc, i0);
        });
}

void k_ms_final(const Ctx& c, uint64_t* out, const uint64_t* ct, const uint64_t* conv, const uint64_t* dinv,
                int Lin, int Lc, int count, hipStream_t st) {
    hipLaunchKernelGGL(ms_final_kernel, ew_grid(c.n, Lc, 2 * count), dim3(EW_THREADS), 0, st, out, ct, conv,
                       c.d_mods, dinv, c.n, Lin, Lc);
}

// element-wise jobs over ciphertexts at level Lc; blockIdx.y = comp * Lc + row
__global__ void ew_jobs_kernel(const EwJob* __restrict__ jobs, const uint64_t* __restrict__ mods,
                               const uint64_t* __restrict__ qinv, int n, int Lc, int mul) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const EwJob jb = jobs[blockIdx.z];
    const int rr = blockIdx.y, row = rr % Lc;
    const uint64_t q = mods[row];
    const size_t o = (size_t)rr * n + x;
    if (mul) jb.out[o] = mont_mul(jb.a[o], jb.b[(size_t)row * n + x], q, qinv[row]);
    else jb.out[o] = add_mod(jb.a[o], jb.b[o], q);
}

__global__ void mask_jobs_kernel(const MaskJob* __restrict__ jobs, const uint64_t* __restrict__ mods,
                                 const uint64_t* __restrict__ qinv, int n, int L) {
    // blockIdx.y = row (the grid covers the rows asked for)
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const MaskJob jb = jobs[blockIdx.z];
    const int row = blockIdx.y;
    const uint64_t q = mods[row], qi = qinv[row];
    const size_t o0 = (size_t)row * n + x, o1 = ((size_t)L + row) * n + x;
    const uint64_t a0 = jb.a[o0], a1 = jb.a[o1];
    #pragma unroll 4
    for (uint32_t col = 0; col < jb.ncol; col++) {
        const uint64_t p = jb.b[col * jb.b_step + o0];
        uint64_t* out = jb.out + col * jb.out_step;
        out[o0] = mont_mul(a0, p, q, qi);
        out[o1] = mont_mul(a1, p, q, qi);
    }
}

void k_mask_jobs(const Ctx& c, const MaskJob* jobs, int M, int rows, int L, hipStream_t st) {
    if (M <= 0 || rows <= 0) return;
    hipLaunchKernelGGL(mask_jobs_kernel, ew_grid(c.n, rows, M), dim3(EW_THREADS), 0, st, jobs, c.d_mods, c.d_qinv,
                       c.n, L);
}

void k_ew_jobs(const Ctx& c, const EwJob* jobs, int M, int Lc, bool mul, hipStream_t st) {
    if (M <= 0) return;
    hipLaunchKernelGGL(ew_jobs_kernel, ew_grid(c.n, 2 * Lc, M), dim3(EW_THREADS), 0, st, jobs, c.d_mods,
                       c.d_qinv, c.n, Lc, mul ? 1 : 0);
}

// ------------------------------------------------------------------ encoding

__global__ void slots_to_eval_kernel(uint32_t* out, const uint32_t* slots, const uint32_t* slotpos,
                                     int n, uint32_t p) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    size_t base = (size_t)blockIdx.z * n;
    out[base + slotpos[x]] = slots[base + x] % p;
}

void k_slots_to_eval(const Ctx& c, uint32_t* out, const uint32_t* slots, int count, hipStream_t st) {
    hipLaunchKernelGGL(slots_to_eval_kernel, ew_grid(c.n, 1, count), dim3(EW_THREADS), 0, st, out,
                       slots, c.d_slotpos, c.n, (uint32_t)c.p);
}

__global__ void lift_kernel(uint64_t* out, const uint32_t* in, const uint64_t* mods,
                            const uint64_t* qinv, const uint64_t* r2, int n, int L, uint32_t p,
                            int mont) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int r = blockIdx.y;
    uint32_t m = in[(size_t)blockIdx.z * n + x];
    uint64_t q = mods[r];
    uint64_t v = (m > p / 2) ? q - (uint64_t)(p - m) : (uint64_t)m;  // centred lift
    if (mont) v = mont_mul(v, r2[r], q, qinv[r]);
    out[((size_t)blockIdx.z * L + r) * n + x] = v;
}

void k_lift(const Ctx& c, uint64_t* out, const uint32_t* in, int count, bool mont, int Lc,
            hipStream_t st) {
    hipLaunchKernelGGL(lift_kernel, ew_grid(c.n, Lc, count), dim3(EW_THREADS), 0, st, out, in,
                       c.d_mods, c.d_qinv, c.d_r2, c.n, Lc, (uint32_t)c.p, mont ? 1 : 0);
}

__device__ __forceinline__ uint32_t mulmod_p(uint32_t a, uint32_t b, uint32_t p, double pinv) {
    uint64_t x = (uint64_t)a * b;
    uint64_t qt = (uint64_t)((double)x * pinv);
    int64_t r = (int64_t)(x - qt * p);
    if (r < 0) r += p;
    if (r >= (int64_t)p) r -= p;
    return (uint32_t)r;
}

// slot (row, m) of the diagonal (beta, gi, b): alpha^e mod p with
// alpha = beta nh + ((m + b) mod nh) + 1, e = ((m - gi B) mod s) + 1; written
// at its NTT-mod-p position.
__global__ void diag_gen_kernel(uint32_t* out, const uint32_t* params, const uint32_t* posslot,
                                int n, int nh, uint32_t p, uint32_t s, uint32_t B) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint32_t* pr = params + 3 * blockIdx.z;
    uint32_t beta = pr[0], gi = pr[1], b = pr[2];
    uint32_t m = posslot[x] % nh;  // column (both rows equal)
    uint64_t alpha = ((uint64_t)beta * nh + ((m + b) % nh) + 1) % p;
    uint32_t e = ((m + s * (uint32_t)nh - (gi * B) % s) % s) + 1;
    double pinv = 1.0 / (double)p;
    uint32_t base = (uint32_t)alpha, acc = 1;
    while (e) {
        if (e & 1) acc = mulmod_p(acc, base, p, pinv);
        base = mulmod_p(base, base, p, pinv);
        e >>= 1;
    }
    out[(size_t)blockIdx.z * n + x] = acc;
}

void k_diag_gen(const Ctx& c, uint32_t* out, const uint32_t* params, int count, uint32_t s,
                uint32_t B, hipStream_t st) {
    hipLaunchKernelGGL(diag_gen_kernel, ew_grid(c.n, 1, count), dim3(EW_THREADS), 0, st, out, params,
                       c.d_posslot, c.n, c.nh, (uint32_t)c.p, s, B);
}

// The unencrypted-database form's diagonals: slot (row r, m) of the diagonal for the
// u-block whose row r holds record block beta_r, giant gi, baby b: alpha^e times, for
// the matrix C diag(DB_c), the value of that record (0 past the database's end), with
// alpha = beta_r nh + ((m + b) mod nh) + 1 and e = ((m - gi B) mod s) + 1.
__global__ void diag_gen_db_kernel(uint32_t* out, const uint32_t* params, const uint32_t* posslot,
                                   const uint32_t* raw, uint64_t Ndb, int n, int nh, uint32_t p, uint32_t s,
                                   uint32_t B) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint32_t* pr = params + 7 * blockIdx.z;
    const uint32_t slot = posslot[x];
    const uint32_t row = slot / (uint32_t)nh, m = slot % (uint32_t)nh;
    const uint32_t beta = pr[row], gi = pr[2], b = pr[3], col = pr[4 + row], rec0 = pr[6];
    uint32_t acc = 0;
    if (col != 0xffffffffu) {
        const uint32_t cc = (m + b) % (uint32_t)nh;
        const uint64_t alpha = ((uint64_t)beta * nh + cc + 1) % p;
        uint32_t e = ((m + s * (uint32_t)nh - (gi * B) % s) % s) + 1;
        const double pinv = 1.0 / (double)p;
        uint32_t base = (uint32_t)alpha;
        acc = 1;
        while (e) {
            if (e & 1) acc = mulmod_p(acc, base, p, pinv);
            base = mulmod_p(base, base, p, pinv);
            e >>= 1;
        }
        if (col > 0) {
            const uint64_t rec = (uint64_t)rec0 + (uint64_t)beta * nh + cc;
            const uint32_t v = rec < Ndb ? raw[(uint64_t)(col - 1) * Ndb + rec] : 0u;
            acc = mulmod_p(acc, v, p, pinv);
        }
    }
    out[(size_t)blockIdx.z * n + x] = acc;
}

void k_diag_gen_db(const Ctx& c, uint32_t* out, const uint32_t* params, int count, uint32_t s, uint32_t B,
                   const uint32_t* raw, uint64_t Ndb, hipStream_t st) {
    hipLaunchKernelGGL(diag_gen_db_kernel, ew_grid(c.n, 1, count), dim3(EW_THREADS), 0, st, out, params,
                       c.d_posslot, raw, Ndb, c.n, c.nh, (uint32_t)c.p, s, B);
}

// ------------------------------------------------------------------ encryption helpers

__global__ void enc_finish_kernel(uint64_t* ct, const uint64_t* e0, const uint64_t* e1,
                                  const uint32_t* m, const uint64_t* mods, const uint64_t* delta,
                                  int n, int L) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int r = blockIdx.y;
    uint64_t q = mods[r];
    size_t o = (size_t)r * n + x;
    uint64_t dm = shoup((uint64_t)m[x], delta[2 * r], delta[2 * r + 1], q);
    ct[o] = add_mod(add_mod(ct[o], e0[o], q), dm, q);
    ct[(size_t)L * n + o] = add_mod(ct[(size_t)L * n + o], e1[o], q);
}

void k_enc_finish(const Ctx& c, uint64_t* ct, const uint64_t* e0, const uint64_t* e1,
                  const uint32_t* m, hipStream_t st) {
    hipLaunchKernelGGL(enc_finish_kernel, ew_grid(c.n, c.L), dim3(EW_THREADS), 0, st, ct, e0, e1, m,
                       c.d_mods, c.d_delta, c.n, c.L);
}

// out = e - a s + g sigma(s)   (s, sigma(s) in Montgomery form; g per row or none)
__global__ void keyrow_kernel(uint64_t* out, const uint64_t* e, const uint64_t* a,
                              const uint64_t* s_mont, const uint64_t* rs_mont, const uint64_t* grow,
                              const uint64_t* mods, const uint64_t* qinv, int n, int lf) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int rr = blockIdx.y, r = lf + rr;
    uint64_t q = mods[r], qi = qinv[r];
    size_t o = (size_t)rr * n + x;
    uint64_t v = sub_mod(e[o], mont_mul(a[o], s_mont[(size_t)r * n + x], q, qi), q);
    if (grow != nullptr && grow[r] != 0)
        v = add_mod(v, mont_mul(grow[r], rs_mont[(size_t)r * n + x], q, qi), q);
    out[o] = v;
}

void k_keyrow(const Ctx& c, uint64_t* out, const uint64_t* e, const uint64_t* a,
              const uint64_t* s_mont, const uint64_t* rot_s_mont, const uint64_t* grow, int lf, int nl,
              hipStream_t st) {
    hipLaunchKernelGGL(keyrow_kernel, ew_grid(c.n, nl), dim3(EW_THREADS), 0, st, out, e, a, s_mont,
                       rot_s_mont, grow, c.d_mods, c.d_qinv, c.n, lf);
}

// ------------------------------------------------------------------ SHAKE-128 samplers (FIPS 202)

__constant__ uint64_t c_keccak_rc[24];
__constant__ uint32_t c_keccak_rho[25];
__constant__ uint32_t c_cdt[20];

__device__ __forceinline__ uint64_t rotl64(uint64_t x, uint32_t r) {
    return r == 0 ? x : ((x << r) | (x >> (64 - r)));
}

// Keccak-f[1600]: lanes A[x + 5y]; theta, rho+pi, chi, iota per round.
__device__ void keccak_f1600(uint64_t A[25]) {
    for (int round = 0; round < 24; round++) {
        uint64_t C[5], D[5], Bm[25];
        #pragma unroll
        for (int x = 0; x < 5; x++) C[x] = A[x] ^ A[x + 5] ^ A[x + 10] ^ A[x + 15] ^ A[x + 20];
        #pragma unroll
        for (int x = 0; x < 5; x++) D[x] = C[(x + 4) % 5] ^ rotl64(C[(x + 1) % 5], 1);
        #pragma unroll
        for (int i = 0; i < 25; i++) A[i] ^= D[i % 5];
        #pragma unroll
        for (int x = 0; x < 5; x++)
            #pragma unroll
            for (int y = 0; y < 5; y++)
                Bm[y + 5 * ((2 * x + 3 * y) % 5)] = rotl64(A[x + 5 * y], c_keccak_rho[x + 5 * y]);
        #pragma unroll
        for (int x = 0; x < 5; x++)
            #pragma unroll
            for (int y = 0; y < 5; y++)
                A[x + 5 * y] = Bm[x + 5 * y] ^ (~Bm[(x + 1) % 5 + 5 * y] & Bm[(x + 2) % 5 + 5 * y]);
        A[0] ^= c_keccak_rc[round];
    }
}

struct Seed32 { uint64_t w[4]; };

// SHAKE-128 of seed || tag || le64(obj) || le64(limb) || le64(block): the
// 64-byte message fits one 168-byte rate block.
struct Shake {
    uint64_t A[25];
    int pos;
    __device__ void init(const Seed32& sd, uint64_t tag, uint64_t obj, uint64_t limb, uint64_t block) {
        #pragma unroll
        for (int i = 0; i < 25; i++) A[i] = 0;
        A[0] = sd.w[0]; A[1] = sd.w[1]; A[2] = sd.w[2]; A[3] = sd.w[3];
        A[4] = tag; A[5] = obj; A[6] = limb; A[7] = block;
        A[8] ^= 0x1Full;                  // SHAKE domain bits + first pad bit
        A[20] ^= 0x8000000000000000ull;   // last pad bit at byte 167
        keccak_f1600(A);
        pos = 0;
    }
    __device__ uint64_t next_lane() {
        if (pos == 21) { keccak_f1600(A); pos = 0; }
        return A[pos++];
    }
};

// x mod q for a 64-bit x (q < 2^62): quotient estimate in double, corrected.
__device__ __forceinline__ uint64_t mod64(uint64_t x, uint64_t q) {
    uint64_t est = (uint64_t)((double)x / (double)q);
    int64_t r = (int64_t)(x - est * q);
    while (r < 0) r += (int64_t)q;
    while (r >= (int64_t)q) r -= (int64_t)q;
    return (uint64_t)r;
}

__global__ void sample_uniform_kernel(uint64_t* out, Seed32 sd, uint64_t tag, uint64_t obj, int lf,
                                      int n, const uint64_t* mods, const uint64_t* qinv,
                                      const uint64_t* r2) {
    const int nblk = n / 256;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk) return;
    const int row = blockIdx.y;
    const int prime = lf + row;
    const uint64_t q = mods[prime];
    Shake sh;
    sh.init(sd, tag, obj, (uint64_t)prime, (uint64_t)t);
    uint64_t* o = out + (size_t)row * n + (size_t)t * 256;
    for (int c = 0; c < 256; c++) {
        uint64_t lo = sh.next_lane();
        uint64_t hi = sh.next_lane();
        // (hi 2^64 + lo) mod q = (hi mod q) 2^64 + lo mod q
        uint64_t h = mont_mul(mod64(hi, q), r2[prime], q, qinv[prime]);
        o[c] = add_mod(h, mod64(lo, q), q);
    }
}

void k_sample_uniform(const Ctx& c, uint64_t* out, const uint8_t* seed, uint64_t tag, uint64_t obj,
                      int lf, int nl, hipStream_t st) {
    Seed32 sd;
    std::memcpy(sd.w, seed, 32);
    int nblk = c.n / 256;
    hipLaunchKernelGGL(sample_uniform_kernel, dim3((nblk + 63) / 64, nl), dim3(64), 0, st, out, sd,
                       tag, obj, lf, c.n, c.d_mods, c.d_qinv, c.d_r2);
}

__global__ void sample_small_kernel(uint64_t* out, int64_t* raw, Seed32 sd, uint64_t tag,
                                    uint64_t obj, int kind, int lf, int nl, int n,
                                    const uint64_t* mods) {
    const int nblk = n / 256;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblk) return;
    Shake sh;
    sh.init(sd, tag, obj, ~0ull, (uint64_t)t);
    uint64_t lane = 0;
    for (int c = 0; c < 256; c++) {
        int64_t v;
        if (kind == 1) {  // ternary: 4 bytes per coefficient
            if ((c & 1) == 0) lane = sh.next_lane();
            uint64_t w = (c & 1) ? (lane >> 32) : (lane & 0xffffffffull);
            v = (int64_t)((3ull * w) >> 32) - 1;
        } else {          // Gaussian: 8 bytes per coefficient
            lane = sh.next_lane();
            uint32_t r = (uint32_t)lane;
            uint32_t neg = (uint32_t)(lane >> 32) & 1u;
            int mag = 0;
            for (int k = 0; k < 19; k++) mag += (r >= c_cdt[k]) ? 1 : 0;
            v = neg ? -mag : mag;
        }
        size_t idx = (size_t)t * 256 + c;
        if (raw) raw[idx] = v;
        for (int rr = 0; rr < nl; rr++) {
            uint64_t q = mods[lf + rr];
            out[(size_t)rr * n + idx] = v < 0 ? q - (uint64_t)(-v) : (uint64_t)v;
        }
    }
}

void k_sample_small(const Ctx& c, uint64_t* out, int64_t* raw, const uint8_t* seed, uint64_t tag,
                    uint64_t obj, int kind, int lf, int nl, hipStream_t st) {
    Seed32 sd;
    std::memcpy(sd.w, seed, 32);
    int nblk = c.n / 256;
    hipLaunchKernelGGL(sample_small_kernel, dim3((nblk + 63) / 64), dim3(64), 0, st, out, raw, sd,
                       tag, obj, kind, lf, nl, c.n, c.d_mods);
}

hc_status upload_keccak_constants(const uint64_t rc[24], const uint32_t rho[25], const uint32_t cdt[20]) {
    HC_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_keccak_rc), rc, sizeof(uint64_t) * 24));
    HC_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_keccak_rho), rho, sizeof(uint32_t) * 25));
    HC_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_cdt), cdt, sizeof(uint32_t) * 20));
    return HC_OK;
}

// ------------------------------------------------------------------ diagonal multiply-accumulate

// A[pp][g] = (A[pp][g] +) sum_{beta < kb, b < B} D(beta, g, b) * R[pp][beta][b], per
// (row, coefficient): for every coefficient this is a small matrix product over
// Z_q, (2 npairs x kb B) times (kb B x G), with D in Montgomery form.
//
// Arithmetic: both operands are stored split, v = v1 2^h + v0 with h = ceil(bits(q)/2),
// as the word v1 2^32 + v0, so a product is four 32 x 32 -> 64-bit multiply-adds
// (v_mad_u64_u32) into three 64-bit sums (low, middle, high) that cannot overflow for
// `chunk` terms; every `chunk` terms they are recombined into one 128-bit value T below
// q 2^64 and T mod q (= REDC(REDC(T) 2^128 mod q)) is carried on in the low sum. The
// last fold is one REDC: with D in Montgomery form that is the plain sum of products.
//
// Work: one wave per (limb, 64 consecutive coefficients, ciphertext pair, GC = 8 giant
// indices), lane = coefficient. The waves of a block are consecutive pairs with the
// same giants: they read the same diagonal words together. Blocks are numbered so
// that each XCD (blocks go to XCDs round robin) works through a contiguous range of
// work items whose fastest index is the giant chunk: the blocks resident on one XCD
// at a time share one tile of the rotated ciphertexts through that XCD's L2.
//
// Operands are tiled so that a block streams two contiguous regions: the rotated
// ciphertexts Rt[r][tile][pp][j][64][2] (term j = beta B + b; written split by
// diag_gather_kernel) and D, whose layout is given by word strides: the split word of
// D(beta, g, b) for limb r at coefficient 64 tile + lane, g = GC c + i (giant chunk c,
// i < GC), is D[r sr + tile st + c sgc + j sj + i sg + lane].
struct DiagMacArgs {
    int n, L, J, Jp, ga, npairs, wp, npg, ngc, ntiles;
    uint32_t work, per_xcd;
    size_t sr, st, sgc, sj, sg;
    int chunk, h, accumulate;
};


// Rt[r][tile][pp][j][lane][k] = R[pp][j] component k at (r, 64 tile + lane), split, for
// j < Jp (J rounded up by diag_terms_padded); nullptr and j >= J -> 0; entries equal to
// kRtInPlace were written into Rt by their producer and are left alone.
__global__ void diag_gather_kernel(uint64_t* __restrict__ Rt, const uint64_t* const* __restrict__ R,
                                   const uint32_t* __restrict__ work, int n, int L, int J, int Jp, int npairs,
                                   int w0, int h) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int r = blockIdx.y;
    const int pj = (int)work[w0 + (int)blockIdx.z];  // pp * Jp + j
    const int pp = pj / Jp, j = pj - pp * Jp;
    const uint64_t* rp = j < J ? R[(size_t)pp * J + j] : nullptr;
    if (rp == kRtInPlace) return;
    const size_t ln = (size_t)L * n;
    const size_t src = (size_t)r * n + x;
    const uint64_t v0 = rp ? rp[src] : 0, v1 = rp ? rp[ln + src] : 0;
    const size_t o = (((size_t)r * (n / 64) + (size_t)(x / 64)) * ((size_t)npairs * Jp) + pj) * 128 + 2 * (x & 63);
    *reinterpret_cast<ulonglong2*>(Rt + o) = ulonglong2{split_word(v0, h), split_word(v1, h)};
}

// The diagonals of a block are read from device memory once and shared through LDS,
// streamed by LDS DMA through a ring of NS stage buffers. A stage's diagonal words (T
// terms x GC giants x 64 coefficients, 16 KB) are written by 16 buffer_load_dwordx4 ...
// lds instructions (each puts 64 lanes x 16 bytes contiguously at the wave-uniform LDS
// base in M0), four per wave of the block (the block's pair waves and helper waves up to
// 4), issued NS - 1 stages before the stage is multiplied; each pair wave loads its
// rotated ciphertexts into NS register slots at the same distance. Per stage a wave
// waits until only the last NS - 2 stages' loads are outstanding (its own share of the
// stage has landed) and the block synchronises on a bare s_barrier: a fenced barrier
// would wait for every outstanding LDS DMA. The buffer a stage refills was multiplied in
// the stage before; the barrier orders that. The buffer (MUBUF) form of the DMA is used
// because the compiler's wait-count tracking treats a pending global (FLAT) LDS DMA as
// both a memory and an LDS access and then waits for all loads at every use of loaded
// registers. The loop covers Jp terms (a multiple of NS T; terms past J have zero
// rotated ciphertexts) with no exit in between.
#define HC_VMCNT(n) (((n) & 15) | (7 << 4) | (15 << 8) | (((n) >> 4) << 14))
// buffer resource word 3 for raw (untyped) buffer access
#define HC_RSRC_WORD3 0x00020000
typedef __attribute__((address_space(3))) void lds_void_t;

// f(integral_constant<int, i>) for i = B..E-1, unrolled at compile time
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// a wave-uniform pointer, held in scalar registers
__device__ __forceinline__ void* uniform_ptr(const void* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (void*)(((uint64_t)hi << 32) | lo);
}

template <int GC, int T, int NS>
__global__ __launch_bounds__(256) void diag_mac_kernel(uint64_t* const* __restrict__ A,
                                                            const uint64_t* __restrict__ Rt,
                                                            const uint64_t* __restrict__ D,
                                                            const uint64_t* __restrict__ mods,
                                                            const uint64_t* __restrict__ qinv,
                                                            const uint64_t* __restrict__ r2, DiagMacArgs a) {
    constexpr int PIECES = T * GC * 32;  // 16-byte pieces per stage
    constexpr int INSTR = PIECES / 64;   // wave instructions per stage
    constexpr int PER_WAVE = INSTR / 4;  // blocks are 4 waves
    static_assert(INSTR % 4 == 0 && GC % 2 == 0, "stage size");
    constexpr int RLOADS = T;            // a pair wave's rotated-ciphertext loads per stage (16 B each)
    __shared__ __attribute__((aligned(1024))) uint64_t lds[NS][T][GC][64];
    const uint32_t bid = blockIdx.x;
    const uint32_t wk = (bid & 7u) * a.per_xcd + (bid >> 3);
    if (wk >= a.work) return;  // uniform over the block
    uint32_t t = wk;
    const int gci = (int)(t % (uint32_t)a.ngc); t /= (uint32_t)a.ngc;
    const int pg = (int)(t % (uint32_t)a.npg); t /= (uint32_t)a.npg;
    const int tile = (int)(t % (uint32_t)a.ntiles);
    const int r = (int)(t / (uint32_t)a.ntiles);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int pp = pg * a.wp + w;
    const bool active = w < a.wp && pp < a.npairs;  // wave-uniform
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t q = mods[r], qi = qinv[r], q2 = r2[r];
    const int g0 = gci * GC;
    const int gc = (a.ga - g0) < GC ? (a.ga - g0) : GC;
    const int h = a.h;
    const int J = a.J, Jp = a.Jp;
    const int nst = Jp / T;  // a multiple of NS

    uint64_t lo[GC][2], mid[GC][2], hi[GC][2];
    #pragma unroll
    for (int g = 0; g < GC; g++)
        #pragma unroll
        for (int k = 0; k < 2; k++) lo[g][k] = mid[g][k] = hi[g][k] = 0;

    auto fold = [&](bool last) __attribute__((always_inline)) {
        #pragma unroll
        for (int g = 0; g < GC; g++)
            #pragma unroll
            for (int k = 0; k < 2; k++) {
                u128p T2{lo[g][k], 0};
                add128(T2, u128p{mid[g][k] << h, mid[g][k] >> (64 - h)});
                add128(T2, u128p{hi[g][k] << (2 * h), hi[g][k] >> (64 - 2 * h)});
                const uint64_t v = redc(T2, q, qi);
                lo[g][k] = last ? v : mont_mul(v, q2, q, qi);
                mid[g][k] = hi[g][k] = 0;
            }
    };

    const uint64_t* Rb = Rt + (((size_t)r * a.ntiles + tile) * a.npairs + (active ? pp : 0)) * (size_t)Jp * 128 + 2 * lane;
    const uint64_t* Db = D + (size_t)r * a.sr + (size_t)tile * a.st + (size_t)(g0 / DIAG_GC) * a.sgc +
                          (size_t)(g0 % DIAG_GC) * a.sg;
    // bytes a term's diagonal words span from their first word (giants g0..g0+gc-1)
    const int nrec = __builtin_amdgcn_readfirstlane((int)(((size_t)(gc - 1) * a.sg + 64) * 8));
    // piece c = 64 m + lane of a stage: term c / (32 GC) = m / (GC / 2), giant (c / 32) % GC,
    // words 2 (c % 32), +1 of the 64-coefficient row; it lands at byte 16 c of the stage
    // buffer. A term's words are addressed from a per-instruction buffer base.
    auto issueD = [&](int s, int buf) __attribute__((always_inline)) {
        #pragma unroll
        for (int k = 0; k < PER_WAVE; k++) {
            const int m = w * PER_WAVE + k;  // wave-uniform, so is the term
            const int tt = m / (GC / 2), g = 2 * (m % (GC / 2)) + (lane >> 5), qd = lane & 31;
            const int jd = (s * T + tt) < J ? (s * T + tt) : J - 1;
            const int gg = g < gc ? g : gc - 1;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(Db + (size_t)jd * a.sj), 0, nrec, HC_RSRC_WORD3);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)((char*)&lds[buf][0][0][0] + m * 1024), 16,
                                                     (uint32_t)((size_t)gg * a.sg + 2 * qd) * 8u, 0, 0, 0);
        }
    };
    uint64_t rv[NS][T][2];
    auto loadR = [&](int s, auto slot_c) __attribute__((always_inline)) {
        constexpr int slot = decltype(slot_c)::value;
        #pragma unroll
        for (int u = 0; u < T; u++) {
            const int jr = (s * T + u) < Jp ? (s * T + u) : Jp - 1;
            const ulonglong2 w = *reinterpret_cast<const ulonglong2*>(Rb + (size_t)jr * 128);
            rv[slot][u][0] = w.x;
            rv[slot][u][1] = w.y;
        }
    };
    int terms = 0;
    auto compute = [&](int buf, auto slot_c) __attribute__((always_inline)) {
        constexpr int slot = decltype(slot_c)::value;
        if (terms + T > a.chunk) {
            fold(false);
            terms = 0;
        }
        #pragma unroll
        for (int u = 0; u < T; u++) {
            const uint32_t r0l = (uint32_t)rv[slot][u][0], r0h = (uint32_t)(rv[slot][u][0] >> 32);
            const uint32_t r1l = (uint32_t)rv[slot][u][1], r1h = (uint32_t)(rv[slot][u][1] >> 32);
            #pragma unroll
            for (int g = 0; g < GC; g++) {
                const uint64_t d = lds[buf][u][g][lane];
                const uint32_t dl = (uint32_t)d, dh = (uint32_t)(d >> 32);
                lo[g][0] += (uint64_t)r0l * dl;
                mid[g][0] += (uint64_t)r0l * dh;
                // keeps the two middle products as two multiply-adds into the sum
                // (the compiler would otherwise add them first and then add the pair)
                asm("" : "+v"(mid[g][0]));
                mid[g][0] += (uint64_t)r0h * dl;
                hi[g][0] += (uint64_t)r0h * dh;
                lo[g][1] += (uint64_t)r1l * dl;
                mid[g][1] += (uint64_t)r1l * dh;
                asm("" : "+v"(mid[g][1]));
                mid[g][1] += (uint64_t)r1h * dl;
                hi[g][1] += (uint64_t)r1h * dh;
            }
        }
        terms += T;
    };
    // Two copies of the stage loop: pair waves (loads, products) and helper waves (their
    // share of the diagonal loads only), so neither carries a branch on the wave's role.
    // A stage's loads: the wave's rotated ciphertexts first, then its diagonal share, so
    // waiting for stage s leaves exactly the later stages' loads outstanding.
    auto run = [&](auto act_c) __attribute__((always_inline)) {
        constexpr bool ACT = decltype(act_c)::value;
        auto stage_loads = [&](int s, auto slot_c) __attribute__((always_inline)) {
            if constexpr (ACT) loadR(s, slot_c);
            issueD(s, decltype(slot_c)::value);
        };
        auto wait_stage = [&]() __attribute__((always_inline)) {
            __builtin_amdgcn_s_waitcnt(HC_VMCNT((NS - 2) * ((ACT ? RLOADS : 0) + PER_WAVE)));
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
        };
        auto mul = [&](int buf, auto slot_c) __attribute__((always_inline)) {
            if constexpr (ACT) compute(buf, slot_c);
            __builtin_amdgcn_sched_barrier(0);
        };
        static_for<0, NS - 1>([&](auto i_c) __attribute__((always_inline)) { stage_loads(i_c.value, i_c); });
        for (int s = 0; s < nst; s += NS) {
            static_for<0, NS>([&](auto i_c) __attribute__((always_inline)) {
                constexpr int i = decltype(i_c)::value;
                wait_stage();
                stage_loads(s + i + NS - 1, std::integral_constant<int, (i + NS - 1) % NS>{});
                mul(i, i_c);
            });
        }
    };
    if (active) run(std::true_type{});
    else run(std::false_type{});
    // the last NS - 1 stages' loads (clamped to valid terms) land before the block's LDS
    // can be handed to another block
    __builtin_amdgcn_s_waitcnt(HC_VMCNT(0));
    if (!active) return;
    fold(true);
    const size_t ln = (size_t)a.L * a.n;
    const size_t off = (size_t)r * a.n + (size_t)tile * 64 + lane;
    #pragma unroll
    for (int g = 0; g < GC; g++) {
        if (g < gc) {
            uint64_t v0 = lo[g][0], v1 = lo[g][1];
            uint64_t* ap = A[(size_t)pp * a.ga + g0 + g];
            if (a.accumulate) {
                v0 = add_mod(v0, ap[off], q);
                v1 = add_mod(v1, ap[ln + off], q);
            }
            ap[off] = v0;
            ap[ln + off] = v1;
        }
    }
}

// Largest number of terms the split sums of diag_mac_kernel take before a fold,
// for residues below qmax < 2^bits split at h: the low sum starts from a residue
// below qmax, every sum stays below 2^64, and the recombined value stays below
// q 2^64 (qmax + terms (q-1)^2 < q 2^64 holds for terms < 2^64 / q).
static int diag_chunk(int bits, int h, uint64_t qmax) {
    const unsigned __int128 one = 1;
    const unsigned __int128 top = (one << 64) - 1;
    const unsigned __int128 m0 = (one << h) - 1, m1 = (one << (bits - h)) - 1;
    unsigned __int128 ch = (top - qmax) / (m0 * m0);
    if (top / (2 * m0 * m1) < ch) ch = top / (2 * m0 * m1);
    if (top / (m1 * m1) < ch) ch = top / (m1 * m1);
    const unsigned __int128 cq = (one << 64) / qmax - 1;
    if (cq < ch) ch = cq;
    if (ch > 4096) ch = 4096;
    return (int)ch;
}

// The split position for the first Lc primes: h = ceil(bits(max q) / 2).
static void diag_split_bits(const Ctx& c, int Lc, int* bits, int* h, uint64_t* qmax) {
    uint64_t m = 0;
    for (int i = 0; i < Lc; i++) m = m > c.primes[i] ? m : c.primes[i];
    int b = 0;
    while (b < 64 && (m >> b)) b++;
    *bits = b;
    *h = (b + 1) / 2;
    *qmax = m;
}

int diag_split_h(const Ctx& c, int Lc) {
    int bits, h;
    uint64_t qmax;
    diag_split_bits(c, Lc, &bits, &h, &qmax);
    return h;
}

__global__ void diag_split_kernel(uint64_t* __restrict__ d, size_t words, int h) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) d[i] = split_word(d[i], h);
}

void k_diag_split(const Ctx& c, uint64_t* d, size_t words, int Lc, hipStream_t st) {
    const size_t blocks = (words + 255) / 256;
    hipLaunchKernelGGL(diag_split_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d, words, diag_split_h(c, Lc));
}

std::vector<uint32_t> diag_gather_list(const std::vector<const uint64_t*>& R, int npairs, int J) {
    const int Jp = diag_terms_padded(J);
    std::vector<uint32_t> w;
    for (int pp = 0; pp < npairs; pp++)
        for (int j = 0; j < Jp; j++)
            if (j >= J || R[(size_t)pp * J + j] != kRtInPlace) w.push_back((uint32_t)(pp * Jp + j));
    return w;
}

void k_diag_gather(const Ctx& c, uint64_t* Rt, const uint64_t* const* R, const uint32_t* work, int nwork, int npairs,
                   int J, int Lc, hipStream_t st) {
    const int Jp = diag_terms_padded(J);
    const int h = diag_split_h(c, Lc);
    for (int w0 = 0; w0 < nwork; w0 += 65535)
        hipLaunchKernelGGL(diag_gather_kernel, ew_grid(c.n, Lc, std::min(65535, nwork - w0)), dim3(EW_THREADS), 0,
                           st, Rt, R, work, c.n, Lc, J, Jp, npairs, w0, h);
}

hc_status k_diag_mac(const Ctx& c, uint64_t* const* A, const uint64_t* Rt, const uint64_t* D,
                     const DiagLayout& lay, int npairs, int J, int ga, bool accumulate, int Lc, hipStream_t st) {
    // the kernel addresses one term's words (DIAG_GC giants) by 32-bit buffer offsets
    if (((size_t)(DIAG_GC - 1) * lay.sg + 64) * 8 >= ((size_t)1 << 31)) return HC_EINVAL;
    int bits, h;
    uint64_t qmax;
    diag_split_bits(c, Lc, &bits, &h, &qmax);
    constexpr int GC = DIAG_GC;
    DiagMacArgs a;
    a.n = c.n;
    a.L = Lc;
    a.J = J;
    a.Jp = diag_terms_padded(J);
    a.ga = ga;
    a.npairs = npairs;
    a.wp = npairs < 4 ? npairs : 4;  // pairs per block (4 waves; two blocks fit a CU)
    a.npg = (npairs + a.wp - 1) / a.wp;
    a.ngc = (ga + GC - 1) / GC;
    a.ntiles = c.n / 64;
    const uint64_t work = (uint64_t)Lc * a.ntiles * a.npg * a.ngc;
    a.work = (uint32_t)work;
    a.per_xcd = (uint32_t)((work + 7) / 8);
    a.sr = lay.sr;
    a.st = lay.st;
    a.sgc = lay.sgc;
    a.sj = lay.sj;
    a.sg = lay.sg;
    a.h = h;
    a.chunk = diag_chunk(bits, h, qmax);  // >= 8 for primes below 2^60 (folds come every DIAG_T terms)
    a.accumulate = accumulate ? 1 : 0;
    const double ln = (double)Lc * c.n;
    // reads each R (both components) and each D once, writes each A once
    TimeScope ts(c, HC_KT_DIAG_MAC, st,
                 8.0 * ln * (2.0 * npairs * J + (double)J * ga + (accumulate ? 4.0 : 2.0) * npairs * ga),
                 2.0 * ln * npairs * J * ga);
    // the tuned variant (hc_autotune): terms per LDS stage x stages in flight, always
    // DIAG_NS DIAG_T terms per round of the ring, so the rotated ciphertexts' padding and
    // every result word are the same for all of them
    static_assert(DIAG_T * DIAG_NS == 16, "variants below assume 16 terms per round");
    switch (c.tune_mac) {
        case 1:
            hc_launch((diag_mac_kernel<GC, 2, 8>), dim3(a.per_xcd * 8), dim3(256), 0, st, A, Rt, D, c.d_mods,
                               c.d_qinv, c.d_r2, a);
            break;
        case 2:
            hc_launch((diag_mac_kernel<GC, 8, 2>), dim3(a.per_xcd * 8), dim3(256), 0, st, A, Rt, D, c.d_mods,
                               c.d_qinv, c.d_r2, a);
            break;
        default:
            hc_launch((diag_mac_kernel<GC, DIAG_T, DIAG_NS>), dim3(a.per_xcd * 8), dim3(256), 0, st, A, Rt,
                               D, c.d_mods, c.d_qinv, c.d_r2, a);
    }
    return HC_OK;
}

// Natural layout (one [Lc][n] polynomial per diagonal, index (beta dG + g) B + b) ->
// the tiled, split layout of resident tables, [Lc][n/64][ceil(dG/GC)][kbt B][GC][64]
// (term j = beta B + b, giant g = GC c + i): the words one block (a 64-coefficient
// tile and one chunk of GC giants) multiplies by form one contiguous run. `count`
// diagonals starting at index i0.
__global__ void diag_tile_kernel(uint64_t* __restrict__ out, const uint64_t* __restrict__ in, size_t i0,
                                 int n, int L, uint32_t kbt, uint32_t B, uint32_t dG, int h) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int r = blockIdx.y;
    const size_t i = i0 + blockIdx.z;
    const uint32_t b = (uint32_t)(i % B);
    const uint32_t g = (uint32_t)((i / B) % dG);
    const uint32_t beta = (uint32_t)(i / ((size_t)B * dG));
    const size_t Jt = (size_t)kbt * B, nch = (dG + DIAG_GC - 1) / DIAG_GC;
    const size_t per_chunk = Jt * DIAG_GC * 64;
    const size_t o = (((size_t)r * (n / 64) + (size_t)(x / 64)) * nch + g / DIAG_GC) * per_chunk +
                     (((size_t)beta * B + b) * DIAG_GC + g % DIAG_GC) * 64 + (x & 63);
    out[o] = split_word(in[((size_t)blockIdx.z * L + r) * n + x], h);
}

void k_diag_tile(const Ctx& c, uint64_t* out, const uint64_t* in, size_t i0, int count, uint32_t kbt,
                 uint32_t B, uint32_t dG, int Lc, hipStream_t st) {
    hipLaunchKernelGGL(diag_tile_kernel, ew_grid(c.n, Lc, count), dim3(EW_THREADS), 0, st, out, in, i0, c.n,
                       Lc, kbt, B, dG, diag_split_h(c, Lc));
}

size_t diag_table_words(const Ctx& c, int Lc, uint32_t Jt, uint32_t dG) {
    return (size_t)Lc * c.n * Jt * ((dG + DIAG_GC - 1) / DIAG_GC) * DIAG_GC;
}

DiagLayout diag_layout_natural(const Ctx& c, int Lc, uint32_t gc) {
    const size_t ln = (size_t)Lc * c.n;
    DiagLayout l;
    l.sr = c.n;
    l.st = 64;
    l.sg = ln;
    l.sgc = DIAG_GC * ln;
    l.sj = (size_t)gc * ln;
    return l;
}

DiagLayout diag_layout_tiled(const Ctx& c, uint32_t Jt, uint32_t dG) {
    DiagLayout l;
    l.sg = 64;
    l.sj = (size_t)DIAG_GC * 64;
    l.sgc = (size_t)Jt * DIAG_GC * 64;
    l.st = ((dG + DIAG_GC - 1) / DIAG_GC) * l.sgc;
    l.sr = (size_t)(c.n / 64) * l.st;
    return l;
}


// ------------------------------------------------------------------ throughput probe

// Eight independent chains of acc = lo32(acc) * b + acc per thread: each step is
// one 32 x 32 -> 64-bit multiply-add (v_mad_u64_u32); registers only.
__global__ void probe_mul32_kernel(uint64_t* sink, uint32_t iters) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t b = tid * 2654435761u + 12345u;
    uint64_t acc[8];
    #pragma unroll
    for (int k = 0; k < 8; k++) acc[k] = (uint64_t)(tid + k) * 0x9E3779B97F4A7C15ull;
    for (uint32_t i = 0; i < iters; i++) {
        #pragma unroll
        for (int k = 0; k < 8; k++) acc[k] = (uint64_t)(uint32_t)acc[k] * b + acc[k];
    }
    uint64_t x = 0;
    #pragma unroll
    for (int k = 0; k < 8; k++) x ^= acc[k];
    sink[tid] = x;
}

}  // namespace hc

namespace hc {
__global__ void probe_copy_kernel(uint64_t* __restrict__ dst, const uint64_t* __restrict__ src, size_t words) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) dst[i] = src[i];
}
}  // namespace hc

extern "C" hc_status hc_probe_copy(hc_context* c, uint64_t bytes) {
    if (!c || bytes < 8) return HC_EINVAL;
    HC_CHECK(hipSetDevice(c->device));
    const size_t words = bytes / 8;
    uint64_t *a = nullptr, *b = nullptr;
    HC_CHECK(hipMalloc((void**)&a, words * 8));
    HC_CHECK(hipMalloc((void**)&b, words * 8));
    hipLaunchKernelGGL(hc::probe_copy_kernel, dim3(4096), dim3(256), 0, 0, b, a, words);
    HC_CHECK(hipDeviceSynchronize());
    HC_CHECK(hipFree(a));
    HC_CHECK(hipFree(b));
    return HC_OK;
}

namespace hc {
// Block b reads `rchunk` consecutive 16-byte units of src (eight per thread per round of
// 4096 units, all issued before use) and, spread evenly over its rounds, writes `wchunk`
// consecutive units of dst; the written values depend on what was read.
__global__ __launch_bounds__(512) void probe_stream_kernel(ulonglong2* __restrict__ dst,
                                                           const ulonglong2* __restrict__ src, size_t runits,
                                                           size_t wunits, size_t rchunk, size_t wchunk) {
    const size_t r0 = (size_t)blockIdx.x * rchunk, w0 = (size_t)blockIdx.x * wchunk;
    const size_t rounds = (rchunk + 4095) / 4096, wpr = (wchunk + rounds - 1) / rounds;
    uint64_t acc = 0;
    size_t wdone = 0;
    for (size_t off = threadIdx.x; off < rchunk + threadIdx.x; off += 4096) {
        ulonglong2 v[8];
        #pragma unroll
        for (int u = 0; u < 8; u++) {
            const size_t o = off + 512 * (size_t)u, k = r0 + o;
            v[u] = (o < rchunk && k < runits) ? src[k] : ulonglong2{0, 0};
        }
        #pragma unroll
        for (int u = 0; u < 8; u++) acc += v[u].x ^ v[u].y;
        const size_t wend = wdone + wpr < wchunk ? wdone + wpr : wchunk;
        for (size_t o = wdone + threadIdx.x; o < wend; o += 512)
            if (w0 + o < wunits) dst[w0 + o] = ulonglong2{acc, o};
        wdone = wend;
    }
}
}  // namespace hc

extern "C" hc_status hc_probe_stream(hc_context* c, uint64_t read_bytes, uint64_t write_bytes, int reps,
                                     double* ms_out) {
    if (!c || !ms_out || read_bytes < 16 || reps < 1) return HC_EINVAL;
    HC_CHECK(hipSetDevice(c->device));
    const size_t runits = read_bytes / 16, wunits = write_bytes / 16;
    const size_t rchunk = 57344;  // 896 KiB per block
    const size_t blocks = (runits + rchunk - 1) / rchunk, wchunk = (wunits + blocks - 1) / blocks;
    if (blocks > 0x7fffffffu) return HC_EINVAL;
    ulonglong2 *src = nullptr, *dst = nullptr;
    HC_CHECK(hipMalloc((void**)&src, runits * 16));
    if (wunits && hipMalloc((void**)&dst, wunits * 16) != hipSuccess) {
        (void)hipFree(src);
        return HC_ENOMEM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hc_status st = HC_OK;
    float ms = 0;
    if (hipMemset(src, 0x5a, runits * 16) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        st = HC_EDEVICE;
    } else {
        auto launch = [&] {
            hipLaunchKernelGGL(hc::probe_stream_kernel, dim3((unsigned)blocks), dim3(512), 0, 0, dst, src, runits, wunits,
                               rchunk, wchunk);
        };
        launch();
        if (hipEventRecord(e0, 0) != hipSuccess) st = HC_EDEVICE;
        for (int i = 0; i < reps && st == HC_OK; i++) launch();
        if (st == HC_OK && (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = HC_EDEVICE;
    }
    if (hipGetLastError() != hipSuccess) st = HC_EDEVICE;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (st == HC_OK) *ms_out = ms / reps;
    return st;
}

extern "C" hc_status hc_probe_mul32_rate(hc_context* c, double ms, double* rate_out) {
    if (!c || !rate_out || ms <= 0) return HC_EINVAL;
    HC_CHECK(hipSetDevice(c->device));
    int cus = 0;
    HC_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    const int threads = 256, blocks = cus * 16;
    uint64_t* sink = nullptr;
    HC_CHECK(hipMalloc((void**)&sink, sizeof(uint64_t) * threads * blocks));
    hipEvent_t a, b;
    HC_CHECK(hipEventCreate(&a));
    HC_CHECK(hipEventCreate(&b));
    uint32_t iters = 1024;
    double rate = 0;
    for (int rep = 0; rep < 3; rep++) {
        HC_CHECK(hipEventRecord(a, 0));
        hipLaunchKernelGGL(hc::probe_mul32_kernel, dim3(blocks), dim3(threads), 0, 0, sink, iters);
        HC_CHECK(hipEventRecord(b, 0));
        HC_CHECK(hipEventSynchronize(b));
        float el = 0;
        HC_CHECK(hipEventElapsedTime(&el, a, b));
        rate = (double)threads * blocks * iters * 8.0 / (el * 1e-3);
        double scale = ms / (el > 0 ? el : 1e-3);
        if (scale > 64) scale = 64;
        if (rep < 2) iters = (uint32_t)(iters * scale) + 1;
    }
    HC_CHECK(hipEventDestroy(a));
    HC_CHECK(hipEventDestroy(b));
    HC_CHECK(hipFree(sink));
    *rate_out = rate;
    return HC_OK;
}
