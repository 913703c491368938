/*
 * hc_kernels.h -- C ABI of libhc's ring-level operations.
 *
 * These are the building blocks hc_compress is made of, exposed one by one
 * so that each can be checked against a reference at full size: the
 * negacyclic NTT per prime, the Galois automorphisms behind the paper's
 * rotations Rot_row / Rot_col (Sec. 5.1), hybrid key switching (basis
 * conversion up and down), the plaintext-ciphertext product (the boxtimes of
 * Sec. 2.2 / Alg. 7 step 2) and the seeded samplers. Conventions as in hc.h:
 * device pointers are caller-owned HIP memory, arrays are uint64_t with
 * canonical residues, work is enqueued on `stream`.
 *
 * "Prime index" i refers to the basis q_1..q_L, p_1..p_K in that order
 * (0-based; 0..L-1 are the ciphertext primes, L..L+K-1 the special primes).
 */
#ifndef HC_KERNELS_H
#define HC_KERNELS_H

#include "hc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* In-place negacyclic NTT of `count` polynomials, each `nlimbs` consecutive
 * rows of n residues for prime indices limb_first..limb_first+nlimbs-1.
 * Forward: coefficients -> evaluations, entry i = a(psi^(2 brv(i) + 1)) with
 * brv the log_n-bit reversal and psi the library's primitive 2n-th root mod
 * the prime; inverse: the exact inverse. Output canonical.
 * Errors: HC_EINVAL (limb range outside L+K). */
hc_status hc_ntt(hc_context* ctx, uint64_t* data, uint32_t count, uint32_t limb_first,
                 uint32_t nlimbs, int inverse, hipStream_t stream);

/* Rotation of one ciphertext by sigma_k with key switching (Sec. 5.1: k = 3^r
 * mod 2n moves both slot rows left by r, k = 2n-1 swaps the rows).
 * Non-hoisted: (sigma_k(c0), sigma_k(c1)), ModUp of each digit of sigma_k(c1),
 * inner product with the key over PQ, ModDown, added to sigma_k(c0).
 * ct_in / ct_out: device [2][L][n], coefficient domain (may not alias).
 * Errors: HC_ENOKEY. */
hc_status hc_rotate(hc_context* ctx, const hc_gk* gk, uint32_t element, const uint64_t* ct_in,
                    uint64_t* ct_out, hipStream_t stream);

/* hc_rotate at a lower level: ct_in / ct_out device [2][level][n] (coefficient
 * domain, may not alias) over the first `level` ciphertext primes, key-switched
 * with the Galois key restricted to those primes, the special primes and the
 * digits inside them (still a valid key for the smaller modulus; this is how the
 * compression rotates after its modulus switch, Sec. 5.3). level: a multiple of
 * K in [K, L]. Errors: HC_EINVAL, HC_ENOKEY, HC_ENOMEM. Synchronises. */
hc_status hc_rotate_level(hc_context* ctx, const hc_gk* gk, uint32_t element, uint32_t level,
                          const uint64_t* ct_in, uint64_t* ct_out, hipStream_t stream);

/* hc_rotate_level without any allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and bit-identical results, but every temporary
 * lives in one fixed device array of HC_NOALLOC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends (found at hc_context_create).
 * The caller passes the input and output as for hc_rotate_level; the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine) and
 * synchronises `stream` before returning. A rotation at `level` needs
 * 8 n (7 level + (level / K) (level + K) + 2 K) bytes plus alignment; larger
 * calls fail with HC_ESCRATCH (ring 2^16 with 3 special primes: levels up to 9,
 * which covers the compression's Comp level; ring 2^15 with 2: every level up to
 * 14). Every call on one GPU shares that GPU's array, so calls that overlap on
 * one GPU (other streams, threads or contexts) race; serialise them. No word of
 * the array needs to start at zero: a call reads only what it wrote first.
 * Errors: as hc_rotate_level, HC_ESCRATCH, HC_EDEVICE (no scratch on the device). */
#define HC_NOALLOC_SCRATCH_BYTES (64ull << 20)
hc_status hc_rotate_level_noalloc(hc_context* ctx, const hc_gk* gk, uint32_t element, uint32_t level,
                                  const uint64_t* ct_in, uint64_t* ct_out, hipStream_t stream);

/* Modulus switching (the BFV form of the paper's move to smaller parameters,
 * Sec. 5.3, and of its single-prime answer, Sec. 6.2): drop the primes
 * level_out..level_in-1 of `count` ciphertexts. With D the product of the dropped
 * primes each component c becomes (c - Conv_{D->Q'}([c]_D)) D^-1 mod Q', Conv the
 * fast basis conversion of the dropped residues; this divides c by D (up to a
 * conversion overflow of fewer than level_in - level_out multiples of Q'), so the
 * result decrypts under Q' = q_1..q_level_out to the same slots.
 * ct_in: device [count][2][level_in][n], ct_out: device [count][2][level_out][n],
 * both coefficient domain (may not alias). 1 <= level_out < level_in <= L.
 * Errors: HC_EINVAL, HC_ENOMEM. Enqueued on `stream`; returns without waiting. */
hc_status hc_mod_switch(hc_context* ctx, const uint64_t* ct_in, uint32_t count, uint32_t level_in,
                        uint32_t level_out, uint64_t* ct_out, hipStream_t stream);

/* Hoisted rotations of one ciphertext by `count` elements: one ModUp of c1,
 * then per element sigma_k applied to the raised digits, inner product and
 * ModDown. cts_out: device [count][2][L][n]. Decrypts like hc_rotate but
 * differs in bits (sigma and the basis conversion commute only modulo D_j). */
hc_status hc_rotate_hoisted(hc_context* ctx, const hc_gk* gk, const uint32_t* elements,
                            uint32_t count, const uint64_t* ct_in, uint64_t* cts_out,
                            hipStream_t stream);

/* ct boxtimes plaintext: both components multiplied by the centred lift
 * (coefficients in (-p/2, p/2]) of the encoding of `slots` (host 2 x n/2).
 * ct_in / ct_out device [2][L][n] coefficient domain (may alias). */
hc_status hc_mul_plain(hc_context* ctx, const uint64_t* ct_in, const uint32_t* slots,
                       uint64_t* ct_out, hipStream_t stream);

/* Fast basis conversion of digit j of x (device [L][n], coefficient domain)
 * to every prime of PQ: out (device [L+K][n]) holds x on the digit's primes
 * and sum_{i in I_j} [x_i (D_j/q_i)^-1]_{q_i} (D_j/q_i) mod r elsewhere. */
hc_status hc_modup(hc_context* ctx, const uint64_t* x, uint32_t digit, uint64_t* out,
                   hipStream_t stream);

/* ModDown: out_i = (T_i - Conv_{P->Q}([T]_P)_i) P^-1 mod q_i for T device
 * [L+K][n] (coefficient domain); out device [L][n]. */
hc_status hc_moddown(hc_context* ctx, const uint64_t* T, uint64_t* out, hipStream_t stream);

/* Seeded samplers over SHAKE-128 stream(seed, tag, obj, limb, block):
 * kind 0: uniform residues mod prime `limb` (16 bytes per coefficient);
 * kind 1: ternary, kind 2: Gaussian sigma = 3.2 (limb ignored, stream limb
 * field 2^64-1), written as int64_t values. out: device, n entries. tag: up to
 * 8 ASCII characters (zero padded). */
hc_status hc_sample(hc_context* ctx, int kind, const uint8_t seed[32], const char* tag,
                    uint64_t obj, uint32_t limb, uint64_t* out, hipStream_t stream);

/* Encoding of one compression diagonal, as a centred-lift polynomial reduced
 * mod each ciphertext prime (device [L][n], coefficient domain): slot m of
 * either row holds (beta n/2 + ((m + b) mod n/2) + 1)^(((m - gi B) mod s) + 1) mod p. */
hc_status hc_encode_diagonal(hc_context* ctx, uint32_t s, uint32_t B, uint32_t beta, uint32_t gi,
                             uint32_t b, uint64_t* out, hipStream_t stream);

/* Export key material to host memory, coefficient domain, canonical:
 * sk: n int64 coefficients in {-1,0,1}; pk: [2][L][n] (b then a);
 * gk: the key for `element`, [dnum][2][L+K][n] (b_j then a_j). Synchronise. */
hc_status hc_export_sk(hc_context* ctx, const hc_sk* sk, int64_t* out);
hc_status hc_export_pk(hc_context* ctx, const hc_pk* pk, uint64_t* out);
hc_status hc_export_gk(hc_context* ctx, const hc_gk* gk, uint32_t element, uint64_t* out);

/* ------------------------------------------------------------------ measurement
 * Kernel timing: while enabled, each launch of a kernel of the given class is
 * bracketed by HIP events recorded on the stream it is launched on, so the
 * totals are device time of exactly those launches. Classes: */
enum {
    HC_KT_NTT_FWD = 0,   /* forward NTT passes (64-bit primes) */
    HC_KT_NTT_INV = 1,   /* inverse NTT passes (64-bit primes) */
    HC_KT_KS_INNER = 2,  /* key-switch inner product with the Galois key */
    HC_KT_DIAG_MAC = 3,  /* diagonal multiply-accumulate */
    HC_KT_MODUP = 4,     /* ModUp basis conversion */
    HC_KT_CONV_FUSED = 5, /* key switching's conversions fused with the NTTs' high-bit passes */
    HC_KT_COUNT = 6
};

/* Start (enable = 1) or stop timing; either call clears the totals (read them with
 * hc_timing_read before stopping). Each timed launch carries its own start/stop events
 * (hipExtLaunchKernel), which keep the launch, and with it the device memory its kernel
 * used, alive: memory the library frees while timing is on is returned to the device
 * only when timing is stopped (or restarted). Synchronises the device. */
hc_status hc_timing_enable(hc_context* ctx, int enable);

/* Totals since timing was enabled for class `kind`: device milliseconds,
 * launches, and the class's algorithmic work summed over those launches
 * (work_bytes: bytes the kernels must read and write; work_ops: butterflies
 * for the NTT classes, modular multiply-adds otherwise). Synchronises. */
hc_status hc_timing_read(hc_context* ctx, int kind, double* total_ms, uint64_t* launches,
                         double* work_bytes, double* work_ops);

/* Throughput probe: runs a register-only kernel of independent 32 x 32 -> 64-bit
 * multiply-adds on every compute unit for about `ms` milliseconds and returns
 * the measured rate in multiply-adds per second (device-wide). */
hc_status hc_probe_mul32_rate(hc_context* ctx, double ms, double* rate_out);

/* Calibration probe for memory counters: one launch of a plain copy kernel
 * (hc::probe_copy_kernel) that reads `bytes` and writes `bytes` of freshly
 * allocated device memory (rounded down to 8-byte words). Synchronises. */
hc_status hc_probe_copy(hc_context* ctx, uint64_t bytes);

/* Ceiling probe for a kernel that streams reads with a share of writes mixed in (the
 * diagonal multiply-accumulate's traffic): allocates `read_bytes` and `write_bytes`
 * of device memory, then times `reps` launches (after one untimed) of
 * hc::probe_stream_kernel, in which each block reads a contiguous 896 KiB of the
 * first buffer and, spread over its reads, writes its contiguous share of the second.
 * *ms_out = mean milliseconds per launch. Frees both buffers; synchronises.
 * Errors: HC_EINVAL (read_bytes < 16, reps < 1), HC_ENOMEM, HC_EDEVICE. */
hc_status hc_probe_stream(hc_context* ctx, uint64_t read_bytes, uint64_t write_bytes, int reps, double* ms_out);

#ifdef __cplusplus
}
#endif
#endif /* HC_KERNELS_H */
