/*
 * hc.h -- C ABI of libhc: SIMD-aware homomorphic compression for private
 * database queries (Cheon, Lee, Park, Yeo, arXiv 2408.17063) on one MI355X.
 *
 * The calls follow the paper's statement of the problem:
 *   - HE syntax KeyGen / Enc / Dec (Sec. 2.2)          -> hc_keygen, hc_galois_keygen,
 *                                                         hc_encrypt, hc_decrypt
 *   - homomorphic compression Comp / Decomp (Def. 3)   -> hc_compress, hc_decompress
 *   - PDQ Query / Answer / Recover (Def. 7, Thm. 3, Alg. 7): Query = keygen +
 *     encrypt of the index vector, Answer = hc_compress (Mask + Comp; the
 *     index vector v is the input, Match is not part of this library),
 *     Recover = hc_decrypt + hc_decompress.
 *
 * Conventions
 *   - Every call returns hc_status; nothing throws across the ABI.
 *   - Ciphertexts exchanged through the ABI are arrays of uint64_t laid out
 *     [2][L][n] (component, prime, coefficient), coefficient domain, canonical
 *     residues 0 <= x < q_i. "device" pointers are HIP device memory owned by
 *     the caller; "host" pointers are ordinary host memory owned by the caller.
 *   - Keys, the encoded database and the context are opaque handles owned by
 *     the library and resident in device memory until their *_destroy call.
 *   - hipStream_t arguments: the call enqueues its device work on that stream
 *     and returns without waiting, unless stated otherwise. Calls that take
 *     host buffers for output synchronise before returning.
 *   - One context per device; calls on one context from several threads must
 *     be serialised by the caller (the context owns a workspace).
 *
 * Scheme (BFV in RNS form; the paper's BGV slot algebra carries over unchanged):
 *   - ring R = Z[X]/(X^n + 1), n = 2^log_n; plaintext prime p = 1 mod 2n, so a
 *     plaintext is a 2 x (n/2) matrix of slots in Z_p (Sec. 5.1);
 *   - ciphertext primes q_1 > ... > q_L: the L largest primes below 2^q_bits
 *     with q = 1 mod 2n; special primes p_1 > ... > p_K: the K largest below
 *     2^p_bits with the same congruence; Delta = floor(Q / p);
 *   - hybrid key switching with digits of alpha = K consecutive primes
 *     (dnum = L / K digits);
 *   - all randomness comes from SHAKE-128 streams keyed by the 32-byte seed,
 *     so every ciphertext is a deterministic function of its inputs.
 */
#ifndef HC_H
#define HC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HC_OK = 0,
    HC_EINVAL = -1,   /* bad parameters or shapes */
    HC_ENOMEM = -2,   /* device or host allocation failed */
    HC_EDEVICE = -3,  /* a HIP call failed */
    HC_ENOKEY = -4,   /* a rotation needs a Galois key that the key set lacks */
    HC_EDECODE = -5,  /* decompression failed: more than s matches or an inconsistent input */
    HC_ENOISE = -6,   /* decryption rounding is ambiguous (noise at the budget) */
    HC_ESCRATCH = -7  /* an allocation-free call needs more than its fixed device scratch */
} hc_status;

typedef struct {
    uint32_t log_n;   /* ring degree n = 2^log_n, 10 <= log_n <= 16 */
    uint64_t p;       /* plaintext prime, p = 1 mod 2n, p < 2^26 */
    uint32_t L;       /* ciphertext primes */
    uint32_t q_bits;  /* bit size bound of the ciphertext primes, 30..60 */
    uint32_t K;       /* special primes (= primes per key-switching digit), 1..4; L % K == 0 */
    uint32_t p_bits;  /* bit size bound of the special primes, <= 61 */
} hc_params;
/* The key inner product sums the dnum = L / K digit products of a row in one
 * 128-bit accumulator before a single Montgomery reduction, so every prime q of
 * the basis must satisfy dnum * q < 2^64 (at most 15 digits of 60-bit primes, 7
 * of 61-bit ones); hc_context_create rejects parameters that break it. */

typedef struct hc_context hc_context;
typedef struct hc_sk hc_sk;
typedef struct hc_pk hc_pk;
typedef struct hc_gk hc_gk;
typedef struct hc_db hc_db;

/* What one compression did (filled by hc_compress / hc_plan). */
typedef struct {
    uint32_t s;            /* sparsity bound 2^ceil(log2 t_bound) = output slots per band */
    uint32_t groups;       /* record groups of at most p-1 records */
    uint32_t streams;      /* vector pairs (v,d_1), (d_2,d_3), ... */
    uint32_t bands;        /* groups * streams; band b occupies slots [b s, (b+1) s) */
    uint32_t n_ct;         /* input ciphertexts ceil(N / n) */
    uint32_t n_keyswitch;  /* key switches performed */
    uint64_t n_ptct;       /* plaintext-ciphertext products performed */
    uint64_t n_diag;       /* diagonal plaintexts encoded during the call */
    uint32_t level;        /* ciphertext primes of the output (out_level, else the Comp level) */
    uint64_t n_diag_resident; /* diagonal plaintexts read from resident tables (hc_diag_prepare) */
    uint32_t comp_level;   /* ciphertext primes Comp ran at */
} hc_compress_info;

/* ------------------------------------------------------------------ context */

/* Derive primes and tables for `params` on HIP device `device` and upload
 * them. Errors: HC_EINVAL (n not a power of two in range, p not prime or
 * p != 1 mod 2n, L % K != 0, not enough primes, dnum * q >= 2^64 for a prime q),
 * HC_EDEVICE, HC_ENOMEM. */
hc_status hc_context_create(const hc_params* params, int device, hc_context** out);
void hc_context_destroy(hc_context* ctx);

/* Free the context's per-call device workspace (it grows again on the next
 * call that needs it). Synchronises the device. */
void hc_context_trim(hc_context* ctx);

/* Copy the derived primes: q_1..q_L then p_1..p_K (host array of L + K). */
hc_status hc_context_primes(const hc_context* ctx, uint64_t* primes_out);

/* ------------------------------------------------------------------ keys (Sec. 2.2, KeyGen) */

/* Secret key s (ternary) and public key (b, a) = ([-a s + e]_Q, a).
 * seed: 32 host bytes. Runs on the device; synchronises before returning. */
hc_status hc_keygen(hc_context* ctx, const uint8_t seed[32], hc_sk** sk, hc_pk** pk);
void hc_sk_destroy(hc_sk* sk);
void hc_pk_destroy(hc_pk* pk);

/* Galois (rotation) keys for the automorphisms X -> X^k, k odd in [1, 2n),
 * one per entry of `elements` (duplicates ignored). Digit j of the key for k:
 *   b_j = [-a_j s + e_j + P (Q/D_j) [(Q/D_j)^-1]_{D_j} sigma_k(s)]_{PQ},
 * a_j uniform over PQ, D_j the product of the primes of digit j.
 * Keys live in device memory (dnum * 2 * (L+K) * n * 8 bytes each).
 * Errors: HC_EINVAL (even or out-of-range element), HC_ENOMEM. Synchronises. */
hc_status hc_galois_keygen(hc_context* ctx, const hc_sk* sk, const uint32_t* elements,
                           uint32_t count, const uint8_t seed[32], hc_gk** gk);
void hc_gk_destroy(hc_gk* gk);

/* The Galois elements a compression of N records, ncol value columns and
 * sparsity bound t_bound needs (the schedule's key set, ascending), and the
 * plan's counts. comp_level and out_level as in hc_compress.
 * *count is the capacity of elements_out on entry and the number written on
 * exit. Errors: HC_EINVAL (the bands do not fit in n/2 slots, s > n/2, N = 0,
 * bad comp_level, capacity too small -- *count then holds the size needed). */
hc_status hc_plan(hc_context* ctx, uint64_t N, uint32_t ncol, uint32_t t_bound, uint32_t comp_level,
                  uint32_t out_level, uint32_t* elements_out, uint32_t* count, hc_compress_info* info);

/* ------------------------------------------------------------------ database */

/* Upload ncol value columns of N records (host, column c at cols + c*N,
 * values < p) and encode them once as plaintext multipliers (the Mask
 * operands of Alg. 7 step 2), resident in device memory. Synchronises. */
hc_status hc_db_upload(hc_context* ctx, const uint32_t* cols, uint32_t ncol, uint64_t N, hc_db** db);
void hc_db_destroy(hc_db* db);

/* ------------------------------------------------------------------ encryption (Sec. 2.2, Enc) */

/* Enc_pk of a slot matrix (host, 2 x n/2 row-major, values < p):
 * ([b u + e0 + Delta m]_Q, [a u + e1]_Q), u ternary, e0, e1 Gaussian (sigma 3.2).
 * ct_out: device [2][L][n]. Synchronises before returning. */
hc_status hc_encrypt(hc_context* ctx, const hc_pk* pk, const uint32_t* slots,
                     const uint8_t seed[32], uint64_t* ct_out, hipStream_t stream);

/* ------------------------------------------------------------------ compression (Alg. 7 steps 2-3; Sec. 5.2) */

/* Answer of a PDQ query: Mask every value column with the index vector and
 * compress [v, d_1, .., d_ncol] with the Vandermonde matrix C[j,i] = i^j mod p
 * (Eq. (1)) into one ciphertext. Mask runs at the input's full modulus; then
 * the ciphertexts are modulus-switched to the first comp_level primes (the
 * BFV form of the paper's switch to smaller parameters before Comp, Sec. 5.3)
 * and the rest of the map runs there with the same Galois keys restricted to
 * those primes. comp_level: 0 = the smallest multiple of K that is >= 2
 * (at most L); L = no switching; otherwise a multiple of K up to L.
 * out_level: 0 = the answer stays at the Comp level; 1..Comp level = the merged
 * answer is modulus-switched once more to its first out_level primes before it
 * is written (the answer the paper sends is one ciphertext modulo one prime,
 * Sec. 6.2; out_level = 1 gives that form). The output decrypts to the same slots.
 *   ct_v: device, n_ct = ceil(N/n) ciphertexts [n_ct][2][L][n] of the index
 *         vector; record r sits in ciphertext r / n, row (r % n) / (n/2),
 *         column r % (n/2).
 *   N, t_bound: records and an upper bound on the matches; s = 2^ceil(log2 t_bound).
 *   db: columns uploaded with hc_db_upload for the same N (ncol may be 0).
 *   ct_out: device, room for [2][L][n]; receives [2][level][n] (info->level).
 *         Band g*streams + sigma, slots [b s, b s + s) of
 *         row 0 / row 1, decrypts to (C a)_j / (C b)_j for group g and stream
 *         sigma = (a, b). With a single band the slots beyond s are not masked.
 *   info: optional, filled on success.
 * The work is enqueued on `stream`; the call returns without waiting.
 * Errors: HC_EINVAL (shapes, bands do not fit), HC_ENOKEY (gk lacks a needed
 * element), HC_ENOMEM (workspace), HC_EDEVICE. */
hc_status hc_compress(hc_context* ctx, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v,
                      uint64_t N, uint32_t t_bound, uint32_t comp_level, uint32_t out_level,
                      uint64_t* ct_out, hc_compress_info* info, hipStream_t stream);

/* The unencrypted-database form (Sec. 5.2, remark on an unencrypted database): the
 * server knows DB in the clear, so C (DB * v) = (C diag(DB)) v and the answer is
 * [C; C diag(DB_1); ...; C diag(DB_ncol)] v computed directly on the index-vector
 * ciphertexts -- no Mask and no per-stream packing. The inputs are switched to the
 * Comp level first; each input ciphertext and its row swap Rot_col serve as the
 * u-blocks of every stream, and the diagonals carry, row by row, the entries of the
 * matrix for the record block that row holds (times the records' values, read from
 * the database db keeps since hc_db_upload; records past its end count as 0). The
 * answer has hc_compress's layout and decrypts to the same slots (its bits differ).
 * Arguments as hc_compress; the key set is hc_plan_plain_db's (hc_plan's plus
 * Rot_col's element 2n - 1 in every case). */
hc_status hc_compress_plain_db(hc_context* ctx, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v,
                               uint64_t N, uint32_t t_bound, uint32_t comp_level, uint32_t out_level,
                               uint64_t* ct_out, hc_compress_info* info, hipStream_t stream);

/* hc_plan for hc_compress_plain_db (its key set and counts). */
hc_status hc_plan_plain_db(hc_context* ctx, uint64_t N, uint32_t ncol, uint32_t t_bound, uint32_t comp_level,
                           uint32_t out_level, uint32_t* elements_out, uint32_t* count, hc_compress_info* info);

/* One entry of a batch for hc_compress_batch. */
typedef struct {
    const uint64_t* ct_v;   /* device, ceil(N/n) ciphertexts */
    uint64_t N;
    uint32_t t_bound;
    uint32_t comp_level;    /* as in hc_compress */
    uint32_t out_level;     /* as in hc_compress */
    uint64_t* ct_out;       /* device, room for [2][L][n] */
    hc_compress_info* info; /* optional */
    hc_status status;       /* per-query result */
} hc_query;

/* Many independent compressions in one call. Each result is bit-identical
 * to hc_compress of the same query; all queries share db and gk. Rotations
 * by the same Galois element across queries are key-switched in one pass so
 * each key byte read from device memory serves every query in the pass.
 * Returns HC_OK if every query succeeded, else the first failing status (and
 * each query's own status in q[i].status). */
hc_status hc_compress_batch(hc_context* ctx, const hc_gk* gk, const hc_db* db,
                            hc_query* q, uint32_t nq, hipStream_t stream);

/* ------------------------------------------------------------------ ciphertext products (Alg. 5, Alg. 7 step 1) */

/* Relinearisation key: the key-switching key from s^2 to s, built like a Galois key
 * with s^2 in place of sigma_k(s) (digit j: b_j = [-a_j s + e_j + P (Q/D_j)
 * [(Q/D_j)^-1]_{D_j} s^2]_{PQ}, a_j uniform; stream tags "rk_a" / "rk_e", object
 * = digit). Returned as a key set holding one key, under element 1; free it with
 * hc_gk_destroy. Synchronises. */
hc_status hc_relin_keygen(hc_context* ctx, const hc_sk* sk, const uint8_t seed[32], hc_gk** rk);

/* Product of two ciphertexts at the full level L (device [2][L][n] each, coefficient
 * domain; ct_out may alias an input): the exact rounding round(p/Q e) mod Q of the
 * integer tensor e = (a0 b0, a0 b1 + a1 b0, a1 b1) of the centred lifts, computed
 * exactly in RNS over Q and an auxiliary basis of L + 1 primes, then relinearised
 * with rk (the key switch of the s^2 component, added in). Decrypts to the
 * slot-wise product while the noise stays inside the budget (BFV multiplication
 * grows it by about log2(2 p n) bits plus the inputs' noise). Synchronises.
 * Errors: HC_ENOKEY (rk is not a relinearisation key), HC_EINVAL, HC_ENOMEM. */
hc_status hc_mul(hc_context* ctx, const hc_gk* rk, const uint64_t* ct_a, const uint64_t* ct_b, uint64_t* ct_out,
                 hipStream_t stream);

/* ct_in^exponent slot-wise (exponent >= 1) by left-to-right binary exponentiation of
 * hc_mul products (after the leading bit: square, then multiply by the input for every
 * set bit). With exponent p - 1 this is the paper's Power_{p-1}: 1 in every nonzero slot,
 * 0 elsewhere (Fermat). Synchronises. Errors: as hc_mul. */
hc_status hc_power(hc_context* ctx, const hc_gk* rk, const uint64_t* ct_in, uint32_t exponent, uint64_t* ct_out,
                   hipStream_t stream);

/* Match (Alg. 7 step 1) for the exact-match predicate P(x, (k_i, v_i)) = [k_i = x] of
 * the paper's key-value example: from ct_x, a ciphertext of the query key x in every
 * slot ([2][L][n]), and the record keys (column 0 of `keys`, uploaded with
 * hc_db_upload), the index-vector ciphertexts ct_v [ceil(N/n)][2][L][n] with
 * v_r = 1 - (x - k_r)^(p-1): the query minus the keys' plaintext, Power_{p-1}, one minus
 * the result; in the last ciphertext the slots past record N are multiplied by 0.
 * Their output feeds hc_compress as ct_v. The powers of up to 16 ciphertexts run in
 * lockstep, each product step one pass over all of them (workspace: about 0.4 GB per
 * ciphertext at 24 primes and ring 2^16). Synchronises. Errors: as hc_mul. */
hc_status hc_match(hc_context* ctx, const hc_gk* rk, const hc_db* keys, const uint64_t* ct_x, uint64_t N,
                   uint64_t* ct_v, hipStream_t stream);

/* Comp of Alg. 5 on ciphertexts of a sparse vector d alone (no index vector given):
 * v = Power_{p-1}(d) at the full level (the ciphertexts in lockstep, as hc_match), then
 * the compression of the pair (v, d) exactly as hc_compress with one value column whose masked
 * ciphertexts are d's own. ct_d: device [ceil(N/n)][2][L][n]. Other arguments as
 * hc_compress (gk: hc_plan's key set for ncol = 1). Synchronises. */
hc_status hc_compress_generic(hc_context* ctx, const hc_gk* gk, const hc_gk* rk, const uint64_t* ct_d, uint64_t N,
                              uint32_t t_bound, uint32_t comp_level, uint32_t out_level, uint64_t* ct_out,
                              hc_compress_info* info, hipStream_t stream);

/* ------------------------------------------------------------------ captured compressions */

typedef struct hc_graph hc_graph;

/* Record the whole device work of hc_compress_batch(ctx, gk, db, q, nq) -- every
 * phase of Mask and Comp for every query -- into one HIP graph, without running it.
 * The schedule of a batch depends only on its queries' shapes (N, t_bound, levels),
 * so the host-side planning is done once here: the graph owns its workspace and its
 * tables, and reads each q[i].ct_v and writes each q[i].ct_out, whose addresses
 * are fixed at creation. Each hc_graph_launch then recomputes the answers of
 * whatever ciphertexts those buffers hold at that moment, bit-identical to
 * hc_compress_batch on them. q[i].info and q[i].status are filled here. gk, db and
 * resident diagonal tables (hc_diag_prepare) must stay unchanged while the graph
 * exists. All queries must share one Comp level. Synchronises the device.
 * Errors: as hc_compress_batch; HC_ENOMEM (the graph's workspace), HC_EDEVICE. */
hc_status hc_graph_create(hc_context* ctx, const hc_gk* gk, const hc_db* db, hc_query* q, uint32_t nq,
                          hc_graph** out);

/* Enqueue one replay of the graph on `stream` and return. Launches of one graph use
 * one workspace: order them (one stream, or synchronise in between). */
hc_status hc_graph_launch(hc_graph* g, hipStream_t stream);

/* Number of nodes (kernels and device copies) the graph holds. */
hc_status hc_graph_nodes(const hc_graph* g, uint64_t* nodes);

/* Wait for the device, then free the graph and its workspace. */
void hc_graph_destroy(hc_graph* g);

/* ------------------------------------------------------------------ kernel autotuning */

/* Bit-neutral kernel variants (every variant computes the same words):
 *   multiply-accumulate: 0 = 4 terms per LDS stage x 4 stages in flight (default),
 *                        1 = 2 x 8, 2 = 8 x 2;
 *   64-bit NTT passes of rings above 2^12: 0 = register budget of 4 waves per SIMD
 *                        (default), 1 = 3 waves, 2 = 5 waves, 3 = a persistent grid over
 *                        the pass's (tile, polynomial, prime) work queue.
 * The compression's schedule itself (rotations, key switches, B) is never tuned. */
#define HC_TUNE_MAC_VARIANTS 3
#define HC_TUNE_NTT_VARIANTS 4
typedef struct {
    uint32_t mac_variant, ntt_variant;     /* chosen, now set in the context */
    double mac_ms[HC_TUNE_MAC_VARIANTS];   /* multiply-accumulate device ms per compression */
    double ntt_ms[HC_TUNE_NTT_VARIANTS];   /* forward + inverse NTT device ms per compression */
} hc_tune_report;

/* Time every variant of each tuned kernel on the caller's own compression
 * (hc_compress of ct_v with N, t_bound, comp_level into ct_out, run a few times
 * per variant with kernel timing on, which clears earlier hc_timing totals), keep
 * the fastest in the context and report the times. Synchronises. Errors: as
 * hc_compress. */
hc_status hc_autotune(hc_context* ctx, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v, uint64_t N,
                      uint32_t t_bound, uint32_t comp_level, uint64_t* ct_out, hc_tune_report* report,
                      hipStream_t stream);

/* Set or read the context's variants (HC_EINVAL for an unknown variant). */
hc_status hc_tune_set(hc_context* ctx, uint32_t mac_variant, uint32_t ntt_variant);
hc_status hc_tune_get(const hc_context* ctx, uint32_t* mac_variant, uint32_t* ntt_variant);

/* ------------------------------------------------------------------ resident diagonals (Sec. 5.2) */

/* Server-side precomputation for the diagonal method of Sec. 5.2. The BSGS
 * diagonals of C that a compression multiplies by depend only on the record
 * groups (through N), on s and on the Comp level: never on the query or on the
 * database. Encode every diagonal that compressions with (N, ncol, t_bound,
 * comp_level) use and keep them resident on the device, one table per
 * (s, B, level) class, NTT domain, k = the most u-blocks of a group, in one of two
 * layouts (see hc_diag_layout): the seven balanced base-256 digits of each centred
 * residue, tiled for the int8 matrix-core multiply-accumulate (7 bytes per residue),
 * or split words in Montgomery form for the vector one (8 bytes). Later hc_compress and
 * hc_compress_batch calls read a class from its table when it holds enough
 * u-blocks, instead of encoding its diagonals on the fly; the results are
 * bit-identical either way. A class already resident with at least k u-blocks
 * is kept; one with fewer is rebuilt. The tables stay until hc_diag_release or
 * hc_context_destroy. bytes_out (optional): device bytes then held by all
 * tables. Synchronises the device.
 * Errors: as hc_plan; HC_ENOMEM when a table does not fit in device memory
 * (tables built before that one in the same call are kept). */
hc_status hc_diag_prepare(hc_context* ctx, uint64_t N, uint32_t ncol, uint32_t t_bound,
                          uint32_t comp_level, uint64_t* bytes_out);

/* Free every resident diagonal table of ctx; later compressions encode their
 * diagonals on the fly. Synchronises the device. */
void hc_diag_release(hc_context* ctx);

/* Layout of the tables later hc_diag_prepare calls build (tables already resident
 * keep theirs; release them to rebuild). HC_DIAG_LAYOUT_AUTO (the default): the
 * matrix-core digit layout for every class it fits -- all Comp-level primes below
 * 2^55, k B <= 128 terms, padding to 16 giants x 64 terms at most doubling the
 * bytes -- else split words. HC_DIAG_LAYOUT_SPLIT: split words for every class.
 * Either way the compressions' results are the same words.
 * Errors: HC_EINVAL (unknown layout). */
enum { HC_DIAG_LAYOUT_AUTO = 0, HC_DIAG_LAYOUT_SPLIT = 1 };
hc_status hc_diag_layout(hc_context* ctx, int layout);

/* ------------------------------------------------------------------ serving loop (Sec. 3, Answer) */

typedef struct hc_server hc_server;

/* A request loop over one context, key set and database, all resident on the
 * device: PDQ queries are submitted as they arrive and answered by continuous
 * batching. A host thread admits waiting requests, oldest first, into a batch
 * while the batch's device workspace fits one lane and the batch holds at most
 * max_batch queries, and runs it (the batched phases of hc_compress_batch) on
 * that lane's own stream. With lanes > 1 a new batch starts while earlier ones
 * are still running, so requests arriving meanwhile share the device with them
 * rather than waiting for them to finish. Every result is bit-identical to
 * hc_compress of the same query.
 *   comp_level, out_level: as in hc_compress, for every request.
 *   lane_bytes: device workspace per lane, allocated at creation.
 *   lanes: 1..4 concurrent batches; max_batch >= 1.
 * ctx, gk and db must outlive the server. Resident diagonal tables
 * (hc_diag_prepare) must not be prepared or released while it runs.
 * Errors: HC_EINVAL, HC_ENOMEM (lanes do not fit), HC_EDEVICE. */
hc_status hc_server_create(hc_context* ctx, const hc_gk* gk, const hc_db* db, uint32_t comp_level,
                           uint32_t out_level, uint64_t lane_bytes, uint32_t lanes, uint32_t max_batch,
                           hc_server** out);

/* Queue one query; returns at once. ct_v and ct_out are device buffers as for
 * hc_compress and must stay valid and unchanged until the request completes.
 * `stream` is the stream the caller produced ct_v on: submit records an event
 * there, and the batch that takes the request waits for it before reading
 * ct_v (so ct_v may still be in flight on that stream at submission).
 * id_out (optional): the request id, increasing from 1. Errors: as hc_plan,
 * HC_ENOKEY, HC_EDEVICE, and HC_ENOMEM when the query alone does not fit one lane. */
hc_status hc_server_submit(hc_server* srv, const uint64_t* ct_v, uint64_t N, uint32_t t_bound,
                           uint64_t* ct_out, hipStream_t stream, uint64_t* id_out);

/* One completed request. Times are CLOCK_MONOTONIC nanoseconds. */
typedef struct {
    uint64_t id;
    hc_status status;
    int64_t submit_ns;        /* hc_server_submit accepted it */
    int64_t start_ns;         /* its batch was enqueued on the device */
    int64_t done_ns;          /* the host saw its batch finish; ct_out is then final */
    uint32_t batch_size;      /* queries in its batch */
    hc_compress_info info;
} hc_server_result;

/* Move up to cap completed requests (in completion order) to out, waiting up to
 * timeout_ms for the first if none is ready; *count may then be 0. */
hc_status hc_server_poll(hc_server* srv, hc_server_result* out, uint32_t cap, uint32_t* count,
                         double timeout_ms);

typedef struct {
    uint64_t submitted, completed, batches;
    uint32_t max_batch_seen;  /* most queries in one batch */
    uint32_t max_lanes_busy;  /* most batches on the device at once */
} hc_server_stats;
hc_status hc_server_stats_get(hc_server* srv, hc_server_stats* out);

/* Finish every queued and running request, stop the loop and free the lanes.
 * Results not yet polled are dropped. */
void hc_server_destroy(hc_server* srv);

/* ------------------------------------------------------------------ client side (host CPU) */

/* Dec: slots of round(p [c0 + c1 s]_Q / Q) mod p, Q the product of the first
 * `level` ciphertext primes (1 <= level <= L). ct: host [2][level][n],
 * coefficient domain. slots_out: host 2 x n/2. Runs on the host.
 * Errors: HC_EINVAL (non-canonical residue, bad level), HC_ENOISE (rounding
 * within 2^-50 of a tie: the noise has reached the budget). */
hc_status hc_decrypt(hc_context* ctx, const hc_sk* sk, const uint64_t* ct, uint32_t level,
                     uint32_t* slots_out);

/* Decomp for one group (Alg. 6 with Alg. 1 and Alg. 4): from w = C v
 * (s values) and e_c = C d_c (ncols x s values, host) recover the matched
 * indices (1-based within the group, ascending) and their values.
 * idx_out: capacity s; val_out: capacity ncols * s, column c at val_out + c*s.
 * Roots are found by Cantor-Zassenhaus. Runs on the host.
 * Errors: HC_EINVAL (p not prime, N_group >= p, s > p-1), HC_EDECODE (root
 * count differs from the degree, a root outside [1, N_group], or the
 * equations beyond the first `count` are violated). */
hc_status hc_decompress(uint64_t p, uint64_t N_group, uint32_t s, uint32_t ncols,
                        const uint32_t* w, const uint32_t* e, uint64_t* idx_out,
                        uint32_t* val_out, uint32_t* count_out);

/* Text of a status code (static string). */
const char* hc_status_str(hc_status st);

#ifdef __cplusplus
}
#endif
#endif /* HC_H */
