// Declarations shared by the host orchestration files (he.cpp, compress.cpp).
#pragma once
#include <initializer_list>

#include "hc_internal.h"

namespace hc {

// key-switching scratch for passes of up to maxM jobs (and maxU raised sources)
struct KsScratch {
    uint64_t* tmpC = nullptr;  // [maxU][Lc][n]
    uint64_t* X = nullptr;     // [maxU][dn][Lc+K][n]
    uint64_t* T = nullptr;     // [maxM][2][Lc+K][n]
    uint64_t* conv = nullptr;  // [maxM][2][Lc][n]
    int maxU = 0, maxM = 0;
};

uint64_t tag_u64(const char* s);
hc_status encode_plain(Ctx& c, uint64_t* out, const uint32_t* host_slots, int count, bool mont,
                       hipStream_t st);
hc_status prefix_mask(Ctx& c, uint32_t s, const uint64_t** out);
// per-call staging of small tables (pinned host -> device, in stream order)
void stage_reset(Lane& l, hipStream_t st);
void* stage_bytes(Lane& l, const void* data, size_t bytes, hipStream_t st);
// Several host arrays staged with one copy: each part's device address goes to *dev.
struct StagePart {
    const void* data;
    size_t bytes;
    void** dev;
};
bool stage_many(Lane& l, std::initializer_list<StagePart> parts, hipStream_t st);
// batched key switching at level Lc (see ks_run in he.cpp)
size_t ks_scratch_bytes(const Ctx& c, int Lc, int max_jobs);
KsScratch ks_scratch(Ctx& c, Arena& a, int Lc, int max_jobs);
hc_status ks_run(Ctx& c, Lane& l, KsScratch& s, const std::vector<KsJob>& jobs,
                 const std::vector<const uint64_t*>* srcs, int Lc, hipStream_t st);
// sums of rotations with one ModDown per sum (see ks_run_sum in he.cpp)
hc_status ks_run_sum(Ctx& c, Lane& l, KsScratch& s, const std::vector<KsJob>& jobs,
                     const std::vector<uint32_t>& group, const std::vector<uint64_t*>& outs, uint64_t* TA,
                     uint64_t* C0A, int Lc, hipStream_t st);
hc_status ew_run(Ctx& c, Lane& l, const std::vector<EwJob>& jobs, int Lc, bool mul, hipStream_t st);
// drop the primes Lc..L-1 of `count` contiguous top-level ciphertexts (NTT domain). The
// first ncoef of them may also be given in coefficient form (coef, same layout): their
// dropped rows are then read from there instead of being transformed back. low_done (ring
// 2^16): the dropped rows of the other count - ncoef already hold the inverse transform's
// first pass (ntt_mask_low).
hc_status mod_switch_batch(Ctx& c, uint64_t* out, uint64_t* in, int count, int Lc, uint64_t* conv,
                           hipStream_t st, const uint64_t* coef = nullptr, int ncoef = 0, bool low_done = false);
// dropping primes from coefficient-domain ciphertexts at level Lin down to Lo
// (count contiguous ciphertexts; conv: 2 Lo n words each)
hc_status mod_switch_coef(const Ctx& c, uint64_t* out, const uint64_t* in, int count, int Lin, int Lo,
                          uint64_t* conv, hipStream_t st);
// the switching constants of every level pair (context creation)
hc_status build_ms_tables(Ctx& c);
const uint64_t* find_key(const hc_gk* gk, uint32_t k);
// key-switching keys from sigma_k(s) for each element, or (relin) from s^2 under element 1
hc_status ks_keygen(Ctx& c, const hc_sk* sk, const uint32_t* elements, uint32_t count, const uint8_t seed[32],
                    bool relin, hc_gk** out);
// Power_e of n_ct ciphertexts at the full level (coefficient domain; out may alias in)
hc_status power_many(Ctx& c, const hc_gk* rk, const uint64_t* in, uint32_t n_ct, uint32_t e, uint64_t* out,
                     hipStream_t st);

}  // namespace hc
