// Declarations shared by the host orchestration files (he.cpp, compress.cpp).
#pragma once
#include "hc_internal.h"

namespace hc {

// key-switching temporaries: tmpC [L][n], X [dnum][nq][n], T [2][nq][n], conv [2][L][n]
struct KSBuf {
    uint64_t* tmpC = nullptr;
    uint64_t* X = nullptr;
    uint64_t* T = nullptr;
    uint64_t* conv = nullptr;
};

uint64_t tag_u64(const char* s);
hc_status encode_plain(Ctx& c, uint64_t* out, const uint32_t* host_slots, int count, bool mont,
                       hipStream_t st);
hc_status prefix_mask(Ctx& c, uint32_t s, const uint64_t** out);
size_t ks_take_bytes(const Ctx& c);
KSBuf ks_take(Ctx& c, Arena& a);
// Key switching at level Lc (ciphertexts [2][Lc][n], NTT domain): rows 0..Lc-1 and
// the special primes, digits inside the first Lc primes. Top-level keys serve every level.
void rotate_plain(Ctx& c, const uint64_t* key, uint32_t k, uint64_t* out, const uint64_t* in,
                  KSBuf& b, int Lc, hipStream_t st);
void hoist_prepare(Ctx& c, const uint64_t* in, KSBuf& b, int Lc, hipStream_t st);
void rotate_hoisted_one(Ctx& c, const uint64_t* key, uint32_t k, uint64_t* out, const uint64_t* in,
                        KSBuf& b, int Lc, hipStream_t st);
// Drop the primes Lc..L-1 of a top-level ciphertext (NTT domain); tmp 2 L n, conv 2 Lc n words.
hc_status mod_switch(Ctx& c, uint64_t* out, const uint64_t* in, int Lc, uint64_t* tmp, uint64_t* conv,
                     hipStream_t st);
const uint64_t* find_key(const hc_gk* gk, uint32_t k);

}  // namespace hc
