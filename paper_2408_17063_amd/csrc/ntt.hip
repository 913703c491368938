// Negacyclic NTT / inverse NTT per prime, batched over polynomials and primes.
//
// Forward transform (merged psi-twist, Cooley-Tukey, natural order in,
// bit-reversed order out): stage st = 0..logn-1 pairs index j with
// j + n/2^(st+1) and multiplies by W[2^st + (j >> (logn - st))],
// W[k] = psi^brv(k). Output entry i = a(psi^(2 brv(i) + 1)).
// Inverse (Gentleman-Sande): stage u = 0..logn-1 pairs j with j + 2^u,
// twiddle Winv[n/2^(u+1) + (j >> (u+1))], Winv[k] = psi^-brv(k), then a
// final multiplication by n^-1 (folded into the last stage, whose one twiddle is
// Winv[1]).
//
// A launch runs S consecutive stages on tiles of 4096 elements (the whole
// ring below 2^12) held in LDS. The stages touch the index bits [BLO, BLO+S);
// a tile is P = 4096 / 2^S independent sub-problems (consecutive values of
// the other bits, so global accesses are contiguous runs) times the 2^S
// elements of each. 256 threads each own 16 elements per round and run up to
// 4 stages in registers between LDS exchanges. Every parameter is a template
// constant, so rounds are fully unrolled. Within a round the twiddles of stage
// u are the 2^u (forward) or 2^(R-1-u) (inverse) consecutive table entries the
// thread's group needs, each one 16-byte load of (w, w') from the interleaved
// table (from a thread-ordered copy in the low-bit pass of a two-pass ring). Rings
// up to 2^12 take one launch per transform; larger rings take two (high bits then
// the low 8 bits forward, the reverse order inverse). The 8-stage high-bit pass
// keeps its first and last rounds' groups in registers between global memory and
// the rounds (see Tile::DIRECT).
//
// The 64-bit butterflies keep the carry flag out of their arithmetic: the product's
// reduction adds qt*(2^64 - q) instead of subtracting qt*q, and the conditional
// subtractions pick their result by the sign bit of x - r (csub_neg), so chains of
// dependent carry and compare results, which stall the SIMD between instructions,
// are rare.
//
// Butterflies are lazy (Harvey). With 32-bit primes the twiddle products are exact
// Shoup products in [0, 2q): forward values stay in [0, 4q), inverse values in
// [0, 2q). With 64-bit primes (q < 2^61) the quotient of a twiddle product is
// taken from the three partial products that reach the high word of x*w' and
// drops their carries, which saves half the multiplies of the exact high word and
// leaves the product in [0, 4q): forward values then stay in [0, 8q), inverse values
// in [0, 4q). For primes below 2^57 (a block checks its row's prime) the forward
// transform makes no conditional subtractions at all: a stage adds at most 4q to
// the bound, so 16 stages from below 8q stay below 72q < 2^64, and the last launch
// reduces with one truncated product by 1. The last launch brings every value to
// [0, q).
#include <algorithm>

#include "hc_internal.h"

namespace hc {

// x - r if x >= r else x, for 64-bit x < 2^63 + r and r < 2^63, given nr = 2^64 - r:
// the sign of x - r picks the result through a bit mask, which keeps the carry flag
// and compare results out of it.
__device__ __forceinline__ uint64_t csub_neg(uint64_t x, uint64_t nr) {
    const uint64_t t = x + nr;
    uint32_t m = (uint32_t)((int32_t)(uint32_t)(t >> 32) >> 31);
    asm("" : "+v"(m));
    const uint64_t mm = ((uint64_t)m << 32) | m;
    return (x & mm) | (t & ~mm);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           __builtin_amdgcn_readfirstlane((uint32_t)v);
}

template <typename T> struct Ar;

template <> struct Ar<uint64_t> {
    static constexpr int LAZY = 2;  // butterfly values are reduced below 4q (forward: 8q)
    // x*w - qt*q with qt = xh*wh' + hi(xh*wl') + hi(xl*wh') for w' = wh'*2^32 + wl':
    // x*w'/2^64 exceeds qt by the dropped low words, less than 3, so qt is at most 2
    // below the exact Shoup quotient and the result lies in [0, 4q) for any 64-bit
    // x. nq = 2^64 - q.
    static __device__ __forceinline__ uint64_t mul(uint64_t x, uint64_t w, uint64_t wp, uint64_t q, uint64_t nq) {
        (void)q;
        const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
        const uint32_t wl = (uint32_t)wp, wh = (uint32_t)(wp >> 32);
        const uint64_t qt = (uint64_t)xh * wh + __umulhi(xh, wl) + __umulhi(xl, wh);
        return x * w + qt * nq;
    }
    static __device__ __forceinline__ uint64_t red(uint64_t x, uint64_t r, uint64_t nr) {
        (void)r;
        return csub_neg(x, nr);
    }
    static __device__ __forceinline__ void load_pair(const uint64_t* p, uint64_t& w, uint64_t& wp) {
        ulonglong2 v = *reinterpret_cast<const ulonglong2*>(p);
        w = v.x;
        wp = v.y;
    }
};

template <> struct Ar<uint32_t> {
    static constexpr int LAZY = 1;  // butterfly values are reduced below 2q (forward: 4q)
    static __device__ __forceinline__ uint32_t shoup_lazy(uint32_t x, uint32_t w, uint32_t wp, uint32_t q) {
        return x * w - __umulhi(x, wp) * q;
    }
    static __device__ __forceinline__ uint32_t mul(uint32_t x, uint32_t w, uint32_t wp, uint32_t q, uint32_t) {
        return shoup_lazy(x, w, wp, q);
    }
    static __device__ __forceinline__ uint32_t red(uint32_t x, uint32_t r, uint32_t) { return x >= r ? x - r : x; }
    static __device__ __forceinline__ void load_pair(const uint32_t* p, uint32_t& w, uint32_t& wp) {
        uint2 v = *reinterpret_cast<const uint2*>(p);
        w = v.x;
        wp = v.y;
    }
};


// Tables for one prime: [2 directions][n][2] = (w, w') pairs, forward then
// inverse; plus n^-1 and Winv[1] n^-1 with their Shoup constants.
template <typename T> struct NttTab {
    const T* base;  // [nprime][2][n][2]
    const T* ninv;  // [nprime][4]: n^-1 and its Shoup constant, W^-1[1] n^-1 and its Shoup constant
    const T* mods;  // [nprime]
    const T* tw2;   // low-bit pass twiddles in thread order (rings above one tile), or nullptr
};

constexpr int TILE_LOG = 12;
constexpr int NTT_EPT_LOG = 4;                          // elements per thread: 2^NTT_EPT_LOG
constexpr int NTT_EPT = 1 << NTT_EPT_LOG;
constexpr int NTT_THREADS = (1 << TILE_LOG) / NTT_EPT;  // block size for full tiles

__device__ __forceinline__ uint32_t insert_bits(uint32_t g, uint32_t v, int pos, int width) {
    uint32_t lowmask = (1u << pos) - 1u;
    return ((g >> pos) << (pos + width)) | (v << pos) | (g & lowmask);
}

template <typename T, bool INV, int LOGN, int S, int BLO, int ST0>
struct Tile {
    static constexpr int TLOG = LOGN < TILE_LOG ? LOGN : TILE_LOG;
    static constexpr int TSIZE = 1 << TLOG;
    static constexpr int LOGP = TLOG - S;
    static constexpr int P = 1 << LOGP;
    static constexpr int N = 1 << LOGN;
    static constexpr int THREADS = TSIZE / NTT_EPT;
    // The pass over the low index bits of a two-pass ring has one round whose
    // twiddles differ from thread to thread (up to one per butterfly in the last
    // forward stages, the first inverse ones). They come from a copy of the table
    // laid out in the order the threads consume them, [tile][ord][thread], so each
    // load instruction reads one contiguous run. In its other round a thread's
    // twiddles depend on its sub-problem only: 16 consecutive table entries serve a
    // block, and they are read from the table itself.
    static constexpr bool TW2 = sizeof(T) == 8 && BLO == 0 && LOGN > TILE_LOG;
    static constexpr int round_r(int done) { return (S - done) >= NTT_EPT_LOG ? NTT_EPT_LOG : (S - done); }
    static constexpr bool tw2_round(int done) { return TW2 && (INV ? done == 0 : done != 0); }
    static constexpr int round_tw(int r) { return (NTT_EPT >> r) * ((1 << r) - 1); }
    static constexpr int tw_before(int done) {
        int o = 0;
        for (int d = 0; d < done; d += round_r(d))
            if (tw2_round(d)) o += round_tw(round_r(d));
        return o;
    }
    static constexpr int TW_PASS = tw_before(S);  // twiddle pairs per thread over the pass
    // The 8-stage pass over the high index bits of a two-pass ring is two rounds of
    // one group per thread whose elements are 128-byte runs in global memory (16
    // consecutive sub-problems) in both rounds' layouts: a thread loads its first
    // round's group straight from global memory and stores its second round's group
    // straight back, so the tile passes through LDS once.
    static constexpr bool DIRECT = BLO != 0 && LOGN > TILE_LOG && S == 2 * NTT_EPT_LOG;  // (no LDS padding)
    // In the 8-stage low-bit pass the round over k's high 4 bits (the forward pass's
    // first, the inverse pass's second) has groups of stride 16 within a sub-problem:
    // with the group index's nibbles swapped (lanes take consecutive k low bits) its
    // elements are 128-byte runs, so the forward pass loads that round's groups
    // straight from global memory and the inverse pass stores them straight back.
    static constexpr bool DIRECT_LO = BLO == 0 && LOGN > TILE_LOG && S == 2 * NTT_EPT_LOG && THREADS == 256;
    static __device__ __forceinline__ uint32_t swap_nibbles(uint32_t t) { return ((t & 15u) << 4) | (t >> 4); }
    // In the low-bit pass of a two-pass ring a thread's global-contiguous loads and
    // stores step through the tile at a stride of P words in LDS, which puts a
    // wavefront's lanes on the same banks. One pad word after every P words spreads
    // them; the rounds' accesses stay (nearly) contiguous.
    static constexpr bool PAD = BLO == 0 && LOGP > 0;
    static constexpr int LDS_WORDS = TSIZE + (PAD ? TSIZE / P : 0);
    static __device__ __forceinline__ uint32_t lpos(uint32_t e) { return PAD ? e + (e >> LOGP) : e; }
    // True if no index bit a thread's group supplies survives the twiddle-index shift
    // of any stage of the round (butterfly bits [kbit, kbit + r) of k, `done` stages
    // before it): the round's twiddles are then the same for the whole block.
    static constexpr bool round_uniform(int kbit, int r, int done) {
        int hi = -1;  // highest j0 bit a group supplies
        for (int b = 0; b < S; b++)
            if (b < kbit || b >= kbit + r) hi = hi > BLO + b ? hi : BLO + b;
        for (int c = 0; c < LOGP; c++) {
            const int pos = BLO == 0 ? S + c : c;
            hi = hi > pos ? hi : pos;
        }
        for (int u = 0; u < r; u++) {
            const int st = ST0 + done + u;
            const int shift = INV ? st + 1 : LOGN - st;
            if (hi >= shift) return false;
        }
        return true;
    }
    // position of twiddle t of stage u in a round of r stages, within a group's run
    static constexpr int tw_off(int r, int u) { return INV ? (1 << r) - (1 << (r - u)) : (1 << u) - 1; }

    // global index of tile element e = (k << LOGP) | spl, sub-problem base sp0
    static __device__ __forceinline__ uint32_t gidx(uint32_t e, uint32_t sp0) {
        uint32_t k = e >> LOGP;
        uint32_t sp = sp0 + (e & (P - 1));
        return ((sp >> BLO) << (BLO + S)) | (k << BLO) | (sp & ((1u << BLO) - 1u));
    }

    // The R stages of one round on one group held in registers: x[v] is tile element
    // insert_bits(g, v, LOGP + KBIT, R); butterfly bits [KBIT, KBIT+R) of k; DONE
    // stages before it; sub: the group's index among the thread's groups.
    // NR (forward, 64-bit primes below 2^57): no conditional subtraction; a forward
    // stage then adds at most 4q to the bound, and 16 stages from below 8q stay below
    // 72q < 2^64.
    // FOLD (the inverse transform's last launch): the last stage, whose one twiddle is
    // W^-1[1], also scales by n^-1: its sums are multiplied by n^-1 and its differences
    // by W^-1[1] n^-1 (ni: the prime's [4] entry of the n^-1 table).
    template <int R, int KBIT, int DONE, bool NR = false, bool FOLD = false>
    static __device__ __forceinline__ void butterflies(T (&x)[1 << R], uint32_t g, int sub, uint32_t sp0, const T* tw,
                                                       const T* tw2, T q, const T* ni = nullptr) {
        constexpr int POS = LOGP + KBIT;
        constexpr int GS = 1 << R;
        const uint32_t j0 = gidx(insert_bits(g, 0, POS, R), sp0);
        const T rq = q << Ar<T>::LAZY;
        T nq = (T)0 - q, nrq = (T)0 - rq;
        // opaque to the compiler, so x*w + qt*nq is not turned back into a
        // subtraction with its carry chain
        if constexpr (sizeof(T) == 8) {
            nq = uniform64(nq);
            nrq = uniform64(nrq);
            asm("" : "+s"(nq), "+s"(nrq));
        }
        // this round holds the transform's last stage (u = R - 1)
        constexpr bool FOLD_HERE = FOLD && INV && ST0 + DONE + R == LOGN;
        #pragma unroll
        for (int u = 0; u < (FOLD_HERE ? R - 1 : R); u++) {
            const int st = ST0 + DONE + u;
            // stage u's twiddles: 2^u (forward) or 2^(R-1-u) (inverse) pairs from base on
            const int cnt = INV ? (1 << (R - 1 - u)) : (1 << u);
            uint32_t base = INV ? ((uint32_t)N >> (st + 1)) + (j0 >> (st + 1)) : (1u << st) + (j0 >> (LOGN - st));
            if constexpr (round_uniform(KBIT, R, DONE)) base = __builtin_amdgcn_readfirstlane(base);
            T w[8], wp[8];
            #pragma unroll
            for (int t = 0; t < cnt; t++) {
                if constexpr (tw2_round(DONE))
                    Ar<T>::load_pair(tw2 + 2 * ((size_t)(tw_before(DONE) + sub * ((1 << R) - 1) + tw_off(R, u) + t) *
                                                    THREADS + threadIdx.x),
                                     w[t], wp[t]);
                else
                    Ar<T>::load_pair(tw + 2 * (base + t), w[t], wp[t]);
            }
            if (!INV) {
                // partner bit R-1-u of v; twiddle base + (v >> (R-u))
                const int half = 1 << (R - 1 - u);
                #pragma unroll
                for (int v = 0; v < GS; v++) {
                    if (!(v & half)) {
                        const int t = v >> (R - u);
                        T X = NR ? x[v] : Ar<T>::red(x[v], rq, nrq);
                        T y = Ar<T>::mul(x[v | half], w[t], wp[t], q, nq);
                        x[v] = X + y;
                        x[v | half] = X - y + rq;
                    }
                }
            } else {
                // partner bit u of v; twiddle base + (v >> (u+1))
                const int half = 1 << u;
                #pragma unroll
                for (int v = 0; v < GS; v++) {
                    if (!(v & half)) {
                        const int t = v >> (u + 1);
                        T X = x[v], Y = x[v | half];
                        x[v] = Ar<T>::red(X + Y, rq, nrq);
                        x[v | half] = Ar<T>::mul(X + rq - Y, w[t], wp[t], q, nq);
                    }
                }
            }
        }
        if constexpr (FOLD_HERE) {
            constexpr int half = 1 << (R - 1);
            const T n0 = ni[0], n1 = ni[1], m0 = ni[2], m1 = ni[3];
            #pragma unroll
            for (int v = 0; v < half; v++) {
                const T X = x[v], Y = x[v | half];
                x[v] = Ar<T>::mul(X + Y, n0, n1, q, nq);
                x[v | half] = Ar<T>::mul(X + rq - Y, m0, m1, q, nq);
            }
        }
    }

    // one round of R stages on the tile in LDS
    template <int R, int KBIT, int DONE, bool NR = false, bool FOLD = false>
    static __device__ __forceinline__ void round(T* lds, uint32_t sp0, const T* tw, const T* tw2, T q,
                                                 const T* ni = nullptr) {
        constexpr int POS = LOGP + KBIT;
        constexpr int GS = 1 << R;
        constexpr int PER = NTT_EPT >> R;  // groups per thread
        // element v of a group sits at lpos(insert_bits(g, 0, POS, R)) + v VSTEP: the
        // group's own bits are disjoint from the others (and POS >= LOGP when padded)
        static_assert(!PAD || POS >= LOGP, "pad step");
        constexpr uint32_t VSTEP = (1u << POS) + (PAD ? (1u << (POS - LOGP)) : 0u);
        #pragma unroll
        for (int sub = 0; sub < PER; sub++) {
            const uint32_t g = threadIdx.x * PER + sub;
            const uint32_t lb = lpos(insert_bits(g, 0, POS, R));
            T x[GS];
            #pragma unroll
            for (int v = 0; v < GS; v++) x[v] = lds[lb + v * VSTEP];
            butterflies<R, KBIT, DONE, NR, FOLD>(x, g, sub, sp0, tw, tw2, q, ni);
            #pragma unroll
            for (int v = 0; v < GS; v++) lds[lb + v * VSTEP] = x[v];
        }
    }

    // rounds: forward processes k bits from the top down, inverse from the bottom up
    template <int DONE, bool NR = false, bool FOLD = false>
    static __device__ __forceinline__ void rounds(T* lds, uint32_t sp0, const T* tw, const T* tw2, T q,
                                                  const T* ni = nullptr) {
        if constexpr (DONE < S) {
            constexpr int R = round_r(DONE);
            constexpr int KBIT = INV ? DONE : (S - DONE - R);
            round<R, KBIT, DONE, NR, FOLD>(lds, sp0, tw, tw2, q, ni);
            __syncthreads();
            rounds<DONE + R, NR, FOLD>(lds, sp0, tw, tw2, q, ni);
        }
    }

    // Writes this thread's twiddles of the pass, in consumption order, to
    // out[ord][THREADS] (pairs): the same indices round() computes.
    template <int DONE>
    static __device__ __forceinline__ void emit(T* out, uint32_t sp0, const T* tw) {
        if constexpr (DONE < S) {
            constexpr int R = round_r(DONE);
            constexpr int KBIT = INV ? DONE : (S - DONE - R);
            constexpr int POS = LOGP + KBIT;
            constexpr int PER = NTT_EPT >> R;
            for (int sub = 0; sub < (tw2_round(DONE) ? PER : 0); sub++) {
                const uint32_t g = threadIdx.x * PER + sub;
                const uint32_t j0 = gidx(insert_bits(g, 0, POS, R), sp0);
                for (int u = 0; u < R; u++) {
                    const int st = ST0 + DONE + u;
                    const uint32_t base = INV ? ((uint32_t)N >> (st + 1)) + (j0 >> (st + 1))
                                              : (1u << st) + (j0 >> (LOGN - st));
                    const int cnt = INV ? (1 << (R - 1 - u)) : (1 << u);
                    for (int t = 0; t < cnt; t++) {
                        const size_t o = 2 * ((size_t)(tw_before(DONE) + sub * ((1 << R) - 1) + tw_off(R, u) + t) *
                                                  THREADS + threadIdx.x);
                        out[o] = tw[2 * (base + t)];
                        out[o + 1] = tw[2 * (base + t) + 1];
                    }
                }
            }
            emit<DONE + R>(out, sp0, tw);
        }
    }
};

// One tile of one pass: tile bx of polynomial by, row (limb) bz; ntiles tiles per row.
// src (nullptr: in place): the pass reads its input there, at data's offsets, and
// writes data.
template <typename T, bool INV, int LOGN, int S, int BLO, int ST0, bool LAST>
__device__ __forceinline__ void ntt_tile(T* __restrict__ data, size_t poly_stride, int limb_first,
                                         const NttTab<T>& tab, T* lds, uint32_t bx, uint32_t by, uint32_t bz,
                                         uint32_t ntiles, const T* __restrict__ src = nullptr) {
    typedef Tile<T, INV, LOGN, S, BLO, ST0> TL;
    constexpr int THREADS = TL::THREADS;  // the launch's block size
    const uint32_t tid = threadIdx.x;
    const int row = (int)bz;  // limb; polynomials along y, so consecutive blocks of one
                              // XCD share a (prime, tile) and its twiddles stay in L2
    const int prime = limb_first + row;
    const T q = tab.mods[prime];
    const T* tw = tab.base + ((size_t)prime * 2 + (INV ? 1 : 0)) * 2 * TL::N;
    T* a = data + (size_t)by * poly_stride + (size_t)row * TL::N;
    const T* ain = src ? src + (a - data) : a;
    const uint32_t sp0 = bx * TL::P;
    const T* ni = tab.ninv + 4 * prime;
    constexpr bool FOLD = INV && LAST;
    // NR: forward transform of a 64-bit prime below 2^57 without conditional subtractions
    auto body = [&](auto nr_c) __attribute__((always_inline)) {
        constexpr bool NR = decltype(nr_c)::value;
        // the last launch: forward values below 8q (4q with 32-bit primes; 72q without
        // conditional subtractions), inverse values times n^-1, down to [0, q)
        auto finish = [&](T v) -> T {
            if constexpr (LAST) {
                T nq1 = (T)0 - q, nq2 = (T)0 - (q << 1), nq4 = (T)0 - (q << 2);
                if constexpr (sizeof(T) == 8) {
                    nq1 = uniform64(nq1);
                    nq2 = uniform64(nq2);
                    nq4 = uniform64(nq4);
                    asm("" : "+s"(nq1), "+s"(nq2), "+s"(nq4));
                }
                if constexpr (INV) {
                    // scaled by n^-1 in the last stage: [0, 4q) (64-bit), [0, 2q)
                } else if constexpr (NR) v = Ar<T>::mul(v, tw[0], tw[1], q, nq1);  // entry 0 is (1, 2^64 / q): [0, 4q)
                else if constexpr (Ar<T>::LAZY == 2) v = Ar<T>::red(v, q << 2, nq4);
                if constexpr (Ar<T>::LAZY == 2 || !INV) v = Ar<T>::red(v, q << 1, nq2);
                v = Ar<T>::red(v, q, nq1);
            }
            return v;
        };

        if constexpr (TL::DIRECT) {
            constexpr int R = NTT_EPT_LOG;
            constexpr int P1 = TL::LOGP + (INV ? 0 : R);  // first round: group bits of k
            constexpr int P2 = TL::LOGP + (INV ? R : 0);  // second round
            T x[NTT_EPT];
            #pragma unroll
            for (int v = 0; v < NTT_EPT; v++) x[v] = ain[TL::gidx(insert_bits(tid, v, P1, R), sp0)];
            TL::template butterflies<R, P1 - TL::LOGP, 0, NR>(x, tid, 0, sp0, tw, nullptr, q);
            #pragma unroll
            for (int v = 0; v < NTT_EPT; v++) lds[insert_bits(tid, v, P1, R)] = x[v];
            __syncthreads();
            #pragma unroll
            for (int v = 0; v < NTT_EPT; v++) x[v] = lds[insert_bits(tid, v, P2, R)];
            TL::template butterflies<R, P2 - TL::LOGP, R, NR, FOLD>(x, tid, 0, sp0, tw, nullptr, q, ni);
            #pragma unroll
            for (int v = 0; v < NTT_EPT; v++) a[TL::gidx(insert_bits(tid, v, P2, R), sp0)] = finish(x[v]);
            return;
        }

        const T* tw2 = nullptr;
        if constexpr (TL::TW2)
            tw2 = tab.tw2 + (((size_t)prime * 2 + (INV ? 1 : 0)) * ntiles + bx) * (size_t)TL::TW_PASS *
                                THREADS * 2;

        if constexpr (TL::DIRECT_LO) {
            constexpr int R = NTT_EPT_LOG;
            constexpr int PH = TL::LOGP + R;  // groups over k's high 4 bits
            const uint32_t gh = TL::swap_nibbles(tid);
            T x[NTT_EPT];
            if constexpr (!INV) {
                #pragma unroll
                for (int v = 0; v < NTT_EPT; v++) x[v] = ain[TL::gidx(insert_bits(gh, v, PH, R), sp0)];
                TL::template butterflies<R, R, 0, NR>(x, gh, 0, sp0, tw, tw2, q);
                #pragma unroll
                for (int v = 0; v < NTT_EPT; v++) lds[TL::lpos(insert_bits(gh, v, PH, R))] = x[v];
                __syncthreads();
                TL::template round<R, 0, R, NR>(lds, sp0, tw, tw2, q);
                __syncthreads();
            } else {
                #pragma unroll
                for (int i = 0; i < NTT_EPT; i++) {
                    const uint32_t f = tid + i * THREADS;
                    const uint32_t e = ((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S);
                    lds[TL::lpos(e)] = ain[TL::gidx(e, sp0)];
                }
                __syncthreads();
                TL::template round<R, 0, 0>(lds, sp0, tw, tw2, q);
                __syncthreads();
                #pragma unroll
                for (int v = 0; v < NTT_EPT; v++) x[v] = lds[TL::lpos(insert_bits(gh, v, PH, R))];
                TL::template butterflies<R, R, R>(x, gh, 0, sp0, tw, tw2, q);
                #pragma unroll
                for (int v = 0; v < NTT_EPT; v++) a[TL::gidx(insert_bits(gh, v, PH, R), sp0)] = finish(x[v]);
                return;
            }
        } else {
            // load in global-contiguous order
            #pragma unroll
            for (int i = 0; i < NTT_EPT; i++) {
                const uint32_t f = tid + i * THREADS;
                uint32_t k, spl;
                if (BLO == 0) { spl = f >> S; k = f & ((1u << S) - 1u); }
                else { k = f >> TL::LOGP; spl = f & (TL::P - 1); }
                const uint32_t e = (k << TL::LOGP) | spl;
                lds[TL::lpos(e)] = ain[TL::gidx(e, sp0)];
            }
            __syncthreads();
            TL::template rounds<0, NR, FOLD>(lds, sp0, tw, tw2, q, ni);
        }

        #pragma unroll
        for (int i = 0; i < NTT_EPT; i++) {
            const uint32_t f = tid + i * THREADS;
            uint32_t k, spl;
            if (BLO == 0) { spl = f >> S; k = f & ((1u << S) - 1u); }
            else { k = f >> TL::LOGP; spl = f & (TL::P - 1); }
            const uint32_t e = (k << TL::LOGP) | spl;
            a[TL::gidx(e, sp0)] = finish(lds[TL::lpos(e)]);
        }
    };
    if constexpr (!INV && sizeof(T) == 8) {
        if (q < ((T)1 << 57)) body(std::true_type{});
        else body(std::false_type{});
    } else {
        body(std::false_type{});
    }
}

// ---------------------------------------------------------------- fused base conversion
// The fast base conversions of key switching sit between two transforms: ModUp takes a
// digit's rows back to coefficients, converts them to every other row of PQ and
// transforms those forward; ModDown does the same from the special rows to the
// ciphertext rows. At ring 2^16 the forward transform's first pass (8 stages over the
// high index bits) loads each thread's 16 elements straight from device memory (the
// DIRECT layout), so the conversion can produce them there instead: per tile and
// output row, the kernel reads the input rows at those 16 positions -- already
// y_a = [x_a (D/q_a)^-1]_{q_a}, the inverse transform having folded the factor into its
// n^-1 -- computes out = sum_a y_a (D/q_a) mod r (the words kb_modup / kb_conv write),
// and runs the pass on them. The converted rows never go through device memory; the
// input rows are read once per output row, from L2 after the first.
struct ConvFused {
    const uint64_t* in;          // input rows: y_a = [x_a (D/q_a)^-1]_{q_a}, canonical (ntt64_inverse_conv)
    uint64_t* out;               // output polynomials
    size_t in_stride, out_stride;  // words between consecutive input / output polynomials
    int in_row0, in_prime0;      // first input row of digit 0 (row r starts r n words in) and its prime
    int digits, alpha;           // grid y = u digits + j: source u, digit j (inputs from row in_row0 + alpha j)
    int out_rows, skip_n;        // output rows 0..out_rows-1 of polynomial y, except skip_n rows from alpha j
    int Lc, L;                   // output row r has prime r < Lc ? r : L + r - Lc
    const uint64_t* cst;         // cst[(alpha j + a) cst_stride + prime]: (D/q_a) mod prime, Montgomery form
    size_t cst_stride;
    const uint64_t* qinv;        // Montgomery constants of the primes
};

// One block per (output row, tile, polynomial), numbered so that the blocks of one
// (tile, polynomial) -- which read the same input words -- run consecutively on one XCD
// (blocks go to the XCDs round robin: block b takes item (b mod 8) per_xcd + b / 8).
template <int A, int LOGN>
__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
conv_fused_kernel(ConvFused f, NttTab<uint64_t> tab, uint32_t nout, uint32_t work, uint32_t per_xcd) {
    static_assert(A >= 1 && A <= 4, "digit size");
    constexpr int R = NTT_EPT_LOG;
    typedef Tile<uint64_t, false, LOGN, LOGN - 8, 8, 0> TF;  // forward transform, first pass
    static_assert(TF::DIRECT, "ring 2^16");
    constexpr int P_LO = TF::LOGP, P_HI = TF::LOGP + R;
    constexpr size_t N = (size_t)1 << LOGN;
    constexpr uint32_t NTILES = 1u << (LOGN - TILE_LOG);
    __shared__ uint64_t lds[TF::LDS_WORDS];
    const uint32_t bid = blockIdx.x;
    const uint32_t wk = (bid & 7u) * per_xcd + (bid >> 3);
    if (wk >= work) return;  // uniform over the block
    const uint32_t ro = wk % nout, rest = wk / nout;
    const uint32_t tid = threadIdx.x, sp0 = (rest % NTILES) * TF::P;
    const int y = (int)(rest / NTILES), u = y / f.digits, j = y % f.digits;
    const int row = (int)ro < f.alpha * j ? (int)ro : (int)ro + f.skip_n;  // past the digit's own rows
    const int prime = row < f.Lc ? row : f.L + row - f.Lc;
    const uint64_t q = tab.mods[prime], qi = f.qinv[prime];
    const uint64_t* src = f.in + (size_t)u * f.in_stride + (size_t)(f.in_row0 + f.alpha * j) * N;
    const uint64_t* cst0 = f.cst + (size_t)(f.alpha * j) * f.cst_stride + prime;
    uint64_t x[NTT_EPT];
    {
        uint64_t c[A];
        #pragma unroll
        for (int a = 0; a < A; a++) c[a] = cst0[(size_t)a * f.cst_stride];
        // the input words of 8 elements are loaded together, then converted
        #pragma unroll
        for (int h = 0; h < NTT_EPT; h += 8) {
            uint64_t sv[8][A];
            #pragma unroll
            for (int v = 0; v < 8; v++) {
                const uint32_t e = TF::gidx(insert_bits(tid, h + v, P_HI, R), sp0);
                #pragma unroll
                for (int a = 0; a < A; a++) sv[v][a] = src[(size_t)a * N + e];
            }
            #pragma unroll
            for (int v = 0; v < 8; v++) {
                u128p acc{0, 0};
                #pragma unroll
                for (int a = 0; a < A; a++) add128(acc, mul128(sv[v][a], c[a]));
                x[h + v] = redc(acc, q, qi);
            }
        }
    }
    const uint64_t* tw = tab.base + ((size_t)prime * 2) * 2 * N;
    uint64_t* dst = f.out + (size_t)y * f.out_stride + (size_t)row * N;
    // the same per-prime choice as the forward transform (no conditional subtractions
    // below 2^57), so its low-bit pass finds the bounds it expects
    auto pass = [&](auto nr_c) __attribute__((always_inline)) {
        constexpr bool NR = decltype(nr_c)::value;
        TF::template butterflies<R, R, 0, NR>(x, tid, 0, sp0, tw, nullptr, q);
        #pragma unroll
        for (int v = 0; v < NTT_EPT; v++) lds[insert_bits(tid, v, P_HI, R)] = x[v];
        __syncthreads();
        #pragma unroll
        for (int v = 0; v < NTT_EPT; v++) x[v] = lds[insert_bits(tid, v, P_LO, R)];
        TF::template butterflies<R, 0, R, NR>(x, tid, 0, sp0, tw, nullptr, q);
        #pragma unroll
        for (int v = 0; v < NTT_EPT; v++) dst[TF::gidx(insert_bits(tid, v, P_LO, R), sp0)] = x[v];
    };
    if (q < ((uint64_t)1 << 57)) pass(std::true_type{});
    else pass(std::false_type{});
}

template <int LOGN>
static void conv_fused_logn(const Ctx& c, const ConvFused& f, int polys, hipStream_t st) {
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods, c.d_tw2};
    const uint32_t nout = (uint32_t)(f.out_rows - f.skip_n);
    const uint64_t work = (uint64_t)nout * (1u << (LOGN - TILE_LOG)) * (uint32_t)polys;
    const uint32_t per_xcd = (uint32_t)((work + 7) / 8);
    const dim3 grid(per_xcd * 8);
    switch (f.alpha) {
        case 1: hc_launch((conv_fused_kernel<1, LOGN>), grid, dim3(NTT_THREADS), 0, st, f, tab, nout, (uint32_t)work, per_xcd); break;
        case 2: hc_launch((conv_fused_kernel<2, LOGN>), grid, dim3(NTT_THREADS), 0, st, f, tab, nout, (uint32_t)work, per_xcd); break;
        case 3: hc_launch((conv_fused_kernel<3, LOGN>), grid, dim3(NTT_THREADS), 0, st, f, tab, nout, (uint32_t)work, per_xcd); break;
        default: hc_launch((conv_fused_kernel<4, LOGN>), grid, dim3(NTT_THREADS), 0, st, f, tab, nout, (uint32_t)work, per_xcd); break;
    }
}

bool conv_fused_ring(const Ctx& c) { return c.logn == 16; }

// ModUp of U sources at level Lc: tmpC [U][Lc][n] (coefficient domain) -> X[U][dn][R][n],
// every row outside each digit through the forward high-bit pass.
void k_modup_fused(const Ctx& c, uint64_t* X, const uint64_t* tmpC, int U, int Lc, hipStream_t st) {
    const int dn = Lc / c.alpha, R = Lc + c.K;
    ConvFused f;
    f.in = tmpC;
    f.out = X;
    f.in_stride = (size_t)Lc * c.n;
    f.out_stride = (size_t)R * c.n;
    f.in_row0 = 0;
    f.in_prime0 = 0;
    f.digits = dn;
    f.alpha = c.alpha;
    f.out_rows = R;
    f.skip_n = c.alpha;
    f.Lc = Lc;
    f.L = c.L;
    f.cst = c.d_modup_c;
    f.cst_stride = (size_t)c.nq;
    f.qinv = c.d_qinv;
    const double n = c.n, polys = (double)U * dn;
    // reads the digit's rows once, writes every converted row once; butterflies of the pass
    TimeScope ts(c, HC_KT_CONV_FUSED, st, 8.0 * n * polys * R, polys * (n / 2) * 8 * (R - c.alpha));
    conv_fused_logn<16>(c, f, U * dn, st);
}

// ModDown's conversion of M jobs (2 components each) at level Lc: the special rows of
// T [M][2][R][n] (coefficient domain) -> conv [M][2][Lc][n] through the forward
// high-bit pass.
void k_moddown_fused(const Ctx& c, uint64_t* conv, const uint64_t* T, int M, int Lc, hipStream_t st) {
    const int R = Lc + c.K;
    ConvFused f;
    f.in = T;
    f.out = conv;
    f.in_stride = (size_t)R * c.n;
    f.out_stride = (size_t)Lc * c.n;
    f.in_row0 = Lc;
    f.in_prime0 = c.L;
    f.digits = 1;
    f.alpha = c.K;
    f.out_rows = Lc;
    f.skip_n = 0;
    f.Lc = Lc;
    f.L = c.L;
    f.cst = c.d_moddown_c;
    f.cst_stride = (size_t)c.L;
    f.qinv = c.d_qinv;
    const double n = c.n, polys = 2.0 * M;
    TimeScope ts(c, HC_KT_CONV_FUSED, st, 8.0 * n * polys * (c.K + Lc), polys * (n / 2) * 8 * Lc);
    conv_fused_logn<16>(c, f, 2 * M, st);
}

// Grid: (tiles of a row, polynomials, rows). WPE: minimum waves per SIMD the
// registers must allow (1 = no constraint).
template <typename T, bool INV, int LOGN, int S, int BLO, int ST0, bool LAST, int WPE>
__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(WPE)))
ntt_tile_kernel(T* __restrict__ data, size_t poly_stride, int limb_first, NttTab<T> tab, const T* __restrict__ src) {
    typedef Tile<T, INV, LOGN, S, BLO, ST0> TL;
    __shared__ T lds[TL::LDS_WORDS];
    ntt_tile<T, INV, LOGN, S, BLO, ST0, LAST>(data, poly_stride, limb_first, tab, lds, blockIdx.x, blockIdx.y,
                                              blockIdx.z, gridDim.x, src);
}

// The same pass as a persistent grid: a fixed number of blocks (the device's resident
// capacity) walks the pass's work queue of (tile, polynomial, row) items, item i =
// (row count + polynomial) ntiles + tile in the regular grid's block order, each block
// taking items blockIdx.x, blockIdx.x + gridDim.x, ... until the queue is exhausted.
// Every item costs the same, so the static order balances like a dynamic one. The
// block's LDS tile is reused item after item (a barrier separates them); every block
// leaves the loop after its last item.
template <typename T, bool INV, int LOGN, int S, int BLO, int ST0, bool LAST, int WPE>
__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(WPE)))
ntt_tile_persistent_kernel(T* __restrict__ data, size_t poly_stride, int limb_first, NttTab<T> tab,
                           uint32_t ntiles, uint32_t count, uint32_t items, const T* __restrict__ src) {
    typedef Tile<T, INV, LOGN, S, BLO, ST0> TL;
    __shared__ T lds[TL::LDS_WORDS];
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        if (it != blockIdx.x) __syncthreads();  // the previous item's LDS reads are done
        const uint32_t bx = it % ntiles, rest = it / ntiles;
        ntt_tile<T, INV, LOGN, S, BLO, ST0, LAST>(data, poly_stride, limb_first, tab, lds, bx, rest % count,
                                                  rest / count, ntiles, src);
    }
}

// Launch one pass; `ops` butterflies and `bytes` moved for the timing record. src: as
// ntt_tile.
template <typename T, bool INV, int LOGN, int S, int BLO, int ST0, bool LAST>
static void pass(const Ctx& c, int kind, T* data, size_t stride, int count, int lf, int nl,
                 NttTab<T> tab, hipStream_t st, const T* src = nullptr) {
    constexpr int TLOG = LOGN < TILE_LOG ? LOGN : TILE_LOG;
    constexpr int THREADS = (1 << TLOG) / NTT_EPT;
    static_assert(THREADS <= NTT_THREADS, "tile");
    // 64-bit passes of two-pass rings: by default four waves per SIMD (128 registers),
    // which the twiddle-heavy passes reach with a few spilled words; the context's tuned
    // variant (hc_autotune) may pick three or five, or the persistent grid. Every
    // variant computes the same words.
    constexpr bool TUNED = sizeof(T) == 8 && LOGN > TILE_LOG;
    const int var = TUNED ? c.tune_ntt : 0;
    dim3 grid(1 << (LOGN - TLOG), count, nl);
    const double bytes = 2.0 * sizeof(T) * (double)count * nl * (1 << LOGN);
    const double ops = (double)count * nl * (1 << (LOGN - 1)) * S;
    auto launch = [&]() {
        if constexpr (TUNED) {
            if (var == 1) {
                hc_launch((ntt_tile_kernel<T, INV, LOGN, S, BLO, ST0, LAST, 3>), grid, dim3(THREADS), 0, st,
                                   data, stride, lf, tab, src);
                return;
            }
            if (var == 2) {
                hc_launch((ntt_tile_kernel<T, INV, LOGN, S, BLO, ST0, LAST, 5>), grid, dim3(THREADS), 0, st,
                                   data, stride, lf, tab, src);
                return;
            }
            if (var == 3) {
                const uint32_t items = grid.x * grid.y * grid.z;
                const uint32_t cap = (uint32_t)c.cus * 4;  // four 4-wave blocks per CU (4 waves per SIMD)
                hc_launch((ntt_tile_persistent_kernel<T, INV, LOGN, S, BLO, ST0, LAST, 4>),
                                   dim3(items < cap ? items : cap), dim3(THREADS), 0, st, data, stride, lf, tab,
                                   grid.x, (uint32_t)count, items, src);
                return;
            }
        }
        hc_launch((ntt_tile_kernel<T, INV, LOGN, S, BLO, ST0, LAST, TUNED ? 4 : 1>), grid, dim3(THREADS), 0,
                           st, data, stride, lf, tab, src);
    };
    if (kind >= 0) {
        TimeScope ts(c, kind, st, bytes, ops);
        launch();
    } else {
        launch();
    }
}

// src (nullptr: in place): the first pass reads the input there, at data's offsets.
template <typename T, bool INV, int LOGN>
static void run_logn(const Ctx& c, int kind, T* data, size_t stride, int count, int lf, int nl,
                     NttTab<T> tab, hipStream_t st, const T* src) {
    if constexpr (LOGN <= TILE_LOG) {
        pass<T, INV, LOGN, LOGN, 0, 0, true>(c, kind, data, stride, count, lf, nl, tab, st, src);
    } else {
        constexpr int SL = 8, SH = LOGN - 8;
        if (!INV) {
            pass<T, false, LOGN, SH, SL, 0, false>(c, kind, data, stride, count, lf, nl, tab, st, src);
            pass<T, false, LOGN, SL, 0, SH, true>(c, kind, data, stride, count, lf, nl, tab, st);
        } else {
            pass<T, true, LOGN, SL, 0, 0, false>(c, kind, data, stride, count, lf, nl, tab, st, src);
            pass<T, true, LOGN, SH, SL, SL, true>(c, kind, data, stride, count, lf, nl, tab, st);
        }
    }
}

template <typename T, bool INV>
static void run_ntt(const Ctx& c, int kind, T* data, size_t stride, int count, int lf, int nl,
                    NttTab<T> tab, hipStream_t st, const T* src = nullptr) {
    switch (c.logn) {
        case 10: run_logn<T, INV, 10>(c, kind, data, stride, count, lf, nl, tab, st, src); break;
        case 11: run_logn<T, INV, 11>(c, kind, data, stride, count, lf, nl, tab, st, src); break;
        case 12: run_logn<T, INV, 12>(c, kind, data, stride, count, lf, nl, tab, st, src); break;
        case 13: run_logn<T, INV, 13>(c, kind, data, stride, count, lf, nl, tab, st, src); break;
        case 14: run_logn<T, INV, 14>(c, kind, data, stride, count, lf, nl, tab, st, src); break;
        case 15: run_logn<T, INV, 15>(c, kind, data, stride, count, lf, nl, tab, st, src); break;
        case 16: run_logn<T, INV, 16>(c, kind, data, stride, count, lf, nl, tab, st, src); break;
        default: break;
    }
}

// Thread-ordered twiddles of the low-bit pass of each direction (see Tile::TW2):
// out[prime][dir][tile][TW_PASS][THREADS][2], one block per (tile, prime).
template <bool INV, int LOGN>
__global__ void __launch_bounds__(NTT_THREADS) ntt_tw2_kernel(uint64_t* __restrict__ out,
                                                              const uint64_t* __restrict__ tw_all) {
    typedef Tile<uint64_t, INV, LOGN, 8, 0, INV ? 0 : LOGN - 8> TL;
    const int prime = blockIdx.y;
    const uint64_t* tw = tw_all + ((size_t)prime * 2 + (INV ? 1 : 0)) * 2 * TL::N;
    uint64_t* o = out + (((size_t)prime * 2 + (INV ? 1 : 0)) * gridDim.x + blockIdx.x) * (size_t)TL::TW_PASS *
                            TL::THREADS * 2;
    TL::template emit<0>(o, blockIdx.x * TL::P, tw);
}

template <int LOGN>
static hc_status build_tw2_logn(Ctx& c) {
    typedef Tile<uint64_t, false, LOGN, 8, 0, LOGN - 8> TF;
    typedef Tile<uint64_t, true, LOGN, 8, 0, 0> TI;
    static_assert(TF::TW2 && TI::TW2 && TF::TW_PASS == TI::TW_PASS, "low-bit passes");
    const int tiles = 1 << (LOGN - TILE_LOG);
    const size_t words = (size_t)c.ntab * 2 * tiles * TF::TW_PASS * TF::THREADS * 2;
    HC_CHECK(hipMalloc((void**)&c.d_tw2, sizeof(uint64_t) * words));
    c.owned.push_back(c.d_tw2);
    hipLaunchKernelGGL((ntt_tw2_kernel<false, LOGN>), dim3(tiles, c.ntab), dim3(TF::THREADS), 0, 0, c.d_tw2, c.d_tw);
    hipLaunchKernelGGL((ntt_tw2_kernel<true, LOGN>), dim3(tiles, c.ntab), dim3(TI::THREADS), 0, 0, c.d_tw2, c.d_tw);
    HC_CHECK(hipGetLastError());
    HC_CHECK(hipDeviceSynchronize());
    return HC_OK;
}

hc_status ntt_build_tw2(Ctx& c) {
    switch (c.logn) {
        case 13: return build_tw2_logn<13>(c);
        case 14: return build_tw2_logn<14>(c);
        case 15: return build_tw2_logn<15>(c);
        case 16: return build_tw2_logn<16>(c);
        default: return HC_OK;  // one-pass rings read the table directly
    }
}

void ntt64(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
           bool inverse, hipStream_t stream, const uint64_t* src) {
    if (count <= 0 || nlimbs <= 0) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods, c.d_tw2};
    if (inverse)
        run_ntt<uint64_t, true>(c, HC_KT_NTT_INV, data, poly_stride, count, limb_first, nlimbs, tab, stream, src);
    else run_ntt<uint64_t, false>(c, HC_KT_NTT_FWD, data, poly_stride, count, limb_first, nlimbs, tab, stream, src);
}

// Only the low-bit pass of a two-pass ring: the inverse transform's first pass or the
// forward transform's last (the other pass runs inside k_modup_fused / k_moddown_fused).
template <int LOGN>
static void low_pass_logn(const Ctx& c, uint64_t* data, size_t stride, int count, int lf, int nl, bool inverse,
                          hipStream_t st) {
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods, c.d_tw2};
    constexpr int SL = 8, SH = LOGN - 8;
    if (inverse) pass<uint64_t, true, LOGN, SL, 0, 0, false>(c, HC_KT_NTT_INV, data, stride, count, lf, nl, tab, st);
    else pass<uint64_t, false, LOGN, SL, 0, SH, true>(c, HC_KT_NTT_FWD, data, stride, count, lf, nl, tab, st);
}

void ntt64_low_pass(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                    bool inverse, hipStream_t stream) {
    if (count <= 0 || nlimbs <= 0 || c.logn != 16) return;
    low_pass_logn<16>(c, data, poly_stride, count, limb_first, nlimbs, inverse, stream);
}

// The forward low-bit pass (ring 2^16) of the ciphertext rows ModUp computes, every
// digit in one launch: polynomial y (stride poly_stride) is digit y % dn of its source,
// and its rows [j alpha, (j + 1) alpha) of digit j are the digit's own (copied in the NTT
// domain), which the blocks of those rows skip.
__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
ntt_low_raise_kernel(uint64_t* __restrict__ data, size_t poly_stride, NttTab<uint64_t> tab, int dn, int alpha) {
    typedef Tile<uint64_t, false, 16, 8, 0, 8> TL;
    __shared__ uint64_t lds[TL::LDS_WORDS];
    if ((int)blockIdx.z / alpha == (int)(blockIdx.y % (uint32_t)dn)) return;  // whole block
    ntt_tile<uint64_t, false, 16, 8, 0, 8, true>(data, poly_stride, 0, tab, lds, blockIdx.x, blockIdx.y, blockIdx.z,
                                                 gridDim.x);
}

void ntt64_low_raise(const Ctx& c, uint64_t* X, size_t poly_stride, int count, int Lc, int dn, hipStream_t st) {
    if (count <= 0 || dn < 2 || c.logn != 16) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods, c.d_tw2};
    const double rows = (double)count * (Lc - c.alpha);  // rows transformed
    TimeScope ts(c, HC_KT_NTT_FWD, st, 16.0 * rows * c.n, rows * (c.n / 2) * 8);
    hc_launch(ntt_low_raise_kernel, dim3(1u << (16 - TILE_LOG), (unsigned)count, (unsigned)Lc), dim3(NTT_THREADS), 0,
              st, X, poly_stride, tab, dn, c.alpha);
}

// The inverse transform's first pass (the low index bits, ring 2^16) of ModUp's inputs,
// loading them from the jobs' ciphertexts: word g of row r of polynomial u is c1 of
// jobs[u].in at sigma_{k_u}'s source of g, and it is also stored to the digit's own row
// of X. Otherwise the pass of ntt_tile (DIRECT_LO, inverse).
__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
ntt_take_c1_low_kernel(const KsJob* __restrict__ jobs, uint64_t* __restrict__ tmpC, uint64_t* __restrict__ X,
                       NttTab<uint64_t> tab, int Lc, int alpha, int R, int dn) {
    constexpr int LOGN = 16, S = 8, RR = NTT_EPT_LOG;
    typedef Tile<uint64_t, true, LOGN, S, 0, 0> TL;
    static_assert(TL::DIRECT_LO && TL::TW2 && TL::THREADS == NTT_THREADS, "ring 2^16 low-bit pass");
    constexpr int PH = TL::LOGP + RR;
    constexpr size_t N = (size_t)1 << LOGN;
    __shared__ uint64_t lds[TL::LDS_WORDS];
    const uint32_t tid = threadIdx.x, bx = blockIdx.x, u = blockIdx.y, r = blockIdx.z;
    const int prime = (int)r;
    const uint64_t q = tab.mods[prime];
    const uint64_t* tw = tab.base + ((size_t)prime * 2 + 1) * 2 * N;
    const uint64_t* tw2 = tab.tw2 + (((size_t)prime * 2 + 1) * gridDim.x + bx) * (size_t)TL::TW_PASS * TL::THREADS * 2;
    const uint32_t sp0 = bx * TL::P;
    const KsJob jb = jobs[u];
    gl_cu64* in = gl(jb.in) + (size_t)(Lc + (int)r) * N;
    uint64_t* own = X + (((size_t)u * dn + r / alpha) * R + r) * N;
    // every gather first, then the stores (a store between two loads of the same
    // thread would keep the second waiting for the first)
    uint64_t vv[NTT_EPT];
    #pragma unroll
    for (int i = 0; i < NTT_EPT; i++) {
        const uint32_t f = tid + i * TL::THREADS;
        const uint32_t e = ((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S);
        const uint32_t g = TL::gidx(e, sp0);
        vv[i] = in[jb.k == 1 ? g : galois_src(g, jb.k, LOGN)];
    }
    #pragma unroll
    for (int i = 0; i < NTT_EPT; i++) {
        const uint32_t f = tid + i * TL::THREADS;
        const uint32_t e = ((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S);
        own[TL::gidx(e, sp0)] = vv[i];
        lds[TL::lpos(e)] = vv[i];
    }
    __syncthreads();
    TL::template round<RR, 0, 0>(lds, sp0, tw, tw2, q);
    __syncthreads();
    const uint32_t gh = TL::swap_nibbles(tid);
    uint64_t x[NTT_EPT];
    #pragma unroll
    for (int v = 0; v < NTT_EPT; v++) x[v] = lds[TL::lpos(insert_bits(gh, v, PH, RR))];
    TL::template butterflies<RR, RR, RR>(x, gh, 0, sp0, tw, tw2, q);
    uint64_t* a = tmpC + ((size_t)u * Lc + r) * N;
    #pragma unroll
    for (int v = 0; v < NTT_EPT; v++) a[TL::gidx(insert_bits(gh, v, PH, RR), sp0)] = x[v];
}

// The inverse transform's first pass (ring 2^16) of Mask's products at the dropped rows
// Lc..L-1, computed while loading: block (tile, (job m, component, column), row Lc + k)
// takes its words of jobs[m].a times the column's plaintext row (Montgomery), runs the
// pass and stores it to the column's output row -- the words mask_jobs writes there,
// after the pass. The blocks of one tile go to one XCD (16 tiles: the block number's
// residue mod 8 is the tile's), so the columns of a row reread its words from that L2.
__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
ntt_mask_low_kernel(const MaskJob* __restrict__ jobs, NttTab<uint64_t> tab, const uint64_t* __restrict__ qinv, int L,
                    int Lc, int cmax) {
    constexpr int LOGN = 16, S = 8, RR = NTT_EPT_LOG;
    typedef Tile<uint64_t, true, LOGN, S, 0, 0> TL;
    static_assert(TL::DIRECT_LO && TL::TW2 && TL::THREADS == NTT_THREADS, "ring 2^16 low-bit pass");
    constexpr int PH = TL::LOGP + RR;
    constexpr size_t N = (size_t)1 << LOGN;
    __shared__ uint64_t lds[TL::LDS_WORDS];
    const uint32_t tid = threadIdx.x, bx = blockIdx.x, k = blockIdx.z;
    const uint32_t mc = blockIdx.y / (uint32_t)cmax, col = blockIdx.y % (uint32_t)cmax;
    const int m = (int)(mc >> 1), comp = (int)(mc & 1);
    const MaskJob jb = jobs[m];
    if (col >= jb.ncol) return;  // uniform over the block
    const int prime = Lc + (int)k;
    const uint64_t q = tab.mods[prime], qi = qinv[prime];
    const uint64_t* tw = tab.base + ((size_t)prime * 2 + 1) * 2 * N;
    const uint64_t* tw2 = tab.tw2 + (((size_t)prime * 2 + 1) * gridDim.x + bx) * (size_t)TL::TW_PASS * TL::THREADS * 2;
    const uint32_t sp0 = bx * TL::P;
    const size_t row = ((size_t)comp * L + prime) * N;
    gl_cu64* av = gl(jb.a) + row;
    gl_cu64* pt = gl(jb.b) + (size_t)col * jb.b_step + (size_t)prime * N;
    // the words of 8 elements are loaded together, then multiplied
    #pragma unroll
    for (int h = 0; h < NTT_EPT; h += 8) {
        uint64_t a[8], b[8];
        #pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t f = tid + (h + i) * TL::THREADS;
            const uint32_t g = TL::gidx(((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S), sp0);
            a[i] = av[g];
            b[i] = pt[g];
        }
        #pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t f = tid + (h + i) * TL::THREADS;
            lds[TL::lpos(((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S))] = mont_mul(a[i], b[i], q, qi);
        }
    }
    __syncthreads();
    TL::template round<RR, 0, 0>(lds, sp0, tw, tw2, q);
    __syncthreads();
    const uint32_t gh = TL::swap_nibbles(tid);
    uint64_t x[NTT_EPT];
    #pragma unroll
    for (int v = 0; v < NTT_EPT; v++) x[v] = lds[TL::lpos(insert_bits(gh, v, PH, RR))];
    TL::template butterflies<RR, RR, RR>(x, gh, 0, sp0, tw, tw2, q);
    gl_mu64* o = gl(jb.out) + (size_t)col * jb.out_step + row;
    #pragma unroll
    for (int v = 0; v < NTT_EPT; v++) o[TL::gidx(insert_bits(gh, v, PH, RR), sp0)] = x[v];
}

void ntt_mask_low(const Ctx& c, const MaskJob* jobs, int M, int cmax, int nprod, int Lc, hipStream_t st) {
    if (M <= 0 || cmax <= 0 || nprod <= 0 || Lc >= c.L || c.logn != 16) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods, c.d_tw2};
    const double n = c.n, nd = c.L - Lc;
    // per job row its words once; per product row the plaintext row and the pass's output
    TimeScope ts(c, HC_KT_NTT_INV, st, 8.0 * n * 2.0 * nd * (M + 2.0 * nprod), 2.0 * nd * nprod * (n / 2) * 8);
    static_assert((1u << (16 - TILE_LOG)) % 8 == 0, "tiles per row a multiple of the XCD count");
    const int per_launch = std::max(1, 65535 / (2 * cmax));  // grid y stays within its limit
    for (int j0 = 0; j0 < M; j0 += per_launch) {
        const int mj = std::min(per_launch, M - j0);
        hc_launch(ntt_mask_low_kernel, dim3(1u << (16 - TILE_LOG), (unsigned)(2 * mj * cmax), (unsigned)(c.L - Lc)),
                  dim3(NTT_THREADS), 0, st, jobs + j0, tab, c.d_qinv, c.L, Lc, cmax);
    }
}

void ntt64_inverse_high_tab(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                            const uint64_t* ninv, hipStream_t stream) {
    if (count <= 0 || nlimbs <= 0 || c.logn != 16) return;
    NttTab<uint64_t> tab{c.d_tw, ninv, c.d_mods, c.d_tw2};
    pass<uint64_t, true, 16, 8, 8, 8, true>(c, HC_KT_NTT_INV, data, poly_stride, count, limb_first, nlimbs, tab, stream);
}

// ModDown's inverse transform, first pass (ring 2^16), of the special rows of the key
// products, computing them while loading: word g of row Lc + k of T[m][comp] is
// sum_j X[xidx_m][j][Lc + k][src(g)] key_m[j][comp][L + k][g] (src: sigma_{k_m}'s source
// if hoisted), one REDC of the 128-bit sum -- the words kb_inner writes. Blocks of
// consecutive jobs at one tile run on one XCD (the grid's x is the 16 tiles), so jobs
// sharing a key read it through that XCD's L2. MULTI: more than one digit (a separate
// build, so the one-digit kernel keeps its registers).
template <bool MULTI>
__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
ntt_inner_low_kernel(const KsJob* __restrict__ jobs, const uint64_t* __restrict__ X, uint64_t* __restrict__ T,
                     NttTab<uint64_t> tab, const uint64_t* __restrict__ qinv, int Lc, int K, int L, int nq, int dn,
                     int hoisted) {
    constexpr int LOGN = 16, S = 8, RR = NTT_EPT_LOG;
    typedef Tile<uint64_t, true, LOGN, S, 0, 0> TL;
    static_assert(TL::DIRECT_LO && TL::TW2 && TL::THREADS == NTT_THREADS, "ring 2^16 low-bit pass");
    constexpr int PH = TL::LOGP + RR;
    constexpr size_t N = (size_t)1 << LOGN;
    __shared__ uint64_t lds[TL::LDS_WORDS];
    const uint32_t tid = threadIdx.x, bx = blockIdx.x, mc = blockIdx.y, k = blockIdx.z;
    const int m = (int)(mc >> 1), comp = (int)(mc & 1), R = Lc + K;
    const int prime = L + (int)k;
    const uint64_t q = tab.mods[prime], qi = qinv[prime];
    const uint64_t* tw = tab.base + ((size_t)prime * 2 + 1) * 2 * N;
    const uint64_t* tw2 = tab.tw2 + (((size_t)prime * 2 + 1) * gridDim.x + bx) * (size_t)TL::TW_PASS * TL::THREADS * 2;
    const uint32_t sp0 = bx * TL::P;
    const KsJob jb = jobs[m];
    const size_t keyrow = (size_t)nq * N;
    gl_cu64* kp = gl(jb.key) + (size_t)comp * keyrow + (size_t)prime * N;
    const uint64_t* xp = X + ((size_t)jb.xidx * dn * R + Lc + k) * N;
    const bool rot = hoisted && jb.k != 1;
    if constexpr (!MULTI) {
        // one digit: the words of 8 elements are loaded together, then multiplied (a
        // loop over the digits between the loads would make each wait for the last)
        #pragma unroll
        for (int h = 0; h < NTT_EPT; h += 8) {
            uint64_t xv[8], kv[8];
            #pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint32_t f = tid + (h + i) * TL::THREADS;
                const uint32_t e = ((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S);
                const uint32_t g = TL::gidx(e, sp0);
                xv[i] = xp[rot ? galois_src(g, jb.k, LOGN) : g];
                kv[i] = kp[g];
            }
            #pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint32_t f = tid + (h + i) * TL::THREADS;
                const uint32_t e = ((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S);
                lds[TL::lpos(e)] = redc(mul128(xv[i], kv[i]), q, qi);
            }
        }
    } else {
        // several digits: per quarter of the thread's elements, digit after digit, each
        // digit's words of the 4 elements loaded together
        gl_cu64* xg = gl(xp);
        #pragma unroll
        for (int h = 0; h < NTT_EPT; h += 4) {
            uint32_t gg[4], ss[4];
            #pragma unroll
            for (int i = 0; i < 4; i++) {
                const uint32_t f = tid + (h + i) * TL::THREADS;
                const uint32_t e = ((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S);
                gg[i] = TL::gidx(e, sp0);
                ss[i] = rot ? galois_src(gg[i], jb.k, LOGN) : gg[i];
            }
            u128p acc[4];
            #pragma unroll
            for (int i = 0; i < 4; i++) acc[i] = u128p{0, 0};
            for (int j = 0; j < dn; j++) {
                uint64_t xv[4], kv[4];
                #pragma unroll
                for (int i = 0; i < 4; i++) {
                    xv[i] = xg[(size_t)j * R * N + ss[i]];
                    kv[i] = kp[(size_t)j * 2 * keyrow + gg[i]];
                }
                #pragma unroll
                for (int i = 0; i < 4; i++) add128(acc[i], mul128(xv[i], kv[i]));
            }
            #pragma unroll
            for (int i = 0; i < 4; i++) {
                const uint32_t f = tid + (h + i) * TL::THREADS;
                const uint32_t e = ((f & ((1u << S) - 1u)) << TL::LOGP) | (f >> S);
                lds[TL::lpos(e)] = redc(acc[i], q, qi);
            }
        }
    }
    __syncthreads();
    TL::template round<RR, 0, 0>(lds, sp0, tw, tw2, q);
    __syncthreads();
    const uint32_t gh = TL::swap_nibbles(tid);
    uint64_t x[NTT_EPT];
    #pragma unroll
    for (int v = 0; v < NTT_EPT; v++) x[v] = lds[TL::lpos(insert_bits(gh, v, PH, RR))];
    TL::template butterflies<RR, RR, RR>(x, gh, 0, sp0, tw, tw2, q);
    uint64_t* a = T + ((size_t)mc * R + Lc + k) * N;
    #pragma unroll
    for (int v = 0; v < NTT_EPT; v++) a[TL::gidx(insert_bits(gh, v, PH, RR), sp0)] = x[v];
}

void ntt_inner_low(const Ctx& c, const KsJob* jobs, const uint64_t* X, uint64_t* T, int M, int Lc, bool hoisted,
                   hipStream_t st) {
    if (M <= 0 || c.logn != 16) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods, c.d_tw2};
    const int dn = Lc / c.alpha;
    const double n = c.n;
    // per job and special row: its digits and the key words of both components, the pass's output
    TimeScope ts(c, HC_KT_NTT_INV, st, 8.0 * n * M * c.K * (dn + 2.0 * dn + 2.0), 2.0 * M * c.K * (n / 2) * 8);
    const dim3 grid(1u << (16 - TILE_LOG), (unsigned)(2 * M), (unsigned)c.K);
    if (dn == 1)
        hc_launch(ntt_inner_low_kernel<false>, grid, dim3(NTT_THREADS), 0, st, jobs, X, T, tab, c.d_qinv, Lc, c.K,
                  c.L, c.nq, dn, hoisted ? 1 : 0);
    else
        hc_launch(ntt_inner_low_kernel<true>, grid, dim3(NTT_THREADS), 0, st, jobs, X, T, tab, c.d_qinv, Lc, c.K,
                  c.L, c.nq, dn, hoisted ? 1 : 0);
}

void ntt_take_c1_low(const Ctx& c, const KsJob* jobs, uint64_t* tmpC, uint64_t* X, int U, int Lc, hipStream_t st) {
    if (U <= 0 || c.logn != 16) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods, c.d_tw2};
    const double n = c.n;
    // reads the rotated c1 rows, writes them to X and the pass's output: 24 bytes per word
    TimeScope ts(c, HC_KT_NTT_INV, st, 24.0 * n * U * Lc, (double)U * Lc * (n / 2) * 8);
    hc_launch(ntt_take_c1_low_kernel, dim3(1u << (16 - TILE_LOG), (unsigned)U, (unsigned)Lc),
                       dim3(NTT_THREADS), 0, st, jobs, tmpC, X, tab, Lc, c.alpha, Lc + c.K, Lc / c.alpha);
}

void ntt64_inverse_high_conv(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                             hipStream_t stream) {
    if (count <= 0 || nlimbs <= 0 || c.logn != 16) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv_conv, c.d_mods, c.d_tw2};
    pass<uint64_t, true, 16, 8, 8, 8, true>(c, HC_KT_NTT_INV, data, poly_stride, count, limb_first, nlimbs, tab, stream);
}

void ntt64_inverse_conv(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                        hipStream_t stream) {
    if (count <= 0 || nlimbs <= 0) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv_conv, c.d_mods, c.d_tw2};
    run_ntt<uint64_t, true>(c, HC_KT_NTT_INV, data, poly_stride, count, limb_first, nlimbs, tab, stream);
}

void ntt32(const Ctx& c, uint32_t* data, int count, bool inverse, hipStream_t stream) {
    if (count <= 0) return;
    NttTab<uint32_t> tab{c.d_twp, c.d_ninvp, c.d_modp, nullptr};
    if (inverse) run_ntt<uint32_t, true>(c, -1, data, (size_t)c.n, count, 0, 1, tab, stream);
    else run_ntt<uint32_t, false>(c, -1, data, (size_t)c.n, count, 0, 1, tab, stream);
}

}  // namespace hc
