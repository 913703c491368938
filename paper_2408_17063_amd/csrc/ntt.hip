// Negacyclic NTT / inverse NTT per prime, batched over polynomials and primes.
//
// Forward transform (merged psi-twist, Cooley-Tukey, natural order in,
// bit-reversed order out): stage st = 0..logn-1 pairs index j with
// j + n/2^(st+1) and multiplies by W[2^st + (j >> (logn - st))],
// W[k] = psi^brv(k). Output entry i = a(psi^(2 brv(i) + 1)).
// Inverse (Gentleman-Sande): stage u = 0..logn-1 pairs j with j + 2^u,
// twiddle Winv[n/2^(u+1) + (j >> (u+1))], Winv[k] = psi^-brv(k), then a
// final multiplication by n^-1.
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
// table. Rings up to 2^12 take one launch per transform; larger rings take two
// (high bits then the low 8 bits forward, the reverse order inverse).
//
// Butterflies are lazy (Harvey): forward values stay in [0, 4q), inverse
// values in [0, 2q); the last launch reduces to [0, q) (and scales by n^-1).
#include "hc_internal.h"

namespace hc {

template <typename T> struct Ar;

template <> struct Ar<uint64_t> {
    typedef ulonglong2 Pair;
    static __device__ __forceinline__ uint64_t shoup_lazy(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
        return x * w - __umul64hi(x, wp) * q;
    }
    static __device__ __forceinline__ void load_pair(const uint64_t* p, uint64_t& w, uint64_t& wp) {
        ulonglong2 v = *reinterpret_cast<const ulonglong2*>(p);
        w = v.x;
        wp = v.y;
    }
};

template <> struct Ar<uint32_t> {
    static __device__ __forceinline__ uint32_t shoup_lazy(uint32_t x, uint32_t w, uint32_t wp, uint32_t q) {
        return x * w - __umulhi(x, wp) * q;
    }
    static __device__ __forceinline__ void load_pair(const uint32_t* p, uint32_t& w, uint32_t& wp) {
        uint2 v = *reinterpret_cast<const uint2*>(p);
        w = v.x;
        wp = v.y;
    }
};

template <typename T>
__device__ __forceinline__ T csubT(T x, T q) { return x >= q ? x - q : x; }

// Tables for one prime: [2 directions][n][2] = (w, w') pairs, forward then
// inverse; plus n^-1 and its Shoup constant.
template <typename T> struct NttTab {
    const T* base;  // [nprime][2][n][2]
    const T* ninv;  // [nprime][2]
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
    // The pass over the low index bits of a two-pass ring reads twiddles that differ
    // from thread to thread (up to one per butterfly in the last stages). They come
    // from a copy of the table laid out in the order the threads consume them,
    // [tile][ord][thread], so each load instruction reads one contiguous run.
    static constexpr bool TW2 = sizeof(T) == 8 && BLO == 0 && LOGN > TILE_LOG;
    static constexpr int round_r(int done) { return (S - done) >= NTT_EPT_LOG ? NTT_EPT_LOG : (S - done); }
    static constexpr int round_tw(int r) { return (NTT_EPT >> r) * ((1 << r) - 1); }
    static constexpr int tw_before(int done) {
        int o = 0;
        for (int d = 0; d < done; d += round_r(d)) o += round_tw(round_r(d));
        return o;
    }
    static constexpr int TW_PASS = tw_before(S);  // twiddle pairs per thread over the pass
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

    // one round of R stages; butterfly bits [KBIT, KBIT+R) of k; DONE stages before it
    template <int R, int KBIT, int DONE>
    static __device__ __forceinline__ void round(T* lds, uint32_t sp0, const T* tw, const T* tw2, T q) {
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
            const uint32_t j0 = gidx(insert_bits(g, 0, POS, R), sp0);
            const T twoq = q << 1;
            #pragma unroll
            for (int u = 0; u < R; u++) {
                const int st = ST0 + DONE + u;
                if (!INV) {
                    // partner bit R-1-u of v; twiddle 2^st + (j0 >> (LOGN-st)) + (v >> (R-u))
                    const int half = 1 << (R - 1 - u);
                    uint32_t base = (1u << st) + (j0 >> (LOGN - st));
                    if constexpr (round_uniform(KBIT, R, DONE)) base = __builtin_amdgcn_readfirstlane(base);
                    T w[8], wp[8];
                    #pragma unroll
                    for (int t = 0; t < (1 << u); t++) {
                        if constexpr (TW2)
                            Ar<T>::load_pair(tw2 + 2 * ((size_t)(tw_before(DONE) + sub * ((1 << R) - 1) +
                                                                 tw_off(R, u) + t) * THREADS + threadIdx.x),
                                             w[t], wp[t]);
                        else
                            Ar<T>::load_pair(tw + 2 * (base + t), w[t], wp[t]);
                    }
                    #pragma unroll
                    for (int v = 0; v < GS; v++) {
                        if (!(v & half)) {
                            const int t = v >> (R - u);
                            T X = csubT<T>(x[v], twoq);
                            T y = Ar<T>::shoup_lazy(x[v | half], w[t], wp[t], q);
                            x[v] = X + y;
                            x[v | half] = X - y + twoq;
                        }
                    }
                } else {
                    // partner bit u of v; twiddle n/2^(st+1) + (j0 >> (st+1)) + (v >> (u+1))
                    const int half = 1 << u;
                    uint32_t base = ((uint32_t)N >> (st + 1)) + (j0 >> (st + 1));
                    if constexpr (round_uniform(KBIT, R, DONE)) base = __builtin_amdgcn_readfirstlane(base);
                    T w[8], wp[8];
                    #pragma unroll
                    for (int t = 0; t < (1 << (R - 1 - u)); t++) {
                        if constexpr (TW2)
                            Ar<T>::load_pair(tw2 + 2 * ((size_t)(tw_before(DONE) + sub * ((1 << R) - 1) +
                                                                 tw_off(R, u) + t) * THREADS + threadIdx.x),
                                             w[t], wp[t]);
                        else
                            Ar<T>::load_pair(tw + 2 * (base + t), w[t], wp[t]);
                    }
                    #pragma unroll
                    for (int v = 0; v < GS; v++) {
                        if (!(v & half)) {
                            const int t = v >> (u + 1);
                            T X = x[v], Y = x[v | half];
                            x[v] = csubT<T>(X + Y, twoq);
                            x[v | half] = Ar<T>::shoup_lazy(X + twoq - Y, w[t], wp[t], q);
                        }
                    }
                }
            }
            #pragma unroll
            for (int v = 0; v < GS; v++) lds[lb + v * VSTEP] = x[v];
        }
    }

    // rounds: forward processes k bits from the top down, inverse from the bottom up
    template <int DONE>
    static __device__ __forceinline__ void rounds(T* lds, uint32_t sp0, const T* tw, const T* tw2, T q) {
        if constexpr (DONE < S) {
            constexpr int R = round_r(DONE);
            constexpr int KBIT = INV ? DONE : (S - DONE - R);
            round<R, KBIT, DONE>(lds, sp0, tw, tw2, q);
            __syncthreads();
            rounds<DONE + R>(lds, sp0, tw, tw2, q);
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
            for (int sub = 0; sub < PER; sub++) {
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

// WPE: minimum waves per SIMD the registers must allow (1 = no constraint); the second
// pass of each direction (forward low bits, inverse high bits) fits four waves (128
// registers) without spills, the first passes would spill.
template <typename T, bool INV, int LOGN, int S, int BLO, int ST0, bool LAST, int WPE>
__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(WPE)))
ntt_tile_kernel(T* __restrict__ data, size_t poly_stride, int limb_first, NttTab<T> tab) {
    typedef Tile<T, INV, LOGN, S, BLO, ST0> TL;
    __shared__ T lds[TL::LDS_WORDS];
    const int row = blockIdx.z;  // limb; polynomials along y, so consecutive blocks of one
                                 // XCD share a (prime, tile) and its twiddles stay in L2
    const int prime = limb_first + row;
    const T q = tab.mods[prime];
    const T* tw = tab.base + ((size_t)prime * 2 + (INV ? 1 : 0)) * 2 * TL::N;
    T* a = data + (size_t)blockIdx.y * poly_stride + (size_t)row * TL::N;
    const uint32_t sp0 = blockIdx.x * TL::P;

    constexpr int THREADS = TL::TSIZE / NTT_EPT;  // the launch's block size
    // load in global-contiguous order
    #pragma unroll
    for (int i = 0; i < NTT_EPT; i++) {
        const uint32_t f = threadIdx.x + i * THREADS;
        uint32_t k, spl;
        if (BLO == 0) { spl = f >> S; k = f & ((1u << S) - 1u); }
        else { k = f >> TL::LOGP; spl = f & (TL::P - 1); }
        const uint32_t e = (k << TL::LOGP) | spl;
        lds[TL::lpos(e)] = a[TL::gidx(e, sp0)];
    }
    __syncthreads();
    const T* tw2 = nullptr;
    if constexpr (TL::TW2)
        tw2 = tab.tw2 + (((size_t)prime * 2 + (INV ? 1 : 0)) * gridDim.x + blockIdx.x) * (size_t)TL::TW_PASS *
                            TL::THREADS * 2;
    TL::template rounds<0>(lds, sp0, tw, tw2, q);

    const T* ni = tab.ninv + 2 * prime;
    #pragma unroll
    for (int i = 0; i < NTT_EPT; i++) {
        const uint32_t f = threadIdx.x + i * THREADS;
        uint32_t k, spl;
        if (BLO == 0) { spl = f >> S; k = f & ((1u << S) - 1u); }
        else { k = f >> TL::LOGP; spl = f & (TL::P - 1); }
        const uint32_t e = (k << TL::LOGP) | spl;
        T v = lds[TL::lpos(e)];
        if (LAST) {
            if (INV) v = csubT<T>(Ar<T>::shoup_lazy(v, ni[0], ni[1], q), q);
            else { v = csubT<T>(v, q << 1); v = csubT<T>(v, q); }
        }
        a[TL::gidx(e, sp0)] = v;
    }
}

// Launch one pass; `ops` butterflies and `bytes` moved for the timing record.
template <typename T, bool INV, int LOGN, int S, int BLO, int ST0, bool LAST>
static void pass(const Ctx& c, int kind, T* data, size_t stride, int count, int lf, int nl,
                 NttTab<T> tab, hipStream_t st) {
    constexpr int TLOG = LOGN < TILE_LOG ? LOGN : TILE_LOG;
    constexpr int THREADS = (1 << TLOG) / NTT_EPT;
    static_assert(THREADS <= NTT_THREADS, "tile");
    dim3 grid(1 << (LOGN - TLOG), count, nl);
    const double bytes = 2.0 * sizeof(T) * (double)count * nl * (1 << LOGN);
    const double ops = (double)count * nl * (1 << (LOGN - 1)) * S;
    constexpr int WPE = (sizeof(T) == 8 && LOGN > TILE_LOG && (INV ? BLO != 0 : BLO == 0)) ? 4 : 1;
    auto launch = [&]() {
        hipLaunchKernelGGL((ntt_tile_kernel<T, INV, LOGN, S, BLO, ST0, LAST, WPE>), grid, dim3(THREADS), 0, st, data,
                           stride, lf, tab);
    };
    if (kind >= 0) {
        TimeScope ts(c, kind, st, bytes, ops);
        launch();
    } else {
        launch();
    }
}

template <typename T, bool INV, int LOGN>
static void run_logn(const Ctx& c, int kind, T* data, size_t stride, int count, int lf, int nl,
                     NttTab<T> tab, hipStream_t st) {
    if constexpr (LOGN <= TILE_LOG) {
        pass<T, INV, LOGN, LOGN, 0, 0, true>(c, kind, data, stride, count, lf, nl, tab, st);
    } else {
        constexpr int SL = 8, SH = LOGN - 8;
        if (!INV) {
            pass<T, false, LOGN, SH, SL, 0, false>(c, kind, data, stride, count, lf, nl, tab, st);
            pass<T, false, LOGN, SL, 0, SH, true>(c, kind, data, stride, count, lf, nl, tab, st);
        } else {
            pass<T, true, LOGN, SL, 0, 0, false>(c, kind, data, stride, count, lf, nl, tab, st);
            pass<T, true, LOGN, SH, SL, SL, true>(c, kind, data, stride, count, lf, nl, tab, st);
        }
    }
}

template <typename T, bool INV>
static void run_ntt(const Ctx& c, int kind, T* data, size_t stride, int count, int lf, int nl,
                    NttTab<T> tab, hipStream_t st) {
    switch (c.logn) {
        case 10: run_logn<T, INV, 10>(c, kind, data, stride, count, lf, nl, tab, st); break;
        case 11: run_logn<T, INV, 11>(c, kind, data, stride, count, lf, nl, tab, st); break;
        case 12: run_logn<T, INV, 12>(c, kind, data, stride, count, lf, nl, tab, st); break;
        case 13: run_logn<T, INV, 13>(c, kind, data, stride, count, lf, nl, tab, st); break;
        case 14: run_logn<T, INV, 14>(c, kind, data, stride, count, lf, nl, tab, st); break;
        case 15: run_logn<T, INV, 15>(c, kind, data, stride, count, lf, nl, tab, st); break;
        case 16: run_logn<T, INV, 16>(c, kind, data, stride, count, lf, nl, tab, st); break;
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
    const size_t words = (size_t)c.nq * 2 * tiles * TF::TW_PASS * TF::THREADS * 2;
    HC_CHECK(hipMalloc((void**)&c.d_tw2, sizeof(uint64_t) * words));
    c.owned.push_back(c.d_tw2);
    hipLaunchKernelGGL((ntt_tw2_kernel<false, LOGN>), dim3(tiles, c.nq), dim3(TF::THREADS), 0, 0, c.d_tw2, c.d_tw);
    hipLaunchKernelGGL((ntt_tw2_kernel<true, LOGN>), dim3(tiles, c.nq), dim3(TI::THREADS), 0, 0, c.d_tw2, c.d_tw);
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
           bool inverse, hipStream_t stream) {
    if (count <= 0 || nlimbs <= 0) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods, c.d_tw2};
    if (inverse) run_ntt<uint64_t, true>(c, HC_KT_NTT_INV, data, poly_stride, count, limb_first, nlimbs, tab, stream);
    else run_ntt<uint64_t, false>(c, HC_KT_NTT_FWD, data, poly_stride, count, limb_first, nlimbs, tab, stream);
}

void ntt32(const Ctx& c, uint32_t* data, int count, bool inverse, hipStream_t stream) {
    if (count <= 0) return;
    NttTab<uint32_t> tab{c.d_twp, c.d_ninvp, c.d_modp, nullptr};
    if (inverse) run_ntt<uint32_t, true>(c, -1, data, (size_t)c.n, count, 0, 1, tab, stream);
    else run_ntt<uint32_t, false>(c, -1, data, (size_t)c.n, count, 0, 1, tab, stream);
}

}  // namespace hc
