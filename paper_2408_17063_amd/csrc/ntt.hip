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
// A launch runs S consecutive stages on tiles held in LDS. The stages touch
// the index bits [blo, blo+S); a tile is P independent sub-problems (values
// of the other bits) times the 2^S elements of each. Every thread owns 16
// elements per round and runs up to 4 stages in registers between LDS
// exchanges. Rings up to 2^12 take one launch per transform; larger rings
// take two (high bits, then the low 8 bits for the forward direction, the
// reverse order for the inverse).
//
// Butterflies are lazy (Harvey): forward values stay in [0, 4q), inverse
// values in [0, 2q); the last launch reduces to [0, q).
#include "hc_internal.h"

namespace hc {

template <typename T> struct Ar;

template <> struct Ar<uint64_t> {
    static __device__ __forceinline__ uint64_t shoup_lazy(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
        return x * w - __umul64hi(x, wp) * q;
    }
};

template <> struct Ar<uint32_t> {
    static __device__ __forceinline__ uint32_t shoup_lazy(uint32_t x, uint32_t w, uint32_t wp, uint32_t q) {
        return x * w - __umulhi(x, wp) * q;
    }
};

template <typename T>
__device__ __forceinline__ T csubT(T x, T q) { return x >= q ? x - q : x; }

// Tables for one prime: fwd W, fwd W', inv W, inv W' (each n entries), plus
// n^-1 and its Shoup constant.
template <typename T> struct NttTab {
    const T* base;  // [nprime][4][n]
    const T* ninv;  // [nprime][2]
    const T* mods;  // [nprime]
};

constexpr int NTT_TILE_LOG = 12;          // 4096 elements per tile (32 KiB for u64)
constexpr int NTT_THREADS = (1 << NTT_TILE_LOG) / 16;

__device__ __forceinline__ uint32_t insert_bits(uint32_t g, uint32_t v, int pos, int width) {
    uint32_t lowmask = (1u << pos) - 1u;
    return ((g >> pos) << (pos + width)) | (v << pos) | (g & lowmask);
}

// data: polynomial-major, each polynomial `nl` rows of n residues; row r of
// polynomial c uses prime index limb_first + r.
template <typename T, bool INVERSE>
__global__ void __launch_bounds__(NTT_THREADS)
ntt_pass_kernel(T* __restrict__ data, size_t poly_stride, int limb_first, int logn, int blo, int S,
                int stage0, int last, NttTab<T> tab) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);

    const int n = 1 << logn;
    const int row = blockIdx.y;
    const int poly = blockIdx.z;
    const int prime = limb_first + row;
    const T q = tab.mods[prime];
    const T* W = tab.base + (size_t)prime * 4 * n + (INVERSE ? 2 * n : 0);
    const T* Wp = W + n;
    T* a = data + (size_t)poly * poly_stride + (size_t)row * n;

    const int tile_log = (logn < NTT_TILE_LOG) ? logn : NTT_TILE_LOG;
    const int tile = 1 << tile_log;
    const int logP = tile_log - S;
    const int P = 1 << logP;
    const uint32_t sp0 = blockIdx.x * P;
    const uint32_t blomask = (1u << blo) - 1u;
    const int nthreads = blockDim.x;

    // global index of tile element e = (k << logP) | spl
    auto gidx = [&](uint32_t e) -> uint32_t {
        uint32_t k = e >> logP;
        uint32_t sp = sp0 + (e & (P - 1));
        return ((sp >> blo) << (blo + S)) | (k << blo) | (sp & blomask);
    };

    // load, in global-contiguous order
    for (int f = threadIdx.x; f < tile; f += nthreads) {
        uint32_t k, spl;
        if (blo == 0) { spl = f >> S; k = f & ((1 << S) - 1); }
        else { k = f >> logP; spl = f & (P - 1); }
        uint32_t e = (k << logP) | spl;
        lds[e] = a[gidx(e)];
    }
    __syncthreads();

    int done = 0;
    while (done < S) {
        const int R = (S - done) >= 4 ? 4 : (S - done);
        const int gsize = 1 << R;
        // butterfly bits of k for this round
        const int kbit = INVERSE ? done : (S - done - R);
        const int pos = logP + kbit;
        const int ngroups = tile >> R;
        for (int g = threadIdx.x; g < ngroups; g += nthreads) {
            T x[16];
            uint32_t e0 = insert_bits(g, 0, pos, R);
            #pragma unroll
            for (int v = 0; v < 16; v++)
                if (v < gsize) x[v] = lds[insert_bits(g, v, pos, R)];
            const uint32_t j0 = gidx(e0);  // global index with the butterfly bits zero
            if (!INVERSE) {
                // stages st = stage0 + done .. + R-1, partner bit (within v) R-1-u
                #pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (u < R) {
                        const int st = stage0 + done + u;
                        const int hb = R - 1 - u;       // partner bit in v
                        const int half = 1 << hb;
                        #pragma unroll
                        for (int v = 0; v < 16; v++) {
                            if (v < gsize && !(v & half)) {
                                // global index of element v: j0 | (v << (blo + kbit))
                                uint32_t j = j0 | ((uint32_t)v << (blo + kbit));
                                uint32_t widx = (1u << st) + (j >> (logn - st));
                                T w = W[widx], wp = Wp[widx];
                                T X = x[v], Y = x[v | half];
                                T twoq = q << 1;
                                X = csubT<T>(X, twoq);
                                T t = Ar<T>::shoup_lazy(Y, w, wp, q);
                                x[v] = X + t;
                                x[v | half] = X - t + twoq;
                            }
                        }
                    }
                }
            } else {
                #pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (u < R) {
                        const int st = stage0 + done + u;   // partner distance 2^st
                        const int hb = u;
                        const int half = 1 << hb;
                        #pragma unroll
                        for (int v = 0; v < 16; v++) {
                            if (v < gsize && !(v & half)) {
                                uint32_t j = j0 | ((uint32_t)v << (blo + kbit));
                                uint32_t widx = ((uint32_t)n >> (st + 1)) + (j >> (st + 1));
                                T w = W[widx], wp = Wp[widx];
                                T X = x[v], Y = x[v | half];
                                T twoq = q << 1;
                                x[v] = csubT<T>(X + Y, twoq);
                                x[v | half] = Ar<T>::shoup_lazy(X + twoq - Y, w, wp, q);
                            }
                        }
                    }
                }
            }
            #pragma unroll
            for (int v = 0; v < 16; v++)
                if (v < gsize) lds[insert_bits(g, v, pos, R)] = x[v];
        }
        done += R;
        __syncthreads();
    }

    // store (final reduction / scaling on the last launch)
    const T* ninv = tab.ninv + 2 * prime;
    for (int f = threadIdx.x; f < tile; f += nthreads) {
        uint32_t k, spl;
        if (blo == 0) { spl = f >> S; k = f & ((1 << S) - 1); }
        else { k = f >> logP; spl = f & (P - 1); }
        uint32_t e = (k << logP) | spl;
        T v = lds[e];
        if (last) {
            if (INVERSE) v = csubT<T>(Ar<T>::shoup_lazy(v, ninv[0], ninv[1], q), q);
            else { v = csubT<T>(v, q << 1); v = csubT<T>(v, q); }
        }
        a[gidx(e)] = v;
    }
}

template <typename T, bool INVERSE>
static void run_ntt(const Ctx& c, T* data, size_t poly_stride, int count, int limb_first, int nlimbs,
                    int logn, NttTab<T> tab, hipStream_t stream) {
    const int n = 1 << logn;
    // timing class (64-bit transforms only), bytes moved and butterflies per pass
    const int kind = sizeof(T) == 8 ? (INVERSE ? HC_KT_NTT_INV : HC_KT_NTT_FWD) : -1;
    const double pass_bytes = 2.0 * sizeof(T) * (double)count * nlimbs * n;
    auto bfly = [&](int S) { return (double)count * nlimbs * (n / 2) * S; };
    const size_t smem = sizeof(T) * (size_t)((logn < NTT_TILE_LOG) ? n : (1 << NTT_TILE_LOG));
    const int threads = ((logn < NTT_TILE_LOG) ? n : (1 << NTT_TILE_LOG)) / 16;
    if (logn <= NTT_TILE_LOG) {
        dim3 grid(1, nlimbs, count);
        if (kind >= 0) {
            TimeScope ts(c, kind, stream, pass_bytes, bfly(logn));
            hipLaunchKernelGGL((ntt_pass_kernel<T, INVERSE>), grid, dim3(threads), smem, stream,
                               data, poly_stride, limb_first, logn, 0, logn, 0, 1, tab);
        } else {
            hipLaunchKernelGGL((ntt_pass_kernel<T, INVERSE>), grid, dim3(threads), smem, stream,
                               data, poly_stride, limb_first, logn, 0, logn, 0, 1, tab);
        }
        return;
    }
    const int S_lo = 8, S_hi = logn - 8;
    const int tiles = n >> NTT_TILE_LOG;
    dim3 grid(tiles, nlimbs, count);
    // pass 1 then pass 2: (blo, S, first stage, last pass?)
    const int fwd[2][4] = {{S_lo, S_hi, 0, 0}, {0, S_lo, S_hi, 1}};
    const int inv[2][4] = {{0, S_lo, 0, 0}, {S_lo, S_hi, S_lo, 1}};
    for (int ps = 0; ps < 2; ps++) {
        const int* a = INVERSE ? inv[ps] : fwd[ps];
        if (kind >= 0) {
            TimeScope ts(c, kind, stream, pass_bytes, bfly(a[1]));
            hipLaunchKernelGGL((ntt_pass_kernel<T, INVERSE>), grid, dim3(threads), smem, stream,
                               data, poly_stride, limb_first, logn, a[0], a[1], a[2], a[3], tab);
        } else {
            hipLaunchKernelGGL((ntt_pass_kernel<T, INVERSE>), grid, dim3(threads), smem, stream,
                               data, poly_stride, limb_first, logn, a[0], a[1], a[2], a[3], tab);
        }
    }
}

void ntt64(const Ctx& c, uint64_t* data, size_t poly_stride, int count, int limb_first, int nlimbs,
           bool inverse, hipStream_t stream) {
    if (count <= 0 || nlimbs <= 0) return;
    NttTab<uint64_t> tab{c.d_tw, c.d_ninv, c.d_mods};
    if (inverse) run_ntt<uint64_t, true>(c, data, poly_stride, count, limb_first, nlimbs, c.logn, tab, stream);
    else run_ntt<uint64_t, false>(c, data, poly_stride, count, limb_first, nlimbs, c.logn, tab, stream);
}

void ntt32(const Ctx& c, uint32_t* data, int count, bool inverse, hipStream_t stream) {
    if (count <= 0) return;
    NttTab<uint32_t> tab{c.d_twp, c.d_ninvp, c.d_modp};
    if (inverse) run_ntt<uint32_t, true>(c, data, (size_t)c.n, count, 0, 1, c.logn, tab, stream);
    else run_ntt<uint32_t, false>(c, data, (size_t)c.n, count, 0, 1, c.logn, tab, stream);
}

}  // namespace hc
