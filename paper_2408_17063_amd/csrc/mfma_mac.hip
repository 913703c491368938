// Diagonal multiply-accumulate on the matrix cores (int8 MFMA), for resident tables.
//
// For every coefficient position x of a limb, the multiply-accumulate of the
// compression (Sec. 5.2: the baby-step/giant-step product of the power-sum matrix with
// the packed vector, Alg. 6) is a small dense product over Z_q,
//     A[row][g](x) = sum_j R[row][j](x) D[j][g](x)   (rows = pairs x 2 components),
// one per x. Each residue is centred (|v| <= q/2 < 2^54) and written in seven balanced
// base-256 digits, v = sum_a v_a 256^a with v_a in [-128, 127]. Then
//     sum_j R D = sum_{s < 13} 256^s C_s,   C_s = sum_{a + b = s} sum_j R_a[j] D_b[j],
// and every C_s is an exact int32 sum of int8 products: v_mfma_i32_16x16x64_i8 computes
// a 16-row x 16-giant x 64-term block of one (a, b) pair at a time. The 13 sums are
// folded into one residue with Montgomery weights W_s = 256^s 2^64 mod q.
//
// Layout of a table (built once by k_diag_digits): 16-byte units
//   D[r][x][t][jb][b][lane]   (t: giant tile of 16, jb: block of 64 terms, b: digit)
// where lane l holds digit b of D(j, g) for g = 16 t + l % 16 and the sixteen terms
// j = 64 jb + 16 (l / 16) + i in byte i. The rotated ciphertexts R come from the split
// words the gather and the baby steps write (Rt[r][tile][pp][j][64][2]); each wave turns
// its rows into the same digit layout in registers (row = l % 16 in place of the giant).
// The instruction pairs byte i of lane group l / 16 of both operands, whatever its own
// order of the 64 terms, so the sum over j is exact for any such assignment.
#include "hc_internal.h"
#include "modarith.h"

namespace hc {

typedef int mf_v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) uint64_t gl_u64;

namespace {

constexpr int MF_ND = 7;              // digits per residue (primes below 2^55)
constexpr int MF_NS = 2 * MF_ND - 1;  // shift classes s = a + b
constexpr int MF_K = 64;              // terms per instruction
constexpr int MF_GT = 16;             // giants per tile
constexpr int MF_XB = 8;              // coefficients per block, one per wave
constexpr int MF_GMAX = 512;          // giants per class (output pointers staged in LDS)
constexpr int MF_RROW = 65;           // words per LDS row of staged rotated ciphertexts
static_assert(2 * 16 * MF_GT * MF_XB <= 128 * MF_RROW, "the output stage fits the staging space");
constexpr uint64_t MF_BIAS = 0x0080808080808080ull;  // 128 in each of the seven digit bytes

// The seven balanced digits of the centred residue of v (v < q < 2^55) as the bytes
// 0..6 of a word (byte 7 zero): u = c + sum_a 128 256^a has the unsigned bytes u_a with
// c = sum_a (u_a - 128) 256^a, and u_a - 128 as an int8 is u_a xor 0x80.
__device__ __forceinline__ uint64_t digit_word(uint64_t v, uint64_t q) {
    const uint64_t c = v > (q >> 1) ? v - q : v;  // two's complement of the centred value
    return (c + MF_BIAS) ^ MF_BIAS;
}

// Digits of four words w[0..3] (terms 4c..4c+3 of a lane) -> dwords d[a]: byte k of d[a]
// is digit a of w[k].
__device__ __forceinline__ void digit_transpose(const uint64_t* w, uint32_t* d) {
    const uint32_t l0 = (uint32_t)w[0], l1 = (uint32_t)w[1], l2 = (uint32_t)w[2], l3 = (uint32_t)w[3];
    const uint32_t h0 = (uint32_t)(w[0] >> 32), h1 = (uint32_t)(w[1] >> 32), h2 = (uint32_t)(w[2] >> 32),
                   h3 = (uint32_t)(w[3] >> 32);
    // perm(hi, lo, sel): byte k of the result is byte sel_k of the 8 bytes {lo, hi}
    // (0..3 from lo, 4..7 from hi)
    const uint32_t x01 = __builtin_amdgcn_perm(l1, l0, 0x05010400u);  // l0.0 l1.0 l0.1 l1.1
    const uint32_t y01 = __builtin_amdgcn_perm(l3, l2, 0x05010400u);
    const uint32_t x23 = __builtin_amdgcn_perm(l1, l0, 0x07030602u);  // l0.2 l1.2 l0.3 l1.3
    const uint32_t y23 = __builtin_amdgcn_perm(l3, l2, 0x07030602u);
    const uint32_t x45 = __builtin_amdgcn_perm(h1, h0, 0x05010400u);
    const uint32_t y45 = __builtin_amdgcn_perm(h3, h2, 0x05010400u);
    const uint32_t x6 = __builtin_amdgcn_perm(h1, h0, 0x07030602u);
    const uint32_t y6 = __builtin_amdgcn_perm(h3, h2, 0x07030602u);
    d[0] = __builtin_amdgcn_perm(y01, x01, 0x05040100u);  // x.0 x.1 y.0 y.1
    d[1] = __builtin_amdgcn_perm(y01, x01, 0x07060302u);  // x.2 x.3 y.2 y.3
    d[2] = __builtin_amdgcn_perm(y23, x23, 0x05040100u);
    d[3] = __builtin_amdgcn_perm(y23, x23, 0x07060302u);
    d[4] = __builtin_amdgcn_perm(y45, x45, 0x05040100u);
    d[5] = __builtin_amdgcn_perm(y45, x45, 0x07060302u);
    d[6] = __builtin_amdgcn_perm(y6, x6, 0x05040100u);
}

}  // namespace

// ------------------------------------------------------------------ table preparation

// One (giant tile t, term block jb) of a table from `ng` x `nj` natural-layout diagonals
// in[(gl nj + jl)][Lc][n] (giant 16 t + gl, term 64 jb + jl; plain residues, NTT domain);
// giants and terms outside are zero. Thread = (limb, coefficient, lane of the unit).
__global__ __launch_bounds__(512) void diag_digits_kernel(mf_v4i* __restrict__ out, const uint64_t* __restrict__ in,
                                                          const uint64_t* __restrict__ mods, int n, int Lc, int Tg,
                                                          int JbT, int t, int jb, int ng, int nj) {
    const int lane = (int)(threadIdx.x & 63);
    const int x = (int)blockIdx.x * MF_XB + (int)(threadIdx.x >> 6);
    const int r = (int)blockIdx.y;
    if (x >= n) return;
    const uint64_t q = mods[r];
    const int gl = lane & 15, kq = lane >> 4;
    const size_t PW = (size_t)Lc * n;
    uint64_t w[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const int jl = 16 * kq + i;
        w[i] = (gl < ng && jl < nj) ? digit_word(in[(size_t)(gl * nj + jl) * PW + (size_t)r * n + x], q) : 0;
    }
    uint32_t d[4][MF_ND];
#pragma unroll
    for (int c4 = 0; c4 < 4; c4++) digit_transpose(w + 4 * c4, d[c4]);
    mf_v4i* o = out + ((((size_t)r * n + x) * Tg + t) * JbT + jb) * MF_ND * 64 + lane;
#pragma unroll
    for (int a = 0; a < MF_ND; a++) o[(size_t)a * 64] = mf_v4i{(int)d[0][a], (int)d[1][a], (int)d[2][a], (int)d[3][a]};
}

bool diag_mfma_fits(const Ctx& c, int Lc, uint32_t Jt, uint32_t G) {
    for (int i = 0; i < Lc; i++)
        if (c.primes[i] >> 55) return false;
    if (Jt == 0 || Jt > 2 * MF_K || G == 0 || G > MF_GMAX) return false;
    const size_t Tg = (G + MF_GT - 1) / MF_GT, Jb = (Jt + MF_K - 1) / MF_K;
    // no more than twice the bytes of the split-word table (padding of small shapes)
    const size_t mf = Tg * MF_GT * Jb * MF_K * MF_ND;
    const size_t va = (size_t)Jt * ((G + DIAG_GC - 1) / DIAG_GC) * DIAG_GC * 8;
    return mf <= 2 * va;
}

size_t diag_mfma_table_bytes(const Ctx& c, int Lc, uint32_t Jt, uint32_t G) {
    const size_t Tg = (G + MF_GT - 1) / MF_GT, Jb = (Jt + MF_K - 1) / MF_K;
    return (size_t)Lc * c.n * Tg * Jb * MF_ND * 64 * 16;
}

void k_diag_digits(const Ctx& c, void* table, const uint64_t* in, uint32_t Jt, uint32_t G, uint32_t t, uint32_t jb,
                   int Lc, hipStream_t st) {
    const int Tg = (int)((G + MF_GT - 1) / MF_GT), JbT = (int)((Jt + MF_K - 1) / MF_K);
    const int ng = (int)std::min<uint32_t>(MF_GT, G - MF_GT * t), nj = (int)std::min<uint32_t>(MF_K, Jt - MF_K * jb);
    hipLaunchKernelGGL(diag_digits_kernel, dim3((unsigned)((c.n + MF_XB - 1) / MF_XB), (unsigned)Lc), dim3(64 * MF_XB),
                       0, st, (mf_v4i*)table, in, c.d_mods, c.n, Lc, Tg, JbT, (int)t, (int)jb, ng, nj);
}

// ------------------------------------------------------------------ multiply-accumulate

struct MfMacArgs {
    int n, L, J, Jp, ga, npairs, npg, Tg, JbT, h;
    uint32_t work, per_xcd;
};

// Block = 8 waves = 8 consecutive coefficients of one limb, and one group of up to 8
// pairs (16 rows). Wave w: coefficient x0 + w. Its rows' digits stay in registers (JB x 7
// fragments); per giant tile it streams the tile's JB x 7 digit fragments of D(x) (two
// tiles ahead of their use), runs JB x 49 MFMAs into 13 accumulators, folds them to
// residues and passes them through LDS so that the block writes runs of 8 coefficients. Blocks are numbered so that the pair groups of one
// coefficient range are consecutive on one XCD (blocks go to XCDs round robin): they read
// the same table words, which the first brings into that XCD's L2.
template <int JB>
__global__ __launch_bounds__(512) void diag_mac_mfma_kernel(uint64_t* const* __restrict__ A,
                                                           const uint64_t* __restrict__ Rt,
                                                           const mf_v4i* __restrict__ D,
                                                           const uint64_t* __restrict__ mods,
                                                           const uint64_t* __restrict__ qinv,
                                                           const uint64_t* __restrict__ wts, MfMacArgs a) {
    // LDS: the rotated-ciphertext staging (128 rows of MF_RROW words), then the output
    // stage [2][16 rows][16 giants][8 coefficients] in the same space
    __shared__ uint64_t lbuf[128 * MF_RROW];
    __shared__ uint64_t* aout[8 * MF_GMAX];  // the block's output pointers [pair][giant]
    const uint32_t bid = blockIdx.x;
    const uint32_t wk = (bid & 7u) * a.per_xcd + (bid >> 3);
    if (wk >= a.work) return;  // uniform over the block
    const int pg = (int)(wk % (uint32_t)a.npg);
    const uint32_t xr = wk / (uint32_t)a.npg;
    const int nxb = a.n / MF_XB;
    const int xb = (int)(xr % (uint32_t)nxb), r = (int)(xr / (uint32_t)nxb);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int x0 = xb * MF_XB, x = x0 + w;
    const uint64_t q = mods[r], qi = qinv[r];
    const int n = a.n;

    // the output pointers first: waiting for them later waits for nothing else
    const int nap = 8 * a.ga;
    uint64_t* apv[8 * MF_GMAX / 512];
#pragma unroll
    for (int k = 0; k < 8 * MF_GMAX / 512; k++) {
        const int i = (int)threadIdx.x + 512 * k;
        const size_t ia = (size_t)pg * 8 * a.ga + i, last = (size_t)a.npairs * a.ga - 1;
        uint64_t* const ap = A[ia < last ? ia : last];
        apv[k] = ia <= last && i < nap ? ap : nullptr;
    }

    // Loads in the order they are needed: the wave's rotated-ciphertext words, then the
    // first giant tile of its table words (so both latencies overlap), then -- after the
    // words are turned into digits -- the second tile. Two register slots of tile
    // fragments: a slot is refilled with the tile two ahead right after its products.
    const size_t per_t = (size_t)a.JbT * MF_ND * 64;
    const mf_v4i* Dx = D + ((size_t)r * n + x) * (size_t)a.Tg * per_t + lane;
    mf_v4i B0[JB][MF_ND], B1[JB][MF_ND];
    // Every load is issued unconditionally (tiles past the last read the table's first
    // words, which stay in L2), so the compiler's wait counts stay exact across the loop.
    auto loadB = [&](mf_v4i(&Bs)[JB][MF_ND], int t) __attribute__((always_inline)) {
        const mf_v4i* Dt = t < a.Tg ? Dx + (size_t)t * per_t : D + lane;
#pragma unroll
        for (int jb = 0; jb < JB; jb++)
#pragma unroll
            for (int b = 0; b < MF_ND; b++) Bs[jb][b] = Dt[((size_t)jb * MF_ND + b) * 64];
    };

    // The wave's rows as the A operand: row m = lane % 16 (pair 8 pg + m / 2, component
    // m % 2), terms j = 64 jb + 16 (lane / 16) + i. The block's words of a 64-term block
    // (8 pairs x 64 terms x its 8 coefficients x 2 components: 128-byte lines) are read
    // whole, 16 bytes per thread, and staged in LDS as rows (w, i) of 64 words in lane
    // order (padded to 65), so that a wave then reads 64 consecutive words per term.
    mf_v4i Aop[JB][MF_ND];
    {
        ulonglong2 rp[JB][8];
        const ulonglong2 zero2{0, 0};
#pragma unroll
        for (int jb = 0; jb < JB; jb++)
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const int idx = k * 512 + (int)threadIdx.x, part = idx & 7, line = idx >> 3;
                const int ppl = line & 7, jl = line >> 3;
                const int pp = pg * 8 + ppl, j = MF_K * jb + jl;
                const bool ok = pp < a.npairs && j < a.Jp;
                const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(
                    Rt + ((((size_t)r * (n / 64) + (x0 >> 6)) * a.npairs + (ok ? pp : 0)) * a.Jp + (ok ? j : 0)) * 128 +
                    2 * (x0 & 63) + 2 * part);
                rp[jb][k] = ok ? v : zero2;
            }
        loadB(B0, 0);
#pragma unroll
        for (int k = 0; k < 8 * MF_GMAX / 512; k++) {
            const int i = (int)threadIdx.x + 512 * k;
            if (i < nap) aout[i] = apv[k];  // read after the first step's barrier
        }
        const uint64_t mask = (1ull << a.h) - 1;
#pragma unroll
        for (int jb = 0; jb < JB; jb++) {
            if (jb) __syncthreads();  // the previous block's rows are read
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const int idx = k * 512 + (int)threadIdx.x, part = idx & 7, line = idx >> 3;
                const int ppl = line & 7, jl = line >> 3;
                uint64_t* dst = lbuf + (part * 16 + (jl & 15)) * MF_RROW + (jl >> 4) * 16 + ppl * 2;
                dst[0] = rp[jb][k].x;
                dst[1] = rp[jb][k].y;
            }
            __syncthreads();
            uint64_t wv[16];
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const uint64_t sw = lbuf[(w * 16 + i) * MF_RROW + lane];
                wv[i] = digit_word(((sw >> 32) << a.h) | (sw & mask), q);  // zero stays zero
            }
            uint32_t d[4][MF_ND];
#pragma unroll
            for (int c4 = 0; c4 < 4; c4++) digit_transpose(wv + 4 * c4, d[c4]);
#pragma unroll
            for (int b = 0; b < MF_ND; b++) Aop[jb][b] = mf_v4i{(int)d[0][b], (int)d[1][b], (int)d[2][b], (int)d[3][b]};
        }
        __syncthreads();  // the staging space becomes the output stage
    }
    loadB(B1, 1);

    // fold weights W_s = 256^s 2^64 mod q, split W = wh 2^31 + wl (both below 2^31)
    int32_t wl[MF_NS], wh[MF_NS];
#pragma unroll
    for (int s = 0; s < MF_NS; s++) {
        const uint64_t W = wts[(size_t)r * 16 + s];
        wl[s] = (int32_t)(W & 0x7fffffffu);
        wh[s] = (int32_t)(W >> 31);
    }
    const uint64_t q35lo = q << 35, q35hi = q >> 29;
    const size_t ln = (size_t)a.L * n;

    auto step = [&](mf_v4i(&Bs)[JB][MF_ND], int t) __attribute__((always_inline)) {
        mf_v4i acc[MF_NS];
#pragma unroll
        for (int s = 0; s < MF_NS; s++) acc[s] = mf_v4i{0, 0, 0, 0};
#pragma unroll
        for (int jb = 0; jb < JB; jb++)
#pragma unroll
            for (int b = 0; b < MF_ND; b++)
#pragma unroll
                for (int aa = 0; aa < MF_ND; aa++)
                    acc[aa + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Aop[jb][aa], Bs[jb][b], acc[aa + b], 0, 0, 0);
        loadB(Bs, t + 2);
        // fold: lane holds rows 4 (lane / 16) + i, giant 16 t + lane % 16. T = sum_s C_s W_s
        // (|C_s| <= 7 J 2^14 < 2^24 for J <= 128, so |T| < 13 2^24 q) plus q 2^35 is in
        // (0, q 2^64): one REDC gives sum_s C_s 256^s mod q.
        uint64_t* stg = lbuf + (t & 1) * (16 * MF_GT * MF_XB);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            int64_t lo = 0, hi = 0;
#pragma unroll
            for (int s = 0; s < MF_NS; s++) {
                lo += (int64_t)acc[s][i] * (int64_t)wl[s];
                hi += (int64_t)acc[s][i] * (int64_t)wh[s];
            }
            // T = hi 2^31 + lo + q 2^35 as 128 bits
            u128p T{(uint64_t)hi << 31, (uint64_t)(hi >> 33)};
            add128(T, u128p{(uint64_t)lo, (uint64_t)(lo >> 63)});
            add128(T, u128p{q35lo, q35hi});
            const int row = 4 * (lane >> 4) + i;
            stg[(row * MF_GT + (lane & 15)) * MF_XB + w] = redc(T, q, qi);
        }
        // A stage buffer is rewritten two tiles later, after the next barrier, which every
        // thread reaches only once its writes from this one are done.
        __syncthreads();
        // runs of 8 coefficients: thread -> (row, giant) = tid / 2, half tid % 2
        const int run = (int)(threadIdx.x >> 1), half = (int)(threadIdx.x & 1);
        const int row = run >> 4, gl = run & 15;
        const int pp = pg * 8 + (row >> 1), g = t * MF_GT + gl;
        if (pp < a.npairs && g < a.ga) {
            const uint64_t* sv = stg + (row * MF_GT + gl) * MF_XB + 4 * half;
            // a global (not generic) store: generic ones also count as LDS accesses, which
            // blurs the wait counts of the loads in flight
            gl_u64* dst = (gl_u64*)(aout[(row >> 1) * a.ga + g] + (row & 1) * ln + (size_t)r * n + x0 + 4 * half);
            dst[0] = sv[0];
            dst[1] = sv[1];
            dst[2] = sv[2];
            dst[3] = sv[3];
        }
    };
    for (int t = 0; t < a.Tg; t += 2) {
        step(B0, t);
        if (t + 1 < a.Tg) step(B1, t + 1);
    }
}

hc_status k_diag_mac_mfma(const Ctx& c, uint64_t* const* A, const uint64_t* Rt, const void* D, uint32_t Jt, int npairs,
                          int J, int ga, int Lc, hipStream_t st) {
    if (J <= 0 || J > 2 * MF_K || (uint32_t)J > Jt || npairs <= 0 || ga <= 0 || ga > MF_GMAX || c.n % 64)
        return HC_EINVAL;
    for (int i = 0; i < Lc; i++)
        if (c.primes[i] >> 55) return HC_EINVAL;
    MfMacArgs a;
    a.n = c.n;
    a.L = Lc;
    a.J = J;
    a.Jp = diag_terms_padded(J);
    a.ga = ga;
    a.npairs = npairs;
    a.npg = (npairs + 7) / 8;
    a.Tg = (ga + MF_GT - 1) / MF_GT;
    a.JbT = (int)((Jt + MF_K - 1) / MF_K);
    a.h = diag_split_h(c, Lc);
    const uint64_t work = (uint64_t)Lc * (c.n / MF_XB) * a.npg;
    a.work = (uint32_t)work;
    a.per_xcd = (uint32_t)((work + 7) / 8);
    const double ln = (double)Lc * c.n;
    // reads each table digit byte, each R word (both components) and writes each A once
    TimeScope ts(c, HC_KT_DIAG_MAC, st, ln * ((double)MF_ND * J * ga + 16.0 * npairs * J + 16.0 * npairs * ga),
                 2.0 * ln * npairs * J * ga);
    const int JB = (J + MF_K - 1) / MF_K;
    if (JB == 1)
        hc_launch((diag_mac_mfma_kernel<1>), dim3(a.per_xcd * 8), dim3(512), 0, st, A, Rt, (const mf_v4i*)D,
                           c.d_mods, c.d_qinv, c.d_mfw, a);
    else
        hc_launch((diag_mac_mfma_kernel<2>), dim3(a.per_xcd * 8), dim3(512), 0, st, A, Rt, (const mf_v4i*)D,
                           c.d_mods, c.d_qinv, c.d_mfw, a);
    return HC_OK;
}

}  // namespace hc
