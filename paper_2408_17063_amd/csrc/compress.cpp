// The compression map on the device: Mask (Alg. 7 step 2) and the SIMD-aware
// Vandermonde product (Alg. 7 step 3, Eq. (1), Sec. 5.2), plus its planner.
//
// Plan (a pure function of n, p, N, ncol, t_bound):
//  * s = 2^ceil(log2 t_bound); records split into G = ceil(n_ct / ((p-1)/n))
//    balanced groups of whole ciphertexts so every group has < p records;
//    a record's Vandermonde column is its 1-based index inside its group;
//  * streams: the vectors [v, d_1, .., d_ncol] in pairs (a, b);
//  * u-block beta of a (group, stream) covers group-local records
//    [beta n/2, (beta+1) n/2): row 0 of ciphertext beta/2 for even beta,
//    row 1 for odd beta, packed as u = [a-part; b-part] with the row masks and
//    Rot_col exactly as the paper's u_1 / u_2 (Sec. 5.2);
//  * baby-step/giant-step: B = the power of two in [1, s] minimising
//    k (B-1) + (s/B - 1), ties to the larger B; baby rotations hoisted;
//  * one rotate-and-sum after all blocks are summed (Sec. 5.2), shifts
//    s, 2s, .., n/4;
//  * bands g*streams + sigma merged into one ciphertext (prefix mask, rotation
//    by -band*s) when there is more than one.
//
// Device flow: inputs -> NTT domain; Mask; u-blocks; hoisted baby steps;
// diagonals encoded on the fly in chunks of giant indices and accumulated by
// one multiply-accumulate kernel that serves every (group, stream) pair with
// the same B at once; giant-step rotations; rotate-and-sum; merge; back to the
// coefficient domain.
#include <string.h>

#include <algorithm>
#include <set>

#include "he.h"

namespace hc {

struct PlanGroup {
    uint32_t ct_start, ct_count;
    uint64_t rec_start, n_rec;
    uint32_t k, B;
};

struct Plan {
    uint32_t s = 0, n_ct = 0, ncol = 0;
    int level = 0;  // ciphertext primes kept for Comp (modulus switched after Mask)
    uint64_t N = 0;
    std::vector<PlanGroup> groups;
    std::vector<std::pair<int, int>> streams;  // vector ids (0 = v, c = d_c), -1 = none
    std::vector<uint32_t> keys;
    uint32_t bands = 0;
    uint32_t n_ks = 0;
    uint64_t n_ptct = 0, n_diag = 0;
};

static uint32_t rot_elt(const Ctx& c, int64_t r) {
    int64_t nh = c.nh;
    int64_t rr = ((r % nh) + nh) % nh;
    return (uint32_t)h_powmod(3, (uint64_t)rr, 2ull * c.n);
}

static uint32_t choose_B(uint32_t s, uint32_t k) {
    uint64_t best = ~0ull;
    uint32_t bestB = 1;
    for (uint32_t B = 1; B <= s; B *= 2) {
        uint64_t cost = (uint64_t)k * (B - 1) + (s / B - 1);
        if (cost <= best) { best = cost; bestB = B; }
    }
    return bestB;
}

// Default level of Comp: the smallest multiple of the digit size that is at least 2 primes.
static int default_level(const Ctx& c) {
    int lvl = c.alpha * ((2 + c.alpha - 1) / c.alpha);
    return lvl < c.L ? lvl : c.L;
}

hc_status make_plan(const Ctx& c, uint64_t N, uint32_t ncol, uint32_t t_bound, uint32_t comp_level,
                    Plan& pl) {
    if (N == 0 || t_bound == 0) return HC_EINVAL;
    if (comp_level == 0) pl.level = default_level(c);
    else if ((int)comp_level > c.L || comp_level % c.alpha) return HC_EINVAL;
    else pl.level = (int)comp_level;
    uint32_t s = 1;
    while (s < t_bound) s *= 2;
    if (s > (uint32_t)c.nh) return HC_EINVAL;
    const uint64_t n = c.n, nh = c.nh;
    pl.s = s;
    pl.N = N;
    pl.ncol = ncol;
    pl.n_ct = (uint32_t)((N + n - 1) / n);
    const uint64_t per_group = (c.p - 1) / n;
    const uint32_t G = (uint32_t)((pl.n_ct + per_group - 1) / per_group);
    uint32_t ct = 0;
    for (uint32_t g = 0; g < G; g++) {
        PlanGroup pg;
        pg.ct_count = pl.n_ct / G + (g < pl.n_ct % G ? 1 : 0);
        pg.ct_start = ct;
        pg.rec_start = (uint64_t)ct * n;
        pg.n_rec = std::min<uint64_t>(N, (uint64_t)(ct + pg.ct_count) * n) - pg.rec_start;
        pg.k = (uint32_t)((pg.n_rec + nh - 1) / nh);
        pg.B = choose_B(s, pg.k);
        pl.groups.push_back(pg);
        ct += pg.ct_count;
    }
    for (uint32_t i = 0; i <= ncol; i += 2) pl.streams.push_back({(int)i, i + 1 <= ncol ? (int)i + 1 : -1});
    pl.bands = (uint32_t)(pl.groups.size() * pl.streams.size());
    if ((uint64_t)pl.bands * s > nh) return HC_EINVAL;

    std::set<uint32_t> keys;
    bool any_b = false;
    for (auto& st : pl.streams) any_b |= st.second >= 0;
    uint32_t fold = 0;
    for (uint64_t sh = s; sh < nh; sh *= 2) { keys.insert(rot_elt(c, (int64_t)sh)); fold++; }
    pl.n_ks = 0;
    pl.n_ptct = (uint64_t)ncol * pl.n_ct;
    for (auto& g : pl.groups) {
        for (uint32_t b = 1; b < g.B; b++) keys.insert(rot_elt(c, b));
        for (uint32_t gi = 1; gi < s / g.B; gi++) keys.insert(rot_elt(c, (int64_t)gi * g.B));
        if (g.k >= 2 || any_b) keys.insert(2u * c.n - 1);
        for (auto& st : pl.streams) {
            bool hb = st.second >= 0;
            for (uint32_t beta = 0; beta < g.k; beta++) {
                bool row0 = (beta % 2) == 0;
                pl.n_ks += row0 ? (hb ? 1 : 0) : 1;           // Rot_col in u-packing
                pl.n_ptct += hb ? 2 : 1;                        // row masks
            }
            pl.n_ks += g.k * (g.B - 1) + (s / g.B - 1) + fold;  // baby, giant, fold
            pl.n_ptct += (uint64_t)g.k * s;                     // diagonals
        }
    }
    for (uint32_t b = 1; b < pl.bands; b++) keys.insert(rot_elt(c, -(int64_t)b * s));
    if (pl.bands > 1) { pl.n_ks += pl.bands - 1; pl.n_ptct += pl.bands; }
    pl.keys.assign(keys.begin(), keys.end());
    // diagonals encoded: per B class, kmax * s
    std::map<uint32_t, uint32_t> kmax;
    for (auto& g : pl.groups) kmax[g.B] = std::max(kmax[g.B], g.k);
    pl.n_diag = 0;
    for (auto& kv : kmax) pl.n_diag += (uint64_t)kv.second * s;
    return HC_OK;
}

static void fill_info(const Plan& pl, hc_compress_info* info) {
    if (!info) return;
    info->s = pl.s;
    info->groups = (uint32_t)pl.groups.size();
    info->streams = (uint32_t)pl.streams.size();
    info->bands = pl.bands;
    info->n_ct = pl.n_ct;
    info->n_keyswitch = pl.n_ks;
    info->n_ptct = pl.n_ptct;
    info->n_diag = pl.n_diag;
    info->level = (uint32_t)pl.level;
}

// bytes of device memory one compression needs beyond its inputs and output
struct Layout {
    size_t ct_words;        // one ciphertext [2][L][n]
    size_t pt_words;        // one plaintext [L][n]
    int npairs;
    uint32_t Gc;            // giant indices per diagonal chunk
    size_t total_bytes;
};

static size_t rup(size_t b) { return (b + 255) & ~(size_t)255; }

// Device-memory budget for the diagonal chunk buffer (plaintexts [L][n] u64).
static const size_t kDiagBudgetBytes = (size_t)16 << 30;

static Layout layout_for(const Ctx& c, const Plan& pl) {
    Layout ly;
    ly.ct_words = 2 * (size_t)pl.level * c.n;   // ciphertexts after the switch
    ly.pt_words = (size_t)pl.level * c.n;
    const size_t full_ct = 2 * (size_t)c.L * c.n;
    ly.npairs = (int)(pl.groups.size() * pl.streams.size());
    uint32_t kmax = 0, Bmax = 1, Gmax = 1;
    size_t ublocks = 0, baby = 0, giants = 0;
    for (auto& g : pl.groups) {
        kmax = std::max(kmax, g.k);
        Bmax = std::max(Bmax, g.B);
        Gmax = std::max(Gmax, pl.s / g.B);
        ublocks += (size_t)g.k * pl.streams.size();
        baby += (size_t)g.k * (g.B - 1) * pl.streams.size();
        giants += (size_t)(pl.s / g.B) * pl.streams.size();
    }
    size_t per_g = (size_t)kmax * Bmax * ly.pt_words * 8;
    uint32_t Gc = (uint32_t)std::max<size_t>(1, kDiagBudgetBytes / std::max<size_t>(per_g, 1));
    Gc = std::min(Gc, Gmax);
    ly.Gc = Gc;
    size_t cnt = (size_t)kmax * Gc * Bmax;  // diagonals per chunk
    size_t t = 0;
    t += rup(full_ct * 8 * pl.n_ct);                                         // inputs in NTT domain
    t += rup(full_ct * 8 * pl.n_ct * std::max<uint32_t>(pl.ncol, 1));       // masked
    t += rup(ly.ct_words * 8 * pl.n_ct * (1 + (size_t)pl.ncol));             // both after the switch
    t += rup(full_ct * 8) + rup(ly.ct_words * 8);                           // switch temporaries
    t += rup(ly.ct_words * 8 * std::max<size_t>(ublocks, 1));               // u-blocks
    t += rup(ly.ct_words * 8 * std::max<size_t>(baby, 1));                  // baby rotations
    t += rup(ly.ct_words * 8 * std::max<size_t>(giants, 1));                // giant accumulators
    t += rup(ly.ct_words * 8 * 4);                           // y, tmp, tmp2, out
    t += rup(ly.pt_words * 8 * cnt);                         // diagonal chunk
    t += rup((size_t)c.n * 4 * cnt);                         // diagonal mod-p stage
    t += rup(cnt * 3 * 4);                                   // diagonal params
    t += rup(sizeof(void*) * ((size_t)ly.npairs * kmax * Bmax + (size_t)ly.npairs * Gmax));
    t += ks_take_bytes(c);
    t += 64 * 256;
    ly.total_bytes = t;
    return ly;
}

struct Compressor {
    Ctx& c;
    const hc_gk* gk;
    hipStream_t st;
    int Lc;
    KSBuf ks;
    hc_status err = HC_OK;

    const uint64_t* key(uint32_t k) {
        const uint64_t* p = find_key(gk, k);
        if (!p && err == HC_OK) err = HC_ENOKEY;
        return p;
    }
    void rot(uint64_t* out, const uint64_t* in, uint32_t k) {
        const uint64_t* kk = key(k);
        if (kk) rotate_plain(c, kk, k, out, in, ks, Lc, st);
    }
    void add(uint64_t* out, const uint64_t* a, const uint64_t* b) {
        k_add(c, out, a, b, 0, Lc, 2, (size_t)Lc * c.n, st);
    }
};

hc_status compress_one(Ctx& c, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v, const Plan& pl,
                       uint64_t* ct_out, hipStream_t st) {
    const size_t n = c.n;
    const Layout ly = layout_for(c, pl);
    const size_t CW = ly.ct_words, PW = ly.pt_words;           // at level Lc
    const size_t CWF = 2 * (size_t)c.L * n, PWF = (size_t)c.L * n;  // at the top level
    const int Lc = pl.level;
    // all keys present?
    for (uint32_t k : pl.keys)
        if (!find_key(gk, k)) return HC_ENOKEY;
    if (pl.ncol && (!db || db->ncol != pl.ncol || db->N != pl.N)) return HC_EINVAL;

    HC_CHECK(hipStreamSynchronize(st));  // the workspace and pointer tables are reused
    if (c.ws.reserve(ly.total_bytes) != HC_OK) return HC_ENOMEM;
    Arena& a = c.ws;
    Compressor cm{c, gk, st, Lc, KSBuf()};
    cm.ks = ks_take(c, a);

    // 1. inputs to the NTT domain
    uint64_t* ctf = a.take<uint64_t>(CWF * pl.n_ct);
    if (!ctf) return HC_ENOMEM;
    HC_CHECK(hipMemcpyAsync(ctf, ct_v, sizeof(uint64_t) * CWF * pl.n_ct, hipMemcpyDeviceToDevice, st));
    ntt64(c, ctf, PWF, 2 * (int)pl.n_ct, 0, c.L, false, st);

    // 2. Mask at the top level: d_c = v boxtimes DB_c per ciphertext
    uint64_t* maskf = a.take<uint64_t>(CWF * pl.n_ct * std::max<uint32_t>(pl.ncol, 1));
    if (!maskf) return HC_ENOMEM;
    for (uint32_t col = 0; col < pl.ncol; col++)
        for (uint32_t i = 0; i < pl.n_ct; i++)
            k_mul_plain(c, maskf + (col * pl.n_ct + i) * CWF, ctf + i * CWF,
                        db->d_pt + ((size_t)col * pl.n_ct + i) * PWF, c.L, st);

    // 3. switch to the Comp level (Sec. 5.3's smaller parameters, as a modulus switch)
    uint64_t *ctv = ctf, *masked = maskf;
    if (Lc < c.L) {
        ctv = a.take<uint64_t>(CW * pl.n_ct * (1 + (size_t)pl.ncol));
        uint64_t* mtmp = a.take<uint64_t>(CWF);
        uint64_t* mconv = a.take<uint64_t>(CW);
        if (!ctv || !mtmp || !mconv) return HC_ENOMEM;
        masked = ctv + CW * pl.n_ct;
        for (uint32_t i = 0; i < pl.n_ct; i++) {
            hc_status s2 = mod_switch(c, ctv + i * CW, ctf + i * CWF, Lc, mtmp, mconv, st);
            if (s2 != HC_OK) return s2;
        }
        for (uint32_t m = 0; m < pl.n_ct * pl.ncol; m++) {
            hc_status s2 = mod_switch(c, masked + m * CW, maskf + m * CWF, Lc, mtmp, mconv, st);
            if (s2 != HC_OK) return s2;
        }
    }
    auto vec_ct = [&](int vid, uint32_t i) -> const uint64_t* {
        return vid == 0 ? ctv + i * CW : masked + ((size_t)(vid - 1) * pl.n_ct + i) * CW;
    };

    // per (group, stream) pair storage
    const int npairs = ly.npairs;
    std::vector<std::vector<uint64_t*>> U(npairs), A(npairs);
    std::vector<std::vector<std::vector<uint64_t*>>> R(npairs);
    size_t ub_total = 0, baby_total = 0, gi_total = 0;
    for (auto& g : pl.groups) {
        ub_total += (size_t)g.k * pl.streams.size();
        baby_total += (size_t)g.k * (g.B - 1) * pl.streams.size();
        gi_total += (size_t)(pl.s / g.B) * pl.streams.size();
    }
    uint64_t* ubuf = a.take<uint64_t>(CW * std::max<size_t>(ub_total, 1));
    uint64_t* bbuf = a.take<uint64_t>(CW * std::max<size_t>(baby_total, 1));
    uint64_t* gbuf = a.take<uint64_t>(CW * std::max<size_t>(gi_total, 1));
    uint64_t* y = a.take<uint64_t>(CW);
    uint64_t* tmp = a.take<uint64_t>(CW);
    uint64_t* tmp2 = a.take<uint64_t>(CW);
    uint64_t* outN = a.take<uint64_t>(CW);
    if (!cm.ks.tmpC || !cm.ks.X || !cm.ks.T || !cm.ks.conv || !ctv || !masked || !ubuf || !bbuf ||
        !gbuf || !y || !tmp || !tmp2 || !outN)
        return HC_ENOMEM;

    // 3. u-blocks and 4. hoisted baby steps
    size_t uo = 0, bo = 0, go = 0;
    int pp = 0;
    for (auto& g : pl.groups) {
        for (auto& sm : pl.streams) {
            U[pp].resize(g.k);
            R[pp].assign(g.k, std::vector<uint64_t*>(g.B, nullptr));
            for (uint32_t beta = 0; beta < g.k; beta++) {
                uint64_t* u = ubuf + (uo++) * CW;
                U[pp][beta] = u;
                uint32_t i = g.ct_start + beta / 2;
                const uint64_t* Act = vec_ct(sm.first, i);
                const uint64_t* Bct = sm.second >= 0 ? vec_ct(sm.second, i) : nullptr;
                if (beta % 2 == 0) {
                    k_mul_plain(c, u, Act, c.d_rowmask[0], Lc, st);
                    if (Bct) {
                        k_mul_plain(c, tmp, Bct, c.d_rowmask[0], Lc, st);
                        cm.rot(tmp2, tmp, 2u * c.n - 1);
                        cm.add(u, u, tmp2);
                    }
                } else {
                    k_mul_plain(c, tmp, Act, c.d_rowmask[1], Lc, st);
                    cm.rot(u, tmp, 2u * c.n - 1);
                    if (Bct) {
                        k_mul_plain(c, tmp, Bct, c.d_rowmask[1], Lc, st);
                        cm.add(u, u, tmp);
                    }
                }
                R[pp][beta][0] = u;
                if (g.B > 1) {
                    hoist_prepare(c, u, cm.ks, Lc, st);
                    for (uint32_t b = 1; b < g.B; b++) {
                        uint64_t* r = bbuf + (bo++) * CW;
                        uint32_t k = rot_elt(c, b);
                        const uint64_t* kk = cm.key(k);
                        if (kk) rotate_hoisted_one(c, kk, k, r, u, cm.ks, Lc, st);
                        R[pp][beta][b] = r;
                    }
                }
            }
            A[pp].resize(pl.s / g.B);
            for (uint32_t gi = 0; gi < pl.s / g.B; gi++) A[pp][gi] = gbuf + (go++) * CW;
            pp++;
        }
    }
    if (cm.err != HC_OK) return cm.err;

    // 5. diagonals + multiply-accumulate, per class of pairs sharing B
    std::set<uint32_t> Bs;
    for (auto& g : pl.groups) Bs.insert(g.B);
    const uint32_t Gc = ly.Gc;
    uint32_t kmax_all = 0;
    for (auto& g : pl.groups) kmax_all = std::max(kmax_all, g.k);
    const size_t max_cnt = (size_t)kmax_all * Gc * (*Bs.rbegin());
    uint64_t* D = a.take<uint64_t>(PW * max_cnt);
    uint32_t* Dp = a.take<uint32_t>((size_t)n * max_cnt);
    uint32_t* prm = a.take<uint32_t>(3 * max_cnt);
    size_t maxG = 1;
    for (auto& g : pl.groups) maxG = std::max<size_t>(maxG, pl.s / g.B);
    uint64_t** ptrs = a.take<uint64_t*>((size_t)npairs * kmax_all * (*Bs.rbegin()) + (size_t)npairs * maxG);
    if (!D || !Dp || !prm || !ptrs) return HC_ENOMEM;
    std::vector<uint32_t> hprm;
    std::vector<uint64_t*> hptr;
    for (uint32_t B : Bs) {
        std::vector<int> cls;
        uint32_t kb = 0;
        for (int q = 0; q < npairs; q++) {
            const PlanGroup& g = pl.groups[q / pl.streams.size()];
            if (g.B == B) { cls.push_back(q); kb = std::max(kb, g.k); }
        }
        const uint32_t G = pl.s / B;
        for (uint32_t g0 = 0; g0 < G; g0 += Gc) {
            uint32_t gc = std::min(Gc, G - g0);
            hprm.clear();
            for (uint32_t beta = 0; beta < kb; beta++)
                for (uint32_t gi = 0; gi < gc; gi++)
                    for (uint32_t b = 0; b < B; b++) {
                        hprm.push_back(beta);
                        hprm.push_back(g0 + gi);
                        hprm.push_back(b);
                    }
            const int cnt = (int)(hprm.size() / 3);
            // R pointers [cls][kb][B], A pointers [cls][gc]
            hptr.assign((size_t)cls.size() * kb * B + cls.size() * gc, nullptr);
            for (size_t ci = 0; ci < cls.size(); ci++) {
                int q = cls[ci];
                for (uint32_t beta = 0; beta < R[q].size(); beta++)
                    for (uint32_t b = 0; b < B; b++) hptr[(ci * kb + beta) * B + b] = R[q][beta][b];
                for (uint32_t gi = 0; gi < gc; gi++)
                    hptr[(size_t)cls.size() * kb * B + ci * gc + gi] = A[q][g0 + gi];
            }
            // synchronous copies: the host vectors are reused for the next chunk
            HC_CHECK(hipMemcpyAsync(prm, hprm.data(), sizeof(uint32_t) * hprm.size(), hipMemcpyHostToDevice, st));
            HC_CHECK(hipMemcpyAsync(ptrs, hptr.data(), sizeof(uint64_t*) * hptr.size(), hipMemcpyHostToDevice, st));
            k_diag_gen(c, Dp, prm, cnt, pl.s, B, st);
            ntt32(c, Dp, cnt, true, st);
            k_lift(c, D, Dp, cnt, true, Lc, st);
            ntt64(c, D, PW, cnt, 0, Lc, false, st);
            k_diag_mac(c, ptrs + (size_t)cls.size() * kb * B, (const uint64_t* const*)ptrs, D,
                       (int)cls.size(), (int)kb, (int)gc, (int)B, false, Lc, st);
            HC_CHECK(hipStreamSynchronize(st));
        }
    }

    // 6. giant steps and rotate-and-sum per pair
    std::vector<uint64_t*> bands;
    uint64_t* band_store = nullptr;
    if (pl.bands > 1) {
        // reuse the u-block buffer for the band results (u-blocks are no longer needed)
        band_store = ubuf;
    }
    pp = 0;
    for (auto& g : pl.groups) {
        for (size_t si = 0; si < pl.streams.size(); si++, pp++) {
            uint64_t* yy = (pl.bands > 1) ? band_store + (size_t)pp * CW : y;
            const uint32_t G = pl.s / g.B;
            HC_CHECK(hipMemcpyAsync(yy, A[pp][0], sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
            for (uint32_t gi = 1; gi < G; gi++) {
                cm.rot(tmp, A[pp][gi], rot_elt(c, (int64_t)gi * g.B));
                cm.add(yy, yy, tmp);
            }
            for (uint64_t sh = pl.s; sh < (uint64_t)c.nh; sh *= 2) {
                cm.rot(tmp, yy, rot_elt(c, (int64_t)sh));
                cm.add(yy, yy, tmp);
            }
            bands.push_back(yy);
        }
    }
    // 7. merge
    uint64_t* res = bands[0];
    if (pl.bands > 1) {
        const uint64_t* ms = nullptr;
        hc_status s2 = prefix_mask(c, pl.s, &ms);
        if (s2 != HC_OK) return s2;
        k_mul_plain(c, outN, bands[0], ms, Lc, st);
        for (uint32_t b = 1; b < pl.bands; b++) {
            k_mul_plain(c, tmp, bands[b], ms, Lc, st);
            cm.rot(tmp2, tmp, rot_elt(c, -(int64_t)b * pl.s));
            cm.add(outN, outN, tmp2);
        }
        res = outN;
    }
    if (cm.err != HC_OK) return cm.err;
    // 8. back to the coefficient domain
    ntt64(c, res, PW, 2, 0, Lc, true, st);
    HC_CHECK(hipMemcpyAsync(ct_out, res, sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
    HC_CHECK(hipGetLastError());
    return HC_OK;
}

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_plan(hc_context* cp, uint64_t N, uint32_t ncol, uint32_t t_bound,
                             uint32_t comp_level, uint32_t* elements_out, uint32_t* count,
                             hc_compress_info* info) {
    if (!cp || !count) return HC_EINVAL;
    Plan pl;
    hc_status s = make_plan(*cp, N, ncol, t_bound, comp_level, pl);
    if (s != HC_OK) return s;
    fill_info(pl, info);
    uint32_t cap = *count;
    *count = (uint32_t)pl.keys.size();
    if (cap < pl.keys.size()) return HC_EINVAL;
    if (elements_out)
        for (size_t i = 0; i < pl.keys.size(); i++) elements_out[i] = pl.keys[i];
    return HC_OK;
}

extern "C" hc_status hc_compress(hc_context* cp, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v,
                                 uint64_t N, uint32_t t_bound, uint32_t comp_level, uint64_t* ct_out,
                                 hc_compress_info* info, hipStream_t st) {
    if (!cp || !gk || !ct_v || !ct_out) return HC_EINVAL;
    HC_CHECK(hipSetDevice(cp->device));
    Plan pl;
    hc_status s = make_plan(*cp, N, db ? db->ncol : 0, t_bound, comp_level, pl);
    if (s != HC_OK) return s;
    s = compress_one(*cp, gk, db, ct_v, pl, ct_out, st);
    if (s == HC_OK) fill_info(pl, info);
    return s;
}

extern "C" hc_status hc_compress_batch(hc_context* cp, const hc_gk* gk, const hc_db* db, hc_query* q,
                                       uint32_t nq, hipStream_t st) {
    if (!cp || !gk || (nq && !q)) return HC_EINVAL;
    hc_status first = HC_OK;
    for (uint32_t i = 0; i < nq; i++) {
        q[i].status = hc_compress(cp, gk, db, q[i].ct_v, q[i].N, q[i].t_bound, q[i].comp_level,
                                  q[i].ct_out, q[i].info, st);
        if (q[i].status != HC_OK && first == HC_OK) first = q[i].status;
    }
    return first;
}
