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

// Device memory one compression needs beyond its inputs and output.
struct Layout {
    size_t CW, PW, CWF;     // ciphertext at the Comp level, plaintext row block, top-level ciphertext
    int npairs;
    uint32_t kmax, Bmax, Gmax, Gc;
    size_t ntot, ub_total, baby_total, gi_total, diag_cnt;
    size_t total_bytes;
};

static size_t rup(size_t b) { return (b + 255) & ~(size_t)255; }

// Device-memory budget for the diagonal chunk buffer (plaintexts [Lc][n] u64).
static const size_t kDiagBudgetBytes = (size_t)16 << 30;

static Layout layout_for(const Ctx& c, const Plan& pl) {
    Layout ly;
    const size_t n = c.n;
    ly.CW = 2 * (size_t)pl.level * n;
    ly.PW = (size_t)pl.level * n;
    ly.CWF = 2 * (size_t)c.L * n;
    ly.npairs = (int)(pl.groups.size() * pl.streams.size());
    ly.kmax = 0;
    ly.Bmax = 1;
    ly.Gmax = 1;
    ly.ub_total = ly.baby_total = ly.gi_total = 0;
    for (auto& g : pl.groups) {
        ly.kmax = std::max(ly.kmax, g.k);
        ly.Bmax = std::max(ly.Bmax, g.B);
        ly.Gmax = std::max(ly.Gmax, pl.s / g.B);
        ly.ub_total += (size_t)g.k * pl.streams.size();
        ly.baby_total += (size_t)g.k * (g.B - 1) * pl.streams.size();
        ly.gi_total += (size_t)(pl.s / g.B) * pl.streams.size();
    }
    const size_t per_g = (size_t)ly.kmax * ly.Bmax * ly.PW * 8;
    ly.Gc = (uint32_t)std::min<size_t>(ly.Gmax, std::max<size_t>(1, kDiagBudgetBytes / std::max<size_t>(per_g, 1)));
    ly.diag_cnt = (size_t)ly.kmax * ly.Gc * ly.Bmax;
    ly.ntot = (size_t)pl.n_ct * (1 + pl.ncol);
    size_t max_jobs = std::max<size_t>({ly.ub_total, ly.baby_total, ly.gi_total, (size_t)pl.bands, 1});
    size_t t = 0;
    t += rup(ly.CWF * 8 * ly.ntot);                      // inputs and masked, top level
    if (pl.level < c.L) t += 2 * rup(ly.CW * 8 * ly.ntot);  // switched copies + conversion scratch
    t += 4 * rup(ly.CW * 8 * std::max<size_t>(ly.ub_total, 1));   // u-blocks and packing temporaries
    t += rup(ly.CW * 8 * std::max<size_t>(ly.baby_total, 1));     // baby-step rotations
    t += 2 * rup(ly.CW * 8 * ly.gi_total);                        // giant accumulators and their rotations
    t += 2 * rup(ly.CW * 8 * ly.npairs);                          // y and fold temporaries
    t += 2 * rup(ly.CW * 8 * pl.bands) + rup(ly.CW * 8);          // merge and output
    t += rup(ly.PW * 8 * ly.diag_cnt) + rup((size_t)n * 4 * ly.diag_cnt);  // diagonal chunk
    t += ks_scratch_bytes(c, pl.level, (int)max_jobs);
    t += 64 * 256;
    ly.total_bytes = t;
    return ly;
}

hc_status compress_one(Ctx& c, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v, const Plan& pl,
                       uint64_t* ct_out, hipStream_t st) {
    const size_t n = c.n;
    const Layout ly = layout_for(c, pl);
    const size_t CW = ly.CW, PW = ly.PW, CWF = ly.CWF, PWF = (size_t)c.L * n;
    const int Lc = pl.level;
    for (uint32_t k : pl.keys)
        if (!find_key(gk, k)) return HC_ENOKEY;
    if (pl.ncol && (!db || db->ncol != pl.ncol || db->N != pl.N)) return HC_EINVAL;

    stage_reset(c, st);  // the workspace and staging area are reused call to call
    if (c.ws.reserve(ly.total_bytes) != HC_OK) return HC_ENOMEM;
    Arena& a = c.ws;
    const size_t max_jobs = std::max<size_t>({ly.ub_total, ly.baby_total, ly.gi_total, (size_t)pl.bands, 1});
    KsScratch ks = ks_scratch(c, a, Lc, (int)max_jobs);
    hc_status err = HC_OK;
#define RUN(x) do { if ((err = (x)) != HC_OK) return err; } while (0)

    // 1. inputs to the NTT domain; Mask at the top level (Alg. 7 step 2)
    uint64_t* ctf = a.take<uint64_t>(CWF * ly.ntot);
    if (!ctf) return HC_ENOMEM;
    HC_CHECK(hipMemcpyAsync(ctf, ct_v, sizeof(uint64_t) * CWF * pl.n_ct, hipMemcpyDeviceToDevice, st));
    ntt64(c, ctf, PWF, 2 * (int)pl.n_ct, 0, c.L, false, st);
    {
        std::vector<EwJob> mj;
        for (uint32_t col = 0; col < pl.ncol; col++)
            for (uint32_t i = 0; i < pl.n_ct; i++)
                mj.push_back(EwJob{ctf + ((size_t)(1 + col) * pl.n_ct + i) * CWF, ctf + i * CWF,
                                   db->d_pt + ((size_t)col * pl.n_ct + i) * PWF});
        RUN(ew_run(c, mj, c.L, true, st));
    }
    // 2. switch to the Comp level (Sec. 5.3's smaller parameters, as a modulus switch)
    uint64_t* cts = ctf;
    if (Lc < c.L) {
        cts = a.take<uint64_t>(CW * ly.ntot);
        uint64_t* conv = a.take<uint64_t>(CW * ly.ntot);
        if (!cts || !conv) return HC_ENOMEM;
        RUN(mod_switch_batch(c, cts, ctf, (int)ly.ntot, Lc, conv, st));
    }
    auto vec_ct = [&](int vid, uint32_t i) -> const uint64_t* { return cts + ((size_t)vid * pl.n_ct + i) * CW; };

    // per-pair storage
    const int npairs = ly.npairs;
    uint64_t* ubuf = a.take<uint64_t>(CW * std::max<size_t>(ly.ub_total, 1));
    uint64_t* tbuf = a.take<uint64_t>(CW * std::max<size_t>(ly.ub_total, 1));
    uint64_t* rbuf = a.take<uint64_t>(CW * std::max<size_t>(ly.ub_total, 1));
    uint64_t* wbuf = a.take<uint64_t>(CW * std::max<size_t>(ly.ub_total, 1));
    uint64_t* bbuf = a.take<uint64_t>(CW * std::max<size_t>(ly.baby_total, 1));
    uint64_t* gbuf = a.take<uint64_t>(CW * ly.gi_total);
    uint64_t* gout = a.take<uint64_t>(CW * ly.gi_total);
    uint64_t* ybuf = a.take<uint64_t>(CW * npairs);
    uint64_t* ytmp = a.take<uint64_t>(CW * npairs);
    uint64_t* mbuf = a.take<uint64_t>(CW * pl.bands);
    uint64_t* mrot = a.take<uint64_t>(CW * pl.bands);
    uint64_t* outN = a.take<uint64_t>(CW);
    if (!ubuf || !tbuf || !rbuf || !wbuf || !bbuf || !gbuf || !gout || !ybuf || !ytmp || !mbuf || !mrot || !outN)
        return HC_ENOMEM;
    const uint32_t col_k = 2u * c.n - 1;
    const uint64_t* col_key = find_key(gk, col_k);

    // 3. u-blocks (Sec. 5.2 remark): row 0: A*[1;0] + Rot_col(B*[1;0]); row 1: Rot_col(A*[0;1]) + B*[0;1]
    std::vector<std::vector<uint64_t*>> U(npairs), A(npairs);
    std::vector<std::vector<std::vector<uint64_t*>>> R(npairs);
    {
        std::vector<EwJob> mul, add;
        std::vector<KsJob> rot;
        size_t uo = 0;
        int pp = 0;
        for (auto& g : pl.groups) {
            for (auto& sm : pl.streams) {
                U[pp].resize(g.k);
                for (uint32_t beta = 0; beta < g.k; beta++, uo++) {
                    uint64_t *u = ubuf + uo * CW, *t = tbuf + uo * CW, *r = rbuf + uo * CW, *w = wbuf + uo * CW;
                    U[pp][beta] = u;
                    const uint32_t i = g.ct_start + beta / 2;
                    const uint64_t* Act = vec_ct(sm.first, i);
                    const uint64_t* Bct = sm.second >= 0 ? vec_ct(sm.second, i) : nullptr;
                    if (beta % 2 == 0) {
                        mul.push_back(EwJob{u, Act, c.d_rowmask[0]});
                        if (Bct) {
                            mul.push_back(EwJob{t, Bct, c.d_rowmask[0]});
                            rot.push_back(KsJob{t, r, col_key, col_k, 0});
                            add.push_back(EwJob{u, u, r});
                        }
                    } else {
                        mul.push_back(EwJob{t, Act, c.d_rowmask[1]});
                        if (Bct) {
                            rot.push_back(KsJob{t, r, col_key, col_k, 0});
                            mul.push_back(EwJob{w, Bct, c.d_rowmask[1]});
                            add.push_back(EwJob{u, r, w});
                        } else {
                            rot.push_back(KsJob{t, u, col_key, col_k, 0});
                        }
                    }
                }
                pp++;
            }
        }
        RUN(ew_run(c, mul, Lc, true, st));
        RUN(ks_run(c, ks, rot, nullptr, Lc, st));
        RUN(ew_run(c, add, Lc, false, st));
    }

    // 4. hoisted baby steps Rot_row(u; b), b = 1..B-1, one raise per u-block
    {
        std::vector<const uint64_t*> srcs;
        std::vector<KsJob> jobs;
        size_t bo = 0;
        int pp = 0;
        for (auto& g : pl.groups) {
            for (size_t si = 0; si < pl.streams.size(); si++, pp++) {
                R[pp].assign(g.k, std::vector<uint64_t*>(g.B, nullptr));
                for (uint32_t beta = 0; beta < g.k; beta++) {
                    R[pp][beta][0] = U[pp][beta];
                    if (g.B == 1) continue;
                    const uint32_t xi = (uint32_t)srcs.size();
                    srcs.push_back(U[pp][beta]);
                    for (uint32_t b = 1; b < g.B; b++) {
                        uint64_t* r = bbuf + (bo++) * CW;
                        const uint32_t k = rot_elt(c, b);
                        jobs.push_back(KsJob{U[pp][beta], r, find_key(gk, k), k, xi});
                        R[pp][beta][b] = r;
                    }
                }
            }
        }
        if (!jobs.empty()) RUN(ks_run(c, ks, jobs, &srcs, Lc, st));
    }

    // 5. diagonals encoded on the fly and accumulated into the giant accumulators,
    //    one chunk of giant indices at a time for every pair that shares B
    {
        size_t go = 0;
        int pp = 0;
        for (auto& g : pl.groups)
            for (size_t si = 0; si < pl.streams.size(); si++, pp++) {
                A[pp].resize(pl.s / g.B);
                for (uint32_t gi = 0; gi < pl.s / g.B; gi++) A[pp][gi] = gbuf + (go++) * CW;
            }
        std::set<uint32_t> Bs;
        for (auto& g : pl.groups) Bs.insert(g.B);
        uint64_t* D = a.take<uint64_t>(PW * ly.diag_cnt);
        uint32_t* Dp = a.take<uint32_t>((size_t)n * ly.diag_cnt);
        if (!D || !Dp) return HC_ENOMEM;
        std::vector<uint32_t> hprm;
        std::vector<const uint64_t*> hptr;
        for (uint32_t B : Bs) {
            std::vector<int> cls;
            uint32_t kb = 0;
            for (int q = 0; q < npairs; q++) {
                const PlanGroup& g = pl.groups[q / pl.streams.size()];
                if (g.B == B) { cls.push_back(q); kb = std::max(kb, g.k); }
            }
            const uint32_t G = pl.s / B;
            for (uint32_t g0 = 0; g0 < G; g0 += ly.Gc) {
                const uint32_t gc = std::min(ly.Gc, G - g0);
                hprm.clear();
                for (uint32_t beta = 0; beta < kb; beta++)
                    for (uint32_t gi = 0; gi < gc; gi++)
                        for (uint32_t b = 0; b < B; b++) {
                            hprm.push_back(beta);
                            hprm.push_back(g0 + gi);
                            hprm.push_back(b);
                        }
                const int cnt = (int)(hprm.size() / 3);
                // R pointers [cls][kb][B], then A pointers [cls][gc]
                hptr.assign((size_t)cls.size() * kb * B + cls.size() * gc, nullptr);
                for (size_t ci = 0; ci < cls.size(); ci++) {
                    const int q = cls[ci];
                    for (uint32_t beta = 0; beta < R[q].size(); beta++)
                        for (uint32_t b = 0; b < B; b++) hptr[(ci * kb + beta) * B + b] = R[q][beta][b];
                    for (uint32_t gi = 0; gi < gc; gi++)
                        hptr[(size_t)cls.size() * kb * B + ci * gc + gi] = A[q][g0 + gi];
                }
                const uint32_t* dprm = (const uint32_t*)stage_bytes(c, hprm.data(), sizeof(uint32_t) * hprm.size(), st);
                uint64_t** dptr = (uint64_t**)stage_bytes(c, hptr.data(), sizeof(uint64_t*) * hptr.size(), st);
                if (!dprm || !dptr) return HC_ENOMEM;
                k_diag_gen(c, Dp, dprm, cnt, pl.s, B, st);
                ntt32(c, Dp, cnt, true, st);
                k_lift(c, D, Dp, cnt, true, Lc, st);
                ntt64(c, D, PW, cnt, 0, Lc, false, st);
                k_diag_mac(c, dptr + (size_t)cls.size() * kb * B, (const uint64_t* const*)dptr, D,
                           (int)cls.size(), (int)kb, (int)gc, (int)B, false, Lc, st);
            }
        }
    }

    // 6. giant steps: y = A_0 + sum_g Rot_row(A_g; g B)
    {
        std::vector<KsJob> jobs;
        size_t go = 0;
        int pp = 0;
        for (auto& g : pl.groups)
            for (size_t si = 0; si < pl.streams.size(); si++, pp++) {
                const uint32_t G = pl.s / g.B;
                HC_CHECK(hipMemcpyAsync(gout + go * CW, A[pp][0], sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
                for (uint32_t gi = 1; gi < G; gi++) {
                    const uint32_t k = rot_elt(c, (int64_t)gi * g.B);
                    jobs.push_back(KsJob{A[pp][gi], gout + (go + gi) * CW, find_key(gk, k), k, 0});
                }
                go += G;
            }
        if (!jobs.empty()) RUN(ks_run(c, ks, jobs, nullptr, Lc, st));
        go = 0;
        pp = 0;
        for (auto& g : pl.groups)
            for (size_t si = 0; si < pl.streams.size(); si++, pp++) {
                const uint32_t G = pl.s / g.B;
                k_sum_cts(c, ybuf + (size_t)pp * CW, gout + go * CW, 1, (int)G, Lc, st);
                go += G;
            }
    }

    // 7. rotate-and-sum, once after the block sums (Sec. 5.2): y += Rot_row(y; s 2^i), all pairs per step
    for (uint64_t sh = pl.s; sh < (uint64_t)c.nh; sh *= 2) {
        const uint32_t k = rot_elt(c, (int64_t)sh);
        std::vector<KsJob> jobs;
        for (int q = 0; q < npairs; q++) jobs.push_back(KsJob{ybuf + q * CW, ytmp + q * CW, find_key(gk, k), k, 0});
        RUN(ks_run(c, ks, jobs, nullptr, Lc, st));
        k_add(c, ybuf, ybuf, ytmp, 0, Lc, 2 * npairs, PW, st);
    }

    // 8. merge the bands into one ciphertext
    uint64_t* res = ybuf;
    if (pl.bands > 1) {
        const uint64_t* ms = nullptr;
        RUN(prefix_mask(c, pl.s, &ms));
        std::vector<EwJob> mul;
        std::vector<KsJob> jobs;
        for (uint32_t b = 0; b < pl.bands; b++) {
            mul.push_back(EwJob{b == 0 ? mrot : mbuf + b * CW, ybuf + b * CW, ms});
            if (b > 0) {
                const uint32_t k = rot_elt(c, -(int64_t)b * pl.s);
                jobs.push_back(KsJob{mbuf + b * CW, mrot + b * CW, find_key(gk, k), k, 0});
            }
        }
        RUN(ew_run(c, mul, Lc, true, st));
        RUN(ks_run(c, ks, jobs, nullptr, Lc, st));
        k_sum_cts(c, outN, mrot, 1, (int)pl.bands, Lc, st);
        res = outN;
    }
#undef RUN
    // 9. back to the coefficient domain
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
