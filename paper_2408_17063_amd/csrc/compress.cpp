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

#include "compress.h"

namespace hc {


uint32_t rot_elt(const Ctx& c, int64_t r) {
    int64_t nh = c.nh;
    int64_t rr = ((r % nh) + nh) % nh;
    return (uint32_t)h_powmod(3, (uint64_t)rr, 2ull * c.n);
}

uint32_t choose_B(uint32_t s, uint32_t k) {
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
                    uint32_t out_level, Plan& pl) {
    if (N == 0 || t_bound == 0) return HC_EINVAL;
    if (comp_level == 0) pl.level = default_level(c);
    else if ((int)comp_level > c.L || comp_level % c.alpha) return HC_EINVAL;
    else pl.level = (int)comp_level;
    if ((int)out_level > pl.level) return HC_EINVAL;
    pl.out_level = out_level ? (int)out_level : pl.level;
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

void fill_info(const Plan& pl, hc_compress_info* info) {
    if (!info) return;
    info->s = pl.s;
    info->groups = (uint32_t)pl.groups.size();
    info->streams = (uint32_t)pl.streams.size();
    info->bands = pl.bands;
    info->n_ct = pl.n_ct;
    info->n_keyswitch = pl.n_ks;
    info->n_ptct = pl.n_ptct;
    info->n_diag = pl.n_diag;
    info->level = (uint32_t)pl.out_level;
    info->comp_level = (uint32_t)pl.level;
    info->n_diag_resident = 0;
}

// Diagonal classes (s, B) of one plan with their largest u-block count.
static std::map<uint32_t, uint32_t> plan_classes(const Plan& pl) {
    std::map<uint32_t, uint32_t> kmax;  // B -> k
    for (auto& g : pl.groups) kmax[g.B] = std::max(kmax[g.B], g.k);
    return kmax;
}


// Device-memory budget for the diagonal chunk buffer (plaintexts [Lc][n] u64).
static const size_t kDiagBudgetBytes = (size_t)16 << 30;

// The resident table of class (s, B) at level Lc if it holds at least kb u-blocks.
static const Ctx::DiagTab* resident_table(const Ctx& c, uint32_t s, uint32_t B, int Lc, uint32_t kb) {
    auto it = c.diag_tabs.find(std::make_tuple(s, B, Lc));
    return (it != c.diag_tabs.end() && it->second.kb >= kb) ? &it->second : nullptr;
}


void fill_info(const QueryRun& q, hc_compress_info* info) {
    if (!info) return;
    fill_info(q.pl, info);
    info->n_diag = q.n_diag;
    info->n_diag_resident = q.n_diag_res;
}

// A batch of compressions run as one sequence of batched phases: every phase
// (Mask, switch, u-packing, baby steps, diagonal chunks, giant steps, each
// rotate-and-sum shift, merge) handles all queries at once, so rotations by the
// same Galois element across queries go through the same key-switching pass and
// pairs with the same (s, B) share each diagonal chunk. All queries must have
// the same Comp level. Each query's result equals its single-query compression.

hc_status batch_shape(const Ctx& c, const hc_gk* gk, const hc_db* db, std::vector<QueryRun>& qs, BatchShape& b) {
    if (qs.empty()) return HC_EINVAL;
    const size_t n = c.n;
    const int Lc = qs[0].pl.level;
    b = BatchShape();
    b.Lc = Lc;
    size_t total = 64 * 256, max_jobs = 1, diag_max = 1;
    auto& cls_k = b.cls_k;
    auto& cls_np = b.cls_np;
    auto& cls_gc = b.cls_gc;
    auto& cls_res = b.cls_res;
    for (auto& q : qs) {
        if (q.pl.level != Lc) return HC_EINVAL;
        for (uint32_t k : q.pl.keys)
            if (!find_key(gk, k)) return HC_ENOKEY;
        if (q.ct_d ? q.pl.ncol != 1 : (q.pl.ncol && (!db || db->ncol != q.pl.ncol || db->N < q.pl.N)))
            return HC_EINVAL;
        q.sizes(c);
        total += q.bytes(c);
        max_jobs = std::max<size_t>({max_jobs, q.ub, q.baby, q.gi, (size_t)q.pl.bands});
        for (auto& g : q.pl.groups) {
            auto key = std::make_pair(q.pl.s, g.B);
            cls_k[key] = std::max(cls_k[key], g.k);
            cls_np[key] += (uint32_t)q.pl.streams.size();
        }
    }
    size_t jobs_all = 0;
    for (auto& q : qs) jobs_all = std::max(jobs_all, q.ub + q.baby + q.gi);
    max_jobs = std::max(max_jobs, jobs_all * qs.size());
    const size_t PW = (size_t)Lc * n;
    for (auto& kv : cls_k) {
        const uint32_t s = kv.first.first, B = kv.first.second, kb = kv.second;
        const Ctx::DiagTab* tab = resident_table(c, s, B, Lc, kb);
        cls_res[kv.first] = tab;
        if (tab) continue;
        const size_t per_g = (size_t)kb * B * PW * 8;
        const uint32_t Gc = (uint32_t)std::min<size_t>(s / B, std::max<size_t>(1, kDiagBudgetBytes / per_g));
        cls_gc[kv.first] = Gc;
        diag_max = std::max(diag_max, (size_t)kb * Gc * B);
    }
    size_t rt_words = 0;  // the rotated ciphertexts of every class in the MAC's layout
    for (auto& kv : cls_k) {
        b.cls_rt[kv.first] = rt_words;
        rt_words += (size_t)cls_np[kv.first] * diag_terms_padded((int)(kv.second * kv.first.second)) * 2 * PW;
    }
    rt_words = std::max<size_t>(rt_words, 1);
    size_t sum_groups = 0;  // giant-step sums (one per pair)
    for (auto& q : qs) sum_groups += (size_t)q.npairs;
    const size_t R = (size_t)Lc + c.K;
    total += rup(PW * 8 * diag_max) + rup(n * 4 * diag_max) + rup(rt_words * 8) +
             rup(sum_groups * 2 * R * n * 8) + rup(sum_groups * PW * 8) + ks_scratch_bytes(c, Lc, (int)max_jobs);

    b.total = total;
    b.max_jobs = max_jobs;
    b.diag_max = diag_max;
    b.rt_words = rt_words;
    b.sum_groups = sum_groups;
    return HC_OK;
}

hc_status compress_many(Ctx& c, Lane& l, const hc_gk* gk, const hc_db* db, std::vector<QueryRun>& qs,
                        hipStream_t st) {
    if (qs.empty()) return HC_OK;
    BatchShape shape;
    hc_status bs = batch_shape(c, gk, db, qs, shape);
    if (bs != HC_OK) return bs;
    const size_t n = c.n;
    const int Lc = shape.Lc;
    const size_t PW = (size_t)Lc * n;
    const size_t total = shape.total, max_jobs = shape.max_jobs, diag_max = shape.diag_max;
    auto& cls_k = shape.cls_k;
    auto& cls_gc = shape.cls_gc;
    auto& cls_res = shape.cls_res;
    stage_reset(l, st);  // the workspace and staging area are reused call to call
    if (l.ws.reserve(total) != HC_OK) return HC_ENOMEM;
    Arena& a = l.ws;
    KsScratch ks = ks_scratch(c, a, Lc, (int)max_jobs);
    for (auto& q : qs)
        if (q.take(a) != HC_OK) return HC_ENOMEM;
    uint64_t* D = a.take<uint64_t>(PW * diag_max);
    uint32_t* Dp = a.take<uint32_t>(n * diag_max);
    uint64_t* Rt = a.take<uint64_t>(shape.rt_words);
    uint64_t* const Rt0 = Rt;
    uint64_t* TA = a.take<uint64_t>(std::max<size_t>(1, shape.sum_groups) * 2 * ((size_t)Lc + c.K) * n);
    uint64_t* C0A = a.take<uint64_t>(std::max<size_t>(1, shape.sum_groups) * PW);
    if (!D || !Dp || !Rt || !TA || !C0A) return HC_ENOMEM;
    for (auto& q : qs) {
        q.n_diag = q.n_diag_res = 0;
        for (auto& kv : plan_classes(q.pl))
            (cls_res[std::make_pair(q.pl.s, kv.first)] ? q.n_diag_res : q.n_diag) += (uint64_t)kv.second * q.pl.s;
    }
    hc_status err = HC_OK;
#define RUN(x) do { if ((err = (x)) != HC_OK) return err; } while (0)
    const uint32_t col_k = 2u * c.n - 1;
    const uint64_t* col_key = find_key(gk, col_k);

    // 1. inputs to the NTT domain; Mask at the top level (Alg. 7 step 2). At ring 2^16 with
    //    a switch to follow, the products at the primes it drops are formed inside the
    //    first pass of their inverse transform (ntt_mask_low), which the switch needs anyway.
    const bool mask_fused = Lc < c.L && c.logn == 16;
    {
        // ciphertext i times every column's plaintext i, into slot (1 + col) n_ct + i
        std::vector<MaskJob> mj;
        for (auto& q : qs) {
            ntt64(c, q.ctf, (size_t)c.L * n, 2 * (int)q.pl.n_ct, 0, c.L, false, st, q.ct_v);
            if (q.ct_d) {  // the value vector given (generic Comp): no Mask
                uint64_t* dst = q.ctf + (size_t)q.pl.n_ct * q.CWF;
                ntt64(c, dst, (size_t)c.L * n, 2 * (int)q.pl.n_ct, 0, c.L, false, st, q.ct_d);
                continue;
            }
            if (q.pl.ncol > 0)
                for (uint32_t i = 0; i < q.pl.n_ct; i++)
                    mj.push_back(MaskJob{q.ctf + i * q.CWF, q.ctf + ((size_t)q.pl.n_ct + i) * q.CWF,
                                         db->d_pt + (size_t)i * c.L * n, (uint64_t)q.pl.n_ct * q.CWF,
                                         (uint64_t)db->n_ct * c.L * n, q.pl.ncol, 0u});
        }
        if (!mj.empty()) {
            const MaskJob* dm = (const MaskJob*)stage_bytes(l, mj.data(), sizeof(MaskJob) * mj.size(), st);
            if (!dm) return HC_ENOMEM;
            k_mask_jobs(c, dm, (int)mj.size(), mask_fused ? Lc : c.L, c.L, st);
            if (mask_fused) {
                int nprod = 0, cmax = 0;
                for (auto& j : mj) {
                    nprod += (int)j.ncol;
                    cmax = std::max(cmax, (int)j.ncol);
                }
                ntt_mask_low(c, dm, (int)mj.size(), cmax, nprod, Lc, st);
            }
        }
    }
    // 2. switch to the Comp level (Sec. 5.3's smaller parameters, as a modulus switch);
    // the input ciphertexts' dropped rows are read from the query (coefficient form)
    if (Lc < c.L)
        for (auto& q : qs)
            RUN(mod_switch_batch(c, q.cts, q.ctf, (int)q.ntot, Lc, q.msconv, st, q.ct_v, (int)q.pl.n_ct,
                                 mask_fused && !q.ct_d && q.pl.ncol > 0));

    // 3. u-blocks (Sec. 5.2 remark): row 0: A*[1;0] + Rot_col(B*[1;0]); row 1: Rot_col(A*[0;1]) + B*[0;1]
    {
        std::vector<EwJob> mul, add;
        std::vector<KsJob> rot;
        for (auto& q : qs) {
            const size_t CW = q.CW;
            q.U.assign(q.npairs, {});
            size_t uo = 0;
            int pp = 0;
            for (auto& g : q.pl.groups) {
                for (auto& sm : q.pl.streams) {
                    q.U[pp].resize(g.k);
                    for (uint32_t beta = 0; beta < g.k; beta++, uo++) {
                        uint64_t *u = q.ubuf + uo * CW, *t = q.tbuf + uo * CW, *r = q.rbuf + uo * CW,
                                 *w = q.wbuf + uo * CW;
                        q.U[pp][beta] = u;
                        const uint32_t i = g.ct_start + beta / 2;
                        const uint64_t* Act = q.vec_ct(sm.first, i);
                        const uint64_t* Bct = sm.second >= 0 ? q.vec_ct(sm.second, i) : nullptr;
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
        }
        RUN(ew_run(c, l, mul, Lc, true, st));
        RUN(ks_run(c, l, ks, rot, nullptr, Lc, st));
        RUN(ew_run(c, l, add, Lc, false, st));
    }

    // Each class (s, B) gathers its pairs' rotated ciphertexts into one region of Rt, in
    // the multiply-accumulate's layout [Lc][n/64][pair][Jp][64][2] (split words); pair
    // ci of the class is its ci-th (query, pair) in query order.
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> cls_seen;
    for (auto& q : qs) {
        q.ci.assign(q.npairs, 0);
        for (int pp = 0; pp < q.npairs; pp++)
            q.ci[pp] = cls_seen[std::make_pair(q.pl.s, q.pl.groups[pp / q.pl.streams.size()].B)]++;
    }

    // 4. hoisted baby steps Rot_row(u; b), b = 1..B-1, one raise per u-block; each
    //    result is written straight into its class's Rt region
    {
        std::vector<const uint64_t*> srcs;
        std::vector<KsJob> jobs;
        for (auto& q : qs) {
            q.R.assign(q.npairs, {});
            int pp = 0;
            for (auto& g : q.pl.groups)
                for (size_t si = 0; si < q.pl.streams.size(); si++, pp++) {
                    const auto key = std::make_pair(q.pl.s, g.B);
                    const size_t Jp = (size_t)diag_terms_padded((int)(cls_k[key] * g.B));
                    const size_t np = shape.cls_np[key];
                    uint64_t* Rc = Rt + shape.cls_rt[key];
                    q.R[pp].assign(g.k, std::vector<const uint64_t*>(g.B, nullptr));
                    for (uint32_t beta = 0; beta < g.k; beta++) {
                        q.R[pp][beta][0] = q.U[pp][beta];
                        if (g.B == 1) continue;
                        const uint32_t xi = (uint32_t)srcs.size();
                        srcs.push_back(q.U[pp][beta]);
                        for (uint32_t b = 1; b < g.B; b++) {
                            const uint32_t k = rot_elt(c, b);
                            KsJob jb{q.U[pp][beta], Rc + ((size_t)q.ci[pp] * Jp + beta * g.B + b) * 128,
                                     find_key(gk, k), k, xi};
                            jb.tstride = np * Jp * 128;
                            jobs.push_back(jb);
                            q.R[pp][beta][b] = kRtInPlace;
                        }
                    }
                }
        }
        if (!jobs.empty()) RUN(ks_run(c, l, ks, jobs, &srcs, Lc, st));
    }

    // 5. diagonals encoded on the fly, one chunk of giant indices at a time, accumulated
    //    for every pair (of every query) with the same (s, B)
    for (auto& q : qs) {
        q.A.assign(q.npairs, {});
        size_t go = 0;
        int pp = 0;
        for (auto& g : q.pl.groups)
            for (size_t si = 0; si < q.pl.streams.size(); si++, pp++) {
                q.A[pp].resize(q.pl.s / g.B);
                for (uint32_t gi = 0; gi < q.pl.s / g.B; gi++) q.A[pp][gi] = q.gbuf + (go++) * q.CW;
            }
    }
    for (auto& kv : cls_k) {
        const uint32_t s = kv.first.first, B = kv.first.second, kb = kv.second, Gc = cls_gc[kv.first];
        std::vector<std::pair<QueryRun*, int>> cls;
        for (auto& q : qs)
            for (int pp = 0; pp < q.npairs; pp++)
                if (q.pl.s == s && q.pl.groups[pp / q.pl.streams.size()].B == B) cls.push_back({&q, pp});
        const uint32_t G = s / B;
        const size_t np = cls.size();
        uint64_t* Rt = Rt0 + shape.cls_rt[kv.first];
        // the rest of the class's rotated ciphertexts (the unrotated u-blocks, zero
        // padding), gathered into its region of the MAC's tiled layout
        std::vector<const uint64_t*> hptr(np * kb * B + np * G, nullptr);
        for (size_t ci = 0; ci < np; ci++) {
            QueryRun& q = *cls[ci].first;
            const int pp = cls[ci].second;
            if (q.ci[pp] != ci) return HC_EINVAL;  // the pair order phase 4 wrote in
            for (uint32_t beta = 0; beta < q.R[pp].size(); beta++)
                for (uint32_t b = 0; b < B; b++) hptr[(ci * kb + beta) * B + b] = q.R[pp][beta][b];
            for (uint32_t gi = 0; gi < G; gi++) hptr[np * kb * B + ci * G + gi] = q.A[pp][gi];
        }
        // the rotated-ciphertext and giant-accumulator pointer tables and the list of
        // entries the gather writes, one copy
        const std::vector<uint32_t> work = diag_gather_list(hptr, (int)np, (int)(kb * B));
        void *drp = nullptr, *dwk = nullptr;
        if (!stage_many(l, {{hptr.data(), sizeof(uint64_t*) * hptr.size(), &drp},
                            {work.data(), sizeof(uint32_t) * work.size(), &dwk}},
                        st))
            return HC_ENOMEM;
        const uint64_t* const* rptr = (const uint64_t* const*)drp;
        k_diag_gather(c, Rt, rptr, (const uint32_t*)dwk, (int)work.size(), (int)np, (int)(kb * B), Lc, st);
        if (const Ctx::DiagTab* tab = cls_res[kv.first]) {
            // resident diagonals: one pass over every giant index
            uint64_t** aptr = (uint64_t**)(rptr + np * kb * B);
            hc_status ms = tab->mfma ? k_diag_mac_mfma(c, aptr, Rt, tab->d, tab->kb * B, (int)np, (int)(kb * B),
                                                       (int)G, Lc, st)
                                     : k_diag_mac(c, aptr, Rt, tab->d, diag_layout_tiled(c, tab->kb * B, G), (int)np,
                                                  (int)(kb * B), (int)G, false, Lc, st);
            if (ms != HC_OK) return ms;
            continue;
        }
        std::vector<uint32_t> hprm;
        std::vector<uint64_t*> haptr;
        for (uint32_t g0 = 0; g0 < G; g0 += Gc) {
            const uint32_t gc = std::min(Gc, G - g0);
            hprm.clear();
            for (uint32_t beta = 0; beta < kb; beta++)  // chunk order (beta, b, g)
                for (uint32_t b = 0; b < B; b++)
                    for (uint32_t gi = 0; gi < gc; gi++) {
                        hprm.push_back(beta);
                        hprm.push_back(g0 + gi);
                        hprm.push_back(b);
                    }
            const int cnt = (int)(hprm.size() / 3);
            haptr.assign(np * gc, nullptr);  // A pointers [cls][gc]
            for (size_t ci = 0; ci < np; ci++)
                for (uint32_t gi = 0; gi < gc; gi++) haptr[ci * gc + gi] = cls[ci].first->A[cls[ci].second][g0 + gi];
            const uint32_t* dprm = (const uint32_t*)stage_bytes(l, hprm.data(), sizeof(uint32_t) * hprm.size(), st);
            uint64_t** aptr = (uint64_t**)stage_bytes(l, haptr.data(), sizeof(uint64_t*) * haptr.size(), st);
            if (!dprm || !aptr) return HC_ENOMEM;
            k_diag_gen(c, Dp, dprm, cnt, s, B, st);
            ntt32(c, Dp, cnt, true, st);
            k_lift(c, D, Dp, cnt, true, Lc, st);
            ntt64(c, D, PW, cnt, 0, Lc, false, st);
            k_diag_split(c, D, (size_t)cnt * PW, Lc, st);
            hc_status ms = k_diag_mac(c, aptr, Rt, D, diag_layout_natural(c, Lc, gc), (int)np, (int)(kb * B),
                                      (int)gc, false, Lc, st);
            if (ms != HC_OK) return ms;
        }
    }

    // 6. giant steps: y = A_0 + sum_{g >= 1} Rot_row(A_g; g B); the giant rotations of
    //    each pair are key-switched as one sum with a single ModDown
    {
        std::vector<KsJob> jobs;
        std::vector<uint32_t> grp;
        std::vector<uint64_t*> outs;
        std::vector<EwJob> add;
        for (auto& q : qs) {
            int pp = 0;
            for (auto& g : q.pl.groups)
                for (size_t si = 0; si < q.pl.streams.size(); si++, pp++) {
                    const uint32_t G = q.pl.s / g.B;
                    uint64_t* y = q.ybuf + (size_t)pp * q.CW;
                    if (G == 1) {
                        HC_CHECK(hipMemcpyAsync(y, q.A[pp][0], sizeof(uint64_t) * q.CW, hipMemcpyDeviceToDevice, st));
                        continue;
                    }
                    uint64_t* o = q.gout + (size_t)pp * q.CW;
                    for (uint32_t gi = 1; gi < G; gi++) {
                        const uint32_t k = rot_elt(c, (int64_t)gi * g.B);
                        jobs.push_back(KsJob{q.A[pp][gi], nullptr, find_key(gk, k), k, 0});
                        grp.push_back((uint32_t)outs.size());
                    }
                    outs.push_back(o);
                    add.push_back(EwJob{y, q.A[pp][0], o});
                }
        }
        if (!jobs.empty()) RUN(ks_run_sum(c, l, ks, jobs, grp, outs, TA, C0A, Lc, st));
        RUN(ew_run(c, l, add, Lc, false, st));
    }

    // 7. rotate-and-sum, once after the block sums (Sec. 5.2): y += Rot_row(y; sh) for
    //    sh = s, 2s, .., n/4; one pass per shift over every query with s <= sh
    for (uint64_t sh = 1; sh < (uint64_t)c.nh; sh *= 2) {
        const uint32_t k = rot_elt(c, (int64_t)sh);
        std::vector<KsJob> jobs;
        for (auto& q : qs)
            if (q.pl.s <= sh)
                for (int pp = 0; pp < q.npairs; pp++)
                    jobs.push_back(KsJob{q.ybuf + pp * q.CW, q.ytmp + pp * q.CW, find_key(gk, k), k, 0});
        if (jobs.empty()) continue;
        RUN(ks_run(c, l, ks, jobs, nullptr, Lc, st));
        for (auto& q : qs)
            if (q.pl.s <= sh) k_add(c, q.ybuf, q.ybuf, q.ytmp, 0, Lc, 2 * q.npairs, q.PW, st);
    }

    // 8. merge the bands of each query into one ciphertext
    {
        std::vector<EwJob> mul;
        std::vector<KsJob> jobs;
        for (auto& q : qs) {
            if (q.pl.bands <= 1) continue;
            const uint64_t* ms = nullptr;
            RUN(prefix_mask(c, q.pl.s, &ms));
            for (uint32_t b = 0; b < q.pl.bands; b++) {
                mul.push_back(EwJob{b == 0 ? q.mrot : q.mbuf + b * q.CW, q.ybuf + b * q.CW, ms});
                if (b > 0) {
                    const uint32_t k = rot_elt(c, -(int64_t)b * q.pl.s);
                    jobs.push_back(KsJob{q.mbuf + b * q.CW, q.mrot + b * q.CW, find_key(gk, k), k, 0});
                }
            }
        }
        RUN(ew_run(c, l, mul, Lc, true, st));
        if (!jobs.empty()) RUN(ks_run(c, l, ks, jobs, nullptr, Lc, st));
    }
    // 9. outputs back to the coefficient domain, then (out_level < Lc) the answer's own
    //    modulus switch, element-wise in the coefficient domain (Sec. 6.2's one-prime answer)
    for (auto& q : qs) {
        uint64_t* res = q.ybuf;
        if (q.pl.bands > 1) {
            k_sum_cts(c, q.outN, q.mrot, 1, (int)q.pl.bands, Lc, st);
            res = q.outN;
        }
        ntt64(c, res, q.PW, 2, 0, Lc, true, st);
        if (q.pl.out_level < Lc)
            RUN(mod_switch_coef(c, q.ct_out, res, 1, Lc, q.pl.out_level, q.ytmp, st));
        else
            HC_CHECK(hipMemcpyAsync(q.ct_out, res, sizeof(uint64_t) * q.CW, hipMemcpyDeviceToDevice, st));
    }
#undef RUN
    HC_CHECK(hipGetLastError());
    return HC_OK;
}

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_plan(hc_context* cp, uint64_t N, uint32_t ncol, uint32_t t_bound,
                             uint32_t comp_level, uint32_t out_level, uint32_t* elements_out, uint32_t* count,
                             hc_compress_info* info) {
    if (!cp || !count) return HC_EINVAL;
    Plan pl;
    hc_status s = make_plan(*cp, N, ncol, t_bound, comp_level, out_level, pl);
    if (s != HC_OK) return s;
    fill_info(pl, info);
    if (info) {
        info->n_diag = 0;
        for (auto& kv : plan_classes(pl))
            (resident_table(*cp, pl.s, kv.first, pl.level, kv.second) ? info->n_diag_resident : info->n_diag) +=
                (uint64_t)kv.second * pl.s;
    }
    uint32_t cap = *count;
    *count = (uint32_t)pl.keys.size();
    if (cap < pl.keys.size()) return HC_EINVAL;
    if (elements_out)
        for (size_t i = 0; i < pl.keys.size(); i++) elements_out[i] = pl.keys[i];
    return HC_OK;
}

extern "C" hc_status hc_compress(hc_context* cp, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v,
                                 uint64_t N, uint32_t t_bound, uint32_t comp_level, uint32_t out_level,
                                 uint64_t* ct_out, hc_compress_info* info, hipStream_t st) {
    if (!cp || !gk || !ct_v || !ct_out) return HC_EINVAL;
    HC_CHECK(hipSetDevice(cp->device));
    std::vector<QueryRun> qs(1);
    hc_status s = make_plan(*cp, N, db ? db->ncol : 0, t_bound, comp_level, out_level, qs[0].pl);
    if (s != HC_OK) return s;
    qs[0].ct_v = ct_v;
    qs[0].ct_out = ct_out;
    s = compress_many(*cp, cp->lane, gk, db, qs, st);
    if (s == HC_OK) fill_info(qs[0], info);
    return s;
}

extern "C" hc_status hc_compress_batch(hc_context* cp, const hc_gk* gk, const hc_db* db, hc_query* q,
                                       uint32_t nq, hipStream_t st) {
    if (!cp || !gk || (nq && !q)) return HC_EINVAL;
    HC_CHECK(hipSetDevice(cp->device));
    // plan every query; queries are batched by Comp level (normally all share one)
    std::map<int, std::vector<QueryRun>> by_level;
    std::map<int, std::vector<uint32_t>> idx;
    hc_status first = HC_OK;
    for (uint32_t i = 0; i < nq; i++) {
        QueryRun r;
        q[i].status = (!q[i].ct_v || !q[i].ct_out)
                          ? HC_EINVAL
                          : make_plan(*cp, q[i].N, db ? db->ncol : 0, q[i].t_bound, q[i].comp_level,
                                      q[i].out_level, r.pl);
        if (q[i].status == HC_OK) {
            for (uint32_t k : r.pl.keys)
                if (!find_key(gk, k)) q[i].status = HC_ENOKEY;
            if (r.pl.ncol && (!db || db->N < r.pl.N)) q[i].status = HC_EINVAL;
        }
        if (q[i].status != HC_OK) {
            if (first == HC_OK) first = q[i].status;
            continue;
        }
        r.ct_v = q[i].ct_v;
        r.ct_out = q[i].ct_out;
        by_level[r.pl.level].push_back(std::move(r));
        idx[r.pl.level].push_back(i);
    }
    for (auto& kv : by_level) {
        hc_status s = compress_many(*cp, cp->lane, gk, db, kv.second, st);
        auto& ids = idx[kv.first];
        for (size_t j = 0; j < ids.size(); j++) {
            q[ids[j]].status = s;
            if (s == HC_OK) fill_info(kv.second[j], q[ids[j]].info);
        }
        if (s != HC_OK && first == HC_OK) first = s;
    }
    return first;
}

extern "C" hc_status hc_diag_prepare(hc_context* cp, uint64_t N, uint32_t ncol, uint32_t t_bound,
                                     uint32_t comp_level, uint64_t* bytes_out) {
    if (!cp) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    Plan pl;
    hc_status s = make_plan(c, N, ncol, t_bound, comp_level, 0, pl);
    if (s != HC_OK) return s;
    const int Lc = pl.level;
    const size_t n = c.n, PW = (size_t)Lc * n;
    const hipStream_t st = nullptr;
    for (auto& kv : plan_classes(pl)) {
        const uint32_t B = kv.first, kb = kv.second, G = pl.s / B;
        if (resident_table(c, pl.s, B, Lc, kb)) continue;
        const auto key = std::make_tuple(pl.s, B, Lc);
        auto old = c.diag_tabs.find(key);
        if (old != c.diag_tabs.end()) {
            HC_CHECK(hipDeviceSynchronize());
            HC_CHECK(hipFree(old->second.d));
            c.diag_tabs.erase(old);
        }
        const size_t count = (size_t)kb * G * B;
        const uint32_t Jt = kb * B;
        Ctx::DiagTab tab;
        tab.kb = kb;
        tab.mfma = c.diag_layout == HC_DIAG_LAYOUT_AUTO && diag_mfma_fits(c, Lc, Jt, G);
        tab.bytes = tab.mfma ? diag_mfma_table_bytes(c, Lc, Jt, G) : diag_table_words(c, Lc, Jt, G) * 8;
        if (hipMalloc((void**)&tab.d, tab.bytes) != hipSuccess) {
            (void)hipGetLastError();
            return HC_ENOMEM;
        }
        if (tab.mfma) {
            // digit layout: one (16-giant tile, 64-term block) of diagonals at a time,
            // encoded as below but lifted as plain residues
            const size_t cmax = 16 * 64;
            stage_reset(c.lane, st);
            if (c.lane.ws.reserve(n * 4 * cmax + PW * 8 * cmax + 4096) != HC_OK) {
                (void)hipFree(tab.d);
                return HC_ENOMEM;
            }
            c.lane.ws.reset();
            uint32_t* Dp = c.lane.ws.take<uint32_t>(n * cmax);
            uint64_t* Dn = c.lane.ws.take<uint64_t>(PW * cmax);
            std::vector<uint32_t> hprm;
            for (uint32_t t = 0; t * 16 < G; t++)
                for (uint32_t jb = 0; jb * 64 < Jt; jb++) {
                    const uint32_t ng = std::min<uint32_t>(16, G - 16 * t), nj = std::min<uint32_t>(64, Jt - 64 * jb);
                    hprm.clear();
                    for (uint32_t gl = 0; gl < ng; gl++)
                        for (uint32_t jl = 0; jl < nj; jl++) {
                            const uint32_t j = 64 * jb + jl;
                            hprm.push_back(j / B);        // beta
                            hprm.push_back(16 * t + gl);  // giant index
                            hprm.push_back(j % B);        // baby index
                        }
                    const int cnt = (int)(ng * nj);
                    stage_reset(c.lane, st);
                    const uint32_t* dprm =
                        (const uint32_t*)stage_bytes(c.lane, hprm.data(), sizeof(uint32_t) * hprm.size(), st);
                    if (!dprm) {
                        (void)hipFree(tab.d);
                        return HC_ENOMEM;
                    }
                    k_diag_gen(c, Dp, dprm, cnt, pl.s, B, st);
                    ntt32(c, Dp, cnt, true, st);
                    k_lift(c, Dn, Dp, cnt, false, Lc, st);
                    ntt64(c, Dn, PW, cnt, 0, Lc, false, st);
                    k_diag_digits(c, tab.d, Dn, Jt, G, t, jb, Lc, st);
                }
            HC_CHECK(hipDeviceSynchronize());
            c.diag_tabs[key] = tab;
            continue;
        }
        // encode in chunks: slot values (Sec. 5.2 diagonals of C), to R_p, lift, NTT per
        // prime, then into the table's tiled layout
        const size_t chunk = std::min<size_t>(count, 2048);
        stage_reset(c.lane, st);
        if (c.lane.ws.reserve(n * 4 * chunk + PW * 8 * chunk + 4096) != HC_OK) {
            (void)hipFree(tab.d);
            return HC_ENOMEM;
        }
        c.lane.ws.reset();
        uint32_t* Dp = c.lane.ws.take<uint32_t>(n * chunk);
        uint64_t* Dn = c.lane.ws.take<uint64_t>(PW * chunk);
        std::vector<uint32_t> hprm;
        for (size_t i0 = 0; i0 < count; i0 += chunk) {
            const size_t cnt = std::min(chunk, count - i0);
            hprm.clear();
            for (size_t i = i0; i < i0 + cnt; i++) {
                hprm.push_back((uint32_t)(i / ((size_t)G * B)));  // beta
                hprm.push_back((uint32_t)((i / B) % G));           // giant index
                hprm.push_back((uint32_t)(i % B));                 // baby index
            }
            stage_reset(c.lane, st);
            const uint32_t* dprm = (const uint32_t*)stage_bytes(c.lane, hprm.data(), sizeof(uint32_t) * hprm.size(), st);
            if (!dprm) {
                (void)hipFree(tab.d);
                return HC_ENOMEM;
            }
            k_diag_gen(c, Dp, dprm, (int)cnt, pl.s, B, st);
            ntt32(c, Dp, (int)cnt, true, st);
            k_lift(c, Dn, Dp, (int)cnt, true, Lc, st);
            ntt64(c, Dn, PW, (int)cnt, 0, Lc, false, st);
            k_diag_tile(c, tab.d, Dn, i0, (int)cnt, kb, B, G, Lc, st);
        }
        HC_CHECK(hipDeviceSynchronize());
        c.diag_tabs[key] = tab;
    }
    if (bytes_out) {
        uint64_t t = 0;
        for (auto& kv : c.diag_tabs) t += kv.second.bytes;
        *bytes_out = t;
    }
    return HC_OK;
}

extern "C" hc_status hc_diag_layout(hc_context* cp, int layout) {
    if (!cp || (layout != HC_DIAG_LAYOUT_AUTO && layout != HC_DIAG_LAYOUT_SPLIT)) return HC_EINVAL;
    cp->diag_layout = layout;
    return HC_OK;
}

extern "C" void hc_diag_release(hc_context* cp) {
    if (!cp) return;
    (void)hipSetDevice(cp->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : cp->diag_tabs) (void)hipFree(kv.second.d);
    cp->diag_tabs.clear();
}
