// The unencrypted-database form of the compression (Sec. 5.2, remark on an unencrypted
// database): with the database in the clear, C (DB * v) = (C diag(DB)) v, so the server
// multiplies the index vector directly by [C; C diag(DB_1); ...] -- no Mask and no
// per-stream packing. The answer has the same layout as hc_compress's (band
// g * streams + sigma, row 0 = M_a v, row 1 = M_b v for the stream pair (M_a, M_b)), so
// it decrypts to the same values.
//
// Device flow: inputs -> NTT domain; switch to the Comp level (the inputs' dropped rows
// read in coefficient form from the query); per input ciphertext X_i its row swap
// Y_i = Rot_col(X_i); both are the u-blocks of every stream of the group (row r of a
// u-block holds record block beta_r: X_i = (2i, 2i+1), Y_i = (2i+1, 2i)); hoisted baby
// steps once per u-block, written into one multiply-accumulate region per group; per
// (group, stream) the diagonals (row r: M_r's entries of block beta_r, times the records'
// values for C diag(DB)) encoded on the fly in chunks of giant indices and accumulated;
// then giant steps, rotate-and-sum, merge and the answer's switch as in compress.cpp.
#include <algorithm>
#include <set>

#include "compress.h"

namespace hc {

// The plan of the unencrypted-database form: make_plan's groups, streams and s, with
// k = 2 (ciphertexts of the group) u-blocks per group, B for that k, and Rot_col's key.
static hc_status make_plan_plain_db(const Ctx& c, uint64_t N, uint32_t ncol, uint32_t t_bound, uint32_t comp_level,
                                    uint32_t out_level, Plan& pl) {
    hc_status s = make_plan(c, N, ncol, t_bound, comp_level, out_level, pl);
    if (s != HC_OK) return s;
    std::set<uint32_t> keys;
    const uint32_t sv = pl.s;
    uint32_t fold = 0;
    for (uint64_t sh = sv; sh < (uint64_t)c.nh; sh *= 2) { keys.insert(rot_elt(c, (int64_t)sh)); fold++; }
    keys.insert(2u * c.n - 1);
    pl.n_ks = pl.n_ct;  // one Rot_col per input ciphertext
    pl.n_ptct = 0;
    pl.n_diag = 0;
    const uint32_t S = (uint32_t)pl.streams.size();
    for (auto& g : pl.groups) {
        g.k = 2 * g.ct_count;
        g.B = choose_B(sv, g.k);
        for (uint32_t b = 1; b < g.B; b++) keys.insert(rot_elt(c, b));
        for (uint32_t gi = 1; gi < sv / g.B; gi++) keys.insert(rot_elt(c, (int64_t)gi * g.B));
        pl.n_ks += g.k * (g.B - 1) + S * ((sv / g.B - 1) + fold);
        pl.n_ptct += (uint64_t)S * g.k * sv;
        pl.n_diag += (uint64_t)S * g.k * sv;
    }
    for (uint32_t b = 1; b < pl.bands; b++) keys.insert(rot_elt(c, -(int64_t)b * sv));
    if (pl.bands > 1) { pl.n_ks += pl.bands - 1; pl.n_ptct += pl.bands; }
    pl.keys.assign(keys.begin(), keys.end());
    return HC_OK;
}

static hc_status compress_plain_db_run(Ctx& c, Lane& l, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v,
                                       uint64_t* ct_out, const Plan& pl, hipStream_t st) {
    const size_t n = c.n;
    const int L = c.L, Lc = pl.level, K = c.K, R = Lc + K;
    const size_t CWF = 2 * (size_t)L * n, CW = 2 * (size_t)Lc * n, PW = (size_t)Lc * n;
    const uint32_t nct = pl.n_ct, S = (uint32_t)pl.streams.size(), G = (uint32_t)pl.groups.size();
    const uint32_t npairs = G * S, sv = pl.s;
    for (uint32_t k : pl.keys)
        if (!find_key(gk, k)) return HC_ENOKEY;
    if (pl.ncol && (!db || db->ncol != pl.ncol || db->N < pl.N || !db->d_raw)) return HC_EINVAL;
    const uint32_t col_k = 2u * c.n - 1;
    const uint64_t* col_key = find_key(gk, col_k);

    // workspace
    size_t max_jobs = std::max<size_t>(nct, npairs), rt_words = 0, giants = 0, cnt_max = 1, baby = 0;
    std::vector<size_t> rt_off(G);
    std::vector<uint32_t> Gc(G);
    const size_t kDiagBudget = (size_t)8 << 30;
    for (uint32_t g = 0; g < G; g++) {
        const PlanGroup& pg = pl.groups[g];
        rt_off[g] = rt_words;
        rt_words += (size_t)diag_terms_padded((int)(pg.k * pg.B)) * 2 * PW;
        giants += (size_t)S * (sv / pg.B);
        baby += (size_t)pg.k * (pg.B - 1);
        const size_t per_g = (size_t)pg.k * pg.B * PW * 8;
        Gc[g] = (uint32_t)std::min<size_t>(sv / pg.B, std::max<size_t>(1, kDiagBudget / per_g));
        cnt_max = std::max(cnt_max, (size_t)pg.k * pg.B * Gc[g]);
        max_jobs = std::max(max_jobs, std::max<size_t>(baby, giants));
    }
    const size_t total = rup(CWF * 8 * nct) + 2 * rup(CW * 8 * nct) + rup(CW * 8 * nct) + rup(rt_words * 8) +
                         rup(CW * 8 * giants) + 5 * rup(CW * 8 * npairs) + 2 * rup(CW * 8 * pl.bands) + rup(CW * 8) +
                         rup(PW * 8 * cnt_max) + rup(n * 4 * cnt_max) + rup(npairs * 2 * (size_t)R * n * 8) +
                         rup(npairs * PW * 8) + ks_scratch_bytes(c, Lc, (int)max_jobs) + 64 * 256;
    stage_reset(l, st);
    if (l.ws.reserve(total) != HC_OK) return HC_ENOMEM;
    Arena& a = l.ws;
    KsScratch ks = ks_scratch(c, a, Lc, (int)max_jobs);
    uint64_t* ctf = a.take<uint64_t>(CWF * nct);
    uint64_t* cts = ctf;
    uint64_t* conv = nullptr;
    if (Lc < L) {
        cts = a.take<uint64_t>(CW * nct);
        conv = a.take<uint64_t>(CW * nct);
    }
    uint64_t* ybl = a.take<uint64_t>(CW * nct);
    uint64_t* Rt = a.take<uint64_t>(std::max<size_t>(rt_words, 1));
    uint64_t* gbuf = a.take<uint64_t>(CW * std::max<size_t>(giants, 1));
    uint64_t* gout = a.take<uint64_t>(CW * npairs);
    uint64_t* ybuf = a.take<uint64_t>(CW * npairs);
    uint64_t* ytmp = a.take<uint64_t>(CW * npairs);
    uint64_t* mbuf = a.take<uint64_t>(CW * pl.bands);
    uint64_t* mrot = a.take<uint64_t>(CW * pl.bands);
    uint64_t* outN = a.take<uint64_t>(CW);
    uint64_t* D = a.take<uint64_t>(PW * cnt_max);
    uint32_t* Dp = a.take<uint32_t>(n * cnt_max);
    uint64_t* TA = a.take<uint64_t>(npairs * 2 * (size_t)R * n);
    uint64_t* C0A = a.take<uint64_t>(npairs * PW);
    if (!ctf || !cts || !ybl || !Rt || !gbuf || !gout || !ybuf || !ytmp || !mbuf || !mrot || !outN || !D || !Dp ||
        !TA || !C0A || (Lc < L && !conv))
        return HC_ENOMEM;
    hc_status err = HC_OK;
#define RUN(x) do { if ((err = (x)) != HC_OK) return err; } while (0)

    // 1-2. inputs to the NTT domain, then down to the Comp level (no Mask in this form)
    HC_CHECK(hipMemcpyAsync(ctf, ct_v, sizeof(uint64_t) * CWF * nct, hipMemcpyDeviceToDevice, st));
    ntt64(c, ctf, (size_t)L * n, 2 * (int)nct, 0, L, false, st);
    if (Lc < L) RUN(mod_switch_batch(c, cts, ctf, (int)nct, Lc, conv, st, ct_v, (int)nct));

    // 3. Y_i = Rot_col(X_i)
    {
        std::vector<KsJob> jobs;
        for (uint32_t i = 0; i < nct; i++) jobs.push_back(KsJob{cts + i * CW, ybl + i * CW, col_key, col_k, 0});
        RUN(ks_run(c, l, ks, jobs, nullptr, Lc, st));
    }
    // u-block beta of group g: X_i (beta = 2i) or Y_i (beta = 2i + 1), i group-local
    auto ublock = [&](const PlanGroup& pg, uint32_t beta) -> const uint64_t* {
        const uint32_t i = pg.ct_start + beta / 2;
        return (beta % 2 == 0 ? cts : ybl) + (size_t)i * CW;
    };
    // 4. hoisted baby steps Rot_row(u; b), once per u-block for every stream, written into
    //    the group's multiply-accumulate region (one "pair" per region)
    {
        std::vector<const uint64_t*> srcs;
        std::vector<KsJob> jobs;
        for (uint32_t g = 0; g < G; g++) {
            const PlanGroup& pg = pl.groups[g];
            const size_t Jp = (size_t)diag_terms_padded((int)(pg.k * pg.B));
            for (uint32_t beta = 0; beta < pg.k && pg.B > 1; beta++) {
                const uint32_t xi = (uint32_t)srcs.size();
                srcs.push_back(ublock(pg, beta));
                for (uint32_t b = 1; b < pg.B; b++) {
                    const uint32_t k = rot_elt(c, b);
                    KsJob jb{ublock(pg, beta), Rt + rt_off[g] + ((size_t)beta * pg.B + b) * 128, find_key(gk, k), k, xi};
                    jb.tstride = Jp * 128;
                    jobs.push_back(jb);
                }
            }
        }
        if (!jobs.empty()) RUN(ks_run(c, l, ks, jobs, &srcs, Lc, st));
    }
    // 5. per group: the unrotated u-blocks and the padding into its region; per (group,
    //    stream): diagonals on the fly, chunk by chunk of giant indices, and the
    //    multiply-accumulate into the pair's giant accumulators
    std::vector<std::vector<uint64_t*>> A(npairs);
    {
        size_t go = 0;
        for (uint32_t pp = 0; pp < npairs; pp++) {
            const PlanGroup& pg = pl.groups[pp / S];
            A[pp].resize(sv / pg.B);
            for (auto& x : A[pp]) x = gbuf + (go++) * CW;
        }
    }
    for (uint32_t g = 0; g < G; g++) {
        const PlanGroup& pg = pl.groups[g];
        const uint32_t J = pg.k * pg.B, Gn = sv / pg.B;
        std::vector<const uint64_t*> hptr(J);
        for (uint32_t beta = 0; beta < pg.k; beta++)
            for (uint32_t b = 0; b < pg.B; b++) hptr[beta * pg.B + b] = b == 0 ? ublock(pg, beta) : kRtInPlace;
        const std::vector<uint32_t> work = diag_gather_list(hptr, 1, (int)J);
        void *drp = nullptr, *dwk = nullptr;
        if (!stage_many(l, {{hptr.data(), sizeof(uint64_t*) * hptr.size(), &drp},
                            {work.data(), sizeof(uint32_t) * work.size(), &dwk}},
                        st))
            return HC_ENOMEM;
        uint64_t* Rg = Rt + rt_off[g];
        k_diag_gather(c, Rg, (const uint64_t* const*)drp, (const uint32_t*)dwk, (int)work.size(), 1, (int)J, Lc, st);
        for (uint32_t si = 0; si < S; si++) {
            const uint32_t pp = g * S + si;
            const auto& sm = pl.streams[si];
            const uint32_t col0 = (uint32_t)sm.first, col1 = sm.second >= 0 ? (uint32_t)sm.second : 0xffffffffu;
            std::vector<uint32_t> hprm;
            std::vector<uint64_t*> haptr;
            for (uint32_t g0 = 0; g0 < Gn; g0 += Gc[g]) {
                const uint32_t gc = std::min(Gc[g], Gn - g0);
                hprm.clear();
                for (uint32_t beta = 0; beta < pg.k; beta++)  // chunk order (beta, b, g)
                    for (uint32_t b = 0; b < pg.B; b++)
                        for (uint32_t gi = 0; gi < gc; gi++) {
                            const uint32_t i = beta / 2;  // group-local ciphertext
                            const bool swapped = beta % 2 == 1;
                            hprm.push_back(swapped ? 2 * i + 1 : 2 * i);
                            hprm.push_back(swapped ? 2 * i : 2 * i + 1);
                            hprm.push_back(g0 + gi);
                            hprm.push_back(b);
                            hprm.push_back(col0);
                            hprm.push_back(col1);
                            hprm.push_back((uint32_t)pg.rec_start);
                        }
                const int cnt = (int)(hprm.size() / 7);
                haptr.assign(A[pp].begin() + g0, A[pp].begin() + g0 + gc);
                void *dprm = nullptr, *dap = nullptr;
                if (!stage_many(l, {{hprm.data(), sizeof(uint32_t) * hprm.size(), &dprm},
                                    {haptr.data(), sizeof(uint64_t*) * haptr.size(), &dap}},
                                st))
                    return HC_ENOMEM;
                k_diag_gen_db(c, Dp, (const uint32_t*)dprm, cnt, sv, pg.B, db ? db->d_raw : nullptr, db ? db->N : 0,
                              st);
                ntt32(c, Dp, cnt, true, st);
                k_lift(c, D, Dp, cnt, true, Lc, st);
                ntt64(c, D, PW, cnt, 0, Lc, false, st);
                k_diag_split(c, D, (size_t)cnt * PW, Lc, st);
                RUN(k_diag_mac(c, (uint64_t* const*)dap, Rg, D, diag_layout_natural(c, Lc, gc), 1, (int)J, (int)gc,
                               false, Lc, st));
            }
        }
    }
    // 6. giant steps: one summed key switch per pair
    {
        std::vector<KsJob> jobs;
        std::vector<uint32_t> grp;
        std::vector<uint64_t*> outs;
        std::vector<EwJob> add;
        for (uint32_t pp = 0; pp < npairs; pp++) {
            const PlanGroup& pg = pl.groups[pp / S];
            const uint32_t Gn = sv / pg.B;
            uint64_t* y = ybuf + (size_t)pp * CW;
            if (Gn == 1) {
                HC_CHECK(hipMemcpyAsync(y, A[pp][0], sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
                continue;
            }
            for (uint32_t gi = 1; gi < Gn; gi++) {
                const uint32_t k = rot_elt(c, (int64_t)gi * pg.B);
                jobs.push_back(KsJob{A[pp][gi], nullptr, find_key(gk, k), k, 0});
                grp.push_back((uint32_t)outs.size());
            }
            outs.push_back(gout + (size_t)pp * CW);
            add.push_back(EwJob{y, A[pp][0], gout + (size_t)pp * CW});
        }
        if (!jobs.empty()) RUN(ks_run_sum(c, l, ks, jobs, grp, outs, TA, C0A, Lc, st));
        RUN(ew_run(c, l, add, Lc, false, st));
    }
    // 7. rotate-and-sum: y += Rot_row(y; sh), sh = s, 2s, .., n/4
    for (uint64_t sh = sv; sh < (uint64_t)c.nh; sh *= 2) {
        const uint32_t k = rot_elt(c, (int64_t)sh);
        std::vector<KsJob> jobs;
        for (uint32_t pp = 0; pp < npairs; pp++)
            jobs.push_back(KsJob{ybuf + pp * CW, ytmp + pp * CW, find_key(gk, k), k, 0});
        RUN(ks_run(c, l, ks, jobs, nullptr, Lc, st));
        k_add(c, ybuf, ybuf, ytmp, 0, Lc, 2 * (int)npairs, PW, st);
    }
    // 8. merge the bands into one ciphertext
    uint64_t* res = ybuf;
    if (pl.bands > 1) {
        const uint64_t* ms = nullptr;
        RUN(prefix_mask(c, sv, &ms));
        std::vector<EwJob> mul;
        std::vector<KsJob> jobs;
        for (uint32_t b = 0; b < pl.bands; b++) {
            mul.push_back(EwJob{b == 0 ? mrot : mbuf + b * CW, ybuf + b * CW, ms});
            if (b > 0) {
                const uint32_t k = rot_elt(c, -(int64_t)b * sv);
                jobs.push_back(KsJob{mbuf + b * CW, mrot + b * CW, find_key(gk, k), k, 0});
            }
        }
        RUN(ew_run(c, l, mul, Lc, true, st));
        RUN(ks_run(c, l, ks, jobs, nullptr, Lc, st));
        k_sum_cts(c, outN, mrot, 1, (int)pl.bands, Lc, st);
        res = outN;
    }
    // 9. the answer in the coefficient domain, switched to out_level primes
    ntt64(c, res, PW, 2, 0, Lc, true, st);
    if (pl.out_level < Lc) RUN(mod_switch_coef(c, ct_out, res, 1, Lc, pl.out_level, ytmp, st));
    else HC_CHECK(hipMemcpyAsync(ct_out, res, sizeof(uint64_t) * CW, hipMemcpyDeviceToDevice, st));
#undef RUN
    HC_CHECK(hipGetLastError());
    return HC_OK;
}

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_plan_plain_db(hc_context* cp, uint64_t N, uint32_t ncol, uint32_t t_bound,
                                      uint32_t comp_level, uint32_t out_level, uint32_t* elements_out,
                                      uint32_t* count, hc_compress_info* info) {
    if (!cp || !count) return HC_EINVAL;
    Plan pl;
    hc_status s = make_plan_plain_db(*cp, N, ncol, t_bound, comp_level, out_level, pl);
    if (s != HC_OK) return s;
    fill_info(pl, info);
    uint32_t cap = *count;
    *count = (uint32_t)pl.keys.size();
    if (cap < pl.keys.size()) return HC_EINVAL;
    if (elements_out)
        for (size_t i = 0; i < pl.keys.size(); i++) elements_out[i] = pl.keys[i];
    return HC_OK;
}

extern "C" hc_status hc_compress_plain_db(hc_context* cp, const hc_gk* gk, const hc_db* db, const uint64_t* ct_v,
                                          uint64_t N, uint32_t t_bound, uint32_t comp_level, uint32_t out_level,
                                          uint64_t* ct_out, hc_compress_info* info, hipStream_t st) {
    if (!cp || !gk || !ct_v || !ct_out) return HC_EINVAL;
    HC_CHECK(hipSetDevice(cp->device));
    Plan pl;
    hc_status s = make_plan_plain_db(*cp, N, db ? db->ncol : 0, t_bound, comp_level, out_level, pl);
    if (s != HC_OK) return s;
    s = compress_plain_db_run(*cp, cp->lane, gk, db, ct_v, ct_out, pl, st);
    if (s == HC_OK) fill_info(pl, info);
    return s;
}
