// Host orchestration of the HE operations: encoding, key generation,
// encryption, key switching (plain and hoisted rotations) and the
// kernel-level ABI. Every step runs in the device kernels of ntt.hip / ops.hip.
#include <string.h>

#include <algorithm>
#include <tuple>

#include "he.h"

namespace hc {

uint64_t tag_u64(const char* s) {
    uint64_t t = 0;
    for (int i = 0; i < 8 && s[i]; i++) t |= (uint64_t)(uint8_t)s[i] << (8 * i);
    return t;
}

// slots (host, count x 2 x nh) -> plaintext multipliers [count][L][n] in the NTT
// domain (Montgomery form if mont), via the inverse slot transform mod p and the
// centred lift.
hc_status encode_plain(Ctx& c, uint64_t* out, const uint32_t* host_slots, int count, bool mont,
                       hipStream_t st) {
    const size_t n = c.n;
    uint32_t *d_slots = nullptr, *d_eval = nullptr;
    HC_CHECK(hipMalloc((void**)&d_slots, sizeof(uint32_t) * n * count));
    HC_CHECK(hipMalloc((void**)&d_eval, sizeof(uint32_t) * n * count));
    HC_CHECK(hipMemcpyAsync(d_slots, host_slots, sizeof(uint32_t) * n * count, hipMemcpyHostToDevice, st));
    k_slots_to_eval(c, d_eval, d_slots, count, st);
    ntt32(c, d_eval, count, true, st);
    k_lift(c, out, d_eval, count, mont, c.L, st);
    ntt64(c, out, (size_t)c.L * n, count, 0, c.L, false, st);
    HC_CHECK(hipStreamSynchronize(st));
    HC_CHECK(hipFree(d_slots));
    HC_CHECK(hipFree(d_eval));
    return HC_OK;
}

hc_status prefix_mask(Ctx& c, uint32_t s, const uint64_t** out) {
    std::lock_guard<std::mutex> g(c.lazy_mu);
    auto it = c.prefix_masks.find(s);
    if (it != c.prefix_masks.end()) { *out = it->second; return HC_OK; }
    std::vector<uint32_t> sl((size_t)c.n, 0);
    for (uint32_t i = 0; i < s; i++) { sl[i] = 1; sl[c.nh + i] = 1; }
    uint64_t* d = nullptr;
    HC_CHECK(hipMalloc((void**)&d, sizeof(uint64_t) * (size_t)c.L * c.n));
    hc_status stt = encode_plain(c, d, sl.data(), 1, true, 0);
    if (stt != HC_OK) { (void)hipFree(d); return stt; }
    c.prefix_masks[s] = d;
    *out = d;
    return HC_OK;
}

// ------------------------------------------------------------------ staging

void stage_reset(Lane& l, hipStream_t st) {
    // The workspace is reused in stream order; on another stream the previous call
    // must be done. The staging area is free once its last copy has run, so on the
    // same stream the host prepares the next call while the GPU finishes this one.
    // A lane being captured into a graph is fresh and the graph's own: nothing to wait for.
    if (l.capture) {
        l.stage_used = 0;
        l.stage_stream = st;
        return;
    }
    if (l.stage_stream != st) (void)hipStreamSynchronize(l.stage_stream);
    if (l.copied) (void)hipEventSynchronize(l.copied);
    l.stage_used = 0;
    l.stage_stream = st;
}

void* stage_bytes(Lane& l, const void* data, size_t bytes, hipStream_t st) {
    size_t off = (l.stage_used + 255) & ~(size_t)255;
    if (off + bytes > l.stage_cap) return nullptr;
    memcpy(l.stage_host + off, data, bytes);
    if (hipMemcpyAsync(l.stage_dev + off, l.stage_host + off, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return nullptr;
    if (!l.capture && l.copied && hipEventRecord(l.copied, st) != hipSuccess) return nullptr;
    l.stage_used = off + bytes;
    return l.stage_dev + off;
}

bool stage_many(Lane& l, std::initializer_list<StagePart> parts, hipStream_t st) {
    const size_t first = (l.stage_used + 255) & ~(size_t)255;
    size_t off = first;
    for (const StagePart& p : parts) {
        off = (off + 255) & ~(size_t)255;
        if (off + p.bytes > l.stage_cap) return false;
        memcpy(l.stage_host + off, p.data, p.bytes);
        *p.dev = l.stage_dev + off;
        off += p.bytes;
    }
    if (off > first) {
        if (hipMemcpyAsync(l.stage_dev + first, l.stage_host + first, off - first, hipMemcpyHostToDevice, st) !=
            hipSuccess)
            return false;
        if (!l.capture && l.copied && hipEventRecord(l.copied, st) != hipSuccess) return false;
    }
    l.stage_used = off;
    return true;
}

// ------------------------------------------------------------------ batched key switching

static size_t ks_src_words(const Ctx& c, int Lc) {
    const int R = Lc + c.K, dn = Lc / c.alpha;
    return (size_t)c.n * (Lc + (size_t)dn * R);
}
static size_t ks_job_words(const Ctx& c, int Lc) {
    const int R = Lc + c.K;
    return (size_t)c.n * (2 * (size_t)R + 2 * (size_t)Lc);
}

static const size_t kKsScratchBudget = (size_t)12 << 30;

size_t ks_scratch_bytes(const Ctx& c, int Lc, int max_jobs) {
    const size_t per = 8 * (ks_src_words(c, Lc) + ks_job_words(c, Lc));
    size_t m = kKsScratchBudget / per;
    if (m > (size_t)max_jobs) m = (size_t)max_jobs;
    if (m < 1) m = 1;
    return m * per + 4 * 256;
}

KsScratch ks_scratch(Ctx& c, Arena& a, int Lc, int max_jobs) {
    KsScratch s;
    const size_t per = 8 * (ks_src_words(c, Lc) + ks_job_words(c, Lc));
    size_t m = kKsScratchBudget / per;
    if (m > (size_t)max_jobs) m = (size_t)max_jobs;
    if (m < 1) m = 1;
    s.maxU = s.maxM = (int)m;
    const int R = Lc + c.K, dn = Lc / c.alpha;
    s.tmpC = a.take<uint64_t>(m * Lc * (size_t)c.n);
    s.X = a.take<uint64_t>(m * (size_t)dn * R * c.n);
    s.T = a.take<uint64_t>(m * 2 * (size_t)R * c.n);
    s.conv = a.take<uint64_t>(m * 2 * (size_t)Lc * c.n);
    return s;
}

// Raise U sources for key switching at level Lc: c1 (rotated by the job's element
// if permute), ModUp into dn digits over PQ, NTT domain. Each digit's own rows are
// copied in the NTT domain before the inverse transform; only the rows ModUp
// computes are transformed forward.
// ModDown's middle for M jobs at level Lc: the special rows of T [M][2][R][n] back to
// coefficients, converted to the ciphertext primes, and forward into conv [M][2][Lc][n]
// (NTT domain). At ring 2^16 the conversion is fused with the forward high-bit pass.
static void moddown_conv(Ctx& c, uint64_t* conv, uint64_t* T, int M, int Lc, hipStream_t st) {
    const size_t n = c.n;
    const int R = Lc + c.K;
    if (conv_fused_ring(c)) {
        ntt64_inverse_conv(c, T + (size_t)Lc * n, (size_t)R * n, 2 * M, c.L, c.K, st);
        k_moddown_fused(c, conv, T, M, Lc, st);
        ntt64_low_pass(c, conv, (size_t)Lc * n, 2 * M, 0, Lc, false, st);
        return;
    }
    ntt64(c, T + (size_t)Lc * n, (size_t)R * n, 2 * M, c.L, c.K, true, st);
    kb_conv(c, conv, T, M, Lc, st);
    ntt64(c, conv, (size_t)Lc * n, 2 * M, 0, Lc, false, st);
}

static void ks_raise(Ctx& c, KsScratch& s, const KsJob* d, int U, int Lc, bool permute, hipStream_t st) {
    const size_t n = c.n;
    const int R = Lc + c.K, dn = Lc / c.alpha, a = c.alpha;
    (void)permute;  // jobs carry their element (k = 1: no rotation)
    if (conv_fused_ring(c)) {
        // the rotated c1 taken inside the inverse transform's first pass, its last pass
        // scaled by the conversion's factor, then the conversion fused with the forward
        // high-bit pass, then the forward low-bit pass of every converted row
        ntt_take_c1_low(c, d, s.tmpC, s.X, U, Lc, st);
        ntt64_inverse_high_conv(c, s.tmpC, (size_t)Lc * n, U, 0, Lc, st);
        k_modup_fused(c, s.X, s.tmpC, U, Lc, st);
        ntt64_low_raise(c, s.X, (size_t)R * n, U * dn, Lc, dn, st);
        ntt64_low_pass(c, s.X + (size_t)Lc * n, (size_t)R * n, U * dn, c.L, c.K, false, st);
        return;
    }
    kb_take_c1(c, s.tmpC, s.X, d, U, Lc, st);
    ntt64(c, s.tmpC, (size_t)Lc * n, U, 0, Lc, true, st);
    kb_modup(c, s.X, s.tmpC, U, Lc, false, st);
    for (int j = 0; j < dn; j++) {
        uint64_t* Xj = s.X + (size_t)j * R * n;
        if (j > 0) ntt64(c, Xj, (size_t)dn * R * n, U, 0, j * a, false, st);
        if ((j + 1) * a < Lc)
            ntt64(c, Xj + (size_t)(j + 1) * a * n, (size_t)dn * R * n, U, (j + 1) * a, Lc - (j + 1) * a, false, st);
    }
    ntt64(c, s.X + (size_t)Lc * n, (size_t)R * n, U * dn, c.L, c.K, false, st);
}

// Jobs of a pass in key order (stable), so that jobs sharing a key are adjacent; the
// order of jobs never changes a result.
static void sort_by_key(std::vector<KsJob>& jb) {
    std::stable_sort(jb.begin(), jb.end(),
                     [](const KsJob& x, const KsJob& y) { return (uintptr_t)x.key < (uintptr_t)y.key; });
}

// Runs of up to KS_RUN adjacent jobs with the same key, for kb_inner.
static std::vector<KsRun> key_runs(const std::vector<KsJob>& jb) {
    std::vector<KsRun> runs;
    for (uint32_t i = 0; i < (uint32_t)jb.size(); i++) {
        if (!runs.empty() && runs.back().cnt < (uint32_t)KS_RUN && jb[runs.back().j0].key == jb[i].key)
            runs.back().cnt++;
        else
            runs.push_back(KsRun{i, 1});
    }
    return runs;
}

// Rotations at level Lc. Plain (srcs == nullptr): each job raises its own rotated c1.
// Hoisted: srcs[u] are raised once (unrotated) and every job with xidx = u rotates
// the raised digits instead. Jobs are processed in passes of at most maxM, each pass
// in key order so that jobs sharing a key read it once (kb_inner). A pass's tables
// (jobs, key runs, and the raised sources when they start a chunk) go to the device
// in one copy.
hc_status ks_run(Ctx& c, Lane& l, KsScratch& s, const std::vector<KsJob>& jobs,
                 const std::vector<const uint64_t*>* srcs, int Lc, hipStream_t st) {
    if (!s.tmpC || !s.X || !s.T || !s.conv) return HC_ENOMEM;
    const size_t n = c.n;
    const int R = Lc + c.K;
    auto raise = [&](const KsJob* d, int U, bool permute) { ks_raise(c, s, d, U, Lc, permute, st); };
    auto finish = [&](const KsJob* d, const KsRun* runs, int nruns, int M, bool hoisted, int maxrun) {
        // the key products' special rows inside the inverse transform's first pass (ring
        // 2^16) or by kb_inner, their ciphertext rows inside the final step
        if (conv_fused_ring(c)) {
            ntt_inner_low(c, d, s.X, s.T, M, Lc, hoisted, st);
            ntt64_inverse_high_conv(c, s.T + (size_t)Lc * n, (size_t)R * n, 2 * M, c.L, c.K, st);
            k_moddown_fused(c, s.conv, s.T, M, Lc, st);
            ntt64_low_pass(c, s.conv, (size_t)Lc * n, 2 * M, 0, Lc, false, st);
        } else {
            kb_inner(c, s.T, s.X, d, runs, nruns, M, Lc, hoisted, st, Lc);
            moddown_conv(c, s.conv, s.T, M, Lc, st);
        }
        kb_final_inner(c, d, runs, nruns, s.X, s.conv, M, Lc, hoisted, st, maxrun);
    };
    auto longest = [](const std::vector<KsRun>& runs) {
        uint32_t m = 0;
        for (const KsRun& r : runs) m = std::max(m, r.cnt);
        return (int)m;
    };
    if (!srcs) {
        std::vector<KsJob> all(jobs);
        sort_by_key(all);
        for (size_t m0 = 0; m0 < all.size(); m0 += s.maxM) {
            const int M = (int)std::min<size_t>(s.maxM, all.size() - m0);
            std::vector<KsJob> jb(all.begin() + m0, all.begin() + m0 + M);
            for (int i = 0; i < M; i++) jb[i].xidx = (uint32_t)i;
            const std::vector<KsRun> runs = key_runs(jb);
            void *d = nullptr, *dr = nullptr;
            if (!stage_many(l, {{jb.data(), sizeof(KsJob) * M, &d}, {runs.data(), sizeof(KsRun) * runs.size(), &dr}},
                            st))
                return HC_ENOMEM;
            raise((const KsJob*)d, M, true);
            finish((const KsJob*)d, (const KsRun*)dr, (int)runs.size(), M, false, longest(runs));
        }
        return HC_OK;
    }
    const size_t U = srcs->size();
    for (size_t u0 = 0; u0 < U; u0 += s.maxU) {
        const int Uc = (int)std::min<size_t>(s.maxU, U - u0);
        std::vector<KsJob> sj(Uc);
        for (int i = 0; i < Uc; i++) sj[i] = KsJob{(*srcs)[u0 + i], nullptr, nullptr, 1u, (uint32_t)i};
        std::vector<KsJob> mine;
        for (const KsJob& j : jobs)
            if (j.xidx >= u0 && j.xidx < u0 + Uc) {
                KsJob t = j;
                t.xidx = (uint32_t)(j.xidx - u0);
                mine.push_back(t);
            }
        sort_by_key(mine);
        for (size_t m0 = 0; m0 < std::max<size_t>(mine.size(), 1); m0 += s.maxM) {
            const int M = (int)std::min<size_t>(s.maxM, mine.size() - std::min(m0, mine.size()));
            std::vector<KsJob> jb(mine.begin() + m0, mine.begin() + m0 + M);
            const std::vector<KsRun> runs = key_runs(jb);
            void *ds = nullptr, *d = nullptr, *dr = nullptr;
            const bool first = m0 == 0;
            if (!stage_many(l, {{sj.data(), first ? sizeof(KsJob) * Uc : 0, &ds},
                                {jb.data(), sizeof(KsJob) * M, &d},
                                {runs.data(), sizeof(KsRun) * runs.size(), &dr}},
                            st))
                return HC_ENOMEM;
            if (first) raise((const KsJob*)ds, Uc, false);
            if (M > 0) finish((const KsJob*)d, (const KsRun*)dr, (int)runs.size(), M, true, longest(runs));
        }
    }
    return HC_OK;
}

// Sums of plain rotations, one ModDown per sum: for each group g, outs[g] = sum of
// Rot_k(in) over the jobs with group[i] == g, whose key products are added over PQ
// (TA, groups x [2][Lc+K][n]) and whose rotated c0 are added (C0A, groups x [Lc][n])
// before a single ModDown. Passes run in key order (jobs of one pass that share a key
// read it together); every sum is exact, so the order does not change a result.
hc_status ks_run_sum(Ctx& c, Lane& l, KsScratch& s, const std::vector<KsJob>& jobs,
                     const std::vector<uint32_t>& group, const std::vector<uint64_t*>& outs, uint64_t* TA,
                     uint64_t* C0A, int Lc, hipStream_t st) {
    if (!s.tmpC || !s.X || !s.T || !s.conv || !TA || !C0A || group.size() != jobs.size()) return HC_ENOMEM;
    const size_t n = c.n, G = outs.size();
    const int R = Lc + c.K;
    k_zero(c, TA, G * 2 * (size_t)R * n, st);
    k_zero(c, C0A, G * (size_t)Lc * n, st);
    // job order by key, carrying each job's group
    std::vector<uint32_t> order(jobs.size());
    for (uint32_t i = 0; i < (uint32_t)jobs.size(); i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return (uintptr_t)jobs[x].key < (uintptr_t)jobs[y].key;
    });
    for (size_t m0 = 0; m0 < jobs.size(); m0 += s.maxM) {
        const int M = (int)std::min<size_t>(s.maxM, jobs.size() - m0);
        std::vector<KsJob> jb(M);
        for (int i = 0; i < M; i++) {
            jb[i] = jobs[order[m0 + i]];
            jb[i].xidx = (uint32_t)i;
        }
        // members of each group within the pass
        std::vector<uint32_t> members(M);
        for (int i = 0; i < M; i++) members[i] = (uint32_t)i;
        std::stable_sort(members.begin(), members.end(),
                         [&](uint32_t x, uint32_t y) { return group[order[m0 + x]] < group[order[m0 + y]]; });
        std::vector<KsGroupRange> rg;
        for (int i = 0; i < M; i++) {
            const uint32_t g = group[order[m0 + members[i]]];
            if (rg.empty() || rg.back().g != g) rg.push_back(KsGroupRange{g, (uint32_t)i, (uint32_t)i + 1, 0});
            else rg.back().j1 = (uint32_t)i + 1;
        }
        int nkeys = 0;
        for (int i = 0; i < M; i++) nkeys += (i == 0 || jb[i].key != jb[i - 1].key) ? 1 : 0;
        void *dv = nullptr, *dgv = nullptr, *dmv = nullptr;
        if (!stage_many(l, {{jb.data(), sizeof(KsJob) * M, &dv}, {rg.data(), sizeof(KsGroupRange) * rg.size(), &dgv},
                            {members.data(), sizeof(uint32_t) * M, &dmv}},
                        st))
            return HC_ENOMEM;
        const KsJob* d = (const KsJob*)dv;
        ks_raise(c, s, d, M, Lc, true, st);
        kb_inner_sum(c, TA, C0A, s.X, d, (const KsGroupRange*)dgv, (const uint32_t*)dmv, (int)rg.size(), M, nkeys,
                     Lc, st);
    }
    // one ModDown per group (TA is consumed in place)
    for (size_t g0 = 0; g0 < G; g0 += s.maxM) {
        const int Mg = (int)std::min<size_t>(s.maxM, G - g0);
        uint64_t* T = TA + g0 * 2 * (size_t)R * n;
        std::vector<KsJob> fj(Mg);
        for (int i = 0; i < Mg; i++) fj[i] = KsJob{C0A + (g0 + i) * (size_t)Lc * n, outs[g0 + i], nullptr, 1u, 0u};
        const KsJob* df = (const KsJob*)stage_bytes(l, fj.data(), sizeof(KsJob) * Mg, st);
        if (!df) return HC_ENOMEM;
        moddown_conv(c, s.conv, T, Mg, Lc, st);
        kb_final(c, df, T, s.conv, Mg, Lc, st);
    }
    return HC_OK;
}

hc_status ew_run(Ctx& c, Lane& l, const std::vector<EwJob>& jobs, int Lc, bool mul, hipStream_t st) {
    if (jobs.empty()) return HC_OK;
    const EwJob* d = (const EwJob*)stage_bytes(l, jobs.data(), sizeof(EwJob) * jobs.size(), st);
    if (!d) return HC_ENOMEM;
    k_ew_jobs(c, d, (int)jobs.size(), Lc, mul, st);
    return HC_OK;
}

// Constants for dropping the primes Lc..Lin-1 (product D) of a ciphertext at level Lin,
// for every 1 <= Lc < Lin <= L, packed in one device buffer (context creation).
hc_status build_ms_tables(Ctx& c) {
    const int L = c.L;
    std::vector<uint64_t> all;
    std::vector<std::tuple<int, size_t, size_t, size_t, size_t>> offs;  // key, inv, cst, dinv, ninv
    const size_t n = c.n;
    for (int Lin = 2; Lin <= L; Lin++)
        for (int Lc = 1; Lc < Lin; Lc++) {
            const int nd = Lin - Lc;
            const size_t oi = all.size(), oc = oi + 2 * (size_t)nd, od = oc + (size_t)nd * Lc;
            const size_t on = od + 2 * (size_t)Lc;
            all.resize(on + (Lin == L ? 4 * (size_t)L : 0));
            for (int j = 0; j < nd; j++) {
                const uint64_t qj = c.primes[Lc + j];
                uint64_t h = 1;  // (D / q_j) mod q_j
                for (int j2 = 0; j2 < nd; j2++)
                    if (j2 != j) h = h_mulmod(h, c.primes[Lc + j2] % qj, qj);
                all[oi + 2 * j] = h_invmod(h, qj);
                all[oi + 2 * j + 1] = h_shoup_const(all[oi + 2 * j], qj);
                for (int i = 0; i < Lc; i++) {
                    const uint64_t qi = c.primes[i];
                    uint64_t hi = 1;
                    for (int j2 = 0; j2 < nd; j2++)
                        if (j2 != j) hi = h_mulmod(hi, c.primes[Lc + j2] % qi, qi);
                    all[oc + (size_t)j * Lc + i] = h_to_mont(hi, qi);
                }
            }
            for (int i = 0; i < Lc; i++) {
                const uint64_t qi = c.primes[i];
                uint64_t D = 1;
                for (int j = 0; j < nd; j++) D = h_mulmod(D, c.primes[Lc + j] % qi, qi);
                all[od + 2 * i] = h_invmod(D, qi);
                all[od + 2 * i + 1] = h_shoup_const(all[od + 2 * i], qi);
            }
            // from the top level: n^-1 and W^-1[1] n^-1 (W^-1[1] the inverse table's word
            // of index 1), times (D/q_j)^-1 on the dropped rows
            if (Lin == L)
                for (int i = 0; i < L; i++) {
                    const uint64_t q = c.primes[i];
                    const uint64_t f = i < Lc ? 1 : all[oi + 2 * (size_t)(i - Lc)];
                    const uint64_t ni = h_mulmod(h_invmod(n % q, q), f, q);
                    const uint64_t w1 = c.h_tw[(size_t)i * 4 * n + 2 * n + 2];
                    all[on + 4 * i] = ni;
                    all[on + 4 * i + 1] = h_shoup_const(ni, q);
                    all[on + 4 * i + 2] = h_mulmod(w1, ni, q);
                    all[on + 4 * i + 3] = h_shoup_const(all[on + 4 * i + 2], q);
                }
            offs.emplace_back(Lin * 256 + Lc, oi, oc, od, Lin == L ? on : SIZE_MAX);
        }
    if (all.empty()) return HC_OK;
    uint64_t* d = nullptr;
    HC_CHECK(hipMalloc((void**)&d, sizeof(uint64_t) * all.size()));
    c.owned.push_back(d);
    HC_CHECK(hipMemcpy(d, all.data(), sizeof(uint64_t) * all.size(), hipMemcpyHostToDevice));
    for (auto& o : offs)
        c.ms_tabs[std::get<0>(o)] = Ctx::MsTab{d + std::get<1>(o), d + std::get<2>(o), d + std::get<3>(o),
                                               std::get<4>(o) == SIZE_MAX ? nullptr : d + std::get<4>(o)};
    return HC_OK;
}

static const Ctx::MsTab* ms_table(const Ctx& c, int Lin, int Lc) {
    auto it = c.ms_tabs.find(Lin * 256 + Lc);
    return it == c.ms_tabs.end() ? nullptr : &it->second;
}

// out [count][2][Lc][n] = in [count][2][L][n] with the primes Lc..L-1 dropped (NTT domain
// in and out). The dropped rows of `in` are left in the coefficient domain. conv: 2 Lc n
// words per ciphertext.
hc_status mod_switch_batch(Ctx& c, uint64_t* out, uint64_t* in, int count, int Lc, uint64_t* conv,
                           hipStream_t st, const uint64_t* coef, int ncoef, bool low_done) {
    const Ctx::MsTab* t = ms_table(c, c.L, Lc);
    if (!t) return HC_EINVAL;
    if (!coef || ncoef < 0) ncoef = 0;
    if (ncoef > count) return HC_EINVAL;
    const bool two_pass = c.logn == 16 && t->ninv;
    if (low_done && !two_pass) return HC_EINVAL;
    const size_t n = c.n, Ln = (size_t)c.L * n, skip = 2 * (size_t)ncoef;
    // the dropped rows in coefficient form: given for the first ncoef, transformed back
    // for the rest (at ring 2^16 already multiplied by their factors (D/q_j)^-1, which the
    // transform's final constants carry)
    const int nt = 2 * (count - ncoef);
    uint64_t* tin = in + skip * Ln + (size_t)Lc * n;
    if (two_pass) {
        if (!low_done) ntt64_low_pass(c, tin, Ln, nt, Lc, c.L - Lc, true, st);
        ntt64_inverse_high_tab(c, tin, Ln, nt, Lc, c.L - Lc, t->ninv, st);
    } else {
        ntt64(c, tin, Ln, nt, Lc, c.L - Lc, true, st);
    }
    if (ncoef > 0) k_ms_conv(c, conv, coef, t->inv, t->cst, c.L, Lc, ncoef, st);
    k_ms_conv(c, conv + skip * Lc * n, in + skip * Ln, two_pass ? nullptr : t->inv, t->cst, c.L, Lc, count - ncoef,
              st);
    ntt64(c, conv, (size_t)Lc * n, 2 * count, 0, Lc, false, st);
    k_ms_final(c, out, in, conv, t->dinv, c.L, Lc, count, st);
    return HC_OK;
}

// out [count][2][Lo][n] = in [count][2][Lin][n] with the primes Lo..Lin-1 dropped, both in the
// coefficient domain (no transform: the conversion and the division are element-wise).
// conv: 2 Lo n words per ciphertext.
hc_status mod_switch_coef(const Ctx& c, uint64_t* out, const uint64_t* in, int count, int Lin, int Lo,
                          uint64_t* conv, hipStream_t st) {
    const Ctx::MsTab* t = ms_table(c, Lin, Lo);
    if (!t || count < 1) return HC_EINVAL;
    k_ms_conv(c, conv, in, t->inv, t->cst, Lin, Lo, count, st);
    k_ms_final(c, out, in, conv, t->dinv, Lin, Lo, count, st);
    return HC_OK;
}

const uint64_t* find_key(const hc_gk* gk, uint32_t k) {
    auto it = gk->keys.find(k);
    return it == gk->keys.end() ? nullptr : it->second;
}

}  // namespace hc

using namespace hc;

// ------------------------------------------------------------------ keys

extern "C" hc_status hc_keygen(hc_context* cp, const uint8_t seed[32], hc_sk** skp, hc_pk** pkp) {
    if (!cp || !seed || !skp || !pkp) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    const size_t n = c.n, nq = c.nq, L = c.L;
    hipStream_t st = 0;
    hc_sk* sk = new hc_sk();
    hc_pk* pk = new hc_pk();
    int64_t* d_raw = nullptr;
    uint64_t *d_e = nullptr;
    HC_CHECK(hipMalloc((void**)&sk->d_s_mont, sizeof(uint64_t) * nq * n));
    HC_CHECK(hipMalloc((void**)&pk->d_a, sizeof(uint64_t) * L * n));
    HC_CHECK(hipMalloc((void**)&pk->d_b, sizeof(uint64_t) * L * n));
    HC_CHECK(hipMalloc((void**)&d_raw, sizeof(int64_t) * n));
    HC_CHECK(hipMalloc((void**)&d_e, sizeof(uint64_t) * L * n));
    // s: ternary, the same integer on every prime of PQ
    k_sample_small(c, sk->d_s_mont, d_raw, seed, tag_u64("sk"), 0, 1, 0, (int)nq, st);
    ntt64(c, sk->d_s_mont, nq * n, 1, 0, (int)nq, false, st);
    k_to_mont(c, sk->d_s_mont, 0, (int)nq, 1, 0, st);
    // pk = (e - a s, a) over Q
    k_sample_uniform(c, pk->d_a, seed, tag_u64("pk_a"), 0, 0, (int)L, st);
    ntt64(c, pk->d_a, L * n, 1, 0, (int)L, false, st);
    k_sample_small(c, d_e, nullptr, seed, tag_u64("pk_e"), 0, 2, 0, (int)L, st);
    ntt64(c, d_e, L * n, 1, 0, (int)L, false, st);
    k_keyrow(c, pk->d_b, d_e, pk->d_a, sk->d_s_mont, nullptr, nullptr, 0, (int)L, st);
    std::vector<int64_t> raw(n);
    HC_CHECK(hipMemcpyAsync(raw.data(), d_raw, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st));
    HC_CHECK(hipStreamSynchronize(st));
    sk->s.resize(n);
    for (size_t i = 0; i < n; i++) sk->s[i] = (int8_t)raw[i];
    HC_CHECK(hipFree(d_raw));
    HC_CHECK(hipFree(d_e));
    *skp = sk;
    *pkp = pk;
    return HC_OK;
}

extern "C" void hc_sk_destroy(hc_sk* sk) {
    if (!sk) return;
    (void)hipFree(sk->d_s_mont);
    delete sk;
}

extern "C" void hc_pk_destroy(hc_pk* pk) {
    if (!pk) return;
    (void)hipFree(pk->d_a);
    (void)hipFree(pk->d_b);
    delete pk;
}

namespace hc {

// Key-switching keys to s from sigma_k(s) (Galois keys, one per element; tags gk_a /
// gk_e, object (k << 16) | digit) or from s^2 (relin: one key stored under element 1;
// tags rk_a / rk_e, object = digit). Digit j of the key for target t:
// b_j = [-a_j s + e_j + P (Q/D_j) [(Q/D_j)^-1]_{D_j} t]_{PQ}.
hc_status ks_keygen(Ctx& c, const hc_sk* sk, const uint32_t* elements, uint32_t count, const uint8_t seed[32],
                    bool relin, hc_gk** out) {
    for (uint32_t i = 0; i < count; i++)
        if ((elements[i] & 1) == 0 || elements[i] >= 2u * c.n) return HC_EINVAL;
    HC_CHECK(hipSetDevice(c.device));
    const size_t n = c.n, nq = c.nq;
    hipStream_t st = 0;
    hc_gk* gk = new hc_gk();
    gk->dnum = c.dnum;
    gk->nq = c.nq;
    gk->n = c.n;
    uint64_t *d_e = nullptr, *d_rs = nullptr, *d_g = nullptr;
    HC_CHECK(hipMalloc((void**)&d_e, sizeof(uint64_t) * nq * n));
    HC_CHECK(hipMalloc((void**)&d_rs, sizeof(uint64_t) * nq * n));
    HC_CHECK(hipMalloc((void**)&d_g, sizeof(uint64_t) * c.dnum * nq));
    // gadget P (Q/D_j) [(Q/D_j)^-1]_{D_j}: P mod q_i on the digit's primes, 0 elsewhere
    std::vector<uint64_t> hmod(c.L);
    HC_CHECK(hipMemcpy(hmod.data(), c.d_pmodq, sizeof(uint64_t) * c.L, hipMemcpyDeviceToHost));
    std::vector<uint64_t> g((size_t)c.dnum * nq, 0);
    for (int j = 0; j < c.dnum; j++)
        for (int a = 0; a < c.alpha; a++) g[(size_t)j * nq + j * c.alpha + a] = hmod[j * c.alpha + a];
    HC_CHECK(hipMemcpy(d_g, g.data(), sizeof(uint64_t) * g.size(), hipMemcpyHostToDevice));
    std::vector<uint32_t> uniq(elements, elements + count);
    if (relin) uniq.assign(1, 1u);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    const uint64_t tag_a = tag_u64(relin ? "rk_a" : "gk_a"), tag_e = tag_u64(relin ? "rk_e" : "gk_e");
    for (uint32_t k : uniq) {
        uint64_t* key = nullptr;
        if (hipMalloc((void**)&key, sizeof(uint64_t) * c.dnum * 2 * nq * n) != hipSuccess) {
            hc_gk_destroy(gk);
            (void)hipFree(d_e); (void)hipFree(d_rs); (void)hipFree(d_g);
            return HC_ENOMEM;
        }
        gk->keys[k] = key;
        if (relin)  // s^2 in Montgomery form: (s R)(s R) R^-1
            k_mul_mont(c, d_rs, sk->d_s_mont, sk->d_s_mont, 0, (int)nq, st);
        else
            k_permute(c, d_rs, sk->d_s_mont, (int)nq, k, 1, 0, st);  // sigma_k(s), NTT domain
        for (int j = 0; j < c.dnum; j++) {
            uint64_t obj = relin ? (uint64_t)j : (((uint64_t)k << 16) | (uint64_t)j);
            uint64_t* b = key + (size_t)j * 2 * nq * n;
            uint64_t* a = b + nq * n;
            k_sample_uniform(c, a, seed, tag_a, obj, 0, (int)nq, st);
            ntt64(c, a, nq * n, 1, 0, (int)nq, false, st);
            k_sample_small(c, d_e, nullptr, seed, tag_e, obj, 2, 0, (int)nq, st);
            ntt64(c, d_e, nq * n, 1, 0, (int)nq, false, st);
            k_keyrow(c, b, d_e, a, sk->d_s_mont, d_rs, d_g + (size_t)j * nq, 0, (int)nq, st);
        }
        k_to_mont(c, key, 0, (int)nq, 2 * c.dnum, nq * n, st);
    }
    HC_CHECK(hipStreamSynchronize(st));
    HC_CHECK(hipFree(d_e));
    HC_CHECK(hipFree(d_rs));
    HC_CHECK(hipFree(d_g));
    *out = gk;
    return HC_OK;
}

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_galois_keygen(hc_context* cp, const hc_sk* sk, const uint32_t* elements,
                                      uint32_t count, const uint8_t seed[32], hc_gk** out) {
    if (!cp || !sk || !seed || !out || (count && !elements)) return HC_EINVAL;
    return ks_keygen(*cp, sk, elements, count, seed, false, out);
}

extern "C" void hc_gk_destroy(hc_gk* gk) {
    if (!gk) return;
    for (auto& kv : gk->keys) (void)hipFree(kv.second);
    delete gk;
}

// ------------------------------------------------------------------ database

extern "C" hc_status hc_db_upload(hc_context* cp, const uint32_t* cols, uint32_t ncol, uint64_t N,
                                  hc_db** out) {
    if (!cp || !out || N == 0 || (ncol && !cols)) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    const size_t n = c.n;
    hc_db* db = new hc_db();
    db->ncol = ncol;
    db->N = N;
    db->n_ct = (uint32_t)((N + n - 1) / n);
    if (ncol) {
        HC_CHECK(hipMalloc((void**)&db->d_pt, sizeof(uint64_t) * ncol * db->n_ct * c.L * n));
        std::vector<uint32_t> sl(n * db->n_ct), raw((size_t)ncol * N);
        for (uint32_t col = 0; col < ncol; col++) {
            std::fill(sl.begin(), sl.end(), 0u);
            for (uint64_t r = 0; r < N; r++) sl[r] = raw[(size_t)col * N + r] = cols[(size_t)col * N + r] % (uint32_t)c.p;
            // record r: ciphertext r / n, row (r % n) / nh, column r % nh = flat r % n
            hc_status s = encode_plain(c, db->d_pt + (size_t)col * db->n_ct * c.L * n, sl.data(),
                                       (int)db->n_ct, true, 0);
            if (s != HC_OK) { hc_db_destroy(db); return s; }
        }
        // the values themselves, for the unencrypted-database form's diagonals
        HC_CHECK(hipMalloc((void**)&db->d_raw, sizeof(uint32_t) * raw.size()));
        HC_CHECK(hipMemcpy(db->d_raw, raw.data(), sizeof(uint32_t) * raw.size(), hipMemcpyHostToDevice));
    }
    *out = db;
    return HC_OK;
}

extern "C" void hc_db_destroy(hc_db* db) {
    if (!db) return;
    (void)hipFree(db->d_pt);
    (void)hipFree(db->d_raw);
    delete db;
}

// ------------------------------------------------------------------ encryption

extern "C" hc_status hc_encrypt(hc_context* cp, const hc_pk* pk, const uint32_t* slots,
                                const uint8_t seed[32], uint64_t* ct_out, hipStream_t st) {
    if (!cp || !pk || !slots || !seed || !ct_out) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    const size_t n = c.n, L = c.L;
    uint64_t *u = nullptr, *e0 = nullptr, *e1 = nullptr;
    uint32_t *d_sl = nullptr, *d_m = nullptr;
    HC_CHECK(hipMalloc((void**)&u, sizeof(uint64_t) * L * n));
    HC_CHECK(hipMalloc((void**)&e0, sizeof(uint64_t) * L * n));
    HC_CHECK(hipMalloc((void**)&e1, sizeof(uint64_t) * L * n));
    HC_CHECK(hipMalloc((void**)&d_sl, sizeof(uint32_t) * n));
    HC_CHECK(hipMalloc((void**)&d_m, sizeof(uint32_t) * n));
    HC_CHECK(hipMemcpyAsync(d_sl, slots, sizeof(uint32_t) * n, hipMemcpyHostToDevice, st));
    k_slots_to_eval(c, d_m, d_sl, 1, st);
    ntt32(c, d_m, 1, true, st);  // m: coefficients in [0, p)
    k_sample_small(c, u, nullptr, seed, tag_u64("enc_u"), 0, 1, 0, (int)L, st);
    ntt64(c, u, L * n, 1, 0, (int)L, false, st);
    k_to_mont(c, u, 0, (int)L, 1, 0, st);
    k_sample_small(c, e0, nullptr, seed, tag_u64("enc_e0"), 0, 2, 0, (int)L, st);
    k_sample_small(c, e1, nullptr, seed, tag_u64("enc_e1"), 0, 2, 0, (int)L, st);
    k_mul_mont(c, ct_out, pk->d_b, u, 0, (int)L, st);
    k_mul_mont(c, ct_out + L * n, pk->d_a, u, 0, (int)L, st);
    ntt64(c, ct_out, L * n, 2, 0, (int)L, true, st);
    k_enc_finish(c, ct_out, e0, e1, d_m, st);
    HC_CHECK(hipStreamSynchronize(st));
    HC_CHECK(hipFree(u));
    HC_CHECK(hipFree(e0));
    HC_CHECK(hipFree(e1));
    HC_CHECK(hipFree(d_sl));
    HC_CHECK(hipFree(d_m));
    return HC_OK;
}

// ------------------------------------------------------------------ kernel-level ABI

extern "C" hc_status hc_ntt(hc_context* cp, uint64_t* data, uint32_t count, uint32_t limb_first,
                            uint32_t nlimbs, int inverse, hipStream_t st) {
    if (!cp || !data || limb_first + nlimbs > (uint32_t)cp->nq) return HC_EINVAL;
    HC_CHECK(hipSetDevice(cp->device));
    ntt64(*cp, data, (size_t)nlimbs * cp->n, (int)count, (int)limb_first, (int)nlimbs, inverse != 0, st);
    HC_CHECK(hipGetLastError());
    return HC_OK;
}

static hc_status rotate_common(hc_context* cp, const hc_gk* gk, const uint32_t* elts, uint32_t count,
                               const uint64_t* ct_in, uint64_t* cts_out, bool hoisted, int Lc, hipStream_t st) {
    if (!cp || !gk || !elts || !ct_in || !cts_out || count == 0) return HC_EINVAL;
    Ctx& c = *cp;
    if (Lc < c.alpha || Lc > c.L || Lc % c.alpha) return HC_EINVAL;
    HC_CHECK(hipSetDevice(c.device));
    const size_t Ln2 = 2 * (size_t)Lc * c.n;
    std::vector<KsJob> jobs(count);
    stage_reset(c.lane, st);
    if (c.lane.ws.reserve(ks_scratch_bytes(c, Lc, (int)count) + sizeof(uint64_t) * Ln2 * (count + 1) + 4096) != HC_OK)
        return HC_ENOMEM;
    KsScratch s = ks_scratch(c, c.lane.ws, Lc, (int)count);
    uint64_t* inN = c.lane.ws.take<uint64_t>(Ln2);
    uint64_t* outN = c.lane.ws.take<uint64_t>(Ln2 * count);
    if (!inN || !outN) return HC_ENOMEM;
    for (uint32_t i = 0; i < count; i++) {
        const uint64_t* key = find_key(gk, elts[i]);
        if (!key) return HC_ENOKEY;
        jobs[i] = KsJob{inN, outN + i * Ln2, key, elts[i], 0};
    }
    ntt64(c, inN, (size_t)Lc * c.n, 2, 0, Lc, false, st, ct_in);
    std::vector<const uint64_t*> srcs{inN};
    hc_status stt = ks_run(c, c.lane, s, jobs, hoisted ? &srcs : nullptr, Lc, st);
    if (stt != HC_OK) return stt;
    ntt64(c, outN, (size_t)Lc * c.n, 2 * (int)count, 0, Lc, true, st);
    HC_CHECK(hipMemcpyAsync(cts_out, outN, sizeof(uint64_t) * Ln2 * count, hipMemcpyDeviceToDevice, st));
    HC_CHECK(hipGetLastError());
    HC_CHECK(hipStreamSynchronize(st));
    return HC_OK;
}

extern "C" hc_status hc_rotate(hc_context* cp, const hc_gk* gk, uint32_t element, const uint64_t* ct_in,
                               uint64_t* ct_out, hipStream_t st) {
    if (!cp) return HC_EINVAL;
    return rotate_common(cp, gk, &element, 1, ct_in, ct_out, false, cp->L, st);
}

extern "C" hc_status hc_rotate_level(hc_context* cp, const hc_gk* gk, uint32_t element, uint32_t level,
                                     const uint64_t* ct_in, uint64_t* ct_out, hipStream_t st) {
    if (!cp) return HC_EINVAL;
    return rotate_common(cp, gk, &element, 1, ct_in, ct_out, false, (int)level, st);
}

extern "C" hc_status hc_rotate_level_noalloc(hc_context* cp, const hc_gk* gk, uint32_t element, uint32_t level,
                                             const uint64_t* ct_in, uint64_t* ct_out, hipStream_t st) {
    if (!cp || !gk || !ct_in || !ct_out || ct_in == ct_out) return HC_EINVAL;
    Ctx& c = *cp;
    const int Lc = (int)level;
    if (Lc < c.alpha || Lc > c.L || Lc % c.alpha) return HC_EINVAL;
    const uint64_t* key = find_key(gk, element);
    if (!key) return HC_ENOKEY;
    if (!c.d_scratch) return HC_EDEVICE;
    HC_CHECK(hipSetDevice(c.device));
    const size_t Ln2 = 2 * (size_t)Lc * c.n;
    // the input in the NTT domain, then one job's key-switching scratch, all carved
    // from the fixed array (an arena over it: take() only hands out offsets)
    Arena a;
    a.base = reinterpret_cast<char*>(c.d_scratch);
    a.cap = HC_NOALLOC_SCRATCH_BYTES;
    if (ks_scratch_bytes(c, Lc, 1) + sizeof(uint64_t) * Ln2 + 256 > a.cap) return HC_ESCRATCH;
    uint64_t* inN = a.take<uint64_t>(Ln2);
    KsScratch s = ks_scratch(c, a, Lc, 1);
    if (!inN || !s.tmpC || !s.X || !s.T || !s.conv) return HC_ESCRATCH;
    stage_reset(c.lane, st);  // job tables go through the context's pinned staging area
    ntt64(c, inN, (size_t)Lc * c.n, 2, 0, Lc, false, st, ct_in);
    // the result goes to the caller's output in the NTT domain and is transformed there
    std::vector<KsJob> jobs{KsJob{inN, ct_out, key, element, 0}};
    hc_status stt = ks_run(c, c.lane, s, jobs, nullptr, Lc, st);
    if (stt != HC_OK) return stt;
    ntt64(c, ct_out, (size_t)Lc * c.n, 2, 0, Lc, true, st);
    HC_CHECK(hipGetLastError());
    HC_CHECK(hipStreamSynchronize(st));
    return HC_OK;
}

extern "C" hc_status hc_rotate_hoisted(hc_context* cp, const hc_gk* gk, const uint32_t* elements,
                                       uint32_t count, const uint64_t* ct_in, uint64_t* cts_out,
                                       hipStream_t st) {
    if (!cp) return HC_EINVAL;
    return rotate_common(cp, gk, elements, count, ct_in, cts_out, true, cp->L, st);
}

extern "C" hc_status hc_mod_switch(hc_context* cp, const uint64_t* ct_in, uint32_t count, uint32_t level_in,
                                   uint32_t level_out, uint64_t* ct_out, hipStream_t st) {
    if (!cp || !ct_in || !ct_out || count == 0 || level_out < 1 || level_out >= level_in ||
        level_in > (uint32_t)cp->L)
        return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    // the workspace is reused in stream order; wait for another stream's last use
    stage_reset(c.lane, st);
    const size_t cw = 2 * (size_t)level_out * c.n * count;
    if (c.lane.ws.reserve(sizeof(uint64_t) * cw + 4096) != HC_OK) return HC_ENOMEM;
    uint64_t* conv = c.lane.ws.take<uint64_t>(cw);
    if (!conv) return HC_ENOMEM;
    hc_status s = mod_switch_coef(c, ct_out, ct_in, (int)count, (int)level_in, (int)level_out, conv, st);
    if (s != HC_OK) return s;
    HC_CHECK(hipGetLastError());
    return HC_OK;
}

extern "C" hc_status hc_mul_plain(hc_context* cp, const uint64_t* ct_in, const uint32_t* slots,
                                  uint64_t* ct_out, hipStream_t st) {
    if (!cp || !ct_in || !slots || !ct_out) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    const size_t Ln = (size_t)c.L * c.n;
    HC_CHECK(hipStreamSynchronize(st));
    if (c.lane.ws.reserve(sizeof(uint64_t) * Ln * 3 + 1024) != HC_OK) return HC_ENOMEM;
    uint64_t* pt = c.lane.ws.take<uint64_t>(Ln);
    uint64_t* tmp = c.lane.ws.take<uint64_t>(2 * Ln);
    if (!pt || !tmp) return HC_ENOMEM;
    hc_status s = encode_plain(c, pt, slots, 1, true, st);
    if (s != HC_OK) return s;
    ntt64(c, tmp, Ln, 2, 0, c.L, false, st, ct_in);
    k_mul_plain(c, tmp, tmp, pt, c.L, st);
    ntt64(c, tmp, Ln, 2, 0, c.L, true, st);
    HC_CHECK(hipMemcpyAsync(ct_out, tmp, sizeof(uint64_t) * 2 * Ln, hipMemcpyDeviceToDevice, st));
    HC_CHECK(hipStreamSynchronize(st));
    return HC_OK;
}

extern "C" hc_status hc_modup(hc_context* cp, const uint64_t* x, uint32_t digit, uint64_t* out,
                              hipStream_t st) {
    if (!cp || !x || !out || digit >= (uint32_t)cp->dnum) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    const size_t n = c.n, R = (size_t)c.nq;
    HC_CHECK(hipStreamSynchronize(st));
    if (c.lane.ws.reserve(sizeof(uint64_t) * (size_t)c.dnum * R * n + 4096) != HC_OK) return HC_ENOMEM;
    uint64_t* X = c.lane.ws.take<uint64_t>((size_t)c.dnum * R * n);
    if (!X) return HC_ENOMEM;
    // x is [L][n], the compact layout of one source at the top level
    kb_modup(c, X, x, 1, c.L, true, st);
    HC_CHECK(hipMemcpyAsync(out, X + (size_t)digit * R * n, sizeof(uint64_t) * R * n,
                            hipMemcpyDeviceToDevice, st));
    HC_CHECK(hipStreamSynchronize(st));
    return HC_OK;
}

__global__ void zero_fill_kernel(uint64_t* p, size_t count) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

extern "C" hc_status hc_moddown(hc_context* cp, const uint64_t* T, uint64_t* out, hipStream_t st) {
    if (!cp || !T || !out) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    const size_t n = c.n;
    stage_reset(c.lane, st);
    if (c.lane.ws.reserve(sizeof(uint64_t) * (2 * c.nq * n + 6 * c.L * n) + 4096) != HC_OK) return HC_ENOMEM;
    // T as component 0 of one job's [2][L+K][n] (component 1 zero); the conversion and the
    // final combination are element-wise, so they apply in the coefficient domain too
    uint64_t* TT = c.lane.ws.take<uint64_t>(2 * c.nq * n);
    uint64_t* conv = c.lane.ws.take<uint64_t>(2 * c.L * n);
    uint64_t* zero = c.lane.ws.take<uint64_t>(2 * c.L * n);
    uint64_t* o2 = c.lane.ws.take<uint64_t>(2 * c.L * n);
    if (!TT || !conv || !zero || !o2) return HC_ENOMEM;
    const size_t zc = 2 * c.nq * n, zc2 = 2 * c.L * n;
    hipLaunchKernelGGL(zero_fill_kernel, dim3((zc + 255) / 256), dim3(256), 0, st, TT, zc);
    hipLaunchKernelGGL(zero_fill_kernel, dim3((zc2 + 255) / 256), dim3(256), 0, st, zero, zc2);
    HC_CHECK(hipMemcpyAsync(TT, T, sizeof(uint64_t) * c.nq * n, hipMemcpyDeviceToDevice, st));
    KsJob j{zero, o2, nullptr, 1u, 0u};
    const KsJob* dj = (const KsJob*)stage_bytes(c.lane, &j, sizeof(j), st);
    if (!dj) return HC_ENOMEM;
    kb_conv(c, conv, TT, 1, c.L, st);
    kb_final(c, dj, TT, conv, 1, c.L, st);
    HC_CHECK(hipMemcpyAsync(out, o2, sizeof(uint64_t) * c.L * n, hipMemcpyDeviceToDevice, st));
    HC_CHECK(hipStreamSynchronize(st));
    return HC_OK;
}

extern "C" hc_status hc_sample(hc_context* cp, int kind, const uint8_t seed[32], const char* tag,
                               uint64_t obj, uint32_t limb, uint64_t* out, hipStream_t st) {
    if (!cp || !seed || !tag || !out || kind < 0 || kind > 2 || strlen(tag) > 8) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    if (kind == 0) {
        if (limb >= (uint32_t)c.nq) return HC_EINVAL;
        k_sample_uniform(c, out, seed, tag_u64(tag), obj, (int)limb, 1, st);
    } else {
        uint64_t* tmp = nullptr;
        HC_CHECK(hipMalloc((void**)&tmp, sizeof(uint64_t) * c.n));
        k_sample_small(c, tmp, reinterpret_cast<int64_t*>(out), seed, tag_u64(tag), obj, kind, 0, 1, st);
        HC_CHECK(hipStreamSynchronize(st));
        HC_CHECK(hipFree(tmp));
    }
    HC_CHECK(hipGetLastError());
    return HC_OK;
}

extern "C" hc_status hc_encode_diagonal(hc_context* cp, uint32_t s, uint32_t B, uint32_t beta,
                                        uint32_t gi, uint32_t b, uint64_t* out, hipStream_t st) {
    if (!cp || !out || s == 0 || B == 0 || s > (uint32_t)cp->nh) return HC_EINVAL;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    uint32_t* d = nullptr;
    HC_CHECK(hipMalloc((void**)&d, sizeof(uint32_t) * (c.n + 4)));
    uint32_t prm[3] = {beta, gi, b};
    HC_CHECK(hipMemcpyAsync(d + c.n, prm, sizeof(prm), hipMemcpyHostToDevice, st));
    k_diag_gen(c, d, d + c.n, 1, s, B, st);
    ntt32(c, d, 1, true, st);
    k_lift(c, out, d, 1, false, c.L, st);
    HC_CHECK(hipStreamSynchronize(st));
    HC_CHECK(hipFree(d));
    return HC_OK;
}

// ------------------------------------------------------------------ exports

extern "C" hc_status hc_export_sk(hc_context* cp, const hc_sk* sk, int64_t* out) {
    if (!cp || !sk || !out) return HC_EINVAL;
    for (size_t i = 0; i < sk->s.size(); i++) out[i] = sk->s[i];
    return HC_OK;
}

static hc_status export_rows(Ctx& c, const uint64_t* d, int count, int nl, bool from_mont, uint64_t* out) {
    const size_t n = c.n;
    uint64_t* tmp = nullptr;
    HC_CHECK(hipMalloc((void**)&tmp, sizeof(uint64_t) * count * nl * n));
    HC_CHECK(hipMemcpy(tmp, d, sizeof(uint64_t) * count * nl * n, hipMemcpyDeviceToDevice));
    if (from_mont) k_from_mont(c, tmp, 0, nl, count, (size_t)nl * n, 0);
    ntt64(c, tmp, (size_t)nl * n, count, 0, nl, true, 0);
    HC_CHECK(hipMemcpy(out, tmp, sizeof(uint64_t) * count * nl * n, hipMemcpyDeviceToHost));
    HC_CHECK(hipFree(tmp));
    return HC_OK;
}

extern "C" hc_status hc_export_pk(hc_context* cp, const hc_pk* pk, uint64_t* out) {
    if (!cp || !pk || !out) return HC_EINVAL;
    HC_CHECK(hipSetDevice(cp->device));
    const size_t Ln = (size_t)cp->L * cp->n;
    hc_status s = export_rows(*cp, pk->d_b, 1, cp->L, false, out);
    if (s != HC_OK) return s;
    return export_rows(*cp, pk->d_a, 1, cp->L, false, out + Ln);
}

extern "C" hc_status hc_export_gk(hc_context* cp, const hc_gk* gk, uint32_t element, uint64_t* out) {
    if (!cp || !gk || !out) return HC_EINVAL;
    const uint64_t* key = find_key(gk, element);
    if (!key) return HC_ENOKEY;
    HC_CHECK(hipSetDevice(cp->device));
    return export_rows(*cp, key, 2 * cp->dnum, cp->nq, true, out);
}
