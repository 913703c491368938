// Internal interface of the compression map (compress.cpp) for the serving loop.
#pragma once
#include <map>
#include <utility>
#include <vector>

#include "he.h"

namespace hc {

struct PlanGroup {
    uint32_t ct_start, ct_count;
    uint64_t rec_start, n_rec;
    uint32_t k, B;
};

struct Plan {
    uint32_t s = 0, n_ct = 0, ncol = 0;
    int level = 0;      // ciphertext primes kept for Comp (modulus switched after Mask)
    int out_level = 0;  // ciphertext primes of the answer (<= level; switched after the merge)
    uint64_t N = 0;
    std::vector<PlanGroup> groups;
    std::vector<std::pair<int, int>> streams;  // vector ids (0 = v, c = d_c), -1 = none
    std::vector<uint32_t> keys;
    uint32_t bands = 0;
    uint32_t n_ks = 0;
    uint64_t n_ptct = 0, n_diag = 0;
};

inline size_t rup(size_t b) { return (b + 255) & ~(size_t)255; }

// One query of a batch and its device regions.
struct QueryRun {
    const uint64_t* ct_v = nullptr;
    // the value vector's ciphertexts themselves (generic Comp, Alg. 5: one column, no
    // database to mask), [n_ct][2][L][n] coefficient domain; nullptr: Mask the database
    const uint64_t* ct_d = nullptr;
    uint64_t* ct_out = nullptr;
    Plan pl;
    size_t CW = 0, PW = 0, CWF = 0, ntot = 0, ub = 0, baby = 0, gi = 0;
    int npairs = 0;
    uint64_t *ctf = nullptr, *cts = nullptr, *ubuf = nullptr, *tbuf = nullptr, *rbuf = nullptr,
             *wbuf = nullptr, *gbuf = nullptr, *gout = nullptr, *ybuf = nullptr,
             *ytmp = nullptr, *mbuf = nullptr, *mrot = nullptr, *outN = nullptr;
    std::vector<std::vector<uint64_t*>> U, A;
    std::vector<std::vector<std::vector<const uint64_t*>>> R;  // [pair][u-block][b] (kRtInPlace: in Rt)
    std::vector<uint32_t> ci;                                    // [pair] index within its (s, B) class

    void sizes(const Ctx& c) {
        const size_t n = c.n;
        CW = 2 * (size_t)pl.level * n;
        PW = (size_t)pl.level * n;
        CWF = 2 * (size_t)c.L * n;
        ntot = (size_t)pl.n_ct * (1 + pl.ncol);
        npairs = (int)(pl.groups.size() * pl.streams.size());
        ub = baby = gi = 0;
        for (auto& g : pl.groups) {
            ub += (size_t)g.k * pl.streams.size();
            baby += (size_t)g.k * (g.B - 1) * pl.streams.size();
            gi += (size_t)(pl.s / g.B) * pl.streams.size();
        }
    }
    size_t bytes(const Ctx& c) const {
        size_t t = rup(CWF * 8 * ntot);
        if (pl.level < c.L) t += 2 * rup(CW * 8 * ntot);
        t += 4 * rup(CW * 8 * std::max<size_t>(ub, 1));
        t += rup(CW * 8 * gi) + rup(CW * 8 * npairs) + 2 * rup(CW * 8 * npairs) + 2 * rup(CW * 8 * pl.bands) +
             rup(CW * 8);
        return t;
    }
    hc_status take(Arena& a) {
        ctf = a.take<uint64_t>(CWF * ntot);
        cts = ctf;
        uint64_t* conv = nullptr;
        if ((int)CW != (int)CWF) {
            cts = a.take<uint64_t>(CW * ntot);
            conv = a.take<uint64_t>(CW * ntot);
            if (!conv) return HC_ENOMEM;
        }
        msconv = conv;
        ubuf = a.take<uint64_t>(CW * std::max<size_t>(ub, 1));
        tbuf = a.take<uint64_t>(CW * std::max<size_t>(ub, 1));
        rbuf = a.take<uint64_t>(CW * std::max<size_t>(ub, 1));
        wbuf = a.take<uint64_t>(CW * std::max<size_t>(ub, 1));
        gbuf = a.take<uint64_t>(CW * gi);
        gout = a.take<uint64_t>(CW * npairs);  // each pair's key-switched giant-step sum
        ybuf = a.take<uint64_t>(CW * npairs);
        ytmp = a.take<uint64_t>(CW * npairs);
        mbuf = a.take<uint64_t>(CW * pl.bands);
        mrot = a.take<uint64_t>(CW * pl.bands);
        outN = a.take<uint64_t>(CW);
        if (!ctf || !cts || !ubuf || !tbuf || !rbuf || !wbuf || !gbuf || !gout || !ybuf || !ytmp ||
            !mbuf || !mrot || !outN)
            return HC_ENOMEM;
        return HC_OK;
    }
    uint64_t* msconv = nullptr;
    uint64_t n_diag = 0, n_diag_res = 0;  // diagonals encoded / read from resident tables
    const uint64_t* vec_ct(int vid, uint32_t i) const { return cts + ((size_t)vid * pl.n_ct + i) * CW; }
};

// Shape and device-memory footprint of a batch (every query at one Comp level):
// the diagonal classes (s, B) with their u-block and pair counts, which of them are
// resident, the on-the-fly chunking, and the workspace bytes compress_many takes.
struct BatchShape {
    int Lc = 0;
    size_t total = 0, max_jobs = 1, diag_max = 1, rt_words = 1, sum_groups = 0;
    std::map<std::pair<uint32_t, uint32_t>, size_t> cls_rt;    // (s, B) -> word offset of its Rt
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> cls_k;   // (s, B) -> max k
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> cls_np;  // (s, B) -> pairs
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> cls_gc;  // (s, B) -> giants per chunk
    std::map<std::pair<uint32_t, uint32_t>, const Ctx::DiagTab*> cls_res;
};

// Galois element of Rot_row(.; r) (k = 3^r mod 2n, r taken mod n/2)
uint32_t rot_elt(const Ctx& c, int64_t r);
// baby steps: the power of two B in [1, s] minimising k (B - 1) + (s / B - 1), ties to the larger
uint32_t choose_B(uint32_t s, uint32_t k);
// Plan one compression (validates N, ncol, t_bound, comp_level and out_level).
hc_status make_plan(const Ctx& c, uint64_t N, uint32_t ncol, uint32_t t_bound, uint32_t comp_level,
                    uint32_t out_level, Plan& pl);
void fill_info(const Plan& pl, hc_compress_info* info);
void fill_info(const QueryRun& q, hc_compress_info* info);
// Shape and workspace bytes of a batch; also sizes each QueryRun.
hc_status batch_shape(const Ctx& c, const hc_gk* gk, const hc_db* db, std::vector<QueryRun>& qs, BatchShape& b);
// Run a batch (one Comp level) on stream st with lane l's workspace and staging.
hc_status compress_many(Ctx& c, Lane& l, const hc_gk* gk, const hc_db* db, std::vector<QueryRun>& qs,
                        hipStream_t st);

}  // namespace hc
