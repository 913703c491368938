// Captured compressions: one hc_compress_batch call's whole device work (Mask, the
// modulus switch, u-packing, the rotation chain with its key-switching passes, the
// multiply-accumulate, giant steps, rotate-and-sum, merge, the answer's switch)
// recorded once into a HIP graph and replayed with one launch.
//
// The plan of a batch depends only on the queries' shapes, so everything the host
// decides per call (job lists, key runs, pointer tables, gather lists) is decided once
// at capture: the graph owns its workspace and a pinned staging area whose tables are
// written once (each launch copies them to the device again, unchanged), and the captured kernels read the
// queries' ct_v buffers and write their ct_out buffers, whose addresses are fixed at
// creation. A launch is then a single hipGraphLaunch: no host planning and no
// per-kernel launch overhead. No memset is recorded (buffers that must start at zero
// are cleared by a kernel), and nothing in the sequence synchronises the host.
#include <stdio.h>

#include <memory>

#include "compress.h"

struct hc_graph {
    hc_context* c = nullptr;
    hc::Lane lane;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t nodes = 0;
};

using namespace hc;

extern "C" void hc_graph_destroy(hc_graph* g) {
    if (!g) return;
    (void)hipSetDevice(g->c->device);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->lane.release();
    g->lane.ws.release();
    delete g;
}

extern "C" hc_status hc_graph_create(hc_context* cp, const hc_gk* gk, const hc_db* db, hc_query* q, uint32_t nq,
                                     hc_graph** out) {
    if (!cp || !gk || !q || nq == 0 || !out) return HC_EINVAL;
    *out = nullptr;
    Ctx& c = *cp;
    HC_CHECK(hipSetDevice(c.device));
    std::vector<QueryRun> runs(nq);
    for (uint32_t i = 0; i < nq; i++) {
        q[i].status = (!q[i].ct_v || !q[i].ct_out)
                          ? HC_EINVAL
                          : make_plan(c, q[i].N, db ? db->ncol : 0, q[i].t_bound, q[i].comp_level, q[i].out_level,
                                      runs[i].pl);
        if (q[i].status != HC_OK) return q[i].status;
        if (runs[i].pl.level != runs[0].pl.level) return q[i].status = HC_EINVAL;
        runs[i].ct_v = q[i].ct_v;
        runs[i].ct_out = q[i].ct_out;
    }
    BatchShape shape;
    hc_status s = batch_shape(c, gk, db, runs, shape);
    if (s != HC_OK) return s;
    // tables the compression builds on first use, built now (outside the capture)
    for (auto& r : runs)
        if (r.pl.bands > 1) {
            const uint64_t* m = nullptr;
            if ((s = prefix_mask(c, r.pl.s, &m)) != HC_OK) return s;
        }
    std::unique_ptr<hc_graph> g(new hc_graph());
    g->c = cp;
    if (g->lane.init((size_t)32 << 20) != HC_OK || g->lane.ws.reserve(shape.total) != HC_OK) {
        g->lane.release();
        g->lane.ws.release();
        return HC_ENOMEM;
    }
    g->lane.capture = true;
    hipStream_t st = nullptr;
    HC_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    const bool timing = c.timing;
    c.timing = false;  // no timing events inside a graph
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        s = compress_many(c, g->lane, gk, db, runs, st);
        if (s != HC_OK) {
            const hipError_t le = hipGetLastError();
            fprintf(stderr, "libhc: capture of the compression failed (status %d, last HIP error %s)\n", (int)s,
                    hipGetErrorString(le));
        }
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(st, &graph);
        g->graph = graph;
    }
    c.timing = timing;
    (void)hipStreamDestroy(st);
    g->lane.capture = false;
    if (e == hipSuccess && s == HC_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e == hipSuccess && s == HC_OK) e = hipGraphGetNodes(g->graph, nullptr, &g->nodes);
    if (e != hipSuccess && s == HC_OK) s = fail_hip(e, "graph capture", __FILE__, __LINE__);
    for (uint32_t i = 0; i < nq; i++) {
        q[i].status = s;
        if (s == HC_OK) fill_info(runs[i], q[i].info);
    }
    if (s != HC_OK) {
        hc_graph_destroy(g.release());
        return s;
    }
    *out = g.release();
    return HC_OK;
}

extern "C" hc_status hc_graph_launch(hc_graph* g, hipStream_t stream) {
    if (!g || !g->exec) return HC_EINVAL;
    HC_CHECK(hipSetDevice(g->c->device));
    HC_CHECK(hipGraphLaunch(g->exec, stream));
    return HC_OK;
}

extern "C" hc_status hc_graph_nodes(const hc_graph* g, uint64_t* nodes) {
    if (!g || !nodes) return HC_EINVAL;
    *nodes = g->nodes;
    return HC_OK;
}
