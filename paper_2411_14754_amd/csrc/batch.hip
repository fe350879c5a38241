// Batched query executor: one hipGraph per batch-size bucket.
//
// Queries arrive in batches of uneven size (1 .. max_batch).  A batch of size
// nq uses the graph of the smallest power-of-two bucket >= nq.  The graph holds
// the whole query path: a stage-in kernel (queries and collision ratios into
// fixed staging buffers, batch size into device memory), then for each pass of
// up to C queries the activate, collide, select, rerank and merge kernels, then a
// stage-out kernel (results to the caller's buffers).  Every kernel strides over
// its items and reads the batch size on the device, so one graph, captured once,
// serves every batch of its bucket.  Per call the host writes the caller's
// pointers and the batch size into a device mailbox with one tiny kernel and
// launches the graph.  A call may also hand over several batches (up to 16) at
// once: the stage-in kernel places them back to back in the staging rows, the
// graph of the bucket of their total runs once, and the stage-out kernel
// returns each batch's results to its own buffers, so batches of uneven size
// that are ready together share one launch.
//
// The launch shapes of a bucket (re-rank rows per work-group, grid caps of the
// collision and re-rank kernels) are chosen on the bucket's first use by timing
// each candidate graph on that batch, and kept in a text file when one is given.
// Every candidate computes the same per-item results, so the choice never
// changes the output: results are bitwise those of suco_query.
#include <array>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>

#include "runtime_impl.h"

namespace suco {

constexpr int kMailBatches = 16;   // batches one call may hand over together

// One call's batches: batch j holds nq queries that take the staging rows
// q0 .. q0 + nq - 1 (the batches in call order, back to back).
struct MailBatch {
    const float *Q;
    const float *alpha_q;
    int32_t *ids;
    float *dists;
    int q0, nq;
};

struct Mail {
    int nq;                 // all the call's queries
    int nb;                 // batches, 1 .. kMailBatches
    int per_query_alpha;
    double alpha;
    MailBatch b[kMailBatches];
};

__global__ void k_set_mail(Mail *dst, Mail m) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = m;
}

// Every batch's queries to their staging rows (float4), collision ratios to
// FP64 staging, the total into device memory.
__global__ __launch_bounds__(256) void k_stage_in(const Mail *mail, float4 *Qs, double *alphas, int *nq_dev,
                                                  int d4) {
    const Mail &m = *mail;
    const int nb = m.nb, pqa = m.per_query_alpha;
    const double alpha = m.alpha;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = 0; j < nb; ++j) {
        const MailBatch bj = m.b[j];
        const float4 *src = reinterpret_cast<const float4 *>(bj.Q);
        float4 *dst = Qs + (int64_t)bj.q0 * d4;
        for (int64_t t = t0; t < (int64_t)bj.nq * d4; t += stride) dst[t] = src[t];
        for (int64_t t = t0; t < bj.nq; t += stride) alphas[bj.q0 + t] = pqa ? (double)bj.alpha_q[t] : alpha;
    }
    if (t0 == 0) *nq_dev = m.nq;
}

// Every batch's results from staging to its caller's buffers.
__global__ __launch_bounds__(256) void k_stage_out(const Mail *mail, const int32_t *ids_s, const float *dists_s,
                                                   int k) {
    const Mail &m = *mail;
    const int nb = m.nb;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = 0; j < nb; ++j) {
        const MailBatch bj = m.b[j];
        const int64_t o = (int64_t)bj.q0 * k;
        for (int64_t t = t0; t < (int64_t)bj.nq * k; t += stride) {
            bj.ids[t] = ids_s[o + t];
            bj.dists[t] = dists_s[o + t];
        }
    }
}

struct Tuned {
    int rpp = 512;     // re-rank rows per work-group
    int cap_c = 0;     // collision grid cap (0: one block per item)
    int cap_r = 0;     // re-rank grid cap
};

struct Bucket {
    int size = 0;
    Tuned t;
    double ms = 0.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<QueryPass> qps;
    std::vector<RerankPass> rps;
    FeatPass fp{};
    InferPass ip{};
    void destroy() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

}  // namespace suco

using namespace suco;

struct suco_batcher {
    uint64_t magic = 0x5375436f42617431ULL;
    const suco_index *ix = nullptr;
    int device = 0, maxb = 0, k = 0, C = 0, cus = 0, parts_max = 0;
    int d4 = 0;                 // kernel arguments of the staging nodes live here
    double beta = 0.0;
    int64_t B = 0;
    RerankCfg rcfg{};
    // staging and pass workspace (device)
    float *Qs = nullptr;
    double *alphas = nullptr;
    int32_t *ids_s = nullptr;
    float *dists_s = nullptr;
    Mail *mail = nullptr;
    int *nq_dev = nullptr;
    uint16_t *cells = nullptr, *lvl = nullptr;
    int32_t *ncells = nullptr, *aprime = nullptr, *order = nullptr, *route = nullptr;
    uint32_t *hist = nullptr, *cand = nullptr;
    uint64_t *part_keys = nullptr;
    std::map<int, Bucket> buckets;
    // attached model: features and alphas computed inside the graph
    suco_mlp *model = nullptr;
    float scale = 1.f, amin = 0.f, amax = 1.f;
    float *Fs = nullptr;
    std::string tune_path;
    std::map<std::string, Tuned> tune_cache;
    std::mutex mu;
    hipEvent_t done = nullptr;
    bool pending = false;

    void release() {
        if (done) { (void)hipEventSynchronize(done); (void)hipEventDestroy(done); done = nullptr; }
        for (auto &kv : buckets) kv.second.destroy();
        buckets.clear();
        if (Fs) (void)hipFree(Fs);
        Fs = nullptr;
        for (void *p : {(void *)Qs, (void *)alphas, (void *)ids_s, (void *)dists_s, (void *)mail, (void *)nq_dev,
                        (void *)cells, (void *)lvl, (void *)ncells, (void *)aprime, (void *)hist, (void *)cand,
                        (void *)part_keys, (void *)order, (void *)route})
            if (p) (void)hipFree(p);
        Qs = nullptr; alphas = nullptr; ids_s = nullptr; dists_s = nullptr; mail = nullptr; nq_dev = nullptr;
        cells = nullptr; lvl = nullptr; ncells = nullptr; aprime = nullptr; hist = nullptr; cand = nullptr;
        order = nullptr;
        route = nullptr;
        part_keys = nullptr;
        magic = 0;
    }
};

namespace {

bool batcher_ok(const suco_batcher *b) { return b != nullptr && b->magic == 0x5375436f42617431ULL; }

std::string tune_key(const suco_batcher *b, int bucket) {
    const suco_index *ix = b->ix;
    std::ostringstream os;
    os << "gfx950 n=" << ix->n << " d=" << ix->d << " ns=" << ix->ns << " sk=" << ix->sk << " P=" << ix->P
       << " TILE=" << ix->TILE << " B=" << b->B << " k=" << b->k << " C=" << b->C << " bucket=" << bucket
       << (b->model ? " learned" : "");
    return os.str();
}

void load_tune_file(suco_batcher *b) {
    if (b->tune_path.empty()) return;
    std::ifstream f(b->tune_path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t bar = line.rfind('|');
        if (bar == std::string::npos) continue;
        std::istringstream vals(line.substr(bar + 1));
        Tuned t;
        if (vals >> t.rpp >> t.cap_c >> t.cap_r && t.rpp >= 64) b->tune_cache[line.substr(0, bar)] = t;
    }
}

void store_tune_entry(const suco_batcher *b, const std::string &key, const Tuned &t) {
    if (b->tune_path.empty()) return;
    std::ofstream f(b->tune_path, std::ios::app);
    if (f) f << key << "|" << t.rpp << " " << t.cap_c << " " << t.cap_r << "\n";
}

hipError_t add_node(hipGraph_t g, hipGraphNode_t *prev, const void *func, dim3 grid, dim3 block, size_t lds,
                    void **args) {
    hipKernelNodeParams p{};
    p.func = const_cast<void *>(func);
    p.gridDim = grid;
    p.blockDim = block;
    p.sharedMemBytes = (unsigned)lds;
    p.kernelParams = args;
    p.extra = nullptr;
    hipGraphNode_t n = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&n, g, *prev ? prev : nullptr, *prev ? 1 : 0, &p);
    if (e == hipSuccess) *prev = n;
    return e;
}

// Build and instantiate the graph of one bucket with the given launch shapes.
hipError_t build_graph(suco_batcher *b, Bucket *bk, const Tuned &t) {
    const suco_index *ix = b->ix;
    bk->destroy();
    bk->t = t;
    hipError_t e = hipGraphCreate(&bk->graph, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t prev = nullptr;
    b->d4 = ix->d / 4;
    {
        void *args[] = {&b->mail, &b->Qs, &b->alphas, &b->nq_dev, &b->d4};
        e = add_node(bk->graph, &prev, reinterpret_cast<const void *>(&k_stage_in), dim3(256), dim3(256), 0, args);
        if (e != hipSuccess) return e;
    }
    if (b->model) {
        bk->fp = FeatPass{};
        bk->fp.ix = ix->view();
        bk->fp.Q = b->Qs;
        bk->fp.nq = bk->size;
        bk->fp.nq_dev = b->nq_dev;
        bk->fp.F = b->Fs;
        bk->ip = InferPass{};
        bk->ip.w = mlp_infer_view(b->model);
        bk->ip.F = b->Fs;
        bk->ip.m = bk->size;
        bk->ip.m_dev = b->nq_dev;
        bk->ip.scale = b->scale;
        bk->ip.amin = b->amin;
        bk->ip.amax = b->amax;
        bk->ip.alpha64 = b->alphas;
        // features and inference in one node
        const Launch La = plan_learned_alpha(bk->fp.ix, half_wmax(ix), bk->size);
        void *aa[] = {&bk->fp, &bk->ip};
        if ((e = add_node(bk->graph, &prev, La.func, La.grid, La.block, La.lds, aa)) != hipSuccess) return e;
    }
    const int passes = (bk->size + b->C - 1) / b->C;
    const int C = std::min(b->C, bk->size);
    bk->qps.assign(passes, QueryPass{});
    bk->rps.assign(passes, RerankPass{});
    const int parts = (int)((b->B + t.rpp - 1) / t.rpp);
    for (int c = 0; c < passes; ++c) {
        QueryPass &qp = bk->qps[c];
        qp.ix = ix->view();
        qp.Q = b->Qs + (int64_t)c * b->C * ix->d;
        qp.nq = C;
        qp.alpha_qd = b->alphas + (int64_t)c * b->C;
        qp.B = b->B;
        qp.k = b->k;
        qp.runs_per_sub = runs_per_sub(ix->ns);
        qp.tgroups = tile_groups(qp.nq, ix->P);
        qp.nq_dev = b->nq_dev;
        qp.q_base = c * b->C;
        qp.cells = b->cells; qp.ncells = b->ncells; qp.aprime = b->aprime; qp.hist = b->hist; qp.lvl = b->lvl;
        if (C <= kOrderWide) { qp.order_out = b->order; qp.order = b->order; }
        qp.cand = b->cand;
        qp.route = ix->sp_cap ? b->route : nullptr;
        qp.tlist = qp.route ? b->route + b->C : nullptr;
        qp.ntl = qp.route ? b->route + 2 * b->C : nullptr;
        qp.sp_cap = ix->sp_cap;
        RerankPass &rp = bk->rps[c];
        rp.X = ix->X; rp.X8 = ix->X8; rp.Q = qp.Q; rp.cand = b->cand; rp.B = b->B; rp.n = ix->n; rp.d = ix->d; rp.k = b->k;
        rp.metric = ix->metric;
        rp.nq = C; rp.parts = parts; rp.nq_dev = b->nq_dev; rp.q_base = c * b->C; rp.rows_per_part = t.rpp;
        rp.G = b->rcfg.G; rp.U = b->rcfg.U; rp.part_keys = b->part_keys;
        rp.ids = b->ids_s + (int64_t)c * b->C * b->k;
        rp.dists = b->dists_s + (int64_t)c * b->C * b->k;
        const Launch La = plan_activate(qp, kActivateGrid), Lc = plan_collide(qp, t.cap_c), Ls = plan_select(qp, 0),
                     Lr = plan_rerank(rp, t.cap_r), Lm = plan_merge(rp, 0);
        void *aq[] = {&qp};
        void *ar[] = {&rp};
        if ((e = add_node(bk->graph, &prev, La.func, La.grid, La.block, La.lds, aq)) != hipSuccess) return e;
        if (qp.order) {
            const Launch Lo = plan_order(qp);
            if ((e = add_node(bk->graph, &prev, Lo.func, Lo.grid, Lo.block, Lo.lds, aq)) != hipSuccess) return e;
        }
        if (qp.route) {
            const Launch Lp = plan_collide_sparse(qp, 0);
            if ((e = add_node(bk->graph, &prev, Lp.func, Lp.grid, Lp.block, Lp.lds, aq)) != hipSuccess) return e;
        }
        if ((e = add_node(bk->graph, &prev, Lc.func, Lc.grid, Lc.block, Lc.lds, aq)) != hipSuccess) return e;
        if ((e = add_node(bk->graph, &prev, Ls.func, Ls.grid, Ls.block, Ls.lds, aq)) != hipSuccess) return e;
        if ((e = add_node(bk->graph, &prev, Lr.func, Lr.grid, Lr.block, Lr.lds, ar)) != hipSuccess) return e;
        if ((e = add_node(bk->graph, &prev, Lm.func, Lm.grid, Lm.block, Lm.lds, ar)) != hipSuccess) return e;
    }
    {
        void *args[] = {&b->mail, &b->ids_s, &b->dists_s, &b->k};
        e = add_node(bk->graph, &prev, reinterpret_cast<const void *>(&k_stage_out), dim3(64), dim3(256), 0, args);
        if (e != hipSuccess) return e;
    }
    return hipGraphInstantiate(&bk->exec, bk->graph, nullptr, nullptr, 0);
}

// Time each candidate on the batch in the mailbox and keep the fastest.
int tune_bucket(suco_batcher *b, Bucket *bk, hipStream_t st) {
    std::vector<Tuned> cands;
    for (int rpp : {256, 512, 1024})
        for (int cc : {0, 2 * b->cus})
            for (int cr : {0, 8 * b->cus}) cands.push_back(Tuned{rpp, cc, cr});
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    double best = 1e30;
    Tuned bt;
    for (const Tuned &t : cands) {
        if ((int)((b->B + t.rpp - 1) / t.rpp) > b->parts_max) continue;
        HIPCHECK(build_graph(b, bk, t));
        HIPCHECK(hipGraphLaunch(bk->exec, st));
        HIPCHECK(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r) HIPCHECK(hipGraphLaunch(bk->exec, st));
        HIPCHECK(hipEventRecord(e1, st));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms / 3.0 < best) { best = ms / 3.0; bt = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHECK(build_graph(b, bk, bt));
    bk->ms = best;
    const std::string key = tune_key(b, bk->size);
    b->tune_cache[key] = bt;
    store_tune_entry(b, key, bt);
    return SUCO_OK;
}

}  // namespace

extern "C" {

int suco_batcher_create(const suco_index *ix, int32_t max_batch, int32_t k, double beta, const char *tune_file,
                        suco_batcher **out) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (!out) return fail(SUCO_E_INVAL, "out must not be NULL");
    if (max_batch < 1 || max_batch > 65536) return fail(SUCO_E_INVAL, "max_batch must be in [1, 65536]");
    if (k < 1 || k > ix->n) return fail(SUCO_E_INVAL, "k must be in [1, n]");
    if (k > kMaxK) return fail(SUCO_E_UNSUPPORTED, "the kernels take k <= 64");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SUCO_E_INVAL, "beta must be in (0, 1]");
    suco_batcher *b = new (std::nothrow) suco_batcher();
    if (!b) return fail(SUCO_E_NOMEM, "host allocation failed");
    b->ix = ix;
    b->device = ix->device;
    DeviceGuard dg(ix->device);
    int cap = 1;
    while (cap < max_batch) cap *= 2;
    b->maxb = cap;
    b->k = k;
    b->beta = beta;
    b->B = count_B_host(beta, ix->n, k);
    int rc = rerank_cfg(ix->d, b->B, &b->rcfg);
    if (rc) { delete b; return rc; }
    b->C = std::min(cap, ix->chunk);
    b->parts_max = (int)((b->B + 255) / 256);
    if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) b->cus = 256;
    if (tune_file) b->tune_path = tune_file;
    const size_t C = (size_t)b->C;
    if ((rc = dev_alloc(&b->Qs, (size_t)cap * ix->d)) || (rc = dev_alloc(&b->alphas, (size_t)cap)) ||
        (rc = dev_alloc(&b->ids_s, (size_t)cap * k)) || (rc = dev_alloc(&b->dists_s, (size_t)cap * k)) ||
        (rc = dev_alloc(&b->mail, 1)) || (rc = dev_alloc(&b->nq_dev, 1)) ||
        (rc = dev_alloc(&b->cells, C * ix->ns * ix->K)) || (rc = dev_alloc(&b->ncells, C * ix->ns)) ||
        (rc = dev_alloc(&b->aprime, C * ix->ns)) || (rc = dev_alloc(&b->hist, C * ix->P * (ix->ns + 2))) ||
        (rc = dev_alloc(&b->order, C)) || (rc = dev_alloc(&b->route, 2 * C + 1)) ||
        (rc = dev_alloc(&b->lvl, C * (size_t)ix->P * ix->TILE + 2 * kSpBucket)) || (rc = dev_alloc(&b->cand, C * (size_t)b->B)) ||
        (rc = dev_alloc(&b->part_keys, C * (size_t)b->parts_max * k))) {
        b->release();
        delete b;
        return rc;
    }
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        b->release();
        delete b;
        return fail(SUCO_E_HIP, "hipEventCreate failed");
    }
    load_tune_file(b);
    *out = b;
    return SUCO_OK;
}

}  // extern "C"

namespace {

// The batches of one call (nb >= 1, checked by the callers) through the graph
// of the bucket of their total.  per_query: alpha_q[j] is given for every batch.
int batcher_run(suco_batcher *b, int nb, const float *const *Q, const int64_t *nq, const float *const *alpha_q,
                double alpha, int32_t *const *ids, float *const *dists, void *stream) {
    if (!batcher_ok(b)) return fail(SUCO_E_STATE, "invalid or freed batcher handle");
    if (!index_ok(b->ix)) return fail(SUCO_E_STATE, "the batcher's index was freed");
    const bool per_query = alpha_q != nullptr;
    if (!b->model && !per_query && !(alpha > 0.0 && alpha <= 1.0)) return fail(SUCO_E_INVAL, "alpha must be in (0, 1]");
    if (b->model && per_query) return fail(SUCO_E_INVAL, "a batcher with a model takes no alpha_q");
    if (b->model && !mlp_valid(b->model)) return fail(SUCO_E_STATE, "the batcher's model was freed");
    Mail m{};
    int64_t total = 0;
    for (int j = 0; j < nb; ++j) {
        if (nq[j] < 0 || nq[j] > b->maxb) return fail(SUCO_E_INVAL, "nq must be in [0, max_batch]");
        if (nq[j] > 0 && (!Q[j] || !ids[j] || !dists[j])) return fail(SUCO_E_INVAL, "Q, ids and dists must not be NULL");
        if (nq[j] > 0 && per_query && !alpha_q[j]) return fail(SUCO_E_INVAL, "alpha_q must not be NULL");
        MailBatch &mb = m.b[m.nb];
        mb.Q = Q[j];
        mb.alpha_q = per_query ? alpha_q[j] : nullptr;
        mb.ids = ids[j];
        mb.dists = dists[j];
        mb.q0 = (int)total;
        mb.nq = (int)nq[j];
        if (nq[j] > 0) ++m.nb;          // empty batches take no entry
        total += nq[j];
        if (total > b->maxb) return fail(SUCO_E_INVAL, "the batches' total must be at most max_batch");
    }
    if (total == 0) return SUCO_OK;
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(b->mu);
    DeviceGuard dg(b->device);
    if (b->model) {
        const int rc = mlp_prepare(b->model, st);
        if (rc) return rc;
        alpha = 1.0;
    }
    if (b->pending) HIPCHECK(hipStreamWaitEvent(st, b->done, 0));
    m.nq = (int)total;
    m.per_query_alpha = per_query;
    m.alpha = alpha;
    const int64_t nq_all = total;
    hipLaunchKernelGGL(k_set_mail, dim3(1), dim3(64), 0, st, b->mail, m);
    HIPCHECK(hipGetLastError());
    int size = 1;
    while (size < nq_all) size *= 2;
    Bucket &bk = b->buckets[size];
    if (!bk.exec) {
        bk.size = size;
        auto it = b->tune_cache.find(tune_key(b, size));
        if (it != b->tune_cache.end()) {
            HIPCHECK(build_graph(b, &bk, it->second));
        } else {
            const int rc = tune_bucket(b, &bk, st);
            if (rc) return rc;
        }
    }
    HIPCHECK(hipGraphLaunch(bk.exec, st));
    HIPCHECK(hipEventRecord(b->done, st));
    b->pending = true;
    return SUCO_OK;
}

}  // namespace

extern "C" {

int suco_batcher_query(suco_batcher *b, const float *Q, int64_t nq, const float *alpha_q, double alpha,
                       int32_t *ids, float *dists, void *stream) {
    const float *const aq[1] = {alpha_q};
    return batcher_run(b, 1, &Q, &nq, alpha_q ? aq : nullptr, alpha, &ids, &dists, stream);
}

int suco_batcher_query_multi(suco_batcher *b, int32_t nb, const float *const *Q, const int64_t *nq,
                             const float *const *alpha_q, double alpha, int32_t *const *ids, float *const *dists,
                             void *stream) {
    if (nb < 1 || nb > kMailBatches) return fail(SUCO_E_INVAL, "nb must be in [1, 16]");
    if (!Q || !nq || !ids || !dists) return fail(SUCO_E_INVAL, "Q, nq, ids and dists must not be NULL");
    return batcher_run(b, nb, Q, nq, alpha_q, alpha, ids, dists, stream);
}

int suco_batcher_set_model(suco_batcher *b, suco_mlp *m, float scale, float alpha_min, float alpha_max) {
    if (!batcher_ok(b)) return fail(SUCO_E_STATE, "invalid or freed batcher handle");
    if (m && !mlp_valid(m)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    if (m && mlp_n_in(m) != 2 * b->ix->ns + 1) return fail(SUCO_E_INVAL, "the model's n_in must be 2*n_s + 1");
    if (m && b->ix->metric)
        return fail(SUCO_E_UNSUPPORTED, "the learned budget's features are Euclidean (not SUCO_BUILD_L1)");
    if (m && !(scale > 0.f)) return fail(SUCO_E_INVAL, "scale must be positive");
    if (m && !(alpha_min > 0.f && alpha_min <= alpha_max && alpha_max <= 1.f))
        return fail(SUCO_E_INVAL, "need 0 < alpha_min <= alpha_max <= 1");
    std::lock_guard<std::mutex> lock(b->mu);
    DeviceGuard dg(b->device);
    if (b->pending) HIPCHECK(hipEventSynchronize(b->done));
    if (m && !b->Fs) {
        const int rc = dev_alloc(&b->Fs, (size_t)b->maxb * (2 * b->ix->ns + 1));
        if (rc) return rc;
    }
    b->model = m;
    b->scale = scale;
    b->amin = alpha_min;
    b->amax = alpha_max;
    // graphs are rebuilt on next use (tuned shapes are kept)
    for (auto &kv : b->buckets) kv.second.destroy();
    return SUCO_OK;
}

int suco_batcher_tuning(const suco_batcher *b, int32_t bucket, int32_t *params, double *ms) {
    if (!batcher_ok(b)) return fail(SUCO_E_STATE, "invalid or freed batcher handle");
    auto it = b->buckets.find(bucket);
    if (it == b->buckets.end() || !it->second.exec) return fail(SUCO_E_INVAL, "bucket not built yet");
    if (params) {
        params[0] = it->second.t.rpp;
        params[1] = it->second.t.cap_c;
        params[2] = it->second.t.cap_r;
    }
    if (ms) *ms = it->second.ms;
    return SUCO_OK;
}

int suco_batcher_free(suco_batcher *b) {
    if (!b) return SUCO_OK;
    if (!batcher_ok(b)) return fail(SUCO_E_STATE, "invalid or freed batcher handle");
    {
        DeviceGuard dg(b->device);
        std::lock_guard<std::mutex> lock(b->mu);
        b->release();
    }
    delete b;
    return SUCO_OK;
}

}  // extern "C"
