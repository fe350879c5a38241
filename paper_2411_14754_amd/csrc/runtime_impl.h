// Host-side internals shared by the SuCo runtime files: error reporting,
// allocation helpers, the index object and per-launch timing.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "suco.h"
#include "suco_impl.h"

namespace suco {

inline thread_local std::string g_err;

inline int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}


#define HIPCHECK(expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(SUCO_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr uint64_t kMagic = 0x5375436f49647831ULL;

// alpha above 1, +inf and NaN activate every point; alpha <= 0 activates one.
inline int64_t count_A_host(double alpha, int64_t n) {
#pragma clang fp contract(off)
    if (!(alpha <= 1.0)) return n;
    if (!(alpha > 0.0)) return 1;
    double prod = alpha * (double)n;
    int64_t a = (int64_t)std::ceil(prod - 1e-9);
    return std::min<int64_t>(std::max<int64_t>(a, 1), n);
}

inline int64_t count_B_host(double beta, int64_t n, int k) {
#pragma clang fp contract(off)
    double prod = beta * (double)n;
    int64_t b = (int64_t)std::floor(prod + 1e-9);
    return std::min<int64_t>(std::max<int64_t>(b, k), n);
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), counter form: output m of a
// stream with the given base.
inline uint64_t splitmix64_at(uint64_t base, uint64_t m) {
    uint64_t z = base + (m + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

template <class T>
inline int dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void **)p, sizeof(T) * count) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(SUCO_E_NOMEM, "device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed");
    }
    return SUCO_OK;
}

}  // namespace suco

struct suco_index {
    // all device buffers are owned by the index and released by release()
    using HalfDims = suco::HalfDims;
    using IndexView = suco::IndexView;
    uint64_t magic = suco::kMagic;
    int device = 0;
    int64_t n = 0;
    int d = 0, ns = 0, sk = 0, K = 0, P = 0, TILE = 0, chunk = 0;
    std::vector<HalfDims> halves_h;
    std::vector<float> cent_h;
    float *X = nullptr;
    float *cent = nullptr;
    HalfDims *halves = nullptr;
    uint32_t *toffs = nullptr;
    uint16_t *ids16 = nullptr;
    uint32_t *csize = nullptr;
    uint8_t *assign = nullptr;
    uint8_t *X8 = nullptr;          // byte copy of X when every coordinate is an integer in 0..255
    uint32_t *coffs = nullptr;      // cell-major copy of the IMI for the sparse collision step
    uint32_t *ids32 = nullptr;
    uint16_t *cbh = nullptr;        // ids of each cell per bucket of the sparse step
    int NB = 0;                     // buckets of the sparse step
    int sp_cap = 0;                 // its ids per round; 0: the step is off
    bool no_sparse = false;
    int act_form = 0;               // SUCO_ACT_* (suco_index_set_activation)
    int metric = 0;                 // 1 with SUCO_BUILD_L1
    bool no_byte_rows = false;
    bool want_bf16 = false;
    int tile_req = 0;               // tile_max and query_chunk as the caller gave them (0 = automatic),
    int chunk_req = 0;              //   recorded by suco_index_save
    // BF16 split precision (built on request)
    uint16_t *Xb = nullptr;         // [n][d] BF16 copy of X
    float *xerr = nullptr;          // [n] upper bound of |bf16(x) - x|
    uint16_t *centb = nullptr;      // BF16 centres, layout of cent
    float *cnorm2 = nullptr;        // [2ns][sqrt_k] squared norms of the BF16 centres
    // query workspace (one arena, grown on demand)
    std::mutex mu;
    hipEvent_t done = nullptr;
    bool pending = false;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    // staging of suco_query_learned (features and alphas), with its own lock
    struct LearnedStage {
        std::mutex mu;
        float *F = nullptr, *alpha = nullptr;
        int64_t cap_f = 0, cap_a = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
    } lstage;
    // optional per-step timing: event pairs around every launch
    struct EvPair { hipEvent_t a, b; int stage; };
    bool prof_on = false;
    std::vector<EvPair> prof_pool;
    size_t prof_used = 0;

    IndexView view() const {
        IndexView v;
        v.X = X; v.cent = cent; v.halves = halves; v.toffs = toffs; v.ids16 = ids16; v.csize = csize;
        v.coffs = coffs; v.ids32 = ids32; v.cbh = cbh;
        v.n = n; v.d = d; v.ns = ns; v.sk = sk; v.K = K; v.P = P; v.TILE = TILE; v.NB = NB;
        v.act_form = act_form;
        v.metric = metric;
        return v;
    }

    void release() {
        if (done) { (void)hipEventSynchronize(done); (void)hipEventDestroy(done); done = nullptr; }
        {
            std::lock_guard<std::mutex> lk(lstage.mu);
            if (lstage.done) { (void)hipEventSynchronize(lstage.done); (void)hipEventDestroy(lstage.done); }
            if (lstage.F) (void)hipFree(lstage.F);
            if (lstage.alpha) (void)hipFree(lstage.alpha);
            lstage.F = nullptr; lstage.alpha = nullptr; lstage.cap_f = lstage.cap_a = 0;
            lstage.done = nullptr; lstage.pending = false;
        }
        for (auto &e : prof_pool) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
        prof_pool.clear();
        prof_used = 0;
        for (void *p : {(void *)X, (void *)cent, (void *)halves, (void *)toffs, (void *)ids16, (void *)csize,
                        (void *)assign, (void *)arena, (void *)X8, (void *)Xb, (void *)xerr, (void *)centb,
                        (void *)cnorm2, (void *)coffs, (void *)ids32, (void *)cbh})
            if (p) (void)hipFree(p);
        coffs = nullptr; ids32 = nullptr; cbh = nullptr;
        X = nullptr; cent = nullptr; halves = nullptr; toffs = nullptr; ids16 = nullptr; csize = nullptr;
        assign = nullptr; arena = nullptr; arena_bytes = 0; X8 = nullptr;
        Xb = nullptr; xerr = nullptr; centb = nullptr; cnorm2 = nullptr;
        magic = 0;
    }
};

namespace suco {


inline bool index_ok(const suco_index *ix) { return ix != nullptr && ix->magic == kMagic; }
// The widest half of the index's subspaces.
inline int half_wmax(const suco_index *ix) {
    int w = 0;
    for (const auto &h : ix->halves_h) w = h.w > w ? h.w : w;
    return w;
}

enum Stage {
    kActivate = 0, kCollide, kSelect, kRerank, kMerge, kCentresBf16, kRerankBf16, kSurvivors, kOrder, kCollideSparse,
    kStages
};

// Launch through `fn`, bracketed by a pair of timing events when profiling is on.
template <class F>
hipError_t timed(suco_index *ix, int stage, hipStream_t st, F &&fn) {
    if (!ix->prof_on) return fn();
    if (ix->prof_used == ix->prof_pool.size()) {
        suco_index::EvPair e{};
        if (hipEventCreate(&e.a) != hipSuccess) return hipErrorOutOfMemory;
        if (hipEventCreate(&e.b) != hipSuccess) { (void)hipEventDestroy(e.a); return hipErrorOutOfMemory; }
        ix->prof_pool.push_back(e);
    }
    auto &ev = ix->prof_pool[ix->prof_used++];
    ev.stage = stage;
    hipError_t e = hipEventRecord(ev.a, st);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    return hipEventRecord(ev.b, st);
}


// Consecutive 256-byte-aligned buffers carved out of one allocation (base ==
// null: only the total size is computed, in off).
struct Carve {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += sizeof(T) * std::max<size_t>(count, 1);
        return p;
    }
};

// Grow the index's query workspace to `bytes` (waiting for the queries that use it).
inline int ensure_arena(suco_index *ix, size_t bytes) {
    if (bytes <= ix->arena_bytes) return SUCO_OK;
    if (ix->pending) HIPCHECK(hipEventSynchronize(ix->done));
    if (ix->arena) (void)hipFree(ix->arena);
    ix->arena = nullptr;
    ix->arena_bytes = 0;
    int rc = dev_alloc(&ix->arena, bytes);
    if (rc) return rc;
    ix->arena_bytes = bytes;
    return SUCO_OK;
}

// the collision kernel (512 threads) takes this many runs of every subspace per batch
inline int runs_per_sub(int ns) {
    int r = 1;
    while (r * 2 * ns <= 512 && r < 64) r *= 2;
    return r;
}

// tile groups per query for the collision step: enough blocks for the pass
// (about 2048) while each block keeps as many tiles of one query as it can
inline int tile_groups(int64_t nq, int P) {
    const int64_t s = (2048 + std::max<int64_t>(nq, 1) - 1) / std::max<int64_t>(nq, 1);
    return (int)std::clamp<int64_t>(s, 1, P);
}

// Queries per pass: nq split into as few passes of at most `chunk` as
// possible, all of the same size but the last.
inline int64_t pass_size(int64_t nq, int chunk) {
    const int64_t passes = (nq + chunk - 1) / chunk;
    return (nq + passes - 1) / passes;
}

struct RerankCfg { int G, U, parts; int64_t rpp; };

// BF16 first pass: G lanes per row, U slices of 8 values per lane.
inline int rerank_bf16_cfg(int d, int64_t B, RerankCfg *c) {
    if (d % 8) return fail(SUCO_E_UNSUPPORTED, "the BF16 re-rank needs d to be a multiple of 8");
    const int d8 = d / 8;
    int G = 1;
    while (G * 2 <= std::max(1, d8 / 2) && G < kWave) G *= 2;
    const int U = (d8 + G - 1) / G;
    if (U > kMaxU16) return fail(SUCO_E_UNSUPPORTED, "the BF16 re-rank supports d <= 2048");
    c->G = G; c->U = U;
    c->rpp = 1024;
    c->parts = (int)((B + c->rpp - 1) / c->rpp);
    return SUCO_OK;
}

inline int rerank_cfg(int d, int64_t B, RerankCfg *c) {
    if (d % 4) return fail(SUCO_E_UNSUPPORTED, "the re-rank needs d to be a multiple of 4");
    const int d4 = d / 4;
    int G = 1;
    while (G * 2 <= std::max(1, d4 / 2) && G < kWave) G *= 2;
    const int U = (d4 + G - 1) / G;
    if (U > kMaxU) return fail(SUCO_E_UNSUPPORTED, "the re-rank supports d <= 2048");
    c->G = G; c->U = U;
    c->rpp = 1024;
    c->parts = (int)((B + c->rpp - 1) / c->rpp);
    return SUCO_OK;
}


}  // namespace suco

namespace suco {
// The learned-budget network, for the batcher's graph (mlp.hip).
MlpView mlp_infer_view(suco_mlp *p);
int mlp_n_in(const suco_mlp *p);
int mlp_prepare(suco_mlp *p, hipStream_t st);
bool mlp_valid(const suco_mlp *p);
Launch plan_mlp_infer(int m_cap);
}  // namespace suco
