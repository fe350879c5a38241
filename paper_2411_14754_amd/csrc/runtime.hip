// Host side of the SuCo library: argument validation, the index object, the
// query workspace and the launch sequences behind the C ABI in suco.h.
#include <cstdio>

#include "runtime_impl.h"

using namespace suco;

namespace {

// Shapes the problem admits (INVAL otherwise) and, among them, those the
// kernels take (UNSUPPORTED otherwise).
int check_shape(int64_t n, int32_t d, int32_t ns, int32_t sk) {
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(SUCO_E_INVAL, "n must be in [1, 2^31)");
    if (d < 2) return fail(SUCO_E_INVAL, "d must be >= 2");
    if (ns < 1 || ns > d / 2) return fail(SUCO_E_INVAL, "n_s must be in [1, d/2]");
    if (sk < 1 || sk > n) return fail(SUCO_E_INVAL, "sqrt_k must be in [1, n]");
    if (ns > kMaxNs) return fail(SUCO_E_UNSUPPORTED, "the kernels take n_s <= 127");
    if (sk > kMaxSqrtK) return fail(SUCO_E_UNSUPPORTED, "the kernels take sqrt_k <= 128");
    return SUCO_OK;
}

// Contiguous division into ns subspaces (the last takes the remainder), each
// split into halves of floor(s/2) and the rest.
std::vector<HalfDims> make_layout(int d, int ns) {
    std::vector<HalfDims> h(2 * ns);
    const int s = d / ns;
    for (int i = 0; i < ns; ++i) {
        const int start = i * s, si = (i == ns - 1) ? d - (ns - 1) * s : s, h1 = si / 2;
        h[2 * i] = {start, h1};
        h[2 * i + 1] = {start + h1, si - h1};
    }
    return h;
}

// Allocate the index object and copy the dataset (D == null: the caller fills
// X); tiles are chosen so that a multiple of 8 tiles (one group per XCD)
// covers the ids when n is large.
int index_common(const float *D, int64_t n, int d, int ns, int sk, const suco_build_params *p,
                 hipStream_t st, suco_index **out) {
    int rc = check_shape(n, d, ns, sk);
    if (rc) return rc;
    int tile_max = p && p->tile_max ? p->tile_max : 65536;
    if (tile_max < 256 || tile_max > 65536 || tile_max % 256)
        return fail(SUCO_E_INVAL, "tile_max must be a multiple of 256 in [256, 65536]");
    int dev = 0, max_lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return fail(SUCO_E_HIP, "no usable HIP device");
    // the collision step keeps a tile of byte scores in LDS next to its static arrays
    const int static_lds = collide_static_lds();
    if (static_lds < 0) return fail(SUCO_E_HIP, "cannot query the collision kernel's attributes");
    tile_max = std::min(tile_max, (max_lds - static_lds) / 256 * 256);
    // by default keep two collision blocks resident per CU
    if (!(p && p->tile_max)) tile_max = std::min(tile_max, std::max(256, (max_lds / 2 - static_lds) / 256 * 256));
    if (tile_max < 256 || (int64_t)sk * sk * 4 > max_lds || (int64_t)sk * (sk + 1) * 4 + 4096 > max_lds)
        return fail(SUCO_E_UNSUPPORTED, "the device has too little LDS per work-group for this shape");
    if (p && (p->flags & SUCO_BUILD_BF16) && d % 8)
        return fail(SUCO_E_UNSUPPORTED, "SUCO_BUILD_BF16 needs d to be a multiple of 8");
    if (p && (p->flags & SUCO_BUILD_BF16) && (p->flags & SUCO_BUILD_L1))
        return fail(SUCO_E_UNSUPPORTED, "the split-precision form is Euclidean only (no SUCO_BUILD_L1)");
    suco_index *ix = new (std::nothrow) suco_index();
    if (!ix) return fail(SUCO_E_NOMEM, "host allocation failed");
    ix->device = dev;
    ix->n = n; ix->d = d; ix->ns = ns; ix->sk = sk; ix->K = sk * sk;
    ix->no_byte_rows = p && (p->flags & SUCO_BUILD_NO_BYTE_ROWS);
    ix->no_sparse = p && (p->flags & SUCO_BUILD_NO_SPARSE);
    ix->want_bf16 = p && (p->flags & SUCO_BUILD_BF16);
    ix->metric = p && (p->flags & SUCO_BUILD_L1) ? 1 : 0;
    ix->tile_req = p ? p->tile_max : 0;
    ix->chunk_req = p ? std::max(0, p->query_chunk) : 0;
    // The sparse collision step: one work-group per CU (160 KB of LDS per CU on
    // gfx950) with its tables, windows and as many ids as fit.
    ix->NB = (int)((n + kSpBucket - 1) / kSpBucket);
    if (!ix->no_sparse && ns <= kSpMaxNs5 && ix->NB <= kSpMaxBuckets) {
        const int sps = sparse_static_lds();
        if (sps < 0) { delete ix; return fail(SUCO_E_HIP, "cannot query the sparse collision kernel's attributes"); }
        const int64_t budget = std::min<int64_t>(max_lds, 160 * 1024) - sps;
        const int64_t cap = (budget - (int64_t)sp_lds_bytes(ix->NB, 0, sp_score_bits(ns))) / 2 / 8 * 8;
        ix->sp_cap = cap >= 4096 ? (int)std::min<int64_t>(cap, (int64_t)kSpMaxChunks * 1024) : 0;
    }
    const int64_t P0 = 8 * ((n + 8LL * tile_max - 1) / (8LL * tile_max));
    const int64_t per = (n + P0 - 1) / P0;
    ix->TILE = (int)((per + 255) / 256 * 256);
    ix->P = (int)((n + ix->TILE - 1) / ix->TILE);
    const int64_t span = (int64_t)ix->P * ix->TILE;
    // Queries per pass: a pass's workspace takes, per query, 2 bytes per point
    // (level lists), 2 bytes per cell and subspace (activated cells) and the
    // tile histograms; passes as large as 16 GiB of that allows (at most 16384
    // queries) cost less per query than small ones (fewer launches, fuller grids).
    const int64_t per_query = 2 * span + 2 * (int64_t)ns * sk * sk + 4 * (int64_t)ix->P * (ns + 2);
    if (p && p->query_chunk > 0) ix->chunk = p->query_chunk;
    else ix->chunk = (int)std::clamp<int64_t>((int64_t(1) << 34) / per_query, 16, 16384);
    ix->halves_h = make_layout(d, ns);
    if ((rc = dev_alloc(&ix->X, (size_t)n * d)) || (rc = dev_alloc(&ix->cent, (size_t)sk * d)) ||
        (rc = dev_alloc(&ix->halves, (size_t)2 * ns)) ||
        (rc = dev_alloc(&ix->toffs, (size_t)ns * ix->P * (ix->K + 1))) ||
        (rc = dev_alloc(&ix->ids16, (size_t)ns * span)) || (rc = dev_alloc(&ix->csize, (size_t)ns * ix->K)) ||
        (rc = dev_alloc(&ix->assign, (size_t)2 * ns * n)) ||
        (ix->sp_cap && ((rc = dev_alloc(&ix->coffs, (size_t)ns * (ix->K + 1))) ||
                        (rc = dev_alloc(&ix->ids32, (size_t)ns * n)) ||
                        (rc = dev_alloc(&ix->cbh, (size_t)ns * ix->K * sp_nb_padded(ix->NB)))))) {
        ix->release();
        delete ix;
        return rc;
    }
    if (hipEventCreateWithFlags(&ix->done, hipEventDisableTiming) != hipSuccess) {
        ix->release(); delete ix;
        return fail(SUCO_E_HIP, "hipEventCreate failed");
    }
    hipError_t e = D ? hipMemcpyAsync(ix->X, D, sizeof(float) * n * d, hipMemcpyDeviceToDevice, st) : hipSuccess;
    if (e == hipSuccess)
        e = hipMemcpyAsync(ix->halves, ix->halves_h.data(), sizeof(HalfDims) * 2 * ns, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(ix->csize, 0, sizeof(uint32_t) * ns * ix->K, st);
    if (e == hipSuccess) e = hipMemsetAsync(ix->ids16, 0, sizeof(uint16_t) * ns * span, st);
    if (e != hipSuccess) {
        ix->release(); delete ix;
        return fail(SUCO_E_HIP, std::string("index upload: ") + hipGetErrorString(e));
    }
    *out = ix;
    return SUCO_OK;
}

// IMI, then a byte copy of X for the re-rank when every coordinate is an
// integer in 0..255 (such rows convert back to FP32 exactly).
int finish_index(suco_index *ix, hipStream_t st) {
    HIPCHECK(launch_imi_build(ix->assign, ix->n, ix->ns, ix->sk, ix->P, ix->TILE, ix->toffs, ix->ids16,
                              ix->csize, st));
    if (ix->sp_cap) {
        HIPCHECK(launch_cell_major(ix->toffs, ix->ids16, ix->csize, ix->n, ix->ns, ix->K, ix->P, ix->TILE, ix->coffs,
                                   ix->ids32, st));
        HIPCHECK(launch_cell_buckets(ix->coffs, ix->ids32, ix->n, ix->ns, ix->K, ix->NB, ix->cbh, st));
    }
    int *bad = nullptr;
    int rc = dev_alloc(&bad, 1);
    if (rc) return rc;
    int hb = 1;
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), st);
    const int64_t m = ix->n * ix->d;
    if (e == hipSuccess) e = launch_check_bytes(ix->X, m, bad, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(SUCO_E_HIP, std::string("byte check: ") + hipGetErrorString(e));
    if (hb == 0 && ix->d % 4 == 0 && !ix->no_byte_rows) {
        if (dev_alloc(&ix->X8, (size_t)m) == SUCO_OK) {
            HIPCHECK(launch_to_bytes(ix->X, m, ix->X8, st));
        } else {
            (void)hipGetLastError();   // keep the FP32 rows only
        }
    }
    if (ix->want_bf16) {
        int rc2;
        if ((rc2 = dev_alloc(&ix->Xb, (size_t)m)) || (rc2 = dev_alloc(&ix->xerr, (size_t)ix->n)) ||
            (rc2 = dev_alloc(&ix->centb, (size_t)ix->sk * ix->d)) ||
            (rc2 = dev_alloc(&ix->cnorm2, (size_t)2 * ix->ns * ix->sk)))
            return rc2;
        HIPCHECK(launch_bf16_rows(ix->X, ix->n, ix->d, ix->Xb, ix->xerr, st));
        HIPCHECK(launch_bf16_centres(ix->cent, ix->halves, 2 * ix->ns, ix->sk, ix->d, ix->centb, ix->cnorm2, st));
    }
    HIPCHECK(hipStreamSynchronize(st));
    return SUCO_OK;
}

// Lloyd's k-means on every half, FP64, on the GPU.
int run_kmeans(suco_index *ix, int iters, uint64_t seed, hipStream_t st) {
    const int64_t n = ix->n;
    const int d = ix->d, ns = ix->ns, sk = ix->sk;
    int wmax = 0;
    for (const auto &h : ix->halves_h) wmax = std::max(wmax, h.w);
    // initial centres: SplitMix64 draws, first sk rows with distinct half-vectors
    const int64_t limit = 16LL * sk + 1024, M = limit + sk;
    std::vector<double> c64((size_t)sk * d);
    int64_t *cand_d = nullptr;
    float *rows_d = nullptr;
    int rc;
    if ((rc = dev_alloc(&cand_d, (size_t)M)) || (rc = dev_alloc(&rows_d, (size_t)M * wmax))) {
        if (cand_d) (void)hipFree(cand_d);
        return rc;
    }
    std::vector<int64_t> cand(M);
    std::vector<float> rows((size_t)M * wmax);
    for (int g = 0; g < 2 * ns && rc == SUCO_OK; ++g) {
        const HalfDims hd = ix->halves_h[g];
        const uint64_t base = seed ^ (0x632BE59BD9B4E019ULL * (uint64_t)(g + 1));
        for (int64_t m = 0; m < M; ++m) cand[m] = (int64_t)(splitmix64_at(base, (uint64_t)m) % (uint64_t)n);
        hipError_t e = hipMemcpyAsync(cand_d, cand.data(), sizeof(int64_t) * M, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = launch_gather_rows(ix->X, d, cand_d, (int)M, hd.dim0, hd.w, rows_d, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rows.data(), rows_d, sizeof(float) * M * hd.w, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { rc = fail(SUCO_E_HIP, std::string("k-means init: ") + hipGetErrorString(e)); break; }
        std::vector<int64_t> chosen;
        for (int64_t m = 0; (int)chosen.size() < sk; ++m) {
            bool ok = true;
            if (m < limit) {
                // distinct by value (a repeated id is a repeated row)
                for (size_t c = 0; c < chosen.size() && ok; ++c) {
                    bool same = true;
                    for (int j = 0; j < hd.w; ++j)
                        if (!(rows[(size_t)chosen[c] * hd.w + j] == rows[(size_t)m * hd.w + j])) { same = false; break; }
                    if (same) ok = false;
                }
            }
            if (ok) chosen.push_back(m);
        }
        for (int c = 0; c < sk; ++c)
            for (int j = 0; j < hd.w; ++j)
                c64[(size_t)sk * hd.dim0 + (size_t)c * hd.w + j] = (double)rows[(size_t)chosen[c] * hd.w + j];
    }
    (void)hipFree(cand_d);
    (void)hipFree(rows_d);
    if (rc) return rc;

    KmeansPass kp{};
    kp.X = ix->X; kp.n = n; kp.d = d; kp.ns = ns; kp.sk = sk; kp.nb = (int)((n + 255) / 256); kp.wmax = wmax;
    kp.halves = ix->halves; kp.assign = ix->assign; kp.metric = ix->metric;
    double *cent64 = nullptr;
    uint32_t *bh = nullptr, *cbase = nullptr, *order = nullptr;
    if ((rc = dev_alloc(&cent64, (size_t)sk * d)) || (rc = dev_alloc(&bh, (size_t)2 * ns * kp.nb * sk)) ||
        (rc = dev_alloc(&cbase, (size_t)2 * ns * (sk + 1))) || (rc = dev_alloc(&order, (size_t)2 * ns * n))) {
        for (void *q : {(void *)cent64, (void *)bh, (void *)cbase, (void *)order}) if (q) (void)hipFree(q);
        return rc;
    }
    kp.cent64 = cent64; kp.bh = bh; kp.cbase = cbase; kp.order = order;
    hipError_t e = hipMemcpyAsync(cent64, c64.data(), sizeof(double) * sk * d, hipMemcpyHostToDevice, st);
    for (int it = 0; it <= iters && e == hipSuccess; ++it) {
        e = launch_km_assign(kp, ix->halves_h.data(), it < iters, st);
        if (it == iters || e != hipSuccess) break;
        if ((e = launch_km_scan(kp, st)) != hipSuccess) break;
        if ((e = launch_km_scatter(kp, st)) != hipSuccess) break;
        e = kp.metric ? launch_km_median(kp, st) : launch_km_update(kp, st);
    }
    if (e == hipSuccess) e = launch_cent_to_f32(cent64, ix->cent, (int64_t)sk * d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(c64.data(), cent64, sizeof(double) * sk * d, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (void *q : {(void *)cent64, (void *)bh, (void *)cbase, (void *)order}) (void)hipFree(q);
    if (e != hipSuccess) return fail(SUCO_E_HIP, std::string("k-means: ") + hipGetErrorString(e));
    ix->cent_h.resize((size_t)sk * d);
    for (size_t t = 0; t < c64.size(); ++t) ix->cent_h[t] = (float)c64[t];
    return SUCO_OK;
}


// ----------------------------------------------------------- persistence --
// File layout (little-endian): a 64-byte header, then the FP32 centres
// [sqrt_k*d], the assignments as bytes [2*n_s][n] and the data [n][d] FP32,
// each section zero-padded to a multiple of 8 bytes.  The header's checksum
// covers everything after the header: a 64-bit word hash (h = (h ^ w) *
// 0x100000001b3 over the little-endian 8-byte words, h0 = 0xcbf29ce484222325,
// the FNV-1a constants).
struct FileHeader {
    char magic[8];          // "SUCOIDX1"
    uint32_t version;       // 1
    uint32_t header_bytes;  // 64
    int64_t n;
    int32_t d, ns, sk;
    int32_t flags;          // SUCO_BUILD_* bits the index was built with
    int32_t tile_max, query_chunk;
    uint64_t checksum;
    uint8_t pad[8];
};
static_assert(sizeof(FileHeader) == 64, "file header is 64 bytes");
constexpr char kFileMagic[8] = {'S', 'U', 'C', 'O', 'I', 'D', 'X', '1'};
constexpr uint64_t kHashInit = 0xcbf29ce484222325ULL, kHashMul = 0x100000001b3ULL;

inline uint64_t pad8(uint64_t b) { return (b + 7) & ~uint64_t(7); }

struct WordHash {
    uint64_t h = kHashInit;
    void add(const void *p, size_t bytes) {   // bytes: a multiple of 8
        const uint8_t *b = static_cast<const uint8_t *>(p);
        for (size_t t = 0; t < bytes; t += 8) {
            uint64_t w;
            std::memcpy(&w, b + t, 8);
            h = (h ^ w) * kHashMul;
        }
    }
};

struct File {
    FILE *f = nullptr;
    ~File() { if (f) std::fclose(f); }
};

// Write `bytes` from `src` followed by zero padding to a multiple of 8, hashing both.
bool write_section(FILE *f, const void *src, uint64_t bytes, WordHash &hs) {
    const uint64_t full = bytes / 8 * 8, rest = bytes - full;
    if (full && std::fwrite(src, 1, full, f) != full) return false;
    hs.add(src, full);
    if (rest) {
        uint8_t tail[8] = {0};
        std::memcpy(tail, static_cast<const uint8_t *>(src) + full, rest);
        if (std::fwrite(tail, 1, 8, f) != 8) return false;
        hs.add(tail, 8);
    }
    return true;
}

bool read_section(FILE *f, void *dst, uint64_t bytes, WordHash &hs) {
    const uint64_t full = bytes / 8 * 8, rest = bytes - full;
    if (full && std::fread(dst, 1, full, f) != full) return false;
    hs.add(dst, full);
    if (rest) {
        uint8_t tail[8];
        if (std::fread(tail, 1, 8, f) != 8) return false;
        hs.add(tail, 8);
        std::memcpy(static_cast<uint8_t *>(dst) + full, tail, rest);
        for (uint64_t t = rest; t < 8; ++t)
            if (tail[t]) return false;
    }
    return true;
}

// Rows of X are moved between the device and the file through a pinned buffer.
constexpr size_t kStageBytes = size_t(64) << 20;

int save_index(const suco_index *ix, const char *path) {
    DeviceGuard dg(ix->device);
    const std::string tmp = std::string(path) + ".tmp";
    File out;
    out.f = std::fopen(tmp.c_str(), "wb");
    if (!out.f) return fail(SUCO_E_INVAL, std::string("cannot open ") + tmp + " for writing");
    FileHeader h{};
    std::memcpy(h.magic, kFileMagic, 8);
    h.version = 1; h.header_bytes = sizeof(FileHeader);
    h.n = ix->n; h.d = ix->d; h.ns = ix->ns; h.sk = ix->sk;
    h.flags = (ix->no_byte_rows ? SUCO_BUILD_NO_BYTE_ROWS : 0) | (ix->want_bf16 ? SUCO_BUILD_BF16 : 0) |
              (ix->no_sparse ? SUCO_BUILD_NO_SPARSE : 0) | (ix->metric ? SUCO_BUILD_L1 : 0);
    h.tile_max = ix->tile_req; h.query_chunk = ix->chunk_req;
    if (std::fwrite(&h, sizeof h, 1, out.f) != 1) return fail(SUCO_E_INVAL, "write failed: " + tmp);
    WordHash hs;
    std::vector<uint8_t> a8((size_t)2 * ix->ns * ix->n);
    HIPCHECK(hipMemcpy(a8.data(), ix->assign, a8.size(), hipMemcpyDeviceToHost));
    if (!write_section(out.f, ix->cent_h.data(), sizeof(float) * ix->cent_h.size(), hs) ||
        !write_section(out.f, a8.data(), a8.size(), hs))
        return fail(SUCO_E_INVAL, "write failed: " + tmp);
    const uint64_t xbytes = sizeof(float) * (uint64_t)ix->n * ix->d;
    void *stage = nullptr;
    HIPCHECK(hipHostMalloc(&stage, kStageBytes, hipHostMallocDefault));
    int rc = SUCO_OK;
    // whole 8-byte words per chunk; the tail (and its padding) is written last
    const uint64_t words = xbytes / 8 * 8;
    for (uint64_t off = 0; off < words && rc == SUCO_OK; off += kStageBytes) {
        const uint64_t len = std::min<uint64_t>(kStageBytes, words - off);
        hipError_t e = hipMemcpy(stage, reinterpret_cast<const char *>(ix->X) + off, len, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(SUCO_E_HIP, std::string("reading X: ") + hipGetErrorString(e));
        else if (!write_section(out.f, stage, len, hs)) rc = fail(SUCO_E_INVAL, "write failed: " + tmp);
    }
    if (rc == SUCO_OK && xbytes > words) {
        hipError_t e = hipMemcpy(stage, reinterpret_cast<const char *>(ix->X) + words, xbytes - words,
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(SUCO_E_HIP, std::string("reading X: ") + hipGetErrorString(e));
        else if (!write_section(out.f, stage, xbytes - words, hs)) rc = fail(SUCO_E_INVAL, "write failed: " + tmp);
    }
    (void)hipHostFree(stage);
    if (rc) return rc;
    h.checksum = hs.h;
    if (std::fseek(out.f, 0, SEEK_SET) != 0 || std::fwrite(&h, sizeof h, 1, out.f) != 1 || std::fflush(out.f) != 0)
        return fail(SUCO_E_INVAL, "write failed: " + tmp);
    std::fclose(out.f);
    out.f = nullptr;
    if (std::rename(tmp.c_str(), path) != 0) return fail(SUCO_E_INVAL, std::string("cannot rename to ") + path);
    return SUCO_OK;
}

// Header and size checks come first, before any device work.
int load_index(const char *path, const suco_build_params *pin, hipStream_t st, suco_index **out) {
    File in;
    in.f = std::fopen(path, "rb");
    if (!in.f) return fail(SUCO_E_INVAL, std::string("cannot open ") + path);
    FileHeader h{};
    if (std::fread(&h, sizeof h, 1, in.f) != 1 || std::memcmp(h.magic, kFileMagic, 8) != 0 || h.version != 1 ||
        h.header_bytes != sizeof(FileHeader))
        return fail(SUCO_E_INVAL, std::string(path) + " is not a SuCo index file");
    int rc = check_shape(h.n, h.d, h.ns, h.sk);
    if (rc) return fail(rc, std::string(path) + ": " + g_err);
    const uint64_t cbytes = sizeof(float) * (uint64_t)h.sk * h.d, abytes = (uint64_t)2 * h.ns * h.n,
                   xbytes = sizeof(float) * (uint64_t)h.n * h.d;
    const uint64_t want = sizeof(FileHeader) + pad8(cbytes) + pad8(abytes) + pad8(xbytes);
    if (std::fseek(in.f, 0, SEEK_END) != 0) return fail(SUCO_E_INVAL, std::string("cannot seek in ") + path);
    const long long size = std::ftell(in.f);
    if (size < 0 || (uint64_t)size != want)
        return fail(SUCO_E_INVAL, std::string(path) + ": size " + std::to_string(size) + " bytes, expected " +
                                      std::to_string(want));
    if (std::fseek(in.f, sizeof(FileHeader), SEEK_SET) != 0) return fail(SUCO_E_INVAL, "seek failed");
    WordHash hs;
    std::vector<float> cent((size_t)h.sk * h.d);
    std::vector<uint8_t> a8((size_t)abytes);
    if (!read_section(in.f, cent.data(), cbytes, hs) || !read_section(in.f, a8.data(), abytes, hs))
        return fail(SUCO_E_INVAL, std::string(path) + ": read failed or bad padding");
    for (uint8_t a : a8)
        if (a >= h.sk) return fail(SUCO_E_INVAL, std::string(path) + ": assignment out of [0, sqrt_k)");
    suco_build_params p{};
    if (pin) p = *pin;
    else { p.flags = h.flags; p.tile_max = h.tile_max; p.query_chunk = h.query_chunk; }
    p.flags = (p.flags & ~SUCO_BUILD_L1) | (h.flags & SUCO_BUILD_L1);   // the metric the centres were built for
    suco_index *ix = nullptr;
    if ((rc = index_common(nullptr, h.n, h.d, h.ns, h.sk, &p, st, &ix))) return rc;
    auto drop = [&](int code) {
        (void)hipStreamSynchronize(st);
        ix->release();
        delete ix;
        return code;
    };
    void *stage = nullptr;
    if (hipHostMalloc(&stage, kStageBytes, hipHostMallocDefault) != hipSuccess)
        return drop(fail(SUCO_E_NOMEM, "pinned staging buffer"));
    // whole 8-byte words per chunk, then the tail with its padding
    const uint64_t words = xbytes / 8 * 8;
    auto upload = [&](uint64_t off, uint64_t len) {
        if (!read_section(in.f, stage, len, hs)) return fail(SUCO_E_INVAL, std::string(path) + ": read failed");
        hipError_t e = hipMemcpyAsync(reinterpret_cast<char *>(ix->X) + off, stage, len, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(SUCO_E_HIP, std::string("uploading X: ") + hipGetErrorString(e));
        return SUCO_OK;
    };
    for (uint64_t off = 0; off < words && rc == SUCO_OK; off += kStageBytes)
        rc = upload(off, std::min<uint64_t>(kStageBytes, words - off));
    if (rc == SUCO_OK && xbytes > words) rc = upload(words, xbytes - words);
    (void)hipHostFree(stage);
    if (rc) return drop(rc);
    if (hs.h != h.checksum) return drop(fail(SUCO_E_INVAL, std::string(path) + ": checksum mismatch"));
    ix->cent_h = cent;
    hipError_t e = hipMemcpyAsync(ix->cent, cent.data(), cbytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ix->assign, a8.data(), abytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return drop(fail(SUCO_E_HIP, std::string("index upload: ") + hipGetErrorString(e)));
    if ((rc = finish_index(ix, st))) return drop(rc);
    *out = ix;
    return SUCO_OK;
}

// ------------------------------------------------------------ workspace --
struct Work {
    uint16_t *cells; int32_t *ncells, *aprime; float *feat; uint32_t *hist; uint16_t *lvl; uint8_t *scores;
    uint32_t *cand; uint64_t *part_keys; int32_t *order, *route;
};

// dense: also room for the dense SC-scores (exported on request only)
Work carve(const suco_index *ix, char *base, size_t C, int64_t B, int k, int parts, bool dense, size_t *bytes) {
    Carve c{base};
    Work w;
    w.cells = c.take<uint16_t>(C * ix->ns * ix->K);
    w.ncells = c.take<int32_t>(C * ix->ns);
    w.aprime = c.take<int32_t>(C * ix->ns);
    w.feat = c.take<float>(C * 2 * ix->ns);
    w.hist = c.take<uint32_t>(C * ix->P * (ix->ns + 2));
    // (the sparse step's unconditional loads may read up to one bucket past a row's end)
    w.lvl = c.take<uint16_t>(C * (size_t)ix->P * ix->TILE + 2 * kSpBucket);
    w.scores = dense ? c.take<uint8_t>(C * (size_t)ix->P * ix->TILE) : nullptr;
    w.cand = c.take<uint32_t>(C * (size_t)B);
    w.order = c.take<int32_t>(C);
    w.route = c.take<int32_t>(2 * C + 1);   // route, then the tiled list and its count
    w.part_keys = c.take<uint64_t>(C * (size_t)parts * k);
    if (bytes) *bytes = c.off;
    return w;
}

struct DebugOut {
    uint8_t *scores = nullptr; int32_t *cand = nullptr; int32_t *ncells = nullptr; int32_t *aprime = nullptr;
    uint16_t *cells = nullptr; float *feat = nullptr;
};

int check_query(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double beta, int32_t *ids,
                float *dists) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (nq < 0) return fail(SUCO_E_INVAL, "nq must be >= 0");
    if (k < 1 || k > ix->n) return fail(SUCO_E_INVAL, "k must be in [1, n]");
    if (k > kMaxK) return fail(SUCO_E_UNSUPPORTED, "the kernels take k <= 64");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SUCO_E_INVAL, "beta must be in (0, 1]");
    if (nq > 0 && (!Q || !ids || !dists)) return fail(SUCO_E_INVAL, "Q, ids and dists must not be NULL");
    return SUCO_OK;
}

// BF16 split precision (suco_query_bf16): optional MFMA centre distances, and
// the re-rank as BF16 first pass, certified survivors, FP32 re-rank of those.
struct Bf16Opts {
    int flags = 0;
    int32_t *nsurv = nullptr;
    double *relerr = nullptr;
    float *cdist = nullptr;
};

// Workspace given by the caller instead of the index's arena (the entry point
// that allocates nothing): passes are sized to fit `bytes`, no timing events
// are recorded and the index's arena bookkeeping is left alone.
struct FixedWork {
    char *base;
    size_t bytes;
};

int run_query(const suco_index *cix, const float *Q, int64_t nq, int32_t k, const float *alpha_q, double alpha,
              double beta, int32_t *ids, float *dists, const DebugOut *dbg, const Bf16Opts *bo, hipStream_t st,
              const FixedWork *fx = nullptr) {
    int rc = check_query(cix, Q, nq, k, beta, ids, dists);
    if (rc) return rc;
    if (!alpha_q && !(alpha > 0.0 && alpha <= 1.0)) return fail(SUCO_E_INVAL, "alpha must be in (0, 1]");
    if (bo) {
        if (bo->flags & ~SUCO_BF16_S1) return fail(SUCO_E_INVAL, "unknown flags");
        if (!cix->Xb) return fail(SUCO_E_STATE, "the index was built without SUCO_BUILD_BF16");
    }
    if (nq == 0) return SUCO_OK;
    suco_index *ix = const_cast<suco_index *>(cix);
    const int64_t B = count_B_host(beta, ix->n, k);
    RerankCfg c32, c16{};
    if ((rc = rerank_cfg(ix->d, B, &c32))) return rc;
    if (bo && (rc = rerank_bf16_cfg(ix->d, B, &c16))) return rc;
    const int parts = std::max(c32.parts, c16.parts);
    std::unique_lock<std::mutex> lock(ix->mu, std::defer_lock);
    if (!fx) lock.lock();
    DeviceGuard dg(ix->device);
    int64_t cap = ix->chunk;
    if (fx) {
        // the largest pass whose workspace fits the fixed buffer
        auto need = [&](int64_t c) { size_t b = 0; carve(ix, nullptr, (size_t)c, B, k, parts, false, &b); return b; };
        int64_t lo = 0, hi = std::min<int64_t>(nq, ix->chunk);
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (need(mid) <= fx->bytes) lo = mid; else hi = mid - 1;
        }
        if (lo == 0)
            return fail(SUCO_E_UNSUPPORTED, "one query needs " + std::to_string(need(1)) +
                                                " bytes of workspace; the fixed scratch holds " +
                                                std::to_string(fx->bytes));
        cap = lo;
    }
    const size_t C = (size_t)pass_size(nq, cap);
    const int nh = 2 * ix->ns;
    const bool dense = dbg && dbg->scores;
    // BF16 buffers follow the common workspace
    float *D = nullptr, *lo = nullptr;
    uint32_t *surv = nullptr;
    int32_t *nsv = nullptr;
    auto extra = [&](char *base, size_t off) {
        Carve cv{base, off};
        D = cv.take<float>(C * nh * ix->sk);
        lo = cv.take<float>(C * (size_t)B);
        surv = cv.take<uint32_t>(C * (size_t)B);
        nsv = cv.take<int32_t>(C);
        return cv.off;
    };
    char *base = fx ? fx->base : nullptr;
    if (!fx) {
        size_t bytes = 0;
        carve(ix, nullptr, C, B, k, parts, dense, &bytes);
        if (bo) bytes = extra(nullptr, bytes);
        if ((rc = ensure_arena(ix, bytes))) return rc;
        if (ix->pending) HIPCHECK(hipStreamWaitEvent(st, ix->done, 0));
        base = ix->arena;
    }
    size_t wbytes = 0;
    Work w = carve(ix, base, C, B, k, parts, dense, &wbytes);
    if (bo) extra(base, wbytes);
    // every launch of a pass, with timing events when profiling is on
    auto T = [&](int stage, auto &&fn) { return fx ? fn() : timed(ix, stage, st, fn); };
    const IndexView v = ix->view();
    for (int64_t c0 = 0; c0 < nq; c0 += (int64_t)C) {
        const int cn = (int)std::min<int64_t>((int64_t)C, nq - c0);
        QueryPass qp{};
        qp.ix = v;
        qp.Q = Q + c0 * ix->d;
        qp.nq = cn;
        qp.alpha_q = alpha_q ? alpha_q + c0 : nullptr;
        qp.alpha = alpha;
        qp.B = B;
        qp.runs_per_sub = runs_per_sub(ix->ns);
        qp.tgroups = tile_groups(qp.nq, ix->P);
        qp.k = k;
        qp.cells = w.cells; qp.ncells = w.ncells; qp.aprime = w.aprime;
        qp.feat = (dbg && dbg->feat) ? dbg->feat + c0 * 2 * ix->ns : nullptr;
        qp.hist = w.hist; qp.lvl = w.lvl; qp.scores = w.scores; qp.cand = w.cand;
        qp.route = ix->sp_cap ? w.route : nullptr;
        qp.tlist = qp.route ? w.route + C : nullptr;
        qp.ntl = qp.route ? w.route + 2 * C : nullptr;
        qp.sp_cap = ix->sp_cap;
        if (bo && (bo->flags & SUCO_BF16_S1)) {
            CentreBf16Pass cp{};
            cp.Q = qp.Q; cp.nq = cn; cp.d = ix->d; cp.sk = ix->sk; cp.nh = nh; cp.halves = ix->halves;
            cp.centb = ix->centb; cp.cnorm2 = ix->cnorm2; cp.D = D;
            HIPCHECK(T(kCentresBf16, [&] { return launch(plan_centre_dists_bf16(cp), &cp, st); }));
            qp.Dext = D;
            if (bo->cdist)
                HIPCHECK(hipMemcpyAsync(bo->cdist + c0 * nh * ix->sk, D, sizeof(float) * cn * nh * ix->sk,
                                        hipMemcpyDeviceToDevice, st));
        }
        HIPCHECK(T(kActivate, [&] { return launch_activate(qp, st); }));
        if (cn <= kOrderWide) {
            qp.order_out = w.order;
            HIPCHECK(T(kOrder, [&] { return launch(plan_order(qp), &qp, st); }));
            qp.order = w.order;
        }
        if (qp.route) HIPCHECK(T(kCollideSparse, [&] { return launch(plan_collide_sparse(qp, 0), &qp, st); }));
        HIPCHECK(T(kCollide, [&] { return launch_collide(qp, st); }));
        HIPCHECK(T(kSelect, [&] { return launch_select(qp, st); }));
        RerankPass rp{};
        rp.X = ix->X; rp.X8 = ix->X8; rp.Q = qp.Q; rp.cand = w.cand; rp.B = B; rp.n = ix->n; rp.d = ix->d; rp.k = k; rp.nq = cn;
        rp.metric = ix->metric;
        rp.parts = c32.parts; rp.rows_per_part = c32.rpp; rp.G = c32.G; rp.U = c32.U;
        rp.part_keys = w.part_keys; rp.ids = ids + c0 * k; rp.dists = dists + c0 * k;
        if (bo) {
            Bf16RerankPass bp{};
            bp.Xb = ix->Xb; bp.xerr = ix->xerr; bp.Q = qp.Q; bp.cand = w.cand; bp.B = B; bp.n = ix->n;
            bp.d = ix->d; bp.k = k; bp.nq = cn; bp.parts = c16.parts; bp.rows_per_part = c16.rpp; bp.G = c16.G;
            bp.U = c16.U; bp.part_keys = w.part_keys; bp.lo = lo; bp.surv = surv; bp.nsurv = nsv;
            HIPCHECK(T(kRerankBf16, [&] { return launch(plan_rerank_bf16(bp, 0), &bp, st); }));
            HIPCHECK(T(kSurvivors, [&] { return launch(plan_survivors(bp), &bp, st); }));
            // the FP32 re-rank of the survivors: one part per query
            rp.cand = surv; rp.rows_dev = nsv; rp.parts = 1; rp.rows_per_part = B;
        }
        HIPCHECK(T(kRerank, [&] { return launch_rerank(rp, st); }));
        HIPCHECK(T(kMerge, [&] { return launch_merge(rp, st); }));
        if (bo && bo->nsurv)
            HIPCHECK(hipMemcpyAsync(bo->nsurv + c0, nsv, sizeof(int32_t) * cn, hipMemcpyDeviceToDevice, st));
        if (bo && bo->relerr) {
            RelErrPass ep{};
            ep.X = ix->X; ep.n = ix->n; ep.Q = qp.Q; ep.ids = rp.ids; ep.dists = rp.dists; ep.nq = cn; ep.d = ix->d; ep.k = k;
            ep.relerr = bo->relerr + c0 * k;
            HIPCHECK(launch(plan_relerr(ep), &ep, st));
        }
        if (dbg) {
            const int ns = ix->ns;
            if (dbg->ncells)
                HIPCHECK(hipMemcpyAsync(dbg->ncells + c0 * ns, w.ncells, sizeof(int32_t) * cn * ns,
                                        hipMemcpyDeviceToDevice, st));
            if (dbg->aprime)
                HIPCHECK(hipMemcpyAsync(dbg->aprime + c0 * ns, w.aprime, sizeof(int32_t) * cn * ns,
                                        hipMemcpyDeviceToDevice, st));
            if (dbg->cells)
                HIPCHECK(hipMemcpyAsync(dbg->cells + c0 * ns * ix->K, w.cells, sizeof(uint16_t) * cn * ns * ix->K,
                                        hipMemcpyDeviceToDevice, st));
            if (dbg->cand)
                HIPCHECK(hipMemcpyAsync(dbg->cand + c0 * B, w.cand, sizeof(uint32_t) * cn * B,
                                        hipMemcpyDeviceToDevice, st));
            if (dbg->scores)
                HIPCHECK(hipMemcpy2DAsync(dbg->scores + c0 * ix->n, (size_t)ix->n, w.scores,
                                          (size_t)ix->P * ix->TILE, (size_t)ix->n, (size_t)cn,
                                          hipMemcpyDeviceToDevice, st));
        }
    }
    if (!fx) {
        HIPCHECK(hipEventRecord(ix->done, st));
        ix->pending = true;
    }
    return SUCO_OK;
}

}  // namespace

// -------------------------------------------------------------- no-alloc --
// Workspace of suco_query_noalloc: a fixed array in the library's device code
// object.  Every device the library runs on holds its own copy until the
// process ends; host code reaches it only through the address
// hipGetSymbolAddress returns with that device current (the array's name is a
// host-side stand-in, not a device address).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch[kScratchDevices] = {};

// The scratch array's address on the current device, looked up once per device.
int scratch_on(int dev, char **out) {
    if (dev < 0 || dev >= kScratchDevices) return fail(SUCO_E_UNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SUCO_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<char *>(p);
    }
    *out = g_scratch[dev];
    return SUCO_OK;
}
}  // namespace

// ================================================================== ABI ==
extern "C" {

int suco_version(void) { return 1; }

const char *suco_last_error(void) { return g_err.c_str(); }

int64_t suco_count_A(double alpha, int64_t n) { return n < 1 ? 0 : count_A_host(alpha, n); }

int64_t suco_count_B(double beta, int64_t n, int32_t k) { return n < 1 ? 0 : count_B_host(beta, n, k); }

int suco_build(const float *D, int64_t n, int32_t d, int32_t n_s, int32_t sqrt_k, const suco_build_params *p,
               void *stream, suco_index **out) {
    if (!D || !out) return fail(SUCO_E_INVAL, "D and out must not be NULL");
    const int iters = p && p->iters > 0 ? p->iters : 25;
    const uint64_t seed = p && p->seed ? p->seed : 1;
    hipStream_t st = (hipStream_t)stream;
    suco_index *ix = nullptr;
    int rc = index_common(D, n, d, n_s, sqrt_k, p, st, &ix);
    if (rc) return rc;
    if ((rc = run_kmeans(ix, iters, seed, st)) || (rc = finish_index(ix, st))) {
        (void)hipStreamSynchronize(st);
        ix->release();
        delete ix;
        return rc;
    }
    *out = ix;
    return SUCO_OK;
}

int suco_build_from_index(const float *D, int64_t n, int32_t d, int32_t n_s, int32_t sqrt_k,
                          const float *centroids, const int32_t *assign, const suco_build_params *p,
                          void *stream, suco_index **out) {
    if (!D || !out || !centroids || !assign) return fail(SUCO_E_INVAL, "NULL argument");
    int rc = check_shape(n, d, n_s, sqrt_k);
    if (rc) return rc;
    std::vector<uint8_t> a8((size_t)2 * n_s * n);
    for (size_t t = 0; t < a8.size(); ++t) {
        if (assign[t] < 0 || assign[t] >= sqrt_k) return fail(SUCO_E_INVAL, "assignment out of [0, sqrt_k)");
        a8[t] = (uint8_t)assign[t];
    }
    hipStream_t st = (hipStream_t)stream;
    suco_index *ix = nullptr;
    if ((rc = index_common(D, n, d, n_s, sqrt_k, p, st, &ix))) return rc;
    ix->cent_h.assign(centroids, centroids + (size_t)sqrt_k * d);
    hipError_t e = hipMemcpyAsync(ix->cent, centroids, sizeof(float) * sqrt_k * d, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ix->assign, a8.data(), a8.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) rc = fail(SUCO_E_HIP, std::string("index upload: ") + hipGetErrorString(e));
    if (!rc) rc = finish_index(ix, st);
    if (rc) {
        (void)hipStreamSynchronize(st);
        ix->release();
        delete ix;
        return rc;
    }
    *out = ix;
    return SUCO_OK;
}

int suco_index_export(const suco_index *ix, float *centroids, int32_t *assign) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (centroids) std::memcpy(centroids, ix->cent_h.data(), sizeof(float) * ix->cent_h.size());
    if (assign) {
        DeviceGuard dg(ix->device);
        std::vector<uint8_t> a8((size_t)2 * ix->ns * ix->n);
        HIPCHECK(hipMemcpy(a8.data(), ix->assign, a8.size(), hipMemcpyDeviceToHost));
        for (size_t t = 0; t < a8.size(); ++t) assign[t] = a8[t];
    }
    return SUCO_OK;
}

int suco_index_save(const suco_index *ix, const char *path) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (!path) return fail(SUCO_E_INVAL, "path must not be NULL");
    return save_index(ix, path);
}

int suco_index_load(const char *path, const suco_build_params *p, void *stream, suco_index **out) {
    if (!path || !out) return fail(SUCO_E_INVAL, "path and out must not be NULL");
    return load_index(path, p, (hipStream_t)stream, out);
}

int suco_index_info(const suco_index *ix, int64_t *n, int32_t *d, int32_t *n_s, int32_t *sqrt_k) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (n) *n = ix->n;
    if (d) *d = ix->d;
    if (n_s) *n_s = ix->ns;
    if (sqrt_k) *sqrt_k = ix->sk;
    return SUCO_OK;
}

int suco_index_flags(const suco_index *ix, int32_t *flags) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (!flags) return fail(SUCO_E_INVAL, "flags must not be NULL");
    *flags = (ix->X8 ? SUCO_INDEX_BYTE_ROWS : 0) | (ix->Xb ? SUCO_INDEX_BF16 : 0) | (ix->metric ? SUCO_INDEX_L1 : 0) |
             (ix->sp_cap ? SUCO_INDEX_SPARSE : 0);
    return SUCO_OK;
}

int suco_index_set_activation(suco_index *ix, int32_t form) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (form != SUCO_ACT_DYNAMIC && form != SUCO_ACT_MULTISEQ) return fail(SUCO_E_INVAL, "unknown activation rule");
    if (form == SUCO_ACT_MULTISEQ && ix->sk > kWave)
        return fail(SUCO_E_UNSUPPORTED, "the Multi-sequence traversal takes sqrt_k <= 64");
    std::lock_guard<std::mutex> lock(ix->mu);
    ix->act_form = form;
    return SUCO_OK;
}

int suco_index_free(suco_index *ix) {
    if (!ix) return SUCO_OK;
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    {
        DeviceGuard dg(ix->device);
        std::lock_guard<std::mutex> lock(ix->mu);
        ix->release();
    }
    delete ix;
    return SUCO_OK;
}

int suco_query(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha, double beta,
               int32_t *ids, float *dists, void *stream) {
    return run_query(ix, Q, nq, k, nullptr, alpha, beta, ids, dists, nullptr, nullptr, (hipStream_t)stream);
}

int suco_query_noalloc(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha, double beta,
                       int32_t *ids, float *dists, void *stream) {
    int rc = check_query(ix, Q, nq, k, beta, ids, dists);
    if (rc) return rc;
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(SUCO_E_INVAL, "alpha must be in (0, 1]");
    if (nq == 0) return SUCO_OK;
    char *base = nullptr;
    {
        DeviceGuard dg(ix->device);
        if ((rc = scratch_on(ix->device, &base))) return rc;
    }
    FixedWork fx{base, kScratchBytes};
    return run_query(ix, Q, nq, k, nullptr, alpha, beta, ids, dists, nullptr, nullptr, (hipStream_t)stream, &fx);
}

int suco_query_alpha(const suco_index *ix, const float *Q, int64_t nq, int32_t k, const float *alpha_q,
                     double beta, int32_t *ids, float *dists, void *stream) {
    if (nq > 0 && !alpha_q) return fail(SUCO_E_INVAL, "alpha_q must not be NULL");
    return run_query(ix, Q, nq, k, alpha_q, 0.0, beta, ids, dists, nullptr, nullptr, (hipStream_t)stream);
}

int suco_query_debug(const suco_index *ix, const float *Q, int64_t nq, int32_t k, const float *alpha_q,
                     double alpha, double beta, int32_t *ids, float *dists, uint8_t *scores, int32_t *cand,
                     int32_t *ncells, int32_t *aprime, uint16_t *cells, float *feat, void *stream) {
    DebugOut dbg;
    dbg.scores = scores; dbg.cand = cand; dbg.ncells = ncells; dbg.aprime = aprime; dbg.cells = cells;
    dbg.feat = feat;
    return run_query(ix, Q, nq, k, alpha_q, alpha, beta, ids, dists, &dbg, nullptr, (hipStream_t)stream);
}

int suco_query_bf16(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha, double beta,
                    int32_t flags, int32_t *ids, float *dists, int32_t *nsurv, double *relerr, float *cdist,
                    void *stream) {
    Bf16Opts bo;
    bo.flags = flags; bo.nsurv = nsurv; bo.relerr = relerr; bo.cdist = cdist;
    return run_query(ix, Q, nq, k, nullptr, alpha, beta, ids, dists, nullptr, &bo, (hipStream_t)stream);
}

int suco_query_bf16_debug(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha, double beta,
                          int32_t flags, int32_t *ids, float *dists, int32_t *nsurv, double *relerr, float *cdist,
                          uint8_t *scores, int32_t *cand, int32_t *ncells, int32_t *aprime, uint16_t *cells,
                          void *stream) {
    Bf16Opts bo;
    bo.flags = flags; bo.nsurv = nsurv; bo.relerr = relerr; bo.cdist = cdist;
    DebugOut dbg;
    dbg.scores = scores; dbg.cand = cand; dbg.ncells = ncells; dbg.aprime = aprime; dbg.cells = cells;
    return run_query(ix, Q, nq, k, nullptr, alpha, beta, ids, dists, &dbg, &bo, (hipStream_t)stream);
}

int suco_collide_select(const suco_index *cix, int64_t nq, const uint16_t *cells, const int32_t *ncells,
                        int32_t k, double beta, uint8_t *scores, int32_t *cand, void *stream) {
    if (!index_ok(cix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (nq < 0) return fail(SUCO_E_INVAL, "nq must be >= 0");
    if (k < 1 || k > cix->n) return fail(SUCO_E_INVAL, "k must be in [1, n]");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SUCO_E_INVAL, "beta must be in (0, 1]");
    if (nq > 0 && (!cells || !ncells || !cand)) return fail(SUCO_E_INVAL, "cells, ncells, cand must not be NULL");
    if (nq == 0) return SUCO_OK;
    suco_index *ix = const_cast<suco_index *>(cix);
    hipStream_t st = (hipStream_t)stream;
    const int64_t B = count_B_host(beta, ix->n, k);
    std::lock_guard<std::mutex> lock(ix->mu);
    DeviceGuard dg(ix->device);
    const size_t C = (size_t)pass_size(nq, ix->chunk);
    size_t bytes = 0;
    carve(ix, nullptr, C, B, k, 1, scores != nullptr, &bytes);
    int rc = ensure_arena(ix, bytes);
    if (rc) return rc;
    if (ix->pending) HIPCHECK(hipStreamWaitEvent(st, ix->done, 0));
    Work w = carve(ix, ix->arena, C, B, k, 1, scores != nullptr, nullptr);
    for (int64_t c0 = 0; c0 < nq; c0 += (int64_t)C) {
        const int cn = (int)std::min<int64_t>((int64_t)C, nq - c0);
        QueryPass qp{};
        qp.ix = ix->view();
        qp.nq = cn;
        qp.B = B;
        qp.runs_per_sub = runs_per_sub(ix->ns);
        qp.tgroups = tile_groups(qp.nq, ix->P);
        qp.k = k;
        qp.cells = const_cast<uint16_t *>(cells) + c0 * ix->ns * ix->K;
        qp.ncells = const_cast<int32_t *>(ncells) + c0 * ix->ns;
        qp.hist = w.hist; qp.lvl = w.lvl; qp.scores = w.scores;
        qp.cand = reinterpret_cast<uint32_t *>(cand) + c0 * B;
        qp.aprime = w.aprime;
        qp.route = ix->sp_cap ? w.route : nullptr;
        qp.tlist = qp.route ? w.route + C : nullptr;
        qp.ntl = qp.route ? w.route + 2 * C : nullptr;
        qp.sp_cap = ix->sp_cap;
        if (qp.route) {
            // the sparse step reads the activated points per subspace
            SizesPass sp{qp.ix, qp.cells, qp.ncells, cn, w.aprime, qp.ntl};
            HIPCHECK(launch(plan_cell_points(sp), &sp, st));
            HIPCHECK(timed(ix, kCollideSparse, st, [&] { return launch(plan_collide_sparse(qp, 0), &qp, st); }));
        }
        HIPCHECK(timed(ix, kCollide, st, [&] { return launch_collide(qp, st); }));
        HIPCHECK(timed(ix, kSelect, st, [&] { return launch_select(qp, st); }));
        if (scores)
            HIPCHECK(hipMemcpy2DAsync(scores + c0 * ix->n, (size_t)ix->n, w.scores, (size_t)ix->P * ix->TILE,
                                      (size_t)ix->n, (size_t)cn, hipMemcpyDeviceToDevice, st));
    }
    HIPCHECK(hipEventRecord(ix->done, st));
    ix->pending = true;
    return SUCO_OK;
}

int suco_rerank(const suco_index *cix, const float *Q, int64_t nq, const int32_t *cand, int64_t B, int32_t k,
                int32_t *ids, float *dists, void *stream) {
    int rc = check_query(cix, Q, nq, k, 1.0, ids, dists);
    if (rc) return rc;
    if (B < k || B > cix->n) return fail(SUCO_E_INVAL, "B must be in [k, n]");
    if (nq > 0 && !cand) return fail(SUCO_E_INVAL, "cand must not be NULL");
    if (nq == 0) return SUCO_OK;
    suco_index *ix = const_cast<suco_index *>(cix);
    hipStream_t st = (hipStream_t)stream;
    RerankCfg c;
    if ((rc = rerank_cfg(ix->d, B, &c))) return rc;
    std::lock_guard<std::mutex> lock(ix->mu);
    DeviceGuard dg(ix->device);
    const size_t C = (size_t)pass_size(nq, ix->chunk);
    size_t bytes = 0;
    carve(ix, nullptr, C, B, k, c.parts, false, &bytes);
    if ((rc = ensure_arena(ix, bytes))) return rc;
    if (ix->pending) HIPCHECK(hipStreamWaitEvent(st, ix->done, 0));
    Work w = carve(ix, ix->arena, C, B, k, c.parts, false, nullptr);
    for (int64_t c0 = 0; c0 < nq; c0 += (int64_t)C) {
        const int cn = (int)std::min<int64_t>((int64_t)C, nq - c0);
        RerankPass rp{};
        rp.X = ix->X; rp.X8 = ix->X8; rp.Q = Q + c0 * ix->d; rp.cand = reinterpret_cast<const uint32_t *>(cand) + c0 * B;
        rp.metric = ix->metric;
        rp.B = B; rp.n = ix->n; rp.d = ix->d; rp.k = k; rp.nq = cn; rp.parts = c.parts; rp.rows_per_part = c.rpp;
        rp.G = c.G; rp.U = c.U; rp.part_keys = w.part_keys; rp.ids = ids + c0 * k; rp.dists = dists + c0 * k;
        HIPCHECK(timed(ix, kRerank, st, [&] { return launch_rerank(rp, st); }));
        HIPCHECK(timed(ix, kMerge, st, [&] { return launch_merge(rp, st); }));
    }
    HIPCHECK(hipEventRecord(ix->done, st));
    ix->pending = true;
    return SUCO_OK;
}

int suco_profile(suco_index *ix, int enable) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    std::lock_guard<std::mutex> lock(ix->mu);
    ix->prof_on = enable != 0;
    return SUCO_OK;
}

int suco_profile_read(suco_index *ix, double *ms, int64_t *launches) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (!ms || !launches) return fail(SUCO_E_INVAL, "ms and launches must not be NULL");
    std::lock_guard<std::mutex> lock(ix->mu);
    DeviceGuard dg(ix->device);
    for (int j = 0; j < kStages; ++j) { ms[j] = 0.0; launches[j] = 0; }
    for (size_t t = 0; t < ix->prof_used; ++t) {
        auto &e = ix->prof_pool[t];
        HIPCHECK(hipEventSynchronize(e.b));
        float m = 0.f;
        HIPCHECK(hipEventElapsedTime(&m, e.a, e.b));
        ms[e.stage] += m;
        launches[e.stage] += 1;
    }
    ix->prof_used = 0;
    return SUCO_OK;
}

}  // extern "C"
