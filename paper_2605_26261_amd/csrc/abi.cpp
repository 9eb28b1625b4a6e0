// C ABI of libftlm (declared in include/ftlm.h): argument checking, handles,
// table layout and kernel launches. No device memory is allocated here; all
// device buffers come from the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ftlm.h"
#include "host_math.hpp"
#include "kernels.hpp"

using namespace ftlm;

struct ftlm_graph {
    int n_sites = 0;
    std::vector<int> bi, bj;   // merged bonds, caller order of first appearance
    std::vector<double> J;
    int n_input = 0;               // bonds as given (before merging)
    std::vector<int> merged_of_input;
    BondTable table{};
};

struct ftlm_sector {
    int n_sites = 0, n_up = 0, mode = 0;
    uint64_t dim = 0;
    void* table = nullptr;
    size_t bytes = 0;
    TableLayout layout{};
    std::vector<uint32_t> binom_host;
    SectorDev dev{};
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return FTLM_OK;
}

#define HIP_CHECK(expr)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(FTLM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

uint64_t binom_u64(int n, int k) {
    if (n < 0 || k < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    unsigned __int128 c = 1;
    for (int i = 1; i <= k; ++i) c = c * unsigned(n - k + i) / unsigned(i);
    return uint64_t(c);
}

// ---- start-vector keys: SplitMix64 (Steele, Lea, Flood 2014) --------------
constexpr uint64_t kGammaHost = 0x9e3779b97f4a7c15ull;
uint64_t mix64_host(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
uint64_t first_output(uint64_t s) { return mix64_host(s + kGammaHost); }
// Key of sample r in the sector with n_up up spins.
uint64_t stream_key(uint64_t seed, int n_up, uint64_t r) {
    uint64_t k = first_output(seed);
    k = first_output(k ^ uint64_t(uint32_t(n_up)));
    return first_output(k ^ r);
}

// ---- stats -------------------------------------------------------------------
struct Stats {
    std::mutex mu;
    bool on = false;
    int64_t launches = 0;
    double ms = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
} g_stats;

struct HvTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    explicit HvTimer(hipStream_t s) : st(s) {
        std::lock_guard<std::mutex> lk(g_stats.mu);
        if (!g_stats.on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        (void)hipEventRecord(a, st);
    }
    ~HvTimer() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> lk(g_stats.mu);
        g_stats.pending.emplace_back(a, b);
    }
};

// ---- column chunking of a [D][ld] block --------------------------------------
// Splits columns [0, nvec) into kernel widths, widest first, keeping every
// vector access naturally aligned (ld, col0 and the base pointers).
std::vector<std::pair<int, int>> column_chunks(int nvec, uint64_t ld, int dtype,
                                               std::initializer_list<const void*> ptrs) {
    const size_t es = dtype == FTLM_F32 ? 4 : 8;
    static const int w32[] = {32, 20, 16, 8, 4, 2, 1};
    static const int w64[] = {16, 8, 4, 2, 1};
    const int* widths = dtype == FTLM_F32 ? w32 : w64;
    const int nw = dtype == FTLM_F32 ? 7 : 5;
    std::vector<std::pair<int, int>> out;
    int col = 0;
    while (col < nvec) {
        for (int i = 0; i < nw; ++i) {
            const int vb = widths[i];
            if (vb > nvec - col) continue;
            size_t vbytes = es;
            if (es == 4 && vb % 4 == 0) vbytes = 16;
            else if (vb % 2 == 0) vbytes = 2 * es;
            bool aligned = (ld * es) % vbytes == 0 && (size_t(col) * es) % vbytes == 0;
            for (const void* p : ptrs) aligned = aligned && (reinterpret_cast<uintptr_t>(p) % vbytes == 0);
            if (!aligned) continue;
            out.emplace_back(col, vb);
            col += vb;
            break;
        }
    }
    return out;
}

int check_dtype(int dtype) {
    if (dtype != FTLM_F32 && dtype != FTLM_F64) return fail(FTLM_E_INVALID, "dtype %d is not FTLM_F32/FTLM_F64", dtype);
    return FTLM_OK;
}

// ---- Lanczos workspace layout -------------------------------------------------
constexpr int kMaxSteps = 4096;
constexpr int kMaxChains = 64;
constexpr int kTickets = 64;

struct WorkLayout {
    size_t u0, u1, partials, chains, alpha, beta, tickets, total;
};

WorkLayout work_layout(uint64_t dim, int R, int dtype) {
    const size_t es = dtype == FTLM_F32 ? 4 : 8;
    WorkLayout w{};
    size_t off = 0;
    w.u0 = off; off = align256(off + size_t(dim) * size_t(R) * es);
    w.u1 = off; off = align256(off + size_t(dim) * size_t(R) * es);
    w.partials = off; off = align256(off + size_t(rows_grid(uint32_t(dim))) * size_t(R) * sizeof(double));
    w.chains = off; off = align256(off + size_t(R) * sizeof(Chain));
    w.alpha = off; off = align256(off + size_t(R) * kMaxSteps * sizeof(double));
    w.beta = off; off = align256(off + size_t(R) * kMaxSteps * sizeof(double));
    w.tickets = off; off = align256(off + kTickets * sizeof(uint32_t));
    w.total = off;
    return w;
}

template <typename P>
P* at(void* base, size_t off) { return reinterpret_cast<P*>(static_cast<char*>(base) + off); }

}  // namespace

extern "C" {

const char* ftlm_last_error(void) { return g_err.c_str(); }

int ftlm_version(void) { return 1; }

// ---- graph ---------------------------------------------------------------------
int ftlm_graph_create(int n_sites, int n_bonds, const int32_t* bi, const int32_t* bj, const double* J,
                      ftlm_graph** out) {
    if (!out || !bi || !bj || !J) return fail(FTLM_E_INVALID, "null argument");
    *out = nullptr;
    if (n_sites < 2 || n_sites > kMaxSites) return fail(FTLM_E_RANGE, "n_sites %d not in [2, %d]", n_sites, kMaxSites);
    if (n_bonds < 1 || n_bonds > kMaxBonds) return fail(FTLM_E_RANGE, "n_bonds %d not in [1, %d]", n_bonds, kMaxBonds);
    ftlm_graph* g = new ftlm_graph();
    g->n_sites = n_sites;
    g->n_input = n_bonds;
    std::map<std::pair<int, int>, int> seen;
    for (int b = 0; b < n_bonds; ++b) {
        int i = bi[b], j = bj[b];
        if (i < 0 || j < 0 || i >= n_sites || j >= n_sites || i == j || !std::isfinite(J[b])) {
            delete g;
            return fail(FTLM_E_INVALID, "bond %d = (%d, %d, %g) is not a pair of distinct sites in [0, %d)", b, i, j,
                        J[b], n_sites);
        }
        if (i > j) std::swap(i, j);
        auto it = seen.find({i, j});
        if (it == seen.end()) {
            seen[{i, j}] = int(g->bi.size());
            g->merged_of_input.push_back(int(g->bi.size()));
            g->bi.push_back(i);
            g->bj.push_back(j);
            g->J.push_back(J[b]);
        } else {
            g->merged_of_input.push_back(it->second);
            g->J[size_t(it->second)] += J[b];
        }
    }
    // Kernel bond table: sorted by the lower site, highest first.
    const int nb = int(g->bi.size());
    std::vector<int> order(static_cast<size_t>(nb));
    for (int b = 0; b < nb; ++b) order[size_t(b)] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        if (g->bi[size_t(a)] != g->bi[size_t(c)]) return g->bi[size_t(a)] > g->bi[size_t(c)];
        return g->bj[size_t(a)] > g->bj[size_t(c)];
    });
    BondTable& T = g->table;
    std::memset(&T, 0, sizeof(T));
    T.n_bonds = nb;
    T.n_sites = n_sites;
    double jsum = 0.0;
    for (int s = 0; s < nb; ++s) {
        const int b = order[size_t(s)];
        T.pack[s] = uint32_t(g->bi[size_t(b)]) | (uint32_t(g->bj[size_t(b)]) << 8) | (uint32_t(b) << 16);
        T.coef_d[s] = 0.5 * g->J[size_t(b)];
        T.coef_f[s] = float(0.5 * g->J[size_t(b)]);
        jsum += g->J[size_t(b)];
    }
    for (int p = 0; p <= kMaxSites; ++p) {
        int c = 0;
        for (int s = 0; s < nb; ++s) c += (int(T.pack[s] & 0xffu) >= p) ? 1 : 0;
        T.ends[p] = uint32_t(p < n_sites ? c : 0);
    }
    T.jsum4_d = 0.25 * jsum;
    T.jsum4_f = float(0.25 * jsum);
    *out = g;
    return ok();
}

void ftlm_graph_destroy(ftlm_graph* g) { delete g; }
int ftlm_graph_n_sites(const ftlm_graph* g) { return g ? g->n_sites : 0; }
int ftlm_graph_n_bonds(const ftlm_graph* g) { return g ? int(g->bi.size()) : 0; }

// ---- sector ---------------------------------------------------------------------
int ftlm_sector_table_bytes(int n_sites, int n_up, int mode, size_t* bytes) {
    if (!bytes) return fail(FTLM_E_INVALID, "null argument");
    if (mode != FTLM_CLT && mode != FTLM_CR) return fail(FTLM_E_INVALID, "mode %d is not FTLM_CLT/FTLM_CR", mode);
    if (n_sites < 1 || n_sites > kMaxSites) return fail(FTLM_E_RANGE, "n_sites %d not in [1, %d]", n_sites, kMaxSites);
    if (n_up < 0 || n_up > n_sites) return fail(FTLM_E_INVALID, "n_up %d not in [0, %d]", n_up, n_sites);
    if (mode == FTLM_CLT && n_sites > kMaxCltSites)
        return fail(FTLM_E_RANGE, "FTLM_CLT holds uint32 labels: n_sites %d > %d", n_sites, kMaxCltSites);
    const uint64_t dim = binom_u64(n_sites, n_up);
    if (dim >= (uint64_t(1) << 32)) return fail(FTLM_E_RANGE, "sector dimension %llu >= 2^32", (unsigned long long)dim);
    *bytes = table_layout(n_sites, n_up, mode, dim).total;
    return ok();
}

int ftlm_sector_create(int n_sites, int n_up, int mode, void* table_dev, size_t bytes, void* stream,
                       ftlm_sector** out) {
    if (!out || !table_dev) return fail(FTLM_E_INVALID, "null argument");
    *out = nullptr;
    size_t need = 0;
    int rc = ftlm_sector_table_bytes(n_sites, n_up, mode, &need);
    if (rc) return rc;
    if (bytes < need) return fail(FTLM_E_NOSPACE, "table buffer holds %zu bytes, %zu needed", bytes, need);
    if (reinterpret_cast<uintptr_t>(table_dev) % 256 != 0) return fail(FTLM_E_INVALID, "table buffer not 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    ftlm_sector* s = new ftlm_sector();
    s->n_sites = n_sites;
    s->n_up = n_up;
    s->mode = mode;
    s->dim = binom_u64(n_sites, n_up);
    s->table = table_dev;
    s->bytes = bytes;
    s->layout = table_layout(n_sites, n_up, mode, s->dim);
    const int w = binom_width(n_up);
    s->binom_host.assign(size_t(n_sites) * size_t(w), 0u);
    for (int p = 0; p < n_sites; ++p)
        for (int k = -1; k <= n_up + 1; ++k)
            s->binom_host[size_t(p) * size_t(w) + size_t(k + 1)] = uint32_t(binom_u64(p, k));
    SectorDev& d = s->dev;
    d.n_sites = n_sites;
    d.n_up = n_up;
    d.mode = mode;
    d.bw = w;
    d.dim = uint32_t(s->dim);
    d.binom = at<uint32_t>(table_dev, s->layout.binom_off);
    d.basis = mode == FTLM_CLT ? at<uint32_t>(table_dev, s->layout.basis_off) : nullptr;
    d.clt = mode == FTLM_CLT ? at<CltEntry>(table_dev, s->layout.clt_off) : nullptr;
    hipError_t e = hipMemcpyAsync(const_cast<uint32_t*>(d.binom), s->binom_host.data(),
                                  s->binom_host.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host copy may be reused at once
    if (e == hipSuccess && mode == FTLM_CLT) {
        e = launch_build_basis(d, st);
        if (e == hipSuccess) e = launch_build_clt(d, st);
    }
    if (e != hipSuccess) {
        delete s;
        return fail(FTLM_E_DEVICE, "sector build: %s", hipGetErrorString(e));
    }
    *out = s;
    return ok();
}

uint64_t ftlm_sector_dim(const ftlm_sector* s) { return s ? s->dim : 0; }
int ftlm_sector_mode(const ftlm_sector* s) { return s ? s->mode : -1; }
void ftlm_sector_destroy(ftlm_sector* s) { delete s; }

int ftlm_rank(const ftlm_sector* s, const uint64_t* labels_dev, uint64_t* idx_dev, uint64_t n, void* stream) {
    if (!s || (n && (!labels_dev || !idx_dev))) return fail(FTLM_E_INVALID, "null argument");
    if (n == 0) return ok();
    HIP_CHECK(launch_rank(s->dev, labels_dev, idx_dev, n, static_cast<hipStream_t>(stream)));
    return ok();
}

int ftlm_unrank(const ftlm_sector* s, const uint64_t* idx_dev, uint64_t* labels_dev, uint64_t n, void* stream) {
    if (!s || (n && (!labels_dev || !idx_dev))) return fail(FTLM_E_INVALID, "null argument");
    if (n == 0) return ok();
    HIP_CHECK(launch_unrank(s->dev, idx_dev, labels_dev, n, static_cast<hipStream_t>(stream)));
    return ok();
}

int ftlm_clt_export(const ftlm_sector* s, uint32_t* mask_host, uint32_t* prefix_host, uint64_t nblocks,
                    void* stream) {
    if (!s || !mask_host || !prefix_host) return fail(FTLM_E_INVALID, "null argument");
    if (s->mode != FTLM_CLT) return fail(FTLM_E_INVALID, "sector is not in FTLM_CLT mode");
    if (nblocks > clt_blocks(s->n_sites)) return fail(FTLM_E_RANGE, "nblocks %llu > %llu", (unsigned long long)nblocks,
                                                     (unsigned long long)clt_blocks(s->n_sites));
    std::vector<CltEntry> tmp(static_cast<size_t>(nblocks));
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_CHECK(hipMemcpyAsync(tmp.data(), s->dev.clt, size_t(nblocks) * sizeof(CltEntry), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (size_t b = 0; b < tmp.size(); ++b) {
        mask_host[b] = tmp[b].mask;
        prefix_host[b] = tmp[b].prefix;
    }
    return ok();
}

int ftlm_neighbors(const ftlm_sector* s, const ftlm_graph* g, uint64_t t0, uint64_t count, uint64_t* idx_dev,
                   void* stream) {
    if (!s || !g || (count && !idx_dev)) return fail(FTLM_E_INVALID, "null argument");
    if (g->n_sites != s->n_sites) return fail(FTLM_E_INVALID, "graph has %d sites, sector %d", g->n_sites, s->n_sites);
    if (t0 > s->dim || count > s->dim - t0) return fail(FTLM_E_RANGE, "rows [%llu, +%llu) outside the sector",
                                                        (unsigned long long)t0, (unsigned long long)count);
    if (count == 0) return ok();
    HIP_CHECK(launch_neighbors(s->dev, g->table, t0, count, idx_dev, static_cast<hipStream_t>(stream)));
    return ok();
}

// ---- H.x -----------------------------------------------------------------------
int ftlm_hv_rows(const ftlm_sector* s, const ftlm_graph* g, const void* x_dev, void* y_dev, int nvec, int dtype,
                 uint64_t row0, uint64_t nrows, void* stream) {
    if (!s || !g || !x_dev || !y_dev) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_dtype(dtype)) return rc;
    if (g->n_sites != s->n_sites) return fail(FTLM_E_INVALID, "graph has %d sites, sector %d", g->n_sites, s->n_sites);
    if (nvec < 1 || nvec > 64) return fail(FTLM_E_RANGE, "nvec %d not in [1, 64]", nvec);
    if (row0 > s->dim || nrows > s->dim - row0) return fail(FTLM_E_RANGE, "rows outside the sector");
    if (nrows == 0) return ok();
    const size_t es = dtype == FTLM_F32 ? 4 : 8;
    const char* xb = static_cast<const char*>(x_dev);
    const char* yb = static_cast<const char*>(y_dev);
    if (xb < yb + nrows * nvec * es && yb < xb + s->dim * nvec * es) return fail(FTLM_E_INVALID, "x and y overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HvLaunch h{};
    h.x = x_dev;
    h.y = y_dev;
    h.ld = uint64_t(nvec);
    h.row0 = uint32_t(row0);
    h.nrows = uint32_t(nrows);
    h.dtype = dtype;
    h.epi = kEpiPlain;
    h.grid = rows_grid(uint32_t(nrows));
    for (auto [col, vb] : column_chunks(nvec, uint64_t(nvec), dtype, {x_dev, y_dev})) {
        h.col0 = uint32_t(col);
        h.vb = vb;
        HvTimer timer(st);
        HIP_CHECK(launch_hv(s->dev, g->table, h, st));
    }
    return ok();
}

int ftlm_hv(const ftlm_sector* s, const ftlm_graph* g, const void* x_dev, void* y_dev, int nvec, int dtype,
            void* stream) {
    if (!s) return fail(FTLM_E_INVALID, "null argument");
    return ftlm_hv_rows(s, g, x_dev, y_dev, nvec, dtype, 0, s->dim, stream);
}

// ---- start vectors and Lanczos ----------------------------------------------------
int ftlm_lanczos_workspace_bytes(const ftlm_sector* s, int R, int dtype, size_t* bytes) {
    if (!s || !bytes) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_dtype(dtype)) return rc;
    if (R < 1 || R > kMaxChains) return fail(FTLM_E_RANGE, "R %d not in [1, %d]", R, kMaxChains);
    *bytes = work_layout(s->dim, R, dtype).total;
    return ok();
}

namespace {

int enqueue_start(const ftlm_sector* s, uint64_t seed, uint64_t r0, int R, int dist, int dtype, void* q,
                  void* work, const WorkLayout& wl, hipStream_t st) {
    StartLaunch a{};
    a.q = q;
    a.ld = uint64_t(R);
    a.col0 = 0;
    a.ncols = R;
    a.dtype = dtype;
    a.dist = dist;
    for (int c = 0; c < R; ++c) {
        a.keys[c] = stream_key(seed, s->n_up, r0 + uint64_t(c));
        a.sample[c] = r0 + uint64_t(c);
    }
    a.grid = rows_grid(uint32_t(s->dim));
    a.pstride = R;
    a.chains = at<Chain>(work, wl.chains);
    a.partials = at<double>(work, wl.partials);
    a.ticket = at<uint32_t>(work, wl.tickets);
    HIP_CHECK(launch_chain_init(a.chains, R, a.ticket, kTickets, st));
    HIP_CHECK(launch_start(s->dev, a, st));
    return FTLM_OK;
}

int check_lanczos_args(const ftlm_sector* s, int R, int dist, int dtype, void* work, size_t work_bytes) {
    if (!s || !work) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_dtype(dtype)) return rc;
    if (dist != FTLM_PM1 && dist != FTLM_GAUSS && dist != FTLM_UNIT) return fail(FTLM_E_INVALID, "bad dist %d", dist);
    if (R < 1 || R > kMaxChains) return fail(FTLM_E_RANGE, "R %d not in [1, %d]", R, kMaxChains);
    const size_t need = work_layout(s->dim, R, dtype).total;
    if (work_bytes < need) return fail(FTLM_E_NOSPACE, "workspace holds %zu bytes, %zu needed", work_bytes, need);
    if (reinterpret_cast<uintptr_t>(work) % 256 != 0) return fail(FTLM_E_INVALID, "workspace not 256-byte aligned");
    return FTLM_OK;
}

}  // namespace

int ftlm_start_vectors(const ftlm_sector* s, uint64_t seed, uint64_t r0, int R, int dist, int dtype, void* q_dev,
                       double* norms_host, void* work_dev, size_t work_bytes, void* stream) {
    if (int rc = check_lanczos_args(s, R, dist, dtype, work_dev, work_bytes)) return rc;
    if (!q_dev || !norms_host) return fail(FTLM_E_INVALID, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const WorkLayout wl = work_layout(s->dim, R, dtype);
    if (int rc = enqueue_start(s, seed, r0, R, dist, dtype, q_dev, work_dev, wl, st)) return rc;
    std::vector<Chain> ch(static_cast<size_t>(R));
    HIP_CHECK(hipMemcpyAsync(ch.data(), at<Chain>(work_dev, wl.chains), size_t(R) * sizeof(Chain),
                             hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (int c = 0; c < R; ++c) norms_host[c] = ch[size_t(c)].norm;
    return ok();
}

int ftlm_lanczos(const ftlm_sector* s, const ftlm_graph* g, uint64_t seed, uint64_t r0, int R, int M, int dist,
                 int dtype, void* work_dev, size_t work_bytes, double* alpha_host, double* beta_host,
                 int32_t* steps_host, void* stream) {
    if (int rc = check_lanczos_args(s, R, dist, dtype, work_dev, work_bytes)) return rc;
    if (!g || !alpha_host || !beta_host || !steps_host) return fail(FTLM_E_INVALID, "null argument");
    if (g->n_sites != s->n_sites) return fail(FTLM_E_INVALID, "graph has %d sites, sector %d", g->n_sites, s->n_sites);
    if (M < 1 || M > kMaxSteps) return fail(FTLM_E_RANGE, "M %d not in [1, %d]", M, kMaxSteps);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const WorkLayout wl = work_layout(s->dim, R, dtype);
    void* U[2] = {at<void>(work_dev, wl.u0), at<void>(work_dev, wl.u1)};
    if (int rc = enqueue_start(s, seed, r0, R, dist, dtype, U[0], work_dev, wl, st)) return rc;
    const int m_eff = int(std::min<uint64_t>(uint64_t(M), s->dim));
    const int grid = rows_grid(uint32_t(s->dim));
    const auto chunks = column_chunks(R, uint64_t(R), dtype, {U[0], U[1]});
    HvLaunch h{};
    h.ld = uint64_t(R);
    h.row0 = 0;
    h.nrows = uint32_t(s->dim);
    h.dtype = dtype;
    h.epi = kEpiLanczos;
    h.pstride = R;
    h.grid = grid;
    h.chains = at<Chain>(work_dev, wl.chains);
    h.partials = at<double>(work_dev, wl.partials);
    h.ticket = at<uint32_t>(work_dev, wl.tickets);
    UpdateLaunch u{};
    u.ld = uint64_t(R);
    u.dtype = dtype;
    u.grid = grid;
    u.pstride = R;
    u.m_eff = m_eff;
    u.eps = dtype == FTLM_F32 ? 1e-6 : 1e-12;
    u.M = kMaxSteps;
    u.chains = h.chains;
    u.partials = h.partials;
    u.ticket = h.ticket;
    u.alpha = at<double>(work_dev, wl.alpha);
    u.beta = at<double>(work_dev, wl.beta);
    for (int k = 1; k <= m_eff; ++k) {
        void* cur = U[(k - 1) & 1];
        void* prev = U[k & 1];
        h.x = cur;
        h.y = prev;
        h.first = k == 1 ? 1 : 0;
        u.u = cur;
        u.w = prev;
        u.step = k;
        for (auto [col, vb] : chunks) {
            h.col0 = uint32_t(col);
            h.vb = vb;
            {
                HvTimer timer(st);
                HIP_CHECK(launch_hv(s->dev, g->table, h, st));
            }
            u.col0 = uint32_t(col);
            u.ncols = vb;
            HIP_CHECK(launch_update(s->dev, u, st));
        }
    }
    std::vector<double> a(size_t(R) * kMaxSteps), b(size_t(R) * kMaxSteps);
    std::vector<Chain> ch(static_cast<size_t>(R));
    HIP_CHECK(hipMemcpyAsync(a.data(), u.alpha, a.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(b.data(), u.beta, b.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(ch.data(), h.chains, ch.size() * sizeof(Chain), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (int r = 0; r < R; ++r) {
        steps_host[r] = ch[size_t(r)].steps;
        for (int k = 0; k < M; ++k) {
            const bool in = k < ch[size_t(r)].steps;
            alpha_host[size_t(r) * M + size_t(k)] = in ? a[size_t(r) * kMaxSteps + size_t(k)] : 0.0;
            beta_host[size_t(r) * M + size_t(k)] = in ? b[size_t(r) * kMaxSteps + size_t(k)] : 0.0;
        }
    }
    return ok();
}

// ---- host FP64 -------------------------------------------------------------------
int ftlm_ritz(int m, const double* alpha, const double* beta, double* theta, double* weight) {
    if (m < 1 || !alpha || !theta || !weight || (m > 1 && !beta)) return fail(FTLM_E_INVALID, "bad argument");
    if (ritz_ql(m, alpha, beta, theta, weight) != 0) return fail(FTLM_E_INVALID, "QL iteration did not converge");
    return ok();
}

int ftlm_thermo(int n_sites, int n_sectors, const ftlm_sector_result* sectors, int nT, const double* T, double g,
                double* E, double* C, double* chi, double* lnZ) {
    if (n_sectors < 1 || !sectors || nT < 0 || (nT && !T)) return fail(FTLM_E_INVALID, "bad argument");
    std::vector<SectorSamples> v(static_cast<size_t>(n_sectors));
    for (int i = 0; i < n_sectors; ++i) {
        const ftlm_sector_result& r = sectors[i];
        if (r.R < 1 || !r.theta || !r.weight || !r.steps || r.stride < 1) return fail(FTLM_E_INVALID, "sector %d malformed", i);
        for (int k = 0; k < r.R; ++k)
            if (r.steps[k] < 1 || r.steps[k] > r.stride) return fail(FTLM_E_INVALID, "sector %d sample %d steps", i, k);
        v[size_t(i)] = SectorSamples{r.n_up, r.R, r.stride, r.dim, r.mult, r.theta, r.weight, r.steps};
    }
    for (int i = 0; i < nT; ++i)
        if (!(T[i] > 0.0)) return fail(FTLM_E_INVALID, "temperature %d not positive", i);
    if (thermo(n_sites, n_sectors, v.data(), nT, T, g, E, C, chi, lnZ) != 0) return fail(FTLM_E_INVALID, "no samples");
    return ok();
}

// ---- measurement hooks --------------------------------------------------------------
int ftlm_stats_enable(int on) {
    std::lock_guard<std::mutex> lk(g_stats.mu);
    g_stats.on = on != 0;
    return ok();
}

int ftlm_stats_reset(void) {
    std::lock_guard<std::mutex> lk(g_stats.mu);
    for (auto& p : g_stats.pending) {
        (void)hipEventSynchronize(p.second);
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    g_stats.pending.clear();
    g_stats.launches = 0;
    g_stats.ms = 0.0;
    return ok();
}

int ftlm_stats_read(int64_t* hv_launches, double* hv_ms) {
    std::lock_guard<std::mutex> lk(g_stats.mu);
    for (auto& p : g_stats.pending) {
        if (hipEventSynchronize(p.second) != hipSuccess) return fail(FTLM_E_DEVICE, "event sync failed");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.first, p.second);
        g_stats.ms += double(ms);
        g_stats.launches += 1;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    g_stats.pending.clear();
    if (hv_launches) *hv_launches = g_stats.launches;
    if (hv_ms) *hv_ms = g_stats.ms;
    return ok();
}

}  // extern "C"
