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
std::vector<std::pair<int, int>> column_chunks_v(int nvec, uint64_t ld, int dtype, const std::vector<const void*>& ptrs) {
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

std::vector<std::pair<int, int>> column_chunks(int nvec, uint64_t ld, int dtype,
                                               std::initializer_list<const void*> ptrs) {
    return column_chunks_v(nvec, ld, dtype, std::vector<const void*>(ptrs));
}

int check_dtype(int dtype) {
    if (dtype != FTLM_F32 && dtype != FTLM_F64) return fail(FTLM_E_INVALID, "dtype %d is not FTLM_F32/FTLM_F64", dtype);
    return FTLM_OK;
}

// ---- Lanczos state layout -----------------------------------------------------
constexpr int kTicketsPerSector = 1;

// Byte offsets of one sector's Lanczos state inside a workspace or arena.
struct SectorState {
    size_t u0, u1, partials, chains, alpha, beta, ticket, keys;
};

// Lays out the state of a sector of dimension `dim` at `off`; returns the end.
size_t layout_state(uint64_t dim, int R, int dtype, size_t off, SectorState& st) {
    const size_t es = dtype == FTLM_F32 ? 4 : 8;
    st.u0 = off; off = align256(off + size_t(dim) * size_t(R) * es);
    st.u1 = off; off = align256(off + size_t(dim) * size_t(R) * es);
    st.partials = off; off = align256(off + size_t(rows_grid(uint32_t(dim))) * size_t(R) * sizeof(double));
    st.chains = off; off = align256(off + size_t(R) * sizeof(Chain));
    st.alpha = off; off = align256(off + size_t(R) * kMaxSteps * sizeof(double));
    st.beta = off; off = align256(off + size_t(R) * kMaxSteps * sizeof(double));
    st.ticket = off; off = align256(off + kTicketsPerSector * sizeof(uint32_t));
    st.keys = off; off = align256(off + size_t(R) * sizeof(uint64_t));
    return off;
}

template <typename P>
P* at(void* base, size_t off) { return reinterpret_cast<P*>(static_cast<char*>(base) + off); }

// A batch of R chains in each of a list of sectors (one sector for
// ftlm_lanczos, all sectors of a plan), with the device descriptors of the
// multi-sector Lanczos kernels. Host copies stay alive until the stream work
// that reads them has been synchronized.
struct LanczosJob {
    int nsec = 0, R = 0, dtype = 0, mode = 0, n_sites = 0, grid = 0;
    size_t lds = 0;
    std::vector<SecWork> secs;           // host copies of the descriptors
    std::vector<uint64_t> keys;          // [nsec][R] stream keys of the run
    SecWork* dev_secs = nullptr;
    uint64_t* dev_keys = nullptr;        // first sector's key block; sector s at dev_keys_of[s]
    std::vector<uint64_t*> key_ptrs;
    std::vector<std::pair<int, int>> chunks;
    int max_steps = 0;                   // largest m_eff over the sectors

    LanczosLaunch launch() const {
        LanczosLaunch a{};
        a.secs = dev_secs;
        a.nsec = nsec;
        a.grid = grid;
        a.ld = uint64_t(R);
        a.dtype = dtype;
        a.eps = dtype == FTLM_F32 ? 1e-6 : 1e-12;
        a.mode = mode;
        a.n_sites = n_sites;
        return a;
    }
};

// Fills job.secs for sectors whose tables are described by `devs` and whose
// state sits at `states` inside `base`; the descriptor array goes to
// `dev_secs` (device). Blocks: each sector gets rows_grid(D) blocks starting
// at a multiple of 8.
void job_layout(LanczosJob& job, const std::vector<SectorDev>& devs, const std::vector<SectorState>& states,
                void* base, int R, int M, int dtype, SecWork* dev_secs) {
    job.nsec = int(devs.size());
    job.R = R;
    job.dtype = dtype;
    job.mode = devs[0].mode;
    job.n_sites = devs[0].n_sites;
    job.dev_secs = dev_secs;
    job.secs.assign(devs.size(), SecWork{});
    job.key_ptrs.clear();
    uint32_t block = 0;
    size_t lds = 0;
    job.max_steps = 0;
    for (size_t i = 0; i < devs.size(); ++i) {
        SecWork& w = job.secs[i];
        const SectorState& st = states[i];
        w.S = devs[i];
        w.u[0] = at<void>(base, st.u0);
        w.u[1] = at<void>(base, st.u1);
        w.chains = at<Chain>(base, st.chains);
        w.partials = at<double>(base, st.partials);
        w.ticket = at<uint32_t>(base, st.ticket);
        w.alpha = at<double>(base, st.alpha);
        w.beta = at<double>(base, st.beta);
        w.keys = at<uint64_t>(base, st.keys);
        job.key_ptrs.push_back(at<uint64_t>(base, st.keys));
        w.G = rows_grid(devs[i].dim);
        w.block0 = block;
        block = (block + w.G + 7) & ~7u;
        w.m_eff = int(std::min<uint64_t>(uint64_t(M), devs[i].dim));
        job.max_steps = std::max(job.max_steps, w.m_eff);
        lds = std::max(lds, hv_lds_bytes(devs[i]));
    }
    job.grid = int(block);
    job.lds = lds;
    std::vector<const void*> ptrs;
    for (auto& w : job.secs) {
        ptrs.push_back(w.u[0]);
        ptrs.push_back(w.u[1]);
    }
    job.chunks = column_chunks_v(R, uint64_t(R), dtype, ptrs);
}

// Start vectors of samples r0 .. r0 + R - 1 in every sector of the job.
int job_start(LanczosJob& job, uint64_t seed, uint64_t r0, int dist, hipStream_t st) {
    job.keys.resize(size_t(job.nsec) * size_t(job.R));
    for (int s = 0; s < job.nsec; ++s) {
        job.secs[size_t(s)].r0 = r0;
        for (int c = 0; c < job.R; ++c)
            job.keys[size_t(s) * job.R + size_t(c)] = stream_key(seed, job.secs[size_t(s)].S.n_up, r0 + uint64_t(c));
    }
    HIP_CHECK(hipMemcpyAsync(job.dev_secs, job.secs.data(), job.secs.size() * sizeof(SecWork),
                             hipMemcpyHostToDevice, st));
    for (int s = 0; s < job.nsec; ++s)
        HIP_CHECK(hipMemcpyAsync(job.key_ptrs[size_t(s)], job.keys.data() + size_t(s) * job.R,
                                 size_t(job.R) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    LanczosLaunch a = job.launch();
    a.dist = dist;
    HIP_CHECK(launch_chain_init(a, st));
    for (int c = 0; c < job.R; c += 4) {
        a.col0 = uint32_t(c);
        a.vb = std::min(4, job.R - c);
        HIP_CHECK(launch_start(a, st));
    }
    return FTLM_OK;
}

// Lanczos steps 1..job.max_steps for every chunk of columns.
int job_steps(const LanczosJob& job, const BondTable& B, hipStream_t st, bool timed = true) {
    LanczosLaunch a = job.launch();
    for (int k = 1; k <= job.max_steps; ++k) {
        a.step = k;
        for (auto [col, vb] : job.chunks) {
            a.col0 = uint32_t(col);
            a.vb = vb;
            if (timed) {
                HvTimer timer(st);
                HIP_CHECK(launch_hv_lanczos(B, a, job.lds, st));
            } else {
                HIP_CHECK(launch_hv_lanczos(B, a, job.lds, st));
            }
            HIP_CHECK(launch_update(a, st));
        }
    }
    return FTLM_OK;
}

// Copies sector s's coefficients into [R][M] host arrays (after a sync).
int job_collect(const LanczosJob& job, int M, double* alpha_host, double* beta_host, int32_t* steps_host,
                hipStream_t st) {
    const size_t R = size_t(job.R);
    std::vector<double> a(size_t(job.nsec) * R * kMaxSteps), b(a.size());
    std::vector<Chain> ch(size_t(job.nsec) * R);
    for (int s = 0; s < job.nsec; ++s) {
        const SecWork& w = job.secs[size_t(s)];
        HIP_CHECK(hipMemcpyAsync(a.data() + size_t(s) * R * kMaxSteps, w.alpha, R * kMaxSteps * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipMemcpyAsync(b.data() + size_t(s) * R * kMaxSteps, w.beta, R * kMaxSteps * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipMemcpyAsync(ch.data() + size_t(s) * R, w.chains, R * sizeof(Chain), hipMemcpyDeviceToHost, st));
    }
    HIP_CHECK(hipStreamSynchronize(st));
    for (int s = 0; s < job.nsec; ++s) {
        for (size_t r = 0; r < R; ++r) {
            const Chain& c = ch[size_t(s) * R + r];
            const size_t row = size_t(s) * R + r;
            steps_host[row] = c.steps;
            for (int k = 0; k < M; ++k) {
                const bool in = k < c.steps;
                alpha_host[row * size_t(M) + size_t(k)] = in ? a[row * kMaxSteps + size_t(k)] : 0.0;
                beta_host[row * size_t(M) + size_t(k)] = in ? b[row * kMaxSteps + size_t(k)] : 0.0;
            }
        }
    }
    return FTLM_OK;
}

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
    h.grid = int(rows_grid(uint32_t(nrows)));
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
// Single-sector workspace: the sector's Lanczos state followed by its device
// descriptor.
namespace {

struct SingleLayout {
    SectorState st;
    size_t secs, total;
};

SingleLayout single_layout(uint64_t dim, int R, int dtype) {
    SingleLayout l{};
    size_t off = layout_state(dim, R, dtype, 0, l.st);
    l.secs = off;
    off = align256(off + sizeof(SecWork));
    l.total = off;
    return l;
}

int check_lanczos_args(const ftlm_sector* s, int R, int dist, int dtype, void* work, size_t work_bytes) {
    if (!s || !work) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_dtype(dtype)) return rc;
    if (dist != FTLM_PM1 && dist != FTLM_GAUSS && dist != FTLM_UNIT) return fail(FTLM_E_INVALID, "bad dist %d", dist);
    if (R < 1 || R > kMaxChains) return fail(FTLM_E_RANGE, "R %d not in [1, %d]", R, kMaxChains);
    const size_t need = single_layout(s->dim, R, dtype).total;
    if (work_bytes < need) return fail(FTLM_E_NOSPACE, "workspace holds %zu bytes, %zu needed", work_bytes, need);
    if (reinterpret_cast<uintptr_t>(work) % 256 != 0) return fail(FTLM_E_INVALID, "workspace not 256-byte aligned");
    return FTLM_OK;
}

void single_job(LanczosJob& job, const ftlm_sector* s, int R, int M, int dtype, void* work) {
    const SingleLayout l = single_layout(s->dim, R, dtype);
    job_layout(job, {s->dev}, {l.st}, work, R, M, dtype, at<SecWork>(work, l.secs));
}

}  // namespace

int ftlm_lanczos_workspace_bytes(const ftlm_sector* s, int R, int dtype, size_t* bytes) {
    if (!s || !bytes) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_dtype(dtype)) return rc;
    if (R < 1 || R > kMaxChains) return fail(FTLM_E_RANGE, "R %d not in [1, %d]", R, kMaxChains);
    *bytes = single_layout(s->dim, R, dtype).total;
    return ok();
}

int ftlm_start_vectors(const ftlm_sector* s, uint64_t seed, uint64_t r0, int R, int dist, int dtype, void* q_dev,
                       double* norms_host, void* work_dev, size_t work_bytes, void* stream) {
    if (int rc = check_lanczos_args(s, R, dist, dtype, work_dev, work_bytes)) return rc;
    if (!q_dev || !norms_host) return fail(FTLM_E_INVALID, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    LanczosJob job;
    single_job(job, s, R, 1, dtype, work_dev);
    job.secs[0].u[0] = q_dev;  // the start block goes to the caller's buffer
    if (int rc = job_start(job, seed, r0, dist, st)) return rc;
    std::vector<Chain> ch(static_cast<size_t>(R));
    HIP_CHECK(hipMemcpyAsync(ch.data(), job.secs[0].chains, size_t(R) * sizeof(Chain), hipMemcpyDeviceToHost, st));
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
    LanczosJob job;
    single_job(job, s, R, M, dtype, work_dev);
    if (int rc = job_start(job, seed, r0, dist, st)) return rc;
    if (int rc = job_steps(job, g->table, st)) return rc;
    if (int rc = job_collect(job, M, alpha_host, beta_host, steps_host, st)) return rc;
    return ok();
}

// ---- batched all-sector plans ------------------------------------------------------
}  // extern "C"

struct ftlm_plan {
    BondTable table{};
    int n_sites = 0, mode = 0, R = 0, M = 0, dtype = 0;
    std::vector<ftlm_sector*> sectors;
    LanczosJob job;
    hipStream_t stream = nullptr;
    hipEvent_t ready = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~ftlm_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ready) (void)hipEventDestroy(ready);
        if (stream) (void)hipStreamDestroy(stream);
        for (auto* s : sectors) delete s;
    }
};

namespace {

// Arena of a plan: the sector descriptors, then per sector its tables and its
// Lanczos state.
struct PlanLayout {
    size_t secs;
    std::vector<size_t> table;
    std::vector<size_t> table_bytes;
    std::vector<SectorState> state;
    size_t total;
};

int plan_layout(int n_sites, int n_sectors, const int32_t* n_ups, int mode, int R, int dtype, PlanLayout& L) {
    L = PlanLayout{};
    size_t off = 0;
    L.secs = off;
    off = align256(off + size_t(n_sectors) * sizeof(SecWork));
    for (int i = 0; i < n_sectors; ++i) {
        size_t tb = 0;
        if (int rc = ftlm_sector_table_bytes(n_sites, n_ups[i], mode, &tb)) return rc;
        L.table.push_back(off);
        L.table_bytes.push_back(tb);
        off = align256(off + tb);
        SectorState st{};
        off = layout_state(binom_u64(n_sites, n_ups[i]), R, dtype, off, st);
        L.state.push_back(st);
    }
    L.total = off;
    return FTLM_OK;
}

int check_plan_args(const ftlm_graph* g, int n_sectors, const int32_t* n_ups, int mode, int R, int dtype) {
    if (!g || !n_ups) return fail(FTLM_E_INVALID, "null argument");
    if (n_sectors < 1 || n_sectors > kMaxPlanSectors)
        return fail(FTLM_E_RANGE, "n_sectors %d not in [1, %d]", n_sectors, kMaxPlanSectors);
    if (int rc = check_dtype(dtype)) return rc;
    if (R < 1 || R > kMaxChains) return fail(FTLM_E_RANGE, "R %d not in [1, %d]", R, kMaxChains);
    for (int i = 0; i < n_sectors; ++i) {
        if (n_ups[i] < 0 || n_ups[i] > g->n_sites) return fail(FTLM_E_INVALID, "n_ups[%d] = %d", i, n_ups[i]);
        for (int j = 0; j < i; ++j)
            if (n_ups[j] == n_ups[i]) return fail(FTLM_E_INVALID, "sector n_up = %d listed twice", n_ups[i]);
    }
    (void)mode;
    return FTLM_OK;
}

}  // namespace

extern "C" {

int ftlm_plan_workspace_bytes(const ftlm_graph* g, int n_sectors, const int32_t* n_ups, int mode, int R, int dtype,
                              size_t* bytes) {
    if (!bytes) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_plan_args(g, n_sectors, n_ups, mode, R, dtype)) return rc;
    PlanLayout L;
    if (int rc = plan_layout(g->n_sites, n_sectors, n_ups, mode, R, dtype, L)) return rc;
    *bytes = L.total;
    return ok();
}

int ftlm_plan_create(const ftlm_graph* g, int n_sectors, const int32_t* n_ups, int mode, int R, int M, int dtype,
                     void* arena_dev, size_t arena_bytes, void* stream, ftlm_plan** out) {
    if (!out || !arena_dev) return fail(FTLM_E_INVALID, "null argument");
    *out = nullptr;
    if (int rc = check_plan_args(g, n_sectors, n_ups, mode, R, dtype)) return rc;
    if (M < 1 || M > kMaxSteps) return fail(FTLM_E_RANGE, "M %d not in [1, %d]", M, kMaxSteps);
    if (reinterpret_cast<uintptr_t>(arena_dev) % 256 != 0) return fail(FTLM_E_INVALID, "arena not 256-byte aligned");
    PlanLayout L;
    if (int rc = plan_layout(g->n_sites, n_sectors, n_ups, mode, R, dtype, L)) return rc;
    if (arena_bytes < L.total) return fail(FTLM_E_NOSPACE, "arena holds %zu bytes, %zu needed", arena_bytes, L.total);
    hipStream_t st = static_cast<hipStream_t>(stream);
    ftlm_plan* p = new ftlm_plan();
    p->table = g->table;
    p->n_sites = g->n_sites;
    p->mode = mode;
    p->R = R;
    p->M = M;
    p->dtype = dtype;
    std::vector<SectorDev> devs;
    for (int i = 0; i < n_sectors; ++i) {
        ftlm_sector* s = nullptr;
        int rc = ftlm_sector_create(g->n_sites, n_ups[i], mode, at<void>(arena_dev, L.table[size_t(i)]),
                                    L.table_bytes[size_t(i)], stream, &s);
        if (rc) {
            delete p;
            return rc;
        }
        p->sectors.push_back(s);
        devs.push_back(s->dev);
    }
    job_layout(p->job, devs, L.state, arena_dev, R, M, dtype, at<SecWork>(arena_dev, L.secs));
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ready, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete p;
        return fail(FTLM_E_DEVICE, "plan setup: %s", hipGetErrorString(e));
    }
    *out = p;
    return ok();
}

int ftlm_plan_run(ftlm_plan* p, uint64_t seed, uint64_t r0, int dist, int use_graph, double* alpha_host,
                  double* beta_host, int32_t* steps_host, void* stream) {
    if (!p || !alpha_host || !beta_host || !steps_host) return fail(FTLM_E_INVALID, "null argument");
    if (dist != FTLM_PM1 && dist != FTLM_GAUSS && dist != FTLM_UNIT) return fail(FTLM_E_INVALID, "bad dist %d", dist);
    hipStream_t caller = static_cast<hipStream_t>(stream);
    HIP_CHECK(hipEventRecord(p->ready, caller));
    HIP_CHECK(hipStreamWaitEvent(p->stream, p->ready, 0));
    if (int rc = job_start(p->job, seed, r0, dist, p->stream)) return rc;
    if (use_graph) {
        if (!p->exec) {
            HIP_CHECK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
            const int rc = job_steps(p->job, p->table, p->stream, false);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(p->stream, &graph);
            if (rc != FTLM_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess) return fail(FTLM_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
            p->graph = graph;
            HIP_CHECK(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
        }
        HIP_CHECK(hipGraphLaunch(p->exec, p->stream));
    } else {
        if (int rc = job_steps(p->job, p->table, p->stream)) return rc;
    }
    if (int rc = job_collect(p->job, p->M, alpha_host, beta_host, steps_host, p->stream)) return rc;
    return ok();
}

void ftlm_plan_destroy(ftlm_plan* p) {
    if (p && p->stream) (void)hipStreamSynchronize(p->stream);
    delete p;
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
