// C ABI of libftlm (declared in include/ftlm.h): argument checking, handles,
// table layout and kernel launches. No device memory is allocated here; all
// device buffers come from the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "host.hpp"

using namespace ftlm;

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
    double jsum = 0.0;
    std::vector<int> orig(g->bi.size());
    for (size_t b = 0; b < g->bi.size(); ++b) {
        orig[b] = int(b);
        jsum += g->J[b];
    }
    g->table = make_bond_table(n_sites, g->bi, g->bj, g->J, orig, jsum);
    *out = g;
    return ok();
}

void ftlm_graph_destroy(ftlm_graph* g) { delete g; }
int ftlm_graph_n_sites(const ftlm_graph* g) { return g ? g->n_sites : 0; }
int ftlm_graph_n_bonds(const ftlm_graph* g) { return g ? int(g->bi.size()) : 0; }

// ---- sector ---------------------------------------------------------------------
int ftlm_sector_info(int n_sites, int n_up, uint64_t* dim, double* mult) {
    if (n_sites < 1 || n_sites > kMaxSites) return fail(FTLM_E_RANGE, "n_sites %d not in [1, %d]", n_sites, kMaxSites);
    if (n_up < 0 || n_up > n_sites) return fail(FTLM_E_INVALID, "n_up %d not in [0, %d]", n_up, n_sites);
    if (dim) *dim = binom_u64(n_sites, n_up);
    if (mult) *mult = sector_multiplicity(n_sites, n_up);
    return ok();
}

int ftlm_sector_table_bytes(int n_sites, int n_up, int mode, size_t* bytes) {
    if (!bytes) return fail(FTLM_E_INVALID, "null argument");
    if (mode != FTLM_CLT && mode != FTLM_CR && mode != FTLM_FULL && mode != FTLM_LIN)
        return fail(FTLM_E_INVALID, "mode %d is not FTLM_CLT/FTLM_CR/FTLM_FULL/FTLM_LIN", mode);
    if (n_sites < 1 || n_sites > kMaxSites) return fail(FTLM_E_RANGE, "n_sites %d not in [1, %d]", n_sites, kMaxSites);
    if (n_up < 0 || n_up > n_sites) return fail(FTLM_E_INVALID, "n_up %d not in [0, %d]", n_up, n_sites);
    if (mode != FTLM_CR && n_sites > kMaxCltSites)
        return fail(FTLM_E_RANGE, "stored maps hold uint32 labels: n_sites %d > %d", n_sites, kMaxCltSites);
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
    d.basis = mode != FTLM_CR ? at<uint32_t>(table_dev, s->layout.basis_off) : nullptr;
    d.clt = mode == FTLM_CLT ? at<CltEntry>(table_dev, s->layout.clt_off) : nullptr;
    d.full = mode == FTLM_FULL ? at<uint32_t>(table_dev, s->layout.full_off) : nullptr;
    d.lin_hi = mode == FTLM_LIN ? at<uint32_t>(table_dev, s->layout.hi_off) : nullptr;
    d.lin_lo = mode == FTLM_LIN ? at<uint32_t>(table_dev, s->layout.lo_off) : nullptr;
    d.lin_lo_bits = lin_low_bits(n_sites);
    d.two_s = 1;
    d.n_labels = n_sites < 64 ? (uint64_t(1) << n_sites) : ~uint64_t(0);
    hipError_t e = hipMemcpyAsync(const_cast<uint32_t*>(d.binom), s->binom_host.data(),
                                  s->binom_host.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host copy may be reused at once
    if (e == hipSuccess && mode != FTLM_CR) {
        e = launch_build_basis(d, st);
        if (e == hipSuccess && mode == FTLM_CLT) e = launch_build_clt(d, st);
        if (e == hipSuccess && mode == FTLM_FULL) e = launch_build_full(d, st);
        if (e == hipSuccess && mode == FTLM_LIN) e = launch_build_lin(d, st);
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

// ---- general local spin (Sec. 2, Eqs. 11-17) ---------------------------------------
}  // extern "C"

namespace {

// D(m, A) for 0 <= m <= N, 0 <= A <= N two_s by the recursion of Eq. (15);
// exact in 64 bits for every size accepted here (D <= d^N <= 8^16).
std::vector<std::vector<uint64_t>> spin_dims(int n_sites, int two_s) {
    const int amax = n_sites * two_s;
    std::vector<std::vector<uint64_t>> D(size_t(n_sites) + 1, std::vector<uint64_t>(size_t(amax) + 1, 0));
    D[0][0] = 1;
    for (int m = 1; m <= n_sites; ++m)
        for (int a = 0; a <= m * two_s; ++a)
            for (int q = 0; q <= two_s && q <= a; ++q) D[size_t(m)][size_t(a)] += D[size_t(m - 1)][size_t(a - q)];
    return D;
}

uint64_t ipow_u64(uint64_t b, int e) {
    uint64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

int check_spin_args(int n_sites, int two_s, int a_tot, int mode) {
    if (mode != FTLM_CLT && mode != FTLM_CR)
        return fail(FTLM_E_INVALID, "mode %d: general spin takes FTLM_CLT or FTLM_CR", mode);
    if (two_s < 1 || two_s > 7) return fail(FTLM_E_RANGE, "2s = %d not in [1, 7]", two_s);
    if (n_sites < 2 || n_sites > 16) return fail(FTLM_E_RANGE, "n_sites %d not in [2, 16] for general spin", n_sites);
    if (a_tot < 0 || a_tot > n_sites * two_s)
        return fail(FTLM_E_INVALID, "digit sum %d not in [0, %d]", a_tot, n_sites * two_s);
    return FTLM_OK;
}

}  // namespace

extern "C" {

int ftlm_sector_info_spin(int n_sites, int two_s, int a_tot, uint64_t* dim, double* mult) {
    if (two_s == 1) return ftlm_sector_info(n_sites, a_tot, dim, mult);
    if (int rc = check_spin_args(n_sites, two_s, a_tot, FTLM_CR)) return rc;
    if (dim) *dim = spin_dims(n_sites, two_s)[size_t(n_sites)][size_t(a_tot)];
    if (mult) *mult = 2 * a_tot == n_sites * two_s ? 1.0 : 2.0;
    return ok();
}

int ftlm_sector_table_bytes_spin(int n_sites, int two_s, int a_tot, int mode, size_t* bytes) {
    if (!bytes) return fail(FTLM_E_INVALID, "null argument");
    if (two_s == 1) return ftlm_sector_table_bytes(n_sites, a_tot, mode, bytes);
    if (int rc = check_spin_args(n_sites, two_s, a_tot, mode)) return rc;
    const uint64_t dim = spin_dims(n_sites, two_s)[size_t(n_sites)][size_t(a_tot)];
    if (dim >= (uint64_t(1) << 32)) return fail(FTLM_E_RANGE, "sector dimension %llu >= 2^32", (unsigned long long)dim);
    const uint64_t labels = ipow_u64(uint64_t(two_s + 1), n_sites);
    if (mode == FTLM_CLT && labels > (uint64_t(1) << 32))
        return fail(FTLM_E_RANGE, "FTLM_CLT holds uint32 labels: d^N = %llu > 2^32", (unsigned long long)labels);
    size_t end = align256(size_t(n_sites) * size_t(a_tot + 3) * size_t(two_s + 1) * 4);
    if (mode == FTLM_CLT) {
        end = align256(end + size_t(dim) * 4);
        end = align256(end + size_t((labels + 31) / 32) * sizeof(CltEntry));
    }
    *bytes = end;
    return ok();
}

int ftlm_sector_create_spin(int n_sites, int two_s, int a_tot, int mode, void* table_dev, size_t bytes,
                            void* stream, ftlm_sector** out) {
    if (!out || !table_dev) return fail(FTLM_E_INVALID, "null argument");
    if (two_s == 1) return ftlm_sector_create(n_sites, a_tot, mode, table_dev, bytes, stream, out);
    *out = nullptr;
    size_t need = 0;
    if (int rc = ftlm_sector_table_bytes_spin(n_sites, two_s, a_tot, mode, &need)) return rc;
    if (bytes < need) return fail(FTLM_E_NOSPACE, "table buffer holds %zu bytes, %zu needed", bytes, need);
    if (reinterpret_cast<uintptr_t>(table_dev) % 256 != 0) return fail(FTLM_E_INVALID, "table buffer not 256-byte aligned");
    const auto D = spin_dims(n_sites, two_s);
    const int d = two_s + 1, bw = a_tot + 3;
    ftlm_sector* s = new ftlm_sector();
    s->n_sites = n_sites;
    s->n_up = a_tot;
    s->two_s = two_s;
    s->mode = mode;
    s->dim = D[size_t(n_sites)][size_t(a_tot)];
    s->table = table_dev;
    s->bytes = bytes;
    // D_c(p, A, a) = sum_{q < a} D(p, A - q) (Eq. 16) for A in [-1, a_tot + 1], mod 2^32
    s->binom_host.assign(size_t(n_sites) * size_t(bw) * size_t(d), 0u);
    for (int p = 0; p < n_sites; ++p)
        for (int A = -1; A <= a_tot + 1; ++A)
            for (int a = 0; a < d; ++a) {
                uint64_t c = 0;
                for (int q = 0; q < a; ++q) {
                    const int r = A - q;
                    if (r >= 0 && r <= p * two_s) c += D[size_t(p)][size_t(r)];
                }
                s->binom_host[(size_t(p) * size_t(bw) + size_t(A + 1)) * size_t(d) + size_t(a)] = uint32_t(c);
            }
    const uint64_t labels = ipow_u64(uint64_t(d), n_sites);
    const size_t tab_end = align256(s->binom_host.size() * 4);
    SectorDev& dv = s->dev;
    dv.n_sites = n_sites;
    dv.n_up = a_tot;
    dv.mode = mode;
    dv.bw = bw;
    dv.dim = uint32_t(s->dim);
    dv.binom = static_cast<const uint32_t*>(table_dev);
    dv.basis = mode == FTLM_CLT ? at<uint32_t>(table_dev, tab_end) : nullptr;
    dv.clt = mode == FTLM_CLT ? at<CltEntry>(table_dev, align256(tab_end + size_t(s->dim) * 4)) : nullptr;
    dv.two_s = two_s;
    dv.n_labels = labels;
    s->layout.binom_off = 0;
    s->layout.basis_off = mode == FTLM_CLT ? tab_end : 0;
    s->layout.clt_off = mode == FTLM_CLT ? align256(tab_end + size_t(s->dim) * 4) : 0;
    s->layout.total = need;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(const_cast<uint32_t*>(dv.binom), s->binom_host.data(), s->binom_host.size() * 4,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host copy may be reused at once
    if (e == hipSuccess && mode == FTLM_CLT) {
        e = launch_build_basis_spin(dv, st);
        if (e == hipSuccess) e = launch_build_clt_spin(dv, st);
    }
    if (e != hipSuccess) {
        delete s;
        return fail(FTLM_E_DEVICE, "sector build: %s", hipGetErrorString(e));
    }
    *out = s;
    return ok();
}

int ftlm_sector_two_s(const ftlm_sector* s) { return s ? s->two_s : 0; }

int ftlm_rank(const ftlm_sector* s, const uint64_t* labels_dev, uint64_t* idx_dev, uint64_t n, void* stream) {
    if (!s || (n && (!labels_dev || !idx_dev))) return fail(FTLM_E_INVALID, "null argument");
    if (n == 0) return ok();
    if (s->two_s > 1) HIP_CHECK(launch_rank_spin(s->dev, labels_dev, idx_dev, n, static_cast<hipStream_t>(stream)));
    else HIP_CHECK(launch_rank(s->dev, labels_dev, idx_dev, n, static_cast<hipStream_t>(stream)));
    return ok();
}

int ftlm_unrank(const ftlm_sector* s, const uint64_t* idx_dev, uint64_t* labels_dev, uint64_t n, void* stream) {
    if (!s || (n && (!labels_dev || !idx_dev))) return fail(FTLM_E_INVALID, "null argument");
    if (n == 0) return ok();
    if (s->two_s > 1) HIP_CHECK(launch_unrank_spin(s->dev, idx_dev, labels_dev, n, static_cast<hipStream_t>(stream)));
    else HIP_CHECK(launch_unrank(s->dev, idx_dev, labels_dev, n, static_cast<hipStream_t>(stream)));
    return ok();
}

int ftlm_clt_export(const ftlm_sector* s, uint32_t* mask_host, uint32_t* prefix_host, uint64_t nblocks,
                    void* stream) {
    if (!s || !mask_host || !prefix_host) return fail(FTLM_E_INVALID, "null argument");
    if (s->mode != FTLM_CLT) return fail(FTLM_E_INVALID, "sector is not in FTLM_CLT mode");
    const uint64_t have = s->two_s > 1 ? (s->dev.n_labels + 31) / 32 : clt_blocks(s->n_sites);
    if (nblocks > have) return fail(FTLM_E_RANGE, "nblocks %llu > %llu", (unsigned long long)nblocks,
                                    (unsigned long long)have);
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
    if (s->two_s > 1)
        HIP_CHECK(launch_neighbors_spin(s->dev, g->table, t0, count, idx_dev, static_cast<hipStream_t>(stream)));
    else HIP_CHECK(launch_neighbors(s->dev, g->table, t0, count, idx_dev, static_cast<hipStream_t>(stream)));
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
    for (auto [col, vb] : column_chunks(nvec, uint64_t(nvec), dtype, {x_dev, y_dev}, max_launch_width(s->two_s))) {
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
}  // extern "C"

namespace {

struct SingleLayout {
    SectorState st;
    size_t secs, bonds, queue, total;
};

SingleLayout single_layout(uint64_t dim, int R, int dtype) {
    SingleLayout l{};
    size_t off = layout_state(dim, R, dtype, 0, l.st);
    l.secs = off;
    off = align256(off + sizeof(SecWork));
    l.bonds = off;
    off = align256(off + kTablesPerGraph * sizeof(BondTable));
    l.queue = off;
    off = align256(off + kQueueBytes);
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

void single_job(LanczosJob& job, const ftlm_sector* s, const ftlm_graph* g, int R, int M, int dtype, void* work) {
    const SingleLayout l = single_layout(s->dim, R, dtype);
    job_layout(job, {s->dev}, {l.st}, work, R, M, dtype, at<SecWork>(work, l.secs), {g},
               {at<BondTable>(work, l.bonds)}, {0});
    job.queue = at<uint32_t>(work, l.queue);
}

}  // namespace

extern "C" {

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
    single_job(job, s, nullptr, R, 1, dtype, work_dev);
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
    single_job(job, s, g, R, M, dtype, work_dev);
    if (int rc = job_start(job, seed, r0, dist, st)) return rc;
    if (int rc = job_steps(job, st)) return rc;
    if (int rc = job_collect(job, M, alpha_host, beta_host, steps_host, st)) return rc;
    return ok();
}

// ---- autotuning ----------------------------------------------------------------------
}  // extern "C"

namespace {

struct TuneCache {
    std::mutex mu;
    bool loaded = false;
    std::map<std::string, std::pair<int, double>> entries;
} g_tune;

// "_c3": the candidate set, cost model and kernel set; a cache file written
// under an older one is not reused.
std::string tune_key(const ftlm_sector* s, const ftlm_graph* g, int R, int dtype) {
    std::string k = "N" + std::to_string(s->n_sites) + "_s" + std::to_string(s->two_s) + "_u" +
                    std::to_string(s->n_up) + "_m" + std::to_string(s->mode) + "_t" + std::to_string(dtype) + "_R" +
                    std::to_string(R) + "_c3_b";
    // the bond structure, so that two graphs with the same size do not share entries
    uint64_t h = 1469598103934665603ull;
    for (size_t b = 0; b < g->bi.size(); ++b) {
        h = (h ^ uint64_t(g->bi[b] * 64 + g->bj[b])) * 1099511628211ull;
    }
    return k + std::to_string(h);
}

void tune_load_file() {
    if (g_tune.loaded) return;
    g_tune.loaded = true;
    const char* path = std::getenv("FTLM_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[256];
    int batch = 0;
    double ms = 0;
    while (std::fscanf(f, "%255s %d %lf", key, &batch, &ms) == 3) g_tune.entries[key] = {batch, ms};
    std::fclose(f);
}

void tune_store_file(const std::string& key, int batch, double ms) {
    const char* path = std::getenv("FTLM_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %.6f\n", key.c_str(), batch, ms);
    std::fclose(f);
}

}  // namespace

extern "C" {

int ftlm_autotune(const ftlm_sector* s, const ftlm_graph* g, int R, int dtype, void* work_dev, size_t work_bytes,
                  void* stream, ftlm_tuning* out) {
    if (!s || !g || !out) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_lanczos_args(s, R, FTLM_PM1, dtype, work_dev, work_bytes)) return rc;
    if (g->n_sites != s->n_sites) return fail(FTLM_E_INVALID, "graph has %d sites, sector %d", g->n_sites, s->n_sites);
    std::memset(out, 0, sizeof(*out));
    const std::string key = tune_key(s, g, R, dtype);
    {
        std::lock_guard<std::mutex> lk(g_tune.mu);
        tune_load_file();
        auto it = g_tune.entries.find(key);
        if (it != g_tune.entries.end()) {
            out->batch = it->second.first;
            out->ms_per_step = it->second.second;
            out->cached = 1;
            return ok();
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // every width a Lanczos launch can take (FP32 only: 10, 12, 20, 32), so
    // that a batch of any size is priced from launches that were measured
    const int widths[] = {1, 2, 4, 8, 10, 12, 16, 20, 32};
    const int widest = max_launch_width(s->two_s);
    EventPair ev;
    HIP_CHECK(ev.create());
    int n = 0;
    for (int B : widths) {
        if (B > R || B > widest || (dtype == FTLM_F64 && (B > 16 || B == 10 || B == 12))) continue;
        // B chains of the sector (their state fits the workspace sized for
        // R >= B); two Lanczos steps per repetition, the first one a warm-up
        LanczosJob job;
        single_job(job, s, g, B, 3, dtype, work_dev);
        float best_ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            int rc = job_start(job, 0, 0, FTLM_PM1, st);
            if (rc == FTLM_OK) rc = job_steps(job, st, false, 1);
            if (rc == FTLM_OK && hipEventRecord(ev.e0, st) != hipSuccess) rc = FTLM_E_DEVICE;
            if (rc == FTLM_OK) rc = job_steps(job, st, false, 1);
            if (rc == FTLM_OK && hipEventRecord(ev.e1, st) != hipSuccess) rc = FTLM_E_DEVICE;
            if (rc == FTLM_OK && hipEventSynchronize(ev.e1) != hipSuccess) rc = FTLM_E_DEVICE;
            if (rc != FTLM_OK) return rc == FTLM_E_DEVICE ? fail(rc, "autotune: HIP error") : rc;
            float ms = 0.f;
            HIP_CHECK(hipEventElapsedTime(&ms, ev.e0, ev.e1));
            if (rep > 0) best_ms = std::min(best_ms, ms);  // the first rep warms up
        }
        out->widths[n] = B;
        out->ms[n] = best_ms;
        ++n;
    }
    // A batch of x chains runs as the column chunks ftlm_lanczos cuts for it;
    // its step costs the measured steps of those widths.
    auto measured = [&](int w) {
        for (int i = 0; i < n; ++i)
            if (out->widths[i] == w) return out->ms[i];
        return 1e300;  // not reached: every chunk width is a candidate <= R
    };
    auto batch_ms = [&](int x) {
        double t = 0.0;
        for (auto [col, w] : column_chunks_v(x, uint64_t(x), dtype, {}, widest)) t += measured(w);
        return t;
    };
    // R chains in batches of b: R / b full batches and one of R mod b
    double best = 1e300;
    int best_b = 1;
    for (int i = 0; i < n; ++i) {
        const int b = out->widths[i];
        const double step = double(R / b) * batch_ms(b) + (R % b ? batch_ms(R % b) : 0.0);
        if (step < best) {
            best = step;
            best_b = b;
        }
    }
    out->n_candidates = n;
    out->batch = best_b;
    out->ms_per_step = best;
    {
        std::lock_guard<std::mutex> lk(g_tune.mu);
        g_tune.entries[key] = {best_b, best};
        tune_store_file(key, best_b, best);
    }
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
    size_t secs, bonds, queue;
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
    L.bonds = off;
    off = align256(off + kTablesPerGraph * sizeof(BondTable));
    L.queue = off;
    off = align256(off + kQueueBytes);
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
    job_layout(p->job, devs, L.state, arena_dev, R, M, dtype, at<SecWork>(arena_dev, L.secs), {g},
               {at<BondTable>(arena_dev, L.bonds)}, std::vector<int>(size_t(n_sectors), 0));
    p->job.queue = at<uint32_t>(arena_dev, L.queue);
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
            const int rc = job_steps(p->job, p->stream, false);
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
        if (int rc = job_steps(p->job, p->stream)) return rc;
    }
    if (int rc = job_collect(p->job, p->M, alpha_host, beta_host, steps_host, p->stream)) return rc;
    return ok();
}

int ftlm_plan_tune(ftlm_plan* p, void* stream, ftlm_plan_tuning* out) {
    if (!p) return fail(FTLM_E_INVALID, "null argument");
    EventPair ev;
    HIP_CHECK(ev.create());
    HIP_CHECK(hipEventRecord(p->ready, static_cast<hipStream_t>(stream)));
    HIP_CHECK(hipStreamWaitEvent(p->stream, p->ready, 0));
    static const int caps32[] = {32, 20, 16, 10, 8, 4}, caps64[] = {16, 8, 4};
    const int* caps = p->dtype == FTLM_F32 ? caps32 : caps64;
    const int ncap = p->dtype == FTLM_F32 ? 6 : 3;
    const auto previous = p->job.chunks;
    std::vector<std::vector<std::pair<int, int>>> seen;
    ftlm_plan_tuning t{};
    double best = 1e300;
    for (int i = 0; i < ncap; ++i) {
        auto chunks = job_chunks(p->job, caps[i]);
        if (std::find(seen.begin(), seen.end(), chunks) != seen.end()) continue;
        seen.push_back(chunks);
        p->job.chunks = chunks;
        float best_ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            int rc = job_start(p->job, 0, 0, FTLM_PM1, p->stream);
            if (rc == FTLM_OK) rc = job_steps(p->job, p->stream, false, 1);
            if (rc == FTLM_OK && hipEventRecord(ev.e0, p->stream) != hipSuccess) rc = FTLM_E_DEVICE;
            if (rc == FTLM_OK) rc = job_steps(p->job, p->stream, false, 1);
            if (rc == FTLM_OK && hipEventRecord(ev.e1, p->stream) != hipSuccess) rc = FTLM_E_DEVICE;
            if (rc == FTLM_OK && hipEventSynchronize(ev.e1) != hipSuccess) rc = FTLM_E_DEVICE;
            float ms = 0.f;
            if (rc == FTLM_OK && hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess) rc = FTLM_E_DEVICE;
            if (rc != FTLM_OK) {
                p->job.chunks = previous;
                return rc == FTLM_E_DEVICE ? fail(rc, "plan tuning: HIP error") : rc;
            }
            best_ms = std::min(best_ms, ms);
        }
        const int n = t.n_candidates++;
        t.max_width[n] = caps[i];
        t.n_launches[n] = int32_t(chunks.size());
        t.ms[n] = best_ms;
        if (best_ms < best) {
            best = best_ms;
            t.chosen = n;
        }
    }
    p->job.chunks = seen[size_t(t.chosen)];
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    if (out) *out = t;
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

int ftlm_ritz_batch(int n, int stride, const int32_t* m, const double* alpha, const double* beta, double* theta,
                    double* weight) {
    if (n < 0 || stride < 1) return fail(FTLM_E_INVALID, "n = %d, stride = %d", n, stride);
    if (n == 0) return ok();
    if (!m || !alpha || !beta || !theta || !weight) return fail(FTLM_E_INVALID, "null argument");
    for (int r = 0; r < n; ++r)
        if (m[r] < 1 || m[r] > stride) return fail(FTLM_E_INVALID, "chain %d: m = %d outside [1, %d]", r, m[r], stride);
    if (ritz_batch(n, stride, m, alpha, beta, theta, weight) != 0)
        return fail(FTLM_E_INVALID, "QL iteration did not converge");
    return ok();
}

int ftlm_ghosts(int m, const double* alpha, const double* beta, double c_tau, double* theta, double* weight,
                double* ell, int32_t* ghost, int32_t* cluster, double* cluster_weight, int32_t* n_clusters,
                double* tau) {
    if (m < 1 || !alpha || (m > 1 && !beta) || !theta || !weight || !ell || !ghost || !cluster || !cluster_weight ||
        !n_clusters || !tau)
        return fail(FTLM_E_INVALID, "bad argument");
    if (!(c_tau >= 0.0) || !std::isfinite(c_tau)) return fail(FTLM_E_INVALID, "c_tau %g is not a finite value >= 0", c_tau);
    if (ghost_test(m, alpha, beta, c_tau, kUnitRoundoffF32, theta, weight, ell, ghost, cluster, cluster_weight,
                   n_clusters, tau) != 0)
        return fail(FTLM_E_INVALID, "QL iteration did not converge");
    return ok();
}

int ftlm_seed_spread(int n_seeds, int n, const double* values, double* mean, double* sigma) {
    if (n_seeds < 1 || n < 0 || (n && (!values || !mean || !sigma)))
        return fail(FTLM_E_INVALID, "n_seeds = %d, n = %d", n_seeds, n);
    seed_spread(n_seeds, n, values, mean, sigma);
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
        if (r.two_s < 0 || r.two_s > 7) return fail(FTLM_E_INVALID, "sector %d: 2s = %d", i, r.two_s);
        v[size_t(i)] = SectorSamples{r.n_up, r.two_s > 1 ? r.two_s : 1, r.R, r.stride, r.dim, r.mult,
                                     r.theta, r.weight, r.steps};
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
