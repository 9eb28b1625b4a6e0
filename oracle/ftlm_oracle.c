/*
 * FP64 CPU oracle for the spin-1/2 Heisenberg FTLM hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It is written for obviousness, not speed:
 * every quantity is computed from its plain definition.
 *
 * Conventions (paper, Sec. 2, Eq. 11 at s = 1/2): a basis state of N sites
 * is the integer n whose bit k is 1 when site k is up (a_k = m_k + 1/2).
 * The S^z sector with n_up up spins (M = n_up - N/2, Eq. 17) holds every
 * such n with popcount(n) = n_up; its basis is ordered by increasing label
 * (Sec. 2, "Compressed lookup table", the ordering convention of Eq. 18).
 * An index of a label outside the sector is UINT64_MAX (the -1 of Alg. 2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NONE UINT64_MAX

static int popcount64(uint64_t x) {
    int c = 0;
    while (x) {
        c += (int)(x & 1u);
        x >>= 1;
    }
    return c;
}

/* Binomial coefficients C(n, k) for 0 <= k <= n <= 64 as exact integers,
 * filled once at load time by Pascal's rule C(n, k) = C(n-1, k-1) + C(n-1, k)
 * (every entry fits in 64 bits). This is the spin-1/2 case of the dimension
 * recursion D(m, A) of Eq. (15): with digits in {0, 1}, D(m, A) = C(m, A). */
static uint64_t pascal[65][65];

__attribute__((constructor)) static void fill_pascal(void) {
    for (int n = 0; n <= 64; ++n) {
        pascal[n][0] = 1;
        for (int k = 1; k <= n; ++k) pascal[n][k] = pascal[n - 1][k - 1] + (k < n ? pascal[n - 1][k] : 0);
    }
}

/* C(n, k), zero outside 0 <= k <= n. */
uint64_t orc_binom(int n, int k) {
    if (n < 0 || k < 0 || k > n || n > 64) return 0;
    return pascal[n][k];
}

/* Sector dimension D_M = C(N, n_up). */
uint64_t orc_sector_dim(int n_sites, int n_up) { return orc_binom(n_sites, n_up); }

/* The sector basis in ascending label order, by scanning the whole label
 * space [0, 2^N) and keeping each label with n_up set bits. Returns the
 * number written, or -1 if `cap` is too small. N <= 34 (the scan is 2^N). */
int64_t orc_enumerate(int n_sites, int n_up, uint64_t* out, uint64_t cap) {
    uint64_t c = 0;
    uint64_t end = (uint64_t)1 << n_sites;
    for (uint64_t x = 0; x < end; ++x) {
        if (popcount64(x) == n_up) {
            if (c >= cap) return -1;
            out[c++] = x;
        }
    }
    return (int64_t)c;
}

/* Number of sector labels strictly smaller than x (any x < 2^N).
 * A sector label y is below x exactly when, at the highest bit p where they
 * differ, x has a 1 and y a 0. For that p, y copies x above p, and its p low
 * bits hold the remaining n_up - (ones of x above p) up spins in any of
 * C(p, remaining) ways. Summing over the set bits p of x counts each smaller
 * y once. */
uint64_t orc_count_below(int n_sites, int n_up, uint64_t x) {
    uint64_t count = 0;
    int ones_above = 0;
    for (int p = n_sites - 1; p >= 0; --p) {
        if ((x >> p) & 1u) {
            int remaining = n_up - ones_above;
            if (remaining >= 0) count += orc_binom(p, remaining);
            ones_above += 1;
        }
    }
    return count;
}

/* Sector index of a label: its position in the ascending basis, i.e. the
 * number of sector labels below it. UINT64_MAX when x is not in the sector. */
uint64_t orc_rank(int n_sites, int n_up, uint64_t x) {
    if (n_sites < 64 && (x >> n_sites) != 0) return ORC_NONE;
    if (popcount64(x) != n_up) return ORC_NONE;
    return orc_count_below(n_sites, n_up, x);
}

/* Position of x in a sorted basis array by binary search; UINT64_MAX if
 * absent. This is the definition of the index when the basis is stored. */
uint64_t orc_rank_bsearch(const uint64_t* basis, uint64_t dim, uint64_t x) {
    uint64_t lo = 0, hi = dim;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (basis[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    if (lo < dim && basis[lo] == x) return lo;
    return ORC_NONE;
}

/* The t-th sector label (inverse of orc_rank), found as the smallest label
 * x whose count of smaller-or-equal sector labels exceeds t, by bisection
 * over the label space. UINT64_MAX if t >= D. N <= 62. */
uint64_t orc_unrank(int n_sites, int n_up, uint64_t t) {
    if (t >= orc_sector_dim(n_sites, n_up)) return ORC_NONE;
    uint64_t lo = 0, hi = ((uint64_t)1 << n_sites) - 1;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (orc_count_below(n_sites, n_up, mid + 1) > t) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

/* Compressed lookup table (Sec. 2, Eqs. 18-21): the label space is split
 * into blocks of 32; mask[b] has bit j set iff label 32b + j is in the
 * sector, and prefix[b] is the number of sector labels in blocks 0..b-1.
 * Built in one pass over the sorted basis, then a running sum. */
void orc_clt(const uint64_t* basis, uint64_t dim, uint64_t nblocks, uint32_t* mask,
             uint32_t* prefix) {
    memset(mask, 0, nblocks * sizeof(uint32_t));
    for (uint64_t t = 0; t < dim; ++t) {
        uint64_t n = basis[t];
        mask[n / 32] |= (uint32_t)1u << (n % 32);
    }
    uint64_t running = 0;
    for (uint64_t b = 0; b < nblocks; ++b) {
        prefix[b] = (uint32_t)running;
        running += (uint64_t)popcount64(mask[b]);
    }
}

/* Index lookup through the table (Alg. 2). */
uint64_t orc_clt_lookup(const uint32_t* mask, const uint32_t* prefix, uint64_t n) {
    uint64_t b = n / 32;
    unsigned j = (unsigned)(n % 32);
    if (((mask[b] >> j) & 1u) == 0) return ORC_NONE;
    uint32_t below = mask[b] & (((uint32_t)1u << j) - 1u);
    return (uint64_t)prefix[b] + (uint64_t)popcount64(below);
}

/* Label of row t: from the stored basis when one is given, else by
 * bisection. */
static uint64_t row_label(int n_sites, int n_up, const uint64_t* basis, uint64_t t) {
    return basis ? basis[t] : orc_unrank(n_sites, n_up, t);
}

static uint64_t index_of(int n_sites, int n_up, const uint64_t* basis, uint64_t dim,
                         uint64_t x) {
    return basis ? orc_rank_bsearch(basis, dim, x) : orc_rank(n_sites, n_up, x);
}

/* Neighbour lists (Eq. 12 at s = 1/2): for each of `count` rows starting at
 * t0, and each bond b in the order given, the sector index of the partner
 * label n XOR (2^i + 2^j) when sites i and j are antiparallel, else
 * UINT64_MAX. out is [count][n_bonds]. */
void orc_neighbors(int n_sites, int n_up, int n_bonds, const int32_t* bi, const int32_t* bj,
                   const uint64_t* basis, uint64_t t0, uint64_t count, uint64_t* out) {
    uint64_t dim = orc_sector_dim(n_sites, n_up);
#pragma omp parallel for schedule(dynamic, 256) if (count > 4096)
    for (int64_t r = 0; r < (int64_t)count; ++r) {
        uint64_t n = row_label(n_sites, n_up, basis, t0 + (uint64_t)r);
        for (int b = 0; b < n_bonds; ++b) {
            uint64_t si = (n >> bi[b]) & 1u, sj = (n >> bj[b]) & 1u;
            uint64_t v = ORC_NONE;
            if (si != sj) {
                uint64_t partner = n ^ (((uint64_t)1 << bi[b]) | ((uint64_t)1 << bj[b]));
                v = index_of(n_sites, n_up, basis, dim, partner);
            }
            out[(uint64_t)r * (uint64_t)n_bonds + (uint64_t)b] = v;
        }
    }
}

/* Matrix-free H.x in row-wise gather form (Eq. 12, coefficients Eqs. 13-14
 * at s = 1/2), in FP64, for the rows [row0, row0 + nrows) of the sector:
 *   y[r] = sum_b J_b s^z_i s^z_j x[t] + sum_{b antiparallel} (J_b / 2) x[idx(n ^ mask_b)]
 * with t = row0 + r, s^z s^z = +1/4 for parallel and -1/4 for antiparallel
 * spins. x has the full sector length; y has nrows entries. The per-bond
 * couplings J_b generalize the single J of Eq. (1). */
void orc_hv(int n_sites, int n_up, int n_bonds, const int32_t* bi, const int32_t* bj,
            const double* J, const uint64_t* basis, const double* x, double* y, uint64_t row0,
            uint64_t nrows) {
    uint64_t dim = orc_sector_dim(n_sites, n_up);
#pragma omp parallel for schedule(dynamic, 1024) if (nrows > 4096)
    for (int64_t r = 0; r < (int64_t)nrows; ++r) {
        uint64_t t = row0 + (uint64_t)r;
        uint64_t n = row_label(n_sites, n_up, basis, t);
        double acc = 0.0;
        for (int b = 0; b < n_bonds; ++b) {
            int up_i = (int)((n >> bi[b]) & 1u), up_j = (int)((n >> bj[b]) & 1u);
            double mi = up_i ? 0.5 : -0.5, mj = up_j ? 0.5 : -0.5;
            acc += J[b] * mi * mj * x[t];
            if (up_i != up_j) {
                uint64_t partner = n ^ (((uint64_t)1 << bi[b]) | ((uint64_t)1 << bj[b]));
                uint64_t idx = index_of(n_sites, n_up, basis, dim, partner);
                acc += 0.5 * J[b] * x[idx];
            }
        }
        y[r] = acc;
    }
}

/* ---- Start vectors ------------------------------------------------------
 * The paper draws normalized random vectors (Sec. 2, FTLM) with seeds shared
 * between precisions (Sec. 3.1) but fixes no generator. This oracle uses the
 * SplitMix64 generator of Steele, Lea and Flood (OOPSLA 2014): state advances
 * by the odd constant GAMMA and each output is the state passed through the
 * MIX64 finalizer. It is counter-based: output i of a stream keyed K is
 * MIX64(K + (i + 1) * GAMMA), so entry i of vector r does not depend on R. */
static const uint64_t GAMMA = 0x9e3779b97f4a7c15ull;

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* First output of a SplitMix64 stream seeded at s. */
static uint64_t first_output(uint64_t s) { return mix64(s + GAMMA); }

/* Stream key of sample r in the sector with n_up up spins. */
uint64_t orc_stream_key(uint64_t seed, int n_up, uint64_t r) {
    uint64_t k = first_output(seed);
    k = first_output(k ^ (uint64_t)(uint32_t)n_up);
    k = first_output(k ^ r);
    return k;
}

/* Distribution codes: 0 = i.i.d. +-1 (sign from the top bit of output i),
 * 1 = standard normal by Box-Muller on two 53-bit uniforms (outputs 2i and
 * 2i + 1), 2 = the unit vector e_r (exact-trace mode, R = D). */
void orc_start_vector(uint64_t seed, int n_up, uint64_t r, int dist, uint64_t dim,
                      double* out) {
    uint64_t key = orc_stream_key(seed, n_up, r);
    const double two_pi = 2.0 * 3.141592653589793;
#pragma omp parallel for schedule(static) if (dim > 65536)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        double v;
        if (dist == 0) {
            uint64_t u = mix64(key + (i + 1) * GAMMA);
            v = (u >> 63) ? -1.0 : 1.0;
        } else if (dist == 1) {
            uint64_t u1 = mix64(key + (2 * i + 1) * GAMMA);
            uint64_t u2 = mix64(key + (2 * i + 2) * GAMMA);
            double a = (double)((u1 >> 11) + 1) * 0x1.0p-53; /* (0, 1] */
            double b = (double)(u2 >> 11) * 0x1.0p-53;       /* [0, 1) */
            v = sqrt(-2.0 * log(a)) * cos(two_pi * b);
        } else {
            v = (i == r) ? 1.0 : 0.0;
        }
        out[i] = v;
    }
}

/* Batch forms of orc_rank / orc_unrank over arrays (OpenMP over entries). */
void orc_rank_many(int n_sites, int n_up, const uint64_t* labels, uint64_t count,
                   uint64_t* out) {
#pragma omp parallel for schedule(static) if (count > 4096)
    for (int64_t i = 0; i < (int64_t)count; ++i) out[i] = orc_rank(n_sites, n_up, labels[i]);
}

void orc_unrank_many(int n_sites, int n_up, const uint64_t* idx, uint64_t count,
                     uint64_t* out) {
#pragma omp parallel for schedule(static) if (count > 1024)
    for (int64_t i = 0; i < (int64_t)count; ++i) out[i] = orc_unrank(n_sites, n_up, idx[i]);
}

/* H.x on an arbitrary list of rows (row-sampled checks at sizes where the
 * full product is too slow for the CPU): y[r] is row rows[r] of H.x. */
void orc_hv_rows(int n_sites, int n_up, int n_bonds, const int32_t* bi, const int32_t* bj,
                 const double* J, const uint64_t* basis, const double* x, double* y,
                 const uint64_t* rows, uint64_t nrows) {
#pragma omp parallel for schedule(dynamic, 64) if (nrows > 256)
    for (int64_t r = 0; r < (int64_t)nrows; ++r)
        orc_hv(n_sites, n_up, n_bonds, bi, bj, J, basis, x, y + r, rows[r], 1);
}

/* Output i (0-based) of a SplitMix64 generator seeded at s, for checking the
 * generator against its published output sequence. */
uint64_t orc_splitmix64_output(uint64_t s, uint64_t i) { return mix64(s + (i + 1) * GAMMA); }

/* Compressed-lookup-table entries of selected blocks straight from the
 * definition (Eqs. 18-19): bit j of block b is set when label 32b + j (below
 * 2^N) has n_up set bits; the prefix is the number of sector labels below
 * 32b. Used where the full basis is too large to enumerate. */
void orc_clt_blocks(int n_sites, int n_up, const uint64_t* blocks, uint64_t count, uint32_t* mask,
                    uint32_t* prefix) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i) {
        uint64_t b = blocks[i];
        uint32_t m = 0;
        for (unsigned j = 0; j < 32; ++j) {
            uint64_t label = b * 32 + j;
            if ((n_sites >= 64 || (label >> n_sites) == 0) && popcount64(label) == n_up) m |= 1u << j;
        }
        mask[i] = m;
        prefix[i] = (uint32_t)orc_count_below(n_sites, n_up, b * 32);
    }
}

/* Full lookup table (Sec. 2, the simplest state-to-index map): one uint32
 * per label of [0, 2^N), holding the sector index of sector labels and
 * 0xFFFFFFFF elsewhere. Built from the sorted basis. 4 * 2^N bytes. */
void orc_full_table(int n_sites, const uint64_t* basis, uint64_t dim, uint32_t* table) {
    uint64_t size = (uint64_t)1 << n_sites;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)size; ++i) table[i] = 0xFFFFFFFFu;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)dim; ++t) table[basis[t]] = (uint32_t)t;
}

/* H.x as orc_hv, with row labels from the stored basis and partner indices
 * read from the full lookup table. */
void orc_hv_table(int n_sites, int n_up, int n_bonds, const int32_t* bi, const int32_t* bj,
                  const double* J, const uint64_t* basis, const uint32_t* table, const double* x,
                  double* y, uint64_t row0, uint64_t nrows) {
    (void)n_sites;
    (void)n_up;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t r = 0; r < (int64_t)nrows; ++r) {
        uint64_t t = row0 + (uint64_t)r;
        uint64_t n = basis[t];
        double acc = 0.0;
        for (int b = 0; b < n_bonds; ++b) {
            int up_i = (int)((n >> bi[b]) & 1u), up_j = (int)((n >> bj[b]) & 1u);
            double mi = up_i ? 0.5 : -0.5, mj = up_j ? 0.5 : -0.5;
            acc += J[b] * mi * mj * x[t];
            if (up_i != up_j) {
                uint64_t partner = n ^ (((uint64_t)1 << bi[b]) | ((uint64_t)1 << bj[b]));
                acc += 0.5 * J[b] * x[table[partner]];
            }
        }
        y[r] = acc;
    }
}

/* Rows of H.x where x is the (unnormalized) start vector of sample r, each
 * entry generated from its stream on demand, so no vector of the full
 * sector is needed: y[k] = row rows[k] of H.x. For sectors too large to hold
 * on the host (N = 34: 2.3e9 entries). */
static double stream_entry(uint64_t key, uint64_t r, int dist, uint64_t i) {
    const double two_pi = 2.0 * 3.141592653589793;
    if (dist == 0) return (mix64(key + (i + 1) * GAMMA) >> 63) ? -1.0 : 1.0;
    if (dist == 1) {
        uint64_t u1 = mix64(key + (2 * i + 1) * GAMMA);
        uint64_t u2 = mix64(key + (2 * i + 2) * GAMMA);
        double a = (double)((u1 >> 11) + 1) * 0x1.0p-53;
        double b = (double)(u2 >> 11) * 0x1.0p-53;
        return sqrt(-2.0 * log(a)) * cos(two_pi * b);
    }
    return (i == r) ? 1.0 : 0.0;
}

void orc_hv_rows_stream(int n_sites, int n_up, int n_bonds, const int32_t* bi, const int32_t* bj,
                        const double* J, uint64_t seed, uint64_t r, int dist, const uint64_t* rows,
                        uint64_t nrows, double* y) {
    uint64_t key = orc_stream_key(seed, n_up, r);
#pragma omp parallel for schedule(dynamic, 64) if (nrows > 256)
    for (int64_t k = 0; k < (int64_t)nrows; ++k) {
        uint64_t t = rows[k];
        uint64_t n = orc_unrank(n_sites, n_up, t);
        double xt = stream_entry(key, r, dist, t);
        double acc = 0.0;
        for (int b = 0; b < n_bonds; ++b) {
            int up_i = (int)((n >> bi[b]) & 1u), up_j = (int)((n >> bj[b]) & 1u);
            double mi = up_i ? 0.5 : -0.5, mj = up_j ? 0.5 : -0.5;
            acc += J[b] * mi * mj * xt;
            if (up_i != up_j) {
                uint64_t partner = n ^ (((uint64_t)1 << bi[b]) | ((uint64_t)1 << bj[b]));
                acc += 0.5 * J[b] * stream_entry(key, r, dist, orc_rank(n_sites, n_up, partner));
            }
        }
        y[k] = acc;
    }
}

/* Next sector label after x in ascending order: the smallest integer above x
 * with the same number of set bits. With c the lowest set bit of x, adding c
 * carries the lowest run of ones one place up; the ones the carry removed,
 * less one, go back to the bottom. */
static uint64_t next_label(uint64_t x) {
    uint64_t c = x & (~x + 1);
    uint64_t r = x + c;
    return r | (((x ^ r) >> 2) / c);
}

/* First-step moments of the start vectors of samples r0 .. r0 + R - 1 over
 * the whole sector, with every entry generated on demand (no stored vector):
 * out[3 r] = <x|x>, out[3 r + 1] = <x|H|x>, out[3 r + 2] = <Hx|Hx> for the
 * unnormalized x of sample r0 + r. For the normalized start vector these give
 * alpha_1 = <x|H|x> / <x|x> and alpha_1^2 + beta_1^2 = <Hx|Hx> / <x|x> (the
 * first Lanczos step, Sec. 2). Rows are walked in chunks of 2^16 in
 * ascending label order; each chunk's sums are added in chunk order, so the
 * result does not depend on the thread count. 1 <= R <= 8. */
void orc_moments_stream(int n_sites, int n_up, int n_bonds, const int32_t* bi, const int32_t* bj,
                        const double* J, uint64_t seed, uint64_t r0, int R, int dist, double* out) {
    const uint64_t dim = orc_sector_dim(n_sites, n_up);
    const uint64_t chunk = (uint64_t)1 << 16;
    const uint64_t nchunks = (dim + chunk - 1) / chunk;
    uint64_t key[8];
    for (int r = 0; r < R; ++r) key[r] = orc_stream_key(seed, n_up, r0 + (uint64_t)r);
    double* part = (double*)calloc((size_t)nchunks * 3 * (size_t)R, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ci = 0; ci < (int64_t)nchunks; ++ci) {
        uint64_t t0 = (uint64_t)ci * chunk;
        uint64_t t1 = t0 + chunk < dim ? t0 + chunk : dim;
        uint64_t n = orc_unrank(n_sites, n_up, t0);
        double* p = part + (size_t)ci * 3 * (size_t)R;
        for (uint64_t t = t0; t < t1; ++t) {
            double xt[8], y[8];
            for (int r = 0; r < R; ++r) {
                xt[r] = stream_entry(key[r], r0 + (uint64_t)r, dist, t);
                y[r] = 0.0;
            }
            for (int b = 0; b < n_bonds; ++b) {
                int up_i = (int)((n >> bi[b]) & 1u), up_j = (int)((n >> bj[b]) & 1u);
                double mi = up_i ? 0.5 : -0.5, mj = up_j ? 0.5 : -0.5;
                for (int r = 0; r < R; ++r) y[r] += J[b] * mi * mj * xt[r];
                if (up_i != up_j) {
                    uint64_t partner = n ^ (((uint64_t)1 << bi[b]) | ((uint64_t)1 << bj[b]));
                    uint64_t idx = orc_rank(n_sites, n_up, partner);
                    for (int r = 0; r < R; ++r)
                        y[r] += 0.5 * J[b] * stream_entry(key[r], r0 + (uint64_t)r, dist, idx);
                }
            }
            for (int r = 0; r < R; ++r) {
                p[3 * r] += xt[r] * xt[r];
                p[3 * r + 1] += xt[r] * y[r];
                p[3 * r + 2] += y[r] * y[r];
            }
            if (t + 1 < t1) n = next_label(n);
        }
    }
    for (int k = 0; k < 3 * R; ++k) out[k] = 0.0;
    for (uint64_t ci = 0; ci < nchunks; ++ci)
        for (int k = 0; k < 3 * R; ++k) out[k] += part[ci * 3 * (uint64_t)R + (uint64_t)k];
    free(part);
}

/* Thread count of the oracle's OpenMP loops (for timing it at 1 thread and
 * at all cores); returns the count now in force. */
#include <omp.h>
int orc_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
