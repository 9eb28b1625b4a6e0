/*
 * FP64 CPU oracle for the general-spin Heisenberg H.x (local spin s = 1/2,
 * 1, 3/2, ...; paper Sec. 2, Eqs. 10-17).
 *
 * TEST INFRASTRUCTURE ONLY, like ftlm_oracle.c: nothing in the product
 * library links, includes or calls this file. Every quantity is computed
 * from its plain definition, for obviousness rather than speed.
 *
 * Conventions (Eq. 11): with d = 2s + 1, a basis state of N sites is the
 * integer n = sum_k a_k d^k whose base-d digit a_k = m_k + s is the shifted
 * S^z quantum number of site k. The sector with total digit sum A holds
 * every such n with a_0 + ... + a_{N-1} = A (S^z = M = A - N s, Eq. 17),
 * ordered by increasing label. two_s = 2s = d - 1 throughout. An index of a
 * label outside the sector is UINT64_MAX.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define SPN_NONE UINT64_MAX

/* Digit sum of label n in base d over N digits. */
static int digit_sum(uint64_t n, int n_sites, int d) {
    int s = 0;
    for (int k = 0; k < n_sites; ++k) {
        s += (int)(n % (uint64_t)d);
        n /= (uint64_t)d;
    }
    return s;
}

static uint64_t ipow(uint64_t b, int e) {
    uint64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

/* D(m, A): number of length-m digit strings over {0..2s} with digit sum A,
 * from the recursion of Eq. (15), D(m, A) = sum_{q=0}^{2s} D(m-1, A-q),
 * D(0, 0) = 1 and D = 0 outside the allowed range. */
uint64_t spn_dim(int m, int two_s, int A) {
    if (m < 0 || A < 0 || A > m * two_s) return 0;
    if (m == 0) return A == 0 ? 1 : 0;
    uint64_t* row = calloc((size_t)(m * two_s + 1), sizeof(uint64_t));
    uint64_t* nxt = calloc((size_t)(m * two_s + 1), sizeof(uint64_t));
    row[0] = 1;
    for (int len = 1; len <= m; ++len) {
        for (int a = 0; a <= len * two_s; ++a) {
            uint64_t c = 0;
            for (int q = 0; q <= two_s && q <= a; ++q) c += row[a - q];
            nxt[a] = c;
        }
        for (int a = 0; a <= len * two_s; ++a) row[a] = nxt[a];
    }
    uint64_t r = row[A];
    free(row);
    free(nxt);
    return r;
}

/* Every label of [0, d^N) with digit sum A, ascending. Returns the count
 * (the labels are written while it stays below cap). */
int64_t spn_enumerate(int n_sites, int two_s, int A, uint64_t* out, uint64_t cap) {
    const int d = two_s + 1;
    const uint64_t total = ipow((uint64_t)d, n_sites);
    uint64_t c = 0;
    for (uint64_t n = 0; n < total; ++n) {
        if (digit_sum(n, n_sites, d) == A) {
            if (c < cap) out[c] = n;
            ++c;
        }
    }
    return (int64_t)c;
}

/* Index of label x in the sorted basis (binary search), SPN_NONE if absent. */
uint64_t spn_rank(const uint64_t* basis, uint64_t dim, uint64_t x) {
    uint64_t lo = 0, hi = dim;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (basis[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return (lo < dim && basis[lo] == x) ? lo : SPN_NONE;
}

/* Digit a_k of label n (Eq. 11). */
static int digit(uint64_t n, int k, int d) {
    for (int i = 0; i < k; ++i) n /= (uint64_t)d;
    return (int)(n % (uint64_t)d);
}

/* sqrt(s(s+1) - m(m+1)) with s = two_s / 2: the matrix element of S^+ from
 * S^z = m (zero at m = s). */
static double ladder_up(int two_s, double m) {
    const double s = 0.5 * two_s;
    const double v = s * (s + 1.0) - m * (m + 1.0);
    return v > 0.0 ? sqrt(v) : 0.0;
}

/* Rows [row0, row0 + nrows) of y = H x in the sector with digit sum A,
 * H = sum_b J_b (S_i^z S_j^z + (S_i^+ S_j^- + S_i^- S_j^+) / 2). Row t with
 * label n: y_t = sum_b J_b m_i m_j x_t + sum_b [c+ x(n+) + c- x(n-)], where
 * n+ has a_i - 1, a_j + 1 (so that S_i^+ S_j^- maps n+ to n) and n- the
 * reverse, with the coefficients of Eqs. (13) and (14): the matrix elements
 * <n| S_i^+ S_j^- |n+> and <n| S_i^- S_j^+ |n->. */
void spn_hv(int n_sites, int two_s, int n_bonds, const int32_t* bi, const int32_t* bj, const double* J,
            const uint64_t* basis, uint64_t dim, const double* x, double* y, uint64_t row0, uint64_t nrows) {
    (void)n_sites;  /* the labels carry every digit */
    const int d = two_s + 1;
    const double s = 0.5 * two_s;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < (int64_t)nrows; ++r) {
        const uint64_t t = row0 + (uint64_t)r;
        const uint64_t n = basis[t];
        double acc = 0.0, diag = 0.0;
        for (int b = 0; b < n_bonds; ++b) {
            const int i = bi[b], j = bj[b];
            const int ai = digit(n, i, d), aj = digit(n, j, d);
            const double mi = ai - s, mj = aj - s;
            diag += J[b] * mi * mj;
            const uint64_t di = ipow((uint64_t)d, i), dj = ipow((uint64_t)d, j);
            /* n+: a_i - 1, a_j + 1 */
            if (ai >= 1 && aj <= two_s - 1) {
                const uint64_t src = n - di + dj;
                /* <n| S_i^+ S_j^- |src> = up(m_i - 1) * up(m_j) (S^- from m_j + 1) */
                const double c = 0.5 * J[b] * ladder_up(two_s, mi - 1.0) * ladder_up(two_s, mj);
                const uint64_t k = spn_rank(basis, dim, src);
                if (k != SPN_NONE) acc += c * x[k];
            }
            /* n-: a_i + 1, a_j - 1 */
            if (ai <= two_s - 1 && aj >= 1) {
                const uint64_t src = n + di - dj;
                const double c = 0.5 * J[b] * ladder_up(two_s, mi) * ladder_up(two_s, mj - 1.0);
                const uint64_t k = spn_rank(basis, dim, src);
                if (k != SPN_NONE) acc += c * x[k];
            }
        }
        y[r] = diag * x[t] + acc;
    }
}

/* Off-diagonal entries of H in the sector with digit sum A: the number of
 * (row, bond, ladder term) with a valid source state, counted over every
 * label of [0, d^N) without storing the basis. Together with the D diagonal
 * entries this is N_nz of Eq. (10) and Table 1. */
uint64_t spn_offdiag_count(int n_sites, int two_s, int A, int n_bonds, const int32_t* bi, const int32_t* bj) {
    const int d = two_s + 1;
    const uint64_t total = ipow((uint64_t)d, n_sites);
    uint64_t count = 0;
#pragma omp parallel for reduction(+ : count) schedule(static, 1 << 16)
    for (int64_t n = 0; n < (int64_t)total; ++n) {
        if (digit_sum((uint64_t)n, n_sites, d) != A) continue;
        for (int b = 0; b < n_bonds; ++b) {
            const int ai = digit((uint64_t)n, bi[b], d), aj = digit((uint64_t)n, bj[b], d);
            if (ai >= 1 && aj <= two_s - 1) ++count;
            if (ai <= two_s - 1 && aj >= 1) ++count;
        }
    }
    return count;
}

/* For rows [t0, t0 + count) and each bond b = (i, j) with i < j: out[(t - t0)
 * * 2 N_B + 2 b] = index of the state with a_i + 1, a_j - 1 and out[... + 2 b
 * + 1] = index of the state with a_i - 1, a_j + 1 (the two ladder terms of
 * Eq. 12), SPN_NONE where a digit would leave [0, 2s]. */
void spn_neighbors(int two_s, int n_bonds, const int32_t* bi, const int32_t* bj, const uint64_t* basis,
                   uint64_t dim, uint64_t t0, uint64_t count, uint64_t* out) {
    const int d = two_s + 1;
    for (uint64_t r = 0; r < count; ++r) {
        const uint64_t n = basis[t0 + r];
        for (int b = 0; b < n_bonds; ++b) {
            const int i = bi[b] < bj[b] ? bi[b] : bj[b], j = bi[b] < bj[b] ? bj[b] : bi[b];
            const int ai = digit(n, i, d), aj = digit(n, j, d);
            const uint64_t di = ipow((uint64_t)d, i), dj = ipow((uint64_t)d, j);
            uint64_t* o = out + r * (uint64_t)(2 * n_bonds) + 2 * (uint64_t)b;
            o[0] = (ai < two_s && aj > 0) ? spn_rank(basis, dim, n + di - dj) : SPN_NONE;
            o[1] = (ai > 0 && aj < two_s) ? spn_rank(basis, dim, n - di + dj) : SPN_NONE;
        }
    }
}

/* ---- ranks by counting (no stored basis) --------------------------------
 * For sectors too large to enumerate in a test: the index of a label is the
 * number of sector labels below it, counted with the dimensions D(m, A) of
 * Eq. (15). Labels compare as integers, i.e. digit strings from the top
 * digit down: a sector label y < x first differs from x at some digit k with
 * y_k < x_k and equal digits above it, and its k lower digits are any string
 * whose digit sum makes up the rest of A. */

/* D(m, a) for m = 0..N and a = 0..N 2s, row m at t[m * (N 2s + 1)]. */
static uint64_t* spn_dim_table(int n_sites, int two_s) {
    const int w = n_sites * two_s + 1;
    uint64_t* t = calloc((size_t)(n_sites + 1) * (size_t)w, sizeof(uint64_t));
    t[0] = 1;
    for (int m = 1; m <= n_sites; ++m)
        for (int a = 0; a <= m * two_s; ++a) {
            uint64_t c = 0;
            for (int q = 0; q <= two_s && q <= a; ++q) c += t[(size_t)(m - 1) * w + (size_t)(a - q)];
            t[(size_t)m * w + (size_t)a] = c;
        }
    return t;
}

static uint64_t dim_at(const uint64_t* t, int n_sites, int two_s, int m, int a) {
    if (a < 0 || a > m * two_s) return 0;
    return t[(size_t)m * (size_t)(n_sites * two_s + 1) + (size_t)a];
}

static uint64_t rank_count(const uint64_t* t, int n_sites, int two_s, int A, uint64_t x) {
    const int d = two_s + 1;
    if (x >= ipow((uint64_t)d, n_sites) || digit_sum(x, n_sites, d) != A) return SPN_NONE;
    uint64_t idx = 0;
    int rem = A;  /* digit sum left for digits k, k - 1, ..., 0 */
    for (int k = n_sites - 1; k >= 0; --k) {
        const int ak = digit(x, k, d);
        for (int q = 0; q < ak; ++q) idx += dim_at(t, n_sites, two_s, k, rem - q);
        rem -= ak;
    }
    return idx;
}

static uint64_t unrank_count(const uint64_t* t, int n_sites, int two_s, int A, uint64_t idx) {
    const int d = two_s + 1;
    uint64_t label = 0;
    int rem = A;
    for (int k = n_sites - 1; k >= 0; --k) {
        int q = 0;
        for (; q <= two_s; ++q) {
            const uint64_t c = dim_at(t, n_sites, two_s, k, rem - q);
            if (idx < c) break;
            idx -= c;
        }
        label += (uint64_t)q * ipow((uint64_t)d, k);
        rem -= q;
    }
    return label;
}

/* out[i] = index of labels[i] by counting (SPN_NONE outside the sector). */
void spn_rank_count(int n_sites, int two_s, int A, const uint64_t* labels, uint64_t n, uint64_t* out) {
    uint64_t* t = spn_dim_table(n_sites, two_s);
    for (uint64_t i = 0; i < n; ++i) out[i] = rank_count(t, n_sites, two_s, A, labels[i]);
    free(t);
}

/* out[i] = label of sector index idx[i] (idx[i] < D). */
void spn_unrank_count(int n_sites, int two_s, int A, const uint64_t* idx, uint64_t n, uint64_t* out) {
    uint64_t* t = spn_dim_table(n_sites, two_s);
    for (uint64_t i = 0; i < n; ++i) out[i] = unrank_count(t, n_sites, two_s, A, idx[i]);
    free(t);
}

/* y[i] = row rows[i] of H x (the sum of spn_hv, term for term in the same
 * order), the row's label and its partners' indices found by counting. */
void spn_hv_rows(int n_sites, int two_s, int A, int n_bonds, const int32_t* bi, const int32_t* bj,
                 const double* J, const double* x, const uint64_t* rows, uint64_t count, double* y) {
    const int d = two_s + 1;
    const double s = 0.5 * two_s;
    uint64_t* tab = spn_dim_table(n_sites, two_s);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < (int64_t)count; ++r) {
        const uint64_t t = rows[r];
        const uint64_t n = unrank_count(tab, n_sites, two_s, A, t);
        double acc = 0.0, diag = 0.0;
        for (int b = 0; b < n_bonds; ++b) {
            const int i = bi[b], j = bj[b];
            const int ai = digit(n, i, d), aj = digit(n, j, d);
            const double mi = ai - s, mj = aj - s;
            diag += J[b] * mi * mj;
            const uint64_t di = ipow((uint64_t)d, i), dj = ipow((uint64_t)d, j);
            if (ai >= 1 && aj <= two_s - 1) {
                const double c = 0.5 * J[b] * ladder_up(two_s, mi - 1.0) * ladder_up(two_s, mj);
                const uint64_t k = rank_count(tab, n_sites, two_s, A, n - di + dj);
                if (k != SPN_NONE) acc += c * x[k];
            }
            if (ai <= two_s - 1 && aj >= 1) {
                const double c = 0.5 * J[b] * ladder_up(two_s, mi) * ladder_up(two_s, mj - 1.0);
                const uint64_t k = rank_count(tab, n_sites, two_s, A, n + di - dj);
                if (k != SPN_NONE) acc += c * x[k];
            }
        }
        y[r] = diag * x[t] + acc;
    }
    free(tab);
}
