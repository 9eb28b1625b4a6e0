// Host FP64 parts of the FTLM path: the Ritz decomposition of the Lanczos
// tridiagonal matrix and the thermal reduction (paper Sec. 2: the small
// tridiagonal problem is solved on the host in FP64; Eqs. 4-9).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <system_error>
#include <thread>
#include <vector>

#include "host_math.hpp"

namespace ftlm {

namespace {

// sqrt(a^2 + b^2): the plain formula where it can neither overflow nor lose
// precision to underflow, std::hypot (several times slower) elsewhere.
inline double givens_norm(double a, double b) {
    const double x = std::fabs(a), y = std::fabs(b);
    const double big = x > y ? x : y;
    if (big > 1e-150 && big < 1e150) return std::sqrt(a * a + b * b);
    return std::hypot(a, b);
}

// Calls f(i) for i in [0, n), split into contiguous ranges over up to
// `threads` host threads (the calling one included). Every index is handled
// by one thread alone, so results do not depend on the split; a thread that
// cannot be started leaves its range to the caller.
template <typename F>
void parallel_for(int n, int threads, F&& f) {
    threads = std::max(1, std::min(threads, n));
    const int per = threads > 1 ? (n + threads - 1) / threads : n;
    std::vector<std::thread> pool;
    std::vector<std::pair<int, int>> left;
    for (int t = 1; t < threads; ++t) {
        const int b = t * per, e = std::min(n, b + per);
        if (b >= e) break;
        try {
            pool.emplace_back([&f, b, e] {
                for (int i = b; i < e; ++i) f(i);
            });
        } catch (const std::system_error&) {
            left.emplace_back(b, e);
        }
    }
    for (int i = 0; i < std::min(n, per); ++i) f(i);
    for (auto [b, e] : left)
        for (int i = b; i < e; ++i) f(i);
    for (auto& th : pool) th.join();
}

// Host threads for `work` elementary steps: one below about a millisecond of
// work (thread start-up would dominate), else up to 16.
int host_threads(double work) {
    if (work < 2e5) return 1;
    const unsigned hw = std::thread::hardware_concurrency();
    return int(std::min(16u, hw ? hw : 1u));
}

}  // namespace

// Implicit-shift QL iteration on the symmetric tridiagonal matrix with
// diagonal d[0..m-1] and off-diagonal e[i] coupling rows i and i+1. Each
// sweep applies Givens rotations from the bottom of the unreduced block
// [l, k] upwards (QL factorization of T - sigma I with the shift sigma taken
// from the eigenvalue of the leading 2x2 block nearer to d[l]), so the
// eigenvalue d[l] converges first. The rotations are also applied to the
// first row of the accumulated eigenvector matrix, which is all FTLM needs:
// w_k = (first component of eigenvector k)^2.
int ritz_ql(int m, const double* alpha, const double* beta, double* theta, double* weight) {
    std::vector<double> d(alpha, alpha + m), e(size_t(m), 0.0), z(size_t(m), 0.0);
    for (int i = 0; i + 1 < m; ++i) e[size_t(i)] = beta[i];
    z[0] = 1.0;
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < m; ++l) {
        for (int iter = 0;; ++iter) {
            int k = l;
            while (k < m - 1 && std::fabs(e[size_t(k)]) > eps * (std::fabs(d[size_t(k)]) + std::fabs(d[size_t(k + 1)])))
                ++k;
            if (k == l) break;
            if (iter >= 200) return -1;
            // shift toward d[l] from the leading 2x2 block
            double g = (d[size_t(l + 1)] - d[size_t(l)]) / (2.0 * e[size_t(l)]);
            double r = givens_norm(g, 1.0);
            g = d[size_t(k)] - d[size_t(l)] + e[size_t(l)] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool deflated = false;
            for (int i = k - 1; i >= l; --i) {
                const double f = s * e[size_t(i)], b = c * e[size_t(i)];
                r = givens_norm(f, g);
                e[size_t(i + 1)] = r;
                if (r == 0.0) {  // the block split: finish this sweep early
                    d[size_t(i + 1)] -= p;
                    e[size_t(k)] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[size_t(i + 1)] - p;
                r = (d[size_t(i)] - g) * s + 2.0 * c * b;
                p = s * r;
                d[size_t(i + 1)] = g + p;
                g = c * r - b;
                const double zi = z[size_t(i)], zn = z[size_t(i + 1)];
                z[size_t(i + 1)] = s * zi + c * zn;
                z[size_t(i)] = c * zi - s * zn;
            }
            if (deflated) continue;
            d[size_t(l)] -= p;
            e[size_t(l)] = g;
            e[size_t(k)] = 0.0;
        }
    }
    std::vector<int> order(static_cast<size_t>(m));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[size_t(a)] < d[size_t(b)]; });
    for (int i = 0; i < m; ++i) {
        theta[i] = d[size_t(order[size_t(i)])];
        const double zi = z[size_t(order[size_t(i)])];
        weight[i] = zi * zi;
    }
    return 0;
}

int ritz_batch(int n, int stride, const int32_t* m, const double* alpha, const double* beta, double* theta,
               double* weight) {
    std::atomic<int> failed{0};
    double work = 0.0;
    for (int r = 0; r < n; ++r) work += double(m[r]) * double(m[r]);
    parallel_for(n, host_threads(4.0 * work), [&](int r) {
        const size_t o = size_t(r) * size_t(stride);
        const int k = m[r];
        if (ritz_ql(k, alpha + o, beta + o, theta + o, weight + o) != 0) failed.store(1);
        for (int j = k; j < stride; ++j) theta[o + size_t(j)] = weight[o + size_t(j)] = 0.0;
    });
    return failed.load() ? -1 : 0;
}

// Cullum-Willoughby ghost test (Sec. 3.2, Eq. 25) of one chain: the Ritz
// values of T, the eigenvalues of T1 (T without its first row and column),
// the deflation distance of every Ritz value to the nearest eigenvalue of
// T1, the flag ell_k < tau with tau = c_tau * u * (theta_max - theta_min),
// and clusters of Ritz values joined along the sorted spectrum wherever two
// neighbours lie within tau, with their total weights.
int ghost_test(int m, const double* alpha, const double* beta, double c_tau, double u, double* theta,
               double* weight, double* ell, int32_t* ghost, int32_t* cluster, double* cluster_weight,
               int32_t* n_clusters, double* tau) {
    if (ritz_ql(m, alpha, beta, theta, weight) != 0) return -1;
    std::vector<double> t1(size_t(m > 1 ? m - 1 : 1)), w1(t1.size());
    if (m > 1 && ritz_ql(m - 1, alpha + 1, beta + 1, t1.data(), w1.data()) != 0) return -1;
    const double tol = c_tau * u * (theta[m - 1] - theta[0]);
    for (int k = 0; k < m; ++k) {
        double best = INFINITY;
        if (m > 1) {
            // t1 is ascending: the nearest value is at or just below the insertion point
            const auto it = std::lower_bound(t1.begin(), t1.begin() + (m - 1), theta[k]);
            if (it != t1.begin() + (m - 1)) best = std::fabs(*it - theta[k]);
            if (it != t1.begin()) best = std::min(best, std::fabs(*(it - 1) - theta[k]));
        }
        ell[k] = best;
        ghost[k] = best < tol ? 1 : 0;
    }
    int c = 0;
    for (int k = 0; k < m; ++k) {
        if (k > 0 && theta[k] - theta[k - 1] > tol) ++c;
        cluster[k] = c;
    }
    for (int k = 0; k < m; ++k) cluster_weight[k] = 0.0;
    for (int k = 0; k < m; ++k) cluster_weight[cluster[k]] += weight[k];
    *n_clusters = c + 1;
    *tau = tol;
    return 0;
}

// Spread over seeds of Eq. (22): per column j of [n_seeds][n] values, the mean
// and sigma = sqrt((1/N_s) sum_s (v_sj - mean_j)^2), summed in seed order.
void seed_spread(int n_seeds, int n, const double* v, double* mean, double* sigma) {
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int r = 0; r < n_seeds; ++r) s += v[size_t(r) * size_t(n) + size_t(j)];
        const double mu = s / double(n_seeds);
        double q = 0.0;
        for (int r = 0; r < n_seeds; ++r) {
            const double d = v[size_t(r) * size_t(n) + size_t(j)] - mu;
            q += d * d;
        }
        mean[j] = mu;
        sigma[j] = std::sqrt(q / double(n_seeds));
    }
}

// FTLM thermal reduction (Eqs. 6-9). Per sector the estimator weighs each
// sample's Gauss-quadrature sum by mult * D / R; Boltzmann factors use
// theta - E0 with E0 the smallest Ritz value of all samples, which cancels in
// every ratio and keeps the exponentials in range.
int thermo(int n_sites, int n_sectors, const SectorSamples* sec, int nT, const double* T,
           double g, double* E, double* C, double* chi, double* lnZ) {
    double e0 = INFINITY;
    for (int s = 0; s < n_sectors; ++s)
        for (int r = 0; r < sec[s].R; ++r)
            for (int k = 0; k < sec[s].steps[r]; ++k)
                e0 = std::min(e0, sec[s].theta[size_t(r) * size_t(sec[s].stride) + size_t(k)]);
    if (!std::isfinite(e0)) return -1;
    double work = 0.0;
    for (int s = 0; s < n_sectors; ++s)
        for (int r = 0; r < sec[s].R; ++r) work += double(sec[s].steps[r]);
    // temperatures are independent: each is summed by one thread, in the
    // same order whatever the split
    parallel_for(nT, host_threads(work * double(nT)), [&](int it) {
        const double beta = 1.0 / T[it];
        double z = 0.0, h1 = 0.0, h2 = 0.0, zm2 = 0.0;
        for (int s = 0; s < n_sectors; ++s) {
            const SectorSamples& q = sec[s];
            const double pref = q.mult * double(q.dim) / double(q.R);
            const double mz = double(q.n_up) - 0.5 * double(n_sites) * double(q.two_s);  // M = A - N s
            double zs = 0.0, a1 = 0.0, a2 = 0.0;
            for (int r = 0; r < q.R; ++r) {
                const double* th = q.theta + size_t(r) * size_t(q.stride);
                const double* w = q.weight + size_t(r) * size_t(q.stride);
                for (int k = 0; k < q.steps[r]; ++k) {
                    const double x = th[k] - e0;
                    const double bw = w[k] * std::exp(-beta * x);
                    zs += bw;
                    a1 += bw * x;
                    a2 += bw * x * x;
                }
            }
            z += pref * zs;
            h1 += pref * a1;
            h2 += pref * a2;
            zm2 += mz * mz * pref * zs;
        }
        const double mean = h1 / z;
        if (E) E[it] = e0 + mean;
        if (C) C[it] = beta * beta * (h2 / z - mean * mean);
        if (chi) chi[it] = g * g * beta * zm2 / z;
        if (lnZ) lnZ[it] = std::log(z) - beta * e0;
    });
    return 0;
}

}  // namespace ftlm
