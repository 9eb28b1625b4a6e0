// Kernel bond tables (host side): the merged bonds of a graph sorted for the
// row kernels, with the coefficients J_b / 2 of the flip terms (Eqs. 13-14 at
// s = 1/2) and the diagonal offset sum_b J_b / 4.
#include <algorithm>
#include <cstring>

#include "host.hpp"

namespace ftlm {

BondTable make_bond_table(int n_sites, const std::vector<int>& lo, const std::vector<int>& hi,
                          const std::vector<double>& J, const std::vector<int>& orig, double jsum_all) {
    const int nb = int(lo.size());
    std::vector<int> order(static_cast<size_t>(nb));
    for (int b = 0; b < nb; ++b) order[size_t(b)] = b;
    // sorted by the lower site, highest first (the combinatorial-ranking pass
    // walks the sites from the top and meets a bond at its lower site)
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        if (lo[size_t(a)] != lo[size_t(c)]) return lo[size_t(a)] > lo[size_t(c)];
        return hi[size_t(a)] > hi[size_t(c)];
    });
    BondTable T;
    std::memset(&T, 0, sizeof(T));
    T.n_bonds = nb;
    T.n_sites = n_sites;
    for (int k = 0; k < nb; ++k) {
        const size_t b = size_t(order[size_t(k)]);
        T.pack[k] = uint32_t(lo[b]) | (uint32_t(hi[b]) << 8) | (uint32_t(orig[b]) << 16);
        T.coef_d[k] = 0.5 * J[b];
        T.coef_f[k] = float(0.5 * J[b]);
    }
    for (int p = 0; p <= kMaxSites; ++p) {
        int c = 0;
        for (int k = 0; k < nb; ++k) c += (int(T.pack[k] & 0xffu) >= p) ? 1 : 0;
        T.ends[p] = uint32_t(p < n_sites ? c : 0);
    }
    T.jsum4_d = 0.25 * jsum_all;
    T.jsum4_f = float(0.25 * jsum_all);
    return T;
}

}  // namespace ftlm
