// Kernel bond tables and the two-pass site split of a graph (host side).
//
// A row-wise gather H.x reads, for every row, the partner rows of its
// antiparallel bonds. With the sector in increasing-label order, a bond
// between low sites keeps the partner near the row, while a bond touching a
// high site sends it far away, so a single pass over the rows re-reads x from
// HBM once per high-site bond class. The split labels the sites as
// [0, c) | [c, s) | [s, N) so that every bond lies inside [0, s) or joins
// [s, N) to [0, c) or to itself. The first pass takes the bonds inside
// [0, s) over rows in index order (a run of rows with equal digits on [s, N)
// holds all their partners); the second pass takes the others over blocks of
// rows with equal digits on [c, s) (again closed under those bonds). Both
// kinds of block hold at most C(s, s/2) and C(N - s + c, (N - s + c)/2) rows,
// which bounds how far a pass reaches for its partners. Measured on gfx950 at
// N = 30 the pair of passes is slower than one pass: the time follows the
// number of scattered row fetches (the same in both forms), not the HBM
// re-reads the split removes, and the second pass's rows come in short runs.
// The split is therefore opt-in (ftlm_set_split_policy).
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

namespace {

// Largest block of a split, in rows (over all sectors of N sites).
uint64_t split_score(int n_sites, int c, int s) {
    const int p = n_sites - s + c;
    return std::max(binom_u64(s, s / 2), binom_u64(p, p / 2));
}

// The best split of the sites as labelled: for each s the smallest c with
// every bond touching [s, N) starting in [0, c) or [s, N).
bool best_split_as_labelled(int n_sites, const std::vector<int>& lo, const std::vector<int>& hi, int& c_out,
                            int& s_out, uint64_t& score_out) {
    bool found = false;
    for (int s = 2; s < n_sites; ++s) {
        int c = 0;
        for (size_t b = 0; b < lo.size(); ++b)
            if (hi[b] >= s && lo[b] < s) c = std::max(c, lo[b] + 1);
        if (c >= s) continue;
        const uint64_t sc = split_score(n_sites, c, s);
        if (!found || sc < score_out) {
            found = true;
            score_out = sc;
            c_out = c;
            s_out = s;
        }
    }
    return found;
}

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

}  // namespace

// Chooses the split order of g's sites and fills the split bond tables.
// Candidates: the caller's labelling as it stands, and for every start site a
// greedy growth of the top set T (each step adds the site that leaves the
// smallest vertex boundary, lowest site first on ties), relabelled as
// boundary of T | other sites | T. The caller's labelling wins ties.
void plan_split(ftlm_graph* g) {
    const int N = g->n_sites;
    const size_t nb = g->bi.size();
    g->split = false;
    g->split_identity = true;
    g->split_site.assign(size_t(N), 0);
    g->user_site.assign(size_t(N), 0);
    for (int k = 0; k < N; ++k) g->split_site[size_t(k)] = g->user_site[size_t(k)] = k;
    if (N < 8) return;

    int best_c = 0, best_s = 0;
    uint64_t best = 0;
    bool have = best_split_as_labelled(N, g->bi, g->bj, best_c, best_s, best);
    std::vector<int> best_order;  // empty: the caller's labelling

    std::vector<uint64_t> adj(size_t(N), 0);
    for (size_t b = 0; b < nb; ++b) {
        adj[size_t(g->bi[b])] |= uint64_t(1) << g->bj[b];
        adj[size_t(g->bj[b])] |= uint64_t(1) << g->bi[b];
    }
    const uint64_t all = N == 64 ? ~uint64_t(0) : ((uint64_t(1) << N) - 1);
    auto boundary = [&](uint64_t T) {
        uint64_t nbr = 0;
        for (int v = 0; v < N; ++v)
            if ((T >> v) & 1) nbr |= adj[size_t(v)];
        return nbr & ~T & all;
    };
    for (int v0 = 0; v0 < N; ++v0) {
        uint64_t T = uint64_t(1) << v0;
        while (popcount64(T) <= N - 2) {
            const uint64_t bd = boundary(T);
            const int k = popcount64(T), c = popcount64(bd), s = N - k;
            if (c < s) {
                const uint64_t sc = split_score(N, c, s);
                if (!have || sc < best) {
                    have = true;
                    best = sc;
                    best_c = c;
                    best_s = s;
                    best_order.assign(size_t(N), -1);
                    int next = 0;
                    for (int u = 0; u < N; ++u)
                        if ((bd >> u) & 1) best_order[size_t(u)] = next++;
                    for (int u = 0; u < N; ++u)
                        if (!((bd >> u) & 1) && !((T >> u) & 1)) best_order[size_t(u)] = next++;
                    for (int u = 0; u < N; ++u)
                        if ((T >> u) & 1) best_order[size_t(u)] = next++;
                }
            }
            const uint64_t cand = bd ? bd : (all & ~T);
            int pick = -1, pick_b = 0;
            for (int u = 0; u < N; ++u) {
                if (!((cand >> u) & 1)) continue;
                const int b = popcount64(boundary(T | (uint64_t(1) << u)));
                if (pick < 0 || b < pick_b) {
                    pick = u;
                    pick_b = b;
                }
            }
            T |= uint64_t(1) << pick;
        }
    }
    // worth it only when a block is a small part of the largest sector
    if (!have || best * 4 > binom_u64(N, N / 2)) return;

    if (!best_order.empty()) {
        g->split_identity = false;
        for (int u = 0; u < N; ++u) {
            g->split_site[size_t(u)] = best_order[size_t(u)];
            g->user_site[size_t(best_order[size_t(u)])] = u;
        }
    }
    std::vector<int> lo1, hi1, o1, lo2, hi2, o2;
    std::vector<double> J1, J2;
    double jsum = 0.0;
    for (size_t b = 0; b < nb; ++b) {
        int i = g->split_site[size_t(g->bi[b])], j = g->split_site[size_t(g->bj[b])];
        if (i > j) std::swap(i, j);
        jsum += g->J[b];
        if (j < best_s) {
            lo1.push_back(i); hi1.push_back(j); J1.push_back(g->J[b]); o1.push_back(int(b));
        } else {
            if (i >= best_c && i < best_s) return;  // not a split (cannot happen by construction)
            lo2.push_back(i); hi2.push_back(j); J2.push_back(g->J[b]); o2.push_back(int(b));
        }
    }
    g->p1 = make_bond_table(N, lo1, hi1, J1, o1, jsum);
    g->p2 = make_bond_table(N, lo2, hi2, J2, o2, 0.0);
    g->split_c = best_c;
    g->split_s = best_s;
    g->split = true;
}

int g_split_policy = FTLM_SPLIT_OFF;

// Whether a sector of dimension `dim` runs the two-pass H.x: the policy asks
// for it, the graph has a split, and the grid has one share per XCD.
bool use_split(const ftlm_graph* g, uint64_t dim, int R, int dtype) {
    (void)R;
    (void)dtype;
    if (!g || !g->split || g_split_policy != FTLM_SPLIT_ON) return false;
    return dim >= 8 * uint64_t(kBlock);
}

}  // namespace ftlm
