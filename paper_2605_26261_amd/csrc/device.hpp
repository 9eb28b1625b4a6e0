// Device-side building blocks shared by the libftlm kernels (gfx950, wave64).
//
// State labels (Sec. 2, Eq. 11 at s = 1/2): bit k of n is 1 when site k is
// up. The sector with n_up up spins is ordered by increasing label, so the
// index of a label is the number of sector labels below it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"

namespace ftlm {

constexpr uint32_t kNone32 = 0xFFFFFFFFu;

// Global-memory accesses through a generic pointer. Every table and vector
// block the kernels touch is device memory, in the global address space;
// saying so lets the compiler emit global instead of flat instructions where
// the pointer came out of a device-memory descriptor (a flat load also holds
// up every LDS wait until it completes).
#define FTLM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const FTLM_GLOBAL T* gptr(const T* p) {
    return (const FTLM_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ FTLM_GLOBAL T* gptr(T* p) {
    return (FTLM_GLOBAL T*)p;
}

// One compressed-lookup-table entry, read as a single 8-byte global load.
__device__ __forceinline__ CltEntry clt_entry(const CltEntry* clt, uint32_t block) {
    const FTLM_GLOBAL CltEntry* q = gptr(clt + block);
    return CltEntry{q->mask, q->prefix};
}

template <typename L>
__device__ __forceinline__ int popc(L x) {
    if constexpr (sizeof(L) == 8) return __popcll(x);
    else return __popc(x);
}

// Binomial table staged in LDS: row p (0 <= p < N) has `w` entries and entry
// [p][k + 1] is C(p, k) mod 2^32 for k in [-1, n_up + 1]. For s = 1/2 this is
// the cumulative dimension table of Eq. (16): D_c(p, A, 1) = C(p, A).
struct Binom {
    const uint32_t* t;
    int w;
    __device__ __forceinline__ uint32_t operator()(int p, int k) const { return t[p * w + k + 1]; }
};

// Copies the sector's binomial table from HBM into LDS (all threads of the
// block take part; ends with a barrier).
__device__ __forceinline__ void stage_binomials(uint32_t* lds, const uint32_t* g, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) lds[i] = *gptr(g + i);
    __syncthreads();
}

// Unranking (the inverse map of Sec. 2, CR): walks the N digit positions
// from the top in a loop of fixed length; at position p with A up spins still
// to place, the C(p, A) labels with a 0 there come first, so the digit is 1
// exactly when the remaining rank reaches C(p, A). Every C(p, A) compared lies
// on the path of a valid rank and is <= D < 2^32, so the table's mod-2^32
// entries are exact where they are compared.
template <typename L>
__device__ __forceinline__ L cr_unrank(uint32_t t, int n_sites, int n_up, Binom C) {
    L n = 0;
    uint32_t rem = t;
    int A = n_up;
    for (int p = n_sites - 1; p >= 0; --p) {
        uint32_t c = C(p, A);
        bool one = (A > 0) && (rem >= c);
        if (one) {
            n |= L(1) << p;
            rem -= c;
            A -= 1;
        }
    }
    return n;
}

// Ranking, Alg. 1 at s = 1/2: over p = N-1..0, a 1 at position p adds
// D_c(p, A, 1) = C(p, A) and lowers A. Sums wrap mod 2^32; the true rank is
// < 2^32, so the wrapped sum is exact. The caller checks sector membership.
template <typename L>
__device__ __forceinline__ uint32_t cr_rank(L x, int n_sites, int n_up, Binom C) {
    uint32_t r = 0;
    int A = n_up;
    for (int p = n_sites - 1; p >= 0; --p) {
        uint32_t bit = uint32_t((x >> p) & 1);
        r += bit ? C(p, A) : 0u;
        A -= int(bit);
    }
    return r;
}

// Alg. 2: index of label n through the compressed lookup table, kNone32 when
// bit n mod 32 of the block's mask is clear.
__device__ __forceinline__ uint32_t clt_lookup(const CltEntry* clt, uint32_t n) {
    CltEntry e = clt_entry(clt, n >> 5);
    uint32_t j = n & 31u;
    if (((e.mask >> j) & 1u) == 0) return kNone32;
    return e.prefix + __popc(e.mask & ((1u << j) - 1u));
}

// Bonds as the kernels see them, passed by value as a kernel argument.
// Every field is a 32-bit word so that each read is a scalar (s_load_dword)
// load: gfx9 has no scalar byte loads, and a vector load of bond data would
// make each bond wait on the gathers still in flight. Bonds are sorted by
// their lower site, highest first, so the combinatorial-ranking pass, which
// walks the sites from the top, meets each bond at its lower site after its
// upper site is known. The bonds with lower site >= p are the first ends[p].
struct BondTable {
    uint32_t pack[kMaxBonds];  // lo | hi << 8 | (position in the caller's order) << 16
    float coef_f[kMaxBonds];   // J_b / 2 (Eqs. 13-14 at s = 1/2)
    double coef_d[kMaxBonds];
    uint32_t ends[kMaxSites + 1];
    int n_bonds;
    int n_sites;
    float jsum4_f;   // sum_b J_b / 4: the diagonal when every bond is parallel
    double jsum4_d;
    __device__ __forceinline__ uint32_t lo(int b) const { return pack[b] & 0xffu; }
    __device__ __forceinline__ uint32_t hi(int b) const { return (pack[b] >> 8) & 0xffu; }
    __device__ __forceinline__ uint32_t orig(int b) const { return pack[b] >> 16; }
};

// Partner-index maps that keep a stored table, read in two phases so that a
// group of lookups is in flight together: fetch(m) issues the table loads of
// label m, index(e, m) turns them into the sector index.
//   CLT (Alg. 2): one 8-byte {mask, prefix} load and a popcount;
//   FULL (the full lookup table of Sec. 2): one 4-byte load of the index;
//   LIN (Lin's two-dimensional search, Sec. 2): the number of sector labels
//   whose high part (label >> L) is smaller, plus the rank of the low part
//   among L-bit strings with its popcount: two 4-byte loads and an add.
template <int MODE>
struct TableMap;

template <>
struct TableMap<kModeClt> {
    using Entry = CltEntry;
    const CltEntry* clt;
    __device__ __forceinline__ Entry none() const { return CltEntry{0u, 0u}; }
    __device__ __forceinline__ Entry fetch(uint32_t m) const { return clt_entry(clt, m >> 5); }
    __device__ __forceinline__ uint32_t index(const Entry& e, uint32_t m) const {
        return e.prefix + __popc(e.mask & ((1u << (m & 31u)) - 1u));
    }
};

template <>
struct TableMap<kModeFull> {
    using Entry = uint32_t;
    const uint32_t* full;
    __device__ __forceinline__ Entry none() const { return 0u; }
    __device__ __forceinline__ Entry fetch(uint32_t m) const { return *gptr(full + m); }
    __device__ __forceinline__ uint32_t index(const Entry& e, uint32_t) const { return e; }
};

template <>
struct TableMap<kModeLin> {
    struct Entry {
        uint32_t hi, lo;
    };
    const uint32_t* hi_tab;
    const uint32_t* lo_tab;
    int lo_bits;
    __device__ __forceinline__ Entry none() const { return Entry{0u, 0u}; }
    __device__ __forceinline__ Entry fetch(uint32_t m) const {
        return Entry{*gptr(hi_tab + (m >> lo_bits)), *gptr(lo_tab + (m & ((1u << lo_bits) - 1u)))};
    }
    __device__ __forceinline__ uint32_t index(const Entry& e, uint32_t) const { return e.hi + e.lo; }
};

// Reports every bond of the row with label n to the visitor, the partner
// indices found through a stored map (the occupancy test always passes for a
// flip inside the sector, Sec. 2):
//   v.flip(b, idx)  for an antiparallel bond b (b in the sorted order), and
//   v.par(b)        for a parallel one;
// or, when the visitor takes groups (V::kGroup > 1), v.group(b0, idx, flips)
// for kGroup consecutive bonds at a time. A group's table loads and then its
// row gathers are in flight together; lanes whose bond is parallel issue
// neither, and the visitor weighs them by zero.
template <typename Map, typename V>
__device__ __forceinline__ void table_bonds(uint32_t n, const BondTable& B, const Map& map, V& v) {
    int b = 0;
    constexpr int G = V::kGroup;
    if constexpr (G > 1) {
        for (; b + G <= B.n_bonds; b += G) {
            uint32_t m[G], idx[G];
            bool anti[G];
            typename Map::Entry e[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const uint32_t lo = B.lo(b + g), hi = B.hi(b + g);
                anti[g] = ((n >> lo) & 1u) != ((n >> hi) & 1u);
                m[g] = n ^ ((1u << lo) | (1u << hi));
                e[g] = map.none();
                if (anti[g]) e[g] = map.fetch(m[g]);
            }
#pragma unroll
            for (int g = 0; g < G; ++g) idx[g] = map.index(e[g], m[g]);
            v.group(b, idx, anti);
        }
    }
    for (; b < B.n_bonds; ++b) {
        const uint32_t si = (n >> B.lo(b)) & 1u, sj = (n >> B.hi(b)) & 1u;
        if (si != sj) {
            const uint32_t m = n ^ ((1u << B.lo(b)) | (1u << B.hi(b)));
            v.flip(b, map.index(map.fetch(m), m));
        } else {
            v.par(b);
        }
    }
}

// Combinatorial ranking of every partner of row t in O(1): one top-down pass
// over the sites either unranks t (FROM_LABEL false: the digit at p is 1 when
// the remaining rank reaches C(p, A)) or reads the digits of a known label n
// (FROM_LABEL true), and ranks the partners on the way. With K = number of up
// spins at positions <= p, Es/Fs the sums over up positions q above p of
// C(q, K_q - 1) - C(q, K_q) and C(q, K_q + 1) - C(q, K_q), define
//   up p:   X = Es - C(p, K),     Y = -C(p, K + 1) - Fs
//   down p: X = C(p, K + 1) + Fs, Y = C(p, K) - Es.
// Moving the up spin of an antiparallel pair lo < hi to the other site changes
// Alg. 1's sum by X(lo) + Y(hi) in both directions (every term between lo and
// hi whose K shifts by one telescopes into Es/Fs), so the partner's index is
// t + X(lo) + Y(hi) mod 2^32. Y of the sites above p sits in LDS at
// ylds[q * 64] (this lane's column of its wave's slab, bank-conflict free).
// Bonds are visited at their lower site. Returns the label.
template <typename L, bool FROM_LABEL, typename V>
__device__ __forceinline__ L cr_bonds(uint32_t t, L n_in, int n_up, const BondTable& B, Binom C, uint32_t* ylds,
                                      V& v) {
    L n = 0;
    uint32_t rem = t, Es = 0, Fs = 0;
    int A = n_up;
    int b = 0;
    for (int p = B.n_sites - 1; p >= 0; --p) {
        const uint32_t cm = C(p, A - 1), c0 = C(p, A), cp = C(p, A + 1);
        bool one;
        if constexpr (FROM_LABEL) one = ((n_in >> p) & 1) != 0;
        else one = (A > 0) && (rem >= c0);
        uint32_t X, Y;
        if (one) {
            X = Es - c0;
            Y = 0u - cp - Fs;
            Es += cm - c0;
            Fs += cp - c0;
            rem -= c0;
            A -= 1;
            n |= L(1) << p;
        } else {
            X = cp + Fs;
            Y = c0 - Es;
        }
        ylds[p * 64] = Y;
        const int end = int(B.ends[p]);
        for (; b < end; ++b) {
            const uint32_t hb = B.hi(b);
            const uint32_t shi = uint32_t((n >> hb) & 1);
            if (shi != uint32_t(one)) v.flip(b, t + X + ylds[hb * 64]);
            else v.par(b);
        }
    }
    return n;
}

// cr_bonds for a visitor that keeps two slots of row gathers in flight
// (V::kPairs): the bonds, in their sorted order, are taken kSiteGroup at a
// time into slot A and slot B in turn, and each slot is accumulated after the
// other slot's next loads have been issued. The two slots are fixed registers
// (the loop body handles one A and one B) loaded by every lane, so the
// compiler can wait for just the older slot's loads. The last bonds (fewer
// than two slots) go one at a time. The top-down pass over the sites runs
// ahead of the bonds only as far as the next bond's lower site, with the loop
// bounds read as wave-uniform values. The partner indices, their order and
// every accumulation are those of cr_bonds.
template <typename L, typename V>
__device__ __forceinline__ L cr_bonds_pairs(uint32_t t, int n_up, const BondTable& B, Binom C, uint32_t* ylds,
                                            V& v) {
    L n = 0;
    uint32_t rem = t, Es = 0, Fs = 0, X = 0;
    int A = n_up;
    bool one = false;
    int p = B.n_sites - 1;  // the next site of the top-down pass
    // runs the pass over the sites down to `lo`; X and `one` are then those of lo
    auto advance = [&](int lo) {
        for (; p >= lo; --p) {
            const uint32_t cm = C(p, A - 1), c0 = C(p, A), cp = C(p, A + 1);
            one = (A > 0) && (rem >= c0);
            uint32_t Y;
            if (one) {
                X = Es - c0;
                Y = 0u - cp - Fs;
                Es += cm - c0;
                Fs += cp - c0;
                rem -= c0;
                A -= 1;
                n |= L(1) << p;
            } else {
                X = cp + Fs;
                Y = c0 - Es;
            }
            ylds[p * 64] = Y;
        }
    };
    constexpr int G = V::kSiteGroup;
    const int nb = B.n_bonds;
    // partner index and flip flag of bond b
    auto prepare = [&](int b, uint32_t& idx, bool& anti) {
        const int lo = __builtin_amdgcn_readfirstlane(int(B.lo(b)));
        advance(lo);
        const uint32_t hb = B.hi(b);
        anti = uint32_t((n >> hb) & 1) != uint32_t(one);
        idx = t;
        if (anti) idx = t + X + ylds[hb * 64];
    };
    v.clear_slots();
    int b = 0;
    for (; b + 2 * G <= nb; b += 2 * G) {
        uint32_t idx[G];
        bool anti[G];
#pragma unroll
        for (int g = 0; g < G; ++g) prepare(b + g, idx[g], anti[g]);
        v.load_slot_a(b, idx, anti);
        v.add_slot_b();
#pragma unroll
        for (int g = 0; g < G; ++g) prepare(b + G + g, idx[g], anti[g]);
        v.load_slot_b(b + G, idx, anti);
        v.add_slot_a();
    }
    v.add_slot_b();
    // the remaining bonds (fewer than 2G) one at a time
    for (; b < nb; ++b) {
        uint32_t idx;
        bool anti;
        prepare(b, idx, anti);
        if (anti) v.flip(b, idx);
        else v.par(b);
    }
    advance(0);
    return n;
}

// Visits one row t of the sector: finds its label n_t and, for every bond,
// either reports a parallel pair or the sector index of the flipped partner
// n_t ^ (2^i + 2^j) (Eq. 12 at s = 1/2). The stored-map modes (CLT, FULL,
// LIN) read n_t from the stored basis; CR mode reconstructs it by unranking
// in the same pass that ranks the partners.
template <typename L, int MODE, typename V, typename Map>
__device__ __forceinline__ L visit_row(uint32_t t, int n_up, const BondTable& B, Binom C,
                                       const uint32_t* __restrict__ basis, const Map& map, uint32_t* ylds, V& v) {
    if constexpr (MODE != kModeCr) {
        const uint32_t n = *gptr(basis + t);
        table_bonds(n, B, map, v);
        return L(n);
    } else {
        if constexpr (V::kPairs) return cr_bonds_pairs<L>(t, n_up, B, C, ylds, v);
        else return cr_bonds<L, false>(t, L(0), n_up, B, C, ylds, v);
    }
}

}  // namespace ftlm
