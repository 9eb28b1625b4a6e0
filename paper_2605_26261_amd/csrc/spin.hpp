// Device building blocks of the general-spin row kernels (local spin s =
// two_s / 2 > 1/2; Sec. 2, Eqs. 11-17).
//
// A basis state is n = sum_p a_p d^p with d = two_s + 1 and digit a_p = m_p +
// s (Eq. 11); the sector with digit sum A (S^z = A - N s, Eq. 17) is ordered
// by increasing label. Kernels hold a row's digits packed four bits per site
// (N <= 16).
#pragma once

#include "kernels.hpp"

namespace ftlm {

constexpr int kMaxSpinSites = 16;  // digits packed 4 bits per site in a uint64
constexpr int kMaxTwoS = 7;        // digits 0..7 fit the 4-bit packing with room to spare

// The cumulative dimension table of Eq. (16) staged in LDS: entry (p, A, a) =
// D_c(p, A, a) = sum_{q < a} D(p, A - q) mod 2^32, the number of length-p
// digit strings with sum A - q over q < a, for 0 <= p < N, -1 <= A <= A_tot + 1
// (zero at A = -1) and 0 <= a <= 2s. Every difference the kernels form is a
// difference of true ranks, so arithmetic mod 2^32 is exact for D < 2^32.
struct CumDim {
    const uint32_t* t;
    int bw;  // A slots: A_tot + 3
    int d;   // digits per position: two_s + 1
    __device__ __forceinline__ uint32_t operator()(int p, int A, int a) const {
        return t[(p * bw + A + 1) * d + a];
    }
};

__device__ __forceinline__ int digit_of(uint64_t packed, int p) { return int((packed >> (4 * p)) & 15u); }

// Unranking (the inverse map of Sec. 2): at position p, with digit sum A left
// for positions <= p, the labels whose digit there is below a come first
// (D_c(p, A, a) of them), so the digit is the largest a with D_c(p, A, a) <=
// the remaining rank. Fixed-length loops over the N positions and the 2s + 1
// digit values. Returns the digits packed.
__device__ __forceinline__ uint64_t spin_unrank_digits(uint32_t t, int n_sites, int a_tot, int two_s, CumDim D) {
    uint64_t dig = 0;
    uint32_t rem = t;
    int A = a_tot;
    for (int p = n_sites - 1; p >= 0; --p) {
        int a = 0;
        for (int q = 1; q <= two_s; ++q)
            if (D(p, A, q) <= rem) a = q;
        rem -= D(p, A, a);
        A -= a;
        dig |= uint64_t(a) << (4 * p);
    }
    return dig;
}

// Alg. 1 (ranking) on packed digits: rank = sum_p D_c(p, A, a_p), A lowered by
// a_p after each position. For a digit string outside the sector the sum stops
// counting once A is exhausted, which makes it the number of sector labels
// below the given one (used for the compressed lookup table's prefix counts).
__device__ __forceinline__ uint32_t spin_rank_digits(uint64_t dig, int n_sites, int a_tot, CumDim D) {
    uint32_t r = 0;
    int A = a_tot;
    for (int p = n_sites - 1; p >= 0 && A >= 0; --p) {
        const int a = digit_of(dig, p);
        r += D(p, A, a);
        A -= a;
    }
    return r;
}

// q = x / d and r = x mod d for 32-bit x and 2 <= d <= 8, from a double
// reciprocal: the product is within 2^-20 of x / d, so the floor is exact
// except one below at exact multiples, which the remainder test repairs.
__device__ __forceinline__ uint32_t divmod_small(uint32_t x, uint32_t d, double inv_d, uint32_t& r) {
    uint32_t q = uint32_t(double(x) * inv_d);
    r = x - q * d;
    if (r >= d) {
        q += 1;
        r -= d;
    }
    return q;
}

// Digits of a 32-bit label, packed.
__device__ __forceinline__ uint64_t label_digits(uint32_t n, int n_sites, uint32_t d, double inv_d) {
    uint64_t dig = 0;
    for (int p = 0; p < n_sites; ++p) {
        uint32_t r;
        n = divmod_small(n, d, inv_d, r);
        dig |= uint64_t(r) << (4 * p);
    }
    return dig;
}

// Digits and digit sum of a 64-bit label (index kernels only: plain division).
__device__ __forceinline__ uint64_t label_digits64(uint64_t n, int n_sites, uint32_t d, int* sum) {
    uint64_t dig = 0;
    int s = 0;
    for (int p = 0; p < n_sites; ++p) {
        const uint32_t r = uint32_t(n % d);
        n /= d;
        s += int(r);
        dig |= uint64_t(r) << (4 * p);
    }
    *sum = s;
    return dig;
}

// One row of the general-spin Hamiltonian (Eq. 12 with the coefficients of
// Eqs. 13-14) reported to a visitor, in combinatorial-ranking mode: a single
// top-down pass unranks t and ranks every partner in O(1).
//
// Moving one unit of digit between the positions lo < hi of a bond (digit
// a_lo + e, a_hi - e for e = +1 or -1) shifts the running digit sum A_q by e at
// the positions lo <= q < hi and nowhere else, so Alg. 1's sum changes by
//   [D_c(lo, A_lo + e, a_lo + e) - D_c(lo, A_lo, a_lo)]
//   + sum_{lo < q < hi} [D_c(q, A_q + e, a_q) - D_c(q, A_q, a_q)]
//   + [D_c(hi, A_hi, a_hi - e) - D_c(hi, A_hi, a_hi)].
// With T_e(q) the middle term's summand and S_e(p) its sum over q > p, that is
// X_e(lo) + Y_e(hi) with
//   X_e(p) = D_c(p, A_p + e, a_p + e) - D_c(p, A_p, a_p) + S_e(p),
//   Y_e(p) = D_c(p, A_p, a_p - e) - D_c(p, A_p, a_p) - S_e(p) - T_e(p),
// all from the same pass (at s = 1/2 they reduce to the X, Y of cr_bonds).
// Y_e of the sites above p sit in LDS at yp/ym[q * 64]. The visitor gets
//   v.diag(b, m_lo m_hi)                       every bond, and
//   v.flip(b, k, idx, f)                       every valid ladder term (k = 0
// for e = +1, 1 for e = -1), with f the product of single-site ladder factors: for e = +1 (the term whose
// source has a_lo + 1, a_hi - 1) f = fu[a_lo] fu[a_hi - 1], for e = -1 f =
// fu[a_lo - 1] fu[a_hi], where fu[a] = sqrt(s(s+1) - m(m+1)), m = a - s.
template <typename T, typename V>
__device__ __forceinline__ void spin_cr_row(uint32_t t, int a_tot, int two_s, const BondTable& B, CumDim D,
                                            const T* fu, uint32_t* yp, uint32_t* ym, V& v) {
    uint64_t dig = 0;
    uint32_t rem = t, Sp = 0, Sm = 0;
    int A = a_tot;
    int b = 0;
    const T s = T(0.5) * T(two_s);
    for (int p = B.n_sites - 1; p >= 0; --p) {
        int a = 0;
        for (int q = 1; q <= two_s; ++q)
            if (D(p, A, q) <= rem) a = q;
        const uint32_t c0 = D(p, A, a);
        const uint32_t Tp = D(p, A + 1, a) - c0, Tm = D(p, A - 1, a) - c0;
        const bool can_up = a < two_s, can_dn = a > 0;
        const uint32_t Xp = (can_up ? D(p, A + 1, a + 1) : 0u) - c0 + Sp;
        const uint32_t Xm = (can_dn ? D(p, A - 1, a - 1) : 0u) - c0 + Sm;
        yp[p * 64] = (can_dn ? D(p, A, a - 1) : 0u) - c0 - Sp - Tp;
        ym[p * 64] = (can_up ? D(p, A, a + 1) : 0u) - c0 - Sm - Tm;
        dig |= uint64_t(a) << (4 * p);
        Sp += Tp;
        Sm += Tm;
        rem -= c0;
        A -= a;
        const T m_lo = T(a) - s;
        const int end = int(B.ends[p]);
        for (; b < end; ++b) {
            const int hi = int(B.hi(b));
            const int ah = digit_of(dig, hi);
            v.diag(b, m_lo * (T(ah) - s));
            if (can_up && ah > 0) v.flip(b, 0, t + Xp + yp[hi * 64], fu[a] * fu[ah - 1]);
            if (can_dn && ah < two_s) v.flip(b, 1, t + Xm + ym[hi * 64], fu[a - 1] * fu[ah]);
        }
    }
}

// spin_cr_row for a visitor that keeps two slots of row gathers in flight
// (V::kPairs): the bonds, in their sorted order, go V::kSlotBonds at a time
// into slot A and slot B in turn, each with its two ladder terms (e = +1,
// then -1), and each slot is accumulated after the other slot's next loads
// are issued. A term that does not exist is loaded from row 0 under weight
// zero, so every lane loads and the compiler can wait for just the older
// slot. The last bonds (fewer than two slots) go one at a time. The top-down
// pass over the sites runs ahead of the bonds only as far as the next bond's
// lower site. The partner indices, the factors and the order of every
// accumulation are those of spin_cr_row.
template <typename T, typename V>
__device__ __forceinline__ void spin_cr_row_pairs(uint32_t t, int a_tot, int two_s, const BondTable& B, CumDim D,
                                                  const T* fu, uint32_t* yp, uint32_t* ym, V& v) {
    uint64_t dig = 0;
    uint32_t rem = t, Sp = 0, Sm = 0, Xp = 0, Xm = 0;
    int A = a_tot, a = 0;
    int p = B.n_sites - 1;  // the next site of the top-down pass
    const T s = T(0.5) * T(two_s);
    // runs the pass down to `lo`; a, Xp and Xm are then those of lo
    auto advance = [&](int lo) {
        for (; p >= lo; --p) {
            int ap = 0;
            for (int q = 1; q <= two_s; ++q)
                if (D(p, A, q) <= rem) ap = q;
            const uint32_t c0 = D(p, A, ap);
            const uint32_t Tp = D(p, A + 1, ap) - c0, Tm = D(p, A - 1, ap) - c0;
            const bool can_up = ap < two_s, can_dn = ap > 0;
            Xp = (can_up ? D(p, A + 1, ap + 1) : 0u) - c0 + Sp;
            Xm = (can_dn ? D(p, A - 1, ap - 1) : 0u) - c0 + Sm;
            yp[p * 64] = (can_dn ? D(p, A, ap - 1) : 0u) - c0 - Sp - Tp;
            ym[p * 64] = (can_up ? D(p, A, ap + 1) : 0u) - c0 - Sm - Tm;
            dig |= uint64_t(ap) << (4 * p);
            Sp += Tp;
            Sm += Tm;
            rem -= c0;
            A -= ap;
            a = ap;
        }
    };
    // the diagonal term of bond b, and its two ladder terms (entries k and
    // k + 1): partner index, existence and single-site factor product
    constexpr int SB = V::kSlotBonds;
    uint32_t idx[2 * SB];
    bool on[2 * SB];
    T f[2 * SB];
    auto prepare = [&](int b, int k) {
        advance(__builtin_amdgcn_readfirstlane(int(B.lo(b))));
        const int hi = int(B.hi(b));
        const int ah = digit_of(dig, hi);
        v.diag(b, (T(a) - s) * (T(ah) - s));
        on[k] = a < two_s && ah > 0;
        on[k + 1] = a > 0 && ah < two_s;
        idx[k] = t + Xp + yp[hi * 64];
        idx[k + 1] = t + Xm + ym[hi * 64];
        f[k] = on[k] ? fu[a] * fu[ah - 1] : T(0);
        f[k + 1] = on[k + 1] ? fu[a - 1] * fu[ah] : T(0);
    };
    const int nb = B.n_bonds;
    v.clear_slots();
    int b = 0;
    for (; b + 2 * SB <= nb; b += 2 * SB) {
#pragma unroll
        for (int g = 0; g < SB; ++g) prepare(b + g, 2 * g);
        v.load_slot_a(b, idx, on, f);
        v.add_slot_b();
#pragma unroll
        for (int g = 0; g < SB; ++g) prepare(b + SB + g, 2 * g);
        v.load_slot_b(b + SB, idx, on, f);
        v.add_slot_a();
    }
    v.add_slot_b();
    for (; b < nb; ++b) {
        prepare(b, 0);
        if (on[0]) v.flip(b, 0, idx[0], f[0]);
        if (on[1]) v.flip(b, 1, idx[1], f[1]);
    }
}

// The same row in compressed-lookup-table mode: the label comes from the
// stored basis, its digits by division, and every partner label is the label
// plus or minus d^lo - d^hi, looked up with Alg. 2. pw[p] = d^p (LDS).
template <typename T, typename V>
__device__ __forceinline__ void spin_clt_row(uint32_t t, int two_s, const BondTable& B, const uint32_t* basis,
                                             const CltEntry* clt, const uint32_t* pw, const T* fu, double inv_d,
                                             V& v) {
    const uint32_t n = *gptr(basis + t);
    const uint64_t dig = label_digits(n, B.n_sites, uint32_t(two_s + 1), inv_d);
    const T s = T(0.5) * T(two_s);
    for (int b = 0; b < B.n_bonds; ++b) {
        const int lo = int(B.lo(b)), hi = int(B.hi(b));
        const int al = digit_of(dig, lo), ah = digit_of(dig, hi);
        v.diag(b, (T(al) - s) * (T(ah) - s));
        const uint32_t step = pw[lo] - pw[hi];  // d^lo - d^hi mod 2^32
        if (al < two_s && ah > 0) v.flip(b, 0, clt_lookup(clt, n + step), fu[al] * fu[ah - 1]);
        if (al > 0 && ah < two_s) v.flip(b, 1, clt_lookup(clt, n - step), fu[al - 1] * fu[ah]);
    }
}

// spin_clt_row for a visitor that takes groups (V::kGroup > 0): the ladder
// terms of kGroup consecutive bonds have their table loads in flight
// together, then their row gathers (v.group); a term that does not exist
// issues neither and is weighed by zero. A partner inside the sector always
// finds its bit set in the table, so the index is prefix plus popcount.
// Partner indices, factors and the order of the accumulations are those of
// spin_clt_row.
template <typename T, typename V>
__device__ __forceinline__ void spin_clt_row_groups(uint32_t t, int two_s, const BondTable& B,
                                                    const uint32_t* basis, const CltEntry* clt, const uint32_t* pw,
                                                    const T* fu, double inv_d, V& v) {
    constexpr int G = V::kGroup;
    const uint32_t n = *gptr(basis + t);
    const uint64_t dig = label_digits(n, B.n_sites, uint32_t(two_s + 1), inv_d);
    const T s = T(0.5) * T(two_s);
    int b = 0;
    for (; b + G <= B.n_bonds; b += G) {
        uint32_t m[2 * G], idx[2 * G];
        bool on[2 * G];
        T f[2 * G];
        CltEntry e[2 * G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int lo = int(B.lo(b + g)), hi = int(B.hi(b + g));
            const int al = digit_of(dig, lo), ah = digit_of(dig, hi);
            v.diag(b + g, (T(al) - s) * (T(ah) - s));
            const uint32_t step = pw[lo] - pw[hi];
            on[2 * g] = al < two_s && ah > 0;
            on[2 * g + 1] = al > 0 && ah < two_s;
            m[2 * g] = n + step;
            m[2 * g + 1] = n - step;
            f[2 * g] = on[2 * g] ? fu[al] * fu[ah - 1] : T(0);
            f[2 * g + 1] = on[2 * g + 1] ? fu[al - 1] * fu[ah] : T(0);
        }
#pragma unroll
        for (int k = 0; k < 2 * G; ++k) {
            e[k] = CltEntry{0u, 0u};
            if (on[k]) e[k] = clt_entry(clt, m[k] >> 5);
        }
#pragma unroll
        for (int k = 0; k < 2 * G; ++k) idx[k] = e[k].prefix + __popc(e[k].mask & ((1u << (m[k] & 31u)) - 1u));
        v.group(b, idx, on, f);
    }
    for (; b < B.n_bonds; ++b) {
        const int lo = int(B.lo(b)), hi = int(B.hi(b));
        const int al = digit_of(dig, lo), ah = digit_of(dig, hi);
        v.diag(b, (T(al) - s) * (T(ah) - s));
        const uint32_t step = pw[lo] - pw[hi];
        if (al < two_s && ah > 0) v.flip(b, 0, clt_lookup(clt, n + step), fu[al] * fu[ah - 1]);
        if (al > 0 && ah < two_s) v.flip(b, 1, clt_lookup(clt, n - step), fu[al - 1] * fu[ah]);
    }
}

}  // namespace ftlm
