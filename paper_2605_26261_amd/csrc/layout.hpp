// Layout of the sector tables in the caller's device buffer, and limits.
// Shared by host and device code of libftlm.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace ftlm {

constexpr int kModeClt = 0;   // FTLM_CLT
constexpr int kModeCr = 1;    // FTLM_CR
constexpr int kModeFull = 2;  // FTLM_FULL: one uint32 index per label of [0, 2^N)
constexpr int kModeLin = 3;   // FTLM_LIN: two half-label tables
constexpr int kMaxSites = 64;
constexpr int kMaxBonds = 128;
constexpr int kMaxCltSites = 32;  // CLT labels are uint32

// One block of 32 labels of the compressed lookup table (Eqs. 18-20): the
// occupancy mask and the number of sector labels in all earlier blocks. The
// two words sit together so one 8-byte load serves a lookup.
struct CltEntry {
    uint32_t mask;
    uint32_t prefix;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Binomial table: N rows of (n_up + 3) uint32; entry [p][k + 1] = C(p, k).
inline int binom_width(int n_up) { return n_up + 3; }
inline size_t binom_bytes(int n_sites, int n_up) {
    return size_t(n_sites) * size_t(binom_width(n_up)) * sizeof(uint32_t);
}

inline uint64_t clt_blocks(int n_sites) {
    return n_sites >= 5 ? (uint64_t(1) << (n_sites - 5)) : 1;
}

// Lin's two-dimensional split of a label: the low lin_low_bits(N) bits and
// the rest.
inline int lin_low_bits(int n_sites) { return n_sites / 2; }

struct TableLayout {
    size_t binom_off, basis_off, clt_off, full_off, hi_off, lo_off, total;
};

// Table buffer of a spin-1/2 sector: the binomial table, then (every mode
// but CR) the basis uint32[D], then the mode's map: CLT {mask, prefix}
// pairs over 2^N / 32 blocks; FULL uint32[2^N]; LIN uint32[2^(N - L)] for the
// high part and uint32[2^L] for the low part (L = lin_low_bits(N)).
inline TableLayout table_layout(int n_sites, int n_up, int mode, uint64_t dim) {
    TableLayout t{};
    t.binom_off = 0;
    size_t end = align256(binom_bytes(n_sites, n_up));
    if (mode != kModeCr) {
        t.basis_off = end;
        end = align256(end + size_t(dim) * sizeof(uint32_t));
    }
    if (mode == kModeClt) {
        t.clt_off = end;
        end = align256(end + size_t(clt_blocks(n_sites)) * sizeof(CltEntry));
    } else if (mode == kModeFull) {
        t.full_off = end;
        end = align256(end + (size_t(1) << n_sites) * sizeof(uint32_t));
    } else if (mode == kModeLin) {
        const int lo = lin_low_bits(n_sites);
        t.hi_off = end;
        end = align256(end + (size_t(1) << (n_sites - lo)) * sizeof(uint32_t));
        t.lo_off = end;
        end = align256(end + (size_t(1) << lo) * sizeof(uint32_t));
    }
    t.total = end;
    return t;
}

}  // namespace ftlm
