/*
 * The paper's CPU method, for the CPU baseline only (Sec. 2, "Computational
 * setup"): a batched row-wise gather H.x in FP64 over B = 8 vectors at once,
 * with the compressed lookup table of Eqs. 18-21 as the state-to-index map
 * and OpenMP over the rows. The row work (label, bond loop, lookup) is done
 * once per row and shared by the 8 vectors, which are stored [D][8].
 *
 * TEST INFRASTRUCTURE ONLY: this is not one of the oracle's definitions and
 * checks nothing. bench.py's cpu_baseline times it next to the oracle; a CPU
 * test checks it against the oracle's H.x. Nothing in the product library
 * links or calls it.
 */
#include <stdint.h>

#define PCPU_B 8

/* y[t][c] = sum over bonds of Eq. 12 at s = 1/2 for rows [row0, row0 +
 * nrows), every column c < 8; x is [D][8], y is [nrows][8]. */
void pcpu_hv_clt_b8(int n_bonds, const int32_t* bi, const int32_t* bj, const double* J, const uint64_t* basis,
                    const uint32_t* mask, const uint32_t* prefix, const double* x, double* y, uint64_t row0,
                    uint64_t nrows) {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < (int64_t)nrows; ++r) {
        const uint64_t t = row0 + (uint64_t)r;
        const uint64_t n = basis[t];
        double acc[PCPU_B] = {0};
        double diag = 0.0;
        for (int b = 0; b < n_bonds; ++b) {
            const uint64_t si = (n >> bi[b]) & 1u, sj = (n >> bj[b]) & 1u;
            if (si == sj) {
                diag += 0.25 * J[b];
                continue;
            }
            diag -= 0.25 * J[b];
            const uint64_t m = n ^ ((1ull << bi[b]) | (1ull << bj[b]));
            const uint64_t blk = m >> 5;
            const uint32_t j = (uint32_t)(m & 31u);
            const uint32_t below = mask[blk] & ((1u << j) - 1u);
            const uint64_t idx = prefix[blk] + (uint64_t)__builtin_popcount(below);
            const double c = 0.5 * J[b];
            const double* xr = x + idx * PCPU_B;
            for (int k = 0; k < PCPU_B; ++k) acc[k] += c * xr[k];
        }
        const double* xt = x + t * PCPU_B;
        double* yr = y + (uint64_t)r * PCPU_B;
        for (int k = 0; k < PCPU_B; ++k) yr[k] = diag * xt[k] + acc[k];
    }
}
