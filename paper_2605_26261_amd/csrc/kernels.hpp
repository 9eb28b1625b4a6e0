// Kernel-side argument structs and the host-visible launchers of libftlm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace ftlm {

constexpr int kBlock = 256;      // threads per workgroup: four wave64s
constexpr int kWaves = kBlock / 64;

// Per-chain Lanczos state, one per vector column, in device memory. The
// stored vector of step k is u_k with q_k = s_cur * u_k (the normalization
// of q_{k+1} = w / beta_k is folded into the next step's scalars instead of
// an extra pass over the vector).
struct Chain {
    double s_cur;      // scale of the current vector u_k
    double s_prev;     // scale of u_{k-1}
    double beta_prev;  // beta_{k-1}
    double amax;       // max_{j<=k}(|alpha_j|, beta_{j-1}) for the stopping rule
    double alpha;      // alpha_k of the step in flight
    double norm;       // |u_1| of the start vector
    // Scalars of the next kernels, precomputed once per step by the last
    // workgroup of the previous kernel so that every thread reads them with
    // scalar loads (no per-thread FP64 work or conversion):
    //   H.x epilogue  w = hv_a * (H u_k) - hv_b * u_{k-1}
    //   update        u_{k+1} = w - up * u_k
    double hv_a_d, hv_b_d, up_d;
    float hv_a_f, hv_b_f, up_f, pad_f;
    int32_t active;
    int32_t steps;
};

// Sets the next-step scalars of a chain from its FP64 state.
__device__ __forceinline__ void chain_set_hv(Chain* ch) {
    ch->hv_a_d = ch->s_cur;
    ch->hv_b_d = ch->beta_prev * ch->s_prev;
    ch->hv_a_f = float(ch->hv_a_d);
    ch->hv_b_f = float(ch->hv_b_d);
}

// A sector as the kernels see it.
struct SectorDev {
    int n_sites;
    int n_up;
    int mode;
    int bw;                  // binomial table row width
    uint32_t dim;
    const uint32_t* binom;   // [N][bw]
    const uint32_t* basis;   // [D] (CLT mode)
    const CltEntry* clt;     // [2^N / 32] (CLT mode)
};

enum Epilogue { kEpiPlain = 0, kEpiLanczos = 1 };

// One multi-vector H.x launch over rows [row0, row0 + nrows) and the
// columns [col0, col0 + vb) of [D][ld] blocks x (input) and y (output).
// In the Lanczos epilogue, y holds u_{k-1} on entry and receives
// w = s_k (H u_k) - beta_{k-1} s_{k-1} u_{k-1}; each workgroup writes its FP64
// partial of <u_k, w> per column to partials[block * pstride + col], and the
// last workgroup to finish sums them in block order into chains[col].alpha.
struct HvLaunch {
    const void* x;
    void* y;
    uint64_t ld;
    uint32_t col0;
    uint32_t row0;
    uint32_t nrows;
    int vb;
    int dtype;
    int epi;
    int first;          // Lanczos step 1: no previous vector
    int pstride;
    int grid;
    Chain* chains;
    double* partials;
    uint32_t* ticket;
};

hipError_t launch_hv(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st);

// Sector table builders and index kernels (sector.hip).
hipError_t launch_build_basis(const SectorDev& s, hipStream_t st);
hipError_t launch_build_clt(const SectorDev& s, hipStream_t st);
hipError_t launch_rank(const SectorDev& s, const uint64_t* labels, uint64_t* idx, uint64_t n,
                       hipStream_t st);
hipError_t launch_unrank(const SectorDev& s, const uint64_t* idx, uint64_t* labels, uint64_t n,
                         hipStream_t st);
hipError_t launch_neighbors(const SectorDev& s, const BondTable& B, uint64_t t0, uint64_t count,
                            uint64_t* out, hipStream_t st);

// Lanczos helpers (lanczos.hip).
struct StartLaunch {
    void* q;              // [D][ld] block, columns [col0, col0 + ncols)
    uint64_t ld;
    uint32_t col0;
    int ncols;
    int dtype;
    int dist;
    uint64_t keys[64];    // SplitMix64 stream key per column
    uint64_t sample[64];  // global sample index per column (FTLM_UNIT)
    int grid;
    int pstride;
    Chain* chains;
    double* partials;
    uint32_t* ticket;
};
hipError_t launch_start(const SectorDev& s, const StartLaunch& a, hipStream_t st);

struct UpdateLaunch {
    void* u;            // u_k, [D][ld]
    void* w;            // w in, u_{k+1} out, [D][ld]
    uint64_t ld;
    uint32_t col0;
    int ncols;
    int dtype;
    int grid;
    int pstride;
    int step;           // k (1-based)
    int m_eff;          // min(M, D)
    double eps;
    int M;              // row stride of the alpha/beta arrays
    Chain* chains;
    double* partials;
    uint32_t* ticket;
    double* alpha;      // [R][M]
    double* beta;       // [R][M]
};
hipError_t launch_update(const SectorDev& s, const UpdateLaunch& a, hipStream_t st);
hipError_t launch_chain_init(Chain* chains, int n, uint32_t* tickets, int nt, hipStream_t st);

// Grid of the persistent row kernels for a row count: a multiple of 8 (one
// share per XCD) capped near the number of resident workgroups, so reduction
// partials depend on the row count only.
inline int rows_grid(uint32_t nrows) {
    const uint32_t tiles = (nrows + kBlock - 1) / kBlock;
    if (tiles < 8) return int(tiles == 0 ? 1 : tiles);
    const uint32_t cap = 2048;
    uint32_t g = tiles < cap ? tiles : cap;
    return int((g + 7) & ~7u);
}

}  // namespace ftlm
