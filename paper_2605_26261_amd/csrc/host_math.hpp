// Host FP64 helpers: Ritz decomposition and thermal reduction.
#pragma once

#include <stdint.h>

namespace ftlm {

struct SectorSamples {
    int n_up;     // digit sum A of the sector (the up-spin count at s = 1/2)
    int two_s;    // 2s of the local spin
    int R;
    int stride;
    uint64_t dim;
    double mult;
    const double* theta;
    const double* weight;
    const int32_t* steps;
};

constexpr double kUnitRoundoffF32 = 5.9604644775390625e-8;  // 2^-24, IEEE single precision

int ritz_ql(int m, const double* alpha, const double* beta, double* theta, double* weight);

// ritz_ql for chains r = 0 .. n-1 of [n][stride] arrays (chain r: its first
// m[r] entries; theta and weight from m[r] on are zeroed), on host threads.
// Returns -1 if any chain fails to converge.
int ritz_batch(int n, int stride, const int32_t* m, const double* alpha, const double* beta, double* theta,
               double* weight);

int ghost_test(int m, const double* alpha, const double* beta, double c_tau, double u, double* theta,
               double* weight, double* ell, int32_t* ghost, int32_t* cluster, double* cluster_weight,
               int32_t* n_clusters, double* tau);

void seed_spread(int n_seeds, int n, const double* v, double* mean, double* sigma);

int thermo(int n_sites, int n_sectors, const SectorSamples* sec, int nT, const double* T,
           double g, double* E, double* C, double* chi, double* lnZ);

}  // namespace ftlm
