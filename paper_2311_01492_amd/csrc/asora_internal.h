// asora_internal.h -- host-side declarations shared by the C ABI and the
// kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "asora_dev.h"

namespace asora {

constexpr int kRBins = 256;                      // radius bins of the scheduling sort
constexpr int kCtlCounter = 0;                   // 3 work counters (one per piece type)
constexpr int kCtlSeg = 4;                       // 4 segment starts
constexpr int kCtlHist = 16;                     // 3*kRBins histogram
constexpr int kCtlOffs = kCtlHist + 3 * kRBins;  // 3*kRBins scatter offsets
constexpr int kCtlSize = kCtlOffs + 3 * kRBins;

struct FwdLaunch {
    int N;
    double alpha, sigma0;
    float tau_w;
    int reading;
    TabParams tp;
    const TabNode *tab;
    const double *nHI;
    double *gacc;
    double *coldens;
    const int32_t *ijk;
    const double *Q;
    const float *R;
    float R_cap;
    const int *order;
    int *ctl;
    int *err;
    int type;
    int ring_cap, row_cap;
};

hipError_t launch_prologue(hipStream_t st, const float *nH, const float *xHI, double *nHI,
                           double *gacc, double *coldens, long n3, int *ctl, int nctl, int n_cu);
hipError_t launch_bucketing(hipStream_t st, const float *R, const int32_t *ijk, long nsrc, int N,
                            float R_max, float R_whole, float R_oct, int *keys, int *ctl,
                            int *order, int *err);
size_t fwd_lds_bytes(int n_tab, int ring_cap, int row_cap);
hipError_t fwd_configure(size_t max_lds);
hipError_t fwd_occupancy(size_t lds, int *blocks_per_cu);
hipError_t launch_fwd_persistent(hipStream_t st, const FwdLaunch &F, int grid);
hipError_t launch_fwd_plain(hipStream_t st, const FwdLaunch &F, int src);
size_t wave_region_bytes(int ring_cap, int row_cap);
hipError_t wave_occupancy(int type, int waves, size_t lds, int *blocks_per_cu);
hipError_t launch_fwd_wave(hipStream_t st, const FwdLaunch &F, int waves, int grid, int plain_src);
hipError_t launch_finalize(hipStream_t st, const double *gacc, float *gamma, long n3, int accumulate,
                           int n_cu);

struct AdjLaunch {
    int N;
    double alpha, sigma0;
    float tau_w;
    int reading;
    TabParams tp;
    const TabNode *tab;
    const double *m64;
    const double *nHI;
    const double *gbar;
    double *nbar;
    double *qbar;
    const int32_t *ijk;
    const double *Q;
    const float *R;
    float R_cap;
    const int *order;
    int *ctl;
    int *err;
    int type;
    int ring_cap, row_cap, shell_cap;
    int waves, grid;
    double *store;
    long store_stride;
};

size_t adj_region_bytes(int ring_cap, int row_cap, int shell_cap);
hipError_t adj_configure(size_t max_lds);
hipError_t adj_occupancy(int type, int waves, size_t lds, int *blocks_per_cu);
hipError_t launch_adj_prologue(hipStream_t st, const float *nH, const float *xHI, double *nHI,
                               double *nbar, long n3, double *qbar, long nsrc, int zero_q, int *ctl,
                               int nctl, int n_cu);
hipError_t launch_adj_wave(hipStream_t st, const AdjLaunch &L);
hipError_t launch_adj_finalize(hipStream_t st, const double *nbar, const float *nH, const float *xHI,
                               float *dnH, float *dxHI, long n3, int accumulate, int n_cu);

// host table builders (asora_tables.cpp)
int table_blackbody(double T_bb, double index, int n, double lg_lo, double lg_hi, double *P,
                    double *dP);
void prepare_table(int n, double lg_lo, double lg_hi, const double *P, const double *dP,
                   TabParams *tp, TabNode *nodes, double *m64);

}  // namespace asora
