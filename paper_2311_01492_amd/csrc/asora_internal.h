// asora_internal.h -- host-side declarations shared by the C ABI and the
// kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "asora_dev.h"

namespace asora {

constexpr int kTypes = 4;                        // piece kinds: whole, octants, shell pyramids, layer pyramids
constexpr int kSBins = 4096;                     // spatial bins per piece kind (16^3 blocks, Morton order)
constexpr int kCtlCounter = 0;                   // work counters: kXcds per piece kind, one per
                                                 // 128-byte line (kCounterPad ints apart)
constexpr int kCtlSeg = kTypes * kXcds * kCounterPad;   // kTypes + 1 segment starts
constexpr int kCtlHist = kCtlSeg + kCounterPad;  // kTypes*kSBins histogram
constexpr int kCtlOffs = kCtlHist + kTypes * kSBins;  // kTypes*kSBins scatter offsets
constexpr int kCtlSize = kCtlOffs + kTypes * kSBins;

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
    const double *nHI_T;    // [k][i][j] copies used by the layer pieces (may be NULL otherwise)
    double *gacc_T;
    char *keep;             // layer pieces: column records per (source, pyramid), or NULL
    size_t keep_piece_bytes;
    long keep_cap;
    size_t keep_rk_off;     // offset of the rate coefficients in a kept record
    const double *m64;      // FP64 node slopes of the table
    bool early_exit;        // layer pieces: stop after the first opaque layer
    int tab_lds;            // layer pieces: table in LDS (1) or read through the caches (0)
    bool sq_table;          // layer pieces: the work-group's LDS table of sqrt(r^2) (else per cell)
    const TabNode *tab_h;   // photo-heating table (same node grid), or NULL: no heating
    double *hacc, *hacc_T;  // heating accumulators (layouts of gacc, gacc_T)
    float dP0_h;            // dH/dtau at the first node
};

hipError_t launch_prologue(hipStream_t st, const float *nH, const float *xHI, double *nHI,
                           double *gacc, double *coldens, long n3, int *ctl, int nctl, int n_cu);
hipError_t launch_bucketing(hipStream_t st, const float *R, const int32_t *ijk, long nsrc, int N,
                            float R_max, float R_whole, float R_oct, int big_type, int *keys,
                            int *ctl, int *order, int *err);
hipError_t launch_transpose_prologue(hipStream_t st, const float *nH, const float *xHI, double *nHI_T,
                                     double *gacc_T, int N);
hipError_t launch_transpose_finalize(hipStream_t st, const double *gacc, const double *gacc_T,
                                     float *gamma, int N, int accumulate);
hipError_t launch_zero(hipStream_t st, double *p, long n, int n_cu);
size_t layer_region_bytes(int S, bool keep);
hipError_t layer_occupancy(bool keep, bool tab_lds, int waves, size_t lds, int *blocks_per_cu);

// hydrogen chemistry step (asora_chem.hip)
struct ChemLaunch {
    long n;
    const float *gamma, *nH;
    const double *y0, *y_prev;     // start-of-step neutral fraction; previous <y> (may be NULL)
    double *y_avg, *y_end;
    float *y_avg32;
    double dt, alpha, c_h, ne_rtol, conv_rtol;
    int max_iter;
    unsigned long long *changed, *unconverged;
    int n_cu;
};
hipError_t launch_chemistry(hipStream_t st, const ChemLaunch &L);
hipError_t launch_chem_prepare(hipStream_t st, long n, const double *y0, double *y_avg, float *y_avg32,
                               unsigned long long *cnt, int n_cu);
hipError_t launch_chem_clear(hipStream_t st, unsigned long long *cnt);
hipError_t launch_fwd_layer(hipStream_t st, const FwdLaunch &F, int S, int waves, int grid,
                            int plain_src);
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
    const double *nHI_T;   // [k][i][j] copies for the layer pieces (may be NULL otherwise)
    const double *gbar_T;
    double *nbar_T;
    const char *kept;      // layer pieces: column records kept by the forward, or NULL
    size_t rec_piece_bytes;   // bytes of one pyramid's column record
    size_t rec_rk_off;        // kept records: offset of the rate coefficients
    long rec_cap;             // cells (and listed cells) per pyramid record
    bool split;               // layer pieces: rate terms of dense chunks in the reverse pass
    bool early_exit;          // layer pieces: stop at the first opaque layer
    bool sq_table;            // layer pieces: the work-group's LDS table of sqrt(r^2) (else per cell)
};

size_t adj_region_bytes(int ring_cap, int row_cap, int shell_cap);
hipError_t adj_configure(size_t max_lds);
hipError_t adj_occupancy(int type, int waves, size_t lds, int *blocks_per_cu);
hipError_t launch_adj_prologue(hipStream_t st, const float *nH, const float *xHI, double *nHI,
                               double *nbar, long n3, double *qbar, long nsrc, int zero_q, int *ctl,
                               int nctl, int n_cu);
hipError_t launch_adj_wave(hipStream_t st, const AdjLaunch &L);
constexpr int kAdjLayerWaves = 16;   // largest work-group of the layer adjoint (waves)
size_t adj_layer_region_bytes(int S);
hipError_t adj_layer_occupancy(bool kept, bool split, int waves, size_t lds, int *blocks_per_cu);
hipError_t launch_adj_layer(hipStream_t st, const AdjLaunch &L, int Mcap, int S);
hipError_t launch_adj_transpose_prologue(hipStream_t st, const float *nH, const float *xHI,
                                         const double *gbar, double *nHI_T, double *gbar_T,
                                         double *nbar_T, int N);
hipError_t launch_adj_transpose_finalize(hipStream_t st, const double *nbar, const double *nbar_T,
                                         const float *nH, const float *xHI, float *dnH, float *dxHI,
                                         int N, int accumulate);
hipError_t launch_adj_finalize(hipStream_t st, const double *nbar, const float *nH, const float *xHI,
                               float *dnH, float *dxHI, long n3, int accumulate, int n_cu);

// two absorbers, hydrogen and helium (asora_he.hip)
struct HeLaunch {
    int N;
    double alpha, sigma0;
    float tau_w;
    int reading;
    int nb, n_tab;
    const TabNode *tab;               // nb x n_tab
    TabParams tp[kMaxBands];
    double sH[kMaxBands], sHe[kMaxBands];
    const double *nHI, *nHeI, *nHI_T, *nHeI_T;
    double *gH, *gHe, *gH_T, *gHe_T;
    const int32_t *ijk;
    const double *Q;
    const float *R;
    float R_cap;
    const int *order;
    int *ctl;
    int *err;
    bool sq_table;                    // the work-group's LDS table of sqrt(r^2) (else per cell)
};
size_t he_region_bytes(int S);
hipError_t he_configure(size_t max_lds);
hipError_t he_occupancy(int waves, size_t lds, int *blocks_per_cu);
hipError_t launch_fwd_layer_he(hipStream_t st, const HeLaunch &H, int S, int waves, int grid, int plain_src);

// host table builders (asora_tables.cpp)
int table_blackbody(double T_bb, double index, int n, double lg_lo, double lg_hi, double *P,
                    double *dP);
int table_blackbody_heat(double T_bb, double index, int n, double lg_lo, double lg_hi, double *H,
                         double *dH);
int table_blackbody_band(double T_bb, double index, double e_lo_ev, double e_hi_ev, int n, double lg_lo,
                         double lg_hi, double *P, double *dP);
void prepare_table(int n, double lg_lo, double lg_hi, const double *P, const double *dP,
                   TabParams *tp, TabNode *nodes, double *m64);

}  // namespace asora
