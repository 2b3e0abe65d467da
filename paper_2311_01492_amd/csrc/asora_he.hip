// asora_he.hip -- forward sweep with two absorbers, hydrogen and helium (the
// extension the paper plans, Sections 2 and 6), for gfx950.
//
// Every source is swept as layer pyramids (asora_dev.h), one wave per
// pyramid.  The layer buffer holds two columns per cell: the HI column as its
// layer-buffer entry (the optical-depth weights of the hydrogen method, on
// the HI column at the HI threshold) and the HeI column itself; both are
// interpolated with the same weights.  The spectrum is split into bands:
// band b has its own table (its photons that survive an optical depth taken
// at its lower edge, on its own node grid) and the cross-sections sH[b],
// sHe[b] of HI and HeI there, so that its optical depth is
// sH[b] N_HI + sHe[b] N_HeI.  A cell's rate of species i is
// Q sum_b s_i,b (-D_b) / (4 pi alpha^2 r^2), D_b the divided difference of
// band b's table over the cell's optical depths (eq. sugg for each band, the
// band's absorbed photons shared between the species in proportion to their
// in-cell optical depths).  Rates are accumulated in FP64 like the hydrogen
// rate; the tables are read through the caches.
#include "asora_dev.h"
#include "asora_internal.h"

namespace asora {

struct HeArgs {
    int N;
    Extent ex;
    double alpha, sigma0;
    float tau_w;
    int reading;
    int nb;                     // bands
    const TabNode *tab;         // nb x n_tab nodes
    int n_tab;
    TabParams tp[kMaxBands];    // node grid (and end slope) of each band's table
    double sH[kMaxBands], sHe[kMaxBands];
    const double *nHI, *nHeI;       // [i][j][k]
    const double *nHI_T, *nHeI_T;   // [k][i][j]
    double *gH, *gHe, *gH_T, *gHe_T;
    const int32_t *ijk;
    const double *Q;
    const float *R;
    float R_cap;
    const int *order;
    const int *seg;
    int *counter;
    int *err;
    int plain_src;
    int lay_S;
    int region_bytes;
    int sq_n;
    double coef_unit;   // 1 / (4 pi alpha^2)
};

// Per-wave queue of cells with a rate: both entry columns, the cell index
// and (m << 16) | r^2 (r^2 < 2^16: the plan checks it).  The in-cell columns
// are recomputed by the batch exactly as the sweep formed them, which keeps
// the queue, and so the LDS per wave, small.
constexpr int kHeQueue = 128;
struct HeQueue {
    double *NinH, *NinHe;
    uint32_t *cp;
    uint32_t *mr;
};

// Rates of one queued cell (one lane): every band's divided difference,
// shared between the species by their cross-sections.  nH, nHe: the fields
// in the piece's layout.
__device__ __forceinline__ void he_rate(const HeArgs &A, const HeQueue &Qa, int pos, double coef, const double *sq,
                                        const double *nH, const double *nHe, double *gH, double *gHe)
{
    const double NH = Qa.NinH[pos], NHe = Qa.NinHe[pos];
    const uint32_t cp = Qa.cp[pos], mr = Qa.mr[pos];
    const int r2 = (int)(mr & 0xffffu), m = (int)(mr >> 16);
    const double ds = (A.sq_n ? sq[r2] : sqrt_fast((double)r2)) * rcp_f64((double)m);
    const double dH = nH[cp] * A.alpha * ds, dHe = nHe[cp] * A.alpha * ds;
    double sumH = 0.0, sumHe = 0.0;
    for (int b = 0; b < A.nb; ++b) {
        const double T = A.sH[b] * NH + A.sHe[b] * NHe;
        const double dT = A.sH[b] * dH + A.sHe[b] * dHe;
        const double nd = (double)neg_divdiff(A.tab + (size_t)b * A.n_tab, A.tp[b], T, dT);
        sumH += A.sH[b] * nd;
        sumHe += A.sHe[b] * nd;
    }
    const double k = coef * (double)rcp_approx((float)r2);
    if (sumH > 0.0) unsafeAtomicAdd(&gH[cp], k * sumH);
    if (sumHe > 0.0) unsafeAtomicAdd(&gHe[cp], k * sumHe);
}

// The source cell: entry column 0, path half a cell, volume alpha^3.
__device__ void he_source_cell(const HeArgs &A, uint32_t cs, double Q)
{
    const double nH = A.nHI[cs], nHe = A.nHeI[cs];
    double GH = 0.0, GHe = 0.0;
    for (int b = 0; b < A.nb; ++b) {
        const double dT = (A.sH[b] * nH + A.sHe[b] * nHe) * A.alpha * 0.5;
        const double nd = (double)neg_divdiff(A.tab + (size_t)b * A.n_tab, A.tp[b], 0.0, dT);
        GH += A.sH[b] * nd;
        GHe += A.sHe[b] * nd;
    }
    const double k = Q / (2.0 * A.alpha * A.alpha);
    if (GH != 0.0) unsafeAtomicAdd(&A.gH[cs], k * GH);
    if (GHe != 0.0) unsafeAtomicAdd(&A.gHe[cs], k * GHe);
}

__device__ void sweep_layer_piece_he(const HeArgs &A, const double *sq, double *lay, double *layHe, Geo *geo,
                                     uint32_t *iu, uint32_t *iv, const HeQueue &Qa, int src, int p, int lane)
{
    const int N = A.N;
    const int si = A.ijk[3 * src], sj = A.ijk[3 * src + 1], sk = A.ijk[3 * src + 2];
    const float R = A.R ? A.R[src] : A.R_cap;
    if (!(R >= 0.f && R <= A.R_cap) || si < 0 || si >= N || sj < 0 || sj >= N || sk < 0 || sk >= N) {
        if (lane == 0) atomicOr(A.err, 1);
        return;
    }
    const double Q = A.Q[src];
    const int Rsq = (int)floor((double)R * (double)R);
    const LayerPiece L = make_layer_piece(p, si, sj, sk, N, A.ex);
    const uint32_t cs = ((uint32_t)si * (uint32_t)N + (uint32_t)sj) * (uint32_t)N + (uint32_t)sk;
    LayerX X;
    X.N = N;
    X.reading = A.reading;
    X.tau_w = A.tau_w;
    X.sigma0 = A.sigma0;
    X.alpha = A.alpha;
    X.half_col = A.nHI[cs] * A.alpha * 0.5;
    X.nHI = L.transposed ? A.nHI_T : A.nHI;
    layer_x_weights(X);
    const double half_he = A.nHeI[cs] * A.alpha * 0.5;
    const double *nHe = L.transposed ? A.nHeI_T : A.nHeI;
    double *gH = L.transposed ? A.gH_T : A.gH;
    double *gHe = L.transposed ? A.gHe_T : A.gHe;
    const double coef = Q * A.coef_unit;
    const int S = A.lay_S;
    if (p == 3 * 0 + 2 && lane == 0) he_source_cell(A, cs, Q);   // once per source
    const int Mx = min(isqrt_floor(Rsq), L.ext_d);
    const int P = S + 1;
    for (int k = lane; k < P * P; k += 64) {
        lay[k] = 0.0;
        layHe[k] = 0.0;
    }
    for (int k = lane; k < S; k += 64) {
        iu[k] = layer_idx_u(L, N, k);
        iv[k] = layer_idx_v(L, N, k);
    }
    wave_sync();
    int head = 0, tail = 0;
    for (int m = 1; m <= Mx; ++m) {
        const LayerRect r = layer_rect(L.ext_u, L.ext_v, Rsq, m);
        const double inv_m = rcp_f64((double)m);
        const int nch = (r.total + 63) / 64;
        for (int k = lane; k < S; k += 64) geo[k] = layer_geo(m, inv_m, k);
        wave_sync();
        RectWalk w;
        w.init(r, (nch - 1) * 64 + lane);
        const int m2 = mul24(m, m);
        const uint32_t idx_d = layer_idx_d(L, N, m);
        for (int c = nch - 1; c >= 0; --c, w.down()) {
            const int g = c * 64 + lane;
            const int u = w.u, v = w.v;
            const int uv2 = mul24(u, u) + mul24(v, v);
            const bool act = g < r.total && uv2 <= r.rem;
            const int pos = layer_slot(u, v, P);
            LayerCell lc;
            lc.owned = false;
            double NinHe = 0.0, dNHe = 0.0;
            if (act) {
                const uint32_t cp = idx_d + iu[u] + iv[v];
                const int r2 = m2 + uv2;
                const double ds = (A.sq_n ? sq[r2] : sqrt_fast((double)r2)) * inv_m;
                const double h[4] = {lay[pos], lay[pos - P], lay[pos - 1], lay[pos - P - 1]};
                layer_cell_core(L, X, m, u, v, geo[u], geo[v], ds, r2, cp, X.nHI[cp], h[0], h[1], h[2], h[3],
                                lc);
                // the helium column with the same weights: N_He = sum s f M_He / sum s f
                if (m == 1) {
                    NinHe = X.reading == 0 ? half_he * ds : half_he;
                } else {
                    const double Mh[4] = {layHe[pos], layHe[pos - P], layHe[pos - 1], layHe[pos - P - 1]};
                    const double sw[4] = {geo[u].om * geo[v].om, geo[u].a * geo[v].om, geo[u].om * geo[v].a,
                                          geo[u].a * geo[v].a};
                    double num = 0.0, W = 0.0;
#pragma unroll
                    for (int n = 0; n < 4; ++n) {
                        const double wn = sw[n] * (h[n] > 0.0 ? h[n] : X.inv_tw);
                        num += wn * Mh[n];
                        W += wn;
                    }
                    NinHe = num * rcp_f64(W);
                }
                dNHe = nHe[cp] * A.alpha * ds;
            }
            wave_sync();   // every read of layer m - 1 before the writes below
            bool want = false;
            if (act) {
                lay[pos] = lc.h;
                layHe[pos] = NinHe + dNHe;
                if (lc.owned)
                    for (int b = 0; b < A.nb; ++b)
                        want = want || A.sH[b] * lc.Nin + A.sHe[b] * NinHe < A.tp[b].tau_hi;
            }
            const uint64_t mask = __ballot(want);
            if (want) {
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                const int q = (tail + rank) & (kHeQueue - 1);
                Qa.NinH[q] = lc.Nin;
                Qa.NinHe[q] = NinHe;
                Qa.cp[q] = lc.cp;
                Qa.mr[q] = ((uint32_t)m << 16) | (uint32_t)lc.r2;
            }
            tail += __popcll(mask);
            if (tail - head >= 64) {
                wave_sync();
                he_rate(A, Qa, (head + lane) & (kHeQueue - 1), coef, sq, X.nHI, nHe, gH, gHe);
                head += 64;
            }
            wave_sync();
        }
    }
    if (tail > head) {
        wave_sync();
        if (lane < tail - head) he_rate(A, Qa, (head + lane) & (kHeQueue - 1), coef, sq, X.nHI, nHe, gH, gHe);
        wave_sync();
    }
}

__global__ __launch_bounds__(1024) void fwd_layer_he(HeArgs A)
{
    extern __shared__ __align__(16) char smem[];
    constexpr int TYPE = 3, npieces = 24;
    if (A.plain_src < 0 && A.seg[TYPE + 1] == A.seg[TYPE]) return;   // no sources
    double *sq = (double *)smem;
    for (int k = threadIdx.x; k < A.sq_n; k += blockDim.x) sq[k] = sqrt((double)k);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    char *region = smem + (A.sq_n ? layer_sqrt_bytes(A.sq_n - 1) : 0) + (size_t)wave * A.region_bytes;
    HeQueue Qa;
    Qa.NinH = (double *)region;
    Qa.NinHe = Qa.NinH + kHeQueue;
    Qa.cp = (uint32_t *)(Qa.NinHe + kHeQueue);
    Qa.mr = Qa.cp + kHeQueue;
    const size_t PP = (size_t)(A.lay_S + 1) * (A.lay_S + 1);
    double *lay = (double *)(Qa.mr + kHeQueue);   // kHeQueue is even: aligned
    double *layHe = lay + PP;
    Geo *geo = (Geo *)(layHe + PP);
    uint32_t *iu = (uint32_t *)(geo + A.lay_S);
    uint32_t *iv = iu + A.lay_S;
    if (A.plain_src >= 0) {
        const int item = blockIdx.x * waves + wave;
        if (item < npieces) sweep_layer_piece_he(A, sq, lay, layHe, geo, iu, iv, Qa, A.plain_src, item, lane);
        return;
    }
    const int base = A.seg[TYPE];
    const int nitems = (A.seg[TYPE + 1] - base) * npieces;
    const int home = (int)(blockIdx.x % kXcds);
    int chunk = home;
    for (;;) {
        const int item = next_item(A.counter, nitems, home, chunk, lane);
        if (item >= nitems) break;
        const int src = A.order[base + item / npieces];
        sweep_layer_piece_he(A, sq, lay, layHe, geo, iu, iv, Qa, src, item % npieces, lane);
    }
}

size_t he_region_bytes(int S)
{
    const size_t b = (size_t)kHeQueue * (2 * sizeof(double) + 2 * sizeof(uint32_t)) +
                     2 * (size_t)(S + 1) * (S + 1) * sizeof(double) + (size_t)S * sizeof(Geo) +
                     2 * (size_t)S * sizeof(uint32_t);
    return (b + 15) & ~(size_t)15;
}

hipError_t he_configure(size_t max_lds)
{
    (void)hipFuncSetAttribute((const void *)fwd_layer_he, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)max_lds - 64);
    (void)hipGetLastError();
    return hipSuccess;
}

hipError_t he_occupancy(int waves, size_t lds, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)fwd_layer_he, waves * 64, lds);
}

hipError_t launch_fwd_layer_he(hipStream_t st, const HeLaunch &H, int S, int waves, int grid, int plain_src)
{
    HeArgs A;
    A.N = H.N;
    A.ex = make_extent(H.N);
    A.alpha = H.alpha;
    A.sigma0 = H.sigma0;
    A.tau_w = H.tau_w;
    A.reading = H.reading;
    A.nb = H.nb;
    A.tab = H.tab;
    A.n_tab = H.n_tab;
    for (int b = 0; b < kMaxBands; ++b) {
        A.tp[b] = H.tp[b < H.nb ? b : 0];
        A.sH[b] = b < H.nb ? H.sH[b] : 0.0;
        A.sHe[b] = b < H.nb ? H.sHe[b] : 0.0;
    }
    A.nHI = H.nHI;
    A.nHeI = H.nHeI;
    A.nHI_T = H.nHI_T;
    A.nHeI_T = H.nHeI_T;
    A.gH = H.gH;
    A.gHe = H.gHe;
    A.gH_T = H.gH_T;
    A.gHe_T = H.gHe_T;
    A.ijk = H.ijk;
    A.Q = H.Q;
    A.R = H.R;
    A.R_cap = H.R_cap;
    A.order = H.order;
    A.seg = H.ctl + kCtlSeg;
    A.counter = H.ctl + kCtlCounter + kXcds * kCounterPad * 3;
    A.err = H.err;
    A.plain_src = plain_src;
    A.lay_S = S;
    A.region_bytes = (int)he_region_bytes(S);
    const int Rsq = (int)floor((double)H.R_cap * (double)H.R_cap);
    const size_t sqb = H.sq_table ? layer_sqrt_bytes(Rsq) : 0;
    A.sq_n = sqb ? Rsq + 1 : 0;
    A.coef_unit = 1.0 / (4.0 * M_PI * H.alpha * H.alpha);
    const size_t lds = sqb + (size_t)waves * A.region_bytes;
    if (plain_src >= 0) grid = (24 + waves - 1) / waves;
    hipLaunchKernelGGL(fwd_layer_he, dim3(grid), dim3(64 * waves), lds, st, A);
    return hipGetLastError();
}

}  // namespace asora
