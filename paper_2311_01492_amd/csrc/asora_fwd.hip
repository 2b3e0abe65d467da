// asora_fwd.hip -- forward ray-tracing kernels for gfx950.
//
// One work-group sweeps one piece of one source (see asora_dev.h): shell by
// shell in L1 distance q (Section 3.3), with the exit columns of the last
// four shells in an LDS ring (FP64), the photoionization table in LDS, and
// the rate of every owned cell added to an FP64 N^3 accumulator with one
// hardware atomic per source-cell.  The persistent kernel pulls
// (source, piece) items from a global counter, largest radius first.
#include <type_traits>

#include "asora_dev.h"
#include "asora_internal.h"

namespace asora {

constexpr int kWG = 256;

struct FwdArgs {
    int N;
    Extent ex;
    double alpha, sigma0;
    float tau_w;            // weight floor, <= 0: geometric weights
    int reading;            // 0: directional source half path, 1: scalar
    TabParams tp;
    const TabNode *tab;
    const double *nHI;
    double *gacc;
    double *coldens;
    const int32_t *ijk;
    const double *Q;
    const float *R;         // may be NULL: every source has R = R_cap
    float R_cap;
    const int *order;       // sources sorted by piece kind, then spatially (Morton blocks)
    const int *seg;         // seg[t] .. seg[t+1]: sources of type t in order[]
    int type, n_pieces;
    int *counter;
    int *err;
    int ring_cap, row_cap;
    int plain_src;          // >= 0: non-persistent launch for this source
    int region_bytes;       // per-wave LDS region (wave kernels)
    double coef_unit;       // sigma0 / (4 pi alpha^2)
    const double *nHI_T;    // n_HI in the [k][i][j] layout (layer pieces with d = k)
    double *gacc_T;         // Gamma accumulator in the [k][i][j] layout
    int lay_S;              // row stride of the per-wave layer buffer (layer pieces)
    char *keep;             // layer pieces: column records, per (source, pyramid); NULL = none
    size_t keep_piece_bytes;
    long keep_cap;          // cells (and listed cells) per pyramid record
    size_t keep_rk_off;     // offset of the rate coefficients in a kept record
    const double *m64;      // FP64 node slopes of the table (rate coefficients of kept records)
    int early_exit;         // layer pieces: stop after the first opaque layer
    const TabNode *tab_h;   // photo-heating table on the same node grid (read through the
                            // caches), or NULL: no heating
    double *hacc, *hacc_T;  // heating accumulators, in the layouts of gacc and gacc_T
    float dP0_h;            // dH/dtau at the first node (slope of the heating table's continuation)
    int sq_n;               // layer pieces: entries of the work-group's LDS table of sqrt(r^2)
                            // (r^2 < sq_n); 0: roots computed per cell
};

// The node grid's parameters with the heating table's end slope.
__device__ __forceinline__ TabParams heat_params(const FwdArgs &A)
{
    TabParams t = A.tp;
    t.dP0 = A.dP0_h;
    return t;
}

// Heating of one cell, added to hacc: the heating table's divided difference
// over the cell's optical depths, with the rate's coefficient (the same
// formula with H in place of P).
__device__ __forceinline__ void add_heating(const FwdArgs &A, double *hacc, uint32_t cp, double ta,
                                            double dt, int r2, double coef)
{
    const float nd = neg_divdiff(A.tab_h, heat_params(A), ta, dt);
    if (nd > 0.f) unsafeAtomicAdd(&hacc[cp], coef * (double)(nd * rcp_approx((float)r2)));
}

struct Lds {
    TabNode *tab;
    double *ring;      // [4][ring_cap]
    int *rowbase;      // [4][row_cap]: slot of (row, B) = rowbase[row] + B
    int *rowstart;     // [row_cap + 1] of the current shell
};

// Sweep one piece of one source.  Called by all threads of the work-group.
__device__ void sweep_piece(const FwdArgs &A, const Lds &L, int src, int p, int *sh_total)
{
    const int tid = threadIdx.x;
    const int N = A.N;
    const int si = A.ijk[3 * src], sj = A.ijk[3 * src + 1], sk = A.ijk[3 * src + 2];
    const float R = A.R ? A.R[src] : A.R_cap;
    if (!(R >= 0.f && R <= A.R_cap) || si < 0 || si >= N || sj < 0 || sj >= N || sk < 0 ||
        sk >= N) {
        if (tid == 0) atomicOr(A.err, 1);
        return;
    }
    const double Q = A.Q[src];
    const int Rsq = (int)floor((double)R * (double)R);
    const Piece pc = make_piece(A.type, p);
    const int Qmax = max_shell(Rsq, A.ex);
    const long cs = ((long)si * N + sj) * N + sk;
    const double n_s = A.nHI[cs];

    CellCtx X;
    X.pc = pc;
    X.N = N;
    X.si = si;
    X.sj = sj;
    X.sk = sk;
    X.reading = A.reading;
    X.tau_w = A.tau_w;
    X.sigma0 = A.sigma0;
    X.alpha = A.alpha;
    X.half_col = n_s * A.alpha * 0.5;
    X.coef = Q * A.coef_unit;
    X.tab = L.tab;
    X.m64 = nullptr;
    X.tp = A.tp;
    X.ring = L.ring;
    X.rowbase = L.rowbase;
    X.ring_cap = A.ring_cap;
    X.row_cap = A.row_cap;
    X.nHI = A.nHI;

    const bool src_owner = (pc.kind == 0) || (pc.oct == 0 && (pc.dom < 0 || pc.dom == 2));
    if (src_owner && tid == 0) {
        const double G = source_cell_rate(L.tab, A.tp, A.sigma0, A.alpha, Q, n_s);
        if (G != 0.0) unsafeAtomicAdd(&A.gacc[cs], G);
        if (A.coldens) A.coldens[cs] = 0.0;
        if (A.hacc) {
            const double H = source_cell_rate(A.tab_h, heat_params(A), A.sigma0, A.alpha, Q, n_s);
            if (H != 0.0) unsafeAtomicAdd(&A.hacc[cs], H);
        }
    }

    for (int q = 1; q <= Qmax; ++q) {
        const int slot = q & 3;
        const int nrows = pc.n_oct * (q + 1);
        // ---- row table of shell q (wave 0): counts, exclusive scan, bases
        if (tid < 64) {
            const int c = (nrows + 63) >> 6;
            const int r0 = tid * c;
            int sum = 0;
            for (int k = 0; k < c; ++k) {
                const int r = r0 + k;
                if (r < nrows) {
                    int blo, cnt;
                    row_range(pc, A.ex, Rsq, q, r, &blo, &cnt);
                    sum += cnt;
                }
            }
            int incl = sum;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(incl, off, 64);
                if (tid >= off) incl += t;
            }
            int run = incl - sum;
            for (int k = 0; k < c; ++k) {
                const int r = r0 + k;
                if (r < nrows) {
                    int blo, cnt;
                    row_range(pc, A.ex, Rsq, q, r, &blo, &cnt);
                    L.rowstart[r] = run;
                    L.rowbase[slot * A.row_cap + r] = run - blo;
                    run += cnt;
                }
            }
            if (tid == 63) {
                L.rowstart[nrows] = incl;
                *sh_total = incl;
            }
        }
        __syncthreads();
        const int total = *sh_total;
        const int *rb_q = L.rowbase + slot * A.row_cap;
        double *ring_q = L.ring + slot * A.ring_cap;
        for (int g = tid; g < total; g += kWG) {
            const int row = find_row(L.rowstart, nrows, g);
            CellOut co;
            cell_update(X, q, g, row, rb_q[row], co);
            ring_q[g] = co.Nout;
            if (co.owned) {
                if (co.G != 0.0) unsafeAtomicAdd(&A.gacc[co.cp], co.G);
                if (A.coldens) A.coldens[co.cp] = co.Nin;
                if (A.hacc)
                    add_heating(A, A.hacc, co.cp, A.sigma0 * co.Nin, A.sigma0 * co.dN, co.r2, X.coef);
            }
        }
        __syncthreads();
    }
}

static FwdArgs make_args(const FwdLaunch &F);

// Per-wave queue of pending rate evaluations (structure of arrays in LDS).
constexpr int kQueue = 128;
struct RateQueue {
    double *ta;     // entry optical depth
    float *dt;      // in-cell optical depth
    uint32_t *cp;   // cell index
    int *r2;        // squared distance (cells)
};

template <bool HEAT>
__device__ __forceinline__ void rate_batch(const FwdArgs &A, const TabNode *T, const RateQueue &Qa,
                                           int head, int lane, double coef, double *acc)
{
    const int pos = (head + lane) & (kQueue - 1);
    const double ta = Qa.ta[pos];
    const float nd = neg_divdiff(T, A.tp, ta, (double)Qa.dt[pos]);
    if (nd > 0.f) {
        const double G = coef * (double)(nd * rcp_approx((float)Qa.r2[pos]));
        unsafeAtomicAdd(&acc[Qa.cp[pos]], G);
    }
    if (HEAT) add_heating(A, A.hacc, Qa.cp[pos], ta, (double)Qa.dt[pos], Qa.r2[pos], coef);
}

template <int TYPE, bool HEAT>
__device__ void sweep_piece_wave(const FwdArgs &A, const TabNode *T, double *ring, int *rowbase,
                                 int *rowstart, const RateQueue &Qa, int src, int p, int lane)
{
    const int N = A.N;
    const int si = A.ijk[3 * src], sj = A.ijk[3 * src + 1], sk = A.ijk[3 * src + 2];
    const float R = A.R ? A.R[src] : A.R_cap;
    if (!(R >= 0.f && R <= A.R_cap) || si < 0 || si >= N || sj < 0 || sj >= N || sk < 0 ||
        sk >= N) {
        if (lane == 0) atomicOr(A.err, 1);
        return;
    }
    const double Q = A.Q[src];
    const int Rsq = (int)floor((double)R * (double)R);
    const Piece pc = make_piece(TYPE, p);
    const int Qmax = max_shell(Rsq, A.ex);
    const long cs = ((long)si * N + sj) * N + sk;
    const double n_s = A.nHI[cs];

    CellCtx X;
    X.pc = pc;
    X.N = N;
    X.si = si;
    X.sj = sj;
    X.sk = sk;
    X.reading = A.reading;
    X.tau_w = A.tau_w;
    X.sigma0 = A.sigma0;
    X.alpha = A.alpha;
    X.half_col = n_s * A.alpha * 0.5;
    X.coef = Q * A.coef_unit;
    X.tab = T;
    X.m64 = nullptr;
    X.tp = A.tp;
    X.ring = ring;
    X.rowbase = rowbase;
    X.ring_cap = A.ring_cap;
    X.row_cap = A.row_cap;
    X.nHI = A.nHI;

    const bool src_owner = (pc.kind == 0) || (pc.oct == 0 && (pc.dom < 0 || pc.dom == 2));
    if (src_owner && lane == 0) {
        const double G = source_cell_rate(T, A.tp, A.sigma0, A.alpha, Q, n_s);
        if (G != 0.0) unsafeAtomicAdd(&A.gacc[cs], G);
        if (A.coldens) A.coldens[cs] = 0.0;
        if (HEAT) {
            const double H = source_cell_rate(A.tab_h, heat_params(A), A.sigma0, A.alpha, Q, n_s);
            if (H != 0.0) unsafeAtomicAdd(&A.hacc[cs], H);
        }
    }
    int head = 0, tail = 0;   // rate queue positions (wave-uniform)

    for (int q = 1; q <= Qmax; ++q) {
        const int slot = q & 3;
        const int nrows = pc.n_oct * (q + 1);
        int *rb_q = rowbase + slot * A.row_cap;
        const int total = wave_build_rows(pc, A.ex, Rsq, q, lane, rowstart, rb_q);
        wave_sync();
        double *ring_q = ring + slot * A.ring_cap;
        // columns for 64 cells at a time; cells whose rate is non-zero (owned,
        // entry optical depth below the table end) go to the wave's queue, and
        // every full 64 queued rates are evaluated by all lanes together
        for (int g0 = 0; g0 < total; g0 += 64) {
            const int g = g0 + lane;
            bool want = false;
            CellOut co;
            co.Nin = 0.0;
            if (g < total) {
                const int row = find_row(rowstart, nrows, g);
                cell_update<false>(X, q, g, row, rb_q[row], co);
                ring_q[g] = co.Nout;
                if (co.owned) {
                    if (A.coldens) A.coldens[co.cp] = co.Nin;
                    want = A.sigma0 * co.Nin < A.tp.tau_hi;
                }
            }
            const uint64_t mask = __ballot(want);
            if (want) {
                const int pos = (tail + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                  __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u))) & (kQueue - 1);
                Qa.ta[pos] = A.sigma0 * co.Nin;
                Qa.dt[pos] = A.sigma0 * co.dN;
                Qa.cp[pos] = co.cp;
                Qa.r2[pos] = co.r2;
            }
            tail += __popcll(mask);
            if (tail - head >= 64) {
                wave_sync();
                rate_batch<HEAT>(A, T, Qa, head, lane, X.coef, A.gacc);
                head += 64;
                wave_sync();
            }
        }
        wave_sync();
    }
    // the rates still queued
    if (tail > head) {
        wave_sync();
        if (lane < tail - head) rate_batch<HEAT>(A, T, Qa, head, lane, X.coef, A.gacc);
        wave_sync();
    }
}

// One wave per piece; the work-group only shares the table.  Persistent
// (items from the global counter) or plain (item = wave index).
template <int TYPE, bool HEAT>
__device__ __forceinline__ void fwd_wave_body(const FwdArgs &A, char *smem)
{
    constexpr int npieces0 = TYPE == 0 ? 1 : (TYPE == 1 ? 8 : 24);
    if (A.plain_src < 0 && A.seg[TYPE + 1] == A.seg[TYPE]) return;   // no sources of this kind
    (void)npieces0;
    TabNode *T = (TabNode *)smem;
    {
        const int4 *s = (const int4 *)A.tab;
        int4 *d = (int4 *)smem;
        for (int k = threadIdx.x; k < A.tp.n; k += blockDim.x) d[k] = s[k];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    char *region = smem + (size_t)A.tp.n * sizeof(TabNode) + (size_t)wave * A.region_bytes;
    double *ring = (double *)region;
    RateQueue Qa;
    Qa.ta = ring + 4 * (size_t)A.ring_cap;
    Qa.dt = (float *)(Qa.ta + kQueue);
    Qa.cp = (uint32_t *)(Qa.dt + kQueue);
    Qa.r2 = (int *)(Qa.cp + kQueue);
    int *rowbase = Qa.r2 + kQueue;
    int *rowstart = rowbase + 4 * A.row_cap;
    constexpr int npieces = TYPE == 0 ? 1 : (TYPE == 1 ? 8 : 24);
    if (A.plain_src >= 0) {
        const int item = blockIdx.x * waves + wave;
        if (item < npieces)
            sweep_piece_wave<TYPE, HEAT>(A, T, ring, rowbase, rowstart, Qa, A.plain_src, item, lane);
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
        sweep_piece_wave<TYPE, HEAT>(A, T, ring, rowbase, rowstart, Qa, src, item % npieces, lane);
    }
}

template <int TYPE>
__global__ __launch_bounds__(1024) void fwd_wave(FwdArgs A)
{
    extern __shared__ __align__(16) char smem[];
    fwd_wave_body<TYPE, false>(A, smem);
}

// The same sweep, adding the photo-heating of every cell to hacc.
template <int TYPE>
__global__ __launch_bounds__(1024) void fwd_wave_heat(FwdArgs A)
{
    extern __shared__ __align__(16) char smem[];
    fwd_wave_body<TYPE, true>(A, smem);
}

// ---- layer pieces --------------------------------------------------------
// One wave sweeps one pyramid layer by layer (see LayerPiece).  Layer m is
// the rectangle of LayerRect, covered in chunks of 64 consecutive cells; the
// previous layer lives in the wave's LDS buffer and is overwritten in place:
// chunks go from the last to the first, and a cell reads only slots at or
// before its own (u, v) in lexicographic order, so every slot a chunk reads
// still holds layer m - 1 (the chunk's own writes follow its reads).  Rates go
// through the same per-wave queue as the shell sweep.  With KEEP the sweep
// also writes the pyramid's column record (the cells' layer-buffer entries and
// the chunks' masks of cells with a rate) for a later adjoint.
// The rate queue of the layer kernel: as RateQueue, with the squared distance
// in 16 bits (a layer buffer that fits the LDS bounds the radius: R^2 stays
// below 2^16, which the plan checks).  The in-cell optical depth is rounded to
// FP32 as in RateQueue (a relative change of 6e-8 in one argument of the
// rate), except with KEEP: the rate coefficients of kept records are FP64
// derivatives that the adjoint combines with cancellation, so they are taken
// at the same point as the adjoint's own.
template <bool KEEP>
struct LayerQueue {
    using dt_t = typename std::conditional<KEEP, double, float>::type;
    double *ta;     // entry optical depth
    dt_t *dt;       // in-cell optical depth
    uint32_t *cp;   // cell index
    uint16_t *r2;   // squared distance (cells)
};

// One batch of queued cells: the rate added to Gamma.  Without KEEP the
// rate comes from the FP32 divided difference; with KEEP from the FP64 one
// that also gives the rate's coefficients for the adjoint (one evaluation
// instead of two), which are stored in the record at the cells' places in
// the order of evaluation (head + lane).
template <bool KEEP, bool HEAT>
__device__ __forceinline__ void layer_rate_batch(const FwdArgs &A, const TabNode *T, const LayerQueue<KEEP> &Qa,
                                                 int head, int lane, double coef, double *acc,
                                                 double *hacc, const LayerRecord &rec)
{
    const int pos = (head + lane) & (kQueue - 1);
    const double ta = Qa.ta[pos], dt = (double)Qa.dt[pos];
    const int r2 = Qa.r2[pos];
    if (!KEEP) {
        const float nd = neg_divdiff(T, A.tp, ta, dt);
        if (nd > 0.f) {
            const double G = coef * (double)(nd * rcp_approx((float)r2));
            unsafeAtomicAdd(&acc[Qa.cp[pos]], G);
        }
    } else {
        double c[3];
        layer_rate_coefs(T, A.m64, A.tp, A.sigma0, ta, dt, r2, c);
        const double G = coef * c[2];   // Gamma = coef (-D) / r2
        if (G != 0.0) unsafeAtomicAdd(&acc[Qa.cp[pos]], G);
        const long q = head + lane;
        rec.rk[q] = c[0];
        rec.rk[A.keep_cap + q] = c[1];
        rec.rk[2 * A.keep_cap + q] = c[2];
    }
    if (HEAT) add_heating(A, hacc, Qa.cp[pos], ta, dt, r2, coef);
}

template <bool KEEP, bool HEAT>
__device__ void sweep_layer_piece(const FwdArgs &A, const TabNode *T, const double *sq, double *lay, Geo *geo,
                                  uint32_t *iu, uint32_t *iv, const LayerQueue<KEEP> &Qa, int src, int p, int lane)
{
    const int N = A.N;
    const int si = A.ijk[3 * src], sj = A.ijk[3 * src + 1], sk = A.ijk[3 * src + 2];
    const float R = A.R ? A.R[src] : A.R_cap;
    if (!(R >= 0.f && R <= A.R_cap) || si < 0 || si >= N || sj < 0 || sj >= N || sk < 0 ||
        sk >= N) {
        if (lane == 0) atomicOr(A.err, 1);
        return;
    }
    const double Q = A.Q[src];
    const int Rsq = (int)floor((double)R * (double)R);
    const LayerPiece L = make_layer_piece(p, si, sj, sk, N, A.ex);
    const uint32_t cs = ((uint32_t)si * (uint32_t)N + (uint32_t)sj) * (uint32_t)N + (uint32_t)sk;
    const double n_s = A.nHI[cs];
    LayerX X;
    X.N = N;
    X.reading = A.reading;
    X.tau_w = A.tau_w;
    X.sigma0 = A.sigma0;
    X.alpha = A.alpha;
    X.half_col = n_s * A.alpha * 0.5;
    X.nHI = L.transposed ? A.nHI_T : A.nHI;
    layer_x_weights(X);
    double *acc = L.transposed ? A.gacc_T : A.gacc;
    double *hacc = HEAT ? (L.transposed ? A.hacc_T : A.hacc) : nullptr;
    const double coef = Q * A.coef_unit;
    const int S = A.lay_S;
    LayerRecord rec;
    if (KEEP)
        rec = layer_record_at(A.keep + ((size_t)src * 24 + p) * A.keep_piece_bytes, A.keep_cap,
                              A.keep_rk_off);

    if (p == 3 * 0 + 2 && lane == 0) {   // the source cell, once per source
        const double G = source_cell_rate(T, A.tp, A.sigma0, A.alpha, Q, n_s);
        if (G != 0.0) unsafeAtomicAdd(&A.gacc[cs], G);
        if (A.coldens) A.coldens[cs] = 0.0;
        if (HEAT) {
            const double H = source_cell_rate(A.tab_h, heat_params(A), A.sigma0, A.alpha, Q, n_s);
            if (H != 0.0) unsafeAtomicAdd(&A.hacc[cs], H);
        }
    }
    const int Mx = min(isqrt_floor(Rsq), L.ext_d);
    const int P = S + 1;   // row stride of the padded layer buffer
    for (int k = lane; k < P * P; k += 64) lay[k] = 0.0;   // finite everywhere it is read
    for (int k = lane; k < S; k += 64) {                   // the pyramid's index terms
        iu[k] = layer_idx_u(L, N, k);
        iv[k] = layer_idx_v(L, N, k);
    }
    wave_sync();
    int head = 0, tail = 0;
    long off = 0;     // first cell of layer m in the record
    long choff = 0;   // first chunk of layer m in the record
    const double opaque = layer_opaque(A.tp.tau_hi);
    // the last layer swept, recorded and visited by the adjoint: every layer,
    // unless the early exit stops the pyramid at its first opaque layer
    int m_last = Mx;
    const bool watch = A.early_exit;
    for (int m = 1; m <= Mx; ++m) {
        const LayerRect r = layer_rect(L.ext_u, L.ext_v, Rsq, m);
        const double inv_m = rcp_f64((double)m);
        const int nch = (r.total + 63) / 64;
        // the bilinear factors of this layer's offsets (the previous layer's
        // readers are done: every chunk ends with a wave barrier)
        for (int k = lane; k < S; k += 64) geo[k] = layer_geo(m, inv_m, k);
        wave_sync();
        RectWalk w;
        w.init(r, (nch - 1) * 64 + lane);
        bool opq = true;   // every cell of layer m so far leaves opaque
        const int m2 = mul24(m, m);
        const uint32_t idx_d = layer_idx_d(L, N, m);
        for (int c = nch - 1; c >= 0; --c, w.down()) {
            const int g = c * 64 + lane;
            const int u = w.u, v = w.v;
            const int uv2 = mul24(u, u) + mul24(v, v);
            const bool act = g < r.total && uv2 <= r.rem;
            const int pos = layer_slot(u, v, P);
            LayerCell lc;
            lc.Nin = 0.0;
            lc.owned = false;
            if (act) {
                const uint32_t cp = idx_d + iu[u] + iv[v];
                const int r2 = m2 + uv2;   // <= Rsq < sq_n when the table is there
                const double rt = A.sq_n ? sq[r2] : sqrt_fast((double)r2);
                layer_cell_core(L, X, m, u, v, geo[u], geo[v], rt * inv_m, r2, cp, X.nHI[cp], lay[pos],
                                lay[pos - P], lay[pos - 1], lay[pos - P - 1], lc);
            }
            wave_sync();   // every read of layer m - 1 before the writes below
            bool want = false;
            if (act) {
                lay[pos] = lc.h;
                if (KEEP) rec.h[off + g] = lc.h;
                if (lc.owned) {
                    if (A.coldens) A.coldens[layer_std_index(L, N, m, u, v)] = lc.Nin;
                    want = A.sigma0 * lc.Nin < A.tp.tau_hi;
                }
            }
            const uint64_t mask = __ballot(want);
            if (KEEP && lane == 0) rec.lit[choff + c] = mask;
            if (watch) opq = opq && __ballot(act && !(A.sigma0 * lc.Nout >= opaque)) == 0;
            if (want) {
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                const int qpos = (tail + rank) & (kQueue - 1);
                Qa.ta[qpos] = A.sigma0 * lc.Nin;
                Qa.dt[qpos] = (typename LayerQueue<KEEP>::dt_t)(A.sigma0 * lc.dN);
                Qa.cp[qpos] = lc.cp;
                Qa.r2[qpos] = (uint16_t)lc.r2;
            }
            tail += __popcll(mask);
            if (tail - head >= 64) {
                wave_sync();
                layer_rate_batch<KEEP, HEAT>(A, T, Qa, head, lane, coef, acc, hacc, rec);
                head += 64;
            }
            wave_sync();
        }
        off += r.total;
        choff += nch;
        if (watch && opq) {
            m_last = m;
            break;   // every later cell has a zero rate
        }
    }
    if (tail > head) {
        wave_sync();
        if (lane < tail - head) layer_rate_batch<KEEP, HEAT>(A, T, Qa, head, lane, coef, acc, hacc, rec);
        wave_sync();
    }
    if (KEEP && lane == 0) {
        ((uint64_t *)rec.rk)[3 * A.keep_cap] = (uint64_t)tail;   // cells with a rate
        ((uint64_t *)rec.rk)[3 * A.keep_cap + 1] = (uint64_t)m_last;
    }
}

// TLDS: the table is copied to LDS once per work-group; otherwise the rate
// batches read it through the caches, which leaves the LDS to more waves.
// The work-group also holds the table of square roots when the launch gives
// one (sq_n > 0: the plan adds it only where it costs no wave); every wave
// its own region (rate queue, layer buffer, per-layer and per-pyramid tables).
template <bool KEEP, bool TLDS, bool HEAT>
__device__ __forceinline__ void fwd_layer_body(const FwdArgs &A, char *smem)
{
    constexpr int TYPE = 3, npieces = 24;
    if (A.plain_src < 0 && A.seg[TYPE + 1] == A.seg[TYPE]) return;   // no sources of this kind
    const TabNode *T = TLDS ? (const TabNode *)smem : A.tab;
    if (TLDS) {
        const int4 *s = (const int4 *)A.tab;
        int4 *d = (int4 *)smem;
        for (int k = threadIdx.x; k < A.tp.n; k += blockDim.x) d[k] = s[k];
    }
    char *wg = smem + (TLDS ? (size_t)A.tp.n * sizeof(TabNode) : 0);
    double *sq = (double *)wg;
    for (int k = threadIdx.x; k < A.sq_n; k += blockDim.x) sq[k] = sqrt((double)k);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    char *region = wg + (A.sq_n ? layer_sqrt_bytes(A.sq_n - 1) : 0) + (size_t)wave * A.region_bytes;
    LayerQueue<KEEP> Qa;
    Qa.ta = (double *)region;
    Qa.dt = (typename LayerQueue<KEEP>::dt_t *)(Qa.ta + kQueue);
    Qa.cp = (uint32_t *)(Qa.dt + kQueue);
    Qa.r2 = (uint16_t *)(Qa.cp + kQueue);
    double *lay = (double *)(Qa.r2 + kQueue);   // kQueue is a multiple of 4: aligned
    Geo *geo = (Geo *)(lay + (size_t)(A.lay_S + 1) * (A.lay_S + 1));
    uint32_t *iu = (uint32_t *)(geo + A.lay_S);
    uint32_t *iv = iu + A.lay_S;
    if (A.plain_src >= 0) {
        const int item = blockIdx.x * waves + wave;
        if (item < npieces) sweep_layer_piece<KEEP, HEAT>(A, T, sq, lay, geo, iu, iv, Qa, A.plain_src, item, lane);
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
        sweep_layer_piece<KEEP, HEAT>(A, T, sq, lay, geo, iu, iv, Qa, src, item % npieces, lane);
    }
}

template <bool KEEP, bool TLDS>
__global__ __launch_bounds__(1024) void fwd_layer(FwdArgs A)
{
    extern __shared__ __align__(16) char smem[];
    fwd_layer_body<KEEP, TLDS, false>(A, smem);
}

// The same sweep, adding the photo-heating of every cell to hacc / hacc_T
// (both tables through the caches).
template <bool KEEP>
__global__ __launch_bounds__(1024) void fwd_layer_heat(FwdArgs A)
{
    extern __shared__ __align__(16) char smem[];
    fwd_layer_body<KEEP, false, true>(A, smem);
}

// Per-wave LDS of the layer kernel: the rate queue (its in-cell optical depths
// in FP64 with keep), the (S + 1) x (S + 1) padded layer buffer, the layer's
// table of bilinear factors and the pyramid's index terms along u and v.
size_t layer_region_bytes(int S, bool keep)
{
    const size_t dt = keep ? sizeof(double) : sizeof(float);
    const size_t b = (size_t)kQueue * (sizeof(double) + dt + sizeof(uint32_t) + sizeof(uint16_t)) +
                     (size_t)(S + 1) * (S + 1) * sizeof(double) + (size_t)S * sizeof(Geo) +
                     2 * (size_t)S * sizeof(uint32_t);
    return (b + 15) & ~(size_t)15;
}

hipError_t layer_occupancy(bool keep, bool tab_lds, int waves, size_t lds, int *blocks_per_cu)
{
    const void *f = keep ? (tab_lds ? (const void *)fwd_layer<true, true> : (const void *)fwd_layer<true, false>)
                         : (tab_lds ? (const void *)fwd_layer<false, true> : (const void *)fwd_layer<false, false>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, waves * 64, lds);
}

hipError_t launch_fwd_layer(hipStream_t st, const FwdLaunch &F, int S, int waves, int grid,
                            int plain_src)
{
    FwdArgs A = make_args(F);
    A.plain_src = plain_src;
    A.lay_S = S;
    A.region_bytes = (int)layer_region_bytes(S, A.keep != nullptr);
    const int Rsq = (int)floor((double)F.R_cap * (double)F.R_cap);
    const size_t sqb = F.sq_table ? layer_sqrt_bytes(Rsq) : 0;
    A.sq_n = sqb ? Rsq + 1 : 0;
    const bool tab_lds = F.tab_lds && !F.hacc;   // the heating sweep reads both tables through the caches
    const size_t lds = (tab_lds ? (size_t)F.tp.n * sizeof(TabNode) : 0) + sqb + (size_t)waves * A.region_bytes;
    if (plain_src >= 0) grid = (24 + waves - 1) / waves;
    const dim3 g(grid), b(64 * waves);
    if (F.hacc && A.keep) hipLaunchKernelGGL((fwd_layer_heat<true>), g, b, lds, st, A);
    else if (F.hacc) hipLaunchKernelGGL((fwd_layer_heat<false>), g, b, lds, st, A);
    else if (A.keep && F.tab_lds) hipLaunchKernelGGL((fwd_layer<true, true>), g, b, lds, st, A);
    else if (A.keep) hipLaunchKernelGGL((fwd_layer<true, false>), g, b, lds, st, A);
    else if (F.tab_lds) hipLaunchKernelGGL((fwd_layer<false, true>), g, b, lds, st, A);
    else hipLaunchKernelGGL((fwd_layer<false, false>), g, b, lds, st, A);
    return hipGetLastError();
}

size_t wave_region_bytes(int ring_cap, int row_cap)
{
    const size_t b = 4 * (size_t)ring_cap * sizeof(double) +
                     (size_t)kQueue * (sizeof(double) + sizeof(float) + sizeof(uint32_t) + sizeof(int)) +
                     (4 * (size_t)row_cap + row_cap + 1) * sizeof(int);
    return (b + 15) & ~(size_t)15;
}

hipError_t wave_occupancy(int type, int waves, size_t lds, int *blocks_per_cu)
{
    const void *f = type == 0 ? (const void *)fwd_wave<0> : (type == 1 ? (const void *)fwd_wave<1> : (const void *)fwd_wave<2>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, waves * 64, lds);
}

hipError_t launch_fwd_wave(hipStream_t st, const FwdLaunch &F, int waves, int grid, int plain_src)
{
    FwdArgs A = make_args(F);
    A.plain_src = plain_src;
    A.region_bytes = (int)wave_region_bytes(F.ring_cap, F.row_cap);
    const size_t lds = (size_t)F.tp.n * sizeof(TabNode) + (size_t)waves * A.region_bytes;
    if (plain_src >= 0) grid = (pieces_of_type(F.type) + waves - 1) / waves;
    if (F.hacc) {
        switch (F.type) {
        case 0: hipLaunchKernelGGL(fwd_wave_heat<0>, dim3(grid), dim3(64 * waves), lds, st, A); break;
        case 1: hipLaunchKernelGGL(fwd_wave_heat<1>, dim3(grid), dim3(64 * waves), lds, st, A); break;
        default: hipLaunchKernelGGL(fwd_wave_heat<2>, dim3(grid), dim3(64 * waves), lds, st, A); break;
        }
        return hipGetLastError();
    }
    switch (F.type) {
    case 0: hipLaunchKernelGGL(fwd_wave<0>, dim3(grid), dim3(64 * waves), lds, st, A); break;
    case 1: hipLaunchKernelGGL(fwd_wave<1>, dim3(grid), dim3(64 * waves), lds, st, A); break;
    default: hipLaunchKernelGGL(fwd_wave<2>, dim3(grid), dim3(64 * waves), lds, st, A); break;
    }
    return hipGetLastError();
}

__device__ Lds carve_lds(char *smem, const FwdArgs &A)
{
    Lds L;
    L.tab = (TabNode *)smem;
    L.ring = (double *)(smem + (size_t)A.tp.n * sizeof(TabNode));
    L.rowbase = (int *)(L.ring + 4 * (size_t)A.ring_cap);
    L.rowstart = L.rowbase + 4 * A.row_cap;
    return L;
}

__device__ void load_table(const FwdArgs &A, TabNode *dst)
{
    const int4 *s = (const int4 *)A.tab;
    int4 *d = (int4 *)dst;
    for (int k = threadIdx.x; k < A.tp.n; k += kWG) d[k] = s[k];
}

__global__ __launch_bounds__(kWG) void fwd_persistent(FwdArgs A)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int sh_item, sh_total;
    const Lds L = carve_lds(smem, A);
    load_table(A, L.tab);
    const int base = A.seg[A.type];
    const long nitems = (long)(A.seg[A.type + 1] - base) * A.n_pieces;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) sh_item = atomicAdd(A.counter, 1);
        __syncthreads();
        const long item = sh_item;
        if (item >= nitems) break;
        const int src = A.order[base + (int)(item / A.n_pieces)];
        const int p = (int)(item % A.n_pieces);
        sweep_piece(A, L, src, p, &sh_total);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void fwd_plain(FwdArgs A)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int sh_total;
    const Lds L = carve_lds(smem, A);
    load_table(A, L.tab);
    __syncthreads();
    sweep_piece(A, L, A.plain_src, blockIdx.x, &sh_total);
}

// ---- small kernels: n_HI, accumulators, bucketing, final conversion --------

__global__ void prologue_kernel(const float *__restrict__ nH, const float *__restrict__ xHI,
                                double *__restrict__ nHI, double *__restrict__ gacc,
                                double *__restrict__ coldens, long n3, int *ctl, int nctl)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n3; c += stride) {
        nHI[c] = (double)nH[c] * (double)xHI[c];   // exact
        gacc[c] = 0.0;
        if (coldens) coldens[c] = 0.0;
    }
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < nctl; k += blockDim.x) ctl[k] = 0;
}

// Morton index of the 16^3 block that holds cell (i, j, k).
__device__ __forceinline__ int block_morton(int i, int j, int k, int N)
{
    const int bi = (int)((long)i * 16 / N), bj = (int)((long)j * 16 / N), bk = (int)((long)k * 16 / N);
    int m = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        m |= (((bi >> b) & 1) << (3 * b + 2)) | (((bj >> b) & 1) << (3 * b + 1)) | (((bk >> b) & 1) << (3 * b));
    return m;
}

// Source pre-pass: piece kind by radius, then the spatial block of the source
// in Morton order, so that sources swept at the same time lie close together
// and share cached field and accumulator lines.
__global__ void classify_kernel(const float *R, const int32_t *ijk, long nsrc, int N, float R_max,
                                float R_whole, float R_oct, int big_type, int *keys, int *hist,
                                int *err)
{
    const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (s >= nsrc) return;
    const float r = R ? R[s] : R_max;
    const int i = ijk[3 * s], j = ijk[3 * s + 1], k = ijk[3 * s + 2];
    int key;
    if (!(r >= 0.f && r <= R_max) || i < 0 || i >= N || j < 0 || j >= N || k < 0 || k >= N) {
        atomicOr(err, 1);
        key = kTypes * kSBins;   // not scheduled
    } else {
        const int type = r <= R_whole ? 0 : (r <= R_oct ? 1 : big_type);
        key = type * kSBins + block_morton(i, j, k, N);
        atomicAdd(&hist[key], 1);
    }
    keys[s] = key;
}

// Exclusive scan of the kTypes*kSBins histogram by one work-group of kScanThreads
// threads (each owns a run of consecutive bins); offsets and per-kind segment
// starts.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void scan_kernel(const int *hist, int *offs, int *seg)
{
    constexpr int n = kTypes * kSBins;
    constexpr int per = (n + kScanThreads - 1) / kScanThreads;
    __shared__ int wsum[kScanThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int v[per];
    int sum = 0;
#pragma unroll
    for (int u = 0; u < per; ++u) {
        const int b = t * per + u;
        v[u] = b < n ? hist[b] : 0;
        sum += v[u];
    }
    int incl = sum;   // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int x = __shfl_up(incl, off, 64);
        if (lane >= off) incl += x;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    int run = before + incl - sum;
#pragma unroll
    for (int u = 0; u < per; ++u) {
        const int b = t * per + u;
        if (b < n) {
            offs[b] = run;
            if (b % kSBins == 0) seg[b / kSBins] = run;
        }
        run += v[u];
    }
    if (t == kScanThreads - 1) seg[kTypes] = run;
}

__global__ void scatter_kernel(const int *keys, long nsrc, int *offs, int *order)
{
    const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (s >= nsrc) return;
    const int key = keys[s];
    if (key >= kTypes * kSBins) return;
    const int pos = atomicAdd(&offs[key], 1);
    order[pos] = (int)s;
}

// n_HI and the zeroed accumulator in the [k][i][j] layout used by the layer
// pieces whose dominant axis is k: one 32 x 32 (j, k) tile of one i plane
// per work-group, staged through LDS so that both the reads (along k) and the
// writes (along j) are contiguous.
constexpr int kTile = 32;
__global__ __launch_bounds__(256) void transpose_prologue_kernel(const float *__restrict__ nH,
                                                                 const float *__restrict__ xHI,
                                                                 double *__restrict__ nHI_T,
                                                                 double *__restrict__ gacc_T, int N)
{
    __shared__ double tile[kTile][kTile + 1];
    const int k0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile, i = blockIdx.z;
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;   // 32 x 8
    for (int jj = ty; jj < kTile; jj += 8) {
        const int j = j0 + jj, k = k0 + tx;
        if (j < N && k < N) {
            const size_t c = ((size_t)i * N + j) * N + k;
            tile[jj][tx] = (double)nH[c] * (double)xHI[c];   // exact
        }
    }
    __syncthreads();
    for (int kk = ty; kk < kTile; kk += 8) {
        const int k = k0 + kk, j = j0 + tx;
        if (j < N && k < N) {
            const size_t t = ((size_t)k * N + i) * N + j;
            nHI_T[t] = tile[tx][kk];
            gacc_T[t] = 0.0;
        }
    }
}

// Gamma = accumulator + transposed accumulator, in the standard layout.
__global__ __launch_bounds__(256) void transpose_finalize_kernel(const double *__restrict__ gacc,
                                                                 const double *__restrict__ gacc_T,
                                                                 float *__restrict__ gamma, int N,
                                                                 int accumulate)
{
    __shared__ double tile[kTile][kTile + 1];
    const int k0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile, i = blockIdx.z;
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    for (int kk = ty; kk < kTile; kk += 8) {
        const int k = k0 + kk, j = j0 + tx;
        if (j < N && k < N) tile[kk][tx] = gacc_T[((size_t)k * N + i) * N + j];
    }
    __syncthreads();
    for (int jj = ty; jj < kTile; jj += 8) {
        const int j = j0 + jj, k = k0 + tx;
        if (j < N && k < N) {
            const size_t c = ((size_t)i * N + j) * N + k;
            const float v = (float)(gacc[c] + tile[tx][jj]);
            gamma[c] = accumulate ? gamma[c] + v : v;
        }
    }
}

// Clears an accumulator (a kernel: no memset node where the caller records
// the launch into a graph).
__global__ void zero_kernel(double *__restrict__ p, long n)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n; c += stride) p[c] = 0.0;
}

__global__ void finalize_kernel(const double *__restrict__ gacc, float *__restrict__ gamma, long n3,
                                int accumulate)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n3; c += stride) {
        const float v = (float)gacc[c];
        gamma[c] = accumulate ? gamma[c] + v : v;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C ABI in asora_api.hip)
// ---------------------------------------------------------------------------
hipError_t launch_prologue(hipStream_t st, const float *nH, const float *xHI, double *nHI,
                           double *gacc, double *coldens, long n3, int *ctl, int nctl, int n_cu)
{
    const int blocks = n_cu * 8;
    hipLaunchKernelGGL(prologue_kernel, dim3(blocks), dim3(256), 0, st, nH, xHI, nHI, gacc,
                       coldens, n3, ctl, nctl);
    return hipGetLastError();
}

hipError_t launch_transpose_prologue(hipStream_t st, const float *nH, const float *xHI, double *nHI_T,
                                     double *gacc_T, int N)
{
    const dim3 grid((N + kTile - 1) / kTile, (N + kTile - 1) / kTile, N);
    hipLaunchKernelGGL(transpose_prologue_kernel, grid, dim3(256), 0, st, nH, xHI, nHI_T, gacc_T, N);
    return hipGetLastError();
}

hipError_t launch_transpose_finalize(hipStream_t st, const double *gacc, const double *gacc_T,
                                     float *gamma, int N, int accumulate)
{
    const dim3 grid((N + kTile - 1) / kTile, (N + kTile - 1) / kTile, N);
    hipLaunchKernelGGL(transpose_finalize_kernel, grid, dim3(256), 0, st, gacc, gacc_T, gamma, N,
                       accumulate);
    return hipGetLastError();
}

hipError_t launch_bucketing(hipStream_t st, const float *R, const int32_t *ijk, long nsrc, int N,
                            float R_max, float R_whole, float R_oct, int big_type, int *keys,
                            int *ctl, int *order, int *err)
{
    int *hist = ctl + kCtlHist, *offs = ctl + kCtlOffs, *seg = ctl + kCtlSeg;
    const int b = (int)((nsrc + 255) / 256);
    if (nsrc > 0) {
        hipLaunchKernelGGL(classify_kernel, dim3(b), dim3(256), 0, st, R, ijk, nsrc, N, R_max,
                           R_whole, R_oct, big_type, keys, hist, err);
    }
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, st, hist, offs, seg);
    if (nsrc > 0)
        hipLaunchKernelGGL(scatter_kernel, dim3(b), dim3(256), 0, st, keys, nsrc, offs, order);
    return hipGetLastError();
}

static FwdArgs make_args(const FwdLaunch &F)
{
    FwdArgs A;
    A.N = F.N;
    A.ex = make_extent(F.N);
    A.alpha = F.alpha;
    A.sigma0 = F.sigma0;
    A.tau_w = F.tau_w;
    A.reading = F.reading;
    A.tp = F.tp;
    A.tab = F.tab;
    A.nHI = F.nHI;
    A.gacc = F.gacc;
    A.coldens = F.coldens;
    A.nHI_T = F.nHI_T;
    A.gacc_T = F.gacc_T;
    A.lay_S = 0;
    A.keep = F.keep;
    A.keep_piece_bytes = F.keep_piece_bytes;
    A.keep_cap = F.keep_cap;
    A.keep_rk_off = F.keep_rk_off;
    A.m64 = F.m64;
    A.early_exit = F.early_exit ? 1 : 0;
    A.tab_h = F.tab_h;
    A.hacc = F.hacc;
    A.hacc_T = F.hacc_T;
    A.dP0_h = F.dP0_h;
    A.ijk = F.ijk;
    A.Q = F.Q;
    A.R = F.R;
    A.R_cap = F.R_cap;
    A.order = F.order;
    A.seg = F.ctl + kCtlSeg;
    A.type = F.type;
    A.n_pieces = pieces_of_type(F.type);
    A.counter = F.ctl + kCtlCounter + kXcds * kCounterPad * F.type;
    A.err = F.err;
    A.ring_cap = F.ring_cap;
    A.row_cap = F.row_cap;
    A.plain_src = -1;
    A.region_bytes = 0;
    A.coef_unit = F.sigma0 / (4.0 * M_PI * F.alpha * F.alpha);
    A.sq_n = 0;
    return A;
}

size_t fwd_lds_bytes(int n_tab, int ring_cap, int row_cap)
{
    return (size_t)n_tab * sizeof(TabNode) + 4 * (size_t)ring_cap * sizeof(double) +
           (4 * (size_t)row_cap + row_cap + 1) * sizeof(int);
}

hipError_t fwd_configure(size_t max_lds)
{
    // Best effort: the dynamic LDS limit of a kernel defaults to what the device
    // offers; raising it explicitly is only an opt-in where a runtime needs it.
    const int dyn = (int)max_lds - 64;   // leave room for the static LDS words
    (void)hipFuncSetAttribute((const void *)fwd_persistent,
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_plain, hipFuncAttributeMaxDynamicSharedMemorySize,
                              dyn);
    (void)hipFuncSetAttribute((const void *)fwd_wave<0>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_wave<1>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_wave<2>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_layer<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_layer<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_layer<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_layer<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_wave_heat<0>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_wave_heat<1>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_wave_heat<2>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_layer_heat<false>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void *)fwd_layer_heat<true>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipGetLastError();
    return hipSuccess;
}

hipError_t fwd_occupancy(size_t lds, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)fwd_persistent,
                                                        kWG, lds);
}

hipError_t launch_fwd_persistent(hipStream_t st, const FwdLaunch &F, int grid)
{
    const FwdArgs A = make_args(F);
    const size_t lds = fwd_lds_bytes(F.tp.n, F.ring_cap, F.row_cap);
    hipLaunchKernelGGL(fwd_persistent, dim3(grid), dim3(kWG), lds, st, A);
    return hipGetLastError();
}

hipError_t launch_fwd_plain(hipStream_t st, const FwdLaunch &F, int src)
{
    FwdArgs A = make_args(F);
    A.plain_src = src;
    const size_t lds = fwd_lds_bytes(F.tp.n, F.ring_cap, F.row_cap);
    hipLaunchKernelGGL(fwd_plain, dim3(A.n_pieces), dim3(kWG), lds, st, A);
    return hipGetLastError();
}

hipError_t launch_zero(hipStream_t st, double *p, long n, int n_cu)
{
    hipLaunchKernelGGL(zero_kernel, dim3(n_cu * 8), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t st, const double *gacc, float *gamma, long n3, int accumulate,
                           int n_cu)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(n_cu * 8), dim3(256), 0, st, gacc, gamma, n3,
                       accumulate);
    return hipGetLastError();
}

}  // namespace asora
