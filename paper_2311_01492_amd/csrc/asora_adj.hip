// asora_adj.hip -- adjoint (reverse-mode) ray-tracing kernels for gfx950.
//
// One wave per source piece, like the forward wave kernels.  For each piece
// the wave first recomputes the exit column of every cell, shell by shell
// (the forward sweep without the rate), keeping the last four shells in an
// LDS ring and storing every shell to the wave's own scratch in global
// memory together with its in-cell columns (so that the reverse pass reads
// them back in order instead of gathering n_HI again).  It then sweeps the
// shells from the outermost inward: the exit
// columns of shells q-1..q-3 (the neighbours of shell q) come back from the
// scratch into the LDS ring, and the adjoints of the exit columns of shells
// q..q-3 live in a second LDS ring that the cells of shell q update with LDS
// atomics when they push their entry-column adjoint to their neighbours.
// dL/dn_HI goes to an FP64 N^3 accumulator with hardware atomics; dL/dQ is
// reduced over the wave and added once per piece.
#include "asora_dev.h"
#include "asora_internal.h"

namespace asora {

// Layer adjoint work-groups: up to kAdjLayerNarrow waves the kernel may hold
// 168 VGPRs per lane (three waves per SIMD); the wide build, up to
// kAdjLayerWaves waves, is held to 128 (four per SIMD) and spills the rest.
// Which wins depends on the workload: the work-group size is tuned.
constexpr int kAdjLayerNarrow = 12;

struct AdjArgs {
    int N;
    Extent ex;
    double alpha, sigma0, coef_unit;
    float tau_w;
    int reading;
    TabParams tp;
    const TabNode *tab;
    const double *m64;       // FP64 node slopes
    const double *nHI;
    const double *gbar;      // dL/dGamma, N^3
    double *nbar;            // dL/dn_HI accumulator, N^3
    double *qbar;            // dL/dQ, n_src
    const int32_t *ijk;
    const double *Q;
    const float *R;
    float R_cap;
    const int *order;
    const int *seg;
    int *counter;
    int *err;
    int ring_cap, row_cap, shell_cap;
    int region_bytes;
    double *store;           // per wave: stored exit columns, then in-cell columns
    long store_stride;       // doubles per wave (twice the largest piece's cell count)
    // layer pieces
    const double *nHI_T;     // [k][i][j] copies for pyramids with dominant axis k
    const double *gbar_T;
    double *nbar_T;
    int Mcap, lay_S;         // largest layer index, row stride of the layer buffers
    const char *kept;        // column records kept by the forward (per source and pyramid), or NULL
    size_t rec_piece_bytes;  // bytes of one pyramid's column record
    size_t rec_rk_off;       // kept records: offset of the rate coefficients
    long rec_cap;            // cells (and listed cells) per pyramid record
    int early_exit;          // layer pieces: stop at the first opaque layer
    int sq_n;                // layer pieces: entries of the work-group's LDS table of sqrt(r^2); 0: none
};

template <int TYPE>
__device__ void adjoint_piece_wave(const AdjArgs &A, const TabNode *T, char *region, double *store,
                                   int src, int p, int lane)
{
    double *store_dN = store + A.store_stride / 2;   // in-cell columns, same indexing as store
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
    const uint32_t cs = ((uint32_t)si * (uint32_t)N + (uint32_t)sj) * (uint32_t)N + (uint32_t)sk;
    const double n_s = A.nHI[cs];

    // LDS region of this wave
    double *ring = (double *)region;                        // [4][ring_cap] exit columns
    double *abar = ring + 4 * (size_t)A.ring_cap;           // [4][ring_cap] their adjoints
    int *rowbase = (int *)(abar + 4 * (size_t)A.ring_cap);  // [4][row_cap]
    int *rowstart = rowbase + 4 * A.row_cap;                // [4][row_cap + 1]
    int *shoff = rowstart + 4 * (A.row_cap + 1);            // [shell_cap + 2] offsets in store

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
    X.m64 = A.m64;
    X.tp = A.tp;
    X.ring = ring;
    X.rowbase = rowbase;
    X.ring_cap = A.ring_cap;
    X.row_cap = A.row_cap;
    X.nHI = A.nHI;

    // ---- forward: exit columns of every shell, kept and stored
    if (lane == 0) shoff[1] = 0;
    wave_sync();
    for (int q = 1; q <= Qmax; ++q) {
        const int slot = q & 3;
        int *rs_q = rowstart + slot * (A.row_cap + 1);
        int *rb_q = rowbase + slot * A.row_cap;
        const int total = wave_build_rows(pc, A.ex, Rsq, q, lane, rs_q, rb_q);
        wave_sync();
        const int off = shoff[q];
        const int nrows = pc.n_oct * (q + 1);
        double *ring_q = ring + slot * (size_t)A.ring_cap;
        for (int g = lane; g < total; g += 64) {
            const int row = find_row(rs_q, nrows, g);
            CellOut co;
            cell_update<false>(X, q, g, row, rb_q[row], co);
            ring_q[g] = co.Nout;
            store[off + g] = co.Nout;
            store_dN[off + g] = co.dN;
        }
        if (lane == 0) shoff[q + 1] = off + total;
        wave_sync();
    }

    // ---- reverse
    for (int k = lane; k < 4 * A.ring_cap; k += 64) abar[k] = 0.0;
    wave_sync();
    double nb_src = 0.0, qb = 0.0;
    for (int q = Qmax; q >= 1; --q) {
        const int slot = q & 3;
        if (q < Qmax && q - 3 >= 1) {
            // shell q-3 enters the rings (its slot held shell q+1, finished)
            const int q3 = q - 3, s3 = q3 & 3;
            const int t3 = wave_build_rows(pc, A.ex, Rsq, q3, lane, rowstart + s3 * (A.row_cap + 1),
                                           rowbase + s3 * A.row_cap);
            const int off3 = shoff[q3];
            for (int g = lane; g < t3; g += 64) {
                ring[s3 * (size_t)A.ring_cap + g] = store[off3 + g];
                abar[s3 * (size_t)A.ring_cap + g] = 0.0;
            }
            wave_sync();
        }
        const int *rs_q = rowstart + slot * (A.row_cap + 1);
        const int *rb_q = rowbase + slot * A.row_cap;
        const int nrows = pc.n_oct * (q + 1);
        const int total = shoff[q + 1] - shoff[q];
        for (int g = lane; g < total; g += 64) {
            const int row = find_row(rs_q, nrows, g);
            CellAdj ca;
            cell_adjoint(X, q, g, row, rb_q[row], abar[slot * (size_t)A.ring_cap + g],
                         store_dN[shoff[q] + g], A.gbar, ca);
            if (ca.nbar != 0.0) unsafeAtomicAdd(&A.nbar[ca.cp], ca.nbar);
            nb_src += ca.nbar_src;
            qb += ca.qbar;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (ca.slot[k] >= 0)
                    atomicAdd(&abar[(ca.qn[k] & 3) * (size_t)A.ring_cap + ca.slot[k]], ca.Mbar[k]);
        }
        wave_sync();
    }
    const bool src_owner = (pc.kind == 0) || (pc.oct == 0 && (pc.dom < 0 || pc.dom == 2));
    if (src_owner && lane == 0) {
        double nb, q1;
        source_cell_adjoint(T, A.m64, A.tp, A.sigma0, A.alpha, Q, n_s, A.gbar[cs], &nb, &q1);
        nb_src += nb;
        qb += q1;
    }
    // wave sums
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        nb_src += __shfl_xor(nb_src, off, 64);
        qb += __shfl_xor(qb, off, 64);
    }
    if (lane == 0) {
        if (nb_src != 0.0) unsafeAtomicAdd(&A.nbar[cs], nb_src);
        if (qb != 0.0) unsafeAtomicAdd(&A.qbar[src], qb / Q);
    }
}

template <int TYPE>
__global__ __launch_bounds__(512) void adj_wave(AdjArgs A)
{
    extern __shared__ __align__(16) char smem[];
    if (A.seg[TYPE + 1] == A.seg[TYPE]) return;   // no sources of this kind
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
    double *store = A.store + (size_t)(blockIdx.x * waves + wave) * A.store_stride;
    constexpr int npieces = TYPE == 0 ? 1 : (TYPE == 1 ? 8 : 24);
    const int base = A.seg[TYPE];
    const int nitems = (A.seg[TYPE + 1] - base) * npieces;
    const int home = (int)(blockIdx.x % kXcds);
    int chunk = home;
    for (;;) {
        const int item = next_item(A.counter, nitems, home, chunk, lane);
        if (item >= nitems) break;
        const int src = A.order[base + item / npieces];
        adjoint_piece_wave<TYPE>(A, T, region, store, src, item % npieces, lane);
    }
}

// ---- layer pieces --------------------------------------------------------
// One wave per pyramid, in two passes.
//  (F) Unless the forward kept the pyramid's column record: the columns layer
//      by layer, in place in the LDS buffer as in the forward kernel, every
//      cell's layer-buffer entry written to the record in the wave's scratch
//      together with each chunk's mask of cells with a rate.  The cells with
//      a rate (SPLIT: only those in sparse chunks, fewer than kDenseChunk of
//      them) go to an LDS queue with their entry optical depth, and 64 at a
//      time, with every lane busy, get the FP64 rate derivatives, the rate's
//      in-cell term of dL/dn_HI, its share of dL/dQ, and its entry-column
//      term g_in, kept per cell in the wave's scratch.  With SPLIT, dense
//      chunks leave theirs to (R), which has the interpolation at hand;
//      without, the kernel holds fewer registers (more waves per SIMD).
//  (R) Layers from the outermost inward, each layer's rectangle in chunks
//      from the first to the last: every cell takes and clears its slot in
//      the LDS adjoint buffer (the adjoint of its exit column, pushed by its
//      consumers), adds its g_in if it has a rate (from (F), or evaluated
//      here in a dense chunk), adds alpha ds times the sum (and, in a dense
//      chunk, the rate's in-cell term) to dL/dn_HI with one atomic and pushes
//      it through the interpolation weights, read
//      from the record's entries of layer m - 1, to its neighbours' slots
//      with LDS atomics.  A neighbour slot precedes the pushing cell in (u, v)
//      order, so it was already taken in this layer.  Chunks with no rate and
//      all slots zero (cells no rate depends on) skip the arithmetic.
// The table is read from global memory (only cells with a rate use it),
// which leaves the LDS to the per-wave buffers.
__device__ __forceinline__ void wave_sync_global()
{
    // this wave's global stores complete before its later global loads by
    // other lanes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

constexpr int kAdjQueue = 128;   // queue entries per wave ((F) rate terms, (R) batches)

// The rate masks of chunks c0 .. c0 + 63 of a layer (first chunk at choff),
// one per lane, held in registers.
__device__ __forceinline__ uint64_t load_masks(const LayerRecord &rec, long choff, int c0, int nch, int lane)
{
    uint32_t lo = 0, hi = 0;
    if (c0 + lane < nch) {
        const uint64_t mk = rec.lit[choff + c0 + lane];
        lo = (uint32_t)mk;
        hi = (uint32_t)(mk >> 32);
    }
    // without this the compiler turns every readlane of the masks back into
    // a global load per chunk
    asm volatile("" : "+v"(lo), "+v"(hi));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t mask_of_chunk(uint64_t masks, int c)
{
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(masks >> 32), c & 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)masks, c & 63);
}

template <bool KEPT, bool SPLIT>
__device__ void adjoint_layer_piece(const AdjArgs &A, const TabNode *T, const double *sq, double *buf, Geo *geo,
                                    uint32_t *iu, uint32_t *iv, int *qk, int *qm, double *qT, char *scratch, int src,
                                    int p, int lane)
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
    const double *gbar = L.transposed ? A.gbar_T : A.gbar;
    double *nbar = L.transposed ? A.nbar_T : A.nbar;
    const double coef = Q * A.coef_unit;
    const int S = A.lay_S;
    const LayerRecord rec = layer_record_at(
        KEPT ? (char *)A.kept + ((size_t)src * 24 + p) * A.rec_piece_bytes : scratch, A.rec_cap,
        KEPT ? A.rec_rk_off : 0);
    double *gin = KEPT ? nullptr : (double *)(scratch + A.rec_piece_bytes);   // g_in by record cell
    const int Mx = min(isqrt_floor(Rsq), L.ext_d);
    constexpr int dense_at = SPLIT ? kDenseChunk : 65;   // popcount of a dense chunk
    // (R) queues the cells with work into full batches, except in the split
    // form (most cells have a rate there, and most lanes work anyway)
    constexpr bool QUEUE = KEPT || !SPLIT;

    // the pyramid's index terms along u and v (every pass)
    for (int k = lane; k < S; k += 64) {
        iu[k] = layer_idx_u(L, N, k);
        iv[k] = layer_idx_v(L, N, k);
    }
    wave_sync();

    // ---- (F), every layer; with the early exit only up to the first layer
    // whose cells all leave opaque (layer_opaque): later layers have no rate
    // and no adjoint.  Kept records hold the layers their forward swept.
    // Unless the forward kept the rate's coefficients, (F) also evaluates the
    // rate's terms (g_in by record cell, dL/dn_HI and dL/dQ shares) of the
    // cells with a rate that (R) does not take in place (all of them in the
    // gathered form, those of sparse chunks in the split one): such cells go
    // to the wave's queue with their entry optical depth and place (m, g),
    // and every full 64 are evaluated by all lanes together.
    double nb_src = 0.0, qb = 0.0;
    long off = 0, choff = 0;   // the record's cells and chunks of layers 1 .. Mt
    int Mt = Mx;   // the last layer (R) visits
    if (KEPT) {
        const int ml = (int)((const uint64_t *)rec.rk)[3 * A.rec_cap + 1];
        Mt = ml < Mx ? ml : Mx;
        for (int m = 1; m <= Mt; ++m) {
            const int t = layer_rect(L.ext_u, L.ext_v, Rsq, m).total;
            off += t;
            choff += (t + 63) / 64;
        }
    } else {
        const bool watch = A.early_exit != 0;
        const int P = S + 1;   // row stride of the padded layer buffer
        for (int k = lane; k < P * P; k += 64) buf[k] = 0.0;   // finite everywhere it is read
        wave_sync();
        const double opaque = layer_opaque(A.tp.tau_hi);
        // the queue: record cell (qk), (m << 16) | g (qm), entry optical depth (qT)
        int head = 0, tail = 0;
        auto batch = [&](int count) {
            if (lane < count) {
                const int q = (head + lane) & (kAdjQueue - 1);
                const int k = qk[q], mg = qm[q];
                const double ta = qT[q];
                const int m = mg >> 16, g = mg & 0xffff;
                int u, v;
                rect_cell(layer_rect(L.ext_u, L.ext_v, Rsq, m), g, u, v);
                // the cell's index, distance and in-cell column as (F) formed them
                const uint32_t cp = layer_idx_d(L, N, m) + iu[u] + iv[v];
                const int r2 = mul24(m, m) + mul24(u, u) + mul24(v, v);
                const double rt = A.sq_n ? sq[r2] : sqrt_fast((double)r2);
                const double ds = rt * rcp_f64((double)m);
                const double gb = gbar[cp];
                double gi = 0.0;
                if (gb != 0.0) {
                    const double dN = X.nHI[cp] * X.alpha * ds;
                    double ne, gG;
                    layer_rate_adjoint_t(T, A.m64, A.tp, A.sigma0, coef, ta, A.sigma0 * dN, X.alpha * ds, r2, gb,
                                         &gi, &ne, &gG);
                    if (ne != 0.0) unsafeAtomicAdd(&nbar[cp], ne);
                    qb += gG;
                }
                gin[k] = gi;
            }
        };
        for (int m = 1; m <= Mx; ++m) {
            const LayerRect r = layer_rect(L.ext_u, L.ext_v, Rsq, m);
            const double inv_m = rcp_f64((double)m);
            const int nch = (r.total + 63) / 64;
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
                lc.Nout = 0.0;
                lc.owned = false;
                if (act) {
                    const uint32_t cp = idx_d + iu[u] + iv[v];
                    const int r2 = m2 + uv2;   // <= Rsq < sq_n when the table is there
                    const double rt = A.sq_n ? sq[r2] : sqrt_fast((double)r2);
                    layer_cell_core(L, X, m, u, v, geo[u], geo[v], rt * inv_m, r2, cp, X.nHI[cp], buf[pos],
                                    buf[pos - P], buf[pos - 1], buf[pos - P - 1], lc);
                }
                wave_sync();
                bool lit = false;
                if (act) {
                    buf[pos] = lc.h;
                    rec.h[off + g] = lc.h;
                    lit = lc.owned && A.sigma0 * lc.Nin < A.tp.tau_hi;
                }
                const uint64_t mask = __ballot(lit);
                if (lane == 0) rec.lit[choff + c] = mask;
                if (watch) opq = opq && __ballot(act && !(A.sigma0 * lc.Nout >= opaque)) == 0;
                if (mask && __popcll(mask) < dense_at) {   // (R) does not take these in place
                    if (lit) {
                        const int q = (tail + (int)__builtin_amdgcn_mbcnt_hi(
                                                  (uint32_t)(mask >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u))) &
                                      (kAdjQueue - 1);
                        qk[q] = (int)(off + g);
                        qm[q] = (m << 16) | g;
                        qT[q] = A.sigma0 * lc.Nin;
                    }
                    tail += __popcll(mask);
                    if (tail - head >= 64) {
                        wave_sync();
                        batch(64);
                        head += 64;
                    }
                }
                wave_sync();
            }
            off += r.total;
            choff += nch;
            if (watch && opq) {
                Mt = m;
                break;
            }
        }
        if (tail > head) {
            wave_sync();
            batch(tail - head);
            wave_sync();
        }
        wave_sync_global();
    }
    for (int k = lane; k < S * S; k += 64) buf[k] = 0.0;   // the adjoint slots
    wave_sync_global();

    // ---- (R)
    {
        // kept records: the cells with a rate were evaluated layer by layer
        // from the first, a layer's chunks from the last, a chunk's lanes in
        // order; lit_end counts those of layers <= m
        long lit_end = KEPT ? (long)((const uint64_t *)rec.rk)[3 * A.rec_cap] : 0;
        for (int m = Mt; m >= 1; --m) {
            const LayerRect r = layer_rect(L.ext_u, L.ext_v, Rsq, m);
            const int nch = (r.total + 63) / 64;
            off -= r.total;    // first cell of layer m in the record
            choff -= nch;      // its first chunk
            // entries of layer m - 1 (its rectangle precedes layer m's)
            const LayerRect rp = layer_rect(L.ext_u, L.ext_v, Rsq, m >= 2 ? m - 1 : 1);
            const double *Hprev = rec.h + (m >= 2 ? off - rp.total : 0);
            // this layer's geometry (the previous layer's readers are done)
            const double inv_m = rcp_f64((double)m);
            const int m2 = mul24(m, m);
            const uint32_t idx_d = layer_idx_d(L, N, m);
            for (int k = lane; k < S; k += 64) geo[k] = layer_geo(m, inv_m, k);
            wave_sync();
            auto interp = [&](int u, int v, LayerInterp &I) {
                const int r2 = m2 + mul24(u, u) + mul24(v, v);
                const double rt = A.sq_n ? sq[r2] : sqrt_fast((double)r2);
                layer_interp_core(X, m, u, v, idx_d + iu[u] + iv[v], r2, rt * inv_m, geo[u], geo[v], Hprev, rp, I);
            };
            // a batch of queued cells of layer m; every slot a cell pushes to
            // precedes it in (u, v) order, so its chunk was taken before the
            // cell was queued
            int qh = 0, qt = 0;
            auto rbatch = [&](int count) {
                if (lane < count) {
                    const int q = (qh + lane) & (kAdjQueue - 1);
                    const int g = qk[q], li = qm[q];
                    double Tin = qT[q];
                    int u, v;
                    rect_cell(r, g, u, v);
                    LayerInterp I;
                    interp(u, v, I);
                    double nbx = 0.0;
                    if (KEPT && li >= 0) {   // the rate's terms, from its coefficients
                        const double gbc = gbar[I.cp] * coef;
                        Tin += gbc * rec.rk[li];
                        nbx = gbc * rec.rk[A.rec_cap + li] * X.alpha * I.ds;
                        qb += gbc * rec.rk[2 * A.rec_cap + li];
                    }
                    LayerRev lr;
                    layer_cell_reverse(X, m, I, Tin, lr);
                    if (m >= 2) {
#pragma unroll
                        for (int n = 0; n < 4; ++n)
                            if (lr.Mbar[n] != 0.0)
                                atomicAdd(&buf[mul24(u - (n & 1), S) + (v - (n >> 1))], lr.Mbar[n]);
                    }
                    const double nb = lr.nbar + nbx;
                    if (nb != 0.0) unsafeAtomicAdd(&nbar[lr.cp], nb);
                    nb_src += lr.nbar_src;
                }
            };
            RectWalk w;
            w.init(r, lane);
            uint64_t masks = 0;
            long run = 0;   // cells with a rate in chunks 0 .. c of this layer
            for (int c = 0; c < nch; ++c, w.up()) {
                if ((c & 63) == 0) masks = load_masks(rec, choff, c, nch, lane);
                const int g = c * 64 + lane;
                const int u = w.u, v = w.v;
                const bool act = g < r.total && mul24(u, u) + mul24(v, v) <= r.rem;
                const uint64_t litmask = mask_of_chunk(masks, c);
                const bool lit = (litmask >> lane) & 1;
                run += __popcll(litmask);
                double Tin = 0.0;
                if (act) {
                    Tin = buf[mul24(u, S) + v];
                    buf[mul24(u, S) + v] = 0.0;
                }
                wave_sync();
                if (QUEUE) {
                    // the cells with work go to the queue with their entry-column
                    // adjoint (gathered form: with the rate's g_in from (F)) and,
                    // with kept records, the place of their rate's coefficients;
                    // full batches run with every lane busy
                    if (!KEPT && lit) Tin += gin[off + g];
                    const bool need = Tin != 0.0 || (KEPT && lit);
                    const uint64_t nm = __ballot(need);
                    if (need) {
                        const int q = (qt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(nm >> 32),
                                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)nm, 0u))) &
                                      (kAdjQueue - 1);
                        long li = -1;
                        if (KEPT && lit) {
                            li = lit_end - run +
                                 (long)__builtin_amdgcn_mbcnt_hi((uint32_t)(litmask >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)litmask, 0u));
                            // in range for any record contents (records of inputs changed since the
                            // forward give wrong gradients, never reads outside the record)
                            li = li < 0 ? 0 : (li >= A.rec_cap ? A.rec_cap - 1 : li);
                        }
                        qk[q] = g;
                        qm[q] = (int)li;
                        qT[q] = Tin;
                    }
                    qt += __popcll(nm);
                    if (qt - qh >= 64) {
                        wave_sync();
                        rbatch(64);
                        qh += 64;
                        wave_sync();
                    }
                } else if (__ballot(Tin != 0.0) | litmask) {
                    // the split form, where most cells have a rate: each chunk
                    // in place (queueing would only add work)
                    const bool dense = __popcll(litmask) >= dense_at;
                    if (lit && !dense) Tin += gin[off + g];
                    if (Tin != 0.0 || (lit && dense)) {
                        LayerInterp I;
                        interp(u, v, I);
                        double extra = 0.0;
                        if (lit && dense) {
                            const double gb = gbar[I.cp];
                            if (gb != 0.0) {
                                double gi, gG;
                                layer_rate_adjoint(T, A.m64, A.tp, X, coef, I, X.nHI[I.cp], gb, &gi, &extra,
                                                   &gG);
                                Tin += gi;
                                qb += gG;
                            }
                        }
                        LayerRev lr;
                        layer_cell_reverse(X, m, I, Tin, lr);
                        if (m >= 2) {
#pragma unroll
                            for (int n = 0; n < 4; ++n)
                                if (lr.Mbar[n] != 0.0)
                                    atomicAdd(&buf[mul24(u - (n & 1), S) + (v - (n >> 1))], lr.Mbar[n]);
                        }
                        const double nb = lr.nbar + extra;
                        if (nb != 0.0) unsafeAtomicAdd(&nbar[lr.cp], nb);
                        nb_src += lr.nbar_src;
                    }
                    wave_sync();
                }
            }
            if (QUEUE && qt > qh) {   // the layer's remaining cells, before layer m - 1 takes its slots
                wave_sync();
                rbatch(qt - qh);
                wave_sync();
            }
            lit_end -= run;
        }
    }
    if (p == 3 * 0 + 2 && lane == 0) {   // the source cell, once per source
        double nb, q1;
        source_cell_adjoint(T, A.m64, A.tp, A.sigma0, A.alpha, Q, n_s, A.gbar[cs], &nb, &q1);
        nb_src += nb;
        qb += q1;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        nb_src += __shfl_xor(nb_src, o, 64);
        qb += __shfl_xor(qb, o, 64);
    }
    if (lane == 0) {
        if (nb_src != 0.0) unsafeAtomicAdd(&A.nbar[cs], nb_src);
        if (qb != 0.0) unsafeAtomicAdd(&A.qbar[src], qb / Q);
    }
}

template <bool KEPT, bool SPLIT, int MAXW>
__global__ __launch_bounds__(64 * MAXW) void adj_layer(AdjArgs A)
{
    extern __shared__ __align__(16) char smem[];
    constexpr int TYPE = 3, npieces = 24;
    if (A.seg[TYPE + 1] == A.seg[TYPE]) return;   // no sources of this kind
    const TabNode *T = A.tab;
    // the work-group's table of square roots, when the launch gives one
    // (every pass takes a cell's root from it)
    double *sq = (double *)smem;
    for (int k = threadIdx.x; k < A.sq_n; k += blockDim.x) sq[k] = sqrt((double)k);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    // per wave: one buffer, the columns in (F) and the adjoints in (R), the
    // queue, the tables of (F)
    double *buf = (double *)(smem + (A.sq_n ? layer_sqrt_bytes(A.sq_n - 1) : 0) + (size_t)wave * A.region_bytes);
    int *qk = (int *)(buf + (size_t)(A.lay_S + 1) * (A.lay_S + 1));
    int *qm = qk + kAdjQueue;
    double *qT = (double *)(qm + kAdjQueue);
    Geo *geo = (Geo *)(qT + kAdjQueue);
    uint32_t *iu = (uint32_t *)(geo + A.lay_S);
    uint32_t *iv = iu + A.lay_S;
    char *scratch = (char *)(A.store + (size_t)(blockIdx.x * waves + wave) * A.store_stride);
    const int base = A.seg[TYPE];
    const int nitems = (A.seg[TYPE + 1] - base) * npieces;
    const int home = (int)(blockIdx.x % kXcds);
    int chunk = home;
    for (;;) {
        const int item = next_item(A.counter, nitems, home, chunk, lane);
        if (item >= nitems) break;
        const int src = A.order[base + item / npieces];
        adjoint_layer_piece<KEPT, SPLIT>(A, T, sq, buf, geo, iu, iv, qk, qm, qT, scratch, src, item % npieces,
                                         lane);
    }
}

// dL/dn_HI of the layer pieces with dominant axis k is accumulated in the
// [k][i][j] layout; this kernel builds that layout's n_HI and dL/dGamma and
// zeroes its accumulator (one 32 x 32 (j, k) tile of one i plane per
// work-group).
constexpr int kTile = 32;
__global__ __launch_bounds__(256) void adj_transpose_prologue_kernel(
    const float *__restrict__ nH, const float *__restrict__ xHI, const double *__restrict__ gbar,
    double *__restrict__ nHI_T, double *__restrict__ gbar_T, double *__restrict__ nbar_T, int N)
{
    __shared__ double tn[kTile][kTile + 1], tg[kTile][kTile + 1];
    const int k0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile, i = blockIdx.z;
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    for (int jj = ty; jj < kTile; jj += 8) {
        const int j = j0 + jj, k = k0 + tx;
        if (j < N && k < N) {
            const size_t c = ((size_t)i * N + j) * N + k;
            if (nHI_T) tn[jj][tx] = (double)nH[c] * (double)xHI[c];
            tg[jj][tx] = gbar[c];
        }
    }
    __syncthreads();
    for (int kk = ty; kk < kTile; kk += 8) {
        const int k = k0 + kk, j = j0 + tx;
        if (j < N && k < N) {
            const size_t t = ((size_t)k * N + i) * N + j;
            if (nHI_T) nHI_T[t] = tn[tx][kk];   // NULL: still in place from the forward
            gbar_T[t] = tg[tx][kk];
            nbar_T[t] = 0.0;
        }
    }
}

// dL/dn_H = x_HI g, dL/dx_HI = n_H g with g = dL/dn_HI from both layouts.
__global__ __launch_bounds__(256) void adj_transpose_finalize_kernel(
    const double *__restrict__ nbar, const double *__restrict__ nbar_T, const float *__restrict__ nH,
    const float *__restrict__ xHI, float *__restrict__ dnH, float *__restrict__ dxHI, int N,
    int accumulate)
{
    __shared__ double tile[kTile][kTile + 1];
    const int k0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile, i = blockIdx.z;
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    for (int kk = ty; kk < kTile; kk += 8) {
        const int k = k0 + kk, j = j0 + tx;
        if (j < N && k < N) tile[kk][tx] = nbar_T[((size_t)k * N + i) * N + j];
    }
    __syncthreads();
    for (int jj = ty; jj < kTile; jj += 8) {
        const int j = j0 + jj, k = k0 + tx;
        if (j < N && k < N) {
            const size_t c = ((size_t)i * N + j) * N + k;
            const double g = nbar[c] + tile[tx][jj];
            const float a = (float)(g * (double)xHI[c]);
            const float b = (float)(g * (double)nH[c]);
            dnH[c] = accumulate ? dnH[c] + a : a;
            dxHI[c] = accumulate ? dxHI[c] + b : b;
        }
    }
}

__global__ void adj_prologue_kernel(const float *__restrict__ nH, const float *__restrict__ xHI,
                                    double *__restrict__ nHI, double *__restrict__ nbar, long n3,
                                    double *__restrict__ qbar, long nsrc, int zero_q, int *ctl,
                                    int nctl)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n3; c += stride) {
        if (nHI) nHI[c] = (double)nH[c] * (double)xHI[c];   // NULL: still in place from the forward
        nbar[c] = 0.0;
    }
    if (zero_q)
        for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < nsrc; s += stride) qbar[s] = 0.0;
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < nctl; k += blockDim.x) ctl[k] = 0;
}

// dL/dn_H = x_HI dL/dn_HI, dL/dx_HI = n_H dL/dn_HI
__global__ void adj_finalize_kernel(const double *__restrict__ nbar, const float *__restrict__ nH,
                                    const float *__restrict__ xHI, float *__restrict__ dnH,
                                    float *__restrict__ dxHI, long n3, int accumulate)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n3; c += stride) {
        const double g = nbar[c];
        const float a = (float)(g * (double)xHI[c]);
        const float b = (float)(g * (double)nH[c]);
        dnH[c] = accumulate ? dnH[c] + a : a;
        dxHI[c] = accumulate ? dxHI[c] + b : b;
    }
}

// ---------------------------------------------------------------------------
size_t adj_region_bytes(int ring_cap, int row_cap, int shell_cap)
{
    const size_t b = 8 * (size_t)ring_cap * sizeof(double) +
                     (4 * (size_t)row_cap + 4 * ((size_t)row_cap + 1) + (size_t)shell_cap + 2) *
                         sizeof(int);
    return (b + 15) & ~(size_t)15;
}

static const void *adj_fn(int type)
{
    return type == 0 ? (const void *)adj_wave<0>
                     : (type == 1 ? (const void *)adj_wave<1> : (const void *)adj_wave<2>);
}

// The layer adjoint's instantiation: kept records (no rate terms to split),
// split rate terms or gathered ones; the wide build above kAdjLayerNarrow waves.
static const void *adj_layer_fn(bool kept, bool split, bool wide)
{
    if (wide)
        return kept ? (const void *)adj_layer<true, false, kAdjLayerWaves>
                    : (split ? (const void *)adj_layer<false, true, kAdjLayerWaves>
                             : (const void *)adj_layer<false, false, kAdjLayerWaves>);
    return kept ? (const void *)adj_layer<true, false, kAdjLayerNarrow>
                : (split ? (const void *)adj_layer<false, true, kAdjLayerNarrow>
                         : (const void *)adj_layer<false, false, kAdjLayerNarrow>);
}

hipError_t adj_configure(size_t max_lds)
{
    const int dyn = (int)max_lds - 64;
    for (int t = 0; t < 3; ++t)
        (void)hipFuncSetAttribute(adj_fn(t), hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    for (bool wide : {false, true})
        for (int v = 0; v < 3; ++v)
            (void)hipFuncSetAttribute(adj_layer_fn(v == 2, v == 1, wide), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      dyn);
    (void)hipGetLastError();
    return hipSuccess;
}

hipError_t adj_occupancy(int type, int waves, size_t lds, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, adj_fn(type), waves * 64, lds);
}

hipError_t launch_adj_prologue(hipStream_t st, const float *nH, const float *xHI, double *nHI,
                               double *nbar, long n3, double *qbar, long nsrc, int zero_q, int *ctl,
                               int nctl, int n_cu)
{
    hipLaunchKernelGGL(adj_prologue_kernel, dim3(n_cu * 8), dim3(256), 0, st, nH, xHI, nHI, nbar,
                       n3, qbar, nsrc, zero_q, ctl, nctl);
    return hipGetLastError();
}

static AdjArgs make_adj_args(const AdjLaunch &L)
{
    AdjArgs A;
    A.N = L.N;
    A.ex = make_extent(L.N);
    A.alpha = L.alpha;
    A.sigma0 = L.sigma0;
    A.coef_unit = L.sigma0 / (4.0 * M_PI * L.alpha * L.alpha);
    A.tau_w = L.tau_w;
    A.reading = L.reading;
    A.tp = L.tp;
    A.tab = L.tab;
    A.m64 = L.m64;
    A.nHI = L.nHI;
    A.gbar = L.gbar;
    A.nbar = L.nbar;
    A.qbar = L.qbar;
    A.ijk = L.ijk;
    A.Q = L.Q;
    A.R = L.R;
    A.R_cap = L.R_cap;
    A.order = L.order;
    A.seg = L.ctl + kCtlSeg;
    A.counter = L.ctl + kCtlCounter + kXcds * kCounterPad * L.type;
    A.err = L.err;
    A.ring_cap = L.ring_cap;
    A.row_cap = L.row_cap;
    A.shell_cap = L.shell_cap;
    A.region_bytes = 0;
    A.store = L.store;
    A.store_stride = L.store_stride;
    A.nHI_T = L.nHI_T;
    A.gbar_T = L.gbar_T;
    A.nbar_T = L.nbar_T;
    A.Mcap = 0;
    A.lay_S = 0;
    A.kept = L.kept;
    A.rec_piece_bytes = L.rec_piece_bytes;
    A.rec_rk_off = L.rec_rk_off;
    A.rec_cap = L.rec_cap;
    A.early_exit = L.early_exit ? 1 : 0;
    A.sq_n = 0;
    return A;
}

hipError_t launch_adj_wave(hipStream_t st, const AdjLaunch &L)
{
    AdjArgs A = make_adj_args(L);
    A.region_bytes = (int)adj_region_bytes(L.ring_cap, L.row_cap, L.shell_cap);
    const size_t lds = (size_t)L.tp.n * sizeof(TabNode) + (size_t)L.waves * A.region_bytes;
    switch (L.type) {
    case 0: hipLaunchKernelGGL(adj_wave<0>, dim3(L.grid), dim3(64 * L.waves), lds, st, A); break;
    case 1: hipLaunchKernelGGL(adj_wave<1>, dim3(L.grid), dim3(64 * L.waves), lds, st, A); break;
    default: hipLaunchKernelGGL(adj_wave<2>, dim3(L.grid), dim3(64 * L.waves), lds, st, A); break;
    }
    return hipGetLastError();
}

// Per-wave LDS of the layer adjoint: the buffer (the padded (S + 1) x (S + 1)
// layer buffer in (F), the S x S adjoint slots in (R)), the queue of cells
// with work and the table of bilinear factors of (F).
size_t adj_layer_region_bytes(int S)
{
    return ((size_t)(S + 1) * (S + 1) * sizeof(double) + kAdjQueue * (2 * sizeof(int) + sizeof(double)) +
            (size_t)S * sizeof(Geo) + 2 * (size_t)S * sizeof(uint32_t) + 15) &
           ~(size_t)15;
}

hipError_t adj_layer_occupancy(bool kept, bool split, int waves, size_t lds, int *blocks_per_cu)
{
    // kept records carry the rate's coefficients: no rate terms to split
    const void *f = adj_layer_fn(kept, !kept && split, waves > kAdjLayerNarrow);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, waves * 64, lds);
}

hipError_t launch_adj_layer(hipStream_t st, const AdjLaunch &L, int Mcap, int S)
{
    AdjArgs A = make_adj_args(L);
    A.Mcap = Mcap;
    A.lay_S = S;
    A.region_bytes = (int)adj_layer_region_bytes(S);
    const int Rsq = (int)floor((double)L.R_cap * (double)L.R_cap);
    const size_t sqb = L.sq_table ? layer_sqrt_bytes(Rsq) : 0;
    A.sq_n = sqb ? Rsq + 1 : 0;
    const size_t lds = sqb + (size_t)L.waves * A.region_bytes;
    const dim3 grid(L.grid), block(64 * L.waves);
    constexpr int W = kAdjLayerWaves, Wn = kAdjLayerNarrow;
    if (L.waves > Wn) {
        if (A.kept) hipLaunchKernelGGL((adj_layer<true, false, W>), grid, block, lds, st, A);
        else if (L.split) hipLaunchKernelGGL((adj_layer<false, true, W>), grid, block, lds, st, A);
        else hipLaunchKernelGGL((adj_layer<false, false, W>), grid, block, lds, st, A);
    } else {
        if (A.kept) hipLaunchKernelGGL((adj_layer<true, false, Wn>), grid, block, lds, st, A);
        else if (L.split) hipLaunchKernelGGL((adj_layer<false, true, Wn>), grid, block, lds, st, A);
        else hipLaunchKernelGGL((adj_layer<false, false, Wn>), grid, block, lds, st, A);
    }
    return hipGetLastError();
}

hipError_t launch_adj_transpose_prologue(hipStream_t st, const float *nH, const float *xHI,
                                         const double *gbar, double *nHI_T, double *gbar_T,
                                         double *nbar_T, int N)
{
    const dim3 grid((N + kTile - 1) / kTile, (N + kTile - 1) / kTile, N);
    hipLaunchKernelGGL(adj_transpose_prologue_kernel, grid, dim3(256), 0, st, nH, xHI, gbar, nHI_T,
                       gbar_T, nbar_T, N);
    return hipGetLastError();
}

hipError_t launch_adj_transpose_finalize(hipStream_t st, const double *nbar, const double *nbar_T,
                                         const float *nH, const float *xHI, float *dnH, float *dxHI,
                                         int N, int accumulate)
{
    const dim3 grid((N + kTile - 1) / kTile, (N + kTile - 1) / kTile, N);
    hipLaunchKernelGGL(adj_transpose_finalize_kernel, grid, dim3(256), 0, st, nbar, nbar_T, nH, xHI,
                       dnH, dxHI, N, accumulate);
    return hipGetLastError();
}

hipError_t launch_adj_finalize(hipStream_t st, const double *nbar, const float *nH, const float *xHI,
                               float *dnH, float *dxHI, long n3, int accumulate, int n_cu)
{
    hipLaunchKernelGGL(adj_finalize_kernel, dim3(n_cu * 8), dim3(256), 0, st, nbar, nH, xHI, dnH,
                       dxHI, n3, accumulate);
    return hipGetLastError();
}

}  // namespace asora
