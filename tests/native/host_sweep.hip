// host_sweep.hip -- test harness (CPU only): a serial driver around the
// library's own per-cell update, row enumeration and rate numerics
// (asora_dev.h), so that tests can compare the kernel logic with the FP64
// oracle without a GPU.  It is the kernel's sweep_piece with the parallel
// parts (wave scan, barriers, atomics) written as plain loops.
#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../paper_2311_01492_amd/csrc/asora_dev.h"
#include "../../paper_2311_01492_amd/csrc/asora_internal.h"

using namespace asora;

extern "C" float hc_neg_divdiff(int n, double lg_lo, double lg_hi, const double *P, const double *dP,
                                double a, double dt)
{
    TabParams tp;
    std::vector<TabNode> T(n);
    std::vector<double> m64(n);
    prepare_table(n, lg_lo, lg_hi, P, dP, &tp, T.data(), m64.data());
    return neg_divdiff(T.data(), tp, a, dt);
}

extern "C" void hc_neg_divdiff_batch(int n, double lg_lo, double lg_hi, const double *P,
                                     const double *dP, long m, const double *a, const double *dt,
                                     float *out)
{
    TabParams tp;
    std::vector<TabNode> T(n);
    std::vector<double> m64(n);
    prepare_table(n, lg_lo, lg_hi, P, dP, &tp, T.data(), m64.data());
    for (long i = 0; i < m; ++i) out[i] = neg_divdiff(T.data(), tp, a[i], dt[i]);
}

// The adjoint's FP64 divided difference and its partial derivatives
// (rate_derivs64) at m points (a, dt): out is D, dD/da, dD/d(dt) per point.
extern "C" void hc_rate_derivs64_batch(int n, double lg_lo, double lg_hi, const double *P, const double *dP,
                                       long m, const double *a, const double *dt, double *out)
{
    TabParams tp;
    std::vector<TabNode> T(n);
    std::vector<double> m64(n);
    prepare_table(n, lg_lo, lg_hi, P, dP, &tp, T.data(), m64.data());
    for (long i = 0; i < m; ++i) rate_derivs64(T.data(), m64.data(), tp, a[i], dt[i], out + 3 * i,
                                               out + 3 * i + 1, out + 3 * i + 2);
}

// The library's FP64 interpolant (tab_eval64: P, dP/dtau, d2P/dtau2, each
// point's own logarithm) at m points: out is [m, 3].
extern "C" void hc_tab_eval64_batch(int n, double lg_lo, double lg_hi, const double *P, const double *dP,
                                    long m, const double *tau, double *out)
{
    TabParams tp;
    std::vector<TabNode> T(n);
    std::vector<double> m64(n);
    prepare_table(n, lg_lo, lg_hi, P, dP, &tp, T.data(), m64.data());
    for (long i = 0; i < m; ++i) tab_eval64(T.data(), m64.data(), tp, tau[i], out + 3 * i, out + 3 * i + 1,
                                            out + 3 * i + 2);
}

// The chunk walk of the layer kernels against plain division: for every row
// width wv in [1, wv_max] and every cell g of rectangles up to 40 rows, the
// lanes' (u, v) after init, down() and up() equal (g / wv, g % wv).  Returns 0
// or the first failing wv.
extern "C" int hc_rectwalk_check(int wv_max)
{
    for (int wv = 1; wv <= wv_max; ++wv) {
        LayerRect r;
        r.rem = 1 << 30;
        r.nu = 40;
        r.wv = wv;
        r.total = r.nu * wv;
        const int nch = (r.total + 63) / 64;
        for (int lane = 0; lane < 64; ++lane) {
            RectWalk d, u;
            d.init(r, (nch - 1) * 64 + lane);
            u.init(r, lane);
            for (int c = 0; c < nch; ++c) {
                const int gd = (nch - 1 - c) * 64 + lane, gu = c * 64 + lane;
                if (d.u != gd / wv || d.v != gd % wv || u.u != gu / wv || u.v != gu % wv) return wv;
                d.down();
                u.up();
            }
        }
    }
    return 0;
}

// Rows of shell q of piece (type, p): writes Blo and counts of nrows rows.
extern "C" int hc_rows(int N, int type, int p, int Rsq, int q, int *blo, int *cnt)
{
    const Piece pc = make_piece(type, p);
    const Extent ex = make_extent(N);
    const int nrows = pc.n_oct * (q + 1);
    for (int r = 0; r < nrows; ++r) row_range(pc, ex, Rsq, q, r, &blo[r], &cnt[r]);
    return nrows;
}

// Full forward on the CPU with the kernels' per-cell code.  n_HI is formed in
// FP32 as on the GPU.  type_force >= 0 uses that piece type for every source.
extern "C" int hc_raytrace(int N, double alpha, double sigma0, int n, double lg_lo, double lg_hi,
                           const double *P, const double *dP, double tau_w, int reading,
                           const float *nH, const float *xHI, long nsrc, const int32_t *ijk,
                           const double *Q, const float *R, float R_whole, float R_oct,
                           int type_force, double *gacc, double *coldens)
{
    TabParams tp;
    std::vector<TabNode> T(n);
    std::vector<double> m64(n);
    prepare_table(n, lg_lo, lg_hi, P, dP, &tp, T.data(), m64.data());
    const long n3 = (long)N * N * N;
    std::vector<double> nhi(n3);
    for (long c = 0; c < n3; ++c) nhi[c] = (double)nH[c] * (double)xHI[c];
    const Extent ex = make_extent(N);
    for (long s = 0; s < nsrc; ++s) {
        const float Rs = R[s];
        const int type = type_force >= 0 ? type_force : (Rs <= R_whole ? 0 : (Rs <= R_oct ? 1 : 2));
        const int Rsq = (int)std::floor((double)Rs * (double)Rs);
        const int Qmax = max_shell(Rsq, ex);
        const int si = ijk[3 * s], sj = ijk[3 * s + 1], sk = ijk[3 * s + 2];
        const long cs = ((long)si * N + sj) * N + sk;
        for (int p = 0; p < pieces_of_type(type); ++p) {
            const Piece pc = make_piece(type, p);
            // capacities: the largest shell of this piece
            int ring_cap = 1;
            const int row_cap = pc.n_oct * (Qmax + 1);
            std::vector<int> rs(row_cap + 1), rbq(row_cap);
            for (int q = 1; q <= Qmax; ++q) {
                const int t = build_rows(pc, ex, Rsq, q, rs.data(), rbq.data());
                ring_cap = t > ring_cap ? t : ring_cap;
            }
            std::vector<double> ring(4 * (size_t)ring_cap, NAN);
            std::vector<int> rowbase(4 * (size_t)row_cap, -(1 << 30));
            std::vector<int> rowstart(row_cap + 1);
            CellCtx X;
            X.pc = pc;
            X.N = N;
            X.si = si;
            X.sj = sj;
            X.sk = sk;
            X.reading = reading;
            X.tau_w = (float)(tau_w > 0 && std::isfinite(tau_w) ? tau_w : 0.0);
            X.sigma0 = sigma0;
            X.alpha = alpha;
            X.half_col = nhi[cs] * alpha * 0.5;
            X.coef = Q[s] * sigma0 / (4.0 * M_PI * alpha * alpha);
            X.tab = T.data();
            X.m64 = m64.data();
            X.tp = tp;
            X.ring = ring.data();
            X.rowbase = rowbase.data();
            X.ring_cap = ring_cap;
            X.row_cap = row_cap;
            X.nHI = nhi.data();
            const bool src_owner = (pc.kind == 0) || (pc.oct == 0 && (pc.dom < 0 || pc.dom == 2));
            if (src_owner) {
                gacc[cs] += source_cell_rate(T.data(), tp, sigma0, alpha, Q[s], nhi[cs]);
                if (coldens) coldens[cs] = 0.0;
            }
            for (int q = 1; q <= Qmax; ++q) {
                const int slot = q & 3;
                const int nrows = pc.n_oct * (q + 1);
                const int total = build_rows(pc, ex, Rsq, q, rowstart.data(),
                                             rowbase.data() + slot * row_cap);
                for (int g = 0; g < total; ++g) {
                    const int row = find_row(rowstart.data(), nrows, g);
                    CellOut co;
                    cell_update(X, q, g, row, rowbase[slot * row_cap + row], co);
                    if (!std::isfinite(co.Nout)) return -5;   // read an unwritten slot
                    ring[slot * (size_t)ring_cap + g] = co.Nout;
                    if (co.owned) {
                        gacc[co.cp] += co.G;
                        if (coldens) coldens[co.cp] = co.Nin;
                    }
                }
                // poison the slot that shell q+1 will overwrite (shell q-3), so
                // that a read of a stale shell shows up as NaN
                if (q + 1 <= Qmax)
                    for (int g = 0; g < ring_cap; ++g) ring[((q + 1) & 3) * (size_t)ring_cap + g] = NAN;
            }
        }
    }
    return 0;
}

// Forward on the CPU through the layer pieces (every source as 24 pyramids
// swept layer by layer), in the kernel's tile order with its in-place layer
// buffer: per tile all 64 lanes read before any writes.  Pyramids with
// dominant axis k read n_HI from the [k][i][j] copy and accumulate into a
// [k][i][j] accumulator, added at the end as on the GPU.  Every read of a
// neighbour of non-zero weight is checked to hold layer m - 1 (returns -6
// otherwise).  tv is the tile width along v (8 or 16).
// One pyramid swept forward in the layer kernels' order: layers m = 1..Mx,
// each layer's rectangle in chunks of 64 cells from the last chunk to the
// first, every chunk reading layer m - 1 from the in-place buffer before it
// writes layer m.  Adds the rates to acc (when acc != NULL) and, when rec is
// given, fills the column record as the kernels do (exit columns in rectangle
// order, listed cells in chunk and lane order; with rec->rk the rate
// coefficients of the cells with a rate in this order of evaluation, and
// their number after the three arrays of cap entries).  With `early` the
// record stops after the first layer whose cells all leave opaque
// (layer_opaque), as in the kernels with the early exit; *m_last (may be
// NULL) receives that layer (Mx without `early` or if there is none).  Every
// layer is swept either way.  Returns -6 if a neighbour of non-zero weight is
// read from a slot that does not hold layer m - 1, -8 if a cell falls outside
// the S x S layer buffer, -10 if a cell after an opaque layer has a rate.
static int layer_forward_piece(const LayerPiece &L, const LayerX &X, int Rsq, const TabNode *T,
                               const double *m64, const TabParams &tp, double coef, int S, double *lay,
                               int *lay_id, double *acc, double *coldens, int N, LayerRecord *rec, long cap,
                               int *m_last = nullptr, bool early = false, double *ta_out = nullptr)
{
    long nlit = 0;
    bool rec_on = rec != nullptr;
    bool past_opaque = false;
    const double opaque = layer_opaque(tp.tau_hi);
    const int Mx = std::min(isqrt_floor(Rsq), L.ext_d);
    if (m_last) *m_last = Mx;
    long off = 0, choff = 0;
    for (int m = 1; m <= Mx; ++m) {
        const LayerRect r = layer_rect(L.ext_u, L.ext_v, Rsq, m);
        const int nch = (r.total + 63) / 64;
        RectWalk wk[64];
        for (int lane = 0; lane < 64; ++lane) wk[lane].init(r, (nch - 1) * 64 + lane);
        bool opq = true;
        for (int c = nch - 1; c >= 0; --c) {
            LayerCell lc[64];
            bool act[64];
            int uu[64], vv[64];
            for (int lane = 0; lane < 64; ++lane) {
                uu[lane] = wk[lane].u;
                vv[lane] = wk[lane].v;
                wk[lane].down();
                act[lane] = c * 64 + lane < r.total && uu[lane] * uu[lane] + vv[lane] * vv[lane] <= r.rem;
                if (!act[lane]) continue;
                const int u = uu[lane], v = vv[lane];
                if (u >= S || v >= S) return -8;   // outside the S x S layer buffer
                if (m > 1) {   // neighbours of non-zero weight must hold layer m - 1
                    const bool a0 = u > 0, a1 = u < m, b0 = v > 0, b1 = v < m;
                    const bool need[4] = {a1 && b1, a0 && b1, a1 && b0, a0 && b0};
                    for (int k = 0; k < 4; ++k)
                        if (need[k] && lay_id[layer_slot(u - (k & 1), v - (k >> 1), S + 1)] != m - 1) return -6;
                }
                layer_cell(L, X, m, u, v, lay, S + 1, lc[lane]);
            }
            uint64_t mask = 0;
            for (int lane = 0; lane < 64; ++lane) {
                if (!act[lane]) continue;
                const int u = uu[lane], v = vv[lane];
                lay[layer_slot(u, v, S + 1)] = lc[lane].h;
                lay_id[layer_slot(u, v, S + 1)] = m;
                if (!(X.sigma0 * lc[lane].Nout >= opaque)) opq = false;
                if (rec_on) rec->h[off + c * 64 + lane] = lc[lane].h;
                if (!lc[lane].owned) continue;
                if (coldens) coldens[layer_std_index(L, N, m, u, v)] = lc[lane].Nin;
                const double ta = X.sigma0 * lc[lane].Nin;
                if (ta >= tp.tau_hi) continue;
                mask |= 1ull << lane;
                if (ta_out && rec_on) ta_out[off + c * 64 + lane] = ta;
                const double dt = X.sigma0 * lc[lane].dN;
                if (acc) {
                    const float nd = neg_divdiff(T, tp, ta, dt);
                    if (nd > 0.f) acc[lc[lane].cp] += coef * (double)(nd * rcp_approx((float)lc[lane].r2));
                }
                if (rec && rec->rk) {
                    double k[3];
                    layer_rate_coefs(T, m64, tp, X.sigma0, ta, dt, lc[lane].r2, k);
                    for (int i = 0; i < 3; ++i) rec->rk[i * cap + nlit] = k[i];
                }
                ++nlit;
            }
            if (rec_on) rec->lit[choff + c] = mask;
            if (past_opaque && mask) return -10;   // a rate after an opaque layer
        }
        off += r.total;
        choff += nch;
        if (opq && !past_opaque) {
            past_opaque = true;
            if (m_last && early) *m_last = m;
        }
        if (rec_on && opq && early) {
            rec_on = false;
            if (rec->rk) ((uint64_t *)rec->rk)[3 * cap + 1] = (uint64_t)m;
        }
    }
    if (rec && rec->rk) {
        ((uint64_t *)rec->rk)[3 * cap] = (uint64_t)nlit;
        if (rec_on) ((uint64_t *)rec->rk)[3 * cap + 1] = (uint64_t)Mx;
    }
    return 0;
}

struct HostLayerSetup {
    TabParams tp;
    std::vector<TabNode> T;
    std::vector<double> m64, nhi, nhiT;
    Extent ex;
    int Mcap, S;
    long cap;
};

static void host_layer_setup(HostLayerSetup &H, int N, int n, double lg_lo, double lg_hi, const double *P,
                             const double *dP, const float *nH, const float *xHI, long nsrc, const float *R)
{
    H.T.resize(n);
    H.m64.resize(n);
    prepare_table(n, lg_lo, lg_hi, P, dP, &H.tp, H.T.data(), H.m64.data());
    const long n3 = (long)N * N * N;
    H.nhi.resize(n3);
    H.nhiT.resize(n3);
    for (long i = 0; i < N; ++i)
        for (long j = 0; j < N; ++j)
            for (long k = 0; k < N; ++k) {
                const long c = (i * N + j) * N + k;
                H.nhi[c] = (double)nH[c] * (double)xHI[c];
                H.nhiT[(k * N + i) * N + j] = H.nhi[c];
            }
    H.ex = make_extent(N);
    float R_cap = 0.f;
    for (long s = 0; s < nsrc; ++s) R_cap = R[s] > R_cap ? R[s] : R_cap;
    const int Rsq_cap = (int)std::floor((double)R_cap * (double)R_cap);
    H.Mcap = std::max(1, std::min(isqrt_floor(Rsq_cap), H.ex.neg));
    H.S = layer_buffer_side(Rsq_cap, H.ex);
    H.cap = std::max(1L, layer_piece_capacity(Rsq_cap, H.ex));
}

static LayerX host_layer_x(const HostLayerSetup &H, const LayerPiece &L, int N, double alpha, double sigma0,
                           double tau_w, int reading, long cs)
{
    LayerX X;
    X.N = N;
    X.reading = reading;
    X.tau_w = (float)(tau_w > 0 && std::isfinite(tau_w) ? tau_w : 0.0);
    X.sigma0 = sigma0;
    X.alpha = alpha;
    X.half_col = H.nhi[cs] * alpha * 0.5;
    X.nHI = L.transposed ? H.nhiT.data() : H.nhi.data();
    layer_x_weights(X);
    return X;
}

extern "C" int hc_raytrace_layer(int N, double alpha, double sigma0, int n, double lg_lo, double lg_hi,
                                 const double *P, const double *dP, double tau_w, int reading,
                                 const float *nH, const float *xHI, long nsrc, const int32_t *ijk,
                                 const double *Q, const float *R, double *gacc, double *coldens)
{
    HostLayerSetup H;
    host_layer_setup(H, N, n, lg_lo, lg_hi, P, dP, nH, xHI, nsrc, R);
    const long n3 = (long)N * N * N;
    std::vector<double> gT(n3, 0.0);
    std::vector<double> lay((size_t)(H.S + 1) * (H.S + 1));   // padded, as in the kernels
    std::vector<int> lay_id((size_t)(H.S + 1) * (H.S + 1));
    const double coef_unit = sigma0 / (4.0 * M_PI * alpha * alpha);
    for (long s = 0; s < nsrc; ++s) {
        const int si = ijk[3 * s], sj = ijk[3 * s + 1], sk = ijk[3 * s + 2];
        const int Rsq = (int)std::floor((double)R[s] * (double)R[s]);
        const long cs = ((long)si * N + sj) * N + sk;
        gacc[cs] += source_cell_rate(H.T.data(), H.tp, sigma0, alpha, Q[s], H.nhi[cs]);
        if (coldens) coldens[cs] = 0.0;
        for (int p = 0; p < 24; ++p) {
            const LayerPiece L = make_layer_piece(p, si, sj, sk, N, H.ex);
            const LayerX X = host_layer_x(H, L, N, alpha, sigma0, tau_w, reading, cs);
            std::fill(lay.begin(), lay.end(), 0.0);
            std::fill(lay_id.begin(), lay_id.end(), -1);
            const int st = layer_forward_piece(L, X, Rsq, H.T.data(), H.m64.data(), H.tp, Q[s] * coef_unit,
                                               H.S, lay.data(), lay_id.data(), L.transposed ? gT.data() : gacc,
                                               coldens, N, nullptr, H.cap);
            if (st) return st;
        }
    }
    for (long i = 0; i < N; ++i)
        for (long j = 0; j < N; ++j)
            for (long k = 0; k < N; ++k) gacc[(i * N + j) * N + k] += gT[(k * N + i) * N + j];
    return 0;
}

// Reverse mode on the CPU through the layer pieces, in the adjoint kernel's
// order, per pyramid: (F) the forward pass fills the column record (the
// cells' layer-buffer entries, each chunk's mask of cells with a rate, and
// the rate terms of the cells with a rate from their entry optical depths);
// (R) layers from the outermost
// inward, each layer's rectangle in chunks from the first to the last, each
// chunk reading its slots and clearing them, adding the rate's entry-column
// terms of its cells with a rate, and pushing to its layer m - 1 neighbours,
// whose entries it reads from the record.  dL/dn_HI of pyramids
// with dominant axis k goes through a [k][i][j] buffer as on the GPU.
// mode 1: chunks with at least kDenseChunk cells with a rate evaluate them in
// (R), as the kernel's split form; 0: all are taken in (F); 2: the forward
// pass keeps the rate coefficients in the record, as a forward with kept
// records does, and (R) reads them (no rate terms in (F)).  mode | 4: the early exit (every
// pass stops at the pyramid's first opaque layer); otherwise all layers.
// Returns -6 if a neighbour of non-zero weight is not an active cell of layer
// m - 1, -7 if a chunk mask marks an inactive lane, -9 if (mode 2) the count
// of cells with a rate disagrees with the chunk masks.
extern "C" int hc_raytrace_layer_grad(int N, double alpha, double sigma0, int n, double lg_lo,
                                      double lg_hi, const double *P, const double *dP, double tau_w,
                                      int reading, const float *nH, const float *xHI, long nsrc,
                                      const int32_t *ijk, const double *Q, const float *R,
                                      const double *gbar, double *nbar, double *qbar, int mode,
                                      long *stats)
{
    // stats (may be NULL): pieces whose adjoint stops before their last
    // layer, cells in the layers the adjoint visits, cells of all layers
    if (stats) stats[0] = stats[1] = stats[2] = 0;
    const bool early = (mode & 4) != 0;
    mode &= 3;
    const int dense_at = mode == 1 ? kDenseChunk : 65;
    const bool kept = mode == 2;
    HostLayerSetup H;
    host_layer_setup(H, N, n, lg_lo, lg_hi, P, dP, nH, xHI, nsrc, R);
    const long n3 = (long)N * N * N;
    std::vector<double> gbT(n3), nbT(n3, 0.0);
    for (long i = 0; i < N; ++i)
        for (long j = 0; j < N; ++j)
            for (long k = 0; k < N; ++k) gbT[(k * N + i) * N + j] = gbar[(i * N + j) * N + k];
    const int S = H.S;
    const size_t SS = (size_t)S * S, PP = (size_t)(S + 1) * (S + 1);
    std::vector<double> cols(PP), abar(SS), gin(H.cap), ta(H.cap);
    std::vector<int> cols_id(PP);
    std::vector<char> recmem(layer_record_bytes(H.cap, H.Mcap, kept));
    LayerRecord rec = layer_record_at(recmem.data(), H.cap, kept ? layer_record_bytes(H.cap, H.Mcap, false) : 0);
    const double coef_unit = sigma0 / (4.0 * M_PI * alpha * alpha);
    for (long s = 0; s < nsrc; ++s) {
        qbar[s] = 0.0;
        const int si = ijk[3 * s], sj = ijk[3 * s + 1], sk = ijk[3 * s + 2];
        const int Rsq = (int)std::floor((double)R[s] * (double)R[s]);
        const long cs = ((long)si * N + sj) * N + sk;
        const double coef = Q[s] * coef_unit;
        double nb_src = 0.0, qb = 0.0;
        for (int p = 0; p < 24; ++p) {
            const LayerPiece L = make_layer_piece(p, si, sj, sk, N, H.ex);
            const LayerX X = host_layer_x(H, L, N, alpha, sigma0, tau_w, reading, cs);
            const double *gb = L.transposed ? gbT.data() : gbar;
            double *nb = L.transposed ? nbT.data() : nbar;
            const int Mx = std::min(isqrt_floor(Rsq), L.ext_d);
            // (F)
            std::fill(cols.begin(), cols.end(), 0.0);
            std::fill(cols_id.begin(), cols_id.end(), -1);
            // unwritten parts of the record read as NaN entries and all-set masks
            std::memset(recmem.data(), 0xff, recmem.size());
            int Mt = Mx;   // the last layer (R) visits
            int st = layer_forward_piece(L, X, Rsq, H.T.data(), H.m64.data(), H.tp, coef, S, cols.data(),
                                         cols_id.data(), nullptr, nullptr, N, &rec, H.cap, &Mt, early,
                                         kept ? nullptr : ta.data());
            if (st) return st;
            if (stats) {
                stats[0] += Mt < Mx;
                for (int m = 1; m <= Mx; ++m) {
                    const long t = layer_rect(L.ext_u, L.ext_v, Rsq, m).total;
                    stats[1] += m <= Mt ? t : 0;
                    stats[2] += t;
                }
            }
            // the rate terms (F) evaluates from its queue: cells with a rate that
            // (R) does not take in place, from their entry optical depth and
            // place (m, g), the rest recomputed as (F) formed it
            long off = 0, choff = 0;
            for (int m = 1; m <= Mt; ++m) {
                const LayerRect r = layer_rect(L.ext_u, L.ext_v, Rsq, m);
                const int nch = (r.total + 63) / 64;
                for (int c = 0; c < nch; ++c) {
                    const uint64_t litmask = rec.lit[choff + c];
                    if (kept || __builtin_popcountll(litmask) >= dense_at) continue;   // left to (R)
                    for (int lane = 0; lane < 64; ++lane) {
                        if (!((litmask >> lane) & 1)) continue;
                        const int g = c * 64 + lane;
                        int u, v;
                        rect_cell(r, g, u, v);
                        if (g >= r.total || u * u + v * v > r.rem) return -7;
                        const uint32_t cp = layer_cp(L, N, m, u, v);
                        const int r2 = m * m + u * u + v * v;
                        const double ds = sqrt_fast((double)r2) * rcp_f64((double)m);
                        double gi = 0.0;
                        const double g_ = gb[cp];
                        if (g_ != 0.0) {
                            const double dN = X.nHI[cp] * X.alpha * ds;
                            double ne, gG;
                            layer_rate_adjoint_t(H.T.data(), H.m64.data(), H.tp, sigma0, coef, ta[off + g],
                                                 sigma0 * dN, X.alpha * ds, r2, g_, &gi, &ne, &gG);
                            nb[cp] += ne;
                            qb += gG;
                        }
                        gin[off + g] = gi;
                    }
                }
                off += r.total;
                choff += nch;
            }
            // (R)
            std::fill(abar.begin(), abar.end(), 0.0);
            long lit_end = kept ? (long)((const uint64_t *)rec.rk)[3 * H.cap] : 0;   // with a rate, layers <= m
            for (int m = Mt; m >= 1; --m) {
                long run = 0;
                const LayerRect r = layer_rect(L.ext_u, L.ext_v, Rsq, m);
                const int nch = (r.total + 63) / 64;
                off -= r.total;   // first cell of layer m
                choff -= nch;
                const LayerRect rp = layer_rect(L.ext_u, L.ext_v, Rsq, m >= 2 ? m - 1 : 1);
                const double *Hprev = rec.h + (m >= 2 ? off - rp.total : 0);
                RectWalk wk[64];
                for (int lane = 0; lane < 64; ++lane) wk[lane].init(r, lane);
                for (int c = 0; c < nch; ++c) {
                    LayerRev lr[64];
                    bool act[64];
                    int uu[64], vv[64];
                    double Tin[64];
                    const uint64_t litmask = rec.lit[choff + c];
                    run += __builtin_popcountll(litmask);
                    for (int lane = 0; lane < 64; ++lane) {
                        uu[lane] = wk[lane].u;
                        vv[lane] = wk[lane].v;
                        wk[lane].up();
                        act[lane] = c * 64 + lane < r.total && uu[lane] * uu[lane] + vv[lane] * vv[lane] <= r.rem;
                        Tin[lane] = act[lane] ? abar[(size_t)uu[lane] * S + vv[lane]] : 0.0;
                    }
                    for (int lane = 0; lane < 64; ++lane)
                        if (act[lane]) abar[(size_t)uu[lane] * S + vv[lane]] = 0.0;
                    const bool dense = !kept && __builtin_popcountll(litmask) >= dense_at;
                    for (int lane = 0; lane < 64; ++lane) {
                        const bool lit = (litmask >> lane) & 1;
                        if (lit && !dense && !kept) Tin[lane] += gin[off + c * 64 + lane];
                        if (!act[lane] || (Tin[lane] == 0.0 && !(lit && (dense || kept)))) continue;
                        const int u = uu[lane], v = vv[lane];
                        if (m > 1) {   // neighbours of non-zero weight: active cells of layer m - 1
                            const bool a0 = u > 0, a1 = u < m, b0 = v > 0, b1 = v < m;
                            const bool need[4] = {a1 && b1, a0 && b1, a1 && b0, a0 && b0};
                            for (int k = 0; k < 4; ++k) {
                                if (!need[k]) continue;
                                const int un = u - (k & 1), vn = v - (k >> 1);
                                if (un >= rp.nu || vn >= rp.wv || un * un + vn * vn > rp.rem) return -6;
                            }
                        }
                        LayerInterp I;
                        layer_interp(L, X, m, u, v, Hprev, rp, I);
                        double extra = 0.0;
                        if (lit && kept) {   // the coefficients at the cell's place in the forward's order
                            const long q = lit_end - run + __builtin_popcountll(litmask & ((1ull << lane) - 1));
                            const double gbc = gb[I.cp] * coef;
                            Tin[lane] += gbc * rec.rk[q];
                            extra = gbc * rec.rk[H.cap + q] * X.alpha * I.ds;
                            qb += gbc * rec.rk[2 * H.cap + q];
                        }
                        if (lit && dense && gb[I.cp] != 0.0) {
                            double gi, gG;
                            layer_rate_adjoint(H.T.data(), H.m64.data(), H.tp, X, coef, I, X.nHI[I.cp], gb[I.cp],
                                               &gi, &extra, &gG);
                            Tin[lane] += gi;
                            qb += gG;
                        }
                        layer_cell_reverse(X, m, I, Tin[lane], lr[lane]);
                        for (int k = 0; k < 4; ++k)
                            if (lr[lane].Mbar[k] != 0.0)
                                abar[(size_t)(u - (k & 1)) * S + (v - (k >> 1))] += lr[lane].Mbar[k];
                        nb[lr[lane].cp] += lr[lane].nbar + extra;
                        nb_src += lr[lane].nbar_src;
                    }
                }
                lit_end -= run;
            }
            if (kept && lit_end != 0) return -9;   // the count of cells with a rate does not add up
        }
        double nb1, q1;
        source_cell_adjoint(H.T.data(), H.m64.data(), H.tp, sigma0, alpha, Q[s], H.nhi[cs], gbar[cs], &nb1, &q1);
        nbar[cs] += nb_src + nb1;
        qbar[s] += (qb + q1) / Q[s];
    }
    for (long i = 0; i < N; ++i)
        for (long j = 0; j < N; ++j)
            for (long k = 0; k < N; ++k) nbar[(i * N + j) * N + k] += nbT[(k * N + i) * N + j];
    return 0;
}

// Reverse mode on the CPU with the kernels' per-cell adjoint: forward column
// pass per piece storing every shell, then shells outermost first.  Outputs
// dL/dn_HI (FP64, accumulated) and dL/dQ.
extern "C" int hc_raytrace_grad(int N, double alpha, double sigma0, int n, double lg_lo, double lg_hi,
                                const double *P, const double *dP, double tau_w, int reading,
                                const float *nH, const float *xHI, long nsrc, const int32_t *ijk,
                                const double *Q, const float *R, float R_whole, float R_oct,
                                int type_force, const double *gbar, double *nbar, double *qbar)
{
    TabParams tp;
    std::vector<TabNode> T(n);
    std::vector<double> m64(n);
    prepare_table(n, lg_lo, lg_hi, P, dP, &tp, T.data(), m64.data());
    const long n3 = (long)N * N * N;
    std::vector<double> nhi(n3);
    for (long c = 0; c < n3; ++c) nhi[c] = (double)nH[c] * (double)xHI[c];
    const Extent ex = make_extent(N);
    for (long s = 0; s < nsrc; ++s) {
        qbar[s] = 0.0;
        const float Rs = R[s];
        const int type = type_force >= 0 ? type_force : (Rs <= R_whole ? 0 : (Rs <= R_oct ? 1 : 2));
        const int Rsq = (int)std::floor((double)Rs * (double)Rs);
        const int Qmax = max_shell(Rsq, ex);
        const int si = ijk[3 * s], sj = ijk[3 * s + 1], sk = ijk[3 * s + 2];
        const long cs = ((long)si * N + sj) * N + sk;
        for (int p = 0; p < pieces_of_type(type); ++p) {
            const Piece pc = make_piece(type, p);
            const int row_cap = pc.n_oct * (Qmax + 1);
            std::vector<std::vector<int>> rs_sh(Qmax + 1), rb_sh(Qmax + 1);
            std::vector<std::vector<double>> nout_sh(Qmax + 1), nbar_sh(Qmax + 1), dn_sh(Qmax + 1);
            int ring_cap = 1;
            for (int q = 1; q <= Qmax; ++q) {
                rs_sh[q].resize(row_cap + 1);
                rb_sh[q].resize(row_cap);
                const int t = build_rows(pc, ex, Rsq, q, rs_sh[q].data(), rb_sh[q].data());
                nout_sh[q].assign(t, 0.0);
                nbar_sh[q].assign(t, 0.0);
                dn_sh[q].assign(t, 0.0);
                ring_cap = t > ring_cap ? t : ring_cap;
            }
            std::vector<double> ring(4 * (size_t)ring_cap, NAN);
            std::vector<int> rowbase(4 * (size_t)row_cap, -(1 << 30));
            CellCtx X;
            X.pc = pc;
            X.N = N;
            X.si = si;
            X.sj = sj;
            X.sk = sk;
            X.reading = reading;
            X.tau_w = (float)(tau_w > 0 && std::isfinite(tau_w) ? tau_w : 0.0);
            X.sigma0 = sigma0;
            X.alpha = alpha;
            X.half_col = nhi[cs] * alpha * 0.5;
            X.coef = Q[s] * sigma0 / (4.0 * M_PI * alpha * alpha);
            X.tab = T.data();
            X.m64 = m64.data();
            X.tp = tp;
            X.ring = ring.data();
            X.rowbase = rowbase.data();
            X.ring_cap = ring_cap;
            X.row_cap = row_cap;
            X.nHI = nhi.data();
            auto load = [&](int qq) {   // shell qq into its ring slot
                if (qq < 1) return;
                const int sl = qq & 3;
                for (int r = 0; r < row_cap; ++r) rowbase[sl * row_cap + r] = rb_sh[qq][r];
                for (size_t g = 0; g < nout_sh[qq].size(); ++g) ring[sl * (size_t)ring_cap + g] = nout_sh[qq][g];
            };
            // forward columns
            for (int q = 1; q <= Qmax; ++q) {
                load(q - 1);
                load(q - 2);
                load(q - 3);
                load(q);
                const int nrows = pc.n_oct * (q + 1);
                for (size_t g = 0; g < nout_sh[q].size(); ++g) {
                    const int row = find_row(rs_sh[q].data(), nrows, (int)g);
                    CellOut co;
                    cell_update<false>(X, q, (int)g, row, rb_sh[q][row], co);
                    nout_sh[q][g] = co.Nout;
                    dn_sh[q][g] = co.dN;
                }
            }
            // reverse
            for (int q = Qmax; q >= 1; --q) {
                load(q - 1);
                load(q - 2);
                load(q - 3);
                load(q);
                const int nrows = pc.n_oct * (q + 1);
                for (size_t g = 0; g < nout_sh[q].size(); ++g) {
                    const int row = find_row(rs_sh[q].data(), nrows, (int)g);
                    CellAdj ca;
                    cell_adjoint(X, q, (int)g, row, rb_sh[q][row], nbar_sh[q][g], dn_sh[q][g], gbar, ca);
                    nbar[ca.cp] += ca.nbar;
                    nbar[cs] += ca.nbar_src;
                    qbar[s] += ca.qbar / Q[s];
                    for (int k = 0; k < 4; ++k)
                        if (ca.slot[k] >= 0) nbar_sh[ca.qn[k]][ca.slot[k]] += ca.Mbar[k];
                }
            }
            const bool src_owner = (pc.kind == 0) || (pc.oct == 0 && (pc.dom < 0 || pc.dom == 2));
            if (src_owner) {
                double nb, qb;
                source_cell_adjoint(T.data(), m64.data(), tp, sigma0, alpha, Q[s], nhi[cs], gbar[cs], &nb, &qb);
                nbar[cs] += nb;
                qbar[s] += qb / Q[s];
            }
        }
    }
    return 0;
}

// The kernels' FP64 logarithms (unit access for their accuracy pins).
extern "C" double hc_log_fast(double a) { return log_fast(a); }
extern "C" double hc_log_f64(double a) { return log_f64(a); }
