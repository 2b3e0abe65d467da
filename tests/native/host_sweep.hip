// host_sweep.hip -- test harness (CPU only): a serial driver around the
// library's own per-cell update, row enumeration and rate numerics
// (asora_dev.h), so that tests can compare the kernel logic with the FP64
// oracle without a GPU.  It is the kernel's sweep_piece with the parallel
// parts (wave scan, barriers, atomics) written as plain loops.
#include <cmath>
#include <cstdint>
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
            std::vector<std::vector<double>> nout_sh(Qmax + 1), nbar_sh(Qmax + 1);
            int ring_cap = 1;
            for (int q = 1; q <= Qmax; ++q) {
                rs_sh[q].resize(row_cap + 1);
                rb_sh[q].resize(row_cap);
                const int t = build_rows(pc, ex, Rsq, q, rs_sh[q].data(), rb_sh[q].data());
                nout_sh[q].assign(t, 0.0);
                nbar_sh[q].assign(t, 0.0);
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
                    cell_adjoint(X, q, (int)g, row, rb_sh[q][row], nbar_sh[q][g], gbar, ca);
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
