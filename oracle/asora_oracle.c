/*
 * asora_oracle.c -- plain, sequential FP64 CPU oracle of the ASORA
 * ray-tracing step (photoionization rate from short characteristics swept in
 * octahedral shells).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file.  It shares no code,
 * header, table or constant with the HIP library: everything below is written
 * from the paper's equations.
 *
 * What is computed, per source s and per cell p inside the ray-tracing ball:
 *   - the column density N_in up to the entry face of p, interpolated from the
 *     exit columns of four neighbours closer to the source (short
 *     characteristics, Section 3.1, eq. raga / eq. interp), weighted
 *     geometrically and by optical depth;
 *   - the in-cell column dN = n_HI alpha ds with ds = r/m (Section 3.1);
 *   - the photon-conserving rate Gamma = [gamma(N_in) - gamma(N_in + dN)] /
 *     (n_HI V_shell), V_shell = 4 pi r^2 ds in physical units
 *     (eq. gamma / eq. tables / eq. sugg), with gamma/Q read from the table;
 *   - the sum of Gamma over sources (Section 2.2, multi-source paragraph).
 * Cells are visited shell by shell in L1 distance q = |di|+|dj|+|dk|
 * (Section 3.3, fig. octa) and, inside a shell, in lexicographic order of
 * (di, dj, dk).  Cells whose distance to the source exceeds R are skipped
 * (Section 3.3, last paragraph), as are cells outside the periodic extent
 * (Appendix A: at most N/2 on the negative and N/2-1 on the positive side on
 * an even mesh, (N-1)/2 on both sides on an odd mesh).
 *
 * Readings of points the paper leaves open (each one is listed with its
 * reason in the design notes of the repository):
 *   - the four neighbours lie in the layer one step closer to the source along
 *     the dominant axis d (the axis with |d| = max): e1 = p - sd*ed,
 *     e2 = e1 - su*eu, e3 = e1 - sv*ev, e4 = e1 - su*eu - sv*ev, with sign(0)=0;
 *   - geometric weights are bilinear in a = |du|/m, b = |dv|/m:
 *     (1-a)(1-b), a(1-b), (1-a)b, ab; neighbours of zero weight are skipped;
 *   - optical-depth weights w = s / max(sigma0*M, tau_w); tau_w = +inf gives
 *     pure geometric weighting;
 *   - the source cell has N_in = 0, path half a cell and volume alpha^3; a
 *     neighbour that interpolates from the source sees the source column
 *     n_HI(s) alpha ds_p / 2 (reading A) or n_HI(s) alpha / 2 (reading B);
 *   - the table interpolant is a cubic Hermite spline of ln P in ln tau with
 *     node slopes tau P'/P; linear below the first node; constant above the
 *     last node;
 *   - inclusion in the ball is r^2 <= R^2 with R in cells; the largest shell
 *     is ceil(sqrt(3) R).
 * Floating point: FP64 throughout; build with -O2 -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ECAUSAL -5
#define ORC_EZERO -6

/* ------------------------------------------------------------------ */
/* Photoionization table: P(tau) = gamma(tau/sigma0) / gamma(0)         */
/* (eq. tables, normalised), tabulated on n nodes uniform in log10 tau. */
/* ------------------------------------------------------------------ */
typedef struct {
    int n;
    double lg_lo, lg_hi;     /* log10 of the first and last node */
    const double *P;         /* P at the nodes */
    const double *dP;        /* dP/dtau at the nodes */
} otab;

/* Evaluate the interpolant P^(tau), its first and second derivative. */
static double tab_eval(const otab *t, double tau, double *d1, double *d2)
{
    const double ln10 = 2.302585092994045684;
    double x_lo = t->lg_lo * ln10;
    double h = (t->lg_hi - t->lg_lo) * ln10 / (double)(t->n - 1);
    double tau_lo = exp(x_lo);
    double tau_hi = exp(x_lo + h * (double)(t->n - 1));
    if (tau < tau_lo) {                       /* linear continuation */
        if (d1) *d1 = t->dP[0];
        if (d2) *d2 = 0.0;
        return t->P[0] + t->dP[0] * (tau - tau_lo);
    }
    if (tau >= tau_hi) {                      /* no absorption beyond the table */
        if (d1) *d1 = 0.0;
        if (d2) *d2 = 0.0;
        return t->P[t->n - 1];
    }
    double x = log(tau);
    int k = (int)floor((x - x_lo) / h);
    if (k < 0) k = 0;
    if (k > t->n - 2) k = t->n - 2;
    double xk = x_lo + h * (double)k;
    double s = (x - xk) / h;
    double tk = exp(xk), tk1 = exp(xk + h);
    double y0 = log(t->P[k]), y1 = log(t->P[k + 1]);
    double m0 = tk * t->dP[k] / t->P[k];          /* d lnP / d ln tau at node k   */
    double m1 = tk1 * t->dP[k + 1] / t->P[k + 1]; /* and at node k+1             */
    /* cubic Hermite basis on [0,1] */
    double h00 = 2 * s * s * s - 3 * s * s + 1;
    double h10 = s * s * s - 2 * s * s + s;
    double h01 = -2 * s * s * s + 3 * s * s;
    double h11 = s * s * s - s * s;
    double y = h00 * y0 + h10 * h * m0 + h01 * y1 + h11 * h * m1;
    double P = exp(y);
    if (d1 || d2) {
        double g00 = 6 * s * s - 6 * s, g10 = 3 * s * s - 4 * s + 1;
        double g01 = -6 * s * s + 6 * s, g11 = 3 * s * s - 2 * s;
        double yx = (g00 * y0 + g10 * h * m0 + g01 * y1 + g11 * h * m1) / h;   /* dy/dx */
        double f00 = 12 * s - 6, f10 = 6 * s - 4, f01 = -12 * s + 6, f11 = 6 * s - 2;
        double yxx = (f00 * y0 + f10 * h * m0 + f01 * y1 + f11 * h * m1) / (h * h);
        /* P = exp(y(x)), x = ln tau */
        double dPdtau = P * yx / tau;
        if (d1) *d1 = dPdtau;
        if (d2) *d2 = P * (yx * yx + yxx - yx) / (tau * tau);
    }
    return P;
}

double oracle_table_eval(int n, double lg_lo, double lg_hi, const double *P, const double *dP,
                         double tau, double *d1, double *d2)
{
    otab t = {n, lg_lo, lg_hi, P, dP};
    return tab_eval(&t, tau, d1, d2);
}

/* ------------------------------------------------------------------ */
/* Short-characteristics interpolation of the incoming column.           */
/* ------------------------------------------------------------------ */
typedef struct {
    int nn;                 /* neighbours with non-zero geometric weight */
    int off[4][3];          /* their offsets from the source              */
    double s[4];            /* geometric weights                           */
} onbr;

static int iabs_(int v) { return v < 0 ? -v : v; }
static int isgn(int v) { return (v > 0) - (v < 0); }

/* Neighbours of the cell at offset d (not the source) with their weights. */
static void neighbours(const int d[3], onbr *nb)
{
    int ad[3] = {iabs_(d[0]), iabs_(d[1]), iabs_(d[2])};
    int m = ad[0];
    if (ad[1] > m) m = ad[1];
    if (ad[2] > m) m = ad[2];
    /* dominant axis: k if tied, then j, then i */
    int dom, u, v;
    if (ad[2] == m) { dom = 2; u = 0; v = 1; }
    else if (ad[1] == m) { dom = 1; u = 0; v = 2; }
    else { dom = 0; u = 1; v = 2; }
    double a = (double)ad[u] / (double)m;
    double b = (double)ad[v] / (double)m;
    double sw[4] = {(1 - a) * (1 - b), a * (1 - b), (1 - a) * b, a * b};
    int shift_u[4] = {0, 1, 0, 1}, shift_v[4] = {0, 0, 1, 1};
    nb->nn = 0;
    for (int n = 0; n < 4; ++n) {
        if (!(sw[n] > 0)) continue;
        int e[3] = {d[0], d[1], d[2]};
        e[dom] -= isgn(d[dom]);
        e[u] -= shift_u[n] * isgn(d[u]);
        e[v] -= shift_v[n] * isgn(d[v]);
        nb->off[nb->nn][0] = e[0];
        nb->off[nb->nn][1] = e[1];
        nb->off[nb->nn][2] = e[2];
        nb->s[nb->nn] = sw[n];
        nb->nn++;
    }
}

/* Unit-level access to the interpolation for pinning it: given the four
 * neighbour columns M (in e1..e4 order; entries with zero weight ignored),
 * return N_in for the cell at offset d.  Also returns the geometric weights. */
double oracle_interp(const int d[3], const double M4[4], double sigma0, double tau_w,
                     double s4_out[4])
{
    int ad[3] = {iabs_(d[0]), iabs_(d[1]), iabs_(d[2])};
    int m = ad[0];
    if (ad[1] > m) m = ad[1];
    if (ad[2] > m) m = ad[2];
    int u, v;
    if (ad[2] == m) { u = 0; v = 1; }
    else if (ad[1] == m) { u = 0; v = 2; }
    else { u = 1; v = 2; }
    double a = (double)ad[u] / (double)m;
    double b = (double)ad[v] / (double)m;
    double sw[4] = {(1 - a) * (1 - b), a * (1 - b), (1 - a) * b, a * b};
    double num = 0, den = 0;
    for (int n = 0; n < 4; ++n) {
        if (s4_out) s4_out[n] = sw[n];
        if (!(sw[n] > 0)) continue;
        double w = isfinite(tau_w) ? sw[n] / fmax(sigma0 * M4[n], tau_w) : sw[n];
        num += w * M4[n];
        den += w;
    }
    return num / den;
}

/* ------------------------------------------------------------------ */
/* The sweep                                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    int N;
    double alpha, sigma0, tau_w;
    int reading;               /* 0: directional source half path, 1: scalar */
    otab tab;
    int lo, hi;                /* periodic extent: lo <= d <= hi per axis    */
} octx;

static void extent(int N, int *lo, int *hi)
{
    if (N % 2 == 0) { *lo = -N / 2; *hi = N / 2 - 1; }
    else { *lo = -(N - 1) / 2; *hi = (N - 1) / 2; }
}

static long cell_index(int N, const int s[3], const int d[3])
{
    int i = ((s[0] + d[0]) % N + N) % N;
    int j = ((s[1] + d[1]) % N + N) % N;
    int k = ((s[2] + d[2]) % N + N) % N;
    return ((long)i * N + j) * N + k;
}

/* Per-source working storage, indexed by global cell. */
typedef struct {
    double *Nout;      /* exit column of each processed cell            */
    double *Nin;       /* entry column                                   */
    int *stamp;        /* source id + 1 of the last source that wrote it */
    int *shell;        /* shell index at which it was written            */
    long *order;       /* processing order: global cell index            */
    int (*order_d)[3]; /* and offset                                     */
    long count;
} owork;

/* Visit all cells of one source in shell order; store N_in, N_out.  When
 * gamma != NULL, accumulate the rate. Returns ORC_ECAUSAL if a neighbour was
 * not yet computed (which would break the causal ordering). */
static int sweep_source(const octx *c, const double *nHI, int sid, const int s[3], double Q,
                        double R, owork *w, double *gamma, double *coldens)
{
    const int N = c->N;
    const double alpha = c->alpha, sig = c->sigma0;
    const double four_pi = 4.0 * M_PI;
    const double R2 = R * R;
    long is = cell_index(N, s, (int[3]){0, 0, 0});
    double n_s = nHI[is];
    int Qmax = (int)ceil(sqrt(3.0) * R);
    w->count = 0;

    /* shell 0: the source cell, path half a cell, volume alpha^3 */
    {
        double tau_s = sig * n_s * alpha / 2;
        double P0 = tab_eval(&c->tab, 0.0, NULL, NULL);
        double G;
        if (n_s > 0) {
            double Ps = tab_eval(&c->tab, tau_s, NULL, NULL);
            G = Q * (P0 - Ps) / (n_s * alpha * alpha * alpha);
        } else {
            double dP;
            tab_eval(&c->tab, 0.0, &dP, NULL);
            G = Q * sig * (-dP) / (2 * alpha * alpha);
        }
        if (gamma) gamma[is] += G;
        w->Nin[is] = 0;
        w->Nout[is] = n_s * alpha / 2;   /* used only by reading B */
        w->stamp[is] = sid + 1;
        w->shell[is] = 0;
        w->order[w->count] = is;
        w->order_d[w->count][0] = w->order_d[w->count][1] = w->order_d[w->count][2] = 0;
        w->count++;
        if (coldens) coldens[is] = 0;
    }

    for (int q = 1; q <= Qmax; ++q) {
        for (int di = -q; di <= q; ++di) {
            int rj = q - iabs_(di);
            for (int dj = -rj; dj <= rj; ++dj) {
                int rk = rj - iabs_(dj);
                for (int t = 0; t < (rk == 0 ? 1 : 2); ++t) {
                    int dk = (rk == 0) ? 0 : (t == 0 ? -rk : rk);
                    int d[3] = {di, dj, dk};
                    if (di < c->lo || di > c->hi || dj < c->lo || dj > c->hi ||
                        dk < c->lo || dk > c->hi)
                        continue;
                    double r2 = (double)di * di + (double)dj * dj + (double)dk * dk;
                    if (r2 > R2) continue;
                    long ip = cell_index(N, s, d);
                    int m = iabs_(di);
                    if (iabs_(dj) > m) m = iabs_(dj);
                    if (iabs_(dk) > m) m = iabs_(dk);
                    double r = sqrt(r2);
                    double ds = r / (double)m;
                    onbr nb;
                    neighbours(d, &nb);
                    double num = 0, den = 0;
                    for (int n = 0; n < nb.nn; ++n) {
                        int *e = nb.off[n];
                        double M;
                        if (e[0] == 0 && e[1] == 0 && e[2] == 0) {
                            M = (c->reading == 0) ? n_s * alpha * ds / 2 : n_s * alpha / 2;
                        } else {
                            long ie = cell_index(N, s, e);
                            if (w->stamp[ie] != sid + 1 || w->shell[ie] >= q) return ORC_ECAUSAL;
                            M = w->Nout[ie];
                        }
                        double wn = isfinite(c->tau_w) ? nb.s[n] / fmax(sig * M, c->tau_w) : nb.s[n];
                        num += wn * M;
                        den += wn;
                    }
                    double Nin = num / den;
                    double n_p = nHI[ip];
                    double dN = n_p * alpha * ds;
                    double Nout = Nin + dN;
                    if (gamma) {
                        double G;
                        if (n_p > 0) {
                            double V = four_pi * (alpha * r) * (alpha * r) * (alpha * ds);
                            double Pin = tab_eval(&c->tab, sig * Nin, NULL, NULL);
                            double Pout = tab_eval(&c->tab, sig * Nout, NULL, NULL);
                            G = Q * (Pin - Pout) / (n_p * V);
                        } else {
                            double dP;
                            tab_eval(&c->tab, sig * Nin, &dP, NULL);
                            G = Q * sig * (-dP) / (four_pi * alpha * alpha * r2);
                        }
                        gamma[ip] += G;
                    }
                    if (coldens) coldens[ip] = Nin;
                    w->Nin[ip] = Nin;
                    w->Nout[ip] = Nout;
                    w->stamp[ip] = sid + 1;
                    w->shell[ip] = q;
                    w->order[w->count] = ip;
                    w->order_d[w->count][0] = di;
                    w->order_d[w->count][1] = dj;
                    w->order_d[w->count][2] = dk;
                    w->count++;
                }
            }
        }
    }
    return ORC_OK;
}

static int make_ctx(octx *c, int N, double alpha, double sigma0, int ntab, double lg_lo,
                    double lg_hi, const double *P, const double *dP, double tau_w, int reading)
{
    if (N <= 0 || ntab < 2 || !(alpha > 0) || !(sigma0 > 0) || !(lg_hi > lg_lo)) return ORC_EINVAL;
    for (int k = 0; k < ntab; ++k)
        if (!(P[k] > 0) || !isfinite(P[k]) || !isfinite(dP[k])) return ORC_EINVAL;
    c->N = N;
    c->alpha = alpha;
    c->sigma0 = sigma0;
    c->tau_w = (tau_w > 0) ? tau_w : INFINITY;
    c->reading = reading;
    c->tab.n = ntab;
    c->tab.lg_lo = lg_lo;
    c->tab.lg_hi = lg_hi;
    c->tab.P = P;
    c->tab.dP = dP;
    extent(N, &c->lo, &c->hi);
    return ORC_OK;
}

static int alloc_work(owork *w, long n3)
{
    w->Nout = (double *)malloc(sizeof(double) * n3);
    w->Nin = (double *)malloc(sizeof(double) * n3);
    w->stamp = (int *)calloc(n3, sizeof(int));
    w->shell = (int *)malloc(sizeof(int) * n3);
    w->order = (long *)malloc(sizeof(long) * n3);
    w->order_d = malloc(sizeof(int[3]) * n3);
    if (!w->Nout || !w->Nin || !w->stamp || !w->shell || !w->order || !w->order_d) return ORC_ENOMEM;
    return ORC_OK;
}

static void free_work(owork *w)
{
    free(w->Nout); free(w->Nin); free(w->stamp); free(w->shell); free(w->order); free(w->order_d);
}

/* Forward: gamma (N^3, accumulated, caller zeroes) and, for a single source,
 * the entry column N_in of every cell of the ball (coldens, may be NULL).
 * n_HI is passed directly (n_H * x_HI formed by the caller in FP64). */
int oracle_raytrace(int N, double alpha, double sigma0, int ntab, double lg_lo, double lg_hi,
                    const double *P, const double *dP, double tau_w, int reading,
                    const double *nHI, long nsrc, const int32_t *ijk, const double *Q,
                    const double *R, double *gamma, double *coldens)
{
    octx c;
    int st = make_ctx(&c, N, alpha, sigma0, ntab, lg_lo, lg_hi, P, dP, tau_w, reading);
    if (st) return st;
    if (coldens && nsrc != 1) return ORC_EINVAL;
    long n3 = (long)N * N * N;
    owork w;
    if (alloc_work(&w, n3)) { free_work(&w); return ORC_ENOMEM; }
    for (long sI = 0; sI < nsrc; ++sI) {
        if (!(R[sI] >= 0)) { st = ORC_EINVAL; break; }
        int s[3] = {ijk[3 * sI], ijk[3 * sI + 1], ijk[3 * sI + 2]};
        st = sweep_source(&c, nHI, (int)sI, s, Q[sI], R[sI], &w, gamma, coldens);
        if (st) break;
    }
    free_work(&w);
    return st;
}

/* Reverse mode of oracle_raytrace: given gbar = dL/dGamma (N^3), accumulate
 * nbar += dL/dn_HI (N^3) and write Qbar[s] = dL/dQ_s.  The chain rule is taken
 * through the same expressions as the forward, cell by cell, in the reverse of
 * the forward visiting order (so every consumer of a column is handled before
 * the cell that produced it).  Cells with n_HI = 0 are rejected (ORC_EZERO). */
int oracle_raytrace_grad(int N, double alpha, double sigma0, int ntab, double lg_lo,
                         double lg_hi, const double *P, const double *dP, double tau_w,
                         int reading, const double *nHI, long nsrc, const int32_t *ijk,
                         const double *Q, const double *R, const double *gbar, double *nbar,
                         double *Qbar)
{
    octx c;
    int st = make_ctx(&c, N, alpha, sigma0, ntab, lg_lo, lg_hi, P, dP, tau_w, reading);
    if (st) return st;
    long n3 = (long)N * N * N;
    owork w;
    double *Nbar = (double *)malloc(sizeof(double) * n3);
    if (!Nbar || alloc_work(&w, n3)) { free(Nbar); free_work(&w); return ORC_ENOMEM; }
    const double a_ = alpha, sig = sigma0, four_pi = 4.0 * M_PI;
    for (long sI = 0; sI < nsrc && !st; ++sI) {
        int s[3] = {ijk[3 * sI], ijk[3 * sI + 1], ijk[3 * sI + 2]};
        double Qs = Q[sI];
        st = sweep_source(&c, nHI, (int)sI, s, Qs, R[sI], &w, NULL, NULL);
        if (st) break;
        long is = w.order[0];
        double n_s = nHI[is];
        for (long t = 0; t < w.count; ++t) Nbar[w.order[t]] = 0;
        double qb = 0;
        for (long t = w.count - 1; t >= 1 && !st; --t) {
            long ip = w.order[t];
            int *d = w.order_d[t];
            double n_p = nHI[ip];
            if (!(n_p > 0)) { st = ORC_EZERO; break; }
            int m = iabs_(d[0]);
            if (iabs_(d[1]) > m) m = iabs_(d[1]);
            if (iabs_(d[2]) > m) m = iabs_(d[2]);
            double r2 = (double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2];
            double r = sqrt(r2), ds = r / (double)m;
            double Nin = w.Nin[ip], Nout = w.Nout[ip];
            double V = four_pi * (a_ * r) * (a_ * r) * (a_ * ds);
            double dPin, dPout;
            double Pin = tab_eval(&c.tab, sig * Nin, &dPin, NULL);
            double Pout = tab_eval(&c.tab, sig * Nout, &dPout, NULL);
            double G = Qs * (Pin - Pout) / (n_p * V);
            double g = gbar[ip];
            qb += g * G / Qs;
            double dG_dNin = Qs * sig * dPin / (n_p * V);
            double dG_dNout = -Qs * sig * dPout / (n_p * V);
            double dG_dn = -G / n_p;                 /* explicit 1/n_HI of eq. sugg */
            double T = Nbar[ip] + g * dG_dNout;      /* total adjoint of N_out       */
            nbar[ip] += T * a_ * ds + g * dG_dn;     /* N_out = N_in + n_HI alpha ds */
            double Nin_bar = T + g * dG_dNin;
            /* back through the interpolation N_in = sum w_n M_n / sum w_n */
            onbr nb;
            neighbours(d, &nb);
            double Mv[4], wv[4], dw[4], W = 0;
            for (int n = 0; n < nb.nn; ++n) {
                int *e = nb.off[n];
                if (e[0] == 0 && e[1] == 0 && e[2] == 0)
                    Mv[n] = (c.reading == 0) ? n_s * a_ * ds / 2 : n_s * a_ / 2;
                else
                    Mv[n] = w.Nout[cell_index(N, s, e)];
                if (isfinite(c.tau_w)) {
                    double tau = sig * Mv[n];
                    if (tau > c.tau_w) { wv[n] = nb.s[n] / tau; dw[n] = -nb.s[n] * sig / (tau * tau); }
                    else { wv[n] = nb.s[n] / c.tau_w; dw[n] = 0; }
                } else {
                    wv[n] = nb.s[n];
                    dw[n] = 0;
                }
                W += wv[n];
            }
            for (int n = 0; n < nb.nn; ++n) {
                int *e = nb.off[n];
                double dNin_dM = (wv[n] + (Mv[n] - Nin) * dw[n]) / W;
                double contrib = Nin_bar * dNin_dM;
                if (e[0] == 0 && e[1] == 0 && e[2] == 0)
                    nbar[is] += contrib * ((c.reading == 0) ? a_ * ds / 2 : a_ / 2);
                else
                    Nbar[cell_index(N, s, e)] += contrib;
            }
        }
        if (st) break;
        /* source cell */
        {
            if (!(n_s > 0)) { st = ORC_EZERO; break; }
            double tau_s = sig * n_s * a_ / 2;
            double dPs;
            double P0 = tab_eval(&c.tab, 0.0, NULL, NULL);
            double Ps = tab_eval(&c.tab, tau_s, &dPs, NULL);
            double V = a_ * a_ * a_;
            double G = Qs * (P0 - Ps) / (n_s * V);
            double g = gbar[is];
            qb += g * G / Qs;
            double dG_dn = -Qs * dPs * sig * a_ / 2 / (n_s * V) - G / n_s;
            nbar[is] += g * dG_dn;
        }
        Qbar[sI] = qb;
    }
    free(Nbar);
    free_work(&w);
    return st;
}

/* Visiting order of one source (offsets, shell by shell) -- for the
 * causality and shell-size checks.  Writes at most cap entries of 3 ints and
 * returns the number of cells (or a negative status). */
long oracle_shell_order(int N, double R, int32_t *out, int32_t *shell_out, long cap)
{
    int lo, hi;
    extent(N, &lo, &hi);
    int Qmax = (int)ceil(sqrt(3.0) * R);
    long cnt = 0;
    for (int q = 0; q <= Qmax; ++q)
        for (int di = -q; di <= q; ++di) {
            int rj = q - iabs_(di);
            for (int dj = -rj; dj <= rj; ++dj) {
                int rk = rj - iabs_(dj);
                for (int t = 0; t < (rk == 0 ? 1 : 2); ++t) {
                    int dk = (rk == 0) ? 0 : (t == 0 ? -rk : rk);
                    if (di < lo || di > hi || dj < lo || dj > hi || dk < lo || dk > hi) continue;
                    double r2 = (double)di * di + (double)dj * dj + (double)dk * dk;
                    if (r2 > R * R) continue;
                    if (cnt < cap) {
                        out[3 * cnt] = di; out[3 * cnt + 1] = dj; out[3 * cnt + 2] = dk;
                        if (shell_out) shell_out[cnt] = q;
                    }
                    cnt++;
                }
            }
        }
    return cnt;
}

/* Neighbours (offsets and geometric weights) of one cell, for the pins. */
int oracle_neighbours(const int32_t d[3], int32_t off_out[12], double s_out[4])
{
    if (d[0] == 0 && d[1] == 0 && d[2] == 0) return 0;
    onbr nb;
    int dd[3] = {d[0], d[1], d[2]};
    neighbours(dd, &nb);
    for (int n = 0; n < nb.nn; ++n) {
        off_out[3 * n] = nb.off[n][0];
        off_out[3 * n + 1] = nb.off[n][1];
        off_out[3 * n + 2] = nb.off[n][2];
        s_out[n] = nb.s[n];
    }
    return nb.nn;
}

/* ------------------------------------------------------------------ */
/* Hydrogen and helium: two absorbers (the extension the paper plans,   */
/* Sections 2 and 6).  Readings where the paper is silent:              */
/*  - the spectrum above 13.6 eV is split into bands at photon energies; */
/*    band b has a table P_b(T): the photons of the band that survive an */
/*    optical depth T measured at the band's lower edge, per photon      */
/*    emitted above 13.6 eV, and the cross-sections sH[b], sHe[b] of HI  */
/*    and HeI at that edge; within a band both cross-sections are taken  */
/*    to follow the band's frequency shape, so the band's optical depth  */
/*    is T_b = sH[b] N_HI + sHe[b] N_HeI;                                */
/*  - a cell absorbs Q [P_b(T_in) - P_b(T_out)] photons of band b (eq.   */
/*    sugg for the band), shared between the species in proportion to   */
/*    their in-cell optical depths; a species' rate is its share over    */
/*    n_i V (the limit sH[b] (-P_b') / (4 pi alpha^2 r^2) where the cell */
/*    holds none of it or nothing absorbs);                              */
/*  - both columns N_HI and N_HeI are carried by the same short          */
/*    characteristics with the hydrogen method's weights, the optical-   */
/*    depth factor taken on the HI column at the HI threshold            */
/*    (sigma0 N_HI): helium does not absorb at 13.6 eV;                  */
/*  - the source cell and its neighbours as for hydrogen, for each       */
/*    column (reading A: the exit column n alpha ds / 2 in the           */
/*    neighbour's direction).                                            */
/* ------------------------------------------------------------------ */
#define ORC_MAX_BANDS 8

typedef struct {
    int nb;
    otab tab[ORC_MAX_BANDS];
    double sH[ORC_MAX_BANDS], sHe[ORC_MAX_BANDS];
} oband;

/* Rates of one cell from its columns: n (species densities), Nin and dN
 * (entry and in-cell columns of HI and HeI), the volume factor 4 pi (alpha
 * r)^2 (alpha ds) as V, and the band loop.  Adds to *GH, *GHe. */
static void he_cell_rates(const oband *bd, double Q, const double n[2], const double Nin[2],
                          const double dN[2], double V, double area, double *GH, double *GHe)
{
    for (int b = 0; b < bd->nb; ++b) {
        const double s[2] = {bd->sH[b], bd->sHe[b]};
        double Tin = s[0] * Nin[0] + s[1] * Nin[1];
        double dT = s[0] * dN[0] + s[1] * dN[1];
        double dPin;
        double Pin = tab_eval(&bd->tab[b], Tin, &dPin, NULL);
        double Pout = tab_eval(&bd->tab[b], Tin + dT, NULL, NULL);
        double A = Q * (Pin - Pout);          /* photons of band b absorbed in the cell */
        double G[2];
        for (int i = 0; i < 2; ++i) {
            if (n[i] > 0 && dT > 0) {
                double share = s[i] * dN[i] / dT;
                G[i] = A * share / (n[i] * V);
            } else if (dT > 0) {
                G[i] = A * s[i] / (dT * area);   /* the same expression as n_i -> 0 */
            } else {
                G[i] = Q * s[i] * (-dPin) / area;
            }
        }
        *GH += G[0];
        *GHe += G[1];
    }
}

static int sweep_source_he(const octx *c, const oband *bd, const double *nH, const double *nHe, int sid,
                           const int s[3], double Q, double R, owork *w, double *NoutHe, double *gH,
                           double *gHe, double *cdH, double *cdHe)
{
    const int N = c->N;
    const double alpha = c->alpha, sig = c->sigma0;
    const double four_pi = 4.0 * M_PI;
    const double R2 = R * R;
    long is = cell_index(N, s, (int[3]){0, 0, 0});
    const double ns[2] = {nH[is], nHe[is]};
    int Qmax = (int)ceil(sqrt(3.0) * R);

    /* shell 0: the source cell, path half a cell, volume alpha^3 */
    {
        const double Nin[2] = {0, 0}, dN[2] = {ns[0] * alpha / 2, ns[1] * alpha / 2};
        double GH = 0, GHe = 0;
        /* area: the limit form with path half a cell, (alpha^3)/(alpha/2) */
        he_cell_rates(bd, Q, ns, Nin, dN, alpha * alpha * alpha, 2 * alpha * alpha, &GH, &GHe);
        gH[is] += GH;
        gHe[is] += GHe;
        w->Nout[is] = ns[0] * alpha / 2;
        NoutHe[is] = ns[1] * alpha / 2;
        w->stamp[is] = sid + 1;
        w->shell[is] = 0;
        if (cdH) cdH[is] = 0;
        if (cdHe) cdHe[is] = 0;
    }

    for (int q = 1; q <= Qmax; ++q) {
        for (int di = -q; di <= q; ++di) {
            int rj = q - iabs_(di);
            for (int dj = -rj; dj <= rj; ++dj) {
                int rk = rj - iabs_(dj);
                for (int t = 0; t < (rk == 0 ? 1 : 2); ++t) {
                    int dk = (rk == 0) ? 0 : (t == 0 ? -rk : rk);
                    int d[3] = {di, dj, dk};
                    if (di < c->lo || di > c->hi || dj < c->lo || dj > c->hi ||
                        dk < c->lo || dk > c->hi)
                        continue;
                    double r2 = (double)di * di + (double)dj * dj + (double)dk * dk;
                    if (r2 > R2) continue;
                    long ip = cell_index(N, s, d);
                    int m = iabs_(di);
                    if (iabs_(dj) > m) m = iabs_(dj);
                    if (iabs_(dk) > m) m = iabs_(dk);
                    double r = sqrt(r2);
                    double ds = r / (double)m;
                    onbr nb;
                    neighbours(d, &nb);
                    double numH = 0, numHe = 0, den = 0;
                    for (int n = 0; n < nb.nn; ++n) {
                        int *e = nb.off[n];
                        double MH, MHe;
                        if (e[0] == 0 && e[1] == 0 && e[2] == 0) {
                            double path = (c->reading == 0) ? alpha * ds / 2 : alpha / 2;
                            MH = ns[0] * path;
                            MHe = ns[1] * path;
                        } else {
                            long ie = cell_index(N, s, e);
                            if (w->stamp[ie] != sid + 1 || w->shell[ie] >= q) return ORC_ECAUSAL;
                            MH = w->Nout[ie];
                            MHe = NoutHe[ie];
                        }
                        /* the hydrogen method's weights, on the HI column */
                        double wn = isfinite(c->tau_w) ? nb.s[n] / fmax(sig * MH, c->tau_w) : nb.s[n];
                        numH += wn * MH;
                        numHe += wn * MHe;
                        den += wn;
                    }
                    const double Nin[2] = {numH / den, numHe / den};
                    const double np[2] = {nH[ip], nHe[ip]};
                    const double dN[2] = {np[0] * alpha * ds, np[1] * alpha * ds};
                    double V = four_pi * (alpha * r) * (alpha * r) * (alpha * ds);
                    double GH = 0, GHe = 0;
                    he_cell_rates(bd, Q, np, Nin, dN, V, four_pi * alpha * alpha * r2, &GH, &GHe);
                    gH[ip] += GH;
                    gHe[ip] += GHe;
                    if (cdH) cdH[ip] = Nin[0];
                    if (cdHe) cdHe[ip] = Nin[1];
                    w->Nout[ip] = Nin[0] + dN[0];
                    NoutHe[ip] = Nin[1] + dN[1];
                    w->stamp[ip] = sid + 1;
                    w->shell[ip] = q;
                }
            }
        }
    }
    return ORC_OK;
}

/* Rates of HI and HeI (N^3 each, accumulated, caller zeroes) for nb bands:
 * tables P, dP as nb x ntab (band b on its own nodes, uniform in log10 tau
 * from lg_lo[b] to lg_hi[b]), cross-sections sH, sHe per band.  nH, nHe:
 * n_HI and n_HeI.  Single source: the entry columns of both species
 * (coldens_H, coldens_He, may be NULL). */
int oracle_raytrace_he(int N, double alpha, double sigma0, int nb, int ntab, const double *lg_lo,
                       const double *lg_hi, const double *P, const double *dP, const double *sH,
                       const double *sHe, double tau_w, int reading, const double *nH, const double *nHe,
                       long nsrc, const int32_t *ijk, const double *Q, const double *R, double *gH,
                       double *gHe, double *coldens_H, double *coldens_He)
{
    if (nb < 1 || nb > ORC_MAX_BANDS) return ORC_EINVAL;
    octx c;
    int st = make_ctx(&c, N, alpha, sigma0, ntab, lg_lo[0], lg_hi[0], P, dP, tau_w, reading);
    if (st) return st;
    if ((coldens_H || coldens_He) && nsrc != 1) return ORC_EINVAL;
    oband bd;
    bd.nb = nb;
    for (int b = 0; b < nb; ++b) {
        if (!(lg_hi[b] > lg_lo[b]) || !(sH[b] >= 0) || !(sHe[b] >= 0)) return ORC_EINVAL;
        for (int k = 0; k < ntab; ++k)
            if (!(P[b * ntab + k] > 0) || !isfinite(P[b * ntab + k]) || !isfinite(dP[b * ntab + k]))
                return ORC_EINVAL;
        bd.tab[b] = (otab){ntab, lg_lo[b], lg_hi[b], P + (long)b * ntab, dP + (long)b * ntab};
        bd.sH[b] = sH[b];
        bd.sHe[b] = sHe[b];
    }
    long n3 = (long)N * N * N;
    owork w;
    double *NoutHe = (double *)malloc(sizeof(double) * n3);
    if (!NoutHe || alloc_work(&w, n3)) { free(NoutHe); free_work(&w); return ORC_ENOMEM; }
    for (long sI = 0; sI < nsrc; ++sI) {
        if (!(R[sI] >= 0)) { st = ORC_EINVAL; break; }
        int s[3] = {ijk[3 * sI], ijk[3 * sI + 1], ijk[3 * sI + 2]};
        st = sweep_source_he(&c, &bd, nH, nHe, (int)sI, s, Q[sI], R[sI], &w, NoutHe, gH, gHe, coldens_H,
                             coldens_He);
        if (st) break;
    }
    free(NoutHe);
    free_work(&w);
    return st;
}
