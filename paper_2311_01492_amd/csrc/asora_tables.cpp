// asora_tables.cpp -- host construction of the photoionization tables
// P(tau) = gamma(tau/sigma0)/gamma(0) and dP/dtau (eq. tables, Section 2.2)
// for a black-body spectrum behind a power-law cross-section (Section 4.1),
// and of the photo-heating table of the same spectrum: H(tau), the energy
// above threshold (eV) that the photons still carry per emitted photon, the
// photon count of P weighted by h nu - h nu_th.
//
// Also the band tables of a spectrum split at photon energies (several
// absorbers): the photons of one band that survive an optical depth tau
// measured at the band's lower edge, per photon emitted above 13.6 eV.
//
// Integration: x = h nu / k T from x0 = 13.6 eV / kT (or a band's lower edge)
// to 800 (the integrand is below e^-790 of its peak beyond) or the band's
// upper edge, substituted x = x_a + u^2 so that panels crowd towards the
// lower edge, and a composite 20-point Gauss-Legendre rule on 240 panels in
// u.  The Legendre nodes are found by Newton's method on the three-term
// recurrence.
#include <cmath>
#include <vector>

#include "asora_dev.h"

namespace asora {

namespace {

constexpr double kBoltzmannEv = 8.617333262e-5;   // eV / K
constexpr double kThresholdEv = 13.6;             // hydrogen ionization threshold
constexpr int kGL = 20;
constexpr int kPanels = 240;
constexpr double kXUpper = 800.0;

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

// Quadrature points of int_{x_a}^{x_b} f(x) dx (x_b <= kXUpper), x = x_a + u^2:
// positions x and weights (Jacobian included).
static void band_points(double x_a, double x_b, std::vector<double> &xs, std::vector<double> &ws)
{
    std::vector<double> gx, gw;
    gauss_legendre(kGL, gx, gw);
    const double u_hi = std::sqrt(x_b - x_a);
    const double du = u_hi / kPanels;
    xs.resize(kGL * kPanels);
    ws.resize(kGL * kPanels);
    for (int p = 0; p < kPanels; ++p) {
        const double c = (p + 0.5) * du;
        for (int k = 0; k < kGL; ++k) {
            const double u = c + 0.5 * du * gx[k];
            xs[p * kGL + k] = x_a + u * u;
            ws[p * kGL + k] = 0.5 * du * gw[k] * 2.0 * u;
        }
    }
}

static double photons(double x) { return x * x * std::exp(-x) / -std::expm1(-x); }   // x^2/(e^x-1)

// The photons of [x_a, x_b) that survive an optical depth tau at x_a, with the
// cross-section shape (x / x_a)^-index, per photon emitted above the hydrogen
// threshold x0 (x_a = x0, x_b = kXUpper: the whole spectrum).  heat = true
// weighs each photon by its energy above x0 (eV).
static int blackbody(double T_bb, double index, double x_a, double x_b, int n, double lg_lo, double lg_hi,
                     bool heat, double *P, double *dP)
{
    if (!(T_bb > 0) || !(n >= 2) || !(lg_hi > lg_lo) || !P || !dP) return -1;
    const double x0 = kThresholdEv / (kBoltzmannEv * T_bb);
    x_b = x_b < kXUpper ? x_b : kXUpper;
    if (!(x0 < kXUpper) || !(x_a >= x0) || !(x_b > x_a)) return -1;
    std::vector<double> xs, ws, xn, wn;
    band_points(x0, kXUpper, xn, wn);
    double norm = 0.0;
    for (size_t i = 0; i < xn.size(); ++i) norm += wn[i] * photons(xn[i]);
    band_points(x_a, x_b, xs, ws);
    const size_t npts = xs.size();
    std::vector<double> wphi(npts), shape(npts);
    for (size_t i = 0; i < npts; ++i) {
        wphi[i] = ws[i] * photons(xs[i]);
        if (heat) wphi[i] *= (xs[i] - x0) * kBoltzmannEv * T_bb;   // energy above threshold
        shape[i] = std::pow(xs[i] / x_a, -index);
    }
    for (int t = 0; t < n; ++t) {
        const double tau = std::pow(10.0, lg_lo + (lg_hi - lg_lo) * t / (double)(n - 1));
        double s0 = 0.0, s1 = 0.0;
        for (size_t i = 0; i < npts; ++i) {
            const double e = wphi[i] * std::exp(-tau * shape[i]);
            s0 += e;
            s1 += e * shape[i];
        }
        P[t] = s0 / norm;
        dP[t] = -s1 / norm;
    }
    return 0;
}

int table_blackbody(double T_bb, double index, int n, double lg_lo, double lg_hi, double *P,
                    double *dP)
{
    const double x0 = kThresholdEv / (kBoltzmannEv * T_bb);
    return blackbody(T_bb, index, x0, kXUpper, n, lg_lo, lg_hi, false, P, dP);
}

int table_blackbody_heat(double T_bb, double index, int n, double lg_lo, double lg_hi, double *H,
                         double *dH)
{
    const double x0 = kThresholdEv / (kBoltzmannEv * T_bb);
    return blackbody(T_bb, index, x0, kXUpper, n, lg_lo, lg_hi, true, H, dH);
}

int table_blackbody_band(double T_bb, double index, double e_lo_ev, double e_hi_ev, int n, double lg_lo,
                         double lg_hi, double *P, double *dP)
{
    if (!(T_bb > 0) || !(e_lo_ev >= kThresholdEv) || !(e_hi_ev > e_lo_ev)) return -1;
    const double kT = kBoltzmannEv * T_bb;
    return blackbody(T_bb, index, e_lo_ev / kT, std::isfinite(e_hi_ev) ? e_hi_ev / kT : kXUpper, n, lg_lo,
                     lg_hi, false, P, dP);
}

// The table in the form the kernels read (see TabNode): node values ln P,
// log-log slopes tau P'/P, FP32 P, and the parameters of the node grid.
void prepare_table(int n, double lg_lo, double lg_hi, const double *P, const double *dP,
                   TabParams *tp, TabNode *nodes, double *m64)
{
    const double ln10 = std::log(10.0);
    tp->n = n;
    tp->x_lo = lg_lo * ln10;
    const double h = (lg_hi - lg_lo) * ln10 / (double)(n - 1);
    tp->inv_h = 1.0 / h;
    tp->h = (float)h;
    tp->inv_hf = (float)(1.0 / h);
    tp->h64 = h;
    tp->tau_lo = std::exp(tp->x_lo);
    tp->tau_hi = std::exp(tp->x_lo + h * (n - 1));
    tp->dP0 = (float)dP[0];
    for (int k = 0; k < n; ++k) {
        const double tk = std::exp(tp->x_lo + h * k);
        nodes[k].y = std::log(P[k]);
        const double m = tk * dP[k] / P[k];
        nodes[k].m = (float)m;
        nodes[k].P = (float)P[k];
        if (m64) m64[k] = m;
    }
}

}  // namespace asora
