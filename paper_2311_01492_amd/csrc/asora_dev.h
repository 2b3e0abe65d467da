// asora_dev.h -- device (and host-planning) building blocks of the ASORA sweep
// for gfx950: table interpolant, shell/row enumeration of a source piece,
// the short-characteristics cell update.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asora {

// Approximate reciprocal (about 1 ulp): the hardware instruction on the GPU.
__host__ __device__ __forceinline__ float rcp_approx(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// 1/x to about half an ulp: hardware estimate and one Newton step.
__host__ __device__ __forceinline__ float rcp_nr(float x)
{
    const float r = rcp_approx(x);
    return r * (2.f - x * r);
}

// 1/x in FP64 for positive x within the FP32 range: FP32 estimate and one
// FP64 Newton step (relative error ~1e-14, far cheaper than a full FP64
// division).
__host__ __device__ __forceinline__ double rcp_f64(double x)
{
    const double r = (double)rcp_approx((float)x);
    return r * (2.0 - x * r);
}

// --------------------------------------------------------------------------
// Photoionization table P(tau) (eq. tables, Section 2.2, normalised to P(0)=1)
// in the form the kernels read it.  Node k sits at x_k = x_lo + k h, x = ln tau.
// Between nodes ln P is the cubic Hermite spline with node values y_k = ln P_k
// and node slopes m_k = d ln P / d ln tau = tau_k P'_k / P_k.  Below the first
// node P is the tangent line there; above the last node it is constant.
// --------------------------------------------------------------------------
struct TabNode {
    double y;   // ln P_k (FP64: differences of y across many nodes must stay exact)
    float m;    // d ln P / d ln tau at node k
    float P;    // P_k (FP32: only multiplied, never subtracted)
};
static_assert(sizeof(TabNode) == 16, "TabNode must be 16 bytes");

struct TabParams {
    int n;          // number of nodes
    double x_lo;    // ln tau_0
    double inv_h;   // 1 / h, h = node spacing in ln tau
    float h, inv_hf;
    double tau_lo;  // tau_0
    double tau_hi;  // tau_{n-1}
    float dP0;      // dP/dtau at tau_0 (slope of the linear continuation)
};

struct Cubic {
    float c1, c2, c3;   // ln P(x_j + t h) - y_j = t (c1 + t (c2 + t c3)), t in [0,1]
};

__host__ __device__ __forceinline__ Cubic cubic_at(const TabNode *T, int j, float h)
{
    const TabNode a = T[j], b = T[j + 1];
    const float d = (float)(b.y - a.y);
    const float hm0 = h * a.m, hm1 = h * b.m;
    Cubic c;
    c.c1 = hm0;
    c.c2 = 3.f * d - 2.f * hm0 - hm1;
    c.c3 = -2.f * d + hm0 + hm1;
    return c;
}

__host__ __device__ __forceinline__ float cubic_val(const Cubic &c, float t)
{
    return t * (c.c1 + t * (c.c2 + t * c.c3));
}

// [p(t2) - p(t1)] / (t2 - t1) for the cubic p, written without the
// subtraction so that it stays exact as t2 -> t1 (then it is p'(t1)).
__host__ __device__ __forceinline__ float cubic_dd(const Cubic &c, float t1, float t2)
{
    return c.c1 + c.c2 * (t1 + t2) + c.c3 * (t1 * t1 + t1 * t2 + t2 * t2);
}

// Divided difference [P(a+dt) - P(a)] / dt of the spline part, for
// tau_lo <= a and a + dt <= tau_hi.  The difference is formed in log space
// (P(a) expm1(delta ln P)) so that it keeps full relative accuracy when dt is
// small against a, and delta ln P is summed piecewise when both ends share an
// interval or sit in neighbouring ones.
__host__ __device__ __forceinline__ float divdiff_spline(const TabNode *T, const TabParams &tp, double a,
                                                double dt)
{
    const double xa = log(a);
    const double ta = (xa - tp.x_lo) * tp.inv_h;
    int ja = (int)floor(ta);
    ja = ja < 0 ? 0 : (ja > tp.n - 2 ? tp.n - 2 : ja);
    const float fa = (float)(ta - (double)ja);
    const Cubic ca = cubic_at(T, ja, tp.h);
    const float corr_a = cubic_val(ca, fa);
    const float Pa = T[ja].P * expf(corr_a);
    const float u = (float)(dt / a);
    if (!(u > 1e-12f)) {
        // zero-width interval: the slope of the interpolant at a
        const float yx = cubic_dd(ca, fa, fa) * tp.inv_hf;
        return Pa * yx / (float)a;
    }
    const float dtn = log1pf(u) * tp.inv_hf;   // (x_b - x_a) / h
    const float tb = fa + dtn;
    float dy;
    if (tb <= 1.f || ja == tp.n - 2) {
        // same interval (on the last interval b <= tau_hi, so tb > 1 is rounding)
        dy = dtn * cubic_dd(ca, fa, fminf(tb, 1.f));
    } else if (tb <= 2.f) {
        const float d1 = 1.f - fa;
        const float d2 = dtn - d1;
        const Cubic cb = cubic_at(T, ja + 1, tp.h);
        dy = d1 * cubic_dd(ca, fa, 1.f) + d2 * cubic_dd(cb, 0.f, d2);
    } else {
        const double tbb = (log(a + dt) - tp.x_lo) * tp.inv_h;
        int jb = (int)floor(tbb);
        jb = jb < 0 ? 0 : (jb > tp.n - 2 ? tp.n - 2 : jb);
        const float fb = (float)(tbb - (double)jb);
        const Cubic cb = cubic_at(T, jb, tp.h);
        dy = (float)(T[jb].y - T[ja].y) + (cubic_val(cb, fb) - corr_a);
    }
    return Pa * expm1f(dy) / (float)dt;
}

// -D = -[P(a+dt) - P(a)] / dt >= 0 of the full interpolant (linear piece,
// spline, constant piece), for a >= 0 and dt >= 0.  An interval that
// straddles a piece boundary is split; the pieces' slopes are averaged with
// their lengths as weights (all of one sign, so nothing cancels).
__host__ __device__ __forceinline__ float neg_divdiff(const TabNode *T, const TabParams &tp, double a,
                                             double dt)
{
    if (a >= tp.tau_hi) return 0.f;
    const double b = a + dt;
    if (b < tp.tau_lo) return -tp.dP0;
    if (a >= tp.tau_lo && b <= tp.tau_hi) return -divdiff_spline(T, tp, a, dt);
    const double aH = a > tp.tau_lo ? a : tp.tau_lo;
    const double bH = b < tp.tau_hi ? b : tp.tau_hi;
    const double lenL = a < tp.tau_lo ? tp.tau_lo - a : 0.0;
    const double lenH = bH - aH;
    const double DH = lenH > 0 ? (double)divdiff_spline(T, tp, aH, lenH) : 0.0;
    return (float)(-((double)tp.dP0 * lenL + DH * lenH) / dt);
}

// --------------------------------------------------------------------------
// Pieces.  The cells of one source split into closed regions whose columns
// depend only on cells of the same region:
//   kind 0 ("whole"): all eight octants, each half-open (a zero coordinate
//          belongs to the + side), no duplicated cells;
//   kind 1: one closed octant (zero planes included).  Cells with a zero
//          coordinate on a negative axis of the octant are "ghosts": computed
//          because the octant's own cells need them, but their rate is added
//          by the octant that owns them.
// With dom >= 0 the piece keeps only cells whose dominant axis (largest |d|,
// ties included) is dom: all their non-zero-weight neighbours keep that axis
// dominant, so the region stays closed; a tied cell is owned by the piece of
// its first dominant axis in the order k, j, i.
// Octant bits: 1 = i negative, 2 = j negative, 4 = k negative.
// Octant coordinates (A, B, C) = (|di|, |dj|, |dk|).
// --------------------------------------------------------------------------
struct Piece {
    int kind;    // 0 whole, 1 single octant
    int oct;     // octant of kind 1
    int dom;     // -1 any, else 0/1/2 = i/j/k
    int n_oct;   // 8 or 1
};

// Periodic extent: offsets in [-ext_neg, ext_pos] (Appendix A).
struct Extent {
    int pos, neg;
};

__host__ __device__ inline Extent make_extent(int N)
{
    Extent e;
    if (N % 2 == 0) { e.pos = N / 2 - 1; e.neg = N / 2; }
    else { e.pos = (N - 1) / 2; e.neg = (N - 1) / 2; }
    return e;
}

// Row r of shell q of a piece: octant slot os = r / (q+1), A = r % (q+1).
// Returns the first B and the number of cells (B contiguous).  Exact integer
// ball test A^2 + B^2 + C^2 <= Rsq.
__host__ __device__ inline void row_range(const Piece &pc, const Extent &ex, int Rsq, int q, int r,
                                          int *Blo, int *cnt)
{
    *Blo = 0;
    *cnt = 0;
    const int os = r / (q + 1);
    const int A = r - os * (q + 1);
    const int o = pc.kind == 0 ? os : pc.oct;
    const int ni = o & 1, nj = (o >> 1) & 1, nk = (o >> 2) & 1;
    const int half = pc.kind == 0;
    const int loA = half & ni, loB = half & nj, loC = half & nk;
    const int hiA = ni ? ex.neg : ex.pos;
    const int hiB = nj ? ex.neg : ex.pos;
    const int hiC = nk ? ex.neg : ex.pos;
    if (A < loA || A > hiA) return;
    const int s = q - A;
    int lo = loB > s - hiC ? loB : s - hiC;
    int hi = hiB < s - loC ? hiB : s - loC;
    if (pc.dom == 0) {
        hi = hi < A ? hi : A;
        lo = lo > s - A ? lo : s - A;
    } else if (pc.dom == 1) {
        const int m = A > (s + 1) / 2 ? A : (s + 1) / 2;
        lo = lo > m ? lo : m;
    } else if (pc.dom == 2) {
        const int m = (s - A) < s / 2 ? (s - A) : s / 2;
        hi = hi < m ? hi : m;
    }
    const int rem = Rsq - A * A;
    if (rem < 0) return;
    const int disc = 2 * rem - s * s;
    if (disc < 0) return;
    const float sq = sqrtf((float)disc);
    int bl = (int)ceilf(0.5f * ((float)s - sq));
    int bh = (int)floorf(0.5f * ((float)s + sq));
    // one correction step each way makes the float bounds exact
    if (bl * bl + (s - bl) * (s - bl) > rem) bl++;
    else if ((bl - 1) * (bl - 1) + (s - bl + 1) * (s - bl + 1) <= rem) bl--;
    if (bh * bh + (s - bh) * (s - bh) > rem) bh--;
    else if ((bh + 1) * (bh + 1) + (s - bh - 1) * (s - bh - 1) <= rem) bh++;
    lo = lo > bl ? lo : bl;
    hi = hi < bh ? hi : bh;
    if (hi >= lo) {
        *Blo = lo;
        *cnt = hi - lo + 1;
    }
}

// Largest L1 shell a source of squared radius Rsq can reach inside the extent.
__host__ __device__ inline int max_shell(int Rsq, const Extent &ex)
{
    int q = (int)floor(sqrt(3.0 * (double)Rsq)) + 1;
    while (q > 0 && (double)q * q > 3.0 * (double)Rsq) --q;
    const int qe = 3 * ex.neg;
    return q < qe ? q : qe;
}

__host__ __device__ inline Piece make_piece(int type, int p)
{
    Piece pc;
    if (type == 0) { pc.kind = 0; pc.oct = 0; pc.dom = -1; pc.n_oct = 8; }
    else if (type == 1) { pc.kind = 1; pc.oct = p; pc.dom = -1; pc.n_oct = 1; }
    else { pc.kind = 1; pc.oct = p / 3; pc.dom = p % 3; pc.n_oct = 1; }
    return pc;
}

__host__ __device__ inline int pieces_of_type(int type)
{
    return type == 0 ? 1 : (type == 1 ? 8 : 24);
}

// Last row r in [0, nrows) with rowstart[r] <= g (rowstart[0] = 0 <= g).
__host__ __device__ __forceinline__ int find_row(const int *rowstart, int nrows, int g)
{
    int lo = 0, hi = nrows;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rowstart[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

__host__ __device__ __forceinline__ int wrap(int v, int N)
{
    v += v < 0 ? N : 0;
    v -= v >= N ? N : 0;
    return v;
}

// Everything one cell update needs that is uniform over a piece.
struct CellCtx {
    Piece pc;
    int N, si, sj, sk;
    int reading;           // 0: directional source half path, 1: scalar
    float tau_w;           // <= 0: geometric weights
    double sigma0, alpha;
    double half_col;       // n_HI(s) alpha / 2
    double coef;           // Q sigma0 / (4 pi alpha^2)
    const TabNode *tab;
    TabParams tp;
    const double *ring;    // [4][ring_cap] exit columns of shells q-1..q-3
    const int *rowbase;    // [4][row_cap]
    int ring_cap, row_cap;
    const double *nHI;     // n_H x_HI, exact product of the FP32 inputs
};

struct CellOut {
    long cp;        // global cell index
    double Nin, Nout;
    double G;       // rate contribution (0 if none)
    bool owned;
};

// The short-characteristics update of the cell with compact index g in shell
// q (row `row` of the shell's row table, base rb = rowbase of that row):
// interpolate the entry column from the neighbours (eq. raga, eq. interp),
// add the in-cell column (Section 3.1) and form the rate (eq. sugg).
__host__ __device__ __forceinline__ void cell_update(const CellCtx &X, int q, int g, int row,
                                                     int rb, CellOut &out)
{
    const int os = row / (q + 1);
    const int cA = row - os * (q + 1);
    const int cB = g - rb;
    const int cC = q - cA - cB;
    const int o = X.pc.kind == 0 ? os : X.pc.oct;
    const int di = (o & 1) ? -cA : cA;
    const int dj = (o & 2) ? -cB : cB;
    const int dk = (o & 4) ? -cC : cC;
    const int N = X.N;
    const long cp = ((long)wrap(X.si + di, N) * N + wrap(X.sj + dj, N)) * N + wrap(X.sk + dk, N);
    const double nhi = X.nHI[cp];

    // geometry: dominant axis, bilinear weights, path length
    const int m = cA > cB ? (cA > cC ? cA : cC) : (cB > cC ? cB : cC);
    const int canon = cC == m ? 2 : (cB == m ? 1 : 0);
    const int dd = X.pc.dom >= 0 ? X.pc.dom : canon;
    // the other two axes, in the order (i, j), (i, k), (j, k)
    const int cu = dd == 0 ? cB : cA;
    const int cv = dd == 2 ? cB : cC;
    const double inv_m = rcp_f64((double)m);
    // a = 1 (b = 1) must be exact: the weights of neighbours that leave the
    // dominant-axis layer then vanish exactly
    const double a = cu == m ? 1.0 : (double)cu * inv_m;
    const double b = cv == m ? 1.0 : (double)cv * inv_m;
    const int r2 = cA * cA + cB * cB + cC * cC;
    const double ds = sqrt((double)r2) * inv_m;
    const double sw[4] = {(1.0 - a) * (1.0 - b), a * (1.0 - b), (1.0 - a) * b, a * b};

    // interpolate the entry column from the (up to) four neighbours,
    // N_in = sum w M / sum w, in FP64: the column is carried along every
    // characteristic, and at optical depths of 10^3 the rate moves ten times
    // faster than the column, so the weights must not leave FP32 rounding in it
    double num = 0.0, W = 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        if (!(sw[n] > 0.0)) continue;
        // offsets: the dominant axis always, u for n = 1, 3 and v for n = 2, 3
        const int su = n & 1, sv = (n >> 1) & 1;
        const int eA = cA - (dd == 0 ? 1 : 0) - (su & (dd != 0 ? 1 : 0));
        const int eB = cB - (dd == 1 ? 1 : 0) - (su & (dd == 0 ? 1 : 0)) - (sv & (dd == 2 ? 1 : 0));
        const int eC = cC - (dd == 2 ? 1 : 0) - (sv & (dd != 2 ? 1 : 0));
        const int qn = q - 1 - su - sv;
        double M;
        if (qn == 0) {
            M = X.reading == 0 ? X.half_col * ds : X.half_col;
        } else {
            int o2 = o;
            if (X.pc.kind == 0) {   // half-open octants: zero planes live in the + octant
                if ((o2 & 1) && eA == 0) o2 &= ~1;
                if ((o2 & 2) && eB == 0) o2 &= ~2;
                if ((o2 & 4) && eC == 0) o2 &= ~4;
            }
            const int ord = X.pc.kind == 0 ? o2 : 0;
            const int sl = qn & 3;
            const int nrow = ord * (qn + 1) + eA;
            M = X.ring[sl * X.ring_cap + X.rowbase[sl * X.row_cap + nrow] + eB];
        }
        double wn = sw[n];
        if (X.tau_w > 0.f) wn *= rcp_f64(fmax(X.sigma0 * M, (double)X.tau_w));
        num += wn * M;
        W += wn;
    }
    const double Nin = num * rcp_f64(W);
    const double dN = nhi * X.alpha * ds;
    const double Nout = Nin + dN;

    // ownership: ghosts of a closed octant, tied cells of a pyramid
    bool owned = true;
    if (X.pc.kind == 1) {
        if (((o & 1) && cA == 0) || ((o & 2) && cB == 0) || ((o & 4) && cC == 0)) owned = false;
        if (X.pc.dom >= 0 && canon != X.pc.dom) owned = false;
    }
    double G = 0.0;
    if (owned) {
        const double ta = X.sigma0 * Nin;
        if (ta < X.tp.tau_hi) {
            const float nd = neg_divdiff(X.tab, X.tp, ta, X.sigma0 * dN);
            if (nd > 0.f) G = X.coef * (double)(nd * rcp_approx((float)r2));
        }
    }
    out.cp = cp;
    out.Nin = Nin;
    out.Nout = Nout;
    out.G = G;
    out.owned = owned;
}

// Rate of the source cell itself: entry column 0, path half a cell, volume
// alpha^3.
__host__ __device__ __forceinline__ double source_cell_rate(const TabNode *T, const TabParams &tp,
                                                            double sigma0, double alpha, double Q,
                                                            double n_s)
{
    const double tau_s = sigma0 * n_s * alpha * 0.5;
    const float nd = neg_divdiff(T, tp, 0.0, tau_s);
    return Q * sigma0 / (2.0 * alpha * alpha) * (double)nd;
}

// Build the row table of shell q of a piece (serial form; the kernel runs
// the same per-row computation in parallel with a wave-wide scan).
__host__ __device__ inline int build_rows(const Piece &pc, const Extent &ex, int Rsq, int q,
                                          int *rowstart, int *rowbase_q)
{
    const int nrows = pc.n_oct * (q + 1);
    int run = 0;
    for (int r = 0; r < nrows; ++r) {
        int blo, cnt;
        row_range(pc, ex, Rsq, q, r, &blo, &cnt);
        rowstart[r] = run;
        rowbase_q[r] = run - blo;
        run += cnt;
    }
    rowstart[nrows] = run;
    return run;
}

}  // namespace asora
