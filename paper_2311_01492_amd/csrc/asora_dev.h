// asora_dev.h -- device (and host-planning) building blocks of the ASORA sweep
// for gfx950: table interpolant, shell/row enumeration of a source piece,
// the short-characteristics cell update.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asora {

constexpr int kXcds = 8;   // accelerator dies (XCDs) of the MI355X, each with its own L2
// Ints between two work counters: every counter has a 128-byte line of its
// own, so that the atomics of different dies do not serialise on one line.
constexpr int kCounterPad = 32;

// Approximate reciprocal (about 1 ulp): the hardware instruction on the GPU.
__host__ __device__ __forceinline__ float rcp_approx(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// 2^x in FP32: the hardware instruction on the GPU (about 1 ulp).
__host__ __device__ __forceinline__ float exp2_fast(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(x);
#else
    return exp2f(x);
#endif
}

// e^x for |x| <~ 1 in FP32, relative error ~1e-7.
__host__ __device__ __forceinline__ float exp_small(float x)
{
    return exp2_fast(x * 1.44269504088896341f);
}

// e^x - 1 in FP32 with full relative accuracy near 0: Taylor series (to x^9)
// for |x| < 0.5, else e^x - 1 (relative error below 3e-7 there).
__host__ __device__ __forceinline__ float expm1_fast(float x)
{
    if (fabsf(x) < 0.5f) {
        float p = 1.f / 362880.f;
        p = p * x + 1.f / 40320.f;
        p = p * x + 1.f / 5040.f;
        p = p * x + 1.f / 720.f;
        p = p * x + 1.f / 120.f;
        p = p * x + 1.f / 24.f;
        p = p * x + 1.f / 6.f;
        p = p * x + 0.5f;
        p = p * x + 1.f;
        return p * x;
    }
    return exp2_fast(x * 1.44269504088896341f) - 1.f;
}

// 1/x to about half an ulp: hardware estimate and one Newton step.
__host__ __device__ __forceinline__ float rcp_nr(float x)
{
    const float r = rcp_approx(x);
    return r * (2.f - x * r);
}

// 1/x in FP64 for positive x within the FP32 normal range (about 1e-38 to
// 3e38): FP32 estimate and one
// FP64 Newton step (relative error ~1e-14, far cheaper than a full FP64
// division).
__host__ __device__ __forceinline__ double rcp_f64(double x)
{
    const double r = (double)rcp_approx((float)x);
    return r * (2.0 - x * r);
}

// sqrt(x) in FP64 for x within the FP32 normal range: FP32 reciprocal square
// root estimate and one Goldschmidt step (relative error ~1e-14).
__host__ __device__ __forceinline__ double sqrt_fast(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = (double)__builtin_amdgcn_rsqf((float)x);
#else
    const double y = 1.0 / (double)sqrtf((float)x);
#endif
    double g = x * y;
    const double h = 0.5 * y;
    const double e = 0.5 - g * h;
    return g + g * e;
}

// ln(a) in FP64 for normal a > 0, absolute error below 2e-11: the mantissa
// is reduced to [1/sqrt2, sqrt2) and ln m = 2 atanh(s), s = (m-1)/(m+1),
// |s| <= 0.172, summed to s^11.  (The table position needs ln tau to ~1e-9
// absolute; a correctly rounded FP64 log costs several times more.)
__host__ __device__ __forceinline__ double log_fast(double a)
{
    int e;
    double m = frexp(a, &e);
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) * rcp_f64(m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 11.0;
    p = p * s2 + 1.0 / 9.0;
    p = p * s2 + 1.0 / 7.0;
    p = p * s2 + 1.0 / 5.0;
    p = p * s2 + 1.0 / 3.0;
    p = p * s2 + 1.0;
    return 2.0 * s * p + (double)e * 0.69314718055994530942;
}

// ln(a) in FP64 for normal a > 0 to about 1e-14 absolute: the reduction of
// log_fast with the series summed to s^19 (the next term is below 1e-16).
// The rate's derivatives for the adjoint take difference quotients over
// in-cell optical depths down to 1e-4 of the entry one, which multiply an
// error of the table position by up to 1e4: log_fast's 2e-11 would reach
// 1e-5 in the gradients.
__host__ __device__ __forceinline__ double log_f64(double a)
{
    int e;
    double m = frexp(a, &e);
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) * rcp_f64(m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 19.0;
    p = p * s2 + 1.0 / 17.0;
    p = p * s2 + 1.0 / 15.0;
    p = p * s2 + 1.0 / 13.0;
    p = p * s2 + 1.0 / 11.0;
    p = p * s2 + 1.0 / 9.0;
    p = p * s2 + 1.0 / 7.0;
    p = p * s2 + 1.0 / 5.0;
    p = p * s2 + 1.0 / 3.0;
    p = p * s2 + 1.0;
    return 2.0 * s * p + (double)e * 0.69314718055994530942;
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
    double h64;     // h
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
// tau_lo <= a and a + dt <= tau_hi.  The difference is formed in log space,
// P(a) expm1(delta ln P), so that it keeps full relative accuracy when dt is
// small against a; delta ln P is the exact difference of the cubic when both
// ends share a node interval, the sum over the two pieces when they sit in
// neighbouring intervals, and node values plus end corrections otherwise.
__host__ __device__ __forceinline__ float divdiff_spline(const TabNode *T, const TabParams &tp, double a,
                                                         double dt)
{
    const double xa = log_fast(a);
    const double ta = (xa - tp.x_lo) * tp.inv_h;
    int ja = (int)floor(ta);
    ja = ja < 0 ? 0 : (ja > tp.n - 2 ? tp.n - 2 : ja);
    const float fa = (float)(ta - (double)ja);
    const Cubic ca = cubic_at(T, ja, tp.h);
    const float corr_a = cubic_val(ca, fa);
    const float Pa = T[ja].P * exp_small(corr_a);
    const float u = (float)dt * rcp_nr((float)a);
    float dy;
    if (u < 1e-3f) {
        if (!(u > 1e-12f)) {
            // zero-width interval: the slope of the interpolant at a
            const float yx = cubic_dd(ca, fa, fa) * tp.inv_hf;
            return Pa * yx * rcp_nr((float)a);
        }
        // ln(1+u) to u^4 (error below u^5/5 < 2e-16): both ends in one or two intervals
        const float dx = u * (1.f - u * (0.5f - u * (1.f / 3.f - u * 0.25f)));
        const float dtn = dx * tp.inv_hf;
        const float tb = fa + dtn;
        if (tb <= 1.f || ja == tp.n - 2) {
            dy = dtn * cubic_dd(ca, fa, fminf(tb, 1.f));
        } else {
            const float d1 = 1.f - fa;
            const float d2 = dtn - d1;
            const Cubic cb = cubic_at(T, ja + 1, tp.h);
            dy = d1 * cubic_dd(ca, fa, 1.f) + d2 * cubic_dd(cb, 0.f, d2);
        }
    } else {
        const double tbb = (log_fast(a + dt) - tp.x_lo) * tp.inv_h;
        int jb = (int)floor(tbb);
        jb = jb < 0 ? 0 : (jb > tp.n - 2 ? tp.n - 2 : jb);
        const float fb = (float)(tbb - (double)jb);
        if (jb == ja) {
            dy = (float)(tbb - ta) * cubic_dd(ca, fa, fb);
        } else if (jb == ja + 1) {
            const Cubic cb = cubic_at(T, jb, tp.h);
            dy = (1.f - fa) * cubic_dd(ca, fa, 1.f) + fb * cubic_dd(cb, 0.f, fb);
        } else {
            const Cubic cb = cubic_at(T, jb, tp.h);
            dy = (float)(T[jb].y - T[ja].y) + (cubic_val(cb, fb) - corr_a);
        }
    }
    return Pa * expm1_fast(dy) * rcp_nr((float)dt);
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
    return (float)(-((double)tp.dP0 * lenL + DH * lenH) * rcp_f64(dt));
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
    const double *m64;     // FP64 node slopes (adjoint only; may be NULL in the forward)
    TabParams tp;
    const double *ring;    // [4][ring_cap] exit columns of shells q-1..q-3
    const int *rowbase;    // [4][row_cap]
    int ring_cap, row_cap;
    const double *nHI;     // n_H x_HI, exact product of the FP32 inputs
};

struct CellOut {
    uint32_t cp;    // global cell index (N^3 < 2^32)
    double Nin, Nout;
    double dN;      // in-cell column
    int r2;         // squared distance to the source (cells)
    double G;       // rate contribution (0 if none; only with the rate evaluated)
    bool owned;
};

// The short-characteristics update of the cell with compact index g in shell
// q (row `row` of the shell's row table, base rb = rowbase of that row):
// interpolate the entry column from the neighbours (eq. raga, eq. interp),
// add the in-cell column (Section 3.1) and form the rate (eq. sugg).
template <bool kRate = true>
__host__ __device__ __forceinline__ void cell_update(const CellCtx &X, int q, int g, int row,
                                                     int rb, CellOut &out)
{
    // octant slot and first coordinate of the row (single-octant pieces: row = A)
    const int os = X.pc.n_oct == 1 ? 0 : (int)(((float)row + 0.5f) * rcp_approx((float)(q + 1)));
    const int cA = row - os * (q + 1);
    const int cB = g - rb;
    const int cC = q - cA - cB;
    const int o = X.pc.kind == 0 ? os : X.pc.oct;
    const int di = (o & 1) ? -cA : cA;
    const int dj = (o & 2) ? -cB : cB;
    const int dk = (o & 4) ? -cC : cC;
    const int N = X.N;
    const uint32_t cp = ((uint32_t)wrap(X.si + di, N) * (uint32_t)N + (uint32_t)wrap(X.sj + dj, N)) *
                            (uint32_t)N + (uint32_t)wrap(X.sk + dk, N);
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
    const double ds = sqrt_fast((double)r2) * inv_m;
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
    if (kRate && owned) {
        const double ta = X.sigma0 * Nin;
        if (ta < X.tp.tau_hi) {
            const float nd = neg_divdiff(X.tab, X.tp, ta, X.sigma0 * dN);
            if (nd > 0.f) G = X.coef * (double)(nd * rcp_approx((float)r2));
        }
    }
    out.cp = cp;
    out.Nin = Nin;
    out.Nout = Nout;
    out.dN = dN;
    out.r2 = r2;
    out.G = G;
    out.owned = owned;
}

// --------------------------------------------------------------------------
// FP64 evaluation of the interpolant and of the rate's partial derivatives,
// for the adjoint.
// --------------------------------------------------------------------------

// e^x in FP64 (relative error ~2e-16): x = k ln2 + r, |r| <= ln2/2, Taylor to r^13.
__host__ __device__ __forceinline__ double exp_f64(double x)
{
    if (x < -745.0) return 0.0;
    const double k = rint(x * 1.4426950408889634);
    const double r = (x - k * 0.69314718055994529) - k * 2.3190468138462996e-17;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

// P(tau), dP/dtau and d2P/dtau2 of the interpolant in FP64 (node slopes m64
// in FP64: gradients can be sums of large terms of both signs), given
// x = ln tau (used only inside the table).
__host__ __device__ __forceinline__ void tab_eval64_x(const TabNode *T, const double *m64,
                                                      const TabParams &tp, double tau, double x, double *P,
                                                      double *d1, double *d2)
{
    if (tau < tp.tau_lo) {
        *P = exp_f64(T[0].y) + (double)tp.dP0 * (tau - tp.tau_lo);
        *d1 = (double)tp.dP0;
        *d2 = 0.0;
        return;
    }
    if (tau >= tp.tau_hi) {
        *P = exp_f64(T[tp.n - 1].y);
        *d1 = 0.0;
        *d2 = 0.0;
        return;
    }
    const double t = (x - tp.x_lo) * tp.inv_h;
    int j = (int)floor(t);
    j = j < 0 ? 0 : (j > tp.n - 2 ? tp.n - 2 : j);
    const double f = t - (double)j;
    const double h = tp.h64;
    const double d = T[j + 1].y - T[j].y;
    const double hm0 = h * m64[j], hm1 = h * m64[j + 1];
    const double c1 = hm0, c2 = 3.0 * d - 2.0 * hm0 - hm1, c3 = -2.0 * d + hm0 + hm1;
    const double y = T[j].y + f * (c1 + f * (c2 + f * c3));
    const double yx = (c1 + f * (2.0 * c2 + 3.0 * f * c3)) * tp.inv_h;
    const double yxx = (2.0 * c2 + 6.0 * f * c3) * tp.inv_h * tp.inv_h;
    const double p = exp_f64(y);
    const double it = rcp_f64(tau);   // tau in [tau_lo, tau_hi): FP32 normal range
    *P = p;
    *d1 = p * yx * it;
    *d2 = p * (yx * yx + yxx - yx) * it * it;
}

__host__ __device__ __forceinline__ void tab_eval64(const TabNode *T, const double *m64,
                                                    const TabParams &tp, double tau, double *P,
                                                    double *d1, double *d2)
{
    tab_eval64_x(T, m64, tp, tau, tau >= tp.tau_lo ? log_f64(tau) : 0.0, P, d1, d2);
}

// ln(1 + e) for |e| <= 1e-4 to 3e-17 absolute (the series to e^3).
__host__ __device__ __forceinline__ double log1p_small(double e)
{
    return e * (1.0 + e * (-0.5 + e * (1.0 / 3.0)));
}

// D = [P(a+dt) - P(a)] / dt and its partial derivatives dD/da (dt fixed) and
// dD/d(dt) (a fixed), FP64.  For dt > 1e-4 a the difference quotients are
// formed directly (their FP64 cancellation costs at most ~1e-8); below that
// the integral forms dD/da = mean of P'' over [a, a+dt] and
// dD/d(dt) = (1/dt^2) int_0^dt t P''(a+t) dt are taken with two-point Gauss
// rules (error O((dt/a)^4)).
__host__ __device__ __forceinline__ void rate_derivs64(const TabNode *T, const double *m64,
                                                       const TabParams &tp, double a, double dt,
                                                       double *D, double *dDda, double *dDddt)
{
    const bool in = a >= tp.tau_lo;   // then a > 0
    const double xa = in ? log_f64(a) : 0.0;
    double Pa, Pa1, Pa2;
    tab_eval64_x(T, m64, tp, a, xa, &Pa, &Pa1, &Pa2);
    if (dt > 1e-4 * a && dt > 0.0) {
        double Pb, Pb1, Pb2;
        tab_eval64(T, m64, tp, a + dt, &Pb, &Pb1, &Pb2);
        const double idt = dt > 1e-30 ? rcp_f64(dt) : 1.0 / dt;
        const double d = (Pb - Pa) * idt;
        *D = d;
        *dDda = (Pb1 - Pa1) * idt;
        *dDddt = (Pb1 - d) * idt;
        return;
    }
    // Gauss-Legendre (mean of P'') and Gauss-Jacobi for the weight t (second)
    const double g1 = 0.21132486540518711, g2 = 0.78867513459481289;
    const double j1 = 0.35505102572168219, j2 = 0.84494897427831781;   // (6 -+ sqrt6)/10
    const double w1 = (9.0 + 2.449489742783178) / 36.0, w2 = (9.0 - 2.449489742783178) / 36.0;
    // the nodes lie within a relative 1e-4 of a: inside the table their
    // logarithms are ln a + ln(1 + g dt / a) (a node can enter the table only
    // from an a just below its start: it takes its own logarithm)
    const double ea = in ? dt * rcp_f64(a) : 0.0;
    auto d2_at = [&](double g) {
        double P_, d1_, d2_;
        if (in) tab_eval64_x(T, m64, tp, a + g * dt, xa + log1p_small(g * ea), &P_, &d1_, &d2_);
        else tab_eval64(T, m64, tp, a + g * dt, &P_, &d1_, &d2_);
        return d2_;
    };
    const double q1 = d2_at(g1), q2 = d2_at(g2), r1 = d2_at(j1), r2 = d2_at(j2);
    *dDda = 0.5 * (q1 + q2);
    *dDddt = w1 * r1 + w2 * r2;
    *D = Pa1 + 0.5 * dt * (*dDda);
}

// Reverse-mode update of one cell (not the source).  Given the total adjoint
// of its exit column from its consumers (Nbar_out), its in-cell column dN as
// the forward computed it, and dL/dGamma of the cell (gbar, owned cells
// only), it recomputes the forward quantities from the
// neighbour columns in the ring and returns the adjoints to push to the
// neighbours (their exit columns; a neighbour that is the source pushes to
// n_HI of the source), the adjoint of the cell's n_HI and of the source rate.
struct CellAdj {
    uint32_t cp;
    int slot[4];            // ring slot of neighbour e_n in shell qn[n]; -1 the source, -2 unused
    int qn[4];              // neighbour shells
    double Mbar[4];         // adjoint pushed to each neighbour's exit column
    double nbar_src;        // pushed to n_HI of the source
    double nbar;            // dL/dn_HI of this cell
    double qbar;            // dL/dQ of the source (times Q: Gbar * Gamma)
};

__host__ __device__ __forceinline__ void cell_adjoint(const CellCtx &X, int q, int g, int row, int rb,
                                                      double Nbar_out, double dN,
                                                      const double *gbar_grid, CellAdj &out)
{
    const int os = X.pc.n_oct == 1 ? 0 : (int)(((float)row + 0.5f) * rcp_approx((float)(q + 1)));
    const int cA = row - os * (q + 1);
    const int cB = g - rb;
    const int cC = q - cA - cB;
    const int o = X.pc.kind == 0 ? os : X.pc.oct;
    const int di = (o & 1) ? -cA : cA;
    const int dj = (o & 2) ? -cB : cB;
    const int dk = (o & 4) ? -cC : cC;
    const int N = X.N;
    const uint32_t cp = ((uint32_t)wrap(X.si + di, N) * (uint32_t)N + (uint32_t)wrap(X.sj + dj, N)) *
                            (uint32_t)N + (uint32_t)wrap(X.sk + dk, N);
    const int m = cA > cB ? (cA > cC ? cA : cC) : (cB > cC ? cB : cC);
    const int canon = cC == m ? 2 : (cB == m ? 1 : 0);
    const int dd = X.pc.dom >= 0 ? X.pc.dom : canon;
    const int cu = dd == 0 ? cB : cA;
    const int cv = dd == 2 ? cB : cC;
    const double inv_m = rcp_f64((double)m);
    const double a = cu == m ? 1.0 : (double)cu * inv_m;
    const double b = cv == m ? 1.0 : (double)cv * inv_m;
    const int r2 = cA * cA + cB * cB + cC * cC;
    const double ds = sqrt_fast((double)r2) * inv_m;
    const double sw[4] = {(1.0 - a) * (1.0 - b), a * (1.0 - b), (1.0 - a) * b, a * b};

    double Mv[4], wv[4], dw[4];
    int nslot[4], nq[4];
    double num = 0.0, W = 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        Mv[n] = 0.0;
        wv[n] = 0.0;
        dw[n] = 0.0;
        nslot[n] = -2;
        nq[n] = 0;
        if (!(sw[n] > 0.0)) continue;
        const int su = n & 1, sv = (n >> 1) & 1;
        const int eA = cA - (dd == 0 ? 1 : 0) - (su & (dd != 0 ? 1 : 0));
        const int eB = cB - (dd == 1 ? 1 : 0) - (su & (dd == 0 ? 1 : 0)) - (sv & (dd == 2 ? 1 : 0));
        const int eC = cC - (dd == 2 ? 1 : 0) - (sv & (dd != 2 ? 1 : 0));
        const int qn = q - 1 - su - sv;
        double M;
        if (qn == 0) {
            M = X.reading == 0 ? X.half_col * ds : X.half_col;
            nslot[n] = -1;
        } else {
            int o2 = o;
            if (X.pc.kind == 0) {
                if ((o2 & 1) && eA == 0) o2 &= ~1;
                if ((o2 & 2) && eB == 0) o2 &= ~2;
                if ((o2 & 4) && eC == 0) o2 &= ~4;
            }
            const int ord = X.pc.kind == 0 ? o2 : 0;
            const int sl = qn & 3;
            const int nrow = ord * (qn + 1) + eA;
            nslot[n] = X.rowbase[sl * X.row_cap + nrow] + eB;
            M = X.ring[sl * X.ring_cap + nslot[n]];
        }
        nq[n] = qn;
        double wn = sw[n];
        if (X.tau_w > 0.f) {
            const double tau = X.sigma0 * M;
            if (tau > (double)X.tau_w) {
                const double it = 1.0 / tau;
                wn *= it;
                dw[n] = -sw[n] * X.sigma0 * it * it;
            } else {
                wn *= 1.0 / (double)X.tau_w;
            }
        }
        Mv[n] = M;
        wv[n] = wn;
        num += wn * M;
        W += wn;
    }
    const double iW = 1.0 / W;
    const double Nin = num * iW;

    // ownership as in the forward
    bool owned = true;
    if (X.pc.kind == 1) {
        if (((o & 1) && cA == 0) || ((o & 2) && cB == 0) || ((o & 4) && cC == 0)) owned = false;
        if (X.pc.dom >= 0 && canon != X.pc.dom) owned = false;
    }
    // N_out = N_in + dN: both receive Nbar_out; the rate adds its own parts
    double Nin_bar = Nbar_out, dN_bar = Nbar_out, qb = 0.0;
    const double ta = X.sigma0 * Nin;
    // dL/dGamma is read only where the rate can be non-zero
    const double gbar = (owned && ta < X.tp.tau_hi) ? gbar_grid[cp] : 0.0;
    if (gbar != 0.0) {
        double D, Da, Ddt;
        rate_derivs64(X.tab, X.m64, X.tp, ta, X.sigma0 * dN, &D, &Da, &Ddt);
        const double k = -X.coef / (double)r2;          // Gamma = k D
        Nin_bar += gbar * k * Da * X.sigma0;
        dN_bar += gbar * k * Ddt * X.sigma0;
        qb = gbar * k * D;                              // = gbar Gamma
    }
    out.cp = cp;
    out.nbar = dN_bar * X.alpha * ds;                   // dN = n_HI alpha ds
    out.qbar = qb;
    out.nbar_src = 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const double dNin_dM = (wv[n] + (Mv[n] - Nin) * dw[n]) * iW;
        const double mb = nslot[n] == -2 ? 0.0 : Nin_bar * dNin_dM;
        if (nslot[n] == -1) out.nbar_src += mb * (X.reading == 0 ? X.alpha * ds * 0.5 : X.alpha * 0.5);
        out.slot[n] = nslot[n];
        out.qn[n] = nq[n];
        out.Mbar[n] = mb;
    }
}

// Adjoint of the source cell's own rate: d Gamma_s / d n_HI(s) and Gamma_s.
__host__ __device__ __forceinline__ void source_cell_adjoint(const TabNode *T, const double *m64,
                                                             const TabParams &tp, double sigma0,
                                                             double alpha, double Q, double n_s,
                                                             double gbar, double *nbar, double *qbar)
{
    const double tau_s = sigma0 * n_s * alpha * 0.5;
    double D, Da, Ddt;
    rate_derivs64(T, m64, tp, 0.0, tau_s, &D, &Da, &Ddt);
    const double k = -Q * sigma0 / (2.0 * alpha * alpha);
    *nbar = gbar * k * Ddt * sigma0 * alpha * 0.5;
    *qbar = gbar * k * D;
}

// Rate of the source cell itself: entry column 0, path half a cell, volume
// alpha^3.
__host__ __device__ __forceinline__ double source_cell_rate(const TabNode *T, const TabParams &tp,
                                                            double sigma0, double alpha, double Q,
                                                            double n_s)
{
    const double tau_s = sigma0 * n_s * alpha * 0.5;
    const float nd = neg_divdiff(T, tp, 0.0, tau_s);
    return Q * sigma0 / (2.0 * alpha * alpha) * (double)nd;   // once per source
}

// --------------------------------------------------------------------------
// Layer pieces.  Within one octant, the cells of a source whose dominant axis
// (largest |d|, ties included) is d form a pyramid; every non-zero-weight
// neighbour of such a cell lies in the same pyramid, one step closer along d
// (the neighbour set of Section 3.1, eq. 11).  The pyramid can therefore be
// swept layer by layer, m = |d_d| = 1, 2, ...: a cell of layer m reads only
// layer m - 1.  In layer m a cell is (u, v) = (|d_u|, |d_v|) in [0, m]^2, for
// the two other axes u, v.  v is the axis that is contiguous in memory: k
// for d = i or j in the field layout [i][j][k]; j for d = k, which reads and
// accumulates in a transposed copy laid out [k][i][j].  A wave's cells are
// then runs of neighbouring addresses, so its gathers and atomics coalesce.
// Pieces are numbered p = 3 * octant + d, octant bits as for Piece.
// --------------------------------------------------------------------------
struct LayerPiece {
    int d, au, av;             // dominant axis and the (u, v) axes (0 = i, 1 = j, 2 = k)
    int oct;                   // octant bits: 1 = i negative, 2 = j negative, 4 = k negative
    // ownership: a cell with u = 0 (v = 0) on a negative axis belongs to the
    // neighbouring octant (neg_u, neg_v); a cell tied with u (v) for the
    // largest offset belongs to the pyramid of the first tied axis in the
    // order k, j, i (tie_u, tie_v: that is not this pyramid)
    bool neg_u, neg_v, tie_u, tie_v;
    int sd, su, sv;            // +1 / -1: direction of the offsets along d, u, v
    int ext_d, ext_u, ext_v;   // periodic extents in those directions
    int c_d, c_u, c_v;         // source coordinates along d, u, v
    uint32_t st_d, st_u;       // memory strides of d and u (v has stride 1)
    bool transposed;           // the piece uses the [k][i][j] copies
};

__host__ __device__ __forceinline__ int axis_sign(int oct, int ax) { return ((oct >> ax) & 1) ? -1 : 1; }

__host__ __device__ inline LayerPiece make_layer_piece(int p, int si, int sj, int sk, int N,
                                                       const Extent &ex)
{
    LayerPiece L;
    L.oct = p / 3;
    L.d = p % 3;
    L.au = L.d == 0 ? 1 : 0;
    L.av = L.d == 2 ? 1 : 2;
    L.transposed = L.d == 2;
    L.sd = axis_sign(L.oct, L.d);
    L.su = axis_sign(L.oct, L.au);
    L.sv = axis_sign(L.oct, L.av);
    L.neg_u = L.su < 0;
    L.neg_v = L.sv < 0;
    L.tie_u = L.d == 0;   // u is j: j comes before i
    L.tie_v = L.d != 2;   // v is k (d = i, j): k comes first
    L.ext_d = L.sd < 0 ? ex.neg : ex.pos;
    L.ext_u = L.su < 0 ? ex.neg : ex.pos;
    L.ext_v = L.sv < 0 ? ex.neg : ex.pos;
    // (selects rather than indexed arrays: no private memory on the GPU)
    L.c_d = L.d == 0 ? si : (L.d == 1 ? sj : sk);
    L.c_u = L.au == 0 ? si : sj;
    L.c_v = L.av == 1 ? sj : sk;
    const uint32_t n = (uint32_t)N;
    // standard [i][j][k]: strides N^2, N, 1; transposed [k][i][j]: i N, j 1, k N^2
    if (L.transposed) {          // d = k, u = i, v = j
        L.st_d = n * n;
        L.st_u = n;
    } else if (L.d == 0) {       // u = j, v = k
        L.st_d = n * n;
        L.st_u = n;
    } else {                     // d = j, u = i, v = k
        L.st_d = n;
        L.st_u = n * n;
    }
    return L;
}

// Largest r with r * r <= x (0 <= x < 2^24).
__host__ __device__ __forceinline__ int isqrt_floor(int x)
{
    int r = (int)sqrtf((float)x);
    if (r * r > x) --r;
    else if ((r + 1) * (r + 1) <= x) ++r;
    return r;
}

// Layer m of a pyramid enumerated as a rectangle: rows u = 0..nu-1 of wv
// cells v = 0..wv-1, cell g = u * wv + v (row-major, so increasing g is
// increasing (u, v) in lexicographic order).  The rectangle is the bounding
// box of the layer's cells inside the ball (u^2 + v^2 <= rem) and the
// periodic extent; the cells outside the ball are inactive.
struct LayerRect {
    int rem;      // Rsq - m^2
    int nu, wv;   // rows, row width
    int total;    // nu * wv
};

__host__ __device__ __forceinline__ LayerRect layer_rect(int ext_u, int ext_v, int Rsq, int m)
{
    LayerRect r;
    r.rem = Rsq - m * m;
    const int s = isqrt_floor(r.rem);
    const int cu = m < ext_u ? m : ext_u, cv = m < ext_v ? m : ext_v;
    r.nu = (cu < s ? cu : s) + 1;
    r.wv = (cv < s ? cv : s) + 1;
    r.total = r.nu * r.wv;
    return r;
}

// (u, v) of cell g of the rectangle; true if the cell is active.
__host__ __device__ __forceinline__ bool rect_cell(const LayerRect &r, int g, int &u, int &v)
{
    int q = (int)((float)g * rcp_approx((float)r.wv));   // off by at most one (g < 2^24)
    if (q * r.wv > g) --q;
    else if ((q + 1) * r.wv <= g) ++q;
    u = q;
    v = g - q * r.wv;
    return g < r.total && u * u + v * v <= r.rem;
}

// Side of the layer buffer of pyramids of squared radius up to Rsq: a cell
// (u, v) of layer m has u, v <= m and u^2 + v^2 + m^2 <= Rsq, hence
// u^2, v^2 <= Rsq / 2 (and u, v within the extent), so an S x S buffer with
// S = floor(sqrt(Rsq / 2)) + 1 holds every layer.
__host__ __device__ inline int layer_buffer_side(int Rsq, const Extent &ex)
{
    const int s = isqrt_floor(Rsq / 2);
    return (s < ex.neg ? s : ex.neg) + 1;
}

// Cells of the largest pyramid of a source of squared radius Rsq, counted as
// layer rectangles (an upper bound for every octant and axis: the negative
// extent is the larger one).
__host__ __device__ inline long layer_piece_capacity(int Rsq, const Extent &ex)
{
    const int r = isqrt_floor(Rsq);
    const int Mx = r < ex.neg ? r : ex.neg;
    long cap = 0;
    for (int m = 1; m <= Mx; ++m) cap += layer_rect(ex.neg, ex.neg, Rsq, m).total;
    return cap;
}

// Column record of one pyramid (a piece of layer kind) in global memory: the
// exit column of every cell as its layer-buffer entry (layer_entry), layer by
// layer in rectangle order, and for every chunk of 64 cells (layers in
// order, chunks of a layer in order) the mask of its cells that carry a rate
// (owned, entry optical depth inside the table).  Written by the forward
// sweep when the columns are kept, or by the adjoint's own forward pass; read
// by the adjoint's reverse pass.  `cap` bounds the cells of one pyramid.
// A record kept by the forward also holds, for the cells with a rate in the
// order the forward evaluated them, the rate's coefficients for the adjoint
// (layer_rate_coefs) in three arrays of cap entries, followed by the number
// of such cells and the last layer the adjoint has to visit (layer_opaque):
// entries and masks of later layers are not written.
struct LayerRecord {
    double *h;        // [cap] layer-buffer entries of the cells
    uint64_t *lit;    // [cap / 64 + Mcap + 1] rate masks, one per chunk
    double *rk;       // kept records: [3][cap] rate coefficients, then the count; else NULL
};

// Bytes of a record of cap cells, with (coefs) or without the rate
// coefficients; the coefficients start at layer_record_bytes(cap, Mcap, false).
__host__ __device__ __forceinline__ size_t layer_record_bytes(long cap, int Mcap, bool coefs)
{
    size_t b = (size_t)cap * sizeof(double) + ((size_t)cap / 64 + Mcap + 1) * sizeof(uint64_t);
    b = (b + 255) & ~(size_t)255;
    if (coefs) b += ((3 * (size_t)cap + 2) * sizeof(double) + 255) & ~(size_t)255;
    return b;
}

// rk_off: layer_record_bytes(cap, Mcap, false) for a record with the
// coefficients, 0 for one without.
__host__ __device__ __forceinline__ LayerRecord layer_record_at(char *base, long cap, size_t rk_off)
{
    LayerRecord s;
    s.h = (double *)base;
    s.lit = (uint64_t *)(s.h + cap);
    s.rk = rk_off ? (double *)(base + rk_off) : nullptr;
    return s;
}

// Everything one layer-cell update needs that is uniform over a piece.
struct LayerX {
    int N;
    int reading;           // 0: directional source half path, 1: scalar
    float tau_w;           // <= 0: geometric weights
    double sigma0, alpha;
    double half_col;       // n_HI(s) alpha / 2
    const double *nHI;     // n_HI in the piece's layout
    double inv_s0;         // 1 / sigma0
    double inv_tw;         // 1 / tau_w, or 1 with geometric weights
};

__host__ __device__ __forceinline__ void layer_x_weights(LayerX &X)
{
    X.inv_s0 = 1.0 / X.sigma0;
    X.inv_tw = X.tau_w > 0.f ? 1.0 / (double)X.tau_w : 1.0;
}

// 24-bit unsigned product (operands below 2^24): a full-rate instruction on
// the GPU, where a 32-bit integer product is a quarter-rate one.
__host__ __device__ __forceinline__ int mul24(int a, int b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return (int)__umul24((unsigned)a, (unsigned)b);
#else
    return a * b;
#endif
}

// The layer buffer holds, for every cell of the previous layer, what its
// consumers need of its exit column M for the optical-depth weights
// w = s / max(sigma0 M, tau_w): the factor f = 1 / max(sigma0 M, tau_w) and the
// product g = f M.  A cell with sigma0 M > tau_w stores h = 1 / (sigma0 M) > 0
// (then f = h, g = 1 / sigma0); any other cell stores h = -M (then
// f = 1 / tau_w, g = M / tau_w).  With geometric weights every cell stores -M
// (f = 1, g = M).  One reciprocal per cell instead of one per neighbour.
__host__ __device__ __forceinline__ double layer_entry(const LayerX &X, double M)
{
    const double t = X.sigma0 * M;
    return (X.tau_w > 0.f && t > (double)X.tau_w) ? rcp_f64(t) : -M;
}

// A layer whose every cell leaves with sigma0 N_out >= layer_opaque(tau_hi)
// ends the pyramid's cells with a rate: a cell's entry column is a convex
// combination of its neighbours' exit columns (weights s / max(sigma0 M,
// tau_w) >= 0) and its exit column adds dN >= 0, so every later cell enters
// with sigma0 N_in >= tau_hi (the margin covers the rounding of tens of
// layers), has no rate, and receives no adjoint.  The forward still sweeps
// those cells; the adjoint need not.
__host__ __device__ __forceinline__ double layer_opaque(double tau_hi)
{
    return tau_hi * (1.0 + 1e-12);
}

struct LayerCell {
    uint32_t cp;    // cell index in the piece's layout
    double Nin, Nout, dN;
    double h;       // layer-buffer entry of the cell (layer_entry of Nout)
    int r2;
    bool owned;
};

// Walks the cells of a layer rectangle 64 at a time: every lane holds cell
// g = c * 64 + lane of chunk c, and down() / up() move all lanes to chunk
// c - 1 / c + 1 without a division (64 = q64 * wv + r64).
struct RectWalk {
    int u, v, wv, q64, r64;
    __host__ __device__ __forceinline__ void init(const LayerRect &r, int g)
    {
        wv = r.wv;
        q64 = 64 / wv;
        r64 = 64 - q64 * wv;
        int q = (int)((float)g * rcp_approx((float)wv));   // off by at most one (g < 2^24)
        if (mul24(q, wv) > g) --q;
        else if (mul24(q + 1, wv) <= g) ++q;
        u = q;
        v = g - mul24(q, wv);
    }
    __host__ __device__ __forceinline__ void down()
    {
        const bool b = v < r64;
        u -= q64 + (b ? 1 : 0);
        v += b ? wv - r64 : -r64;
    }
    __host__ __device__ __forceinline__ void up()
    {
        v += r64;
        const bool c = v >= wv;
        u += q64 + (c ? 1 : 0);
        v -= c ? wv : 0;
    }
};

// Index of layer cell (u, v) of layer m in the piece's field layout, as the
// sum of one term per axis: layer_idx_d(m) + layer_idx_u(u) + layer_idx_v(v)
// (a sweep keeps the u and v terms of its pyramid in per-wave tables).
// Strides are N or N^2 (< 2^22); the N^2 stride is applied with a full product.
__host__ __device__ __forceinline__ uint32_t layer_idx_d(const LayerPiece &L, int N, int m)
{
    return (uint32_t)wrap(L.c_d + L.sd * m, N) * L.st_d;
}

__host__ __device__ __forceinline__ uint32_t layer_idx_u(const LayerPiece &L, int N, int u)
{
    return (uint32_t)wrap(L.c_u + L.su * u, N) * L.st_u;
}

__host__ __device__ __forceinline__ uint32_t layer_idx_v(const LayerPiece &L, int N, int v)
{
    return (uint32_t)wrap(L.c_v + L.sv * v, N);
}

__host__ __device__ __forceinline__ uint32_t layer_cp(const LayerPiece &L, int N, int m, int u, int v)
{
    return layer_idx_d(L, N, m) + layer_idx_u(L, N, u) + layer_idx_v(L, N, v);
}

// Largest number of spectral bands of the two-absorber sweep.
constexpr int kMaxBands = 8;

// Largest r^2 with an entry in a sweep's table of square roots (r^2 up to the
// squared radius of the call); beyond it the root is computed per cell.
constexpr int kSqrtTable = 4096;

// Bytes of a layer sweep's table of square roots (sqrt of every r^2 up to
// the squared radius Rsq of the call), or 0 when it would exceed kSqrtTable
// entries (the roots are then computed per cell).
__host__ __device__ inline size_t layer_sqrt_bytes(int Rsq)
{
    return Rsq < kSqrtTable ? (((size_t)(Rsq + 1) * sizeof(double) + 15) & ~(size_t)15) : 0;
}

// The layer buffer of a sweep: (S + 1) x (S + 1) doubles, cell (u, v) at
// slot (u + 1)(S + 1) + v + 1.  Row 0 and column 0 stay zero: a cell on a
// zero plane (u = 0 or v = 0) reads its neighbours (u - 1, .) or (., v - 1),
// whose weights vanish, from those finite slots, so the four reads need no
// clamp and come in two adjacent pairs.
__host__ __device__ __forceinline__ int layer_slot(int u, int v, int P)
{
    return mul24(u + 1, P) + v + 1;
}

// Bilinear factors of an offset u (or v) of layer m: (1 - a, a), a = u / m.
// a = 1 exactly at u = m: the weights of neighbours that leave the pyramid
// then vanish exactly.  A sweep keeps them for u = 0 .. S - 1 in a per-layer
// table.
struct Geo {
    double om, a;
};

__host__ __device__ __forceinline__ Geo layer_geo(int m, double inv_m, int u)
{
    Geo g;
    g.a = u == m ? 1.0 : (double)u * inv_m;
    g.om = 1.0 - g.a;
    return g;
}

// The short-characteristics update of cell (u, v) of layer m of a pyramid
// (eqs. 9-12): entry column interpolated from the layer-buffer entries
// (layer_entry) h0 .. h3 of its four neighbours in layer m - 1, (u, v),
// (u - 1, v), (u, v - 1), (u - 1, v - 1), with bilinear geometric weights
// from gu = layer_geo(u), gv = layer_geo(v) times the optical-depth factors
// (for m = 1 the only neighbour of non-zero weight is the source, whose
// column the cell sees directly); in-cell column n_HI alpha ds with
// ds = r / m; ownership.  The weights must be finite wherever they are zero.
__host__ __device__ __forceinline__ void layer_cell_core(const LayerPiece &L, const LayerX &X, int m, int u,
                                                         int v, const Geo &gu, const Geo &gv, double ds, int r2,
                                                         uint32_t cp, double nhi, double h0, double h1,
                                                         double h2, double h3, LayerCell &out)
{
    double Nin;
    if (m == 1) {
        Nin = X.reading == 0 ? X.half_col * ds : X.half_col;
    } else {
        const double h[4] = {h0, h1, h2, h3};
        const double sw[4] = {gu.om * gv.om, gu.a * gv.om, gu.om * gv.a, gu.a * gv.a};
        double num = 0.0, W = 0.0;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const bool thick = h[n] > 0.0;
            const double f = thick ? h[n] : X.inv_tw;
            const double g = thick ? X.inv_s0 : -h[n] * X.inv_tw;
            num += sw[n] * g;
            W += sw[n] * f;
        }
        Nin = num * rcp_f64(W);
    }
    const double dN = nhi * X.alpha * ds;
    out.cp = cp;
    out.Nin = Nin;
    out.Nout = Nin + dN;
    out.h = layer_entry(X, out.Nout);
    out.dN = dN;
    out.r2 = r2;
    out.owned = !(L.neg_u && u == 0) && !(L.neg_v && v == 0) && !(L.tie_u && u == m) && !(L.tie_v && v == m);
}

// The same update from the padded layer buffer lay (row stride P = S + 1) of
// layer m - 1, with the geometry computed in place: the reference form of
// what the sweep kernels do with their per-layer tables.
__host__ __device__ __forceinline__ void layer_cell(const LayerPiece &L, const LayerX &X, int m, int u, int v,
                                                    const double *lay, int P, LayerCell &out)
{
    const uint32_t cp = layer_cp(L, X.N, m, u, v);
    const double inv_m = rcp_f64((double)m);
    const int r2 = mul24(m, m) + mul24(u, u) + mul24(v, v);
    const int pos = layer_slot(u, v, P);
    layer_cell_core(L, X, m, u, v, layer_geo(m, inv_m, u), layer_geo(m, inv_m, v),
                    sqrt_fast((double)r2) * inv_m, r2, cp, X.nHI[cp], lay[pos], lay[pos - P], lay[pos - 1],
                    lay[pos - P - 1], out);
}

// Cell (i, j, k) of layer cell (m, u, v), in the standard layout.
__host__ __device__ __forceinline__ uint32_t layer_std_index(const LayerPiece &L, int N, int m, int u,
                                                             int v)
{
    const int cd = wrap(L.c_d + L.sd * m, N), cu = wrap(L.c_u + L.su * u, N),
              cv = wrap(L.c_v + L.sv * v, N);
    const int ci = L.d == 0 ? cd : cu;                      // u is i unless d = i
    const int cj = L.d == 1 ? cd : (L.d == 0 ? cu : cv);
    const int ck = L.d == 2 ? cd : cv;                      // v is k unless d = k
    return ((uint32_t)ci * (uint32_t)N + (uint32_t)cj) * (uint32_t)N + (uint32_t)ck;
}

// The entry column of layer cell (u, v) of layer m recomputed from the
// layer-buffer entries (layer_entry) of layer m - 1, kept as Hprev[u' * wvp +
// v'] (its rectangle), with what the adjoint needs: the geometric weights s,
// the weight factors f, which neighbours are optically thick, W = sum s f
// (as 1/W) and N_in = sum s g / W.  For m = 1 the entry column is the
// source's.
// A chunk of 64 layer cells with at least this many cells with a rate has
// their rate terms evaluated in the reverse pass itself (the lanes are mostly
// busy anyway); sparser chunks have them evaluated beforehand in batches of
// 64 gathered from many chunks.
constexpr int kDenseChunk = 32;

struct LayerInterp {
    uint32_t cp;
    int r2;
    double ds, Nin, iW;
    double sw[4], f[4];
    bool thick[4];
};

// The interpolation of cell (u, v) of layer m from its four neighbours in
// layer m - 1, whose entries Hprev holds in layer m - 1's rectangle rp (for
// m = 1 the only neighbour of non-zero weight is the source: N_in is its
// column), given the cell's index cp, r2, ds and bilinear factors gu, gv
// (layer_geo).  Neighbours of zero weight may lie outside layer m - 1 and
// are not read.
__host__ __device__ __forceinline__ void layer_interp_core(const LayerX &X, int m, int u, int v, uint32_t cp,
                                                           int r2, double ds, const Geo &gu, const Geo &gv,
                                                           const double *Hprev, const LayerRect &rp,
                                                           LayerInterp &I)
{
    I.cp = cp;
    I.r2 = r2;
    I.ds = ds;
    I.sw[0] = gu.om * gv.om;
    I.sw[1] = gu.a * gv.om;
    I.sw[2] = gu.om * gv.a;
    I.sw[3] = gu.a * gv.a;
    I.iW = 1.0;
    if (m == 1) {
        I.Nin = X.reading == 0 ? X.half_col * I.ds : X.half_col;
#pragma unroll
        for (int n = 0; n < 4; ++n) { I.f[n] = 0.0; I.thick[n] = false; }
        return;
    }
    double num = 0.0, W = 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const double h = I.sw[n] > 0.0 ? Hprev[(u - (n & 1)) * rp.wv + (v - (n >> 1))] : 0.0;
        I.thick[n] = h > 0.0;
        I.f[n] = I.thick[n] ? h : X.inv_tw;
        const double g = I.thick[n] ? X.inv_s0 : -h * X.inv_tw;
        num += I.sw[n] * g;
        W += I.sw[n] * I.f[n];
    }
    I.iW = rcp_f64(W);
    I.Nin = num * I.iW;
}

// The same with the cell's geometry computed in place (the reference form of
// what the adjoint kernel does with its tables).
__host__ __device__ __forceinline__ void layer_interp(const LayerPiece &L, const LayerX &X, int m, int u, int v,
                                                      const double *Hprev, const LayerRect &rp, LayerInterp &I)
{
    const double inv_m = rcp_f64((double)m);
    const int r2 = mul24(m, m) + mul24(u, u) + mul24(v, v);
    layer_interp_core(X, m, u, v, layer_cp(L, X.N, m, u, v), r2, sqrt_fast((double)r2) * inv_m,
                      layer_geo(m, inv_m, u), layer_geo(m, inv_m, v), Hprev, rp, I);
}

// The rate's share of the adjoint of a cell with a rate (owned, entry optical
// depth inside the table): with Gamma = k D(tau_in, dtau), k = -coef / r2,
// g_in = gbar dGamma/dN_in and g_dN = gbar dGamma/d(dN) from the FP64
// derivatives of the divided difference.  Returns g_in (added to the cell's
// exit-column adjoint before the interpolation is reversed), the part of
// dL/dn_HI of the cell that the reverse does not produce,
// (g_dN - g_in) alpha ds, and gbar Gamma.  Given the cell's entry and
// in-cell optical depths ta = sigma0 N_in and dt = sigma0 dN, alpha ds (ads)
// and r2.
__host__ __device__ __forceinline__ void layer_rate_adjoint_t(const TabNode *T, const double *m64,
                                                              const TabParams &tp, double sigma0, double coef,
                                                              double ta, double dt, double ads, int r2,
                                                              double gbar, double *g_in, double *nbar_extra,
                                                              double *gG)
{
    double D, Da, Ddt;
    rate_derivs64(T, m64, tp, ta, dt, &D, &Da, &Ddt);
    const double k = -coef * rcp_f64((double)r2);
    const double gi = gbar * k * Da * sigma0;
    const double gd = gbar * k * Ddt * sigma0;
    *g_in = gi;
    *nbar_extra = (gd - gi) * ads;
    *gG = gbar * k * D;
}

__host__ __device__ __forceinline__ void layer_rate_adjoint(const TabNode *T, const double *m64,
                                                            const TabParams &tp, const LayerX &X,
                                                            double coef, const LayerInterp &I, double nhi,
                                                            double gbar, double *g_in, double *nbar_extra,
                                                            double *gG)
{
    // the same from the cell's interpolation I and n_HI, dt formed as the
    // column sweep forms it: sigma0 (n_HI alpha ds)
    layer_rate_adjoint_t(T, m64, tp, X.sigma0, coef, X.sigma0 * I.Nin, X.sigma0 * (nhi * X.alpha * I.ds),
                         X.alpha * I.ds, I.r2, gbar, g_in, nbar_extra, gG);
}

// The rate's coefficients of a cell with a rate for the adjoint, from its
// entry and in-cell optical depths (a = sigma0 N_in, dt = sigma0 dN) and r2:
// with k = -1 / r2 (the source's Q coef factored out), dGamma/dN_in =
// coef c[0], dGamma/d(dN) - dGamma/dN_in = coef c[1] and Gamma = coef c[2].
// The same FP64 derivatives as layer_rate_adjoint, taken once in the forward
// when the columns are kept, so that the adjoint only scales them by
// coef dL/dGamma.
__host__ __device__ __forceinline__ void layer_rate_coefs(const TabNode *T, const double *m64,
                                                          const TabParams &tp, double sigma0, double a,
                                                          double dt, int r2, double c[3])
{
    double D, Da, Ddt;
    rate_derivs64(T, m64, tp, a, dt, &D, &Da, &Ddt);
    const double k = -rcp_f64((double)r2);
    c[0] = k * Da * sigma0;
    c[1] = k * (Ddt - Da) * sigma0;
    c[2] = k * D;
}

// Reverse-mode update of layer cell (u, v) of layer m through the
// interpolation.  Tin is the total adjoint of the cell's entry column: what
// its consumers pushed to its exit column plus, for a cell with a rate, the
// rate's entry-column term g_in.  Since N_out = N_in + dN, the exit-column
// adjoint flows unchanged into N_in and dN, so the cell's dL/dn_HI is
// Tin alpha ds here (the rate's remaining part comes from layer_rate_adjoint).
// With N_in = sum s g / sum s f (f, g as in layer_entry),
// dN_in/dM_n = s_n sigma0 N_in f_n^2 / W for a neighbour with
// sigma0 M_n > tau_w (f_n = 1/(sigma0 M_n)) and s_n f_n / W for any other
// (f_n constant), W = sum s f: the entries alone suffice.  Returns the
// adjoints to push to the four neighbours of layer m - 1 (Mbar[n] for
// neighbour (u - (n & 1), v - (n >> 1)); zero where the weight is zero; for
// m = 1 the source takes them through nbar_src) and dL/dn_HI of the cell.
// I is the cell's layer_interp.
struct LayerRev {
    uint32_t cp;
    double Mbar[4];
    double nbar_src;
    double nbar;
};

__host__ __device__ __forceinline__ void layer_cell_reverse(const LayerX &X, int m, const LayerInterp &I,
                                                            double Tin, LayerRev &out)
{
    out.cp = I.cp;
    out.nbar = Tin * X.alpha * I.ds;                  // dN = n_HI alpha ds
    out.nbar_src = 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n) out.Mbar[n] = 0.0;
    if (m == 1) {
        out.nbar_src = Tin * (X.reading == 0 ? X.alpha * I.ds * 0.5 : X.alpha * 0.5);
        return;
    }
    const double tk = Tin * I.iW, tt = tk * X.sigma0 * I.Nin;
#pragma unroll
    for (int n = 0; n < 4; ++n) out.Mbar[n] = I.sw[n] * I.f[n] * (I.thick[n] ? tt * I.f[n] : tk);
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

#if defined(__HIPCC__)
constexpr int kRowsPerLane = 4;   // wave sweeps: rows per shell <= 64 * kRowsPerLane

// Order LDS traffic of one wave: its own writes before its later reads.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Next work item of a wave.  The items of a launch (in the spatial order of
// their sources) are split into kXcds contiguous chunks with one counter each;
// the waves of work-group b start on chunk b % kXcds, which keeps the cells
// that one die's L2 sees in a compact region of the grid, and move on to the
// following chunks once theirs is used up.  Returns nitems when no chunk has
// work left.
//
// Every lane takes part in each atomic (lane 0 adds 1, the others 0) and the
// result is lane 0's, read into a scalar register.  There is no branch on the
// lane index: with `if (lane == 0) fetch` followed by a broadcast, the compiler
// may merge that branch with a lane-0 branch at the end of the previous item
// and run lane 0 and lanes 1..63 around separate loops, so that the broadcast
// runs without lane 0 and lanes 1..63 never see the end of the work.  The
// scalar result also makes everything derived from the item wave-uniform.
__device__ __forceinline__ int next_item(int *counters, int nitems, int home, int &chunk, int lane)
{
    for (;;) {
        const int lo = (int)((long)nitems * chunk / kXcds);
        const int hi = (int)((long)nitems * (chunk + 1) / kXcds);
        const int got = atomicAdd(&counters[chunk * kCounterPad], lane == 0 ? 1 : 0);
        const int k = __builtin_amdgcn_readfirstlane(got);
        if (lo + k < hi) return lo + k;
        chunk = chunk + 1 == kXcds ? 0 : chunk + 1;
        if (chunk == home) return nitems;
    }
}

// Row table of shell q built by one wave: every lane owns up to kRowsPerLane
// consecutive rows, counts them, and a wave-wide exclusive scan gives the
// row starts.  Returns the shell's cell count (same value in every lane).
__device__ __forceinline__ int wave_build_rows(const Piece &pc, const Extent &ex, int Rsq, int q,
                                               int lane, int *rowstart, int *rowbase_q)
{
    const int nrows = pc.n_oct * (q + 1);
    const int c = (nrows + 63) >> 6;
    const int r0 = lane * c;
    int blo_k[kRowsPerLane], cnt_k[kRowsPerLane];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kRowsPerLane; ++k) {
        const int r = r0 + k;
        blo_k[k] = 0;
        cnt_k[k] = 0;
        if (k < c && r < nrows) row_range(pc, ex, Rsq, q, r, &blo_k[k], &cnt_k[k]);
        sum += cnt_k[k];
    }
    int incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    int run = incl - sum;
#pragma unroll
    for (int k = 0; k < kRowsPerLane; ++k) {
        const int r = r0 + k;
        if (k < c && r < nrows) {
            rowstart[r] = run;
            rowbase_q[r] = run - blo_k[k];
            run += cnt_k[k];
        }
    }
    const int total = __shfl(incl, 63, 64);
    if (lane == 0) rowstart[nrows] = total;
    return total;
}
#endif

}  // namespace asora
