// asora_api.hip -- the C ABI declared in include/asora.h: argument checks,
// context and scratch memory, table preparation, launch planning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/asora.h"
#include "asora_internal.h"

using namespace asora;

struct PlanKey {
    int type, Rsq;
    bool operator<(const PlanKey &o) const { return type != o.type ? type < o.type : Rsq < o.Rsq; }
};

struct Plan {
    int ring_cap, row_cap, Qmax;
    int S;              // layer pieces: side of the per-wave layer buffer
    long piece_cells;   // largest number of cells of one piece (adjoint scratch)
    long scratch;       // adjoint: doubles of scratch per wave
    int Mcap;           // layer pieces: largest layer index
    long rec_cap;       // layer pieces: cells per pyramid record
    size_t rec_bytes;   // layer pieces: bytes of one pyramid record (the adjoint's own)
    size_t keep_bytes;  // layer pieces: bytes of one record kept by the forward (with rate coefficients)
    int wave_mode;   // 1: one wave per piece (waves per work-group below); 0: one work-group per piece
    int waves;
    size_t lds;
    int grid;
    bool sq_table;      // layer pieces: the work-group holds the table of sqrt(r^2)
    // layer forward that keeps the column records (a larger rate queue)
    int kwaves, kgrid;
    bool ksq_table;
};

static const int kProfSlots = 64;

struct asora_ctx {
    int magic;
    int device;
    int N;
    double alpha, sigma0, tau_w;
    uint32_t flags;
    int reading;
    TabParams tp;
    TabNode *d_tab;
    double *d_m64;          // FP64 node slopes for the adjoint
    double lg_lo, lg_hi;    // log10 of the first and last table node
    TabNode *d_tab_h;       // photo-heating table on the same nodes (NULL until set)
    float dP0_h;            // its slope at the first node
    double *d_hacc;         // heating accumulators (allocated by the first heating forward)
    double *d_hacc_T;
    // two absorbers (asora_set_helium): band tables, cross-sections; n_HeI and
    // the HeI rate accumulator in both layouts (allocated by the first call)
    int he_nb, he_ntab;
    TabNode *d_tab_he;
    TabParams he_tp[kMaxBands];
    double he_sH[kMaxBands], he_sHe[kMaxBands];
    double *d_nhe, *d_nhe_T, *d_ghe, *d_ghe_T;
    double *d_nhi;
    double *d_gacc;
    int *d_ctl;
    int *d_err;
    int *d_keys;
    int *d_order;
    long src_cap;
    int n_cu;
    size_t max_lds;
    float R_whole, R_oct;   // radius thresholds of the piece types
    int min_waves, max_waves;   // wave-per-piece mode bounds
    std::map<PlanKey, Plan> plans;
    int big_kind;           // piece kind of the forward above R_oct: 2 shell pyramids, 3 layer pyramids
    int tab_lds;            // layer forward: table in LDS (1) or through the caches (0)
    int adj_waves;          // layer adjoint: waves per work-group
    int adj_split;          // layer adjoint: rate terms of dense chunks in the reverse pass (1) or all gathered (0)
    double *d_nhi_T;        // [k][i][j] copies for the layer pieces (allocated on first use)
    double *d_gacc_T;
    double *d_gbar_T;       // adjoint: dL/dGamma and dL/dn_HI in the [k][i][j] layout
    double *d_nbar_T;
    double *d_nbar;         // dL/dn_HI accumulator (allocated by the first backward call)
    double *d_store;        // stored exit columns of the adjoint pieces in flight
    size_t store_cap;       // doubles
    // column records kept by a forward call made with ASORA_STORE (layer pieces)
    char *d_keep;
    size_t keep_alloc;      // bytes allocated
    size_t keep_need;       // bytes the most recent ASORA_STORE forward needed
    size_t keep_budget;     // 0: half the free device memory at the call
    bool keep_valid;
    const void *keep_sig[5];    // n_H, x_HI, src_ijk, src_Q, src_R of that call
    int64_t keep_nsrc;
    float keep_Rmax;
    bool keep_early;        // that call stopped its pyramids at their first opaque layer
    // the source order (bucketing) in d_order and the segment table: a
    // generation counted at every bucketing, and the one the keeping forward
    // made (-1: none), which a backward with its records may reuse
    long order_gen;
    long keep_order_gen;
    // n_HI in d_nhi (and d_nhi_T): a generation counted at every write, and
    // the one the keeping forward wrote (-1: none), which its backward reuses
    long nhi_gen;
    long keep_nhi_gen;
    std::map<PlanKey, Plan> adj_plans;
    // profiling: a ring of event quadruples (call start, sweep start, sweep
    // stop, call stop), one per call made with ASORA_PROFILE
    hipEvent_t pev[kProfSlots][4];
    long prof_count;        // profiled calls so far
    int prof_pending;       // profiled calls since the last summary reset (<= kProfSlots)
    int live_graphs;        // graphs recorded from this context and not yet freed: they
                            // hold its buffers' addresses, so no buffer may move
    std::map<std::string, std::vector<float>> tuned;   // autotune results by workload key
    std::string dev_tag;    // device name and compute-unit count (part of the tuning keys)
    char *d_static;         // this device's `scratch` array (asora_raytrace_static), or NULL
    asora_tune_progress_fn tune_cb;   // called after every timed autotune candidate (may be NULL)
    void *tune_cb_user;
    // chemistry: counters (cells changed, cells whose n_e iteration did not
    // converge); the time step's <y> in two FP64 grids and one FP32 grid
    unsigned long long *d_chem_cnt;
    double *d_chem_y[2];
    float *d_chem_y32;
    std::string err;
};

static const int kMagic = 0x4153524f;
static std::string g_init_err;
static std::mutex g_init_mu;

static asora_status fail(asora_ctx *c, asora_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else {
        std::lock_guard<std::mutex> g(g_init_mu);
        g_init_err = buf;
    }
    return st;
}

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, e_ == hipErrorOutOfMemory ? ASORA_ENOMEM : ASORA_EHIP, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                        \
    } while (0)

static bool ctx_ok(const asora_ctx *c) { return c && c->magic == kMagic; }

// ---------------------------------------------------------------------------
extern "C" asora_status asora_table_blackbody(double T_bb, double index, int32_t n, double lg_lo,
                                              double lg_hi, double *P, double *dPdtau)
{
    if (table_blackbody(T_bb, index, n, lg_lo, lg_hi, P, dPdtau) != 0)
        return fail(nullptr, ASORA_EINVAL, "asora_table_blackbody: invalid argument");
    return ASORA_OK;
}

extern "C" asora_status asora_table_blackbody_heat(double T_bb, double index, int32_t n, double lg_lo,
                                                   double lg_hi, double *H, double *dHdtau)
{
    if (table_blackbody_heat(T_bb, index, n, lg_lo, lg_hi, H, dHdtau) != 0)
        return fail(nullptr, ASORA_EINVAL, "asora_table_blackbody_heat: invalid argument");
    return ASORA_OK;
}

extern "C" asora_status asora_table_blackbody_band(double T_bb, double index, double e_lo_eV, double e_hi_eV,
                                                   int32_t n, double lg_lo, double lg_hi, double *P, double *dPdtau)
{
    if (table_blackbody_band(T_bb, index, e_lo_eV, e_hi_eV, n, lg_lo, lg_hi, P, dPdtau) != 0)
        return fail(nullptr, ASORA_EINVAL, "asora_table_blackbody_band: invalid argument");
    return ASORA_OK;
}

extern "C" asora_status asora_table_grey(int32_t n, double lg_lo, double lg_hi, double *P,
                                         double *dPdtau)
{
    if (n < 2 || !(lg_hi > lg_lo) || !P || !dPdtau)
        return fail(nullptr, ASORA_EINVAL, "asora_table_grey: invalid argument");
    for (int t = 0; t < n; ++t) {
        const double tau = std::pow(10.0, lg_lo + (lg_hi - lg_lo) * t / (double)(n - 1));
        P[t] = std::exp(-tau);
        dPdtau[t] = -std::exp(-tau);
    }
    return ASORA_OK;
}

// ---------------------------------------------------------------------------
// First node of a table that the kernels cannot take (values must be positive
// normal FP32 numbers, non-increasing, slopes finite and <= 0), or -1.
static int bad_table_node(int n, const double *P, const double *dP)
{
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(P[k]) || !(P[k] >= 1.2e-38) || !std::isfinite(dP[k]) || dP[k] > 0 ||
            (k > 0 && P[k] > P[k - 1]))
            return k;
    return -1;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free forward (asora_raytrace_static): a file-scope
// device array of fixed size, of which every device holds its own copy for
// the life of the process.  Host code never uses the array's name as an
// address: asora_init looks up each device's copy once with
// hipGetSymbolAddress and every later use goes through that pointer.
// Layout: n_HI, the rate accumulator and their [k][i][j] copies (FP64, up to
// kStaticMaxN^3 cells each), the control block, the source keys and the
// scheduling order (up to kStaticMaxSources each).
constexpr int kStaticMaxN = 64;
constexpr long kStaticMaxSources = 1L << 16;
constexpr size_t kStaticCells = (size_t)kStaticMaxN * kStaticMaxN * kStaticMaxN;
constexpr size_t pad256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kStaticGrid = pad256(kStaticCells * sizeof(double));
constexpr size_t kStaticOffCtl = 4 * kStaticGrid;
constexpr size_t kStaticOffKeys = kStaticOffCtl + pad256((size_t)kCtlSize * sizeof(int));
constexpr size_t kStaticOffOrder = kStaticOffKeys + pad256((size_t)kStaticMaxSources * sizeof(int));
constexpr size_t kStaticBytes = kStaticOffOrder + pad256((size_t)kStaticMaxSources * sizeof(int));

static __device__ __align__(256) char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices];   // each device's copy of `scratch` (NULL: not looked up yet)

// This device's copy of `scratch` (the device must be current), looked up
// once per device.
static hipError_t device_scratch(int device, char **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (char *)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

extern "C" asora_status asora_init(asora_ctx **out, int32_t N, double cell_cm, double sigma0_cm2,
                                   double lg_tau_lo, double lg_tau_hi, int32_t n_tab,
                                   const double *P, const double *dPdtau,
                                   double tau_weight_floor, uint32_t flags, int32_t device)
{
    if (!out) return fail(nullptr, ASORA_EINVAL, "asora_init: out is NULL");
    *out = nullptr;
    if (N < 1 || N > 1600) return fail(nullptr, ASORA_EINVAL, "asora_init: N=%d out of [1,1600]", N);
    if (!(cell_cm > 0) || !std::isfinite(cell_cm))
        return fail(nullptr, ASORA_EINVAL, "asora_init: cell size must be positive and finite");
    if (!(sigma0_cm2 > 0) || !std::isfinite(sigma0_cm2))
        return fail(nullptr, ASORA_EINVAL, "asora_init: sigma0 must be positive and finite");
    if (!(lg_tau_hi > lg_tau_lo) || !std::isfinite(lg_tau_lo) || !std::isfinite(lg_tau_hi))
        return fail(nullptr, ASORA_EINVAL, "asora_init: table range must satisfy lo < hi");
    if (n_tab < 2 || n_tab > 4096)
        return fail(nullptr, ASORA_EINVAL, "asora_init: n_tab=%d out of [2,4096]", n_tab);
    if (!P || !dPdtau) return fail(nullptr, ASORA_EINVAL, "asora_init: table pointer is NULL");
    const int bad = bad_table_node(n_tab, P, dPdtau);
    if (bad >= 0)
        return fail(nullptr, ASORA_EINVAL,
                    "asora_init: table node %d invalid (P must be positive, >= 1.2e-38, "
                    "non-increasing; dP/dtau finite and <= 0)", bad);
    if (std::isnan(tau_weight_floor) || tau_weight_floor < 0)
        return fail(nullptr, ASORA_EINVAL, "asora_init: tau_weight_floor must be >= 0 or +inf");
    if (flags & ~ASORA_INIT_SOURCE_HALFPATH_SCALAR)
        return fail(nullptr, ASORA_EINVAL, "asora_init: unknown flags 0x%x", flags);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(nullptr, ASORA_EINVAL, "asora_init: device %d not available", device);

    asora_ctx *c = new asora_ctx();
    c->magic = kMagic;
    c->device = device;
    c->N = N;
    c->alpha = cell_cm;
    c->sigma0 = sigma0_cm2;
    c->tau_w = (tau_weight_floor > 0 && std::isfinite(tau_weight_floor)) ? tau_weight_floor : 0.0;
    c->flags = flags;
    c->reading = (flags & ASORA_INIT_SOURCE_HALFPATH_SCALAR) ? 1 : 0;
    c->R_whole = 6.f;
    c->R_oct = 15.f;
    c->min_waves = 4;
    c->max_waves = 16;
    c->big_kind = 3;
    c->tab_lds = 1;
    c->keep_order_gen = -1;
    c->keep_nhi_gen = -1;
    c->adj_waves = 4;
    c->adj_split = 1;

    // table in the kernels' form
    std::vector<TabNode> nodes(n_tab);
    std::vector<double> m64(n_tab);
    prepare_table(n_tab, lg_tau_lo, lg_tau_hi, P, dPdtau, &c->tp, nodes.data(), m64.data());
    c->lg_lo = lg_tau_lo;
    c->lg_hi = lg_tau_hi;

    auto bail = [&](asora_status st) {
        asora_free(c);
        return st;
    };
    if (hipSetDevice(device) != hipSuccess)
        return bail(fail(nullptr, ASORA_EHIP, "asora_init: hipSetDevice(%d) failed", device));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return bail(fail(nullptr, ASORA_EHIP, "asora_init: hipGetDeviceProperties failed"));
    c->n_cu = prop.multiProcessorCount;
    c->max_lds = prop.sharedMemPerBlock;
    {
        char tag[96];
        snprintf(tag, sizeof tag, "%s:%d", prop.gcnArchName, c->n_cu);
        c->dev_tag = tag;
        for (char &ch : c->dev_tag)
            if (ch == ' ' || ch == '/') ch = '_';
    }
    const long n3 = (long)N * N * N;
    if (hipMalloc(&c->d_tab, sizeof(TabNode) * n_tab) != hipSuccess ||
        hipMalloc(&c->d_m64, sizeof(double) * n_tab) != hipSuccess ||
        hipMalloc(&c->d_nhi, sizeof(double) * n3) != hipSuccess ||
        hipMalloc(&c->d_gacc, sizeof(double) * n3) != hipSuccess ||
        hipMalloc(&c->d_ctl, sizeof(int) * kCtlSize) != hipSuccess ||
        hipMalloc(&c->d_err, sizeof(int)) != hipSuccess)
        return bail(fail(nullptr, ASORA_ENOMEM, "asora_init: device allocation of %.1f MB failed",
                         16.0 * n3 / 1e6));
    if (hipMemcpy(c->d_tab, nodes.data(), sizeof(TabNode) * n_tab, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_m64, m64.data(), sizeof(double) * n_tab, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->d_err, 0, sizeof(int)) != hipSuccess ||
        hipMemset(c->d_ctl, 0, sizeof(int) * kCtlSize) != hipSuccess)
        return bail(fail(nullptr, ASORA_EHIP, "asora_init: copy to device failed"));
    for (int sl = 0; sl < kProfSlots; ++sl)
        for (int k = 0; k < 4; ++k)
            if (hipEventCreate(&c->pev[sl][k]) != hipSuccess)
                return bail(fail(nullptr, ASORA_EHIP, "asora_init: hipEventCreate failed"));
    if (fwd_configure(c->max_lds) != hipSuccess || adj_configure(c->max_lds) != hipSuccess ||
        he_configure(c->max_lds) != hipSuccess)
        return bail(fail(nullptr, ASORA_EHIP, "asora_init: kernel attribute setup failed"));
    if (device < kMaxDevices) {   // beyond, the context works without asora_raytrace_static
        const hipError_t e = device_scratch(device, &c->d_static);
        if (e != hipSuccess)
            return bail(fail(nullptr, ASORA_EHIP, "asora_init: hipGetSymbolAddress of the static scratch: %s",
                             hipGetErrorString(e)));
    }
    *out = c;
    return ASORA_OK;
}

extern "C" asora_status asora_free(asora_ctx *c)
{
    if (!c) return ASORA_OK;
    if (c->magic != kMagic) return ASORA_ESTATE;
    if (c->live_graphs)
        return fail(c, ASORA_ESTATE, "asora_free: %d recorded graph(s) still use this context",
                    c->live_graphs);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->d_tab);
    (void)hipFree(c->d_m64);
    (void)hipFree(c->d_tab_h);
    (void)hipFree(c->d_hacc);
    (void)hipFree(c->d_hacc_T);
    (void)hipFree(c->d_tab_he);
    (void)hipFree(c->d_nhe);
    (void)hipFree(c->d_nhe_T);
    (void)hipFree(c->d_ghe);
    (void)hipFree(c->d_ghe_T);
    (void)hipFree(c->d_nhi);
    (void)hipFree(c->d_gacc);
    (void)hipFree(c->d_ctl);
    (void)hipFree(c->d_err);
    (void)hipFree(c->d_keys);
    (void)hipFree(c->d_order);
    (void)hipFree(c->d_nhi_T);
    (void)hipFree(c->d_gacc_T);
    (void)hipFree(c->d_gbar_T);
    (void)hipFree(c->d_nbar_T);
    (void)hipFree(c->d_nbar);
    (void)hipFree(c->d_store);
    (void)hipFree(c->d_keep);
    (void)hipFree(c->d_chem_cnt);
    (void)hipFree(c->d_chem_y[0]);
    (void)hipFree(c->d_chem_y[1]);
    (void)hipFree(c->d_chem_y32);
    for (int sl = 0; sl < kProfSlots; ++sl)
        for (int k = 0; k < 4; ++k)
            if (c->pev[sl][k]) (void)hipEventDestroy(c->pev[sl][k]);
    c->magic = 0;
    delete c;
    return ASORA_OK;
}

extern "C" const char *asora_last_error(const asora_ctx *c)
{
    if (!c) {
        std::lock_guard<std::mutex> g(g_init_mu);
        return g_init_err.c_str();
    }
    return c->err.c_str();
}

extern "C" asora_status asora_check(asora_ctx *c, void *stream)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    int e = 0;
    HIPCHK(c, hipMemcpy(&e, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (e) {
        HIPCHK(c, hipMemset(c->d_err, 0, sizeof(int)));
        return fail(c, ASORA_ERANGE,
                    "a source had a radius above the call's R_max (or was outside the grid) and "
                    "was skipped");
    }
    return ASORA_OK;
}

// ---------------------------------------------------------------------------
// Launch planning: on-chip buffer sizes of one piece type for radii <= R_cap.
static int type_of(const asora_ctx *c, float R)
{
    return R <= c->R_whole ? 0 : (R <= c->R_oct ? 1 : 2);
}

static asora_status get_layer_plan(asora_ctx *c, float R_cap, Plan *out, bool store = true);

// store = false: the plan is not added to the context's table (no host
// allocation; the allocation-free entry point plans every call)
static asora_status get_plan(asora_ctx *c, int type, float R_cap, Plan *out, bool store = true)
{
    if (type == 3) return get_layer_plan(c, R_cap, out, store);
    const int Rsq = (int)std::floor((double)R_cap * (double)R_cap);
    const PlanKey key{type, Rsq};
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
        *out = it->second;
        return ASORA_OK;
    }
    const Extent ex = make_extent(c->N);
    const int Qmax = max_shell(Rsq, ex);
    int ring = 1;
    long cells = 1;
    for (int p = 0; p < pieces_of_type(type); ++p) {
        const Piece pc = make_piece(type, p);
        long pcells = 0;
        for (int q = 1; q <= Qmax; ++q) {
            int tot = 0;
            for (int r = 0; r < pc.n_oct * (q + 1); ++r) {
                int blo, cnt;
                row_range(pc, ex, Rsq, q, r, &blo, &cnt);
                tot += cnt;
            }
            ring = tot > ring ? tot : ring;
            pcells += tot;
        }
        cells = pcells > cells ? pcells : cells;
    }
    Plan P;
    P.piece_cells = cells;
    P.ring_cap = ring;
    P.row_cap = (type == 0 ? 8 : 1) * (Qmax + 1);
    P.Qmax = Qmax;
    // one wave per piece when at least c->min_waves per-wave regions fit next to
    // the table; else a whole work-group per piece
    const size_t tab = (size_t)c->tp.n * sizeof(TabNode);
    const size_t region = wave_region_bytes(P.ring_cap, P.row_cap);
    const long fit = c->max_lds > tab + 64 ? (long)((c->max_lds - tab - 64) / region) : 0;
    int bpc = 0;
    if (fit >= c->min_waves && P.row_cap <= 256) {
        P.wave_mode = 1;
        P.waves = (int)(fit < c->max_waves ? fit : c->max_waves);
        P.lds = tab + (size_t)P.waves * region;
        HIPCHK(c, wave_occupancy(type, P.waves, P.lds, &bpc));
    } else {
        P.wave_mode = 0;
        P.waves = 4;
        P.lds = fwd_lds_bytes(c->tp.n, P.ring_cap, P.row_cap);
        if (P.lds + 64 > c->max_lds)
            return fail(c, ASORA_ENOSYS,
                        "R_max=%.1f needs %zu bytes of LDS per work-group (limit %zu) for this "
                        "table and grid", R_cap, P.lds, c->max_lds);
        HIPCHK(c, fwd_occupancy(P.lds, &bpc));
    }
    P.grid = c->n_cu * (bpc > 0 ? bpc : 1);
    if (store) c->plans[key] = P;
    *out = P;
    return ASORA_OK;
}

// Waves of a layer sweep's work-group: as many per-wave regions as fit in the
// LDS next to the work-group's own bytes (wg), up to cap.  The table of square
// roots (sqb bytes) is added only when it costs no wave: a wave more hides
// more latency than the table saves (a root is a handful of instructions per
// cell).  0 when not even one region fits.
static int layer_waves(const asora_ctx *c, size_t wg, size_t sqb, size_t region, int cap, bool *sq_table)
{
    auto fit = [&](size_t b) -> long {
        const long f = c->max_lds > b + 64 ? (long)((c->max_lds - b - 64) / region) : 0;
        return f < cap ? f : cap;
    };
    const long with = sqb ? fit(wg + sqb) : 0, without = fit(wg);
    *sq_table = sqb && with >= without;
    return (int)(*sq_table ? with : without);
}

// Layer pieces: one wave per pyramid, the wave's LDS holds one layer.
static asora_status get_layer_plan(asora_ctx *c, float R_cap, Plan *out, bool store)
{
    const int Rsq = (int)std::floor((double)R_cap * (double)R_cap);
    const PlanKey key{c->tab_lds ? 3 : 5, Rsq};
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
        *out = it->second;
        return ASORA_OK;
    }
    const Extent ex = make_extent(c->N);
    Plan P = Plan();
    int r = (int)std::floor(std::sqrt((double)Rsq));
    while ((long)r * r > Rsq) --r;
    while ((long)(r + 1) * (r + 1) <= Rsq) ++r;
    P.Mcap = r < ex.neg ? r : ex.neg;
    if (P.Mcap < 1) P.Mcap = 1;
    P.S = layer_buffer_side(Rsq, ex);
    P.rec_cap = layer_piece_capacity(Rsq, ex);
    if (P.rec_cap < 1) P.rec_cap = 1;
    P.rec_bytes = layer_record_bytes(P.rec_cap, P.Mcap, false);
    P.keep_bytes = layer_record_bytes(P.rec_cap, P.Mcap, true);
    P.wave_mode = 1;
    // the work-group's LDS: the table (if placed there), the table of square
    // roots (if it costs no wave), one region per wave
    const size_t tab = c->tab_lds ? (size_t)c->tp.n * sizeof(TabNode) : 0;
    const size_t sqb = layer_sqrt_bytes(Rsq);
    for (bool keep : {false, true}) {
        const size_t region = layer_region_bytes(P.S, keep);
        bool sq = false;
        const int waves = layer_waves(c, tab, sqb, region, c->max_waves, &sq);
        if (waves < 1 || Rsq > 65535)   // the rate queue holds r^2 in 16 bits
            return fail(c, ASORA_ENOSYS,
                        "R_max=%.1f needs %zu bytes of LDS per wave (limit %zu) for this table and grid",
                        R_cap, region + tab, c->max_lds);
        const size_t lds = tab + (sq ? sqb : 0) + (size_t)waves * region;
        int bpc = 0;
        HIPCHK(c, layer_occupancy(keep, c->tab_lds != 0, waves, lds, &bpc));
        const int grid = c->n_cu * (bpc > 0 ? bpc : 1);
        if (keep) {
            P.kwaves = waves, P.kgrid = grid, P.ksq_table = sq;
        } else {
            P.waves = waves, P.grid = grid, P.sq_table = sq;
            P.lds = lds;
        }
    }
    if (store) c->plans[key] = P;
    *out = P;
    return ASORA_OK;
}

static asora_status ensure_layer_buffers(asora_ctx *c)
{
    if (c->d_nhi_T) return ASORA_OK;
    const size_t n3 = (size_t)c->N * c->N * c->N;
    HIPCHK(c, hipMalloc(&c->d_nhi_T, sizeof(double) * n3));
    if (hipMalloc(&c->d_gacc_T, sizeof(double) * n3) != hipSuccess) {
        (void)hipFree(c->d_nhi_T);
        c->d_nhi_T = nullptr;
        return fail(c, ASORA_ENOMEM, "allocation of the transposed field copies failed");
    }
    return ASORA_OK;
}

static asora_status pinned(asora_ctx *c, const char *what)
{
    return fail(c, ASORA_ESTATE,
                "%s would have to grow while a recorded graph holds the current buffers; free the "
                "graphs (asora_graph_free) first", what);
}

static asora_status ensure_src_cap(asora_ctx *c, long n)
{
    if (n <= c->src_cap) return ASORA_OK;
    if (c->live_graphs) return pinned(c, "the source order buffer");
    long cap = c->src_cap ? c->src_cap : 1024;
    while (cap < n) cap *= 2;
    (void)hipFree(c->d_keys);
    (void)hipFree(c->d_order);
    c->d_keys = c->d_order = nullptr;
    c->src_cap = 0;
    HIPCHK(c, hipMalloc(&c->d_keys, sizeof(int) * cap));
    HIPCHK(c, hipMalloc(&c->d_order, sizeof(int) * cap));
    c->src_cap = cap;
    return ASORA_OK;
}

// Device memory for the kept column records: `need` bytes if they fit the
// budget (the explicit one, else half of the free device memory plus what is
// already allocated).  *ok = false leaves nothing kept.  Growing frees the old
// allocation, which waits for the device.
static asora_status reserve_keep(asora_ctx *c, size_t need, bool *ok)
{
    *ok = false;
    if (need == 0) return ASORA_OK;
    if (need <= c->keep_alloc && (c->keep_budget == 0 || need <= c->keep_budget)) {
        *ok = true;   // fits what is held (no device query: this may run while a graph records)
        return ASORA_OK;
    }
    size_t budget = c->keep_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        HIPCHK(c, hipMemGetInfo(&fr, &tot));
        budget = fr / 2 + c->keep_alloc;
    }
    if (need > budget) return ASORA_OK;
    if (need > c->keep_alloc) {
        if (c->live_graphs) return pinned(c, "the kept column records");
        (void)hipFree(c->d_keep);
        c->d_keep = nullptr;
        c->keep_alloc = 0;
        if (hipMalloc(&c->d_keep, need) != hipSuccess) {
            (void)hipGetLastError();
            return ASORA_OK;   // treated as not fitting
        }
        c->keep_alloc = need;
    }
    *ok = true;
    return ASORA_OK;
}

extern "C" asora_status asora_store_info(const asora_ctx *c, int32_t *valid, uint64_t *bytes_needed,
                                         uint64_t *bytes_allocated)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (valid) *valid = c->keep_valid ? 1 : 0;
    if (bytes_needed) *bytes_needed = c->keep_need;
    if (bytes_allocated) *bytes_allocated = c->keep_alloc;
    return ASORA_OK;
}

extern "C" asora_status asora_set_store_budget(asora_ctx *c, uint64_t bytes)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    c->keep_budget = (size_t)bytes;
    return ASORA_OK;
}

// Largest source list of one call: the persistent kernels number their work
// items (source, piece) in 32-bit integers, up to 24 pieces per source.
static const int64_t kMaxSources = (int64_t)INT32_MAX / 24;

extern "C" int64_t asora_max_sources(void) { return kMaxSources; }

static asora_status check_common(asora_ctx *c, const float *n_H, const float *x_HI, int64_t n_src,
                                 const int32_t *ijk, const double *Q, float R_max)
{
    if (!n_H || !x_HI) return fail(c, ASORA_EINVAL, "n_H and x_HI must not be NULL");
    if (n_src < 0 || n_src > kMaxSources)
        return fail(c, ASORA_EINVAL, "n_src=%lld out of [0, %lld]", (long long)n_src, (long long)kMaxSources);
    if (n_src > 0 && (!ijk || !Q)) return fail(c, ASORA_EINVAL, "source arrays must not be NULL");
    if (!(R_max >= 0.f) || !(R_max <= 4096.f))
        return fail(c, ASORA_EINVAL, "R_max must be in [0, 4096]");
    return ASORA_OK;
}

extern "C" asora_status asora_set_heating_table(asora_ctx *c, const double *H, const double *dHdtau)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (!H || !dHdtau) return fail(c, ASORA_EINVAL, "asora_set_heating_table: table pointer is NULL");
    const int n = c->tp.n;
    const int bad = bad_table_node(n, H, dHdtau);
    if (bad >= 0)
        return fail(c, ASORA_EINVAL,
                    "asora_set_heating_table: node %d invalid (H must be positive, >= 1.2e-38, "
                    "non-increasing; dH/dtau finite and <= 0)", bad);
    std::vector<TabNode> nodes(n);
    TabParams tp;
    prepare_table(n, c->lg_lo, c->lg_hi, H, dHdtau, &tp, nodes.data(), nullptr);
    HIPCHK(c, hipSetDevice(c->device));
    if (!c->d_tab_h) HIPCHK(c, hipMalloc(&c->d_tab_h, sizeof(TabNode) * n));
    // ordered after the work already queued on the device: a sweep in flight
    // reads the table it started with
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(c->d_tab_h, nodes.data(), sizeof(TabNode) * n, hipMemcpyHostToDevice));
    c->dP0_h = tp.dP0;
    return ASORA_OK;
}

static asora_status forward(asora_ctx *c, const float *n_H, const float *x_HI, int64_t n_src,
                            const int32_t *src_ijk, const double *src_Q, const float *src_R, float R_max,
                            float *gamma, float *heating, double *coldens_in, uint32_t flags,
                            void *stream);

extern "C" asora_status asora_raytrace(asora_ctx *c, const float *n_H, const float *x_HI,
                                       int64_t n_src, const int32_t *src_ijk, const double *src_Q,
                                       const float *src_R, float R_max, float *gamma,
                                       double *coldens_in, uint32_t flags, void *stream)
{
    return forward(c, n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max, gamma, nullptr, coldens_in, flags,
                   stream);
}

extern "C" asora_status asora_raytrace_heating(asora_ctx *c, const float *n_H, const float *x_HI,
                                               int64_t n_src, const int32_t *src_ijk, const double *src_Q,
                                               const float *src_R, float R_max, float *gamma,
                                               float *heating, uint32_t flags, void *stream)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (!heating) return fail(c, ASORA_EINVAL, "heating must not be NULL");
    if (!c->d_tab_h)
        return fail(c, ASORA_ESTATE, "asora_raytrace_heating: no heating table (asora_set_heating_table)");
    return forward(c, n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max, gamma, heating, nullptr, flags,
                   stream);
}

// Device buffers of one forward call: n_HI and the rate accumulator in both
// layouts, the control block (work counters, segment table, histogram), the
// source keys and the scheduling order.
struct FwdBufs {
    double *nhi, *gacc, *nhi_T, *gacc_T;
    int *ctl, *keys, *order;
};

// Plans of the piece kinds a forward up to R_max uses (plans[t], t <= *tmax;
// kind 2 is skipped when the large kind is 3).
static asora_status forward_plans(asora_ctx *c, float R_max, bool store, Plan plans[4], int *tmax_out)
{
    const int tbig = type_of(c, R_max);
    const int tmax = tbig == 2 ? c->big_kind : tbig;
    for (int t = 0; t <= tmax; ++t) {
        if (t == 2 && tmax == 3) continue;
        const float cap = t == tmax ? R_max : (t == 0 ? c->R_whole : c->R_oct);
        asora_status st = get_plan(c, t, cap, &plans[t], store);
        if (st) return st;
    }
    *tmax_out = tmax;
    return ASORA_OK;
}

// The launches of one forward call on buffers B (no allocation).
static asora_status forward_launch(asora_ctx *c, const FwdBufs &B, const Plan plans[4], int tmax,
                                   const float *n_H, const float *x_HI, int64_t n_src, const int32_t *src_ijk,
                                   const double *src_Q, const float *src_R, float R_max, float *gamma,
                                   float *heating, double *coldens_in, uint32_t flags, bool keep,
                                   hipStream_t s)
{
    const bool prof = (flags & ASORA_PROFILE) != 0;
    hipEvent_t *ev = c->pev[c->prof_count % kProfSlots];
    const long n3 = (long)c->N * c->N * c->N;
    const bool layers = tmax == 3;
    FwdLaunch F;
    F.N = c->N;
    F.alpha = c->alpha;
    F.sigma0 = c->sigma0;
    F.tau_w = (float)c->tau_w;
    F.reading = c->reading;
    F.tp = c->tp;
    F.tab = c->d_tab;
    F.nHI = B.nhi;
    F.gacc = B.gacc;
    F.coldens = coldens_in;
    F.ijk = src_ijk;
    F.Q = src_Q;
    F.R = src_R;
    F.order = B.order;
    F.ctl = B.ctl;
    F.err = c->d_err;
    F.nHI_T = B.nhi_T;
    F.gacc_T = B.gacc_T;
    F.keep = keep ? c->d_keep : nullptr;
    F.keep_piece_bytes = layers ? plans[3].keep_bytes : 0;
    F.keep_cap = layers ? plans[3].rec_cap : 0;
    F.keep_rk_off = layers ? plans[3].rec_bytes : 0;
    F.m64 = c->d_m64;
    F.tab_lds = c->tab_lds;
    F.sq_table = layers && (keep ? plans[3].ksq_table : plans[3].sq_table);
    F.early_exit = (flags & ASORA_EARLY_EXIT) != 0;
    F.tab_h = heating ? c->d_tab_h : nullptr;
    F.hacc = heating ? c->d_hacc : nullptr;
    F.hacc_T = heating && layers ? c->d_hacc_T : nullptr;
    F.dP0_h = c->dP0_h;

    if (prof) HIPCHK(c, hipEventRecord(ev[0], s));
    HIPCHK(c, launch_prologue(s, n_H, x_HI, B.nhi, B.gacc, coldens_in, n3, B.ctl, kCtlSize, c->n_cu));
    if (layers) HIPCHK(c, launch_transpose_prologue(s, n_H, x_HI, B.nhi_T, B.gacc_T, c->N));
    if (heating) {
        HIPCHK(c, launch_zero(s, c->d_hacc, n3, c->n_cu));
        if (layers) HIPCHK(c, launch_zero(s, c->d_hacc_T, n3, c->n_cu));
    }
    const bool bucketed = n_src > 0 && !(flags & ASORA_PLAIN);
    if (bucketed)
        HIPCHK(c, launch_bucketing(s, src_R, src_ijk, n_src, c->N, R_max, c->R_whole, c->R_oct,
                                   tmax == 3 ? 3 : 2, B.keys, B.ctl, B.order, c->d_err));
    if (prof) HIPCHK(c, hipEventRecord(ev[1], s));
    if (n_src > 0) {
        if (flags & ASORA_PLAIN) {
            F.type = tmax;
            F.R_cap = R_max;
            F.ring_cap = plans[tmax].ring_cap;
            F.row_cap = plans[tmax].row_cap;
            for (long k = 0; k < n_src; ++k) {
                if (tmax == 3)
                    HIPCHK(c, launch_fwd_layer(s, F, plans[3].S, keep ? plans[3].kwaves : plans[3].waves, 0,
                                               (int)k));
                else if (plans[tmax].wave_mode)
                    HIPCHK(c, launch_fwd_wave(s, F, plans[tmax].waves, 0, (int)k));
                else
                    HIPCHK(c, launch_fwd_plain(s, F, (int)k));
            }
        } else {
            for (int t = tmax; t >= 0; --t) {
                if (t == 2 && tmax == 3) continue;
                F.type = t;
                F.R_cap = t == tmax ? R_max : (t == 0 ? c->R_whole : c->R_oct);
                F.ring_cap = plans[t].ring_cap;
                F.row_cap = plans[t].row_cap;
                if (t == 3)
                    HIPCHK(c, launch_fwd_layer(s, F, plans[3].S, keep ? plans[3].kwaves : plans[3].waves,
                                               keep ? plans[3].kgrid : plans[3].grid, -1));
                else if (plans[t].wave_mode)
                    HIPCHK(c, launch_fwd_wave(s, F, plans[t].waves, plans[t].grid, -1));
                else
                    HIPCHK(c, launch_fwd_persistent(s, F, plans[t].grid));
            }
        }
    }
    if (prof) HIPCHK(c, hipEventRecord(ev[2], s));
    if (layers)
        HIPCHK(c, launch_transpose_finalize(s, B.gacc, B.gacc_T, gamma, c->N, (flags & ASORA_ACCUMULATE) ? 1 : 0));
    else
        HIPCHK(c, launch_finalize(s, B.gacc, gamma, n3, (flags & ASORA_ACCUMULATE) ? 1 : 0, c->n_cu));
    if (heating && layers)
        HIPCHK(c, launch_transpose_finalize(s, c->d_hacc, c->d_hacc_T, heating, c->N,
                                            (flags & ASORA_ACCUMULATE) ? 1 : 0));
    else if (heating)
        HIPCHK(c, launch_finalize(s, c->d_hacc, heating, n3, (flags & ASORA_ACCUMULATE) ? 1 : 0, c->n_cu));
    if (prof) {
        HIPCHK(c, hipEventRecord(ev[3], s));
        c->prof_count++;
        if (c->prof_pending < kProfSlots) c->prof_pending++;
    }
    return ASORA_OK;
}

static asora_status forward(asora_ctx *c, const float *n_H, const float *x_HI, int64_t n_src,
                            const int32_t *src_ijk, const double *src_Q, const float *src_R, float R_max,
                            float *gamma, float *heating, double *coldens_in, uint32_t flags,
                            void *stream)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    asora_status st = check_common(c, n_H, x_HI, n_src, src_ijk, src_Q, R_max);
    if (st) return st;
    if (!gamma) return fail(c, ASORA_EINVAL, "gamma must not be NULL");
    if (coldens_in && n_src != 1) return fail(c, ASORA_EINVAL, "coldens_in requires n_src == 1");
    if (flags & ~(ASORA_ACCUMULATE | ASORA_PLAIN | ASORA_PROFILE | ASORA_STORE | ASORA_EARLY_EXIT))
        return fail(c, ASORA_EINVAL, "unknown flags");
    if (coldens_in && (flags & ASORA_EARLY_EXIT))
        return fail(c, ASORA_EINVAL, "ASORA_EARLY_EXIT does not give entry columns (coldens_in)");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const long n3 = (long)c->N * c->N * c->N;
    Plan plans[4];
    int tmax = 0;
    if ((st = forward_plans(c, R_max, true, plans, &tmax))) return st;
    const bool layers = tmax == 3;
    if ((st = ensure_src_cap(c, n_src))) return st;
    if (layers && (st = ensure_layer_buffers(c))) return st;
    if (heating) {
        if (!c->d_hacc) HIPCHK(c, hipMalloc(&c->d_hacc, sizeof(double) * n3));
        if (layers && !c->d_hacc_T) HIPCHK(c, hipMalloc(&c->d_hacc_T, sizeof(double) * n3));
    }
    // ASORA_STORE: keep the pyramids' column records for the adjoint when
    // they fit the budget; any other forward with the flag replaces them
    bool keep = false;
    if (flags & ASORA_STORE) {
        c->keep_valid = false;
        c->keep_need = layers ? (size_t)n_src * 24 * plans[3].keep_bytes : 0;
        if ((st = reserve_keep(c, c->keep_need, &keep))) return st;
    }
    // n_HI and the source order are rewritten from here on (even if a launch fails)
    ++c->nhi_gen;
    const bool bucketed = n_src > 0 && !(flags & ASORA_PLAIN);
    if (bucketed) ++c->order_gen;
    const FwdBufs B{c->d_nhi, c->d_gacc, c->d_nhi_T, c->d_gacc_T, c->d_ctl, c->d_keys, c->d_order};
    if ((st = forward_launch(c, B, plans, tmax, n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max, gamma, heating,
                             coldens_in, flags, keep, s)))
        return st;
    if (keep) {
        c->keep_valid = true;
        c->keep_order_gen = bucketed ? c->order_gen : -1;
        c->keep_nhi_gen = c->nhi_gen;
        c->keep_sig[0] = n_H;
        c->keep_sig[1] = x_HI;
        c->keep_sig[2] = src_ijk;
        c->keep_sig[3] = src_Q;
        c->keep_sig[4] = src_R;
        c->keep_nsrc = n_src;
        c->keep_Rmax = R_max;
        c->keep_early = (flags & ASORA_EARLY_EXIT) != 0;
    }
    return ASORA_OK;
}

// ---------------------------------------------------------------------------
// Two absorbers: hydrogen and helium.
extern "C" asora_status asora_set_helium(asora_ctx *c, int32_t n_bands, int32_t n_tab, const double *lg_lo,
                                         const double *lg_hi, const double *P, const double *dPdtau,
                                         const double *sigma_HI, const double *sigma_HeI)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (n_bands < 1 || n_bands > kMaxBands || n_tab < 2 || n_tab > 4096)
        return fail(c, ASORA_EINVAL, "asora_set_helium: need 1 <= n_bands <= %d and 2 <= n_tab <= 4096",
                    kMaxBands);
    if (!lg_lo || !lg_hi || !P || !dPdtau || !sigma_HI || !sigma_HeI)
        return fail(c, ASORA_EINVAL, "asora_set_helium: NULL argument");
    std::vector<TabNode> nodes((size_t)n_bands * n_tab);
    TabParams tp[kMaxBands];
    for (int b = 0; b < n_bands; ++b) {
        if (!(lg_hi[b] > lg_lo[b]) || !std::isfinite(lg_lo[b]) || !std::isfinite(lg_hi[b]))
            return fail(c, ASORA_EINVAL, "asora_set_helium: band %d: table range must satisfy lo < hi", b);
        if (!(sigma_HI[b] >= 0) || !(sigma_HeI[b] >= 0) || !std::isfinite(sigma_HI[b]) ||
            !std::isfinite(sigma_HeI[b]) || !(sigma_HI[b] + sigma_HeI[b] > 0))
            return fail(c, ASORA_EINVAL, "asora_set_helium: band %d: cross-sections must be >= 0, finite, "
                                         "not both 0", b);
        const int bad = bad_table_node(n_tab, P + (size_t)b * n_tab, dPdtau + (size_t)b * n_tab);
        if (bad >= 0)
            return fail(c, ASORA_EINVAL, "asora_set_helium: band %d: table node %d invalid (P must be positive, "
                                         ">= 1.2e-38, non-increasing; dP/dtau finite and <= 0)", b, bad);
        prepare_table(n_tab, lg_lo[b], lg_hi[b], P + (size_t)b * n_tab, dPdtau + (size_t)b * n_tab, &tp[b],
                      nodes.data() + (size_t)b * n_tab, nullptr);
    }
    HIPCHK(c, hipSetDevice(c->device));
    if (c->live_graphs) return pinned(c, "the helium tables");
    // ordered after the work already queued: a sweep in flight reads its tables
    HIPCHK(c, hipDeviceSynchronize());
    if (c->d_tab_he && (c->he_nb != n_bands || c->he_ntab != n_tab)) {
        (void)hipFree(c->d_tab_he);
        c->d_tab_he = nullptr;
    }
    if (!c->d_tab_he) HIPCHK(c, hipMalloc(&c->d_tab_he, sizeof(TabNode) * nodes.size()));
    HIPCHK(c, hipMemcpy(c->d_tab_he, nodes.data(), sizeof(TabNode) * nodes.size(), hipMemcpyHostToDevice));
    c->he_nb = n_bands;
    c->he_ntab = n_tab;
    for (int b = 0; b < n_bands; ++b) {
        c->he_tp[b] = tp[b];
        c->he_sH[b] = sigma_HI[b];
        c->he_sHe[b] = sigma_HeI[b];
    }
    return ASORA_OK;
}

// The two-absorber sweep's plan: layer pyramids, one wave each, the
// work-group's table of square roots and one region per wave.
static asora_status get_he_plan(asora_ctx *c, float R_cap, Plan *out)
{
    const int Rsq = (int)std::floor((double)R_cap * (double)R_cap);
    const PlanKey key{6, Rsq};
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
        *out = it->second;
        return ASORA_OK;
    }
    const Extent ex = make_extent(c->N);
    Plan P = Plan();
    P.S = layer_buffer_side(Rsq, ex);
    P.wave_mode = 1;
    const size_t sqb = layer_sqrt_bytes(Rsq);
    const size_t region = he_region_bytes(P.S);
    P.waves = layer_waves(c, 0, sqb, region, c->max_waves, &P.sq_table);
    if (P.waves < 1 || Rsq > 65535)   // the rate queue holds r^2 in 16 bits
        return fail(c, ASORA_ENOSYS, "asora_raytrace_helium: R_max=%.1f needs %zu bytes of LDS per wave (limit %zu)",
                    R_cap, region, c->max_lds);
    P.lds = (P.sq_table ? sqb : 0) + (size_t)P.waves * region;
    int bpc = 0;
    HIPCHK(c, he_occupancy(P.waves, P.lds, &bpc));
    P.grid = c->n_cu * (bpc > 0 ? bpc : 1);
    c->plans[key] = P;
    *out = P;
    return ASORA_OK;
}

extern "C" asora_status asora_raytrace_helium(asora_ctx *c, const float *n_H, const float *x_HI, const float *n_He,
                                              const float *x_HeI, int64_t n_src, const int32_t *src_ijk,
                                              const double *src_Q, const float *src_R, float R_max,
                                              float *gamma_HI, float *gamma_HeI, uint32_t flags, void *stream)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    asora_status st = check_common(c, n_H, x_HI, n_src, src_ijk, src_Q, R_max);
    if (st) return st;
    if (!n_He || !x_HeI || !gamma_HI || !gamma_HeI)
        return fail(c, ASORA_EINVAL, "asora_raytrace_helium: n_He, x_HeI and both outputs must not be NULL");
    if (flags & ~(ASORA_ACCUMULATE | ASORA_PLAIN | ASORA_PROFILE))
        return fail(c, ASORA_EINVAL, "asora_raytrace_helium: flags may be ACCUMULATE, PLAIN, PROFILE");
    if (!c->d_tab_he) return fail(c, ASORA_ESTATE, "asora_raytrace_helium: no band tables (asora_set_helium)");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const long n3 = (long)c->N * c->N * c->N;
    Plan plan;
    if ((st = get_he_plan(c, R_max, &plan))) return st;
    if ((st = ensure_src_cap(c, n_src))) return st;
    if ((st = ensure_layer_buffers(c))) return st;
    double **grids[4] = {&c->d_nhe, &c->d_nhe_T, &c->d_ghe, &c->d_ghe_T};
    for (double **g : grids)
        if (!*g) {
            if (c->live_graphs) return pinned(c, "the helium grids");
            HIPCHK(c, hipMalloc(g, sizeof(double) * n3));
        }
    const bool prof = (flags & ASORA_PROFILE) != 0;
    hipEvent_t *ev = c->pev[c->prof_count % kProfSlots];
    const int acc = (flags & ASORA_ACCUMULATE) ? 1 : 0;
    // n_HI, n_HeI and zeroed accumulators in both layouts; every source as layer pyramids
    ++c->nhi_gen;
    if (prof) HIPCHK(c, hipEventRecord(ev[0], s));
    HIPCHK(c, launch_prologue(s, n_H, x_HI, c->d_nhi, c->d_gacc, nullptr, n3, c->d_ctl, kCtlSize, c->n_cu));
    HIPCHK(c, launch_prologue(s, n_He, x_HeI, c->d_nhe, c->d_ghe, nullptr, n3, c->d_ctl, 0, c->n_cu));
    HIPCHK(c, launch_transpose_prologue(s, n_H, x_HI, c->d_nhi_T, c->d_gacc_T, c->N));
    HIPCHK(c, launch_transpose_prologue(s, n_He, x_HeI, c->d_nhe_T, c->d_ghe_T, c->N));
    const bool bucketed = n_src > 0 && !(flags & ASORA_PLAIN);
    if (bucketed) {
        HIPCHK(c, launch_bucketing(s, src_R, src_ijk, n_src, c->N, R_max, -1.f, -1.f, 3, c->d_keys, c->d_ctl,
                                   c->d_order, c->d_err));
        ++c->order_gen;
    }
    if (prof) HIPCHK(c, hipEventRecord(ev[1], s));
    if (n_src > 0) {
        HeLaunch H;
        H.N = c->N;
        H.alpha = c->alpha;
        H.sigma0 = c->sigma0;
        H.tau_w = (float)c->tau_w;
        H.reading = c->reading;
        H.nb = c->he_nb;
        H.n_tab = c->he_ntab;
        H.tab = c->d_tab_he;
        for (int b = 0; b < kMaxBands; ++b) {
            H.tp[b] = c->he_tp[b < c->he_nb ? b : 0];
            H.sH[b] = b < c->he_nb ? c->he_sH[b] : 0.0;
            H.sHe[b] = b < c->he_nb ? c->he_sHe[b] : 0.0;
        }
        H.nHI = c->d_nhi;
        H.nHeI = c->d_nhe;
        H.nHI_T = c->d_nhi_T;
        H.nHeI_T = c->d_nhe_T;
        H.gH = c->d_gacc;
        H.gHe = c->d_ghe;
        H.gH_T = c->d_gacc_T;
        H.gHe_T = c->d_ghe_T;
        H.ijk = src_ijk;
        H.Q = src_Q;
        H.R = src_R;
        H.R_cap = R_max;
        H.order = c->d_order;
        H.ctl = c->d_ctl;
        H.err = c->d_err;
        H.sq_table = plan.sq_table;
        if (flags & ASORA_PLAIN) {
            for (long k = 0; k < n_src; ++k)
                HIPCHK(c, launch_fwd_layer_he(s, H, plan.S, plan.waves, 0, (int)k));
        } else {
            HIPCHK(c, launch_fwd_layer_he(s, H, plan.S, plan.waves, plan.grid, -1));
        }
    }
    if (prof) HIPCHK(c, hipEventRecord(ev[2], s));
    HIPCHK(c, launch_transpose_finalize(s, c->d_gacc, c->d_gacc_T, gamma_HI, c->N, acc));
    HIPCHK(c, launch_transpose_finalize(s, c->d_ghe, c->d_ghe_T, gamma_HeI, c->N, acc));
    if (prof) {
        HIPCHK(c, hipEventRecord(ev[3], s));
        c->prof_count++;
        if (c->prof_pending < kProfSlots) c->prof_pending++;
    }
    return ASORA_OK;
}

extern "C" asora_status asora_raytrace_static(asora_ctx *c, const float *n_H, const float *x_HI, int64_t n_src,
                                              const int32_t *src_ijk, const double *src_Q, const float *src_R,
                                              float R_max, float *gamma, double *coldens_in, uint32_t flags,
                                              void *stream)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    asora_status st = check_common(c, n_H, x_HI, n_src, src_ijk, src_Q, R_max);
    if (st) return st;
    if (!gamma) return fail(c, ASORA_EINVAL, "gamma must not be NULL");
    if (coldens_in && n_src != 1) return fail(c, ASORA_EINVAL, "coldens_in requires n_src == 1");
    if (flags & ~(ASORA_ACCUMULATE | ASORA_PLAIN | ASORA_PROFILE | ASORA_EARLY_EXIT))
        return fail(c, ASORA_EINVAL, "asora_raytrace_static: flags may be ACCUMULATE, PLAIN, PROFILE, EARLY_EXIT");
    if (coldens_in && (flags & ASORA_EARLY_EXIT))
        return fail(c, ASORA_EINVAL, "ASORA_EARLY_EXIT does not give entry columns (coldens_in)");
    if (c->N > kStaticMaxN)
        return fail(c, ASORA_EINVAL, "asora_raytrace_static: N=%d exceeds the static scratch (N <= %d)", c->N,
                    kStaticMaxN);
    if (n_src > kStaticMaxSources)
        return fail(c, ASORA_EINVAL, "asora_raytrace_static: n_src=%lld exceeds the static scratch (<= %ld)",
                    (long long)n_src, kStaticMaxSources);
    if (!c->d_static) return fail(c, ASORA_ESTATE, "asora_raytrace_static: no static scratch on this device");
    HIPCHK(c, hipSetDevice(c->device));
    Plan plans[4];
    int tmax = 0;
    if ((st = forward_plans(c, R_max, false, plans, &tmax))) return st;
    char *base = c->d_static;
    const FwdBufs B{(double *)base, (double *)(base + kStaticGrid), (double *)(base + 2 * kStaticGrid),
                    (double *)(base + 3 * kStaticGrid), (int *)(base + kStaticOffCtl), (int *)(base + kStaticOffKeys),
                    (int *)(base + kStaticOffOrder)};
    return forward_launch(c, B, plans, tmax, n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max, gamma, nullptr,
                          coldens_in, flags, false, (hipStream_t)stream);
}

extern "C" asora_status asora_set_tuning(asora_ctx *c, float R_whole, float R_oct, int32_t max_waves,
                                         int32_t pyramid_sweep, int32_t table_place, int32_t adj_waves,
                                         int32_t adj_rate)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    const float w = R_whole > 0 ? R_whole : c->R_whole;
    const float o = R_oct > 0 ? R_oct : c->R_oct;
    if (!(o >= w) || !std::isfinite(w) || !std::isfinite(o) || max_waves > 16 ||
        !(pyramid_sweep == 0 || pyramid_sweep == 2 || pyramid_sweep == 3) || table_place < 0 ||
        table_place > 2 || adj_waves > kAdjLayerWaves || adj_rate < 0 || adj_rate > 2)
        return fail(c, ASORA_EINVAL,
                    "asora_set_tuning: need 0 < R_whole <= R_oct, max_waves <= 16, pyramid_sweep 0/2/3, "
                    "table_place 0/1/2, adj_waves <= %d, adj_rate 0/1/2", kAdjLayerWaves);
    if (c->live_graphs) return pinned(c, "the tuning");
    c->R_whole = w;
    c->R_oct = o;
    if (max_waves > 0) c->max_waves = max_waves;
    if (c->min_waves > c->max_waves) c->min_waves = c->max_waves;
    if (pyramid_sweep) c->big_kind = pyramid_sweep;
    if (table_place) c->tab_lds = table_place == 1 ? 1 : 0;
    if (adj_waves > 0) c->adj_waves = adj_waves;
    if (adj_rate) c->adj_split = adj_rate == 2 ? 1 : 0;
    c->plans.clear();
    c->adj_plans.clear();
    c->keep_valid = false;   // record layouts follow the plans
    return ASORA_OK;
}

extern "C" asora_status asora_get_tuning(const asora_ctx *c, float *R_whole, float *R_oct,
                                         int32_t *max_waves, int32_t *pyramid_sweep,
                                         int32_t *table_place, int32_t *adj_waves, int32_t *adj_rate)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (R_whole) *R_whole = c->R_whole;
    if (R_oct) *R_oct = c->R_oct;
    if (max_waves) *max_waves = c->max_waves;
    if (pyramid_sweep) *pyramid_sweep = c->big_kind;
    if (table_place) *table_place = c->tab_lds ? 1 : 2;
    if (adj_waves) *adj_waves = c->adj_waves;
    if (adj_rate) *adj_rate = c->adj_split ? 2 : 1;
    return ASORA_OK;
}

extern "C" asora_status asora_profile(asora_ctx *c, double *sweep_ms, double *total_ms)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (c->prof_count == 0) return fail(c, ASORA_ESTATE, "asora_profile: no profiled call yet");
    HIPCHK(c, hipSetDevice(c->device));
    hipEvent_t *ev = c->pev[(c->prof_count - 1) % kProfSlots];
    HIPCHK(c, hipEventSynchronize(ev[3]));
    float a = 0.f, b = 0.f;
    HIPCHK(c, hipEventElapsedTime(&a, ev[1], ev[2]));
    HIPCHK(c, hipEventElapsedTime(&b, ev[0], ev[3]));
    if (sweep_ms) *sweep_ms = a;
    if (total_ms) *total_ms = b;
    return ASORA_OK;
}

extern "C" asora_status asora_profile_read(asora_ctx *c, int32_t max_calls, int32_t *n_calls,
                                           double *sweep_ms, double *total_ms)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (max_calls < 0 || (max_calls > 0 && (!sweep_ms || !total_ms)))
        return fail(c, ASORA_EINVAL, "asora_profile_read: need max_calls >= 0 and both arrays");
    HIPCHK(c, hipSetDevice(c->device));
    const int n = c->prof_pending < max_calls ? c->prof_pending : max_calls;
    for (int i = 0; i < n; ++i) {   // output i = the (n-1-i)-th most recent call
        hipEvent_t *ev = c->pev[(c->prof_count - n + i) % kProfSlots];
        HIPCHK(c, hipEventSynchronize(ev[3]));
        float a = 0.f, b = 0.f;
        HIPCHK(c, hipEventElapsedTime(&a, ev[1], ev[2]));
        HIPCHK(c, hipEventElapsedTime(&b, ev[0], ev[3]));
        sweep_ms[i] = a;
        total_ms[i] = b;
    }
    if (n_calls) *n_calls = n;
    c->prof_pending = 0;
    return ASORA_OK;
}

// Adjoint plan: the forward plan's sizes with the adjoint's per-wave region.
static asora_status get_adj_plan(asora_ctx *c, int type, float R_cap, Plan *out)
{
    const int Rsq = (int)std::floor((double)R_cap * (double)R_cap);
    const PlanKey key{type, Rsq};
    auto it = c->adj_plans.find(key);
    if (it != c->adj_plans.end()) {
        *out = it->second;
        return ASORA_OK;
    }
    Plan P;
    asora_status st = get_plan(c, type, R_cap, &P);   // ring/row/cell sizes
    if (st) return st;
    if (P.row_cap > 256)
        return fail(c, ASORA_ENOSYS,
                    "asora_raytrace_backward: R_max=%.1f too large for the shell adjoint", R_cap);
    const size_t tab = (size_t)c->tp.n * sizeof(TabNode);
    const size_t region = adj_region_bytes(P.ring_cap, P.row_cap, P.Qmax);
    const long fit = c->max_lds > tab + 64 ? (long)((c->max_lds - tab - 64) / region) : 0;
    if (fit < 1)
        return fail(c, ASORA_ENOSYS,
                    "asora_raytrace_backward: R_max=%.1f needs %zu bytes of LDS per wave (limit %zu)",
                    R_cap, region + tab, c->max_lds);
    P.wave_mode = 1;
    P.scratch = 2 * P.piece_cells;   // exit and in-cell columns of a piece
    const int cap = c->max_waves < 8 ? c->max_waves : 8;   // adjoint work-groups: <= 512 threads
    P.waves = (int)(fit < cap ? fit : cap);
    P.lds = tab + (size_t)P.waves * region;
    int bpc = 0;
    HIPCHK(c, adj_occupancy(type, P.waves, P.lds, &bpc));
    P.grid = c->n_cu * (bpc > 0 ? bpc : 1);
    c->adj_plans[key] = P;
    *out = P;
    return ASORA_OK;
}

// Adjoint layer pieces: one layer buffer and a small queue per wave in LDS; a
// pyramid column record and the rate's entry-column terms in the wave's
// scratch.
static asora_status get_adj_layer_plan(asora_ctx *c, float R_cap, bool kept, Plan *out)
{
    const int Rsq = (int)std::floor((double)R_cap * (double)R_cap);
    const PlanKey key{kept ? 4 : 3, Rsq};
    auto it = c->adj_plans.find(key);
    if (it != c->adj_plans.end()) {
        *out = it->second;
        return ASORA_OK;
    }
    Plan P;
    asora_status st = get_layer_plan(c, R_cap, &P);   // Mcap, record sizes
    if (st) return st;
    const size_t region = adj_layer_region_bytes(P.S);
    const size_t sqb = layer_sqrt_bytes(Rsq);   // the work-group's table of square roots
    P.waves = layer_waves(c, 0, sqb, region, c->adj_waves, &P.sq_table);
    if (P.waves < 1)
        return fail(c, ASORA_ENOSYS,
                    "asora_raytrace_backward: R_max=%.1f needs %zu bytes of LDS per wave (limit %zu)",
                    R_cap, region, c->max_lds);
    P.lds = (P.sq_table ? sqb : 0) + (size_t)P.waves * region;
    int bpc = 0;
    HIPCHK(c, adj_layer_occupancy(kept, c->adj_split != 0, P.waves, P.lds, &bpc));
    P.grid = c->n_cu * (bpc > 0 ? bpc : 1);
    P.piece_cells = P.rec_cap;
    // the record, then g_in per cell (unused when the forward kept the records,
    // but sized alike, so that both forms run on the same buffers: a recorded
    // graph of one leaves room for eager calls of the other)
    P.scratch = (long)(P.rec_bytes / sizeof(double)) + P.rec_cap;
    c->adj_plans[key] = P;
    *out = P;
    return ASORA_OK;
}

static asora_status ensure_adj_layer_buffers(asora_ctx *c)
{
    asora_status st = ensure_layer_buffers(c);
    if (st) return st;
    if (c->d_gbar_T) return ASORA_OK;
    const size_t n3 = (size_t)c->N * c->N * c->N;
    HIPCHK(c, hipMalloc(&c->d_gbar_T, sizeof(double) * n3));
    if (hipMalloc(&c->d_nbar_T, sizeof(double) * n3) != hipSuccess) {
        (void)hipFree(c->d_gbar_T);
        c->d_gbar_T = nullptr;
        return fail(c, ASORA_ENOMEM, "allocation of the transposed adjoint buffers failed");
    }
    return ASORA_OK;
}

extern "C" asora_status asora_raytrace_backward(asora_ctx *c, const float *n_H, const float *x_HI,
                                                int64_t n_src, const int32_t *src_ijk,
                                                const double *src_Q, const float *src_R,
                                                float R_max, const double *dL_dgamma,
                                                float *dL_dnH, float *dL_dxHI, double *dL_dQ,
                                                uint32_t flags, void *stream)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    asora_status st = check_common(c, n_H, x_HI, n_src, src_ijk, src_Q, R_max);
    if (st) return st;
    if (!dL_dgamma || !dL_dnH || !dL_dxHI || (n_src > 0 && !dL_dQ))
        return fail(c, ASORA_EINVAL, "gradient buffers must not be NULL");
    if (flags & ~(ASORA_ACCUMULATE | ASORA_PROFILE | ASORA_STORE | ASORA_EARLY_EXIT))
        return fail(c, ASORA_EINVAL, "unknown flags");
    const bool prof = (flags & ASORA_PROFILE) != 0;
    const bool acc = (flags & ASORA_ACCUMULATE) != 0;
    const bool early = (flags & ASORA_EARLY_EXIT) != 0;
    hipEvent_t *ev = c->pev[c->prof_count % kProfSlots];
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const long n3 = (long)c->N * c->N * c->N;
    const int tbig = type_of(c, R_max);
    const int tmax = tbig == 2 ? c->big_kind : tbig;
    const bool layers = tmax == 3;
    // ASORA_STORE: the records kept by the forward call with these inputs
    // (and the same early-exit choice: records of an early-exit forward end at
    // the opaque layers)
    const bool kept = (flags & ASORA_STORE) && layers && c->keep_valid && c->keep_nsrc == n_src &&
                      c->keep_Rmax == R_max && c->keep_sig[0] == n_H && c->keep_sig[1] == x_HI &&
                      c->keep_sig[2] == src_ijk && c->keep_sig[3] == src_Q && c->keep_sig[4] == src_R &&
                      c->keep_early == early;
    Plan plans[4];
    size_t store_need = 0;
    for (int t = 0; t <= tmax; ++t) {
        if (t == 2 && layers) continue;
        const float cap = t == tmax ? R_max : (t == 0 ? c->R_whole : c->R_oct);
        if ((st = t == 3 ? get_adj_layer_plan(c, cap, kept, &plans[t]) : get_adj_plan(c, t, cap, &plans[t])))
            return st;
        size_t need = (size_t)plans[t].grid * plans[t].waves * (size_t)plans[t].scratch;
        if (t == 3) {   // room for the other form too (kept records or not): see get_adj_layer_plan
            Plan o;
            if ((st = get_adj_layer_plan(c, cap, !kept, &o))) return st;
            const size_t n2 = (size_t)o.grid * o.waves * (size_t)o.scratch;
            need = n2 > need ? n2 : need;
        }
        store_need = need > store_need ? need : store_need;
    }
    if ((st = ensure_src_cap(c, n_src))) return st;
    if (layers && (st = ensure_adj_layer_buffers(c))) return st;
    if (!c->d_nbar) HIPCHK(c, hipMalloc(&c->d_nbar, sizeof(double) * n3));
    if (store_need > c->store_cap) {
        if (c->live_graphs) return pinned(c, "the adjoint scratch");
        (void)hipFree(c->d_store);
        c->d_store = nullptr;
        c->store_cap = 0;
        HIPCHK(c, hipMalloc(&c->d_store, sizeof(double) * store_need));
        c->store_cap = store_need;
    }
    if (prof) HIPCHK(c, hipEventRecord(ev[0], s));
    // with the forward's records and its source order still in place (no
    // bucketing since), only the work counters are cleared and the order is
    // reused; otherwise the sources are bucketed again
    const bool reuse_order = kept && n_src > 0 && c->keep_order_gen == c->order_gen;
    // n_HI (both layouts) as the keeping forward left it, if nothing wrote it since
    const bool reuse_nhi = kept && c->keep_nhi_gen == c->nhi_gen;
    // dL/dQ accumulates over pieces: zero it unless the caller accumulates
    HIPCHK(c, launch_adj_prologue(s, n_H, x_HI, reuse_nhi ? nullptr : c->d_nhi, c->d_nbar, n3, dL_dQ, n_src,
                                  acc ? 0 : 1, c->d_ctl, reuse_order ? kCtlSeg : kCtlSize, c->n_cu));
    if (layers)
        HIPCHK(c, launch_adj_transpose_prologue(s, n_H, x_HI, dL_dgamma, reuse_nhi ? nullptr : c->d_nhi_T,
                                                c->d_gbar_T, c->d_nbar_T, c->N));
    if (!reuse_nhi) ++c->nhi_gen;
    if (n_src > 0 && !reuse_order) {
        HIPCHK(c, launch_bucketing(s, src_R, src_ijk, n_src, c->N, R_max, c->R_whole, c->R_oct,
                                   layers ? 3 : 2, c->d_keys, c->d_ctl, c->d_order, c->d_err));
        ++c->order_gen;
    }
    if (prof) HIPCHK(c, hipEventRecord(ev[1], s));
    if (n_src > 0) {
        AdjLaunch L;
        L.N = c->N;
        L.alpha = c->alpha;
        L.sigma0 = c->sigma0;
        L.tau_w = (float)c->tau_w;
        L.reading = c->reading;
        L.tp = c->tp;
        L.tab = c->d_tab;
        L.m64 = c->d_m64;
        L.nHI = c->d_nhi;
        L.gbar = dL_dgamma;
        L.nbar = c->d_nbar;
        L.qbar = dL_dQ;
        L.ijk = src_ijk;
        L.Q = src_Q;
        L.R = src_R;
        L.order = c->d_order;
        L.ctl = c->d_ctl;
        L.err = c->d_err;
        L.store = c->d_store;
        L.nHI_T = c->d_nhi_T;
        L.gbar_T = c->d_gbar_T;
        L.nbar_T = c->d_nbar_T;
        L.kept = kept ? c->d_keep : nullptr;
        L.rec_piece_bytes = layers ? (kept ? plans[3].keep_bytes : plans[3].rec_bytes) : 0;
        L.rec_rk_off = kept ? plans[3].rec_bytes : 0;
        L.rec_cap = layers ? plans[3].rec_cap : 0;
        L.split = c->adj_split != 0;
        L.early_exit = early;
        L.sq_table = layers && plans[3].sq_table;
        for (int t = tmax; t >= 0; --t) {
            if (t == 2 && layers) continue;
            L.type = t;
            L.R_cap = t == tmax ? R_max : (t == 0 ? c->R_whole : c->R_oct);
            L.ring_cap = plans[t].ring_cap;
            L.row_cap = plans[t].row_cap;
            L.shell_cap = plans[t].Qmax;
            L.waves = plans[t].waves;
            L.grid = plans[t].grid;
            L.store_stride = plans[t].scratch;
            if (t == 3) HIPCHK(c, launch_adj_layer(s, L, plans[3].Mcap, plans[3].S));
            else HIPCHK(c, launch_adj_wave(s, L));
        }
    }
    if (prof) HIPCHK(c, hipEventRecord(ev[2], s));
    if (layers)
        HIPCHK(c, launch_adj_transpose_finalize(s, c->d_nbar, c->d_nbar_T, n_H, x_HI, dL_dnH, dL_dxHI,
                                                c->N, acc ? 1 : 0));
    else
        HIPCHK(c, launch_adj_finalize(s, c->d_nbar, n_H, x_HI, dL_dnH, dL_dxHI, n3, acc ? 1 : 0,
                                      c->n_cu));
    if (prof) {
        HIPCHK(c, hipEventRecord(ev[3], s));
        c->prof_count++;
        if (c->prof_pending < kProfSlots) c->prof_pending++;
    }
    return ASORA_OK;
}

// ---------------------------------------------------------------------------
// Graphs: one step recorded once and replayed.
struct asora_graph {
    int magic;
    asora_ctx *ctx;
    hipGraph_t graph;
    hipGraphExec_t exec;
};
static const int kGraphMagic = 0x41475248;

extern "C" asora_status asora_graph_create(asora_ctx *c, const float *n_H, const float *x_HI,
                                           int64_t n_src, const int32_t *src_ijk, const double *src_Q,
                                           const float *src_R, float R_max, float *gamma,
                                           const double *dL_dgamma, float *dL_dnH, float *dL_dxHI,
                                           double *dL_dQ, uint32_t flags, asora_graph **out)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (!out) return fail(c, ASORA_EINVAL, "asora_graph_create: out is NULL");
    *out = nullptr;
    if (flags & ~(ASORA_ACCUMULATE | ASORA_PLAIN | ASORA_STORE | ASORA_EARLY_EXIT))
        return fail(c, ASORA_EINVAL, "asora_graph_create: flags may be ACCUMULATE, PLAIN, STORE, EARLY_EXIT");
    const bool adj = dL_dgamma != nullptr;
    const uint32_t ff = flags, bf = flags & (ASORA_ACCUMULATE | ASORA_STORE | ASORA_EARLY_EXIT);
    HIPCHK(c, hipSetDevice(c->device));
    // the inputs may still be in production on other streams
    HIPCHK(c, hipDeviceSynchronize());
    hipStream_t s = nullptr;
    HIPCHK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    auto step = [&]() -> asora_status {
        asora_status st = asora_raytrace(c, n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max, gamma,
                                         nullptr, ff, s);
        if (st || !adj) return st;
        return asora_raytrace_backward(c, n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max, dL_dgamma,
                                       dL_dnH, dL_dxHI, dL_dQ, bf, s);
    };
    // one eager step sizes every buffer, so that recording allocates nothing
    asora_status st = step();
    if (!st && hipStreamSynchronize(s) != hipSuccess) st = fail(c, ASORA_EHIP, "warm-up step failed");
    asora_graph *g = nullptr;
    if (!st) {
        g = new asora_graph();
        g->magic = kGraphMagic;
        g->ctx = c;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
            st = fail(c, ASORA_EHIP, "hipStreamBeginCapture failed");
        } else {
            st = step();
            hipGraph_t gr = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &gr);
            g->graph = gr;
            if (!st && (e != hipSuccess || !gr)) st = fail(c, ASORA_EHIP, "hipStreamEndCapture failed");
            if (!st && hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0) != hipSuccess)
                st = fail(c, ASORA_EHIP, "hipGraphInstantiate failed");
        }
    }
    (void)hipStreamDestroy(s);
    if (st) {
        if (g) {
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            if (g->graph) (void)hipGraphDestroy(g->graph);
            delete g;
        }
        (void)hipGetLastError();
        return st;
    }
    c->live_graphs++;
    *out = g;
    return ASORA_OK;
}

extern "C" asora_status asora_graph_launch(asora_graph *g, void *stream)
{
    if (!g || g->magic != kGraphMagic || !ctx_ok(g->ctx)) return ASORA_ESTATE;
    asora_ctx *c = g->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipGraphLaunch(g->exec, (hipStream_t)stream));
    return ASORA_OK;
}

extern "C" asora_status asora_graph_free(asora_graph *g)
{
    if (!g) return ASORA_OK;
    if (g->magic != kGraphMagic) return ASORA_ESTATE;
    asora_ctx *c = g->ctx;
    if (ctx_ok(c)) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        c->live_graphs--;
    }
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    g->magic = 0;
    delete g;
    return ASORA_OK;
}

// ---------------------------------------------------------------------------
// Tuning keys: the device, the grid, the number of sources, R_max, the pass
// count and a 64-bin histogram of the radii (FNV-1a hash of the counts), so
// that a tuning found once is reused for workloads of the same shape, in this
// process (the context's table) or across processes (asora_tuning_save /
// asora_tuning_load).
static asora_status tuning_key(asora_ctx *c, const float *src_R, int64_t n_src, float R_max, int passes,
                               void *stream, std::string *key)
{
    constexpr int kBins = 64;
    uint64_t cnt[kBins] = {};
    if (src_R && n_src > 0) {
        std::vector<float> R((size_t)n_src);
        HIPCHK(c, hipMemcpyAsync(R.data(), src_R, sizeof(float) * (size_t)n_src, hipMemcpyDeviceToHost,
                                 (hipStream_t)stream));
        HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
        for (float r : R) {
            int b = R_max > 0.f ? (int)((double)r / (double)R_max * kBins) : 0;
            b = b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
            cnt[b]++;
        }
    } else {
        cnt[kBins - 1] = (uint64_t)n_src;
    }
    uint64_t h = 1469598103934665603ull;
    for (int b = 0; b < kBins; ++b)
        for (int k = 0; k < 8; ++k) {
            h ^= (cnt[b] >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    char buf[256];
    snprintf(buf, sizeof buf, "%s/N%d/n%lld/R%.4f/h%016llx/p%d", c->dev_tag.c_str(), c->N, (long long)n_src,
             (double)R_max, (unsigned long long)h, passes);
    *key = buf;
    return ASORA_OK;
}

static const int kTuneVals = 8;   // the seven tuning values and the best time (ms)

// Entries of a tuning file: one per line, the key and kTuneVals numbers.
static bool read_tuning_file(const char *path, std::map<std::string, std::vector<float>> *out)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char key[300];
        float v[kTuneVals];
        if (sscanf(line, "%299s %f %f %f %f %f %f %f %f", key, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
                   &v[6], &v[7]) == 1 + kTuneVals)
            (*out)[key] = std::vector<float>(v, v + kTuneVals);
    }
    fclose(f);
    return true;
}

extern "C" asora_status asora_set_tune_progress(asora_ctx *c, asora_tune_progress_fn fn, void *user)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    c->tune_cb = fn;
    c->tune_cb_user = user;
    return ASORA_OK;
}

extern "C" asora_status asora_tuning_load(asora_ctx *c, const char *path, int32_t *n_loaded)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (!path) return fail(c, ASORA_EINVAL, "asora_tuning_load: path is NULL");
    std::map<std::string, std::vector<float>> m;
    if (n_loaded) *n_loaded = 0;
    if (!read_tuning_file(path, &m)) return ASORA_OK;   // no file yet: nothing known
    for (auto &kv : m) c->tuned[kv.first] = kv.second;
    if (n_loaded) *n_loaded = (int32_t)m.size();
    return ASORA_OK;
}

extern "C" asora_status asora_tuning_save(asora_ctx *c, const char *path)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (!path) return fail(c, ASORA_EINVAL, "asora_tuning_save: path is NULL");
    std::map<std::string, std::vector<float>> m;
    read_tuning_file(path, &m);   // entries of other workloads and devices stay
    for (auto &kv : c->tuned) m[kv.first] = kv.second;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return fail(c, ASORA_EINVAL, "asora_tuning_save: cannot write %s", tmp.c_str());
    fprintf(f, "# ASORA autotuner results: key (device:CUs/N/n_src/R_max/radius histogram/passes), "
               "R_whole R_oct max_waves pyramid_sweep table_place adj_waves adj_rate best_ms\n");
    for (auto &kv : m) {
        fprintf(f, "%s", kv.first.c_str());
        for (float v : kv.second) fprintf(f, " %.9g", (double)v);
        fprintf(f, "\n");
    }
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0)
        return fail(c, ASORA_EINVAL, "asora_tuning_save: cannot write %s", path);
    return ASORA_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate scheduling parameters on the caller's inputs and
// keeps the fastest.  Coordinate descent over the large-source sweep (layers,
// shells), the table's place, the waves per work-group, the layer adjoint's
// rate split and work-group size, and the whole / octant radius thresholds;
// each candidate is one warm-up call and the median of three timed calls.
constexpr int kTuneRow = 8;   // floats per report row
extern "C" asora_status asora_autotune(asora_ctx *c, const float *n_H, const float *x_HI,
                                       int64_t n_src, const int32_t *src_ijk, const double *src_Q,
                                       const float *src_R, float R_max, int32_t passes,
                                       uint32_t flags, void *stream, float *best_ms,
                                       int32_t max_report, int32_t *n_report, float *report)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    asora_status st = check_common(c, n_H, x_HI, n_src, src_ijk, src_Q, R_max);
    if (st) return st;
    if (passes != 1 && passes != 2) return fail(c, ASORA_EINVAL, "asora_autotune: passes must be 1 or 2");
    if (flags & ~ASORA_TUNE_RETUNE) return fail(c, ASORA_EINVAL, "asora_autotune: unknown flags");
    if (max_report < 0 || (max_report > 0 && !report))
        return fail(c, ASORA_EINVAL, "asora_autotune: need max_report >= 0 and a report array");
    if (c->live_graphs) return pinned(c, "the tuning");
    if (n_report) *n_report = 0;
    HIPCHK(c, hipSetDevice(c->device));
    std::string key;
    if ((st = tuning_key(c, src_R, n_src, R_max, passes, stream, &key))) return st;
    auto hit = c->tuned.find(key);
    if (hit != c->tuned.end() && !(flags & ASORA_TUNE_RETUNE)) {
        const std::vector<float> &v = hit->second;
        st = asora_set_tuning(c, v[0], v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5], (int)v[6]);
        if (!st && best_ms) *best_ms = v[7];
        return st;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t n3 = (size_t)c->N * c->N * c->N;
    float *gamma = nullptr, *dn = nullptr, *dx = nullptr;
    double *gb = nullptr, *dq = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        (void)hipFree(gamma);
        (void)hipFree(dn);
        (void)hipFree(dx);
        (void)hipFree(gb);
        (void)hipFree(dq);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    bool ok = hipMalloc(&gamma, sizeof(float) * n3) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
              hipEventCreate(&e1) == hipSuccess;
    if (ok && passes == 2) {
        ok = hipMalloc(&dn, sizeof(float) * n3) == hipSuccess && hipMalloc(&dx, sizeof(float) * n3) == hipSuccess &&
             hipMalloc(&gb, sizeof(double) * n3) == hipSuccess &&
             hipMalloc(&dq, sizeof(double) * (n_src > 0 ? n_src : 1)) == hipSuccess;
        if (ok) {   // dL/dGamma = 1 everywhere
            std::vector<double> ones(n3, 1.0);
            ok = hipMemcpy(gb, ones.data(), sizeof(double) * n3, hipMemcpyHostToDevice) == hipSuccess;
        }
    }
    if (!ok) {
        cleanup();
        return fail(c, ASORA_ENOMEM, "asora_autotune: scratch allocation failed");
    }
    const uint32_t sf = passes == 2 ? ASORA_STORE : 0;
    auto one = [&](uint32_t f) -> asora_status {
        asora_status r = asora_raytrace(c, n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max, gamma, nullptr,
                                        f, s);
        if (r || passes == 1) return r;
        return asora_raytrace_backward(c, n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max, gb, dn, dx, dq,
                                       f, s);
    };
    int nrep = 0;
    struct Cand {
        float w, o;
        int waves, sweep, place, aw, ar;
        bool operator==(const Cand &x) const
        {
            return w == x.w && o == x.o && waves == x.waves && sweep == x.sweep && place == x.place &&
                   aw == x.aw && ar == x.ar;
        }
    };
    auto apply = [&](const Cand &k) {
        return asora_set_tuning(c, k.w, k.o, k.waves, k.sweep, k.place, k.aw, k.ar);
    };
    // f: the step's flags; only steps of the tuned form (sf) enter the report
    auto trial = [&](const Cand &k, float *ms, uint32_t f) -> asora_status {
        asora_status r = apply(k);
        if (r) return r;
        if ((r = one(f))) return r;   // plans, buffers, warm caches
        float t[3];
        for (int i = 0; i < 3; ++i) {
            HIPCHK(c, hipEventRecord(e0, s));
            if ((r = one(f))) return r;
            HIPCHK(c, hipEventRecord(e1, s));
            HIPCHK(c, hipEventSynchronize(e1));
            HIPCHK(c, hipEventElapsedTime(&t[i], e0, e1));
        }
        std::sort(t, t + 3);
        *ms = t[1];
        const float v[kTuneRow] = {k.w, k.o, (float)k.waves, (float)k.sweep, (float)k.place,
                                   (float)k.aw, (float)k.ar, *ms};
        if (c->tune_cb) c->tune_cb(v, f == sf ? 1 : 0, c->tune_cb_user);
        if (f != sf) return ASORA_OK;
        if (nrep < max_report) std::copy(v, v + kTuneRow, report + kTuneRow * nrep);
        ++nrep;
        return ASORA_OK;
    };
    Cand b{c->R_whole, c->R_oct, c->max_waves, c->big_kind, c->tab_lds ? 1 : 2, c->adj_waves,
           c->adj_split ? 2 : 1};
    Cand k;
    // With the records kept (they fit) the tuned step's adjoint reads them and
    // does not use the rate form; the form serves the steps that recompute the
    // columns, so it is chosen on such steps, once, before the search, and
    // every candidate carries it.
    bool ar_fixed = false;
    if (passes == 2 && !(st = apply(b)) && !(st = one(sf)) && c->keep_valid) {
        float t_ar[2] = {0.f, 0.f};
        for (int ar : {1, 2})
            if (!st) (k = b).ar = ar, st = trial(k, &t_ar[ar - 1], 0u);
        if (!st) {
            b.ar = t_ar[0] <= t_ar[1] ? 1 : 2;
            ar_fixed = true;
        }
    }
    float best = 0.f;
    if (!st) st = trial(b, &best, sf);
    auto consider = [&](Cand k) -> asora_status {
        if (!(k.o >= k.w) || k == b) return ASORA_OK;
        float ms = 0.f;
        asora_status r = trial(k, &ms, sf);
        if (r) return r;
        if (ms < best) {
            best = ms;
            b = k;
        }
        return ASORA_OK;
    };
    if (!st && R_max > b.o)
        for (int sw : {3, 2})
            if (!st) (k = b).sweep = sw, st = consider(k);
    if (R_max > b.o && b.sweep == 3)
        for (int pl : {1, 2})
            if (!st) (k = b).place = pl, st = consider(k);
    for (int wv : {4, 8, 12, 16})
        if (!st) (k = b).waves = wv, st = consider(k);
    if (passes == 2 && R_max > b.o && b.sweep == 3) {   // the layer adjoint
        // the rate form and the work-group size jointly: the wide build's
        // register limit suits the gathered form and not the split one
        const Cand b0 = b;
        for (int aw : {2, 4, 8, 12, 16})
            for (int ar : {1, 2}) {
                if (st || (ar_fixed && ar != b0.ar)) continue;
                (k = b0).aw = aw, k.ar = ar, st = consider(k);
            }
    }
    if (R_max > 8.f)
        for (float o : {8.f, 10.f, 12.f, 15.f, 20.f})
            if (!st) (k = b).o = o, st = consider(k);
    for (float w : {3.f, 4.f, 6.f, 8.f})
        if (!st) (k = b).w = w, st = consider(k);
    cleanup();
    if (st) return st;
    if ((st = apply(b))) return st;
    c->tuned[key] = {b.w, b.o, (float)b.waves, (float)b.sweep, (float)b.place, (float)b.aw, (float)b.ar, best};
    if (best_ms) *best_ms = best;
    if (n_report) *n_report = nrep < max_report ? nrep : max_report;
    return ASORA_OK;
}

// ---------------------------------------------------------------------------
// Hydrogen chemistry (Section 2.1) and one time step of the ray-tracing <->
// chemistry iteration.

static constexpr double kNeRtol = 1e-12;   // n_e iteration: relative change of <y>
static constexpr int kNeMaxIter = 100;

static asora_status ensure_chem_counters(asora_ctx *c)
{
    if (!c->d_chem_cnt) HIPCHK(c, hipMalloc(&c->d_chem_cnt, 2 * sizeof(unsigned long long)));
    return ASORA_OK;
}

static asora_status chem_check(asora_ctx *c, double dt, double alpha_H, double C_H, double conv_rtol)
{
    if (!(dt >= 0.0) || !std::isfinite(dt) || !(alpha_H >= 0.0) || !std::isfinite(alpha_H) || !(C_H >= 0.0) ||
        !std::isfinite(C_H) || !(conv_rtol >= 0.0))
        return fail(c, ASORA_EINVAL, "chemistry: need dt, alpha_H, C_H, conv_rtol finite and >= 0");
    return ASORA_OK;
}

static asora_status chem_launch(asora_ctx *c, hipStream_t s, const float *gamma, const float *n_H,
                                const double *y0, const double *y_prev, double dt, double alpha_H, double C_H,
                                double conv_rtol, double *y_avg, double *y_end, float *y_avg32)
{
    ChemLaunch L;
    L.n = (long)c->N * c->N * c->N;
    L.gamma = gamma;
    L.nH = n_H;
    L.y0 = y0;
    L.y_prev = y_prev;
    L.y_avg = y_avg;
    L.y_end = y_end;
    L.y_avg32 = y_avg32;
    L.dt = dt;
    L.alpha = alpha_H;
    L.c_h = C_H;
    L.ne_rtol = kNeRtol;
    L.conv_rtol = conv_rtol;
    L.max_iter = kNeMaxIter;
    L.changed = c->d_chem_cnt;
    L.unconverged = c->d_chem_cnt + 1;
    L.n_cu = c->n_cu;
    HIPCHK(c, launch_chemistry(s, L));
    return ASORA_OK;
}

// the two counters, after waiting for the stream
static asora_status chem_counts(asora_ctx *c, hipStream_t s, unsigned long long out[2])
{
    HIPCHK(c, hipMemcpyAsync(out, c->d_chem_cnt, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (out[1]) return fail(c, ASORA_ERANGE, "chemistry: the n_e iteration of %llu cells did not converge", out[1]);
    return ASORA_OK;
}

extern "C" asora_status asora_chemistry(asora_ctx *c, const float *gamma, const float *n_H, const double *xHI_0,
                                        const double *xHI_avg_prev, double dt, double alpha_H, double C_H,
                                        double conv_rtol, double *xHI_avg, double *xHI_end, float *xHI_avg32,
                                        uint64_t *n_changed, void *stream)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (!gamma || !n_H || !xHI_0 || !xHI_avg || !xHI_end || !xHI_avg32)
        return fail(c, ASORA_EINVAL, "asora_chemistry: gamma, n_H, xHI_0 and the outputs must not be NULL");
    if (n_changed && !xHI_avg_prev)
        return fail(c, ASORA_EINVAL, "asora_chemistry: n_changed needs xHI_avg_prev");
    asora_status st = chem_check(c, dt, alpha_H, C_H, conv_rtol);
    if (st) return st;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_chem_counters(c))) return st;
    HIPCHK(c, launch_chem_clear(s, c->d_chem_cnt));
    if ((st = chem_launch(c, s, gamma, n_H, xHI_0, xHI_avg_prev, dt, alpha_H, C_H, conv_rtol, xHI_avg, xHI_end,
                          xHI_avg32)))
        return st;
    if (n_changed) {
        unsigned long long cnt[2];
        if ((st = chem_counts(c, s, cnt))) return st;
        *n_changed = cnt[0];
    }
    return ASORA_OK;
}

extern "C" asora_status asora_time_step(asora_ctx *c, const float *n_H, const double *xHI_0, int64_t n_src,
                                        const int32_t *src_ijk, const double *src_Q, const float *src_R,
                                        float R_max, double dt, double alpha_H, double C_H, double conv_rtol,
                                        double conv_frac, int32_t max_passes, int32_t fixed_passes,
                                        double *xHI_end, double *xHI_avg, float *gamma, int32_t *passes,
                                        void *stream)
{
    if (!ctx_ok(c)) return ASORA_ESTATE;
    if (!n_H || !xHI_0 || !xHI_end || !gamma)
        return fail(c, ASORA_EINVAL, "asora_time_step: n_H, xHI_0, xHI_end and gamma must not be NULL");
    asora_status st = chem_check(c, dt, alpha_H, C_H, conv_rtol);
    if (st) return st;
    if (!(conv_frac >= 0.0) || max_passes < 1 || fixed_passes < 0)
        return fail(c, ASORA_EINVAL, "asora_time_step: need conv_frac >= 0, max_passes >= 1, fixed_passes >= 0");
    if (c->live_graphs) return pinned(c, "the time-step buffers");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const long n3 = (long)c->N * c->N * c->N;
    if ((st = ensure_chem_counters(c))) return st;
    for (int k = 0; k < 2; ++k)
        if (!c->d_chem_y[k]) HIPCHK(c, hipMalloc(&c->d_chem_y[k], sizeof(double) * n3));
    if (!c->d_chem_y32) HIPCHK(c, hipMalloc(&c->d_chem_y32, sizeof(float) * n3));
    // <y> of the pass before: y0 at first; the ray tracing reads its FP32 copy
    int cur = 0;
    HIPCHK(c, launch_chem_prepare(s, n3, xHI_0, c->d_chem_y[cur], c->d_chem_y32, c->d_chem_cnt, c->n_cu));
    int pass = 0;
    for (;;) {
        if ((st = asora_raytrace(c, n_H, c->d_chem_y32, n_src, src_ijk, src_Q, src_R, R_max, gamma, nullptr, 0,
                                 stream)))
            return st;
        HIPCHK(c, launch_chem_clear(s, c->d_chem_cnt));
        if ((st = chem_launch(c, s, gamma, n_H, xHI_0, c->d_chem_y[cur], dt, alpha_H, C_H, conv_rtol,
                              c->d_chem_y[1 - cur], xHI_end, c->d_chem_y32)))
            return st;
        cur = 1 - cur;
        ++pass;
        if (fixed_passes > 0) {
            if (pass >= fixed_passes) break;
            continue;
        }
        unsigned long long cnt[2];
        if ((st = chem_counts(c, s, cnt))) return st;
        if ((double)cnt[0] <= conv_frac * (double)n3 || pass >= max_passes) break;
    }
    if (xHI_avg) HIPCHK(c, hipMemcpyAsync(xHI_avg, c->d_chem_y[cur], sizeof(double) * n3, hipMemcpyDeviceToDevice, s));
    if (passes) *passes = pass;
    if (fixed_passes > 0) {   // report a non-converged n_e iteration here too
        unsigned long long cnt[2];
        if ((st = chem_counts(c, s, cnt))) return st;
    }
    return ASORA_OK;
}
