/*
 * asora.h -- C ABI of the MI355X (gfx950) ASORA ray-tracing library.
 *
 * The library computes, for a set of point sources on a periodic cubic grid,
 * the hydrogen photoionization rate Gamma of every cell (eq. gamma / eq. sugg
 * of Section 2.2, summed over sources as in the multi-source paragraph of
 * Section 2.2), with the neutral-hydrogen column densities obtained by short
 * characteristics (Section 3.1) swept outward in octahedral shells
 * (Section 3.3, Appendix A), and the adjoint of that map.
 *
 * Conventions shared by every entry point:
 *   - Grids are N^3, C order [i][j][k] with k fastest, cell index
 *     (i*N + j)*N + k.  Units: cm, cm^-3, photons/s, s^-1, cm^-2.
 *   - "device" pointers are HIP device memory of the device given to
 *     asora_init; "host" pointers are ordinary host memory.  The caller owns
 *     every buffer it passes; the library only reads inputs and writes outputs
 *     and keeps no reference after the call returns.  The library owns its
 *     context, copies of the tables and its scratch memory.
 *   - Work is enqueued on the HIP stream passed as `stream` (a hipStream_t;
 *     NULL = the default stream) and is asynchronous: outputs are valid once
 *     that stream has reached the call.  A context must not be used from two
 *     streams or threads at the same time.
 *   - Argument errors are detected before anything is enqueued and returned
 *     as ASORA_EINVAL; nothing is written then.  Errors seen by the kernels
 *     (a source radius above the bound given to the call) are recorded in the
 *     context and reported by asora_check.  asora_last_error describes the
 *     most recent failure.
 */
#ifndef ASORA_H
#define ASORA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct asora_ctx asora_ctx;

typedef enum {
    ASORA_OK = 0,
    ASORA_EINVAL = -1,    /* invalid argument                                   */
    ASORA_ENOMEM = -2,    /* device or host allocation failed                   */
    ASORA_EHIP = -3,      /* a HIP runtime call failed                           */
    ASORA_ESTATE = -4,    /* context not usable (NULL, freed, wrong device)      */
    ASORA_ERANGE = -5,    /* a kernel met a source outside the call's bounds    */
    ASORA_ENOSYS = -6     /* combination of options not supported               */
} asora_status;

/* asora_init flags */
#define ASORA_INIT_SOURCE_HALFPATH_SCALAR 0x1u
/*   Column that a cell interpolating from the source cell sees for it.
 *   Default (flag clear): the exit column of the source cell along the cell's
 *   own ray, n_HI(s) alpha ds / 2 (exact on axes and diagonals).  With the
 *   flag: the scalar n_HI(s) alpha / 2.  The source cell itself always has
 *   entry column 0, path half a cell and volume alpha^3. */

/* asora_raytrace / asora_raytrace_backward flags */
#define ASORA_ACCUMULATE 0x1u  /* gamma += result (forward); gradients += (backward) */
#define ASORA_PROFILE    0x4u  /* record HIP events around the sweep kernels and the
                                  whole call on `stream`; read with asora_profile or
                                  asora_profile_read                                */
#define ASORA_STORE      0x8u  /* forward: keep the column record of every pyramid
                                  piece (sources above R_oct, swept in layers) in
                                  library-owned device memory, if it fits the store
                                  budget (asora_set_store_budget); otherwise nothing
                                  is kept (asora_store_info tells which); the records
                                  also hold the rate's FP64 derivatives for every cell
                                  with a rate.  backward: take the columns, the cells
                                  with a rate and those derivatives from the records
                                  instead of re-sweeping the pyramids forward and
                                  re-evaluating the rate, provided the most recent
                                  forward call with
                                  ASORA_STORE kept them for the same n_H, x_HI,
                                  src_ijk, src_Q, src_R pointers, n_src and R_max and
                                  the tuning has not changed since; otherwise the
                                  adjoint recomputes them.  The caller guarantees that
                                  the contents of those buffers did not change in
                                  between (if they did, the gradients are wrong, but
                                  every access stays inside the records).  Whole-source
                                  and octant pieces are always recomputed.  Results
                                  are the same either way up to rounding.            */
#define ASORA_EARLY_EXIT 0x10u /* forward: stop each layer pyramid (sources above
                                  R_oct, swept in layers) after its first layer whose
                                  cells all leave with sigma0 N_out >= tau_hi (a
                                  relative margin of 1e-12): every later cell of the
                                  pyramid enters at tau >= tau_hi, where the table is
                                  constant, so its rate is exactly zero (Section 2.2,
                                  the table's range; the photon-loss cut of Section
                                  3.3, made exact).  Gamma is the same as without the
                                  flag up to the order of floating-point sums; fewer
                                  cells are swept than the ball holds.  Not with
                                  coldens_in (later cells get no entry column).
                                  backward: the same stop in the adjoint's passes
                                  (no adjoint reaches a cell past such a layer, so
                                  the gradients are the same up to rounding).  Kept
                                  records are used only by a backward with the same
                                  choice as the forward that kept them.  Without
                                  the flag both passes sweep every layer.          */
#define ASORA_PLAIN      0x2u  /* one kernel launch per source, in input order: the
                                  unbatched baseline form (Section 3.3, one block per
                                  source).  Default: all sources in one persistent
                                  launch per piece kind, longest first.  Results are
                                  the same up to the order of floating-point sums.   */

/*
 * asora_max_sources -- the largest n_src one call accepts (host only, no GPU
 * use).  The persistent sweep kernels number their work items (source, piece)
 * in 32-bit integers with up to 24 pieces per source, so n_src is bounded by
 * INT32_MAX / 24; a call with more sources returns ASORA_EINVAL before
 * anything is enqueued (split the source list over several calls with
 * ASORA_ACCUMULATE: Gamma is a sum over sources, Section 2.2).
 */
int64_t asora_max_sources(void);

/*
 * asora_init -- create a context for one grid and one photoionization table.
 *
 * The table is P(tau) = gamma(tau/sigma0)/gamma(0), the number of ionizing
 * photons per second that survive an optical depth tau at the threshold
 * frequency, normalised to P(0) = 1 (eq. tables, Section 2.2), and its
 * derivative dP/dtau.  It is sampled on n_tab nodes uniform in log10 tau from
 * lg_tau_lo to lg_tau_hi.  Between nodes the library uses the cubic Hermite
 * spline of ln P in ln tau with node slopes tau P'/P ("a simple
 * interpolation", Section 2.2); below the first node the tangent line at the
 * first node; above the last node the constant P(tau_hi) (nothing absorbed
 * beyond the table).
 *
 *   out          host, receives the new context.
 *   N            grid size (cells per side), 1 <= N <= 1600 (N^3 < 2^32).
 *   cell_cm      cell size alpha in cm (> 0).
 *   sigma0_cm2   HI cross-section at the threshold (> 0); tau = sigma0 N_HI.
 *   lg_tau_lo, lg_tau_hi   log10 tau of the first and last node (lo < hi).
 *   n_tab        number of nodes, 2 <= n_tab <= 4096.
 *   P, dPdtau    host arrays of n_tab doubles; copied.  P must be positive,
 *                finite, non-increasing and representable as a normal FP32
 *                number (>= 1.2e-38); dPdtau finite and <= 0.
 *   tau_weight_floor   optical-depth floor of the interpolation weights
 *                w = s / max(sigma0 M, floor) (0.6 is the customary value);
 *                +INFINITY or 0 selects purely geometric weights.
 *   flags        ASORA_INIT_* flags.
 *   device       HIP device ordinal.
 * Allocates about 16 N^3 bytes of device memory (FP64 rate accumulator and
 * FP64 n_HI, the exact product of the FP32 inputs).  Returns ASORA_OK,
 * ASORA_EINVAL, ASORA_ENOMEM or ASORA_EHIP.
 */
asora_status asora_init(asora_ctx **out, int32_t N, double cell_cm, double sigma0_cm2,
                        double lg_tau_lo, double lg_tau_hi, int32_t n_tab, const double *P,
                        const double *dPdtau, double tau_weight_floor, uint32_t flags,
                        int32_t device);

/*
 * asora_raytrace -- photoionization rate of all cells from n_src sources.
 *
 * For each source s and each cell p with |p - s|^2 <= R_s^2 (in cells, the
 * hard photon radius of Section 3.2/3.3) inside the periodic extent
 * (Appendix A: at most N/2 cells on the negative and N/2-1 on the positive
 * side of the source on an even mesh, (N-1)/2 on both sides on an odd mesh):
 * interpolate the column N_in up to the entry face of p from the exit columns
 * of its four neighbours one layer closer to the source along the dominant
 * axis (eq. raga, eq. interp; bilinear geometric weights times optical-depth
 * weights), add the in-cell column n_HI alpha ds with ds = r/m (Section 3.1),
 * and add Gamma_p = Q_s [P(sigma0 N_in) - P(sigma0 N_out)] /
 * (n_HI V_shell), V_shell = 4 pi (alpha r)^2 alpha ds (eq. sugg), to gamma[p].
 * Cells are swept in shells of equal L1 distance from the source
 * (Section 3.3), which is a causal order for the interpolation.
 *
 *   n_H, x_HI    device, N^3 floats: total hydrogen density (cm^-3) and neutral
 *                fraction; n_HI = n_H x_HI.
 *   n_src        number of sources, 0 <= n_src <= asora_max_sources() (0 writes
 *                zeros / leaves gamma).
 *   src_ijk      device, n_src x 3 int32 cell indices in [0, N).
 *   src_Q        device, n_src doubles, ionizing photons per second (>= 0).
 *   src_R        device, n_src floats, radius in cells; NULL = R_max for all.
 *   R_max        host, an upper bound of every src_R (cells, 0 <= R_max <=
 *                4096).  Used to size on-chip buffers; a source with a larger
 *                radius is skipped and flagged (asora_check returns ERANGE).
 *   gamma        device, N^3 floats, output (s^-1); overwritten unless
 *                ASORA_ACCUMULATE.  Summation runs in FP64 and is rounded once.
 *   coldens_in   device, N^3 doubles or NULL.  Only with n_src == 1: receives
 *                N_in (cm^-2) for every cell of the ball, 0 elsewhere.
 *   flags        ASORA_ACCUMULATE | ASORA_PLAIN | ASORA_PROFILE | ASORA_STORE.
 *   stream       hipStream_t.
 */
asora_status asora_raytrace(asora_ctx *ctx, const float *n_H, const float *x_HI, int64_t n_src,
                            const int32_t *src_ijk, const double *src_Q, const float *src_R,
                            float R_max, float *gamma, double *coldens_in, uint32_t flags,
                            void *stream);

/*
 * asora_raytrace_static -- asora_raytrace for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): the call allocates nothing.  Its scratch (n_HI and
 * the FP64 rate accumulator in both layouts, work counters, source keys and
 * scheduling order) lives in a fixed-size device array of the library, about
 * 8.6 MiB, which every device the library runs on holds until the process
 * ends; the tables and parameters come from the context as asora_init made
 * them.  Limits: N <= 64 and n_src <= 65536; larger calls return ASORA_EINVAL
 * before anything is enqueued; on devices numbered 64 and above the call
 * returns ASORA_ESTATE (the library keeps the array's address for devices
 * 0 to 63).  The caller passes every input and output as
 * for asora_raytrace (same arguments and meaning).
 *   flags        ASORA_ACCUMULATE | ASORA_PLAIN | ASORA_PROFILE |
 *                ASORA_EARLY_EXIT (not ASORA_STORE: kept records need memory).
 * Every call on a device uses that device's one array and leaves its contents
 * there; the call clears what must start at zero itself.  Calls that overlap
 * on one device (several streams, threads or contexts) race on the array and
 * give wrong results; serialise them.  Results equal asora_raytrace's up to
 * the order of floating-point sums.
 */
asora_status asora_raytrace_static(asora_ctx *ctx, const float *n_H, const float *x_HI, int64_t n_src,
                                   const int32_t *src_ijk, const double *src_Q, const float *src_R,
                                   float R_max, float *gamma, double *coldens_in, uint32_t flags,
                                   void *stream);

/*
 * asora_set_heating_table -- give the context a photo-heating table: H(tau)
 * and dH/dtau (host arrays of the context's n_tab doubles, copied) on the
 * node grid of its photoionization table, for the same source spectrum, in
 * the energy unit the heating rate is wanted in (asora_table_blackbody_heat
 * builds it in eV).  H is the energy above the ionization threshold that the
 * photons still carry after optical depth tau, per emitted photon: the
 * energy analogue of the photon count P of eq. tables (Section 2.2).  The
 * paper computes photoionization only and names photo-heating as the next
 * extension (Sections 2 and 6).  Replaces an earlier heating table; waits for
 * the device first.  EINVAL for a NULL pointer or a node that is not positive,
 * >= 1.2e-38 and non-increasing with a finite slope <= 0.
 */
asora_status asora_set_heating_table(asora_ctx *ctx, const double *H, const double *dHdtau);

/*
 * asora_raytrace_heating -- asora_raytrace that also gives the photo-heating
 * rate per HI atom, from the same sweep: every cell whose rate is evaluated
 * also evaluates the heating table at the same optical depths,
 *   heating_p = Q_s [H(sigma0 N_in) - H(sigma0 N_out)] / (n_HI V_shell),
 * the energy its neutral hydrogen absorbs above threshold (eq. sugg with H in
 * place of P; the source cell as for the rate).  Two table lookups per cell,
 * one column computation.
 *
 *   n_H ... gamma, flags, stream: as for asora_raytrace (flags ASORA_ACCUMULATE
 *                | ASORA_PLAIN | ASORA_PROFILE | ASORA_STORE | ASORA_EARLY_EXIT;
 *                the kept records serve the rate's adjoint only; the early
 *                exit is exact for the heating too, which is also zero beyond
 *                the table's last node).
 *   heating      device, N^3 floats, output (heating-table energy unit per
 *                second per HI atom); overwritten unless ASORA_ACCUMULATE.
 *                FP64 accumulation, rounded once.
 * ESTATE without a heating table (asora_set_heating_table).  Scratch: 16 N^3
 * bytes more than asora_raytrace (two heating accumulators), allocated by
 * the first call.  Both tables are read through the caches by the layer
 * pieces (the table placement of asora_set_tuning does not apply).
 */
asora_status asora_raytrace_heating(asora_ctx *ctx, const float *n_H, const float *x_HI, int64_t n_src,
                                    const int32_t *src_ijk, const double *src_Q, const float *src_R,
                                    float R_max, float *gamma, float *heating, uint32_t flags,
                                    void *stream);

/*
 * asora_set_helium / asora_raytrace_helium -- the sweep with two absorbers,
 * HI and HeI (the extension the paper plans, Sections 2 and 6).
 *
 * The spectrum above 13.6 eV is split into bands (asora_table_blackbody_band
 * builds a black body's).  Band b has its own table P_b(T): the photons of the
 * band that survive an optical depth T measured at the band's lower edge, per
 * photon emitted above 13.6 eV, on n_tab nodes uniform in log10 T from
 * lg_lo[b] to lg_hi[b] (interpolated as the hydrogen table; constant beyond
 * the last node), and the cross-sections sigma_HI[b], sigma_HeI[b] (cm^2) of
 * the two species at that edge; inside a band both follow the band's
 * frequency shape, so its optical depth is sigma_HI[b] N_HI + sigma_HeI[b] N_HeI.
 * Both column densities are carried by the same short characteristics
 * (Section 3.1) with the weights of the hydrogen sweep (their optical-depth
 * factor on sigma0 N_HI: helium does not absorb at 13.6 eV).  A cell absorbs
 * Q [P_b(T_in) - P_b(T_out)] photons of band b, shared between the species in
 * proportion to their in-cell optical depths; a species' rate is its share
 * over n_i V (eq. sugg for each band), i.e. Q sum_b sigma_i[b] (-D_b) /
 * (4 pi alpha^2 r^2) with D_b the divided difference of P_b over the cell.
 *
 * asora_set_helium: n_bands in [1, 8]; lg_lo, lg_hi, sigma_HI, sigma_HeI host
 * arrays of n_bands; P, dPdtau host arrays of n_bands x n_tab (band-major),
 * with the rules of asora_init's table per band; copied (waits for the
 * device).  sigma_HI[b], sigma_HeI[b] >= 0, not both 0.  ASORA_EINVAL on
 * invalid input, ASORA_ESTATE while a recorded graph exists.
 *
 * asora_raytrace_helium: as asora_raytrace with, in addition, n_He (total
 * helium density, cm^-3) and x_HeI (its neutral fraction), device N^3 floats
 * (n_HeI = n_He x_HeI formed exactly in FP64), and two outputs gamma_HI,
 * gamma_HeI (device N^3 floats, s^-1, overwritten unless ASORA_ACCUMULATE;
 * FP64 accumulation).  Every source is swept as layer pyramids (no whole or
 * octant pieces); flags ASORA_ACCUMULATE | ASORA_PLAIN | ASORA_PROFILE.
 * ESTATE without band tables.  Scratch: 32 N^3 bytes more than
 * asora_raytrace (n_HeI and the HeI accumulator in both layouts), allocated
 * by the first call.
 */
asora_status asora_set_helium(asora_ctx *ctx, int32_t n_bands, int32_t n_tab, const double *lg_lo,
                              const double *lg_hi, const double *P, const double *dPdtau,
                              const double *sigma_HI, const double *sigma_HeI);
asora_status asora_raytrace_helium(asora_ctx *ctx, const float *n_H, const float *x_HI, const float *n_He,
                                   const float *x_HeI, int64_t n_src, const int32_t *src_ijk,
                                   const double *src_Q, const float *src_R, float R_max, float *gamma_HI,
                                   float *gamma_HeI, uint32_t flags, void *stream);

/*
 * asora_raytrace_backward -- adjoint of asora_raytrace.
 *
 * Given dL/dgamma, computes dL/dn_H, dL/dx_HI and dL/dQ of the forward map
 * with the same inputs (reverse mode through eq. sugg, the in-cell column
 * and the interpolation of eq. interp, with the optical-depth weights
 * differentiated as functions of the neighbour columns).  For every source
 * piece the exit columns are first recomputed into scratch memory (or, with
 * ASORA_STORE, taken from the records the forward kept), then the shells or
 * layers are swept from the outermost inward and every cell pushes the
 * adjoint of its entry column to its neighbours.
 *
 *   n_H, x_HI, n_src, src_ijk, src_Q, src_R, R_max: as for asora_raytrace.
 *   dL_dgamma    device, N^3 doubles (FP64: a cell's gradient can be a sum of
 *                large terms of both signs, so FP32 rounding of dL/dgamma
 *                would be amplified).
 *   dL_dnH, dL_dxHI   device, N^3 floats, outputs (overwritten unless
 *                ASORA_ACCUMULATE); accumulated in FP64, rounded once.
 *   dL_dQ        device, n_src doubles, output (overwritten unless
 *                ASORA_ACCUMULATE).
 *   flags        ASORA_ACCUMULATE | ASORA_PROFILE (asora_profile then reports
 *                the reverse sweep as sweep_ms) | ASORA_STORE (use the column
 *                records kept by the forward, see ASORA_STORE) |
 *                ASORA_EARLY_EXIT (stop each layer pyramid at its first opaque
 *                layer, see ASORA_EARLY_EXIT).
 * Scratch: about 16 N^3 bytes more than the forward, plus the stored columns
 * of the pieces in flight (allocated at the first call, grown on demand).
 * The derivative of the rate is taken on the interpolant as it is (a cubic
 * spline, so its second derivative is piecewise continuous); at exactly zero
 * n_HI the limit of the rate for vanishing in-cell optical depth is used.
 */
asora_status asora_raytrace_backward(asora_ctx *ctx, const float *n_H, const float *x_HI,
                                     int64_t n_src, const int32_t *src_ijk, const double *src_Q,
                                     const float *src_R, float R_max, const double *dL_dgamma,
                                     float *dL_dnH, float *dL_dxHI, double *dL_dQ,
                                     uint32_t flags, void *stream);

/*
 * asora_table_blackbody -- build P(tau) and dP/dtau for a black-body source of
 * temperature T_bb (K) behind a power-law cross-section sigma0 (nu/nu_th)^-index
 * (Section 4.1, Test 3), threshold h nu_th = 13.6 eV, on n nodes uniform in
 * log10 tau in [lg_lo, lg_hi]:
 *   P(tau)   = int_x0^inf phi(x) exp(-tau (x/x0)^-index) dx / int_x0^inf phi(x) dx
 *   P'(tau)  = -int_x0^inf phi(x) (x/x0)^-index exp(..) dx / (same)
 * with phi(x) = x^2/(e^x - 1) and x0 = 13.6 eV / (k T_bb).  Host only (no
 * GPU use); P, dPdtau are host arrays of n doubles.  Relative accuracy ~1e-12.
 */
asora_status asora_table_blackbody(double T_bb, double index, int32_t n, double lg_lo,
                                   double lg_hi, double *P, double *dPdtau);

/*
 * asora_table_blackbody_heat -- the photo-heating table of the same source:
 *   H(tau)  =  k T_bb int_x0^inf phi(x) (x - x0) exp(-tau (x/x0)^-index) dx / int_x0^inf phi(x) dx
 *   H'(tau) = -k T_bb int_x0^inf phi(x) (x - x0) (x/x0)^-index exp(..) dx / (same)
 * in eV, on the nodes of asora_table_blackbody with the same arguments.  Host
 * only; H, dHdtau are host arrays of n doubles.
 */
asora_status asora_table_blackbody_heat(double T_bb, double index, int32_t n, double lg_lo,
                                        double lg_hi, double *H, double *dHdtau);

/*
 * asora_table_blackbody_band -- one band [e_lo_eV, e_hi_eV) of the black body
 * of asora_table_blackbody, for several absorbers: the photons of the band
 * that survive an optical depth tau measured at the band's lower edge, with
 * the cross-section shape (nu / nu_lo)^-index inside the band, per photon
 * emitted above 13.6 eV, and its derivative:
 *   P_b(tau) = int_{x_lo}^{x_hi} phi(x) exp(-tau (x/x_lo)^-index) dx / int_x0^inf phi(x) dx.
 * The bands of a spectrum with tau_b = tau (e_b / 13.6 eV)^-index add up to
 * asora_table_blackbody's P(tau).  e_hi_eV = +INFINITY: an open band.  Host
 * only; P, dPdtau host arrays of n doubles.  ASORA_EINVAL unless
 * 13.6 <= e_lo_eV < e_hi_eV.
 */
asora_status asora_table_blackbody_band(double T_bb, double index, double e_lo_eV, double e_hi_eV, int32_t n,
                                        double lg_lo, double lg_hi, double *P, double *dPdtau);

/* asora_table_grey -- P = exp(-tau), dP/dtau = -exp(-tau) (grey opacity). */
asora_status asora_table_grey(int32_t n, double lg_lo, double lg_hi, double *P, double *dPdtau);

/*
 * asora_check -- wait for `stream` and report errors recorded by kernels since
 * the previous check (ASORA_ERANGE: a source radius exceeded the R_max of its
 * call, or a source index was outside the grid; that source was skipped).
 * Clears the record.
 */
asora_status asora_check(asora_ctx *ctx, void *stream);

/*
 * asora_store_info -- state of the kept column records: *valid = 1 if the
 * most recent forward call with ASORA_STORE kept them; *bytes_needed = what
 * that call needed (0 if it swept no pyramid pieces); *bytes_allocated = the
 * device memory held for them.  Any pointer may be NULL.
 */
asora_status asora_store_info(const asora_ctx *ctx, int32_t *valid, uint64_t *bytes_needed,
                              uint64_t *bytes_allocated);

/*
 * asora_set_store_budget -- largest number of bytes of device memory the kept
 * column records may take (n_src x 24 x one pyramid's record, about 32 bytes
 * per cell of the largest pyramid: its entry and room for the rate's three
 * derivatives).  0 (the default) means half of the free
 * device memory at the time of the forward call, plus what is already held.
 * A forward call with ASORA_STORE that needs more keeps nothing.
 */
asora_status asora_set_store_budget(asora_ctx *ctx, uint64_t bytes);

/*
 * asora_set_tuning -- scheduling parameters of the sweep (results do not
 * depend on them beyond the order of floating-point sums).  Sources with
 * R <= R_whole are swept whole by one wave; R_whole < R <= R_oct as eight
 * closed octants; larger R as 24 octant x dominant-axis pyramids (cells on
 * shared planes are computed by each piece and owned by one).  Those
 * pyramids are swept either shell by shell in L1 distance (pyramid_sweep 2)
 * or layer by layer along their dominant axis, each layer in chunks of 64
 * memory-contiguous cells (pyramid_sweep 3, the default), in the forward and
 * in the adjoint.  table_place: where the layer forward reads the table, 1 =
 * a copy in LDS per work-group (the default), 2 = through the caches (which
 * leaves the LDS to more waves).  max_waves (1..16) caps the waves per
 * work-group.  The adjoint of layer pyramids: adj_waves (1..16, default 4)
 * waves per work-group (above 12 a build held to four waves per SIMD, which
 * may spill registers); adj_rate 1 = the rate terms of every cell with a rate
 * gathered into full waves before the reverse pass (fewer registers: suits
 * sources whose rate reaches few cells), 2 = those of chunks where at least
 * half the cells have a rate evaluated in the reverse pass itself (the
 * default: suits sources that ionise most of their sphere); it applies when
 * the adjoint re-sweeps the pyramids (records kept with ASORA_STORE carry the
 * rate's derivatives).  Values <= 0
 * keep the current setting.  ASORA_EINVAL if R_oct < R_whole, max_waves > 16,
 * pyramid_sweep is not 0, 2 or 3, table_place not 0, 1 or 2, adj_waves > 16
 * or adj_rate not 0, 1 or 2; ASORA_ESTATE while a recorded graph of the
 * context exists.
 */
asora_status asora_set_tuning(asora_ctx *ctx, float R_whole, float R_oct, int32_t max_waves,
                              int32_t pyramid_sweep, int32_t table_place, int32_t adj_waves,
                              int32_t adj_rate);

/* asora_autotune flags */
#define ASORA_TUNE_RETUNE 0x1u  /* time again even if this workload was tuned before */

/*
 * asora_autotune -- pick the scheduling parameters of asora_set_tuning by
 * timing candidates on the given inputs (the sources' independence, Section
 * 2.2, leaves the order and grouping of the work free; this chooses it by
 * measurement, not by rule).  Coordinate descent over: the sweep of pyramid
 * pieces (layers, shells), the place of the table (LDS, caches), the waves
 * per work-group (4, 8, 12, 16), for passes = 2 with layer pyramids the
 * layer adjoint's adj_rate (1, 2) jointly with adj_waves (2, 4, 8, 12, 16), R_oct (8, 10,
 * 12, 15, 20) and R_whole (3, 4, 6, 8); every candidate is one
 * warm-up call and the median of three calls timed with HIP events on
 * `stream`.  passes = 1 times the forward; passes = 2 the forward with
 * ASORA_STORE followed by the adjoint (with dL/dgamma = 1).  The best
 * candidate is kept in the context (asora_get_tuning reads it) and cached
 * under a key of the workload's shape: the device (name and compute-unit
 * count), N, n_src, R_max, passes and a 64-bin histogram of the radii.  A
 * later call with the same key sets the cached parameters without timing,
 * unless flags has ASORA_TUNE_RETUNE; asora_tuning_load fills that cache from
 * a file.  The key is formed on the host from a copy of src_R (the call
 * waits for `stream` for it).
 *
 *   n_H .. R_max  as for asora_raytrace (device buffers; only read).
 *   passes        1 or 2.
 *   best_ms       host, may be NULL: time of the best candidate (ms).
 *   report        host array of max_report x 8 floats (may be NULL when
 *                 max_report = 0): per timed candidate R_whole, R_oct,
 *                 max_waves, pyramid_sweep, table_place, adj_waves, adj_rate,
 *                 ms; *n_report (may be NULL) receives the number of rows
 *                 written.
 * Allocates scratch outputs of the size of the grid for its duration and
 * waits for `stream`.  ASORA_ESTATE while a recorded graph of the context
 * exists.
 */
asora_status asora_autotune(asora_ctx *ctx, const float *n_H, const float *x_HI, int64_t n_src,
                            const int32_t *src_ijk, const double *src_Q, const float *src_R,
                            float R_max, int32_t passes, uint32_t flags, void *stream,
                            float *best_ms, int32_t max_report, int32_t *n_report, float *report);

/*
 * asora_set_tune_progress -- a host function that asora_autotune calls after
 * every candidate it has timed, on the calling thread: row = the candidate's
 * R_whole, R_oct, max_waves, pyramid_sweep, table_place, adj_waves, adj_rate
 * and its time in ms (host array of 8 floats, valid during the call);
 * in_report = 1 if the candidate is of the tuned form (it enters the report),
 * 0 for the preliminary choice of adj_rate.  fn = NULL removes it.  For
 * callers that show the progress of a long tuning run.
 */
typedef void (*asora_tune_progress_fn)(const float *row, int32_t in_report, void *user);
asora_status asora_set_tune_progress(asora_ctx *ctx, asora_tune_progress_fn fn, void *user);

/*
 * asora_tuning_save / asora_tuning_load -- keep autotuner results across
 * processes, so that a workload tuned once is not searched again (the search
 * itself is asora_autotune).
 * The file is text, one line per key: the key of asora_autotune and eight
 * numbers (R_whole R_oct max_waves pyramid_sweep table_place adj_waves
 * adj_rate best_ms); lines starting with '#' are comments.
 *   save  writes every result the context holds into `path` (host string),
 *         keeping the file's entries of other keys; written to path".tmp"
 *         and renamed.  ASORA_EINVAL if the file cannot be written.
 *   load  adds the file's entries to the context's cache (a missing file
 *         adds nothing and is not an error); *n_loaded (may be NULL)
 *         receives their number.  The tuning in force changes only when
 *         asora_autotune later meets one of these keys.
 * Host only (no GPU use).
 */
asora_status asora_tuning_save(asora_ctx *ctx, const char *path);
asora_status asora_tuning_load(asora_ctx *ctx, const char *path, int32_t *n_loaded);

/*
 * asora_graph_create -- record one ray-tracing step into a HIP graph owned
 * by the library, to be replayed with asora_graph_launch: asora_raytrace with
 * the given arguments (no column output) and, if dL_dgamma is not NULL,
 * asora_raytrace_backward right after it (flags ASORA_ACCUMULATE and
 * ASORA_STORE carried over).  The step is first run once eagerly on a
 * private stream (this sizes every library buffer, so that recording
 * allocates nothing; it writes the outputs), then recorded.  A replay reads
 * the inputs' current contents and writes the same outputs; every buffer
 * given here must stay allocated while the graph exists.  While a graph of a
 * context exists, a call that would have to grow one of the context's
 * buffers (more sources, a larger R_max, kept records of another size, a
 * retuning) fails with ASORA_ESTATE instead.
 *
 *   flags   ASORA_ACCUMULATE | ASORA_PLAIN | ASORA_STORE (not ASORA_PROFILE).
 *   out     host, receives the graph.
 */
typedef struct asora_graph asora_graph;
asora_status asora_graph_create(asora_ctx *ctx, const float *n_H, const float *x_HI, int64_t n_src,
                                const int32_t *src_ijk, const double *src_Q, const float *src_R,
                                float R_max, float *gamma, const double *dL_dgamma, float *dL_dnH,
                                float *dL_dxHI, double *dL_dQ, uint32_t flags, asora_graph **out);

/* asora_graph_launch -- replay the recorded step on `stream` (asynchronous). */
asora_status asora_graph_launch(asora_graph *graph, void *stream);

/* asora_graph_free -- wait for the device and release the graph.  NULL is
 * accepted.  Free every graph of a context before the context. */
asora_status asora_graph_free(asora_graph *graph);

/*
 * asora_get_tuning -- the current scheduling parameters (any pointer may be
 * NULL).
 */
asora_status asora_get_tuning(const asora_ctx *ctx, float *R_whole, float *R_oct,
                              int32_t *max_waves, int32_t *pyramid_sweep, int32_t *table_place,
                              int32_t *adj_waves, int32_t *adj_rate);

/*
 * asora_profile -- durations (ms) of the most recent call made with
 * ASORA_PROFILE on ctx: sweep_ms covers the ray-tracing sweep kernels only
 * (all piece kinds; for ASORA_PLAIN every per-source launch), total_ms the
 * whole call (n_HI and accumulator set-up, scheduling sort, sweep, final
 * conversion).  Waits for those events.  Either pointer may be NULL.
 * ASORA_ESTATE if no profiled call was made.
 */
asora_status asora_profile(asora_ctx *ctx, double *sweep_ms, double *total_ms);

/*
 * asora_profile_read -- the same two durations (ms) for every call made with
 * ASORA_PROFILE since the previous asora_profile_read, oldest first, into the
 * host arrays sweep_ms[max_calls] and total_ms[max_calls].  The library keeps
 * the events of the 64 most recent profiled calls; when more calls are pending
 * than max_calls (or than 64), the most recent ones are returned.  *n_calls
 * (may be NULL) receives the count written.  Waits for those events, so a
 * timed loop of profiled calls can be read once at its end without a wait per
 * call.  Afterwards no call is pending.  ASORA_EINVAL if max_calls < 0, or
 * max_calls > 0 with a NULL array.
 */
asora_status asora_profile_read(asora_ctx *ctx, int32_t max_calls, int32_t *n_calls,
                                double *sweep_ms, double *total_ms);

/*
 * asora_chemistry -- the hydrogen chemistry step (Section 2.1, eq. chemistry
 * and eq. time_avrg_sol): for every cell, the time-averaged solution of
 * dx/dt = (1 - x)(Gamma + n_e C_H) - x n_e alpha_H over a step dt with Gamma,
 * n_e, C_H and alpha_H held fixed, the electron density iterated as
 * n_e = n_H <x> (starting from n_H x0) until <x> changes by at most 1e-12
 * relative (100 passes at most).  Everything is in the neutral fraction
 * x_HI = 1 - x (y below): y_eq = n_e alpha_H t_i, t_i = 1 / (Gamma +
 * n_e (C_H + alpha_H)), <y> = y_eq + (y0 - y_eq)(1 - e^(-dt/t_i)) t_i/dt,
 * y(dt) = y_eq + (y0 - y_eq) e^(-dt/t_i), FP64.  With xHI_avg_prev the n_e
 * iteration starts from it instead (the same fixed point, in fewer passes).
 *
 *   gamma        device, N^3 FP32: the time-averaged photoionization rate
 *                (s^-1; what asora_raytrace returns).
 *   n_H          device, N^3 FP32 (cm^-3).
 *   xHI_0        device, N^3 FP64: the neutral fraction at the start of the step.
 *   xHI_avg_prev device, N^3 FP64, may be NULL: the <y> of the previous pass of
 *                the ray-tracing <-> chemistry iteration, for n_changed.
 *   dt           the step (s); alpha_H, C_H: recombination and collisional
 *                ionization coefficients (cm^3 s^-1), the same in every cell.
 *   conv_rtol    a cell counts as changed when |<y> - prev| > conv_rtol <y>.
 *   xHI_avg      device, N^3 FP64 out: <y>;  xHI_end: y(dt);  xHI_avg32:
 *                <y> in FP32, the next ray tracing's x_HI.
 *   n_changed    host, may be NULL (then nothing waits): the number of
 *                changed cells; the call then waits for `stream`.
 * All outputs are written on `stream`.  ASORA_EINVAL for NULL buffers,
 * negative or non-finite dt / coefficients; ASORA_ERANGE if the n_e iteration
 * of some cell did not converge (only reported when the call waits).
 */
asora_status asora_chemistry(asora_ctx *ctx, const float *gamma, const float *n_H, const double *xHI_0,
                             const double *xHI_avg_prev, double dt, double alpha_H, double C_H,
                             double conv_rtol, double *xHI_avg, double *xHI_end, float *xHI_avg32,
                             uint64_t *n_changed, void *stream);

/*
 * asora_time_step -- one time step of the ray-tracing <-> chemistry
 * iteration (Section 2.1, the flowchart): the ray tracing (asora_raytrace on
 * the sources, no flags) runs on the time-averaged neutral fraction <y>
 * (the start-of-step xHI_0 the first time), the chemistry step
 * (asora_chemistry) turns the summed rate into a new <y>, and the two
 * alternate.  With fixed_passes > 0 exactly that many passes run; otherwise
 * until at most conv_frac N^3 cells changed <y> by more than conv_rtol
 * relative, or max_passes passes.  The photoionization rate is assumed
 * constant over the step (the paper's time-averaged rate).
 *
 *   n_H          device, N^3 FP32; xHI_0: device, N^3 FP64.
 *   sources      as for asora_raytrace (device buffers; R_max bounds src_R).
 *   dt, alpha_H, C_H, conv_rtol   as for asora_chemistry.
 *   xHI_end      device, N^3 FP64 out: the neutral fraction at the end of the step.
 *   xHI_avg      device, N^3 FP64 out, may be NULL: the converged <y>.
 *   gamma        device, N^3 FP32 out: the last pass's rate.
 *   passes       host, may be NULL: the passes made.
 * Holds two FP64 and one FP32 grid of its own in the context.  Waits for
 * `stream` after every pass (the convergence count) unless fixed_passes > 0.
 * ASORA_EINVAL for bad arguments; ASORA_ESTATE while a recorded graph of the
 * context exists; errors of asora_raytrace and asora_chemistry pass through.
 */
asora_status asora_time_step(asora_ctx *ctx, const float *n_H, const double *xHI_0, int64_t n_src,
                             const int32_t *src_ijk, const double *src_Q, const float *src_R, float R_max,
                             double dt, double alpha_H, double C_H, double conv_rtol, double conv_frac,
                             int32_t max_passes, int32_t fixed_passes, double *xHI_end, double *xHI_avg,
                             float *gamma, int32_t *passes, void *stream);

/* asora_last_error -- text of the most recent error on ctx (or of the most
 * recent failed asora_init when ctx is NULL).  Owned by the library. */
const char *asora_last_error(const asora_ctx *ctx);

/* asora_free -- release the context and its device memory (waits for the
 * device).  NULL is accepted.  ASORA_ESTATE (nothing freed) while a recorded
 * graph of the context exists. */
asora_status asora_free(asora_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* ASORA_H */
