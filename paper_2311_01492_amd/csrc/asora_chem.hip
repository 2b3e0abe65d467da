// Hydrogen chemistry step (Section 2.1): the time-averaged solution of the
// chemistry equation over a step dt for the time-averaged rate Gamma, with
// the electron density iterated per cell.  Elementwise over the grid: 44
// bytes per cell move (Gamma, n_H FP32; y0, the previous <y> FP64 in; <y>,
// y(dt) FP64 and <y> FP32 out), one thread per cell, grid-stride; the FP64
// exponentials of the n_e passes, not the bytes, set its time.
//
// Carried in the neutral fraction y = 1 - x_HII:
//   rate = Gamma + n_e (C_H + alpha_H),  y_eq = n_e alpha_H / rate,
//   <y>  = y_eq + (y0 - y_eq) (1 - e^-u) / u,  y(dt) = y_eq + (y0 - y_eq) e^-u,
//   u = rate dt,  n_e = n_H (1 - <y>), starting from n_H (1 - y0).
#include <hip/hip_runtime.h>

#include "asora_internal.h"

namespace asora {

namespace {

constexpr int kChemThreads = 256;

struct ChemArgs {
    long n;
    const float *gamma, *nH;
    const double *y0, *y_prev;
    double *y_avg, *y_end;
    float *y_avg32;
    double dt, alpha, c_h, ne_rtol, conv_rtol;
    int max_iter;
    unsigned long long *changed;   // cells whose <y> moved by more than conv_rtol relative (may be NULL)
    unsigned long long *unconverged;   // cells whose n_e iteration hit max_iter
};

__device__ __forceinline__ void time_average(double gamma, double n_e, double y0, double dt, double alpha,
                                             double c_h, double &y_avg, double &y_end)
{
    const double rate = gamma + n_e * (c_h + alpha);
    const double y_eq = rate > 0.0 ? n_e * alpha / rate : 1.0;
    const double u = rate * dt;
    // (1 - e^-u) / u without cancellation for small u; 1 at u = 0
    const double frac = u > 0.0 ? -expm1(-u) / u : 1.0;
    y_avg = y_eq + (y0 - y_eq) * frac;
    y_end = y_eq + (y0 - y_eq) * exp(-u);
}

__global__ __launch_bounds__(kChemThreads) void chem_kernel(ChemArgs A)
{
    unsigned int changed = 0, unconverged = 0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < A.n; i += (long)gridDim.x * blockDim.x) {
        const double g = (double)A.gamma[i], nH = (double)A.nH[i], y0 = A.y0[i];
        // n_e from the previous pass's <y> when there is one: the same fixed
        // point, reached in fewer passes
        double ya = A.y_prev ? A.y_prev[i] : y0, ye = y0;
        int it = 0;
        for (; it < A.max_iter; ++it) {
            double a, e;
            time_average(g, nH * (1.0 - ya), y0, A.dt, A.alpha, A.c_h, a, e);
            const bool done = fabs(a - ya) <= A.ne_rtol * a;
            ya = a;
            ye = e;
            if (done) break;
        }
        if (it == A.max_iter) ++unconverged;
        A.y_avg[i] = ya;
        A.y_end[i] = ye;
        A.y_avg32[i] = (float)ya;
        if (A.y_prev && fabs(ya - A.y_prev[i]) > A.conv_rtol * ya) ++changed;
    }
    // one atomic per wave for each count
    unsigned int c = changed, u = unconverged;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        u += __shfl_xor(u, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (A.changed && c) atomicAdd(A.changed, (unsigned long long)c);
        if (u) atomicAdd(A.unconverged, (unsigned long long)u);
    }
}

// Start of a time step: <y> := y0 (FP64 copy and FP32 for the ray tracing);
// counters cleared (by a kernel: no memset node if the caller records it).
__global__ __launch_bounds__(kChemThreads) void chem_prepare_kernel(long n, const double *y0, double *y_avg,
                                                                    float *y_avg32, unsigned long long *cnt)
{
    if (blockIdx.x == 0 && threadIdx.x < 2) cnt[threadIdx.x] = 0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double y = y0[i];
        if (y_avg) y_avg[i] = y;
        y_avg32[i] = (float)y;
    }
}

__global__ void chem_clear_kernel(unsigned long long *cnt)
{
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_chem_prepare(hipStream_t st, long n, const double *y0, double *y_avg, float *y_avg32,
                               unsigned long long *cnt, int n_cu)
{
    long blocks = (n + kChemThreads - 1) / kChemThreads;
    if (blocks > (long)n_cu * 16) blocks = (long)n_cu * 16;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(chem_prepare_kernel, dim3((unsigned)blocks), dim3(kChemThreads), 0, st, n, y0, y_avg,
                       y_avg32, cnt);
    return hipGetLastError();
}

hipError_t launch_chem_clear(hipStream_t st, unsigned long long *cnt)
{
    hipLaunchKernelGGL(chem_clear_kernel, dim3(1), dim3(64), 0, st, cnt);
    return hipGetLastError();
}

hipError_t launch_chemistry(hipStream_t st, const ChemLaunch &L)
{
    ChemArgs A;
    A.n = L.n;
    A.gamma = L.gamma;
    A.nH = L.nH;
    A.y0 = L.y0;
    A.y_prev = L.y_prev;
    A.y_avg = L.y_avg;
    A.y_end = L.y_end;
    A.y_avg32 = L.y_avg32;
    A.dt = L.dt;
    A.alpha = L.alpha;
    A.c_h = L.c_h;
    A.ne_rtol = L.ne_rtol;
    A.conv_rtol = L.conv_rtol;
    A.max_iter = L.max_iter;
    A.changed = L.changed;
    A.unconverged = L.unconverged;
    long blocks = (L.n + kChemThreads - 1) / kChemThreads;
    const long cap = (long)L.n_cu * 16;   // grid-stride beyond 16 work-groups per CU
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(chem_kernel, dim3((unsigned)blocks), dim3(kChemThreads), 0, st, A);
    return hipGetLastError();
}

}  // namespace asora
