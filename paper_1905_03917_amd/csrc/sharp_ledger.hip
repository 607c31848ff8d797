// sharp_ledger.hip -- conservation ledger: the total content
// sum_c dV (alpha U)_k of every fluid and component (the quantity whose
// drift the paper reports for its conservation checks, Sec. 4.2), by a
// fixed-order two-pass tree reduction on the device (deterministic: the
// same state gives the same bits).
#include <hip/hip_runtime.h>

#include "sharp_internal.h"

namespace sharp {

namespace {

constexpr int LEDGER_WG = 256;
constexpr int LEDGER_BLOCKS = 512;   // fixed grid: the summation order does not depend on the device

// pass 1: block b sums the cells of its contiguous chunk for every (fluid,
// component) and writes 10 partial sums
__global__ void __launch_bounds__(LEDGER_WG) k_ledger_partial(Dev g, int nv, double* part)
{
    __shared__ double sred[LEDGER_WG / 64][10];
    const long long chunk = ((long long)g.nc + gridDim.x - 1) / gridDim.x;
    const long long lo = blockIdx.x * chunk, hi = lo + chunk < g.nc ? lo + chunk : g.nc;
    double acc[10];
#pragma unroll
    for (int j = 0; j < 10; j++) acc[j] = 0.0;
    for (long long c = lo + threadIdx.x; c < hi; c += blockDim.x)
        for (int k = 0; k < 2; k++)
            for (int q = 0; q < nv; q++) acc[k * 5 + q] += g.X[k][(size_t)q * g.nc + c];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 10; j++) {
        double v = acc[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sred[wid][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        double v = 0.0;
        for (int w = 0; w < LEDGER_WG / 64; w++) v += sred[w][threadIdx.x];
        part[(size_t)blockIdx.x * 10 + threadIdx.x] = v;
    }
}

// pass 2: one thread per (fluid, component) sums the partials in block order
__global__ void k_ledger_final(const double* part, int nblocks, double dv, double* out)
{
    const int j = threadIdx.x;
    if (j >= 10) return;
    double v = 0.0;
    for (int b = 0; b < nblocks; b++) v += part[(size_t)b * 10 + j];
    out[j] = v * dv;
}

}  // namespace

sim_status engine_totals(Sim& s, double* out10)
{
    Dev& g = s.g;
    const int nv = g.D + 2;
    double* buf = nullptr;
    if (hipMalloc((void**)&buf, sizeof(double) * (10 * LEDGER_BLOCKS + 10)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("ledger allocation failed");
        return SIM_ENOMEM;
    }
    double dv = 1.0;
    for (int d = 0; d < g.D; d++) dv *= g.h;
    k_ledger_partial<<<LEDGER_BLOCKS, LEDGER_WG, 0, s.stream>>>(g, nv, buf);
    k_ledger_final<<<1, 64, 0, s.stream>>>(buf, LEDGER_BLOCKS, dv, buf + 10 * LEDGER_BLOCKS);
    hipError_t e = hipMemcpyAsync(out10, buf + 10 * LEDGER_BLOCKS, sizeof(double) * 10, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    (void)hipFree(buf);
    if (e != hipSuccess) {
        set_error("ledger readback failed: %s", hipGetErrorString(e));
        return SIM_EDEVICE;
    }
    return SIM_OK;
}

}  // namespace sharp
