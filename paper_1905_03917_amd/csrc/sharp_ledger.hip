// sharp_ledger.hip -- conservation ledger: the total content
// sum_c dV (alpha U)_k of every fluid and component (the quantity whose
// drift the paper reports for its conservation checks, Sec. 4.2), by a
// fixed-order two-pass tree reduction on the device (deterministic: the
// same state gives the same bits).
#include <hip/hip_runtime.h>

#include <mutex>

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

// Scratch of the allocation-free ledger (sim_totals_noalloc): the partial
// sums of the fixed grid and the ten totals, whatever the grid size.  One
// copy per device, held until the process ends; every call on a device
// shares it (calls that overlap on one device race).  Host code never passes
// this name to a kernel or a copy: it reaches the array only through the
// device address hipGetSymbolAddress returns (scratch_ptr).
constexpr int SCRATCH_DOUBLES = 10 * LEDGER_BLOCKS + 10;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[MAX_DEVICES] = {nullptr};

}  // namespace

// Device address of this device's scratch array, looked up once per device
// with that device current.  Called by sim_create for the simulation's
// device.
sim_status ledger_scratch_attach(int device)
{
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("device %d: the allocation-free ledger supports devices 0..%d", device, MAX_DEVICES - 1);
        return SIM_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[device]) return SIM_OK;
    int cur = -1;
    SHARP_HIP(hipGetDevice(&cur));
    if (cur != device) SHARP_HIP(hipSetDevice(device));
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
        set_error("hipGetSymbolAddress of the ledger scratch failed: %s", hipGetErrorString(e));
        return SIM_EDEVICE;
    }
    scratch_ptr[device] = static_cast<double*>(p);
    return SIM_OK;
}

// sim_totals through the device's scratch array: the same kernels, grid and
// summation order as engine_totals (so the same bits), no allocation.  With
// on_device the totals are written to out10 on the simulation's stream and
// nothing waits; otherwise they are copied to the host array out10.
sim_status engine_totals_noalloc(Sim& s, double* out10, int on_device)
{
    static_assert(SCRATCH_DOUBLES >= 10 * LEDGER_BLOCKS + 10, "ledger scratch too small for its fixed grid");
    if (s.device < 0 || s.device >= MAX_DEVICES) {
        set_error("no ledger scratch for device %d", s.device);
        return SIM_EDEVICE;
    }
    double* buf = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        buf = scratch_ptr[s.device];
    }
    if (!buf) {
        set_error("the ledger scratch of device %d was not set up", s.device);
        return SIM_ESTATE;
    }
    Dev& g = s.g;
    const int nv = g.D + 2;
    double dv = 1.0;
    for (int d = 0; d < g.D; d++) dv *= g.h;
    double* tot = on_device ? out10 : buf + 10 * LEDGER_BLOCKS;
    k_ledger_partial<<<LEDGER_BLOCKS, LEDGER_WG, 0, s.stream>>>(g, nv, buf);
    k_ledger_final<<<1, 64, 0, s.stream>>>(buf, LEDGER_BLOCKS, dv, tot);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && !on_device) {
        e = hipMemcpyAsync(out10, tot, sizeof(double) * 10, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    }
    if (e != hipSuccess) {
        set_error("allocation-free ledger failed: %s", hipGetErrorString(e));
        return SIM_EDEVICE;
    }
    return SIM_OK;
}

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
