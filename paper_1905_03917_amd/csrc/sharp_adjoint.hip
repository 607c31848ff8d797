// sharp_adjoint.hip -- reverse-mode derivative (adjoint) of single-dt runs
// in which one fluid fills the grid: the Shu-Osher stages (Sec. 2.1, Sec. 3)
// of the finite-volume update with the WENO5 flux under local Lax-Friedrichs
// splitting, and the stiffened-gas EOS.  The step lengths are frozen at
// their forward values.
//
// Forward tape: the state of the fluid every `ckpt_every` steps and each
// step's length.  Backward: per segment (last first), the stage states are
// recomputed from the segment's checkpoint with the forward stage kernel,
// then the reverse sweep runs through them.  One stage
//     U_s = a_s U_0 + (1 - a_s) (U_{s-1} + dt L(U_{s-1}))
// reverses to
//     lam_0 += a_s lam_s,   lam_{s-1} = (1 - a_s) lam_s + J_L(U_{s-1})^T mu,
//     mu = (1 - a_s) dt lam_s,
// and J_L^T mu is evaluated face by face: with L_c = sum_d (F_lo - F_hi)/h
// the flux of face f receives (mu_right - mu_left)/h, and the face's
// vector-Jacobian product is written per stencil slot, then gathered per
// cell in a fixed order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "sharp_internal.h"

namespace sharp {

namespace {

constexpr int ADJ_WG = 256;
constexpr int ADJ_BLOCKS = 1024;   // fixed grid of the kernels with per-block parameter partials

const double ADJ_RK3_A[3] = {0.0, 0.75, 1.0 / 3.0};
const double ADJ_RK2_A[2] = {0.0, 0.5};

// reverse of the WENO5-JS value w(v0..v4) (left-biased, at the right edge
// of v2): vb += gb * dw/dv.  With candidate values q_k, smoothness
// indicators b_k, e_k = eps + b_k, alpha_k = d_k / e_k^2 and omega_k =
// alpha_k / sum(alpha):
//   dw/dv = sum_k omega_k dq_k/dv - 2 sum_k omega_k (q_k - w) / e_k db_k/dv.
__host__ __device__ __forceinline__ void weno5_vjp(const double* v, double eps, double gb, double* vb)
{
    const double c13_12 = 13.0 / 12.0, c13_6 = 13.0 / 6.0;
    double q0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) * (1.0 / 6.0);
    double q1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) * (1.0 / 6.0);
    double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) * (1.0 / 6.0);
    double t0 = v[0] - 2.0 * v[1] + v[2], u0 = v[0] - 4.0 * v[1] + 3.0 * v[2];
    double t1 = v[1] - 2.0 * v[2] + v[3], u1 = v[1] - v[3];
    double t2 = v[2] - 2.0 * v[3] + v[4], u2 = 3.0 * v[2] - 4.0 * v[3] + v[4];
    double e0 = eps + c13_12 * t0 * t0 + 0.25 * u0 * u0;
    double e1 = eps + c13_12 * t1 * t1 + 0.25 * u1 * u1;
    double e2 = eps + c13_12 * t2 * t2 + 0.25 * u2 * u2;
    double a0 = 0.1 / (e0 * e0), a1 = 0.6 / (e1 * e1), a2 = 0.3 / (e2 * e2);
    double S = a0 + a1 + a2;
    double w0 = a0 / S, w1 = a1 / S, w2 = a2 / S;
    double w = w0 * q0 + w1 * q1 + w2 * q2;
    // candidate values at fixed weights
    double g0 = gb * w0 * (1.0 / 6.0), g1 = gb * w1 * (1.0 / 6.0), g2 = gb * w2 * (1.0 / 6.0);
    vb[0] += 2.0 * g0;
    vb[1] += -7.0 * g0 - g1;
    vb[2] += 11.0 * g0 + 5.0 * g1 + 2.0 * g2;
    vb[3] += 2.0 * g1 + 5.0 * g2;
    vb[4] += -g2;
    // weights through the smoothness indicators
    double c0 = -2.0 * gb * w0 * (q0 - w) / e0;
    double c1 = -2.0 * gb * w1 * (q1 - w) / e1;
    double c2 = -2.0 * gb * w2 * (q2 - w) / e2;
    // b0 = 13/12 t0^2 + 1/4 u0^2, t0 ~ (1,-2,1), u0 ~ (1,-4,3)
    double x0 = c13_6 * t0 * c0, y0 = 0.5 * u0 * c0;
    vb[0] += x0 + y0;
    vb[1] += -2.0 * x0 - 4.0 * y0;
    vb[2] += x0 + 3.0 * y0;
    // b1: t1 ~ (0,1,-2,1,0), u1 ~ (0,1,0,-1,0)
    double x1 = c13_6 * t1 * c1, y1 = 0.5 * u1 * c1;
    vb[1] += x1 + y1;
    vb[2] += -2.0 * x1;
    vb[3] += x1 - y1;
    // b2: t2 ~ (0,0,1,-2,1), u2 ~ (0,0,3,-4,1)
    double x2 = c13_6 * t2 * c2, y2 = 0.5 * u2 * c2;
    vb[2] += x2 + 3.0 * y2;
    vb[3] += -2.0 * x2 - 4.0 * y2;
    vb[4] += x2 + y2;
}

// Reverse of one face flux along d (LLF splitting, WENO5 per component) of
// the six stencil states U[m] (cells -3..+2 from the face), for the upstream
// flux weights Fb.  Adds dF/dU^T Fb to Ub and the partials with respect to
// gamma and p_inf (U fixed) to *gb, *pb.
// (the direction is a template parameter: with every index static the
// stencil arrays stay in registers)
template <int D, int DIR>
__host__ __device__ __forceinline__ void face_vjp(const double (*U)[D + 2], double gm, double pi, double eps,
                                                  const double* Fb, double (*Ub)[D + 2], double* gb, double* pb)
{
    constexpr int NV = D + 2;
    constexpr int d = DIR;
    double rho[6], vel[6][D], E[6], p[6], c[6], un[6], ke[6];
    double amax = -1.0;
    int ms = 0;
#pragma unroll
    for (int m = 0; m < 6; m++) {
        rho[m] = U[m][0];
        double k2 = 0.0;
#pragma unroll
        for (int e = 0; e < D; e++) {
            vel[m][e] = U[m][1 + e] / rho[m];
            k2 += vel[m][e] * vel[m][e];
        }
        ke[m] = 0.5 * rho[m] * k2;
        E[m] = U[m][NV - 1];
        p[m] = (gm - 1.0) * (E[m] - ke[m]) - gm * pi;
        c[m] = sqrt(gm * (p[m] + pi) / rho[m]);
        un[m] = vel[m][d];
        double s = fabs(un[m]) + c[m];
        if (s > amax) { amax = s; ms = m; }
    }
    const double a = amax;
    double Fp[6][NV], Ud[6][NV], ab = 0.0;
#pragma unroll
    for (int m = 0; m < 6; m++)
#pragma unroll
        for (int q = 0; q < NV; q++) { Fp[m][q] = 0.0; Ud[m][q] = 0.0; }
#pragma unroll
    for (int q = 0; q < NV; q++) {
        double F[6];
#pragma unroll
        for (int m = 0; m < 6; m++) {
            if (q == 0) F[m] = U[m][1 + d];
            else if (q == NV - 1) F[m] = (E[m] + p[m]) * un[m];
            else F[m] = U[m][q] * un[m] + ((q - 1) == d ? p[m] : 0.0);
        }
        double vp[5], vm[5], bp[5] = {0, 0, 0, 0, 0}, bm[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 5; j++) {
            vp[j] = 0.5 * (F[j] + a * U[j][q]);               // f+ at cells 0..4
            vm[j] = 0.5 * (F[5 - j] - a * U[5 - j][q]);       // f- at cells 5..1
        }
        weno5_vjp(vp, eps, Fb[q], bp);
        weno5_vjp(vm, eps, Fb[q], bm);
#pragma unroll
        for (int j = 0; j < 5; j++) {
            Fp[j][q] += 0.5 * bp[j];
            Ud[j][q] += 0.5 * a * bp[j];
            ab += 0.5 * U[j][q] * bp[j];
            Fp[5 - j][q] += 0.5 * bm[j];
            Ud[5 - j][q] -= 0.5 * a * bm[j];
            ab -= 0.5 * U[5 - j][q] * bm[j];
        }
    }
#pragma unroll
    for (int m = 0; m < 6; m++) {
        double unb = 0.0, pbm = 0.0, cb = 0.0, rb = 0.0;
        if (m == ms) {
            unb += (un[m] > 0.0 ? 1.0 : (un[m] < 0.0 ? -1.0 : 0.0)) * ab;
            cb += ab;
        }
        // physical flux
        Ub[m][1 + d] += Fp[m][0];
#pragma unroll
        for (int e = 0; e < D; e++) {
            Ub[m][1 + e] += Fp[m][1 + e] * un[m];
            unb += Fp[m][1 + e] * U[m][1 + e];
        }
        pbm += Fp[m][1 + d];
        Ub[m][NV - 1] += Fp[m][NV - 1] * un[m];
        pbm += Fp[m][NV - 1] * un[m];
        unb += Fp[m][NV - 1] * (E[m] + p[m]);
        // c = sqrt(gamma (p + p_inf) / rho)
        double ic = 1.0 / (2.0 * rho[m] * c[m]);
        pbm += cb * gm * ic;
        rb += -cb * c[m] / (2.0 * rho[m]);
        *gb += cb * (p[m] + pi) * ic;
        *pb += cb * gm * ic;
        // u_n = m_d / rho
        Ub[m][1 + d] += unb / rho[m];
        rb += -unb * un[m] / rho[m];
        // p = (gamma - 1)(E - ke) - gamma p_inf, ke = |m|^2 / (2 rho)
        Ub[m][NV - 1] += pbm * (gm - 1.0);
        double k2 = 0.0;
#pragma unroll
        for (int e = 0; e < D; e++) {
            Ub[m][1 + e] += -pbm * (gm - 1.0) * vel[m][e];
            k2 += vel[m][e] * vel[m][e];
        }
        rb += pbm * (gm - 1.0) * 0.5 * k2;
        *gb += pbm * (E[m] - ke[m] - pi);
        *pb += -pbm * gm;
        Ub[m][0] += rb;
#pragma unroll
        for (int q = 0; q < NV; q++) Ub[m][q] += Ud[m][q];
    }
}

__device__ __forceinline__ void block_add_pair(double x, double y, double* acc)
{
    __shared__ double sx[ADJ_WG / 64], sy[ADJ_WG / 64];
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_down(x, off, 64);
        y += __shfl_down(y, off, 64);
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sx[wid] = x; sy[wid] = y; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < ADJ_WG / 64; w++) { x += sx[w]; y += sy[w]; }
        acc[2 * blockIdx.x] += x;       // this block's slot: launches add in stream order
        acc[2 * blockIdx.x + 1] += y;
    }
}

// face lattice normal to d: n[e] + (e == d) faces per direction e
__device__ __forceinline__ void face_coords(const Dev& g, int d, long long f, int* fc)
{
    int n0 = g.n[0] + (d == 0), n1 = g.n[1] + (d == 1);
    fc[0] = (int)(f % n0);
    fc[1] = (int)((f / n0) % n1);
    fc[2] = (int)(f / ((long long)n0 * n1));
}

__device__ __forceinline__ long long face_index(const Dev& g, int d, const int* fc)
{
    long long n0 = g.n[0] + (d == 0), n1 = g.n[1] + (d == 1);
    return fc[0] + n0 * (fc[1] + n1 * (long long)fc[2]);
}

// two waves per SIMD (a few spills) measured 3% faster than one without
template <int D, int DIR>
__global__ void __launch_bounds__(ADJ_WG, 2) k_adj_face(Dev g, int k, const double* U, const double* lam,
                                                     double scale, double* fb, double* pacc)
{
    constexpr int NV = D + 2;
    constexpr int d = DIR;
    const long long nf = (long long)(g.n[0] + (d == 0)) * (g.n[1] + (d == 1)) * (g.n[2] + (d == 2));
    const double gm = g.gam[k], pi = g.pinf[k];
    double gsum = 0.0, psum = 0.0;
    for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nf; f += (long long)gridDim.x * blockDim.x) {
        int fc[3];
        face_coords(g, d, f, fc);
        const int x = fc[d], n = g.n[d];
        int cc[3] = {fc[0], fc[1], fc[2]};
        double Fb[NV];
        const int cr = x < n ? cc[0] + g.n[0] * (cc[1] + g.n[1] * cc[2]) : -1;
        cc[d] = x - 1;
        const int cl = x > 0 ? cc[0] + g.n[0] * (cc[1] + g.n[1] * cc[2]) : -1;
#pragma unroll
        for (int q = 0; q < NV; q++)
            Fb[q] = scale * ((cr >= 0 ? lam[(size_t)q * g.nc + cr] : 0.0) - (cl >= 0 ? lam[(size_t)q * g.nc + cl] : 0.0));
        double Us[6][NV], Ub[6][NV];
#pragma unroll
        for (int m = 0; m < 6; m++) {
            cc[d] = x - 3 + m;
            int c = cidx(g, cc[0], cc[1], cc[2]);
#pragma unroll
            for (int q = 0; q < NV; q++) {
                Us[m][q] = U[(size_t)q * g.nc + c];
                Ub[m][q] = 0.0;
            }
        }
        face_vjp<D, DIR>(Us, gm, pi, g.eps, Fb, Ub, &gsum, &psum);
        double* o = fb + (size_t)f * 6 * NV;
#pragma unroll
        for (int m = 0; m < 6; m++)
#pragma unroll
            for (int q = 0; q < NV; q++) o[m * NV + q] = Ub[m][q];
    }
    block_add_pair(gsum, psum, pacc);
}

// v (+)= sum over the faces normal to d of the slots that map to each cell:
// the in-grid positions first (faces x+3 .. x-2), then, near the grid ends,
// the positions outside the grid whose boundary image is the cell
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj_gather(Dev g, int d, const double* fb, double* v, int accumulate)
{
    constexpr int NV = D + 2;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        int cc[3];
        coords(g, c, cc[0], cc[1], cc[2]);
        const int x = cc[d], n = g.n[d];
        double acc[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) acc[q] = 0.0;
        int fc[3] = {cc[0], cc[1], cc[2]};
        for (int m = 0; m < 6; m++) {
            int fd = x + 3 - m;
            if (fd < 0 || fd > n) continue;
            fc[d] = fd;
            const double* s = fb + ((size_t)face_index(g, d, fc) * 6 + m) * NV;
#pragma unroll
            for (int q = 0; q < NV; q++) acc[q] += s[q];
        }
        if (x < 3 || x > n - 4) {
            for (int fd = 0; fd <= n; fd++) {
                if (fd >= 3 && fd <= n - 3) { fd = n - 3; continue; }
                fc[d] = fd;
                for (int m = 0; m < 6; m++) {
                    int pos = fd - 3 + m;
                    if (pos >= 0 && pos < n) continue;
                    if (bcmap(pos, n, g.bc[d]) != x) continue;
                    const double* s = fb + ((size_t)face_index(g, d, fc) * 6 + m) * NV;
#pragma unroll
                    for (int q = 0; q < NV; q++) acc[q] += s[q];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NV; q++) {
            size_t e = (size_t)q * g.nc + c;
            v[e] = accumulate ? v[e] + acc[q] : acc[q];
        }
    }
}

// stage combination of the reverse sweep (element-wise over NV*cells):
// top (s = last stage) starts lam0; the first stage folds everything into lam
__global__ void __launch_bounds__(ADJ_WG) k_adj_comb(long long n, double* lam, double* lam0, const double* v,
                                                     double a, double w, int top, int first)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        double l = lam[e];
        double l0 = (top ? 0.0 : lam0[e]) + a * l;
        if (first) lam[e] = l0 + w * l + v[e];
        else { lam[e] = w * l + v[e]; lam0[e] = l0; }
    }
}

// reverse of the initial map prim -> cons (rho u, E = (p + gamma p_inf)/(gamma - 1) + rho |u|^2 / 2)
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj_prim0(Dev g, int k, const double* W, const double* lam, double* gp,
                                                      double* pacc)
{
    constexpr int NV = D + 2;
    const double gm = g.gam[k], pi = g.pinf[k];
    double gsum = 0.0, psum = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        double rho = W[c], p = W[(size_t)(NV - 1) * g.nc + c];
        double lE = lam[(size_t)(NV - 1) * g.nc + c];
        double r = lam[c], k2 = 0.0;
#pragma unroll
        for (int e = 0; e < D; e++) {
            double u = W[(size_t)(1 + e) * g.nc + c], lm = lam[(size_t)(1 + e) * g.nc + c];
            r += lm * u;
            k2 += u * u;
            gp[(size_t)(1 + e) * g.nc + c] = lm * rho + lE * rho * u;
        }
        gp[c] = r + lE * 0.5 * k2;
        gp[(size_t)(NV - 1) * g.nc + c] = lE / (gm - 1.0);
        gsum += -lE * (p + pi) / ((gm - 1.0) * (gm - 1.0));
        psum += lE * gm / (gm - 1.0);
    }
    block_add_pair(gsum, psum, pacc);
}

template <int D>
struct Adjoint {
    static constexpr int NV = D + 2;
    Sim& s;
    Dev& g;
    explicit Adjoint(Sim& sim) : s(sim), g(sim.g) {}

    static int blocks(long long n)
    {
        long long b = (n + ADJ_WG - 1) / ADJ_WG;
        return (int)(b < 1 ? 1 : (b > 65535 ? 65535 : b));
    }

    // v = J_L(U)^T (scale * lam), per direction through the face buffer
    void jlt(int k, const double* U, const double* lam, double scale, double* v, double* fb, double* pacc)
    {
        for (int d = 0; d < D; d++) {
            if (d == 0)
                k_adj_face<D, 0><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, U, lam, scale / g.h, fb, pacc);
            if constexpr (D > 1)
                if (d == 1) k_adj_face<D, 1><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, U, lam, scale / g.h, fb, pacc);
            if constexpr (D > 2)
                if (d == 2) k_adj_face<D, 2><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, U, lam, scale / g.h, fb, pacc);
            k_adj_gather<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, d, fb, v, d > 0);
        }
    }

    sim_status run(const double* g_cons, double* g_prim0, double* g_eos)
    {
        std::vector<void*> own;
        sim_status rc = sweep(g_cons, g_prim0, g_eos, own);
        (void)hipStreamSynchronize(s.stream);
        for (void* p : own) (void)hipFree(p);
        return rc;
    }

    sim_status sweep(const double* g_cons, double* g_prim0, double* g_eos, std::vector<void*>& own)
    {
        const int k = s.tape_fluid;
        const int ns = s.o.rk;
        const double* A = ns == 3 ? ADJ_RK3_A : ADJ_RK2_A;
        const size_t nv = (size_t)NV * g.nc;
        const long long N = (long long)s.tape_dt.size();
        const int K = s.o.ckpt_every;
        g.use_sched = 0;   // stage lengths come from the tape
        long long nfmax = 0;
        for (int d = 0; d < D; d++)
            nfmax = std::max(nfmax, (long long)(g.n[0] + (d == 0)) * (g.n[1] + (d == 1)) * (g.n[2] + (d == 2)));
        // buffers: the stage inputs of one segment (ns per step), lam, lam0,
        // v, the face buffer (6 NV per face), the per-block parameter partials
        const size_t nstore = (size_t)std::min<long long>(N > 0 ? N : 1, K) * ns;
        auto alloc = [&](size_t bytes) -> double* {
            void* p = nullptr;
            if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
            own.push_back(p);
            return (double*)p;
        };
        double* store = alloc(sizeof(double) * nv * nstore);
        double* lam = alloc(sizeof(double) * nv);
        double* lam0 = alloc(sizeof(double) * nv);
        double* v = alloc(sizeof(double) * nv);
        double* fb = alloc(sizeof(double) * (size_t)nfmax * 6 * NV);
        double* pacc = alloc(sizeof(double) * 2 * ADJ_BLOCKS);
        if (!store || !lam || !lam0 || !v || !fb || !pacc) {
            set_error("adjoint buffers do not fit in device memory (%zu MB for the recomputed stages)",
                      sizeof(double) * nv * nstore >> 20);
            return SIM_ENOMEM;
        }
        SHARP_HIP(hipMemsetAsync(pacc, 0, sizeof(double) * 2 * ADJ_BLOCKS, s.stream));
        SHARP_HIP(hipMemcpyAsync(lam, g_cons + (size_t)k * nv, sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
        const long long nseg = (N + K - 1) / K;
        for (long long seg = nseg - 1; seg >= 0; seg--) {
            const long long s0 = seg * K, s1 = std::min(N, s0 + K);
            // recompute the stage inputs U_0 .. U_{ns-1} of every step of the
            // segment with the forward stage kernel (bit-identical)
            SHARP_HIP(hipMemcpyAsync(store, s.tape_ckpt[(size_t)seg], sizeof(double) * nv, hipMemcpyDeviceToDevice,
                                     s.stream));
            for (long long st = s0; st < s1; st++) {
                double* U = store + (size_t)(st - s0) * ns * nv;
                const double dt = s.tape_dt[(size_t)st];
                for (int q = 1; q < ns; q++)
                    engine_bulk_stage(s, k, U + (size_t)(q - 1) * nv, U, U + (size_t)q * nv, A[q - 1], dt);
                if (st + 1 < s1)
                    engine_bulk_stage(s, k, U + (size_t)(ns - 1) * nv, U, U + (size_t)ns * nv, A[ns - 1], dt);
            }
            // reverse sweep
            for (long long st = s1 - 1; st >= s0; st--) {
                const double* U = store + (size_t)(st - s0) * ns * nv;
                const double dt = s.tape_dt[(size_t)st];
                for (int q = ns; q >= 1; q--) {
                    const double w = 1.0 - A[q - 1];
                    jlt(k, U + (size_t)(q - 1) * nv, lam, w * dt, v, fb, pacc);
                    k_adj_comb<<<blocks((long long)nv), ADJ_WG, 0, s.stream>>>((long long)nv, lam, lam0, v, A[q - 1], w,
                                                                               q == ns, q == 1);
                }
            }
        }
        // initial map; the other fluid holds no cell
        SHARP_HIP(hipMemsetAsync(g_prim0, 0, sizeof(double) * 2 * nv, s.stream));
        k_adj_prim0<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, s.tape_prim0, lam, g_prim0 + (size_t)k * nv, pacc);
        std::vector<double> h(2 * ADJ_BLOCKS);
        SHARP_HIP(hipMemcpyAsync(h.data(), pacc, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s.stream));
        SHARP_HIP(hipStreamSynchronize(s.stream));
        SHARP_HIP(hipGetLastError());
        double gsum = 0.0, psum = 0.0;
        for (int b = 0; b < ADJ_BLOCKS; b++) { gsum += h[2 * b]; psum += h[2 * b + 1]; }
        for (int i = 0; i < 4; i++) g_eos[i] = 0.0;
        g_eos[2 * k] = gsum;
        g_eos[2 * k + 1] = psum;
        return SIM_OK;
    }
};

}  // namespace

void tape_clear(Sim& s)
{
    for (double* p : s.tape_ckpt) (void)hipFree(p);
    s.tape_ckpt.clear();
    s.tape_dt.clear();
    if (s.tape_prim0) (void)hipFree(s.tape_prim0);
    s.tape_prim0 = nullptr;
    s.tape_fluid = -1;
}

sim_status tape_begin(Sim& s, const double* prim_dev)
{
    tape_clear(s);
    const bool none0 = s.bulk_cells[0] == 0, none1 = s.bulk_cells[1] == 0;
    if (s.lcount[LIST_BAND] != 0 || none0 == none1) {
        s.tape_why = "the level set places an interface (or its band) in the grid: the adjoint covers runs in "
                     "which one fluid fills the grid";
        return SIM_OK;
    }
    const int k = none0 ? 1 : 0;
    const size_t nv = (size_t)(s.g.D + 2) * s.g.nc;
    if (hipMalloc((void**)&s.tape_prim0, sizeof(double) * nv) != hipSuccess) {
        (void)hipGetLastError();
        s.tape_prim0 = nullptr;
        set_error("tape allocation failed");
        return SIM_ENOMEM;
    }
    SHARP_HIP(hipMemcpyAsync(s.tape_prim0, prim_dev + (size_t)k * nv, sizeof(double) * nv, hipMemcpyDeviceToDevice,
                             s.stream));
    s.tape_fluid = k;
    s.tape_why.clear();
    return SIM_OK;
}

sim_status tape_step(Sim& s, double dt)
{
    if (s.tape_fluid < 0) return SIM_OK;
    if (s.tape_dt.size() % (size_t)s.o.ckpt_every == 0) {
        const size_t nv = (size_t)(s.g.D + 2) * s.g.nc;
        double* p = nullptr;
        if (hipMalloc((void**)&p, sizeof(double) * nv) != hipSuccess) {
            (void)hipGetLastError();
            set_error("tape checkpoint allocation failed");
            return SIM_ENOMEM;
        }
        s.tape_ckpt.push_back(p);
        SHARP_HIP(hipMemcpyAsync(p, s.g.X[s.tape_fluid], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
    }
    s.tape_dt.push_back(dt);
    return SIM_OK;
}

sim_status engine_backward(Sim& s, const double* g_cons, double* g_prim0, double* g_eos)
{
    (void)hipStreamSynchronize(s.stream);
    for (int k = 0; k < 2; k++)
        if (s.side[k]) (void)hipStreamSynchronize(s.side[k]);
    switch (s.g.D) {
    case 1: return Adjoint<1>(s).run(g_cons, g_prim0, g_eos);
    case 2: return Adjoint<2>(s).run(g_cons, g_prim0, g_eos);
    default: return Adjoint<3>(s).run(g_cons, g_prim0, g_eos);
    }
}

}  // namespace sharp
