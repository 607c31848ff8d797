// sharp_adjoint.hip -- reverse-mode derivative (adjoint) of single-dt runs:
// the Shu-Osher stages (Sec. 2.1, Sec. 3) of the cut-cell finite-volume
// update (Eq. Eulerdiscrete) with the WENO5 flux under local Lax-Friedrichs
// splitting, the exchange term of the interface Riemann problem, the
// ghost-fluid extension and small-cell mixing (Sec. 2.3, Sec. 2.2), and the
// stiffened-gas EOS.  The step lengths are frozen at their forward values,
// and so is the geometry: every stage's level set is the recorded one.
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
//
// With an interface (tape_fluid = 2) the forward also records the level set
// after every stage, and the backward replays each segment from its
// checkpoint through the forward engine with those level sets, copying
// every stage's inputs, extended primitives, interface solution and
// geometry to a stage record.  Per stage and fluid k the map is
//     out_k = Mix_k(a U_0,k + (1 - a)(U_k + dt L_k)),
//     L_k = sum_d (A_k,lo F_lo - A_k,hi F_hi)/h + X_k(p*, u*),
// where a face flux reads, at each stencil cell, U/alpha_k on the fluid's
// real cells (alpha_k >= alpha_mix) and U(W) of the extended primitives W
// elsewhere; W = Ext_k(W(U/alpha_k) on real cells); (p*, u*) solve the
// Riemann problem between the two fluids' W at each cut cell.  Its reverse:
// Mix_k^T, then the face products (weighted by A_k), the exchange term's
// product with dp*, du* from the implicit function theorem on
// f_L(p) + f_R(p) + u_R - u_L = 0, Ext_k^T (the transposed Jacobi sweeps)
// and the primitive recovery's transpose.
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
// stage times (c) and quadrature weights (b) of the Shu-Osher tables: the
// accelerated cycle's interpolation and correction weights (Sec. 3.1)
const double ADJ_RK3_B[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
const double ADJ_RK3_C[3] = {0.0, 1.0, 0.5};
const double ADJ_RK2_B[2] = {0.5, 0.5};
const double ADJ_RK2_C[2] = {0.0, 1.0};

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

// parameter partials (gamma_0, p_inf_0, gamma_1, p_inf_1) of a block, added
// to its slot acc[4 block + i]: launches add in stream order
__device__ __forceinline__ void block_add4(const double (&x)[4], double* acc)
{
    __shared__ double sx[4][ADJ_WG / 64];
    double v[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        v[i] = x[i];
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, 64);
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 4; i++) sx[i][wid] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            double t = v[i];
            for (int w = 1; w < ADJ_WG / 64; w++) t += sx[i][w];
            acc[4 * blockIdx.x + i] += t;
        }
}
__device__ __forceinline__ void block_add_pair(int k, double x, double y, double* acc)
{
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    v[2 * k] = x;
    v[2 * k + 1] = y;
    block_add4(v, acc);
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

// two waves per SIMD (a few spills) measured 3% faster than one without.
// ap: fluid 0's aperture of the faces normal to d (padded face index), the
// flux weight of fluid k (1 - ap for fluid 1); null: every face open.  A
// face with no weight writes zero slots and reads no stencil state.
template <int D, int DIR>
__global__ void __launch_bounds__(ADJ_WG, 2) k_adj_face(Dev g, int k, const double* U, const double* lam,
                                                     double scale, const double* ap, double* fb, double* pacc)
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
        double wk = 1.0;
        if (ap) {
            const double a0 = ap[fidx(g, fc[0], fc[1], fc[2])];
            wk = k == 0 ? a0 : 1.0 - a0;
        }
        bool any = false;
#pragma unroll
        for (int q = 0; q < NV; q++) {
            Fb[q] = wk * scale *
                    ((cr >= 0 ? lam[(size_t)q * g.nc + cr] : 0.0) - (cl >= 0 ? lam[(size_t)q * g.nc + cl] : 0.0));
            any = any || Fb[q] != 0.0;
        }
        double* o = fb + (size_t)f * 6 * NV;
        if (!any) {
            for (int m = 0; m < 6 * NV; m++) o[m] = 0.0;
            continue;
        }
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
#pragma unroll
        for (int m = 0; m < 6; m++)
#pragma unroll
            for (int q = 0; q < NV; q++) o[m * NV + q] = Ub[m][q];
    }
    block_add_pair(k, gsum, psum, pacc);
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

// x += y (element-wise over n)
__global__ void __launch_bounds__(ADJ_WG) k_adj_add(long long n, double* x, const double* y)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        x[e] += y[e];
}

// reverse of the initial map prim -> cons, alpha_k U(W) with
// U = (rho, rho u, (p + gamma p_inf)/(gamma - 1) + rho |u|^2 / 2);
// al: fluid 0's volume fraction of the initial geometry (null: 1)
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj_prim0(Dev g, int k, const double* W, const double* lam, double* gp,
                                                      const double* al, double* pacc)
{
    constexpr int NV = D + 2;
    const double gm = g.gam[k], pi = g.pinf[k];
    double gsum = 0.0, psum = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        const double a = al ? (k == 0 ? al[c] : 1.0 - al[c]) : 1.0;
        double rho = W[c], p = W[(size_t)(NV - 1) * g.nc + c];
        double lE = a * lam[(size_t)(NV - 1) * g.nc + c];
        double r = a * lam[c], k2 = 0.0;
#pragma unroll
        for (int e = 0; e < D; e++) {
            double u = W[(size_t)(1 + e) * g.nc + c], lm = a * lam[(size_t)(1 + e) * g.nc + c];
            r += lm * u;
            k2 += u * u;
            gp[(size_t)(1 + e) * g.nc + c] = lm * rho + lE * rho * u;
        }
        gp[c] = r + lE * 0.5 * k2;
        gp[(size_t)(NV - 1) * g.nc + c] = lE / (gm - 1.0);
        if (lE != 0.0) {
            gsum += -lE * (p + pi) / ((gm - 1.0) * (gm - 1.0));
            psum += lE * gm / (gm - 1.0);
        }
    }
    block_add_pair(k, gsum, psum, pacc);
}

// ---------------------------------------------------------------------------
// Two fluids with frozen geometry: the reverse of one stage's band physics.
// Every kernel reads the stage record's arrays (see StageRec).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double frac_k(const double* al, int k, int c) { return k == 0 ? al[c] : 1.0 - al[c]; }

// level-set gradient by central differences over the domain's neighbours
template <int D>
__device__ __forceinline__ double grad_at(const Dev& g, const double* phi, int c, double* gr)
{
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; d++) {
        gr[d] = (phi[nbr(g, c, d, 1)] - phi[nbr(g, c, d, -1)]) / (2.0 * g.h);
        g2 += gr[d] * gr[d];
    }
    return sqrt(g2);
}

// stencil state of fluid k at every cell: the content over the volume
// fraction on real cells, U(W) of the extended primitives elsewhere
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_sten(Dev g, int k, const double* in, const double* al, const double* W,
                                                      double* S)
{
    constexpr int NV = D + 2;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        const double a = frac_k(al, k, c);
        double U[NV];
        if (a >= g.amix) {
#pragma unroll
            for (int q = 0; q < NV; q++) U[q] = in[(size_t)q * g.nc + c] / a;
        } else {
            double Wc[NV];
#pragma unroll
            for (int q = 0; q < NV; q++) Wc[q] = W[(size_t)q * g.nc + c];
            prim2cons<D>(g.gam[k], g.pinf[k], Wc, U);
        }
#pragma unroll
        for (int q = 0; q < NV; q++) S[(size_t)q * g.nc + c] = U[q];
    }
}

// the stencil states' adjoint v: real cells -> d(content) = v / alpha_k (in
// place); ghost cells -> the primitives' adjoint Wb = (dU/dW)^T v (v := 0),
// with the EOS partials of U(W)
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_split(Dev g, int k, const double* al, const double* W, double* v,
                                                       double* Wb, double* pacc)
{
    constexpr int NV = D + 2;
    const double gm = g.gam[k], pi = g.pinf[k];
    double gsum = 0.0, psum = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        const double a = frac_k(al, k, c);
        double ub[NV];
        bool any = false;
#pragma unroll
        for (int q = 0; q < NV; q++) {
            ub[q] = v[(size_t)q * g.nc + c];
            any = any || ub[q] != 0.0;
        }
        if (a >= g.amix) {
#pragma unroll
            for (int q = 0; q < NV; q++) {
                v[(size_t)q * g.nc + c] = ub[q] / a;
                Wb[(size_t)q * g.nc + c] = 0.0;
            }
            continue;
        }
#pragma unroll
        for (int q = 0; q < NV; q++) {
            v[(size_t)q * g.nc + c] = 0.0;
            Wb[(size_t)q * g.nc + c] = 0.0;
        }
        if (!any) continue;
        const double rho = W[c], p = W[(size_t)(NV - 1) * g.nc + c], lE = ub[NV - 1];
        double r = ub[0], k2 = 0.0;
#pragma unroll
        for (int e = 0; e < D; e++) {
            const double u = W[(size_t)(1 + e) * g.nc + c];
            r += ub[1 + e] * u;
            k2 += u * u;
            Wb[(size_t)(1 + e) * g.nc + c] = ub[1 + e] * rho + lE * rho * u;
        }
        Wb[c] = r + lE * 0.5 * k2;
        Wb[(size_t)(NV - 1) * g.nc + c] = lE / (gm - 1.0);
        gsum += -lE * (p + pi) / ((gm - 1.0) * (gm - 1.0));
        psum += lE * gm / (gm - 1.0);
    }
    block_add_pair(k, gsum, psum, pacc);
}

// one side's wave function f(p) of the interface Riemann problem and its
// partials: df = df/dp, a = df/d(rho, p_side, gamma, p_inf) at fixed p
// (shock: Hugoniot branch; rarefaction: isentropic branch)
__device__ inline double wave_partials(double rho, double ps, double gm, double pi, double p, double* df, double* a)
{
    const double pk = ps + pi, pb = p + pi;
    if (p > ps) {
        const double A = 2.0 / ((gm + 1.0) * rho), m = (gm - 1.0) / (gm + 1.0), B = m * pk;
        const double t = 1.0 / (pb + B), q = sqrt(A * t), f = (p - ps) * q, hq = -0.5 * (p - ps) * q * t;
        *df = q * (1.0 - 0.5 * (p - ps) * t);
        a[0] = -0.5 * f / rho;
        a[1] = -q + hq * m;
        a[2] = 0.5 * f * (-1.0 / (gm + 1.0)) + hq * 2.0 * pk / ((gm + 1.0) * (gm + 1.0));
        a[3] = hq * (1.0 + m);
        return f;
    }
    const double c = sqrt(gm * pk / rho), z = (gm - 1.0) / (2.0 * gm), r = pb / pk;
    const double rz = r > 0.0 ? pow(r, z) : 0.0, lr = r > 0.0 ? log(r) : 0.0;
    const double f = 2.0 * c / (gm - 1.0) * (rz - 1.0);
    *df = r > 0.0 ? rz / (r * rho * c) : 0.0;
    a[0] = -0.5 * f / rho;
    a[1] = 0.5 * f / pk - c * rz / (gm * pk);
    a[2] = 0.5 * f / gm + (2.0 * c / (gm - 1.0)) * rz * lr / (2.0 * gm * gm) - f / (gm - 1.0);
    a[3] = a[1] + (pb > 0.0 ? c * rz / (gm * pb) : 0.0);
    return f;
}

// Reverse of the exchange term at every cut cell: X_0 = (0, -p* g, -p* u*
// |g|) per unit volume, X_1 = -(0, -p_1 g, -p_1 u* |g|) with fluid 1's
// interface pressure p_1 = p* - j (j the Laplace jump of Eq.
// (surfacetension), 0 without surface tension), g = (A_lo - A_hi)/h of fluid
// 0's apertures (Sec. 2.1, Eq. Eulerdiscrete).  mu_k = scale lam_k; the
// primitives' adjoints Wb_k (+=) and the four EOS partials follow from
// dp*/dtheta = -(df/dtheta)/(df/dp) at the root of f_L(p) + f_R(p - j) +
// u_R - u_L and u* = (u_L + u_R)/2 + (f_R(p* - j) - f_L(p*))/2.  With the
// geometry frozen, j is a constant of the cut cell (from the level set phi
// the interaction saw), and f_R(p - j) is the wave curve of fluid 1's state
// with (p, p_inf) shifted by (+j, -j), whose partials in p and p_inf are
// those in fluid 1's own.  At the cavitation floor p* is held fixed.
template <int D>
__device__ __forceinline__ double adj_jump(const Dev& g, const double* phi, int i, int j, int k)
{
    return (g.pj && phi) ? laplace_jump<D>(g, phi, i, j, k) : 0.0;
}
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_riemann(Dev g, const double* ap, const double* W0, const double* W1,
                                                         const double* ps, const double* us, const double* lam0,
                                                         const double* lam1, double scale, double* Wb0, double* Wb1,
                                                         double* pacc, const double* phi)
{
    constexpr int NV = D + 2;
    double par[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        int i, j, kk;
        coords(g, c, i, j, kk);
        double gv[3], g2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; d++) {
            const double* a = ap + (size_t)d * g.nfc;
            gv[d] = (a[fidx(g, i, j, kk)] - a[fidx(g, i + (d == 0), j + (d == 1), kk + (d == 2))]) / g.h;
            g2 += gv[d] * gv[d];
        }
        const double gn = sqrt(g2);
        if (!(gn > 0.0)) continue;
        const double pst = ps[c], ust = us[c];
        const double jmp = adj_jump<D>(g, phi, i, j, kk);
        double pb = 0.0, ub = 0.0;
        for (int k = 0; k < 2; k++) {
            const double* lam = k == 0 ? lam0 : lam1;
            const double sg = k == 0 ? 1.0 : -1.0;
            const double pk = k == 0 ? pst : pst - jmp;
            double dot = 0.0;
#pragma unroll
            for (int d = 0; d < D; d++) dot += gv[d] * lam[(size_t)(1 + d) * g.nc + c];
            const double lE = lam[(size_t)(NV - 1) * g.nc + c];
            pb += sg * scale * (-dot - ust * gn * lE);
            ub += sg * scale * (-pk * gn * lE);
        }
        if (pb == 0.0 && ub == 0.0) continue;
        // (the wave functions depend on the normal velocities only through
        // u_R - u_L, whose partials are the sides' velocity adjoints below)
        const double r0 = W0[c], p0 = W0[(size_t)(NV - 1) * g.nc + c];
        const double r1 = W1[c], p1 = W1[(size_t)(NV - 1) * g.nc + c] + jmp;
        const double pi1 = g.pinf[1] - jmp;
        double dfl, dfr, al4[4], ar4[4];
        wave_partials(r0, p0, g.gam[0], g.pinf[0], pst, &dfl, al4);
        wave_partials(r1, p1, g.gam[1], pi1, pst, &dfr, ar4);
        const double pfl = -(g.pinf[0] < pi1 ? g.pinf[0] : pi1);
        const double G = 0.5 * (dfr - dfl);
        const bool cav = !(pst > pfl);
        const double sig = cav ? 0.0 : (pb + ub * G) / (dfl + dfr);
        const double uL = sig + 0.5 * ub, uR = -sig + 0.5 * ub;
        // the sides' (rho, p, gamma, p_inf)
        const double cl = -(sig + 0.5 * ub), cr = -(sig - 0.5 * ub);
        Wb0[c] += cl * al4[0];
        Wb0[(size_t)(NV - 1) * g.nc + c] += cl * al4[1];
        Wb1[c] += cr * ar4[0];
        Wb1[(size_t)(NV - 1) * g.nc + c] += cr * ar4[1];
#pragma unroll
        for (int d = 0; d < D; d++) {
            Wb0[(size_t)(1 + d) * g.nc + c] += uL * gv[d] / gn;
            Wb1[(size_t)(1 + d) * g.nc + c] += uR * gv[d] / gn;
        }
        par[0] += cl * al4[2];
        par[1] += cl * al4[3];
        par[2] += cr * ar4[2];
        par[3] += cr * ar4[3];
    }
    block_add4(par, pacc);
}

// the Laplace jumps of every cut cell of the current geometry, from the
// level set phi: what the interaction whose p*, u* a checkpoint restores
// stored beside them (the jumps are not part of the checkpoint; the band
// stages read them)
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_jump(Dev g, const double* phi)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        int i, j, kk;
        coords(g, c, i, j, kk);
        double g2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; d++) {
            const double gd = (g.ap[d][fidx(g, i, j, kk)] - g.ap[d][fidx(g, i + (d == 0), j + (d == 1), kk + (d == 2))]) /
                              g.h;
            g2 += gd * gd;
        }
        g.pj[c] = g2 > 0.0 ? laplace_jump<D>(g, phi, i, j, kk) : 0.0;
    }
}

// the exchange term's partials of one of its uses, accumulated per cut
// cell: X_k = s_k (0, -p_k g, -p_k u* |g|) of fluid k (p_0 = p*, p_1 = p* -
// j) enters with weight `scale` against the adjoint lam (a stage's (1 - a)
// dt, or a correction weight), s_0 = 1, s_1 = -1; pb += dJ/dp*, ub += dJ/du*
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_xacc(Dev g, const double* ap, const double* ps, const double* us,
                                                      const double* lam, double scale, double* pb, double* ub, int k,
                                                      const double* phi)
{
    constexpr int NV = D + 2;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        int i, j, kk;
        coords(g, c, i, j, kk);
        double gv[3], g2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; d++) {
            const double* a = ap + (size_t)d * g.nfc;
            gv[d] = (a[fidx(g, i, j, kk)] - a[fidx(g, i + (d == 0), j + (d == 1), kk + (d == 2))]) / g.h;
            g2 += gv[d] * gv[d];
        }
        const double gn = sqrt(g2);
        if (!(gn > 0.0)) continue;
        double dot = 0.0;
#pragma unroll
        for (int d = 0; d < D; d++) dot += gv[d] * lam[(size_t)(1 + d) * g.nc + c];
        const double lE = lam[(size_t)(NV - 1) * g.nc + c];
        const double pk = k == 0 ? ps[c] : ps[c] - adj_jump<D>(g, phi, i, j, kk);
        pb[c] += scale * (-dot - us[c] * gn * lE);
        ub[c] += scale * (-pk * gn * lE);
    }
}

// the Riemann problem's reverse from accumulated dJ/dp*, dJ/du* (see
// k_adj2_riemann, which forms them from the two fluids' stage adjoints)
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_riemann2(Dev g, const double* ap, const double* W0, const double* W1,
                                                          const double* ps, const double* pbv, const double* ubv,
                                                          double* Wb0, double* Wb1, double* pacc, const double* phi)
{
    constexpr int NV = D + 2;
    double par[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        const double pb = pbv[c], ub = ubv[c];
        if (pb == 0.0 && ub == 0.0) continue;
        int i, j, kk;
        coords(g, c, i, j, kk);
        double gv[3], g2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; d++) {
            const double* a = ap + (size_t)d * g.nfc;
            gv[d] = (a[fidx(g, i, j, kk)] - a[fidx(g, i + (d == 0), j + (d == 1), kk + (d == 2))]) / g.h;
            g2 += gv[d] * gv[d];
        }
        const double gn = sqrt(g2);
        if (!(gn > 0.0)) continue;
        const double pst = ps[c];
        const double jmp = adj_jump<D>(g, phi, i, j, kk), pi1 = g.pinf[1] - jmp;
        double dfl, dfr, al4[4], ar4[4];
        wave_partials(W0[c], W0[(size_t)(NV - 1) * g.nc + c], g.gam[0], g.pinf[0], pst, &dfl, al4);
        wave_partials(W1[c], W1[(size_t)(NV - 1) * g.nc + c] + jmp, g.gam[1], pi1, pst, &dfr, ar4);
        const double pfl = -(g.pinf[0] < pi1 ? g.pinf[0] : pi1);
        const double G = 0.5 * (dfr - dfl);
        const double sig = !(pst > pfl) ? 0.0 : (pb + ub * G) / (dfl + dfr);
        const double uL = sig + 0.5 * ub, uR = -sig + 0.5 * ub;
        const double cl = -(sig + 0.5 * ub), cr = -(sig - 0.5 * ub);
        Wb0[c] += cl * al4[0];
        Wb0[(size_t)(NV - 1) * g.nc + c] += cl * al4[1];
        Wb1[c] += cr * ar4[0];
        Wb1[(size_t)(NV - 1) * g.nc + c] += cr * ar4[1];
#pragma unroll
        for (int d = 0; d < D; d++) {
            Wb0[(size_t)(1 + d) * g.nc + c] += uL * gv[d] / gn;
            Wb1[(size_t)(1 + d) * g.nc + c] += uR * gv[d] / gn;
        }
        par[0] += cl * al4[2];
        par[1] += cl * al4[3];
        par[2] += cr * ar4[2];
        par[3] += cr * ar4[3];
    }
    block_add4(par, pacc);
}

// reverse of X_S += corr on the momentum and energy components: the
// correction's adjoint gains the slow fluid's
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_corrT(Dev g, const double* lx, double* lc)
{
    constexpr int NV = D + 2;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x)
#pragma unroll
        for (int q = 1; q < NV; q++) lc[(size_t)q * g.nc + c] += lx[(size_t)q * g.nc + c];
}

// x = a x + b y (element-wise over n)
__global__ void __launch_bounds__(ADJ_WG) k_adj_axpby(long long n, double* x, double a, const double* y, double b)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        x[e] = a * x[e] + b * y[e];
}

// the level set a stage saw over every cell (its band-mask cells from the
// working buffer, the others from the base one)
__global__ void __launch_bounds__(ADJ_WG) k_adj_phi(Dev g, const double* cur, double* out)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x)
        out[c] = g.M[c] ? cur[c] : g.phiP[c];
}

// Extension of fluid k (Sec. 2.3): target cells are band cells with
// alpha_k < alpha_mix within ext_band cells on the far side of the
// interface with a nonzero level-set gradient; each Jacobi sweep sets a
// target to sum_d w_d W[up_d] with n = s_k grad phi / |grad phi|, w_d =
// |n_d| / sum |n|, up_d the neighbour against n_d (s_0 = 1, s_1 = -1).
template <int D>
__device__ __forceinline__ bool ext_target(const Dev& g, int k, const double* phi, const double* al,
                                           const uint8_t* M, int c, double* w, int* up)
{
    const double sk = k == 0 ? 1.0 : -1.0;
    if (!M[c] || !(frac_k(al, k, c) < g.amix) || sk * phi[c] > g.extb * g.h) return false;
    double gr[3];
    const double gm = grad_at<D>(g, phi, c, gr);
    if (!(gm > 0.0)) return false;
    double ws = 0.0;
#pragma unroll
    for (int d = 0; d < D; d++) {
        const double nd = sk * gr[d] / gm;
        up[d] = nbr(g, c, d, nd > 0.0 ? -1 : 1);
        w[d] = fabs(nd);
        ws += w[d];
    }
#pragma unroll
    for (int d = 0; d < D; d++) w[d] /= ws;
    return true;
}

// The transposed sweep's gather for every cell, computed once per stage and
// fluid (every sweep of a stage has the same targets and weights): the
// cell's own entry passes (tx = 0) or is replaced (tx = 1), and up to 2D + 1
// (source cell, weight) pairs are added; slots past `cnt` are unused.
// Layout: cnt[c] = number of pairs | tx << 7; idx[m * nc + c], wt[m * nc + c].
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_extprep(Dev g, int k, const double* phi, const double* al,
                                                         const uint8_t* M, uint8_t* cnt, int* idx, double* wt)
{
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < g.nc; x += gridDim.x * blockDim.x) {
        double w[3];
        int up[3];
        const bool tx = ext_target<D>(g, k, phi, al, M, x, w, up);
        int cand[1 + 2 * D], nc = 0, np = 0;
        cand[nc++] = x;
#pragma unroll
        for (int d = 0; d < D; d++)
            for (int o = -1; o <= 1; o += 2) {
                const int c = nbr(g, x, d, o);
                bool seen = false;
                for (int m = 0; m < nc; m++) seen = seen || cand[m] == c;
                if (!seen) cand[nc++] = c;
            }
        for (int m = 0; m < nc; m++) {
            const int c = cand[m];
            if (!ext_target<D>(g, k, phi, al, M, c, w, up)) continue;
            for (int d = 0; d < D; d++) {
                if (up[d] != x || w[d] == 0.0) continue;
                idx[(size_t)np * g.nc + x] = c;
                wt[(size_t)np * g.nc + x] = w[d];
                np++;
            }
        }
        cnt[x] = (uint8_t)(np | (tx ? 0x80 : 0));
    }
}

// one transposed Jacobi sweep from the precomputed gathers (k_adj2_extprep)
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_extT2(Dev g, const uint8_t* cnt, const int* idx, const double* wt,
                                                       const double* Wi, double* Wo)
{
    constexpr int NV = D + 2;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < g.nc; x += gridDim.x * blockDim.x) {
        const int cx = cnt[x], np = cx & 0x7f;
        double acc[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) acc[q] = (cx & 0x80) ? 0.0 : Wi[(size_t)q * g.nc + x];
        for (int m = 0; m < np; m++) {
            const int c = idx[(size_t)m * g.nc + x];
            const double w = wt[(size_t)m * g.nc + x];
#pragma unroll
            for (int q = 0; q < NV; q++) acc[q] += w * Wi[(size_t)q * g.nc + c];
        }
#pragma unroll
        for (int q = 0; q < NV; q++) Wo[(size_t)q * g.nc + x] = acc[q];
    }
}

// the primitives' adjoint left on the cells that are not real cells of
// fluid k (alpha_k < alpha_mix): there the extension's first sweep read the
// values the previous extension left (or those sim_set_state gave)
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_ghost(Dev g, int k, const double* al, const double* Wb, double* carry)
{
    constexpr int NV = D + 2;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        const bool real = frac_k(al, k, c) >= g.amix;
#pragma unroll
        for (int q = 0; q < NV; q++) carry[(size_t)q * g.nc + c] = real ? 0.0 : Wb[(size_t)q * g.nc + c];
    }
}

// reverse of the primitive recovery W = W(U), U = content / alpha_k, on the
// real cells of fluid k: v += (dW/dU)^T Wb / alpha_k, with its EOS partials
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_c2pT(Dev g, int k, const double* in, const double* al,
                                                      const double* Wb, double* v, double* pacc)
{
    constexpr int NV = D + 2;
    const double gm = g.gam[k], pi = g.pinf[k];
    double gsum = 0.0, psum = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.nc; c += gridDim.x * blockDim.x) {
        const double a = frac_k(al, k, c);
        if (!(a >= g.amix)) continue;
        double wb[NV];
        bool any = false;
#pragma unroll
        for (int q = 0; q < NV; q++) {
            wb[q] = Wb[(size_t)q * g.nc + c];
            any = any || wb[q] != 0.0;
        }
        if (!any) continue;
        const double rho = in[c] / a, E = in[(size_t)(NV - 1) * g.nc + c] / a;
        double u[3], k2 = 0.0;
#pragma unroll
        for (int e = 0; e < D; e++) {
            u[e] = in[(size_t)(1 + e) * g.nc + c] / a / rho;
            k2 += u[e] * u[e];
        }
        const double pbw = wb[NV - 1];
        double r = wb[0] + pbw * (gm - 1.0) * 0.5 * k2;
#pragma unroll
        for (int e = 0; e < D; e++) {
            r -= wb[1 + e] * u[e] / rho;
            v[(size_t)(1 + e) * g.nc + c] += (wb[1 + e] / rho - pbw * (gm - 1.0) * u[e]) / a;
        }
        v[c] += r / a;
        v[(size_t)(NV - 1) * g.nc + c] += pbw * (gm - 1.0) / a;
        gsum += pbw * (E - 0.5 * rho * k2 - pi);
        psum += -pbw * gm;
    }
    block_add_pair(k, gsum, psum, pacc);
}

// Small-cell mixing of fluid k (Sec. 2.2): a source s (alpha_k < alpha_mix,
// |phi| <= mix_band cells, nonzero gradient) exchanges
// M = beta [(aU)_t a_s - (aU)_s a_t] / (a_s + a_t) with each target t
// toward the bulk of fluid k along a non-empty subset of the axes (weights
// |n_d|^2, |n_a n_b|, |n_x n_y n_z|^(2/3), normalised); s gains M, t loses
// it.  mix_target returns the target of subset m and its weight (t = -1:
// none).
template <int D>
__device__ __forceinline__ bool mix_source(const Dev& g, int k, const double* phi, const double* al, int c,
                                           double* beta, int* sx)
{
    if (!(frac_k(al, k, c) < g.amix) || !(fabs(phi[c]) <= g.mixb * g.h)) return false;
    double gr[3];
    const double gm = grad_at<D>(g, phi, c, gr);
    if (!(gm > 0.0)) return false;
    double dir[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < D; d++) {
        dir[d] = (k == 0 ? -1.0 : 1.0) * gr[d] / gm;
        sx[d] = dir[d] < 0.0 ? -1 : 1;
    }
    double bs = 0.0;
    for (int m = 1; m < (1 << D); m++) {
        int cnt = 0;
        double prod = 1.0;
        for (int d = 0; d < D; d++)
            if (m & (1 << d)) { cnt++; prod *= fabs(dir[d]); }
        const double b = cnt == 1 ? prod * prod : (cnt == 2 ? prod : pow(prod, 2.0 / 3.0));
        beta[m - 1] = b;
        bs += b;
    }
    for (int m = 1; m < (1 << D); m++) beta[m - 1] /= bs;
    return true;
}

template <int D>
__device__ __forceinline__ int mix_target(const Dev& g, int c, int m, const int* sx)
{
    int i, j, kk;
    coords(g, c, i, j, kk);
    return cidx(g, i + ((m & 1) ? sx[0] : 0), j + (D > 1 && (m & 2) ? sx[1] : 0), kk + (D > 2 && (m & 4) ? sx[2] : 0));
}

// lo = Mix_k^T li, gathered per cell: its own exchanges as a source and
// those of the sources in its 3^D neighbourhood that target it
template <int D>
__global__ void __launch_bounds__(ADJ_WG) k_adj2_mixT(Dev g, int k, const double* al, const double* phi,
                                                      const double* li, double* lo)
{
    constexpr int NV = D + 2;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < g.nc; x += gridDim.x * blockDim.x) {
        double lx[NV], acc[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) acc[q] = lx[q] = li[(size_t)q * g.nc + x];
        const double ax = frac_k(al, k, x);
        double beta[7];
        int sx[3] = {1, 1, 1};
        if (mix_source<D>(g, k, phi, al, x, beta, sx)) {
            for (int m = 1; m < (1 << D); m++) {
                const double b = beta[m - 1];
                if (!(b > 0.0)) continue;
                const int t = mix_target<D>(g, x, m, sx);
                if (t == x) continue;
                const double at = frac_k(al, k, t);
                if (!(ax + at > 0.0)) continue;
                const double f = b * at / (ax + at);
#pragma unroll
                for (int q = 0; q < NV; q++) acc[q] -= f * (lx[q] - li[(size_t)q * g.nc + t]);
            }
        }
        int i, j, kk;
        coords(g, x, i, j, kk);
        int seen[27], ns = 0;
        for (int oz = (D > 2 ? -1 : 0); oz <= (D > 2 ? 1 : 0); oz++)
            for (int oy = (D > 1 ? -1 : 0); oy <= (D > 1 ? 1 : 0); oy++)
                for (int ox = -1; ox <= 1; ox++) {
                    const int c = cidx(g, i + ox, j + oy, kk + oz);
                    if (c == x) continue;
                    bool dup = false;
                    for (int m = 0; m < ns; m++) dup = dup || seen[m] == c;
                    if (dup) continue;
                    seen[ns++] = c;
                    int sc[3] = {1, 1, 1};
                    if (!mix_source<D>(g, k, phi, al, c, beta, sc)) continue;
                    const double ac = frac_k(al, k, c);
                    if (!(ac + ax > 0.0)) continue;
                    for (int m = 1; m < (1 << D); m++) {
                        const double b = beta[m - 1];
                        if (!(b > 0.0) || mix_target<D>(g, c, m, sc) != x) continue;
                        const double f = b * ac / (ac + ax);
#pragma unroll
                        for (int q = 0; q < NV; q++) acc[q] += f * (li[(size_t)q * g.nc + c] - lx[q]);
                    }
                }
#pragma unroll
        for (int q = 0; q < NV; q++) lo[(size_t)q * g.nc + x] = acc[q];
    }
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

    // v = J^T (scale * lam) of the face fluxes of fluid k, per direction
    // through the face buffer (ap: fluid 0's apertures, D padded face
    // arrays; null: every face open)
    void jlt(int k, const double* U, const double* lam, double scale, double* v, double* fb, double* pacc,
             const double* ap = nullptr)
    {
        for (int d = 0; d < D; d++) {
            const double* a = ap ? ap + (size_t)d * g.nfc : nullptr;
            if (d == 0)
                k_adj_face<D, 0><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, U, lam, scale / g.h, a, fb, pacc);
            if constexpr (D > 1)
                if (d == 1) k_adj_face<D, 1><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, U, lam, scale / g.h, a, fb, pacc);
            if constexpr (D > 2)
                if (d == 2) k_adj_face<D, 2><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, U, lam, scale / g.h, a, fb, pacc);
            k_adj_gather<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, d, fb, v, d > 0);
        }
    }

    sim_status run(const double* g_cons, double* g_prim0, double* g_eos)
    {
        std::vector<void*> own;
        bool cycles = false;
        for (const Sim::TapeUnit& u : s.tape_units) cycles = cycles || u.cycle;
        sim_status rc = s.tape_fluid != 2 ? sweep(g_cons, g_prim0, g_eos, own)
                                          : (cycles ? sweep3(g_cons, g_prim0, g_eos, own)
                                                    : sweep2(g_cons, g_prim0, g_eos, own));
        (void)hipStreamSynchronize(s.stream);
        for (void* p : own) (void)hipFree(p);
        return rc;
    }

    // what the last interaction left (both fluids' extended primitives, p*,
    // u* and the extended level-set velocity) to or from p (2 NV + 2 + D
    // cells values): the state a step starts from besides the contents and
    // the level set
    hipError_t save_interaction(double* p, bool back)
    {
        const size_t nv = (size_t)NV * g.nc, nc = (size_t)g.nc;
        double* dst[4 + D];
        double* src[4 + D];
        size_t n[4 + D];
        dst[0] = p; src[0] = g.Wb[0][s.wcur]; n[0] = nv;
        dst[1] = p + nv; src[1] = g.Wb[1][s.wcur]; n[1] = nv;
        dst[2] = p + 2 * nv; src[2] = g.ps; n[2] = nc;
        dst[3] = p + 2 * nv + nc; src[3] = g.us; n[3] = nc;
        for (int d = 0; d < D; d++) {
            dst[4 + d] = p + 2 * nv + (2 + d) * nc;
            src[4 + d] = g.v[s.vcur][d];
            n[4 + d] = nc;
        }
        hipError_t e = hipSuccess;
        for (int i = 0; i < 4 + D && e == hipSuccess; i++)
            e = hipMemcpyAsync(back ? src[i] : dst[i], back ? dst[i] : src[i], n[i] * sizeof(double),
                               hipMemcpyDeviceToDevice, s.stream);
        return e;
    }

    double* alloc(std::vector<void*>& own, size_t bytes)
    {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
        own.push_back(p);
        return (double*)p;
    }

    long long max_faces() const
    {
        long long nfmax = 0;
        for (int d = 0; d < D; d++)
            nfmax = std::max(nfmax, (long long)(g.n[0] + (d == 0)) * (g.n[1] + (d == 1)) * (g.n[2] + (d == 2)));
        return nfmax;
    }

    // the four parameter partials, summed over the blocks in a fixed order
    sim_status read_params(const double* pacc, double* g_eos)
    {
        std::vector<double> h(4 * ADJ_BLOCKS);
        SHARP_HIP(hipMemcpyAsync(h.data(), pacc, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s.stream));
        SHARP_HIP(hipStreamSynchronize(s.stream));
        SHARP_HIP(hipGetLastError());
        for (int i = 0; i < 4; i++) {
            double t = 0.0;
            for (int b = 0; b < ADJ_BLOCKS; b++) t += h[4 * b + i];
            g_eos[i] = t;
        }
        return SIM_OK;
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
        // buffers: the stage inputs of one segment (ns per step), lam, lam0,
        // v, the face buffer (6 NV per face), the per-block parameter partials
        const size_t nstore = (size_t)std::min<long long>(N > 0 ? N : 1, K) * ns;
        double* store = alloc(own, sizeof(double) * nv * nstore);
        double* lam = alloc(own, sizeof(double) * nv);
        double* lam0 = alloc(own, sizeof(double) * nv);
        double* v = alloc(own, sizeof(double) * nv);
        double* fb = alloc(own, sizeof(double) * (size_t)max_faces() * 6 * NV);
        double* pacc = alloc(own, sizeof(double) * 4 * ADJ_BLOCKS);
        if (!store || !lam || !lam0 || !v || !fb || !pacc) {
            set_error("adjoint buffers do not fit in device memory (%zu MB for the recomputed stages)",
                      sizeof(double) * nv * nstore >> 20);
            return SIM_ENOMEM;
        }
        SHARP_HIP(hipMemsetAsync(pacc, 0, sizeof(double) * 4 * ADJ_BLOCKS, s.stream));
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
        k_adj_prim0<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, s.tape_prim0, lam, g_prim0 + (size_t)k * nv, nullptr,
                                                            pacc);
        return read_params(pacc, g_eos);
    }

    // Two fluids and an interface, geometry frozen at the recorded stage
    // level sets.  Per segment (last first): the state is set to the
    // segment's checkpoint and its steps are replayed by the forward engine
    // (every kernel on the simulation's stream) into one stage record per
    // stage; then the reverse sweep runs through the records.  The state
    // the forward ended with is restored at the end.
    sim_status sweep2(const double* g_cons, double* g_prim0, double* g_eos, std::vector<void*>& own)
    {
        const int ns = s.o.rk;
        const double* A = ns == 3 ? ADJ_RK3_A : ADJ_RK2_A;
        const size_t nv = (size_t)NV * g.nc;
        const long long N = (long long)s.tape_dt.size();
        const int K = s.o.ckpt_every;
        StageRec rec;
        rec.layout(D, (size_t)g.nc, (size_t)g.nfc);
        const size_t nrec = (size_t)std::min<long long>(N > 0 ? N : 1, K) * ns;
        double* store = alloc(own, sizeof(double) * rec.stride * nrec);
        double *lam[2], *lam0[2], *v[2], *Wb[2][2];
        for (int k = 0; k < 2; k++) {
            lam[k] = alloc(own, sizeof(double) * nv);
            lam0[k] = alloc(own, sizeof(double) * nv);
            v[k] = alloc(own, sizeof(double) * nv);
            Wb[k][0] = alloc(own, sizeof(double) * nv);
            Wb[k][1] = alloc(own, sizeof(double) * nv);
        }
        double* S = alloc(own, sizeof(double) * nv);
        double* tmp = alloc(own, sizeof(double) * nv);
        // adjoint of the ghost values an extension starts from (the previous
        // interaction's extension results), carried to the stage before
        double* carry[2] = {alloc(own, sizeof(double) * nv), alloc(own, sizeof(double) * nv)};
        // the transposed extension's gathers of one stage and fluid
        uint8_t* xcnt = reinterpret_cast<uint8_t*>(alloc(own, (size_t)g.nc + 8));
        int* xidx = reinterpret_cast<int*>(alloc(own, sizeof(int) * (size_t)(2 * D + 1) * g.nc));
        double* xwt = alloc(own, sizeof(double) * (size_t)(2 * D + 1) * g.nc);
        double* fb = alloc(own, sizeof(double) * (size_t)max_faces() * 6 * NV);
        double* pacc = alloc(own, sizeof(double) * 4 * ADJ_BLOCKS);
        double* fin = alloc(own, sizeof(double) * (4 * nv + (3 + D) * g.nc));
        bool ok = store && S && tmp && fb && pacc && fin && xcnt && xidx && xwt && carry[0] && carry[1];
        for (int k = 0; k < 2; k++) ok = ok && lam[k] && lam0[k] && v[k] && Wb[k][0] && Wb[k][1];
        if (!ok) {
            set_error("adjoint buffers do not fit in device memory (%zu MB for %zu stage records)",
                      sizeof(double) * rec.stride * nrec >> 20, nrec);
            return SIM_ENOMEM;
        }
        // the state the forward ended with, restored afterwards
        SHARP_HIP(hipMemcpyAsync(fin, g.X[0], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(hipMemcpyAsync(fin + nv, g.X[1], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(hipMemcpyAsync(fin + 2 * nv, g.phiP, sizeof(double) * g.nc, hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(save_interaction(fin + 2 * nv + g.nc, false));
        SHARP_HIP(hipMemsetAsync(pacc, 0, sizeof(double) * 4 * ADJ_BLOCKS, s.stream));
        for (int k = 0; k < 2; k++) {
            SHARP_HIP(hipMemcpyAsync(lam[k], g_cons + (size_t)k * nv, sizeof(double) * nv, hipMemcpyDeviceToDevice,
                                     s.stream));
            SHARP_HIP(hipMemsetAsync(carry[k], 0, sizeof(double) * nv, s.stream));
        }
        const double t_end = s.t;
        const bool serial = s.run_serial;
        s.run_serial = true;
        g.use_sched = 0;
        s.ls_src.clear();
        for (double* p : s.tape_ls)
            for (int q = 0; q < ns; q++) s.ls_src.push_back(p + (size_t)q * g.nc);
        sim_status rc = SIM_OK;
        const long long nseg = (N + K - 1) / K;
        for (long long seg = nseg - 1; seg >= 0 && rc == SIM_OK; seg--) {
            const long long s0 = seg * K, s1 = std::min(N, s0 + K);
            const double* ck = s.tape_ckpt[(size_t)seg];
            rc = engine_restore(s, ck, ck + nv, ck + 2 * nv);
            if (rc != SIM_OK) break;
            // the step-start interaction's results as the forward had them:
            // the first step of the segment starts with its stages
            for (int k = 0; k < 2; k++)
                SHARP_HIP(hipMemcpyAsync(g.Wb[k][s.wcur], ck + 2 * nv + g.nc + (size_t)k * nv, sizeof(double) * nv,
                                         hipMemcpyDeviceToDevice, s.stream));
            SHARP_HIP(hipMemcpyAsync(g.ps, ck + 4 * nv + g.nc, sizeof(double) * g.nc, hipMemcpyDeviceToDevice,
                                     s.stream));
            SHARP_HIP(hipMemcpyAsync(g.us, ck + 4 * nv + 2 * g.nc, sizeof(double) * g.nc, hipMemcpyDeviceToDevice,
                                     s.stream));
            if (g.pj) k_adj2_jump<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, g.phiP);
            s.ls_pos = (size_t)s0 * ns;
            rec.base = store;
            rec.next = 0;
            for (long long st = s0; st < s1 && rc == SIM_OK; st++)
                rc = engine_replay_step(s, s.tape_dt[(size_t)st], &rec, st == s0);
            if (rc != SIM_OK) break;
            for (long long st = s1 - 1; st >= s0; st--) {
                const double dt = s.tape_dt[(size_t)st];
                for (int q = ns; q >= 1; q--) {
                    const double* R = store + ((size_t)(st - s0) * ns + (q - 1)) * rec.stride;
                    const double w = 1.0 - A[q - 1];
                    // mixing after the stage, with the stage's new geometry
                    for (int k = 0; k < 2; k++) {
                        k_adj2_mixT<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, k, R + rec.aln, R + rec.phin, lam[k],
                                                                             tmp);
                        std::swap(lam[k], tmp);
                    }
                    // face fluxes: content adjoints on real cells, primitive
                    // adjoints on ghost cells
                    for (int k = 0; k < 2; k++) {
                        k_adj2_sten<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, k, R + rec.in[k], R + rec.al,
                                                                             R + rec.W[k], S);
                        jlt(k, S, lam[k], w * dt, v[k], fb, pacc, R + rec.ap);
                        k_adj2_split<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, R + rec.al, R + rec.W[k], v[k],
                                                                            Wb[k][0], pacc);
                    }
                    // exchange term
                    k_adj2_riemann<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, R + rec.ap, R + rec.W[0], R + rec.W[1],
                                                                          R + rec.ps, R + rec.us, lam[0], lam[1],
                                                                          w * dt, Wb[0][0], Wb[1][0], pacc, R + rec.phi);
                    const uint8_t* Mk = reinterpret_cast<const uint8_t*>(R + rec.M);
                    for (int k = 0; k < 2; k++) {
                        int cur = 0;
                        // the later stage's extension started from this
                        // one's results
                        k_adj_add<<<blocks((long long)nv), ADJ_WG, 0, s.stream>>>((long long)nv, Wb[k][0], carry[k]);
                        if (s.o.ext_iters > 0)
                            k_adj2_extprep<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, k, R + rec.phi, R + rec.al, Mk,
                                                                                    xcnt, xidx, xwt);
                        for (int it = 0; it < s.o.ext_iters; it++) {
                            k_adj2_extT2<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, xcnt, xidx, xwt, Wb[k][cur],
                                                                                  Wb[k][1 - cur]);
                            cur ^= 1;
                        }
                        k_adj2_c2pT<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, R + rec.in[k], R + rec.al, Wb[k][cur],
                                                                           v[k], pacc);
                        k_adj2_ghost<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, k, R + rec.al, Wb[k][cur], carry[k]);
                        k_adj_comb<<<blocks((long long)nv), ADJ_WG, 0, s.stream>>>((long long)nv, lam[k], lam0[k], v[k],
                                                                                   A[q - 1], w, q == ns, q == 1);
                    }
                }
            }
            if (seg == 0) {
                // initial map alpha_k U(W_k) with the initial geometry (the
                // first record's); the first extension started from the
                // given primitives outside each fluid's real cells
                for (int k = 0; k < 2; k++) {
                    k_adj_prim0<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, s.tape_prim0 + (size_t)k * nv, lam[k],
                                                                        g_prim0 + (size_t)k * nv, store + rec.al, pacc);
                    k_adj_add<<<blocks((long long)nv), ADJ_WG, 0, s.stream>>>((long long)nv, g_prim0 + (size_t)k * nv,
                                                                              carry[k]);
                }
            }
        }
        s.ls_src.clear();
        s.ls_pos = 0;
        s.run_serial = serial;
        sim_status r2 = engine_restore(s, fin, fin + nv, fin + 2 * nv);
        if (r2 == SIM_OK && save_interaction(fin + 2 * nv + g.nc, true) != hipSuccess) r2 = SIM_EDEVICE;
        s.t = t_end;
        if (rc != SIM_OK) return rc;
        if (r2 != SIM_OK) return r2;
        return read_params(pacc, g_eos);
    }
    // ---- accelerated cycles (Sec. 3.1) with an interface ----
    // The segment's units (single-dt steps and accelerated cycles) are
    // recomputed by a forward composed of single engine operations in the
    // order of the method's steps, which records every interaction (its two
    // inputs, the extended primitives, p*, u*, the geometry and level set)
    // and the geometry of every mixing, and lists the operations; the
    // reverse walks that list backwards with one adjoint per state buffer
    // and, per interaction, the accumulated dJ/dp*, dJ/du* and primitive
    // adjoints, which it turns into its inputs' adjoints once every use of
    // the interaction is reversed.
    enum { BX0, BX1, BY0, BY1, BZ0, BZ1, BT2, BFH, BCORR, NBUF };
    enum OpKind { OP_IX, OP_STAGE, OP_MIX, OP_INTERP, OP_COPY, OP_CORR, OP_CORR_ZERO, OP_CORR_APPLY };
    struct Op {
        OpKind kind;
        int k, r, in, base, out;   // fluid, record (interaction or geometry), buffers
        double a, dt;              // stage coefficient and length; interpolation weight; correction weight
    };
    double* bufptr(int id) const
    {
        switch (id) {
        case BX0: return g.X[0];
        case BX1: return g.X[1];
        case BY0: return g.Y[0];
        case BY1: return g.Y[1];
        case BZ0: return g.Z[0];
        case BZ1: return g.Z[1];
        case BT2: return g.T2;
        case BFH: return g.Fh;
        default: return g.corr;
        }
    }

    sim_status sweep3(const double* g_cons, double* g_prim0, double* g_eos, std::vector<void*>& own)
    {
        const int ns = s.o.rk;
        const double* A = ns == 3 ? ADJ_RK3_A : ADJ_RK2_A;
        const double* B = ns == 3 ? ADJ_RK3_B : ADJ_RK2_B;
        const double* C = ns == 3 ? ADJ_RK3_C : ADJ_RK2_C;
        const size_t nv = (size_t)NV * g.nc, nc = (size_t)g.nc;
        const long long N = (long long)s.tape_units.size();
        const int K = s.o.ckpt_every;
        const long long nseg = (N + K - 1) / K;
        // records per unit: interactions and mixings
        auto counts = [&](const Sim::TapeUnit& u, size_t& nix, size_t& ngeo) {
            if (!u.cycle) { nix += ns; ngeo += 2 * ns; return; }
            const size_t m = u.sub.size();
            nix += 1 + (m - 1) + m * (ns - 1) + (ns == 3 ? 1 : 0);
            ngeo += (m - 1) + m * (ns - 1) + m * ns + (ns == 3 ? 1 : 0) + 1;
        };
        size_t maxix = 1, maxgeo = 1;
        for (long long seg = 0; seg < nseg; seg++) {
            size_t a = 0, b = 0;
            for (long long u = seg * K; u < std::min(N, (seg + 1) * K); u++) counts(s.tape_units[(size_t)u], a, b);
            maxix = std::max(maxix, a);
            maxgeo = std::max(maxgeo, b);
        }
        StageRec rec;
        rec.layout(D, nc, (size_t)g.nfc);
        const size_t gstride = 2 * nc;                       // geometry record: alpha, level set
        const size_t astride = 2 * nv + 2 * nc;              // per interaction: W-bar 0, 1, p*-bar, u*-bar
        double* store = alloc(own, sizeof(double) * rec.stride * maxix);
        double* geo = alloc(own, sizeof(double) * gstride * maxgeo);
        double* acc = alloc(own, sizeof(double) * astride * maxix);
        double* lam[NBUF];
        bool ok = store && geo && acc;
        for (int b = 0; b < NBUF; b++) ok = ok && (lam[b] = alloc(own, sizeof(double) * nv)) != nullptr;
        double* L = alloc(own, sizeof(double) * nv);
        double* v = alloc(own, sizeof(double) * nv);
        double* Wt = alloc(own, sizeof(double) * nv);
        double* Wx[2] = {alloc(own, sizeof(double) * nv), alloc(own, sizeof(double) * nv)};
        double* S = alloc(own, sizeof(double) * nv);
        double* tmp = alloc(own, sizeof(double) * nv);
        double* carry[2] = {alloc(own, sizeof(double) * nv), alloc(own, sizeof(double) * nv)};
        uint8_t* xcnt = reinterpret_cast<uint8_t*>(alloc(own, nc + 8));
        int* xidx = reinterpret_cast<int*>(alloc(own, sizeof(int) * (size_t)(2 * D + 1) * nc));
        double* xwt = alloc(own, sizeof(double) * (size_t)(2 * D + 1) * nc);
        double* fb = alloc(own, sizeof(double) * (size_t)max_faces() * 6 * NV);
        double* pacc = alloc(own, sizeof(double) * 4 * ADJ_BLOCKS);
        double* fin = alloc(own, sizeof(double) * (4 * nv + (3 + D) * nc));
        ok = ok && L && v && Wt && Wx[0] && Wx[1] && S && tmp && carry[0] && carry[1] && xcnt && xidx && xwt && fb &&
             pacc && fin;
        if (!ok) {
            set_error("adjoint buffers do not fit in device memory (%zu interaction records of %zu MB)", maxix,
                      sizeof(double) * rec.stride >> 20);
            return SIM_ENOMEM;
        }
        SHARP_HIP(hipMemcpyAsync(fin, g.X[0], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(hipMemcpyAsync(fin + nv, g.X[1], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(hipMemcpyAsync(fin + 2 * nv, g.phiP, sizeof(double) * nc, hipMemcpyDeviceToDevice, s.stream));
        SHARP_HIP(save_interaction(fin + 2 * nv + nc, false));
        SHARP_HIP(hipMemsetAsync(pacc, 0, sizeof(double) * 4 * ADJ_BLOCKS, s.stream));
        for (int b = 0; b < NBUF; b++) SHARP_HIP(hipMemsetAsync(lam[b], 0, sizeof(double) * nv, s.stream));
        for (int k = 0; k < 2; k++) {
            SHARP_HIP(hipMemcpyAsync(lam[BX0 + k], g_cons + (size_t)k * nv, sizeof(double) * nv,
                                     hipMemcpyDeviceToDevice, s.stream));
            SHARP_HIP(hipMemsetAsync(carry[k], 0, sizeof(double) * nv, s.stream));
        }
        const double t_end = s.t;
        const bool serial = s.run_serial;
        s.run_serial = true;
        g.use_sched = 0;
        s.ls_src.clear();
        for (double* p : s.tape_ls)
            for (int q = 0; q < ns; q++) s.ls_src.push_back(p + (size_t)q * nc);
        const int nb = blocks((long long)nv);
        std::vector<Op> ops;
        size_t nix = 0, ngeo = 0;
        // ---- recording helpers of the composed forward ----
        auto ix = [&](int id0, int id1, const double* cur) {
            double* b = store + nix * rec.stride;
            const double* in[2] = {bufptr(id0), bufptr(id1)};
            for (int k = 0; k < 2; k++) {
                (void)hipMemcpyAsync(b + rec.in[k], in[k], nv * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
                (void)hipMemcpyAsync(b + rec.W[k], g.Wb[k][s.wcur], nv * sizeof(double), hipMemcpyDeviceToDevice,
                                     s.stream);
            }
            (void)hipMemcpyAsync(b + rec.ps, g.ps, nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
            (void)hipMemcpyAsync(b + rec.us, g.us, nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
            (void)hipMemcpyAsync(b + rec.al, g.alpha, nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
            for (int d = 0; d < D; d++)
                (void)hipMemcpyAsync(b + rec.ap + (size_t)d * g.nfc, g.ap[d], (size_t)g.nfc * sizeof(double),
                                     hipMemcpyDeviceToDevice, s.stream);
            k_adj_phi<<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, cur, b + rec.phi);
            (void)hipMemcpyAsync(b + rec.M, g.M, nc, hipMemcpyDeviceToDevice, s.stream);
            ops.push_back({OP_IX, 0, (int)nix, id0, id1, 0, 0.0, 0.0});
            return (int)nix++;
        };
        auto mixop = [&](int k, int id, const double* cur) {
            engine_op_mix(s, k, bufptr(id), cur);
            double* b = geo + ngeo * gstride;
            (void)hipMemcpyAsync(b, g.alpha, nc * sizeof(double), hipMemcpyDeviceToDevice, s.stream);
            k_adj_phi<<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, cur, b + nc);
            ops.push_back({OP_MIX, k, (int)ngeo++, id, id, id, 0.0, 0.0});
        };
        auto stageop = [&](int k, int r, int in, int base, int out, double a, double dt) {
            engine_op_stage(s, k, bufptr(in), bufptr(base), bufptr(out), a, dt);
            ops.push_back({OP_STAGE, k, r, in, base, out, a, dt});
        };
        auto interp = [&](int S_, double th) {
            engine_op_axpby(s, 1.0 - th, bufptr(BX0 + S_), th, bufptr(BY0 + S_), g.T2);
            ops.push_back({OP_INTERP, S_, 0, BX0 + S_, BY0 + S_, BT2, th, 0.0});
        };
        const bool use_corr = !s.o.no_correction;
        auto corr = [&](int r, double w, int S_) {
            if (!use_corr) return;
            engine_op_corr_add(s, w, S_);
            ops.push_back({OP_CORR, S_, r, 0, 0, 0, w, 0.0});
        };
        sim_status rc = SIM_OK;
        for (long long seg = nseg - 1; seg >= 0 && rc == SIM_OK; seg--) {
            const long long u0 = seg * K, u1 = std::min(N, u0 + K);
            const double* ck = s.tape_ckpt[(size_t)seg];
            rc = engine_restore(s, ck, ck + nv, ck + 2 * nv);
            if (rc != SIM_OK) break;
            for (int k = 0; k < 2; k++)
                SHARP_HIP(hipMemcpyAsync(g.Wb[k][s.wcur], ck + 2 * nv + nc + (size_t)k * nv, sizeof(double) * nv,
                                         hipMemcpyDeviceToDevice, s.stream));
            SHARP_HIP(hipMemcpyAsync(g.ps, ck + 4 * nv + nc, sizeof(double) * nc, hipMemcpyDeviceToDevice, s.stream));
            SHARP_HIP(hipMemcpyAsync(g.us, ck + 4 * nv + 2 * nc, sizeof(double) * nc, hipMemcpyDeviceToDevice,
                                     s.stream));
            if (g.pj) k_adj2_jump<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, g.phiP);
            SHARP_HIP(hipMemsetAsync(g.corr, 0, sizeof(double) * nv, s.stream));
            s.ls_pos = s.tape_units[(size_t)u0].ls_block * ns;
            ops.clear();
            nix = ngeo = 0;
            // ---- the composed forward of the segment ----
            for (long long ui = u0; ui < u1 && rc == SIM_OK; ui++) {
                const Sim::TapeUnit& u = s.tape_units[(size_t)ui];
                if (ui > u0) rc = engine_op_prepare(s);
                if (rc != SIM_OK) break;
                if (!u.cycle) {
                    int in[2] = {BX0, BX1};
                    const double* phin = g.phiP;
                    for (int q = 0; q < ns; q++) {
                        if (q > 0) engine_op_interaction(s, bufptr(in[0]), bufptr(in[1]), phin);
                        const int r = ix(in[0], in[1], phin);
                        int out[2];
                        for (int k = 0; k < 2; k++) {
                            out[k] = q == ns - 1 ? BX0 + k : (q == 0 ? BY0 + k : BZ0 + k);
                            stageop(k, r, in[k], BX0 + k, out[k], A[q], u.t1);
                        }
                        const double* cur = engine_op_ls(s, q, q == ns - 1, A[q], u.t1, phin);
                        for (int k = 0; k < 2; k++) mixop(k, out[k], cur);
                        in[0] = out[0];
                        in[1] = out[1];
                        phin = cur;
                    }
                    continue;
                }
                const int Sf = u.S, F = 1 - Sf;
                const double t1 = u.t1;
                const int XS = BX0 + Sf, XF = BX0 + F;
                auto order = [&](int sid, int fid, int& id0, int& id1) {
                    id0 = Sf == 0 ? sid : fid;
                    id1 = Sf == 0 ? fid : sid;
                };
                const int r0 = ix(BX0, BX1, g.phiP);
                ops.push_back({OP_CORR_ZERO, 0, 0, 0, 0, 0, 0.0, 0.0});
                stageop(Sf, r0, XS, XS, BY0 + Sf, A[0], t1);
                double tau = 0.0;
                int last = r0;
                for (size_t j = 0; j < u.sub.size(); j++) {
                    const double dl = u.sub[j].dl;
                    const int hh = u.sub[j].hh, fin_ = u.sub[j].fin;
                    int in = XF;
                    const double* phin = g.phiP;
                    if (j > 0) {
                        engine_op_mask(s);
                        interp(Sf, tau / t1);
                        mixop(Sf, BT2, g.phiP);
                        int i0, i1;
                        order(BT2, XF, i0, i1);
                        engine_op_interaction(s, bufptr(i0), bufptr(i1), g.phiP);
                        last = ix(i0, i1, g.phiP);
                    } else {
                        corr(r0, -B[0] * t1 + B[0] * dl, Sf);
                    }
                    for (int q = 0; q < ns; q++) {
                        if (q > 0) {
                            const bool shared = fin_ && C[q] == 1.0;
                            const double th = shared ? 1.0 : (tau + C[q] * dl) / t1;
                            interp(Sf, th);
                            mixop(Sf, BT2, phin);
                            int i0, i1;
                            order(BT2, in, i0, i1);
                            engine_op_interaction(s, bufptr(i0), bufptr(i1), phin);
                            last = ix(i0, i1, phin);
                            corr(last, shared ? -B[q] * t1 + B[q] * dl : B[q] * dl, Sf);
                            if (shared) stageop(Sf, last, BT2, XS, ns == 2 ? XS : BZ0 + Sf, A[q], t1);
                        } else if (j > 0) {
                            corr(last, B[0] * dl, Sf);
                        }
                        const int out = q == ns - 1 ? XF : (q == 0 ? BY0 + F : BZ0 + F);
                        stageop(F, last, in, XF, out, A[q], dl);
                        const double* cur = engine_op_ls(s, q, q == ns - 1, A[q], dl, phin);
                        mixop(F, out, cur);
                        in = out;
                        phin = cur;
                    }
                    tau = hh ? 0.5 * t1 : (fin_ ? t1 : tau + dl);
                    if (hh) {
                        SHARP_HIP(hipMemcpyAsync(g.Fh, g.X[F], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
                        SHARP_HIP(hipMemcpyAsync(g.phiH, g.phiP, sizeof(double) * nc, hipMemcpyDeviceToDevice,
                                                 s.stream));
                        ops.push_back({OP_COPY, 0, 0, XF, 0, BFH, 0.0, 0.0});
                    }
                }
                if (ns == 3) {
                    engine_op_geom(s, g.phiH);
                    SHARP_HIP(hipMemcpyAsync(g.T2, g.Z[Sf], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
                    ops.push_back({OP_COPY, 0, 0, BZ0 + Sf, 0, BT2, 0.0, 0.0});
                    mixop(Sf, BT2, g.phiH);
                    int i0, i1;
                    order(BT2, BFH, i0, i1);
                    engine_op_interaction(s, bufptr(i0), bufptr(i1), g.phiH);
                    const int rh = ix(i0, i1, g.phiH);
                    corr(rh, -B[2] * t1, Sf);
                    stageop(Sf, rh, BT2, XS, XS, A[2], t1);
                    engine_op_geom(s, g.phiP);
                }
                if (use_corr) {
                    engine_op_corr_apply(s, Sf);
                    ops.push_back({OP_CORR_APPLY, Sf, 0, 0, 0, 0, 0.0, 0.0});
                }
                mixop(Sf, XS, g.phiP);
            }
            if (rc != SIM_OK) break;
            // ---- the reverse of the segment ----
            SHARP_HIP(hipMemsetAsync(acc, 0, sizeof(double) * astride * nix, s.stream));
            for (size_t oi = ops.size(); oi-- > 0;) {
                const Op& o = ops[oi];
                switch (o.kind) {
                case OP_CORR_APPLY:
                    k_adj2_corrT<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, lam[BX0 + o.k], lam[BCORR]);
                    break;
                case OP_MIX: {
                    const double* gr = geo + (size_t)o.r * gstride;
                    k_adj2_mixT<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, o.k, gr, gr + nc, lam[o.out], tmp);
                    std::swap(lam[o.out], tmp);
                    break;
                }
                case OP_INTERP:
                    k_adj_axpby<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, lam[o.in], 1.0, lam[o.out], 1.0 - o.a);
                    k_adj_axpby<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, lam[o.base], 1.0, lam[o.out], o.a);
                    SHARP_HIP(hipMemsetAsync(lam[o.out], 0, sizeof(double) * nv, s.stream));
                    break;
                case OP_COPY:
                    k_adj_add<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, lam[o.in], lam[o.out]);
                    SHARP_HIP(hipMemsetAsync(lam[o.out], 0, sizeof(double) * nv, s.stream));
                    break;
                case OP_CORR_ZERO:
                    SHARP_HIP(hipMemsetAsync(lam[BCORR], 0, sizeof(double) * nv, s.stream));
                    break;
                case OP_CORR: {
                    const double* R = store + (size_t)o.r * rec.stride;
                    double* a = acc + (size_t)o.r * astride;
                    const double sg = o.k == 0 ? 1.0 : -1.0;
                    k_adj2_xacc<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, R + rec.ap, R + rec.ps, R + rec.us,
                                                                         lam[BCORR], sg * o.a, a + 2 * nv,
                                                                         a + 2 * nv + nc, o.k, R + rec.phi);
                    break;
                }
                case OP_STAGE: {
                    const double* R = store + (size_t)o.r * rec.stride;
                    double* a = acc + (size_t)o.r * astride;
                    const int k = o.k;
                    const double w = 1.0 - o.a, sg = k == 0 ? 1.0 : -1.0;
                    SHARP_HIP(hipMemcpyAsync(L, lam[o.out], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
                    SHARP_HIP(hipMemsetAsync(lam[o.out], 0, sizeof(double) * nv, s.stream));
                    if (o.a != 0.0) k_adj_axpby<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, lam[o.base], 1.0, L, o.a);
                    k_adj2_sten<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, k, R + rec.in[k], R + rec.al, R + rec.W[k],
                                                                         S);
                    jlt(k, S, L, w * o.dt, v, fb, pacc, R + rec.ap);
                    k_adj2_split<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, R + rec.al, R + rec.W[k], v, Wt, pacc);
                    k_adj_add<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, a + (size_t)k * nv, Wt);
                    k_adj_axpby<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, lam[o.in], 1.0, L, w);
                    k_adj_add<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, lam[o.in], v);
                    k_adj2_xacc<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, R + rec.ap, R + rec.ps, R + rec.us, L,
                                                                         sg * w * o.dt, a + 2 * nv, a + 2 * nv + nc,
                                                                         k, R + rec.phi);
                    break;
                }
                case OP_IX: {
                    const double* R = store + (size_t)o.r * rec.stride;
                    double* a = acc + (size_t)o.r * astride;
                    k_adj2_riemann2<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, R + rec.ap, R + rec.W[0], R + rec.W[1],
                                                                           R + rec.ps, a + 2 * nv, a + 2 * nv + nc,
                                                                           a, a + nv, pacc, R + rec.phi);
                    const uint8_t* Mk = reinterpret_cast<const uint8_t*>(R + rec.M);
                    const int ids[2] = {o.in, o.base};
                    for (int k = 0; k < 2; k++) {
                        SHARP_HIP(hipMemcpyAsync(Wx[0], a + (size_t)k * nv, sizeof(double) * nv,
                                                 hipMemcpyDeviceToDevice, s.stream));
                        k_adj_add<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, Wx[0], carry[k]);
                        int cur = 0;
                        if (s.o.ext_iters > 0)
                            k_adj2_extprep<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, k, R + rec.phi, R + rec.al, Mk,
                                                                                    xcnt, xidx, xwt);
                        for (int it = 0; it < s.o.ext_iters; it++) {
                            k_adj2_extT2<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, xcnt, xidx, xwt, Wx[cur],
                                                                                  Wx[1 - cur]);
                            cur ^= 1;
                        }
                        k_adj2_c2pT<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, R + rec.in[k], R + rec.al, Wx[cur],
                                                                           lam[ids[k]], pacc);
                        k_adj2_ghost<D><<<blocks(g.nc), ADJ_WG, 0, s.stream>>>(g, k, R + rec.al, Wx[cur], carry[k]);
                    }
                    break;
                }
                }
            }
            if (seg == 0) {
                for (int k = 0; k < 2; k++) {
                    k_adj_prim0<D><<<ADJ_BLOCKS, ADJ_WG, 0, s.stream>>>(g, k, s.tape_prim0 + (size_t)k * nv,
                                                                        lam[BX0 + k], g_prim0 + (size_t)k * nv,
                                                                        store + rec.al, pacc);
                    k_adj_add<<<nb, ADJ_WG, 0, s.stream>>>((long long)nv, g_prim0 + (size_t)k * nv, carry[k]);
                }
            }
        }
        s.ls_src.clear();
        s.ls_pos = 0;
        s.run_serial = serial;
        sim_status r2 = engine_restore(s, fin, fin + nv, fin + 2 * nv);
        if (r2 == SIM_OK && save_interaction(fin + 2 * nv + g.nc, true) != hipSuccess) r2 = SIM_EDEVICE;
        SHARP_HIP(hipMemsetAsync(g.corr, 0, sizeof(double) * nv, s.stream));
        s.t = t_end;
        if (rc != SIM_OK) return rc;
        if (r2 != SIM_OK) return r2;
        return read_params(pacc, g_eos);
    }
};

}  // namespace

void tape_clear(Sim& s)
{
    for (double* p : s.tape_ckpt) (void)hipFree(p);
    s.tape_ckpt.clear();
    for (double* p : s.tape_ls) (void)hipFree(p);
    s.tape_ls.clear();
    s.tape_units.clear();
    s.tape_dt.clear();
    if (s.tape_prim0) (void)hipFree(s.tape_prim0);
    s.tape_prim0 = nullptr;
    s.tape_fluid = -1;
}

sim_status tape_begin(Sim& s, const double* prim_dev)
{
    tape_clear(s);
    const bool none0 = s.bulk_cells[0] == 0, none1 = s.bulk_cells[1] == 0;
    // one fluid fills the grid (k), or an interface (2): both fluids
    const bool two = s.lcount[LIST_BAND] != 0 || none0 == none1;
    const int k = two ? 2 : (none0 ? 1 : 0);
    const size_t nv = (size_t)(s.g.D + 2) * s.g.nc, n0 = two ? 2 * nv : nv;
    if (hipMalloc((void**)&s.tape_prim0, sizeof(double) * n0) != hipSuccess) {
        (void)hipGetLastError();
        s.tape_prim0 = nullptr;
        set_error("tape allocation failed");
        return SIM_ENOMEM;
    }
    SHARP_HIP(hipMemcpyAsync(s.tape_prim0, prim_dev + (two ? 0 : (size_t)k * nv), sizeof(double) * n0,
                             hipMemcpyDeviceToDevice, s.stream));
    s.tape_fluid = k;
    s.tape_why.clear();
    return SIM_OK;
}

// a checkpoint of a two-fluid tape: contents, level set, and what the
// unit's start interaction left
static sim_status tape_checkpoint2(Sim& s)
{
    const size_t nv = (size_t)(s.g.D + 2) * s.g.nc, nc = (size_t)s.g.nc;
    double* p = nullptr;
    if (hipMalloc((void**)&p, sizeof(double) * (4 * nv + 3 * nc)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("tape checkpoint allocation failed");
        return SIM_ENOMEM;
    }
    s.tape_ckpt.push_back(p);
    SHARP_HIP(hipMemcpyAsync(p, s.g.X[0], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
    SHARP_HIP(hipMemcpyAsync(p + nv, s.g.X[1], sizeof(double) * nv, hipMemcpyDeviceToDevice, s.stream));
    SHARP_HIP(hipMemcpyAsync(p + 2 * nv, s.g.phiP, sizeof(double) * nc, hipMemcpyDeviceToDevice, s.stream));
    for (int k = 0; k < 2; k++)
        SHARP_HIP(hipMemcpyAsync(p + 2 * nv + nc + (size_t)k * nv, s.g.Wb[k][s.wcur], sizeof(double) * nv,
                                 hipMemcpyDeviceToDevice, s.stream));
    SHARP_HIP(hipMemcpyAsync(p + 4 * nv + nc, s.g.ps, sizeof(double) * nc, hipMemcpyDeviceToDevice, s.stream));
    SHARP_HIP(hipMemcpyAsync(p + 4 * nv + 2 * nc, s.g.us, sizeof(double) * nc, hipMemcpyDeviceToDevice, s.stream));
    return SIM_OK;
}

// one block of stage level sets (a single-dt step or a fast sub-step)
static sim_status tape_ls_block(Sim& s)
{
    double* p = nullptr;
    if (hipMalloc((void**)&p, sizeof(double) * (size_t)s.o.rk * s.g.nc) != hipSuccess) {
        (void)hipGetLastError();
        set_error("level-set tape allocation failed");
        return SIM_ENOMEM;
    }
    s.tape_ls.push_back(p);
    return SIM_OK;
}

sim_status tape_cycle(Sim& s, int S, double t1)
{
    if (s.tape_fluid != 2) return SIM_OK;
    if (s.tape_units.size() % (size_t)s.o.ckpt_every == 0) {
        sim_status rc = tape_checkpoint2(s);
        if (rc != SIM_OK) return rc;
    }
    Sim::TapeUnit u;
    u.cycle = 1;
    u.S = S;
    u.t1 = t1;
    u.ls_block = s.tape_ls.size();
    s.tape_units.push_back(u);
    return SIM_OK;
}

sim_status tape_sub(Sim& s)
{
    if (s.tape_fluid != 2 || s.tape_units.empty()) return SIM_OK;
    s.tape_units.back().sub.push_back({0.0, 0, 0});
    return tape_ls_block(s);
}

sim_status tape_step(Sim& s, double dt)
{
    if (s.tape_fluid < 0) return SIM_OK;
    const size_t nv = (size_t)(s.g.D + 2) * s.g.nc;
    const bool two = s.tape_fluid == 2;
    if (two) {
        if (s.tape_units.size() % (size_t)s.o.ckpt_every == 0) {
            sim_status rc = tape_checkpoint2(s);
            if (rc != SIM_OK) return rc;
        }
        Sim::TapeUnit u;
        u.t1 = dt;
        u.ls_block = s.tape_ls.size();
        s.tape_units.push_back(u);
        sim_status rc = tape_ls_block(s);
        if (rc != SIM_OK) return rc;
        s.tape_dt.push_back(dt);
        return SIM_OK;
    }
    if (s.tape_dt.size() % (size_t)s.o.ckpt_every == 0) {
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
    if (s.ls_stream) (void)hipStreamSynchronize(s.ls_stream);
    if (s.snap_stream) (void)hipStreamSynchronize(s.snap_stream);
    s.snap_pending = false;   // the cycle-start copies are complete
    switch (s.g.D) {
    case 1: return Adjoint<1>(s).run(g_cons, g_prim0, g_eos);
    case 2: return Adjoint<2>(s).run(g_cons, g_prim0, g_eos);
    default: return Adjoint<3>(s).run(g_cons, g_prim0, g_eos);
    }
}

}  // namespace sharp
