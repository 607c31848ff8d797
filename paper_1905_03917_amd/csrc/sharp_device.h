// sharp_device.h -- device-side building blocks of the gfx950 path of the
// accelerated sharp-interface method (Long, Cai & Pan, Sec. 2 and 3.1).
//
// Everything here is per-cell or per-face arithmetic used by the kernels in
// sharp_kernels.hip: stiffened-gas EOS, WENO5 reconstruction, the exact
// two-material Riemann problem of the interface interaction, and the
// level-set geometry (vertex values, apertures, volume fraction).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SHARP_WG 256

namespace sharp {

// ---------------------------------------------------------------------------
// Block coordinates seen by a kernel body: the block's index among the blocks
// working on one simulation, and their number.  A launch for one simulation
// passes its grid; a fused launch over several simulations passes each
// block's place in its own simulation's share of the grid.
// ---------------------------------------------------------------------------
struct VB {
    int b, n;
    static __device__ __forceinline__ VB grid() { return {(int)blockIdx.x, (int)gridDim.x}; }
};

// ---------------------------------------------------------------------------
// Device view of one simulation: grid, tiling, parameters and buffers.
// Passed by value to every kernel.
// ---------------------------------------------------------------------------
struct Dev {
    int D;            // 1, 2, 3
    int n[3];         // cells per direction (1 if unused)
    int nf[3];        // padded face lattice (n+1 in active directions)
    int nc;           // number of cells
    int nfc;          // number of padded faces per direction array
    int T[3];         // tile dims
    int nt[3];        // tiles per direction
    int ntiles;
    int bc[3];        // 0 zero-gradient, 1 periodic
    double h;
    double gam[2], pinf[2];
    double amix, lsb, extb, mixb, eps;
    int bface_off[3][2];  // offsets of the boundary-face accumulators
    int nbface;
    // state
    double* X[2];
    double* Y[2];
    double* Z[2];
    double* T2;       // slow-fluid temporary (interpolated and mixed)
    double* Tm[2];    // per fluid: band-stage output of the inner tiles, before mixing
    double* Fh;       // fast-fluid snapshot at t1/2
    double* Wb[2][2]; // primitives, two Jacobi buffers per fluid
    double* phiP;     // level set, base/current
    double* phiB[3];  // level-set stage / reinitialisation buffers
    double* phiH;     // level-set snapshot at t1/2
    double* alpha;    // fluid-0 volume fraction
    double* ap[3];    // fluid-0 aperture of the low face, padded index
    double* ps;       // interface pressure (cut cells)
    double* us;       // interface normal velocity (cut cells)
    double* ss[2];    // star-state CFL speed per fluid (cut cells)
    double sigma;     // surface tension coefficient (0: none)
    double* pj;       // with sigma: Laplace jump sigma kappa per cut cell; fluid 1's
                      // interface pressure is ps - pj (nullptr without sigma)
    double* v[2][3];  // level-set velocity, two Jacobi buffers
    uint8_t* M;       // band mask of the (sub)step
    uint8_t* nearif;  // sign change within the 3^D neighbourhood (reinit)
    double* corr;     // interfacial flux correction [NV][cells]
    double* dmix;     // mixing increments [NV][cells]
    double* bacc[2];  // boundary inflow accumulators [NV][nbface]
    // tiles
    double* tphimin;  // per tile: min |phi| over the tile and its one-cell halo at the last geometry
    // 3-D extension: the first Jacobi sweep of each extension records its
    // targets and their upwind stencils; the later sweeps walk these lists.
    // Wave w of the tile at inner-list position ti owns the slots from
    // (4 ti + w) * WL_WAVE (primitives) or * VL_WAVE (velocity).
    int* wl_n;        // [4 ntiles] entries per wave, primitive list
    int* wl_c;        // primitive list: cell | fluid << 31
    int* wl_up;       // [3][wl_cap] upwind neighbours
    double* wl_w;     // [4][wl_cap] weights along x, y, z and their sum
    int* vl_n;        // [4 ntiles] entries per wave, velocity list
    int* vl_c;        // velocity list: cell
    int* vl_up;       // [3][vl_cap]
    double* vl_w;     // [4][vl_cap]
    int wl_cap, vl_cap;
    int* tcore;       // tile holds band cells
    int* tflag;       // bit0 band tile, bit1 candidate tile, bit2 ring tile
    int* tsign;       // fluid of a tile outside the band
    int* lists;       // [6][ntiles]: band, candidate, bulk0, bulk1, all, inner
    int* counts;      // [16]: tiles per list (0..5), cells per list (8 + list, lists 0..3 and 5)
    // scalars
    unsigned long long* red;   // [0..1] max speed bits, [2..3] active counts, [4] error flags
    // schedule of a fast sub-step planned on the device (SCHED_* slots); with
    // use_sched set, the kernels of its first stage take dt and the weights
    // from there instead of their arguments
    double* sched;
    int use_sched;
};
enum { SCHED_DT = 0, SCHED_W0 = 1, SCHED_TH1 = 2, SCHED_HH = 3, SCHED_FIN = 4, SCHED_DTF = 5, SCHED_CNT = 6 };

// band: tiles within one tile of a band-mask tile; inner: band tiles all of
// whose neighbours are band tiles (every band-mask cell of a cycle lies in
// one, or the cycle fails with a band overflow)
enum { LIST_BAND = 0, LIST_CAND = 1, LIST_BULK0 = 2, LIST_BULK1 = 3, LIST_ALL = 4, LIST_INNER = 5, NLISTS = 6 };
enum { ERR_NONPHYS = 1, ERR_BAND_OVERFLOW = 2 };

// ---------------------------------------------------------------------------
// indexing
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bcmap(int i, int n, int bc)
{
    if (bc == 1) { i %= n; return i < 0 ? i + n : i; }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ __forceinline__ int cidx(const Dev& g, int i, int j, int k)
{
    i = bcmap(i, g.n[0], g.bc[0]);
    j = g.D > 1 ? bcmap(j, g.n[1], g.bc[1]) : 0;
    k = g.D > 2 ? bcmap(k, g.n[2], g.bc[2]) : 0;
    return i + g.n[0] * (j + g.n[1] * k);
}

__device__ __forceinline__ int fidx(const Dev& g, int i, int j, int k)
{
    return i + g.nf[0] * (j + g.nf[1] * k);
}

__device__ __forceinline__ void coords(const Dev& g, int c, int& i, int& j, int& k)
{
    i = c % g.n[0];
    j = (c / g.n[0]) % g.n[1];
    k = c / (g.n[0] * g.n[1]);
}

__device__ __forceinline__ int nbr(const Dev& g, int c, int d, int off)
{
    int i, j, k;
    coords(g, c, i, j, k);
    if (d == 0) i += off; else if (d == 1) j += off; else k += off;
    return cidx(g, i, j, k);
}

// level set of the (sub)step: band cells are read from the working buffer,
// every other cell keeps its value in the base buffer
__device__ __forceinline__ double phi_at(const Dev& g, const double* cur, int c)
{
    return g.M[c] ? cur[c] : g.phiP[c];
}

// ---------------------------------------------------------------------------
// stiffened-gas EOS
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void prim2cons(double gm, double pi, const double* W, double* U)
{
    double rho = W[0], ke = 0.0;
    U[0] = rho;
#pragma unroll
    for (int d = 0; d < D; d++) { U[1 + d] = rho * W[1 + d]; ke += W[1 + d] * W[1 + d]; }
    U[D + 1] = (W[D + 1] + gm * pi) / (gm - 1.0) + 0.5 * rho * ke;
}

template <int D>
__device__ __forceinline__ bool cons2prim(double gm, double pi, const double* U, double* W)
{
    double rho = U[0], ir = 1.0 / rho, ke = 0.0;
    W[0] = rho;
#pragma unroll
    for (int d = 0; d < D; d++) { W[1 + d] = U[1 + d] * ir; ke += W[1 + d] * W[1 + d]; }
    double p = (gm - 1.0) * (U[D + 1] - 0.5 * rho * ke) - gm * pi;
    W[D + 1] = p;
    return (rho > 0.0) && (p + pi > 0.0) && isfinite(p);
}

__device__ __forceinline__ double csound(double gm, double pi, double rho, double p)
{
    return sqrt(gm * (p + pi) / rho);
}

// ---------------------------------------------------------------------------
// WENO5 (Jiang & Shu), left-biased value at the right edge of v2, written
// with a single division: the normalised nonlinear weights share the common
// factor prod_r (eps + beta_r)^2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double weno5(double v0, double v1, double v2, double v3, double v4, double eps)
{
    const double c13_12 = 13.0 / 12.0;
    double q0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) * (1.0 / 6.0);
    double q1 = (-v1 + 5.0 * v2 + 2.0 * v3) * (1.0 / 6.0);
    double q2 = (2.0 * v2 + 5.0 * v3 - v4) * (1.0 / 6.0);
    double t0 = v0 - 2.0 * v1 + v2, u0 = v0 - 4.0 * v1 + 3.0 * v2;
    double t1 = v1 - 2.0 * v2 + v3, u1 = v1 - v3;
    double t2 = v2 - 2.0 * v3 + v4, u2 = 3.0 * v2 - 4.0 * v3 + v4;
    double e0 = eps + c13_12 * t0 * t0 + 0.25 * u0 * u0;
    double e1 = eps + c13_12 * t1 * t1 + 0.25 * u1 * u1;
    double e2 = eps + c13_12 * t2 * t2 + 0.25 * u2 * u2;
    double s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
    double w0 = 0.1 * (s1 * s2), w1 = 0.6 * (s0 * s2), w2 = 0.3 * (s0 * s1);
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

// Reciprocal: hardware estimate refined by two Newton steps (within a few
// ulp of the correctly rounded quotient).
__device__ __forceinline__ double rcp_nr(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
}

// WENO5 of the face flux in the form used by the stage kernels: for
// v = F +- a U (the LLF split flux without its factor 1/2) returns num/den
// with value = num / (6 den); eps4 = 4 eps keeps the weights identical to
// weno5(v/2, eps), since the smoothness indicators are quadratic in v.
__device__ __forceinline__ double weno5_q(double v0, double v1, double v2, double v3, double v4, double eps4)
{
    const double c13_12 = 13.0 / 12.0;
    double P0 = 2.0 * v0 - 7.0 * v1 + 11.0 * v2;
    double P1 = -v1 + 5.0 * v2 + 2.0 * v3;
    double P2 = 2.0 * v2 + 5.0 * v3 - v4;
    double t0 = v0 - 2.0 * v1 + v2, u0 = v0 - 4.0 * v1 + 3.0 * v2;
    double t1 = v1 - 2.0 * v2 + v3, u1 = v1 - v3;
    double t2 = v2 - 2.0 * v3 + v4, u2 = 3.0 * v2 - 4.0 * v3 + v4;
    double e0 = fma(c13_12 * t0, t0, fma(0.25 * u0, u0, eps4));
    double e1 = fma(c13_12 * t1, t1, fma(0.25 * u1, u1, eps4));
    double e2 = fma(c13_12 * t2, t2, fma(0.25 * u2, u2, eps4));
    double s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
    double w0 = s1 * s2, w1 = 6.0 * (s0 * s2), w2 = 3.0 * (s0 * s1);
    return (w0 * P0 + w1 * P1 + w2 * P2) * rcp_nr(w0 + w1 + w2);
}

// ---------------------------------------------------------------------------
// exact Riemann problem of two stiffened gases (wave curves in p + p_inf)
// ---------------------------------------------------------------------------
struct Side { double rho, u, p, g, pi; };

// Positive powers x^y (x >= 0, |y log x| moderate) for the rarefaction
// branches, as exp(y log x) with short, branch-free evaluations:
//  - log: x = m 2^e, m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s) with
//    s = (m - 1)/(m + 1), |s| <= 0.172, summed as its Taylor series in s^2
//    through s^21 (truncation below 1e-18 relative);
//  - exp: y = k ln 2 + r, |r| <= ln 2 / 2, by Cody-Waite reduction with ln 2
//    split into a 29-bit head (k * head exact) and a tail; exp r by its
//    Taylor series through r^13 (truncation below 1e-17 relative).
// A few ulp against a correctly rounded power; the Riemann solver only needs
// its root to 1e-13.
constexpr double LN2_HI = 0x1.62e42ffp-1;                 // 29 significant bits
constexpr double LN2_LO = -4.2009150726810846e-11;        // ln 2 - LN2_HI
constexpr double INV_LN2 = 1.4426950408889634;

__host__ __device__ __forceinline__ double log_pos(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752) { m *= 2.0; e -= 1; }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = fma(p, z, 1.0);
    double de = (double)e;
    return fma(de, LN2_HI, fma(de, LN2_LO, 2.0 * s * p));
}

__host__ __device__ __forceinline__ double exp_fin(double y)
{
    double k = rint(y * INV_LN2);
    double r = fma(-k, LN2_HI, y);
    r = fma(-k, LN2_LO, r);
    double p = 1.0 / 6227020800.0;           // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

__host__ __device__ __forceinline__ double pow_pos(double x, double y)
{
    return x > 0.0 ? exp_fin(y * log_pos(x)) : 0.0;
}

// One side of the two-material Riemann problem with its p-independent
// constants: shock branch f = (p - p_s) sqrt(A / (p + p_inf + B)),
// rarefaction branch f = 2c/(g-1) (((p + p_inf)/(p_s + p_inf))^((g-1)/(2g)) - 1).
struct WaveSide {
    double p, pi, g, rho;
    double A, B;          // shock
    double e, cf, irc, ipk;   // rarefaction: exponent, 2c/(g-1), 1/(rho c), 1/(p_s + p_inf)
};

__device__ __forceinline__ WaveSide wave_side(const Side& s)
{
    WaveSide w;
    double pk = s.p + s.pi, c = csound(s.g, s.pi, s.rho, s.p);
    w.p = s.p;
    w.pi = s.pi;
    w.g = s.g;
    w.rho = s.rho;
    w.A = 2.0 / ((s.g + 1.0) * s.rho);
    w.B = (s.g - 1.0) / (s.g + 1.0) * pk;
    w.e = (s.g - 1.0) / (2.0 * s.g);
    w.cf = 2.0 * c / (s.g - 1.0);
    w.irc = 1.0 / (s.rho * c);
    w.ipk = 1.0 / pk;
    return w;
}

// f and f' of one side at p; both branches are evaluated (independent
// chains, no divergence) and the one for p is selected.  rz returns the
// rarefaction factor ((p + p_inf)/(p_s + p_inf))^((g-1)/(2g)).
__device__ __forceinline__ double wave_fs(const WaveSide& w, double p, double& df, double& rz)
{
    double pb = p + w.pi;
    double t = 1.0 / (pb + w.B);
    double q = sqrt(w.A * t);
    double fs = (p - w.p) * q;
    double dfs = q * (1.0 - 0.5 * (p - w.p) * t);
    double r = pb * w.ipk;
    rz = pow_pos(r, w.e);
    double fr = w.cf * (rz - 1.0);
    double dfr = rz * w.irc / r;
    bool shock = p > w.p;
    df = shock ? dfs : dfr;
    return shock ? fs : fr;
}

// star-state density behind the wave of side w at p (rz from wave_fs at p):
// shock Hugoniot, or the isentrope rho (r)^(1/g) = rho r / rz^2
__device__ __forceinline__ double star_rho_w(const WaveSide& w, double p, double rz)
{
    double pb = p + w.pi;
    if (pb <= 0.0) return 0.0;
    double r = pb * w.ipk;
    if (p > w.p) {
        double m = (w.g - 1.0) / (w.g + 1.0);
        return w.rho * (r + m) / (m * r + 1.0);
    }
    return w.rho * r / (rz * rz);
}

// Exact two-material Riemann problem: the root p* of
//   f(p) = f_L(p) + f_R(p) + (u_R - u_L),
// which is increasing in p, by safeguarded Newton iteration; p* is the floor
// -min(p_inf) when f(floor) >= 0.  out: p*, u*, rho*_L, rho*_R.
// p0 is a start value (the cell's previous solution); when it does not lie
// above the floor, the geometric mean of the side pressures (relative to the
// floor) starts the iteration.  The floor value f(floor) is evaluated only
// when an iterate would leave the bracket through the floor: if the root lies
// above the floor the iterates never depend on it, and if it does not, every
// Newton step moves down until one reaches the floor.
__device__ inline void riemann(const Side& L, const Side& R, double p0, double* out)
{
    const WaveSide wl = wave_side(L), wr = wave_side(R);
    double du = R.u - L.u, dfl, dfr, rzl, rzr;
    double pfloor = -(L.pi < R.pi ? L.pi : R.pi);
    double p;
    if (p0 > pfloor && p0 < INFINITY) {
        p = p0;
    } else if (L.p > pfloor && R.p > pfloor) {
        p = pfloor + sqrt((L.p - pfloor) * (R.p - pfloor));
    } else {
        double cL = csound(L.g, L.pi, L.rho, L.p), cR = csound(R.g, R.pi, R.rho, R.p);
        p = 0.5 * (L.p + R.p) - 0.125 * du * (L.rho + R.rho) * (cL + cR);
        double pmax = L.p > R.p ? L.p : R.p;
        if (!(p > pfloor)) p = pfloor + 0.5 * (pmax - pfloor);
    }
    double lo = pfloor, hi = INFINITY;
    double scale = fabs(L.pi) + fabs(R.pi) + 1e-300;
    bool floor_known = false, at_floor = false;
    for (int it = 1; it <= 200; it++) {
        double f = wave_fs(wl, p, dfl, rzl) + wave_fs(wr, p, dfr, rzr) + du;
        if (f > 0.0) { if (p < hi) hi = p; }
        else { if (p > lo) lo = p; }
        double pn = p - f / (dfl + dfr);
        if (fabs(pn - p) <= 1e-13 * (fabs(p) + scale)) {
            // converged: a step this small can fall below the rounding of p
            // (pn == p == lo), which the bracket test below would take for
            // a step out of the bracket and answer with a bisection away
            // from the root
            if (pn > lo && pn < hi) p = pn;
            break;
        }
        if (!(pn > lo && pn < hi)) {
            if (!floor_known && !(pn > lo) && lo == pfloor) {
                floor_known = true;
                if (wave_fs(wl, pfloor, dfl, rzl) + wave_fs(wr, pfloor, dfr, rzr) + du >= 0.0) {
                    at_floor = true;
                    break;
                }
            }
            pn = isfinite(hi) ? 0.5 * (lo + hi) : lo + 2.0 * (p - lo);
        }
        double dp = pn - p;
        p = pn;
        if (fabs(dp) <= 1e-13 * (fabs(p) + scale)) break;
    }
    if (at_floor) p = pfloor;
    double fl = wave_fs(wl, p, dfl, rzl), fr = wave_fs(wr, p, dfr, rzr);
    out[0] = p;
    out[1] = 0.5 * (L.u + R.u) + 0.5 * (fr - fl);
    out[2] = star_rho_w(wl, p, rzl);
    out[3] = star_rho_w(wr, p, rzr);
}

// Laplace pressure jump sigma kappa of Eq. (surfacetension) at cut cell
// (i, j, k): kappa = div(grad phi / |grad phi|) = (|G|^2 tr H - G.H.G) / |G|^3
// with G and H from central differences of phi, positive where fluid 0 is
// convex, moved from the cell centre to the nearest interface point as for
// a circle or sphere (each principal curvature k at distance phi is
// k / (1 + phi k)): kappa / (1 - phi kappa / (D - 1)), the denominator held
// at >= 1/2; 0 in 1-D
template <int D>
__device__ __forceinline__ double laplace_jump(const Dev& g, const double* phi, int i, int j, int k)
{
    if constexpr (D < 2) {
        return 0.0;
    } else {
        const double pc = phi[i + g.n[0] * (j + g.n[1] * k)];
        const double h = g.h;
        double G[D], H[D][D];
#pragma unroll
        for (int d = 0; d < D; d++) {
            const int u = d == 0, v = d == 1, w = d == 2;
            const double pp = phi[cidx(g, i + u, j + v, k + w)], pm = phi[cidx(g, i - u, j - v, k - w)];
            G[d] = (pp - pm) / (2.0 * h);
            H[d][d] = (pp - 2.0 * pc + pm) / (h * h);
#pragma unroll
            for (int e = d + 1; e < D; e++) {
                const int a = e == 0, b = e == 1, f = e == 2;
                const double q1 = phi[cidx(g, i + u + a, j + v + b, k + w + f)];
                const double q2 = phi[cidx(g, i + u - a, j + v - b, k + w - f)];
                const double q3 = phi[cidx(g, i - u + a, j - v + b, k - w + f)];
                const double q4 = phi[cidx(g, i - u - a, j - v - b, k - w - f)];
                H[d][e] = H[e][d] = (q1 - q2 - q3 + q4) / (4.0 * h * h);
            }
        }
        double g2 = 0.0, tr = 0.0, ghg = 0.0;
#pragma unroll
        for (int d = 0; d < D; d++) {
            g2 += G[d] * G[d];
            tr += H[d][d];
#pragma unroll
            for (int e = 0; e < D; e++) ghg += G[d] * H[d][e] * G[e];
        }
        if (!(g2 > 1e-24)) return 0.0;
        const double kap = (g2 * tr - ghg) / (g2 * sqrt(g2));
        const double den = fmax(1.0 - pc * kap / (double)(D - 1), 0.5);
        return g.sigma * (kap / den);
    }
}

// ---------------------------------------------------------------------------
// geometry of the level set (vertex = mean of the adjacent cell centres,
// interface linear along every cell edge)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double edge_frac(double a, double b)
{
    bool na = a < 0.0, nb = b < 0.0;
    if (na && nb) return 1.0;
    if (!na && !nb) return 0.0;
    double t = a / (a - b);
    return na ? t : 1.0 - t;
}

// wetted area of the unit square with corner values v0..v3 at (0,0),(1,0),(1,1),(0,1)
__device__ __forceinline__ double clip_area(const double* v)
{
    const double cx[4] = {0.0, 1.0, 1.0, 0.0}, cy[4] = {0.0, 0.0, 1.0, 1.0};
    double px[8], py[8];
    int m = 0;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        int a = e, b = (e + 1) & 3;
        if (v[a] < 0.0) { px[m] = cx[a]; py[m] = cy[a]; m++; }
        if ((v[a] < 0.0) != (v[b] < 0.0)) {
            double t = v[a] / (v[a] - v[b]);
            px[m] = cx[a] + t * (cx[b] - cx[a]);
            py[m] = cy[a] + t * (cy[b] - cy[a]);
            m++;
        }
    }
    double area = 0.0;
    for (int e = 0; e < m; e++) {
        int f = (e + 1 == m) ? 0 : e + 1;
        area += px[e] * py[f] - px[f] * py[e];
    }
    area = 0.5 * fabs(area);
    return area > 1.0 ? 1.0 : area;
}

}  // namespace sharp
