/*
 * sharp_oracle.c -- plain FP64 CPU oracle of the accelerated sharp-interface
 * method of Long, Cai & Pan (Sec. 2 and Sec. 3.1 of the paper), on a uniform
 * Cartesian grid in 1, 2 or 3 dimensions.
 *
 * TEST INFRASTRUCTURE ONLY: a slow, loop-per-cell reference.  Every array is
 * a full-grid array and every step visits every cell; there is no tiling,
 * fusion or reordering.  Nothing in the GPU library includes, links or calls
 * this file.
 *
 * What it computes, in the paper's order:
 *   - per fluid, the cut-cell finite-volume update of Eq. (Eulerdiscrete):
 *     (alpha U)^{new} = (alpha U) + dt/dV X(dGamma) + dt/dx sum_faces A F
 *     with F a WENO5 flux (Sec. 2.1, Sec. 4: "fifth-order WENO-LF"), here with
 *     local Lax-Friedrichs splitting, and a Shu-Osher Runge-Kutta integrator
 *     (Sec. 3: the paper's TVD-RK2, and SSP-RK3 as the default);
 *   - the level-set geometry: volume fraction alpha, face apertures A and the
 *     interface segment dGamma*n of each cut cell (Sec. 2.1, Sec. 2.3);
 *   - the interface exchange X from the exact two-material stiffened-gas
 *     Riemann problem, and the level-set velocity it implies (Sec. 2.3);
 *     with surface tension, the Laplace pressure jump sigma kappa of Eq.
 *     (surfacetension) across the contact, each fluid taking its own
 *     interface pressure (Sec. 3.1: X_1 / X_2 = p_I1 / p_I2);
 *   - ghost-fluid extension of each fluid's state normal to the interface,
 *     level-set advection, Eq. (LS:linearadvection), and reinitialisation
 *     (Sec. 2.3);
 *   - small-cell mixing (Sec. 2.2, last paragraph);
 *   - the original single-time-step method and the accelerated cycle of
 *     Sec. 3.1: per-fluid CFL steps, truncation of n with threshold 0.7,
 *     interpolation of the slow fluid by Eq. (interpolation), interfacial
 *     flux correction by Eqs. (firstcorrection) and (secondcorrection).
 *
 * Readings where the paper is silent (the constitutive choices of the
 * interaction, extension, mixing and reinitialisation are deferred to the
 * cited works) are listed in the design notes.  Each function is pinned by
 * the test suite to something other than itself: closed forms (exact Riemann
 * solutions, planar extensions, translated and reinitialised circles and
 * spheres, the CFL steps of the gas-water tube, linear acoustics),
 * invariants (conservation, equilibrium, closure of cut cells) and
 * convergence orders; the unit entry points at the end of this file run
 * single steps for those pins.  The particular values that follow only from
 * the silent choices (the mixing weights, the number of extension and
 * reinitialisation sweeps, the band widths) are "parity unpinned" by the
 * paper: the invariants and GPU/oracle parity pin them, no printed number
 * does.
 */
#include "sharp_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define NVMAX 5

static char g_err[256];
const char* or_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* Equation of state: stiffened gas p = (gamma-1) rho e - gamma p_inf.        */
/* (The paper's Tait water is this EOS on an isentrope, p_inf = B - p0.)     */
/* ------------------------------------------------------------------------ */

void or_prim2cons(int D, double g, double pinf, const double* W, double* U)
{
    double rho = W[0], ke = 0.0;
    U[0] = rho;
    for (int d = 0; d < D; d++) {
        U[1 + d] = rho * W[1 + d];
        ke += W[1 + d] * W[1 + d];
    }
    double p = W[D + 1];
    U[D + 1] = (p + g * pinf) / (g - 1.0) + 0.5 * rho * ke;
}

int or_cons2prim(int D, double g, double pinf, const double* U, double* W)
{
    double rho = U[0], ke = 0.0;
    W[0] = rho;
    for (int d = 0; d < D; d++) {
        W[1 + d] = U[1 + d] / rho;
        ke += W[1 + d] * W[1 + d];
    }
    double p = (g - 1.0) * (U[D + 1] - 0.5 * rho * ke) - g * pinf;
    W[D + 1] = p;
    if (!(rho > 0.0) || !(p + pinf > 0.0) || !isfinite(p)) return -1;
    return 0;
}

static double sound(double g, double pinf, double rho, double p)
{
    return sqrt(g * (p + pinf) / rho);
}

/* ------------------------------------------------------------------------ */
/* Exact Riemann problem for two stiffened gases (interaction model).        */
/* The wave functions are the textbook ideal-gas ones written in p + p_inf.  */
/* ------------------------------------------------------------------------ */

typedef struct { double rho, u, p, g, pi; } side_t;

static double wave_f(const side_t* s, double p, double* df)
{
    double pk = s->p + s->pi, pb = p + s->pi;
    if (p > s->p) {                                  /* shock */
        double A = 2.0 / ((s->g + 1.0) * s->rho);
        double B = (s->g - 1.0) / (s->g + 1.0) * pk;
        double q = sqrt(A / (pb + B));
        *df = q * (1.0 - 0.5 * (p - s->p) / (pb + B));
        return (p - s->p) * q;
    } else {                                         /* rarefaction */
        double c = sound(s->g, s->pi, s->rho, s->p);
        double z = (s->g - 1.0) / (2.0 * s->g);
        double r = pb / pk, rz = pow(r, z);
        *df = rz / r / (s->rho * c);            /* r^(z-1) / (rho c) */
        return 2.0 * c / (s->g - 1.0) * (rz - 1.0);
    }
}

static double star_density(const side_t* s, double ps)
{
    double pk = s->p + s->pi, pb = ps + s->pi;
    if (pb <= 0.0) return 0.0;
    if (ps > s->p) {
        double m = (s->g - 1.0) / (s->g + 1.0);
        return s->rho * (pb / pk + m) / (m * pb / pk + 1.0);
    }
    return s->rho * pow(pb / pk, 1.0 / s->g);
}

/* The contact carries the pressure jump p_L - p_R = jump (0 without surface
 * tension): the root is p = p*_L of f_L(p) + f_R(p - jump) + (u_R - u_L) = 0,
 * increasing in p, each side's wave function taken at its own contact
 * pressure.  Cavitation floor: the larger of the two sides' lower bounds
 * on p, -p_inf_L and jump - p_inf_R. */
static int riemann_core(const double* WL, const double* WR, double gL, double piL,
                        double gR, double piR, double jump, double* out)
{
    side_t L = {WL[0], WL[1], WL[2], gL, piL};
    side_t R = {WR[0], WR[1], WR[2], gR, piR};
    double du = R.u - L.u, dfl, dfr;
    double fl_lo = -piL, fr_lo = jump - piR;
    double pfloor = fl_lo > fr_lo ? fl_lo : fr_lo;
    double pR = R.p + jump;   /* the right side's pressure on the left side's scale */
    int it = 0;
    double p;
    /* cavitation: no positive root above the floor */
    double fl0 = wave_f(&L, pfloor, &dfl), fr0 = wave_f(&R, pfloor - jump, &dfr);
    if (fl0 + fr0 + du >= 0.0) {
        p = pfloor;
    } else {
        /* start from the geometric mean of the side pressures measured from
         * the floor; a side below the floor (possible for the larger p_inf)
         * falls back to the linearised (PVRS) estimate */
        if (L.p > pfloor && pR > pfloor) {
            p = pfloor + sqrt((L.p - pfloor) * (pR - pfloor));
        } else {
            double cL = sound(gL, piL, L.rho, L.p), cR = sound(gR, piR, R.rho, R.p);
            p = 0.5 * (L.p + pR) - 0.125 * du * (L.rho + R.rho) * (cL + cR);
            /* the side with the smaller p_inf has p > pfloor; the other side may not */
            double pmax = (L.p > pR ? L.p : pR);
            if (!(p > pfloor)) p = pfloor + 0.5 * (pmax - pfloor);
        }
        double lo = pfloor, hi = INFINITY;
        double scale = fabs(piL) + fabs(piR) + fabs(jump) + 1e-300;
        for (it = 1; it <= 200; it++) {
            double f = wave_f(&L, p, &dfl) + wave_f(&R, p - jump, &dfr) + du;
            if (f > 0.0) { if (p < hi) hi = p; }
            else { if (p > lo) lo = p; }
            double pn = p - f / (dfl + dfr);
            if (!(pn > lo && pn < hi))
                pn = isfinite(hi) ? 0.5 * (lo + hi) : lo + 2.0 * (p - lo);
            double dp = pn - p;
            p = pn;
            if (fabs(dp) <= 1e-13 * (fabs(p) + scale)) break;
        }
    }
    double fl = wave_f(&L, p, &dfl), fr = wave_f(&R, p - jump, &dfr);
    out[0] = p;
    out[1] = 0.5 * (L.u + R.u) + 0.5 * (fr - fl);
    out[2] = star_density(&L, p);
    out[3] = star_density(&R, p - jump);
    out[4] = (double)it;
    return 0;
}

int or_riemann(const double* WL, const double* WR, double gL, double piL,
               double gR, double piR, double* out)
{
    return riemann_core(WL, WR, gL, piL, gR, piR, 0.0, out);
}

int or_riemann_jump(const double* WL, const double* WR, double gL, double piL,
                    double gR, double piR, double jump, double* out)
{
    return riemann_core(WL, WR, gL, piL, gR, piR, jump, out);
}

void or_riemann_sample(const double* WL, const double* WR, double gL, double piL,
                       double gR, double piR, double xi, double* out)
{
    double st[5];
    or_riemann(WL, WR, gL, piL, gR, piR, st);
    double ps = st[0], us = st[1];
    int left = (xi <= us);
    const double* W = left ? WL : WR;
    double g = left ? gL : gR, pi = left ? piL : piR;
    double rho = W[0], u = W[1], p = W[2];
    double c = sound(g, pi, rho, p);
    double sgn = left ? 1.0 : -1.0;   /* mirror the right side onto the left */
    double x = sgn * xi, uu = sgn * u, uss = sgn * us;
    double r, v, q;
    if (ps > p) {
        double S = uu - c * sqrt((g + 1.0) / (2.0 * g) * (ps + pi) / (p + pi) + (g - 1.0) / (2.0 * g));
        if (x <= S) { r = rho; v = uu; q = p; }
        else { r = left ? st[2] : st[3]; v = uss; q = ps; }
    } else {
        double sh = uu - c;
        double rs = left ? st[2] : st[3];
        double cs = (rs > 0.0) ? sound(g, pi, rs, ps) : 0.0;
        double stl = uss - cs;
        if (x <= sh) { r = rho; v = uu; q = p; }
        else if (x >= stl) { r = rs; v = uss; q = ps; }
        else {
            double cf = 2.0 / (g + 1.0) * (c + 0.5 * (g - 1.0) * (uu - x));
            v = 2.0 / (g + 1.0) * (c + 0.5 * (g - 1.0) * uu + x);
            r = rho * pow(cf / c, 2.0 / (g - 1.0));
            q = (p + pi) * pow(cf / c, 2.0 * g / (g - 1.0)) - pi;
        }
    }
    out[0] = r; out[1] = sgn * v; out[2] = q; out[3] = left ? 0.0 : 1.0;
}

/* ------------------------------------------------------------------------ */
/* WENO5 reconstruction (Jiang & Shu), value at the right edge of cell v2     */
/* from the left-biased stencil v0..v4, textbook form.                        */
/* ------------------------------------------------------------------------ */

double or_weno5(double v0, double v1, double v2, double v3, double v4, double eps)
{
    double q0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) / 6.0;
    double q1 = (-v1 + 5.0 * v2 + 2.0 * v3) / 6.0;
    double q2 = (2.0 * v2 + 5.0 * v3 - v4) / 6.0;
    double b0 = 13.0 / 12.0 * (v0 - 2.0 * v1 + v2) * (v0 - 2.0 * v1 + v2)
              + 0.25 * (v0 - 4.0 * v1 + 3.0 * v2) * (v0 - 4.0 * v1 + 3.0 * v2);
    double b1 = 13.0 / 12.0 * (v1 - 2.0 * v2 + v3) * (v1 - 2.0 * v2 + v3)
              + 0.25 * (v1 - v3) * (v1 - v3);
    double b2 = 13.0 / 12.0 * (v2 - 2.0 * v3 + v4) * (v2 - 2.0 * v3 + v4)
              + 0.25 * (3.0 * v2 - 4.0 * v3 + v4) * (3.0 * v2 - 4.0 * v3 + v4);
    double a0 = 0.1 / ((eps + b0) * (eps + b0));
    double a1 = 0.6 / ((eps + b1) * (eps + b1));
    double a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* Physical flux of direction d and conserved vector of primitive W. */
static void phys(int D, int d, double g, double pi, const double* W, double* U, double* F, double* s)
{
    or_prim2cons(D, g, pi, W, U);
    double un = W[1 + d], p = W[D + 1];
    F[0] = U[0] * un;
    for (int e = 0; e < D; e++) F[1 + e] = U[1 + e] * un;
    F[1 + d] += p;
    F[D + 1] = (U[D + 1] + p) * un;
    *s = fabs(un) + sound(g, pi, W[0], p);
}

/* LLF-WENO5 flux of one face from six stencil states j = i-2 .. i+3 (the face
 * sits between j = 2 and j = 3).  U6 are the conserved vectors used in the
 * splitting (for real cells the cell's own content / alpha). */
static void face_flux(int D, int d, double g, double pi, double eps,
                      const double (*W6)[NVMAX], const double (*U6)[NVMAX], double* Fh)
{
    int NV = D + 2;
    double U[6][NVMAX], F[6][NVMAX], Ut[NVMAX], a = 0.0, s;
    for (int j = 0; j < 6; j++) {
        phys(D, d, g, pi, W6[j], Ut, F[j], &s);
        for (int q = 0; q < NV; q++) U[j][q] = U6[j][q];
        if (s > a) a = s;
    }
    for (int q = 0; q < NV; q++) {
        double fp[6], fm[6];
        for (int j = 0; j < 6; j++) {
            fp[j] = 0.5 * (F[j][q] + a * U[j][q]);
            fm[j] = 0.5 * (F[j][q] - a * U[j][q]);
        }
        Fh[q] = or_weno5(fp[0], fp[1], fp[2], fp[3], fp[4], eps)
              + or_weno5(fm[5], fm[4], fm[3], fm[2], fm[1], eps);
    }
}

void or_face_flux_1d(const double* W6, double gamma, double pinf, double eps, double* F)
{
    double W[6][NVMAX], U[6][NVMAX];
    for (int j = 0; j < 6; j++) {
        W[j][0] = W6[3 * j]; W[j][1] = W6[3 * j + 1]; W[j][2] = W6[3 * j + 2];
        or_prim2cons(1, gamma, pinf, W[j], U[j]);
    }
    face_flux(1, 0, gamma, pinf, eps, (const double (*)[NVMAX])W, (const double (*)[NVMAX])U, F);
}

/* ------------------------------------------------------------------------ */
/* Simulation object                                                          */
/* ------------------------------------------------------------------------ */

struct or_sim {
    or_params P;
    int D, NV;
    long n[3], nc;        /* cells */
    long nf[3], nfc;      /* padded face lattice: n+1 in active directions */
    double h, t;
    double* X[2];         /* state (alpha U) */
    double* Y[2];         /* stage buffers */
    double* Z[2];
    double* W[2];         /* primitives: real cells and extended ghost cells */
    double* Wn;           /* Jacobi scratch */
    double* phi;          /* level set */
    double* phib;         /* level set at the start of the (sub)step */
    double* phi0;         /* level set before reinitialisation */
    double* phit;         /* scratch */
    double* phih;         /* level-set snapshot at t1/2 (RK3 cycle) */
    double* Fh;           /* fast-fluid snapshot at t1/2 */
    double* T;            /* slow fluid interpolated / mixed state */
    double* alpha;        /* fluid-0 volume fraction */
    double* ap[3];        /* fluid-0 aperture of the low face (padded index) */
    double* ps;           /* interface pressure p*   (cut cells) */
    double* pj;           /* Laplace jump sigma kappa: fluid 1's interface pressure is ps - pj */
    double* us;           /* interface normal velocity u* (cut cells) */
    double* ss[2];        /* star-state CFL speed of each fluid (cut cells) */
    double* v[3];         /* level-set velocity */
    double* vn[3];
    unsigned char* M;     /* level-set band mask of the (sub)step */
    double* corr;         /* interfacial flux correction, [NV][cells] */
    double* dlt;          /* mixing increments */
    double bflux[2][NVMAX];
    long err_cell;
    double* replay;       /* prescribed CFL steps (copy of P.dt_replay) */
    long n_replay, replay_pos;
    double* log;          /* CFL steps taken */
    long n_log, cap_log;
    double* ls_rep;       /* prescribed stage level sets (copy of P.ls_replay) */
    long n_ls_rep, ls_pos;
    double* lslog;        /* stage level sets taken (P.log_levelset) */
    long n_lslog, cap_lslog;
};

void or_default_params(or_params* p)
{
    memset(p, 0, sizeof(*p));
    p->ndim = 1;
    p->n[0] = p->n[1] = p->n[2] = 1;
    p->h = 1.0;
    p->gamma[0] = p->gamma[1] = 1.4;
    p->cfl = 0.6;
    p->rk = 3;
    p->n_thr = 0.7;
    p->alpha_mix = 0.5;
    p->ls_band = 8.0;
    p->ext_band = 5.0;
    p->mix_band = 3.0;
    p->ext_iters = 8;
    p->reinit_iters = 2;
    p->weno_eps = 1e-6;
}

static double* dalloc(long n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

or_sim* or_create(const or_params* p)
{
    if (p->ndim < 1 || p->ndim > 3 || !(p->h > 0.0) || (p->rk != 2 && p->rk != 3)) {
        snprintf(g_err, sizeof g_err, "invalid parameters");
        return NULL;
    }
    if (p->n_dt_replay < 0 || (p->n_dt_replay > 0 && !p->dt_replay)) {
        snprintf(g_err, sizeof g_err, "invalid dt_replay");
        return NULL;
    }
    if (p->n_ls_replay < 0 || (p->n_ls_replay > 0 && !p->ls_replay)) {
        snprintf(g_err, sizeof g_err, "invalid ls_replay");
        return NULL;
    }
    or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
    s->P = *p;
    s->P.dt_replay = NULL;
    s->P.ls_replay = NULL;
    if (p->n_dt_replay > 0) {
        s->replay = (double*)malloc(sizeof(double) * (size_t)p->n_dt_replay);
        memcpy(s->replay, p->dt_replay, sizeof(double) * (size_t)p->n_dt_replay);
        s->n_replay = p->n_dt_replay;
    }
    if (p->n_ls_replay > 0) {
        s->ls_rep = (double*)malloc(sizeof(double) * (size_t)p->n_ls_replay);
        memcpy(s->ls_rep, p->ls_replay, sizeof(double) * (size_t)p->n_ls_replay);
        s->n_ls_rep = p->n_ls_replay;
    }
    s->D = p->ndim;
    s->NV = p->ndim + 2;
    s->nc = 1; s->nfc = 1;
    for (int d = 0; d < 3; d++) {
        s->n[d] = d < s->D ? p->n[d] : 1;
        s->nf[d] = d < s->D ? s->n[d] + 1 : 1;
        s->nc *= s->n[d];
        s->nfc *= s->nf[d];
    }
    s->h = p->h;
    long nv = s->NV * s->nc;
    for (int k = 0; k < 2; k++) {
        s->X[k] = dalloc(nv); s->Y[k] = dalloc(nv); s->Z[k] = dalloc(nv);
        s->W[k] = dalloc(nv); s->ss[k] = dalloc(s->nc);
    }
    s->Wn = dalloc(nv);
    s->T = dalloc(nv); s->Fh = dalloc(nv); s->corr = dalloc(nv); s->dlt = dalloc(nv);
    s->phi = dalloc(s->nc); s->phib = dalloc(s->nc); s->phi0 = dalloc(s->nc);
    s->phit = dalloc(s->nc); s->phih = dalloc(s->nc);
    s->alpha = dalloc(s->nc);
    for (int d = 0; d < 3; d++) {
        s->ap[d] = dalloc(s->nfc);
        s->v[d] = dalloc(s->nc);
        s->vn[d] = dalloc(s->nc);
    }
    s->ps = dalloc(s->nc); s->us = dalloc(s->nc); s->pj = dalloc(s->nc);
    s->M = (unsigned char*)calloc((size_t)s->nc, 1);
    /* finite placeholder for ghost states never reached by the extension */
    for (int k = 0; k < 2; k++)
        for (long c = 0; c < s->nc; c++) {
            s->W[k][c] = 1.0;
            s->W[k][(s->D + 1) * s->nc + c] = 1.0;
        }
    return s;
}

void or_destroy(or_sim* s)
{
    if (!s) return;
    for (int k = 0; k < 2; k++) {
        free(s->X[k]); free(s->Y[k]); free(s->Z[k]); free(s->W[k]); free(s->ss[k]);
    }
    free(s->Wn); free(s->T); free(s->Fh); free(s->corr); free(s->dlt);
    free(s->phi); free(s->phib); free(s->phi0); free(s->phit); free(s->phih);
    free(s->alpha);
    for (int d = 0; d < 3; d++) { free(s->ap[d]); free(s->v[d]); free(s->vn[d]); }
    free(s->ps); free(s->us); free(s->pj); free(s->M);
    free(s->replay); free(s->log);
    free(s->ls_rep); free(s->lslog);
    free(s);
}

long or_schedule(const or_sim* s, double* out, long cap)
{
    for (long i = 0; out && i < s->n_log && i < cap; i++) out[i] = s->log[i];
    return s->n_log;
}

long or_levelset_log(const or_sim* s, double* out, long cap)
{
    for (long i = 0; out && i < s->n_lslog && i < cap; i++) out[i] = s->lslog[i];
    return s->n_lslog;
}

/* The CFL step of fluid k at a (sub)step start: the prescribed one when the
 * simulation replays a schedule; every step taken is logged.  -1 when the
 * schedule has run out. */
static int take_cfl(or_sim* s, double* dt)
{
    if (s->n_replay > 0) {
        if (s->replay_pos >= s->n_replay) {
            snprintf(g_err, sizeof g_err, "dt_replay exhausted after %ld steps", s->replay_pos);
            return -1;
        }
        *dt = s->replay[s->replay_pos++];
    }
    if (s->n_log == s->cap_log) {
        s->cap_log = s->cap_log ? 2 * s->cap_log : 64;
        s->log = (double*)realloc(s->log, sizeof(double) * (size_t)s->cap_log);
    }
    s->log[s->n_log++] = *dt;
    return 0;
}

/* ---- indexing with domain boundary conditions (no ghost storage) ---- */

static long bcmap(long i, long n, int bc)
{
    if (bc == 1) { i %= n; if (i < 0) i += n; return i; }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

static long cell(const or_sim* s, long i, long j, long k)
{
    i = bcmap(i, s->n[0], s->P.bc[0]);
    j = s->D > 1 ? bcmap(j, s->n[1], s->P.bc[1]) : 0;
    k = s->D > 2 ? bcmap(k, s->n[2], s->P.bc[2]) : 0;
    return i + s->n[0] * (j + s->n[1] * k);
}

static long face(const or_sim* s, long i, long j, long k)
{
    return i + s->nf[0] * (j + s->nf[1] * k);
}

static void coords(const or_sim* s, long c, long* i, long* j, long* k)
{
    *i = c % s->n[0];
    *j = (c / s->n[0]) % s->n[1];
    *k = c / (s->n[0] * s->n[1]);
}

static long nbr(const or_sim* s, long c, int d, int off)
{
    long i, j, k;
    coords(s, c, &i, &j, &k);
    if (d == 0) i += off; else if (d == 1) j += off; else k += off;
    return cell(s, i, j, k);
}

/* ------------------------------------------------------------------------ */
/* Level-set geometry (Sec. 2.1, Fig. 1; Sec. 2.3).                           */
/* Vertex values are the mean of the adjacent cell-centre values; the        */
/* interface is linear along every cell edge.  Apertures are the wetted      */
/* (phi < 0) fraction of each face, alpha is the clipped polygon area (2-D)  */
/* or the divergence-theorem volume (3-D).                                   */
/* ------------------------------------------------------------------------ */

static double vertex(const or_sim* s, const double* phi, long i, long j, long k)
{
    double sum = 0.0;
    int m = 1 << s->D;
    for (int b = 0; b < m; b++) {
        long ii = i - 1 + (b & 1);
        long jj = s->D > 1 ? j - 1 + ((b >> 1) & 1) : 0;
        long kk = s->D > 2 ? k - 1 + ((b >> 2) & 1) : 0;
        sum += phi[cell(s, ii, jj, kk)];
    }
    return sum / (double)m;
}

/* wetted fraction of a segment with end values a, b */
static double edge_frac(double a, double b)
{
    int na = a < 0.0, nb = b < 0.0;
    if (na && nb) return 1.0;
    if (!na && !nb) return 0.0;
    double t = a / (a - b);
    return na ? t : 1.0 - t;
}

/* wetted area of the unit square with corner values v[0..3] at (0,0), (1,0),
 * (1,1), (0,1): the polygon of wetted corners and edge crossings */
double or_clip_area(const double* v)
{
    static const double cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
    double px[8], py[8];
    int m = 0;
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
        int f = (e + 1) % m;
        area += px[e] * py[f] - px[f] * py[e];
    }
    area = 0.5 * fabs(area);
    return area > 1.0 ? 1.0 : area;
}

static double aperture(const or_sim* s, const double* phi, int d, long i, long j, long k)
{
    if (s->D == 1) return vertex(s, phi, i, j, k) < 0.0 ? 1.0 : 0.0;
    if (s->D == 2) {
        if (d == 0) return edge_frac(vertex(s, phi, i, j, k), vertex(s, phi, i, j + 1, k));
        return edge_frac(vertex(s, phi, i, j, k), vertex(s, phi, i + 1, j, k));
    }
    double v[4];
    if (d == 0) {
        v[0] = vertex(s, phi, i, j, k);     v[1] = vertex(s, phi, i, j + 1, k);
        v[2] = vertex(s, phi, i, j + 1, k + 1); v[3] = vertex(s, phi, i, j, k + 1);
    } else if (d == 1) {
        v[0] = vertex(s, phi, i, j, k);     v[1] = vertex(s, phi, i + 1, j, k);
        v[2] = vertex(s, phi, i + 1, j, k + 1); v[3] = vertex(s, phi, i, j, k + 1);
    } else {
        v[0] = vertex(s, phi, i, j, k);     v[1] = vertex(s, phi, i + 1, j, k);
        v[2] = vertex(s, phi, i + 1, j + 1, k); v[3] = vertex(s, phi, i, j + 1, k);
    }
    return or_clip_area(v);
}

static void geometry_of(const or_sim* s, const double* phi, double* alpha, double* const* ap)
{
    int D = s->D;
    /* apertures on every face of the padded lattice */
    for (int d = 0; d < D; d++)
        for (long k = 0; k < (d == 2 ? s->nf[2] : s->n[2]); k++)
            for (long j = 0; j < (d == 1 ? s->nf[1] : s->n[1]); j++)
                for (long i = 0; i < (d == 0 ? s->nf[0] : s->n[0]); i++)
                    ap[d][face(s, i, j, k)] = aperture(s, phi, d, i, j, k);
    for (long c = 0; c < s->nc; c++) {
        long i, j, k;
        coords(s, c, &i, &j, &k);
        double a;
        if (D == 1) {
            a = edge_frac(vertex(s, phi, i, 0, 0), vertex(s, phi, i + 1, 0, 0));
        } else if (D == 2) {
            double v[4] = {vertex(s, phi, i, j, 0), vertex(s, phi, i + 1, j, 0),
                           vertex(s, phi, i + 1, j + 1, 0), vertex(s, phi, i, j + 1, 0)};
            a = or_clip_area(v);
        } else {
            /* divergence theorem on the wetted part of the unit cube:
             * 3 alpha = sum_faces A (x.n) + |dGamma n| (x_Gamma . n),
             * x.n = 1/2 on every face, x_Gamma . n = -phi_c/h (planar cut) */
            double sumA = 0.0, g2 = 0.0;
            for (int d = 0; d < 3; d++) {
                long fl = face(s, i, j, k);
                long fh = face(s, i + (d == 0), j + (d == 1), k + (d == 2));
                sumA += ap[d][fl] + ap[d][fh];
                double gd = ap[d][fl] - ap[d][fh];
                g2 += gd * gd;
            }
            a = (0.5 * sumA + sqrt(g2) * (-phi[c] / s->h)) / 3.0;
            a = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
        }
        alpha[c] = a;
    }
}

static void geometry(or_sim* s) { geometry_of(s, s->phi, s->alpha, s->ap); }

long or_face_count(const or_sim* s) { return s->nfc; }

void or_geometry(const or_sim* s, double* alpha, double* ap)
{
    double* a3[3] = {ap, ap + s->nfc, ap + 2 * s->nfc};
    geometry_of(s, s->phi, alpha, a3);
}

/* interface segment per unit volume, g = dGamma n / dV, of fluid 0 (n points
 * from fluid 0 into fluid 1), from the closure of the wetted region */
static double interface_vec(const or_sim* s, long c, double* g)
{
    long i, j, k;
    coords(s, c, &i, &j, &k);
    double g2 = 0.0;
    for (int d = 0; d < s->D; d++) {
        long fl = face(s, i, j, k);
        long fh = face(s, i + (d == 0), j + (d == 1), k + (d == 2));
        g[d] = (s->ap[d][fl] - s->ap[d][fh]) / s->h;
        g2 += g[d] * g[d];
    }
    return sqrt(g2);
}

static double alpha_k(const or_sim* s, int k, long c) { return k == 0 ? s->alpha[c] : 1.0 - s->alpha[c]; }

static double grad_phi(const or_sim* s, const double* phi, long c, double* gr)
{
    double g2 = 0.0;
    for (int d = 0; d < s->D; d++) {
        gr[d] = (phi[nbr(s, c, d, 1)] - phi[nbr(s, c, d, -1)]) / (2.0 * s->h);
        g2 += gr[d] * gr[d];
    }
    return sqrt(g2);
}

/* Curvature of the level set for the Laplace jump of Eq. (surfacetension):
 * kappa = div(grad phi / |grad phi|), expanded as
 *   (|g|^2 trace(H) - g.H.g) / |g|^3
 * with the gradient g and the Hessian H of phi by second-order central
 * differences at the cell centre; positive where fluid 0 (phi < 0) is
 * convex.  The cell centre lies phi from the interface: each principal
 * curvature k of a signed distance function is k / (1 + phi k) there, so
 * the value at the nearest interface point is taken, with the principal
 * curvatures assumed equal (exact for circles and spheres):
 *   kappa_I = kappa / (1 - phi kappa / (D - 1)),
 * the denominator held at >= 1/2 where the level set is not resolved.
 * 0 in 1-D (a point interface has no curvature) and where |g| vanishes. */
static double curvature(const or_sim* s, const double* phi, long c)
{
    int D = s->D;
    if (D < 2) return 0.0;
    double h = s->h, g[3], H[3][3];
    for (int d = 0; d < D; d++) {
        double pp = phi[nbr(s, c, d, 1)], pm = phi[nbr(s, c, d, -1)];
        g[d] = (pp - pm) / (2.0 * h);
        H[d][d] = (pp - 2.0 * phi[c] + pm) / (h * h);
        for (int e = d + 1; e < D; e++) {
            double a = phi[nbr(s, nbr(s, c, d, 1), e, 1)], b = phi[nbr(s, nbr(s, c, d, 1), e, -1)];
            double cc = phi[nbr(s, nbr(s, c, d, -1), e, 1)], dd = phi[nbr(s, nbr(s, c, d, -1), e, -1)];
            H[d][e] = H[e][d] = (a - b - cc + dd) / (4.0 * h * h);
        }
    }
    double g2 = 0.0, tr = 0.0, gHg = 0.0;
    for (int d = 0; d < D; d++) {
        g2 += g[d] * g[d];
        tr += H[d][d];
        for (int e = 0; e < D; e++) gHg += g[d] * H[d][e] * g[e];
    }
    if (!(g2 > 1e-24)) return 0.0;
    double kap = (g2 * tr - gHg) / (g2 * sqrt(g2));
    double den = 1.0 - phi[c] * kap / (double)(D - 1);
    if (den < 0.5) den = 0.5;
    return kap / den;
}

/* ------------------------------------------------------------------------ */
/* Band mask of the (sub)step: a cell is in the level-set band when it or one */
/* of its axis neighbours is closer than ls_band cells to the interface.      */
/* ------------------------------------------------------------------------ */

static void band_mask(or_sim* s)
{
    double R = s->P.ls_band * s->h;
    for (long c = 0; c < s->nc; c++) {
        double m = fabs(s->phi[c]);
        for (int d = 0; d < s->D; d++) {
            double a = fabs(s->phi[nbr(s, c, d, -1)]), b = fabs(s->phi[nbr(s, c, d, 1)]);
            if (a < m) m = a;
            if (b < m) m = b;
        }
        s->M[c] = m < R;
    }
}

/* ------------------------------------------------------------------------ */
/* Primitive recovery on real cells: alpha_k >= alpha_mix.                    */
/* ------------------------------------------------------------------------ */

static int prims(or_sim* s, int k, const double* cons)
{
    int D = s->D, NV = s->NV;
    for (long c = 0; c < s->nc; c++) {
        double a = alpha_k(s, k, c);
        if (a < s->P.alpha_mix) continue;
        double U[NVMAX], W[NVMAX];
        for (int q = 0; q < NV; q++) U[q] = cons[q * s->nc + c] / a;
        if (or_cons2prim(D, s->P.gamma[k], s->P.pinf[k], U, W) != 0) {
            s->err_cell = c;
            snprintf(g_err, sizeof g_err, "non-physical state of fluid %d in cell %ld", k, c);
            return -4;
        }
        for (int q = 0; q < NV; q++) s->W[k][q * s->nc + c] = W[q];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Extension (Sec. 2.3): first-order upwind steady state of                  */
/* dq/dtau + n . grad q = 0, Jacobi sweeps.  Fluid k's ghost cells are band  */
/* cells with alpha_k < alpha_mix within ext_band cells on the far side;     */
/* information travels away from fluid k.  The level-set velocity is        */
/* extended from the cut cells to the rest of the band, away from the        */
/* interface on both sides.                                                   */
/* ------------------------------------------------------------------------ */

static int is_cut(const or_sim* s, long c)
{
    double g[3];
    return interface_vec(s, c, g) > 0.0;
}

static void extend_w(or_sim* s)
{
    int D = s->D, NV = s->NV;
    double band = s->P.ext_band * s->h;
    for (int it = 0; it < s->P.ext_iters; it++) {
        for (int k = 0; k < 2; k++) {
            double sk = (k == 0) ? 1.0 : -1.0;   /* ghost side of fluid 0 is phi > 0 */
            memcpy(s->Wn, s->W[k], sizeof(double) * (size_t)(NV * s->nc));
            for (long c = 0; c < s->nc; c++) {
                if (!s->M[c] || alpha_k(s, k, c) >= s->P.alpha_mix || sk * s->phi[c] > band) continue;
                double gr[3], nn[3], wsum = 0.0;
                double gm = grad_phi(s, s->phi, c, gr);
                if (!(gm > 0.0)) continue;
                long up[3];
                for (int d = 0; d < D; d++) {
                    nn[d] = sk * gr[d] / gm;
                    up[d] = nbr(s, c, d, nn[d] > 0.0 ? -1 : 1);
                    wsum += fabs(nn[d]);
                }
                for (int q = 0; q < NV; q++) {
                    double acc = 0.0;
                    for (int d = 0; d < D; d++) acc += fabs(nn[d]) * s->W[k][q * s->nc + up[d]];
                    s->Wn[q * s->nc + c] = acc / wsum;
                }
            }
            memcpy(s->W[k], s->Wn, sizeof(double) * (size_t)(NV * s->nc));
        }
    }
}

static void extend_v(or_sim* s)
{
    int D = s->D;
    for (int it = 0; it < s->P.ext_iters; it++) {
        for (int d = 0; d < D; d++) memcpy(s->vn[d], s->v[d], sizeof(double) * (size_t)s->nc);
        for (long c = 0; c < s->nc; c++) {
            if (!s->M[c] || is_cut(s, c)) continue;
            double gr[3], nn[3], wsum = 0.0;
            double gm = grad_phi(s, s->phi, c, gr);
            if (!(gm > 0.0)) continue;
            double sg = s->phi[c] < 0.0 ? -1.0 : 1.0;   /* away from the interface */
            long up[3];
            for (int d = 0; d < D; d++) {
                nn[d] = sg * gr[d] / gm;
                up[d] = nbr(s, c, d, nn[d] > 0.0 ? -1 : 1);
                wsum += fabs(nn[d]);
            }
            for (int e = 0; e < D; e++) {
                double acc = 0.0;
                for (int d = 0; d < D; d++) acc += fabs(nn[d]) * s->v[e][up[d]];
                s->vn[e][c] = acc / wsum;
            }
        }
        for (int d = 0; d < D; d++) memcpy(s->v[d], s->vn[d], sizeof(double) * (size_t)s->nc);
    }
}

/* ------------------------------------------------------------------------ */
/* Interface interaction: per cut cell, the exact Riemann problem between     */
/* the two fluids' states projected on the interface normal.  The exchange    */
/* term of fluid 0 per unit volume is X/dV = (0, -p* g, -p* u* |g|) and       */
/* fluid 1 receives the opposite; the level-set velocity is u* n.            */
/* ------------------------------------------------------------------------ */

static void interaction(or_sim* s)
{
    int D = s->D;
    for (long c = 0; c < s->nc; c++) {
        double g[3];
        double gm = interface_vec(s, c, g);
        s->ps[c] = 0.0; s->us[c] = 0.0; s->ss[0][c] = 0.0; s->ss[1][c] = 0.0; s->pj[c] = 0.0;
        if (!(gm > 0.0)) continue;
        double WL[3], WR[3], un0 = 0.0, un1 = 0.0;
        for (int d = 0; d < D; d++) {
            un0 += s->W[0][(1 + d) * s->nc + c] * g[d] / gm;
            un1 += s->W[1][(1 + d) * s->nc + c] * g[d] / gm;
        }
        WL[0] = s->W[0][c]; WL[1] = un0; WL[2] = s->W[0][(D + 1) * s->nc + c];
        WR[0] = s->W[1][c]; WR[1] = un1; WR[2] = s->W[1][(D + 1) * s->nc + c];
        double st[5];
        /* Laplace jump of Eq. (surfacetension): fluid 0's interface
         * pressure exceeds fluid 1's by sigma kappa */
        double jump = s->P.sigma != 0.0 ? s->P.sigma * curvature(s, s->phi, c) : 0.0;
        riemann_core(WL, WR, s->P.gamma[0], s->P.pinf[0], s->P.gamma[1], s->P.pinf[1], jump, st);
        s->ps[c] = st[0];
        s->us[c] = st[1];
        s->pj[c] = jump;
        for (int k = 0; k < 2; k++) {
            double rs = st[2 + k];
            double pk = k == 0 ? st[0] : st[0] - jump;
            double cs = rs > 0.0 ? sound(s->P.gamma[k], s->P.pinf[k], rs, pk) : 0.0;
            double sum = 0.0;
            for (int d = 0; d < D; d++) sum += (fabs(st[1] * g[d] / gm) + cs) / s->h;
            s->ss[k][c] = sum;
        }
        for (int d = 0; d < D; d++) s->v[d][c] = st[1] * g[d] / gm;
    }
}

/* exchange term of fluid k in cell c, per unit volume, at fluid k's own
 * interface pressure (fluid 1's is lower by the Laplace jump) */
static void exchange(const or_sim* s, int k, long c, double* Xh)
{
    int D = s->D;
    double g[3];
    double gm = interface_vec(s, c, g);
    for (int q = 0; q < s->NV; q++) Xh[q] = 0.0;
    if (!(gm > 0.0)) return;
    double sg = (k == 0) ? 1.0 : -1.0;
    double p = k == 0 ? s->ps[c] : s->ps[c] - s->pj[c];
    for (int d = 0; d < D; d++) Xh[1 + d] = -sg * p * g[d];
    Xh[D + 1] = -sg * p * s->us[c] * gm;
}

/* Eqs. (firstcorrection)/(secondcorrection): corr += w * X_slow */
static void corr_add(or_sim* s, int S, double w)
{
    double Xh[NVMAX];
    for (long c = 0; c < s->nc; c++) {
        exchange(s, S, c, Xh);
        for (int q = 1; q < s->NV; q++) s->corr[q * s->nc + c] += w * Xh[q];
    }
}

/* ------------------------------------------------------------------------ */
/* CFL time step of each fluid: cfl / max sum_d (|u_d| + c)/dx over cells     */
/* holding the fluid, including the star state of cut cells.                 */
/* ------------------------------------------------------------------------ */

static void cfl_dt(or_sim* s, double* dt, long* cnt)
{
    int D = s->D;
    for (int k = 0; k < 2; k++) {
        double m = 0.0;
        long n = 0;
        for (long c = 0; c < s->nc; c++) {
            if (!(alpha_k(s, k, c) > 0.0)) continue;
            n++;
            double rho = s->W[k][c], p = s->W[k][(D + 1) * s->nc + c];
            double cs = sound(s->P.gamma[k], s->P.pinf[k], rho, p), sum = 0.0;
            for (int d = 0; d < D; d++) sum += (fabs(s->W[k][(1 + d) * s->nc + c]) + cs) / s->h;
            if (sum > m) m = sum;
            if (s->ss[k][c] > m) m = s->ss[k][c];
        }
        cnt[k] = n;
        dt[k] = (n > 0 && m > 0.0) ? s->P.cfl / m : INFINITY;
    }
}

/* ------------------------------------------------------------------------ */
/* One Shu-Osher stage of fluid k, Eq. (Eulerdiscrete) with the RK form:      */
/*   out = a*base + (1-a)*(in + dt*L(in)),                                    */
/*   L = sum_d (A_lo F_lo - A_hi F_hi)/dx + X/dV.                             */
/* W[k] must hold the primitives of `in` on real cells and the extension on   */
/* ghost cells.  Boundary-face inflow is accumulated with weight wflux.       */
/* ------------------------------------------------------------------------ */

static void state_of(const or_sim* s, int k, const double* in, long c, double* W, double* U)
{
    int NV = s->NV;
    double a = alpha_k(s, k, c);
    for (int q = 0; q < NV; q++) W[q] = s->W[k][q * s->nc + c];
    if (a >= s->P.alpha_mix) {
        for (int q = 0; q < NV; q++) U[q] = in[q * s->nc + c] / a;
    } else {
        or_prim2cons(s->D, s->P.gamma[k], s->P.pinf[k], W, U);
    }
}

static double ap_k(const or_sim* s, int k, int d, long f)
{
    return k == 0 ? s->ap[d][f] : 1.0 - s->ap[d][f];
}

/* flux through the low face of cell (i,j,k) in direction d (times aperture) */
static void low_face_flux(const or_sim* s, int kf, const double* in, int d, long i, long j, long k, double* Fa)
{
    double W6[6][NVMAX], U6[6][NVMAX], Fh[NVMAX];
    for (int m = 0; m < 6; m++) {
        long off = m - 3;
        long c = cell(s, i + (d == 0) * off, j + (d == 1) * off, k + (d == 2) * off);
        state_of(s, kf, in, c, W6[m], U6[m]);
    }
    face_flux(s->D, d, s->P.gamma[kf], s->P.pinf[kf], s->P.weno_eps,
              (const double (*)[NVMAX])W6, (const double (*)[NVMAX])U6, Fh);
    double A = ap_k(s, kf, d, face(s, i, j, k));
    for (int q = 0; q < s->NV; q++) Fa[q] = A * Fh[q];
}

static void stage(or_sim* s, int kf, const double* in, const double* base, double* out,
                  double a, double dt, double wflux)
{
    int D = s->D, NV = s->NV;
    double farea = pow(s->h, D - 1);
    for (long c = 0; c < s->nc; c++) {
        long i, j, k;
        coords(s, c, &i, &j, &k);
        double L[NVMAX], Xh[NVMAX];
        exchange(s, kf, c, Xh);
        for (int q = 0; q < NV; q++) L[q] = Xh[q];
        for (int d = 0; d < D; d++) {
            double Flo[NVMAX], Fhi[NVMAX];
            low_face_flux(s, kf, in, d, i, j, k, Flo);
            low_face_flux(s, kf, in, d, i + (d == 0), j + (d == 1), k + (d == 2), Fhi);
            for (int q = 0; q < NV; q++) L[q] += (Flo[q] - Fhi[q]) / s->h;
            if (s->P.bc[d] == 0) {
                long id = d == 0 ? i : (d == 1 ? j : k);
                if (id == 0)
                    for (int q = 0; q < NV; q++) s->bflux[kf][q] += wflux * farea * Flo[q];
                if (id == s->n[d] - 1)
                    for (int q = 0; q < NV; q++) s->bflux[kf][q] -= wflux * farea * Fhi[q];
            }
        }
        for (int q = 0; q < NV; q++) {
            long e = q * s->nc + c;
            double b = base[e];
            out[e] = a * b + (1.0 - a) * (in[e] + dt * L[q]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Level set: one Shu-Osher stage of Eq. (LS:linearadvection) with WENO5     */
/* upwind derivatives, on band cells only.                                   */
/* ------------------------------------------------------------------------ */

static void ls_stage(or_sim* s, double a, double dt)
{
    int D = s->D;
    double eps = s->P.weno_eps;
    for (long c = 0; c < s->nc; c++) {
        if (!s->M[c]) { s->phit[c] = s->phi[c]; continue; }
        double rhs = 0.0;
        for (int d = 0; d < D; d++) {
            double vd = s->v[d][c];
            if (vd == 0.0) continue;
            double p[7];
            for (int m = 0; m < 7; m++) p[m] = s->phi[nbr(s, c, d, m - 3)];
            double D1[6];
            for (int m = 0; m < 6; m++) D1[m] = (p[m + 1] - p[m]) / s->h;
            double der = vd > 0.0 ? or_weno5(D1[0], D1[1], D1[2], D1[3], D1[4], eps)
                                  : or_weno5(D1[5], D1[4], D1[3], D1[2], D1[1], eps);
            rhs -= vd * der;
        }
        s->phit[c] = a * s->phib[c] + (1.0 - a) * (s->phi[c] + dt * rhs);
    }
    memcpy(s->phi, s->phit, sizeof(double) * (size_t)s->nc);
}

/* ------------------------------------------------------------------------ */
/* Reinitialisation (Sec. 2.3): phi_tau + S(phi0)(|grad phi| - 1) = 0,         */
/* first-order Godunov upwind, dtau = h/2, Jacobi sweeps on band cells.      */
/* Cells near the interface are left untouched so that the reinitialisation  */
/* never moves the cut-cell geometry: a cell is frozen when one of its        */
/* 3^D neighbours sees both signs of phi0 in its own 3^D neighbourhood.       */
/* ------------------------------------------------------------------------ */

static int near_sign_change(const or_sim* s, const double* phi, long c)
{
    long i, j, k;
    coords(s, c, &i, &j, &k);
    int neg = 0, pos = 0;
    for (int dk = (s->D > 2 ? -1 : 0); dk <= (s->D > 2 ? 1 : 0); dk++)
        for (int dj = (s->D > 1 ? -1 : 0); dj <= (s->D > 1 ? 1 : 0); dj++)
            for (int di = -1; di <= 1; di++) {
                double v = phi[cell(s, i + di, j + dj, k + dk)];
                if (v < 0.0) neg = 1; else pos = 1;
            }
    return neg && pos;
}

static int frozen(const or_sim* s, const unsigned char* nearif, long c)
{
    long i, j, k;
    coords(s, c, &i, &j, &k);
    for (int dk = (s->D > 2 ? -1 : 0); dk <= (s->D > 2 ? 1 : 0); dk++)
        for (int dj = (s->D > 1 ? -1 : 0); dj <= (s->D > 1 ? 1 : 0); dj++)
            for (int di = -1; di <= 1; di++)
                if (nearif[cell(s, i + di, j + dj, k + dk)]) return 1;
    return 0;
}

static void reinit(or_sim* s)
{
    int D = s->D;
    double h = s->h, dtau = 0.5 * h;
    memcpy(s->phi0, s->phi, sizeof(double) * (size_t)s->nc);
    unsigned char* nearif = (unsigned char*)calloc((size_t)s->nc, 1);
    for (long c = 0; c < s->nc; c++) nearif[c] = (unsigned char)near_sign_change(s, s->phi0, c);
    for (int it = 0; it < s->P.reinit_iters; it++) {
        for (long c = 0; c < s->nc; c++) {
            s->phit[c] = s->phi[c];
            if (!s->M[c] || frozen(s, nearif, c)) continue;
            double p0 = s->phi0[c], pc = s->phi[c];
            double S = p0 / sqrt(p0 * p0 + h * h), g2 = 0.0;
            for (int d = 0; d < D; d++) {
                double am = (pc - s->phi[nbr(s, c, d, -1)]) / h;
                double bp = (s->phi[nbr(s, c, d, 1)] - pc) / h;
                double x, y;
                if (S > 0.0) { x = am > 0.0 ? am : 0.0; y = bp < 0.0 ? bp : 0.0; }
                else { x = am < 0.0 ? am : 0.0; y = bp > 0.0 ? bp : 0.0; }
                g2 += (x * x > y * y) ? x * x : y * y;
            }
            s->phit[c] = pc - dtau * S * (sqrt(g2) - 1.0);
        }
        memcpy(s->phi, s->phit, sizeof(double) * (size_t)s->nc);
    }
    free(nearif);
}

/* ------------------------------------------------------------------------ */
/* Small-cell mixing (Sec. 2.2): a cell with alpha_k < alpha_mix near the      */
/* interface exchanges M = beta [(aU)_t a_s - (aU)_s a_t] / (a_s + a_t) with   */
/* its neighbours t toward the bulk of fluid k (axis, face-diagonal and body-  */
/* diagonal), beta from the normal.  All M use the pre-mixing values.         */
/* ------------------------------------------------------------------------ */

static void mix(or_sim* s, int k, double* cons)
{
    int D = s->D, NV = s->NV;
    double band = s->P.mix_band * s->h;
    memset(s->dlt, 0, sizeof(double) * (size_t)(NV * s->nc));
    for (long c = 0; c < s->nc; c++) {
        double as = alpha_k(s, k, c);
        if (!(as < s->P.alpha_mix) || !(fabs(s->phi[c]) <= band)) continue;
        double gr[3];
        double gm = grad_phi(s, s->phi, c, gr);
        if (!(gm > 0.0)) continue;
        double dir[3] = {0, 0, 0};
        int sx[3] = {1, 1, 1};
        for (int d = 0; d < D; d++) {
            dir[d] = (k == 0 ? -1.0 : 1.0) * gr[d] / gm;  /* toward the bulk of fluid k */
            sx[d] = dir[d] < 0.0 ? -1 : 1;
        }
        /* candidate targets: every non-empty subset of the axes */
        int nsub = (1 << D) - 1;
        double beta[7];
        double bsum = 0.0;
        for (int m = 1; m <= nsub; m++) {
            int cnt = 0;
            double prod = 1.0;
            for (int d = 0; d < D; d++)
                if (m & (1 << d)) { cnt++; prod *= fabs(dir[d]); }
            double b;
            if (cnt == 1) b = prod * prod;
            else if (cnt == 2) b = prod;
            else b = pow(prod, 2.0 / 3.0);
            beta[m - 1] = b;
            bsum += b;
        }
        long i, j, kk;
        coords(s, c, &i, &j, &kk);
        for (int m = 1; m <= nsub; m++) {
            double b = beta[m - 1] / bsum;
            if (!(b > 0.0)) continue;
            long t = cell(s, i + ((m & 1) ? sx[0] : 0), j + ((m & 2) ? sx[1] : 0), kk + ((m & 4) ? sx[2] : 0));
            if (t == c) continue;
            double at = alpha_k(s, k, t);
            if (!(as + at > 0.0)) continue;
            for (int q = 0; q < NV; q++) {
                double Mq = b * (cons[q * s->nc + t] * as - cons[q * s->nc + c] * at) / (as + at);
                s->dlt[q * s->nc + c] += Mq;
                s->dlt[q * s->nc + t] -= Mq;
            }
        }
    }
    for (long e = 0; e < (long)NV * s->nc; e++) cons[e] += s->dlt[e];
}

/* ------------------------------------------------------------------------ */
/* Runge-Kutta tables (Shu-Osher form).  out_s = a_s base + (1-a_s)(in + dt L) */
/* c_s: time of the stage input relative to the step; b_s: the equivalent     */
/* quadrature weights, used for the flux bookkeeping of Sec. 3.1.             */
/* ------------------------------------------------------------------------ */

static const double RK3_A[3] = {0.0, 0.75, 1.0 / 3.0};
static const double RK3_C[3] = {0.0, 1.0, 0.5};
static const double RK3_B[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
static const double RK2_A[2] = {0.0, 0.5};
static const double RK2_C[2] = {0.0, 1.0};
static const double RK2_B[2] = {0.5, 0.5};

/* ------------------------------------------------------------------------ */
/* State set-up: cell contents alpha_k * U_k of piecewise-constant data.      */
/* ------------------------------------------------------------------------ */

static int prepare(or_sim* s, double* dt, long* cnt);

int or_set_state(or_sim* s, const double* phi, const double* prim)
{
    int NV = s->NV;
    memcpy(s->phi, phi, sizeof(double) * (size_t)s->nc);
    geometry(s);
    for (int k = 0; k < 2; k++)
        for (long c = 0; c < s->nc; c++) {
            double W[NVMAX], U[NVMAX];
            for (int q = 0; q < NV; q++) W[q] = prim[(k * NV + q) * s->nc + c];
            or_prim2cons(s->D, s->P.gamma[k], s->P.pinf[k], W, U);
            double a = alpha_k(s, k, c);
            for (int q = 0; q < NV; q++) s->X[k][q * s->nc + c] = a * U[q];
            /* the given states outside fluid k's region start its ghost states */
            for (int q = 0; q < NV; q++) s->W[k][q * s->nc + c] = W[q];
        }
    s->t = 0.0;
    memset(s->bflux, 0, sizeof s->bflux);
    return 0;
}

void or_get_state(const or_sim* s, double* phi, double* cons, double* alpha)
{
    if (phi) memcpy(phi, s->phi, sizeof(double) * (size_t)s->nc);
    if (cons)
        for (int k = 0; k < 2; k++)
            memcpy(cons + (size_t)k * s->NV * s->nc, s->X[k], sizeof(double) * (size_t)(s->NV * s->nc));
    if (alpha) memcpy(alpha, s->alpha, sizeof(double) * (size_t)s->nc);
}

void or_totals(const or_sim* s, double* out)
{
    double dv = pow(s->h, s->D);
    for (int k = 0; k < 2; k++)
        for (int q = 0; q < 5; q++) {
            double sum = 0.0;
            if (q < s->NV)
                for (long c = 0; c < s->nc; c++) sum += s->X[k][q * s->nc + c];
            out[k * 5 + q] = sum * dv;
        }
}

/* Start of a (sub)step: band mask, primitives, extension, interaction, CFL. */
static int prepare(or_sim* s, double* dt, long* cnt)
{
    band_mask(s);
    int rc = prims(s, 0, s->X[0]);
    if (!rc) rc = prims(s, 1, s->X[1]);
    if (rc) return rc;
    extend_w(s);
    interaction(s);
    extend_v(s);
    cfl_dt(s, dt, cnt);
    if (take_cfl(s, &dt[0]) || take_cfl(s, &dt[1])) return -2;
    return 0;
}

/* One stage of the level set (advection, and reinitialisation after a step's
 * last stage), or, with ls_replay, the level set this stage had in the
 * recorded run (frozen geometry); logged with log_levelset. */
static int ls_step(or_sim* s, double a, double dt, int last)
{
    if (s->n_ls_rep > 0) {
        if (s->ls_pos + s->nc > s->n_ls_rep) {
            snprintf(g_err, sizeof g_err, "ls_replay exhausted after %ld stages", s->ls_pos / s->nc);
            return -2;
        }
        memcpy(s->phi, s->ls_rep + s->ls_pos, sizeof(double) * (size_t)s->nc);
        s->ls_pos += s->nc;
    } else {
        ls_stage(s, a, dt);
        if (last) reinit(s);
    }
    if (s->P.log_levelset) {
        if (s->n_lslog + s->nc > s->cap_lslog) {
            s->cap_lslog = s->cap_lslog ? 2 * s->cap_lslog : 4 * s->nc;
            if (s->cap_lslog < s->n_lslog + s->nc) s->cap_lslog = s->n_lslog + s->nc;
            s->lslog = (double*)realloc(s->lslog, sizeof(double) * (size_t)s->cap_lslog);
        }
        memcpy(s->lslog + s->n_lslog, s->phi, sizeof(double) * (size_t)s->nc);
        s->n_lslog += s->nc;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The original method: both fluids and the level set advance with one dt.    */
/* Expects prepare() to have run on the current state.                        */
/* ------------------------------------------------------------------------ */

static int step_single(or_sim* s, double dt)
{
    int ns = s->P.rk;
    const double* A = ns == 3 ? RK3_A : RK2_A;
    const double* B = ns == 3 ? RK3_B : RK2_B;
    double* in[2] = {s->X[0], s->X[1]};
    memcpy(s->phib, s->phi, sizeof(double) * (size_t)s->nc);
    for (int st = 0; st < ns; st++) {
        if (st > 0) {
            int rc = prims(s, 0, in[0]);
            if (!rc) rc = prims(s, 1, in[1]);
            if (rc) return rc;
            extend_w(s);
            interaction(s);
            extend_v(s);
        }
        double* out[2];
        for (int k = 0; k < 2; k++) {
            out[k] = (st == ns - 1) ? s->X[k] : (st == 0 ? s->Y[k] : s->Z[k]);
            stage(s, k, in[k], s->X[k], out[k], A[st], dt, B[st] * dt);
        }
        int rc = ls_step(s, A[st], dt, st == ns - 1);
        if (rc) return rc;
        geometry(s);
        mix(s, 0, out[0]);
        mix(s, 1, out[1]);
        in[0] = out[0];
        in[1] = out[1];
    }
    s->t += dt;
    return 0;
}

/* slow fluid's intermediate state, Eq. (interpolation), mixed with the
 * current geometry unless it is the (already mixed) previous state */
static void interp_slow(or_sim* s, int S, double theta)
{
    long n = (long)s->NV * s->nc;
    for (long e = 0; e < n; e++) s->T[e] = (1.0 - theta) * s->X[S][e] + theta * s->Y[S][e];
    if (theta != 0.0) mix(s, S, s->T);
}

/* ------------------------------------------------------------------------ */
/* Scheduler helpers of Sec. 3.1.                                             */
/* ------------------------------------------------------------------------ */

void or_plan_cycle(double dt_slow, double dt_fast, double remaining, double thr,
                   double* dt_slow_out, int* single)
{
    double n = dt_slow / dt_fast;
    double fl = floor(n);
    double dts = (n - fl < thr) ? fl * dt_fast : dt_slow;
    if (dts > remaining) dts = remaining;
    *dt_slow_out = dts;
    *single = !(dts > dt_fast * (1.0 + 1e-12));
}

double or_substep(double tau, double t1, double dt_fast, int rk, int half_done,
                  int* hits_half, int* final_step)
{
    *hits_half = 0;
    *final_step = 0;
    double half = 0.5 * t1;
    if (rk == 3 && !half_done && tau < half) {
        if (tau + dt_fast * (1.0 + 1e-9) >= half) { *hits_half = 1; return half - tau; }
        return dt_fast;
    }
    if (tau + dt_fast * (1.0 + 1e-9) >= t1) { *final_step = 1; return t1 - tau; }
    return dt_fast;
}

/* ------------------------------------------------------------------------ */
/* The accelerated cycle of Sec. 3.1, generalised from RK2 to any Shu-Osher   */
/* table: the slow fluid S takes one step dt_S, the fast fluid F and the     */
/* level set take CFL sub-steps until t2 = t1; S's interaction states are    */
/* interpolated; every exchange term is booked into the correction so that  */
/* S finally receives minus what F received.  For RK3 the fast sub-steps     */
/* stop at t1/2 as well, where S's third stage is evaluated.                  */
/* ------------------------------------------------------------------------ */

static int cycle(or_sim* s, const double* dt, const long* cnt, double t_end, or_stats* st)
{
    int ns = s->P.rk, NV = s->NV;
    const double* A = ns == 3 ? RK3_A : RK2_A;
    const double* C = ns == 3 ? RK3_C : RK2_C;
    const double* B = ns == 3 ? RK3_B : RK2_B;
    int S = dt[0] >= dt[1] ? 0 : 1, F = 1 - S;
    double dtS, rem = t_end - s->t;
    int single;
    if (!isfinite(dt[F])) { S = F; F = 1 - S; }
    if (!isfinite(dt[S]) || !isfinite(dt[F])) {
        double d = dt[0] < dt[1] ? dt[0] : dt[1];
        if (d > rem) d = rem;
        single = 1;
        dtS = d;
    } else {
        or_plan_cycle(dt[S], dt[F], rem, s->P.n_thr, &dtS, &single);
        if (single && s->P.force_cycle && dtS >= dt[F] * (1.0 - 1e-12)) single = 0;
    }
    if (single) {
        int rc = step_single(s, dtS);
        if (rc) return rc;
        st->cycles++;
        for (int k = 0; k < 2; k++) { st->steps[k]++; st->cell_updates[k] += cnt[k]; }
        st->last_n = 1.0;
        return 0;
    }
    double t1 = dtS;
    st->last_n = t1 / dt[F];
    memset(s->corr, 0, sizeof(double) * (size_t)(NV * s->nc));
    /* (1) S's first stage with dt_S on I0; keep previous (X) and future (Y) */
    stage(s, S, s->X[S], s->X[S], s->Y[S], A[0], t1, B[0] * t1);
    double tau = 0.0, dtF = dt[F];
    int first = 1, half_done = 0, rc;
    long cntF = cnt[F];
    for (;;) {
        if (!first) {
            double d2[2];
            long c2[2];
            band_mask(s);
            interp_slow(s, S, tau / t1);
            rc = prims(s, S, s->T);
            if (!rc) rc = prims(s, F, s->X[F]);
            if (rc) return rc;
            extend_w(s);
            interaction(s);
            extend_v(s);
            cfl_dt(s, d2, c2);
            if (take_cfl(s, &d2[F])) return -2;
            dtF = d2[F];
            cntF = c2[F];
            if (!isfinite(dtF) || !(dtF > 0.0)) {
                snprintf(g_err, sizeof g_err, "invalid fast-fluid time step");
                return -4;
            }
        }
        int hh, fin;
        double dl = or_substep(tau, t1, dtF, ns, half_done, &hh, &fin);
        if (first && !s->P.no_correction) corr_add(s, S, -B[0] * t1 + B[0] * dl);
        memcpy(s->phib, s->phi, sizeof(double) * (size_t)s->nc);
        double* in = s->X[F];
        for (int q = 0; q < ns; q++) {
            if (q > 0) {
                double theta = (fin && C[q] == 1.0) ? 1.0 : (tau + C[q] * dl) / t1;
                interp_slow(s, S, theta);
                rc = prims(s, S, s->T);
                if (!rc) rc = prims(s, F, in);
                if (rc) return rc;
                extend_w(s);
                interaction(s);
                extend_v(s);
                if (fin && C[q] == 1.0) {
                    /* shared with S's second stage: Eq. (firstcorrection) */
                    if (!s->P.no_correction) corr_add(s, S, -B[q] * t1 + B[q] * dl);
                    stage(s, S, s->T, s->X[S], ns == 2 ? s->X[S] : s->Z[S], A[q], t1, B[q] * t1);
                } else if (!s->P.no_correction) {
                    corr_add(s, S, B[q] * dl);    /* Eq. (secondcorrection) */
                }
            } else if (!first && !s->P.no_correction) {
                corr_add(s, S, B[0] * dl);
            }
            double* out = (q == ns - 1) ? s->X[F] : (q == 0 ? s->Y[F] : s->Z[F]);
            stage(s, F, in, s->X[F], out, A[q], dl, B[q] * dl);
            rc = ls_step(s, A[q], dl, q == ns - 1);
            if (rc) return rc;
            geometry(s);
            mix(s, F, out);
            in = out;
        }
        st->steps[F]++;
        st->cell_updates[F] += cntF;
        tau = hh ? 0.5 * t1 : (fin ? t1 : tau + dl);
        if (hh) {
            half_done = 1;
            memcpy(s->Fh, s->X[F], sizeof(double) * (size_t)(NV * s->nc));
            memcpy(s->phih, s->phi, sizeof(double) * (size_t)s->nc);
        }
        first = 0;
        if (fin) break;
    }
    if (ns == 3) {
        /* S's third stage at t1/2 against the snapshot of F and the level set */
        memcpy(s->phit, s->phi, sizeof(double) * (size_t)s->nc);
        memcpy(s->phi, s->phih, sizeof(double) * (size_t)s->nc);
        memcpy(s->phi0, s->phit, sizeof(double) * (size_t)s->nc);  /* keep phi(t1) */
        geometry(s);
        memcpy(s->T, s->Z[S], sizeof(double) * (size_t)(NV * s->nc));
        mix(s, S, s->T);
        rc = prims(s, S, s->T);
        if (!rc) rc = prims(s, F, s->Fh);
        if (rc) return rc;
        extend_w(s);
        interaction(s);
        extend_v(s);
        if (!s->P.no_correction) corr_add(s, S, -B[2] * t1);
        stage(s, S, s->T, s->X[S], s->X[S], A[2], t1, B[2] * t1);
        memcpy(s->phi, s->phi0, sizeof(double) * (size_t)s->nc);
        geometry(s);
    }
    /* interfacial flux correction of the slow fluid, then mixing */
    if (!s->P.no_correction)
        for (int q = 1; q < NV; q++)
            for (long c = 0; c < s->nc; c++) s->X[S][q * s->nc + c] += s->corr[q * s->nc + c];
    mix(s, S, s->X[S]);
    s->t += t1;
    st->cycles++;
    st->steps[S]++;
    st->cell_updates[S] += cnt[S];
    return 0;
}

int or_advance(or_sim* s, double t_end, int mode, long max_cycles, or_stats* st)
{
    or_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    long done = 0;
    int rc = 0;
    while (s->t < t_end && (max_cycles <= 0 || done < max_cycles)) {
        double dt[2];
        long cnt[2];
        rc = prepare(s, dt, cnt);
        if (rc) break;
        st->last_dt[0] = dt[0];
        st->last_dt[1] = dt[1];
        if (!(fmin(dt[0], dt[1]) > 0.0)) { snprintf(g_err, sizeof g_err, "invalid time step"); rc = -4; break; }
        if (mode == 0) {
            double d = dt[0] < dt[1] ? dt[0] : dt[1];
            if (d > t_end - s->t) d = t_end - s->t;
            rc = step_single(s, d);
            if (rc) break;
            st->cycles++;
            for (int k = 0; k < 2; k++) { st->steps[k]++; st->cell_updates[k] += cnt[k]; }
            st->last_n = 1.0;
        } else {
            rc = cycle(s, dt, cnt, t_end, st);
            if (rc) break;
        }
        if (t_end - s->t <= 1e-14 * t_end) s->t = t_end;
        done++;
    }
    st->t = s->t;
    memcpy(st->bflux, s->bflux, sizeof s->bflux);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Unit-level runs of single method steps, for the pin tests: each creates a  */
/* simulation object, runs the step exactly as the schedule above does, and   */
/* copies the result out.                                                     */
/* ------------------------------------------------------------------------ */

/* Level-set transport, Eq. (LS:linearadvection) of Sec. 2.3, by a prescribed
 * velocity field vel[D][cells] held fixed: nsteps steps of length dt, each
 * the band of the step start, the Shu-Osher stages of ls_stage and the
 * reinitialisation (reinit_iters sweeps), as in step_single.  phi in/out. */
int or_ls_transport(const or_params* p, double* phi, const double* vel, double dt, int nsteps)
{
    or_sim* s = or_create(p);
    if (!s) return -1;
    size_t nb = sizeof(double) * (size_t)s->nc;
    memcpy(s->phi, phi, nb);
    for (int d = 0; d < s->D; d++) memcpy(s->v[d], vel + (size_t)d * s->nc, nb);
    int ns = s->P.rk;
    const double* A = ns == 3 ? RK3_A : RK2_A;
    for (int it = 0; it < nsteps; it++) {
        band_mask(s);
        memcpy(s->phib, s->phi, nb);
        for (int st = 0; st < ns; st++) ls_stage(s, A[st], dt);
        reinit(s);
    }
    memcpy(phi, s->phi, nb);
    or_destroy(s);
    return 0;
}

/* Reinitialisation alone (Sec. 2.3): the band of phi, then reinit_iters
 * Jacobi sweeps with the cells next to the interface held.  phi in/out. */
int or_reinit_run(const or_params* p, double* phi)
{
    or_sim* s = or_create(p);
    if (!s) return -1;
    size_t nb = sizeof(double) * (size_t)s->nc;
    memcpy(s->phi, phi, nb);
    band_mask(s);
    reinit(s);
    memcpy(phi, s->phi, nb);
    or_destroy(s);
    return 0;
}

/* Extension of the level-set velocity v[D][cells] (in/out) from the cut
 * cells of the geometry of phi over the band (ext_iters sweeps). */
int or_extend_v_run(const or_params* p, const double* phi, double* v)
{
    or_sim* s = or_create(p);
    if (!s) return -1;
    size_t nb = sizeof(double) * (size_t)s->nc;
    memcpy(s->phi, phi, nb);
    geometry(s);
    band_mask(s);
    for (int d = 0; d < s->D; d++) memcpy(s->v[d], v + (size_t)d * s->nc, nb);
    extend_v(s);
    for (int d = 0; d < s->D; d++) memcpy(v + (size_t)d * s->nc, s->v[d], nb);
    or_destroy(s);
    return 0;
}

/* Extension of the primitives W[2][NV][cells] (in/out) of each fluid into
 * its ghost cells of the geometry of phi (ext_iters sweeps). */
int or_extend_w_run(const or_params* p, const double* phi, double* W)
{
    or_sim* s = or_create(p);
    if (!s) return -1;
    size_t nb = sizeof(double) * (size_t)s->nc * (size_t)s->NV;
    memcpy(s->phi, phi, sizeof(double) * (size_t)s->nc);
    geometry(s);
    band_mask(s);
    for (int k = 0; k < 2; k++) memcpy(s->W[k], W + (size_t)k * s->NV * s->nc, nb);
    extend_w(s);
    for (int k = 0; k < 2; k++) memcpy(W + (size_t)k * s->NV * s->nc, s->W[k], nb);
    or_destroy(s);
    return 0;
}

int or_curvature_run(const or_params* p, const double* phi, double* kappa)
{
    or_sim* s = or_create(p);
    if (!s) return -1;
    for (long c = 0; c < s->nc; c++) kappa[c] = curvature(s, phi, c);
    or_destroy(s);
    return 0;
}
