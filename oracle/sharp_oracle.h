/*
 * sharp_oracle.h -- plain FP64 CPU oracle of the accelerated sharp-interface
 * method (Long, Cai & Pan, "An accelerated sharp-interface method for
 * multiphase flows simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke entry point and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU path.
 *
 * Conventions (all arrays are host memory, FP64, structure of arrays,
 * x fastest):
 *   cell index    c = i + n0*(j + n1*k)
 *   fluid 0       the fluid where phi < 0; fluid 1 where phi >= 0
 *   prim[k][q][c] primitive state of fluid k: q = 0 rho, 1..D velocity, D+1 p
 *   cons[k][q][c] conserved cell content of fluid k divided by the cell
 *                 volume, i.e. alpha_k * U_k (Sec. 2.1, Eq. Eulerdiscrete)
 */
#ifndef SHARP_ORACLE_H
#define SHARP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_sim or_sim;

typedef struct {
    int ndim;            /* 1, 2 or 3 */
    int n[3];            /* cells per direction (unused directions: 1) */
    double lo[3];        /* lower domain corner */
    double h;            /* uniform cell size, equal in all directions */
    int bc[3];           /* 0 zero-gradient, 1 periodic (per direction) */
    double gamma[2];     /* stiffened-gas gamma of fluid 0 / fluid 1 */
    double pinf[2];      /* stiffened-gas p_inf of fluid 0 / fluid 1 */
    double cfl;          /* CFL number (0.6 in Sec. 4) */
    int rk;              /* 3: SSP-RK3 (default), 2: the paper's TVD-RK2 */
    double n_thr;        /* threshold on the fractional part of n (0.7, Sec. 3.1) */
    double alpha_mix;    /* small-cell threshold of the mixing step (0.5) */
    double ls_band;      /* level-set band half width, in cells (8) */
    double ext_band;     /* ghost-fluid extension depth, in cells (5) */
    double mix_band;     /* |phi| limit for mixing sources, in cells (3) */
    int ext_iters;       /* Jacobi sweeps of the extension (8) */
    int reinit_iters;    /* reinitialisation sweeps per level-set step (2) */
    double weno_eps;     /* WENO epsilon (1e-6) */
    int force_cycle;     /* test hook: run the accelerated cycle even when n < 2 */
    int no_correction;   /* test hook: skip the interfacial flux correction */
    const double* dt_replay;  /* n_dt_replay > 0: CFL steps taken instead of the
                                 computed ones, in or_schedule's order (copied) */
    long n_dt_replay;
    int log_levelset;    /* record the level set after every stage that advances it */
    const double* ls_replay;  /* n_ls_replay > 0: the stages that advance the level set
                                 (every single-dt stage; every fast sub-step stage of an
                                 accelerated cycle) take these level sets (cells each,
                                 in or_levelset_log's order) instead of advecting and
                                 reinitialising (copied) */
    long n_ls_replay;
    double sigma;        /* surface tension coefficient of the interface (0: none);
                            the interaction then takes the Laplace pressure jump
                            p_0 - p_1 = sigma kappa of Eq. (surfacetension) */
} or_params;

typedef struct {
    long cycles;          /* cycles (multi_dt) or steps (single_dt) */
    long steps[2];        /* complete RK steps taken by each fluid */
    long cell_updates[2]; /* sum over those steps of cells with alpha_k > 0 */
    double t;             /* simulation time reached */
    double last_n;        /* time-step ratio n of the last cycle (1 for single_dt) */
    double last_dt[2];    /* last CFL time step of each fluid */
    double bflux[2][5];   /* time-integrated boundary inflow of each fluid */
} or_stats;

void or_default_params(or_params* p);
or_sim* or_create(const or_params* p);
void or_destroy(or_sim* s);
/* phi[cells], prim[2][NV][cells]; returns 0 or a negative error code */
int or_set_state(or_sim* s, const double* phi, const double* prim);
/* mode 0 single_dt (the original method), 1 multi_dt (the accelerated one).
 * Stops at t_end or after max_cycles cycles/steps (if > 0). */
int or_advance(or_sim* s, double t_end, int mode, long max_cycles, or_stats* st);

/* CFL steps taken since or_create, in the order they were taken: both
 * fluids' (fluid 0 first) at each cycle or single-dt step start, the fast
 * fluid's at each later fast sub-step start (the order dt_replay follows).
 * Copies up to cap values to out (may be NULL); returns the total count. */
long or_schedule(const or_sim* s, double* out, long cap);
/* Level sets recorded with log_levelset: after each stage that advances the
 * level set (each single-dt stage, each fast sub-step stage of an
 * accelerated cycle; the reinitialised one after a step's last stage),
 * cells values each.
 * Copies up to cap values to out (may be NULL); returns the total count.
 * Replaying them (ls_replay) fixes the geometry of every stage, so that the
 * state at the end of the run is a function of the initial state and the
 * EOS alone: the map the adjoint with frozen geometry differentiates. */
long or_levelset_log(const or_sim* s, double* out, long cap);
void or_get_state(const or_sim* s, double* phi, double* cons, double* alpha);
/* total content sum_c dV * cons[k][q][c]  -> out[k*5+q] */
void or_totals(const or_sim* s, double* out);
const char* or_last_error(void);

/* ---- unit-level entry points, exported for the pin tests ---- */
void or_prim2cons(int D, double gamma, double pinf, const double* W, double* U);
int or_cons2prim(int D, double gamma, double pinf, const double* U, double* W);
double or_weno5(double v0, double v1, double v2, double v3, double v4, double eps);
/* exact two-material stiffened-gas Riemann problem: out = {p*, u*, rho*L, rho*R, iters} */
int or_riemann(const double* WL, const double* WR, double gL, double piL,
               double gR, double piR, double* out);
/* the same problem with the pressure jump p_L - p_R = jump across the
 * contact (Eq. surfacetension): out = {p*_L, u*, rho*L, rho*R, iters}, and
 * the right side's contact pressure is p*_L - jump */
int or_riemann_jump(const double* WL, const double* WR, double gL, double piL,
                    double gR, double piR, double jump, double* out);
/* sample the exact solution at xi = x/t: out = {rho, u, p, side} */
void or_riemann_sample(const double* WL, const double* WR, double gL, double piL,
                       double gR, double piR, double xi, double* out);
double or_clip_area(const double* v4);
/* one LLF-WENO5 face flux of a 1-D six-cell primitive stencil (rho,u,p) */
void or_face_flux_1d(const double* W6, double gamma, double pinf, double eps, double* F);
/* geometry of the current level set: alpha[cells], ap[d][padded faces] */
void or_geometry(const or_sim* s, double* alpha, double* ap);
long or_face_count(const or_sim* s);
/* scheduler helpers (Sec. 3.1) */
void or_plan_cycle(double dt_slow, double dt_fast, double remaining, double thr,
                   double* dt_slow_out, int* single);
double or_substep(double tau, double t1, double dt_fast, int rk, int half_done,
                  int* hits_half, int* final_step);
/* single method steps run alone (Sec. 2.3), arrays [D or NV][cells] */
int or_ls_transport(const or_params* p, double* phi, const double* vel, double dt, int nsteps);
int or_reinit_run(const or_params* p, double* phi);
int or_extend_v_run(const or_params* p, const double* phi, double* v);
int or_extend_w_run(const or_params* p, const double* phi, double* W);
/* curvature of the level set at the interface point nearest each cell
 * centre, kappa[cells] (0 in 1-D) */
int or_curvature_run(const or_params* p, const double* phi, double* kappa);

#ifdef __cplusplus
}
#endif
#endif
