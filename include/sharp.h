/*
 * sharp.h -- C ABI of the gfx950 (MI355X) implementation of the accelerated
 * sharp-interface method of Long, Cai & Pan, "An accelerated sharp-interface
 * method for multiphase flows simulations".
 *
 * The library advances two compressible fluids separated by a level-set
 * interface on a uniform Cartesian grid (1-D, 2-D or 3-D, FP64):
 *   - each fluid's cut-cell finite-volume update, Eq. (Eulerdiscrete) of
 *     Sec. 2.1, with a WENO5 flux (local Lax-Friedrichs splitting) and a
 *     Shu-Osher Runge-Kutta stage (SSP-RK3 by default, the paper's TVD-RK2
 *     on request, Sec. 3);
 *   - the level-set geometry, interface interaction (exact two-material
 *     stiffened-gas Riemann problem), ghost-fluid extension, small-cell
 *     mixing, level-set advection Eq. (LS:linearadvection) and
 *     reinitialisation (Sec. 2.2-2.3);
 *   - the original method (one CFL time step for both fluids) or the
 *     accelerated cycle of Sec. 3.1 (each fluid with its own CFL step, the
 *     slow fluid's intermediate states by Eq. (interpolation), interfacial
 *     flux correction by Eqs. (firstcorrection)/(secondcorrection)).
 *
 * Conventions.  Fluid 0 occupies phi < 0, fluid 1 phi >= 0.  Arrays are FP64
 * structure-of-arrays with x fastest: cell c = i + n0*(j + n1*k).
 *   phi[c]          level set (signed distance to the interface)
 *   prim[k][q][c]   primitive state of fluid k, q = rho, u_1..u_D, p
 *   cons[k][q][c]   cell content of fluid k per cell volume, alpha_k * U_k,
 *                   q = rho, rho u_1..rho u_D, E
 *   alpha[c]        volume fraction of fluid 0
 * NV = D + 2 components.
 *
 * Ownership and errors.  The library allocates and owns every device buffer
 * of a simulation.  Caller arrays are only read or written during a call;
 * `on_device` tells whether they are device pointers (ordered on the
 * simulation's stream) or host pointers.  Handles are not thread safe.  No
 * exception crosses the ABI: every call returns a sim_status, and
 * sim_last_error() returns a description of the last failure on this thread.
 */
#ifndef SHARP_H
#define SHARP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest grid (cells) on which opts->graph = 1 captures single-dt steps:
 * 512^2, where a captured step of the 2-D shock-bubble case still measured
 * 1.01x the launches it replaces (1.5x on a 400-cell tube). */
#define SIM_GRAPH_MAX_CELLS 262144
/* ... and accelerated cycles with prescribed steps (opts->dt_fixed_fluid):
 * 256^2, where a captured cycle of the shock-bubble case measured 1.04x
 * (0.95x at 512^2, 1.37x on a 400-cell tube). */
#define SIM_GRAPH_MAX_CELLS_CYCLE 65536

typedef struct sim sim_t;

typedef enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,    /* invalid argument */
    SIM_ENOMEM = -2,    /* device allocation failed */
    SIM_EDEVICE = -3,   /* HIP runtime error, or the interface band outran its tiles */
    SIM_ENONPHYS = -4,  /* rho <= 0, p + p_inf <= 0, NaN, or no valid time step */
    SIM_ESTATE = -5     /* call out of order (e.g. advance before set_state) */
} sim_status;

typedef enum { SIM_SINGLE_DT = 0, SIM_MULTI_DT = 1 } sim_mode;

/* Uniform grid: n cells per direction on [lo, lo + n h]; unused directions
 * have n = 1.  bc: 0 zero-gradient, 1 periodic (per direction). */
typedef struct {
    int ndim;
    int64_t n[3];
    double lo[3];
    double h;
    int bc[3];
} sim_grid;

/* Stiffened gas p = (gamma - 1) rho e - gamma p_inf (p_inf finite; the
 * states must keep p + p_inf > 0).  The paper's Tait fluids (Sec. 2.2, Eq.
 * Tait's equation) are the isentropes with p_inf = B - p0, negative where
 * B < p0 (the gas-like fluid of Sec. 4.3). */
typedef struct {
    double gamma;
    double pinf;
} sim_eos;

/* Options; sim_default_opts() fills the values in brackets. */
typedef struct {
    double cfl;          /* CFL number [0.6] (Sec. 4) */
    int rk;              /* 3: SSP-RK3 [3]; 2: the paper's TVD-RK2 */
    double n_thr;        /* fractional-part threshold of n [0.7] (Sec. 3.1) */
    double alpha_mix;    /* small-cell mixing threshold [0.5] */
    double ls_band;      /* level-set band half width, cells [8] */
    double ext_band;     /* extension depth, cells [5] */
    double mix_band;     /* |phi| limit of mixing sources, cells [3] */
    int ext_iters;       /* Jacobi sweeps of the extension [8] */
    int reinit_iters;    /* reinitialisation sweeps per level-set step [2] */
    double weno_eps;     /* WENO epsilon [1e-6] */
    int force_cycle;     /* run the accelerated cycle even when n truncates to 1 [0] */
    int no_correction;   /* skip the interfacial flux correction (diagnostic) [0] */
    int serial;          /* run every kernel on the simulation's stream instead of
                            overlapping the bulk-tile stages with the band work on
                            two library-owned streams; results are identical [0] */
    int tape;            /* record the run (single-dt steps and, with an
                            interface, accelerated cycles) for sim_backward [0] */
    int ckpt_every;      /* taped steps between stored states (checkpoints) [20] */
    double dt_fixed;     /* > 0: single-dt steps of this length (the last one
                            clamped to t_end) instead of the CFL step, so that
                            perturbed runs share one schedule [0] */
    int autotune;        /* time the first cycles with each candidate launch
                            (bulk-tile stage grid bound 1024-8192 with the
                            bulk stages overlapped, and the serial schedule)
                            and keep the fastest; results do not depend on
                            the choice [0] */
    int graph;           /* with dt_fixed > 0: capture a whole single-dt step
                            of that length (with dt_fixed_fluid: a whole
                            accelerated cycle, all its fast sub-steps; the same
                            rules hold) (band tiles, interaction and CFL
                            reductions, then all stages of both fluids, level
                            set, mixing; every kernel in one chain, with no
                            side streams) into a HIP graph once per launch
                            configuration, and enqueue the whole steps of a
                            sim_advance call as replays without waiting for
                            any: the active-cell counts are summed on the
                            device and read back, with the error flags, once
                            after them (an error is reported at the end of
                            that run of steps).  Results are identical to the
                            launches issued one by one.  Steps under a tape, a
                            batch, kernel profiling or an unfinished autotuner,
                            and a step shortened to reach t_end, are issued
                            one by one.  1: capture on grids of at most
                            SIM_GRAPH_MAX_CELLS cells (measured faster up to
                            there; on larger grids the bulk stages overlapped
                            on side streams win and the steps are issued one
                            by one; SIM_GRAPH_MAX_CELLS_CYCLE cells for
                            accelerated cycles); 2: capture at any size [0] */
    int no_rollback;     /* do not keep the state of the last cycle start: a
                            call that fails with SIM_ENONPHYS then leaves the
                            state of the failing step instead of rolling it
                            back (saves one copy of the contents and level
                            set per cycle, 2 NV + 1 fields of memory) [0] */
    int grid_cap;        /* > 0: at most this many blocks for every kernel that
                            walks a tile list (each block then loops over
                            several tiles; a multiple of 8 keeps the XCD-aware
                            tile order, other values use a plain stride).  The
                            kernels loop over the device-side list counts, so
                            results do not depend on it; for tests and
                            tuning [0] */
    const double* dt_replay;   /* with n_dt_replay > 0: the CFL steps to take
                            instead of the computed ones, in the order
                            sim_schedule reports them (both fluids' at each
                            cycle or single-dt step start, fluid 0 first; the
                            fast fluid's at each later fast sub-step start).
                            Copied at sim_create.  A parity run replays the
                            other library's schedule, so that a rounding
                            difference in a CFL step cannot change a sub-step
                            count (a reading of Sec. 3.1's truncation test);
                            running past the end fails with SIM_EINVAL [NULL] */
    int64_t n_dt_replay; /* entries of dt_replay [0] */
    const double* ls_replay;   /* with n_ls_replay > 0: the level set of every
                            stage of the single-dt steps to take, in stage
                            order, as sim_levelset_tape reports them
                            (n_ls_replay = stages x cells), used instead of
                            the stage's advection and reinitialisation.  Each
                            stage then has the recorded cut-cell geometry
                            (Sec. 2.3), so that the contents at the end of a
                            run are a function of the initial state and the
                            EOS alone: the map sim_backward differentiates
                            when an interface is present, and what finite
                            differences of it perturb.  Host array, copied at
                            sim_create; every sim_set_state starts again from
                            its first level set.  Single-dt steps only
                            (SIM_EINVAL for accelerated cycles, when it runs
                            out, and together with opts.tape) [NULL] */
    int64_t n_ls_replay; /* entries of ls_replay [0] */
    double sigma;        /* surface tension coefficient of the interface
                            (Sec. 3.1, Eq. surfacetension).  Nonzero: each cut
                            cell's interaction takes the Laplace pressure jump
                            p*_0 - p*_1 = sigma kappa across the contact, kappa
                            = div(grad phi / |grad phi|) from central
                            differences of the level set, moved to the
                            interface point nearest the cell centre as for a
                            circle or sphere (positive where fluid 0, phi < 0,
                            is convex); each fluid's exchange term takes its
                            own interface pressure, and the interfacial flux
                            correction books the slow fluid's (Eqs.
                            firstcorrection_surfacetension and
                            secondcorrection_surface_tension).  No effect in
                            1-D.  sim_backward differentiates it with the
                            geometry frozen (the jump of each cut cell a
                            constant of the recorded level set) [0] */
    double dt_fixed_fluid[2]; /* both > 0: accelerated cycles (SIM_MULTI_DT)
                            take these steps of fluid 0 and fluid 1 instead of
                            their CFL steps; the cycle's plan (Sec. 3.1: the
                            slow fluid's step, n with the 0.7 truncation, the
                            fast sub-steps stopping at t1/2 for RK3 and at t1)
                            follows from them as from CFL steps.  With
                            opts.graph, every whole cycle before t_end is
                            captured into a HIP graph once per launch
                            configuration and replayed, without host
                            readbacks between cycles.  Both 0 or both > 0;
                            not together with dt_replay or tape (SIM_EINVAL)
                            [0, 0] */
} sim_opts;

typedef struct {
    int64_t cycles;          /* accelerated cycles, or original steps */
    int64_t steps[2];        /* complete RK steps taken by each fluid */
    int64_t cell_updates[2]; /* sum over those steps of the cells holding the fluid */
    double t;                /* simulation time reached */
    double last_n;           /* time-step ratio of the last cycle (1 for a single-dt step) */
    double last_dt[2];       /* last CFL time step of each fluid */
    double bflux[2][5];      /* time-integrated inflow through the domain boundary,
                                per fluid and component (x dV units) */
    int64_t active_cells[2]; /* cells holding each fluid (alpha_k > 0) at the start
                                of the call's last cycle or step */
} sim_stats;

/* Fill *o with the defaults listed above. */
void sim_default_opts(sim_opts* o);

/* Create a simulation of the two-fluid problem of Sec. 2.1 (the Euler
 * equations of each fluid, Eq. (EulerEquation), on one uniform grid, with
 * the interface the zero level set of Sec. 2.3).  eos[0] is fluid 0
 * (phi < 0), eos[1] fluid 1.
 * stream: a hipStream_t to order all work on, or NULL for a private stream.
 * Unless opts->serial is set, the library also creates two non-blocking
 * streams for the bulk-tile stages; every call joins them back into `stream`
 * before it returns, so callers see all work ordered on `stream`.
 * Requires equal spacing in every direction (h), 1 <= ndim <= 3,
 * n[d] >= 1, gamma > 1, p_inf finite, rk in {2, 3}.  Returns SIM_EINVAL on bad
 * arguments, SIM_ENOMEM if device memory runs out. */
sim_status sim_create(const sim_grid* grid, const sim_eos eos[2], const sim_opts* opts,
                      void* stream, sim_t** out);

/* Set the state from a level set phi[cells] and primitives prim[2][NV][cells]
 * (Sec. 2.1: the cut cells receive alpha_k * U_k of the given piecewise
 * states).  The primitives given outside a fluid's region initialise that
 * fluid's ghost states.  Resets time and the boundary-flux ledger. */
sim_status sim_set_state(sim_t* s, const double* phi, const double* prim, int on_device);

/* Advance to t_end with the original method of Sec. 3.1 (SIM_SINGLE_DT: one
 * CFL time step for both fluids and the level set) or the accelerated cycle
 * of Sec. 3.1 (SIM_MULTI_DT: the slow fluid takes one step of its own CFL
 * length, truncated to a whole number of fast steps when the fractional
 * part of n is below 0.7; the fast fluid sub-steps with its CFL step,
 * interacting with the slow fluid's states interpolated by Eq.
 * (interpolation); the interfacial flux correction of Eqs.
 * (firstcorrection)/(secondcorrection) keeps the update conservative),
 * stopping early after max_cycles cycles/steps when max_cycles > 0.  The
 * last cycle is shortened so that t lands on t_end.  Statistics of this
 * call go to *out (nullable).
 * On SIM_ENONPHYS (a state with rho <= 0, p + p_inf <= 0 or NaN, or no valid
 * time step) the contents, level set, boundary ledger and time are rolled
 * back to the start of the failing cycle or step, the last completed one
 * (unless opts->no_rollback); *out then counts the completed cycles only,
 * and sim_last_error() names the fluid, the cell and the time of the
 * failing cycle.  The extension's and the Riemann solver's warm-start values
 * are not rolled back, so a repeated call can differ from the first at the
 * level of their stopping tolerances.  A run of captured steps (opts->graph)
 * learns of a failure only after the whole run: it rolls back to the start
 * of that run.  Batched simulations (sim_batch_advance) are not rolled back:
 * they keep the state of the failing step. */
sim_status sim_advance(sim_t* s, double t_end, int mode, int64_t max_cycles, sim_stats* out);

/* Copy the level set, the cell contents cons[2][NV][cells] = alpha_k U_k
 * (the per-volume contents that Eq. (Eulerdiscrete) of Sec. 2.1 advances)
 * and the fluid-0 volume fraction out (any pointer may be NULL). */
sim_status sim_get_state(sim_t* s, double* phi, double* cons, double* alpha, int on_device);

/* Conservation ledger (the totals whose drift Sec. 4.2 tracks): the total
 * content sum_c dV cons[k][q][c] -> out[k*5 + q] (q < NV; 0 for q >= NV),
 * by a fixed-order tree reduction on the device (the same state always gives
 * the same bits).  out10 is a host array. */
sim_status sim_totals(sim_t* s, double* out10);

/* sim_totals for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same totals, bit for bit, with the reduction's partial sums kept in a
 * file-scope device array of 41 KB per device (512 x 10 partial sums and the
 * 10 totals; its size does not depend on the grid, so no grid is refused for
 * it) instead of a buffer allocated per call.  No hipMalloc, hipFree or
 * other allocation.  on_device = 1: out10 is a device pointer, written on
 * the simulation's stream without waiting (ordered like the other work of
 * the simulation); 0: out10 is a host array and the call waits for it.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (simulations on different streams, or threads) race, and
 * must be ordered by the caller.  SIM_ESTATE before sim_set_state. */
sim_status sim_totals_noalloc(sim_t* s, double* out10, int on_device);

/* Kernel timing of the fused face-flux/RK stage kernel on bulk tiles: when
 * enabled, sim_advance brackets every launch of it with HIP events on the
 * stream the kernel runs on.  sim_profile_read returns the summed duration
 * (ms), the number of launches, the cells those launches advanced by one
 * stage (summed over launches), and how many of them were first stages of a
 * step (which read no base state).  Enabling resets the counters. */
sim_status sim_profile(sim_t* s, int enable);
sim_status sim_profile_read(sim_t* s, double* ms, int64_t* launches, int64_t* cells, int64_t* first_cells);

/* Adjoint of the taped run (opts->tape = 1): the gradient of a scalar J
 * through every sim_advance call since the last sim_set_state (single-dt
 * steps and, with an interface, accelerated cycles), with the step lengths
 * frozen at their forward values.
 * The map is the composition of the Shu-Osher stages (Sec. 2.1, Sec. 3) of
 * the cut-cell finite-volume update (Eq. Eulerdiscrete: WENO5-LLF face
 * fluxes times the fluid's apertures, and the exchange term of the
 * interface Riemann problem) with the primitive recovery, the ghost-fluid
 * extension and the small-cell mixing of each stage, and of the initial
 * prim -> cons map (alpha_k U(W_k)).  With an interface, the geometry is
 * frozen: every stage's level set is the recorded one (see
 * opts.ls_replay), so the derivative is that of the replayed run; the
 * exchange term's p*, u* are differentiated by the implicit function
 * theorem on the Riemann root (with surface tension, opts.sigma, across the
 * Laplace jump of the recorded level set, a constant of each cut cell);
 * extension and mixing are linear maps with
 * their recorded coefficients, and the ghost values an extension starts
 * from (the previous extension's results; sim_set_state's primitives at
 * the first) are differentiated through.  A run in which one fluid fills
 * the grid has no interface and none of these steps.  Accelerated cycles
 * (Sec. 3.1) add the slow fluid's interpolation, Eq. (interpolation), and
 * the interfacial flux correction, Eqs. (firstcorrection) and
 * (secondcorrection), both linear maps of the recorded states.  The forward
 * stores the state every ckpt_every steps or cycles (with an interface:
 * both fluids' contents, the level set and the start interaction's
 * results, and the level set of every stage that advances it); the
 * backward replays each segment from its checkpoint, every kernel on the
 * simulation's stream, and runs the reverse sweep through it; the gradient
 * does not depend on ckpt_every.
 * Afterwards the simulation holds the state the forward ended with.
 *   g_cons[2][NV][cells]  dJ/dcons at the end of the run (input)
 *   g_prim0[2][NV][cells] dJ/dprim given to sim_set_state (output; zero for
 *                         a fluid that holds no cell)
 *   g_eos[4]              dJ/dgamma_0, dJ/dpinf_0, dJ/dgamma_1, dJ/dpinf_1
 *                         through the dynamics and the initial prim -> cons
 *                         map (host array, output; nullable)
 * Returns SIM_EINVAL when the run is not covered (accelerated cycles of a
 * run in which one fluid fills the grid, a rolled-back step; the message
 * says why), SIM_ESTATE without a tape, SIM_ENOMEM when the recomputation
 * buffers (one fluid: 3 ckpt_every states; with an interface: a record of
 * about 4 NV + 2 D + 6 fields per interaction of ckpt_every steps or
 * cycles) do not fit. */
sim_status sim_backward(sim_t* s, const double* g_cons, double* g_prim0, double* g_eos, int on_device);

/* The level sets a taped run with an interface recorded: after each stage
 * of each single-dt step and of each fast sub-step of an accelerated cycle
 * (after the reinitialisation at a step's last stage), cells values each,
 * in stage order; opts.ls_replay takes the single-dt ones.
 * Up to cap values are copied to the host array out, and *n (if not NULL)
 * receives the total count.  SIM_ESTATE when the simulation holds no such
 * tape. */
sim_status sim_levelset_tape(sim_t* s, double* out, int64_t cap, int64_t* n);

/* Launch configuration in use: the bulk-tile stage's grid bound (blocks),
 * the schedule (serial = 1: every kernel on the simulation's stream; 0: the
 * bulk-tile stages overlapped on the side streams), and whether the
 * autotuner (opts->autotune) has finished choosing them.  Any pointer may be
 * NULL. */
sim_status sim_tuned(sim_t* s, int* bulk_blocks, int* serial, int* done);

/* The CFL steps the simulation has taken since sim_create (or replayed from
 * opts->dt_replay), in the order described there: up to cap values are
 * copied to the host array out, and *n (if not NULL) receives the total
 * count.  out may be NULL to query the count.  Single-dt steps of the fixed
 * length opts->dt_fixed take no CFL step and add nothing. */
sim_status sim_schedule(sim_t* s, double* out, int64_t cap, int64_t* n);

/* Captured steps (opts->graph): the number of single-dt steps captured into
 * HIP graphs and the number replayed from one (the capturing step included),
 * and the graphs held (at most 4, one per launch configuration: the grid
 * sizes follow the tile counts rounded up to powers of two).  Any pointer
 * may be NULL.  The graphs are released by sim_destroy. */
sim_status sim_graph_info(sim_t* s, long long* captures, long long* replays, int* held);

/* ---- batches: many simulations advanced together ----
 * A batch advances independent simulations (any sizes, dimensions and
 * options; each created, filled and read with the calls above) to their own
 * end times, running each one's single-dt steps or accelerated cycles
 * (Sec. 3.1) unchanged, while the kernel launches of all of them are fused:
 * the launches of every simulation up to its next host decision (CFL steps,
 * tile lists, sub-step plan: a readback of its reduction block) are merged
 * into one launch per kernel over all simulations that have it next, and
 * one copy brings every simulation's readback to the host.  Each
 * simulation takes the steps sim_advance would take on it alone and reaches
 * the same state up to round-off (the fused kernels are the same kernel
 * bodies compiled in another context).
 *   sims[n]     simulations (1 <= n <= SIM_BATCH_MAX), distinct, without a
 *               tape; borrowed: they must outlive the batch and must not be
 *               used from another thread during sim_batch_advance
 * The batch splits the simulations into two groups (alternate members)
 * whose passes overlap, each on a stream the batch creates.
 * sim_batch_advance first waits for
 * the work already on each simulation's streams and returns with all of the
 * batch's work complete.  Returns SIM_EINVAL on bad arguments, SIM_ENOMEM
 * if the batch's buffers do not fit, SIM_EDEVICE if its stream or events
 * cannot be created. */
#define SIM_BATCH_MAX 4096
typedef struct sim_batch sim_batch_t;
sim_status sim_batch_create(sim_t* const* sims, int n, sim_batch_t** out);

/* Advance simulation i to t_end[i] (host array of n) in `mode`, at most
 * max_cycles cycles or steps each when max_cycles > 0.  stats[i] and
 * status[i] (nullable host arrays of n) receive what sim_advance would
 * return for simulation i.  Returns SIM_OK when every simulation succeeded,
 * else the first failing simulation's status (sim_last_error names it);
 * a failing simulation stops, the others go on. */
sim_status sim_batch_advance(sim_batch_t* b, const double* t_end, int mode, int64_t max_cycles, sim_stats* stats,
                             sim_status* status);

/* Totals since creation: passes (one per host decision point: each ends
 * with one synchronisation), fused launches issued,
 * and launch records they carried (each a launch that the simulations would
 * have issued on their own). */
sim_status sim_batch_info(sim_batch_t* b, int64_t* passes, int64_t* fused_launches, int64_t* records);
void sim_batch_destroy(sim_batch_t* b);

void sim_destroy(sim_t* s);
const char* sim_strerror(sim_status st);
const char* sim_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
