// sharp_internal.h -- host-side simulation object shared by the engine
// (sharp_kernels.hip) and the C ABI (sharp_capi.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "../../include/sharp.h"
#include "sharp_device.h"

// grid bound of the bulk-tile stage kernels: below the tile count it leaves
// room on the chip for the band kernels that run beside them
#ifndef SHARP_BULK_BLOCKS
#define SHARP_BULK_BLOCKS 2048
#endif

namespace sharp {

// layout of the reduction block (64-bit words): reductions at 0..7, the
// device-planned sub-step (doubles) from word RED_SCHED, the list counts
// (16 ints) from word RED_COUNTS; each group on its own cache line
constexpr int RED_SCHED = 16;
constexpr int RED_COUNTS = 32;
constexpr int RED_WORDS = RED_COUNTS + 8;

// Recording of one simulation's launches for a batch (sharp_batch.hip).
// While a Sim has a recorder, the engine enqueues nothing: each launch is
// appended here (kernel, block size, grid, argument record) and the batch
// driver issues the launches of all its simulations as fused launches, in
// each simulation's order.  A readback of the reduction block becomes a
// recorded copy into the batch's readback slot, and waiting for it hands
// control back to the driver (yield), which resumes the simulation once the
// slot has reached s.h_red.
struct FusedOp {
    const void* fn;    // fused kernel (one per kernel body and argument list)
    int block;         // threads per block
    int nblk;          // blocks of this simulation's share
    size_t off, size;  // argument record in Recorder::args (its first int is the device-view index)
};
struct Recorder {
    std::vector<FusedOp> ops;
    std::vector<unsigned char> args;
    std::vector<Dev> devs;        // device views the records refer to (index local to this simulation)
    unsigned long long* slot = nullptr;   // device readback slot of this simulation (RED_WORDS words)
    bool rb_pending = false;
    sim_status status = SIM_OK;   // of the driver's last pass, returned by the wait
    void (*yield)(void*) = nullptr;
    void* yield_arg = nullptr;
    int dev_index(const Dev& d)
    {
        if (devs.empty() || std::memcmp(&devs.back(), &d, sizeof(Dev)) != 0) devs.push_back(d);
        return (int)devs.size() - 1;
    }
    void add(const void* fn, int block, int nblk, const void* rec, size_t size)
    {
        size_t off = (args.size() + 15) & ~(size_t)15;
        args.resize(off + size);
        std::memcpy(args.data() + off, rec, size);
        ops.push_back({fn, block, nblk, off, size});
    }
    void clear()
    {
        ops.clear();
        args.clear();
        devs.clear();
    }
};

// Where a replayed single-dt step copies what its stages saw (the adjoint's
// recomputation of a segment): one record per stage, each holding, at the
// offsets below (doubles), the stage inputs of both fluids, their
// primitives after the extension, the interface solution, the geometry and
// the level set the stage's interaction used, the volume fraction and level
// set after the stage's level-set update (those of its mixing), and the
// band mask of the step (bytes).
struct StageRec {
    double* base = nullptr;   // first record
    size_t stride = 0;        // doubles per record
    int next = 0;             // record the next stage fills
    size_t in[2], W[2], ps, us, al, ap, phi, aln, phin, M;
    void layout(int D, size_t nc, size_t nfc)
    {
        const size_t nv = (size_t)(D + 2) * nc;
        in[0] = 0;
        in[1] = nv;
        W[0] = 2 * nv;
        W[1] = 3 * nv;
        ps = 4 * nv;
        us = ps + nc;
        al = us + nc;
        ap = al + nc;   // D padded face arrays
        phi = ap + (size_t)D * nfc;
        aln = phi + nc;
        phin = aln + nc;
        M = phin + nc;
        stride = M + (nc + 7) / 8;
    }
};

struct Sim {
    Dev g;                 // device view (pointers live in device memory)
    Recorder* rec = nullptr;   // set while a batch advances this simulation
    sim_opts o;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = -1;       // device current at sim_create (the simulation's device)
    // bulk-tile stages run on one side stream per fluid, ordered against the
    // band work on `stream` by events (none when o.serial is set)
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t ev_band[2] = {nullptr, nullptr};   // on stream: latest band stage of fluid k
    hipEvent_t ev_bulk[2] = {nullptr, nullptr};   // on side[k]: latest bulk stage of fluid k
    bool band_rec[2] = {false, false};
    bool bulk_pending[2] = {false, false};        // stream has not yet waited for side[k]
    // second geometry buffer set: a new geometry is written there while
    // kernels (and other blocks of the writing kernel) read the current one
    double* alpha_alt = nullptr;
    double* ap_alt[3] = {nullptr, nullptr, nullptr};
    double* tphimin_alt = nullptr;     // per-tile |phi| minima of the geometry being built
    // level-set stream: a stage's level-set chain (velocity extension,
    // advection, reinitialisation, geometry) beside its band stage
    hipStream_t ls_stream = nullptr;
    hipEvent_t ev_ls_go = nullptr;     // on stream: the interaction the chain starts from
    hipEvent_t ev_ls_done = nullptr;   // on ls_stream: end of the chain
    bool ls_pending = false;           // stream has not yet waited for ev_ls_done
    // the velocity extension of the last interaction, left to the level-set
    // chain that follows it (run there, beside the band stage)
    std::vector<double> dt_log;        // CFL steps taken (sim_schedule)
    std::vector<double> dt_replay;     // prescribed CFL steps (opts.dt_replay)
    size_t replay_pos = 0;
    bool vel_deferred = false;
    const double* vel_cur = nullptr;   // the level set that interaction saw
    int max_blocks = 2048; // grid-stride bound for tile-list kernels
    int bulk_blocks = SHARP_BULK_BLOCKS;  // the same bound for the bulk-tile stages
    // autotuner of the bulk stage's launch and of the schedule (o.autotune):
    // candidate being timed (-1: the warm-up cycle), wall seconds per
    // cell-update of each candidate; candidates 0-3 overlap the bulk stages
    // on the side streams with grid bounds 1024-8192, candidate 4 issues
    // every kernel on the simulation's stream (bound 2048)
    static constexpr int NTUNE = 5;
    int tune_cur = -2;                    // -2: not started, NTUNE: done
    double tune_cost[NTUNE] = {0, 0, 0, 0, 0};
    bool run_serial = false;              // the schedule in use: no side streams
    double tune_t0 = 0.0;
    long long tune_cells0 = 0;
    bool tune_open = false;
    bool has_state = false;
    double t = 0.0;
    int wcur = 0;          // Jacobi buffer holding the latest primitives
    int vcur = 0;          // Jacobi buffer holding the latest level-set velocity
    unsigned long long* h_red = nullptr;  // pinned readback of the reduction block
    hipEvent_t ev_rb = nullptr;           // readback of a device-planned sub-step
    std::vector<void*> dev_allocs;
    // kernel timing of the bulk stage kernel
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<long long> prof_cells;    // cells of each pending timed launch (negative: first stage)
    double prof_ms = 0.0;
    long long prof_launches = 0, prof_cell_stages = 0, prof_first_stages = 0;
    long long bulk_cells[2] = {0, 0};   // cells in the bulk lists (host copy)
    int lcount[NLISTS] = {1, 1, 1, 1, 1, 1};   // tiles per list (host copy, sizes the grids)
    // tape of the adjoint (o.tape): single-dt steps
    int tape_fluid = -1;                // the fluid holding every cell, 2 with an interface; -1: not differentiable
    std::string tape_why;               // why this run cannot be differentiated
    std::vector<double> tape_dt;        // length of each taped step
    // state before steps 0, K, 2K, ... (K = o.ckpt_every): the contents of
    // tape_fluid, or (tape_fluid = 2) of both fluids, the level set, and the
    // results of the step-start interaction: both fluids' primitives after
    // the extension (whose ghost values the next extension starts from) and
    // the interface solution p*, u* (p* starts the next Riemann iterations)
    std::vector<double*> tape_ckpt;
    double* tape_prim0 = nullptr;       // primitives given to sim_set_state (tape_fluid, or both)
    std::vector<double*> tape_ls;       // tape_fluid = 2: per step or fast sub-step, the level set after each stage
    // tape_fluid = 2: every single-dt step and accelerated cycle, in order
    // (checkpoints every ckpt_every of them); a cycle lists its slow fluid,
    // length and fast sub-steps
    struct TapeSub { double dl; int hh, fin; };
    struct TapeUnit {
        int cycle = 0;          // 0: a single-dt step of length t1
        int S = 0;
        double t1 = 0.0;
        size_t ls_block = 0;    // index of its first tape_ls block
        std::vector<TapeSub> sub;
    };
    std::vector<TapeUnit> tape_units;
    // level-set replay: the stages of single-dt steps take these level sets
    // (device arrays of cells values, in stage order) instead of their own
    // advection and reinitialisation, which fixes every stage's geometry
    std::vector<const double*> ls_src;
    size_t ls_pos = 0;
    double* ls_rep = nullptr;           // device copy of opts.ls_replay
    size_t n_ls_rep = 0;                // its level sets
    StageRec* stage_rec = nullptr;      // set while the adjoint replays a step
    // single-dt steps of the fixed length o.dt_fixed captured in HIP graphs
    // (o.graph): one graph per launch configuration, i.e. per value of the
    // host state the step's launches are made from (`key`); `after` holds
    // the host state the step leaves, restored after each replay
    struct StepGraph {
        std::vector<unsigned char> key, after;
        hipGraphExec_t exec = nullptr;
        double adv = 0.0;              // time one replay advances
        long long steps[2] = {0, 0};   // steps of each fluid in one replay (a cycle's)
        double last_n = 1.0;           // the cycle's time-step ratio
    };
    static constexpr size_t MAX_GRAPHS = 4;
    std::vector<StepGraph> graphs;      // oldest first
    hipStream_t cap_stream = nullptr;   // library-owned stream the captures run on
    bool capturing = false;             // grids are sized for a capture (see Engine::grid)
    long long graph_captures = 0, graph_replays = 0;
    // Rollback (unless o.no_rollback): at every cycle start the contents and
    // the level set are copied on snap_stream (beside the cycle's first
    // stages, which write only stage buffers) and the boundary ledger on
    // the stream; every kernel that writes X or phiP waits for ev_snap first.
    // A non-physical state restores the copies and the time.
    double* snapX[2] = {nullptr, nullptr};
    double* snapPhi = nullptr;
    double* snapBacc[2] = {nullptr, nullptr};
    hipStream_t snap_stream = nullptr;
    hipEvent_t ev_cs = nullptr, ev_snap = nullptr;
    bool snap_valid = false;            // the copies hold the start of the current cycle
    bool snap_pending = false;          // writers of X / phiP must still wait for ev_snap
    bool snap_waited[3] = {false, false, false};   // stream, side[0], side[1] have waited
    double snap_t = 0.0;
    sim_stats snap_stats;               // the call's statistics at that cycle start
    long long rollbacks = 0;
};

void set_error(const char* fmt, ...);

// engine entry points (sharp_kernels.hip)
sim_status engine_set_state(Sim& s, const double* phi_dev, const double* prim_dev);
sim_status engine_advance(Sim& s, double t_end, int mode, long long max_cycles, sim_stats* st);
sim_status engine_bflux(Sim& s, double out[2][5]);
// one bulk-tile stage of fluid k on the simulation stream (the forward
// recomputation of the adjoint): out = a*base + (1-a)*(in + dt*L(in))
void engine_bulk_stage(Sim& s, int k, const double* in, const double* base, double* out, double a, double dt);
// the adjoint's recomputation with an interface: the state set to the
// contents X0, X1 and level set phi (device), geometry and tile lists
// rebuilt from phi; then single-dt steps of length dt, every kernel on the
// simulation's stream, their stage level sets taken from s.ls_src and
// their stages copied to *rec (`prepared`: the step-start interaction's
// results are in place already, so the step starts with its stages)
sim_status engine_restore(Sim& s, const double* X0, const double* X1, const double* phi);
sim_status engine_replay_step(Sim& s, double dt, StageRec* rec, bool prepared);
// conservation ledger (sharp_ledger.hip): out10[k*5 + q] = sum_c dV cons[k][q][c], zero for q >= NV
sim_status engine_totals(Sim& s, double* out10);
// the same through the device's file-scope scratch array (sharp_ledger.hip):
// ledger_scratch_attach looks up its address once per device
sim_status ledger_scratch_attach(int device);
sim_status engine_totals_noalloc(Sim& s, double* out10, int on_device);
// adjoint (sharp_adjoint.hip)
void tape_clear(Sim& s);
sim_status tape_begin(Sim& s, const double* prim_dev);
sim_status tape_step(Sim& s, double dt);
// an accelerated cycle (slow fluid S, length t1) starts / one of its fast
// sub-steps starts (its length and flags are set once known)
sim_status tape_cycle(Sim& s, int S, double t1);
sim_status tape_sub(Sim& s);
// the composed forward of the adjoint's recomputation: one engine
// operation each, every kernel on the simulation's stream
sim_status engine_op_prepare(Sim& s);
void engine_op_interaction(Sim& s, const double* in0, const double* in1, const double* cur);
void engine_op_stage(Sim& s, int k, const double* in, const double* base, double* out, double a, double dt);
const double* engine_op_ls(Sim& s, int q, bool last, double a, double dt, const double* phin);
void engine_op_mix(Sim& s, int k, double* buf, const double* cur);
void engine_op_mask(Sim& s);
void engine_op_geom(Sim& s, const double* phi);
void engine_op_corr_add(Sim& s, double w, int S);
void engine_op_corr_apply(Sim& s, int S);
void engine_op_axpby(Sim& s, double a1, const double* x, double a2, const double* y, double* dst);
sim_status engine_backward(Sim& s, const double* g_cons, double* g_prim0, double* g_eos);

// reduction word holding the lowest (cell << 1 | fluid) code of a cell found
// non-physical (all ones when none)
constexpr int RED_CELL = 8;

#define SHARP_HIP(call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::sharp::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                               __FILE__, __LINE__);                                  \
            return SIM_EDEVICE;                                                      \
        }                                                                            \
    } while (0)

}  // namespace sharp

// the C ABI's handle (include/sharp.h)
struct sim {
    sharp::Sim s;
};
