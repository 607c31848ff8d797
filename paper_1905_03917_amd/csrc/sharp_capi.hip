// sharp_capi.hip -- C ABI of the gfx950 sharp-interface library (include/sharp.h):
// argument checking, device allocation, host/device staging.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "sharp_internal.h"

namespace sharp {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

template <typename T>
static sim_status dalloc(Sim& s, T** p, size_t n)
{
    void* q = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed", n * sizeof(T));
        return SIM_ENOMEM;
    }
    s.dev_allocs.push_back(q);
    if (hipMemsetAsync(q, 0, n * sizeof(T), s.stream) != hipSuccess) {
        set_error("hipMemsetAsync failed");
        return SIM_EDEVICE;
    }
    *p = static_cast<T*>(q);
    return SIM_OK;
}

static void release(Sim& s)
{
    tape_clear(s);
    for (auto& sg : s.graphs)
        if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
    s.graphs.clear();
    if (s.cap_stream) (void)hipStreamDestroy(s.cap_stream);
    s.cap_stream = nullptr;
    if (s.snap_stream) (void)hipStreamDestroy(s.snap_stream);
    if (s.ev_cs) (void)hipEventDestroy(s.ev_cs);
    if (s.ev_snap) (void)hipEventDestroy(s.ev_snap);
    s.snap_stream = nullptr;
    s.ev_cs = s.ev_snap = nullptr;
    for (void* p : s.dev_allocs) (void)hipFree(p);
    s.dev_allocs.clear();
    for (hipEvent_t e : s.ev_pool) (void)hipEventDestroy(e);
    s.ev_pool.clear();
    if (s.h_red) (void)hipHostFree(s.h_red);
    s.h_red = nullptr;
    if (s.ev_rb) (void)hipEventDestroy(s.ev_rb);
    s.ev_rb = nullptr;
    if (s.ls_stream) (void)hipStreamDestroy(s.ls_stream);
    if (s.ev_ls_go) (void)hipEventDestroy(s.ev_ls_go);
    if (s.ev_ls_done) (void)hipEventDestroy(s.ev_ls_done);
    s.ls_stream = nullptr;
    s.ev_ls_go = s.ev_ls_done = nullptr;
    for (int k = 0; k < 2; k++) {
        if (s.side[k]) (void)hipStreamDestroy(s.side[k]);
        if (s.ev_band[k]) (void)hipEventDestroy(s.ev_band[k]);
        if (s.ev_bulk[k]) (void)hipEventDestroy(s.ev_bulk[k]);
        s.side[k] = nullptr;
        s.ev_band[k] = s.ev_bulk[k] = nullptr;
    }
    if (s.own_stream && s.stream) (void)hipStreamDestroy(s.stream);
    s.stream = nullptr;
}

}  // namespace sharp

using namespace sharp;

extern "C" {

void sim_default_opts(sim_opts* o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->cfl = 0.6;
    o->rk = 3;
    o->n_thr = 0.7;
    o->alpha_mix = 0.5;
    o->ls_band = 8.0;
    o->ext_band = 5.0;
    o->mix_band = 3.0;
    o->ext_iters = 8;
    o->reinit_iters = 2;
    o->weno_eps = 1e-6;
    o->ckpt_every = 20;
}

const char* sim_strerror(sim_status st)
{
    switch (st) {
    case SIM_OK: return "ok";
    case SIM_EINVAL: return "invalid argument";
    case SIM_ENOMEM: return "out of device memory";
    case SIM_EDEVICE: return "device error";
    case SIM_ENONPHYS: return "non-physical state";
    case SIM_ESTATE: return "invalid call order";
    }
    return "unknown status";
}

const char* sim_last_error(void) { return g_err; }

sim_status sim_create(const sim_grid* grid, const sim_eos eos[2], const sim_opts* opts, void* stream, sim_t** out)
{
    if (!grid || !eos || !out) { set_error("null argument"); return SIM_EINVAL; }
    *out = nullptr;
    int D = grid->ndim;
    if (D < 1 || D > 3) { set_error("ndim must be 1, 2 or 3"); return SIM_EINVAL; }
    if (!(grid->h > 0.0) || !std::isfinite(grid->h)) { set_error("h must be positive"); return SIM_EINVAL; }
    long long nc = 1;
    for (int d = 0; d < 3; d++) {
        long long n = d < D ? grid->n[d] : 1;
        if (n < 1 || (d >= D && grid->n[d] != 1 && grid->n[d] != 0)) { set_error("bad cell count in direction %d", d); return SIM_EINVAL; }
        if (d < D && grid->bc[d] != 0 && grid->bc[d] != 1) { set_error("bc must be 0 or 1"); return SIM_EINVAL; }
        if (d < D && grid->bc[d] == 1 && n < 6) { set_error("periodic direction needs >= 6 cells"); return SIM_EINVAL; }
        nc *= n;
    }
    if (nc * 5 >= (1ll << 31)) { set_error("grid too large for 32-bit cell indexing"); return SIM_EINVAL; }
    for (int k = 0; k < 2; k++)
        if (!(eos[k].gamma > 1.0) || !std::isfinite(eos[k].pinf)) { set_error("eos %d: need gamma > 1 and a finite p_inf", k); return SIM_EINVAL; }
    sim_opts o;
    if (opts) o = *opts; else sim_default_opts(&o);
    if (o.rk != 2 && o.rk != 3) { set_error("rk must be 2 or 3"); return SIM_EINVAL; }
    if (!(o.cfl > 0.0) || o.ext_iters < 0 || o.reinit_iters < 0) { set_error("invalid options"); return SIM_EINVAL; }
    if (o.tape && o.ckpt_every < 1) { set_error("ckpt_every must be >= 1"); return SIM_EINVAL; }
    if (!std::isfinite(o.sigma)) { set_error("sigma must be finite"); return SIM_EINVAL; }
    {
        const double* f = o.dt_fixed_fluid;
        const bool none = f[0] == 0.0 && f[1] == 0.0;
        const bool both = f[0] > 0.0 && f[1] > 0.0 && std::isfinite(f[0]) && std::isfinite(f[1]);
        if (!none && !both) { set_error("dt_fixed_fluid: both 0 or both positive and finite"); return SIM_EINVAL; }
        if (both && (o.tape || o.n_dt_replay > 0)) { set_error("dt_fixed_fluid together with tape or dt_replay"); return SIM_EINVAL; }
    }
    if (!(o.dt_fixed >= 0.0) || !std::isfinite(o.dt_fixed)) { set_error("dt_fixed must be >= 0"); return SIM_EINVAL; }
    if (o.graph < 0 || o.graph > 2) { set_error("graph must be 0, 1 or 2 (got %d)", o.graph); return SIM_EINVAL; }
    if (o.graph && !(o.dt_fixed > 0.0) && !(o.dt_fixed_fluid[0] > 0.0)) {
        set_error("graph needs dt_fixed > 0 or dt_fixed_fluid");
        return SIM_EINVAL;
    }
    if (o.grid_cap < 0) { set_error("grid_cap must be >= 0"); return SIM_EINVAL; }
    if (o.n_dt_replay < 0 || (o.n_dt_replay > 0 && !o.dt_replay)) {
        set_error("dt_replay needs n_dt_replay >= 0 values");
        return SIM_EINVAL;
    }
    for (int64_t i = 0; i < o.n_dt_replay; i++)
        if (!(o.dt_replay[i] > 0.0)) {   // +inf: a fluid that holds no cell
            set_error("dt_replay[%lld] = %g is not a positive step", (long long)i, o.dt_replay[i]);
            return SIM_EINVAL;
        }
    if (o.n_ls_replay < 0 || (o.n_ls_replay > 0 && !o.ls_replay) || o.n_ls_replay % nc != 0) {
        set_error("ls_replay needs a whole number of level sets (%lld values each)", nc);
        return SIM_EINVAL;
    }
    if (o.n_ls_replay > 0 && o.tape) {
        set_error("a run that replays level sets cannot record a tape");
        return SIM_EINVAL;
    }

    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) { set_error("hipGetDevice failed"); return SIM_EDEVICE; }
    {
        sim_status r = ledger_scratch_attach(device);
        if (r != SIM_OK) return r;
    }
    sim_t* h = new sim_t();
    Sim& s = h->s;
    s.o = o;
    s.device = device;
    if (o.n_dt_replay > 0) s.dt_replay.assign(o.dt_replay, o.dt_replay + o.n_dt_replay);
    s.o.dt_replay = nullptr;   // the copy is used; the caller's buffer need not outlive the call
    s.o.ls_replay = nullptr;   // copied to the device below
    // 3-D bulk lists are long (the slow fluid fills most of the grid): a
    // larger grid bound measured faster there (the autotuner's choice at 256^3)
    if (D == 3) s.bulk_blocks = 4 * SHARP_BULK_BLOCKS;
    if (stream) {
        s.stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreate(&s.stream) != hipSuccess) { delete h; set_error("hipStreamCreate failed"); return SIM_EDEVICE; }
        s.own_stream = true;
    }
    if (!o.serial) {
        bool ok = true;
        for (int k = 0; k < 2 && ok; k++)
            ok = hipStreamCreateWithFlags(&s.side[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&s.ev_band[k], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&s.ev_bulk[k], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            release(s);
            delete h;
            set_error("stream/event creation failed");
            return SIM_EDEVICE;
        }
    }
    Dev& g = s.g;
    memset(&g, 0, sizeof g);
    g.D = D;
    const int TT[3][3] = {{256, 1, 1}, {16, 16, 1}, {8, 8, 4}};
    g.nc = 1;
    g.nfc = 1;
    g.ntiles = 1;
    for (int d = 0; d < 3; d++) {
        g.n[d] = d < D ? (int)grid->n[d] : 1;
        g.nf[d] = d < D ? g.n[d] + 1 : 1;
        g.bc[d] = d < D ? grid->bc[d] : 0;
        g.T[d] = TT[D - 1][d];
        g.nt[d] = (g.n[d] + g.T[d] - 1) / g.T[d];
        g.nc *= g.n[d];
        g.nfc *= g.nf[d];
        g.ntiles *= g.nt[d];
    }
    g.h = grid->h;
    for (int k = 0; k < 2; k++) { g.gam[k] = eos[k].gamma; g.pinf[k] = eos[k].pinf; }
    g.amix = o.alpha_mix;
    g.lsb = o.ls_band;
    g.extb = o.ext_band;
    g.mixb = o.mix_band;
    g.eps = o.weno_eps;
    g.sigma = o.sigma;
    // boundary faces: two sides per direction, product of the other extents
    int off = 0;
    for (int d = 0; d < 3; d++) {
        int other = 1;
        for (int e = 0; e < 3; e++)
            if (e != d) other *= g.n[e];
        for (int sd = 0; sd < 2; sd++) {
            g.bface_off[d][sd] = off;
            if (d < D) off += other;
        }
    }
    g.nbface = off;

    int NV = D + 2;
    size_t nv = (size_t)NV * g.nc;
    sim_status rc = SIM_OK;
#define A(ptr, n) if (rc == SIM_OK) rc = dalloc(s, &(ptr), (n))
    for (int k = 0; k < 2; k++) {
        A(g.X[k], nv); A(g.Y[k], nv); A(g.Z[k], nv);
        A(g.Wb[k][0], nv); A(g.Wb[k][1], nv);
        A(g.ss[k], (size_t)g.nc);
        A(g.bacc[k], (size_t)NV * (g.nbface > 0 ? g.nbface : 1));
    }
    A(g.T2, nv); A(g.Fh, nv); A(g.corr, nv); A(g.dmix, nv);
    A(g.Tm[0], nv); A(g.Tm[1], nv);
    A(g.phiP, (size_t)g.nc);
    for (int b = 0; b < 3; b++) A(g.phiB[b], (size_t)g.nc);
    A(g.phiH, (size_t)g.nc);
    A(g.alpha, (size_t)g.nc);
    for (int d = 0; d < 3; d++) A(g.ap[d], d < D ? (size_t)g.nfc : 1);
    A(s.alpha_alt, (size_t)g.nc);
    for (int d = 0; d < 3; d++) A(s.ap_alt[d], d < D ? (size_t)g.nfc : 1);
    A(g.ps, (size_t)g.nc); A(g.us, (size_t)g.nc);
    // a point interface (1-D) has no curvature: no jump to keep
    if (o.sigma != 0.0 && D > 1) A(g.pj, (size_t)g.nc);
    for (int b = 0; b < 2; b++)
        for (int d = 0; d < 3; d++) A(g.v[b][d], d < D ? (size_t)g.nc : 1);
    A(g.M, (size_t)g.nc); A(g.nearif, (size_t)g.nc);
    A(g.tcore, (size_t)g.ntiles); A(g.tflag, (size_t)g.ntiles); A(g.tsign, (size_t)g.ntiles);
    A(g.tphimin, (size_t)g.ntiles); A(s.tphimin_alt, (size_t)g.ntiles);
    A(g.lists, (size_t)NLISTS * g.ntiles);
    // extension stencil lists (3-D): a cell is a target of the primitive
    // extension at most once per fluid and of the velocity extension once
    g.wl_cap = D == 3 ? 4 * g.ntiles * 128 : 0;   // 64 cells x 2 fluids per wave
    g.vl_cap = D == 3 ? 4 * g.ntiles * 64 : 0;
    A(g.wl_n, D == 3 ? (size_t)4 * g.ntiles : 1); A(g.vl_n, D == 3 ? (size_t)4 * g.ntiles : 1);
    A(g.wl_c, (size_t)g.wl_cap); A(g.wl_up, (size_t)3 * g.wl_cap); A(g.wl_w, (size_t)4 * g.wl_cap);
    A(g.vl_c, (size_t)g.vl_cap); A(g.vl_up, (size_t)3 * g.vl_cap); A(g.vl_w, (size_t)4 * g.vl_cap);
    // reductions (8 words) and list counts (16 ints) share one block, read
    // back with one copy; the counts, read by every grid-stride loop, sit
    // 256 bytes away from the words the reductions update atomically
    A(g.red, RED_WORDS);
    if (o.n_ls_replay > 0) {
        A(s.ls_rep, (size_t)o.n_ls_replay);
        s.n_ls_rep = (size_t)(o.n_ls_replay / nc);
    }
    if (!o.no_rollback) {
        for (int k = 0; k < 2; k++) {
            A(s.snapX[k], nv);
            A(s.snapBacc[k], (size_t)NV * (g.nbface > 0 ? g.nbface : 1));
        }
        A(s.snapPhi, (size_t)g.nc);
        if (rc == SIM_OK && (hipStreamCreateWithFlags(&s.snap_stream, hipStreamNonBlocking) != hipSuccess ||
                             hipEventCreateWithFlags(&s.ev_cs, hipEventDisableTiming) != hipSuccess ||
                             hipEventCreateWithFlags(&s.ev_snap, hipEventDisableTiming) != hipSuccess)) {
            set_error("snapshot stream/event creation failed");
            rc = SIM_EDEVICE;
        }
    }
    if (rc == SIM_OK) {
        g.counts = reinterpret_cast<int*>(g.red + RED_COUNTS);
        g.sched = reinterpret_cast<double*>(g.red + RED_SCHED);
        g.use_sched = 0;
    }
    if (rc == SIM_OK && hipEventCreateWithFlags(&s.ev_rb, hipEventDisableTiming) != hipSuccess) {
        set_error("event creation failed");
        rc = SIM_EDEVICE;
    }
#undef A
    if (rc == SIM_OK) {
        std::vector<int> all(g.ntiles);
        for (int t = 0; t < g.ntiles; t++) all[t] = t;
        int cnt[16] = {0};
        cnt[LIST_ALL] = g.ntiles;
        if (hipMemcpyAsync(g.lists + (size_t)LIST_ALL * g.ntiles, all.data(), sizeof(int) * g.ntiles,
                           hipMemcpyHostToDevice, s.stream) != hipSuccess ||
            hipMemcpyAsync(g.counts, cnt, sizeof cnt, hipMemcpyHostToDevice, s.stream) != hipSuccess ||
            (s.ls_rep && hipMemcpyAsync(s.ls_rep, o.ls_replay, sizeof(double) * (size_t)o.n_ls_replay,
                                        hipMemcpyHostToDevice, s.stream) != hipSuccess) ||
            hipStreamSynchronize(s.stream) != hipSuccess) {
            set_error("initial upload failed");
            rc = SIM_EDEVICE;
        }
    }
    if (rc == SIM_OK && hipHostMalloc((void**)&s.h_red, RED_WORDS * sizeof(unsigned long long)) != hipSuccess) {
        set_error("pinned host allocation failed");
        rc = SIM_ENOMEM;
    }
    if (rc != SIM_OK) {
        release(s);
        delete h;
        return rc;
    }
    *out = h;
    return SIM_OK;
}

void sim_destroy(sim_t* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->s.stream);
    for (int k = 0; k < 2; k++)
        if (h->s.side[k]) (void)hipStreamSynchronize(h->s.side[k]);
    if (h->s.snap_stream) (void)hipStreamSynchronize(h->s.snap_stream);
    if (h->s.ls_stream) (void)hipStreamSynchronize(h->s.ls_stream);
    release(h->s);
    delete h;
}

static sim_status stage_in(Sim& s, const double* src, size_t n, int on_device, double** tmp)
{
    *tmp = nullptr;
    if (on_device) return SIM_OK;
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) { (void)hipGetLastError(); set_error("staging allocation failed"); return SIM_ENOMEM; }
    if (hipMemcpyAsync(p, src, n * sizeof(double), hipMemcpyHostToDevice, s.stream) != hipSuccess) {
        (void)hipFree(p);
        set_error("host-to-device copy failed");
        return SIM_EDEVICE;
    }
    *tmp = (double*)p;
    return SIM_OK;
}

sim_status sim_set_state(sim_t* h, const double* phi, const double* prim, int on_device)
{
    if (!h || !phi || !prim) { set_error("null argument"); return SIM_EINVAL; }
    Sim& s = h->s;
    int NV = s.g.D + 2;
    double *tphi = nullptr, *tprim = nullptr;
    sim_status rc = stage_in(s, phi, s.g.nc, on_device, &tphi);
    if (rc == SIM_OK) rc = stage_in(s, prim, (size_t)2 * NV * s.g.nc, on_device, &tprim);
    if (rc == SIM_OK) rc = engine_set_state(s, tphi ? tphi : phi, tprim ? tprim : prim);
    (void)hipStreamSynchronize(s.stream);
    if (tphi) (void)hipFree(tphi);
    if (tprim) (void)hipFree(tprim);
    return rc;
}

sim_status sim_advance(sim_t* h, double t_end, int mode, int64_t max_cycles, sim_stats* out)
{
    if (!h) { set_error("null handle"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (!s.has_state) { set_error("sim_set_state has not been called"); return SIM_ESTATE; }
    if (mode != SIM_SINGLE_DT && mode != SIM_MULTI_DT) { set_error("bad mode"); return SIM_EINVAL; }
    if (!std::isfinite(t_end)) { set_error("t_end must be finite"); return SIM_EINVAL; }
    sim_stats st;
    memset(&st, 0, sizeof st);
    sim_status rc = engine_advance(s, t_end, mode, (long long)max_cycles, &st);
    if (rc == SIM_OK) {
        rc = engine_bflux(s, st.bflux);
    } else if (rc == SIM_ENONPHYS && s.snap_valid) {
        // the rolled-back ledger; the failure's message is kept
        std::string msg = sim_last_error();
        if (engine_bflux(s, st.bflux) != SIM_OK) memset(st.bflux, 0, sizeof st.bflux);
        set_error("%s", msg.c_str());
    }
    if (out) *out = st;
    return rc;
}

sim_status sim_backward(sim_t* h, const double* g_cons, double* g_prim0, double* g_eos, int on_device)
{
    if (!h || !g_cons || !g_prim0) { set_error("null argument"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (!s.o.tape || !s.has_state) { set_error("no tape: create with opts.tape = 1, then set_state and advance"); return SIM_ESTATE; }
    if (s.tape_fluid < 0) { set_error("%s", s.tape_why.c_str()); return SIM_EINVAL; }
    size_t n = (size_t)2 * (s.g.D + 2) * s.g.nc;
    double *tg = nullptr, *tp = nullptr;
    sim_status rc = stage_in(s, g_cons, n, on_device, &tg);
    if (rc == SIM_OK && !on_device) {
        if (hipMalloc((void**)&tp, n * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("staging allocation failed");
            rc = SIM_ENOMEM;
        }
    }
    double eos[4] = {0.0, 0.0, 0.0, 0.0};
    if (rc == SIM_OK) rc = engine_backward(s, tg ? tg : g_cons, tp ? tp : g_prim0, eos);
    if (rc == SIM_OK && tp && hipMemcpyAsync(g_prim0, tp, n * sizeof(double), hipMemcpyDeviceToHost, s.stream) != hipSuccess) {
        set_error("device-to-host copy failed");
        rc = SIM_EDEVICE;
    }
    (void)hipStreamSynchronize(s.stream);
    if (tg) (void)hipFree(tg);
    if (tp) (void)hipFree(tp);
    if (rc == SIM_OK && g_eos)
        for (int i = 0; i < 4; i++) g_eos[i] = eos[i];
    return rc;
}

sim_status sim_get_state(sim_t* h, double* phi, double* cons, double* alpha, int on_device)
{
    if (!h) { set_error("null handle"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (!s.has_state) { set_error("no state"); return SIM_ESTATE; }
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    size_t nc = s.g.nc, nv = (size_t)(s.g.D + 2) * nc;
    SHARP_HIP(hipStreamSynchronize(s.stream));
    if (phi) SHARP_HIP(hipMemcpyAsync(phi, s.g.phiP, nc * sizeof(double), kind, s.stream));
    if (cons)
        for (int k = 0; k < 2; k++) SHARP_HIP(hipMemcpyAsync(cons + k * nv, s.g.X[k], nv * sizeof(double), kind, s.stream));
    if (alpha) SHARP_HIP(hipMemcpyAsync(alpha, s.g.alpha, nc * sizeof(double), kind, s.stream));
    SHARP_HIP(hipStreamSynchronize(s.stream));
    return SIM_OK;
}

sim_status sim_totals(sim_t* h, double* out10)
{
    if (!h || !out10) { set_error("null argument"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (!s.has_state) { set_error("no state"); return SIM_ESTATE; }
    return engine_totals(s, out10);
}

sim_status sim_totals_noalloc(sim_t* h, double* out10, int on_device)
{
    if (!h || !out10) { set_error("null argument"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (!s.has_state) { set_error("no state"); return SIM_ESTATE; }
    return engine_totals_noalloc(s, out10, on_device);
}

sim_status sim_tuned(sim_t* h, int* bulk_blocks, int* serial, int* done)
{
    if (!h) { set_error("null handle"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (bulk_blocks) *bulk_blocks = s.bulk_blocks;
    if (serial) *serial = (s.o.serial || s.run_serial) ? 1 : 0;
    if (done) *done = s.o.autotune ? (s.tune_cur >= Sim::NTUNE) : 1;
    return SIM_OK;
}

sim_status sim_schedule(sim_t* h, double* out, int64_t cap, int64_t* n)
{
    if (!h || cap < 0 || (cap > 0 && !out)) { set_error("bad arguments"); return SIM_EINVAL; }
    const std::vector<double>& v = h->s.dt_log;
    const int64_t m = (int64_t)v.size();
    for (int64_t i = 0; i < m && i < cap; i++) out[i] = v[(size_t)i];
    if (n) *n = m;
    return SIM_OK;
}

sim_status sim_levelset_tape(sim_t* h, double* out, int64_t cap, int64_t* n)
{
    if (!h || cap < 0 || (cap > 0 && !out)) { set_error("bad arguments"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (!s.o.tape || s.tape_fluid != 2) {
        set_error("no level-set tape: it is recorded by a taped run (opts.tape = 1) with an interface");
        return SIM_ESTATE;
    }
    const size_t per = (size_t)s.o.rk * s.g.nc;
    const int64_t m = (int64_t)(per * s.tape_ls.size());
    if (n) *n = m;
    for (size_t i = 0; i < s.tape_ls.size(); i++) {
        const int64_t o0 = (int64_t)(i * per);
        if (o0 >= cap) break;
        const size_t cnt = (size_t)std::min<int64_t>((int64_t)per, cap - o0);
        if (hipMemcpyAsync(out + o0, s.tape_ls[i], cnt * sizeof(double), hipMemcpyDeviceToHost, s.stream) != hipSuccess) {
            set_error("device-to-host copy failed");
            return SIM_EDEVICE;
        }
    }
    if (hipStreamSynchronize(s.stream) != hipSuccess) { set_error("stream synchronisation failed"); return SIM_EDEVICE; }
    return SIM_OK;
}

sim_status sim_graph_info(sim_t* h, long long* captures, long long* replays, int* held)
{
    if (!h) { set_error("null handle"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (captures) *captures = s.graph_captures;
    if (replays) *replays = s.graph_replays;
    if (held) *held = (int)s.graphs.size();
    return SIM_OK;
}

sim_status sim_profile(sim_t* h, int enable)
{
    if (!h) { set_error("null handle"); return SIM_EINVAL; }
    Sim& s = h->s;
    s.prof = enable != 0;
    if (s.prof && s.ev_pool.empty()) {
        s.ev_pool.resize(4096);
        for (auto& e : s.ev_pool) SHARP_HIP(hipEventCreate(&e));
    }
    s.prof_ms = 0.0;
    s.prof_launches = 0;
    s.prof_cell_stages = 0;
    s.prof_first_stages = 0;
    s.ev_used = 0;
    s.prof_cells.clear();
    return SIM_OK;
}

sim_status sim_profile_read(sim_t* h, double* ms, int64_t* launches, int64_t* cells, int64_t* first_cells)
{
    if (!h) { set_error("null handle"); return SIM_EINVAL; }
    Sim& s = h->s;
    if (ms) *ms = s.prof_ms;
    if (launches) *launches = s.prof_launches;
    if (cells) *cells = s.prof_cell_stages;
    if (first_cells) *first_cells = s.prof_first_stages;
    return SIM_OK;
}

}  // extern "C"
