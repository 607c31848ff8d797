// sharp_batch.hip -- batches of simulations advanced together (the
// batched form of the hot path: many independent instances of uneven sizes,
// each running the unchanged single-dt step or accelerated cycle of
// Sec. 3.1, with their launches fused across instances).
//
// Each simulation of a batch runs its engine in a coroutine of its own with
// a Recorder attached: the engine's launches become records, and a readback
// of its reduction block (the host decisions of the method: the CFL steps,
// the tile lists, the sub-step plan) becomes a recorded copy into a slot
// followed by a yield.  The driver resumes every unfinished simulation in
// turn until each has yielded or finished (a pass), then merges the
// recorded launches: it repeatedly takes the kernel that heads the most
// simulations' queues and issues one fused launch for all of them, so that
// each simulation's launches keep their order.  One upload carries the
// pass's device views and argument records, one copy brings every slot
// back, and an event marks the end of the pass.  The simulations form
// groups (two by default; alternate members) with a stream, staging buffers
// and slot range each: while the GPU runs one group's pass, the host resumes
// another group and records its next one.  The work a pass enqueues is what
// the simulations would have enqueued on their own, in the
// same order per simulation: the same steps, with states equal to those of
// separate runs up to round-off (a fused kernel is the same body compiled
// in another context, where the compiler may contract other multiply-adds).
#include <sys/mman.h>
#include <ucontext.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "sharp_internal.h"

namespace sharp {

struct BatchInst {
    Sim* s = nullptr;
    int slot = 0;                 // readback slot index
    Recorder rec;
    ucontext_t ctx;
    bool done = false;
    sim_status rc = SIM_OK;
    std::string err;
    sim_stats st;
    double t_end = 0.0;
    struct sim_batch_impl* b = nullptr;
};

static constexpr size_t CO_STACK = 1u << 20;   // per simulation (mapped lazily)
// groups of a batch (passes in flight at once); 3 measured the same as 2 on
// the 512-instance batch, 4 slower
#ifndef SHARP_BATCH_GROUPS
#define SHARP_BATCH_GROUPS 2
#endif

// a group of a batch's simulations: its members' passes run on its stream,
// in its buffers, and fill its range of readback slots
struct BatchGroup {
    std::vector<int> members;                // simulation indices, in order
    int slot0 = 0;                           // first readback slot (member m has slot0 + m)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev = nullptr;                 // end of the pass in flight
    bool pending = false;                    // a pass is in flight
    unsigned char* d_buf = nullptr;          // device views, record offsets and argument records of a pass
    unsigned char* h_buf = nullptr;          // pinned staging of d_buf
    size_t cap = 0;
    std::vector<unsigned char> stage;
};

struct sim_batch_impl {
    std::vector<BatchInst> in;
    std::vector<BatchGroup> grp;
    std::vector<void*> stacks;
    ucontext_t sched;
    int mode = 0;
    long long max_cycles = 0;
    unsigned long long* d_slots = nullptr;   // n * RED_WORDS readback slots
    unsigned long long* h_slots = nullptr;   // pinned copy of the slots
    long long passes = 0, fused = 0, recorded = 0;
};

static void co_entry(unsigned lo, unsigned hi)
{
    BatchInst* bi = reinterpret_cast<BatchInst*>(((uintptr_t)hi << 32) | (uintptr_t)lo);
    std::memset(&bi->st, 0, sizeof bi->st);
    bi->rc = engine_advance(*bi->s, bi->t_end, bi->b->mode, bi->b->max_cycles, &bi->st);
    if (bi->rc != SIM_OK) bi->err = sim_last_error();
    bi->done = true;
    // returning resumes the driver (uc_link)
}

static void co_yield(void* p)
{
    BatchInst* bi = static_cast<BatchInst*>(p);
    swapcontext(&bi->ctx, &bi->b->sched);
}

static size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

struct FusedLaunch {
    const void* fn;
    int block, grid, nrec;
    size_t pre_off, rec_off;
};

// merge and issue the recorded launches of group G's members, then the copy
// of its readback slots and the event that ends the pass
static sim_status pass_issue(sim_batch_impl& B, BatchGroup& G)
{
    const int n = (int)G.members.size();
    auto rec = [&](int m) -> Recorder& { return B.in[G.members[m]].rec; };
    std::vector<unsigned char>& H = G.stage;
    H.clear();
    std::vector<size_t> dbase(n);
    size_t ndev = 0;
    for (int m = 0; m < n; m++) {
        dbase[m] = ndev;
        ndev += rec(m).devs.size();
    }
    H.resize(ndev * sizeof(Dev));
    for (int m = 0; m < n; m++)
        if (!rec(m).devs.empty())
            std::memcpy(H.data() + dbase[m] * sizeof(Dev), rec(m).devs.data(), rec(m).devs.size() * sizeof(Dev));
    std::vector<size_t> cur(n, 0);
    std::vector<FusedLaunch> L;
    std::vector<std::pair<const void*, int>> heads;
    std::vector<int> members, pre;
    for (;;) {
        heads.clear();
        for (int m = 0; m < n; m++) {
            const Recorder& r = rec(m);
            if (cur[m] >= r.ops.size()) continue;
            const void* f = r.ops[cur[m]].fn;
            size_t h = 0;
            while (h < heads.size() && heads[h].first != f) h++;
            if (h == heads.size()) heads.push_back({f, 0});
            heads[h].second++;
        }
        if (heads.empty()) break;
        size_t best = 0;
        for (size_t h = 1; h < heads.size(); h++)
            if (heads[h].second > heads[best].second) best = h;
        const void* f = heads[best].first;
        members.clear();
        pre.clear();
        int grid = 0, block = 0;
        size_t rsize = 0;
        for (int m = 0; m < n; m++) {
            const Recorder& r = rec(m);
            if (cur[m] >= r.ops.size() || r.ops[cur[m]].fn != f) continue;
            const FusedOp& op = r.ops[cur[m]];
            if (members.empty()) { block = op.block; rsize = op.size; }
            if (op.block != block || op.size != rsize) { set_error("batch: inconsistent fused launch"); return SIM_EDEVICE; }
            int start = grid;
            if (op.nblk >= 8 && (op.nblk & 7) == 0) start = (grid + 7) & ~7;
            pre.push_back(start);
            grid = start + op.nblk;
            members.push_back(m);
        }
        FusedLaunch fl;
        fl.fn = f;
        fl.block = block;
        fl.grid = grid;
        fl.nrec = (int)members.size();
        fl.pre_off = align16(H.size());
        H.resize(fl.pre_off + pre.size() * sizeof(int));
        std::memcpy(H.data() + fl.pre_off, pre.data(), pre.size() * sizeof(int));
        fl.rec_off = align16(H.size());
        H.resize(fl.rec_off + members.size() * rsize);
        for (size_t q = 0; q < members.size(); q++) {
            const int m = members[q];
            const FusedOp& op = rec(m).ops[cur[m]];
            unsigned char* dst = H.data() + fl.rec_off + q * rsize;
            std::memcpy(dst, rec(m).args.data() + op.off, rsize);
            int dev;
            std::memcpy(&dev, dst, sizeof dev);
            dev += (int)dbase[m];
            std::memcpy(dst, &dev, sizeof dev);
            cur[m]++;
        }
        L.push_back(fl);
        B.recorded += fl.nrec;
    }
    if (!H.empty()) {
        if (H.size() > G.cap) {
            // the group's previous pass has completed: its buffers are free
            size_t c = H.size() * 2;
            if (G.d_buf) (void)hipFree(G.d_buf);
            if (G.h_buf) (void)hipHostFree(G.h_buf);
            G.d_buf = nullptr;
            G.h_buf = nullptr;
            G.cap = 0;
            SHARP_HIP(hipMalloc((void**)&G.d_buf, c));
            SHARP_HIP(hipHostMalloc((void**)&G.h_buf, c, hipHostMallocDefault));
            G.cap = c;
        }
        std::memcpy(G.h_buf, H.data(), H.size());
        SHARP_HIP(hipMemcpyAsync(G.d_buf, G.h_buf, H.size(), hipMemcpyHostToDevice, G.stream));
    }
    for (const FusedLaunch& fl : L) {
        const Dev* devs = reinterpret_cast<const Dev*>(G.d_buf);
        const void* recs = G.d_buf + fl.rec_off;
        const int* pre_d = reinterpret_cast<const int*>(G.d_buf + fl.pre_off);
        int nrec = fl.nrec;
        void* args[4] = {(void*)&devs, (void*)&recs, (void*)&pre_d, (void*)&nrec};
        SHARP_HIP(hipLaunchKernel(fl.fn, dim3(fl.grid), dim3(fl.block), args, 0, G.stream));
        B.fused++;
    }
    bool rb = false;
    for (int m = 0; m < n; m++) rb = rb || rec(m).rb_pending;
    if (rb)
        SHARP_HIP(hipMemcpyAsync(B.h_slots + (size_t)G.slot0 * RED_WORDS, B.d_slots + (size_t)G.slot0 * RED_WORDS,
                                 (size_t)n * RED_WORDS * sizeof(unsigned long long), hipMemcpyDeviceToHost, G.stream));
    SHARP_HIP(hipEventRecord(G.ev, G.stream));
    G.pending = true;
    B.passes++;
    return SIM_OK;
}

// wait for group G's pass and hand its readbacks to the simulations
static sim_status pass_complete(sim_batch_impl& B, BatchGroup& G)
{
    G.pending = false;
    SHARP_HIP(hipEventSynchronize(G.ev));
    for (int i : G.members) {
        Recorder& r = B.in[i].rec;
        if (r.rb_pending) {
            std::memcpy(B.in[i].s->h_red, B.h_slots + (size_t)B.in[i].slot * RED_WORDS,
                        RED_WORDS * sizeof(unsigned long long));
            r.rb_pending = false;
        }
        r.clear();
    }
    return SIM_OK;
}

static void batch_free(sim_batch_impl* B)
{
    if (!B) return;
    for (BatchGroup& G : B->grp) {
        if (G.stream) (void)hipStreamSynchronize(G.stream);
        if (G.d_buf) (void)hipFree(G.d_buf);
        if (G.h_buf) (void)hipHostFree(G.h_buf);
        if (G.ev) (void)hipEventDestroy(G.ev);
        if (G.own_stream && G.stream) (void)hipStreamDestroy(G.stream);
    }
    for (void* p : B->stacks) munmap(p, CO_STACK);
    if (B->d_slots) (void)hipFree(B->d_slots);
    if (B->h_slots) (void)hipHostFree(B->h_slots);
    delete B;
}

}  // namespace sharp

using namespace sharp;

struct sim_batch {
    sim_batch_impl* b;
};

extern "C" {

sim_status sim_batch_create(sim_t* const* sims, int n, sim_batch_t** out)
{
    if (!sims || !out) { set_error("null argument"); return SIM_EINVAL; }
    *out = nullptr;
    if (n < 1 || n > SIM_BATCH_MAX) { set_error("batch size must be in [1, %d]", SIM_BATCH_MAX); return SIM_EINVAL; }
    for (int i = 0; i < n; i++) {
        if (!sims[i]) { set_error("null simulation %d", i); return SIM_EINVAL; }
        for (int j = 0; j < i; j++)
            if (sims[j] == sims[i]) { set_error("simulation %d appears twice", i); return SIM_EINVAL; }
        if (sims[i]->s.o.tape) { set_error("simulation %d records a tape (not batched)", i); return SIM_EINVAL; }
    }
    sim_batch_impl* B = new sim_batch_impl();
    B->in.resize(n);
    // groups of alternate members (fewer when n is smaller), each on a
    // stream of the batch's own, created one after the other (the runtime
    // spreads consecutive streams over its hardware queues, so the groups'
    // passes overlap; a caller's stream may share a queue with them)
    const int ng = n < SHARP_BATCH_GROUPS ? n : SHARP_BATCH_GROUPS;
    B->grp.resize(ng);
    for (int i = 0; i < n; i++) B->grp[i % ng].members.push_back(i);
    sim_status rc = SIM_OK;
    int slot = 0;
    for (int g = 0; g < ng && rc == SIM_OK; g++) {
        BatchGroup& G = B->grp[g];
        G.slot0 = slot;
        for (size_t m = 0; m < G.members.size(); m++) B->in[G.members[m]].slot = slot++;
        if (hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking) == hipSuccess) {
            G.own_stream = true;
        } else {
            set_error("batch: stream creation failed");
            rc = SIM_EDEVICE;
        }
        if (rc == SIM_OK && hipEventCreateWithFlags(&G.ev, hipEventDisableTiming) != hipSuccess) {
            set_error("batch: event creation failed");
            rc = SIM_EDEVICE;
        }
    }
    if (rc == SIM_OK &&
        (hipMalloc((void**)&B->d_slots, (size_t)n * RED_WORDS * sizeof(unsigned long long)) != hipSuccess ||
         hipHostMalloc((void**)&B->h_slots, (size_t)n * RED_WORDS * sizeof(unsigned long long), hipHostMallocDefault) !=
             hipSuccess)) {
        (void)hipGetLastError();
        set_error("batch: allocation of the readback slots failed");
        rc = SIM_ENOMEM;
    }
    for (int i = 0; i < n && rc == SIM_OK; i++) {
        BatchInst& bi = B->in[i];
        bi.s = &sims[i]->s;
        bi.b = B;
        bi.rec.slot = B->d_slots + (size_t)bi.slot * RED_WORDS;
        bi.rec.yield = co_yield;
        bi.rec.yield_arg = &bi;
        void* st = mmap(nullptr, CO_STACK, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
        if (st == MAP_FAILED) { set_error("batch: stack allocation failed"); rc = SIM_ENOMEM; break; }
        B->stacks.push_back(st);
    }
    if (rc != SIM_OK) {
        batch_free(B);
        return rc;
    }
    sim_batch* h = new sim_batch;
    h->b = B;
    *out = h;
    return SIM_OK;
}

sim_status sim_batch_advance(sim_batch_t* h, const double* t_end, int mode, int64_t max_cycles, sim_stats* stats,
                             sim_status* status)
{
    if (!h || !t_end) { set_error("null argument"); return SIM_EINVAL; }
    sim_batch_impl& B = *h->b;
    const int n = (int)B.in.size();
    if (mode != SIM_SINGLE_DT && mode != SIM_MULTI_DT) { set_error("bad mode"); return SIM_EINVAL; }
    for (int i = 0; i < n; i++) {
        if (!B.in[i].s->has_state) { set_error("simulation %d: sim_set_state has not been called", i); return SIM_ESTATE; }
        if (!std::isfinite(t_end[i])) { set_error("simulation %d: t_end must be finite", i); return SIM_EINVAL; }
    }
    // work the simulations enqueued on their own streams comes first
    for (int i = 0; i < n; i++) {
        Sim& s = *B.in[i].s;
        SHARP_HIP(hipStreamSynchronize(s.stream));
        for (int k = 0; k < 2; k++)
            if (s.side[k]) SHARP_HIP(hipStreamSynchronize(s.side[k]));
    }
    B.mode = mode;
    B.max_cycles = (long long)max_cycles;
    std::vector<char> prof(n);
    for (int i = 0; i < n; i++) {
        BatchInst& bi = B.in[i];
        prof[i] = bi.s->prof;
        bi.s->prof = false;
        bi.s->rec = &bi.rec;
        bi.rec.clear();
        bi.rec.rb_pending = false;
        bi.rec.status = SIM_OK;
        bi.done = false;
        bi.rc = SIM_OK;
        bi.err.clear();
        bi.t_end = t_end[i];
        getcontext(&bi.ctx);
        bi.ctx.uc_stack.ss_sp = B.stacks[i];
        bi.ctx.uc_stack.ss_size = CO_STACK;
        bi.ctx.uc_link = &B.sched;
        const uintptr_t p = reinterpret_cast<uintptr_t>(&bi);
        makecontext(&bi.ctx, (void (*)())co_entry, 2, (unsigned)(p & 0xffffffffu), (unsigned)(p >> 32));
    }
    sim_status frc = SIM_OK;
    // resume a group's unfinished members until each yields or finishes,
    // then issue their pass; returns whether any member was resumed
    auto step = [&](BatchGroup& G) -> bool {
        int live = 0;
        for (int i : G.members) {
            BatchInst& bi = B.in[i];
            if (bi.done) continue;
            swapcontext(&B.sched, &bi.ctx);
            live++;
        }
        if (live == 0) return false;
        if (frc == SIM_OK) frc = pass_issue(B, G);
        if (frc != SIM_OK) {
            // every waiting simulation sees the failure at its readback and returns
            for (int i = 0; i < n; i++) {
                B.in[i].rec.status = frc;
                B.in[i].rec.rb_pending = false;
                B.in[i].rec.clear();
            }
            for (BatchGroup& H : B.grp) H.pending = false;
        }
        return true;
    };
    // the groups alternate: while one group's pass runs on the GPU, the
    // other group is resumed and its next pass recorded and issued
    for (BatchGroup& G : B.grp) step(G);
    for (;;) {
        bool any = false;
        for (BatchGroup& G : B.grp) {
            if (G.pending) {
                sim_status rc = pass_complete(B, G);
                if (rc != SIM_OK && frc == SIM_OK) frc = rc;
            }
            any = step(G) || any;
        }
        if (!any) break;
    }
    for (BatchGroup& G : B.grp) (void)hipStreamSynchronize(G.stream);
    sim_status first = frc;
    std::string msg = frc != SIM_OK ? std::string(sim_last_error()) : std::string();
    for (int i = 0; i < n; i++) {
        BatchInst& bi = B.in[i];
        bi.s->rec = nullptr;
        bi.s->prof = prof[i];
        if (bi.rc == SIM_OK && stats) bi.rc = engine_bflux(*bi.s, bi.st.bflux);
        if (stats) stats[i] = bi.st;
        if (status) status[i] = bi.rc;
        if (bi.rc != SIM_OK && first == SIM_OK) {
            first = bi.rc;
            msg = "simulation " + std::to_string(i) + ": " + bi.err;
        }
    }
    if (first != SIM_OK) set_error("%s", msg.c_str());
    return first;
}

sim_status sim_batch_info(sim_batch_t* h, int64_t* passes, int64_t* fused_launches, int64_t* records)
{
    if (!h) { set_error("null handle"); return SIM_EINVAL; }
    if (passes) *passes = h->b->passes;
    if (fused_launches) *fused_launches = h->b->fused;
    if (records) *records = h->b->recorded;
    return SIM_OK;
}

void sim_batch_destroy(sim_batch_t* h)
{
    if (!h) return;
    for (BatchInst& bi : h->b->in)
        if (bi.s) bi.s->rec = nullptr;
    batch_free(h->b);
    delete h;
}

}  // extern "C"
