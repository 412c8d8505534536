// batch.hip -- ensemble of independent, uneven lattices advanced together.
//
// Each channel is a full lattice handle.  When every channel runs the dense
// tau = 1 path in one storage precision, a step is one launch per kernel for
// all channels: the channels are grouped by kernel variant and block shape,
// and a group's launch holds the channels' own grids back to back; each block
// finds its channel in a block table and works on that channel's device
// arguments (both roles of the population buffers are uploaded once, so the
// launches alternate between two argument tables).  Otherwise each channel
// enqueues its own step sequence on its own stream between a fork and join
// events.  Either form is captured into one HIP graph.  An even number of
// steps is captured so that the two population buffers of every channel are
// back in their starting roles after each replay; the step index lives in
// device memory, so replays advance it.  The autotuner times the fused LB
// kernel for a set of tile shapes on one channel of each width class and
// applies the fastest.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sim.h"

using namespace cgb;

struct cgb_batch {
    std::vector<cgb_sim*> ch;
    hipStream_t master = nullptr;
    // fused step: the cell list and pair forces run on a side stream beside
    // the lattice kernels, between a fork after the rasterisation and a join
    // before the integrator
    hipStream_t side = nullptr;
    hipEvent_t ev_fk = nullptr, ev_jn = nullptr;
    hipEvent_t fork = nullptr, done = nullptr;  // captured fork; end of replays
    std::vector<hipEvent_t> join, pre;          // captured joins; eager work before a replay
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_steps = 0;
    // Per channel, the device arguments and launch shape baked into the
    // graph; a replay is refused once any channel's differ (buffers swapped
    // by an odd number of eager steps, arrays reallocated by a new cell set
    // or a new tile shape).
    std::vector<DevArgs> cap_args;
    std::vector<LaunchCfg> cap_cfg;
    std::string err;
    // One launch per kernel for every channel (the captured graph holds the
    // step's kernels once, not once per channel): the launches in step
    // order, their per-channel block tables, and each channel's device
    // arguments for the two roles of its population buffers.
    std::vector<MultiLaunch> plan;
    void* plan_mem = nullptr;  // [2][nch] DevArgs, then the ChanGrid tables
    size_t plan_bytes = 0;
    const DevArgs* plan_args[2] = {nullptr, nullptr};
};


#define BFAIL(b, code, ...)                         \
    do {                                            \
        char _m[512];                               \
        snprintf(_m, sizeof _m, __VA_ARGS__);       \
        (b)->err = _m;                              \
        return code;                                \
    } while (0)
#define BCHK(b, call)                                                                    \
    do {                                                                                 \
        hipError_t _e = (call);                                                          \
        if (_e != hipSuccess) BFAIL(b, CGB_EDEVICE, "%s: %s", #call, hipGetErrorString(_e)); \
    } while (0)

namespace cgb {
bool multi_grid(int kind, const DevArgs& a, LaunchCfg lb, int* variant, unsigned* bx, unsigned* by, dim3* grid,
                int* arg) {
    if (kind == MK_LB) {
        *arg = 0;
        return multi_grid_lb(a, lb, variant, bx, by, grid);
    }
    if (kind == MK_TRACK || kind == MK_TRACK_FIN) return multi_grid_fields(kind, a, variant, bx, by, grid, arg);
    return multi_grid_particles(kind, a, variant, bx, by, grid, arg);
}
hipError_t launch_multi(const MultiLaunch& m, const DevArgs* args, hipStream_t st) {
    if (m.kind == MK_LB) return launch_multi_lb(m, args, st);
    if (m.kind == MK_TRACK || m.kind == MK_TRACK_FIN) return launch_multi_fields(m, args, st);
    return launch_multi_particles(m, args, st);
}
}  // namespace cgb

// kernels of one channel's step in the order cgb_step launches them (a
// batch's channels step alone on their streams: no side stream)
static const int kStepKinds[] = {MK_PREP, MK_CLAIM, MK_RESOLVE, MK_TRANS, MK_LMOM, MK_LB, MK_MEM, MK_TRACK,
                                 MK_TRACK_FIN, MK_BIN_CLEAR, MK_BIN_COUNT, MK_SCAN_LOCAL, MK_SCAN_TOP, MK_SCAN_ADD,
                                 MK_BIN_FILL, MK_BIN_SORT, MK_SORTED_POS, MK_POT, MK_INT};

static void drop_plan(cgb_batch* b) {
    if (b->plan_mem) (void)hipFree(b->plan_mem);
    b->plan_mem = nullptr;
    b->plan_bytes = 0;
    b->plan.clear();
    b->plan_args[0] = b->plan_args[1] = nullptr;
}

// every channel can take the one-launch-per-kernel step: the tau = 1 dense
// kernel, one precision, no viscometer
static bool fusable(const cgb_batch* b) {
    for (const cgb_sim* s : b->ch) {
        const DevArgs& a = s->a;
        if (a.tau != 1.0 || a.big || a.cidx || a.le_u != 0.0 || !a.lmom || a.precision != b->ch[0]->a.precision)
            return false;
    }
    return true;
}

static void drop_graph(cgb_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = 0;
    drop_plan(b);
}

// The launch plan of the current channel states: per kernel of the step,
// the channels grouped by kernel variant and block shape, each group one
// launch whose blocks are the channels' own grids back to back.
static int build_plan(cgb_batch* b) {
    drop_plan(b);
    const int nch = (int)b->ch.size();
    struct Group {
        int kind, variant;
        unsigned bx, by;
        std::vector<ChanGrid> cg;
        std::vector<int> chans;
    };
    std::vector<Group> groups;
    for (int kind : kStepKinds) {
        std::map<std::tuple<int, unsigned, unsigned>, size_t> at;
        for (int c = 0; c < nch; c++) {
            const cgb_sim* s = b->ch[(size_t)c];
            int variant = 0, arg = 0;
            unsigned bx = 0, by = 0;
            dim3 g;
            if (!multi_grid(kind, s->a, s->lbcfg, &variant, &bx, &by, &g, &arg)) continue;
            const auto key = std::make_tuple(variant, bx, by);
            auto it = at.find(key);
            if (it == at.end()) {
                at[key] = groups.size();
                groups.push_back(Group{kind, variant, bx, by, {}, {}});
                it = at.find(key);
            }
            Group& G = groups[it->second];
            const unsigned start = G.cg.empty() ? 0u : G.cg.back().start + G.cg.back().gx * G.cg.back().gy * G.cg.back().gz;
            G.cg.push_back(ChanGrid{start, g.x, g.y, g.z, arg, {0, 0, 0}});
            G.chans.push_back(c);
        }
    }
    // device memory: both argument arrays, then every group's table (with its
    // own argument arrays, since a group holds a subset of the channels)
    size_t ntab = 0, tab_bytes = 0;
    for (const Group& G : groups) {
        ntab += G.cg.size();
        const unsigned blocks = G.cg.back().start + G.cg.back().gx * G.cg.back().gy * G.cg.back().gz;
        // the group's table, its block -> channel list, rounded to whole entries
        tab_bytes += G.cg.size() * sizeof(ChanGrid) + ((size_t)blocks * 4 + sizeof(ChanGrid) - 1) / sizeof(ChanGrid) * sizeof(ChanGrid);
    }
    const size_t args_bytes = 2 * (size_t)nch * sizeof(DevArgs);
    const size_t grp_args = 2 * ntab * sizeof(DevArgs);
    b->plan_bytes = args_bytes + grp_args + tab_bytes;
    BCHK(b, hipMalloc(&b->plan_mem, b->plan_bytes));
    std::vector<char> host(b->plan_bytes);
    DevArgs* ha = (DevArgs*)host.data();
    for (int q = 0; q < 2; q++)
        for (int c = 0; c < nch; c++) {
            cgb_sim* s = b->ch[(size_t)c];
            const int cur = s->cur;
            s->cur = (cur + q) & 1;
            sim_bind(s);
            memcpy(&ha[(size_t)q * nch + c], &s->a, sizeof(DevArgs));
            s->cur = cur;
            sim_bind(s);
        }
    char* dev = (char*)b->plan_mem;
    DevArgs* garg = (DevArgs*)(host.data() + args_bytes);
    size_t off = 0, toff = args_bytes + grp_args;
    for (const Group& G : groups) {
        const size_t k = G.cg.size();
        for (int q = 0; q < 2; q++)
            for (size_t j = 0; j < k; j++) garg[(size_t)q * ntab + off + j] = ha[(size_t)q * nch + G.chans[j]];
        MultiLaunch m;
        m.kind = G.kind;
        m.variant = G.variant;
        m.bx = G.bx;
        m.by = G.by;
        m.blocks = G.cg.back().start + G.cg.back().gx * G.cg.back().gy * G.cg.back().gz;
        m.nch = (int)k;
        ChanGrid* tab = (ChanGrid*)(host.data() + toff);
        memcpy(tab, G.cg.data(), k * sizeof(ChanGrid));
        int* blk = (int*)(tab + k);
        for (size_t j = 0; j < k; j++) {
            const unsigned nb = G.cg[j].gx * G.cg[j].gy * G.cg[j].gz;
            for (unsigned t = 0; t < nb; t++) blk[G.cg[j].start + t] = (int)j;
        }
        m.cg = (const ChanGrid*)(dev + toff);
        b->plan.push_back(m);
        off += k;
        toff += k * sizeof(ChanGrid) + ((size_t)m.blocks * 4 + sizeof(ChanGrid) - 1) / sizeof(ChanGrid) * sizeof(ChanGrid);
    }
    BCHK(b, hipMemcpy(b->plan_mem, host.data(), b->plan_bytes, hipMemcpyHostToDevice));
    // per launch: the argument array of its group (offset into the group arrays)
    b->plan_args[0] = (const DevArgs*)(dev + args_bytes);
    b->plan_args[1] = (const DevArgs*)(dev + args_bytes) + ntab;
    return CGB_OK;
}

// one time step of every channel: the plan's launches with the arguments of
// buffer role q
// (the cell list and the pair forces need only the step start's positions
// and kinematics, and write arrays the lattice kernels do not read: the same
// split as one lattice's step)
static bool on_side(int kind) { return kind >= MK_BIN_CLEAR && kind <= MK_POT; }
static int fused_step(cgb_batch* b, int q) {
    size_t off = 0;
    bool forked = false, side_open = false;
    for (const MultiLaunch& m : b->plan) {
        const DevArgs* args = b->plan_args[q] + off;
        off += (size_t)m.nch;
        if (!forked && m.kind > MK_RESOLVE) {
            BCHK(b, hipEventRecord(b->ev_fk, b->master));
            forked = true;
        }
        if (on_side(m.kind)) {
            if (!side_open) {
                BCHK(b, hipStreamWaitEvent(b->side, b->ev_fk, 0));
                side_open = true;
            }
            BCHK(b, launch_multi(m, args, b->side));
            continue;
        }
        if (m.kind == MK_INT && side_open) {
            BCHK(b, hipEventRecord(b->ev_jn, b->side));
            BCHK(b, hipStreamWaitEvent(b->master, b->ev_jn, 0));
            side_open = false;
        }
        BCHK(b, launch_multi(m, args, b->master));
    }
    if (side_open) {
        BCHK(b, hipEventRecord(b->ev_jn, b->side));
        BCHK(b, hipStreamWaitEvent(b->master, b->ev_jn, 0));
    }
    return CGB_OK;
}

extern "C" {

void cgb_batch_destroy(cgb_batch* b) {
    if (!b) return;
    if (b->master) (void)hipStreamSynchronize(b->master);
    if (b->side) (void)hipStreamSynchronize(b->side);
    drop_graph(b);
    for (cgb_sim* s : b->ch) cgb_destroy(s);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->pre) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->ev_fk) (void)hipEventDestroy(b->ev_fk);
    if (b->ev_jn) (void)hipEventDestroy(b->ev_jn);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->master) (void)hipStreamDestroy(b->master);
    delete b;
}

const char* cgb_batch_last_error(const cgb_batch* b) { return b ? b->err.c_str() : "null handle"; }

int cgb_batch_create(int32_t nch, const cgb_params* ch, cgb_batch** out) {
    if (!out || nch < 1 || !ch) return CGB_EINVAL;
    *out = nullptr;
    cgb_batch* b = new cgb_batch();
    if (hipStreamCreateWithFlags(&b->master, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_fk, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_jn, hipEventDisableTiming) != hipSuccess) {
        cgb_batch_destroy(b);
        return CGB_EDEVICE;
    }
    for (int c = 0; c < nch; c++) {
        cgb_sim* s = nullptr;
        const int rc = cgb_create(&ch[c], nullptr, nullptr, &s);
        if (rc) {
            cgb_batch_destroy(b);
            return rc;
        }
        // the channels run concurrently with each other: each steps on its own
        // stream alone (the captured graph holds one chain per channel)
        s->fork = false;
        b->ch.push_back(s);
        hipEvent_t e1, e2;
        if (hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess) {
            cgb_batch_destroy(b);
            return CGB_EDEVICE;
        }
        b->join.push_back(e1);
        if (hipEventCreateWithFlags(&e2, hipEventDisableTiming) != hipSuccess) {
            cgb_batch_destroy(b);
            return CGB_EDEVICE;
        }
        b->pre.push_back(e2);
    }
    *out = b;
    return CGB_OK;
}

int cgb_batch_channel(cgb_batch* b, int32_t c, cgb_sim** out) {
    if (!b || !out || c < 0 || c >= (int)b->ch.size()) return CGB_EINVAL;
    *out = b->ch[(size_t)c];
    return CGB_OK;
}

// The LB launches of the fused plan alone, for the current tiles: they read
// the current populations and write only buffers that every step rewrites
// before reading them (the other population buffer and its densities, the
// cell nodes' momenta, the mixture partials), so the state is unchanged.
static int time_fused_lb(cgb_batch* b, int reps, double* ms_avg) {
    int rc = build_plan(b);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto lb_pass = [&]() {
        size_t off = 0;
        for (const MultiLaunch& m : b->plan) {
            if (m.kind == MK_LB && e == hipSuccess) e = launch_multi(m, b->plan_args[0] + off, b->master);
            off += (size_t)m.nch;
        }
    };
    for (int k = 0; k < 2; k++) lb_pass();
    if (e == hipSuccess) e = hipEventRecord(e0, b->master);
    for (int k = 0; k < reps; k++) lb_pass();
    if (e == hipSuccess) e = hipEventRecord(e1, b->master);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    drop_plan(b);
    if (e != hipSuccess) BFAIL(b, CGB_EDEVICE, "LB timing: %s", hipGetErrorString(e));
    *ms_avg = (double)ms / reps;
    return CGB_OK;
}

// Chooses the LB tile shape per width class of the channels.  Fused batches
// (one launch per kernel for every channel): what counts is the time of the
// whole fused LB launch, so each class in turn tries every candidate with the
// other classes' shapes fixed, and keeps the one whose fused launches take
// least; then every candidate for all channels at once is timed against that
// result.  Otherwise: the LB kernel alone on the first channel of each class.
// chosen: nullable, nch*3 ints (bx, by, tz).
int cgb_batch_autotune(cgb_batch* b, int32_t reps, int32_t* chosen) {
    if (!b || reps < 1) return CGB_EINVAL;
    drop_graph(b);
    std::map<int, std::vector<int>> classes;  // width class -> channels
    for (size_t c = 0; c < b->ch.size(); c++) {
        const int w = b->ch[c]->a.nx;
        classes[w < 48 ? 0 : (w < 80 ? 1 : 2)].push_back((int)c);
    }
    int rc = CGB_OK;
    if (fusable(b)) {
        // plane-linear tiles (by = 0) keep every lane busy on rows of any width
        static const LaunchCfg fcand[] = {{64, 0, 8}, {128, 0, 8}, {256, 0, 8}, {64, 0, 16}, {256, 0, 16},
                                          {32, 8, 8}, {64, 4, 8}, {32, 8, 16}, {64, 4, 16}};
        for (cgb_sim* s : b->ch) BCHK(b, hipStreamSynchronize(s->st));
        for (auto& kv : classes) {
            LaunchCfg best = b->ch[(size_t)kv.second[0]]->lbcfg;
            double best_ms = 1e30;
            for (const LaunchCfg& cf : fcand) {
                for (int c : kv.second)
                    if ((rc = sim_set_tiles(b->ch[(size_t)c], cf)) != CGB_OK) break;
                if (rc) break;
                double ms = 0.0;
                if ((rc = time_fused_lb(b, reps, &ms)) != CGB_OK) return rc;
                if (ms < best_ms) { best_ms = ms; best = cf; }
            }
            if (rc) break;
            for (int c : kv.second)
                if ((rc = sim_set_tiles(b->ch[(size_t)c], best)) != CGB_OK) break;
            if (rc) break;
        }
        // one shape for every channel (one LB launch): a change no single
        // class's step above can make once the classes' shapes differ
        if (!rc && classes.size() > 1) {
            std::vector<LaunchCfg> tuned;
            for (cgb_sim* s : b->ch) tuned.push_back(s->lbcfg);
            double best_ms = 0.0;
            if ((rc = time_fused_lb(b, reps, &best_ms)) != CGB_OK) return rc;
            const LaunchCfg* uni = nullptr;
            for (const LaunchCfg& cf : fcand) {
                for (cgb_sim* s : b->ch)
                    if ((rc = sim_set_tiles(s, cf)) != CGB_OK) break;
                if (rc) break;
                double ms = 0.0;
                if ((rc = time_fused_lb(b, reps, &ms)) != CGB_OK) return rc;
                if (ms < best_ms) { best_ms = ms; uni = &cf; }
            }
            for (size_t c = 0; c < b->ch.size() && !rc; c++)
                rc = sim_set_tiles(b->ch[c], uni ? *uni : tuned[c]);
        }
    } else {
        static const LaunchCfg cand[] = {{64, 4, 8}, {64, 4, 16}, {32, 8, 8}, {32, 8, 16}, {16, 16, 16}, {64, 2, 16}, {32, 4, 16}};
        for (auto& kv : classes) {
            cgb_sim* s = b->ch[(size_t)kv.second[0]];
            LaunchCfg best = s->lbcfg;
            double best_ms = 1e30;
            for (const LaunchCfg& cf : cand) {
                if ((rc = sim_set_tiles(s, cf)) != CGB_OK) break;
                double ms = 0.0;
                if ((rc = cgb_time_lb(s, reps, &ms)) != CGB_OK) break;
                if (ms < best_ms) { best_ms = ms; best = cf; }
            }
            if (rc) break;
            for (int c : kv.second)
                if ((rc = sim_set_tiles(b->ch[(size_t)c], best)) != CGB_OK) break;
            if (rc) break;
        }
    }
    if (rc) BFAIL(b, rc, "autotune failed: %s", cgb_last_error(b->ch[0]));
    if (chosen)
        for (size_t c = 0; c < b->ch.size(); c++) {
            const LaunchCfg& k = b->ch[c]->lbcfg;
            chosen[3 * c] = k.bx; chosen[3 * c + 1] = k.by; chosen[3 * c + 2] = k.tz;
        }
    return CGB_OK;
}

// Captures `steps` (even) time steps of every channel into one graph.
int cgb_batch_capture(cgb_batch* b, int32_t steps) {
    if (!b || steps < 2 || (steps & 1)) return CGB_EINVAL;
    drop_graph(b);
    for (cgb_sim* s : b->ch) {
        if (!s->fluid_ready) BFAIL(b, CGB_ESTATE, "channel not initialised");
        BCHK(b, hipStreamSynchronize(s->st));
        if (s->prof) cgb_profile(s, 0);
    }
    std::vector<int> cur(b->ch.size());
    std::vector<long long> stp(b->ch.size());
    for (size_t c = 0; c < b->ch.size(); c++) { cur[c] = b->ch[c]->cur; stp[c] = b->ch[c]->step; }
    if (fusable(b)) {
        // one launch per kernel for every channel
        int rc = build_plan(b);
        if (rc) return rc;
        BCHK(b, hipStreamBeginCapture(b->master, hipStreamCaptureModeRelaxed));
        for (int k = 0; k < steps && rc == CGB_OK; k++) rc = fused_step(b, k & 1);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(b->master, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e2 != hipSuccess) BFAIL(b, CGB_EDEVICE, "end capture: %s", hipGetErrorString(e2));
        b->graph = g;
        BCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_steps = steps;
        b->cap_args.resize(b->ch.size());
        b->cap_cfg.resize(b->ch.size());
        for (size_t c = 0; c < b->ch.size(); c++) {
            memcpy(&b->cap_args[c], &b->ch[c]->a, sizeof(DevArgs));
            b->cap_cfg[c] = b->ch[c]->lbcfg;
        }
        return CGB_OK;
    }
    BCHK(b, hipStreamBeginCapture(b->master, hipStreamCaptureModeRelaxed));
    hipError_t e = hipEventRecord(b->fork, b->master);
    int rc = CGB_OK;
    for (size_t c = 0; c < b->ch.size() && e == hipSuccess && rc == CGB_OK; c++) {
        cgb_sim* s = b->ch[c];
        e = hipStreamWaitEvent(s->st, b->fork, 0);
        if (e != hipSuccess) break;
        rc = cgb_step(s, steps);
        if (rc) break;
        e = hipEventRecord(b->join[c], s->st);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->master, b->join[c], 0);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->master, &g);
    for (size_t c = 0; c < b->ch.size(); c++) {
        b->ch[c]->cur = cur[c];
        b->ch[c]->step = stp[c];
        sim_bind(b->ch[c]);
    }
    if (rc) { if (g) (void)hipGraphDestroy(g); BFAIL(b, rc, "capture: %s", cgb_last_error(b->ch[0])); }
    if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); BFAIL(b, CGB_EDEVICE, "capture: %s", hipGetErrorString(e)); }
    if (e2 != hipSuccess) BFAIL(b, CGB_EDEVICE, "end capture: %s", hipGetErrorString(e2));
    b->graph = g;
    BCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_steps = steps;
    b->cap_args.resize(b->ch.size());
    b->cap_cfg.resize(b->ch.size());
    for (size_t c = 0; c < b->ch.size(); c++) {
        memcpy(&b->cap_args[c], &b->ch[c]->a, sizeof(DevArgs));
        b->cap_cfg[c] = b->ch[c]->lbcfg;
    }
    return CGB_OK;
}

// Replays the captured graph nsteps / graph_steps times (asynchronous).
int cgb_batch_run(cgb_batch* b, int32_t nsteps) {
    if (!b || nsteps < 0) return CGB_EINVAL;
    if (!b->exec) BFAIL(b, CGB_ESTATE, "no captured graph");
    if (nsteps % b->graph_steps) BFAIL(b, CGB_EINVAL, "steps must be a multiple of %d", b->graph_steps);
    for (size_t c = 0; c < b->ch.size(); c++) {
        cgb_sim* s = b->ch[c];
        const LaunchCfg& k = b->cap_cfg[c];
        if (!sim_same_args(s->a, b->cap_args[c]) || s->lbcfg.bx != k.bx || s->lbcfg.by != k.by || s->lbcfg.tz != k.tz)
            BFAIL(b, CGB_ESTATE, "channel %zu changed since the capture (odd eager steps, new cells or tiles); capture again", c);
        // the channel streams may hold eager work issued since the last replay
        BCHK(b, hipEventRecord(b->pre[c], s->st));
        BCHK(b, hipStreamWaitEvent(b->master, b->pre[c], 0));
    }
    for (int k = 0; k < nsteps / b->graph_steps; k++) BCHK(b, hipGraphLaunch(b->exec, b->master));
    // later eager work on a channel stream waits for the replays
    BCHK(b, hipEventRecord(b->done, b->master));
    for (cgb_sim* s : b->ch) {
        BCHK(b, hipStreamWaitEvent(s->st, b->done, 0));
        s->step += nsteps;
    }
    return CGB_OK;
}

int cgb_batch_sync(cgb_batch* b) {
    if (!b) return CGB_EINVAL;
    BCHK(b, hipStreamSynchronize(b->master));
    for (size_t c = 0; c < b->ch.size(); c++) {
        const int rc = cgb_sync(b->ch[c]);
        if (rc) BFAIL(b, rc, "channel %zu: %s", c, cgb_last_error(b->ch[c]));
    }
    return CGB_OK;
}

// Per-step mixture record on every channel (cgb_track); captured graphs
// record too, so capture after enabling it.
int cgb_batch_track(cgb_batch* b, int32_t cap) {
    if (!b || cap < 0) return CGB_EINVAL;
    drop_graph(b);
    for (size_t c = 0; c < b->ch.size(); c++) {
        const int rc = cgb_track(b->ch[c], cap);
        if (rc) BFAIL(b, rc, "channel %zu: %s", c, cgb_last_error(b->ch[c]));
    }
    return CGB_OK;
}

// Apparent relative viscosity of every channel from its record (cgb_mu_rel).
int cgb_batch_mu_rel(cgb_batch* b, int32_t first, double* mu) {
    if (!b || !mu) return CGB_EINVAL;
    BCHK(b, hipStreamSynchronize(b->master));
    for (size_t c = 0; c < b->ch.size(); c++) {
        const int rc = cgb_mu_rel(b->ch[c], first, mu + c);
        if (rc) BFAIL(b, rc, "channel %zu: %s", c, cgb_last_error(b->ch[c]));
    }
    return CGB_OK;
}

}  // extern "C"
