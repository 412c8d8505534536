// sim.h -- internal definition of the lattice handle shared by the runtime
// translation units (runtime.hip, batch.hip).
#pragma once
#include <cstring>
#include <string>
#include <vector>

#include "cgb_dev.h"

struct LaunchRec {
    int kind;
    hipEvent_t e0, e1;
};

enum { K_PREP, K_RASTER, K_TRANS, K_LB, K_MEM, K_CELLS, K_POT, K_INT, K_TRACK, K_NKIND };

// where a handle's device memory comes from
enum { MEM_OWN = 0, MEM_ARENA = 1, MEM_COUNT = 2 };

struct cgb_sim {
    double n_nonwall = 0;  // non-wall nodes (normalisation of the tracked sums)
    cgb_params P;
    cgb::DevArgs a;
    hipStream_t st = nullptr;
    bool own_stream = false;
    // the cell list and the potentials, which need only the cells' positions
    // and axes, run on a side stream beside the lattice part of the step;
    // events order them (default priorities throughout)
    bool fork = false;
    hipStream_t st_pot = nullptr;
    hipEvent_t ev_ras = nullptr, ev_pot = nullptr;
    int cur = 0;
    void* pop[2] = {nullptr, nullptr};
    void* rho[2] = {nullptr, nullptr};
    size_t esize = 8;
    int ncap = 0;
    long long step = 0;
    bool fluid_ready = false;
    std::string err;
    int64_t dev_bytes = 0;
    std::vector<void*> allocs;
    // MEM_ARENA: every device array is a piece of the caller's arena, sized
    // once at creation for cell_cap cells and track_max recorded steps
    int mem_mode = MEM_OWN;
    char* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0, arena_state = 0;
    int cell_cap = -1;
    int track_max = 0;
    double* track_buf = nullptr;
    double* le_rec_buf = nullptr;
    double* tmp = nullptr;  // FP64 staging for uploads/downloads
    void* zero_buf = nullptr;  // 256 zeroed bytes (large-lattice layout)
    // a captured step sequence (cgb_capture / cgb_replay) and what it was
    // captured with
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_steps = 0;
    cgb::DevArgs cap_args{};
    cgb::LaunchCfg cap_cfg{0, 0, 0};
    bool cap_fork = false;
    long long n_stored = 0;    // indexed layout: stored (non-wall) nodes
    size_t tmp_bytes = 0;
    double* obs_partial = nullptr;
    int obs_nblk = 512;
    int* pair_buf = nullptr;
    int* pair_cnt = nullptr;
    int pair_cap = 0;
    cgb::LaunchCfg lbcfg{64, 4, 16};
    bool prof = false;
    std::vector<LaunchRec> recs;
    std::vector<hipEvent_t> ev_pool;
    double ktime[K_NKIND] = {0};
    long long kcount[K_NKIND] = {0};
};


namespace cgb {
// internal entry points of runtime.hip used by the batch
int sim_set_tiles(cgb_sim* s, LaunchCfg cfg);
void sim_bind(cgb_sim* s);
}  // namespace cgb

// the device arguments a launch sequence was recorded with still hold (the
// host-side step index aside, which no kernel reads)
inline bool sim_same_args(const cgb::DevArgs& live, const cgb::DevArgs& snap) {
    cgb::DevArgs t;
    memcpy(&t, &live, sizeof t);
    t.step = snap.step;
    return memcmp(&t, &snap, sizeof t) == 0;
}
