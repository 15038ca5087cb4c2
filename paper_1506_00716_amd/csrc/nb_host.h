// nb_host.h -- host-side handle types shared by the libnb C-ABI sources.
#pragma once

#include "../../include/nb.h"
#include "nb_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

struct nb_ctx {
    int device;
    int n_cu;  // compute units of the device
    hipStream_t stream;
    std::string err;
};

struct nb_sys {
    nb_ctx* ctx;
    nb_params p;
    int M, G, jtile, fx_bits;
    int ncx, ncy;
    int max_groups, cand_cap, ent_cap, item_cap;
    void* arena;
    size_t arena_bytes;
    size_t needed_bytes;
    nbi::SysDev h;        // host copy of the descriptor
    nbi::SysDev* d_desc;  // device copy (inside the arena)
    int* d_prefix;        // [2] item prefix for single-system launches
    int* d_done;          // [1] relaxation flag
    std::vector<double> q, sig, eps, mass;
    bool has_particles, has_mass;
    bool list_valid;
    bool list_exact;  // the list carries the exact FP64 atom-pair masks
    int64_t step;
    nbi::Bounds bounds;
    double ew_fit_err;    // max relative error of the Ewald force and energy tables on [0, rc]
    bool pme_on;          // reciprocal-space Ewald (pme_grid set)
    nbi::PmeDev pme;      // its grids and constants (inside the arena)
    // a second stream (default priority) for PME systems: the pair kernel and
    // the reciprocal part run side by side, one of them forked from the
    // context stream at side_in and joined back at side_out
    hipStream_t side_stream;
    hipEvent_t side_in, side_out;
    nb_ens* ens;          // ensemble the system belongs to (or NULL)
    int64_t list_step;    // step counter when the current list was built (dynamic-prune schedule)
    int pg_cur;           // partial buffer of the next prune-guard interval
    bool pg_pending;      // the other buffer holds an interval not folded yet
    bool f_current;       // f holds F(x) for the current x and list (kept by the ensemble
                          // between its calls, so a call opens without a force pass)
    // the descriptor as last copied to d_desc (a call whose descriptor is
    // unchanged copies nothing)
    nbi::SysDev desc_sent;
    bool desc_sent_valid = false;
    // pinned host buffer (md_step): the energy-trace ring rows and the status
    // words of a call come back in one copy round and one synchronisation
    void* mailbox = nullptr;
    // per-phase HIP-event timers (md_step): pairs of events around each launch
    bool timing;
    int timing_every;     // mark one of every timing_every force launches / rebuilds
    int64_t mark_seq[2];  // force launches and rebuilds seen since set_timing
    bool mark_open;       // the last mark_begin recorded (its mark_end records too)
    bool check_builds;    // md_step: synchronise after each rebuild to check capacity
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used;
    std::vector<std::pair<size_t, int>> ev_marks;  // (first event index, phase)
    double t_ms[4];       // accumulated ms: force kernel, list build, whole md_step
    int64_t t_n[4];       // launches / builds / calls
};

namespace nbh {

// A roctx range over a host scope (the library's phases: list rebuilds, force
// passes, PME, ensemble steps, server batches), shown by rocprofv3
// --marker-trace beside the kernels the scope enqueued; a cheap no-op when no
// tool is attached
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

nb_status fail(nb_ctx* ctx, nb_status code, const std::string& msg);
nb_status upload_desc(nb_sys* s);
nb_status read_status(nb_sys* s, int st[nbi::ST_COUNT]);
nb_status capacity_error(nb_sys* s, const int st[nbi::ST_COUNT]);
nb_status do_build(nb_sys* s, bool exact = true);
// cleared: the gather that ended the step did the build's clears (md_step)
nb_status enqueue_build(nb_sys* s, bool exact, int status_clear, bool first, bool cleared = false);
nb_status make_exact(nb_sys* s);
nb_status read_candidates(nb_sys* s, int ng, std::vector<int>& cc, std::vector<int2>& cand,
                          std::vector<unsigned long long>& msk);
// open_next > 0 (md_step's first positions): the gather also applies the first
// step's half-kick and drift (and with 2 the staging), with time step dt.
// clear_status: the staging kernel clears the status words first
nb_status eval_forces(nb_sys* s, bool ener, int trace_row, bool with_ke, double step_value, int open_next = 0,
                      double dt = 0.0, bool clear_status = false);
nb_status check_after(nb_sys* s);
// the error (if any) that a call's status words report
nb_status status_result(nb_sys* s, const int st[nbi::ST_COUNT]);
// A PME system's step runs the pair kernel and the reciprocal part side by
// side; whichever takes longer stays on the context stream, where its
// dependencies on the kernels before and after it (the gathers, the list
// build) are ordered inside one queue: a dependency between two queues costs
// about 10 us each way on MI355X.
//  pme_fork / pme_join: PME of positions x on the side stream, after the work
//    queued so far on the context stream; the join makes the context stream
//    wait for it (steps with a list build: PME beside the build and the pair
//    kernel)
//  pair_beside_pme: the pair kernel on the side stream, PME of x on the context
//    stream, joined before the caller's gather (the other steps, and single
//    evaluations, where the PME chain is the longer)
nb_status pme_fork(nb_sys* s, const double* x, bool ener);
nb_status pme_join(nb_sys* s);
nb_status pair_beside_pme(nb_sys* s, const double* x, bool ener, bool prune);
// the pair kernel's grid beside the PME kernels: 3 blocks of 4 waves per CU
// (of the 4 it can hold at <= 128 VGPRs), so they find a free wave slot on
// every SIMD
int pair_grid_beside_pme(const nb_ctx* c);
// dynamic-prune guard (no-op without pruning): check = the prune interval that
// ends here is measured; either way x_prune = x
nb_status prune_guard(nb_sys* s, bool check);

}  // namespace nbh

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return nbh::fail((ctx), NB_ERR_DEVICE,                                           \
                             std::string(#expr) + ": " + hipGetErrorString(_e));             \
    } while (0)
