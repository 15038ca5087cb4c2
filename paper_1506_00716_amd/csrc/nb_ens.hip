// nb_ens.hip -- batched ensembles and the cluster/tile autotuner.
//
// Many independent systems (paper, Section "Ensemble simulations") advance
// together: every per-step kernel is launched once over a device table of the
// members' descriptors (2-D grids: y = member), and the force kernel once per
// kernel class (cluster size, interaction type) as a persistent launch over the
// concatenated work items of that class.  The step without a list rebuild is
// captured once into a HIP graph and replayed.  Each member's arithmetic
// depends only on its own descriptor and list, so its trajectory is bitwise
// the same alone and in any batch.
#include "nb_host.h"

#include <algorithm>
#include <cstring>
#include <tuple>
#include <vector>

using namespace nbi;

namespace {

__global__ void k_ens_energy(const SysDev* __restrict__ table, int n, double* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[3 * i] = table[i].eout[0];
    out[3 * i + 1] = table[i].eout[1];
    out[3 * i + 2] = table[i].eout[8];
}

size_t al(size_t v) { return (v + 255) & ~size_t(255); }

struct EnsClass {
    int M, coul, lj, fp32;
    int off, cnt;
    int item_cap;
    int prefix_off;
};

}  // namespace

struct nb_ens {
    nb_ctx* ctx;
    int max_systems;
    void* arena;
    size_t arena_bytes;
    SysDev* d_table;
    int* d_prefix;
    int* d_prefix2;   // item prefixes of the opening force pass (members that need it)
    int* d_flags;     // build modes per member
    int* d_eflags;    // opening force pass per member (1 = needed)
    int* d_status;
    double* d_energy;
    std::vector<nb_sys*> members;
    std::vector<double*> xs, vs;
    std::vector<float*> fs;
    std::vector<SysDev> h_table;
    std::vector<EnsClass> classes;
    std::vector<int> h_eflags;  // host copy of d_eflags (kept until the upload has run)
    Bounds bounds;
    bool dirty;
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_ok;
    double graph_dt;
};

namespace {

size_t ens_layout(int max_systems, char* base, nb_ens* e)
{
    size_t off = 0;
    auto take = [&](size_t b) -> char* {
        char* p = base ? base + off : nullptr;
        off = al(off + b);
        return p;
    };
    char* t = take(sizeof(SysDev) * (size_t)max_systems);
    char* p = take(sizeof(int) * (size_t)(2 * max_systems + 64));
    char* p2 = take(sizeof(int) * (size_t)(2 * max_systems + 64));
    char* f = take(sizeof(int) * (size_t)max_systems);
    char* ef = take(sizeof(int) * (size_t)max_systems);
    char* s = take(sizeof(int) * 4);
    char* en = take(sizeof(double) * 3 * (size_t)max_systems);
    if (e) {
        e->d_table = (SysDev*)t;
        e->d_prefix = (int*)p;
        e->d_prefix2 = (int*)p2;
        e->d_flags = (int*)f;
        e->d_eflags = (int*)ef;
        e->d_status = (int*)s;
        e->d_energy = (double*)en;
    }
    return off + 256;
}

void drop_graph(nb_ens* e)
{
    if (e->graph_ok) {
        hipGraphExecDestroy(e->gexec);
        hipGraphDestroy(e->graph);
        e->graph_ok = false;
    }
}

nb_status refresh_table(nb_ens* e)
{
    const int n = (int)e->members.size();
    // order members by kernel class so each class is a contiguous table range
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto key = [&](int i) {
        const nb_sys* s = e->members[i];
        return std::make_tuple(s->M, s->p.coulomb, s->p.lj, (int)((s->p.flags & NB_FP32_REDUCE) != 0));
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    std::vector<nb_sys*> m2(n);
    std::vector<double*> x2(n), v2(n);
    std::vector<float*> f2(n);
    for (int i = 0; i < n; ++i) {
        m2[i] = e->members[order[i]];
        x2[i] = e->xs[order[i]];
        v2[i] = e->vs[order[i]];
        f2[i] = e->fs[order[i]];
    }
    e->members.swap(m2);
    e->xs.swap(x2);
    e->vs.swap(v2);
    e->fs.swap(f2);
    e->h_table.resize(n);
    e->classes.clear();
    e->bounds = Bounds{0, 0, 0, 0, 0, false, true};
    int poff = 0;
    for (int i = 0; i < n; ++i) {
        nb_sys* s = e->members[i];
        s->h.x = e->xs[i];
        s->h.v = e->vs[i];
        s->h.f = e->fs[i];
        e->h_table[i] = s->h;
        e->bounds.max_atoms = std::max(e->bounds.max_atoms, s->bounds.max_atoms);
        e->bounds.max_cols = std::max(e->bounds.max_cols, s->bounds.max_cols);
        e->bounds.max_groups = std::max(e->bounds.max_groups, s->bounds.max_groups);
        e->bounds.max_slots = std::max(e->bounds.max_slots, s->bounds.max_slots);
        e->bounds.max_ent = std::max(e->bounds.max_ent, s->bounds.max_ent);
        e->bounds.any_tric = e->bounds.any_tric || s->bounds.any_tric;
        e->bounds.all_m8 = e->bounds.all_m8 && s->bounds.all_m8;
        const bool fp32 = (s->p.flags & NB_FP32_REDUCE) != 0;
        if (e->classes.empty() || e->classes.back().M != s->M || e->classes.back().coul != s->p.coulomb ||
            e->classes.back().lj != s->p.lj || e->classes.back().fp32 != (int)fp32) {
            EnsClass c;
            c.M = s->M;
            c.coul = s->p.coulomb;
            c.lj = s->p.lj;
            c.fp32 = fp32;
            c.off = i;
            c.cnt = 0;
            c.item_cap = 0;
            c.prefix_off = poff;
            e->classes.push_back(c);
        }
        EnsClass& c = e->classes.back();
        c.cnt += 1;
        c.item_cap += s->item_cap;
        poff = c.prefix_off + c.cnt + 1;
    }
    if (n > 0)
        HIPCHK(e->ctx, hipMemcpyAsync(e->d_table, e->h_table.data(), sizeof(SysDev) * n, hipMemcpyHostToDevice,
                                      e->ctx->stream));
    HIPCHK(e->ctx, hipStreamSynchronize(e->ctx->stream));
    drop_graph(e);
    e->dirty = false;
    return NB_OK;
}

// item prefixes per kernel class into `prefix`; flags (NULL = all): members
// with flag 0 get no items
nb_status ens_prefixes(nb_ens* e, hipStream_t st, int* prefix = nullptr, const int* flags = nullptr)
{
    if (!prefix) prefix = e->d_prefix;
    for (const EnsClass& c : e->classes)
        HIPCHK(e->ctx, launch_item_prefix(e->d_table + c.off, c.cnt, prefix + c.prefix_off, st,
                                          flags ? flags + c.off : nullptr));
    return NB_OK;
}

// faults: also report saturated / non-finite members (end of a call); a
// rebuild inside the call checks capacity only, so every member still takes
// all the steps of the call and a failing one can be isolated afterwards.
// over (may be NULL): per member, whether its list ran out of capacity (each
// such member gets its needed arena size and loses its list)
nb_status ens_check(nb_ens* e, bool faults, std::vector<char>* over = nullptr)
{
    int st[2];
    hipStream_t s = e->ctx->stream;
    const int n = (int)e->members.size();
    if (over) over->assign(n, 0);
    HIPCHK(e->ctx, launch_ens_status(e->d_table, n, e->d_status, s));
    HIPCHK(e->ctx, hipMemcpyAsync(st, e->d_status, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(e->ctx, hipStreamSynchronize(s));
    if (st[0]) {
        // the members that overflowed, with their needed sizes
        std::string who;
        for (int i = 0; i < n; ++i) {
            nb_sys* m = e->members[i];
            int stv[ST_COUNT];
            nb_status r = nbh::read_status(m, stv);
            if (r) return r;
            if (stv[ST_OVERFLOW]) {
                nbh::capacity_error(m, stv);
                if (over) (*over)[i] = 1;
                if (who.empty()) who = m->ctx->err;
            }
        }
        return nbh::fail(e->ctx, NB_ERR_CAPACITY, "ensemble member pair-list capacity exceeded: " + who);
    }
    if (faults && st[1])
        return nbh::fail(e->ctx, NB_ERR_NONFINITE, "non-finite position or force beyond the fixed-point range in an ensemble member");
    return NB_OK;
}

// one step without list rebuild (the graph body): the same kernel sequence as
// md_step's plain step, so members evolve bitwise as they would alone
nb_status ens_plain_step(nb_ens* e, hipStream_t st, double dt, bool ener)
{
    const int n = (int)e->members.size();
    HIPCHK(e->ctx, launch_kick_drift_stage(e->d_table, n, e->bounds, dt, st));
    for (const EnsClass& c : e->classes)
        HIPCHK(e->ctx, launch_force(e->d_table + c.off, c.cnt, e->d_prefix + c.prefix_off, c.M, c.coul, c.lj, ener,
                                    0, c.item_cap, st));
    HIPCHK(e->ctx, launch_gather_kick(e->d_table, n, e->bounds, dt, ener, st));
    return NB_OK;
}

// F(x) for the members with need[i] != 0 (the others keep their forces)
nb_status ens_forces(nb_ens* e, hipStream_t st, const std::vector<int>& need)
{
    const int n = (int)e->members.size();
    e->h_eflags = need;  // (every call ends with a synchronisation, after which it may change)
    HIPCHK(e->ctx, hipMemcpyAsync(e->d_eflags, e->h_eflags.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIPCHK(e->ctx, launch_stage(e->d_table, n, e->bounds, st, e->d_eflags));
    nb_status r = ens_prefixes(e, st, e->d_prefix2, e->d_eflags);
    if (r) return r;
    for (const EnsClass& c : e->classes)
        HIPCHK(e->ctx, launch_force(e->d_table + c.off, c.cnt, e->d_prefix2 + c.prefix_off, c.M, c.coul, c.lj,
                                    false, 0, c.item_cap, st));
    HIPCHK(e->ctx, launch_finalize(e->d_table, n, e->bounds, false, st, e->d_eflags));
    return NB_OK;
}

// exact: FP64 masks; otherwise as md_step builds (the search's FP32 atom-pair
// prune decides the list)
nb_status ens_build(nb_ens* e, const std::vector<int>& flags, bool exact)
{
    const int n = (int)e->members.size();
    hipStream_t st = e->ctx->stream;
    // per member: 0 = not rebuilt, 1 = rebuilt (list-buffer guard measured),
    // 2 = first build (positions only recorded)
    std::vector<int> mode(n, 0);
    for (int i = 0; i < n; ++i)
        if (flags[i]) mode[i] = e->members[i]->list_valid ? 1 : 2;
    HIPCHK(e->ctx, hipMemcpyAsync(e->d_flags, mode.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIPCHK(e->ctx, launch_build(e->d_table, n, e->bounds, e->d_flags, st, exact, 2));
    nb_status r = ens_prefixes(e, st);
    if (r) return r;
    // (synchronises, so `mode` outlives its upload)
    std::vector<char> over;
    r = ens_check(e, false, &over);
    if (r && r != NB_ERR_CAPACITY) return r;
    // members whose build fitted hold a valid list even if another member's did not
    for (int i = 0; i < n; ++i)
        if (flags[i] && !over[i]) {
            e->members[i]->list_valid = true;
            e->members[i]->list_exact = exact;
        }
    return r;
}

}  // namespace

extern "C" {

nb_status nb_ens_arena_bytes(int32_t max_systems, size_t* bytes)
{
    if (max_systems < 1 || !bytes) return nbh::fail(nullptr, NB_ERR_ARG, "bad arguments");
    *bytes = ens_layout(max_systems, nullptr, nullptr);
    return NB_OK;
}

nb_status nb_ens_create(nb_ctx* ctx, int32_t max_systems, void* dev_arena, size_t arena_bytes, nb_ens** out)
{
    if (!ctx || !out || !dev_arena || max_systems < 1) return nbh::fail(ctx, NB_ERR_ARG, "bad arguments");
    *out = nullptr;
    const size_t need = ens_layout(max_systems, nullptr, nullptr);
    if (arena_bytes < need) return nbh::fail(ctx, NB_ERR_CAPACITY, "ensemble arena too small");
    nb_ens* e = new nb_ens;
    e->ctx = ctx;
    e->max_systems = max_systems;
    e->arena = dev_arena;
    e->arena_bytes = arena_bytes;
    char* base = (char*)(((uintptr_t)dev_arena + 255) & ~uintptr_t(255));
    ens_layout(max_systems, base, e);
    e->dirty = true;
    e->graph_ok = false;
    e->graph_dt = 0.0;
    e->bounds = Bounds{0, 0, 0, 0, 0, false, true};
    hipError_t err = hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking);
    if (err != hipSuccess) {
        delete e;
        return nbh::fail(ctx, NB_ERR_DEVICE, hipGetErrorString(err));
    }
    *out = e;
    return NB_OK;
}

nb_status nb_ens_destroy(nb_ens* e)
{
    if (!e) return nbh::fail(nullptr, NB_ERR_ARG, "ens is NULL");
    hipStreamSynchronize(e->ctx->stream);
    drop_graph(e);
    hipStreamDestroy(e->cap_stream);
    for (nb_sys* m : e->members) m->ens = nullptr;
    delete e;
    return NB_OK;
}

nb_status nb_ens_add(nb_ens* e, nb_sys* s, double* x_dev, double* v_dev, float* f_dev)
{
    if (!e || !s || !x_dev || !v_dev || !f_dev) return nbh::fail(e ? e->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    if ((int)e->members.size() >= e->max_systems) return nbh::fail(e->ctx, NB_ERR_CAPACITY, "ensemble is full");
    if (s->ens) return nbh::fail(e->ctx, NB_ERR_STATE, "system already belongs to an ensemble");
    if (s->ctx->stream != e->ctx->stream) return nbh::fail(e->ctx, NB_ERR_ARG, "system on another stream");
    if (!s->has_particles || !s->has_mass) return nbh::fail(e->ctx, NB_ERR_STATE, "particles/masses not set");
    if (s->pme_on) return nbh::fail(e->ctx, NB_ERR_ARG, "ensemble members run without PME (pme_grid must be zero)");
    e->members.push_back(s);
    e->xs.push_back(x_dev);
    e->vs.push_back(v_dev);
    e->fs.push_back(f_dev);
    s->ens = e;
    s->list_valid = false;  // the member's list is rebuilt inside the ensemble
    s->f_current = false;
    e->dirty = true;
    return NB_OK;
}

nb_status nb_ens_remove(nb_ens* e, nb_sys* s)
{
    if (!e || !s) return nbh::fail(e ? e->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    auto it = std::find(e->members.begin(), e->members.end(), s);
    if (it == e->members.end()) return nbh::fail(e->ctx, NB_ERR_ARG, "not a member");
    const size_t i = it - e->members.begin();
    HIPCHK(e->ctx, hipStreamSynchronize(e->ctx->stream));
    e->members.erase(e->members.begin() + i);
    e->xs.erase(e->xs.begin() + i);
    e->vs.erase(e->vs.begin() + i);
    e->fs.erase(e->fs.begin() + i);
    s->ens = nullptr;
    s->f_current = false;
    e->dirty = true;
    return NB_OK;
}

nb_status nb_ens_size(const nb_ens* e, int32_t* n)
{
    if (!e || !n) return nbh::fail(nullptr, NB_ERR_ARG, "NULL argument");
    *n = (int32_t)e->members.size();
    return NB_OK;
}

nb_status nb_ens_step(nb_ens* e, int32_t n_steps, double dt, int32_t nstlist, int32_t use_graph,
                      double* energies_host)
{
    if (!e || n_steps < 0 || !(dt > 0.0) || nstlist < 1) return nbh::fail(e ? e->ctx : nullptr, NB_ERR_ARG, "bad arguments");
    const int n = (int)e->members.size();
    if (n == 0) return NB_OK;
    nbh::Range range("nb ensemble step");
    nb_status r;
    if (e->dirty) {
        r = refresh_table(e);
        if (r) return r;
    }
    hipStream_t st = e->ctx->stream;
    HIPCHK(e->ctx, launch_clear_status(e->d_table, n, st));
    // lists for members that have none, then F(x) for the members whose forces
    // are not those of their current positions and list (new members, lists
    // dropped since); the others keep the forces their last step left, so a
    // member continues exactly as within one call
    std::vector<int> flags(n, 0), need(n, 0);
    bool any = false, any_need = false;
    for (int i = 0; i < n; ++i) {
        nb_sys* m = e->members[i];
        if (!m->list_valid) {
            flags[i] = 1;
            any = true;
        }
        need[i] = (!m->list_valid || !m->f_current) ? 1 : 0;
        any_need = any_need || need[i];
    }
    if (any) {
        r = ens_build(e, flags, false);
        if (r) return r;
    } else {
        r = ens_prefixes(e, st);
        if (r) return r;
    }
    if (any_need) {
        r = ens_forces(e, st, need);
        if (r) return r;
    }
    for (nb_sys* m : e->members) m->f_current = true;
    if (use_graph && (!e->graph_ok || e->graph_dt != dt)) {
        drop_graph(e);
        // capture the plain step on a private stream, replay on the context stream
        HIPCHK(e->ctx, hipStreamSynchronize(st));
        HIPCHK(e->ctx, hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
        nb_status rc = ens_plain_step(e, e->cap_stream, dt, false);
        hipGraph_t g;
        hipError_t ce = hipStreamEndCapture(e->cap_stream, &g);
        if (rc) return rc;
        if (ce != hipSuccess) return nbh::fail(e->ctx, NB_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        hipError_t ie = hipGraphInstantiate(&e->gexec, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            hipGraphDestroy(g);
            return nbh::fail(e->ctx, NB_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
        }
        e->graph = g;
        e->graph_ok = true;
        e->graph_dt = dt;
    }
    for (int32_t k = 0; k < n_steps; ++k) {
        const bool last = (k == n_steps - 1);
        const bool ener = last && energies_host;
        bool rebuild = false;
        for (int i = 0; i < n; ++i) {
            flags[i] = ((e->members[i]->step + 1) % nstlist == 0) ? 1 : 0;
            rebuild = rebuild || flags[i];
        }
        if (!rebuild && !ener && use_graph) {
            HIPCHK(e->ctx, hipGraphLaunch(e->gexec, st));
        } else if (!rebuild) {
            r = ens_plain_step(e, st, dt, ener);
            if (r) return r;
        } else {
            // members due for a rebuild move first, are rebuilt and staged; the
            // others take the fused plain step (flags select per member).  The
            // full-step x, v of every member are kept: if a rebuild runs out of
            // capacity, the whole batch goes back to this step, so every member
            // stops at the same step with its state intact (forces and, for the
            // members whose rebuild fitted, a list that the repeated step
            // rebuilds identically) and the call reports NB_ERR_CAPACITY
            HIPCHK(e->ctx, launch_state_copy(e->d_table, n, e->bounds, 0, st));
            HIPCHK(e->ctx, launch_kick_drift(e->d_table, n, e->bounds, dt, st));
            r = ens_build(e, flags, false);
            if (r == NB_ERR_CAPACITY) {
                HIPCHK(e->ctx, launch_state_copy(e->d_table, n, e->bounds, 1, st));
                HIPCHK(e->ctx, hipStreamSynchronize(st));
                // the members that overflowed lost their list (and need a force
                // pass once rebuilt); the others' forces are those of their x
                for (nb_sys* m : e->members) m->f_current = m->list_valid;
                return r;
            }
            if (r) return r;
            HIPCHK(e->ctx, launch_stage(e->d_table, n, e->bounds, st));
            for (const EnsClass& c : e->classes)
                HIPCHK(e->ctx, launch_force(e->d_table + c.off, c.cnt, e->d_prefix + c.prefix_off, c.M, c.coul, c.lj,
                                            ener, 0, c.item_cap, st));
            HIPCHK(e->ctx, launch_gather_kick(e->d_table, n, e->bounds, dt, ener, st));
        }
        for (int i = 0; i < n; ++i) e->members[i]->step += 1;
    }
    if (energies_host && n_steps > 0) {
        HIPCHK(e->ctx, launch_energy_reduce(e->d_table, n, -1, true, 0.0, st));
        hipLaunchKernelGGL(k_ens_energy, dim3((n + 255) / 256), dim3(256), 0, st, e->d_table, n, e->d_energy);
        HIPCHK(e->ctx, hipGetLastError());
        std::vector<double> buf((size_t)3 * n);
        HIPCHK(e->ctx, hipMemcpyAsync(buf.data(), e->d_energy, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, st));
        HIPCHK(e->ctx, hipStreamSynchronize(st));
        // back to the caller's member order is the table order: report per table entry
        std::memcpy(energies_host, buf.data(), sizeof(double) * 3 * n);
    }
    return ens_check(e, true);
}

// index of a member in the ensemble's current (class-sorted) order
nb_status nb_ens_member_index(const nb_ens* e, const nb_sys* s, int32_t* idx)
{
    if (!e || !s || !idx) return nbh::fail(nullptr, NB_ERR_ARG, "NULL argument");
    auto it = std::find(e->members.begin(), e->members.end(), s);
    if (it == e->members.end()) return nbh::fail(e->ctx, NB_ERR_ARG, "not a member");
    *idx = (int32_t)(it - e->members.begin());
    return NB_OK;
}

nb_status nb_autotune(nb_sys* sys, const double* x_dev, float* f_dev, void* scratch_dev, size_t scratch_bytes,
                      const int32_t* clusters, int32_t n_clusters, const int32_t* jtiles, int32_t n_jtiles,
                      int32_t reps, int32_t* best_cluster, int32_t* best_jtile, double* best_us)
{
    if (!sys || !x_dev || !f_dev || !scratch_dev || !clusters || !jtiles || n_clusters < 1 || n_jtiles < 1 ||
        reps < 1 || !best_cluster || !best_jtile)
        return nbh::fail(sys ? sys->ctx : nullptr, NB_ERR_ARG, "bad arguments");
    hipStream_t st = sys->ctx->stream;
    hipEvent_t e0, e1;
    HIPCHK(sys->ctx, hipEventCreate(&e0));
    HIPCHK(sys->ctx, hipEventCreate(&e1));
    double best = 1e300;
    int bc = -1, bj = -1;
    float* fdev = f_dev;
    for (int ic = 0; ic < n_clusters; ++ic)
        for (int ij = 0; ij < n_jtiles; ++ij) {
            nb_params p = sys->p;
            p.cluster = clusters[ic];
            p.jtile = jtiles[ij];
            size_t need = 0;
            if (nb_arena_bytes(&p, &need) != NB_OK || need > scratch_bytes) continue;
            nb_sys* t = nullptr;
            if (nb_sys_create(sys->ctx, &p, scratch_dev, scratch_bytes, &t) != NB_OK) continue;
            nb_status r = nb_sys_set_particles(t, sys->q.data(), sys->sig.data(), sys->eps.data(),
                                               sys->has_mass ? sys->mass.data() : nullptr);
            if (r == NB_OK) r = nb_build_pairlist(t, x_dev);
            if (r == NB_OK) {
                t->h.f = fdev;
                r = nbh::upload_desc(t);
            }
            if (r == NB_OK) {
                // warm-up, then time `reps` force evaluations
                nbh::eval_forces(t, false, -1, false, 0.0);
                hipEventRecord(e0, st);
                for (int k = 0; k < reps; ++k) nbh::eval_forces(t, false, -1, false, 0.0);
                hipEventRecord(e1, st);
                hipEventSynchronize(e1);
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                const double us = 1000.0 * ms / reps;
                if (us < best) {
                    best = us;
                    bc = p.cluster;
                    bj = p.jtile;
                }
            }
            nb_sys_destroy(t);
        }
    hipStreamSynchronize(st);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (bc < 0) return nbh::fail(sys->ctx, NB_ERR_CAPACITY, "no candidate fitted the scratch arena");
    *best_cluster = bc;
    *best_jtile = bj;
    if (best_us) *best_us = best;
    return NB_OK;
}

}  // extern "C"
