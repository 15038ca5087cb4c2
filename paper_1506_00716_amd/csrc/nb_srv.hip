// nb_srv.hip -- continuous-batching MD job server (host runtime, C++).
//
// The paper runs many independent simulations under an ensemble controller
// that keeps every run going to completion (Section "Ensemble simulations").
// Here one GPU serves a stream of MD jobs: a host thread admits queued jobs
// while the device memory budget and the slot count allow, joins them to the
// running batch at the next list-rebuild boundary, advances the whole batch
// with the ensemble kernels (graph replay between rebuilds), and retires jobs
// as they reach their step counts, copying results back and freeing memory.
// Coordinates, velocities, forces and pair lists stay resident on the device
// for the life of the job.  Each job's arithmetic depends only on its own data,
// so its result is bitwise the same alone and in any mix.
#include "nb_host.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace {

using Clock = std::chrono::steady_clock;

// first-fit allocator over the caller's device pool (256-byte granules)
struct Pool {
    char* base = nullptr;
    size_t bytes = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    void init(void* b, size_t n)
    {
        char* a = (char*)(((uintptr_t)b + 255) & ~uintptr_t(255));
        base = a;
        bytes = n - (size_t)(a - (char*)b);
        bytes &= ~size_t(255);
        free_.clear();
        free_[0] = bytes;
    }
    static size_t round(size_t n) { return (n + 255) & ~size_t(255); }
    void* alloc(size_t n)
    {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                const size_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > n) free_[off + n] = sz - n;
                return base + off;
            }
        return nullptr;
    }
    void release(void* p, size_t n)
    {
        n = round(n);
        size_t off = (size_t)((char*)p - base);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Job {
    uint64_t id;
    nb_params p;
    int32_t n_steps;
    std::vector<double> x, v, q, sig, eps, mass;
    int32_t state;  // 0 queued, 1 running, 2 done, 3 failed, 4 rejected
    nb_status error;
    double t_submit, t_admit, t_done;
    double energies[3];
    // device residency
    void* block;
    size_t block_bytes;
    nb_sys* sys;
    double* dx;
    double* dv;
    float* df;
    int64_t steps_done;
};

}  // namespace

struct nb_srv {
    nb_ctx* ctx;
    hipStream_t stream;
    nb_ens* ens;
    void* ens_arena;
    Pool pool;
    int max_slots;
    double dt;
    int nstlist;
    int use_graph;
    std::mutex mu;
    std::condition_variable cv, cv_idle;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Job*> jobs;
    std::vector<Job*> active;
    uint64_t next_id;
    bool stop;
    std::thread worker;
    Clock::time_point t0;
    int64_t global_step;
    double atom_steps, busy_s;
    int64_t n_done, n_failed, n_rejected;
    std::string err;
};

namespace {

double now_s(const nb_srv* s) { return std::chrono::duration<double>(Clock::now() - s->t0).count(); }

size_t job_bytes(const nb_params& p)
{
    size_t a = 0;
    nb_arena_bytes(&p, &a);
    const size_t N = (size_t)p.n_atoms;
    // arena with headroom for density fluctuations, then x, v (FP64) and f (FP32)
    return Pool::round(a + a / 4) + Pool::round(24 * N) * 2 + Pool::round(12 * N) + 1024;
}

// admit one queued job onto the device (called by the worker, lock held by caller)
bool admit(nb_srv* s, Job* j)
{
    const size_t need = job_bytes(j->p);
    void* blk = s->pool.alloc(need);
    if (!blk) return false;
    j->block = blk;
    j->block_bytes = need;
    size_t a = 0;
    nb_arena_bytes(&j->p, &a);
    a = Pool::round(a + a / 4);
    const size_t N = (size_t)j->p.n_atoms;
    char* c = (char*)blk;
    j->dx = (double*)(c + a);
    j->dv = (double*)(c + a + Pool::round(24 * N));
    j->df = (float*)(c + a + 2 * Pool::round(24 * N));
    nb_status r = nb_sys_create(s->ctx, &j->p, blk, a, &j->sys);
    if (r == NB_OK)
        r = nb_sys_set_particles(j->sys, j->q.data(), j->sig.empty() ? nullptr : j->sig.data(),
                                 j->eps.empty() ? nullptr : j->eps.data(), j->mass.data());
    if (r == NB_OK && hipMemcpyAsync(j->dx, j->x.data(), 24 * N, hipMemcpyHostToDevice, s->stream) != hipSuccess)
        r = NB_ERR_DEVICE;
    if (r == NB_OK && hipMemcpyAsync(j->dv, j->v.data(), 24 * N, hipMemcpyHostToDevice, s->stream) != hipSuccess)
        r = NB_ERR_DEVICE;
    if (r == NB_OK && hipMemsetAsync(j->df, 0, 12 * N, s->stream) != hipSuccess) r = NB_ERR_DEVICE;
    if (r == NB_OK) r = nb_ens_add(s->ens, j->sys, j->dx, j->dv, j->df);
    if (r != NB_OK) {
        if (j->sys) nb_sys_destroy(j->sys);
        j->sys = nullptr;
        s->pool.release(blk, need);
        j->block = nullptr;
        j->state = 3;
        j->error = r;
        j->t_done = now_s(s);
        s->n_failed++;
        return true;  // consumed (failed)
    }
    j->state = 1;
    j->t_admit = now_s(s);
    j->steps_done = 0;
    s->active.push_back(j);
    return true;
}

// A job whose list outgrew its arena (a build inside the batch ran out of
// capacity; the batch then stopped at the job's last full step): move it to a
// block with the arena size the library asked for, state copied over, and put
// it back in the batch, where its list is rebuilt at its current positions --
// what a lone run does when it grows its arena.  False if the pool has no room.
bool regrow(nb_srv* s, Job* j)
{
    size_t need = 0;
    if (nb_sys_needed_bytes(j->sys, &need) != NB_OK) return false;
    const size_t N = (size_t)j->p.n_atoms;
    const size_t a = Pool::round(need);
    const size_t total = a + 2 * Pool::round(24 * N) + Pool::round(12 * N) + 1024;
    void* blk = s->pool.alloc(total);
    if (!blk) return false;
    char* c = (char*)blk;
    double* dx = (double*)(c + a);
    double* dv = (double*)(c + a + Pool::round(24 * N));
    float* df = (float*)(c + a + 2 * Pool::round(24 * N));
    bool ok = hipMemcpyAsync(dx, j->dx, 24 * N, hipMemcpyDeviceToDevice, s->stream) == hipSuccess &&
              hipMemcpyAsync(dv, j->dv, 24 * N, hipMemcpyDeviceToDevice, s->stream) == hipSuccess &&
              hipMemcpyAsync(df, j->df, 12 * N, hipMemcpyDeviceToDevice, s->stream) == hipSuccess;
    nb_ens_remove(s->ens, j->sys);  // (synchronises the stream)
    ok = ok && nb_sys_set_arena(j->sys, blk, a) == NB_OK;
    if (!ok) {
        hipStreamSynchronize(s->stream);
        s->pool.release(blk, total);
        return false;
    }
    s->pool.release(j->block, j->block_bytes);
    j->block = blk;
    j->block_bytes = total;
    j->dx = dx;
    j->dv = dv;
    j->df = df;
    return nb_ens_add(s->ens, j->sys, dx, dv, df) == NB_OK;
}

void retire(nb_srv* s, Job* j, int32_t state, nb_status err)
{
    const size_t N = (size_t)j->p.n_atoms;
    if (state == 2) {
        hipMemcpyAsync(j->x.data(), j->dx, 24 * N, hipMemcpyDeviceToHost, s->stream);
        hipMemcpyAsync(j->v.data(), j->dv, 24 * N, hipMemcpyDeviceToHost, s->stream);
        hipStreamSynchronize(s->stream);
    }
    nb_ens_remove(s->ens, j->sys);
    nb_sys_destroy(j->sys);
    j->sys = nullptr;
    s->pool.release(j->block, j->block_bytes);
    j->block = nullptr;
    j->state = state;
    j->error = err;
    j->t_done = now_s(s);
    if (state == 2) s->n_done++; else s->n_failed++;
}

void worker_loop(nb_srv* s)
{
    hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        // an empty batch has no phase: move the clock to the next boundary
        if (s->active.empty() && s->global_step % s->nstlist != 0)
            s->global_step += s->nstlist - s->global_step % s->nstlist;
        // admissions only at list-rebuild boundaries of the global clock, so every
        // member of the batch rebuilds at the same steps
        if (s->global_step % s->nstlist == 0) {
            while (!s->queue.empty() && (int)s->active.size() < s->max_slots) {
                Job* j = s->jobs[s->queue.front()];
                if (!admit(s, j)) break;  // no memory now: wait for a retirement (FIFO)
                s->queue.pop_front();
            }
        }
        if (s->active.empty()) {
            s->cv_idle.notify_all();
            if (!s->queue.empty()) {
                // nothing running and the head job does not fit: it never will
                Job* j = s->jobs[s->queue.front()];
                s->queue.pop_front();
                j->state = 4;
                j->error = NB_ERR_CAPACITY;
                j->t_done = now_s(s);
                s->n_rejected++;
                continue;
            }
            s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
            continue;
        }
        int64_t chunk = s->nstlist - (s->global_step % s->nstlist);
        for (Job* j : s->active) chunk = std::min<int64_t>(chunk, j->n_steps - j->steps_done);
        const bool last_for_some = [&] {
            for (Job* j : s->active)
                if (j->steps_done + chunk >= j->n_steps) return true;
            return false;
        }();
        std::vector<double> en(3 * s->active.size());
        std::vector<int64_t> before(s->active.size());
        for (size_t k = 0; k < s->active.size(); ++k) before[k] = s->active[k]->sys->step;
        lk.unlock();
        const double tb = now_s(s);
        nb_status r = nb_ens_step(s->ens, (int32_t)chunk, s->dt, s->nstlist, s->use_graph,
                                  last_for_some ? en.data() : nullptr);
        const double te = now_s(s);
        lk.lock();
        s->busy_s += te - tb;
        // the steps each member took (all of the chunk, or fewer if a list
        // build ran out of capacity and the batch stopped at the last full step);
        // the members move in lockstep, so the clock follows them
        int64_t adv = 0;
        for (size_t k = 0; k < s->active.size(); ++k) {
            Job* j = s->active[k];
            const int64_t d = j->sys->step - before[k];
            j->steps_done += d;
            s->atom_steps += (double)d * j->p.n_atoms;
            adv = std::max(adv, d);
        }
        s->global_step += adv;
        std::vector<Job*> keep;
        std::map<Job*, int32_t> row;  // energy rows in the batch order of this chunk
        if (last_for_some && r == NB_OK)
            for (Job* j : s->active) {
                int32_t idx = 0;
                nb_ens_member_index(s->ens, j->sys, &idx);
                row[j] = idx;
            }
        if (r != NB_OK) {
            // isolate: fail the members whose forces or positions went bad, move
            // the ones whose list outgrew its arena to a larger block (or fail
            // them if the pool has no room), keep the rest as they are
            s->err = nb_last_error(s->ctx);
            std::vector<Job*> ok;
            bool attributed = false;
            for (Job* j : s->active) {
                int st[8] = {0};
                hipMemcpy(st, j->sys->h.status, sizeof(st), hipMemcpyDeviceToHost);
                if (st[5] || st[7]) {
                    retire(s, j, 3, r);
                    attributed = true;
                } else if (st[0]) {
                    attributed = true;
                    if (regrow(s, j)) ok.push_back(j);
                    else retire(s, j, 3, NB_ERR_CAPACITY);
                } else {
                    ok.push_back(j);
                }
            }
            if (!attributed) {  // not attributable: fail everyone
                for (Job* j : ok) retire(s, j, 3, r);
                ok.clear();
            }
            s->active.swap(ok);
        }
        for (Job* j : s->active) {
            if (j->steps_done >= j->n_steps) {
                if (last_for_some && r == NB_OK)
                    for (int k = 0; k < 3; ++k) j->energies[k] = en[3 * row[j] + k];
                retire(s, j, 2, NB_OK);
            } else {
                keep.push_back(j);
            }
        }
        s->active.swap(keep);
    }
}

}  // namespace

extern "C" {

nb_status nb_srv_create(nb_ctx* ctx, void* pool_dev, size_t pool_bytes, void* ens_arena_dev, size_t ens_arena_bytes,
                        int32_t max_slots, double dt_ps, int32_t nstlist, int32_t use_graph, nb_srv** out)
{
    if (!ctx || !pool_dev || !ens_arena_dev || !out || max_slots < 1 || !(dt_ps > 0.0) || nstlist < 1)
        return nbh::fail(ctx, NB_ERR_ARG, "bad nb_srv_create arguments");
    *out = nullptr;
    nb_srv* s = new nb_srv;
    s->ctx = new nb_ctx;
    s->ctx->device = ctx->device;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        delete s->ctx;
        delete s;
        return nbh::fail(ctx, NB_ERR_DEVICE, "stream creation failed");
    }
    s->ctx->stream = s->stream;
    nb_status r = nb_ens_create(s->ctx, max_slots, ens_arena_dev, ens_arena_bytes, &s->ens);
    if (r != NB_OK) {
        hipStreamDestroy(s->stream);
        delete s->ctx;
        delete s;
        return nbh::fail(ctx, r, "ensemble creation failed");
    }
    s->ens_arena = ens_arena_dev;
    s->pool.init(pool_dev, pool_bytes);
    s->max_slots = max_slots;
    s->dt = dt_ps;
    s->nstlist = nstlist;
    s->use_graph = use_graph;
    s->next_id = 1;
    s->stop = false;
    s->t0 = Clock::now();
    s->global_step = 0;
    s->atom_steps = 0.0;
    s->busy_s = 0.0;
    s->n_done = s->n_failed = s->n_rejected = 0;
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return NB_OK;
}

nb_status nb_srv_submit(nb_srv* s, const nb_params* p, const double* x, const double* v, const double* q,
                        const double* sigma, const double* epsilon, const double* mass, int32_t n_steps,
                        uint64_t* job_id)
{
    if (!s || !p || !x || !v || !q || !mass || n_steps < 1 || !job_id)
        return nbh::fail(nullptr, NB_ERR_ARG, "bad nb_srv_submit arguments");
    size_t a = 0;
    nb_status r = nb_arena_bytes(p, &a);
    if (r != NB_OK) return r;
    if (p->lj == NB_LJ_LB && (!sigma || !epsilon)) return nbh::fail(nullptr, NB_ERR_ARG, "LB needs sigma/epsilon");
    if (p->pme_grid[0] || p->pme_grid[1] || p->pme_grid[2])
        return nbh::fail(nullptr, NB_ERR_ARG, "served jobs run without PME (pme_grid must be zero)");
    Job* j = new Job;
    const size_t N = (size_t)p->n_atoms;
    j->p = *p;
    j->n_steps = n_steps;
    j->x.assign(x, x + 3 * N);
    j->v.assign(v, v + 3 * N);
    j->q.assign(q, q + N);
    if (sigma) j->sig.assign(sigma, sigma + N);
    if (epsilon) j->eps.assign(epsilon, epsilon + N);
    j->mass.assign(mass, mass + N);
    j->state = 0;
    j->error = NB_OK;
    j->t_admit = j->t_done = -1.0;
    j->energies[0] = j->energies[1] = j->energies[2] = 0.0;
    j->block = nullptr;
    j->sys = nullptr;
    j->steps_done = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        j->id = s->next_id++;
        j->t_submit = now_s(s);
        if (job_bytes(*p) > s->pool.bytes) {
            j->state = 4;
            j->error = NB_ERR_CAPACITY;
            j->t_done = j->t_submit;
            s->n_rejected++;
        } else {
            s->queue.push_back(j->id);
        }
        s->jobs[j->id] = j;
        *job_id = j->id;
    }
    s->cv.notify_all();
    return NB_OK;
}

nb_status nb_srv_poll(nb_srv* s, uint64_t job_id, int32_t* state, double times[3], double energies[3],
                      nb_status* job_error)
{
    if (!s || !state) return nbh::fail(nullptr, NB_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return nbh::fail(nullptr, NB_ERR_ARG, "unknown job id");
    Job* j = it->second;
    *state = j->state;
    if (times) {
        times[0] = j->t_submit;
        times[1] = j->t_admit;
        times[2] = j->t_done;
    }
    if (energies)
        for (int k = 0; k < 3; ++k) energies[k] = j->energies[k];
    if (job_error) *job_error = j->error;
    return NB_OK;
}

nb_status nb_srv_fetch(nb_srv* s, uint64_t job_id, double* x_host, double* v_host)
{
    if (!s) return nbh::fail(nullptr, NB_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return nbh::fail(nullptr, NB_ERR_ARG, "unknown job id");
    Job* j = it->second;
    if (j->state != 2) return nbh::fail(nullptr, NB_ERR_STATE, "job not done");
    const size_t N = (size_t)j->p.n_atoms;
    if (x_host) std::memcpy(x_host, j->x.data(), 24 * N);
    if (v_host) std::memcpy(v_host, j->v.data(), 24 * N);
    return NB_OK;
}

nb_status nb_srv_release(nb_srv* s, uint64_t job_id)
{
    if (!s) return nbh::fail(nullptr, NB_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return nbh::fail(nullptr, NB_ERR_ARG, "unknown job id");
    if (it->second->state <= 1) return nbh::fail(nullptr, NB_ERR_STATE, "job still queued or running");
    delete it->second;
    s->jobs.erase(it);
    return NB_OK;
}

nb_status nb_srv_wait_idle(nb_srv* s, double timeout_s)
{
    if (!s) return nbh::fail(nullptr, NB_ERR_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->cv_idle.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                        [&] { return s->queue.empty() && s->active.empty(); });
    return ok ? NB_OK : nbh::fail(nullptr, NB_ERR_STATE, "server still busy at timeout");
}

nb_status nb_srv_stats(nb_srv* s, double out[8])
{
    if (!s || !out) return nbh::fail(nullptr, NB_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->atom_steps;
    out[1] = (double)s->n_done;
    out[2] = (double)s->n_failed;
    out[3] = (double)s->n_rejected;
    out[4] = s->busy_s;
    out[5] = now_s(s);
    out[6] = (double)s->active.size();
    out[7] = (double)s->queue.size();
    return NB_OK;
}

nb_status nb_srv_destroy(nb_srv* s)
{
    if (!s) return nbh::fail(nullptr, NB_ERR_ARG, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
    for (Job* j : s->active)
        if (j->sys) {
            nb_ens_remove(s->ens, j->sys);
            nb_sys_destroy(j->sys);
        }
    for (auto& kv : s->jobs) delete kv.second;
    nb_ens_destroy(s->ens);
    hipStreamSynchronize(s->stream);
    hipStreamDestroy(s->stream);
    delete s->ctx;
    delete s;
    return NB_OK;
}

}  // extern "C"
