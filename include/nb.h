/*
 * nb.h -- C ABI of libnb: short-range non-bonded forces for periodic molecular
 * dynamics on one AMD MI355X (gfx950), with the cluster-pair neighbour scheme.
 *
 * The method: atoms are placed on a grid in x and y and binned in z, grouped
 * into clusters of exactly M atoms, and a buffered list of cluster pairs whose
 * atoms may come within the interaction range is built once and reused over
 * several force evaluations (paper, Section "SIMD parallelism").  The kernel
 * evaluates all M x N atom pairs of a listed cluster pair at once, keeping the
 * i-cluster in registers (same section).  The problem statement -- positions
 * and velocities per particle, forces from the model physics, update by
 * Newton's second law with a finite time step -- is the paper's Section
 * "Introduction"; integrators take position, velocity and force vectors without
 * knowing the kernels (Section "C -> C++").
 *
 * Conventions for every call:
 *  - Units: nm, ps, amu, kJ/mol, elementary charge.  Boxes are rectangular or
 *    triclinic (nb_params.box_off).
 *  - Every call returns nb_status: NB_OK (0) or a negative error code.  No call
 *    throws or aborts across the ABI.  nb_last_error(ctx) returns a message for
 *    the last failure on that context (valid until the next call on it).
 *  - Arguments are validated before any work is enqueued; a call that fails
 *    validation has no side effects.
 *  - Device pointers ("_dev") are HIP device addresses owned by the caller; the
 *    library reads/writes them only inside work it enqueues on the context's
 *    stream.  Host pointers ("_host") are read or written before the call returns.
 *  - Calls enqueue asynchronously on the context's stream, except calls with host
 *    outputs, which synchronise the stream before returning.
 *  - One nb_ctx per stream; a context and everything created from it must be
 *    used from one host thread at a time.
 */
#ifndef NB_H
#define NB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nb_status;
enum {
    NB_OK = 0,
    NB_ERR_ARG = -1,       /* invalid argument (null pointer, size, mode) */
    NB_ERR_BOX = -2,       /* r_list >= half the smallest box edge, or bad box */
    NB_ERR_CAPACITY = -3,  /* arena or list capacity too small; nb_sys_needed_bytes tells the size */
    NB_ERR_DEVICE = -4,    /* HIP runtime error; message in nb_last_error */
    NB_ERR_NONFINITE = -5, /* non-finite force/energy, or a force beyond the fixed-point range */
    NB_ERR_BUFFER = -6,    /* list-buffer check: a pair inside r_cut was missing from the list */
    NB_ERR_STATE = -7      /* call out of order (e.g. forces before particles were set) */
};

enum { NB_COUL_NONE = 0, NB_COUL_RF = 1, NB_COUL_EWALD = 2 };
enum { NB_LJ_SINGLE = 0, NB_LJ_LB = 1 };

/* flags */
#define NB_POT_SHIFT 1u    /* shift LJ and Ewald pair energies to zero at r_cut (forces unshifted) */
#define NB_FP32_REDUCE 2u  /* precision variant V32: the per-atom force partials and the
                              per-system energy/virial sums are added in FP32 (positions and
                              velocities stay FP64).  Default V64r: the force partials are
                              added in int64 fixed point (exact, order-independent, bitwise
                              deterministic) and energies/virial in FP64.  No variant uses
                              atomics for forces: every partial has one writer. */

/*
 * Model and layout parameters of one system.
 *  n_atoms         number of atoms N >= 1
 *  box             the box's diagonal (nm), > 0: the edges L_x, L_y, L_z of a
 *                  rectangular box, or a_x, b_y, c_z of a triclinic one (box_off)
 *  r_cut, r_list   0 < r_cut <= r_list < min(box)/2 (else NB_ERR_BOX)
 *  coulomb         NB_COUL_NONE, NB_COUL_RF (reaction field) or NB_COUL_EWALD (real-space erfc)
 *  eps_r           relative dielectric constant (> 0)
 *  eps_rf          reaction-field dielectric; <= 0 means infinity
 *  ewald_beta      Ewald splitting parameter (nm^-1), > 0 for NB_COUL_EWALD
 *  lj              NB_LJ_SINGLE (c6, c12 below for every pair) or NB_LJ_LB (per-atom
 *                  sigma/epsilon with Lorentz-Berthelot mixing)
 *  c6, c12         single-type LJ coefficients (kJ/mol nm^6, kJ/mol nm^12)
 *  cluster         cluster size M = N: 0 (auto = 8), 1 (plain Verlet list), 4 or 8
 *  jtile           size of a force-kernel work item in list entries, 0 = auto (16 for
 *                  M = 8, 32 for M = 4, 128 for M = 1).  For M = 8 items are cut by
 *                  cost: an entry weighs 7 + 2 x the i-clusters it lists, an item
 *                  about 16 * jtile
 *  force_fixed_bits  fixed-point fraction bits of the V64r force sums, 0 = auto (20:
 *                  resolution ~1e-6 kJ/mol/nm); every force partial added to an atom
 *                  must stay below 2^(50 - bits) kJ/mol/nm (~1e9 at 20 bits), else the
 *                  call fails with NB_ERR_NONFINITE.  nb_minimize uses at most 12 bits.
 *  flags           NB_POT_SHIFT | NB_FP32_REDUCE
 *  r_inner, nstprune  dynamic list pruning (paper, Section "Heterogeneous
 *                  parallelization": the list is pruned on the GPU, so it can be kept
 *                  for many more steps with a larger buffer).  r_inner = 0: off.
 *                  Otherwise r_cut <= r_inner <= r_list, nstprune >= 1: md_step's
 *                  force pass of every nstprune-th step after a list build (the
 *                  build's own step included) keeps, per listed cluster pair, only
 *                  the i-clusters with an atom pair within r_inner at that step, and
 *                  the steps until the next prune evaluate only those.  A pruned
 *                  cluster pair has no pair inside r_cut unless two atoms moved by
 *                  (r_inner - r_cut)/2 each within the interval (counted by
 *                  nb_sys_buffer_stats), so forces are bitwise those of the unpruned
 *                  list.  Ensembles and the server run the full list.
 *  box_off         off-diagonal b_x, c_x, c_y (nm) of a triclinic box with lattice
 *                  vectors a = (box[0], 0, 0), b = (b_x, box[1], 0), c = (c_x, c_y,
 *                  box[2]) -- e.g. the rhombic dodecahedron the paper runs (Section
 *                  "Heterogeneous parallelization", Fig. 6): a = (d,0,0), b = (0,d,0),
 *                  c = (d/2, d/2, d/sqrt(2)).  All zero: rectangular.  Requires
 *                  |b_x| <= box[0]/2, |c_x| <= box[0]/2, |c_y| <= box[1]/2 (else
 *                  NB_ERR_BOX).  The minimum image removes the nearest multiples of c,
 *                  b, a from a displacement's z, y, x components in that order.
 *  pme_grid, pme_order  reciprocal-space Ewald by smooth particle-mesh Ewald, the
 *                  long-range lattice part that the paper computes beside the pair
 *                  forces (Section "Multi-level parallelism", Fig. 2; Section
 *                  "Heterogeneous parallelization"); here on the GPU.  pme_grid all
 *                  zero: off (coulomb then is the real-space pair term alone).
 *                  Otherwise coulomb must be NB_COUL_EWALD, pme_order 4 or 6 (0 =
 *                  4: cardinal B-splines of that order) and each pme_grid[k] (grid
 *                  points along lattice vector k) within [pme_order, 256]; a spacing
 *                  of about 0.12 nm suits beta ~ 3.1 nm^-1.  With PME on, forces,
 *                  E_coul and the virial of nb_compute_forces, md_step and
 *                  nb_minimize are the full Ewald sums: real space + reciprocal
 *                  space + the self term -f beta/sqrt(pi) sum q^2 + the neutralising
 *                  background -f pi (sum q)^2 / (2 V beta^2).  The reciprocal
 *                  influence function is left out at m = 0 and at the Nyquist
 *                  frequency of an even pme_grid[k].  Single systems only
 *                  (ensembles, the server and nb_compute_forces_noalloc return
 *                  NB_ERR_ARG for it).
 */
typedef struct {
    int32_t n_atoms;
    double box[3];
    double r_cut, r_list;
    int32_t coulomb;
    double eps_r, eps_rf, ewald_beta;
    int32_t lj;
    double c6, c12;
    int32_t cluster;
    int32_t jtile;
    int32_t force_fixed_bits;
    uint32_t flags;
    double r_inner;
    int32_t nstprune;
    double box_off[3];
    int32_t pme_grid[3];
    int32_t pme_order;
} nb_params;

typedef struct nb_ctx nb_ctx;
typedef struct nb_sys nb_sys;
typedef struct nb_ens nb_ens;
typedef struct nb_srv nb_srv;

/* Static description of a message code; never NULL. */
const char *nb_strerror(nb_status s);
/* Message of the last failure on ctx ("" if none); NULL ctx gives the last global message. */
const char *nb_last_error(const nb_ctx *ctx);

/* Create a context bound to HIP device `device` and the HIP stream `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  *out receives the handle. */
nb_status nb_ctx_create(int device, void *hip_stream, nb_ctx **out);
nb_status nb_ctx_destroy(nb_ctx *ctx);

/* Device memory a system needs for `p` (bytes, 256-aligned arena).  Host-only; the
 * list capacity inside is an estimate from the mean density: a build that
 * overflows it fails with NB_ERR_CAPACITY and nb_sys_needed_bytes reports the size. */
nb_status nb_arena_bytes(const nb_params *p, size_t *bytes);

/* Create a system on `dev_arena` (caller-owned device memory of `arena_bytes`,
 * 256-byte aligned, which must outlive the system and is never freed by it). */
nb_status nb_sys_create(nb_ctx *ctx, const nb_params *p, void *dev_arena, size_t arena_bytes,
                        nb_sys **out);
nb_status nb_sys_destroy(nb_sys *sys);
/* Arena size that the last failed build asked for (>= the current size). */
nb_status nb_sys_needed_bytes(const nb_sys *sys, size_t *bytes);
/* Move a system onto a new arena (e.g. a larger one after NB_ERR_CAPACITY).  The
 * pair list is discarded; particle data are re-uploaded from the system's host copy. */
nb_status nb_sys_set_arena(nb_sys *sys, void *dev_arena, size_t arena_bytes);

/* Per-atom data, host FP64 arrays of length N, copied before return:
 *  q        charges (e)
 *  sigma, epsilon  LJ parameters for NB_LJ_LB (ignored, may be NULL, for NB_LJ_SINGLE)
 *  mass     masses (amu, > 0); may be NULL if md_step is never called */
nb_status nb_sys_set_particles(nb_sys *sys, const double *q, const double *sigma,
                               const double *epsilon, const double *mass);

/* Build the cluster-pair list at positions x_dev (device FP64 [N,3], any periodic
 * image): grid binning in x/y, z sort, clusters of M atoms, bounding-box search
 * within r_list, and an exact FP64 atom-pair prune (paper, Sections "SIMD
 * parallelism" and "Heterogeneous parallelization").  Synchronises once to check
 * capacity (NB_ERR_CAPACITY). */
nb_status nb_build_pairlist(nb_sys *sys, const double *x_dev);

/* Export the exact atom-pair set of the current list: every unordered pair {i,j}
 * whose minimum-image distance at build time is below r_list, as (i, j) with i < j
 * (original indices), sorted lexicographically, into pairs_host[cap][2].  *n_pairs
 * receives the total count even if it exceeds cap.  Lists built inside md_step or
 * an ensemble keep the result of the build's conservative FP32 atom-pair prune on
 * the GPU (in the non-bonded kernel's frame; Section "Heterogeneous
 * parallelization") instead of the exact test; for those the exact FP64 masks are
 * computed here from the stored build positions, without changing the list the
 * forces run on.  Synchronises. */
nb_status nb_pairlist_export(nb_sys *sys, int32_t *pairs_host, int64_t cap, int64_t *n_pairs);

/* List statistics (host, synchronises): out[0] clusters, out[1] cluster-pair
 * entries, out[2] cluster pairs (entry x i-cluster bits), out[3] atom pairs within
 * r_list, out[4] evaluated pair slots per force call (cluster pairs x M x N),
 * out[5] work items, out[6] groups, out[7] padded atom slots, out[8] atom pairs
 * within r_cut at build time (FP64), out[9] candidate cluster pairs of the
 * bounding-box search (before the atom-pair prune). */
nb_status nb_pairlist_stats(nb_sys *sys, int64_t out[10]);

/* Forces at x_dev (device FP64 [N,3]) into f_dev (device FP32 [N,3], kJ/mol/nm),
 * using the current list (built first if there is none): the cluster-pair kernel
 * of Section "SIMD parallelism" (all M x N pairs of each listed cluster pair;
 * Lennard-Jones plus reaction-field or real-space Ewald Coulomb, the short-range
 * non-bonded interactions of Section "Introduction" and Section "Multi-level
 * parallelism").  Each listed pair with r < r_cut is evaluated once (Newton's
 * third law).  ener_host[2] = {E_LJ, E_coul}
 * and virial_host[9] = Xi = -1/2 sum_{i<j} r_ij (x) F_ij (row-major) are FP64;
 * either may be NULL (then no energy pass is run and the call is asynchronous). */
nb_status nb_compute_forces(nb_sys *sys, const double *x_dev, float *f_dev, double *ener_host,
                            double *virial_host);

/* The reciprocal-space part alone of a system with PME (pme_grid set): smooth PME
 * at x_dev (device FP64 [N,3], any periodic image) -- charges spread on the grid
 * with cardinal B-splines, 3D transform, influence function
 * exp(-pi^2 m^2/beta^2) B(m) / (pi V m^2), inverse transform, forces from the
 * spline gradients (the long-range part of Section "Multi-level parallelism",
 * Fig. 2) -- into f_dev (device FP32 [N,3], kJ/mol/nm).  energy_host (may be
 * NULL) receives E_recip + E_self + E_background and virial_host[9] (may be
 * NULL) their virial, row-major, as nb_compute_forces.  No pair list is needed.
 * NB_ERR_STATE without PME or particles.  Synchronises if energy or virial is
 * asked for, else asynchronous. */
nb_status nb_pme_forces(nb_sys *sys, const double *x_dev, float *f_dev, double *energy_host,
                        double *virial_host);

/* n_steps velocity-Verlet steps in FP64 (x_dev, v_dev FP64 [N,3] updated in place;
 * f_dev FP32 [N,3] holds F(x) on return): forces from positions, then positions
 * and velocities from forces, step after step (Section "Introduction"), with the
 * buffered list reused for nstlist steps (Section "Heterogeneous
 * parallelization").  Per step: v += dt/2 F/m; x += dt v; list rebuilt when the
 * system's step counter is a multiple of nstlist (and before the first step if no
 * list exists); F = F(x); v += dt/2 F/m.  Energies are evaluated every nstenergy
 * steps (0 = never); ener_trace_host receives one row {step, E_LJ, E_coul, E_kin,
 * E_total} (5 doubles) per evaluated step, at most trace_cap rows; *n_rows (may be
 * NULL) the count.  Synchronises at the end.
 * Errors: if a rebuild inside the call needs more list capacity than the arena
 * holds (with build checks on, the default), the call returns NB_ERR_CAPACITY
 * with x, v and the step counter at the last completed step, the energy rows of
 * the completed steps in ener_trace_host / *n_rows, and nb_sys_needed_bytes set:
 * grow the arena (nb_sys_set_arena) and call again for the remaining steps. */
nb_status md_step(nb_sys *sys, double *x_dev, double *v_dev, float *f_dev, double dt_ps,
                  int32_t n_steps, int32_t nstlist, int32_t nstenergy, double *ener_trace_host,
                  int32_t trace_cap, int32_t *n_rows);

/* Steepest-descent relaxation on the same force path: each iteration moves every
 * atom by max_disp * F_i / max_j |F_j| (the atom with the largest force moves
 * max_disp nm), until max|F| < f_tol or n_iter iterations.  The list is rebuilt
 * every nstlist iterations.  x_dev is updated in place and f_dev holds the forces
 * at the final positions; *f_max_host and *iters_host (either may be NULL)
 * receive the final max|F| and the iteration count.  Synchronises. */
nb_status nb_minimize(nb_sys *sys, double *x_dev, float *f_dev, int32_t n_iter, double f_tol,
                      double max_disp, int32_t nstlist, double *f_max_host, int32_t *iters_host);

/* Step counter of the system (number of md_step steps done). */
nb_status nb_sys_get_step(const nb_sys *sys, int64_t *step);
nb_status nb_sys_set_step(nb_sys *sys, int64_t step);

/* Checkpoint: state = {step, N, x[N,3], v[N,3]} as host bytes, so a run of an
 * ensemble can be stopped and continued (Section "Ensemble simulations": many
 * runs managed to completion by a controller).  nb_state_bytes
 * gives the size; export copies from x_dev/v_dev; import writes them back and
 * drops the list (so a checkpoint taken at a list-build step resumes bitwise). */
nb_status nb_state_bytes(const nb_sys *sys, size_t *bytes);
nb_status nb_state_export(nb_sys *sys, const double *x_dev, const double *v_dev, void *host,
                          size_t bytes);
nb_status nb_state_import(nb_sys *sys, double *x_dev, double *v_dev, const void *host,
                          size_t bytes);

/* ------------------------------------------------------------------------ */
/* Batched ensembles (paper, Section "Ensemble simulations": many independent
 * simulations of one problem).  Members keep their own arenas and state; the
 * ensemble runs every per-step kernel once for all members (one launch per
 * kernel, the force kernel once per kernel class = cluster size x interaction
 * type), and replays the step without a list rebuild from a captured HIP graph.
 * A member's arithmetic depends only on its own data, so its trajectory is
 * bitwise the same alone (md_step) and in any ensemble (V64r precision). */

/* Device memory for the ensemble's own tables (max_systems members). */
nb_status nb_ens_arena_bytes(int32_t max_systems, size_t *bytes);
nb_status nb_ens_create(nb_ctx *ctx, int32_t max_systems, void *dev_arena, size_t arena_bytes,
                        nb_ens **out);
nb_status nb_ens_destroy(nb_ens *ens);
/* Add a member with its device state (FP64 x, v [N,3]; FP32 f [N,3]).  The member's
 * list is rebuilt inside the ensemble.  NB_ERR_CAPACITY if the ensemble is full. */
nb_status nb_ens_add(nb_ens *ens, nb_sys *sys, double *x_dev, double *v_dev, float *f_dev);
nb_status nb_ens_remove(nb_ens *ens, nb_sys *sys);
nb_status nb_ens_size(const nb_ens *ens, int32_t *n);
/* Position of a member in the ensemble's internal order (the order of
 * nb_ens_step's energy rows). */
nb_status nb_ens_member_index(const nb_ens *ens, const nb_sys *sys, int32_t *idx);
/* n_steps velocity-Verlet steps for every member, exactly as md_step would do for
 * each alone (own step counter; list rebuilt when its counter is a multiple of
 * nstlist).  use_graph != 0 replays a captured graph for steps without a rebuild.
 * energies_host (may be NULL) receives per member, in nb_ens_member_index order,
 * {E_LJ, E_coul, E_kin} of the last step.  Synchronises at the end. */
nb_status nb_ens_step(nb_ens *ens, int32_t n_steps, double dt_ps, int32_t nstlist, int32_t use_graph,
                      double *energies_host);

/* Autotuner (Section "SIMD parallelism": the cluster size is chosen per hardware
 * to fit its SIMD width; here it is measured per system): for sys's model and
 * particles at positions x_dev, build a throw-away
 * copy in scratch_dev for every cluster size in clusters[] and j-tile in jtiles[],
 * time `reps` force evaluations (HIP events; f_dev is FP32 [N,3] scratch) and
 * return the fastest pair.  Candidates that do not fit the scratch arena are
 * skipped.  Synchronises. */
nb_status nb_autotune(nb_sys *sys, const double *x_dev, float *f_dev, void *scratch_dev,
                      size_t scratch_bytes, const int32_t *clusters, int32_t n_clusters,
                      const int32_t *jtiles, int32_t n_jtiles, int32_t reps, int32_t *best_cluster,
                      int32_t *best_jtile, double *best_us);

/* ------------------------------------------------------------------------ */
/* Serving: a continuous-batching MD job server (paper, Section "Ensemble
 * simulations": a controller that keeps many independent runs going to
 * completion).  A host thread admits queued jobs while the device pool (the HBM
 * budget) and the slot count allow, joins them to the running batch at the next
 * list-rebuild boundary, advances the batch with the ensemble kernels and retires
 * jobs at their step counts.  Job state stays resident on the device while the
 * job runs.  Results are bitwise the same as running the job alone (V64r).
 *
 * nb_srv_create: pool_dev/pool_bytes is the caller's device memory budget for job
 *   state (sub-allocated first-fit by the server); ens_arena_dev must hold
 *   nb_ens_arena_bytes(max_slots).  The server runs on its own HIP stream of
 *   device ctx->device.
 * nb_srv_submit: host arrays are copied before return; x, v FP64 [N,3]; sigma/
 *   epsilon may be NULL for NB_LJ_SINGLE.  A job larger than the whole pool is
 *   rejected (state 4, NB_ERR_CAPACITY).
 * nb_srv_poll: state 0 queued, 1 running, 2 done, 3 failed, 4 rejected; times =
 *   {submit, admit, done} in seconds since server creation (-1 if not yet);
 *   energies = {E_LJ, E_coul, E_kin} after the last step.
 * nb_srv_fetch copies a finished job's final x, v; nb_srv_release forgets a
 *   finished job.  nb_srv_wait_idle blocks until nothing is queued or running.
 * nb_srv_stats: {atom-steps done, jobs done, failed, rejected, busy seconds,
 *   seconds since creation, running, queued}. */
nb_status nb_srv_create(nb_ctx *ctx, void *pool_dev, size_t pool_bytes, void *ens_arena_dev,
                        size_t ens_arena_bytes, int32_t max_slots, double dt_ps, int32_t nstlist,
                        int32_t use_graph, nb_srv **out);
nb_status nb_srv_submit(nb_srv *srv, const nb_params *p, const double *x, const double *v,
                        const double *q, const double *sigma, const double *epsilon,
                        const double *mass, int32_t n_steps, uint64_t *job_id);
nb_status nb_srv_poll(nb_srv *srv, uint64_t job_id, int32_t *state, double times[3],
                      double energies[3], nb_status *job_error);
nb_status nb_srv_fetch(nb_srv *srv, uint64_t job_id, double *x_host, double *v_host);
nb_status nb_srv_release(nb_srv *srv, uint64_t job_id);
nb_status nb_srv_wait_idle(nb_srv *srv, double timeout_s);
nb_status nb_srv_stats(nb_srv *srv, double out[8]);
nb_status nb_srv_destroy(nb_srv *srv);

/* Per-phase HIP-event timers of md_step (on the context stream).  on = 0: off;
 * on = k >= 1: one of every k force-kernel launches and one of every k list
 * rebuilds (counted from this call), and each whole md_step call, are bracketed
 * by events (an event record between two kernels costs the stream a few
 * microseconds, so a stride above 1 keeps the timed run close to an untimed
 * one).  nb_sys_get_timings returns {force ms total, force launches timed,
 * rebuild ms total, rebuilds timed, md_step ms total, md_step calls} since the
 * last nb_sys_set_timing.  NB_ERR_ARG for on < 0. */
nb_status nb_sys_set_timing(nb_sys *sys, int32_t on);
nb_status nb_sys_get_timings(nb_sys *sys, double out[6]);
/* List-buffer guard: at every rebuild the largest atom displacement since the
 * previous build is measured (FP64).  out[0] = the largest such displacement seen
 * (nm), out[1] = number of list lifetimes in which it reached (r_list - r_cut)/2,
 * the only way a pair could have entered r_cut without being listed.  With
 * dynamic pruning the same for the prune intervals: out[2] = the largest
 * displacement within one interval, out[3] = intervals in which it reached
 * (r_inner - r_cut)/2 (0 and 0 without pruning).  Synchronises. */
nb_status nb_sys_buffer_stats(nb_sys *sys, double out[4]);
/* md_step checks list capacity after every rebuild by default (one host
 * synchronisation per rebuild); off defers the check to the end of the call
 * (a capacity overflow then fails the call after the fact). */
nb_status nb_sys_set_build_checks(nb_sys *sys, int32_t on);

/* ------------------------------------------------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work of
 * nb_sys_create + nb_sys_set_particles + nb_compute_forces for one system --
 * list build at x_dev and forces (energies/virial if asked) -- with all working
 * memory (pair list, partials, staging, counters) in a fixed device array
 * inside the library, NB_NOALLOC_MAX_BYTES per GPU, held from the first
 * context on that GPU until the process ends.  The call allocates nothing:
 * no hipMalloc, hipFree or other allocating routine, no system handle.
 *  p               system parameters (as for nb_sys_create)
 *  q, sigma, epsilon  host FP64 [N] per-atom data (sigma/epsilon only for
 *                  NB_LJ_LB; may be NULL otherwise), read before return
 *  x_dev, f_dev    device FP64 [N,3] positions, device FP32 [N,3] forces out
 *  ener_host[2], virial_host[9]  as for nb_compute_forces (may be NULL)
 * Results are bitwise those of the three calls above.  Synchronises.
 * Errors: NB_ERR_CAPACITY if the system's working memory exceeds
 * NB_NOALLOC_MAX_BYTES (also after growing a list that outgrew its estimate);
 * NB_ERR_DEVICE if the array could not be located on this GPU.
 * Every call on a GPU uses that GPU's one array and leaves its contents there
 * (each call clears what it reads before use): calls that overlap on one GPU
 * (other threads, or other streams before this one's call returned) race. */
#define NB_NOALLOC_MAX_BYTES ((size_t)64 << 20)
nb_status nb_compute_forces_noalloc(nb_ctx *ctx, const nb_params *p, const double *q,
                                    const double *sigma, const double *epsilon,
                                    const double *x_dev, float *f_dev, double *ener_host,
                                    double *virial_host);

/* Introspection: max relative error over [0, r_cut] of the kernel's Ewald
 * tables (the force factor erfc(beta r) + 2 beta r/sqrt(pi) exp(-beta^2 r^2)
 * and erfc(beta r), piecewise cubic with FP32 coefficients), evaluated in FP64
 * at system creation; 0 for non-Ewald systems. */
nb_status nb_sys_ewald_fit_error(const nb_sys *sys, double *err);

#ifdef __cplusplus
}
#endif
#endif /* NB_H */
