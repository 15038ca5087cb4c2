// nb_internal.h -- device data layout and launch helpers of libnb (gfx950).
//
// One system lives in one caller-provided arena.  Its descriptor (SysDev) is a
// plain struct of sizes, model constants and device pointers into the arena; a
// copy sits at the start of the arena so that kernels can read it, and batched
// launches read an array of such descriptors (one per member system).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace nbi {

constexpr int kWave = 64;
constexpr int kGroup = 8;            // clusters per i-group (2 x 2 x 2 split of a column chunk)
// periodic shift (sx, sy, sz) of a list entry: sx a + sy b + sz c, sx in -2..2
// (a skewed box's rows can reach two a-images), sy, sz in -1..1
__host__ __device__ constexpr int shift_id(int sx, int sy, int sz) { return (sx + 2) + 5 * (sy + 1) + 15 * (sz + 1); }
constexpr int kShiftZero = shift_id(0, 0, 0);
constexpr int kSortLds = 4096;       // column keys sorted in LDS (larger columns sort in HBM)
constexpr int kTraceCap = 1024;      // device energy-trace ring rows
constexpr int kStatusBytes = 64;     // the status words, padded; the trace ring follows them
constexpr int kKeBlocks = 1024;      // max blocks of the per-system partial sums (kinetic energy, max|F|)
constexpr int kEnerPart = 8;         // per-item partials: E_lj, E_c, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz
constexpr int kEwTab = 256;          // cubic intervals of the Ewald tables on [0, r_cut]
constexpr int kEwTabN = kEwTab + 1;  // plus one interval past r_cut: an FP32 r that rounds to r_cut reads a valid one

// List entry meta word: bits 0-7 shift id, 8-15 the i-clusters the force
// kernel evaluates (after a dynamic prune: those with a pair within r_inner),
// 16-19 real atoms of the j-cluster, 20-27 the i-clusters the build listed.
constexpr int kMetaInner = 8;
constexpr int kMetaNreal = 16;
constexpr int kMetaOuter = 20;

// Work items of the force kernel cut by cost.  With 8-atom clusters a list
// entry costs a fixed part (its loads, the j-force reduction and store: about
// 3.5 times the cost of one listed cluster pair, measured per item on MI355X)
// plus a part per i-cluster it lists: weight kEntW0 + kEntW1 popcount(mask).
// A group's kept entries, in list order, cover consecutive weight ranges
// [P, P + w); an entry whose range holds a multiple of the item weight W starts
// an item, so a group has ceil(total / W) items of about equal cost.  Other
// cluster sizes weigh every entry 1 (items of jtile entries).
constexpr int kEntW0 = 7;
constexpr int kEntW1 = 2;
constexpr int kEntWMax = kEntW0 + kEntW1 * kGroup;
constexpr int kEntWNom = 16;  // jtile counts nominal entries of this weight
__host__ __device__ inline int entry_weight(int M, unsigned int im)
{
    return M == 8 ? kEntW0 + kEntW1 * __builtin_popcount(im & 255u) : 1;
}
__host__ __device__ inline int item_weight(int M, int jtile)
{
    return M == 8 ? (jtile * kEntWNom > kEntWMax ? jtile * kEntWNom : kEntWMax) : jtile;
}
// items for ent entries in n_groups groups, at most
__host__ __device__ inline double item_bound(int M, int jtile, double ent, int n_groups)
{
    return ent * (M == 8 ? kEntWMax : 1) / item_weight(M, jtile) + n_groups;
}

// global-address-space loads (the pointers live in a descriptor, so the compiler
// would otherwise emit flat loads); vector types go through ext_vector_type
// because aggregate copies would drop the address space
typedef float nb_v4f __attribute__((ext_vector_type(4)));
typedef float nb_v2f __attribute__((ext_vector_type(2)));
typedef int nb_v2i __attribute__((ext_vector_type(2)));
typedef int nb_v4i __attribute__((ext_vector_type(4)));
#define NB_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ float4 gld(const float4* p)
{
    const nb_v4f v = *(const NB_GLOBAL nb_v4f*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 gld(const float2* p)
{
    const nb_v2f v = *(const NB_GLOBAL nb_v2f*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ int2 gld(const int2* p)
{
    const nb_v2i v = *(const NB_GLOBAL nb_v2i*)p;
    return make_int2(v.x, v.y);
}
__device__ __forceinline__ int4 gld(const int4* p)
{
    const nb_v4i v = *(const NB_GLOBAL nb_v4i*)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
// scalars (int, float, double, 64-bit words)
template <class T>
__device__ __forceinline__ T gld(const T* p)
{
    return *(const NB_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ void gst(T* p, T v)
{
    *(NB_GLOBAL T*)p = v;
}
__device__ __forceinline__ void gst(int2* p, int2 v) { *(NB_GLOBAL nb_v2i*)p = nb_v2i{v.x, v.y}; }
__device__ __forceinline__ void gst(float4* p, float4 v) { *(NB_GLOBAL nb_v4f*)p = nb_v4f{v.x, v.y, v.z, v.w}; }
__device__ __forceinline__ void gst(float2* p, float2 v) { *(NB_GLOBAL nb_v2f*)p = nb_v2f{v.x, v.y}; }
// device-scope integer add in the global address space (a flat atomic would
// also count against the LDS wait counter)
__device__ __forceinline__ int gatomic_add(int* p, int v)
{
    return __hip_atomic_fetch_add((NB_GLOBAL int*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Blocks per system for per-atom loops: a function of the system alone, so the
// kinetic-energy partial sums decompose the same way alone and in a batch.
__device__ inline int sys_blocks(int n_atoms)
{
    int b = (n_atoms + 255) / 256;
    return b > kKeBlocks ? kKeBlocks : (b < 1 ? 1 : b);
}


// status word indices
enum { ST_OVERFLOW = 0, ST_NEED_CAND = 1, ST_NEED_ENT = 2, ST_NEED_ITEM = 3, ST_NEED_GROUPS = 4,
       ST_SATURATE = 5, ST_BIGCOL = 6, ST_BADPOS = 7, ST_COUNT = 8 };

struct SysDev {
    // ---- sizes -------------------------------------------------------
    int n_atoms;
    int M;              // cluster size
    int G;              // clusters per group (kGroup)
    int ncx, ncy;       // coarse columns
    int n_cols;
    int max_groups;
    int cand_cap;       // candidates per group
    int ent_cap;        // entries (total)
    int item_cap;       // work items (total)
    int jtile;          // entries per work item (nominal entries with 8-atom clusters)
    int item_w;         // weight per work item: item_weight(M, jtile)
    int mask_words;     // u64 words of atom masks per entry (G*M*M/64 rounded up)
    int coulomb, lj, pot_shift, fp32_reduce;
    // ---- geometry (FP64) ---------------------------------------------
    double box[3], invbox[3];
    double box_off[3];  // triclinic b_x, c_x, c_y (a = (box0,0,0), b = (b_x,box1,0), c = (c_x,c_y,box2))
    int tric;           // box_off not all zero
    double cell[2], inv_cell[2];
    double rlist2;      // exact pair criterion r^2 < rlist2
    double rcut2;       // FP64 r_cut^2 (list statistics only)
    double rbb;         // bounding-box search radius (r_list + margin)
    // ---- model (FP32 pair arithmetic) ---------------------------------
    float rc2;
    float rl2_prune;                // r_list^2 (1 + 2^-14): the search's FP32 atom-pair prune
    float rin2;                     // r_inner^2 (dynamic pruning in the force kernel; 0: off)
    int prune_on;                   // dynamic pruning configured
    double prune_half;              // (r_inner - r_cut) / 2: the prune interval's displacement guard
    float c6, c12, c6x6, c12x12;   // single-type LJ
    float lj_shift;                 // single type: c12/rc^12 - c6/rc^6
    float irc6, irc12;              // 1/rc^6, 1/rc^12 (LB shift)
    float krf2, krf, crf;           // 2 k_rf, k_rf, c_rf
    float ew_shift;                 // erfc(beta rc)/rc (0 without shift)
    float qscale;                   // sqrt(1/(4 pi eps0 eps_r))
    float ew_tinv;                  // kEwTab / r_cut
    float4* ew_tab;                 // [kEwTabN] cubic coefficients of q(r) = erfc(beta r) + 2 beta r/sqrt(pi) exp(-beta^2 r^2)
    float4* ew_etab;                // [kEwTabN] cubic coefficients of e(r) = erfc(beta r) (energies)
    double fx_scale, fx_inv;        // fixed-point 2^bits, 2^-bits
    float fx_lim;                   // max |partial| representable
    // ---- per-atom inputs (device copies, original order) ----------------
    const double* q;      // [N]
    const double* sig;    // [N] (LB)
    const double* eps;    // [N] (LB)
    const double* mass;   // [N]
    // ---- caller state (set per call) -----------------------------------
    const double* x;      // [N,3]
    double* v;            // [N,3]
    float* f;             // [N,3]
    // ---- binning -------------------------------------------------------
    int* atom_col;        // [N]
    int* atom_wrap;       // [N,3]
    unsigned int* atom_zkey; // [N]
    int* col_count;       // [n_cols]
    int* col_fill;        // [n_cols]
    int* col_start;       // [n_cols+1]
    int* col_gstart;      // [n_cols+1]
    unsigned long long* sort_key; // [N] (z key, atom) words in column segments, unsorted
    unsigned long long* sort_out; // [N] the same, sorted within each column
    // ---- slots (cluster order) ----------------------------------------
    int* slot_atom;       // [max_slots] original atom or -1
    float4* xq;           // [max_slots] local x,y,z, scaled charge
    float2* ljs;          // [max_slots] sigma/2, 2 sqrt(eps)
    int* slot_wrap;       // [max_slots*3]
    double* slot_x;       // [max_slots*3] original FP64 positions at build (exact prune)
    // ---- clusters and groups -------------------------------------------
    int* n_groups;        // [1]
    int* cl_nreal;        // [max_groups*G]
    double* cl_bb;        // [max_groups*G*6] lo.xyz, hi.xyz (wrapped frame)
    double* gr_ref;       // [max_groups*3]
    double* gr_bb;        // [max_groups*6]
    int* grp_col;         // [max_groups] column of each group
    int2* grp_range;      // [max_groups] each group's atoms: {first sorted key, count}
    // ---- candidates ------------------------------------------------------
    int* cand_count;      // [max_groups]
    int2* cand;           // [max_groups*cand_cap] {cj, sid | imask<<8}
    unsigned long long* cand_mask; // [max_groups*cand_cap*mask_words]
    int* cand_kept;       // [max_groups]
    int* grp_rc;          // [max_groups] atom pairs within r_cut at build (statistics)
    int* grp_w;           // [max_groups] weight of the kept entries (work-item cutting)
    // ---- list ------------------------------------------------------------
    int* ent_start;       // [max_groups+1]
    int* item_start;      // [max_groups+1]
    int2* ent;            // [ent_cap] {cj, sid | imask<<8 | nreal(cj)<<16}
    float4* ent_S;        // [ent_cap] shift vector (FP32); w: the row of the entry's j-partial (int bits)
    int4* items;          // [item_cap] {group, e0, e1, j-cluster of entry e0}
    // ---- force partials (written by the force kernel, summed by the gather) --
    float* jpart;         // [ent_cap*M*3] j-atom forces of each entry
    float* ipart;         // [item_cap*G*M*3] i-atom forces of each work item
    int* jstart;          // [max_groups*G+1] entries that list each cluster as j (CSR)
    int* jfill;           // [max_groups*G] fill cursor / counts
    int* n_items;         // [1]
    int* n_ent;           // [1]
    // ---- reductions and outputs -----------------------------------------
    float* epart;         // [item_cap*kEnerPart]
    double* ke_part;      // [kKeBlocks]
    double* eout;         // [16]: E_lj, E_c, Xi xx,yy,zz,xy,xz,yz, KE
    double* trace;        // [kTraceCap*5], kStatusBytes after status
    double* fmax_part;    // [kKeBlocks]
    int* status;          // [ST_COUNT]
    double* x_build;      // [N,3] positions at the last list build
    double* x_bak;        // [N,3] x, v at the last full step before a rebuild step
    double* v_bak;        //       (restored if that rebuild runs out of capacity)
    double* disp;         // [kKeBlocks] per-block max displacement^2; [kKeBlocks..+2): max, violations
    double* x_prune;      // [N,3] positions at the last dynamic prune (or build)
    double* pg_part;      // [2 kKeBlocks + 2]: two buffers of per-block max displacement^2 of a
                          // prune interval, then the statistics {max displacement, violations}
    double buffer;        // r_list - r_cut
    int* stats;           // [8] scratch for statistics
    // pair export scratch
    long long* exp_count; // [max_groups+1]
    // ---- reciprocal-space Ewald (PME), NULL without it -------------------
    const float* pme_f;   // [N,3] reciprocal-space forces, added by the gather
    const double* pme_e;  // [8] reciprocal + self + background energy, Xi xx,yy,zz,xy,xz,yz
};

// Smooth particle-mesh Ewald of one system: a K0 x K1 x K2 grid along the
// lattice vectors a, b, c, cardinal B-splines of order `order`.
struct PmeDev {
    int n_atoms;
    int K[3];
    int H2;                // K2/2 + 1 half-complex points along c
    int order;
    int tile;              // h_c columns per LDS tile of the b and a passes
    int solve_blocks;      // blocks of the a pass (rows of energy partials)
    double rec[6];         // a* = (rec0, rec1, rec2), b* = (0, rec3, rec4), c* = (0, 0, rec5)
    double fel;            // 1/(4 pi eps0 eps_r)
    double beta, vol;
    double pi2_b2;         // pi^2 / beta^2
    const double* q;       // [N] charges (the system's device copy)
    int col_cap;           // atoms a column bucket holds (twice the mean occupancy + 16)
    int* col_count;        // [K0*K1] atoms per (base_a, base_b) grid column; all zero between evaluations
    int* col_list;         // [K0*K1][col_cap] each column's bucket of atoms (any order within it)
    int* ovf_count;        // [1] atoms past their column's bucket; zero between evaluations
    int* ovf_list;         // [N] those atoms (any order)
    int4* atom_base;       // [N] spline base points (a, b, c) and column
    double* theta;         // [N][3*order] spline weights M_P(w + j) along a, b, c (k*order + j)
    double* dtheta;        // [N][3*order] their derivatives M_P'(w + j)
    double* conv;          // [K0*K1*K2] potential grid (theta_rec * Q)
    double2* cgrid;        // [K0*K1*H2] transforms in place, k_c fastest
    double* bmod;          // [K0+K1+K2] |b(m)|^2 of each dimension
    double* gtab;          // [K0*K1*H2] influence function G(m) on the half-complex grid
    double2* tw;           // [K0+K1+K2] (cos, sin)(2 pi j / K) of each dimension
    double* epart;         // [solve_blocks*8] energy and virial partials of the a pass
    double* qsum;          // [2] sum q, sum q^2
    double* eout;          // [8] E_recip + E_self + E_background, Xi xx,yy,zz,xy,xz,yz
    float* frec;           // [N,3] reciprocal-space forces
};

// A position moved into the primary cell by its integer lattice counts w
// (x - w_a a - w_b b - w_c c), FP64 without contraction, components in the
// order ((x - w_a a_x) - w_b b_x) - w_c c_x, (y - w_b b_y) - w_c c_y,
// z - w_c c_z (for a rectangular box: x - w L per dimension).
__device__ __forceinline__ void wrapped_pos(const SysDev& d, const double x[3], const int w[3], double u[3])
{
#pragma clang fp contract(off)
    u[0] = ((x[0] - (double)w[0] * d.box[0]) - (double)w[1] * d.box_off[0]) - (double)w[2] * d.box_off[1];
    u[1] = (x[1] - (double)w[1] * d.box[1]) - (double)w[2] * d.box_off[2];
    u[2] = x[2] - (double)w[2] * d.box[2];
}

// Group-local FP32 coordinates of a position: its wrapped position minus the
// group's reference point in FP64, rounded once.  Every kernel that stages
// positions uses it, so a slot's staged value does not depend on which kernel
// wrote it.
__device__ __forceinline__ void stage_pos(const SysDev& d, const double x[3], const int w[3], const double ref[3],
                                          float4& p)
{
#pragma clang fp contract(off)
    double u[3];
    wrapped_pos(d, x, w, u);
    p.x = (float)(u[0] - ref[0]);
    p.y = (float)(u[1] - ref[1]);
    p.z = (float)(u[2] - ref[2]);
}

// ---- launch entry points (implemented in the .hip files) ------------------
// All take a device array of `n_sys` descriptors and the per-launch grid bounds
// the host knows statically (max over members).
struct Bounds {
    int max_atoms;
    int max_cols;
    int max_groups;
    int max_slots;
    int max_ent;    // largest entry capacity of the members
    bool any_tric;  // some member has a triclinic box
    bool all_m8;    // every member has 8-atom clusters
};

// the whole list build with its transpose, after the list-buffer guard (the
// largest displacement since the previous build, then x recorded for the next
// one).  The search prunes every candidate at the atom level in FP32 (the force
// kernel's frame).  exact: then the FP64 atom-pair prune (export-ready masks)
// decides the list; otherwise the FP32 result is the list (masks left undefined
// until launch_refine).  item_prefix: also the prefix over the systems of their
// work-item counts.  flags (per system, NULL = the one system): 0 = skip, 1 =
// rebuild, 2 = first build (x only recorded); without flags, first says which.
// cleared: the gather before it already cleared the counters and status words
// and took the list-buffer guard's partials (md_step's rebuilds)
hipError_t launch_build(const SysDev* table, int n_sys, const Bounds& b, const int* flags, hipStream_t s,
                        bool exact, int status_clear = 0, int* item_prefix = nullptr, bool first = false,
                        bool cleared = false);
// exact masks (cand_mask) and pair counts for a list built without them, from
// the stored build positions; the force list itself is not touched
hipError_t launch_refine(const SysDev* table, int n_sys, const Bounds& b, hipStream_t s);
hipError_t launch_ens_status(const SysDev* table, int n_sys, int* out, hipStream_t s);
// flags (per system, NULL = every system): 0 = skip that system; clear_status:
// also every status word, as launch_clear_status would before it
hipError_t launch_stage(const SysDev* table, int n_sys, const Bounds& b, hipStream_t s,
                        const int* flags = nullptr, bool clear_status = false);
// mode 0: x, v -> x_bak, v_bak of every system; mode 1: back again
hipError_t launch_state_copy(const SysDev* table, int n_sys, const Bounds& b, int mode, hipStream_t s);
// prune: the force pass also prunes every entry's i-cluster mask to r_inner
// (from the build's mask), and later passes evaluate the pruned mask.
// max_blocks > 0 caps the persistent grid (its waves loop over the work items).
// red_row >= 0 (one system, no energies, no pruning): an extra block writes the
// previous energy pass's energy row as launch_energy_reduce(table, 1, red_row,
// true, red_step) would
hipError_t launch_force(const SysDev* table, int n_sys, const int* item_prefix, int M, int coulomb,
                        int lj, bool ener, int max_blocks, int total_item_cap, hipStream_t s, bool prune = false,
                        int red_row = -1, double red_step = 0.0);
// dynamic-prune guard of one system: check = 1: the largest displacement since
// x_prune into partial buffer cur; then x_prune = x.  fold: first fold the
// previous interval's partials (buffer 1 - cur) into the statistics
hipError_t launch_prune_guard_k(const SysDev* table, int n_atoms, int check, int cur, int fold, hipStream_t s);
hipError_t launch_finalize(const SysDev* table, int n_sys, const Bounds& b, bool fp32, hipStream_t s,
                           const int* flags = nullptr);
hipError_t launch_energy_reduce(const SysDev* table, int n_sys, int trace_row, bool with_ke,
                                double step_value, hipStream_t s);
hipError_t launch_kick_drift(const SysDev* table, int n_sys, const Bounds& b, double dt, hipStream_t s);
hipError_t launch_kick(const SysDev* table, int n_sys, const Bounds& b, double dt, bool ke,
                       hipStream_t s);
hipError_t launch_item_prefix(const SysDev* table, int n_sys, int* item_prefix, hipStream_t s,
                              const int* flags = nullptr);
// fused plain-step kernels: kick + drift + staging; gather + kick (+ kinetic energy)
hipError_t launch_kick_drift_stage(const SysDev* table, int n_sys, const Bounds& b, double dt, hipStream_t s);
// next: 0 = gather + half-kick; 1 = and the next step's half-kick + drift, and
// the list build's clears and buffer-guard partials (a rebuild follows);
// 2 = and also the staging of the new positions (no list rebuild due).
// open: the first positions of a run (no half-kick closes a step; next 1 or 2)
hipError_t launch_gather_kick(const SysDev* table, int n_sys, const Bounds& b, double dt, bool ke, hipStream_t s,
                              int next = 0, bool open = false);
hipError_t launch_export_count(const SysDev* table, const Bounds& b, hipStream_t s);
hipError_t launch_export_write(const SysDev* table, const Bounds& b, int* pairs_dev,
                               long long cap, hipStream_t s);
hipError_t launch_stats(const SysDev* table, const Bounds& b, hipStream_t s);
hipError_t launch_minimize_step(const SysDev* table, const Bounds& b, double* x, double max_disp,
                                double f_tol, int* done_flag, hipStream_t s);
hipError_t launch_fmax(const SysDev* table, const Bounds& b, hipStream_t s);
// PME: twiddles, spline moduli and charge sums (after the charges are on the
// device); then per evaluation the spread, transforms, solve and gather of the
// positions x (device FP64 [N,3]) into p.frec, and with ener the energy and
// virial into p.eout
hipError_t launch_pme_setup(const PmeDev& p, hipStream_t s);
hipError_t launch_pme(const PmeDev& p, const double* x, bool ener, hipStream_t s);
// keep_faults: leave the saturation / bad-position flags of earlier steps set
// (clears inside a multi-step call); otherwise every flag is cleared
hipError_t launch_clear_status(const SysDev* table, int n_sys, hipStream_t s, bool keep_faults = false);

// Per-system energy/virial (and kinetic energy) from the per-item partials, in
// a fixed order: FP64 (V64r) or FP32 (V32).  Xi = -1/2 sum r_ij (x) F_ij.
// One block of 256 threads per system: thread t sums items t, t + 256, ... (two
// 16-byte loads per item, all of a thread's loads issued before its sums), then
// each wave sums its lanes with a fixed shuffle tree and the four wave totals
// are added in wave order -- the same decomposition alone and in a batch.
template <class T>
__device__ __forceinline__ T wave_tree_sum(T v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <class T>
__device__ inline void energy_reduce_block(const SysDev& d, int n, int with_ke, T out[kEnerPart + 1])
{
    __shared__ T sh[4][kEnerPart + 1];
    T acc[kEnerPart + 1];
    for (int k = 0; k <= kEnerPart; ++k) acc[k] = T(0);
    const nb_v4f* ep = (const nb_v4f*)d.epart;
    constexpr int kU = 4;
    for (int i0 = threadIdx.x; i0 < n; i0 += 256 * kU) {
        nb_v4f lo[kU], hi[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = min(i0 + 256 * u, n - 1);  // (rows past the end are loaded, dropped)
            lo[u] = *(const NB_GLOBAL nb_v4f*)&ep[2 * i];
            hi[u] = *(const NB_GLOBAL nb_v4f*)&ep[2 * i + 1];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (i0 + 256 * u >= n) break;
            acc[0] += T(lo[u].x); acc[1] += T(lo[u].y); acc[2] += T(lo[u].z); acc[3] += T(lo[u].w);
            acc[4] += T(hi[u].x); acc[5] += T(hi[u].y); acc[6] += T(hi[u].z); acc[7] += T(hi[u].w);
        }
    }
    if (with_ke)
        for (int i = threadIdx.x; i < kKeBlocks; i += 256) acc[kEnerPart] += T(gld(&d.ke_part[i]));
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = 0; k <= kEnerPart; ++k) {
        const T w = wave_tree_sum(acc[k]);
        if (lane == 0) sh[wid][k] = w;
    }
    __syncthreads();
    for (int k = 0; k <= kEnerPart; ++k) out[k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
}

// The energy row of one system, by one block of 256 threads: the reduction
// above, then eout (E_lj, E_coul, the virial -1/2 sum r (x) F, the
// reciprocal-space terms when PME is on, E_kin) and, for trace_row >= 0, the
// trace ring row {step, E_lj, E_coul, E_kin, E_tot}.  Run by its own kernel or
// by an extra block of the next step's pair kernel (the same arithmetic).
__device__ inline void energy_reduce_system(const SysDev& d, int trace_row, int with_ke, double step_value)
{
    const int n = d.n_items[0];
    double out[kEnerPart + 1];
    if (d.fp32_reduce) {
        float o[kEnerPart + 1];
        energy_reduce_block<float>(d, n, with_ke, o);
        for (int k = 0; k <= kEnerPart; ++k) out[k] = o[k];
    } else {
        energy_reduce_block<double>(d, n, with_ke, out);
    }
    if (threadIdx.x == 0) {
        d.eout[0] = out[0];
        d.eout[1] = out[1];
        for (int k = 2; k < kEnerPart; ++k) d.eout[k] = -0.5 * out[k];
        if (d.pme_e) {
            // reciprocal space, self and background terms of the Ewald sum
            d.eout[1] += d.pme_e[0];
            for (int k = 2; k < kEnerPart; ++k) d.eout[k] += d.pme_e[k - 1];
            out[1] = d.eout[1];
        }
        if (with_ke) d.eout[8] = out[kEnerPart];
        if (trace_row >= 0) {
            double* t = d.trace + (size_t)(trace_row % kTraceCap) * 5;
            t[0] = step_value;
            t[1] = out[0];
            t[2] = out[1];
            t[3] = with_ke ? out[kEnerPart] : 0.0;
            t[4] = out[0] + out[1] + t[3];
        }
    }
}

}  // namespace nbi
