// nb_build.hip -- cluster-pair list construction on the GPU (gfx950).
//
// The paper's scheme (Section "SIMD parallelism"): place atoms on a grid in x
// and y, bin them in z, cut the z-ordered columns into clusters of exactly M
// atoms, and list every cluster pair that may contain atoms close enough to
// interact, with a buffer (r_list > r_cut) so the list can be reused over
// several steps.  The GPU additionally prunes the list (Section "Heterogeneous
// parallelization"); here the prune is an exact FP64 atom-pair test that also
// yields the list's exact atom-pair set.
//
// MI355X design: the whole build runs on the device with no host round trip.
//   1. k_bin          wrap into the box (integer image counts kept), xy column id
//   2. k_col_scan     per-system column offsets and group counts (one block)
//   3. k_scatter      counting-sort scatter of (z key, atom) into columns
//   4. k_col_sort     per-column bitonic sort in LDS;
//      k_group_split  one wave per 8*M-atom chunk of a column: split 2 x 2 x 2
//                     (z, then y, then x halves) into an i-group of 8 clusters
//                     of M atoms; bounding boxes; staging of the new slots
//   5. k_search       one block per i-group: bounding-box culling against the
//                     clusters of the neighbouring columns, all periodic images;
//                     candidates sorted by (j-cluster, shift)
//   6. k_prune        exact FP64 atom-pair masks (ballot of one pair per lane),
//                     the group's i-atoms in LDS.  Explicit builds only: the
//                     rebuilds inside MD runs keep the bounding-box candidates
//                     and the force kernel prunes them on first use (Section
//                     "Heterogeneous parallelization": the list is pruned on the
//                     GPU by the non-bonded kernel)
//   7. k_list_scan    per-system CSR offsets of kept entries and work items
//   8. k_list_write   compacted entries, FP32 shift vectors, work items
// Every step is deterministic (no order depends on atomics).
#include "nb_internal.h"

#pragma clang fp contract(off)

namespace nbi {

namespace {

__device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

__device__ inline double box_gap(double lo1, double hi1, double lo2, double hi2)
{
    double g = lo2 - hi1;
    double h = lo1 - hi2;
    double m = g > h ? g : h;
    return m > 0.0 ? m : 0.0;
}

// box fraction of a wrapped coordinate as a 32-bit key (non-finite -> 0)
// FP32 shift vector of a list entry in the force kernel's frame: j-group
// reference plus the periodic shift, minus the i-group reference (FP64, then
// rounded once)
__device__ inline float4 entry_shift(const SysDev& d, const double rj[3], int sid, const double ri[3])
{
    const int s0 = sid % 5 - 2, s1 = (sid / 5) % 3 - 1, s2 = sid / 15 - 1;
    // the shift s0 a + s1 b + s2 c (rectangular: s L per dimension)
    const double tx = (s0 * d.box[0] + s1 * d.box_off[0]) + s2 * d.box_off[1];
    const double ty = s1 * d.box[1] + s2 * d.box_off[2];
    float4 S;
    S.x = (float)((rj[0] + tx) - ri[0]);
    S.y = (float)((rj[1] + ty) - ri[1]);
    S.z = (float)((rj[2] + s2 * d.box[2]) - ri[2]);
    S.w = 0.0f;
    return S;
}

__device__ inline unsigned int coord_key(double v, double inv)
{
    const double f = v * inv * 4294967296.0;
    if (!(f >= 0.0)) return 0u;
    if (f >= 4294967295.0) return 0xffffffffu;
    return (unsigned int)f;
}

// exclusive block scan of one int per thread (blockDim.x == 1024)
__device__ int block_exclusive_scan(int v, int* smem, int* total)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) smem[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        int w = lane < (int)(blockDim.x >> 6) ? smem[lane] : 0;
        int wi = w;
        for (int o = 1; o < 16; o <<= 1) {
            int t = __shfl_up(wi, o, 64);
            if (lane >= o) wi += t;
        }
        if (lane < 16) smem[16 + lane] = wi - w;
        if (lane == 15) smem[32] = wi;
    }
    __syncthreads();
    int res = incl - v + smem[16 + wid];
    *total = smem[32];
    __syncthreads();
    return res;
}

// Ascending sort of n <= 2 * blockDim.x distinct keys in LDS (16-byte aligned,
// room for n + 1) by rank: each thread counts the keys below its own
// (broadcast reads of two keys at a time, no barrier per stage; waves without
// a key skip the count), then every key moves to its rank
typedef unsigned long long nb_u64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void rank_sort_lds(unsigned long long* keys, int n)
{
    if (threadIdx.x == 0) keys[n] = ~0ull;  // pad: above every key
    __syncthreads();
    const int t0 = threadIdx.x, t1 = threadIdx.x + blockDim.x;
    const unsigned long long k0 = t0 < n ? keys[t0] : ~0ull, k1 = t1 < n ? keys[t1] : ~0ull;
    int r0 = 0, r1 = 0;
    if ((int)(threadIdx.x & ~63u) < n) {
        const nb_u64x2* kv = (const nb_u64x2*)keys;
#pragma unroll 4
        for (int u = 0; u < (n + 1) / 2; ++u) {
            const nb_u64x2 ku = kv[u];
            r0 += (ku.x < k0 ? 1 : 0) + (ku.y < k0 ? 1 : 0);
            r1 += (ku.x < k1 ? 1 : 0) + (ku.y < k1 ? 1 : 0);
        }
    }
    __syncthreads();
    if (t0 < n) keys[r0] = k0;
    if (t1 < n) keys[r1] = k1;
    __syncthreads();
}

// Ascending bitonic sort of keys[0..n) (n <= P, P a power of two), all
// comparators min-to-lower-index so the implicit +inf padding never moves.
__device__ __forceinline__ void bitonic_sort(unsigned long long* keys, int n, int P)
{
    const int nthr = blockDim.x;
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (P >> 1); t += nthr) {
                int i, p;
                if (j == (k >> 1)) {
                    i = (t / j) * k + (t % j);
                    p = i ^ (k - 1);
                } else {
                    i = (t / j) * 2 * j + (t % j);
                    p = i + j;
                }
                if (p < n) {
                    unsigned long long u = keys[i], w = keys[p];
                    if (u > w) {
                        keys[i] = w;
                        keys[p] = u;
                    }
                }
            }
            __syncthreads();
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// the build mode of a system: 0 = not rebuilt, 1 = rebuilt, 2 = first build
__device__ inline int build_mode(const int* flags, int sys, int first)
{
    return flags ? flags[sys] : (first ? 2 : 1);
}

// 0. clear the build counters, and the list-buffer guard: per block the largest
//    squared displacement since the previous build (mode 1), x recorded for the
//    next one.  status_clear: 1 = clear the status words too, 2 = all but the
//    fault flags of earlier steps (saturation, bad positions).  Inside md_step
//    the gather that ends the step before a rebuild does all of this instead
//    (the kernel is then not launched); the slot map is reset by k_bin.
__global__ __launch_bounds__(256) void k_build_clear(const SysDev* __restrict__ table, const int* flags,
                                                     int status_clear, int first)
{
    const int mode = build_mode(flags, blockIdx.y, first);
    if (mode == 0) return;
    const SysDev& d = table[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (status_clear && i < ST_COUNT && !(status_clear == 2 && (i == ST_SATURATE || i == ST_BADPOS)))
        gst(&d.status[i], 0);
    if (i < d.n_cols) {
        gst(&d.col_count[i], 0);
        gst(&d.col_fill[i], 0);
    }
    if (i < d.max_groups) {
        gst(&d.cand_count[i], 0);
        gst(&d.cand_kept[i], 0);
        gst(&d.grp_w[i], 0);
    }
    if (i < d.max_groups * d.G) gst(&d.jfill[i], 0);
    // displacement partials: blocks [0, sys_blocks) stride over the atoms (the
    // same decomposition alone and in a batch); the other partial slots are 0
    const int nb = sys_blocks(d.n_atoms);
    if ((int)blockIdx.x >= nb) {
        if ((int)blockIdx.x < kKeBlocks && threadIdx.x == 0) d.disp[blockIdx.x] = 0.0;
        return;
    }
    __shared__ double sh[256];
    double m = 0.0;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < d.n_atoms; a += nb * blockDim.x) {
        double s2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double x = gld(&d.x[3 * a + k]);
            if (mode == 1) {
                const double dd = x - gld(&d.x_build[3 * a + k]);
                s2 += dd * dd;
            }
            gst(&d.x_build[3 * a + k], x);
        }
        m = (s2 > m || s2 != s2) ? s2 : m;  // NaN wins
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double u = sh[threadIdx.x + o];
            if (u > sh[threadIdx.x] || u != u) sh[threadIdx.x] = u;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) d.disp[blockIdx.x] = sh[0];
}

// 1. wrap, column id, z key; column counts through a block-private LDS
//    histogram (device-scope atomics to one counter serialise)
constexpr int kHistLds = 4096;

__global__ __launch_bounds__(256) void k_bin(const SysDev* __restrict__ table, const int* flags)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    // every slot starts empty (the group split fills the real ones)
    const int slots = d.max_groups * d.G * d.M;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < slots; k += gridDim.x * blockDim.x)
        gst(&d.slot_atom[k], -1);
    __shared__ int hist[kHistLds];
    const bool priv = d.n_cols <= kHistLds;
    if (priv)
        for (int c = threadIdx.x; c < d.n_cols; c += blockDim.x) hist[c] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.n_atoms) {
        double xw[3];
        bool finite = true;
        const double x0 = d.x[3 * i], x1 = d.x[3 * i + 1], x2 = d.x[3 * i + 2];
        int wl[3] = {0, 0, 0};
        // lattice counts in the order c, b, a: each component is reduced after
        // the higher lattice vectors were removed from it (rectangular: per
        // dimension)
        for (int k = 2; k >= 0; --k) {
            const double xk = k == 2 ? x2
                            : k == 1 ? x1 - (double)wl[2] * d.box_off[2]
                                     : (x0 - (double)wl[1] * d.box_off[0]) - (double)wl[2] * d.box_off[1];
            finite = finite && (fabs(xk) <= 1.7976931348623157e308);
            double t = floor(xk * d.invbox[k]);
            if (!(fabs(t) < 1e9)) t = 0.0;  // non-finite or absurd input: image 0
            int w = (int)t;
            double r = xk - t * d.box[k];
            if (r >= d.box[k]) {
                r -= d.box[k];
                w += 1;
            }
            if (r < 0.0) {
                r += d.box[k];
                w -= 1;
            }
            if (r >= d.box[k]) r = 0.0;  // r was -tiny: rounds to L; keep the image count, clamp
            xw[k] = r;
            wl[k] = w;
            d.atom_wrap[3 * i + k] = w;
        }
        const double fx = xw[0] * d.inv_cell[0], fy = xw[1] * d.inv_cell[1];
        int cx = (fx >= 0.0 && fx < 1e9) ? (int)fx : 0;  // non-finite input lands in column 0
        int cy = (fy >= 0.0 && fy < 1e9) ? (int)fy : 0;
        cx = cx < 0 ? 0 : (cx >= d.ncx ? d.ncx - 1 : cx);
        cy = cy < 0 ? 0 : (cy >= d.ncy ? d.ncy - 1 : cy);
        const int col = cx + d.ncx * cy;
        d.atom_col[i] = col;
        d.atom_zkey[i] = coord_key(xw[2], d.invbox[2]);
        if (!finite) atomicOr(&d.status[ST_BADPOS], 1);
        if (priv) atomicAdd(&hist[col], 1);
        else gatomic_add(&d.col_count[col], 1);
    }
    __syncthreads();
    if (priv)
        for (int c = threadIdx.x; c < d.n_cols; c += blockDim.x)
            if (hist[c]) gatomic_add(&d.col_count[c], hist[c]);
}

// 2. column offsets and group counts
__global__ __launch_bounds__(1024) void k_col_scan(const SysDev* __restrict__ table, const int* flags, int first)
{
    const int mode = build_mode(flags, blockIdx.x, first);
    if (mode == 0) return;
    const SysDev& d = table[blockIdx.x];
    __shared__ int smem[40];
    if (mode == 1) {
        // list-buffer guard: the largest displacement of this list lifetime
        // from the per-block partials (NaN wins), and whether it reached half
        // the buffer (the only way a pair could enter r_cut unlisted)
        __shared__ double shd[1024];
        double m = 0.0;
        for (int k = threadIdx.x; k < kKeBlocks; k += blockDim.x) {
            const double u = d.disp[k];
            m = (u > m || u != u) ? u : m;
        }
        shd[threadIdx.x] = m;
        __syncthreads();
        for (int o = 512; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                const double u = shd[threadIdx.x + o];
                if (u > shd[threadIdx.x] || u != u) shd[threadIdx.x] = u;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double mm = sqrt(shd[0]);
            if (mm > d.disp[kKeBlocks]) d.disp[kKeBlocks] = mm;
            if (!(2.0 * mm < d.buffer)) d.disp[kKeBlocks + 1] += 1.0;
        }
    }
    const int GM = d.G * d.M;
    int carry_a = 0, carry_g = 0;
    for (int base = 0; base < d.n_cols; base += 1024) {
        const int c = base + threadIdx.x;
        const int cnt = c < d.n_cols ? gld(&d.col_count[c]) : 0;
        const int ng = (cnt + GM - 1) / GM;
        int tot_a, tot_g;
        int ea = block_exclusive_scan(cnt, smem, &tot_a);
        int eg = block_exclusive_scan(ng, smem, &tot_g);
        if (c < d.n_cols) {
            gst(&d.col_start[c], carry_a + ea);
            gst(&d.col_gstart[c], carry_g + eg);
        }
        carry_a += tot_a;
        carry_g += tot_g;
    }
    if (threadIdx.x == 0) {
        d.col_start[d.n_cols] = carry_a;
        d.col_gstart[d.n_cols] = carry_g;
        int ng = carry_g;
        if (ng > d.max_groups) {
            d.status[ST_OVERFLOW] = 1;
            atomicMax(&d.status[ST_NEED_GROUPS], ng);
            ng = d.max_groups;
        }
        d.n_groups[0] = ng;
    }
}

// 3. scatter (z key, atom) into column segments: rank inside the block from an
//    LDS counter, one global reservation per (block, column); the per-column
//    sort makes the final order independent of the atomic order here.
__global__ __launch_bounds__(256) void k_scatter(const SysDev* __restrict__ table, const int* flags)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    __shared__ int cnt[kHistLds];
    __shared__ int base[kHistLds];
    const bool priv = d.n_cols <= kHistLds;
    if (priv)
        for (int c = threadIdx.x; c < d.n_cols; c += blockDim.x) cnt[c] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < d.n_atoms;
    int col = 0, rank = 0;
    if (valid) {
        col = d.atom_col[i];
        if (priv) rank = atomicAdd(&cnt[col], 1);
    }
    __syncthreads();
    if (priv)
        for (int c = threadIdx.x; c < d.n_cols; c += blockDim.x)
            if (cnt[c]) base[c] = gatomic_add(&d.col_fill[c], cnt[c]);
    __syncthreads();
    if (valid) {
        const int pos = d.col_start[col] + (priv ? base[col] + rank : gatomic_add(&d.col_fill[col], 1));
        d.sort_key[pos] = ((unsigned long long)d.atom_zkey[i] << 32) | (unsigned int)i;
    }
}

// 4a. per-column sort of the (z key, atom) words into sort_out, kColParts
//     blocks per column: each loads the column's keys into LDS and moves its
//     share of them to their rank (the keys are distinct: the atom index is in
//     the low word), so the column sort spreads over more CUs than there are
//     columns.  Longer columns: the first block sorts them with a bitonic
//     network, in LDS up to kSortLds keys, else in place in HBM.  The first
//     block also records each group's column.
constexpr int kColParts = 4;
constexpr int kColRankMax = 2048;  // longer columns: a bitonic network (the rank sort is quadratic)

__global__ __launch_bounds__(256) void k_col_sort(const SysDev* __restrict__ table, const int* flags)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    const int col = blockIdx.x / kColParts, part = blockIdx.x % kColParts;
    if (col >= d.n_cols) return;
    const int n = gld(&d.col_count[col]);
    const int base = gld(&d.col_start[col]);
    if (part == 0) {
        // each group's column and its chunk of the column's sorted keys
        const int GM = d.G * d.M;
        const int g_begin = gld(&d.col_gstart[col]);
        const int n_grp = gld(&d.col_gstart[col + 1]) - g_begin;
        for (int t = threadIdx.x; t < n_grp; t += blockDim.x)
            if (g_begin + t < d.max_groups) {
                gst(&d.grp_col[g_begin + t], col);
                gst(&d.grp_range[g_begin + t], make_int2(base + t * GM, min(GM, n - t * GM)));
            }
    }
    __shared__ __align__(16) unsigned long long skeys[kSortLds + 2];
    if (n <= kColRankMax) {
        const int per = kColParts * (int)blockDim.x;
        if (part * (int)blockDim.x >= n) return;  // no key of this part
        for (int t = threadIdx.x; t < n; t += blockDim.x) skeys[t] = gld(&d.sort_key[base + t]);
        if (threadIdx.x == 0) skeys[n] = ~0ull;  // pad: above every key
        __syncthreads();
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
        const u64x2* kv = (const u64x2*)skeys;
        for (int t0 = part * (int)blockDim.x; t0 < n; t0 += per) {
            const int t = t0 + (int)threadIdx.x;
            const unsigned long long k = t < n ? skeys[t] : ~0ull;
            int r = 0;
#pragma unroll 4
            for (int u = 0; u < (n + 1) / 2; ++u) {
                const u64x2 ku = kv[u];
                r += (ku.x < k ? 1 : 0) + (ku.y < k ? 1 : 0);
            }
            if (t < n) gst(&d.sort_out[base + r], k);
        }
    } else if (part == 0) {
        int P = 1;
        while (P < n) P <<= 1;
        if (n <= kSortLds) {
            for (int t = threadIdx.x; t < n; t += blockDim.x) skeys[t] = gld(&d.sort_key[base + t]);
            __syncthreads();
            bitonic_sort(skeys, n, P);
            for (int t = threadIdx.x; t < n; t += blockDim.x) gst(&d.sort_out[base + t], skeys[t]);
        } else {
            if (threadIdx.x == 0) d.status[ST_BIGCOL] = 1;
            bitonic_sort(d.sort_key + base, n, P);  // block-coherent in HBM
            __syncthreads();
            for (int t = threadIdx.x; t < n; t += blockDim.x) d.sort_out[base + t] = d.sort_key[base + t];
        }
    }
}

// 4b. one wave per i-group: the 2x2x2 split of its chunk of 8*M atoms (in z
//     order) into 8 clusters of M atoms, its slots and bounding boxes
// (one wave per block: the groups are independent, so a block barrier only
//  orders one wave's LDS traffic, and the groups spread over all CUs)
constexpr int kSplitWaves = 1;

__global__ __launch_bounds__(64 * kSplitWaves) void k_group_split(const SysDev* __restrict__ table, const int* flags)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    const int M = d.M, G = d.G, GM = G * M;
    __shared__ double px[kSplitWaves][64], py[kSplitWaves][64], pz[kSplitWaves][64];
    __shared__ double pq[kSplitWaves][64], psg[kSplitWaves][64], pep[kSplitWaves][64];  // charge, sigma, epsilon
    __shared__ unsigned int kx[kSplitWaves][64], ky[kSplitWaves][64];
    __shared__ int pid[kSplitWaves][64], pk[kSplitWaves][64], pyh[kSplitWaves][64], pslot[kSplitWaves][64];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    {
        const int gg = blockIdx.x * kSplitWaves + wid;
        // the group's key range (written by the column sort) is loaded together
        // with the group count (gg < max_groups: in bounds either way)
        const int ng_now = gld(&d.n_groups[0]);
        const int2 rg = gld(&d.grp_range[min(gg, d.max_groups - 1)]);
        const bool active = gg < ng_now;
        const int cnt = active ? rg.y : 0;
        const unsigned long long* keys = d.sort_out + (active ? rg.x : 0);
        // load chunk atoms: every load of the lane's atom at once (positions,
        // image counts, the staging's parameters); the lane keeps the original
        // position and image counts for the slot arrays below
        double xo[3] = {0.0, 0.0, 0.0};
        int wo[3] = {0, 0, 0};
        if (lane < cnt) {
            const unsigned long long key = gld(keys + lane);
            const int idx = (int)(key & 0xffffffffull);
            for (int c = 0; c < 3; ++c) {
                xo[c] = gld(&d.x[3 * idx + c]);
                wo[c] = gld(&d.atom_wrap[3 * idx + c]);
            }
            const double qv = gld(&d.q[idx]);
            const double sgv = d.lj == 1 ? gld(&d.sig[idx]) : 0.0;
            const double epv = d.lj == 1 ? gld(&d.eps[idx]) : 0.0;
            double u[3];
            wrapped_pos(d, xo, wo, u);
            px[wid][lane] = u[0];
            py[wid][lane] = u[1];
            pz[wid][lane] = u[2];
            pid[wid][lane] = idx;
            pq[wid][lane] = qv;
            psg[wid][lane] = sgv;
            pep[wid][lane] = epv;
            // integer rank keys (a strict total order with the atom index, also for
            // non-finite input)
            kx[wid][lane] = coord_key(px[wid][lane], d.invbox[0]);
            ky[wid][lane] = coord_key(py[wid][lane], d.invbox[1]);
        }
        __syncthreads();
        // z half by position in the z order, y half by rank in the z half
        const int H = 4 * M;
        int zh = 0, yh = 0, myk = 0, myp = 0;
        if (lane < cnt) {
            zh = lane >= H ? 1 : 0;
            const int lo = zh * H, hi = min(cnt, lo + H);
            const unsigned int yme = ky[wid][lane];
            const int ime = pid[wid][lane];
            int yr = 0;
            for (int m = lo; m < hi; ++m) {
                const unsigned int ym = ky[wid][m];
                yr += (ym < yme || (ym == yme && pid[wid][m] < ime)) ? 1 : 0;
            }
            yh = yr >= 2 * M ? 1 : 0;
            pyh[wid][lane] = yh;
        }
        __syncthreads();
        if (lane < cnt) {
            const int lo = zh * H, hi = min(cnt, lo + H);
            const unsigned int xme = kx[wid][lane];
            const int ime = pid[wid][lane];
            int xr = 0;
            for (int m = lo; m < hi; ++m) {
                if (pyh[wid][m] != yh) continue;
                const unsigned int xm = kx[wid][m];
                xr += (xm < xme || (xm == xme && pid[wid][m] < ime)) ? 1 : 0;
            }
            const int xh = xr >= M ? 1 : 0;
            myk = zh * 4 + yh * 2 + xh;
            myp = xr - xh * M;
            const int slot = (gg * G + myk) * M + myp;
            pk[wid][lane] = myk;
            gst(&d.slot_atom[slot], pid[wid][lane]);
            for (int c = 0; c < 3; ++c) {
                gst(&d.slot_wrap[3 * slot + c], wo[c]);
                gst(&d.slot_x[3 * slot + c], xo[c]);
            }
        }
        __syncthreads();
        // cluster bounding boxes: move every atom to the lane of its slot in the
        // group (lane = k*M + p), then min/max over the M lanes of each cluster
        // and over all lanes for the group box, with shuffles
        if (lane < GM) pslot[wid][lane] = -1;
        __syncthreads();
        if (lane < cnt) {
            const int q = myk * M + myp;
            pslot[wid][q] = lane;
        }
        __syncthreads();
        if (active) {
            const int src = lane < GM ? pslot[wid][lane] : -1;
            const bool real = src >= 0;
            double lo[3], hi[3];
            lo[0] = real ? px[wid][src] : 1e300;
            lo[1] = real ? py[wid][src] : 1e300;
            lo[2] = real ? pz[wid][src] : 1e300;
            for (int k = 0; k < 3; ++k) hi[k] = real ? lo[k] : -1e300;
            const unsigned long long rb = __ballot(real);
            for (int o = 1; o < M; o <<= 1)
                for (int k = 0; k < 3; ++k) {
                    lo[k] = fmin(lo[k], __shfl_xor(lo[k], o, 64));
                    hi[k] = fmax(hi[k], __shfl_xor(hi[k], o, 64));
                }
            if (lane < GM && (lane % M) == 0) {
                const int k = lane / M;
                const int ci = gg * G + k;
                const unsigned long long cm = (M >= 64) ? ~0ull : (((1ull << M) - 1ull) << lane);
                gst(&d.cl_nreal[ci], (int)__popcll(rb & cm));
                for (int c = 0; c < 3; ++c) {
                    gst(&d.cl_bb[6 * ci + c], lo[c]);
                    gst(&d.cl_bb[6 * ci + 3 + c], hi[c]);
                }
            }
            for (int o = M; o < 64; o <<= 1)
                for (int k = 0; k < 3; ++k) {
                    lo[k] = fmin(lo[k], __shfl_xor(lo[k], o, 64));
                    hi[k] = fmax(hi[k], __shfl_xor(hi[k], o, 64));
                }
            double ref[3];
            for (int c = 0; c < 3; ++c) ref[c] = 0.5 * (lo[c] + hi[c]);
            if (lane == 0)
                for (int c = 0; c < 3; ++c) {
                    gst(&d.gr_bb[6 * gg + c], lo[c]);
                    gst(&d.gr_bb[6 * gg + 3 + c], hi[c]);
                    gst(&d.gr_ref[3 * gg + c], ref[c]);
                }
            // stage the group's slots at these positions (the force kernel's
            // frame; the same arithmetic as every other staging)
            if (lane < GM) {
                const int slot = gg * GM + lane;
                float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
                float2 l = make_float2(0.f, 0.f);
                if (real) {
                    // px is the wrapped position of stage_pos (FP64, no
                    // contraction), so (float)(px - ref) is the staged value
                    p.x = (float)(px[wid][src] - ref[0]);
                    p.y = (float)(py[wid][src] - ref[1]);
                    p.z = (float)(pz[wid][src] - ref[2]);
                    p.w = (float)(pq[wid][src] * (double)d.qscale);
                    if (d.lj == 1) {
                        l.x = (float)(0.5 * psg[wid][src]);
                        l.y = (float)(2.0 * sqrt(pep[wid][src]));
                    }
                }
                gst(&d.xq[slot], p);
                if (d.lj == 1) gst(&d.ljs[slot], l);
            }
        }
        __syncthreads();
    }
}

// 5. bounding-box search: one block of 8 waves per i-group; the waves share
//    out the column cells within reach, and a wave tests 8 j-clusters against
//    the 8 i-clusters of the group at once (lane = j * 8 + i-cluster), so the
//    byte j of the ballot is that j-cluster's i-cluster mask.  Candidates are
//    appended in any order, then sorted by (j-cluster, shift) so the list is
//    canonical (deterministic) and j-ordered for cache locality.  Each
//    candidate's mask is then pruned at the atom level in FP32 (below).
constexpr int kCandLds = 4096;
constexpr int kSearchWaves = 8;
constexpr int kPruneXj = 2048;  // shifted j-atoms staged per chunk of candidates

// fast: the FP32-pruned candidates are the list (kept count set here);
// otherwise the exact FP64 prune follows.  TRIC: some system of the launch has
// a triclinic box (the rectangular-only variant leaves that search out)
// M8: every system of the launch has 8-atom clusters (the cluster size a
// compile-time constant: the code for other sizes, and the scalar registers it
// holds, drop out of the variant)
template <bool TRIC, bool M8>
__global__ __launch_bounds__(64 * kSearchWaves) void k_search(const SysDev* __restrict__ table, const int* flags,
                                                              int fast)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    const int gi = blockIdx.x;
    if (gi >= d.n_groups[0]) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    __shared__ __align__(16) unsigned long long keys_lds[kCandLds];
    __shared__ double ibb[kGroup][6];
    __shared__ float4 ixq[64];      // the group's staged i-atoms (slot order)
    __shared__ float4 xjs[kPruneXj];
    __shared__ int inr_s[kGroup];   // real atoms per i-cluster
    __shared__ int ireal_s;
    __shared__ int count_s, kept_s, kw_s;
    const int G = d.G;
    const int M = M8 ? 8 : d.M;
    if (threadIdx.x < kGroup * 6) ibb[threadIdx.x / 6][threadIdx.x % 6] = d.cl_bb[6 * (gi * G) + threadIdx.x];
    if (threadIdx.x < G * M) ixq[threadIdx.x] = d.xq[(size_t)gi * G * M + threadIdx.x];
    if (threadIdx.x < kGroup) inr_s[threadIdx.x] = d.cl_nreal[gi * G + threadIdx.x];
    if (threadIdx.x == 0) {
        count_s = 0;
        kept_s = 0;
        kw_s = 0;
        int m = 0;
        for (int g = 0; g < kGroup; ++g) m |= (d.cl_nreal[gi * G + g] > 0) ? (1 << g) : 0;
        ireal_s = m;
    }
    const double rl = d.rbb;
    const double rl2 = rl * rl;
    double gb[6];
    for (int k = 0; k < 6; ++k) gb[k] = d.gr_bb[6 * gi + k];
    const int ci0 = gi * G;
    const int ng_tot = d.n_groups[0];
    const int cap = d.cand_cap;
    // the group's column (unwrapped cell coordinates of the search start there)
    const int colg = gld(&d.grp_col[gi]);
    const int cxi = colg % d.ncx, cyi = colg / d.ncx;
    // keys past the LDS array are staged in the group's own candidate region
    // (8 bytes each)
    unsigned long long* gkeys = (unsigned long long*)(d.cand + (size_t)gi * cap);
    bool finite = true;
    for (int k = 0; k < 6; ++k) finite = finite && (fabs(gb[k]) < 1e9);
    __syncthreads();
    // this lane's i-cluster and its box
    const int g = lane & 7, jj = lane >> 3;
    const bool ireal = (ireal_s >> g) & 1;
    double ib[6];
    for (int k = 0; k < 6; ++k) ib[k] = ibb[g][k];
    if (finite) {
        const int ci = ci0 + g;
        // Test the j-clusters [c_lo, c_hi) of one column, 8 per wave
        // instruction (lane = j * 8 + i-cluster), with the j offset (ox, oy)
        // in x and y and each z image t of tmask (z shift t - 1, offset
        // (t - 1) c_z); the boxes of a chunk are loaded once (all loads issued
        // together) and the next chunk's are in flight while it is tested.  The
        // group owns the pair in its own column (no x/y shift) with the z shift
        // +1, or without a z shift with cj >= ci (cj == ci: the cluster with
        // itself).
        auto scan_col = [&](int c_lo, int c_hi, int sx, int sy, bool own_col, unsigned int tmask, double ox,
                            double oy) {
            int nrj_n = 0;
            double bn[6];
            auto load_chunk = [&](int cb) {
                const int cjc = min(cb + jj, c_hi - 1);
                nrj_n = gld(&d.cl_nreal[cjc]);
                const double* bb = d.cl_bb + 6 * cjc;
                for (int k = 0; k < 6; ++k) bn[k] = gld(bb + k);
            };
            load_chunk(c_lo);
            for (int cb = c_lo; cb < c_hi; cb += 8) {
                const int cj = cb + jj;
                const int nrj = nrj_n;
                const double b0 = bn[0], b1 = bn[1], b2 = bn[2], b3 = bn[3], b4 = bn[4], b5 = bn[5];
                if (cb + 8 < c_hi) load_chunk(cb + 8);
                const bool okj = cj < c_hi && ireal && nrj > 0;
                const double fx = box_gap(ib[0], ib[3], b0 + ox, b3 + ox);
                const double fy = box_gap(ib[1], ib[4], b1 + oy, b4 + oy);
                const double fxy = fx * fx + fy * fy;
                for (int t = 0; t < 3; ++t) {
                    if (!((tmask >> t) & 1u)) continue;
                    const double zoff = (t - 1) * d.box[2];
                    const double fz = box_gap(ib[2], ib[5], b2 + zoff, b5 + zoff);
                    const int sid = shift_id(sx, sy, t - 1);
                    const bool owns = !own_col || t == 2 || (t == 1 && cj >= ci);
                    const bool hit = okj && owns && fxy + fz * fz < rl2;
                    const unsigned long long bal = __ballot(hit);
                    if (bal == 0ull) continue;
                    // byte jj of the ballot: the i-cluster mask of j-cluster cb + jj
                    const unsigned long long nz = __ballot(g == 0 && ((bal >> (8 * jj)) & 255ull) != 0ull);
                    const int n = __popcll(nz);
                    int base = 0;
                    if (lane == 0) base = atomicAdd(&count_s, n);  // LDS atomic
                    base = __shfl(base, 0, 64);
                    if ((nz >> lane) & 1ull) {
                        const int pos = base + __popcll(nz & ((1ull << lane) - 1ull));
                        const unsigned long long im = (bal >> (8 * jj)) & 255ull;
                        // appended into LDS; only keys past the LDS array go to HBM
                        const unsigned long long key =
                            ((unsigned long long)cj << 16) | ((unsigned long long)sid << 8) | im;
                        if (pos < min(cap, kCandLds)) keys_lds[pos] = key;
                        else if (pos < cap) gst(gkeys + pos, key);
                    }
                }
            }
        };
        // Half list by half-space, the same share for every group: in unwrapped
        // cell coordinates (periodic images included) the group owns its pairs
        // with the columns above it in y, with those above it in x in its own
        // row, and in its own column as above.  Seen from the other cluster a
        // pair has the opposite offset, so every cluster pair and shift is
        // listed once.  The cell coordinates count lattice images, not
        // distances, so the rule holds in triclinic boxes too.
        if (!TRIC || !d.tric) {
            // gb lies in [0, L) and r_list < L/2, so the ranges span at most [-n, 2n)
            const int cx0 = max(-d.ncx, (int)floor((gb[0] - rl) * d.inv_cell[0]));
            const int cx1 = min(2 * d.ncx - 1, (int)floor((gb[3] + rl) * d.inv_cell[0]));
            const int cy0 = max(-d.ncy, (int)floor((gb[1] - rl) * d.inv_cell[1]));
            const int cy1 = min(2 * d.ncy - 1, (int)floor((gb[4] + rl) * d.inv_cell[1]));
            const int nxc = cx1 - cx0 + 1;
            const int ncell = nxc * (cy1 - cy0 + 1);
            for (int cell = wid; cell < ncell; cell += kSearchWaves) {
                const int cy = cy0 + cell / nxc, cx = cx0 + cell % nxc;
                const int dcy = cy - cyi, dcx = cx - cxi;
                if (dcy < 0 || (dcy == 0 && dcx < 0)) continue;
                const bool own_col = dcy == 0 && dcx == 0;
                const int sy = floor_div(cy, d.ncy);
                const int cyw = cy - sy * d.ncy;
                const double ylo = cyw * d.cell[1] + sy * d.box[1];
                const double gy = box_gap(gb[1], gb[4], ylo, ylo + d.cell[1]);
                const int sx = floor_div(cx, d.ncx);
                const int cxw = cx - sx * d.ncx;
                const double xlo = cxw * d.cell[0] + sx * d.box[0];
                const double gx = box_gap(gb[0], gb[3], xlo, xlo + d.cell[0]);
                if (gx * gx + gy * gy >= rl2) continue;
                const int col = cxw + d.ncx * cyw;
                const int g0 = gld(&d.col_gstart[col]);
                const int g1 = min(gld(&d.col_gstart[col + 1]), ng_tot);
                if (g0 >= g1) continue;
                // the (up to 3) periodic z images in reach: j images occupy [zoff, zoff + L)
                unsigned int tmask = 0u;
                for (int t = 0; t < 3; ++t) {
                    const double zoff = (t - 1) * d.box[2];
                    if (!(gb[2] - rl >= zoff + d.box[2] || gb[5] + rl < zoff)) tmask |= 1u << t;
                }
                scan_col(g0 * G, g1 * G, sx, sy, own_col, tmask, sx * d.box[0], sy * d.box[1]);
            }
        } else {
            // triclinic: the j-image with lattice shift (sx, sy, sz) of column
            // (cxw, cyw) is offset by sx a + sy b + sz c, so each z image moves the
            // cells in x and y (sz c_x, sz c_y) and each y image moves a row in x
            // (sy b_x); per z image the rows in reach, per row its cells
            const int nxc = (int)floor((gb[3] - gb[0] + 2.0 * rl) * d.inv_cell[0]) + 2;
            for (int t = 0; t < 3; ++t) {
                const int sz = t - 1;
                const double zoff = sz * d.box[2];
                if (gb[2] - rl >= zoff + d.box[2] || gb[5] + rl < zoff) continue;
                const double cxo = sz * d.box_off[1], cyo = sz * d.box_off[2];
                const int cy0 = (int)floor((gb[1] - rl - cyo) * d.inv_cell[1]);
                const int cy1 = (int)floor((gb[4] + rl - cyo) * d.inv_cell[1]);
                const int ncell = nxc * (cy1 - cy0 + 1);
                for (int cell = wid; cell < ncell; cell += kSearchWaves) {
                    const int cy = cy0 + cell / nxc;
                    const int sy = floor_div(cy, d.ncy);
                    const int cyw = cy - sy * d.ncy;
                    const double xo = sy * d.box_off[0] + cxo;  // this row's image offset in x (without sx)
                    const int cx = (int)floor((gb[0] - rl - xo) * d.inv_cell[0]) + cell % nxc;
                    if (cx > (int)floor((gb[3] + rl - xo) * d.inv_cell[0])) continue;
                    const int dcy = cy - cyi, dcx = cx - cxi;
                    if (dcy < 0 || (dcy == 0 && dcx < 0)) continue;
                    const bool own_col = dcy == 0 && dcx == 0;
                    if (own_col && sz < 0) continue;  // (owned from the other side)
                    const int sx = floor_div(cx, d.ncx);
                    const int cxw = cx - sx * d.ncx;
                    const double ylo = cyw * d.cell[1] + sy * d.box[1] + cyo;
                    const double gy = box_gap(gb[1], gb[4], ylo, ylo + d.cell[1]);
                    const double xlo = cxw * d.cell[0] + sx * d.box[0] + xo;
                    const double gx = box_gap(gb[0], gb[3], xlo, xlo + d.cell[0]);
                    if (gx * gx + gy * gy >= rl2) continue;
                    const int col = cxw + d.ncx * cyw;
                    const int g0 = gld(&d.col_gstart[col]);
                    const int g1 = min(gld(&d.col_gstart[col + 1]), ng_tot);
                    if (g0 >= g1) continue;
                    scan_col(g0 * G, g1 * G, sx, sy, own_col, 1u << t, sx * d.box[0] + xo, sy * d.box[1] + cyo);
                }
            }
        }
    }
    __syncthreads();
    const int count = count_s;
    const int n = min(count, cap);
    int P = 1;
    while (P < n) P <<= 1;
    // sorted in LDS when they fit, else in place in HBM (each branch with its
    // own address space, so LDS accesses are not flat ones)
    const bool in_lds = n <= kCandLds;
    if (in_lds) {
        // the keys are distinct (one per j-cluster and shift)
        if (n <= 2 * 64 * kSearchWaves && n < kCandLds) rank_sort_lds(keys_lds, n);
        else bitonic_sort(keys_lds, n, P);
    } else {
        for (int t = threadIdx.x; t < kCandLds; t += blockDim.x) gst(gkeys + t, keys_lds[t]);
        __syncthreads();
        bitonic_sort(gkeys, n, P);
    }
    __syncthreads();
    // keys -> candidate words, in chunks (in place: a chunk's keys are read
    // before its words are written).  The i-cluster mask of each candidate is
    // pruned in the force kernel's FP32 frame (the positions staged at this
    // build, the entry's FP32 shift vector): a bit stays if the cluster pair has
    // an atom pair within r_list (1 + 2^-14), a margin far above that frame's
    // rounding, so every cluster pair the exact FP64 test keeps is kept.
    //  (a) one thread per (candidate, j-atom): the shifted j-atoms of the chunk
    //      into LDS (w = 1 for a real atom), all loads in flight together;
    //  (b) one wave per candidate: pair p = k*64 + lane of the group's
    //      8*M*M pairs is (i-cluster p/(M*M), i-atom (p/M) mod M, j-atom p mod M),
    //      as in the exact prune's mask words; which lanes hold a pair to test
    //      is a scalar lane mask, so each pair costs a difference, r^2 and a
    //      compare.
    const int LM = (M == 8) ? 3 : (M == 4) ? 2 : 0;  // M is 1, 4 or 8
    const int MM = M * M;
    const int K = (kGroup * MM + 63) / 64;  // 64-pair words per cluster pair
    const float rlp = d.rl2_prune;
    const double ri[3] = {d.gr_ref[3 * gi], d.gr_ref[3 * gi + 1], d.gr_ref[3 * gi + 2]};
    // this lane's i-atom of word k (registers); the real atoms of i-cluster g,
    // 4 bits each, in one scalar
    float4 xr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int p = k * 64 + lane;
        xr[k] = (k < K && p < kGroup * MM) ? ixq[p >> LM] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    unsigned int inr_pk = 0u;
    for (int g = 0; g < kGroup; ++g) inr_pk |= (unsigned int)inr_s[g] << (4 * g);
    inr_pk = (unsigned int)__builtin_amdgcn_readfirstlane((int)inr_pk);
    const unsigned long long segm = (MM >= 64) ? ~0ull : ((1ull << MM) - 1ull);
    const unsigned long long tri8 = __ballot((lane >> 3) < (lane & 7));  // M = 8: a < b
    // a wave's kept candidates and their weight (wave-uniform), added to the
    // group's totals once at the end
    int kept_w = 0, kw_w = 0;
    for (int t0 = 0; t0 < n; t0 += kPruneXj / M) {
        const int cnt = min(n - t0, kPruneXj / M);
        // the chunk's keys are read from LDS only (keys sorted in HBM are
        // copied into the then unused key array first), so no read below
        // waits on the stores of the candidate words
        int k0 = t0;
        if (!in_lds) {
            for (int q = threadIdx.x; q < cnt; q += blockDim.x) keys_lds[q] = gld(gkeys + t0 + q);
            __syncthreads();
            k0 = 0;
        }
        // (a) a fixed number of items per thread with clamped indices: all their
        //     loads are issued first, then the shifts are formed
        constexpr int kU = kPruneXj / (64 * kSearchWaves);
        float4 xjv[kU];
        double rjv[kU][3];
        int nrv[kU], sidv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int qc = min((int)threadIdx.x + u * 64 * kSearchWaves, cnt * M - 1);
            const unsigned long long kv = keys_lds[k0 + (qc >> LM)];
            const int cj = (int)(kv >> 16), gj = cj / G;
            sidv[u] = (int)((kv >> 8) & 255ull);
            xjv[u] = gld(&d.xq[(size_t)cj * M + (qc & (M - 1))]);
            nrv[u] = gld(&d.cl_nreal[cj]);
            for (int c = 0; c < 3; ++c) rjv[u][c] = gld(&d.gr_ref[3 * gj + c]);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int q = threadIdx.x + u * 64 * kSearchWaves;
            const float4 S = entry_shift(d, rjv[u], sidv[u], ri);
            if (q < cnt * M)
                xjs[q] = make_float4(xjv[u].x + S.x, xjv[u].y + S.y, xjv[u].z + S.z,
                                     (q & (M - 1)) < nrv[u] ? 1.0f : 0.0f);
        }
        __syncthreads();
        // (b) the next candidate's key and j-atoms are read while this one is tested
        unsigned long long kv_n = 0ull;
        float4 xj_n = make_float4(0.f, 0.f, 0.f, 0.f);
        if (wid < cnt) {
            kv_n = keys_lds[k0 + wid];
            xj_n = xjs[wid * M + (lane & (M - 1))];
        }
        // the wave's q-th candidate of the chunk is recorded by lane q mod 64;
        // its word (and the j-cluster count) is written with the wave's others
        // once 64 are recorded or the chunk ends: one store for them all
        int rec_c = -1, rec_cj = 0, rec_w = 0;
        auto write_recorded = [&]() {
            if (rec_c >= 0) {
                gst(&d.cand[(size_t)gi * cap + t0 + rec_c], make_int2(rec_cj, rec_w));
                // the list's entries per j-cluster (the transpose's counts)
                if (fast && (rec_w >> 8) != 0) gatomic_add(&d.jfill[rec_cj], 1);
            }
            rec_c = -1;
        };
        for (int c = wid; c < cnt; c += kSearchWaves) {
            // key = cj << 16 | sid << 8 | imask (the same for the whole wave)
            const unsigned long long kv = kv_n;
            const float4 xj = xj_n;
            if (c + kSearchWaves < cnt) {
                kv_n = keys_lds[k0 + c + kSearchWaves];
                xj_n = xjs[(c + kSearchWaves) * M + (lane & (M - 1))];
            }
            const int cj = __builtin_amdgcn_readfirstlane((int)(kv >> 16));
            const int sid = __builtin_amdgcn_readfirstlane((int)((kv >> 8) & 255ull));
            const unsigned int im = (unsigned int)__builtin_amdgcn_readfirstlane((int)(kv & 255ull));
            const unsigned long long jm = __ballot(xj.w != 0.0f);
            // a cluster with itself at zero shift: each pair once (a < b)
            const int gself = __builtin_amdgcn_readfirstlane((sid == kShiftZero) ? cj - ci0 : -1);
            unsigned int keep = 0u;
            if (M == 8) {
                // word g = i-cluster g: lanes (a, b) with a < nr_g, real b;
                // with itself at zero shift also a < b
#pragma unroll
                for (int g = 0; g < kGroup; ++g) {
                    if (!((im >> g) & 1u)) continue;
                    const int nl = (int)((inr_pk >> (4 * g)) & 15u) * 8;
                    unsigned long long on = (nl >= 64 ? ~0ull : ((1ull << nl) - 1ull)) & jm;
                    if (g == gself) on &= tri8;
                    if (on == 0ull) continue;
                    const float dx = xr[g].x - xj.x, dy = xr[g].y - xj.y, dz = xr[g].z - xj.z;
                    if (__ballot(fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < rlp) & on) keep |= 1u << g;
                }
            } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k >= K) break;
                // i-clusters of word k, and its lanes that hold a pair to test:
                // the first nr*M lanes of i-cluster g's MM lanes (real i-atoms)
                const int glo = (k * 64) >> (2 * LM), ghi = min(kGroup - 1, (k * 64 + 63) >> (2 * LM));
                unsigned long long on = 0ull;
                for (int g = glo; g <= ghi; ++g) {
                    if (!((im >> g) & 1u)) continue;
                    const int nl = (int)((inr_pk >> (4 * g)) & 15u) * M;
                    unsigned long long sg = (nl >= 64 ? ~0ull : ((1ull << nl) - 1ull)) << ((g * MM) & 63);
                    if (g == gself) sg &= __ballot(((k * 64 + lane) >> LM & (M - 1)) < (lane & (M - 1)));
                    on |= sg;
                }
                on &= jm;
                if (on == 0ull) continue;
                const float dx = xr[k].x - xj.x, dy = xr[k].y - xj.y, dz = xr[k].z - xj.z;
                const unsigned long long hit = __ballot(fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < rlp) & on;
                for (int g = glo; g <= ghi; ++g)
                    if (hit & (segm << ((g * MM) & 63))) keep |= 1u << g;
            }
            }
            if (keep) {
                kept_w += 1;
                kw_w += entry_weight(M, keep);
            }
            const int q = (c - wid) / kSearchWaves;
            if (lane == (q & 63)) {
                rec_c = c;
                rec_cj = cj;
                rec_w = sid | (int)(keep << 8);
            }
            if ((q & 63) == 63) write_recorded();
        }
        write_recorded();
        __syncthreads();
    }
    if (lane == 0 && kept_w > 0) {
        atomicAdd(&kept_s, kept_w);  // LDS atomics
        atomicAdd(&kw_s, kw_w);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        d.cand_count[gi] = count;
        if (fast) {  // the FP32-pruned candidates are the list
            d.cand_kept[gi] = kept_s;
            d.grp_w[gi] = kw_s;
            d.grp_rc[gi] = 0;
        }
        if (count > cap) {
            d.status[ST_OVERFLOW] = 1;
            atomicMax(&d.status[ST_NEED_CAND], count);
        }
    }
}

// 6. exact FP64 atom-pair prune: kPruneBlocks blocks of 4 waves per i-group,
//    waves stride over the group's candidates, one atom pair per lane.  The
//    new i-cluster mask and the pairs-within-r_cut count go back into the
//    candidate word.
constexpr int kPruneBlocks = 8;

// refine: masks and pair count only; the candidate's i-cluster mask (the one the
// force list was written from) is left as it is
__global__ __launch_bounds__(256) void k_prune(const SysDev* __restrict__ table, const int* flags, int refine)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    const int gi = blockIdx.x / kPruneBlocks;
    if (gi >= d.n_groups[0]) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wg = (blockIdx.x % kPruneBlocks) * 4 + wid;
    const int lane = threadIdx.x & 63;
    const int M = d.M, G = d.G, MM = M * M, GM = G * M;
    const int ncand = min(d.cand_count[gi], d.cand_cap);
    const int words = d.mask_words;  // <= 8: G * M * M / 64 rounded up, M <= 8
    // the group's i-atoms (<= 64 slots), shared by the block's 4 waves; a
    // padding slot has atom -1
    __shared__ double ix[64][3];
    __shared__ int iw[64][3];
    __shared__ int ireal[64];
    if (threadIdx.x < GM) {
        const int sa = gi * GM + threadIdx.x;
        const bool real = d.slot_atom[sa] >= 0;
        ireal[threadIdx.x] = real ? 1 : 0;
        for (int q = 0; q < 3; ++q) {
            ix[threadIdx.x][q] = real ? d.slot_x[3 * sa + q] : 0.0;
            iw[threadIdx.x][q] = real ? d.slot_wrap[3 * sa + q] : 0;
        }
    }
    __syncthreads();
    if (wg >= ncand) return;
    // word p, lane l is pair (k, a, b) with p*64 + l = k*M*M + a*M + b: its
    // i-atom is group slot (p*64 + l) / M, its j-atom b is the same in every word
    const int b = lane % M;
    const double box0 = d.box[0], box1 = d.box[1], box2 = d.box[2];
    const double off0 = d.box_off[0], off1 = d.box_off[1], off2 = d.box_off[2];  // b_x, c_x, c_y
    const double ib0 = d.invbox[0], ib1 = d.invbox[1], ib2 = d.invbox[2];
    const double rl2 = d.rlist2, rc2 = d.rcut2;
    // software pipeline: the next candidate and its j-atom are loaded while the
    // current one is tested
    int2 cd_n = d.cand[(size_t)gi * d.cand_cap + wg];
    int sb_n = cd_n.x * M + b;
    int jat_n = d.slot_atom[sb_n];
    double xb_n[3] = {d.slot_x[3 * sb_n], d.slot_x[3 * sb_n + 1], d.slot_x[3 * sb_n + 2]};
    int wb_n[3] = {d.slot_wrap[3 * sb_n], d.slot_wrap[3 * sb_n + 1], d.slot_wrap[3 * sb_n + 2]};
    for (int c = wg; c < ncand; c += kPruneBlocks * 4) {
        const size_t ce = (size_t)gi * d.cand_cap + c;
        const int2 cd = cd_n;
        const bool jreal = jat_n >= 0;
        const double xb[3] = {xb_n[0], xb_n[1], xb_n[2]};
        const int wb[3] = {wb_n[0], wb_n[1], wb_n[2]};
        if (c + kPruneBlocks * 4 < ncand) {
            cd_n = d.cand[ce + kPruneBlocks * 4];
            sb_n = cd_n.x * M + b;
            jat_n = d.slot_atom[sb_n];
            for (int q = 0; q < 3; ++q) {
                xb_n[q] = d.slot_x[3 * sb_n + q];
                wb_n[q] = d.slot_wrap[3 * sb_n + q];
            }
        }
        const int cj = cd.x;
        const int sid = cd.y & 255;
        const unsigned int im = (unsigned int)(cd.y >> 8) & 255u;
        const int s0 = sid % 5 - 2, s1 = (sid / 5) % 3 - 1, s2 = sid / 15 - 1;
        unsigned int newim = 0;
        int nrc = 0;
        for (int p = 0; p < words; ++p) {
            // i-clusters covered by this 64-pair word: [p*64/MM, (p*64+63)/MM]
            const int k_lo = (p * 64) / MM, k_hi = min(G - 1, (p * 64 + 63) / MM);
            const unsigned int wmask = ((2u << k_hi) - 1u) & ~((1u << k_lo) - 1u);
            if (!(im & wmask)) {  // no listed i-cluster in this word
                if (lane == 0) d.cand_mask[ce * words + p] = 0ull;
                continue;
            }
            const int pi = p * 64 + lane;
            const int k = pi / MM, a = (pi / M) % M, ia = min(pi / M, 63);
            bool bit = false, inrc = false;
            if (jreal && k < G && ((im >> k) & 1u) && ireal[ia] &&
                !(gi * G + k == cj && sid == kShiftZero && a >= b)) {
                // the minimum image as the pair-set definition takes it: the
                // nearest multiples of c, b, a removed from z, y, x in that
                // order (per dimension in a rectangular box)
                double e0 = xb[0] - ix[ia][0], e1 = xb[1] - ix[ia][1], e2 = xb[2] - ix[ia][2];
                const double k2 = rint(e2 * ib2);
                e0 = e0 - k2 * off1;
                e1 = e1 - k2 * off2;
                e2 = e2 - k2 * box2;
                const double k1 = rint(e1 * ib1);
                e0 = e0 - k1 * off0;
                e1 = e1 - k1 * box1;
                const double k0 = rint(e0 * ib0);
                e0 = e0 - k0 * box0;
                const bool own = (wb[0] - iw[ia][0] - (int)k0 == s0) && (wb[1] - iw[ia][1] - (int)k1 == s1) &&
                                 (wb[2] - iw[ia][2] - (int)k2 == s2);
                const double t = e0 * e0 + e1 * e1;
                const double r2 = t + e2 * e2;
                bit = own && (r2 < rl2);
                inrc = bit && (r2 < rc2);
            }
            nrc += __popcll(__ballot(inrc));
            const unsigned long long w = __ballot(bit);
            if (lane == 0) d.cand_mask[ce * words + p] = w;
            // i-clusters of this word with at least one pair: lanes k*MM.. of the word
            const unsigned long long per_k = (MM >= 64) ? ~0ull : ((1ull << MM) - 1ull);
            for (int kk = k_lo; kk <= k_hi; ++kk)
                if (w & (per_k << ((kk * MM) % 64))) newim |= 1u << kk;
        }
        const int y = refine ? (cd.y & 0xffff) : (sid | (int)(newim << 8));
        if (lane == 0) d.cand[ce] = make_int2(cj, y | (min(nrc, 4095) << 16));
    }
}

// 6b. kept candidates and pairs within r_cut per i-group (one wave per group);
//     count_j: also the list's entries per j-cluster (the transpose's counts)
__global__ __launch_bounds__(256) void k_count_kept(const SysDev* __restrict__ table, const int* flags, int count_j)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gi = blockIdx.x * 4 + wid;
    if (gi >= d.n_groups[0]) return;
    const int ncand = min(d.cand_count[gi], d.cand_cap);
    int kept = 0, nrc = 0, kw = 0;
    for (int cb = 0; cb < ncand; cb += 64) {
        const int c = cb + lane;
        int2 cd = make_int2(0, 0);
        if (c < ncand) cd = d.cand[(size_t)gi * d.cand_cap + c];
        const int y = cd.y;
        const bool kp = ((y >> 8) & 255) != 0;
        kept += __popcll(__ballot(kp));
        if (kp) kw += entry_weight(d.M, (unsigned int)(y >> 8));
        if (count_j && kp) gatomic_add(&d.jfill[cd.x], 1);
        nrc += (y >> 16) & 4095;
    }
    for (int o = 32; o > 0; o >>= 1) {
        nrc += __shfl_xor(nrc, o, 64);
        kw += __shfl_xor(kw, o, 64);
    }
    if (lane == 0) {
        d.cand_kept[gi] = kept;
        d.grp_w[gi] = kw;
        d.grp_rc[gi] = nrc;
    }
}

// 7. CSR offsets of kept entries and work items, and of the transpose (per
//    j-cluster, the rows of the entries that name it; the counts come from the
//    search or the exact prune, and go back to 0 for the list writer to place
//    the entries).  One block per system; item_prefix (one system only): the
//    prefix {0, items} the force kernel reads.
__global__ __launch_bounds__(1024) void k_list_scan(const SysDev* __restrict__ table, const int* flags,
                                                     int* item_prefix)
{
    if (flags && !flags[blockIdx.x]) return;
    const SysDev& d = table[blockIdx.x];
    __shared__ int smem[40];
    const int ng = d.n_groups[0];
    const int W = d.item_w;
    int carry_e = 0, carry_i = 0;
    for (int base = 0; base < ng; base += 1024) {
        const int g = base + threadIdx.x;
        const int kept = g < ng ? gld(&d.cand_kept[g]) : 0;
        const int nit = g < ng ? (gld(&d.grp_w[g]) + W - 1) / W : 0;
        int te, ti;
        const int ee = block_exclusive_scan(kept, smem, &te);
        const int ei = block_exclusive_scan(nit, smem, &ti);
        if (g < ng) {
            gst(&d.ent_start[g], carry_e + ee);
            gst(&d.item_start[g], carry_i + ei);
        }
        carry_e += te;
        carry_i += ti;
    }
    if (threadIdx.x == 0) {
        d.ent_start[ng] = carry_e;
        d.item_start[ng] = carry_i;
        int ne = carry_e, ni = carry_i;
        if (ne > d.ent_cap) {
            d.status[ST_OVERFLOW] = 1;
            atomicMax(&d.status[ST_NEED_ENT], ne);
        }
        if (ni > d.item_cap) {
            d.status[ST_OVERFLOW] = 1;
            atomicMax(&d.status[ST_NEED_ITEM], ni);
        }
        const bool over = ne > d.ent_cap || ni > d.item_cap;
        d.n_ent[0] = over ? 0 : ne;
        d.n_items[0] = over ? 0 : ni;
        if (item_prefix) {
            item_prefix[0] = 0;
            item_prefix[1] = over ? 0 : ni;
        }
    }
    const int ncl = ng * d.G;
    int carry = 0;
    for (int base = 0; base < ncl; base += 1024) {
        const int c = base + threadIdx.x;
        const int v = c < ncl ? gld(&d.jfill[c]) : 0;
        int tot;
        const int ex = block_exclusive_scan(v, smem, &tot);
        if (c < ncl) {
            gst(&d.jstart[c], carry + ex);
            gst(&d.jfill[c], 0);
        }
        carry += tot;
    }
    if (threadIdx.x == 0) d.jstart[ncl] = carry;
}

// 8. compacted entries, shift vectors and work items: one wave per i-group
__global__ __launch_bounds__(256) void k_list_write(const SysDev* __restrict__ table, const int* flags)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gi = blockIdx.x * 4 + wid;
    if (gi >= d.n_groups[0]) return;
    if (d.n_ent[0] == 0) return;  // empty list, or overflow: list unusable
    const int G = d.G, M = d.M;
    const int W = d.item_w;
    const int ncand = min(d.cand_count[gi], d.cand_cap);
    const int e0 = d.ent_start[gi];
    const int e1 = d.ent_start[gi + 1];
    const double ri[3] = {d.gr_ref[3 * gi], d.gr_ref[3 * gi + 1], d.gr_ref[3 * gi + 2]};
    const int it0 = d.item_start[gi];
    const int nit = d.item_start[gi + 1] - it0;
    // the group's weight wg is cut into its nit = ceil(wg / W) items at the
    // points floor(k wg / nit), so its items weigh the same (not nit - 1 of W
    // and a remainder); when those points lie closer together than an entry
    // can weigh, at the multiples of W instead
    const long long wg = d.grp_w[gi];
    const bool even = nit > 0 && wg / nit >= (M == 8 ? kEntWMax : 1);
    int pos = e0, wpos = 0;
    for (int cb = 0; cb < ncand; cb += 64) {
        const int c = cb + lane;
        int2 cd = make_int2(0, 0);
        bool keep = false;
        if (c < ncand) {
            cd = d.cand[(size_t)gi * d.cand_cap + c];
            keep = ((cd.y >> 8) & 255) != 0;
        }
        const unsigned long long bal = __ballot(keep);
        // the entry's weight range [P, P + w) in the group's kept entries
        const int w = keep ? entry_weight(M, (unsigned int)(cd.y >> 8)) : 0;
        int inc = w;
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        const int P = wpos + inc - w;
        if (keep) {
            const int e = pos + __popcll(bal & ((1ull << lane) - 1ull));
            const int cj = cd.x, sid = cd.y & 255;
            // meta: shift id, the i-clusters to evaluate (all the build kept,
            // until a dynamic prune narrows them), j real atoms, the build's
            // i-clusters
            d.ent[e] = make_int2(cj, (cd.y & 0xffff) | (d.cl_nreal[cj] << kMetaNreal) |
                                         (((cd.y >> 8) & 255) << kMetaOuter));
            // the row of this entry's j-force partial, carried in the shift
            // vector's w word: the j-cluster's rows are contiguous; the order
            // inside them depends on atomics, and the gather's int64
            // fixed-point sums do not depend on it
            const int jpos = d.jstart[cj] + gatomic_add(&d.jfill[cj], 1);
            const int gj = cj / G;
            const double rj[3] = {d.gr_ref[3 * gj], d.gr_ref[3 * gj + 1], d.gr_ref[3 * gj + 2]};
            float4 S = entry_shift(d, rj, sid, ri);
            S.w = __int_as_float(jpos);
            d.ent_S[e] = S;
            // the entry whose range holds item k's point starts work item k:
            // {group, first entry, end, its j-cluster} (the force kernel loads
            // the first j-atoms with the item).  The points lie at least an
            // entry's weight apart, so a range holds at most one; the end is
            // the next item's first entry
            int k;
            bool starts;
            if (even) {
                k = (int)(((long long)P * nit + wg - 1) / wg);  // the first point >= P
                starts = k < nit && ((long long)k * wg) / nit < P + w;
            } else {
                k = (P + W - 1) / W;
                starts = k * W < P + w;
            }
            if (starts) {
                int* item = (int*)&d.items[it0 + k];
                item[0] = gi;
                item[1] = e;
                item[3] = cj;
                if (k > 0) item[-2] = e;  // .z of item k - 1
                if (k == nit - 1) item[2] = e1;
            }
        }
        pos += __popcll(bal);
        wpos += __shfl(inc, 63, 64);
    }
}

__global__ void k_clear_status(const SysDev* __restrict__ table, int keep_faults)
{
    const SysDev& d = table[blockIdx.x];
    const int t = threadIdx.x;
    if (t < ST_COUNT && !(keep_faults && (t == ST_SATURATE || t == ST_BADPOS))) d.status[t] = 0;
}

hipError_t launch_clear_status(const SysDev* table, int n_sys, hipStream_t s, bool keep_faults)
{
    hipLaunchKernelGGL(k_clear_status, dim3(n_sys), dim3(64), 0, s, table, keep_faults ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_build(const SysDev* table, int n_sys, const Bounds& b, const int* flags, hipStream_t s,
                        bool exact, int status_clear, int* item_prefix, bool first, bool cleared)
{
    const int clear_n = max(max(b.max_cols, b.max_groups * kGroup), (int)ST_COUNT);
    // enough blocks for the clears and for the displacement partials
    const int atom_b = min(kKeBlocks, max(1, (b.max_atoms + 255) / 256));
    const int fst = first ? 1 : 0;
    if (!cleared)
        hipLaunchKernelGGL(k_build_clear, dim3(max((clear_n + 255) / 256, atom_b), n_sys), dim3(256), 0, s, table,
                           flags, status_clear, fst);
    hipLaunchKernelGGL(k_bin, dim3((b.max_atoms + 255) / 256, n_sys), dim3(256), 0, s, table, flags);
    hipLaunchKernelGGL(k_col_scan, dim3(n_sys), dim3(1024), 0, s, table, flags, fst);
    hipLaunchKernelGGL(k_scatter, dim3((b.max_atoms + 255) / 256, n_sys), dim3(256), 0, s, table, flags);
    hipLaunchKernelGGL(k_col_sort, dim3(b.max_cols * kColParts, n_sys), dim3(256), 0, s, table, flags);
    hipLaunchKernelGGL(k_group_split, dim3((b.max_groups + kSplitWaves - 1) / kSplitWaves, n_sys),
                       dim3(64 * kSplitWaves), 0, s, table, flags);
    hipLaunchKernelGGL(b.any_tric ? (b.all_m8 ? k_search<true, true> : k_search<true, false>)
                                  : (b.all_m8 ? k_search<false, true> : k_search<false, false>),
                       dim3(b.max_groups, n_sys),
                       dim3(64 * kSearchWaves), 0, s, table, flags,
                       exact ? 0 : 1);
    if (exact) {
        hipLaunchKernelGGL(k_prune, dim3(b.max_groups * kPruneBlocks, n_sys), dim3(256), 0, s, table, flags, 0);
        hipLaunchKernelGGL(k_count_kept, dim3((b.max_groups + 3) / 4, n_sys), dim3(256), 0, s, table, flags, 1);
    }
    hipLaunchKernelGGL(k_list_scan, dim3(n_sys), dim3(1024), 0, s, table, flags, n_sys == 1 ? item_prefix : nullptr);
    hipLaunchKernelGGL(k_list_write, dim3((b.max_groups + 3) / 4, n_sys), dim3(256), 0, s, table, flags);
    return hipGetLastError();
}

hipError_t launch_refine(const SysDev* table, int n_sys, const Bounds& b, hipStream_t s)
{
    hipLaunchKernelGGL(k_prune, dim3(b.max_groups * kPruneBlocks, n_sys), dim3(256), 0, s, table, nullptr, 1);
    hipLaunchKernelGGL(k_count_kept, dim3((b.max_groups + 3) / 4, n_sys), dim3(256), 0, s, table, nullptr, 0);
    return hipGetLastError();
}

// OR of the members' overflow / saturation flags into out[0..1]
__global__ void k_ens_status(const SysDev* __restrict__ table, int n_sys, int* out)
{
    int ov = 0, sat = 0;
    for (int i = threadIdx.x; i < n_sys; i += blockDim.x) {
        ov |= table[i].status[ST_OVERFLOW];
        sat |= table[i].status[ST_SATURATE] | table[i].status[ST_BADPOS];
    }
    if (ov) atomicOr(&out[0], 1);
    if (sat) atomicOr(&out[1], 1);
}

__global__ void k_zero_ints(int* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_ens_status(const SysDev* table, int n_sys, int* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, out, 2);
    hipLaunchKernelGGL(k_ens_status, dim3(1), dim3(256), 0, s, table, n_sys, out);
    return hipGetLastError();
}

}  // namespace nbi
