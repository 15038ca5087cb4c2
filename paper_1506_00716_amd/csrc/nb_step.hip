// nb_step.hip -- per-step kernels around the force kernel (gfx950):
// position staging, force gather, FP64 energy/virial/kinetic reductions,
// velocity Verlet, and the steepest-descent relaxation step.
//
// Positions and velocities stay FP64 in HBM; the force kernel sees FP32
// coordinates relative to each i-group's reference point (its bounding-box
// centre), so FP32 rounding is set by the group size (< 1 nm), not by the box.
#include "nb_internal.h"

namespace nbi {

// FP64 master x -> FP32 group-local SoA (+ scaled charge, LB parameters);
// flags (per system, NULL = every system): 0 = skip.  clear: block 0 also
// clears the status words (no kernel before it in the stream is still running,
// and this one writes none)
__global__ __launch_bounds__(256) void k_stage(const SysDev* __restrict__ table, const int* flags, int clear)
{
    if (flags && !flags[blockIdx.y]) return;
    const SysDev& d = table[blockIdx.y];
    if (clear && blockIdx.x == 0 && threadIdx.x < ST_COUNT) d.status[threadIdx.x] = 0;
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    const int GM = d.G * d.M;
    if (slot >= d.n_groups[0] * GM) return;
    const int a = d.slot_atom[slot];
    const int g = slot / GM;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    float2 l = make_float2(0.f, 0.f);
    if (a >= 0) {
        const double xa[3] = {d.x[3 * a], d.x[3 * a + 1], d.x[3 * a + 2]};
        const int wa[3] = {d.slot_wrap[3 * slot], d.slot_wrap[3 * slot + 1], d.slot_wrap[3 * slot + 2]};
        const double ref[3] = {d.gr_ref[3 * g], d.gr_ref[3 * g + 1], d.gr_ref[3 * g + 2]};
        stage_pos(d, xa, wa, ref, p);
        p.w = (float)(d.q[a] * (double)d.qscale);
        if (d.lj == 1) {
            l.x = (float)(0.5 * d.sig[a]);
            l.y = (float)(2.0 * sqrt(d.eps[a]));
        }
    }
    d.xq[slot] = p;
    if (d.lj == 1) d.ljs[slot] = l;
}

__device__ __forceinline__ long long to_fixed(float v, double scale)
{
    // v * scale rounded to an integer: 1.5 * 2^52 puts the integer in the low
    // mantissa bits for |v * scale| < 2^51.
    const double t = fma((double)v, scale, 6755399441055744.0);
    return __double_as_longlong(t) - 0x4338000000000000LL;
}

// one block per system (the energy pass's trace row, see energy_reduce_system)
__global__ __launch_bounds__(256) void k_energy_reduce(const SysDev* __restrict__ table,
                                                       int trace_row, int with_ke, double step_value)
{
    energy_reduce_system(table[blockIdx.x], trace_row, with_ke, step_value);
}


// v += dt/2 F/m ; x += dt v  (every velocity-Verlet update in this file is
// written with explicit FMAs, so fused and separate kernels agree bitwise)
__global__ __launch_bounds__(256) void k_kick_drift(const SysDev* __restrict__ table, double dt)
{
    const SysDev& d = table[blockIdx.y];
    const int nb = sys_blocks(d.n_atoms);
    if ((int)blockIdx.x >= nb) return;
    const int stride = nb * blockDim.x;
    double* x = (double*)d.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n_atoms; i += stride) {
        const double h = 0.5 * dt / d.mass[i];
        for (int k = 0; k < 3; ++k) {
            const double v = fma(h, (double)d.f[3 * i + k], d.v[3 * i + k]);
            d.v[3 * i + k] = v;
            x[3 * i + k] = fma(dt, v, x[3 * i + k]);
        }
    }
}

// v += dt/2 F/m ; per-block kinetic-energy partial sums (fixed decomposition)
__global__ __launch_bounds__(256) void k_kick(const SysDev* __restrict__ table, double dt, int ke)
{
    const SysDev& d = table[blockIdx.y];
    __shared__ double sh[256];
    const int nb = sys_blocks(d.n_atoms);
    if ((int)blockIdx.x >= nb) {
        if (ke && threadIdx.x == 0) d.ke_part[blockIdx.x] = 0.0;
        return;
    }
    const int stride = nb * blockDim.x;
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n_atoms; i += stride) {
        const double m = d.mass[i];
        const double h = 0.5 * dt / m;
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double v = fma(h, (double)d.f[3 * i + k], d.v[3 * i + k]);
            d.v[3 * i + k] = v;
            s += v * v;
        }
        acc += 0.5 * m * s;
    }
    if (!ke) return;
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.ke_part[blockIdx.x] = sh[0];
}

// List-buffer guard (Verlet displacement criterion): at each rebuild, the
// largest displacement since the previous build; a pair can only have entered
// r_cut unlisted if two atoms moved by >= (r_list - r_cut)/2 each.
// max over n >= 0 per-block partials (NaN wins), by all threads of a 256-thread
// block; every thread gets the result
__device__ double block_max_partials(const double* p, int n)
{
    __shared__ double sh[256];
    double m = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        const double u = p[k];
        m = (u > m || u != u) ? u : m;
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double u = sh[threadIdx.x + o];
            if (u > sh[threadIdx.x] || u != u) sh[threadIdx.x] = u;
        }
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Dynamic-prune guard of one system, launched at the end of every prune
// interval (check = 1) and when a list is built afresh (check = 0): per block
// the largest squared displacement since x_prune (the positions at the last
// prune) into partial buffer `cur`, then x_prune = x.  Block 0 first folds the
// previous interval's partials (buffer 1 - cur, complete since that launch
// ended) into the interval statistics: the largest displacement, and the
// intervals in which it reached (r_inner - r_cut)/2 -- the only way a cluster
// pair pruned at the interval's start could have had a pair inside r_cut.
__global__ __launch_bounds__(256) void k_prune_guard(const SysDev* __restrict__ table, int check, int cur,
                                                     int fold)
{
    const SysDev& d = table[0];
    const int nb = sys_blocks(d.n_atoms);
    if (fold && blockIdx.x == 0) {
        const double m2 = block_max_partials(d.pg_part + (1 - cur) * kKeBlocks, nb);
        if (threadIdx.x == 0) {
            const double mm = sqrt(m2);
            double* st = d.pg_part + 2 * kKeBlocks;
            if (mm > st[0] || mm != mm) st[0] = mm;
            if (!(mm < d.prune_half)) st[1] += 1.0;
        }
    }
    double m = 0.0;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < d.n_atoms; a += nb * blockDim.x) {
        double s2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double x = gld(&d.x[3 * a + k]);
            if (check) {
                const double dd = x - gld(&d.x_prune[3 * a + k]);
                s2 += dd * dd;
            }
            gst(&d.x_prune[3 * a + k], x);
        }
        m = (s2 > m || s2 != s2) ? s2 : m;  // NaN wins
    }
    if (!check) return;
    __shared__ double sh[256];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double u = sh[threadIdx.x + o];
            if (u > sh[threadIdx.x] || u != u) sh[threadIdx.x] = u;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) d.pg_part[cur * kKeBlocks + blockIdx.x] = sh[0];
}

// per-block max |F| (relaxation)
__global__ __launch_bounds__(256) void k_fmax(const SysDev* __restrict__ table)
{
    const SysDev& d = table[0];
    __shared__ double sh[256];
    double m = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n_atoms; i += gridDim.x * blockDim.x) {
        const double fx = d.f[3 * i], fy = d.f[3 * i + 1], fz = d.f[3 * i + 2];
        const double f2 = fx * fx + fy * fy + fz * fz;
        m = (f2 > m || f2 != f2) ? f2 : m;
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double u = sh[threadIdx.x + o];
            if (u > sh[threadIdx.x] || u != u) sh[threadIdx.x] = u;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) d.fmax_part[blockIdx.x] = sh[0];
}

// steepest descent: x += max_disp * F / max|F| (largest move = max_disp)
__global__ __launch_bounds__(256) void k_minimize_step(const SysDev* __restrict__ table, double* x,
                                                       double max_disp, double f_tol, int* done)
{
    const SysDev& d = table[0];
    const double fm = sqrt(block_max_partials(d.fmax_part, kKeBlocks));
    if (!(fm >= f_tol)) {  // converged (or NaN: stop)
        if (blockIdx.x == 0 && threadIdx.x == 0) *done = 1;
        return;
    }
    const double s = max_disp / fm;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n_atoms; i += gridDim.x * blockDim.x)
        for (int k = 0; k < 3; ++k) x[3 * i + k] += s * (double)d.f[3 * i + k];
}

// prefix over member systems of their work-item counts (one small block);
// a system with flag 0 contributes no items
__global__ void k_item_prefix(const SysDev* __restrict__ table, int n_sys, int* prefix, const int* flags)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int acc = 0;
    prefix[0] = 0;
    for (int s = 0; s < n_sys; ++s) {
        acc += (flags && !flags[s]) ? 0 : table[s].n_items[0];
        prefix[s + 1] = acc;
    }
}

// mode 0: x, v -> x_bak, v_bak (every atom); mode 1: back again
__global__ __launch_bounds__(256) void k_state_copy(const SysDev* __restrict__ table, int mode)
{
    const SysDev& d = table[blockIdx.y];
    const int n3 = 3 * d.n_atoms;
    double* x = (double*)d.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += gridDim.x * blockDim.x) {
        if (mode == 0) {
            gst(&d.x_bak[i], gld(&x[i]));
            gst(&d.v_bak[i], gld(&d.v[i]));
        } else {
            gst(&x[i], gld(&d.x_bak[i]));
            gst(&d.v[i], gld(&d.v_bak[i]));
        }
    }
}

// ---- fused per-slot step kernels (plain steps without a list rebuild) --------
// Every real atom owns exactly one slot, so per-atom updates can run in cluster
// order and the FP64 arithmetic is the same as in k_kick_drift / k_kick.

// v += dt/2 F/m ; x += dt v ; stage the new x into the group-local FP32 SoA
__global__ __launch_bounds__(256) void k_kick_drift_stage(const SysDev* __restrict__ table, double dt)
{
    const SysDev& d = table[blockIdx.y];
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    const int GM = d.G * d.M;
    if (slot >= d.n_groups[0] * GM) return;
    const int a = d.slot_atom[slot];
    if (a < 0) return;  // padding slots keep their staged values
    const int g = slot / GM;
    double* x = (double*)d.x;
    const double h = 0.5 * dt / d.mass[a];
    double xn[3];
    for (int k = 0; k < 3; ++k) {
        const double v = fma(h, (double)d.f[3 * a + k], d.v[3 * a + k]);
        d.v[3 * a + k] = v;
        xn[k] = fma(dt, v, x[3 * a + k]);
        x[3 * a + k] = xn[k];
    }
    float4 p;
    {
        const int wa[3] = {d.slot_wrap[3 * slot], d.slot_wrap[3 * slot + 1], d.slot_wrap[3 * slot + 2]};
        const double ref[3] = {d.gr_ref[3 * g], d.gr_ref[3 * g + 1], d.gr_ref[3 * g + 2]};
        stage_pos(d, xn, wa, ref, p);
    }
    p.w = (float)(d.q[a] * (double)d.qscale);
    d.xq[slot] = p;
}

// Force gather: an atom's force is the sum of its i-partials (one per work item
// of its group) and its j-partials (one per list entry with its cluster as j;
// the force kernel writes them in rows grouped by j-cluster, so a cluster's
// j-partials are contiguous).
// One wave per cluster: lane (r, a) handles atom a of the cluster and every
// R-th partial (R = 64/M rows), then the rows are summed with shuffles.  V64r
// sums in int64 fixed point (exact, so the result does not depend on the order:
// bitwise reproducible); V32 sums in FP32.  The force goes to the caller's
// f[N,3] in original atom order; with KICK the velocity half-kick
// v += dt/2 F/m follows (plus kinetic-energy partials), fusing the end of a
// velocity-Verlet step.  The block count per system depends only on the system
// (cluster count), so the kinetic-energy decomposition is the same alone and
// in a batch.
__device__ inline int cluster_blocks(int n_clusters)
{
    int b = (n_clusters + 3) / 4;
    return b > kKeBlocks ? kKeBlocks : (b < 1 ? 1 : b);
}

// next (with KICK): 0 = stop after the half-kick; 1 = also the next step's
// half-kick and drift (v += dt/2 F/m, x += dt v: the same FP64 operations as
// k_kick_drift), keeping the full-step x, v in x_bak, v_bak, and the work of
// the list build's first kernel (a rebuild follows: its counters and status
// words cleared, the list-buffer guard's largest squared displacement since the
// last build per block, x recorded for the next one); 2 = half-kick, drift and
// the staging of the new x (as k_kick_drift_stage).  open: the forces of a run's first positions, with no
// step to close: only the next step's half-kick and drift (next 1 or 2)
template <bool KICK>
__global__ __launch_bounds__(256) void k_gather(const SysDev* __restrict__ table, double dt, int ke, int next,
                                                int open, const int* flags)
{
    if (flags && !flags[blockIdx.y]) return;  // (only the force-only gather takes flags)
    const SysDev& d = table[blockIdx.y];
    __shared__ double sh[4];
    const bool pre_build = KICK && next == 1;
    if (pre_build) {
        // the build's counters and status words (all but the fault flags of
        // earlier steps); none of them is read before the build
        const int t = blockIdx.x * blockDim.x + threadIdx.x, ts = gridDim.x * blockDim.x;
        for (int i = t; i < d.n_cols; i += ts) {
            gst(&d.col_count[i], 0);
            gst(&d.col_fill[i], 0);
        }
        for (int i = t; i < d.max_groups; i += ts) {
            gst(&d.cand_count[i], 0);
            gst(&d.cand_kept[i], 0);
            gst(&d.grp_w[i], 0);
        }
        for (int i = t; i < d.max_groups * d.G; i += ts) gst(&d.jfill[i], 0);
        if (t < ST_COUNT && t != ST_SATURATE && t != ST_BADPOS) gst(&d.status[t], 0);
        // guard partials past this grid
        if (blockIdx.x == 0)
            for (int k = gridDim.x + threadIdx.x; k < kKeBlocks; k += blockDim.x) d.disp[k] = 0.0;
    }
    const int M = d.M, G = d.G;
    const int n_cl = d.n_groups[0] * G;
    const int nb = cluster_blocks(n_cl);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if ((int)blockIdx.x >= nb) {
        if (KICK && ke && threadIdx.x == 0) d.ke_part[blockIdx.x] = 0.0;
        if (pre_build && threadIdx.x == 0) d.disp[blockIdx.x] = 0.0;
        return;
    }
    const int R = 64 / M;
    const int a = lane % M, r = lane / M;
    const size_t istride = (size_t)G * M * 3;
    const bool f32 = d.fp32_reduce != 0;
    const float lim = d.fx_lim;
    const double sc = d.fx_scale;
    // partial rows written by the force kernel: a list whose build ran out of
    // capacity has none (its offsets may point past the partial arrays, so the
    // row ranges below are clamped to what exists)
    const int n_it = gld(&d.n_items[0]), n_en = gld(&d.n_ent[0]);
    bool bad = false;
    double kin = 0.0;
    double disp_m = 0.0;  // (pre_build) largest squared displacement since the last build
    for (int cl = blockIdx.x * 4 + wid; cl < n_cl; cl += nb * 4) {
        // Two memory round trips per cluster: (1) its size, row ranges and
        // atoms, (2) its partials together with the finishing lanes' atom data.
        // No branch or conditional load sits between the loads of a round trip,
        // so none waits on another.  Empty clusters (no partials are written
        // for them) and padding lanes get empty row ranges and no atom.
        const int g = cl / G, k = cl % G;
        const int nr_l = gld(&d.cl_nreal[cl]);
        const int it0 = gld(&d.item_start[g]), it1 = gld(&d.item_start[g + 1]);
        const int js0 = gld(&d.jstart[cl]), js1 = gld(&d.jstart[cl + 1]);
        const int atom_l = gld(&d.slot_atom[cl * M + a]);
        const bool real = a < nr_l;
        const int t0 = min(it0, n_it), t1 = real ? max(t0, min(it1, n_it)) : t0;
        const int j0 = min(js0, n_en), j1 = real ? max(j0, min(js1, n_en)) : j0;
        const bool fin = (r == 0) && real;
        const int atom = fin ? atom_l : -1;
        // the atom data are loaded for every lane (a clamped index), used by
        // the finishing lanes only
        const int ac = atom >= 0 ? atom : 0;
        double m = 1.0, v0[3] = {0.0, 0.0, 0.0}, x0[3] = {0.0, 0.0, 0.0}, xb[3] = {0.0, 0.0, 0.0};
        if (KICK) {
            m = gld(&d.mass[ac]);
            for (int c = 0; c < 3; ++c) v0[c] = gld(&d.v[3 * ac + c]);
            for (int c = 0; c < 3; ++c) x0[c] = gld(&d.x[3 * ac + c]);
            if (pre_build)
                for (int c = 0; c < 3; ++c) xb[c] = gld(&d.x_build[3 * ac + c]);
        }
        long long sx = 0, sy = 0, sz = 0;
        float fx = 0.f, fy = 0.f, fz = 0.f;
        // one row space over the cluster's i-partials, then its j-partials;
        // rows go in batches of 4 per lane whose loads are all issued before
        // any of them is summed
        const int ni = t1 - t0, nrow = ni + (j1 - j0);
        const float* ipl = d.ipart + (size_t)t0 * istride + ((size_t)k * M + a) * 3;
        const float* jpl = d.jpart + ((size_t)j0 * M + a) * 3;
        const size_t jstr = (size_t)M * 3;
        auto row = [&](int q) -> const float* {
            return q < ni ? ipl + (size_t)q * istride : jpl + (size_t)(q - ni) * jstr;
        };
        if (f32) {
            for (int q0 = r; q0 < nrow; q0 += 4 * R) {
                float v[4][3];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // rows past the end read row q0 (loaded unconditionally, dropped)
                    const int q = q0 + u * R;
                    const float* pr = row(q < nrow ? q : q0);
                    for (int c = 0; c < 3; ++c) {
                        const float w = gld(pr + c);
                        v[u][c] = q < nrow ? w : 0.0f;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);  // all loads of the batch first
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    fx += v[u][0];
                    fy += v[u][1];
                    fz += v[u][2];
                }
            }
        } else {
            for (int q0 = r; q0 < nrow; q0 += 4 * R) {
                float v[4][3];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // rows past the end read row q0 (loaded unconditionally, dropped)
                    const int q = q0 + u * R;
                    const float* pr = row(q < nrow ? q : q0);
                    for (int c = 0; c < 3; ++c) {
                        const float w = gld(pr + c);
                        v[u][c] = q < nrow ? w : 0.0f;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);  // all loads of the batch first
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bad = bad || !(fabsf(v[u][0]) < lim) || !(fabsf(v[u][1]) < lim) || !(fabsf(v[u][2]) < lim);
                    sx += to_fixed(v[u][0], sc);
                    sy += to_fixed(v[u][1], sc);
                    sz += to_fixed(v[u][2], sc);
                }
            }
        }
        for (int o = M; o < 64; o <<= 1) {
            if (f32) {
                fx += __shfl_xor(fx, o, 64);
                fy += __shfl_xor(fy, o, 64);
                fz += __shfl_xor(fz, o, 64);
            } else {
                sx += __shfl_xor(sx, o, 64);
                sy += __shfl_xor(sy, o, 64);
                sz += __shfl_xor(sz, o, 64);
            }
        }
        if (fin && atom >= 0 && d.pme_f) {
            // the reciprocal-space force of the atom joins the same sum
            float pf[3];
            for (int c = 0; c < 3; ++c) pf[c] = gld(&d.pme_f[3 * atom + c]);
            if (f32) {
                fx += pf[0];
                fy += pf[1];
                fz += pf[2];
            } else {
                bad = bad || !(fabsf(pf[0]) < lim) || !(fabsf(pf[1]) < lim) || !(fabsf(pf[2]) < lim);
                sx += to_fixed(pf[0], sc);
                sy += to_fixed(pf[1], sc);
                sz += to_fixed(pf[2], sc);
            }
        }
        if (fin) {
            if (atom >= 0) {
                float F[3];
                if (f32) {
                    F[0] = fx;
                    F[1] = fy;
                    F[2] = fz;
                    bad = bad || !(fabsf(fx) <= 3.4e38f) || !(fabsf(fy) <= 3.4e38f) || !(fabsf(fz) <= 3.4e38f);
                } else {
                    F[0] = (float)((double)sx * d.fx_inv);
                    F[1] = (float)((double)sy * d.fx_inv);
                    F[2] = (float)((double)sz * d.fx_inv);
                }
                if (KICK) {
                    const double h = 0.5 * dt / m;
                    double s2 = 0.0;
                    double vn[3];
                    for (int c = 0; c < 3; ++c) {
                        d.f[3 * atom + c] = F[c];
                        vn[c] = open ? v0[c] : fma(h, (double)F[c], v0[c]);
                        s2 += vn[c] * vn[c];
                    }
                    kin += 0.5 * m * s2;
                    if (next == 0) {
                        for (int c = 0; c < 3; ++c) d.v[3 * atom + c] = vn[c];
                    } else {
                        double* x = (double*)d.x;
                        double xn[3];
                        if (next == 1)  // a rebuild step follows: keep the full step
                            for (int c = 0; c < 3; ++c) {
                                d.x_bak[3 * atom + c] = x0[c];
                                d.v_bak[3 * atom + c] = vn[c];
                            }
                        for (int c = 0; c < 3; ++c) {
                            const double v2 = fma(h, (double)F[c], vn[c]);
                            d.v[3 * atom + c] = v2;
                            xn[c] = fma(dt, v2, x0[c]);
                            x[3 * atom + c] = xn[c];
                        }
                        if (next == 1) {  // (the same operations as k_build_clear)
                            double s2 = 0.0;
                            for (int c = 0; c < 3; ++c) {
                                const double dd = xn[c] - xb[c];
                                s2 += dd * dd;
                                d.x_build[3 * atom + c] = xn[c];
                            }
                            disp_m = (s2 > disp_m || s2 != s2) ? s2 : disp_m;  // NaN wins
                        }
                        if (next == 2) {
                            const int slot = cl * M + a;
                            float4 p;
                            const int wa[3] = {d.slot_wrap[3 * slot], d.slot_wrap[3 * slot + 1],
                                               d.slot_wrap[3 * slot + 2]};
                            const double ref[3] = {d.gr_ref[3 * g], d.gr_ref[3 * g + 1], d.gr_ref[3 * g + 2]};
                            stage_pos(d, xn, wa, ref, p);
                            p.w = (float)(d.q[atom] * (double)d.qscale);
                            d.xq[slot] = p;
                        }
                    }
                } else {
                    for (int c = 0; c < 3; ++c) d.f[3 * atom + c] = F[c];
                }
            }
        }
    }
    if (bad) atomicOr(&d.status[ST_SATURATE], 1);
    if (pre_build) {
        // the block's largest squared displacement (NaN wins)
        for (int o = 1; o < 64; o <<= 1) {
            const double u = __shfl_xor(disp_m, o, 64);
            disp_m = (u > disp_m || u != u) ? u : disp_m;
        }
        __shared__ double shd[4];
        if (lane == 0) shd[wid] = disp_m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double mm = shd[0];
            for (int w = 1; w < 4; ++w) mm = (shd[w] > mm || shd[w] != shd[w]) ? shd[w] : mm;
            d.disp[blockIdx.x] = mm;
        }
    }
    if (!(KICK && ke)) return;
    // fixed-order kinetic-energy partial of the block
    for (int o = 1; o < 64; o <<= 1) kin += __shfl_xor(kin, o, 64);
    if (lane == 0) sh[wid] = kin;
    __syncthreads();
    if (threadIdx.x == 0) d.ke_part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

static int atom_blocks(int max_atoms)
{
    int b = (max_atoms + 255) / 256;
    if (b > kKeBlocks) b = kKeBlocks;
    return b < 1 ? 1 : b;
}

hipError_t launch_stage(const SysDev* table, int n_sys, const Bounds& b, hipStream_t s, const int* flags,
                        bool clear_status)
{
    hipLaunchKernelGGL(k_stage, dim3((b.max_slots + 255) / 256, n_sys), dim3(256), 0, s, table, flags,
                       clear_status ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_state_copy(const SysDev* table, int n_sys, const Bounds& b, int mode, hipStream_t s)
{
    const int blocks = min(kKeBlocks, max(1, (3 * b.max_atoms + 255) / 256));
    hipLaunchKernelGGL(k_state_copy, dim3(blocks, n_sys), dim3(256), 0, s, table, mode);
    return hipGetLastError();
}

static int gather_blocks(const Bounds& b)
{
    const int ncl = b.max_groups * kGroup;
    int nb = (ncl + 3) / 4;
    return nb > kKeBlocks ? kKeBlocks : (nb < 1 ? 1 : nb);
}

hipError_t launch_finalize(const SysDev* table, int n_sys, const Bounds& b, bool fp32, hipStream_t s,
                           const int* flags)
{
    (void)fp32;
    hipLaunchKernelGGL(k_gather<false>, dim3(gather_blocks(b), n_sys), dim3(256), 0, s, table, 0.0, 0, 0, 0, flags);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(const SysDev* table, int n_sys, int trace_row, bool with_ke,
                                double step_value, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_reduce, dim3(n_sys), dim3(256), 0, s, table, trace_row,
                       with_ke ? 1 : 0, step_value);
    return hipGetLastError();
}

hipError_t launch_kick_drift(const SysDev* table, int n_sys, const Bounds& b, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_kick_drift, dim3(atom_blocks(b.max_atoms), n_sys), dim3(256), 0, s, table, dt);
    return hipGetLastError();
}

hipError_t launch_kick(const SysDev* table, int n_sys, const Bounds& b, double dt, bool ke,
                       hipStream_t s)
{
    // blocks beyond a member's own count write zero partials and exit; partials
    // past the grid stay zero from system creation
    hipLaunchKernelGGL(k_kick, dim3(atom_blocks(b.max_atoms), n_sys), dim3(256), 0, s, table, dt,
                       ke ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_kick_drift_stage(const SysDev* table, int n_sys, const Bounds& b, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_kick_drift_stage, dim3((b.max_slots + 255) / 256, n_sys), dim3(256), 0, s, table, dt);
    return hipGetLastError();
}

hipError_t launch_gather_kick(const SysDev* table, int n_sys, const Bounds& b, double dt, bool ke, hipStream_t s,
                              int next, bool open)
{
    hipLaunchKernelGGL(k_gather<true>, dim3(gather_blocks(b), n_sys), dim3(256), 0, s, table, dt, ke ? 1 : 0, next,
                       open ? 1 : 0, (const int*)nullptr);
    return hipGetLastError();
}

hipError_t launch_item_prefix(const SysDev* table, int n_sys, int* item_prefix, hipStream_t s, const int* flags)
{
    hipLaunchKernelGGL(k_item_prefix, dim3(1), dim3(64), 0, s, table, n_sys, item_prefix, flags);
    return hipGetLastError();
}

hipError_t launch_prune_guard_k(const SysDev* table, int n_atoms, int check, int cur, int fold, hipStream_t s)
{
    hipLaunchKernelGGL(k_prune_guard, dim3(atom_blocks(n_atoms)), dim3(256), 0, s, table, check, cur, fold);
    return hipGetLastError();
}

hipError_t launch_fmax(const SysDev* table, const Bounds& b, hipStream_t s)
{
    (void)b;
    hipLaunchKernelGGL(k_fmax, dim3(kKeBlocks), dim3(256), 0, s, table);
    return hipGetLastError();
}

hipError_t launch_minimize_step(const SysDev* table, const Bounds& b, double* x, double max_disp,
                                double f_tol, int* done_flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_minimize_step, dim3(atom_blocks(b.max_atoms)), dim3(256), 0, s, table, x,
                       max_disp, f_tol, done_flag);
    return hipGetLastError();
}

}  // namespace nbi
