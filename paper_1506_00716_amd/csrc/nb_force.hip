// nb_force.hip -- the cluster-pair non-bonded kernel (gfx950, wave64).
//
// The paper's kernel (Section "SIMD parallelism") keeps the atoms of an
// i-cluster in registers and, for each listed j-cluster, evaluates all M x N
// atom pairs without reloading particle data; its GPU variant groups 8
// clusters so each loaded j-cluster serves several i-clusters.  Newton's third
// law is used: every listed pair is evaluated once and the j-atoms receive the
// opposite force.
//
// MI355X mapping.  One wave64 processes one work item = (i-group of 8
// clusters, a run of `jtile` list entries).  Lane l handles pair (a, b) =
// ((l / M) % M, l % M) of entry (l / M^2), so for M = 8 a wave evaluates one
// full 8 x 8 cluster pair per instruction, for M = 4 four entries at once and
// for M = 1 (plain Verlet list) 64 entries at once.  The 8 i-clusters of the
// group sit in registers (lane holds i-atom a of each), their forces
// accumulate in registers over the whole item; each entry's j-forces are
// summed over the a-lanes with cross-lane shuffles once per entry (amortised
// over up to 8 i-clusters).  The kernel issues no atomics: each entry stores
// its j-atom forces and each item its i-atom forces as partials, and the
// gather kernel sums an atom's partials (int64 fixed point, so the result is
// independent of order and bitwise reproducible; FP32 in the V32 variant).
// Device-scope atomics from many waves to the same atom serialise at the
// memory side on this GPU, which is why they are avoided.  Pair arithmetic is
// FP32 on group-local coordinates; Ewald's force factor q(r) and, for
// energies, erfc(beta r) come from cubic tables in LDS (the same force table
// in every pass).
#include "nb_internal.h"

namespace nbi {

namespace {


// keep a wave-uniform constant in an SGPR for the whole item (no re-loads inside
// the unrolled i-cluster loop)
__device__ __forceinline__ float pin(float v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// the same for a wave-uniform base pointer
template <class T>
__device__ __forceinline__ T* pinp(T* p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// lane ^ D exchange: DPP for 1, 2, 8; ds_swizzle for 4, 16; ds_bpermute for 32
template <int D>
__device__ __forceinline__ float xshfl(float v)
{
    const int i = __float_as_int(v);
    int r;
    if (D == 1) r = __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false);        // quad_perm [1,0,3,2]
    else if (D == 2) r = __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    else if (D == 8) r = __builtin_amdgcn_mov_dpp(i, 0x128, 0xF, 0xF, false);  // row_ror:8
    else if (D == 4) r = __builtin_amdgcn_ds_swizzle(i, 0x101F);               // xor 4 in 32 lanes
    else if (D == 16) r = __builtin_amdgcn_ds_swizzle(i, 0x401F);              // xor 16 in 32 lanes
    else r = __shfl_xor(i, D, 64);
    return __int_as_float(r);
}

// Sum (x, y, z) over the 2^L lanes lane ^ (S * m), m < 2^L, splitting the
// components across lanes so the butterfly moves one value per step instead of
// three: L = 3 takes 4 exchanges (not 9), L = 2 takes 3 (not 6).  Returns the
// total of component `comp` (0 x, 1 y, 2 z) held by this lane; `own` marks one
// lane per component.
template <int S, int L>
__device__ __forceinline__ float reduce3(float x, float y, float z, int idx, int& comp, bool& own)
{
    if (L == 3) {
        const bool lo = idx < 4;
        const float r1 = xshfl<4 * S>(lo ? z : x);
        const float r2 = xshfl<4 * S>(y);
        if (lo) {
            x += r1;
            y += r2;
        } else {
            z += r1;
        }
        const int h = idx & 3;  // within the half
        const float snd = lo ? (h < 2 ? y : x) : z;
        const float r3 = xshfl<2 * S>(snd);
        float v = lo ? (h < 2 ? x : y) : z;
        v += r3;
        v += xshfl<S>(v);
        comp = lo ? (h < 2 ? 0 : 1) : 2;
        own = (idx == 0) || (idx == 2) || (idx == 4);
        return v;
    } else if (L == 2) {
        const bool lo = idx < 2;
        const float r1 = xshfl<2 * S>(lo ? z : x);
        const float r2 = xshfl<2 * S>(y);
        if (lo) {
            x += r1;
            y += r2;
        } else {
            z += r1;
        }
        const float snd = idx == 0 ? y : (idx == 1 ? x : z);
        float v = idx == 0 ? x : (idx == 1 ? y : z);
        v += xshfl<S>(snd);
        comp = idx == 0 ? 0 : (idx == 1 ? 1 : 2);
        own = idx <= 2;
        return v;
    } else {
        comp = -1;  // no reduction: the lane holds all three
        own = true;
        return 0.0f;
    }
}

// the component and ownership reduce3<S, L> assigns to lane index idx
template <int L>
__device__ __forceinline__ void reduce3_slot(int idx, int& comp, bool& own)
{
    if (L == 3) {
        comp = idx < 4 ? ((idx & 3) < 2 ? 0 : 1) : 2;
        own = (idx == 0) || (idx == 2) || (idx == 4);
    } else if (L == 2) {
        comp = idx == 0 ? 0 : (idx == 1 ? 1 : 2);
        own = idx <= 2;
    } else {
        comp = -1;
        own = true;
    }
}

__device__ __forceinline__ float wave_sum(float v)
{
    v += xshfl<1>(v);
    v += xshfl<2>(v);
    v += xshfl<4>(v);
    v += xshfl<8>(v);
    v += xshfl<16>(v);
    v += xshfl<32>(v);
    return v;
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

}  // namespace

// PRUNE: the pass evaluates each entry's build mask and stores the mask pruned
// to r_inner (a separate variant, so the plain pass carries none of it)
//
// red_row >= 0 (one system, force-only passes without pruning): the grid has
// 8 blocks in front of the pair work (one per XCD, dispatched first); block 0
// writes the previous energy pass's energy row (trace row red_row, step
// red_step) with the kinetic energy while the pair blocks run.  That pass's
// partials are complete, this pass writes none of them, and no list build has
// run in between, so the row is the one the energy-reduction kernel would
// write, and its launch is saved.
template <int M, int COUL, int LJ, bool ENER, bool PRUNE>
__global__ __launch_bounds__(256) void k_force(const SysDev* __restrict__ table, int n_sys,
                                               const int* __restrict__ item_prefix, int red_row,
                                               double red_step)
{
    constexpr bool prune = PRUNE;
    constexpr int MM = M * M;
    constexpr int E = 64 / MM;
    constexpr int G = kGroup;
    constexpr int LM = ilog2(M);
    const int lane = threadIdx.x & 63;
    const int esub = lane / MM;
    const int a = (lane / M) % M;
    const int b = lane % M;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the entry of a cluster with itself (zero shift) counts each pair once: a < b
    const unsigned long long tri = __builtin_amdgcn_ballot_w64(a < b);

    // XCD-aware order: blocks are dispatched round-robin over the 8 XCDs
    // (XCD = block id mod 8).  Give each XCD a contiguous eighth of the items
    // (items of nearby i-groups share j-clusters in that XCD's L2) and spread
    // it over that XCD's blocks, so all XCDs work whatever the item count.
    int pair0 = 0;  // the first pair block
    if constexpr (!ENER && !PRUNE) {
        if (red_row >= 0) {
            if (blockIdx.x < 8) {
                if (blockIdx.x == 0) energy_reduce_system(table[0], red_row, 1, red_step);
                return;
            }
            pair0 = 8;
        }
    }
    const int total = item_prefix[n_sys];
    const int bx = (int)blockIdx.x - pair0;  // (bx mod 8 is still the block's XCD)
    const int xcd = bx % 8;
    const int bj = bx / 8;
    const int per_xcd = ((int)gridDim.x - pair0) / 8;  // the pair blocks are a multiple of 8
    const int chunk = (total + 7) / 8;
    const int it_end = min(total, (xcd + 1) * chunk);
    const int nwave = per_xcd * 4;
    // Ewald tables: the force table (every pass) and, with energies, the erfc
    // table; one private copy per wave, reloaded when the wave moves to an
    // item of another system
    constexpr bool TAB = (COUL == 2);
    constexpr bool ETAB = TAB && ENER;
    // per wave kTabU * 64 rows: every lane writes each of its kTabU rows (the
    // rows past the table repeat its last interval and are never read)
    constexpr int kTabU = (kEwTabN + 63) / 64;
    __shared__ float4 tab_lds[TAB ? 4 * kTabU * 64 : 1];
    __shared__ float4 etab_lds[ETAB ? 4 * kTabU * 64 : 1];
    float4* tab = tab_lds + (TAB ? wid * kTabU * 64 : 0);
    float4* etab = etab_lds + (ETAB ? wid * kTabU * 64 : 0);
    int tab_sys = -1;

    for (int it = xcd * chunk + bj * 4 + wid; it < it_end; it += nwave) {
        int s = 0;
        if (n_sys > 1) {
            int lo = 0, hi = n_sys - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (item_prefix[mid] <= it) lo = mid; else hi = mid - 1;
            }
            s = lo;
        }
        s = __builtin_amdgcn_readfirstlane(s);
        const SysDev& d = table[s];
        // the table (when the wave needs a new one) and the work item are
        // loaded in one memory round trip, then the i-atoms, cluster sizes,
        // first entries and first j-atoms (through the item's j-cluster)
        // together: a fixed number of unconditional loads per lane, so none is
        // moved behind a branch.  With per-atom LJ parameters the variant is
        // short of registers for the table in flight: it loads one row per
        // lane at a time (its waves take several items each in the large
        // systems it serves, and refill only for another system), and so do the
        // energy passes (the rare ones) for both their tables
        constexpr bool TAB1 = TAB && LJ == 0 && !ENER;
        const bool fill = TAB && s != tab_sys;
        float4 tv[TAB1 ? kTabU : 1];
        if (TAB1 && fill) {
#pragma unroll
            for (int u = 0; u < kTabU; ++u) tv[u] = gld(&d.ew_tab[min(lane + 64 * u, kEwTabN - 1)]);
        }
        const int li = n_sys > 1 ? it - item_prefix[s] : it;  // item_prefix[0] = 0
        const int4 item = gld(&d.items[li]);
        if (fill) {
            if (TAB1) {
#pragma unroll
                for (int u = 0; u < kTabU; ++u) tab[lane + 64 * u] = tv[u];
            } else {
                for (int k = lane; k < kEwTabN; k += 64) tab[k] = gld(&d.ew_tab[k]);
            }
            if (ETAB)
                for (int k = lane; k < kEwTabN; k += 64) etab[k] = gld(&d.ew_etab[k]);
            // LDS accesses of one wave complete in order; the fence keeps the
            // compiler from moving the table reads above these writes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            tab_sys = s;
        }
        const int gi = item.x, e0 = item.y, e1 = item.z;

        // model constants, one SGPR each for the item; only those this variant
        // uses are loaded (a pinned value is never dropped by the compiler)
        const float rc2 = pin(d.rc2);
        const float rmask2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * d.rc2)));
        constexpr bool LJ1 = LJ == 0;                  // one LJ type
        const float c6 = (LJ1 && ENER) ? pin(d.c6) : 0.f, c12 = (LJ1 && ENER) ? pin(d.c12) : 0.f;
        const float c6x6 = LJ1 ? pin(d.c6x6) : 0.f, c12x12 = LJ1 ? pin(d.c12x12) : 0.f;
        // 6 C6 in a vector register: the LJ FMA takes one scalar operand only
        float c6v = 0.f;
        if (LJ1) asm volatile("v_mov_b32 %0, %1" : "=v"(c6v) : "s"(c6x6));
        const float krf = (COUL == 1 && ENER) ? pin(d.krf) : 0.f, crf = (COUL == 1 && ENER) ? pin(d.crf) : 0.f;
        const float krf2 = COUL == 1 ? pin(d.krf2) : 0.f;
        const float ew_tinv = TAB ? pin(d.ew_tinv) : 0.f;
        // dynamic pruning (a pass that prunes evaluates the build's i-cluster
        // mask and keeps, per entry, the i-clusters with a pair within r_inner)
        const float rin2 = prune ? pin(d.rin2) : 0.f;

        float4 xi[G];
        float2 lji[G];
        unsigned int ireal = 0, iany = 0;
        unsigned long long irm[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int slot = (gi * G + g) * M + a;
            xi[g] = gld(&d.xq[slot]);
            if (LJ == 1) lji[g] = gld(&d.ljs[slot]);
        }
        // the group's 8 cluster sizes (32-byte aligned)
        const int4 nr03 = gld((const int4*)&d.cl_nreal[gi * G]);
        const int4 nr47 = gld((const int4*)&d.cl_nreal[gi * G + 4]);
        float fix[G], fiy[G], fiz[G];
#pragma unroll
        for (int g = 0; g < G; ++g) fix[g] = fiy[g] = fiz[g] = 0.0f;
        float elj = 0.f, ec = 0.f, wxx = 0.f, wyy = 0.f, wzz = 0.f, wxy = 0.f, wxz = 0.f, wyz = 0.f;

        // software pipeline, two stages deep: the list data of the entry after
        // next and the j-atoms of the next entry are in flight while the current
        // entry is evaluated, so no load waits on another load inside the loop
        const int2* ent = pinp(d.ent);
        const float4* entS = pinp(d.ent_S);
        const float4* xq = pinp(d.xq);
        const float2* ljs = pinp(d.ljs);
        float* jpart = pinp(d.jpart);
        int* entw = PRUNE ? pinp((int*)d.ent) : nullptr;
        int2 en_n, en_nn;
        float4 S_n, xj_n;
        float2 ljj_n = make_float2(0.f, 0.f);
        {
            const int e = min(e0 + esub, e1 - 1);
            en_n = gld(&ent[e]);
            S_n = gld(&entS[e]);
            en_nn = gld(&ent[min(e0 + E + esub, e1 - 1)]);
            // one entry per wave (E == 1): its j-cluster comes with the item
            const int cj0 = E == 1 ? item.w : en_n.x;
            xj_n = gld(&xq[cj0 * M + b]);
            if (LJ == 1) ljj_n = gld(&ljs[cj0 * M + b]);
        }
        // ireal: per lane, the i-clusters whose atom a is real; irm[g]: the same
        // as a wave lane mask (scalar registers), used when the wave holds one
        // entry (M = 8)
        {
            const int nrg[G] = {nr03.x, nr03.y, nr03.z, nr03.w, nr47.x, nr47.y, nr47.z, nr47.w};
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (a < nrg[g]) ireal |= 1u << g;
                if (nrg[g] > 0) iany |= 1u << g;
                irm[g] = (E == 1) ? __builtin_amdgcn_ballot_w64(a < nrg[g]) : 0ull;
            }
            iany = __builtin_amdgcn_readfirstlane(iany);
        }
        bool pend = false;  // a j-partial of the previous entry waits to be stored
        float* pend_p = jpart;
        float pend_x = 0.f, pend_y = 0.f, pend_z = 0.f;
        bool pend_m = false;  // (pruning) its pruned meta word, stored with it
        int* pend_mp = entw;
        int pend_mv = 0;
        for (int eb = e0; eb < e1; eb += E) {
            const int e = eb + esub;
            const bool valid = e < e1;
            const int2 en = en_n;
            const float4 S = S_n;
            float4 xj = xj_n;
            const float2 ljj = ljj_n;
            // this entry's data and the next entry's j-cluster are used first, so
            // the wait for the prefetched loads comes before this iteration's store
            int cj_next = en_nn.x;
            asm volatile("" : "+v"(cj_next));  // materialised (waited for) here
            xj.x += S.x;
            xj.y += S.y;
            xj.z += S.z;
            __builtin_amdgcn_sched_barrier(0);
            // the previous entry's j-partial, stored one entry late: issued after
            // that wait and before this iteration's prefetch, so no wait for a
            // prefetch also waits for a store issued after it
            if (pend) {
                if (LM == 0) {
                    gst(pend_p, pend_x);
                    gst(pend_p + 1, pend_y);
                    gst(pend_p + 2, pend_z);
                } else {
                    gst(pend_p, pend_x);
                }
            }
            if (pend_m) gst(pend_mp, pend_mv);
            // issued on every iteration (indices clamped to the item's last
            // entry; the last iteration's loads go unused): with a fixed number
            // of loads per iteration the compiler waits for the current entry's
            // data only, not for the prefetch just issued
            en_n = en_nn;
            S_n = gld(&entS[min(eb + E + esub, e1 - 1)]);
            xj_n = gld(&xq[cj_next * M + b]);
            if (LJ == 1) ljj_n = gld(&ljs[cj_next * M + b]);
            en_nn = gld(&ent[min(eb + 2 * E + esub, e1 - 1)]);
            // row of this entry's j-partial (the shift vector's w word)
            const int jrow = __float_as_int(S.w);
            const int cj = en.x;
            const unsigned int meta = (unsigned int)en.y;
            const int sid = meta & 255u;
            const unsigned int im = (meta >> (prune ? kMetaOuter : kMetaInner)) & 255u;
            const int nrj = (meta >> kMetaNreal) & 15u;
            unsigned int pin_m = 0u;  // (pruning) i-clusters with a pair within r_inner
            bool anyw = false;        // some cluster pair of the entry was evaluated
            const int jslot = cj * M + b;
            const bool jreal = valid && (b < nrj);
            // i-clusters this lane interacts with in this entry; the entry of a
            // cluster with itself (zero shift) counts each pair once (a < b)
            const int gself = (sid == kShiftZero) ? (cj - gi * G) : -1;
            // E > 1: per lane bits; E == 1: wave lane masks (the entry is uniform)
            unsigned int act = 0u;
            unsigned long long jm = 0ull;
            unsigned int gneed;
            int gsu = -1;
            if (E == 1) {
                gneed = __builtin_amdgcn_readfirstlane(im) & iany;
                jm = __builtin_amdgcn_ballot_w64(jreal);
                gsu = __builtin_amdgcn_readfirstlane(gself);
            } else {
                act = jreal ? (im & ireal) : 0u;
                if (gself >= 0 && gself < G && a >= b) act &= ~(1u << gself);
                gneed = 0xffu;
            }
            float fjx = 0.f, fjy = 0.f, fjz = 0.f;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (!((gneed >> g) & 1u)) continue;
                // lanes of this cluster pair that hold a pair to evaluate, as a
                // wave mask: the tests below stay scalar
                unsigned long long onm;
                if (E == 1) {
                    onm = irm[g] & jm;
                    if (g == gsu) onm &= tri;
                } else {
                    onm = __builtin_amdgcn_ballot_w64(((act >> g) & 1u) != 0u);
                    if (onm == 0ull) continue;
                }
                const float dx = xi[g].x - xj.x;
                const float dy = xi[g].y - xj.y;
                const float dz = xi[g].z - xj.z;
                const float r2 = dx * dx + dy * dy + dz * dz;
                if (prune) {
                    if (E == 1) {
                        if (__builtin_amdgcn_ballot_w64(r2 < rin2) & onm) pin_m |= 1u << g;
                    } else if (((act >> g) & 1u) && r2 < rin2) {
                        pin_m |= 1u << g;
                    }
                }
                const unsigned long long cm = __builtin_amdgcn_ballot_w64(r2 < rc2) & onm;
                if (cm == 0ull) continue;  // listed cluster pair with no pair inside r_cut now
                anyw = true;
                const bool c = __builtin_amdgcn_inverse_ballot_w64(cm);
                // lanes without a pair get r^2 = r_cut^2 / 2: finite, and a table
                // index inside the table (their result is discarded below)
                const float r2s = c ? r2 : rmask2;
                const float rinv = __builtin_amdgcn_rsqf(r2s);
                const float rinv2 = rinv * rinv;
                const float rinv6 = rinv2 * rinv2 * rinv2;
                float c6p, c12p, fl;
                if (LJ == 1) {
                    const float sg = lji[g].x + ljj.x;
                    const float ep = lji[g].y * ljj.y;
                    const float s2 = sg * sg;
                    const float s6 = s2 * s2 * s2;
                    c6p = ep * s6;
                    c12p = c6p * s6;
                    fl = (12.0f * c12p * rinv6 - 6.0f * c6p) * rinv6;
                } else {
                    c6p = c6;
                    c12p = c12;
                    fl = fmaf(c12x12, rinv6, -c6v) * rinv6;
                }
                float fs = fl * rinv2;
                float vc = 0.f;
                const float qq = xi[g].w * xj.w;
                if (COUL == 1) {
                    fs += qq * (rinv * rinv2 - krf2);
                    if (ENER) vc = qq * (rinv + krf * r2s - crf);
                } else if (COUL == 2) {
                    // q(r) from the cubic table: F_coul = qq q(r) r_ij / r^3;
                    // energies: erfc(beta r) from the second table
                    const float r = r2s * rinv;
                    const float rs = r * ew_tinv;
                    const int k = (int)rs;  // <= kEwTab: the tables have one interval past r_cut
                    const float w = __builtin_amdgcn_fractf(rs);
                    const float4 cf = tab[k];
                    const float qv = fmaf(fmaf(fmaf(cf.w, w, cf.z), w, cf.y), w, cf.x);
                    fs = fmaf(qq * qv, rinv, fl) * rinv2;
                    if (ENER) {
                        const float4 ce = etab[k];
                        const float ev = fmaf(fmaf(fmaf(ce.w, w, ce.z), w, ce.y), w, ce.x);
                        vc = qq * fmaf(ev, rinv, -d.ew_shift);
                    }
                }
                fs = c ? fs : 0.0f;
                const float tx = fs * dx, ty = fs * dy, tz = fs * dz;
                fix[g] += tx;
                fiy[g] += ty;
                fiz[g] += tz;
                fjx -= tx;
                fjy -= ty;
                fjz -= tz;
                if (ENER) {
                    float vl = (c12p * rinv6 - c6p) * rinv6;
                    if (d.pot_shift) vl -= (LJ == 1) ? (c12p * d.irc12 - c6p * d.irc6) : d.lj_shift;
                    elj += c ? vl : 0.0f;
                    ec += c ? vc : 0.0f;
                    wxx += tx * dx;
                    wyy += ty * dy;
                    wzz += tz * dz;
                    wxy += tx * dy;
                    wxz += tx * dz;
                    wyz += ty * dz;
                }
            }
            // j-forces: sum over the a-lanes of each (entry, b), one component per
            // lane, this entry's partial (summed per atom by the gather; an entry
            // without any pair inside r_cut gives zeros), stored at the next entry
            {
                float* jp = jpart + ((size_t)jrow * M + b) * 3;
                if (LM == 0) {
                    pend = valid;
                    pend_p = jp;
                    pend_x = fjx;
                    pend_y = fjy;
                    pend_z = fjz;
                } else {
                    int comp;
                    bool own;
                    // (one entry per wave: an entry without an evaluated cluster
                    // pair stores zeros, no reduction needed)
                    if (PRUNE && E == 1 && !anyw) {
                        reduce3_slot<LM>(a, comp, own);
                        pend_x = 0.0f;
                    } else {
                        pend_x = reduce3<M, LM>(fjx, fjy, fjz, a, comp, own);
                    }
                    pend = valid && own;
                    pend_p = jp + comp;
                }
            }
            if (prune) {
                // the entry's pruned mask, one lane per entry (the OR over the
                // entry's lanes when a wave holds several entries)
                if (E > 1)
                    for (int o = 1; o < MM; o <<= 1) pin_m |= (unsigned int)__shfl_xor((int)pin_m, o, 64);
                pend_m = valid && (lane % MM) == 0;
                pend_mp = entw + 2 * (size_t)e + 1;
                pend_mv = (int)((meta & ~(255u << kMetaInner)) | (pin_m << kMetaInner));
            }
        }
        if (pend) {  // the item's last entry
            gst(pend_p, pend_x);
            if (LM == 0) {
                gst(pend_p + 1, pend_y);
                gst(pend_p + 2, pend_z);
            }
        }
        if (pend_m) gst(pend_mp, pend_mv);
        // i-forces: sum over b (3-component butterfly), then over the entries of
        // the wave; stored as this item's partial
        float* ip = d.ipart + (size_t)li * (G * M * 3);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (!((iany >> g) & 1u)) continue;
            if (LM == 0) {
                float x = fix[g], y = fiy[g], z = fiz[g];
#pragma unroll
                for (int m = 1; m < 64; m <<= 1) {
                    x += __shfl_xor(x, m, 64);
                    y += __shfl_xor(y, m, 64);
                    z += __shfl_xor(z, m, 64);
                }
                if (lane == 0) {
                    gst(ip + g * 3, x);
                    gst(ip + g * 3 + 1, y);
                    gst(ip + g * 3 + 2, z);
                }
            } else {
                int comp;
                bool own;
                float v = reduce3<1, LM>(fix[g], fiy[g], fiz[g], b, comp, own);
                if (E >= 2) v += xshfl<MM>(v);
                if (E >= 4) v += xshfl<2 * MM>(v);
                if (own && esub == 0) gst(ip + (g * M + a) * 3 + comp, v);
            }
        }
        if (ENER) {
            const float v0 = wave_sum(elj), v1 = wave_sum(ec), v2 = wave_sum(wxx), v3 = wave_sum(wyy),
                        v4 = wave_sum(wzz), v5 = wave_sum(wxy), v6 = wave_sum(wxz), v7 = wave_sum(wyz);
            if (lane == 0) {
                float* o = d.epart + (size_t)li * kEnerPart;
                o[0] = v0; o[1] = v1; o[2] = v2; o[3] = v3;
                o[4] = v4; o[5] = v5; o[6] = v6; o[7] = v7;
            }
        }
    }
}

// ---- dispatch table (the C++ analogue of the paper's kernel function table) ----
typedef void (*ForceFn)(const SysDev*, int, const int*, int, double);

template <int M, int C, int L>
static ForceFn pick(bool ener, bool prune)
{
    if (prune) return ener ? k_force<M, C, L, true, true> : k_force<M, C, L, false, true>;
    return ener ? k_force<M, C, L, true, false> : k_force<M, C, L, false, false>;
}

template <int M>
static ForceFn pick_m(int coul, int lj, bool ener, bool prune)
{
    switch (coul * 2 + lj) {
    case 0: return pick<M, 0, 0>(ener, prune);
    case 1: return pick<M, 0, 1>(ener, prune);
    case 2: return pick<M, 1, 0>(ener, prune);
    case 3: return pick<M, 1, 1>(ener, prune);
    case 4: return pick<M, 2, 0>(ener, prune);
    default: return pick<M, 2, 1>(ener, prune);
    }
}

hipError_t launch_force(const SysDev* table, int n_sys, const int* item_prefix, int M, int coulomb,
                        int lj, bool ener, int max_blocks, int total_item_cap, hipStream_t s, bool prune,
                        int red_row, double red_step)
{
    if (red_row >= 0 && (n_sys != 1 || ener || prune)) return hipErrorInvalidValue;
    ForceFn fn;
    if (M == 8) fn = pick_m<8>(coulomb, lj, ener, prune);
    else if (M == 4) fn = pick_m<4>(coulomb, lj, ener, prune);
    else if (M == 1) fn = pick_m<1>(coulomb, lj, ener, prune);
    else return hipErrorInvalidValue;
    // persistent grid: up to one wave per work item (4096 blocks at most), more
    // than the CUs hold at once: on the 1M-atom slab one resident round of
    // blocks (1024) is 4 % slower.  max_blocks > 0 caps it (a multiple of 8 so
    // the XCD-aware block remap in the kernel is a bijection)
    int blocks = (total_item_cap + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
    if (blocks < 8) blocks = 8;
    blocks = (blocks + 7) / 8 * 8;
    if (red_row >= 0) blocks += 8;  // the energy row's block, and 7 that exit
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, s, table, n_sys, item_prefix, red_row, red_step);
    return hipGetLastError();
}

}  // namespace nbi
