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
// over up to 8 i-clusters) and added to the j-atoms.  Force sums cross waves
// as int64 fixed point (order independent, so bitwise reproducible), or as
// FP32 atomics in the V32 precision variant.  Pair arithmetic is FP32 on
// cluster-local coordinates; Ewald's erfc uses exp2 and a fitted polynomial
// in t = 1/(1 + p beta r).
#include "nb_internal.h"

namespace nbi {

namespace {

__device__ __forceinline__ long long to_fixed(float v, double scale)
{
    // v * scale rounded to an integer: 1.5 * 2^52 puts the integer in the low
    // mantissa bits for |v * scale| < 2^51.
    const double t = fma((double)v, scale, 6755399441055744.0);
    return __double_as_longlong(t) - 0x4338000000000000LL;
}

__device__ __forceinline__ void add_force(const SysDev& d, int slot, float fx, float fy, float fz,
                                          bool fp32)
{
    if (fp32) {
        atomicAdd(&d.facc32[3 * slot], fx);
        atomicAdd(&d.facc32[3 * slot + 1], fy);
        atomicAdd(&d.facc32[3 * slot + 2], fz);
    } else {
        const float m = fmaxf(fmaxf(fabsf(fx), fabsf(fy)), fabsf(fz));
        if (!(m < d.fx_lim)) {
            atomicOr(&d.status[ST_SATURATE], 1);
            return;
        }
        unsigned long long* p = (unsigned long long*)(d.facc + 3 * slot);
        __hip_atomic_fetch_add(p, (unsigned long long)to_fixed(fx, d.fx_scale), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(p + 1, (unsigned long long)to_fixed(fy, d.fx_scale),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(p + 2, (unsigned long long)to_fixed(fz, d.fx_scale),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ float wave_sum(float v)
{
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace

template <int M, int COUL, int LJ, bool ENER, bool FP32>
__global__ __launch_bounds__(256) void k_force(const SysDev* __restrict__ table, int n_sys,
                                               const int* __restrict__ item_prefix)
{
    constexpr int MM = M * M;
    constexpr int E = 64 / MM;
    constexpr int G = kGroup;
    const int lane = threadIdx.x & 63;
    const int esub = lane / MM;
    const int a = (lane / M) % M;
    const int b = lane % M;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // XCD-aware order: blocks are dispatched round-robin over the 8 XCDs, so
    // give each XCD a contiguous range of logical blocks (items of nearby
    // i-groups share j-clusters in that XCD's L2).
    const int nb = gridDim.x;
    const int per = (nb + 7) / 8;
    const int bx = blockIdx.x;
    const int lb = (bx % 8) * per + bx / 8;
    const int nwave = per * 8 * 4;
    const int total = item_prefix[n_sys];

    for (int it = lb * 4 + wid; it < total; it += nwave) {
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
        const int li = it - item_prefix[s];
        const int4 item = d.items[li];
        const int gi = item.x, e0 = item.y, e1 = item.z;

        float4 xi[G];
        float2 lji[G];
        unsigned int ireal = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int ci = gi * G + g;
            const int slot = ci * M + a;
            xi[g] = d.xq[slot];
            if (LJ == 1) lji[g] = d.ljs[slot];
            if (a < d.cl_nreal[ci]) ireal |= 1u << g;
        }
        float fix[G], fiy[G], fiz[G];
#pragma unroll
        for (int g = 0; g < G; ++g) fix[g] = fiy[g] = fiz[g] = 0.0f;
        float elj = 0.f, ec = 0.f, wxx = 0.f, wyy = 0.f, wzz = 0.f, wxy = 0.f, wxz = 0.f, wyz = 0.f;

        const float rc2 = d.rc2;
        for (int eb = e0; eb < e1; eb += E) {
            const int e = eb + esub;
            const bool valid = e < e1;
            const int2 en = d.ent[valid ? e : e0];
            const float4 S = d.ent_S[valid ? e : e0];
            const int cj = en.x;
            const int sid = en.y & 255;
            const unsigned int im = ((unsigned int)en.y >> 8) & 255u;
            const int jslot = cj * M + b;
            float4 xj = d.xq[jslot];
            float2 ljj = make_float2(0.f, 0.f);
            if (LJ == 1) ljj = d.ljs[jslot];
            const bool jreal = valid && (b < d.cl_nreal[cj]);
            const unsigned int act = jreal ? (im & ireal) : 0u;
            const int gself = (sid == kShiftZero) ? (cj - gi * G) : -1;
            xj.x += S.x;
            xj.y += S.y;
            xj.z += S.z;
            float fjx = 0.f, fjy = 0.f, fjz = 0.f;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                bool on = (act >> g) & 1u;
                if (g == gself && a >= b) on = false;
                if (!__any(on)) continue;
                const float dx = xi[g].x - xj.x;
                const float dy = xi[g].y - xj.y;
                const float dz = xi[g].z - xj.z;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const bool c = on && (r2 < rc2);
                const float r2s = c ? r2 : 1.0f;
                const float rinv = __builtin_amdgcn_rsqf(r2s);
                const float rinv2 = rinv * rinv;
                const float rinv6 = rinv2 * rinv2 * rinv2;
                float c6, c12;
                if (LJ == 1) {
                    const float sg = lji[g].x + ljj.x;
                    const float ep = lji[g].y * ljj.y;
                    const float s2 = sg * sg;
                    const float s6 = s2 * s2 * s2;
                    c6 = ep * s6;
                    c12 = c6 * s6;
                } else {
                    c6 = d.c6;
                    c12 = d.c12;
                }
                float fl;
                if (LJ == 1)
                    fl = (12.0f * c12 * rinv6 - 6.0f * c6) * rinv6;
                else
                    fl = (d.c12x12 * rinv6 - d.c6x6) * rinv6;
                float fs = fl * rinv2;
                float vc = 0.f;
                const float qq = xi[g].w * xj.w;
                if (COUL == 1) {
                    fs += qq * (rinv * rinv2 - d.krf2);
                    if (ENER) vc = qq * (rinv + d.krf * r2s - d.crf);
                } else if (COUL == 2) {
                    const float r = r2s * rinv;
                    const float t = __builtin_amdgcn_rcpf(fmaf(d.ew_pb, r, 1.0f));
                    const float u = fmaf(d.ew_u1, t, d.ew_u0);
                    float p = d.ew_poly[kPolyDeg];
#pragma unroll
                    for (int k = kPolyDeg - 1; k >= 0; --k) p = fmaf(p, u, d.ew_poly[k]);
                    const float ex = __builtin_amdgcn_exp2f(d.ew_kexp * r2s);
                    const float erfc_r = ex * p * rinv;
                    fs += qq * fmaf(d.ew_c2b, ex, erfc_r) * rinv2;
                    if (ENER) vc = qq * (erfc_r - d.ew_shift);
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
                    float vl = (c12 * rinv6 - c6) * rinv6;
                    if (d.pot_shift) vl -= (LJ == 1) ? (c12 * d.irc12 - c6 * d.irc6) : d.lj_shift;
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
            // j-forces: sum over the a-lanes of each (entry, b)
#pragma unroll
            for (int m = M; m < MM; m <<= 1) {
                fjx += __shfl_xor(fjx, m, 64);
                fjy += __shfl_xor(fjy, m, 64);
                fjz += __shfl_xor(fjz, m, 64);
            }
            if (a == 0 && jreal) add_force(d, jslot, fjx, fjy, fjz, FP32);
        }
        // i-forces: sum over b and over the entries of the wave
#pragma unroll
        for (int g = 0; g < G; ++g) {
            float x = fix[g], y = fiy[g], z = fiz[g];
#pragma unroll
            for (int m = 1; m < M; m <<= 1) {
                x += __shfl_xor(x, m, 64);
                y += __shfl_xor(y, m, 64);
                z += __shfl_xor(z, m, 64);
            }
#pragma unroll
            for (int m = MM; m < 64; m <<= 1) {
                x += __shfl_xor(x, m, 64);
                y += __shfl_xor(y, m, 64);
                z += __shfl_xor(z, m, 64);
            }
            if (b == 0 && esub == 0 && ((ireal >> g) & 1u))
                add_force(d, (gi * G + g) * M + a, x, y, z, FP32);
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
typedef void (*ForceFn)(const SysDev*, int, const int*);

template <int M, int C, int L>
static ForceFn pick(bool ener, bool fp32)
{
    if (ener) return fp32 ? k_force<M, C, L, true, true> : k_force<M, C, L, true, false>;
    return fp32 ? k_force<M, C, L, false, true> : k_force<M, C, L, false, false>;
}

template <int M>
static ForceFn pick_m(int coul, int lj, bool ener, bool fp32)
{
    switch (coul * 2 + lj) {
    case 0: return pick<M, 0, 0>(ener, fp32);
    case 1: return pick<M, 0, 1>(ener, fp32);
    case 2: return pick<M, 1, 0>(ener, fp32);
    case 3: return pick<M, 1, 1>(ener, fp32);
    case 4: return pick<M, 2, 0>(ener, fp32);
    default: return pick<M, 2, 1>(ener, fp32);
    }
}

hipError_t launch_force(const SysDev* table, int n_sys, const int* item_prefix, int M, int coulomb,
                        int lj, bool ener, bool fp32, int total_item_cap, hipStream_t s)
{
    ForceFn fn;
    if (M == 8) fn = pick_m<8>(coulomb, lj, ener, fp32);
    else if (M == 4) fn = pick_m<4>(coulomb, lj, ener, fp32);
    else if (M == 1) fn = pick_m<1>(coulomb, lj, ener, fp32);
    else return hipErrorInvalidValue;
    // persistent grid: enough waves to fill 256 CUs several times over
    // (a multiple of 8 so the XCD-aware block remap in the kernel is a bijection)
    int blocks = (total_item_cap + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 8) blocks = 8;
    blocks = (blocks + 7) / 8 * 8;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, s, table, n_sys, item_prefix);
    return hipGetLastError();
}

}  // namespace nbi
