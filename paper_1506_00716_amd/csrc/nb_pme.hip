// nb_pme.hip -- reciprocal-space Ewald by smooth particle-mesh Ewald (gfx950).
//
// The paper splits the electrostatics into the short-range pair part of the
// cluster-pair kernel and a long-range lattice part computed by PME, a 3D FFT
// on a charge grid (Section "Multi-level parallelism", Fig. 2), which it runs
// on the CPU beside the GPU's pair forces (Section "Heterogeneous
// parallelization").  Here every stage runs on the GPU, in the same stream as
// the pair kernel, in FP64 except the charge grid (64-bit fixed point: sums of
// integers do not depend on the order of the atoms) and the output forces
// (FP32, as the pair forces):
//   prep     per atom its cardinal B-spline weights of order P (M_P(w + j)
//            from the recursion that defines M_P), their derivatives and its
//            base grid point; the atoms binned by their (a, b) grid column
//            (count, scan, place);
//   spread   one wave per grid line along c gathers the atoms of the P x P
//            columns that reach it into an LDS copy of the line, then the
//            line's real DFT along c to its K2/2 + 1 half-complex points;
//   b pass   complex DFT along b, tiles of h_c columns staged in LDS;
//   a pass   complex DFT along a, the influence function
//            G(m) = exp(-pi^2 m^2/beta^2) B(m) / (pi V m^2) (tabulated per
//            system), the energy and virial partials, and the inverse DFT
//            along a, in one LDS tile;
//   b pass   inverse DFT along b;
//   inv_z    half-complex-to-real inverse DFT along c: the potential grid;
//   gather   F_i = -f q_i sum_k grad_i(spline weights) (theta * Q)(k).
// G is zero at m = 0 and at the Nyquist frequency of an even dimension (which
// has no partner of opposite sign on the grid, so a skewed box would make G(m)
// differ from G(-m) there).  The transforms are direct DFTs of each grid line
// held in LDS (K terms per output in FP64, the twiddle of each term rotated
// from the previous one in registers): the grids of the target systems have a
// few tens of points per dimension, where a line transform inside LDS is
// cheaper than a mixed-radix FFT's passes through memory.
#include "nb_internal.h"

#include <math.h>

namespace nbi {
namespace {

constexpr double kPmeFx = 17179869184.0;  // 2^34: fixed-point scale of the charge grid
constexpr double kPmeFxInv = 1.0 / 17179869184.0;
constexpr int kLanesPerAtom = 16;

// Cardinal B-spline weights A[j] = M_P(w + j) and derivatives D[j] = M_P'(w + j),
// j = 0..P-1, w in [0, 1]: M_2(u) = 1 - |u - 1| on [0, 2],
// M_n(u) = (u M_{n-1}(u) + (n - u) M_{n-1}(u - 1)) / (n - 1) and
// M_n'(u) = M_{n-1}(u) - M_{n-1}(u - 1).
template <int P>
__device__ __forceinline__ void bspline(double w, double A[P], double D[P])
{
    A[0] = w;
    A[1] = 1.0 - w;
#pragma unroll
    for (int j = 2; j < P; ++j) A[j] = 0.0;
#pragma unroll
    for (int n = 3; n <= P; ++n) {
        if (n == P) {
#pragma unroll
            for (int j = 0; j < P; ++j) D[j] = (j < P - 1 ? A[j] : 0.0) - (j >= 1 ? A[j - 1] : 0.0);
        }
        const double inv = 1.0 / (n - 1);
        // downwards, so A[j] and A[j - 1] still hold M_{n-1}
#pragma unroll
        for (int j = n - 1; j >= 0; --j) {
            const double u = w + j;
            const double here = j < n - 1 ? A[j] : 0.0;
            const double left = j >= 1 ? A[j - 1] : 0.0;
            A[j] = (u * here + (n - u) * left) * inv;
        }
    }
}

// Scaled fractional coordinate u = K (r . a*_k) modulo K: the spline's base
// grid point and offset w = u - base in [0, 1).
__device__ __forceinline__ void grid_coord(double s, int K, int& base, double& w)
{
#pragma clang fp contract(off)
    const double Kd = (double)K;
    double u = s * Kd;
    u = u - floor(u / Kd) * Kd;
    int b = (int)floor(u);
    if (b >= K) {  // (u rounded up to K)
        b -= K;
        u -= Kd;
    }
    base = b;
    w = u - (double)b;
}

template <int P>
__device__ __forceinline__ void atom_splines(const PmeDev& p, const double* __restrict__ x, int atom, int base[3],
                                             double A[3][P], double D[3][P])
{
    const double r0 = gld(&x[3 * atom]), r1 = gld(&x[3 * atom + 1]), r2 = gld(&x[3 * atom + 2]);
    double s[3];
    s[0] = r0 * p.rec[0] + r1 * p.rec[1] + r2 * p.rec[2];
    s[1] = r1 * p.rec[3] + r2 * p.rec[4];
    s[2] = r2 * p.rec[5];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double w;
        grid_coord(s[k], p.K[k], base[k], w);
        bspline<P>(w, A[k], D[k]);
    }
}

// grid index base - j, wrapped (K >= P, so one period suffices)
__device__ __forceinline__ int wrap_down(int base, int j, int K)
{
    const int i = base - j;
    return i < 0 ? i + K : i;
}

// complex multiply-add helpers (FP64)
__device__ __forceinline__ void cmac(double& re, double& im, double vr, double vi, double wr, double wi)
{
    re = fma(vr, wr, re);
    re = fma(-vi, wi, re);
    im = fma(vr, wi, im);
    im = fma(vi, wr, im);
}
// w <- w * s (the twiddle of the next term: rotating by s costs four FMAs
// and no table read; after K steps its error is K FP64 roundings)
__device__ __forceinline__ void rotate(double& wr, double& wi, double sr, double si)
{
    const double t = wr * sr - wi * si;
    wi = fma(wr, si, wi * sr);
    wr = t;
}

// Per atom: spline base points, weights and derivatives, and its place in its
// (a, b) grid column's bucket, or past a full bucket in the overflow list (the
// counts are all zero on entry).  Weights are stored atom by atom (3P values
// each); the block stages them in LDS so that its stores are contiguous.
template <int P>
__global__ __launch_bounds__(256) void k_pme_prep(PmeDev p, const double* __restrict__ x)
{
    __shared__ double stage[256 * 3 * P];
    const int a0 = blockIdx.x * 256;
    const int atom = a0 + threadIdx.x;
    const bool real = atom < p.n_atoms;
    double A[3][P], D[3][P];
    if (real) {
        int base[3];
        atom_splines<P>(p, x, atom, base, A, D);
        const int col = base[0] * p.K[1] + base[1];
        p.atom_base[atom] = make_int4(base[0], base[1], base[2], col);
        const int r = gatomic_add(&p.col_count[col], 1);
        if (r < p.col_cap) gst(&p.col_list[(size_t)col * p.col_cap + r], atom);
        else gst(&p.ovf_list[gatomic_add(p.ovf_count, 1)], atom);
    }
    const int na = min(256, p.n_atoms - a0);
    for (int pass = 0; pass < 2; ++pass) {
        if (real)
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < P; ++j) stage[threadIdx.x * 3 * P + k * P + j] = pass ? D[k][j] : A[k][j];
        __syncthreads();
        double* out = (pass ? p.dtheta : p.theta) + (size_t)a0 * 3 * P;
        for (int i = threadIdx.x; i < na * 3 * P; i += 256) gst(&out[i], stage[i]);
        __syncthreads();
    }
}

// One wave per grid line along c at (i_a, i_b): the atoms of the P x P columns
// whose splines reach the line add q M(a) M(b) M(c) into an LDS copy of the
// line (64-bit fixed point: integer adds, so the order of the atoms does not
// matter), then the line's real DFT along c goes to its K2/2 + 1 half-complex
// points, two lanes per output (each sums half the line).  No global atomics:
// every grid value has one writer.
template <int P>
__global__ __launch_bounds__(256) void k_pme_spread_z(PmeDev p)
{
    extern __shared__ double lds[];
    __shared__ int cstart[4][P * P + 1], cbase[4][P * P];
    __shared__ int novf_s;
    const int K0 = p.K[0], K1 = p.K[1], K2 = p.K[2], H2 = p.H2;
    double2* tw = (double2*)lds;
    long long* lines = (long long*)(lds + 2 * K2);
    for (int j = threadIdx.x; j < K2; j += 256) tw[j] = p.tw[K0 + K1 + j];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + wid;
    const bool live = row < K0 * K1;
    long long* line = lines + wid * K2;
    for (int n = lane; n < K2; n += 64) line[n] = 0;
    if (threadIdx.x == 0) novf_s = gld(p.ovf_count);
    int total = 0;
    int i0 = 0, i1 = 0;
    if (live) {
        i0 = row / K1;
        i1 = row % K1;
        // column (i0 + a, i1 + b) holds the atoms with base (i0 + a, i1 + b):
        // their weights j = a and j = b land on this line
        int cnt = 0, st = 0;
        if (lane < P * P) {
            const int a = lane / P, b = lane % P;
            const int ca = i0 + a < K0 ? i0 + a : i0 + a - K0, cb = i1 + b < K1 ? i1 + b : i1 + b - K1;
            const int col = ca * K1 + cb;
            st = col * p.col_cap;
            cnt = min(gld(&p.col_count[col]), p.col_cap);
        }
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane < P * P) {
            cstart[wid][lane + 1] = incl;
            cbase[wid][lane] = st;
        }
        if (lane == 0) cstart[wid][0] = 0;
        total = __shfl(incl, P * P - 1, 64);
    }
    __syncthreads();
    // atom `atom` with weights j = a along a and j = b along b on this line
    auto add_atom = [&](int atom, int a, int b, int b2) {
        const double* th = p.theta + (size_t)atom * 3 * P;
        const double wab = gld(&p.q[atom]) * gld(&th[a]) * gld(&th[P + b]) * kPmeFx;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            const long long v = __double2ll_rn(wab * gld(&th[2 * P + c]));
            atomicAdd((unsigned long long*)&line[wrap_down(b2, c, K2)], (unsigned long long)v);
        }
    };
    for (int e = lane; e < total; e += 64) {
        int ab = 0;
        while (cstart[wid][ab + 1] <= e) ++ab;
        const int atom = gld(&p.col_list[cbase[wid][ab] + (e - cstart[wid][ab])]);
        add_atom(atom, ab / P, ab % P, p.atom_base[atom].z);
    }
    // atoms past their column's bucket: those whose column is in reach
    const int novf = live ? novf_s : 0;
    for (int e = lane; e < novf; e += 64) {
        const int atom = gld(&p.ovf_list[e]);
        const int4 bs = p.atom_base[atom];
        const int a = bs.x >= i0 ? bs.x - i0 : bs.x - i0 + K0, b = bs.y >= i1 ? bs.y - i1 : bs.y - i1 + K1;
        if (a < P && b < P) add_atom(atom, a, b, bs.z);
    }
    __syncthreads();
    if (!live) return;
    const int half = lane & 1, nmid = K2 / 2;
    const int n0 = half ? nmid : 0, n1 = half ? K2 : nmid;
    for (int hc = 0; hc < H2; hc += 32) {
        const int h = hc + (lane >> 1);
        double re = 0.0, im = 0.0;
        if (h < H2) {
            // exp(-2 pi i h n / K2) from n = n0 on
            const double2 t0 = tw[(int)(((long long)h * n0) % K2)], ts = tw[h];
            double wr = t0.x, wi = -t0.y;
            const double sr = ts.x, si = -ts.y;
            for (int n = n0; n < n1; ++n) {
                const double v = (double)line[n] * kPmeFxInv;
                re = fma(v, wr, re);
                im = fma(v, wi, im);
                rotate(wr, wi, sr, si);
            }
        }
        re += __shfl_xor(re, 1, 64);
        im += __shfl_xor(im, 1, 64);
        if (!half && h < H2) p.cgrid[(size_t)row * H2 + h] = make_double2(re, im);
    }
}

// Part of a strided DFT sum: sum over k in [kb, ke) of v[k T + c] w^k with
// w = exp(i sg 2 pi h / K), v a tile in LDS
__device__ __forceinline__ void dft_part(const double2* tile, int T, int c, int K, int h, double sg, int kb, int ke,
                                         const double2* __restrict__ tw, double& re, double& im)
{
    const double2 t0 = tw[(int)(((long long)h * kb) % K)], ts = tw[h];
    double wr = t0.x, wi = sg * t0.y;
    const double sr = ts.x, si = sg * ts.y;
    for (int k = kb; k < ke; ++k) {
        const double2 v = tile[k * T + c];
        cmac(re, im, v.x, v.y, wr, wi);
        rotate(wr, wi, sr, si);
    }
}

// The b and a passes give each output kSplit consecutive lanes, each summing a
// kSplit-th of the line, so a pass runs several thousand waves
constexpr int kSplit = 4;

// complex DFT along b (sign -1 forward, +1 inverse) of a tile of h_c columns
__global__ __launch_bounds__(256) void k_pme_y(PmeDev p, double sg)
{
    extern __shared__ double lds[];
    const int K1 = p.K[1], H2 = p.H2, T = p.tile;
    double2* tile = (double2*)lds;
    const double2* tw = p.tw + p.K[0];
    const int ntile = (H2 + T - 1) / T;
    const int k0 = blockIdx.x / ntile, c0 = (blockIdx.x % ntile) * T;
    double2* g = p.cgrid + (size_t)k0 * K1 * H2;
    for (int e = threadIdx.x; e < K1 * T; e += 256) {
        const int k1 = e / T, c = e % T;
        tile[e] = (c0 + c < H2) ? g[(size_t)k1 * H2 + c0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int items = K1 * T * kSplit;
    for (int e0 = 0; e0 < items; e0 += 256) {
        const int e = e0 + threadIdx.x;
        const int o = e / kSplit, sp = e % kSplit;
        const int h1 = o / T, c = o % T;
        double re = 0.0, im = 0.0;
        if (e < items) dft_part(tile, T, c, K1, h1, sg, sp * K1 / kSplit, (sp + 1) * K1 / kSplit, tw, re, im);
#pragma unroll
        for (int m = 1; m < kSplit; m <<= 1) {
            re += __shfl_xor(re, m, 64);
            im += __shfl_xor(im, m, 64);
        }
        if (e < items && sp == 0 && c0 + c < H2) g[(size_t)h1 * H2 + c0 + c] = make_double2(re, im);
    }
}

// signed frequency of index h on a K-point grid (numpy's FFT order), and
// whether it is the unpaired Nyquist point of an even K
__device__ __forceinline__ int signed_freq(int h, int K, bool& nyq)
{
    nyq = (K % 2 == 0) && (h == K / 2);
    return h < (K + 1) / 2 ? h : h - K;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// DFT along a, influence function (energy and virial partials with ener),
// inverse DFT along a, for a tile of h_c columns at one h_b
__global__ __launch_bounds__(256) void k_pme_x_solve(PmeDev p, int ener)
{
    extern __shared__ double lds[];
    __shared__ double red[4][8];
    const int K0 = p.K[0], K1 = p.K[1], K2 = p.K[2], H2 = p.H2, T = p.tile;
    double2* tA = (double2*)lds;
    double2* tB = tA + K0 * T;
    const double2* tw = p.tw;
    const int ntile = (H2 + T - 1) / T;
    const int h1 = blockIdx.x / ntile, c0 = (blockIdx.x % ntile) * T;
    const size_t rstride = (size_t)K1 * H2;
    double2* g = p.cgrid + (size_t)h1 * H2 + c0;
    for (int e = threadIdx.x; e < K0 * T; e += 256) {
        const int k0 = e / T, c = e % T;
        tA[e] = (c0 + c < H2) ? g[(size_t)k0 * rstride + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    bool ny1;
    const int f1 = signed_freq(h1, K1, ny1);
    double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int items = K0 * T * kSplit;
    for (int e0 = 0; e0 < items; e0 += 256) {
        const int e = e0 + threadIdx.x;
        const int o = e / kSplit, sp = e % kSplit;
        const int h0 = o / T, c = o % T;
        double re = 0.0, im = 0.0;
        if (e < items) dft_part(tA, T, c, K0, h0, -1.0, sp * K0 / kSplit, (sp + 1) * K0 / kSplit, tw, re, im);
#pragma unroll
        for (int m = 1; m < kSplit; m <<= 1) {
            re += __shfl_xor(re, m, 64);
            im += __shfl_xor(im, m, 64);
        }
        if (e >= items || sp != 0) continue;
        const int h2 = c0 + c;
        bool ny0;
        const int f0 = signed_freq(h0, K0, ny0);
        const bool ny2 = (K2 % 2 == 0) && (h2 == K2 / 2);
        const bool zero = (h2 >= H2) || ny0 || ny1 || ny2 || (f0 == 0 && f1 == 0 && h2 == 0);
        // the influence function of this point, tabulated per system
        const double G = zero ? 0.0 : gld(&p.gtab[((size_t)h0 * K1 + h1) * H2 + h2]);
        if (!zero) {
            if (ener) {
                const double mx = f0 * p.rec[0];
                const double my = f0 * p.rec[1] + f1 * p.rec[3];
                const double mz = f0 * p.rec[2] + f1 * p.rec[4] + h2 * p.rec[5];
                const double m2 = mx * mx + my * my + mz * mz;
                // the half-complex point stands for itself and its mirror,
                // except on the plane h_c = 0 (the plane K2/2 is left out)
                const double wz = h2 == 0 ? 1.0 : 2.0;
                const double Em = 0.5 * wz * G * (re * re + im * im);
                const double fac = Em * 2.0 * (1.0 + p.pi2_b2 * m2) / m2;
                acc[0] += Em;
                acc[1] += -0.5 * (Em - fac * mx * mx);
                acc[2] += -0.5 * (Em - fac * my * my);
                acc[3] += -0.5 * (Em - fac * mz * mz);
                acc[4] += 0.5 * fac * mx * my;
                acc[5] += 0.5 * fac * mx * mz;
                acc[6] += 0.5 * fac * my * mz;
            }
        }
        tB[h0 * T + c] = make_double2(re * G, im * G);
    }
    __syncthreads();
    for (int e0 = 0; e0 < items; e0 += 256) {
        const int e = e0 + threadIdx.x;
        const int o = e / kSplit, sp = e % kSplit;
        const int k0 = o / T, c = o % T;
        double re = 0.0, im = 0.0;
        if (e < items) dft_part(tB, T, c, K0, k0, 1.0, sp * K0 / kSplit, (sp + 1) * K0 / kSplit, tw, re, im);
#pragma unroll
        for (int m = 1; m < kSplit; m <<= 1) {
            re += __shfl_xor(re, m, 64);
            im += __shfl_xor(im, m, 64);
        }
        if (e < items && sp == 0 && c0 + c < H2) g[(size_t)k0 * rstride + c] = make_double2(re, im);
    }
    if (!ener) return;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        const int k = threadIdx.x;
        gst(&p.epart[(size_t)blockIdx.x * 8 + k], (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]));
    }
}

// inverse DFT along c from the half-complex points to K2 real values (one wave per line)
__global__ __launch_bounds__(256) void k_pme_inv_z(PmeDev p)
{
    extern __shared__ double lds[];
    const int K2 = p.K[2], H2 = p.H2;
    double2* rows = (double2*)lds;
    const double2* tw = p.tw + p.K[0] + p.K[1];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + wid;
    const int nrows = p.K[0] * p.K[1];
    double2* r = rows + wid * H2;
    if (row < nrows)
        for (int h = lane; h < H2; h += 64) r[h] = p.cgrid[(size_t)row * H2 + h];
    __syncthreads();
    if (row >= nrows) return;
    // h = 1 .. (K2-1)/2 pair with K2 - h; the Nyquist point of an even K2 is zero
    const int hmax = (K2 - 1) / 2;
    for (int n = lane; n < K2; n += 64) {
        const double2 ts = tw[n];
        double wr = ts.x, wi = ts.y, s = 0.0;
        for (int h = 1; h <= hmax; ++h) {
            const double2 v = r[h];
            s = fma(v.x, wr, s);
            s = fma(-v.y, wi, s);
            rotate(wr, wi, ts.x, ts.y);
        }
        gst(&p.conv[(size_t)row * K2 + n], r[0].x + 2.0 * s);
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_pme_gather(PmeDev p)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int atom_l = t / kLanesPerAtom, l = t % kLanesPerAtom;
    const bool real = atom_l < p.n_atoms;
    const int atom = real ? atom_l : 0;
    const int4 base = p.atom_base[atom];
    const double* th = p.theta + (size_t)atom * 3 * P;
    const double* dth = p.dtheta + (size_t)atom * 3 * P;
    double A2[P], D2[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        A2[c] = gld(&th[2 * P + c]);
        D2[c] = gld(&dth[2 * P + c]);
    }
    const int K1 = p.K[1], K2 = p.K[2];
    // the spread has read the column counts: cleared for the next evaluation
    for (int i = t; i < p.K[0] * K1; i += gridDim.x * 256) gst(&p.col_count[i], 0);
    if (t == 0) gst(p.ovf_count, 0);
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int ab = l; ab < P * P; ab += kLanesPerAtom) {
        const int a = ab / P, b = ab % P;
        const int i0 = wrap_down(base.x, a, p.K[0]), i1 = wrap_down(base.y, b, K1);
        const double* row = p.conv + ((size_t)i0 * K1 + i1) * K2;
        const double A0 = gld(&th[a]), A1 = gld(&th[P + b]), D0 = gld(&dth[a]), D1 = gld(&dth[P + b]);
        const double aa = A0 * A1, da = D0 * A1, ad = A0 * D1;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            const double cv = gld(&row[wrap_down(base.z, c, K2)]);
            g0 = fma(da * A2[c], cv, g0);
            g1 = fma(ad * A2[c], cv, g1);
            g2 = fma(aa * D2[c], cv, g2);
        }
    }
#pragma unroll
    for (int o = kLanesPerAtom / 2; o >= 1; o >>= 1) {
        g0 += __shfl_xor(g0, o, 64);
        g1 += __shfl_xor(g1, o, 64);
        g2 += __shfl_xor(g2, o, 64);
    }
    if (l != 0 || !real) return;
    // dE/du_k times du_k/dr = K_k a*_k
    g0 *= p.K[0];
    g1 *= K1;
    g2 *= K2;
    const double fq = -p.fel * gld(&p.q[atom]);
    gst(&p.frec[3 * atom + 0], (float)(fq * (g0 * p.rec[0])));
    gst(&p.frec[3 * atom + 1], (float)(fq * (g0 * p.rec[1] + g1 * p.rec[3])));
    gst(&p.frec[3 * atom + 2], (float)(fq * (g0 * p.rec[2] + g1 * p.rec[4] + g2 * p.rec[5])));
}

// energy and virial of the a pass's partials (fixed order) plus the self and
// background terms: -f beta/sqrt(pi) sum q^2 and -f pi (sum q)^2 / (2 V beta^2)
__global__ __launch_bounds__(256) void k_pme_energy(PmeDev p)
{
    __shared__ double red[4][8];
    double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < p.solve_blocks; b += 256)
#pragma unroll
        for (int k = 0; k < 7; ++k) acc[k] += gld(&p.epart[(size_t)b * 8 + k]);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double s[7];
    for (int k = 0; k < 7; ++k) s[k] = p.fel * ((red[0][k] + red[1][k]) + (red[2][k] + red[3][k]));
    const double Q = gld(&p.qsum[0]), Q2 = gld(&p.qsum[1]);
    const double e_self = -p.fel * p.beta / sqrt(M_PI) * Q2;
    const double e_bg = -p.fel * M_PI * Q * Q / (2.0 * p.vol * p.beta * p.beta);
    p.eout[0] = s[0] + e_self + e_bg;
    // the background energy scales as 1/V: its virial is -E_bg/2 on the diagonal
    for (int k = 1; k <= 3; ++k) p.eout[k] = s[k] - 0.5 * e_bg;
    for (int k = 4; k <= 6; ++k) p.eout[k] = s[k];
}

// twiddles, spline moduli |b(m)|^2 = 1 / |sum_j M_P(j) exp(2 pi i m j / K)|^2
// The influence function G(m) = exp(-pi^2 m^2/beta^2) B(m) / (pi V m^2) on the
// half-complex grid (zero at m = 0 and on the Nyquist planes of even
// dimensions): it depends on the box and the grid only, so it is tabulated
// once per system (after the moduli)
__global__ __launch_bounds__(256) void k_pme_gtab(PmeDev p)
{
    const int K0 = p.K[0], K1 = p.K[1], K2 = p.K[2], H2 = p.H2;
    const int n = K0 * K1 * H2;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const int h2 = i % H2, h1 = (i / H2) % K1, h0 = i / (H2 * K1);
        bool ny0, ny1;
        const int f0 = signed_freq(h0, K0, ny0), f1 = signed_freq(h1, K1, ny1);
        const bool ny2 = (K2 % 2 == 0) && (h2 == K2 / 2);
        double G = 0.0;
        if (!(ny0 || ny1 || ny2 || (f0 == 0 && f1 == 0 && h2 == 0))) {
            const double mx = f0 * p.rec[0];
            const double my = f0 * p.rec[1] + f1 * p.rec[3];
            const double mz = f0 * p.rec[2] + f1 * p.rec[4] + h2 * p.rec[5];
            const double m2 = mx * mx + my * my + mz * mz;
            G = exp(-p.pi2_b2 * m2) * p.bmod[h0] * p.bmod[K0 + h1] * p.bmod[K0 + K1 + h2] / (M_PI * p.vol * m2);
        }
        gst(&p.gtab[i], G);
    }
}

// and the charge sums (one block)
template <int P>
__global__ __launch_bounds__(256) void k_pme_setup(PmeDev p)
{
    __shared__ double red[4][2];
    double Mi[P], Di[P];
    bspline<P>(0.0, Mi, Di);
    int off = 0;
    for (int d = 0; d < 3; ++d) {
        const int K = p.K[d];
        for (int m = threadIdx.x; m < K; m += 256) {
            double sn, cs;
            sincospi(2.0 * m / K, &sn, &cs);
            p.tw[off + m] = make_double2(cs, sn);
            double re = 0.0, im = 0.0;
            for (int j = 0; j < P; ++j) {
                double sj, cj;
                sincospi(2.0 * (double)((m * j) % K) / K, &sj, &cj);
                re += Mi[j] * cj;
                im += Mi[j] * sj;
            }
            p.bmod[off + m] = 1.0 / (re * re + im * im);
        }
        off += K;
    }
    double q1 = 0.0, q2 = 0.0;
    for (int i = threadIdx.x; i < p.n_atoms; i += 256) {
        const double v = gld(&p.q[i]);
        q1 += v;
        q2 += v * v;
    }
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    q1 = wave_sum(q1);
    q2 = wave_sum(q2);
    if (lane == 0) {
        red[wid][0] = q1;
        red[wid][1] = q2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        p.qsum[0] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
        p.qsum[1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    }
}

}  // namespace

hipError_t launch_pme_setup(const PmeDev& p, hipStream_t s)
{
    if (p.order == 6)
        hipLaunchKernelGGL(k_pme_setup<6>, dim3(1), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL(k_pme_setup<4>, dim3(1), dim3(256), 0, s, p);
    const int n = p.K[0] * p.K[1] * p.H2;
    hipLaunchKernelGGL(k_pme_gtab, dim3(min(1024, (n + 255) / 256)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_pme(const PmeDev& p, const double* x, bool ener, hipStream_t s)
{
    const int K0 = p.K[0], K1 = p.K[1], K2 = p.K[2];
    const int nb = (p.n_atoms + 255) / 256;
    const int ab = (int)(((long long)p.n_atoms * kLanesPerAtom + 255) / 256);
    const int lines = (K0 * K1 + 3) / 4;
    const int ntile = (p.H2 + p.tile - 1) / p.tile;
    const size_t lz = sizeof(double) * 2 * K2 + sizeof(long long) * 4 * K2;
    const size_t ly = sizeof(double2) * (size_t)K1 * p.tile;
    const size_t lx = sizeof(double2) * (size_t)K0 * 2 * p.tile;
    const size_t lc = sizeof(double2) * 4 * p.H2;
    if (p.order == 6) {
        hipLaunchKernelGGL(k_pme_prep<6>, dim3(nb), dim3(256), 0, s, p, x);
        hipLaunchKernelGGL(k_pme_spread_z<6>, dim3(lines), dim3(256), lz, s, p);
    } else {
        hipLaunchKernelGGL(k_pme_prep<4>, dim3(nb), dim3(256), 0, s, p, x);
        hipLaunchKernelGGL(k_pme_spread_z<4>, dim3(lines), dim3(256), lz, s, p);
    }
    hipLaunchKernelGGL(k_pme_y, dim3(K0 * ntile), dim3(256), ly, s, p, -1.0);
    hipLaunchKernelGGL(k_pme_x_solve, dim3(K1 * ntile), dim3(256), lx, s, p, ener ? 1 : 0);
    hipLaunchKernelGGL(k_pme_y, dim3(K0 * ntile), dim3(256), ly, s, p, 1.0);
    hipLaunchKernelGGL(k_pme_inv_z, dim3(lines), dim3(256), lc, s, p);
    if (p.order == 6)
        hipLaunchKernelGGL(k_pme_gather<6>, dim3(ab), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL(k_pme_gather<4>, dim3(ab), dim3(256), 0, s, p);
    if (ener) hipLaunchKernelGGL(k_pme_energy, dim3(1), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace nbi
