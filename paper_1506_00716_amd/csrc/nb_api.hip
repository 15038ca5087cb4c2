// nb_api.hip -- host side of libnb: the C ABI declared in include/nb.h.
//
// Validation, arena layout, model constants (including the Ewald erfc fit),
// and the orchestration of the device kernels on the context's stream.
#include "../../include/nb.h"
#include "nb_host.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace nbi;

namespace nbh {
thread_local std::string g_last_error;
}  // namespace nbh

using namespace nbh;

namespace {

const double kOneOver4PiEps0 = 138.935458;  // kJ mol^-1 nm e^-2

// Working memory of nb_compute_forces_noalloc: one fixed array per GPU, held by
// the loaded library until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: the device address of each GPU's copy
// comes from hipGetSymbolAddress, taken once per device (at context creation,
// with that device current) and kept in scratch_dev[device].
constexpr size_t kNoallocBytes = size_t(64) << 20;
constexpr int kNoallocMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoallocBytes];
std::mutex g_scratch_mu;
void* scratch_dev[kNoallocMaxDevices];
hipError_t scratch_err[kNoallocMaxDevices];

// address of this device's scratch array (device current), looked up once
void scratch_setup(int device)
{
    if (device < 0 || device >= kNoallocMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (scratch_dev[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    scratch_err[device] = e;
    if (e == hipSuccess) scratch_dev[device] = ptr;
}

}  // namespace

namespace nbh {

nb_status fail(nb_ctx* ctx, nb_status code, const std::string& msg)
{
    g_last_error = msg;
    if (ctx) ctx->err = msg;
    return code;
}

}  // namespace nbh

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool pme_on(const nb_params* p) { return p->pme_grid[0] != 0 || p->pme_grid[1] != 0 || p->pme_grid[2] != 0; }
int pme_order(const nb_params* p) { return p->pme_order == 0 ? 4 : p->pme_order; }

nb_status validate(const nb_params* p, std::string* why)
{
    if (!p) { *why = "params is NULL"; return NB_ERR_ARG; }
    if (p->n_atoms < 1) { *why = "n_atoms must be >= 1"; return NB_ERR_ARG; }
    for (int k = 0; k < 3; ++k)
        if (!(p->box[k] > 0.0) || !std::isfinite(p->box[k])) { *why = "box edges must be > 0"; return NB_ERR_BOX; }
    if (!(p->r_cut > 0.0) || !(p->r_list >= p->r_cut)) {
        *why = "need 0 < r_cut <= r_list";
        return NB_ERR_ARG;
    }
    const double lmin = std::min(p->box[0], std::min(p->box[1], p->box[2]));
    if (!(p->r_list < 0.5 * lmin)) { *why = "r_list must be < half the smallest box edge"; return NB_ERR_BOX; }
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->box_off[k])) { *why = "box_off must be finite"; return NB_ERR_BOX; }
    if (!(std::fabs(p->box_off[0]) <= 0.5 * p->box[0]) || !(std::fabs(p->box_off[1]) <= 0.5 * p->box[0]) ||
        !(std::fabs(p->box_off[2]) <= 0.5 * p->box[1])) {
        *why = "triclinic box needs |b_x| <= a_x/2, |c_x| <= a_x/2, |c_y| <= b_y/2";
        return NB_ERR_BOX;
    }
    if (p->coulomb < 0 || p->coulomb > 2) { *why = "coulomb must be 0, 1 or 2"; return NB_ERR_ARG; }
    if (p->lj < 0 || p->lj > 1) { *why = "lj must be 0 or 1"; return NB_ERR_ARG; }
    if (p->coulomb != NB_COUL_NONE && !(p->eps_r > 0.0)) { *why = "eps_r must be > 0"; return NB_ERR_ARG; }
    if (p->coulomb == NB_COUL_EWALD && !(p->ewald_beta > 0.0)) { *why = "ewald_beta must be > 0"; return NB_ERR_ARG; }
    if (!(p->cluster == 0 || p->cluster == 1 || p->cluster == 4 || p->cluster == 8)) {
        *why = "cluster must be 0, 1, 4 or 8";
        return NB_ERR_ARG;
    }
    if (p->jtile < 0 || p->jtile > 4096) { *why = "jtile out of range"; return NB_ERR_ARG; }
    if (p->force_fixed_bits < 0 || p->force_fixed_bits > 40) { *why = "force_fixed_bits out of range"; return NB_ERR_ARG; }
    if (p->flags & ~(NB_POT_SHIFT | NB_FP32_REDUCE)) { *why = "unknown flag"; return NB_ERR_ARG; }
    if (p->r_inner != 0.0 && !(p->r_inner >= p->r_cut && p->r_inner <= p->r_list)) {
        *why = "r_inner must be 0 (no dynamic pruning) or within [r_cut, r_list]";
        return NB_ERR_ARG;
    }
    if (p->r_inner != 0.0 && p->nstprune < 1) { *why = "nstprune must be >= 1 with r_inner > 0"; return NB_ERR_ARG; }
    if (p->pme_order != 0 && p->pme_order != 4 && p->pme_order != 6) { *why = "pme_order must be 0, 4 or 6"; return NB_ERR_ARG; }
    if (pme_on(p)) {
        if (p->coulomb != NB_COUL_EWALD) { *why = "PME needs coulomb = NB_COUL_EWALD"; return NB_ERR_ARG; }
        const int order = pme_order(p);
        for (int k = 0; k < 3; ++k)
            if (p->pme_grid[k] < order || p->pme_grid[k] > 256) {
                *why = "each pme_grid[k] must be within [pme_order, 256]";
                return NB_ERR_ARG;
            }
    }
    return NB_OK;
}

struct Shape {
    int M, G, jtile, fx_bits, ncx, ncy, max_groups, cand_cap, ent_cap, item_cap;
};

// Grid and capacity estimates from the mean density (a build that overflows
// reports the sizes it needed).
Shape shape_of(const nb_params* p)
{
    Shape s;
    s.M = p->cluster == 0 ? 8 : p->cluster;
    s.G = kGroup;
    s.jtile = p->jtile > 0 ? p->jtile : (s.M == 8 ? 16 : (s.M == 4 ? 32 : 128));
    s.fx_bits = p->force_fixed_bits > 0 ? p->force_fixed_bits : 20;
    const double vol = p->box[0] * p->box[1] * p->box[2];
    const double rho = p->n_atoms / vol;
    const int GM = s.G * s.M;
    const double side = std::cbrt(GM / rho);
    s.ncx = std::max(1, std::min(4096, (int)(p->box[0] / side)));
    s.ncy = std::max(1, std::min(4096, (int)(p->box[1] / side)));
    const int ncols = s.ncx * s.ncy;
    s.max_groups = p->n_atoms / GM + ncols + 1;  // sum over columns of ceil(n_c / GM)
    const double cx = p->box[0] / s.ncx, cy = p->box[1] / s.ncy;
    const double hz = std::min(p->box[2], GM / (rho * cx * cy));
    const double r = p->r_list;
    const double reach = (cx * 1.5 + 2 * r) * (cy * 1.5 + 2 * r) * (hz + 0.5 * hz + 2 * r);
    // a group owns about half of its neighbourhood (the balanced half list)
    double cand = 0.6 * rho * reach / s.M;
    cand = std::min(cand, (double)s.max_groups * s.G * 3.0);  // cannot exceed all images
    s.cand_cap = (int)(cand * 1.3) + 32;
    const double ent = (double)s.max_groups * s.cand_cap * 0.75 + 1024;
    s.ent_cap = (int)std::min(ent, 2.0e9);
    s.item_cap = (int)std::min(item_bound(s.M, s.jtile, s.ent_cap, s.max_groups) + 16, 2.0e9);
    return s;
}

// Carve the arena (base == nullptr: only measure).  Returns the byte size.
size_t layout(const nb_params* p, const Shape& s, char* base, SysDev* d, int** prefix, int** done,
              SysDev** d_desc, PmeDev* pm = nullptr)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* ptr = base ? base + off : nullptr;
        off = align256(off + bytes);
        return ptr;
    };
    const size_t N = (size_t)p->n_atoms;
    const int GM = s.G * s.M;
    const size_t slots = (size_t)s.max_groups * GM;
    const size_t ncl = (size_t)s.max_groups * s.G;
    const int ncols = s.ncx * s.ncy;
    const int words = (s.G * s.M * s.M + 63) / 64;
    SysDev tmp;
    SysDev& o = d ? *d : tmp;
    *d_desc = (SysDev*)take(sizeof(SysDev));
    *prefix = (int*)take(sizeof(int) * 2);
    *done = (int*)take(sizeof(int) * 4);
    o.q = (const double*)take(sizeof(double) * N);
    o.sig = (const double*)take(sizeof(double) * N);
    o.eps = (const double*)take(sizeof(double) * N);
    o.mass = (const double*)take(sizeof(double) * N);
    o.atom_col = (int*)take(sizeof(int) * N);
    o.atom_wrap = (int*)take(sizeof(int) * 3 * N);
    o.atom_zkey = (unsigned int*)take(sizeof(unsigned int) * N);
    o.col_count = (int*)take(sizeof(int) * ncols);
    o.col_fill = (int*)take(sizeof(int) * ncols);
    o.col_start = (int*)take(sizeof(int) * (ncols + 1));
    o.col_gstart = (int*)take(sizeof(int) * (ncols + 1));
    o.sort_key = (unsigned long long*)take(sizeof(unsigned long long) * N);
    o.sort_out = (unsigned long long*)take(sizeof(unsigned long long) * N);
    o.slot_atom = (int*)take(sizeof(int) * slots);
    o.xq = (float4*)take(sizeof(float4) * slots);
    o.ljs = (float2*)take(sizeof(float2) * slots);
    o.slot_wrap = (int*)take(sizeof(int) * 3 * slots);
    o.slot_x = (double*)take(sizeof(double) * 3 * slots);
    o.n_groups = (int*)take(sizeof(int) * 4);
    o.cl_nreal = (int*)take(sizeof(int) * ncl);
    o.cl_bb = (double*)take(sizeof(double) * 6 * ncl);
    o.gr_ref = (double*)take(sizeof(double) * 3 * s.max_groups);
    o.gr_bb = (double*)take(sizeof(double) * 6 * s.max_groups);
    o.grp_col = (int*)take(sizeof(int) * s.max_groups);
    o.grp_range = (int2*)take(sizeof(int2) * s.max_groups);
    o.cand_count = (int*)take(sizeof(int) * s.max_groups);
    o.cand = (int2*)take(sizeof(int2) * (size_t)s.max_groups * s.cand_cap);
    o.cand_mask = (unsigned long long*)take(sizeof(unsigned long long) * (size_t)s.max_groups *
                                            s.cand_cap * words);
    o.cand_kept = (int*)take(sizeof(int) * s.max_groups);
    o.grp_rc = (int*)take(sizeof(int) * s.max_groups);
    o.grp_w = (int*)take(sizeof(int) * s.max_groups);
    o.ent_start = (int*)take(sizeof(int) * (s.max_groups + 1));
    o.item_start = (int*)take(sizeof(int) * (s.max_groups + 1));
    o.ent = (int2*)take(sizeof(int2) * (size_t)s.ent_cap);
    o.ent_S = (float4*)take(sizeof(float4) * (size_t)s.ent_cap);
    o.items = (int4*)take(sizeof(int4) * (size_t)s.item_cap);
    o.jpart = (float*)take(sizeof(float) * 3 * (size_t)s.ent_cap * s.M);
    o.ipart = (float*)take(sizeof(float) * 3 * (size_t)s.item_cap * GM);
    o.jstart = (int*)take(sizeof(int) * (ncl + 1));
    o.jfill = (int*)take(sizeof(int) * ncl);
    o.n_items = (int*)take(sizeof(int) * 4);
    o.n_ent = (int*)take(sizeof(int) * 4);
    o.epart = (float*)take(sizeof(float) * kEnerPart * (size_t)s.item_cap);
    o.ke_part = (double*)take(sizeof(double) * kKeBlocks);
    o.eout = (double*)take(sizeof(double) * 16);
    // the status words, then the energy-row ring (one copy returns both)
    static_assert(sizeof(int) * ST_COUNT <= kStatusBytes, "status words exceed their slot");
    o.status = (int*)take(kStatusBytes + sizeof(double) * 5 * kTraceCap);
    o.trace = o.status ? (double*)((char*)o.status + kStatusBytes) : nullptr;
    o.fmax_part = (double*)take(sizeof(double) * kKeBlocks);
    o.stats = (int*)take(sizeof(int) * 8);
    o.x_build = (double*)take(sizeof(double) * 3 * N);
    o.x_bak = (double*)take(sizeof(double) * 3 * N);
    o.v_bak = (double*)take(sizeof(double) * 3 * N);
    o.disp = (double*)take(sizeof(double) * (kKeBlocks + 2));
    o.x_prune = (double*)take(sizeof(double) * 3 * N);
    o.pg_part = (double*)take(sizeof(double) * (2 * kKeBlocks + 2));
    o.exp_count = (long long*)take(sizeof(long long) * (s.max_groups + 1));
    o.ew_tab = (float4*)take(sizeof(float4) * kEwTabN);
    o.ew_etab = (float4*)take(sizeof(float4) * kEwTabN);
    o.pme_f = nullptr;
    o.pme_e = nullptr;
    if (pme_on(p)) {
        PmeDev ptmp;
        PmeDev& P = pm ? *pm : ptmp;
        const int K0 = p->pme_grid[0], K1 = p->pme_grid[1], K2 = p->pme_grid[2];
        const int H2 = K2 / 2 + 1;
        const size_t grid = (size_t)K0 * K1 * K2, half = (size_t)K0 * K1 * H2, ks = (size_t)K0 + K1 + K2;
        // b and a passes: tiles of 2 h_c columns (LDS 2 tile K complex values)
        P.tile = 2;
        P.solve_blocks = K1 * ((H2 + P.tile - 1) / P.tile);
        const int order = pme_order(p);
        // column buckets: twice the mean occupancy plus 16 keeps a uniform
        // liquid far from overflow (a Poisson count past it is below 1e-12);
        // crowded columns spill into the overflow list
        const size_t ncol = (size_t)K0 * K1;
        const size_t mean = ((size_t)N + ncol - 1) / ncol;
        P.col_cap = (int)((2 * mean + 16 + 3) / 4 * 4);
        P.col_count = (int*)take(sizeof(int) * ncol);
        P.col_list = (int*)take(sizeof(int) * ncol * P.col_cap);
        P.ovf_count = (int*)take(sizeof(int));
        P.ovf_list = (int*)take(sizeof(int) * N);
        P.atom_base = (int4*)take(sizeof(int4) * N);
        P.theta = (double*)take(sizeof(double) * 3 * order * N);
        P.dtheta = (double*)take(sizeof(double) * 3 * order * N);
        P.conv = (double*)take(sizeof(double) * grid);
        P.cgrid = (double2*)take(sizeof(double2) * half);
        P.bmod = (double*)take(sizeof(double) * ks);
        P.gtab = (double*)take(sizeof(double) * half);
        P.tw = (double2*)take(sizeof(double2) * ks);
        P.epart = (double*)take(sizeof(double) * 8 * (size_t)P.solve_blocks);
        P.qsum = (double*)take(sizeof(double) * 2);
        P.eout = (double*)take(sizeof(double) * 8);
        P.frec = (float*)take(sizeof(float) * 3 * N);
        o.pme_f = P.frec;
        o.pme_e = P.eout;
    }
    return off + 256;  // slack for aligning the caller's pointer
}

// PME constants of a lower-triangular box: reciprocal vectors a*, b*, c* (the
// rows of inv(L)^T for lattice rows a, b, c), volume, 1/(4 pi eps0 eps_r)
void fill_pme(const nb_params* p, const SysDev& d, PmeDev& P)
{
    P.n_atoms = p->n_atoms;
    for (int k = 0; k < 3; ++k) P.K[k] = p->pme_grid[k];
    P.H2 = P.K[2] / 2 + 1;
    P.order = pme_order(p);
    const double ax = p->box[0], by = p->box[1], cz = p->box[2];
    const double bx = p->box_off[0], cx = p->box_off[1], cy = p->box_off[2];
    P.rec[0] = 1.0 / ax;
    P.rec[1] = -bx / (ax * by);
    P.rec[2] = (bx * cy - by * cx) / (ax * by * cz);
    P.rec[3] = 1.0 / by;
    P.rec[4] = -cy / (by * cz);
    P.rec[5] = 1.0 / cz;
    P.vol = ax * by * cz;
    P.fel = kOneOver4PiEps0 / p->eps_r;
    P.beta = p->ewald_beta;
    P.pi2_b2 = M_PI * M_PI / (p->ewald_beta * p->ewald_beta);
    P.q = d.q;
}

// Piecewise-cubic tables of the Ewald real-space factors on kEwTab equal
// intervals of [0, rc] plus one past rc (kEwTabN in all): per interval the
// cubic through 4 Chebyshev points in w in [0, 1], FP64, stored as FP32
// coefficients.
//   force:     q(r) = erfc(beta r) + (2 beta r / sqrt(pi)) exp(-beta^2 r^2)
//              (F = f qq q(r) r_ij / r^3)
//   potential: e(r) = erfc(beta r)  (V = f qq (e(r) / r - shift))
// The same force table serves every pass, so a step's forces do not depend on
// whether its energies are asked for.  Returns the max relative error of the
// two FP32 tables on [0, rc] (evaluated in FP64).
double fit_ewald_tables(double beta, double rc, float4* ftab, float4* etab)
{
    double tn[4], inv[4][4];
    for (int k = 0; k < 4; ++k) tn[k] = 0.5 * (1.0 - std::cos((2 * k + 1) * M_PI / 8.0));
    // inverse of the 4x4 Vandermonde matrix by Gauss-Jordan
    double a[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            a[i][j] = std::pow(tn[i], j);
            a[i][4 + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
        for (int j = 0; j < 8; ++j) std::swap(a[c][j], a[piv][j]);
        const double dv = a[c][c];
        for (int j = 0; j < 8; ++j) a[c][j] /= dv;
        for (int r = 0; r < 4; ++r)
            if (r != c) {
                const double f = a[r][c];
                for (int j = 0; j < 8; ++j) a[r][j] -= f * a[c][j];
            }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) inv[i][j] = a[i][4 + j];
    const double h = rc / kEwTab;
    double worst = 0.0;
    auto fit = [&](auto fn, float4* tab) {
        for (int k = 0; k < kEwTabN; ++k) {
            double v[4], c[4];
            for (int i = 0; i < 4; ++i) v[i] = fn((k + tn[i]) * h);
            for (int i = 0; i < 4; ++i) {
                c[i] = 0.0;
                for (int j = 0; j < 4; ++j) c[i] += inv[i][j] * v[j];
            }
            tab[k] = make_float4((float)c[0], (float)c[1], (float)c[2], (float)c[3]);
            if (k >= kEwTab) continue;
            for (int t = 0; t <= 16; ++t) {
                const double w = t / 16.0;
                const double e = ((tab[k].w * w + tab[k].z) * w + tab[k].y) * w + tab[k].x;
                const double ref = fn((k + w) * h);
                worst = std::max(worst, std::fabs(e / ref - 1.0));
            }
        }
    };
    fit([&](double r) {
        const double x = beta * r;
        return std::erfc(x) + 2.0 * x / std::sqrt(M_PI) * std::exp(-x * x);
    }, ftab);
    fit([&](double r) { return std::erfc(beta * r); }, etab);
    return worst;
}

void fill_model(const nb_params* p, const Shape& s, SysDev& d)
{
    d.n_atoms = p->n_atoms;
    d.M = s.M;
    d.G = s.G;
    d.ncx = s.ncx;
    d.ncy = s.ncy;
    d.n_cols = s.ncx * s.ncy;
    d.max_groups = s.max_groups;
    d.cand_cap = s.cand_cap;
    d.ent_cap = s.ent_cap;
    d.item_cap = s.item_cap;
    d.jtile = s.jtile;
    d.item_w = item_weight(s.M, s.jtile);
    d.mask_words = (s.G * s.M * s.M + 63) / 64;
    d.coulomb = p->coulomb;
    d.lj = p->lj;
    d.pot_shift = (p->flags & NB_POT_SHIFT) ? 1 : 0;
    d.fp32_reduce = (p->flags & NB_FP32_REDUCE) ? 1 : 0;
    for (int k = 0; k < 3; ++k) {
        d.box[k] = p->box[k];
        d.invbox[k] = 1.0 / p->box[k];
        d.box_off[k] = p->box_off[k];
    }
    d.tric = (p->box_off[0] != 0.0 || p->box_off[1] != 0.0 || p->box_off[2] != 0.0) ? 1 : 0;
    d.cell[0] = p->box[0] / s.ncx;
    d.cell[1] = p->box[1] / s.ncy;
    d.inv_cell[0] = s.ncx / p->box[0];
    d.inv_cell[1] = s.ncy / p->box[1];
    d.rlist2 = p->r_list * p->r_list;
    d.rcut2 = p->r_cut * p->r_cut;
    d.buffer = p->r_list - p->r_cut;
    d.rbb = p->r_list + 1e-6;
    const double rc = p->r_cut;
    d.rc2 = (float)(rc * rc);
    d.rl2_prune = (float)(p->r_list * p->r_list * (1.0 + 1.0 / 16384.0));
    d.prune_on = p->r_inner > 0.0 ? 1 : 0;
    // a cluster pair is kept if an atom pair is within r_inner (1 + 2^-14) in the
    // kernel's FP32 frame: the margin dwarfs that frame's rounding
    d.rin2 = d.prune_on ? (float)(p->r_inner * p->r_inner * (1.0 + 1.0 / 16384.0)) : 0.0f;
    d.prune_half = d.prune_on ? 0.5 * (p->r_inner - p->r_cut) : 0.0;
    d.c6 = (float)p->c6;
    d.c12 = (float)p->c12;
    d.c6x6 = (float)(6.0 * p->c6);
    d.c12x12 = (float)(12.0 * p->c12);
    const double irc6 = 1.0 / (rc * rc * rc * rc * rc * rc);
    d.irc6 = (float)irc6;
    d.irc12 = (float)(irc6 * irc6);
    d.lj_shift = d.pot_shift ? (float)(p->c12 * irc6 * irc6 - p->c6 * irc6) : 0.0f;
    double krf = 0.0;
    if (p->coulomb == NB_COUL_RF)
        krf = p->eps_rf <= 0.0 ? 1.0 / (2.0 * rc * rc * rc)
                               : (p->eps_rf - p->eps_r) / ((2.0 * p->eps_rf + p->eps_r) * rc * rc * rc);
    d.krf = (float)krf;
    d.krf2 = (float)(2.0 * krf);
    d.crf = (float)(1.0 / rc + krf * rc * rc);
    const double beta = p->ewald_beta;
    d.ew_shift = (d.pot_shift && p->coulomb == NB_COUL_EWALD) ? (float)(std::erfc(beta * rc) / rc) : 0.0f;
    d.qscale = p->coulomb == NB_COUL_NONE ? 0.0f : (float)std::sqrt(kOneOver4PiEps0 / p->eps_r);
    d.ew_tinv = (float)(kEwTab / rc);
    d.fx_scale = std::ldexp(1.0, s.fx_bits);
    d.fx_inv = std::ldexp(1.0, -s.fx_bits);
    d.fx_lim = (float)std::ldexp(1.0, 50 - s.fx_bits);
}

Shape shape_of_sys(const nb_sys* s)
{
    Shape sh;
    sh.M = s->M;
    sh.G = s->G;
    sh.jtile = s->jtile;
    sh.fx_bits = s->fx_bits;
    sh.ncx = s->ncx;
    sh.ncy = s->ncy;
    sh.max_groups = s->max_groups;
    sh.cand_cap = s->cand_cap;
    sh.ent_cap = s->ent_cap;
    sh.item_cap = s->item_cap;
    return sh;
}

// HIP-event timer marks (recorded on the context stream around a phase)
hipEvent_t next_event(nb_sys* s)
{
    if (s->ev_used == s->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        s->ev_pool.push_back(e);
    }
    return s->ev_pool[s->ev_used++];
}

// (st: the stream the marked work runs on; NULL = the context stream)
void mark_begin(nb_sys* s, int phase, hipStream_t st = nullptr)
{
    s->mark_open = false;
    if (!s->timing) return;
    // force launches and rebuilds are sampled: each event record between two
    // kernels costs the stream a few microseconds
    if (phase < 2 && (s->mark_seq[phase]++ % s->timing_every) != 0) return;
    const size_t i = s->ev_used;
    hipEvent_t e = next_event(s);
    hipEvent_t f = next_event(s);
    if (!e || !f) return;
    hipEventRecord(e, st ? st : s->ctx->stream);
    s->ev_marks.push_back({i, phase});
    s->mark_open = true;
}

void mark_end(nb_sys* s, hipStream_t st = nullptr)
{
    if (!s->timing || !s->mark_open || s->ev_marks.empty()) return;
    s->mark_open = false;
    hipEventRecord(s->ev_pool[s->ev_marks.back().first + 1], st ? st : s->ctx->stream);
}

// after a synchronisation: fold the recorded pairs into the accumulators
void collect_marks(nb_sys* s)
{
    for (auto& m : s->ev_marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s->ev_pool[m.first], s->ev_pool[m.first + 1]) == hipSuccess) {
            s->t_ms[m.second] += ms;
            s->t_n[m.second] += 1;
        }
    }
    s->ev_marks.clear();
    s->ev_used = 0;
}

// lay the system out on its arena and upload descriptor and particle data
nb_status place(nb_sys* s)
{
    const Shape sh = shape_of_sys(s);
    char* base = (char*)(((uintptr_t)s->arena + 255) & ~uintptr_t(255));
    const size_t need = layout(&s->p, sh, nullptr, nullptr, &s->d_prefix, &s->d_done, &s->d_desc);
    if (need > s->arena_bytes) {
        s->needed_bytes = need;
        return fail(s->ctx, NB_ERR_CAPACITY, "arena too small for this system");
    }
    SysDev d;
    std::memset(&d, 0, sizeof(d));
    fill_model(&s->p, sh, d);
    s->ew_fit_err = 0.0;  // (set below for Ewald, when the tables are fitted)
    std::memset(&s->pme, 0, sizeof(s->pme));
    layout(&s->p, sh, base, &d, &s->d_prefix, &s->d_done, &s->d_desc, &s->pme);
    s->pme_on = pme_on(&s->p);
    if (s->pme_on) fill_pme(&s->p, d, s->pme);
    d.x = nullptr;
    d.v = nullptr;
    d.f = nullptr;
    s->h = d;
    float4 tab[2][kEwTabN];  // (uploaded before the synchronisation below)
    if (s->p.coulomb == NB_COUL_EWALD) {
        s->ew_fit_err = fit_ewald_tables(s->p.ewald_beta, s->p.r_cut, tab[0], tab[1]);
        HIPCHK(s->ctx, hipMemcpyAsync(d.ew_tab, tab[0], sizeof(float4) * kEwTabN, hipMemcpyHostToDevice,
                                      s->ctx->stream));
        HIPCHK(s->ctx, hipMemcpyAsync(d.ew_etab, tab[1], sizeof(float4) * kEwTabN, hipMemcpyHostToDevice,
                                      s->ctx->stream));
        HIPCHK(s->ctx, hipStreamSynchronize(s->ctx->stream));
    }
    s->bounds.max_atoms = s->p.n_atoms;
    s->bounds.max_cols = d.n_cols;
    s->bounds.max_groups = d.max_groups;
    s->bounds.max_slots = d.max_groups * d.G * d.M;
    s->bounds.max_ent = d.ent_cap;
    s->bounds.any_tric = d.tric != 0;
    s->bounds.all_m8 = d.M == 8;
    hipStream_t st = s->ctx->stream;
    HIPCHK(s->ctx, hipMemsetAsync(d.status, 0, sizeof(int) * ST_COUNT, st));
    HIPCHK(s->ctx, hipMemsetAsync(d.ke_part, 0, sizeof(double) * kKeBlocks, st));
    HIPCHK(s->ctx, hipMemsetAsync(d.fmax_part, 0, sizeof(double) * kKeBlocks, st));
    HIPCHK(s->ctx, hipMemsetAsync(d.n_groups, 0, sizeof(int) * 4, st));
    HIPCHK(s->ctx, hipMemsetAsync(d.n_items, 0, sizeof(int) * 4, st));
    HIPCHK(s->ctx, hipMemsetAsync(d.eout, 0, sizeof(double) * 16, st));
    HIPCHK(s->ctx, hipMemsetAsync(d.disp, 0, sizeof(double) * (kKeBlocks + 2), st));
    HIPCHK(s->ctx, hipMemsetAsync(d.pg_part, 0, sizeof(double) * (2 * kKeBlocks + 2), st));
    if (s->pme_on) {
        // the binning counts into cleared columns; the force gather of each
        // evaluation clears them again
        const PmeDev& P = s->pme;
        HIPCHK(s->ctx, hipMemsetAsync(P.col_count, 0, sizeof(int) * P.K[0] * P.K[1], st));
        HIPCHK(s->ctx, hipMemsetAsync(P.ovf_count, 0, sizeof(int), st));
        HIPCHK(s->ctx, hipMemsetAsync(P.eout, 0, sizeof(double) * 8, st));
        HIPCHK(s->ctx, hipMemsetAsync(P.qsum, 0, sizeof(double) * 2, st));
    }
    s->pg_cur = 0;
    s->pg_pending = false;
    s->desc_sent_valid = false;
    HIPCHK(s->ctx, hipMemcpyAsync(s->d_desc, &s->h, sizeof(SysDev), hipMemcpyHostToDevice, st));
    s->desc_sent = s->h;
    s->desc_sent_valid = true;
    const size_t N = (size_t)s->p.n_atoms;
    if (s->has_particles) {
        HIPCHK(s->ctx, hipMemcpyAsync((void*)d.q, s->q.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
        HIPCHK(s->ctx, hipMemcpyAsync((void*)d.sig, s->sig.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
        HIPCHK(s->ctx, hipMemcpyAsync((void*)d.eps, s->eps.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
    }
    if (s->has_mass)
        HIPCHK(s->ctx, hipMemcpyAsync((void*)d.mass, s->mass.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
    if (s->pme_on && s->has_particles) HIPCHK(s->ctx, launch_pme_setup(s->pme, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    s->list_valid = false;
    return NB_OK;
}

// energies at this step (s->step already counts it)
bool ener_step(const nb_sys* s, int32_t nstenergy) { return nstenergy > 0 && (s->step % nstenergy == 0); }

void release_side_stream(nb_sys* s)
{
    if (s->side_stream) {
        hipStreamSynchronize(s->side_stream);
        hipStreamDestroy(s->side_stream);
    }
    if (s->side_in) hipEventDestroy(s->side_in);
    if (s->side_out) hipEventDestroy(s->side_out);
    s->side_stream = nullptr;
    s->side_in = s->side_out = nullptr;
}

// the host fields of a system on `arena` (nothing placed yet)
void init_sys(nb_sys* s, nb_ctx* ctx, const nb_params* p, void* dev_arena, size_t arena_bytes)
{
    s->list_exact = false;
    s->ctx = ctx;
    s->p = *p;
    const Shape sh = shape_of(p);
    s->M = sh.M;
    s->G = sh.G;
    s->jtile = sh.jtile;
    s->fx_bits = sh.fx_bits;
    s->ncx = sh.ncx;
    s->ncy = sh.ncy;
    s->max_groups = sh.max_groups;
    s->cand_cap = sh.cand_cap;
    s->ent_cap = sh.ent_cap;
    s->item_cap = sh.item_cap;
    s->arena = dev_arena;
    s->arena_bytes = arena_bytes;
    s->needed_bytes = 0;
    s->has_particles = false;
    s->has_mass = false;
    s->list_valid = false;
    s->step = 0;
    s->ew_fit_err = 0;
    s->pme_on = false;
    s->side_stream = nullptr;
    s->side_in = s->side_out = nullptr;
    s->ens = nullptr;
    s->f_current = false;
    s->list_step = 0;
    s->pg_cur = 0;
    s->pg_pending = false;
    s->timing = false;
    s->timing_every = 1;
    s->mark_seq[0] = s->mark_seq[1] = 0;
    s->mark_open = false;
    s->check_builds = true;
    s->ev_used = 0;
    for (int k = 0; k < 4; ++k) {
        s->t_ms[k] = 0.0;
        s->t_n[k] = 0;
    }
}

}  // namespace

nb_status nbh::upload_desc(nb_sys* s)
{
    if (s->desc_sent_valid && std::memcmp(&s->desc_sent, &s->h, sizeof(SysDev)) == 0) return NB_OK;
    HIPCHK(s->ctx, hipMemcpyAsync(s->d_desc, &s->h, sizeof(SysDev), hipMemcpyHostToDevice, s->ctx->stream));
    s->desc_sent = s->h;
    s->desc_sent_valid = true;
    return NB_OK;
}

nb_status nbh::read_status(nb_sys* s, int st[ST_COUNT])
{
    HIPCHK(s->ctx, hipMemcpyAsync(st, s->h.status, sizeof(int) * ST_COUNT, hipMemcpyDeviceToHost, s->ctx->stream));
    HIPCHK(s->ctx, hipStreamSynchronize(s->ctx->stream));
    return NB_OK;
}

// grow the capacities that overflowed and report the arena size needed
nb_status nbh::capacity_error(nb_sys* s, const int st[ST_COUNT])
{
    if (st[ST_NEED_CAND] > s->cand_cap) s->cand_cap = (int)(st[ST_NEED_CAND] * 1.2) + 16;
    if (st[ST_NEED_ENT] > s->ent_cap) s->ent_cap = (int)(st[ST_NEED_ENT] * 1.2) + 1024;
    if (st[ST_NEED_ITEM] > s->item_cap) s->item_cap = (int)(st[ST_NEED_ITEM] * 1.2) + 64;
    if (st[ST_NEED_CAND] > 0) {
        // entries follow the candidates
        const double ent = (double)s->max_groups * s->cand_cap * 0.75 + 1024;
        s->ent_cap = std::max(s->ent_cap, (int)std::min(ent, 2.0e9));
        s->item_cap = std::max(s->item_cap,
                               (int)std::min(item_bound(s->M, s->jtile, s->ent_cap, s->max_groups) + 16, 2.0e9));
    }
    int* pp;
    int* dd;
    SysDev* ds;
    s->needed_bytes = layout(&s->p, shape_of_sys(s), nullptr, nullptr, &pp, &dd, &ds);
    s->list_valid = false;
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "pair-list capacity exceeded (candidates %d, entries %d, items %d); arena of %zu bytes needed",
                  st[ST_NEED_CAND], st[ST_NEED_ENT], st[ST_NEED_ITEM], s->needed_bytes);
    return fail(s->ctx, NB_ERR_CAPACITY, buf);
}

// a list built inside an MD run has only the conservative cluster masks: compute
// the exact FP64 atom-pair masks of its candidates from the stored build
// positions (for export and statistics; the force list is left as it is, so
// asking for them does not change a run)
nb_status nbh::make_exact(nb_sys* s)
{
    if (s->list_exact) return NB_OK;
    HIPCHK(s->ctx, launch_refine(s->d_desc, 1, s->bounds, s->ctx->stream));
    s->list_exact = true;
    return NB_OK;
}

// the candidates of every group with their exact masks (after make_exact)
nb_status nbh::read_candidates(nb_sys* s, int ng, std::vector<int>& cc, std::vector<int2>& cand,
                               std::vector<unsigned long long>& msk)
{
    hipStream_t st = s->ctx->stream;
    const size_t cap = (size_t)s->cand_cap, words = (size_t)s->h.mask_words;
    cc.assign(ng > 0 ? ng : 1, 0);
    cand.assign(ng > 0 ? (size_t)ng * cap : 1, make_int2(0, 0));
    msk.assign(ng > 0 ? (size_t)ng * cap * words : 1, 0ull);
    if (ng > 0) {
        HIPCHK(s->ctx, hipMemcpyAsync(cc.data(), s->h.cand_count, sizeof(int) * ng, hipMemcpyDeviceToHost, st));
        HIPCHK(s->ctx, hipMemcpyAsync(cand.data(), s->h.cand, sizeof(int2) * ng * cap, hipMemcpyDeviceToHost, st));
        HIPCHK(s->ctx, hipMemcpyAsync(msk.data(), s->h.cand_mask, sizeof(unsigned long long) * ng * cap * words,
                                      hipMemcpyDeviceToHost, st));
    }
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    for (int g = 0; g < ng; ++g) cc[g] = std::min(cc[g], (int)cap);
    return NB_OK;
}

// The list-build sequence of one system, enqueued.  The search prunes its
// candidates at the atom level in FP32 in the force kernel's frame (the paper's
// GPU-side prune, done at the build so every force of the list lifetime sees
// the same list).  exact: the FP64 atom-pair prune then decides the list
// (explicit builds, export-ready masks).  The build starts with the list-buffer
// guard (displacement since the previous build; first: positions only recorded).
nb_status nbh::enqueue_build(nb_sys* s, bool exact, int status_clear, bool first, bool cleared)
{
    Range range("nb list build");
    hipStream_t st = s->ctx->stream;
    HIPCHK(s->ctx, launch_build(s->d_desc, 1, s->bounds, nullptr, st, exact, status_clear, s->d_prefix, first,
                                cleared));
    s->list_exact = exact;
    return NB_OK;
}

nb_status nbh::prune_guard(nb_sys* s, bool check)
{
    if (!s->h.prune_on) return NB_OK;
    HIPCHK(s->ctx, launch_prune_guard_k(s->d_desc, s->p.n_atoms, check ? 1 : 0, s->pg_cur, s->pg_pending ? 1 : 0,
                                        s->ctx->stream));
    s->pg_pending = check;
    if (check) s->pg_cur ^= 1;
    return NB_OK;
}

nb_status nbh::do_build(nb_sys* s, bool exact)
{
    nb_status rb = enqueue_build(s, exact, 1, !s->list_valid);
    if (rb) return rb;
    int stv[ST_COUNT];
    nb_status r = read_status(s, stv);
    if (r) return r;
    if (stv[ST_OVERFLOW]) return capacity_error(s, stv);
    s->list_valid = true;
    // a list built afresh starts the dynamic-prune schedule and its guard here
    s->list_step = s->step;
    return prune_guard(s, false);
}

nb_status nbh::eval_forces(nb_sys* s, bool ener, int trace_row, bool with_ke, double step_value, int open_next,
                           double dt, bool clear_status)
{
    Range range("nb forces");
    hipStream_t st = s->ctx->stream;
    HIPCHK(s->ctx, launch_stage(s->d_desc, 1, s->bounds, st, nullptr, clear_status));
    if (s->pme_on) {
        // the pair kernel beside the reciprocal part; the gather adds both
        nb_status r = pair_beside_pme(s, s->h.x, ener, false);
        if (r) return r;
    } else {
        HIPCHK(s->ctx, launch_force(s->d_desc, 1, s->d_prefix, s->M, s->p.coulomb, s->p.lj, ener,
                                    0, s->item_cap, st));
    }
    if (open_next > 0)
        HIPCHK(s->ctx, launch_gather_kick(s->d_desc, 1, s->bounds, dt, false, st, open_next, true));
    else
        HIPCHK(s->ctx, launch_finalize(s->d_desc, 1, s->bounds, false, st));
    if (ener) HIPCHK(s->ctx, launch_energy_reduce(s->d_desc, 1, trace_row, with_ke, step_value, st));
    return NB_OK;
}

nb_status nbh::pme_fork(nb_sys* s, const double* x, bool ener)
{
    Range range("nb pme");
    HIPCHK(s->ctx, hipEventRecord(s->side_in, s->ctx->stream));
    HIPCHK(s->ctx, hipStreamWaitEvent(s->side_stream, s->side_in, 0));
    HIPCHK(s->ctx, launch_pme(s->pme, x, ener, s->side_stream));
    HIPCHK(s->ctx, hipEventRecord(s->side_out, s->side_stream));
    return NB_OK;
}

nb_status nbh::pme_join(nb_sys* s)
{
    HIPCHK(s->ctx, hipStreamWaitEvent(s->ctx->stream, s->side_out, 0));
    return NB_OK;
}

int nbh::pair_grid_beside_pme(const nb_ctx* c)
{
    return 3 * c->n_cu;
}

nb_status nbh::pair_beside_pme(nb_sys* s, const double* x, bool ener, bool prune)
{
    hipStream_t st = s->ctx->stream;
    HIPCHK(s->ctx, hipEventRecord(s->side_in, st));
    HIPCHK(s->ctx, hipStreamWaitEvent(s->side_stream, s->side_in, 0));
    mark_begin(s, 0, s->side_stream);
    HIPCHK(s->ctx, launch_force(s->d_desc, 1, s->d_prefix, s->M, s->p.coulomb, s->p.lj, ener,
                                pair_grid_beside_pme(s->ctx), s->item_cap, s->side_stream, prune));
    mark_end(s, s->side_stream);
    HIPCHK(s->ctx, hipEventRecord(s->side_out, s->side_stream));
    {
        Range range("nb pme");
        HIPCHK(s->ctx, launch_pme(s->pme, x, ener, st));
    }
    HIPCHK(s->ctx, hipStreamWaitEvent(st, s->side_out, 0));
    return NB_OK;
}

nb_status nbh::check_after(nb_sys* s)
{
    int stv[ST_COUNT];
    nb_status r = read_status(s, stv);
    if (r) return r;
    return status_result(s, stv);
}

nb_status nbh::status_result(nb_sys* s, const int stv[ST_COUNT])
{
    if (stv[ST_BADPOS]) return fail(s->ctx, NB_ERR_NONFINITE, "a position was not finite");
    if (stv[ST_SATURATE])
        return fail(s->ctx, NB_ERR_NONFINITE,
                    "a force partial exceeded the fixed-point range (or was not finite); lower force_fixed_bits");
    if (stv[ST_OVERFLOW]) return capacity_error(s, stv);
    return NB_OK;
}


// ===========================================================================
extern "C" {

const char* nb_strerror(nb_status s)
{
    switch (s) {
    case NB_OK: return "ok";
    case NB_ERR_ARG: return "invalid argument";
    case NB_ERR_BOX: return "box too small for r_list (r_list must be < L/2) or invalid box";
    case NB_ERR_CAPACITY: return "capacity exceeded";
    case NB_ERR_DEVICE: return "HIP device error";
    case NB_ERR_NONFINITE: return "non-finite or out-of-range force";
    case NB_ERR_BUFFER: return "pair-list buffer violated";
    case NB_ERR_STATE: return "call out of order";
    default: return "unknown status";
    }
}

const char* nb_last_error(const nb_ctx* ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_last_error.c_str();
}

nb_status nb_ctx_create(int device, void* hip_stream, nb_ctx** out)
{
    if (!out) return fail(nullptr, NB_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(nullptr, NB_ERR_DEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(nullptr, NB_ERR_ARG, "device index out of range");
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, NB_ERR_DEVICE, hipGetErrorString(e));
    scratch_setup(device);  // (a failure is reported by the call that needs it)
    int n_cu = 0;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess || n_cu <= 0) return fail(nullptr, NB_ERR_DEVICE, "cannot read the compute unit count");
    nb_ctx* c = new nb_ctx;
    c->device = device;
    c->n_cu = n_cu;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return NB_OK;
}

nb_status nb_ctx_destroy(nb_ctx* ctx)
{
    if (!ctx) return fail(nullptr, NB_ERR_ARG, "ctx is NULL");
    delete ctx;
    return NB_OK;
}

nb_status nb_arena_bytes(const nb_params* p, size_t* bytes)
{
    std::string why;
    nb_status r = validate(p, &why);
    if (r) return fail(nullptr, r, why);
    if (!bytes) return fail(nullptr, NB_ERR_ARG, "bytes is NULL");
    int* pp;
    int* dd;
    SysDev* ds;
    *bytes = layout(p, shape_of(p), nullptr, nullptr, &pp, &dd, &ds);
    return NB_OK;
}

nb_status nb_sys_create(nb_ctx* ctx, const nb_params* p, void* dev_arena, size_t arena_bytes, nb_sys** out)
{
    if (!ctx || !out) return fail(ctx, NB_ERR_ARG, "ctx/out is NULL");
    *out = nullptr;
    std::string why;
    nb_status r = validate(p, &why);
    if (r) return fail(ctx, r, why);
    if (!dev_arena) return fail(ctx, NB_ERR_ARG, "arena is NULL");
    nb_sys* s = new nb_sys;
    init_sys(s, ctx, p, dev_arena, arena_bytes);
    r = place(s);
    if (r) {
        delete s;
        return r;
    }
    if (s->pme_on) {
        if (hipStreamCreateWithFlags(&s->side_stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->side_in, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s->side_out, hipEventDisableTiming) != hipSuccess) {
            release_side_stream(s);
            delete s;
            return fail(ctx, NB_ERR_DEVICE, "cannot create the PME stream and its events");
        }
    }
    *out = s;
    return NB_OK;
}

nb_status nb_sys_destroy(nb_sys* s)
{
    if (!s) return fail(nullptr, NB_ERR_ARG, "sys is NULL");
    if (s->ens) nb_ens_remove(s->ens, s);
    for (hipEvent_t e : s->ev_pool) hipEventDestroy(e);
    release_side_stream(s);
    if (s->mailbox) hipHostFree(s->mailbox);
    delete s;
    return NB_OK;
}

nb_status nb_sys_needed_bytes(const nb_sys* s, size_t* bytes)
{
    if (!s || !bytes) return fail(nullptr, NB_ERR_ARG, "NULL argument");
    *bytes = std::max(s->needed_bytes, s->arena_bytes);
    return NB_OK;
}

nb_status nb_sys_set_arena(nb_sys* s, void* dev_arena, size_t arena_bytes)
{
    if (!s || !dev_arena) return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    HIPCHK(s->ctx, hipStreamSynchronize(s->ctx->stream));
    void* old = s->arena;
    size_t oldb = s->arena_bytes;
    s->arena = dev_arena;
    s->arena_bytes = arena_bytes;
    nb_status r = place(s);
    if (r) {
        s->arena = old;
        s->arena_bytes = oldb;
        nb_status r2 = place(s);
        (void)r2;
        return r;
    }
    return NB_OK;
}

nb_status nb_sys_set_particles(nb_sys* s, const double* q, const double* sigma, const double* epsilon,
                               const double* mass)
{
    if (!s) return fail(nullptr, NB_ERR_ARG, "sys is NULL");
    if (!q) return fail(s->ctx, NB_ERR_ARG, "q is NULL");
    if (s->p.lj == NB_LJ_LB && (!sigma || !epsilon)) return fail(s->ctx, NB_ERR_ARG, "LB needs sigma and epsilon");
    const size_t N = (size_t)s->p.n_atoms;
    for (size_t i = 0; i < N; ++i) {
        if (!std::isfinite(q[i])) return fail(s->ctx, NB_ERR_ARG, "non-finite charge");
        if (s->p.lj == NB_LJ_LB && (!(sigma[i] >= 0.0) || !(epsilon[i] >= 0.0)))
            return fail(s->ctx, NB_ERR_ARG, "sigma/epsilon must be >= 0");
        if (mass && !(mass[i] > 0.0)) return fail(s->ctx, NB_ERR_ARG, "masses must be > 0");
    }
    s->q.assign(q, q + N);
    if (sigma && epsilon) {
        s->sig.assign(sigma, sigma + N);
        s->eps.assign(epsilon, epsilon + N);
    } else {
        s->sig.assign(N, 0.0);
        s->eps.assign(N, 0.0);
    }
    s->has_particles = true;
    if (mass) {
        s->mass.assign(mass, mass + N);
        s->has_mass = true;
    }
    hipStream_t st = s->ctx->stream;
    HIPCHK(s->ctx, hipMemcpyAsync((void*)s->h.q, s->q.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHK(s->ctx, hipMemcpyAsync((void*)s->h.sig, s->sig.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
    HIPCHK(s->ctx, hipMemcpyAsync((void*)s->h.eps, s->eps.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
    if (mass)
        HIPCHK(s->ctx, hipMemcpyAsync((void*)s->h.mass, s->mass.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
    // charge sums of the PME self and background terms (and its tables)
    if (s->pme_on) HIPCHK(s->ctx, launch_pme_setup(s->pme, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    return NB_OK;
}

nb_status nb_build_pairlist(nb_sys* s, const double* x_dev)
{
    if (!s || !x_dev) return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    s->h.x = x_dev;
    nb_status r = upload_desc(s);
    if (r) return r;
    s->list_valid = false;  // an explicit build starts a new displacement record
    return do_build(s);
}

nb_status nb_pairlist_export(nb_sys* s, int32_t* pairs_host, int64_t cap, int64_t* n_pairs)
{
    if (!s || !n_pairs || cap < 0 || (cap > 0 && !pairs_host))
        return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "bad export arguments");
    if (!s->list_valid) return fail(s->ctx, NB_ERR_STATE, "no valid pair list");
    nb_status rr = make_exact(s);
    if (rr) return rr;
    hipStream_t st = s->ctx->stream;
    int ng = 0;
    HIPCHK(s->ctx, hipMemcpyAsync(&ng, s->h.n_groups, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    const int G = s->G, M = s->M, MM = M * M, words = s->h.mask_words;
    std::vector<int> slot_atom((size_t)ng * G * M + 1);
    HIPCHK(s->ctx, hipMemcpyAsync(slot_atom.data(), s->h.slot_atom, sizeof(int) * ((size_t)ng * G * M),
                                  hipMemcpyDeviceToHost, st));
    std::vector<int> cc;
    std::vector<int2> cand;
    std::vector<unsigned long long> msk;
    rr = read_candidates(s, ng, cc, cand, msk);
    if (rr) return rr;
    const size_t ccap = (size_t)s->cand_cap;
    std::vector<unsigned long long> keys;
    for (int gi = 0; gi < ng; ++gi)
        for (int c = 0; c < cc[gi]; ++c) {
            const size_t ce = (size_t)gi * ccap + c;
            const int cj = cand[ce].x;
            for (int pi = 0; pi < G * MM; ++pi) {
                if (!((msk[ce * words + pi / 64] >> (pi % 64)) & 1ull)) continue;
                const int k = pi / MM, a = (pi / M) % M, b = pi % M;
                const int ia = slot_atom[(size_t)(gi * G + k) * M + a];
                const int jb = slot_atom[(size_t)cj * M + b];
                const unsigned lo = (unsigned)std::min(ia, jb), hi = (unsigned)std::max(ia, jb);
                keys.push_back(((unsigned long long)lo << 32) | hi);
            }
        }
    std::sort(keys.begin(), keys.end());
    *n_pairs = (int64_t)keys.size();
    const int64_t nw = std::min<int64_t>(cap, (int64_t)keys.size());
    for (int64_t i = 0; i < nw; ++i) {
        pairs_host[2 * i] = (int32_t)(keys[i] >> 32);
        pairs_host[2 * i + 1] = (int32_t)(keys[i] & 0xffffffffull);
    }
    return NB_OK;
}

nb_status nb_pairlist_stats(nb_sys* s, int64_t out[10])
{
    if (!s || !out) return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    if (!s->list_valid) return fail(s->ctx, NB_ERR_STATE, "no valid pair list");
    nb_status rr = make_exact(s);
    if (rr) return rr;
    hipStream_t st = s->ctx->stream;
    int ng = 0, nit = 0;
    HIPCHK(s->ctx, hipMemcpyAsync(&ng, s->h.n_groups, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipMemcpyAsync(&nit, s->h.n_items, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    const int G = s->G, M = s->M, words = s->h.mask_words;
    std::vector<int> es(ng + 1), nreal((size_t)ng * G), grc(ng > 0 ? ng : 1);
    HIPCHK(s->ctx, hipMemcpyAsync(es.data(), s->h.ent_start, sizeof(int) * (ng + 1), hipMemcpyDeviceToHost, st));
    if (ng > 0)
        HIPCHK(s->ctx, hipMemcpyAsync(grc.data(), s->h.grp_rc, sizeof(int) * ng, hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipMemcpyAsync(nreal.data(), s->h.cl_nreal, sizeof(int) * nreal.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    const int ne = es[ng];
    std::vector<int2> ent(ne > 0 ? ne : 1);
    if (ne > 0) {
        HIPCHK(s->ctx, hipMemcpyAsync(ent.data(), s->h.ent, sizeof(int2) * ne, hipMemcpyDeviceToHost, st));
        HIPCHK(s->ctx, hipStreamSynchronize(st));
    }
    // the exact atom pairs come from the candidates' exact masks; entries and
    // cluster pairs are those of the list the force kernel runs on
    std::vector<int> cc;
    std::vector<int2> cand;
    std::vector<unsigned long long> msk;
    rr = read_candidates(s, ng, cc, cand, msk);
    if (rr) return rr;
    int64_t ncl = 0, cpairs = 0, apairs = 0;
    for (int v : nreal) ncl += v > 0;
    for (int e = 0; e < ne; ++e) cpairs += __builtin_popcount((unsigned)(ent[e].y >> kMetaOuter) & 255u);
    for (int gi = 0; gi < ng; ++gi)
        for (int c = 0; c < cc[gi]; ++c)
            for (int w = 0; w < words; ++w)
                apairs += __builtin_popcountll(msk[((size_t)gi * s->cand_cap + c) * words + w]);
    out[0] = ncl;
    out[1] = ne;
    out[2] = cpairs;
    out[3] = apairs;
    out[4] = cpairs * M * M;
    out[5] = nit;
    out[6] = ng;
    out[7] = (int64_t)ng * G * M;
    int64_t nrc = 0;
    for (int g = 0; g < ng; ++g) nrc += grc[g];
    out[8] = nrc;
    int64_t ncand = 0;
    for (int g = 0; g < ng; ++g) ncand += cc[g];
    out[9] = ncand;
    return NB_OK;
}

nb_status nb_compute_forces(nb_sys* s, const double* x_dev, float* f_dev, double* ener_host, double* virial_host)
{
    if (!s || !x_dev || !f_dev) return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    if (!s->has_particles) return fail(s->ctx, NB_ERR_STATE, "particles not set");
    s->h.x = x_dev;
    s->h.f = f_dev;
    nb_status r = upload_desc(s);
    if (r) return r;
    if (!s->list_valid) {
        r = do_build(s);
        if (r) return r;
    }
    const bool ener = ener_host || virial_host;
    // (the staging kernel clears the status words first)
    r = eval_forces(s, ener, -1, false, 0.0, 0, 0.0, true);
    if (r) return r;
    if (ener) {
        double eo[16];
        HIPCHK(s->ctx, hipMemcpyAsync(eo, s->h.eout, sizeof(eo), hipMemcpyDeviceToHost, s->ctx->stream));
        r = check_after(s);
        if (r) return r;
        if (ener_host) {
            ener_host[0] = eo[0];
            ener_host[1] = eo[1];
        }
        if (virial_host) {
            // eout[2..7] = xx, yy, zz, xy, xz, yz
            virial_host[0] = eo[2];
            virial_host[4] = eo[3];
            virial_host[8] = eo[4];
            virial_host[1] = virial_host[3] = eo[5];
            virial_host[2] = virial_host[6] = eo[6];
            virial_host[5] = virial_host[7] = eo[7];
        }
    }
    return NB_OK;
}

nb_status nb_pme_forces(nb_sys* s, const double* x_dev, float* f_dev, double* energy_host, double* virial_host)
{
    if (!s || !x_dev || !f_dev) return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    if (!s->pme_on) return fail(s->ctx, NB_ERR_STATE, "the system has no PME (pme_grid not set)");
    if (!s->has_particles) return fail(s->ctx, NB_ERR_STATE, "particles not set");
    hipStream_t st = s->ctx->stream;
    PmeDev P = s->pme;
    P.frec = f_dev;
    const bool ener = energy_host || virial_host;
    HIPCHK(s->ctx, launch_pme(P, x_dev, ener, st));
    if (!ener) return NB_OK;
    double eo[8];
    HIPCHK(s->ctx, hipMemcpyAsync(eo, P.eout, sizeof(eo), hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    if (energy_host) *energy_host = eo[0];
    if (virial_host) {
        // eo[1..6] = xx, yy, zz, xy, xz, yz
        virial_host[0] = eo[1];
        virial_host[4] = eo[2];
        virial_host[8] = eo[3];
        virial_host[1] = virial_host[3] = eo[4];
        virial_host[2] = virial_host[6] = eo[5];
        virial_host[5] = virial_host[7] = eo[6];
    }
    return NB_OK;
}

nb_status md_step(nb_sys* s, double* x_dev, double* v_dev, float* f_dev, double dt_ps, int32_t n_steps,
                  int32_t nstlist, int32_t nstenergy, double* trace_host, int32_t trace_cap, int32_t* n_rows)
{
    if (!s || !x_dev || !v_dev || !f_dev) return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    if (!(dt_ps > 0.0) || n_steps < 0 || nstlist < 1 || nstenergy < 0 || trace_cap < 0 ||
        (trace_cap > 0 && !trace_host))
        return fail(s->ctx, NB_ERR_ARG, "bad md_step arguments");
    if (!s->has_particles || !s->has_mass) return fail(s->ctx, NB_ERR_STATE, "particles/masses not set");
    Range range("nb md_step");
    hipStream_t st = s->ctx->stream;
    s->h.x = x_dev;
    s->h.v = v_dev;
    s->h.f = f_dev;
    if (!s->mailbox &&
        hipHostMalloc(&s->mailbox, kStatusBytes + sizeof(double) * 5 * kTraceCap, hipHostMallocDefault) !=
            hipSuccess) {
        s->mailbox = nullptr;
        return fail(s->ctx, NB_ERR_DEVICE, "cannot allocate the pinned trace buffer");
    }
    nb_status r = upload_desc(s);
    if (r) return r;
    if (!s->list_valid) {
        // built as the rebuilds inside the run are (the search's FP32 prune
        // decides the list), so a run resumed at a rebuild step, or the same
        // system in an ensemble, takes the same lists
        r = do_build(s, false);
        if (r) return r;
    }
    // F(x0) with the current list (bitwise the same as the previous call's last
    // force); its gather also applies the first step's half-kick and drift.
    // The staging kernel clears the status words first
    const int next0 = n_steps > 0 ? (((s->step + 1) % nstlist == 0) ? 1 : 2) : 0;
    r = eval_forces(s, false, -1, false, 0.0, next0, dt_ps, true);
    if (r) return r;
    int rows = 0, pending = 0, ring0 = 0;
    // the pending rows of the device ring (and with stv the status words) in
    // one round of copies to the pinned mailbox and one synchronisation.  The
    // mailbox mirrors the device layout (status words, then the ring), so the
    // status words with the rows from the ring's start are one copy
    int* mb_status = (int*)s->mailbox;
    double* mb_rows = (double*)((char*)s->mailbox + kStatusBytes);
    auto flush = [&](int* stv) -> nb_status {
        if (pending == 0 && !stv) return NB_OK;
        if (stv && ring0 == 0) {
            HIPCHK(s->ctx, hipMemcpyAsync(s->mailbox, s->h.status, kStatusBytes + sizeof(double) * 5 * pending,
                                          hipMemcpyDeviceToHost, st));
        } else {
            for (int k = 0; k < pending;) {  // at most two contiguous runs of the ring
                const int row = (ring0 + k) % kTraceCap;
                const int run = std::min(pending - k, kTraceCap - row);
                HIPCHK(s->ctx, hipMemcpyAsync(mb_rows + (size_t)row * 5, s->h.trace + (size_t)row * 5,
                                              sizeof(double) * 5 * run, hipMemcpyDeviceToHost, st));
                k += run;
            }
            if (stv)
                HIPCHK(s->ctx,
                       hipMemcpyAsync(mb_status, s->h.status, sizeof(int) * ST_COUNT, hipMemcpyDeviceToHost, st));
        }
        HIPCHK(s->ctx, hipStreamSynchronize(st));
        for (int k = 0; k < pending; ++k) {
            const int row = (ring0 + k) % kTraceCap;
            if (rows < trace_cap)
                std::memcpy(trace_host + (size_t)rows * 5, mb_rows + (size_t)row * 5, sizeof(double) * 5);
            ++rows;
        }
        if (stv) std::memcpy(stv, mb_status, sizeof(int) * ST_COUNT);
        ring0 = (ring0 + pending) % kTraceCap;
        pending = 0;
        return NB_OK;
    };
    mark_begin(s, 2);
    // the gather of step k also applies step k+1's half-kick and drift (and the
    // staging when no rebuild is due): moved = that part of this step is done
    bool moved = next0 > 0;
    // an energy row left to the next step's pair kernel (its extra block)
    int red_row = -1;
    double red_step = 0.0;
    for (int32_t k = 0; k < n_steps; ++k) {
        const bool rebuild = ((s->step + 1) % nstlist == 0);
        s->step += 1;
        if (rebuild) {
            // x must move before the list is rebuilt at the new positions; the
            // full-step x, v are kept (by the previous gather, or copied here)
            // so a rebuild that runs out of capacity can hand them back
            if (!moved) {
                if (s->check_builds) {
                    const size_t nb3 = sizeof(double) * 3 * (size_t)s->p.n_atoms;
                    HIPCHK(s->ctx, hipMemcpyAsync(s->h.x_bak, x_dev, nb3, hipMemcpyDeviceToDevice, st));
                    HIPCHK(s->ctx, hipMemcpyAsync(s->h.v_bak, v_dev, nb3, hipMemcpyDeviceToDevice, st));
                }
                HIPCHK(s->ctx, launch_kick_drift(s->d_desc, 1, s->bounds, dt_ps, st));
            }
            // reciprocal space of the new positions beside the rebuild
            if (s->pme_on) {
                r = pme_fork(s, x_dev, ener_step(s, nstenergy));
                if (r) return r;
            }
            // the dynamic-prune interval that ends at this rebuild
            r = prune_guard(s, true);
            if (r) return r;
            mark_begin(s, 1);
            // (after a gather that ended the step, its clears are done)
            r = enqueue_build(s, false, 2, false, moved);
            if (r) return r;
            mark_end(s);
            s->list_step = s->step;
            if (s->check_builds) {
                int stv[ST_COUNT];
                r = read_status(s, stv);
                if (r) return r;
                if (stv[ST_OVERFLOW]) {
                    // stop at the last full step: x, v and the step count go
                    // back to it, the energy rows so far are returned, and the
                    // caller can grow the arena and run the remaining steps
                    // (after the PME pass that still reads x)
                    if (s->pme_on) {
                        r = pme_join(s);
                        if (r) return r;
                    }
                    const size_t nb3 = sizeof(double) * 3 * (size_t)s->p.n_atoms;
                    HIPCHK(s->ctx, hipMemcpyAsync(x_dev, s->h.x_bak, nb3, hipMemcpyDeviceToDevice, st));
                    HIPCHK(s->ctx, hipMemcpyAsync(v_dev, s->h.v_bak, nb3, hipMemcpyDeviceToDevice, st));
                    s->step -= 1;
                    s->list_valid = false;
                    r = flush(nullptr);
                    if (r) return r;
                    if (n_rows) *n_rows = rows;
                    for (auto& m : s->ev_marks)
                        if (m.second == 2) hipEventRecord(s->ev_pool[m.first + 1], st);
                    HIPCHK(s->ctx, hipStreamSynchronize(st));
                    collect_marks(s);
                    return capacity_error(s, stv);
                }
            }
            // (the build staged the new slots at these positions)
        } else {
            if (!moved) HIPCHK(s->ctx, launch_kick_drift_stage(s->d_desc, 1, s->bounds, dt_ps, st));
        }
        const bool ener = ener_step(s, nstenergy);
        // dynamic pruning: every nstprune-th step of the list's life (its first
        // included) the force pass prunes the list for the steps that follow
        const bool prune = s->h.prune_on && ((s->step - s->list_step) % s->p.nstprune == 0);
        if (prune && !rebuild) {
            r = prune_guard(s, true);
            if (r) return r;
        }
        if (s->pme_on && !rebuild) {
            // the pair kernel beside this step's PME (joined before the gather)
            r = pair_beside_pme(s, x_dev, ener, prune);
            if (r) return r;
        } else {
            // (a rebuild step's PME, forked before the build, has run beside the
            // build: the pair kernel takes the whole GPU, and PME joins before
            // the gather)
            mark_begin(s, 0);
            HIPCHK(s->ctx, launch_force(s->d_desc, 1, s->d_prefix, s->M, s->p.coulomb, s->p.lj, ener,
                                        0, s->item_cap, st, prune, red_row, red_step));
            red_row = -1;
            mark_end(s);
            if (s->pme_on) {
                r = pme_join(s);
                if (r) return r;
            }
        }
        // the last step of the call leaves x, v at the full step
        const int next = (k + 1 < n_steps) ? (((s->step + 1) % nstlist == 0) ? 1 : 2) : 0;
        HIPCHK(s->ctx, launch_gather_kick(s->d_desc, 1, s->bounds, dt_ps, ener, st, next));
        moved = next > 0;
        if (ener) {
            // the energy row: by an extra block of the next step's pair kernel
            // when that step exists and builds no list, evaluates no energies,
            // prunes nothing and runs no PME (its pair kernel then reads and
            // writes nothing the row depends on), and no flush of the rows comes
            // first; else by the reduction kernel now
            const int row = (ring0 + pending) % kTraceCap;
            const int64_t s1 = s->step + 1;
            const bool next_ener = nstenergy > 0 && s1 % nstenergy == 0;
            const bool next_prune = s->h.prune_on && ((s1 - s->list_step) % s->p.nstprune == 0);
            if (next == 2 && !s->pme_on && !next_ener && !next_prune && pending + 1 < kTraceCap) {
                red_row = row;
                red_step = (double)s->step;
            } else {
                HIPCHK(s->ctx, launch_energy_reduce(s->d_desc, 1, row, true, (double)s->step, st));
            }
            ++pending;
            if (pending == kTraceCap) {
                r = flush(nullptr);
                if (r) return r;
            }
        }
    }
    if (!s->ev_marks.empty()) {
        // close the whole-call mark (index of the first mark of this call)
        for (auto& m : s->ev_marks)
            if (m.second == 2) hipEventRecord(s->ev_pool[m.first + 1], st);
    }
    int stv[ST_COUNT];
    r = flush(stv);
    if (r) return r;
    if (n_rows) *n_rows = rows;
    r = status_result(s, stv);
    collect_marks(s);
    if (r == NB_ERR_CAPACITY && !s->check_builds)
        // the overflow was found after the fact: the steps after that rebuild
        // ran without their list (the force kernel and the gather skip a list
        // that did not fit), so x and v are not a valid trajectory
        return fail(s->ctx, NB_ERR_CAPACITY,
                    s->ctx->err + "; build checks were off, so the steps after the overflowing rebuild ran "
                                  "without a list: x and v are not a valid trajectory");
    return r;
}

nb_status nb_minimize(nb_sys* s, double* x_dev, float* f_dev, int32_t n_iter, double f_tol, double max_disp,
                      int32_t nstlist, double* f_max_host, int32_t* iters_host)
{
    if (!s || !x_dev || !f_dev || n_iter < 0 || !(max_disp > 0.0) || nstlist < 1)
        return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "bad nb_minimize arguments");
    if (!s->has_particles) return fail(s->ctx, NB_ERR_STATE, "particles not set");
    hipStream_t st = s->ctx->stream;
    // unrelaxed inputs carry pair forces far beyond MD's: relax with a coarse
    // fixed-point scale (2^-12 kJ/mol/nm, range 2^38) and restore it afterwards
    struct ScaleGuard {
        nb_sys* s;
        double sc, inv;
        float lim;
        ~ScaleGuard()
        {
            s->h.fx_scale = sc;
            s->h.fx_inv = inv;
            s->h.fx_lim = lim;
            nbh::upload_desc(s);
        }
    } guard{s, s->h.fx_scale, s->h.fx_inv, s->h.fx_lim};
    const int bits = std::min(s->fx_bits, 12);
    s->h.fx_scale = std::ldexp(1.0, bits);
    s->h.fx_inv = std::ldexp(1.0, -bits);
    s->h.fx_lim = (float)std::ldexp(1.0, 50 - bits);
    s->h.x = x_dev;
    s->h.f = f_dev;
    nb_status r = upload_desc(s);
    if (r) return r;
    r = do_build(s);
    if (r) return r;
    HIPCHK(s->ctx, launch_clear_status(s->d_desc, 1, st));
    int done = 0, it = 0;
    HIPCHK(s->ctx, hipMemsetAsync(s->d_done, 0, sizeof(int), st));
    for (it = 0; it < n_iter; ++it) {
        if (it > 0 && it % nstlist == 0) {
            r = do_build(s);
            if (r) return r;
        }
        r = eval_forces(s, false, -1, false, 0.0);
        if (r) return r;
        HIPCHK(s->ctx, launch_fmax(s->d_desc, s->bounds, st));
        HIPCHK(s->ctx, launch_minimize_step(s->d_desc, s->bounds, x_dev, max_disp, f_tol, s->d_done, st));
        HIPCHK(s->ctx, hipMemcpyAsync(&done, s->d_done, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(s->ctx, hipStreamSynchronize(st));
        if (done) break;
    }
    // final forces at the final positions
    r = do_build(s);
    if (r) return r;
    r = eval_forces(s, false, -1, false, 0.0);
    if (r) return r;
    HIPCHK(s->ctx, launch_fmax(s->d_desc, s->bounds, st));
    std::vector<double> parts(kKeBlocks);
    HIPCHK(s->ctx, hipMemcpyAsync(parts.data(), s->h.fmax_part, sizeof(double) * kKeBlocks, hipMemcpyDeviceToHost, st));
    r = check_after(s);
    if (r) return r;
    double m2 = 0.0;
    for (double v : parts) m2 = std::max(m2, v);
    if (f_max_host) *f_max_host = std::sqrt(m2);
    if (iters_host) *iters_host = it;
    s->list_valid = false;
    return NB_OK;
}

nb_status nb_sys_get_step(const nb_sys* s, int64_t* step)
{
    if (!s || !step) return fail(nullptr, NB_ERR_ARG, "NULL argument");
    *step = s->step;
    return NB_OK;
}

nb_status nb_sys_set_step(nb_sys* s, int64_t step)
{
    if (!s || step < 0) return fail(nullptr, NB_ERR_ARG, "bad argument");
    s->step = step;
    return NB_OK;
}

nb_status nb_state_bytes(const nb_sys* s, size_t* bytes)
{
    if (!s || !bytes) return fail(nullptr, NB_ERR_ARG, "NULL argument");
    *bytes = 16 + sizeof(double) * 6 * (size_t)s->p.n_atoms;
    return NB_OK;
}

nb_status nb_state_export(nb_sys* s, const double* x_dev, const double* v_dev, void* host, size_t bytes)
{
    if (!s || !x_dev || !v_dev || !host) return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    const size_t N = (size_t)s->p.n_atoms;
    if (bytes < 16 + sizeof(double) * 6 * N) return fail(s->ctx, NB_ERR_ARG, "state buffer too small");
    char* h = (char*)host;
    int64_t hdr[2] = {s->step, (int64_t)N};
    std::memcpy(h, hdr, 16);
    hipStream_t st = s->ctx->stream;
    HIPCHK(s->ctx, hipMemcpyAsync(h + 16, x_dev, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipMemcpyAsync(h + 16 + sizeof(double) * 3 * N, v_dev, sizeof(double) * 3 * N,
                                  hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    return NB_OK;
}

nb_status nb_state_import(nb_sys* s, double* x_dev, double* v_dev, const void* host, size_t bytes)
{
    if (!s || !x_dev || !v_dev || !host) return fail(s ? s->ctx : nullptr, NB_ERR_ARG, "NULL argument");
    const size_t N = (size_t)s->p.n_atoms;
    if (bytes < 16 + sizeof(double) * 6 * N) return fail(s->ctx, NB_ERR_ARG, "state buffer too small");
    const char* h = (const char*)host;
    int64_t hdr[2];
    std::memcpy(hdr, h, 16);
    if (hdr[1] != (int64_t)N || hdr[0] < 0) return fail(s->ctx, NB_ERR_ARG, "state does not match this system");
    hipStream_t st = s->ctx->stream;
    HIPCHK(s->ctx, hipMemcpyAsync(x_dev, h + 16, sizeof(double) * 3 * N, hipMemcpyHostToDevice, st));
    HIPCHK(s->ctx, hipMemcpyAsync(v_dev, h + 16 + sizeof(double) * 3 * N, sizeof(double) * 3 * N,
                                  hipMemcpyHostToDevice, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    s->step = hdr[0];
    s->list_valid = false;
    return NB_OK;
}

nb_status nb_sys_set_timing(nb_sys* s, int32_t on)
{
    if (!s) return fail(nullptr, NB_ERR_ARG, "NULL argument");
    if (on < 0) return fail(s->ctx, NB_ERR_ARG, "timing stride must be >= 0");
    s->timing = on != 0;
    s->timing_every = on > 0 ? on : 1;
    s->mark_seq[0] = s->mark_seq[1] = 0;
    s->mark_open = false;
    for (int k = 0; k < 4; ++k) {
        s->t_ms[k] = 0.0;
        s->t_n[k] = 0;
    }
    return NB_OK;
}

nb_status nb_sys_get_timings(nb_sys* s, double out[6])
{
    if (!s || !out) return fail(nullptr, NB_ERR_ARG, "NULL argument");
    out[0] = s->t_ms[0];
    out[1] = (double)s->t_n[0];
    out[2] = s->t_ms[1];
    out[3] = (double)s->t_n[1];
    out[4] = s->t_ms[2];
    out[5] = (double)s->t_n[2];
    return NB_OK;
}

nb_status nb_sys_buffer_stats(nb_sys* s, double out[4])
{
    if (!s || !out) return fail(nullptr, NB_ERR_ARG, "NULL argument");
    hipStream_t st = s->ctx->stream;
    double pg[2] = {0.0, 0.0};
    const int nb = std::min(kKeBlocks, std::max(1, (s->p.n_atoms + 255) / 256));
    std::vector<double> part(nb, 0.0);
    HIPCHK(s->ctx, hipMemcpyAsync(out, s->h.disp + kKeBlocks, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipMemcpyAsync(pg, s->h.pg_part + 2 * kKeBlocks, sizeof(pg), hipMemcpyDeviceToHost, st));
    if (s->pg_pending)  // the last interval, not folded on the device yet
        HIPCHK(s->ctx, hipMemcpyAsync(part.data(), s->h.pg_part + (1 - s->pg_cur) * kKeBlocks,
                                      sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    HIPCHK(s->ctx, hipStreamSynchronize(st));
    if (s->pg_pending) {
        double m2 = 0.0;
        for (double v : part) m2 = (v > m2 || v != v) ? v : m2;
        const double mm = std::sqrt(m2);
        if (mm > pg[0] || mm != mm) pg[0] = mm;
        if (!(mm < s->h.prune_half)) pg[1] += 1.0;
    }
    out[2] = pg[0];
    out[3] = pg[1];
    return NB_OK;
}

nb_status nb_sys_set_build_checks(nb_sys* s, int32_t on)
{
    if (!s) return fail(nullptr, NB_ERR_ARG, "NULL argument");
    s->check_builds = on != 0;
    return NB_OK;
}

// One system's list build and forces with every piece of working memory in
// this device's scratch array: the same placement, build and force kernels as
// nb_sys_create + nb_sys_set_particles + nb_compute_forces, on an arena that
// is not allocated.  A build that outgrows the capacity estimate is redone
// with the grown capacities while they fit the array.
nb_status nb_compute_forces_noalloc(nb_ctx* ctx, const nb_params* p, const double* q, const double* sigma,
                                    const double* epsilon, const double* x_dev, float* f_dev,
                                    double* ener_host, double* virial_host)
{
    if (!ctx || !p || !q || !x_dev || !f_dev) return fail(ctx, NB_ERR_ARG, "NULL argument");
    std::string why;
    nb_status r = validate(p, &why);
    if (r) return fail(ctx, r, why);
    if (pme_on(p)) return fail(ctx, NB_ERR_ARG, "the allocation-free entry point has no PME (pme_grid must be zero)");
    if (p->lj == NB_LJ_LB && (!sigma || !epsilon)) return fail(ctx, NB_ERR_ARG, "LB needs sigma and epsilon");
    for (int32_t i = 0; i < p->n_atoms; ++i) {
        if (!std::isfinite(q[i])) return fail(ctx, NB_ERR_ARG, "non-finite charge");
        if (p->lj == NB_LJ_LB && (!(sigma[i] >= 0.0) || !(epsilon[i] >= 0.0)))
            return fail(ctx, NB_ERR_ARG, "sigma/epsilon must be >= 0");
    }
    {
        int* pp;
        int* dd;
        SysDev* ds;
        const size_t need = layout(p, shape_of(p), nullptr, nullptr, &pp, &dd, &ds);
        if (need > kNoallocBytes) {
            char buf[200];
            std::snprintf(buf, sizeof buf,
                          "the system needs %zu bytes of working memory; the allocation-free entry point "
                          "holds at most %zu per GPU",
                          need, kNoallocBytes);
            return fail(ctx, NB_ERR_CAPACITY, buf);
        }
    }
    if (ctx->device < 0 || ctx->device >= kNoallocMaxDevices || !scratch_dev[ctx->device])
        return fail(ctx, NB_ERR_DEVICE,
                    std::string("no scratch array on this device: ") +
                        (ctx->device >= 0 && ctx->device < kNoallocMaxDevices
                             ? hipGetErrorString(scratch_err[ctx->device])
                             : "device index beyond the supported range"));
    HIPCHK(ctx, hipSetDevice(ctx->device));
    nb_sys s;
    init_sys(&s, ctx, p, scratch_dev[ctx->device], kNoallocBytes);
    const size_t N = (size_t)p->n_atoms;
    for (int attempt = 0; attempt < 4; ++attempt) {
        // place() clears the counters and flags a build reads; the per-atom data
        // go straight from the caller's arrays into the array's particle slots
        r = place(&s);
        if (r) return r;
        hipStream_t st = ctx->stream;
        HIPCHK(ctx, hipMemcpyAsync((void*)s.h.q, q, sizeof(double) * N, hipMemcpyHostToDevice, st));
        if (p->lj == NB_LJ_LB) {
            HIPCHK(ctx, hipMemcpyAsync((void*)s.h.sig, sigma, sizeof(double) * N, hipMemcpyHostToDevice, st));
            HIPCHK(ctx, hipMemcpyAsync((void*)s.h.eps, epsilon, sizeof(double) * N, hipMemcpyHostToDevice, st));
        }
        s.has_particles = true;
        s.h.x = x_dev;
        s.h.f = f_dev;
        r = upload_desc(&s);
        if (r) return r;
        r = do_build(&s);
        if (r == NB_ERR_CAPACITY && s.needed_bytes <= kNoallocBytes) continue;
        if (r) return r;
        const bool ener = ener_host || virial_host;
        HIPCHK(ctx, launch_clear_status(s.d_desc, 1, st));
        r = eval_forces(&s, ener, -1, false, 0.0);
        if (r) return r;
        double eo[16];
        if (ener) HIPCHK(ctx, hipMemcpyAsync(eo, s.h.eout, sizeof(eo), hipMemcpyDeviceToHost, st));
        // (synchronises: the caller's host arrays and the next call's use of
        // the array wait for this call's kernels)
        r = check_after(&s);
        if (r) return r;
        if (ener_host) {
            ener_host[0] = eo[0];
            ener_host[1] = eo[1];
        }
        if (virial_host) {
            virial_host[0] = eo[2];
            virial_host[4] = eo[3];
            virial_host[8] = eo[4];
            virial_host[1] = virial_host[3] = eo[5];
            virial_host[2] = virial_host[6] = eo[6];
            virial_host[5] = virial_host[7] = eo[7];
        }
        return NB_OK;
    }
    return fail(ctx, NB_ERR_CAPACITY, "pair-list capacity did not converge in the scratch array");
}

// debug/introspection: max relative error of the Ewald erfc fit (FP64 evaluation)
nb_status nb_sys_ewald_fit_error(const nb_sys* s, double* err)
{
    if (!s || !err) return fail(nullptr, NB_ERR_ARG, "NULL argument");
    *err = s->ew_fit_err;
    return NB_OK;
}

}  // extern "C"
