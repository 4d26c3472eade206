// fk_solver.hip -- one simulation context: tables, time step, state I/O.
//
// Kernels per step: the fused sweep over all tiles of f (HBM-bound; a
// second launch for the tiles outside the main body), the plane sums of
// the tile partials, then the one-workgroup field kernel that reduces the
// wall partials, updates sigma and prepares the next step.  Steps are
// replayed from captured HIP graphs.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>

#include "fk_field.h"
#include "fk_kernels.h"
#include "fk_sweep_fast.h"
#include "fk_sweep2.h"

namespace fk {

// ---------------------------------------------------------------- tables

struct TableArgs {
    double* delta;
    double* ghat;
    double* fsrc64;
    double* wband;
    double* srck;
    double* consts;
    void* fsrc;
    void* gx;
    void* gy;
    int is_f32;
    int nx, nvx, nvy;
    double vmax_x, vmax_y, dvx, dvy, dx, dt;
    double delta_max, a_max_ev, ks, t_se_ev, t_src_ev, t_e_ev;
    double j_src, x_lo, x_hi;
    uint32_t mask;
};

// One velocity axis of the collisional equilibrium (Eq 5 is a product of a
// v_x and a v_y Maxwellian at T_e): exp(-m v^2 / 2 T_e) normalised so that
// its sum times dv is one, written in f's element type.  The product of
// the two factors then has unit discrete integral over the grid.
__device__ void equilibrium_axis(int n, double dv, double t_ev, bool on, int is_f32, void* out, double* sh)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = cell_v(i, n, dv);
        s += on ? exp(-kMe * v * v / (2.0 * t_ev * kE)) * dv : 0.0;
    }
    s = block_sum(s, sh);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = cell_v(i, n, dv);
        const double g = (on && s > 0.0) ? exp(-kMe * v * v / (2.0 * t_ev * kE)) / s : 0.0;
        if (is_f32) static_cast<float*>(out)[i] = (float)g;
        else static_cast<double*>(out)[i] = g;
    }
}

// SEY of Eq 8-9 at incident energy a_ev (Eq 10) and angle alpha (Eq 11).
__device__ double sey_yield(double delta_max, double a_max_ev, double ks, double a_ev, double alpha)
{
    const double z = 1.284 * a_ev / (a_max_ev * (1.0 + ks * alpha * alpha / kPi));
    if (!(z > 0.0)) return 0.0;
    const double rise = -expm1(-pow(z, 1.725));   // 1 - exp(-z^1.725)
    return 1.526 * delta_max * (1.0 + ks * alpha * alpha / (2.0 * kPi)) * rise / pow(z, 0.725);
}

// Per velocity cell: SEY on v_x < 0, emission shape on v_x > 0, source VDF
// on v_y > 0 (unnormalised).
__global__ void k_tables_cells(TableArgs a)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.nvx * a.nvy) return;
    const int i = m / a.nvy, j = m % a.nvy;
    const double vx = cell_v(i, a.nvx, a.dvx);
    const double vy = cell_v(j, a.nvy, a.dvy);
    const double v2 = vx * vx + vy * vy;
    double dl = 0.0, g = 0.0, s = 0.0;
    if (vx < 0.0) {
        const double a_ev = 0.5 * kMe * v2 / kE;
        const double alpha = atan(fabs(vy / vx));
        dl = sey_yield(a.delta_max, a.a_max_ev, a.ks, a_ev, alpha);
    }
    if (vx > 0.0) g = exp(-kMe * v2 / (2.0 * a.t_se_ev * kE));
    if (vy > 0.0) s = exp(-kMe * v2 / (2.0 * a.t_src_ev * kE));
    a.delta[m] = dl;
    a.ghat[m] = g;
    a.fsrc64[m] = s;
}

// Normalisations (one workgroup): Z = sum v_x ghat dv^2, the source VDF
// scaled to unit integral, the band weights and per-plane source
// coefficients, and the particles injected per step.
__global__ void __launch_bounds__(kFieldThreads) k_tables_norm(TableArgs a)
{
    __shared__ double sh[kFieldThreads];
    const int t = threadIdx.x, T = blockDim.x;
    const int nv = a.nvx * a.nvy;
    const double dv2 = a.dvx * a.dvy;
    double z = 0.0, s = 0.0;
    for (int m = t; m < nv; m += T) {
        const int i = m / a.nvy;
        const double vx = cell_v(i, a.nvx, a.dvx);
        if (vx > 0.0) z += vx * a.ghat[m] * dv2;
        s += a.fsrc64[m] * dv2;
    }
    z = block_sum(z, sh);
    s = block_sum(s, sh);
    double norm = 0.0;
    for (int m = t; m < nv; m += T) {
        const double v = s > 0.0 ? a.fsrc64[m] / s : 0.0;
        a.fsrc64[m] = v;
        if (a.is_f32) static_cast<float*>(a.fsrc)[m] = (float)v;
        else static_cast<double*>(a.fsrc)[m] = v;
        norm += v * dv2;
    }
    norm = block_sum(norm, sh);
    const double band = a.x_hi - a.x_lo;
    double inj = 0.0;
    for (int k = t; k < a.nx; k += T) {
        const double lo = fmax(k * a.dx, a.x_lo), hi = fmin((k + 1) * a.dx, a.x_hi);
        const double w = hi > lo ? (hi - lo) / a.dx : 0.0;
        a.wband[k] = w;
        const double c = (band > 0.0 && (a.mask & FK_PHYS_SRC)) ? a.dt * (a.j_src / kE) * w / band : 0.0;
        a.srck[k] = c;
        inj += c * a.dx;
    }
    inj = block_sum(inj, sh);
    if (t == 0) {
        a.consts[0] = z;
        a.consts[1] = norm;
        a.consts[2] = inj * norm;
        const double mt = kMe / (a.t_se_ev * kE);
        a.consts[3] = pow(mt, 1.5) / sqrt(2.0 * kPi);   // Eq 15 prefactor per unit Gamma_see
    }
    const bool bgk = (a.mask & FK_PHYS_BGK) && a.t_e_ev > 0.0;
    equilibrium_axis(a.nvx, a.dvx, a.t_e_ev, bgk, a.is_f32, a.gx, sh);
    equilibrium_axis(a.nvy, a.dvy, a.t_e_ev, bgk, a.is_f32, a.gy, sh);
}

// ---------------------------------------------------------------- kernels

template <typename T, int TI>
__global__ void __launch_bounds__(1024) k_moments(SweepArgs<T> a)
{
    extern __shared__ double smem[];
    moments_tile<T, TI>(a, blockIdx.x, smem);
}

__global__ void __launch_bounds__(64) k_plane_sums(const double* __restrict__ part_n, int nx, int n_it,
                                                    double* __restrict__ plane_sum)
{
    plane_sums(part_n, nx, n_it, plane_sum);
}

__global__ void __launch_bounds__(kFieldThreads) k_field(FieldArgs a)
{
    __shared__ double sh[2 * kFieldThreads];
    field_block(a, sh);
}

// ---------------------------------------------------------------- profile

// Value of the x-resolved enclosed charge sigma_enc(x) = 2 eps0 E_x(x),
// piecewise linear through (0, sigma), the cell centres (x_k, 2 eps0 E_x,k)
// and flat beyond the last centre.
// Enclosed charge sigma_enc(x) = sigma - 2 e int_0^x n_e dx' (2 eps0 times the
// self field of the 1D Gauss solve, Section 2) with n_e constant over each
// cell, at npts uniform points x_p = L p / (npts - 1).  One thread per point
// sums the cells below it in order.
__global__ void k_profile(const double* __restrict__ ne, const DevState* __restrict__ st, int nx, double dx,
                          double length, int npts, double* __restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const double x = length * p / (npts - 1);
    int k = (int)floor(x / dx);
    k = max(0, min(k, nx));
    double below = 0.0;
    for (int q = 0; q < k; ++q) below += ne[q];
    double s = (st->sigma + st->sigma_lo) - 2.0 * kE * dx * below;
    if (k < nx) s -= 2.0 * kE * ne[k] * (x - k * dx);
    out[p] = s;
}

// Piecewise-linear interpolation of a profile given at npts uniform points.
__device__ double profile_at(const double* prof, int npts, double length, double x)
{
    const double u = fmin(fmax(x / length, 0.0), 1.0) * (npts - 1);
    int q = (int)floor(u);
    if (q >= npts - 1) q = npts - 2;
    const double w = u - q;
    return (1.0 - w) * prof[q] + w * prof[q + 1];
}

// Normalisation of the emission-temperature Maxwellian on the velocity grid:
// out = 1 / sum exp(-m v^2 / 2T) dv_x dv_y (one workgroup).
__global__ void __launch_bounds__(kFieldThreads) k_warm_norm(int nvx, int nvy, double dvx, double dvy, double t_ev,
                                                             double* out)
{
    __shared__ double sh[kFieldThreads];
    double s = 0.0;
    for (int m = threadIdx.x; m < nvx * nvy; m += blockDim.x) {
        const double vx = cell_v(m / nvy, nvx, dvx), vy = cell_v(m % nvy, nvy, dvy);
        s += exp(-kMe * (vx * vx + vy * vy) / (2.0 * t_ev * kE)) * dvx * dvy;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *out = s > 0.0 ? 1.0 / s : 0.0;
}

// Warm start: f(x_k, v) = n_k M(v) with n_k = (S(k dx) - S((k+1) dx)) / (2 e dx)
// (clamped at 0): the electron density whose enclosed charge is the profile
// S, averaged over cell k, times the normalised Maxwellian at t_ev.
template <typename T>
__global__ void k_warm_start(T* __restrict__ f, const double* __restrict__ prof, int npts, double length, int nx,
                             int nvx, int nvy, double dx, double dvx, double dvy, double t_ev,
                             const double* __restrict__ norm)
{
    const size_t cells = (size_t)nx * nvx * nvy;
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int k = (int)(c / ((size_t)nvx * nvy));
    const int m = (int)(c % ((size_t)nvx * nvy));
    const double s0 = profile_at(prof, npts, length, k * dx);
    const double s1 = profile_at(prof, npts, length, (k + 1) * dx);
    const double nk = fmax(0.0, (s0 - s1) / (2.0 * kE * dx));
    const double vx = cell_v(m / nvy, nvx, dvx), vy = cell_v(m % nvy, nvy, dvy);
    f[c] = T(nk * *norm * exp(-kMe * (vx * vx + vy * vy) / (2.0 * t_ev * kE)));
}

}  // namespace fk

using namespace fk;

// ---------------------------------------------------------------- context

struct fk_ctx {
    fk_params p;
    Layout L;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    bool own_f = true;
    Buffers b{};
    void* pool = nullptr;         // small buffers
    int cur = 0;                  // which f buffer holds the state
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_steps = 0;          // steps per graph launch (even)
    bool graph_ready = false;
    int sticky = FK_OK;
    std::string err;
    // trace
    std::vector<fk_state> history;
    int64_t drained_step = -1;    // last step whose record has been drained
    // profiling
    int prof = 0;                  // 0: off; n: events around every n-th step
    int64_t prof_count = 0;        // steps launched since profiling was switched on
    struct Ev { hipEvent_t a, b, c; };   // sweep launch a->b, reduction and field b->c
    std::vector<Ev> events;
    std::vector<hipEvent_t> spare;
    std::vector<int> tile_order;   // host copy of the tile list (kept alive for the async upload)
    bool batch_member = false;     // stepped by a batch, not by fk_step
    int64_t host_step = 0;         // step counter of the state, as the queued work will leave it
};

namespace {

int hip_fail(fk_ctx* c, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(c ? &c->err : nullptr, FK_E_HIP, m);
}

#define FK_HIP(c, call)                                        \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
    } while (0)

// ---- sweep launch shape (begin): the code that decides the upwind sweep
// kernels' arguments, tiling and grid.  The benchmark keys its committed HBM
// counter figures to a hash of this region and the sweep's device code.
template <typename T>
SweepArgs<T> sweep_args(const fk_ctx* c, int from)
{
    SweepArgs<T> a{};
    a.fin = static_cast<const T*>(c->b.f[from]);
    a.fout = static_cast<T*>(c->b.f[from ^ 1]);
    a.dxk = c->b.dxk;
    a.srck = c->b.srck;
    a.fsrc = static_cast<const T*>(c->b.fsrc);
    a.nudt = c->b.nudt;
    a.nudt_n = c->b.nudt_n;
    a.gx = static_cast<const T*>(c->b.gx);
    a.gy = static_cast<const T*>(c->b.gy);
    a.ghat = c->b.ghat;
    a.delta = c->b.delta;
    a.st = c->b.st;
    a.part_n = c->b.part_n;
    a.part_wall = c->b.part_wall;
    a.part_top = c->b.part_top;
    a.part_lv = c->b.part_lv;
    a.part_abs = c->b.part_abs;
    a.nx = c->p.nx;
    a.nvx = c->p.nvx;
    a.nvy = c->p.nvy;
    a.n_it = c->L.n_it;
    a.kc = c->L.kc;
    a.dvx = c->L.dvx;
    a.dt_dx = c->L.dt / c->L.dx;
    a.dy = c->L.dy;
    a.r_refl = c->p.r_refl;
    a.x_on = (c->p.physics_mask & FK_PHYS_X) ? 1 : 0;
    // non-temporal stores pay when every row of f starts on a 128-byte line,
    // so that each wave writes whole lines; a row that shares lines with its
    // neighbours is better merged in L2 first
    const bool rows_on_lines = ((size_t)c->p.nvy * sizeof(T)) % 128 == 0 &&
                               reinterpret_cast<uintptr_t>(c->b.f[0]) % 128 == 0 &&
                               reinterpret_cast<uintptr_t>(c->b.f[1]) % 128 == 0;
    a.store_nt = rows_on_lines ? 1 : 0;
    a.tile_list = c->b.tiles;
    a.n_list = c->L.n_it;
    return a;
}

template <typename T, int TI, int MAXB, bool BGK>
void launch_sweep_b(const fk_ctx* c, int from, hipStream_t s)
{
    SweepArgs<T> a = sweep_args<T>(c, from);
    if (c->L.n_fast > 0) {
        a.tile_list = c->b.tiles;
        a.n_list = c->L.n_fast;
        // inner rows streamed where the stores are non-temporal too (rows on 128-byte lines)
        if (a.store_nt)
            hipLaunchKernelGGL((k_sweep<T, TI, MAXB, BGK, true>), dim3(c->L.n_fast * c->L.n_kc), dim3(c->L.block),
                               c->L.lds_sweep, s, a);
        else
            hipLaunchKernelGGL((k_sweep<T, TI, MAXB, BGK, false>), dim3(c->L.n_fast * c->L.n_kc), dim3(c->L.block),
                               c->L.lds_sweep, s, a);
    }
    if (c->L.n_generic > 0) {
        a.tile_list = c->b.tiles + c->L.n_fast;
        a.n_list = c->L.n_generic;
        hipLaunchKernelGGL((k_sweep_generic<T, TI, MAXB, BGK>), dim3(c->L.n_generic * c->L.n_kc),
                           dim3(c->L.block), c->L.lds_sweep, s, a);
    }
}

template <typename T, int TI, int MAXB>
void launch_sweep_t(const fk_ctx* c, int from, hipStream_t s)
{
    if (c->L.bgk) launch_sweep_b<T, TI, MAXB, true>(c, from, s);
    else launch_sweep_b<T, TI, MAXB, false>(c, from, s);
}

// second-order scheme (defined after this region): forward order on even
// steps, reversed on odd ones
void launch_sweep2(const fk_ctx* c, int from, hipStream_t s, int rev);

void launch_sweep(const fk_ctx* c, int from, hipStream_t s, int rev = 0)
{
    if (c->L.scheme == FK_SCHEME_LIMITED2) {
        launch_sweep2(c, from, s, rev);
        return;
    }
    const bool small = c->L.block <= 512;
    if (c->L.elem == 4) {
        switch (c->L.ti) {
        case 16: launch_sweep_t<float, 16, 512>(c, from, s); break;
        case 12: launch_sweep_t<float, 12, 512>(c, from, s); break;
        case 8: small ? launch_sweep_t<float, 8, 512>(c, from, s) : launch_sweep_t<float, 8, 1024>(c, from, s); break;
        default: launch_sweep_t<float, 4, 1024>(c, from, s); break;
        }
    } else {
        switch (c->L.ti) {
        case 8: launch_sweep_t<double, 8, 512>(c, from, s); break;
        default: launch_sweep_t<double, 4, 1024>(c, from, s); break;
        }
    }
}

// Workgroups of a layout's main sweep kernel that fit on one compute unit.
template <bool BGK>
int sweep_wgs_per_cu_b(const Layout& L)
{
    int occ = 0;
    hipError_t e;
    const bool small = L.block <= 512;
    if (L.elem == 4) {
        if (L.ti == 16)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep<float, 16, 512, BGK>, L.block, L.lds_sweep);
        else if (L.ti == 12)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep<float, 12, 512, BGK>, L.block, L.lds_sweep);
        else if (L.ti == 8)
            e = small ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep<float, 8, 512, BGK>, L.block, L.lds_sweep)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep<float, 8, 1024, BGK>, L.block, L.lds_sweep);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep<float, 4, 1024, BGK>, L.block, L.lds_sweep);
    } else {
        e = L.ti == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep<double, 8, 512, BGK>, L.block, L.lds_sweep)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep<double, 4, 1024, BGK>, L.block, L.lds_sweep);
    }
    return e == hipSuccess ? occ : 0;
}

int sweep2_wgs_per_cu(const Layout& L)
{
    // the main launch's kernel (the fast bodies) sets the pace
    int occ = 0;
    hipError_t e;
    const bool small = L.block <= 512;
    if (L.elem == 4) {
        if (L.ti == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep2_fast<float, 8, 512, false>, L.block, L.lds_sweep);
        else if (small) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep2_fast<float, 4, 512, false>, L.block, L.lds_sweep);
        else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep2_fast<float, 4, 1024, false>, L.block, L.lds_sweep);
    } else {
        if (L.ti == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep2_fast<double, 8, 512, false>, L.block, L.lds_sweep);
        else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep2_fast<double, 4, 512, false>, L.block, L.lds_sweep);
    }
    return e == hipSuccess ? occ : 0;
}

int sweep_wgs_per_cu(const Layout& L)
{
    if (L.scheme == FK_SCHEME_LIMITED2) return sweep2_wgs_per_cu(L);
    return L.bgk ? sweep_wgs_per_cu_b<true>(L) : sweep_wgs_per_cu_b<false>(L);
}

// x planes per tile when the caller leaves it open, among 16 .. 128 (steps
// of 8).  The pick is the longest x run whose launch keeps at least 8 waves
// resident on every compute unit (2 per SIMD, or all that a unit can hold
// if that is fewer) and spreads its workgroups evenly: the last round of
// the device's workgroup slots (or, below one round, each unit's share) as
// full as any other candidate's.  With the prefetch overlapped, more waves
// than that only add concurrent streams: at 2048 x 256 x 256, 2 workgroups
// of 4 waves per unit (128 planes) beat 4 (64 planes) by 7%, while 150 v_y
// lanes (3-wave workgroups) needed the 4.  A launch of 4.03 rounds of
// one 6-wave workgroup per unit ran 14% slower than a whole number.  Grids
// too small for the wave target fall back to the fullest last round.
void choose_planes(const fk_params* p, Layout* L)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        return;
    double best = -1.0, best_fill = -1.0;
    Layout pick = *L, pick_fill = *L;
    for (int kc = 16; kc <= 128 && kc <= std::max(16, p->nx); kc += 8) {
        fk_params q = *p;
        q.tile_rows = L->ti;
        q.tile_planes = std::min(kc, p->nx);
        Layout t;
        if (derive_layout(&q, &t, nullptr) != FK_OK) continue;
        const int occ = sweep_wgs_per_cu(t);
        if (occ < 1) continue;
        const int wpw = (t.block + 63) / 64;
        const double slots = (double)cus * occ;
        const double rounds = t.nwg / slots;
        const double fill = t.nwg / (std::ceil(rounds) * slots);
        if (fill >= best_fill - 1e-9) {    // ties go to the longer x runs (later kc)
            best_fill = fill;
            pick_fill = t;
        }
        const double per_cu = (double)t.nwg / cus;
        const int resident = std::min((int)per_cu, occ) * wpw;
        if (resident < std::min(8, occ * wpw)) continue;
        const double even = rounds >= 1.0 ? fill : per_cu / std::ceil(per_cu);
        if (even >= best - 1e-9) {
            best = even;
            pick = t;
        }
    }
    if (best > 0.0) *L = pick;
    else if (best_fill > 0.0) *L = pick_fill;
    (void)hipGetLastError();
}

// ---- sweep launch shape (end)

template <typename T, int TI, int MAXB, bool REV>
void launch_sweep2_r(const fk_ctx* c, int from, hipStream_t s)
{
    SweepArgs<T> a = sweep_args<T>(c, from);
    if (c->L.n_fast > 0 && c->L.n_generic > 0) {
        // one launch: the generic tiles' workgroups first (padded to a
        // multiple of 8), then the fast tiles'
        const int n_gen = (c->L.n_generic * c->L.n_kc + 7) / 8 * 8;
        hipLaunchKernelGGL((k_sweep2_all<T, TI, MAXB, REV>), dim3(n_gen + c->L.n_fast * c->L.n_kc), dim3(c->L.block),
                           c->L.lds_sweep, s, a, (const int*)c->b.tiles, c->L.n_fast, c->L.n_generic, n_gen,
                           c->L.n_kc);
        return;
    }
    if (c->L.n_fast > 0) {
        a.tile_list = c->b.tiles;
        a.n_list = c->L.n_fast;
        hipLaunchKernelGGL((k_sweep2_fast<T, TI, MAXB, REV>), dim3(c->L.n_fast * c->L.n_kc), dim3(c->L.block),
                           c->L.lds_sweep, s, a);
    }
    if (c->L.n_generic > 0) {
        a.tile_list = c->b.tiles + c->L.n_fast;
        a.n_list = c->L.n_generic;
        hipLaunchKernelGGL((k_sweep2<T, TI, MAXB, REV>), dim3(c->L.n_generic * c->L.n_kc), dim3(c->L.block),
                           c->L.lds_sweep, s, a);
    }
}

template <typename T, int TI, int MAXB>
void launch_sweep2_t(const fk_ctx* c, int from, hipStream_t s, int rev)
{
    if (rev) launch_sweep2_r<T, TI, MAXB, true>(c, from, s);
    else launch_sweep2_r<T, TI, MAXB, false>(c, from, s);
}

// second-order scheme: forward order on even steps, reversed on odd ones
void launch_sweep2(const fk_ctx* c, int from, hipStream_t s, int rev)
{
    const bool small = c->L.block <= 512;
    if (c->L.elem == 4) {
        if (c->L.ti == 8) launch_sweep2_t<float, 8, 512>(c, from, s, rev);
        else small ? launch_sweep2_t<float, 4, 512>(c, from, s, rev) : launch_sweep2_t<float, 4, 1024>(c, from, s, rev);
    } else {
        if (c->L.ti == 8) launch_sweep2_t<double, 8, 512>(c, from, s, rev);
        else launch_sweep2_t<double, 4, 512>(c, from, s, rev);
    }
}

void launch_moments(const fk_ctx* c, hipStream_t s)
{
    if (c->L.elem == 4) {
        auto a = sweep_args<float>(c, c->cur);
        switch (c->L.ti) {
        case 16: hipLaunchKernelGGL((k_moments<float, 16>), dim3(c->L.nwg), dim3(c->L.block), c->L.lds_moments, s, a); break;
        case 12: hipLaunchKernelGGL((k_moments<float, 12>), dim3(c->L.nwg), dim3(c->L.block), c->L.lds_moments, s, a); break;
        case 8: hipLaunchKernelGGL((k_moments<float, 8>), dim3(c->L.nwg), dim3(c->L.block), c->L.lds_moments, s, a); break;
        default: hipLaunchKernelGGL((k_moments<float, 4>), dim3(c->L.nwg), dim3(c->L.block), c->L.lds_moments, s, a); break;
        }
    } else {
        auto a = sweep_args<double>(c, c->cur);
        switch (c->L.ti) {
        case 8: hipLaunchKernelGGL((k_moments<double, 8>), dim3(c->L.nwg), dim3(c->L.block), c->L.lds_moments, s, a); break;
        default: hipLaunchKernelGGL((k_moments<double, 4>), dim3(c->L.nwg), dim3(c->L.block), c->L.lds_moments, s, a); break;
        }
    }
}

FieldArgs field_args(const fk_ctx* c, int advance)
{
    FieldArgs a{};
    a.part_n = c->b.part_n;
    a.part_wall = c->b.part_wall;
    a.part_top = c->b.part_top;
    a.part_lv = c->b.part_lv;
    a.n_it = c->L.n_it;
    a.nwg = c->L.nwg;
    a.consts = c->b.consts;
    a.ne = c->b.ne;
    a.ex = c->b.ex;
    a.dxk = c->b.dxk;
    a.nudt = c->b.nudt;
    a.nudt_n = c->b.nudt_n;
    a.st = c->b.st;
    a.ring = c->b.ring;
    a.nx = c->p.nx;
    a.advance = advance;
    a.mask = c->p.physics_mask;
    a.emission_norm = c->p.emission_norm;
    a.trace_stride = c->p.trace_stride;
    a.trace_cap = c->p.trace_cap;
    a.dx = c->L.dx;
    a.dv2 = c->L.dvx * c->L.dvy;
    a.dt = c->L.dt;
    a.dvx = c->L.dvx;
    a.ex_ext = c->p.ex_external;
    a.r_refl = c->p.r_refl;
    a.r_inel = c->p.r_inel;
    a.part_abs = c->b.part_abs;
    a.abs_from_sweep = 0;
    if (c->L.bgk) {
        // Eq 4: nu_ee = n_e e^4 ln(Lambda) / (12 pi^1.5 eps0^2 sqrt(m_e) T_e^1.5), T_e in joules
        const double te = c->p.t_e_ev * kE;
        a.nudt_per_n = c->L.dt * kE * kE * kE * kE * c->p.ln_lambda /
                       (12.0 * pow(kPi, 1.5) * kEps0 * kEps0 * sqrt(kMe) * te * sqrt(te));
    }
    return a;
}

void launch_field(const fk_ctx* c, int advance, hipStream_t s, int rev = 0)
{
    // many narrow workgroups for the plane sums (the bulk of the reduction),
    // then the one-workgroup field solve on them
    hipLaunchKernelGGL(k_plane_sums, dim3((c->p.nx + 63) / 64), dim3(64), 0, s, c->b.part_n, c->p.nx, c->L.n_it,
                       c->b.plane_sum);
    FieldArgs a = field_args(c, advance);
    a.plane_sum = c->b.plane_sum;
    a.abs_from_sweep = (advance && rev) ? 1 : 0;
    hipLaunchKernelGGL(k_field, dim3(1), dim3(kFieldThreads), 0, s, a);
}

// whether step `step` (from f^step) runs in the reversed split order
int reversed_step(const fk_ctx* c, int64_t step)
{
    return (c->L.scheme == FK_SCHEME_LIMITED2 && (step & 1)) ? 1 : 0;
}

// one step from buffer `from` into the other
void enqueue_step(const fk_ctx* c, int from, hipStream_t s, int rev = 0)
{
    launch_sweep(c, from, s, rev);
    launch_field(c, 1, s, rev);
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// v_x tiles of the current layout: fast ones first, then the generic ones
int upload_tiles(fk_ctx* c)
{
    std::vector<int> order;
    for (int it = 0; it < c->L.n_it; ++it)
        if (tile_main(it, c->L.ti, c->p.nvx, c->L.scheme)) order.push_back(it);
    for (int it = 0; it < c->L.n_it; ++it)
        if (!tile_main(it, c->L.ti, c->p.nvx, c->L.scheme)) order.push_back(it);
    c->tile_order = order;
    FK_HIP(c, hipMemcpyAsync(c->b.tiles, c->tile_order.data(), order.size() * sizeof(int),
                             hipMemcpyHostToDevice, c->stream));
    return FK_OK;
}

// Layout of an instance's tables, partials and small state in one block of
// device memory (everything but f); returns its size in bytes and, with a
// base address, points b's members into it.
size_t carve_buffers(const fk_params& p, const Layout& L, char* base, Buffers* b)
{
    const size_t v2 = (size_t)p.nvx * p.nvy;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    const size_t o_delta = take(v2 * 8), o_ghat = take(v2 * 8), o_fsrc64 = take(v2 * 8),
                 o_fsrc = take(v2 * L.elem), o_wband = take(p.nx * 8), o_srck = take(p.nx * 8),
                 o_pn = take((size_t)p.nx * L.n_it_cap * 8), o_pw = take((size_t)L.n_it_cap * 16),
                 o_pt = take((size_t)L.n_it_cap * 8), o_plv = take((size_t)L.nwg_cap * 8),
                 o_pab = take((size_t)L.n_it_cap * 16),
                 o_ne = take(p.nx * 8), o_ex = take(p.nx * 8), o_dxk = take(p.nx * 8),
                 o_nudt = take(p.nx * 8), o_nudtn = take(p.nx * 8), o_gx = take((size_t)p.nvx * L.elem),
                 o_gy = take((size_t)p.nvy * L.elem),
                 o_consts = take(64), o_tiles = take((size_t)L.n_it_cap * sizeof(int)),
                 o_psum = take((size_t)p.nx * 8), o_st = take(sizeof(DevState)),
                 o_ring = take((size_t)p.trace_cap * sizeof(fk_state));
    if (!base) return off;
    b->delta = (double*)(base + o_delta);
    b->ghat = (double*)(base + o_ghat);
    b->fsrc64 = (double*)(base + o_fsrc64);
    b->fsrc = base + o_fsrc;
    b->wband = (double*)(base + o_wband);
    b->srck = (double*)(base + o_srck);
    b->part_n = (double*)(base + o_pn);
    b->part_wall = (double*)(base + o_pw);
    b->part_top = (double*)(base + o_pt);
    b->part_lv = (double*)(base + o_plv);
    b->part_abs = (double*)(base + o_pab);
    b->ne = (double*)(base + o_ne);
    b->ex = (double*)(base + o_ex);
    b->dxk = (double*)(base + o_dxk);
    b->nudt = (double*)(base + o_nudt);
    b->nudt_n = (double*)(base + o_nudtn);
    b->gx = base + o_gx;
    b->gy = base + o_gy;
    b->consts = (double*)(base + o_consts);
    b->tiles = (int*)(base + o_tiles);
    b->plane_sum = (double*)(base + o_psum);
    b->st = (DevState*)(base + o_st);
    b->ring = (fk_state*)(base + o_ring);
    return off;
}

int alloc_buffers(fk_ctx* c, void* fa, void* fb)
{
    const fk_params& p = c->p;
    const Layout& L = c->L;
    const size_t off = carve_buffers(p, L, nullptr, nullptr);
    if (hipMalloc(&c->pool, off) != hipSuccess) {
        c->pool = nullptr;
        return set_error(&c->err, FK_E_OOM, "device allocation of tables and partials failed");
    }
    carve_buffers(p, L, static_cast<char*>(c->pool), &c->b);
    FK_HIP(c, hipMemsetAsync(c->pool, 0, off, c->stream));
    {
        int rc = upload_tiles(c);
        if (rc) return rc;
    }
    const size_t fbytes = (size_t)L.cells * L.elem;
    if (fa) {
        c->own_f = false;
        c->b.f[0] = fa;
        c->b.f[1] = fb;
    } else {
        c->own_f = true;
        if (hipMalloc(&c->b.f[0], fbytes) != hipSuccess) {
            c->b.f[0] = nullptr;
            return set_error(&c->err, FK_E_OOM, "device allocation of f failed");
        }
        if (hipMalloc(&c->b.f[1], fbytes) != hipSuccess) {
            c->b.f[1] = nullptr;
            return set_error(&c->err, FK_E_OOM, "device allocation of f failed");
        }
    }
    FK_HIP(c, hipMemsetAsync(c->b.f[0], 0, fbytes, c->stream));
    FK_HIP(c, hipMemsetAsync(c->b.f[1], 0, fbytes, c->stream));
    return FK_OK;
}

int build_tables(fk_ctx* c)
{
    const fk_params& p = c->p;
    TableArgs a{};
    a.delta = c->b.delta;
    a.ghat = c->b.ghat;
    a.fsrc64 = c->b.fsrc64;
    a.wband = c->b.wband;
    a.srck = c->b.srck;
    a.consts = c->b.consts;
    a.fsrc = c->b.fsrc;
    a.gx = c->b.gx;
    a.gy = c->b.gy;
    a.is_f32 = c->L.elem == 4;
    a.nx = p.nx;
    a.nvx = p.nvx;
    a.nvy = p.nvy;
    a.vmax_x = p.vmax_x;
    a.vmax_y = p.vmax_y;
    a.dvx = c->L.dvx;
    a.dvy = c->L.dvy;
    a.dx = c->L.dx;
    a.dt = c->L.dt;
    a.delta_max = p.delta_max;
    a.a_max_ev = p.a_max_ev;
    a.ks = p.ks;
    a.t_se_ev = p.t_se_ev;
    a.t_src_ev = p.t_src_ev;
    a.t_e_ev = p.t_e_ev;
    a.j_src = p.j_src;
    a.x_lo = p.x_src_lo;
    a.x_hi = p.x_src_hi;
    a.mask = p.physics_mask;
    const int nv = p.nvx * p.nvy;
    hipLaunchKernelGGL(k_tables_cells, dim3((nv + 255) / 256), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_tables_norm, dim3(1), dim3(kFieldThreads), 0, c->stream, a);
    FK_HIP(c, hipGetLastError());
    return FK_OK;
}

// recompute the prologue quantities of the current f and state
int refresh(fk_ctx* c)
{
    launch_moments(c, c->stream);
    launch_field(c, 0, c->stream);
    FK_HIP(c, hipGetLastError());
    return FK_OK;
}

int capture_graphs(fk_ctx* c)
{
    c->graph_ready = false;
    for (auto& g : c->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    if (c->batch_member) return FK_OK;   // a batch replays its own graphs
    c->graph_steps = 16;
    for (int start = 0; start < 2; ++start) {
        hipGraph_t g = nullptr;
        FK_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        for (int s = 0; s < c->graph_steps; ++s) enqueue_step(c, (start + s) & 1, c->cap_stream, reversed_step(c, s));
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&c->graph[start], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
    }
    c->graph_ready = true;
    return FK_OK;
}

hipEvent_t get_event(fk_ctx* c)
{
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int read_devstate(fk_ctx* c, DevState* out)
{
    FK_HIP(c, hipMemcpyAsync(out, c->b.st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    FK_HIP(c, hipStreamSynchronize(c->stream));
    return FK_OK;
}

int flags_to_code(uint32_t f)
{
    if (f & kFlagNonfinite) return FK_E_NONFINITE;
    if (f & kFlagCfl) return FK_E_CFL;
    return FK_OK;
}

int drain(fk_ctx* c, size_t* fresh_begin)
{
    DevState s;
    int rc = read_devstate(c, &s);
    if (rc) return rc;
    *fresh_begin = c->history.size();
    const int64_t stride = c->p.trace_stride, cap = c->p.trace_cap;
    const int64_t last_rec = s.step / stride;               // index of the newest record
    int64_t first_rec = c->drained_step < 0 ? 0 : c->drained_step / stride + 1;
    int code = FK_OK;
    if (last_rec - first_rec + 1 > cap) {
        first_rec = last_rec - cap + 1;
        code = FK_E_STATE;
    }
    const int64_t n = last_rec - first_rec + 1;
    if (n > 0) {
        // copy only the slots of the new records (one or two ranges of the ring)
        std::vector<fk_state> tmp((size_t)n);
        const int64_t s0 = first_rec % cap;
        const int64_t n1 = std::min(n, cap - s0);
        FK_HIP(c, hipMemcpyAsync(tmp.data(), c->b.ring + s0, sizeof(fk_state) * n1, hipMemcpyDeviceToHost, c->stream));
        if (n1 < n)
            FK_HIP(c, hipMemcpyAsync(tmp.data() + n1, c->b.ring, sizeof(fk_state) * (n - n1), hipMemcpyDeviceToHost,
                                     c->stream));
        FK_HIP(c, hipStreamSynchronize(c->stream));
        c->history.insert(c->history.end(), tmp.begin(), tmp.end());
        c->drained_step = last_rec * stride;
    }
    if (code) set_error(&c->err, code, "trace ring overflowed; older records were lost");
    return code;
}

void release(fk_ctx* c)
{
    if (!c) return;
    if (c->stream || c->pool) (void)hipStreamSynchronize(c->stream);
    for (auto& g : c->graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto& e : c->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
        (void)hipEventDestroy(e.c);
    }
    for (auto e : c->spare) (void)hipEventDestroy(e);
    if (c->own_f) {
        if (c->b.f[0]) (void)hipFree(c->b.f[0]);
        if (c->b.f[1]) (void)hipFree(c->b.f[1]);
    }
    if (c->pool) (void)hipFree(c->pool);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

// Switch the context to another tiling (v_x rows, x planes per tile); the
// partial buffers are sized for any tiling.  Recomputes the prologue of the
// current state and recaptures the step graphs.
int retile(fk_ctx* c, int ti, int kc)
{
    fk_params q = c->p;
    q.tile_rows = ti;
    q.tile_planes = kc;
    Layout L;
    std::string why;
    int rc = derive_layout(&q, &L, &why);
    if (rc) return set_error(&c->err, rc, why);
    FK_HIP(c, hipStreamSynchronize(c->stream));
    c->p.tile_rows = ti;
    c->p.tile_planes = kc;
    c->L = L;
    rc = upload_tiles(c);
    if (!rc) rc = refresh(c);
    if (!rc) rc = capture_graphs(c);
    if (!rc) FK_HIP(c, hipStreamSynchronize(c->stream));
    return rc;
}

// Candidate tilings of a parameter set (the autotuner's search space).
std::vector<std::pair<int, int>> tile_candidates(const fk_params& p)
{
    std::vector<std::pair<int, int>> out;
    const int tis[4] = {4, 8, 12, 16};
    const int kcs[4] = {16, 32, 64, 128};
    for (int ti : tis)
        for (int kc : kcs) {
            fk_params q = p;
            q.tile_rows = ti;
            q.tile_planes = kc;
            Layout L;
            if (derive_layout(&q, &L, nullptr) == FK_OK && L.kc == kc) out.push_back({ti, kc});
        }
    if (out.empty()) out.push_back({0, 0});
    return out;
}

int create_impl(const fk_params* p, void* stream, void* fa, void* fb, fk_ctx** out, bool member = false)
{
    if (!out) return set_error(nullptr, FK_E_INVALID, "out is NULL");
    *out = nullptr;
    Layout L;
    std::string why;
    int rc = derive_layout(p, &L, &why);
    if (rc) return set_error(nullptr, rc, why);
    // the chunk length from the upwind sweep's occupancy; the second-order
    // sweep keeps its short chunks (it is bound by the vector ALU)
    if (p->tile_planes == 0 && p->scheme == FK_SCHEME_UPWIND) choose_planes(p, &L);
    if ((fa == nullptr) != (fb == nullptr)) return set_error(nullptr, FK_E_INVALID, "borrowed buffers: give both or neither");
    if (fa && fa == fb) return set_error(nullptr, FK_E_INVALID, "borrowed buffers must differ");
    fk_ctx* c = new (std::nothrow) fk_ctx();
    if (!c) return set_error(nullptr, FK_E_OOM, "host allocation failed");
    c->p = *p;
    c->L = L;
    c->stream = static_cast<hipStream_t>(stream);
    c->batch_member = member;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess && !member) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        std::string m = std::string("HIP initialisation failed: ") + hipGetErrorString(e);
        release(c);
        return set_error(nullptr, FK_E_HIP, m);
    }
    rc = alloc_buffers(c, fa, fb);
    if (!rc) rc = build_tables(c);
    if (!rc) rc = refresh(c);
    if (!rc) rc = capture_graphs(c);
    if (!rc) {
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = hip_fail(c, e, "create");
    }
    if (rc) {
        std::string m = c->err;
        release(c);
        return set_error(nullptr, rc, m);
    }
    *out = c;
    return FK_OK;
}

}  // namespace

extern "C" const char* fk_last_error(const fk_ctx* c) { return c ? c->err.c_str() : global_error(); }

extern "C" int fk_create(const fk_params* p, void* stream, fk_ctx** out)
{
    return create_impl(p, stream, nullptr, nullptr, out);
}

extern "C" int fk_create_borrowed(const fk_params* p, void* stream, void* f_a, void* f_b, fk_ctx** out)
{
    if (!f_a || !f_b) return set_error(nullptr, FK_E_INVALID, "borrowed buffers must not be NULL");
    return create_impl(p, stream, f_a, f_b, out);
}

extern "C" int fk_destroy(fk_ctx* c)
{
    if (!c) return FK_E_INVALID;
    release(c);
    return FK_OK;
}

extern "C" int fk_query(const fk_ctx* c, fk_info* out)
{
    if (!c || !out) return FK_E_INVALID;
    out->dx = c->L.dx; out->dvx = c->L.dvx; out->dvy = c->L.dvy; out->dt = c->L.dt;
    out->courant_x = c->L.courant_x; out->courant_vy = c->L.courant_vy;
    out->cells = c->L.cells; out->tile_rows = c->L.ti; out->tile_planes = c->L.kc;
    out->block = c->L.block; out->n_tiles = c->L.nwg; out->bytes_device = c->L.bytes_device;
    return FK_OK;
}

extern "C" int fk_step(fk_ctx* c, int64_t n)
{
    if (!c || n < 0) return set_error(c ? &c->err : nullptr, FK_E_INVALID, "bad arguments to fk_step");
    if (c->batch_member) return set_error(&c->err, FK_E_STATE, "a batch member is stepped through fk_batch_step");
    if (c->sticky) return c->sticky;
    auto direct = [&]() {
        enqueue_step(c, c->cur, c->stream, reversed_step(c, c->host_step));
        c->cur ^= 1;
        c->host_step += 1;
    };
    if (c->prof) {
        // direct launches; a sampled step gets three events: before and
        // after its sweep launch and after its reduction and field kernels
        for (int64_t s = 0; s < n; ++s) {
            if (c->prof_count++ % c->prof != 0) {
                direct();
                continue;
            }
            hipEvent_t e0 = get_event(c), e1 = get_event(c), e2 = get_event(c);
            if (!e0 || !e1 || !e2) return set_error(&c->err, FK_E_HIP, "hipEventCreate failed");
            const int rev = reversed_step(c, c->host_step);
            FK_HIP(c, hipEventRecord(e0, c->stream));
            launch_sweep(c, c->cur, c->stream, rev);
            FK_HIP(c, hipEventRecord(e1, c->stream));
            launch_field(c, 1, c->stream, rev);
            FK_HIP(c, hipEventRecord(e2, c->stream));
            c->events.push_back({e0, e1, e2});
            c->cur ^= 1;
            c->host_step += 1;
        }
        FK_HIP(c, hipGetLastError());
        return FK_OK;
    }
    int64_t left = n;
    // the graphs start at an even step (the second-order scheme alternates
    // its split order with the step's parity)
    if (left > 0 && (c->host_step & 1) && c->L.scheme == FK_SCHEME_LIMITED2) {
        direct();
        left -= 1;
    }
    if (c->graph_ready) {
        while (left >= c->graph_steps) {
            FK_HIP(c, hipGraphLaunch(c->graph[c->cur], c->stream));
            left -= c->graph_steps;   // graph_steps is even: cur and the step parity unchanged
            c->host_step += c->graph_steps;
        }
    }
    for (; left > 0; --left) direct();
    FK_HIP(c, hipGetLastError());
    return FK_OK;
}

extern "C" int fk_sync(fk_ctx* c)
{
    if (!c) return FK_E_INVALID;
    DevState s;
    int rc = read_devstate(c, &s);
    if (rc) return rc;
    int code = flags_to_code(s.flags);
    if (code) {
        c->sticky = code;
        return set_error(&c->err, code, code == FK_E_CFL ? "v_x Courant number or nu_ee dt above one (E_x or n_e too large for dt)"
                                                          : "non-finite moment, flux or surface charge");
    }
    return FK_OK;
}

extern "C" int fk_read_f(fk_ctx* c, void* dst, size_t bytes, int on_device)
{
    if (!c || !dst) return FK_E_INVALID;
    const size_t need = (size_t)c->L.cells * c->L.elem;
    if (bytes < need) return set_error(&c->err, FK_E_INVALID, "destination too small");
    FK_HIP(c, hipMemcpyAsync(dst, c->b.f[c->cur], need, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    FK_HIP(c, hipStreamSynchronize(c->stream));
    return FK_OK;
}

extern "C" int fk_read_state(fk_ctx* c, fk_state* out)
{
    if (!c || !out) return FK_E_INVALID;
    DevState s;
    int rc = read_devstate(c, &s);
    if (rc) return rc;
    out->step = s.step;
    out->t = (double)s.step * c->L.dt;
    out->sigma = s.sigma;
    out->sigma_lo = s.sigma_lo;
    out->g_pe = s.g_pe;
    out->g_see = s.g_see;
    out->g_top = s.g_top;
    out->emitted = s.emitted;
    out->loss_v = s.loss_v;
    out->n_total = s.n_total;
    out->resid = s.resid;
    return FK_OK;
}

extern "C" int fk_read_field(fk_ctx* c, double* ex, double* ne, int on_device)
{
    if (!c) return FK_E_INVALID;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (ex) FK_HIP(c, hipMemcpyAsync(ex, c->b.ex, c->p.nx * sizeof(double), k, c->stream));
    if (ne) FK_HIP(c, hipMemcpyAsync(ne, c->b.ne, c->p.nx * sizeof(double), k, c->stream));
    FK_HIP(c, hipStreamSynchronize(c->stream));
    return FK_OK;
}

extern "C" int fk_read_tables(fk_ctx* c, double* delta, double* ghat, double* fsrc, double* wband)
{
    if (!c) return FK_E_INVALID;
    const size_t v2 = (size_t)c->p.nvx * c->p.nvy * sizeof(double);
    if (delta) FK_HIP(c, hipMemcpyAsync(delta, c->b.delta, v2, hipMemcpyDeviceToHost, c->stream));
    if (ghat) FK_HIP(c, hipMemcpyAsync(ghat, c->b.ghat, v2, hipMemcpyDeviceToHost, c->stream));
    if (fsrc) FK_HIP(c, hipMemcpyAsync(fsrc, c->b.fsrc64, v2, hipMemcpyDeviceToHost, c->stream));
    if (wband) FK_HIP(c, hipMemcpyAsync(wband, c->b.wband, c->p.nx * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    FK_HIP(c, hipStreamSynchronize(c->stream));
    return FK_OK;
}

extern "C" int fk_read_trace(fk_ctx* c, fk_state* dst, size_t cap, size_t* n_out)
{
    if (!c || !n_out || (!dst && cap)) return FK_E_INVALID;
    size_t begin = 0;
    int rc = drain(c, &begin);
    if (rc && rc != FK_E_STATE) return rc;
    size_t n = std::min(cap, c->history.size() - begin);
    if (n) std::memcpy(dst, c->history.data() + begin, n * sizeof(fk_state));
    *n_out = n;
    return rc;
}

extern "C" int fk_write_state(fk_ctx* c, const void* f, int on_device, double sigma, double sigma_lo, int64_t step)
{
    if (!c || step < 0 || !std::isfinite(sigma) || !std::isfinite(sigma_lo)) return FK_E_INVALID;
    FK_HIP(c, hipStreamSynchronize(c->stream));
    if (f) {
        const size_t need = (size_t)c->L.cells * c->L.elem;
        FK_HIP(c, hipMemcpyAsync(c->b.f[c->cur], f, need, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    }
    DevState s{};
    s.step = step;
    s.sigma = sigma;
    s.sigma_lo = sigma_lo;
    FK_HIP(c, hipMemcpyAsync(c->b.st, &s, sizeof(s), hipMemcpyHostToDevice, c->stream));
    int rc = refresh(c);
    if (rc) return rc;
    FK_HIP(c, hipStreamSynchronize(c->stream));
    c->sticky = FK_OK;
    c->host_step = step;
    c->history.clear();
    c->drained_step = step - 1;
    // the record of the restored state itself is drained from the ring only
    // if it falls on the stride
    if (step % c->p.trace_stride != 0) c->drained_step = step;
    return FK_OK;
}

extern "C" int fk_saturated(fk_ctx* c, double window_s, double rtol, int* out)
{
    if (!c || !out) return FK_E_INVALID;
    size_t begin = 0;
    int rc = drain(c, &begin);
    if (rc && rc != FK_E_STATE) return rc;
    return fk_saturation_check(c->history.data(), c->history.size(), window_s, rtol, out);
}

extern "C" int fk_set_profiling(fk_ctx* c, int every)
{
    if (!c || every < 0) return FK_E_INVALID;
    FK_HIP(c, hipStreamSynchronize(c->stream));
    for (auto& e : c->events) {
        c->spare.push_back(e.a);
        c->spare.push_back(e.b);
        c->spare.push_back(e.c);
    }
    c->events.clear();
    c->prof = every;
    c->prof_count = 0;
    return FK_OK;
}

extern "C" int fk_kernel_times(fk_ctx* c, double* sweep_ms, int64_t* sweep_n, double* field_ms, int64_t* field_n)
{
    if (!c) return FK_E_INVALID;
    FK_HIP(c, hipStreamSynchronize(c->stream));
    double t[2] = {0, 0};
    int64_t n[2] = {0, 0};
    for (const auto& e : c->events) {
        float ms = 0;
        FK_HIP(c, hipEventElapsedTime(&ms, e.a, e.b));
        t[0] += ms;
        n[0] += 1;
        FK_HIP(c, hipEventElapsedTime(&ms, e.b, e.c));
        t[1] += ms;
        n[1] += 1;
    }
    if (sweep_ms) *sweep_ms = t[0];
    if (sweep_n) *sweep_n = n[0];
    if (field_ms) *field_ms = t[1];
    if (field_n) *field_n = n[1];
    return FK_OK;
}

extern "C" int fk_autotune(fk_ctx* c, int trial_steps, fk_info* chosen)
{
    if (!c || trial_steps < 2) return FK_E_INVALID;
    if (c->batch_member) return set_error(&c->err, FK_E_STATE, "batch members are tuned by their batch");
    if (c->sticky) return c->sticky;
    const int prof = c->prof;
    c->prof = 0;
    size_t begin = 0;
    int rc = drain(c, &begin);
    if (rc && rc != FK_E_STATE) return rc;
    DevState saved;
    rc = read_devstate(c, &saved);
    if (rc) return rc;
    const int64_t saved_step = c->host_step;
    // keep the state while the trials step it
    const size_t fbytes = (size_t)c->L.cells * c->L.elem;
    void* keep = nullptr;
    std::vector<char> host_keep;
    if (hipMalloc(&keep, fbytes) == hipSuccess) {
        FK_HIP(c, hipMemcpyAsync(keep, c->b.f[c->cur], fbytes, hipMemcpyDeviceToDevice, c->stream));
    } else {
        keep = nullptr;
        host_keep.resize(fbytes);
        FK_HIP(c, hipMemcpyAsync(host_keep.data(), c->b.f[c->cur], fbytes, hipMemcpyDeviceToHost, c->stream));
    }
    hipEvent_t e0 = get_event(c), e1 = get_event(c);
    if (!e0 || !e1) rc = set_error(&c->err, FK_E_HIP, "hipEventCreate failed");
    int best_ti = c->L.ti, best_kc = c->L.kc;
    float best_ms = 1e30f;
    for (auto cand : tile_candidates(c->p)) {
        if (rc) break;
        rc = retile(c, cand.first, cand.second);
        if (rc) break;
        rc = fk_step(c, 2);
        if (rc) break;
        if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = FK_E_HIP; break; }
        rc = fk_step(c, trial_steps);
        if (rc) break;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = FK_E_HIP; break; }
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = FK_E_HIP; break; }
        if (ms < best_ms) {
            best_ms = ms;
            best_ti = c->L.ti;
            best_kc = c->L.kc;
        }
    }
    if (e0) c->spare.push_back(e0);
    if (e1) c->spare.push_back(e1);
    if (!rc) rc = retile(c, best_ti, best_kc);
    // restore the state
    if (keep) {
        if (hipMemcpyAsync(c->b.f[c->cur], keep, fbytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess && !rc)
            rc = FK_E_HIP;
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(keep);
    } else if (hipMemcpyAsync(c->b.f[c->cur], host_keep.data(), fbytes, hipMemcpyHostToDevice, c->stream) != hipSuccess && !rc) {
        rc = FK_E_HIP;
    }
    if (hipMemcpyAsync(c->b.st, &saved, sizeof(saved), hipMemcpyHostToDevice, c->stream) != hipSuccess && !rc) rc = FK_E_HIP;
    c->host_step = saved_step;
    if (!rc) rc = refresh(c);
    if (!rc) FK_HIP(c, hipStreamSynchronize(c->stream));
    c->prof = prof;
    if (rc) return rc;
    if (chosen) return fk_query(c, chosen);
    return FK_OK;
}

// ================================================================ no allocation
//
// fk_step_noalloc: borrowed create, steps and state read-out in one call
// that allocates nothing.  Everything but f (tables, tile partials, the
// small state, the trace ring) lives in one file-scope device array per
// GPU; the caller's two f buffers hold the state.

namespace fk {

constexpr size_t kScratchBytes = (size_t)32 << 20;   // 32 MiB per device, held until the process ends
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

__global__ void k_fill_zero(uint64_t* __restrict__ p, size_t n)
{
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n; m += (size_t)gridDim.x * blockDim.x)
        p[m] = 0;
}

// the v_x tile list of a layout (fast tiles first, then the others), made
// on the device so that no host buffer has to outlive the call
__global__ void k_tile_list(int* __restrict__ tiles, int n_it, int ti, int nvx, int scheme)
{
    if (threadIdx.x != 0) return;
    int m = 0;
    for (int it = 0; it < n_it; ++it)
        if (tile_main(it, ti, nvx, scheme)) tiles[m++] = it;
    for (int it = 0; it < n_it; ++it)
        if (!tile_main(it, ti, nvx, scheme)) tiles[m++] = it;
}

__global__ void k_state_init(DevState* __restrict__ st, double sigma, double sigma_lo, int64_t step)
{
    if (threadIdx.x != 0) return;
    DevState s{};
    s.step = step;
    s.sigma = sigma;
    s.sigma_lo = sigma_lo;
    *st = s;
}

__global__ void k_state_out(const DevState* __restrict__ st, double dt, fk_state* __restrict__ out,
                            uint32_t* __restrict__ flags)
{
    if (threadIdx.x != 0) return;
    const DevState s = *st;
    if (out) {
        fk_state r;
        r.step = s.step;
        r.t = (double)s.step * dt;
        r.sigma = s.sigma;
        r.sigma_lo = s.sigma_lo;
        r.g_pe = s.g_pe;
        r.g_see = s.g_see;
        r.g_top = s.g_top;
        r.emitted = s.emitted;
        r.loss_v = s.loss_v;
        r.n_total = s.n_total;
        r.resid = s.resid;
        *out = r;
    }
    if (flags) *flags = s.flags;
}

}  // namespace fk

namespace {

// device address of the scratch array on each device, taken once per device
// with that device current
std::atomic<void*> g_scratch_addr[fk::kMaxDevices];

void* scratch_address(int dev)
{
    if (dev < 0 || dev >= fk::kMaxDevices) return nullptr;
    void* p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (p) return p;
    void* q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(fk::scratch)) != hipSuccess || !q) {
        (void)hipGetLastError();
        return nullptr;
    }
    g_scratch_addr[dev].store(q, std::memory_order_release);
    return q;
}

}  // namespace

extern "C" int fk_step_noalloc(const fk_params* p, void* stream, void* f_a, void* f_b, double sigma,
                               double sigma_lo, int64_t step, int64_t nsteps, fk_state* state_out,
                               uint32_t* flags_out)
{
    if (!p || !f_a || !f_b || f_a == f_b || nsteps < 0 || step < 0 || !std::isfinite(sigma) || !std::isfinite(sigma_lo))
        return set_static_error(FK_E_INVALID, "fk_step_noalloc: bad arguments");
    Layout L;
    int rc = derive_layout(p, &L, nullptr);
    if (rc) return set_static_error(rc, "fk_step_noalloc: invalid parameters (fk_validate gives the reason)");
    // the chunk length from the upwind sweep's occupancy; the second-order
    // sweep keeps its short chunks (it is bound by the vector ALU)
    if (p->tile_planes == 0 && p->scheme == FK_SCHEME_UPWIND) choose_planes(p, &L);
    const size_t need = carve_buffers(*p, L, nullptr, nullptr);
    if (need > kScratchBytes)
        return set_static_error(FK_E_INVALID,
                                "fk_step_noalloc: tables, partials and trace ring need more than the 32 MiB scratch "
                                "(fewer x planes, velocity cells or trace records)");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_static_error(FK_E_HIP, "fk_step_noalloc: hipGetDevice failed");
    void* base = scratch_address(dev);
    if (!base) return set_static_error(FK_E_HIP, "fk_step_noalloc: hipGetSymbolAddress of the scratch array failed");

    // a context on the stack: members that own memory stay empty
    fk_ctx c;
    c.p = *p;
    c.L = L;
    c.stream = static_cast<hipStream_t>(stream);
    c.own_f = false;
    c.b.f[0] = f_a;
    c.b.f[1] = f_b;
    carve_buffers(*p, L, static_cast<char*>(base), &c.b);
    hipStream_t s = c.stream;
    // clear the part of the array this call uses (earlier calls leave their
    // contents): a fill kernel, as callers may capture the call in a graph
    const size_t words = (need + 7) / 8;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<size_t>((words + 255) / 256, 2048)), dim3(256), 0, s,
                       static_cast<uint64_t*>(base), words);
    hipLaunchKernelGGL(k_tile_list, dim3(1), dim3(64), 0, s, c.b.tiles, L.n_it, L.ti, p->nvx, L.scheme);
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, c.b.st, sigma, sigma_lo, step);
    if (hipGetLastError() != hipSuccess) return set_static_error(FK_E_HIP, "fk_step_noalloc: a set-up launch failed");
    if (build_tables(&c) || refresh(&c)) return set_static_error(FK_E_HIP, "fk_step_noalloc: a set-up launch failed");
    for (int64_t n = 0; n < nsteps; ++n) {
        enqueue_step(&c, c.cur, s, reversed_step(&c, step + n));
        c.cur ^= 1;
    }
    hipLaunchKernelGGL(k_state_out, dim3(1), dim3(64), 0, s, c.b.st, L.dt, state_out, flags_out);
    if (hipGetLastError() != hipSuccess) return set_static_error(FK_E_HIP, "fk_step_noalloc: a step launch failed");
    return FK_OK;
}

// ================================================================ batch
//
// Independent instances of uneven sizes advanced together.  Each step runs
// two persistent sweep launches, one over the tiles that take the fast body
// and one over the rest (ragged or straddling v_x = 0), so each kernel is
// compiled for one body and keeps its own register budget.  Workgroups pull
// (instance, x chunk, up to 256 / block v_x tiles) work items from an
// atomic counter, largest first, and run the item's tiles side by side.
// One more launch reduces every instance's moments and solves its field
// (a workgroup per instance); the launches of a step are replayed from
// captured HIP graphs.

namespace fk {

constexpr int kBatchThreads = 256;
constexpr int kBatchMaxGroup = kBatchThreads / 64;
// Work classes, one sweep launch each.  Split mode (mode 0) uses four:
// main-body or other tiles, workgroups of 256 threads (v_y blocks of 64,
// 128 or 256 lanes: 4, 2 or 1 tiles side by side) or of 192 threads (one
// tile of a 192-lane block, no idle wave).  Single mode (modes 2 and 3)
// puts every tile in class 4: one launch per step in workgroups of 256 or
// 192 threads, each tile taking its body at run time.
constexpr int kBatchClasses = 5;
enum BatchBody { BODY_FAST = 0, BODY_REST = 1, BODY_ANY = 2 };
__host__ __device__ constexpr int class_body(int k) { return k < 2 ? BODY_FAST : (k < 4 ? BODY_REST : BODY_ANY); }
__host__ __device__ constexpr int class_threads(int k) { return (k == 1 || k == 3) ? 192 : 256; }

struct BatchInst {
    SweepArgs<float> sw[2];   // from buffer 0 / from buffer 1
    FieldArgs fd;
    int block, group, kc, nx, lds_doubles;
};

struct BatchItem {
    int inst, kci, ntiles;
    int tile[kBatchMaxGroup];
};

// sched 0: items taken from an atomic counter (dynamic); sched 1: workgroup
// w takes items w, w + grid, ... of the cost-sorted list (static).  The
// launch bound asks for 4 workgroups of 256 threads per compute unit, i.e.
// at most 128 VGPRs: the kernels that carry the generic body then keep 4
// waves per SIMD instead of 3 (131 -> 127 VGPRs, no spills).  BGK: the
// variant with the collision term (any member has it; members without it
// have zero coefficients and skip it), bounded at 2 workgroups per unit so
// its larger bodies do not spill.
template <int TI, int BODY, bool BGK = false>
__global__ void __launch_bounds__(kBatchThreads, BGK ? 2 : 4) k_batch_sweep(const BatchInst* __restrict__ insts,
                                                               const BatchItem* __restrict__ items,
                                                               int n_items, int* __restrict__ counter, int from,
                                                               int sched)
{
    extern __shared__ double smem[];
    __shared__ int next;
    for (int round = 0;; ++round) {
        if (sched == 0) {
            if (threadIdx.x == 0) next = atomicAdd(counter, 1);
            __syncthreads();
        }
        const int m = sched == 0 ? __builtin_amdgcn_readfirstlane(next) : (int)blockIdx.x + round * (int)gridDim.x;
        __syncthreads();
        if (m >= n_items) break;
        const BatchItem& item = items[m];
        const BatchInst* in = insts + item.inst;
        // B is a multiple of 64, so a wavefront lies in one sub-tile slot:
        // the slot, its tile and everything derived from them are uniform
        // per wave and stay in scalar registers
        const int B = __builtin_amdgcn_readfirstlane(in->block);
        const int sub = __builtin_amdgcn_readfirstlane((int)threadIdx.x / B);
        const int j = (int)threadIdx.x - sub * B;
        const int kci = __builtin_amdgcn_readfirstlane(item.kci);
        const int k0 = kci * in->kc;
        const int np = min(in->kc, in->nx - k0);
        if (sub < __builtin_amdgcn_readfirstlane(item.ntiles)) {
            const int it = __builtin_amdgcn_readfirstlane(item.tile[sub]);
            double* slot = smem + (size_t)sub * in->lds_doubles;
            const SweepArgs<float>& a = in->sw[from];
            if (BODY == BODY_FAST || (BODY == BODY_ANY && tile_is_fast(it, TI, a.nvx)))
                sweep_fast_dispatch<float, TI, BGK>(a, it, kci, slot, j, B);
            else
                sweep_rest<float, TI, BGK>(a, it, kci, slot, j, B);
        } else {
            sweep_idle(np);
        }
    }
}

// counters[0 .. kBatchClasses-1]: the sweep launches' work counters, cleared
// for the next step once the sweeps of this one have finished
__global__ void __launch_bounds__(kFieldThreads) k_batch_field(const BatchInst* __restrict__ insts, int* counters,
                                                               int advance)
{
    __shared__ double sh[2 * kFieldThreads];
    FieldArgs a = insts[blockIdx.x].fd;
    a.advance = advance;
    field_block(a, sh);
    if (blockIdx.x == 0 && threadIdx.x < kBatchClasses) counters[threadIdx.x] = 0;
}

}  // namespace fk

struct fk_batch {
    std::vector<fk_ctx*> inst;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int ti = 8;
    int bgk = 0;                  // 1: a member has the collision term (the sweep variant with it)
    int sched = 0;                // 0 dynamic (atomic counter), 1 static round-robin
    int single = 0;               // 1: one sweep launch per step (class 4 only)
    int single_width = 0;         // threads per workgroup of that launch asked for: 192, or 0 (256)
    int single_threads = 256;     // the width in use
    int occ = 0;                  // workgroups per compute unit (0 = occupancy limit)
    std::vector<char> active;     // instances still stepped
    int n_active = 0;
    int grid = 0;
    size_t lds = 0;
    std::vector<BatchInst> inst_host;
    std::vector<BatchItem> items_host;   // the classes' items, one range each
    int cls_off[kBatchClasses] = {0}, cls_n[kBatchClasses] = {0}, cls_grid[kBatchClasses] = {0};
    BatchInst* d_inst = nullptr;
    BatchItem* d_items = nullptr;
    int* d_counter = nullptr;           // [kBatchClasses] sweep work counters
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_steps = 8;
    int cur = 0;
    int sticky = FK_OK;
    std::string err;
};

namespace {

int bfail(fk_batch* b, hipError_t e, const char* what)
{
    return set_error(&b->err, FK_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define FK_BHIP(b, call)                                     \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return bfail((b), e_, #call);  \
    } while (0)

size_t batch_slice_doubles(int ti, int block, int kc, bool bgk)
{
    return (sweep_lds(ti, block, kc, 4, bgk) + 7) / 8;
}

int batch_threads(const fk_batch* b, int k) { return k == 4 ? b->single_threads : class_threads(k); }

template <int TI, bool BGK>
void batch_launch_sweeps(const fk_batch* b, int from, hipStream_t s)
{
    for (int k = 0; k < kBatchClasses; ++k) {
        if (b->cls_n[k] == 0) continue;
        const BatchItem* items = b->d_items + b->cls_off[k];
        const dim3 grid(b->cls_grid[k]), block(batch_threads(b, k));
        int* ctr = b->d_counter + k;
        switch (class_body(k)) {
        case BODY_FAST:
            hipLaunchKernelGGL((k_batch_sweep<TI, BODY_FAST, BGK>), grid, block, b->lds, s, b->d_inst, items,
                               b->cls_n[k], ctr, from, b->sched);
            break;
        case BODY_REST:
            hipLaunchKernelGGL((k_batch_sweep<TI, BODY_REST, BGK>), grid, block, b->lds, s, b->d_inst, items,
                               b->cls_n[k], ctr, from, b->sched);
            break;
        default:
            hipLaunchKernelGGL((k_batch_sweep<TI, BODY_ANY, BGK>), grid, block, b->lds, s, b->d_inst, items,
                               b->cls_n[k], ctr, from, b->sched);
            break;
        }
    }
}

void batch_launch_step(const fk_batch* b, int from, hipStream_t s)
{
    if (b->bgk) {
        if (b->ti == 4) batch_launch_sweeps<4, true>(b, from, s);
        else batch_launch_sweeps<8, true>(b, from, s);
    } else {
        if (b->ti == 4) batch_launch_sweeps<4, false>(b, from, s);
        else batch_launch_sweeps<8, false>(b, from, s);
    }
    hipLaunchKernelGGL(k_batch_field, dim3(b->n_active), dim3(kFieldThreads), 0, s, b->d_inst, b->d_counter, 1);
}

template <int TI, bool BGK>
hipError_t batch_occupancy_t(int k, int nt, size_t lds, int* occ)
{
    switch (class_body(k)) {
    case BODY_FAST: return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_batch_sweep<TI, BODY_FAST, BGK>, nt, lds);
    case BODY_REST: return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_batch_sweep<TI, BODY_REST, BGK>, nt, lds);
    default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_batch_sweep<TI, BODY_ANY, BGK>, nt, lds);
    }
}

int batch_occupancy(int ti, bool bgk, int k, int nt, size_t lds, int* occ)
{
    hipError_t e;
    if (bgk) e = ti == 4 ? batch_occupancy_t<4, true>(k, nt, lds, occ) : batch_occupancy_t<8, true>(k, nt, lds, occ);
    else e = ti == 4 ? batch_occupancy_t<4, false>(k, nt, lds, occ) : batch_occupancy_t<8, false>(k, nt, lds, occ);
    return e == hipSuccess ? FK_OK : FK_E_HIP;
}

// (Re)build the instance descriptors and the work lists for the members'
// current tiling, and capture the step graphs.
int batch_build(fk_batch* b, int wgs_per_cu)
{
    FK_BHIP(b, hipStreamSynchronize(b->stream));
    b->inst_host.clear();
    b->items_host.clear();
    for (int k = 0; k < kBatchClasses; ++k) b->cls_off[k] = b->cls_n[k] = b->cls_grid[k] = 0;
    b->lds = 0;
    b->occ = wgs_per_cu;
    if (b->active.size() != b->inst.size()) b->active.assign(b->inst.size(), 1);
    std::vector<int> compact;
    for (size_t m = 0; m < b->inst.size(); ++m)
        if (b->active[m]) compact.push_back((int)m);
    b->n_active = (int)compact.size();
    if (b->n_active == 0) return FK_OK;
    if (b->single) {
        // width of the single launch's workgroups.  256 threads hold 4, 2 or
        // 1 tiles of 64-, 128- or 256-lane v_y blocks (a wave idles beside a
        // 192-lane block); 192 threads hold 3, 1 or 1 tiles of 64-, 128- or
        // 192-lane blocks.  256 unless the caller (the autotuner) picked 192
        // and every block fits: on 64 uneven instances, 82% of whose cells
        // have 129-192 v_y lanes, 192 still ran 2% slower than 256.
        int max_block = 0;
        for (int m : compact) max_block = std::max(max_block, b->inst[m]->L.block);
        b->single_threads = (b->single_width == 192 && max_block <= 192) ? 192 : 256;
    }
    std::vector<BatchItem> cls[kBatchClasses];
    for (size_t q = 0; q < compact.size(); ++q) {
        fk_ctx* c = b->inst[compact[q]];
        BatchInst d{};
        d.sw[0] = sweep_args<float>(c, 0);
        d.sw[1] = sweep_args<float>(c, 1);
        d.fd = field_args(c, 1);
        d.block = c->L.block;
        d.group = b->single ? b->single_threads / c->L.block : std::min(kBatchMaxGroup, kBatchThreads / c->L.block);
        d.kc = c->L.kc;
        d.nx = c->p.nx;
        d.lds_doubles = (int)batch_slice_doubles(b->ti, c->L.block, c->L.kc, b->bgk != 0);
        b->lds = std::max(b->lds, (size_t)d.group * d.lds_doubles * 8);
        b->inst_host.push_back(d);
        // tiles by body, in groups of d.group for every x chunk
        std::vector<int> tf, tg;
        for (int it = 0; it < c->L.n_it; ++it)
            (tile_is_fast(it, b->ti, c->p.nvx) ? tf : tg).push_back(it);
        const int narrow = d.group * d.block == 192 ? 1 : 0;   // 192-thread workgroups
        if (b->single) {
            // one class: consecutive tiles in groups of d.group, any body
            for (int kci = 0; kci < c->L.n_kc; ++kci)
                for (int g0 = 0; g0 < c->L.n_it; g0 += d.group) {
                    BatchItem it{};
                    it.inst = (int)q;
                    it.kci = kci;
                    it.ntiles = std::min(c->L.n_it - g0, d.group);
                    for (int u = 0; u < it.ntiles; ++u) it.tile[u] = g0 + u;
                    cls[4].push_back(it);
                }
            continue;
        }
        for (int kci = 0; kci < c->L.n_kc; ++kci)
            for (int body = 0; body < 2; ++body) {
                const std::vector<int>& t = body == 0 ? tf : tg;
                for (size_t g0 = 0; g0 < t.size(); g0 += d.group) {
                    BatchItem it{};
                    it.inst = (int)q;
                    it.kci = kci;
                    it.ntiles = (int)std::min(t.size() - g0, (size_t)d.group);
                    for (int u = 0; u < it.ntiles; ++u) it.tile[u] = t[g0 + u];
                    cls[2 * body + narrow].push_back(it);
                }
            }
    }
    // largest items first
    auto by_cost = [&](const BatchItem& x, const BatchItem& y) {
        auto cost = [&](const BatchItem& t) {
            const fk_ctx* c = b->inst[compact[t.inst]];
            const int np = std::min(c->L.kc, c->p.nx - t.kci * c->L.kc);
            return (double)t.ntiles * np * c->p.nvy;
        };
        return cost(x) > cost(y);
    };
    for (int k = 0; k < kBatchClasses; ++k) {
        std::stable_sort(cls[k].begin(), cls[k].end(), by_cost);
        b->cls_off[k] = (int)b->items_host.size();
        b->cls_n[k] = (int)cls[k].size();
        b->items_host.insert(b->items_host.end(), cls[k].begin(), cls[k].end());
    }
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_inst = nullptr;
    b->d_items = nullptr;
    FK_BHIP(b, hipMalloc(&b->d_inst, sizeof(BatchInst) * b->inst_host.size()));
    FK_BHIP(b, hipMalloc(&b->d_items, sizeof(BatchItem) * b->items_host.size()));
    FK_BHIP(b, hipMemcpy(b->d_inst, b->inst_host.data(), sizeof(BatchInst) * b->inst_host.size(), hipMemcpyHostToDevice));
    FK_BHIP(b, hipMemcpy(b->d_items, b->items_host.data(), sizeof(BatchItem) * b->items_host.size(), hipMemcpyHostToDevice));
    // persistent grids: every compute unit holds wgs_per_cu workgroups (or
    // as many as fit), at most one per item
    int dev = 0, cus = 0;
    FK_BHIP(b, hipGetDevice(&dev));
    FK_BHIP(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    b->grid = 0;
    for (int k = 0; k < kBatchClasses; ++k) {
        if (b->cls_n[k] == 0) continue;
        int occ = 0;
        if (batch_occupancy(b->ti, b->bgk != 0, k, batch_threads(b, k), b->lds, &occ))
            return set_error(&b->err, FK_E_HIP, "hipOccupancyMaxActiveBlocksPerMultiprocessor failed");
        if (occ < 1) return set_error(&b->err, FK_E_INVALID, "batch tiles need more LDS than a compute unit has");
        // the fast classes carry the bulk: they take the tuned occupancy
        const int per_cu = (class_body(k) != BODY_REST && wgs_per_cu > 0) ? std::min(wgs_per_cu, occ) : occ;
        b->cls_grid[k] = std::max(1, std::min(cus * per_cu, b->cls_n[k]));
        b->grid = std::max(b->grid, b->cls_grid[k]);
    }
    // graphs of graph_steps steps from either buffer
    for (auto& g : b->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    for (int start = 0; start < 2; ++start) {
        hipGraph_t g = nullptr;
        FK_BHIP(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
        for (int s = 0; s < b->graph_steps; ++s) batch_launch_step(b, (start + s) & 1, b->cap_stream);
        hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (e != hipSuccess) return bfail(b, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->graph[start], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return bfail(b, e, "hipGraphInstantiate");
    }
    return FK_OK;
}

void batch_release(fk_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (auto& g : b->graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto c : b->inst) release(c);
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

int batch_steps(fk_batch* b, int64_t n)
{
    if (b->n_active == 0) return FK_OK;
    int64_t left = n;
    while (left >= b->graph_steps) {
        FK_BHIP(b, hipGraphLaunch(b->graph[b->cur], b->stream));
        left -= b->graph_steps;
    }
    for (; left > 0; --left) {
        batch_launch_step(b, b->cur, b->stream);
        b->cur ^= 1;
    }
    FK_BHIP(b, hipGetLastError());
    for (size_t m = 0; m < b->inst.size(); ++m)
        if (b->active[m]) b->inst[m]->cur = b->cur;
    return FK_OK;
}

// zero f and the scalars of every member
int batch_reset(fk_batch* b)
{
    for (auto c : b->inst) {
        const size_t fbytes = (size_t)c->L.cells * c->L.elem;
        FK_BHIP(b, hipMemsetAsync(c->b.f[0], 0, fbytes, b->stream));
        FK_BHIP(b, hipMemsetAsync(c->b.f[1], 0, fbytes, b->stream));
        FK_BHIP(b, hipMemsetAsync(c->b.st, 0, sizeof(DevState), b->stream));
        c->history.clear();
        c->drained_step = -1;
        c->sticky = FK_OK;
        if (refresh(c)) return set_error(&b->err, FK_E_HIP, c->err);
    }
    FK_BHIP(b, hipStreamSynchronize(b->stream));
    return FK_OK;
}

}  // namespace

extern "C" int fk_batch_create(const fk_params* params, int n, void* stream, int mode, fk_batch** out)
{
    if (!out || !params || n < 1) return set_error(nullptr, FK_E_INVALID, "bad arguments to fk_batch_create");
    *out = nullptr;
    for (int m = 0; m < n; ++m) {
        Layout L;
        std::string why;
        int rc = derive_layout(&params[m], &L, &why);
        if (rc) return set_error(nullptr, rc, "instance " + std::to_string(m) + ": " + why);
        if (params[m].dtype != FK_F32) return set_error(nullptr, FK_E_INVALID, "batched instances are FK_F32");
        if (L.block > kBatchThreads) return set_error(nullptr, FK_E_INVALID, "batched instances need nvy <= 256");
        if (params[m].scheme != FK_SCHEME_UPWIND)
            return set_error(nullptr, FK_E_INVALID, "batched instances take the first-order scheme");
    }
    fk_batch* b = new (std::nothrow) fk_batch();
    if (!b) return set_error(nullptr, FK_E_OOM, "host allocation failed");
    b->stream = static_cast<hipStream_t>(stream);
    if (mode < 0 || mode > 3) {
        delete b;
        return set_error(nullptr, FK_E_INVALID, "batch mode must be 0, 1, 2 or 3");
    }
    b->single = mode >= 2 ? 1 : 0;
    b->single_width = mode == 3 ? 192 : 0;
    for (int m = 0; m < n; ++m)
        if (params[m].physics_mask & FK_PHYS_BGK) b->bgk = 1;
    int rc = FK_OK;
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) rc = bfail(b, e, "hipStreamCreateWithFlags");
    if (!rc && (e = hipMalloc(&b->d_counter, kBatchClasses * sizeof(int))) != hipSuccess) rc = bfail(b, e, "hipMalloc");
    if (!rc && (e = hipMemset(b->d_counter, 0, kBatchClasses * sizeof(int))) != hipSuccess) rc = bfail(b, e, "hipMemset");
    for (int m = 0; m < n && !rc; ++m) {
        fk_params q = params[m];
        q.tile_rows = b->ti;
        if (q.tile_planes == 0) q.tile_planes = 16;   // the fastest untuned choice on 64 uneven instances
        fk_ctx* c = nullptr;
        rc = create_impl(&q, stream, nullptr, nullptr, &c, true);
        if (rc) b->err = "instance " + std::to_string(m) + ": " + global_error();
        else b->inst.push_back(c);
    }
    if (!rc) rc = batch_build(b, 0);
    if (!rc && mode == 1) {
        // search the tiling (rows, planes) and the persistent grid size on a
        // short run, then start the instances again from f = 0
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = FK_E_HIP;
        int best_ti = 8, best_kc = 32, best_occ = 0, best_sched = 0, best_single = 0, best_width = 0;
        float best_ms = 1e30f;
        const int tis[2] = {4, 8};
        const int kcs[3] = {16, 32, 64};
        const int occs[4] = {2, 3, 4, 0};
        for (int ti : tis)
            for (int kc : kcs)
                for (int occ : occs)
                for (int sched = 0; sched < 2; ++sched)
                for (int variant = 0; variant < 3; ++variant) {   // split; single at 256 or 192 threads
                    if (rc) break;
                    const int single = variant > 0 ? 1 : 0;
                    b->ti = ti;
                    b->sched = sched;
                    b->single = single;
                    b->single_width = variant == 1 ? 256 : (variant == 2 ? 192 : 0);
                    for (auto c : b->inst) {
                        const int kcc = std::min(kc, c->p.nx);
                        if (!rc) rc = retile(c, ti, kcc < 4 ? 0 : kcc);
                    }
                    if (!rc) rc = batch_build(b, occ);
                    if (!rc) rc = batch_steps(b, 2);
                    if (rc) break;
                    (void)hipEventRecord(e0, b->stream);
                    rc = batch_steps(b, 16);
                    (void)hipEventRecord(e1, b->stream);
                    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = FK_E_HIP;
                    float ms = 0;
                    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = FK_E_HIP;
                    if (!rc && ms < best_ms) {
                        best_ms = ms;
                        best_ti = ti;
                        best_kc = kc;
                        best_occ = occ;
                        best_sched = sched;
                        best_single = single;
                        best_width = b->single_width;
                    }
                }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (!rc) {
            b->ti = best_ti;
            b->sched = best_sched;
            b->single = best_single;
            b->single_width = best_width;
            for (auto c : b->inst) {
                const int kcc = std::min(best_kc, c->p.nx);
                if (!rc) rc = retile(c, best_ti, kcc < 4 ? 0 : kcc);
            }
            if (!rc) rc = batch_build(b, best_occ);
            if (!rc) rc = batch_reset(b);
            b->cur = 0;
            for (auto c : b->inst) c->cur = 0;
        }
    }
    if (rc) {
        std::string m = b->err;
        for (auto c : b->inst)
            if (!c->err.empty()) m += " / " + c->err;
        batch_release(b);
        return set_error(nullptr, rc, m.empty() ? std::string("batch creation failed") : m);
    }
    *out = b;
    return FK_OK;
}

extern "C" int fk_batch_destroy(fk_batch* b)
{
    if (!b) return FK_E_INVALID;
    batch_release(b);
    return FK_OK;
}

extern "C" int fk_batch_step(fk_batch* b, int64_t n)
{
    if (!b || n < 0) return FK_E_INVALID;
    if (b->sticky) return b->sticky;
    return batch_steps(b, n);
}

extern "C" int fk_batch_sync(fk_batch* b, int* first_bad)
{
    if (!b) return FK_E_INVALID;
    FK_BHIP(b, hipStreamSynchronize(b->stream));
    if (first_bad) *first_bad = -1;
    for (size_t m = 0; m < b->inst.size(); ++m) {
        if (!b->active[m]) continue;
        int rc = fk_sync(b->inst[m]);
        if (rc) {
            b->sticky = rc;
            if (first_bad) *first_bad = (int)m;
            return set_error(&b->err, rc, "instance " + std::to_string(m) + ": " + b->inst[m]->err);
        }
    }
    return FK_OK;
}

extern "C" int fk_batch_get(fk_batch* b, int i, fk_ctx** view)
{
    if (!b || !view || i < 0 || i >= (int)b->inst.size()) return FK_E_INVALID;
    *view = b->inst[i];
    return FK_OK;
}

extern "C" int fk_batch_info(const fk_batch* b, fk_batch_info_t* out)
{
    if (!b || !out) return FK_E_INVALID;
    out->n = (int)b->inst.size();
    out->tile_rows = b->ti;
    out->grid = b->grid;
    out->items = (int)b->items_host.size();
    out->lds_bytes = (int64_t)b->lds;
    int64_t cells = 0;
    for (auto c : b->inst) cells += c->L.cells;
    out->cells = cells;
    out->tile_planes = b->inst.empty() ? 0 : b->inst[0]->L.kc;
    out->schedule = b->sched;
    int launches = 0;
    for (int k = 0; k < kBatchClasses; ++k) launches += b->cls_n[k] > 0;
    out->sweep_launches = launches;
    out->single_threads = b->single ? b->single_threads : 0;
    return FK_OK;
}

extern "C" const char* fk_batch_last_error(const fk_batch* b) { return b ? b->err.c_str() : global_error(); }


extern "C" int fk_read_profile(fk_ctx* c, int npts, double* out, int dst_on_device)
{
    if (!c || !out || npts < 2) return FK_E_INVALID;
    double* d = out;
    double* tmp = nullptr;
    if (!dst_on_device) {
        FK_HIP(c, hipMalloc(&tmp, (size_t)npts * sizeof(double)));
        d = tmp;
    }
    hipLaunchKernelGGL(k_profile, dim3((npts + 255) / 256), dim3(256), 0, c->stream, c->b.ne, c->b.st, c->p.nx,
                       c->L.dx, c->p.length_m, npts, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && tmp) e = hipMemcpyAsync(out, tmp, (size_t)npts * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(c, e, "fk_read_profile");
    return FK_OK;
}

extern "C" int fk_warm_start(fk_ctx* c, const double* profile, int npts, int src_on_device, double t_ev,
                             int64_t step)
{
    if (!c || !profile || npts < 2 || !(t_ev > 0) || step < 0) return FK_E_INVALID;
    FK_HIP(c, hipStreamSynchronize(c->stream));
    std::vector<double> host(npts);
    if (src_on_device)
        FK_HIP(c, hipMemcpy(host.data(), profile, npts * sizeof(double), hipMemcpyDeviceToHost));
    else
        std::memcpy(host.data(), profile, npts * sizeof(double));
    for (double v : host)
        if (!std::isfinite(v)) return set_error(&c->err, FK_E_INVALID, "profile has non-finite values");
    double* dprof = nullptr;
    FK_HIP(c, hipMalloc(&dprof, npts * sizeof(double)));
    hipError_t e = hipMemcpyAsync(dprof, host.data(), npts * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_warm_norm, dim3(1), dim3(kFieldThreads), 0, c->stream, c->p.nvx, c->p.nvy, c->L.dvx,
                           c->L.dvy, t_ev, c->b.consts + 4);
        const size_t cells = (size_t)c->L.cells;
        const dim3 grid((unsigned)((cells + 255) / 256));
        if (c->L.elem == 4)
            hipLaunchKernelGGL(k_warm_start<float>, grid, dim3(256), 0, c->stream, static_cast<float*>(c->b.f[c->cur]),
                               dprof, npts, c->p.length_m, c->p.nx, c->p.nvx, c->p.nvy, c->L.dx, c->L.dvx, c->L.dvy,
                               t_ev, c->b.consts + 4);
        else
            hipLaunchKernelGGL(k_warm_start<double>, grid, dim3(256), 0, c->stream, static_cast<double*>(c->b.f[c->cur]),
                               dprof, npts, c->p.length_m, c->p.nx, c->p.nvx, c->p.nvy, c->L.dx, c->L.dvx, c->L.dvy,
                               t_ev, c->b.consts + 4);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dprof);
    if (e != hipSuccess) return hip_fail(c, e, "fk_warm_start");
    return fk_write_state(c, nullptr, 0, host[0], 0.0, step);
}

extern "C" int fk_batch_retire(fk_batch* b, const int* idx, int n)
{
    if (!b || (n && !idx)) return FK_E_INVALID;
    for (int q = 0; q < n; ++q) {
        if (idx[q] < 0 || idx[q] >= (int)b->inst.size()) return set_error(&b->err, FK_E_INVALID, "bad instance index");
        b->active[idx[q]] = 0;
    }
    // instances are independent: once the flagged ones are retired the rest
    // may go on (the next fk_batch_sync checks the active ones again)
    b->sticky = FK_OK;
    return batch_build(b, b->occ);
}
