// fk_field.h -- the per-step reduction and field kernel bodies: the plane
// sums of the sweep's tile partials, then one workgroup that reduces the wall
// partials, updates sigma (Eq 18), solves the 1D field and prepares the next
// step (emission row scale, Courant numbers, trace record).
#pragma once

#include "fk_kernels.h"

namespace fk {

// Compensated sum (Neumaier): the value is s + c, with c collecting the
// rounding error of every addition into s.
struct CSum {
    double s = 0.0, c = 0.0;
};

__device__ __forceinline__ void cadd(CSum& a, double x)
{
    const double t = a.s + x;
    a.c += fabs(a.s) >= fabs(x) ? (a.s - t) + x : (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ CSum cmerge(CSum a, const CSum& b)
{
    cadd(a, b.s);
    a.c += b.c;
    return a;
}

__device__ __forceinline__ double cvalue(const CSum& a) { return a.s + a.c; }

// A compensated sum across the 64 lanes in the fixed order of wave_total
// (lane 63 holds the total; lanes shifted in from outside a row add zero).
template <int CTRL, int ROWS>
__device__ __forceinline__ void cmerge_dpp(CSum& v)
{
    CSum o;
    o.s = dpp_move<CTRL, ROWS>(v.s);
    o.c = dpp_move<CTRL, ROWS>(v.c);
    v = cmerge(v, o);
}

__device__ __forceinline__ CSum wave_csum(CSum v)
{
    cmerge_dpp<0x111, 0xf>(v);
    cmerge_dpp<0x112, 0xf>(v);
    cmerge_dpp<0x114, 0xf>(v);
    cmerge_dpp<0x118, 0xf>(v);
    cmerge_dpp<0x142, 0xa>(v);
    cmerge_dpp<0x143, 0xc>(v);
    CSum r;
    r.s = lane63(v.s);
    r.c = lane63(v.c);
    return r;
}

// Plane sums over the v_x tiles, one thread per x plane (coalesced over
// consecutive planes), tiles added in order with compensation: the same
// sums the field workgroup forms itself when it is given no plane_sum.
__device__ __forceinline__ void plane_sums(const double* __restrict__ part_n, int nx, int n_it,
                                           double* __restrict__ plane_sum)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nx) return;
    CSum s;
#pragma unroll 16
    for (int u = 0; u < n_it; ++u) cadd(s, part_n[(size_t)u * nx + k]);
    plane_sum[k] = cvalue(s);
}

// ---------------------------------------------------------------- field

struct FieldArgs {
    const double* __restrict__ plane_sum;   // [nx] plane sums already reduced over the tiles, or null
    const double* __restrict__ part_n;      // [n_it][nx] plane sums of the v_x tiles
    const double* __restrict__ part_wall;   // [n_it][2]  wall primary, wall secondary
    const double* __restrict__ part_top;    // [n_it]     flux through x = L
    const double* __restrict__ part_lv;     // [nwg]      velocity-box outflow
    const double* __restrict__ part_abs;    // [n_it][2]  absorbed at the wall and at x = L by a reversed
                                            //            second-order step (read when abs_from_sweep)
    const double* __restrict__ consts;  // zsum, srcnorm, injected per step, Eq 15 prefactor
    double* __restrict__ ne;
    double* __restrict__ ex;
    double* __restrict__ dxk;
    double* __restrict__ nudt;      // [nx] out: nu_ee dt per plane (collision term)
    double* __restrict__ nudt_n;    // [nx] out: nu_ee dt n_e per plane
    DevState* __restrict__ st;
    fk_state* __restrict__ ring;
    int nx, n_it, nwg, advance;
    uint32_t mask;
    int emission_norm, trace_stride, trace_cap;
    double dx, dv2, dt, dvx, ex_ext;
    double nudt_per_n;              // dt nu_ee / n_e of Eq 4 (0: no collision term)
    double r_refl;                  // elastic (specular) share of the wall reflection R_f
    double r_inel;                  // inelastic share of R_f, re-emitted in the Eq 15 shape
    int abs_from_sweep;             // 1: the step's x sweep transported f after the velocity sweeps
                                    //    (reversed second-order step); its absorbed fluxes are in part_abs
};

// Reduction of the moment partials of the new f over the v_x tiles (fixed
// order), the 1D field solve and the wall bookkeeping; one workgroup of
// kFieldThreads threads.  Thread t owns a contiguous segment of x planes and
// keeps their densities in registers.  sh holds 2 * kFieldThreads doubles.
constexpr int kFieldSegMax = 8;

// Plane sums of planes kb .. kb + SEG - 1 (tiles in order) into n[0 .. SEG).
// Either read from the reduced plane sums or added here from the tile
// partials, four tiles' loads in flight before their adds.
template <int SEG>
__device__ __forceinline__ void plane_densities(const FieldArgs& a, int kb, double (&n)[kFieldSegMax])
{
    const int klast = a.nx - 1;
#pragma unroll
    for (int q = 0; q < kFieldSegMax; ++q) n[q] = 0.0;
    if (a.plane_sum) {
#pragma unroll
        for (int q = 0; q < SEG; ++q) n[q] = a.plane_sum[min(kb + q, klast)];
        return;
    }
    CSum acc[SEG];
    constexpr int kChunk = 4;
    for (int u0 = 0; u0 < a.n_it; u0 += kChunk) {
        double v[kChunk][SEG];
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            const double* row = a.part_n + (size_t)min(u0 + c, a.n_it - 1) * a.nx;
#pragma unroll
            for (int q = 0; q < SEG; ++q) v[c][q] = row[min(kb + q, klast)];
        }
#pragma unroll
        for (int c = 0; c < kChunk; ++c)
            if (u0 + c < a.n_it) {
#pragma unroll
                for (int q = 0; q < SEG; ++q) cadd(acc[q], v[c][q]);
            }
    }
#pragma unroll
    for (int q = 0; q < SEG; ++q) n[q] = cvalue(acc[q]);
}

__device__ __forceinline__ void field_block(const FieldArgs& a, double* sh)
{
    const int t = threadIdx.x;
    const int T = blockDim.x;
    const int lane = t & 63, wave = t >> 6, nw = T >> 6;
    const int seg = (a.nx + T - 1) / T;
    const int kb = min(t * seg, a.nx), ke = min(kb + seg, a.nx);
    const DevState old = *a.st;     // issued early: needed after the scans
    const double zsum = a.consts[0], inj_step = a.consts[2], emit_pref = a.consts[3];

    // Every global load comes before the first global store: one counter
    // tracks both, so a load waited for after a store waits for the store
    // too.  Loads use clamped indices and stay unconditional (values past
    // the thread's segment are dropped).
    //
    // electron density per plane: sum over the v_x tiles in tile order
    double nloc[kFieldSegMax];
    double local = 0.0;
    CSum ltot;                      // the same sum, compensated, for the electron total
    const bool in_regs = seg <= kFieldSegMax;
    if (in_regs) {
        if (seg == 1) plane_densities<1>(a, kb, nloc);
        else if (seg == 2) plane_densities<2>(a, kb, nloc);
        else if (seg <= 4) plane_densities<4>(a, kb, nloc);
        else plane_densities<kFieldSegMax>(a, kb, nloc);
#pragma unroll
        for (int q = 0; q < kFieldSegMax; ++q)
            if (kb + q < ke) {
                nloc[q] *= a.dv2;
                local += nloc[q];
                cadd(ltot, nloc[q]);
            }
    } else {
        for (int k = kb; k < ke; ++k) {
            CSum sk;
            if (a.plane_sum) cadd(sk, a.plane_sum[k]);
            else
                for (int u = 0; u < a.n_it; ++u) cadd(sk, a.part_n[(size_t)u * a.nx + k]);
            a.ne[k] = cvalue(sk) * a.dv2;
            local += cvalue(sk) * a.dv2;
            cadd(ltot, cvalue(sk) * a.dv2);
        }
    }
    // wall, top, velocity-box and absorbed partials: compensated sums.  The
    // n_it tile partials go to wave 0, strided over its lanes (the other
    // waves hold zeros, which leave a compensated sum unchanged); the nwg
    // box-loss partials (one per sweep workgroup, thousands) are strided
    // over the whole workgroup.
    constexpr int kParts = 6;       // primary, secondary, top, box loss, absorbed at wall / top
    CSum part[kParts];
    if (wave == 0) {
        for (int u = lane; u < a.n_it; u += 64) {
            cadd(part[0], a.part_wall[2 * u]);
            cadd(part[1], a.part_wall[2 * u + 1]);
            cadd(part[2], a.part_top[u]);
            if (a.abs_from_sweep) {
                cadd(part[4], a.part_abs[2 * u]);
                cadd(part[5], a.part_abs[2 * u + 1]);
            }
        }
    }
    if (a.advance) {
        // four loads in flight per thread before their adds
        for (int w0 = t; w0 < a.nwg; w0 += T * 4) {
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = a.part_lv[min(w0 + T * q, a.nwg - 1)];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (w0 + T * q < a.nwg) cadd(part[3], v[q]);
        }
    }

    // exclusive prefix of the segment sums over the workgroup: wave scans,
    // then a scan of the wave totals
    const double incl = wave_total(local);     // inclusive scan over the wave
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 0.0;
    double* wtot = sh;              // [nw]
    double* red = sh + 64;          // [nw][kParts + 1][2]: (s, c) pairs of the partials and the electron total
    double* tots = red + 16 * (kParts + 1) * 2 + 32;   // [kParts + 1] the totals over the waves
    if (lane == 63) wtot[wave] = incl;
    ltot = wave_csum(ltot);
    if (wave == 0) {
        part[0] = wave_csum(part[0]);
        part[1] = wave_csum(part[1]);
        part[2] = wave_csum(part[2]);
        if (a.abs_from_sweep) {
            part[4] = wave_csum(part[4]);
            part[5] = wave_csum(part[5]);
        }
    }
    part[3] = wave_csum(part[3]);
    if (lane == 0) {
        double* r = red + wave * (kParts + 1) * 2;
#pragma unroll
        for (int m = 0; m < kParts; ++m) {
            r[2 * m] = part[m].s;
            r[2 * m + 1] = part[m].c;
        }
        r[2 * kParts] = ltot.s;
        r[2 * kParts + 1] = ltot.c;
    }
    __syncthreads();
    double wave_below = 0.0;
    for (int w = 0; w < wave; ++w) wave_below += wtot[w];
    const double below0 = wave_below + excl;
    // the partials and the electron total over the waves, in order: thread m
    // of wave 0 merges quantity m
    if (t <= kParts) {
        CSum acc;
        for (int w = 0; w < nw; ++w) {
            CSum x;
            x.s = red[w * (kParts + 1) * 2 + 2 * t];
            x.c = red[w * (kParts + 1) * 2 + 2 * t + 1];
            acc = cmerge(acc, x);
        }
        tots[t] = cvalue(acc);
    }
    __syncthreads();
    double tot[kParts + 1];
#pragma unroll
    for (int m = 0; m <= kParts; ++m) tot[m] = tots[m];
    const double pe = tot[0], see = tot[1], top = tot[2], lv = tot[3];
    const double total = tot[kParts];

    // electrons the step's x sweep absorbed at the wall and let out at x = L:
    // the fluxes of f^n, or on a reversed second-order step those of the
    // array after the velocity sweeps
    double g_abs = old.g_pe, top_abs = old.g_top;
    if (a.abs_from_sweep && (a.mask & FK_PHYS_X)) {
        g_abs = tot[4] * a.dv2;
        top_abs = tot[5] * a.dv2;
    }
    double sig = old.sigma, sig_lo = old.sigma_lo;
    if (a.advance) {
        // Eq 18 with the fluxes of f^n, Neumaier-compensated across steps;
        // reflected electrons of both shares leave the wall again
        const double inc = kE * a.dt * (old.g_see + (a.r_refl + a.r_inel) * old.g_pe - g_abs);
        const double s = sig + inc;
        if (fabs(sig) >= fabs(inc)) sig_lo += (sig - s) + inc;
        else sig_lo += (inc - s) + sig;
        sig = s;
    }
    const double sigma_now = sig + sig_lo;

    // E_x at the cell centres: sigma / 2 eps0 minus the electron charge below
    double run = below0, cmax = 0.0, bmax = 0.0;
    const double e_wall = sigma_now / (2.0 * kEps0), e_per_n = kE / kEps0 * a.dx;
    const double d_per_e = (a.mask & FK_PHYS_VX) ? -kE / kMe * a.dt / a.dvx : 0.0;   // Courant number per V/m
    auto field_at = [&](int k, double nk) {
        double e = 0.0;
        if (a.mask & FK_PHYS_SELF_FIELD)
            e = (a.mask & FK_PHYS_NO_SPACE_CHARGE) ? e_wall : e_wall - e_per_n * (run + 0.5 * nk);
        e += a.ex_ext;
        a.ex[k] = e;
        const double d = d_per_e * e;
        a.dxk[k] = d;
        cmax = fmax(cmax, fabs(d));
        if (a.nudt_per_n != 0.0) {
            // collision term of the next step (Eq 3-4): nu_ee is linear in n_e
            const double b = a.nudt_per_n * nk;
            a.nudt[k] = b;
            a.nudt_n[k] = b * nk;
            bmax = fmax(bmax, b);
        }
        run += nk;
    };
    if (in_regs) {
#pragma unroll
        for (int q = 0; q < kFieldSegMax; ++q)
            if (kb + q < ke) {
                a.ne[kb + q] = nloc[q];
                field_at(kb + q, nloc[q]);
            }
    } else {
        for (int k = kb; k < ke; ++k) field_at(k, a.ne[k]);
    }
    cmax = wave_max_nonneg(cmax);
    bmax = wave_max_nonneg(bmax);
    double* redm = red + 16 * (kParts + 1) * 2;   // [nw][2]
    if (lane == 0) {
        redm[wave * 2 + 0] = cmax;
        redm[wave * 2 + 1] = bmax;
    }
    __syncthreads();
    if (t == 0) {
        cmax = bmax = 0.0;
        for (int w = 0; w < nw; ++w) {
            cmax = fmax(cmax, redm[w * 2 + 0]);
            bmax = fmax(bmax, redm[w * 2 + 1]);
        }
    }

    if (t == 0) {
        const bool x_on = a.mask & FK_PHYS_X;
        const bool see_on = x_on && (a.mask & FK_PHYS_SEE);
        const double g_pe = x_on ? pe * a.dv2 : 0.0;
        const double g_see = see_on ? see * a.dv2 * (1.0 - a.r_refl - a.r_inel) : 0.0;   // 1 - R_f induce SEE
        const double g_top = x_on ? top * a.dv2 : 0.0;
        // the emission shape carries the secondaries and the inelastically
        // reflected electrons
        const double g_shape = g_see + (x_on ? a.r_inel * g_pe : 0.0);
        double gscale = 0.0;
        if (x_on) {
            if (a.emission_norm == FK_EMIT_DISCRETE) gscale = zsum > 0.0 ? g_shape / zsum : 0.0;
            else gscale = g_shape * emit_pref;
        }
        const double emitted = gscale * zsum + (x_on ? a.r_refl * g_pe : 0.0);
        const double n_total = total * a.dx;
        const double loss_v = a.advance ? lv * a.dx * a.dv2 : 0.0;
        double resid = 0.0;
        if (a.advance) {
            const double inj = (a.mask & FK_PHYS_SRC) ? inj_step : 0.0;
            resid = (n_total - old.n_total) - (a.dt * (old.emitted - g_abs - top_abs) + inj - loss_v);
        }
        DevState ns = old;
        ns.step = old.step + (a.advance ? 1 : 0);
        ns.sigma = sig;
        ns.sigma_lo = sig_lo;
        ns.g_pe = g_pe;
        ns.g_see = g_see;
        ns.g_top = g_top;
        ns.emitted = emitted;
        ns.loss_v = loss_v;
        ns.n_total = n_total;
        ns.resid = resid;
        ns.gscale = gscale;
        ns.courant_vx_max = fmax(old.courant_vx_max, cmax);
        if (cmax > 1.0 || bmax > 1.0) ns.flags |= kFlagCfl;
        if (!isfinite(n_total) || !isfinite(g_pe) || !isfinite(g_see) || !isfinite(g_top) ||
            !isfinite(sigma_now))
            ns.flags |= kFlagNonfinite;
        *a.st = ns;
        // trace slot: 32-bit arithmetic while the step count fits
        int64_t rec = -1;
        if (ns.step >= 0 && ns.step <= 0xffffffffLL) {
            const unsigned st32 = (unsigned)ns.step, q = st32 / (unsigned)a.trace_stride;
            if (q * (unsigned)a.trace_stride == st32) rec = q % (unsigned)a.trace_cap;
        } else if (ns.step % a.trace_stride == 0) {
            rec = (ns.step / a.trace_stride) % a.trace_cap;
        }
        if (rec >= 0) {
            fk_state r;
            r.step = ns.step;
            r.t = (double)ns.step * a.dt;
            r.sigma = sig;
            r.sigma_lo = sig_lo;
            r.g_pe = g_pe;
            r.g_see = g_see;
            r.g_top = g_top;
            r.emitted = emitted;
            r.loss_v = loss_v;
            r.n_total = n_total;
            r.resid = resid;
            a.ring[rec] = r;
        }
    }
}

}  // namespace fk
