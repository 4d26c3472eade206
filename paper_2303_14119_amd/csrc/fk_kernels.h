// fk_kernels.h -- the device kernels of one time step, shared by the single
// context and the batched driver.
//
// Step n (Section 2 of the paper), from f^n and sigma^n:
//   field kernel (one workgroup): n_k from the moment partials of f^n,
//     E_x from the 1D Gauss law with E_x(0) = sigma^n / 2 eps0, the v_x
//     Courant number of every plane, the wall fluxes of f^n (Eq 13-14),
//     sigma^{n+1} by Eq 18 and the scale of the emission row (Eq 15-16).
//   sweep kernel (all tiles): x, v_x, v_y upwind transport and the band
//     source fused in one pass over f, writing f^{n+1} and its moment
//     partials (plane sums, wall and top fluxes, velocity-box outflow).
#pragma once

#include "fk_internal.h"

namespace fk {

// Workgroup -> tile map.  Consecutive workgroup ids are dealt round-robin
// to the 8 XCDs; remap so each XCD works on a contiguous range of tiles
// (neighbouring v_x tiles of the same x planes share their halo rows in that
// XCD's L2).
__device__ __forceinline__ int xcd_remap(int wg, int nwg)
{
    const int per = nwg >> 3, rem = nwg & 7;
    const int xcd = wg & 7, pos = wg >> 3;
    return xcd < rem ? xcd * (per + 1) + pos : rem * (per + 1) + (xcd - rem) * per + pos;
}

// Centre of velocity cell i of n on [-vmax, vmax]: (i + 1/2 - n/2) dv.  The
// factor is exact, so the middle cell of an odd grid is exactly 0 and the
// signs that select wall, emission and source cells never depend on rounding.
__device__ __forceinline__ double cell_v(int i, int n, double dv) { return (i + 0.5 - 0.5 * n) * dv; }

// Sum over the 64 lanes of a wavefront; lane 0 holds a result that does not
// depend on scheduling (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fixed-order sum over a workgroup of blockDim.x (a power of two, <= 1024)
// threads; sh holds blockDim.x doubles.  Every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- sweep

template <typename T>
struct SweepArgs {
    const T* __restrict__ fin;
    T* __restrict__ fout;
    const double* __restrict__ dxk;     // [nx] v_x Courant number per plane (0 if v_x advection off)
    const double* __restrict__ srck;    // [nx] source coefficient per plane (0 outside the band)
    const T* __restrict__ fsrc;         // [nvx][nvy] normalised source VDF
    const double* __restrict__ ghat;    // [nvx][nvy] emission shape
    const double* __restrict__ delta;   // [nvx][nvy] SEY
    const DevState* __restrict__ st;    // gscale of this step
    double* __restrict__ part_n;        // [nx][n_it]
    double* __restrict__ part_wall;     // [n_it][2]
    double* __restrict__ part_top;      // [n_it]
    double* __restrict__ part_lv;       // [nwg]
    int nx, nvx, nvy, n_it, kc;
    double dvx, dt_dx;                  // v_x of row i is cell_v(i, nvx, dvx)
    double dy;                          // signed v_y Courant number
    int x_on;
    int tile_base, nwg_total;           // batched launches: first tile of the instance, grid size
};

// One workgroup owns v_x rows [i0, i0+TI) for all v_y columns (one thread per
// column) and marches over x planes [k0, k0+kc).  Each thread keeps three x
// planes of its rows (plus one halo row on each side) in registers:
//   x sweep     upwind on sign(v_x) -- the plane below or above, in registers;
//   v_x sweep   upwind on sign(a_x) -- the neighbouring row, in registers;
//   v_y sweep   upwind on sign(a_y) -- the neighbouring column, through LDS;
//   source      added on the planes overlapping the band.
// f is read once and written once per cell (plus halo re-reads that mostly
// hit L2).
template <typename T, int TI>
__device__ __forceinline__ void sweep_tile(const SweepArgs<T>& a, int wg, double* smem)
{
    const int it = wg % a.n_it;
    const int kci = wg / a.n_it;
    const int i0 = it * TI;
    const int k0 = kci * a.kc;
    const int k1 = min(k0 + a.kc, a.nx);
    const int j = threadIdx.x;
    const int B = blockDim.x;
    const int nw = B >> 6;
    const int lane = j & 63, wave = j >> 6;
    const bool jok = j < a.nvy;
    const int W = B + 2;
    const size_t plane = (size_t)a.nvx * a.nvy;

    T* xb = reinterpret_cast<T*>(smem);                       // [2][TI][W]
    double* wsum = reinterpret_cast<double*>(xb + 2 * TI * W); // [kc][nw]
    double* red = wsum + a.kc * nw;                           // [nw][4]

    for (int m = j; m < 2 * TI; m += B) {
        xb[m * W] = T(0);
        xb[m * W + W - 1] = T(0);
    }

    bool ok[TI + 2];
    T c[TI + 2];
#pragma unroll
    for (int r = 0; r < TI + 2; ++r) {
        const int i = i0 - 1 + r;
        ok[r] = jok && i >= 0 && i < a.nvx;
        const double v = cell_v(i, a.nvx, a.dvx);
        c[r] = (a.x_on && ok[r]) ? T(v * a.dt_dx) : T(0);
    }

    T fm[TI + 2], fc[TI + 2], fp[TI + 2];
    const T* __restrict__ fin = a.fin + j;
    if (k0 == 0) {
        // below the dielectric: the emission row of this step (Eq 15)
        const double gs = a.st->gscale;
#pragma unroll
        for (int r = 0; r < TI + 2; ++r) {
            const int i = i0 - 1 + r;
            fm[r] = ok[r] ? T(gs * a.ghat[(size_t)i * a.nvy + j]) : T(0);
        }
    } else {
        const T* p = fin + (size_t)(k0 - 1) * plane;
#pragma unroll
        for (int r = 0; r < TI + 2; ++r) fm[r] = ok[r] ? p[(size_t)(i0 - 1 + r) * a.nvy] : T(0);
    }
    {
        const T* p = fin + (size_t)k0 * plane;
#pragma unroll
        for (int r = 0; r < TI + 2; ++r) fc[r] = ok[r] ? p[(size_t)(i0 - 1 + r) * a.nvy] : T(0);
    }

    double lv = 0.0, spe = 0.0, ssee = 0.0, stop = 0.0;
    const T dy = T(a.dy);

    for (int k = k0; k < k1; ++k) {
        if (k + 1 < a.nx) {
            const T* p = fin + (size_t)(k + 1) * plane;
#pragma unroll
            for (int r = 0; r < TI + 2; ++r) fp[r] = ok[r] ? p[(size_t)(i0 - 1 + r) * a.nvy] : T(0);
        } else {
#pragma unroll
            for (int r = 0; r < TI + 2; ++r) fp[r] = T(0);   // nothing enters at x = L (Eq 17)
        }

        // x sweep: f' = f - c (f - f_up), upwind on the sign of v_x
        T f1[TI + 2];
#pragma unroll
        for (int r = 0; r < TI + 2; ++r) {
            const T diff = c[r] > T(0) ? (fc[r] - fm[r]) : (fp[r] - fc[r]);
            f1[r] = fc[r] - c[r] * diff;
        }

        // v_x sweep by a_x(x_k): upwind on the sign of the plane's Courant number
        const T d = T(a.dxk[k]);
        T f2[TI];
#pragma unroll
        for (int r = 1; r <= TI; ++r) {
            const T diff = d > T(0) ? (f1[r] - f1[r - 1]) : (f1[r + 1] - f1[r]);
            f2[r - 1] = ok[r] ? f1[r] - d * diff : T(0);
        }
        if (d > T(0)) {
#pragma unroll
            for (int r = 1; r <= TI; ++r)
                if (ok[r] && i0 - 1 + r == a.nvx - 1) lv += (double)d * (double)f1[r];
        } else if (d < T(0)) {
#pragma unroll
            for (int r = 1; r <= TI; ++r)
                if (ok[r] && i0 - 1 + r == 0) lv -= (double)d * (double)f1[r];
        }

        // v_y sweep by a_y: the neighbouring column comes from LDS
        T* buf = xb + (k & 1) * TI * W;
#pragma unroll
        for (int r = 0; r < TI; ++r) buf[r * W + j + 1] = f2[r];
        __syncthreads();
        T f3[TI];
#pragma unroll
        for (int r = 0; r < TI; ++r) {
            const T left = buf[r * W + j], right = buf[r * W + j + 2];
            const T diff = dy > T(0) ? (f2[r] - left) : (right - f2[r]);
            f3[r] = jok ? f2[r] - dy * diff : T(0);
        }
        if (dy > T(0) && j == a.nvy - 1) {
#pragma unroll
            for (int r = 0; r < TI; ++r) lv += (double)dy * (double)f2[r];
        } else if (dy < T(0) && j == 0) {
#pragma unroll
            for (int r = 0; r < TI; ++r) lv -= (double)dy * (double)f2[r];
        }

        // band source (Eq 7)
        const double s = a.srck[k];
        if (s != 0.0) {
            const T ts = T(s);
            const T* sp = a.fsrc + j;
#pragma unroll
            for (int r = 0; r < TI; ++r)
                if (ok[r + 1]) f3[r] += ts * sp[(size_t)(i0 + r) * a.nvy];
        }

        T* op = a.fout + (size_t)k * plane + j;
#pragma unroll
        for (int r = 0; r < TI; ++r)
            if (ok[r + 1]) op[(size_t)(i0 + r) * a.nvy] = f3[r];

        // moments of f^{n+1}
        double sn = 0.0;
#pragma unroll
        for (int r = 0; r < TI; ++r) sn += (double)f3[r];
        sn = wave_sum(sn);
        if (lane == 0) wsum[(k - k0) * nw + wave] = sn;
        if (k == 0) {
#pragma unroll
            for (int r = 0; r < TI; ++r) {
                const int i = i0 + r;
                const double v = cell_v(i, a.nvx, a.dvx);
                if (ok[r + 1] && v < 0.0) {
                    const double g = -v * (double)f3[r];
                    spe += g;
                    ssee += a.delta[(size_t)i * a.nvy + j] * g;
                }
            }
        }
        if (k == a.nx - 1) {
#pragma unroll
            for (int r = 0; r < TI; ++r) {
                const double v = cell_v(i0 + r, a.nvx, a.dvx);
                if (ok[r + 1] && v > 0.0) stop += v * (double)f3[r];
            }
        }

#pragma unroll
        for (int r = 0; r < TI + 2; ++r) {
            fm[r] = fc[r];
            fc[r] = fp[r];
        }
    }

    __syncthreads();
    for (int kk = j; kk < k1 - k0; kk += B) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += wsum[kk * nw + w];
        a.part_n[(size_t)(k0 + kk) * a.n_it + it] = s;
    }
    lv = wave_sum(lv);
    spe = wave_sum(spe);
    ssee = wave_sum(ssee);
    stop = wave_sum(stop);
    if (lane == 0) {
        red[wave * 4 + 0] = lv;
        red[wave * 4 + 1] = spe;
        red[wave * 4 + 2] = ssee;
        red[wave * 4 + 3] = stop;
    }
    __syncthreads();
    if (j == 0) {
        double t0 = 0, t1 = 0, t2 = 0, t3 = 0;
        for (int w = 0; w < nw; ++w) {
            t0 += red[w * 4 + 0];
            t1 += red[w * 4 + 1];
            t2 += red[w * 4 + 2];
            t3 += red[w * 4 + 3];
        }
        a.part_lv[wg] = t0;
        if (k0 == 0) {
            a.part_wall[it * 2 + 0] = t1;
            a.part_wall[it * 2 + 1] = t2;
        }
        if (k1 == a.nx) a.part_top[it] = t3;
    }
}

// Moment partials of the current f without advancing it (after create and
// fk_write_state); same tiling and output slots as the sweep.
template <typename T, int TI>
__device__ __forceinline__ void moments_tile(const SweepArgs<T>& a, int wg, double* smem)
{
    const int it = wg % a.n_it;
    const int kci = wg / a.n_it;
    const int i0 = it * TI;
    const int k0 = kci * a.kc;
    const int k1 = min(k0 + a.kc, a.nx);
    const int j = threadIdx.x;
    const int nw = blockDim.x >> 6;
    const int lane = j & 63, wave = j >> 6;
    const bool jok = j < a.nvy;
    const size_t plane = (size_t)a.nvx * a.nvy;
    double* wsum = smem;
    double* red = wsum + a.kc * nw;
    double spe = 0.0, ssee = 0.0, stop = 0.0;
    for (int k = k0; k < k1; ++k) {
        const T* p = a.fin + (size_t)k * plane + j;
        double sn = 0.0;
        for (int r = 0; r < TI; ++r) {
            const int i = i0 + r;
            if (!jok || i >= a.nvx) continue;
            const double fv = (double)p[(size_t)i * a.nvy];
            sn += fv;
            const double v = cell_v(i, a.nvx, a.dvx);
            if (k == 0 && v < 0.0) {
                spe += -v * fv;
                ssee += a.delta[(size_t)i * a.nvy + j] * (-v * fv);
            }
            if (k == a.nx - 1 && v > 0.0) stop += v * fv;
        }
        sn = wave_sum(sn);
        if (lane == 0) wsum[(k - k0) * nw + wave] = sn;
    }
    __syncthreads();
    for (int kk = j; kk < k1 - k0; kk += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += wsum[kk * nw + w];
        a.part_n[(size_t)(k0 + kk) * a.n_it + it] = s;
    }
    spe = wave_sum(spe);
    ssee = wave_sum(ssee);
    stop = wave_sum(stop);
    if (lane == 0) {
        red[wave * 4 + 1] = spe;
        red[wave * 4 + 2] = ssee;
        red[wave * 4 + 3] = stop;
    }
    __syncthreads();
    if (j == 0) {
        double t1 = 0, t2 = 0, t3 = 0;
        for (int w = 0; w < nw; ++w) {
            t1 += red[w * 4 + 1];
            t2 += red[w * 4 + 2];
            t3 += red[w * 4 + 3];
        }
        a.part_lv[wg] = 0.0;
        if (k0 == 0) {
            a.part_wall[it * 2 + 0] = t1;
            a.part_wall[it * 2 + 1] = t2;
        }
        if (k1 == a.nx) a.part_top[it] = t3;
    }
}

// ---------------------------------------------------------------- field

struct FieldArgs {
    const double* __restrict__ part_n;
    const double* __restrict__ part_wall;
    const double* __restrict__ part_top;
    const double* __restrict__ part_lv;
    const double* __restrict__ consts;  // zsum, srcnorm, injected per step, Eq 15 prefactor
    double* __restrict__ ne;
    double* __restrict__ ex;
    double* __restrict__ dxk;
    DevState* __restrict__ st;
    fk_state* __restrict__ ring;
    int nx, n_it, nwg, advance;
    uint32_t mask;
    int emission_norm, trace_stride, trace_cap;
    double dx, dv2, dt, dvx, ex_ext;
};

// Reduction of the moment partials of the new f, the 1D field solve and the
// wall bookkeeping; one workgroup of kFieldThreads threads.
__device__ __forceinline__ void field_block(const FieldArgs& a, double* sh)
{
    const int t = threadIdx.x;
    const int T = blockDim.x;
    const int seg = (a.nx + T - 1) / T;
    const int kb = min(t * seg, a.nx), ke = min(kb + seg, a.nx);

    // electron density per plane (sum over the v_x tiles, fixed order)
    double local = 0.0;
    for (int k = kb; k < ke; ++k) {
        double s = 0.0;
        for (int u = 0; u < a.n_it; ++u) s += a.part_n[(size_t)k * a.n_it + u];
        const double nk = s * a.dv2;
        a.ne[k] = nk;
        local += nk;
    }

    // exclusive prefix over the thread segments (Hillis-Steele on LDS)
    double* s0 = sh;
    double* s1 = sh + T;
    s0[t] = local;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        double v = s0[t];
        if (t >= off) v += s0[t - off];
        s1[t] = v;
        __syncthreads();
        double* tmp = s0; s0 = s1; s1 = tmp;
    }
    const double below0 = t > 0 ? s0[t - 1] : 0.0;
    const double total = s0[T - 1];
    __syncthreads();

    const DevState old = *a.st;
    double sig = old.sigma, sig_lo = old.sigma_lo;
    if (a.advance) {
        // Eq 18 with the fluxes of f^n, Neumaier-compensated across steps
        const double inc = kE * a.dt * (old.g_see - old.g_pe);
        const double s = sig + inc;
        if (fabs(sig) >= fabs(inc)) sig_lo += (sig - s) + inc;
        else sig_lo += (inc - s) + sig;
        sig = s;
    }
    const double sigma_now = sig + sig_lo;

    // E_x at the cell centres: sigma / 2 eps0 minus the electron charge below
    double run = below0, cmax = 0.0;
    for (int k = kb; k < ke; ++k) {
        const double nk = a.ne[k];
        double e = (a.mask & FK_PHYS_SELF_FIELD)
                       ? sigma_now / (2.0 * kEps0) - kE / kEps0 * a.dx * (run + 0.5 * nk)
                       : 0.0;
        e += a.ex_ext;
        a.ex[k] = e;
        const double d = (a.mask & FK_PHYS_VX) ? (-kE * e / kMe) * a.dt / a.dvx : 0.0;
        a.dxk[k] = d;
        cmax = fmax(cmax, fabs(d));
        run += nk;
    }
    cmax = block_max(cmax, s1);

    double pe = 0.0, see = 0.0, top = 0.0, lv = 0.0;
    for (int u = t; u < a.n_it; u += T) {
        pe += a.part_wall[2 * u];
        see += a.part_wall[2 * u + 1];
        top += a.part_top[u];
    }
    if (a.advance)
        for (int w = t; w < a.nwg; w += T) lv += a.part_lv[w];
    pe = block_sum(pe, s1);
    see = block_sum(see, s1);
    top = block_sum(top, s1);
    lv = block_sum(lv, s1);

    if (t == 0) {
        const bool x_on = a.mask & FK_PHYS_X;
        const bool see_on = x_on && (a.mask & FK_PHYS_SEE);
        const double g_pe = x_on ? pe * a.dv2 : 0.0;
        const double g_see = see_on ? see * a.dv2 : 0.0;
        const double g_top = x_on ? top * a.dv2 : 0.0;
        const double zsum = a.consts[0];
        double gscale = 0.0;
        if (see_on) {
            if (a.emission_norm == FK_EMIT_DISCRETE) gscale = zsum > 0.0 ? g_see / zsum : 0.0;
            else gscale = g_see * a.consts[3];
        }
        const double emitted = gscale * zsum;
        const double n_total = total * a.dx;
        const double loss_v = a.advance ? lv * a.dx * a.dv2 : 0.0;
        double resid = 0.0;
        if (a.advance) {
            const double inj = (a.mask & FK_PHYS_SRC) ? a.consts[2] : 0.0;
            resid = (n_total - old.n_total) - (a.dt * (old.emitted - old.g_pe - old.g_top) + inj - loss_v);
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
        if (cmax > 1.0) ns.flags |= kFlagCfl;
        if (!isfinite(n_total) || !isfinite(g_pe) || !isfinite(g_see) || !isfinite(g_top) ||
            !isfinite(sigma_now))
            ns.flags |= kFlagNonfinite;
        *a.st = ns;
        if (ns.step % a.trace_stride == 0) {
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
            a.ring[(ns.step / a.trace_stride) % a.trace_cap] = r;
        }
    }
}

}  // namespace fk
