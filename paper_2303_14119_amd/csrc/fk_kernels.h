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

// A double moved across lanes by a DPP control (two 32-bit halves); lanes
// whose source is outside the row or whose row is masked off read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWS, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront in the vector ALU (no LDS traffic),
// fixed order: an inclusive scan inside each row of 16 lanes (shifts by 1,
// 2, 4, 8), then row totals passed on by the row broadcasts; lane 63 holds
// the total.
__device__ __forceinline__ double wave_total(double v)
{
    v += dpp_move<0x111, 0xf>(v);   // row_shr:1
    v += dpp_move<0x112, 0xf>(v);   // row_shr:2
    v += dpp_move<0x114, 0xf>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v);   // row_shr:8
    v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// Value of lane 63, the same in every lane.
__device__ __forceinline__ double lane63(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a wavefront (the fixed order of wave_total), the
// same in every lane.
__device__ __forceinline__ double wave_sum(double v) { return lane63(wave_total(v)); }

// Maximum over the 64 lanes of a wavefront of values >= 0, the same in every
// lane (lanes shifted in from outside a row read 0, which no value is below).
__device__ __forceinline__ double wave_max_nonneg(double v)
{
    v = fmax(v, dpp_move<0x111, 0xf>(v));
    v = fmax(v, dpp_move<0x112, 0xf>(v));
    v = fmax(v, dpp_move<0x114, 0xf>(v));
    v = fmax(v, dpp_move<0x118, 0xf>(v));
    v = fmax(v, dpp_move<0x142, 0xa>(v));
    v = fmax(v, dpp_move<0x143, 0xc>(v));
    return lane63(v);
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
    const double* __restrict__ nudt;    // [nx] nu_ee dt per plane (collision term, Eq 3-4)
    const double* __restrict__ nudt_n;  // [nx] nu_ee dt n_e per plane
    const T* __restrict__ gx;           // [nvx] v_x factor of the normalised equilibrium (Eq 5)
    const T* __restrict__ gy;           // [nvy] v_y factor
    const double* __restrict__ ghat;    // [nvx][nvy] emission shape
    const double* __restrict__ delta;   // [nvx][nvy] SEY
    const DevState* __restrict__ st;    // gscale of this step
    double* __restrict__ part_n;        // [n_it][nx] plane sums of each v_x tile
    double* __restrict__ part_wall;     // [n_it][2]
    double* __restrict__ part_top;      // [n_it]
    double* __restrict__ part_lv;       // [nwg]
    double* __restrict__ part_abs;      // [n_it][2] absorbed at the wall / x = L (reversed second-order steps)
    int nx, nvx, nvy, n_it, kc;
    double dvx, dt_dx;                  // v_x of row i is cell_v(i, nvx, dvx)
    double dy;                          // signed v_y Courant number
    double r_refl;                      // wall reflection: share of the wall cell's -v_x electrons returned at +v_x
    int x_on;
    int store_nt;                       // 1: stores of f^{n+1} are non-temporal (whole 128 B lines per row)
    const int* __restrict__ tile_list;  // v_x tile indices handled by this launch
    int n_list;
};

// Buffer-resource access (CDNA raw buffer instructions).  A descriptor
// covers one x plane; the row offset is a scalar, the column a 32-bit lane
// offset.  Accesses at or beyond the descriptor's byte range read 0 and
// drop stores (the hardware range check), which is how rows outside the
// grid (null descriptor, range 0) and idle lanes (lane offset past the
// plane) are masked without branches.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kIdleLaneOffset = 0x7ffffff0;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}

// Cache policy operand of the buffer instructions: bit 1 marks the access
// non-temporal (streamed through L2 without being kept).
constexpr int kCpDefault = 0, kCpStream = 2;

template <typename T, int CP = kCpDefault> __device__ __forceinline__ T bload(rsrc_t r, int voff, int soff)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, CP));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, CP));
}
template <typename T, int CP = kCpDefault> __device__ __forceinline__ void bstore(T v, rsrc_t r, int voff, int soff)
{
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, voff, soff, CP);
    } else {
        typedef int v2i __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, voff, soff, CP);
    }
}

// One workgroup owns v_x rows [i0, i0+TI) for all v_y columns (one thread per
// column) and marches over x planes [k0, k0+kc).  Each thread keeps three x
// planes of its rows (plus one halo row on each side) in registers and
// prefetches the fourth:
//   x sweep     upwind on sign(v_x) -- the plane below or above, in registers;
//   v_x sweep   upwind on sign(a_x) -- the neighbouring row, in registers;
//   v_y sweep   upwind on sign(a_y) -- the neighbouring column, through LDS;
//   source      added on the planes overlapping the band.
// f is read once and written once per cell, plus the two halo rows (mostly
// L2 hits: the neighbouring tiles run on the same XCD) and one halo plane per
// chunk.
template <typename T, int TI, bool EDGE, bool BGK = false>
__device__ __forceinline__ void sweep_body(const SweepArgs<T>& a, int it, int kci, double* smem, int j, int B)
{
    const int i0 = it * TI;
    const int k0 = kci * a.kc;
    const int k1 = min(k0 + a.kc, a.nx);
    const int nw = B >> 6;
    const int lane = j & 63, wave = j >> 6;
    const bool jok = j < a.nvy;
    const int W = B + 2;
    const size_t plane = (size_t)a.nvx * a.nvy;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));
    const int rowbytes = a.nvy * (int)sizeof(T);

    T* xb = reinterpret_cast<T*>(smem);                       // [2][TI][W]
    double* wsum = reinterpret_cast<double*>(xb + 2 * TI * W); // [kc][nw]
    double* red = wsum + a.kc * nw;                           // [nw][4]

    for (int m = j; m < 2 * TI; m += B) {
        xb[m * W] = T(0);
        xb[m * W + W - 1] = T(0);
    }

    // per-row data: row inside the grid (uniform), the lane's byte offset in
    // a plane (out of range for rows outside the grid and idle lanes, so
    // those read 0 and store nothing), and the signed x Courant number
    // The sign of v_x of row i is the sign of 2i + 1 - nvx (exact integer
    // test, uniform); the x sweep uses the split coefficients
    // cp = max(c, 0), cn = min(c, 0) so it needs no per-row lane masks.
    bool rv[TI + 2];
    int vo[TI + 2];
    T cp[TI + 2], cn[TI + 2];
#pragma unroll
    for (int r = 0; r < TI + 2; ++r) {
        const int i = i0 - 1 + r;
        rv[r] = EDGE ? (i >= 0 && i < a.nvx) : true;   // interior tiles: every row is in the grid
        vo[r] = (rv[r] && jok) ? i * rowbytes + j * (int)sizeof(T) : kIdleLaneOffset;
        const T c = (a.x_on && rv[r]) ? T(cell_v(i, a.nvx, a.dvx) * a.dt_dx) : T(0);
        cp[r] = 2 * i + 1 > a.nvx ? c : T(0);
        cn[r] = 2 * i + 1 < a.nvx ? c : T(0);
    }
    auto up_row = [&](int r) { return a.x_on && 2 * (i0 - 1 + r) + 1 > a.nvx; };   // v_x > 0
    auto down_row = [&](int r) { return a.x_on && 2 * (i0 - 1 + r) + 1 < a.nvx; }; // v_x < 0
    auto plane_in = [&](int kk) { return make_rsrc(a.fin + (size_t)kk * plane, pbytes); };
    auto plane_out = [&](int kk) { return make_rsrc(a.fout + (size_t)kk * plane, pbytes); };

    // Rolling window of x planes k-1, k, k+1 and the prefetched k+2.  The
    // planes just outside [k0, k1) are read only by the rows whose upwind
    // side they are: the plane below by rows with v_x > 0, the plane above
    // by rows with v_x < 0.
    T fm[TI + 2], fc[TI + 2], fp[TI + 2], fn[TI + 2];
    if (k0 == 0) {
        // below the dielectric: the emission row of this step (Eq 15)
        const double gs = a.st->gscale;
#pragma unroll
        for (int r = 0; r < TI + 2; ++r) {
            const int i = i0 - 1 + r;
            // plus the specular reflection of the wall cell (v_x row nvx-1-i
            // holds -v_x of row i)
            double g = 0.0;
            if (rv[r] && up_row(r) && jok) {
                g = gs * a.ghat[(size_t)i * a.nvy + j];
                if (a.r_refl != 0.0) g += a.r_refl * (double)a.fin[(size_t)(a.nvx - 1 - i) * a.nvy + j];
            }
            fm[r] = T(g);
        }
    } else {
        const rsrc_t pr = plane_in(k0 - 1);
#pragma unroll
        for (int r = 0; r < TI + 2; ++r) fm[r] = up_row(r) ? bload<T>(pr, vo[r], 0) : T(0);
    }
    {
        const rsrc_t pr = plane_in(k0);
#pragma unroll
        for (int r = 0; r < TI + 2; ++r) fc[r] = bload<T>(pr, vo[r], 0);
    }
    // Loads without branches (exact wait counts for the compiler): a plane
    // past x = L gets an empty descriptor and reads 0 (nothing enters there,
    // Eq 17), and rows that must not read the plane get an out-of-range
    // lane offset.  Past k1 only the rows with v_x < 0 read the plane.
    auto load_ahead = [&](int kk, T (&dst)[TI + 2]) {
        const bool in = kk < a.nx, inner = kk < k1;
        const rsrc_t pr = make_rsrc(a.fin + (size_t)(in ? kk : 0) * plane, in ? pbytes : 0u);
#pragma unroll
        for (int r = 0; r < TI + 2; ++r)
            dst[r] = bload<T>(pr, (inner || down_row(r)) ? vo[r] : kIdleLaneOffset, 0);
    };
    load_ahead(k0 + 1, fp);

    double lv = 0.0, spe = 0.0, ssee = 0.0, stop = 0.0;
    const T dy = T(a.dy);

    // the planes' v_x Courant numbers and source coefficients (used in T
    // precision only), staged per wave in LDS: the plane loop then issues no
    // memory operation but its plane loads and stores, so the compiler's
    // waits for the prefetched plane never cover a later load.  A wave reads
    // only what its own lanes wrote, so no workgroup barrier is needed.
    // With the collision term the table also holds nu_ee dt and nu_ee dt n_e
    // per plane and the tile's rows of the equilibrium's v_x factor.
    T* tab = reinterpret_cast<T*>(red + nw * 4) + wave * (BGK ? 4 * a.kc + TI : 2 * a.kc);
    for (int m = lane; m < k1 - k0; m += 64) {
        tab[m] = T(a.dxk[k0 + m]);
        tab[a.kc + m] = T(a.srck[k0 + m]);
        if (BGK) {
            tab[2 * a.kc + m] = T(a.nudt[k0 + m]);
            tab[3 * a.kc + m] = T(a.nudt_n[k0 + m]);
        }
    }
    T gyj = T(0);
    if (BGK) {
        for (int m = lane; m < TI; m += 64) tab[4 * a.kc + m] = i0 + m < a.nvx ? a.gx[i0 + m] : T(0);
        gyj = jok ? a.gy[j] : T(0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int k = k0; k < k1; ++k) {
        const T d_k = tab[k - k0];
        const T s_k = tab[a.kc + k - k0];
        load_ahead(k + 2, fn);   // reads nothing useful on the last iteration

        // x sweep: f' = f - c (f - f_up), upwind on the sign of v_x
        T f1[TI + 2];
#pragma unroll
        for (int r = 0; r < TI + 2; ++r) f1[r] = fc[r] - cp[r] * (fc[r] - fm[r]) - cn[r] * (fp[r] - fc[r]);

        // v_x sweep by a_x(x_k): upwind on the sign of the plane's Courant number
        const T d = T(d_k);
        T f2[TI];
#pragma unroll
        for (int r = 1; r <= TI; ++r) {
            const T diff = d > T(0) ? (f1[r] - f1[r - 1]) : (f1[r + 1] - f1[r]);
            f2[r - 1] = (rv[r] && jok) ? f1[r] - d * diff : T(0);
        }
        if (d > T(0)) {
#pragma unroll
            for (int r = 1; r <= TI; ++r)
                if (rv[r] && i0 - 1 + r == a.nvx - 1) lv += (double)d * (double)f1[r];
        } else if (d < T(0)) {
#pragma unroll
            for (int r = 1; r <= TI; ++r)
                if (rv[r] && i0 - 1 + r == 0) lv -= (double)d * (double)f1[r];
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
        if (s_k != 0) {
            const T ts = T(s_k);
#pragma unroll
            for (int r = 0; r < TI; ++r)
                if (rv[r + 1] && jok) f3[r] += ts * a.fsrc[(size_t)(i0 + r) * a.nvy + j];
        }

        // electron-electron collisions (Eq 3): dt nu_ee (n_e gx gy - f^n).
        // Rows outside the grid and idle lanes have gx, gy and f^n all 0.
        if (BGK) {
            const T bk = tab[2 * a.kc + k - k0];
            if (bk != T(0)) {
                const T agy = tab[3 * a.kc + k - k0] * gyj;
#pragma unroll
                for (int r = 0; r < TI; ++r) f3[r] += agy * tab[4 * a.kc + r] - bk * fc[r + 1];
            }
        }

        {
            const rsrc_t po = plane_out(k);
            if (a.store_nt) {
#pragma unroll
                for (int r = 0; r < TI; ++r) bstore<T, kCpStream>(f3[r], po, vo[r + 1], 0);
            } else {
#pragma unroll
                for (int r = 0; r < TI; ++r) bstore<T>(f3[r], po, vo[r + 1], 0);
            }
        }

        // moments of f^{n+1}
        double sn = 0.0;
#pragma unroll
        for (int r = 0; r < TI; ++r) sn += (double)f3[r];
        sn = wave_total(sn);
        if (lane == 63) wsum[(k - k0) * nw + wave] = sn;
        if (k == 0) {
#pragma unroll
            for (int r = 0; r < TI; ++r) {
                const int i = i0 + r;
                const double v = cell_v(i, a.nvx, a.dvx);
                if (rv[r + 1] && jok && v < 0.0) {
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
                if (rv[r + 1] && jok && v > 0.0) stop += v * (double)f3[r];
            }
        }

#pragma unroll
        for (int r = 0; r < TI + 2; ++r) {
            fm[r] = fc[r];
            fc[r] = fp[r];
            fp[r] = fn[r];
        }
    }

    __syncthreads();
    for (int kk = j; kk < k1 - k0; kk += B) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += wsum[kk * nw + w];
        a.part_n[(size_t)it * a.nx + k0 + kk] = s;
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
        a.part_lv[kci * a.n_it + it] = t0;
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
        sn = wave_total(sn);
        if (lane == 63) wsum[(k - k0) * nw + wave] = sn;
    }
    __syncthreads();
    for (int kk = j; kk < k1 - k0; kk += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += wsum[kk * nw + w];
        a.part_n[(size_t)it * a.nx + k0 + kk] = s;
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

}  // namespace fk
