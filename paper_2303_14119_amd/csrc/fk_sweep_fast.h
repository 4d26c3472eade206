// fk_sweep_fast.h -- the sweep of one tile whose v_x rows split at a
// compile-time row S: rows r < S have v_x <= 0 (their upwind x neighbour is
// the plane above), rows r >= S have v_x > 0 (upwind is the plane below).
// Rows are r = 0 .. TI+1 for v_x rows i = i0 - 1 + r (r = 0 and r = TI+1
// are the halo rows of the v_x sweep).
//
// Two launches per step: the main one over full tiles split at an edge
// (S = 0, 1, TI+1, TI+2), which covers almost every tile and keeps the
// register budget low; the second over the rest, where tiles of 4 or 8 rows
// split inside the tile or ragged at +v_max still take a compiled fast body
// and only the remainder takes the generic masked body.
//
// Per row the thread keeps the two x planes the upwind update reads plus
// one prefetched plane.  Rows outside the grid (the halo below the first
// tile, above the last) and lanes past nvy read 0 and store nothing through
// the buffer range check, so the body has no per-row lane masks.  Inside
// the plane loop the only memory operations are the next plane's loads and
// this plane's stores (the per-plane coefficients sit in LDS), so the
// prefetch stays in flight while the plane is computed.
#pragma once

#include "fk_kernels.h"

namespace fk {

// STREAM: the tile's inner rows are read with non-temporal loads (see the
// row loads below); only where every row of f starts on a 128-byte line.
template <typename T, int TI, int S, bool RAGGED = false, bool BGK = false, bool STREAM = false>
__device__ __forceinline__ void sweep_fast(const SweepArgs<T>& a, int it, int kci, double* smem, int j, int B)
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
    const int rb = a.nvy * (int)sizeof(T);
    const int es = (int)sizeof(T);
    const bool first = it == 0;
    const bool last = i0 + TI >= a.nvx;
    // lane byte offsets within a plane: output rows r = 1..TI at vb + (r-1)*rb,
    // halo rows at vlo / vhi (out of range outside the grid)
    const int vb = jok ? i0 * rb + j * es : kIdleLaneOffset;
    const int vlo = (jok && !first) ? (i0 - 1) * rb + j * es : kIdleLaneOffset;
    const int vhi = (jok && !last) ? (i0 + TI) * rb + j * es : kIdleLaneOffset;
    // a ragged last tile (RAGGED) holds R < TI rows: rows past the grid get
    // an out-of-range lane offset of their own, so they read 0 and store
    // nothing
    const int R = RAGGED ? a.nvx - i0 : TI;
    const int vb0 = i0 * rb + j * es;
    auto roff = [&](int r) { return (jok && r <= R) ? vb0 + (r - 1) * rb : kIdleLaneOffset; };

    T* xb = reinterpret_cast<T*>(smem);                       // [2][TI][W]
    double* wsum = reinterpret_cast<double*>(xb + 2 * TI * W); // [kc][nw]
    double* red = wsum + a.kc * nw;                           // [nw][4]
    for (int m = j; m < 2 * TI; m += B) {
        xb[m * W] = T(0);
        xb[m * W + W - 1] = T(0);
    }

    T c[TI + 2];
#pragma unroll
    for (int r = 0; r < TI + 2; ++r) {
        const int i = i0 - 1 + r;
        c[r] = a.x_on ? T(cell_v(i, a.nvx, a.dvx) * a.dt_dx) : T(0);
    }

    auto plane_in = [&](int kk) { return make_rsrc(a.fin + (size_t)kk * plane, pbytes); };
    // With STREAM the rows read by this tile alone, the inner rows
    // 2 .. TI-1, are streamed past L2 (non-temporal loads).  The halo rows
    // and the tile's first and last rows (the halo rows of the neighbouring
    // tiles, read again by them) keep the default policy and stay in L2.
    // Sweep time, default -> inner rows streamed: 4096 x 384 x 384 836.4 ->
    // 823.3 us; 2048 x 384 x 384 423.4 -> 412.8; 2048 x 256 x 256 194.9 ->
    // 190.6; the same in FP64 406.9 -> 403.7.  Streaming the first and last
    // rows too raised the reads at 4096 x 384 x 384 from 1.004x to 1.035x
    // the algorithmic bytes and gave back most of the gain.  Where rows share
    // lines with their neighbours (v_y widths off multiples of 32 FP32
    // values) streaming cost the 64-instance batch 8%, so it follows the
    // rule of the non-temporal stores.
    constexpr int kInnerCp = STREAM ? kCpStream : kCpDefault;
    auto ldrow = [&](const rsrc_t& pr, int r) -> T {
        if (r == 0) return bload<T>(pr, vlo, 0);
        if (r == TI + 1) return bload<T>(pr, vhi, 0);
        if (r == 1 || r == TI) return RAGGED ? bload<T>(pr, roff(r), 0) : bload<T>(pr, vb, (r - 1) * rb);
        if (RAGGED) return bload<T, kInnerCp>(pr, roff(r), 0);
        return bload<T, kInnerCp>(pr, vb, (r - 1) * rb);
    };

    // w0/w1: the two planes the row's upwind update reads; w2: prefetch.
    //   rows r < S  (v_x <= 0): w0 = f(k),   w1 = f(k+1)
    //   rows r >= S (v_x > 0):  w0 = f(k-1), w1 = f(k)
    T w0[TI + 2], w1[TI + 2], w2[TI + 2];
    {
        const rsrc_t pk = plane_in(k0);
        const bool has_up = k0 + 1 < a.nx;           // nothing enters at x = L (Eq 17)
        const rsrc_t pu = plane_in(has_up ? k0 + 1 : k0);
#pragma unroll
        for (int r = 0; r < S; ++r) {
            w0[r] = ldrow(pk, r);
            w1[r] = has_up ? ldrow(pu, r) : T(0);
        }
#pragma unroll
        for (int r = S; r < TI + 2; ++r) w1[r] = ldrow(pk, r);
        if (k0 == 0) {
            // below the dielectric: the emission row of this step (Eq 15)
            const double gs = a.st->gscale;
#pragma unroll
            for (int r = S; r < TI + 2; ++r) {
                const int i = i0 - 1 + r;
                // plus the specular reflection of the wall cell (v_x row
                // nvx-1-i holds -v_x of row i)
                double g = 0.0;
                if (jok && i < a.nvx) {
                    g = gs * a.ghat[(size_t)i * a.nvy + j];
                    if (a.r_refl != 0.0) g += a.r_refl * (double)a.fin[(size_t)(a.nvx - 1 - i) * a.nvy + j];
                }
                w0[r] = T(g);
            }
        } else {
            const rsrc_t pd = plane_in(k0 - 1);
#pragma unroll
            for (int r = S; r < TI + 2; ++r) w0[r] = ldrow(pd, r);
        }
    }

    const int nvl = a.nvy;
    const T dy = T(a.dy);
    double lv = 0.0, spe = 0.0, ssee = 0.0, stop = 0.0;
    const rsrc_t psrc = make_rsrc(a.fsrc, pbytes);

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
        // prefetch the planes of the next iteration.  The loads are issued on
        // every iteration (no branch, so the compiler's wait counts stay
        // exact); a plane that does not exist gets an empty descriptor and
        // reads 0, as nothing enters at x = L (Eq 17)
        {
            const bool n1 = k + 1 < k1, n2 = n1 && k + 2 < a.nx;
            const rsrc_t p1 = make_rsrc(a.fin + (size_t)(n1 ? k + 1 : k) * plane, n1 ? pbytes : 0u);
            const rsrc_t p2 = make_rsrc(a.fin + (size_t)(n2 ? k + 2 : k) * plane, n2 ? pbytes : 0u);
#pragma unroll
            for (int r = S; r < TI + 2; ++r) w2[r] = ldrow(p1, r);
#pragma unroll
            for (int r = 0; r < S; ++r) w2[r] = ldrow(p2, r);
        }

        // x sweep (upwind on the sign of v_x)
        T f1[TI + 2];
#pragma unroll
        for (int r = 0; r < TI + 2; ++r)
            f1[r] = r < S ? w0[r] - c[r] * (w1[r] - w0[r]) : w1[r] - c[r] * (w1[r] - w0[r]);

        // v_x sweep by a_x(x_k), upwind on the sign of the plane's Courant number
        const T d = T(d_k);
        T f2[TI];
        if (d > T(0)) {
#pragma unroll
            for (int r = 1; r <= TI; ++r) f2[r - 1] = f1[r] - d * (f1[r] - f1[r - 1]);
            if (RAGGED) {
#pragma unroll
                for (int r = 1; r <= TI; ++r)
                    if (r == R) lv += (double)d * (double)f1[r];  // leaves through +v_max
            } else if (last) {
                lv += (double)d * (double)f1[TI];                 // leaves through +v_max
            }
        } else {
#pragma unroll
            for (int r = 1; r <= TI; ++r) f2[r - 1] = f1[r] - d * (f1[r + 1] - f1[r]);
            if (first) lv -= (double)d * (double)f1[1];          // leaves through -v_max
        }
        if (RAGGED) {
#pragma unroll
            for (int r = 1; r <= TI; ++r)
                if (r > R) f2[r - 1] = T(0);                      // no cells past +v_max
        }

        // v_y sweep by a_y: the neighbouring column comes from LDS
        T* buf = xb + (k & 1) * TI * W;
#pragma unroll
        for (int r = 0; r < TI; ++r) buf[r * W + j + 1] = f2[r];
        __syncthreads();
        T f3[TI];
        if (dy > T(0)) {
#pragma unroll
            for (int r = 0; r < TI; ++r) f3[r] = f2[r] - dy * (f2[r] - buf[r * W + j]);
            if (j == nvl - 1) {
#pragma unroll
                for (int r = 0; r < TI; ++r) lv += (double)dy * (double)f2[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < TI; ++r) f3[r] = f2[r] - dy * (buf[r * W + j + 2] - f2[r]);
            if (j == 0) {
#pragma unroll
                for (int r = 0; r < TI; ++r) lv -= (double)dy * (double)f2[r];
            }
        }

        // band source (Eq 7)
        if (s_k != 0) {
            const T ts = T(s_k);
#pragma unroll
            for (int r = 0; r < TI; ++r)
                f3[r] += ts * (RAGGED ? bload<T>(psrc, roff(r + 1), 0) : bload<T>(psrc, vb, r * rb));
        }

        // electron-electron collisions (Eq 3): dt nu_ee (n_e gx gy - f^n),
        // with f^n of output row r in w0 (v_x <= 0) or w1 (v_x > 0).  Rows
        // past the grid and idle lanes have gx, gy and f^n all 0.
        if (BGK) {
            const T bk = tab[2 * a.kc + k - k0];
            if (bk != T(0)) {
                const T agy = tab[3 * a.kc + k - k0] * gyj;
#pragma unroll
                for (int r = 0; r < TI; ++r) f3[r] += agy * tab[4 * a.kc + r] - bk * (r + 1 < S ? w0[r + 1] : w1[r + 1]);
            }
        }

        {
            const rsrc_t po = make_rsrc(a.fout + (size_t)k * plane, pbytes);
            if (a.store_nt) {
#pragma unroll
                for (int r = 0; r < TI; ++r) {
                    if (RAGGED) bstore<T, kCpStream>(f3[r], po, roff(r + 1), 0);
                    else bstore<T, kCpStream>(f3[r], po, vb, r * rb);
                }
            } else {
#pragma unroll
                for (int r = 0; r < TI; ++r) {
                    if (RAGGED) bstore<T>(f3[r], po, roff(r + 1), 0);
                    else bstore<T>(f3[r], po, vb, r * rb);
                }
            }
        }

        // moments of f^{n+1}
        double sn = 0.0;
#pragma unroll
        for (int r = 0; r < TI; ++r) sn += (double)f3[r];
        sn = wave_total(jok ? sn : 0.0);
        if (lane == 63) wsum[(k - k0) * nw + wave] = sn;
        if (k == 0 && jok) {
#pragma unroll
            for (int r = 1; r < (S < TI + 1 ? S : TI + 1); ++r) {   // output rows with v_x <= 0
                const int i = i0 - 1 + r;
                const double g = -cell_v(i, a.nvx, a.dvx) * (double)f3[r - 1];
                spe += g;
                ssee += a.delta[(size_t)i * a.nvy + j] * g;
            }
        }
        if (k == a.nx - 1 && jok) {
#pragma unroll
            for (int r = (S > 1 ? S : 1); r <= TI; ++r)                // output rows with v_x > 0
                stop += cell_v(i0 - 1 + r, a.nvx, a.dvx) * (double)f3[r - 1];
        }

        if (k + 1 < k1) {
#pragma unroll
            for (int r = 0; r < TI + 2; ++r) {
                w0[r] = w1[r];
                w1[r] = w2[r];
            }
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

template <typename T, int TI, bool BGK = false, bool STREAM = false>
__device__ __forceinline__ void sweep_fast_dispatch(const SweepArgs<T>& a, int it, int kci, double* smem, int j, int B)
{
    switch (tile_split(it, TI, a.nvx)) {
    case 0: sweep_fast<T, TI, 0, false, BGK, STREAM>(a, it, kci, smem, j, B); break;
    case 1: sweep_fast<T, TI, 1, false, BGK, STREAM>(a, it, kci, smem, j, B); break;
    case TI + 1: sweep_fast<T, TI, TI + 1, false, BGK, STREAM>(a, it, kci, smem, j, B); break;
    default: sweep_fast<T, TI, TI + 2, false, BGK, STREAM>(a, it, kci, smem, j, B); break;
    }
}

// Splits inside the tile (S = 2 .. TI) as a chain of uniform branches.
template <typename T, int TI, int S, bool BGK = false>
__device__ __forceinline__ void sweep_mid_chain(const SweepArgs<T>& a, int it, int kci, double* smem, int j, int B,
                                                int s)
{
    if constexpr (S == TI) {
        sweep_fast<T, TI, S, false, BGK>(a, it, kci, smem, j, B);
    } else {
        if (s == S) sweep_fast<T, TI, S, false, BGK>(a, it, kci, smem, j, B);
        else sweep_mid_chain<T, TI, S + 1, BGK>(a, it, kci, smem, j, B, s);
    }
}

// Tiles outside the edge-split set: the fast body compiled for their split
// (full tiles of 4 or 8 rows split inside the tile) or for a ragged last
// tile whose rows all have v_x > 0; any other tile takes the generic body.
template <typename T, int TI, bool BGK = false>
__device__ __forceinline__ void sweep_rest(const SweepArgs<T>& a, int it, int kci, double* smem, int j, int B)
{
    if constexpr (TI == 4 || TI == 8) {
        if (tile_is_special(it, TI, a.nvx)) {
            if ((it + 1) * TI > a.nvx) sweep_fast<T, TI, 0, true, BGK>(a, it, kci, smem, j, B);
            else sweep_mid_chain<T, TI, 2, BGK>(a, it, kci, smem, j, B, tile_split(it, TI, a.nvx));
            return;
        }
    }
    sweep_body<T, TI, true, BGK>(a, it, kci, smem, j, B);
}

// Tiles of a launch: blockIdx -> (x chunk, entry of the launch's v_x tile
// list), remapped so each XCD takes a contiguous range.
// BGK: compiled with the collision term (a kernel of its own, so the
// register budget of the plain sweep does not carry it).  STREAM: the inner
// rows are read with non-temporal loads (rows on 128-byte lines).
template <typename T, int TI, int MAXB, bool BGK = false, bool STREAM = false>
__global__ void __launch_bounds__(MAXB) k_sweep(SweepArgs<T> a)
{
    extern __shared__ double smem[];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int it = a.tile_list[wg % a.n_list];
    sweep_fast_dispatch<T, TI, BGK, STREAM>(a, it, wg / a.n_list, smem, threadIdx.x, blockDim.x);
}

template <typename T, int TI, int MAXB, bool BGK = false>
__global__ void __launch_bounds__(MAXB) k_sweep_generic(SweepArgs<T> a)
{
    extern __shared__ double smem[];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int it = a.tile_list[wg % a.n_list];
    sweep_rest<T, TI, BGK>(a, it, wg / a.n_list, smem, threadIdx.x, blockDim.x);
}

// A sub-tile slot of a batched workgroup with no tile: take part in the same
// number of workgroup barriers as a tile of nplanes x planes.
__device__ __forceinline__ void sweep_idle(int nplanes)
{
    for (int k = 0; k < nplanes; ++k) __syncthreads();
    __syncthreads();
    __syncthreads();
}

}  // namespace fk
