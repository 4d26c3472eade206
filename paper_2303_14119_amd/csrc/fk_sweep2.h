// fk_sweep2.h -- the fused sweep of the second-order scheme
// (FK_SCHEME_LIMITED2), one pass over f per step.
//
// Every 1D advection at Courant number c (constant along its line) is taken
// in flux form: the face right of cell m carries, for c > 0, the cell's value
// moved towards the face, f_m + (1 - c)/2 s_m, and the face left of cell m,
// for c < 0, f_m - (1 + c)/2 s_m, where s_m is the minmod of the cell's two
// one-sided differences (zero in the first and last cell of every line, so
// the boundary faces carry the plain upwind values: the emission row at the
// dielectric, nothing through x = L or into the velocity box, and the same
// wall, escape and box-loss tallies as the first-order step).  The update is
// f'_m = f_m - c (right face - left face).  This is an accuracy extension
// beyond the paper's first-order upwind step (Section 2, after Eq 2).
//
// Split order: x, v_x, v_y, source on even steps (the forward body) and
// source, v_y, v_x, x on odd steps (the reversed body), so that two steps
// form a symmetric composition.
//
// Layout as in the first-order sweep: one thread per v_y column j, a tile of
// TI v_x rows, a chunk of kc x planes.  The limited stencils reach two cells:
//   forward:  the x update runs on TI + 4 rows (the v_x sweep's halo), each
//             row keeping planes k-1 .. k+2 and the face value it carried
//             into plane k; v_y neighbours j-2 .. j+2 come through LDS;
//   reversed: each plane is first advanced in velocity (source, v_y on
//             TI + 4 rows, v_x down to TI rows) two planes ahead of the x
//             update, which then runs on the tile's TI rows; the velocity
//             work of the two planes on each side of a chunk is repeated by
//             the neighbouring chunks (only the chunk's own planes tally).
// Rows outside the grid and lanes past nvy read 0 and store nothing through
// the buffer range check, as in the first-order bodies.
#pragma once

#include "fk_kernels.h"

namespace fk {

// minmod of two differences: the one nearer zero if they agree in sign,
// else 0.  In FP32 it is the median of (a, b, 0), one v_med3 instruction; in
// FP64 min, max and an addition of zero.  Both are exact.
template <typename T>
__device__ __forceinline__ T minmod(T a, T b)
{
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_fmed3f(a, b, 0.0f);
    else return fmax(fmin(a, b), T(0)) + fmin(fmax(a, b), T(0));
}

// The limited 1D update along a line of values held by one thread (v_x
// rows), c uniform.  u[0 .. R-1] are rows i0 - 2 .. i0 + R - 3; out[o] is
// row i0 + o for o = 0 .. R-5.  edge[r]: row r's slope is zero (first or
// last cell of the line, or outside it).  Returns the amount leaving through
// the box edges (in cell units, times c) for the rows of this tile.
template <typename T, int R>
__device__ __forceinline__ double vx_update(const T (&u)[R], const bool (&edge)[R], const bool (&in_grid)[R], T d,
                                            T (&out)[R - 4], int first_row, int last_row)
{
    double lv = 0.0;
    T s[R];
#pragma unroll
    for (int r = 1; r < R - 1; ++r) s[r] = edge[r] ? T(0) : minmod(u[r] - u[r - 1], u[r + 1] - u[r]);
    if (d > T(0)) {
        const T h = T(0.5) * (T(1) - d);
        T g[R];
#pragma unroll
        for (int r = 1; r < R - 2; ++r) g[r] = u[r] + h * s[r];   // right face of row r
#pragma unroll
        for (int o = 0; o < R - 4; ++o) out[o] = in_grid[o + 2] ? u[o + 2] - d * (g[o + 2] - g[o + 1]) : T(0);
#pragma unroll
        for (int o = 0; o < R - 4; ++o)
            if (o == last_row) lv += (double)d * (double)u[o + 2];   // leaves through +v_max
    } else {
        const T h = T(0.5) * (T(1) + d);
        T g[R];
#pragma unroll
        for (int r = 2; r < R - 1; ++r) g[r] = u[r] - h * s[r];   // left face of row r
#pragma unroll
        for (int o = 0; o < R - 4; ++o) out[o] = in_grid[o + 2] ? u[o + 2] - d * (g[o + 3] - g[o + 2]) : T(0);
#pragma unroll
        for (int o = 0; o < R - 4; ++o)
            if (o == first_row) lv -= (double)d * (double)u[o + 2];  // leaves through -v_max
    }
    return lv;
}

// The limited v_y update of NR rows held one column per thread: values go
// through LDS (buf: NR rows of W = B + 4 columns, the lane at column j + 2),
// one barrier.  Returns the box loss of this lane over rows [own_lo, own_hi)
// (the tile's own rows; halo rows are tallied by their own tile).  jok false
// zeroes the output (callers whose idle lanes never reach memory or the sums
// pass true).
template <typename T, int NR>
__device__ __forceinline__ double vy_update(const T (&v)[NR], T (&out)[NR], T* buf, int W, int j, int nvy, T dy,
                                            bool jok, int own_lo, int own_hi)
{
#pragma unroll
    for (int r = 0; r < NR; ++r) buf[r * W + j + 2] = v[r];
    __syncthreads();
    // With s(m) the minmod slope of column m and h the face coefficient:
    // dy > 0: res = b0 - dy (b0 - a1) - dy h s(j) + dy h s(j - 1);
    // dy < 0: res = b0 - dy (c1 - b0) + dy h s(j + 1) - dy h s(j).
    // Slopes are zero in the first and last column and outside the grid;
    // those factors are folded into the per-lane coefficients e0, em, ep.
    const T fm = (j - 1 <= 0 || j - 1 >= nvy - 1) ? T(0) : T(1);
    const T f0 = (j <= 0 || j >= nvy - 1) ? T(0) : T(1);
    const T fpl = (j + 1 >= nvy - 1) ? T(0) : T(1);
    const T h = dy > T(0) ? T(0.5) * (T(1) - dy) : T(0.5) * (T(1) + dy);
    const T e0 = dy * h * f0;
    T lvr = T(0);   // the lane's outflow over its own rows (only the edge lanes use it)
    // one uniform branch on the sign of dy, outside the row loop
    if (dy > T(0)) {
        const T em = dy * h * fm;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const T* row = buf + r * W + j + 2;
            const T a2 = row[-2], a1 = row[-1], b0 = v[r], c1 = row[1];
            const T d = b0 - a1;
            const T res = fma(em, minmod(a1 - a2, d), fma(-e0, minmod(d, c1 - b0), fma(-dy, d, b0)));
            out[r] = jok ? res : T(0);
            if (r >= own_lo && r < own_hi) lvr += b0;
        }
    } else {
        const T ep = dy * h * fpl;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const T* row = buf + r * W + j + 2;
            const T a1 = row[-1], b0 = v[r], c1 = row[1], c2 = row[2];
            const T d = c1 - b0;
            const T res = fma(-e0, minmod(b0 - a1, d), fma(ep, minmod(d, c2 - c1), fma(-dy, d, b0)));
            out[r] = jok ? res : T(0);
            if (r >= own_lo && r < own_hi) lvr += b0;
        }
    }
    // what leaves through +v_max (dy > 0, last column) or -v_max (dy < 0,
    // first column): dy times the edge cell (its slope is zero)
    if ((dy > T(0) && j == nvy - 1) || (dy < T(0) && j == 0)) return fabs((double)dy) * (double)lvr;
    return 0.0;
}

// The x update of one output plane k for the rows of a tile (one value per
// row): window planes k-1, k, k+1, k+2 and the face value carried into plane
// k (fp).  up[r]: v_x > 0.  zk, zk1: the slope of plane k / k+1 is zero.
template <typename T, int NR>
__device__ __forceinline__ void x_update(const T (&wm)[NR], const T (&w0)[NR], const T (&w1)[NR], const T (&w2)[NR],
                                         const T (&c)[NR], const bool (&up)[NR], bool zk, bool zk1, T (&fp)[NR],
                                         T (&out)[NR])
{
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        // the face right of plane k: carried from plane k (v_x > 0) or from
        // plane k + 1 (v_x < 0)
        const T a = up[r] ? wm[r] : w0[r];
        const T b = up[r] ? w0[r] : w1[r];
        const T e = up[r] ? w1[r] : w2[r];
        const bool z = up[r] ? zk : zk1;
        const T s = z ? T(0) : minmod(b - a, e - b);
        const T h = up[r] ? T(0.5) * (T(1) - c[r]) : -(T(0.5) * (T(1) + c[r]));
        const T f = b + h * s;
        out[r] = w0[r] - c[r] * (f - fp[r]);
        fp[r] = f;
    }
}

// The face value carried into plane k0 (the face left of k0) from the
// planes k0 - 2 .. k0 + 1, or the emission row at the dielectric.
template <typename T, int NR>
__device__ __forceinline__ void x_first_face(const T (&wmm)[NR], const T (&wm)[NR], const T (&w0)[NR],
                                             const T (&w1)[NR], const T (&ghost)[NR], const T (&c)[NR],
                                             const bool (&up)[NR], int k0, int nx, T (&fp)[NR])
{
    const bool zm = k0 - 1 <= 0 || k0 - 1 >= nx - 1;
    const bool z0 = k0 <= 0 || k0 >= nx - 1;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (up[r]) {
            const T s = zm ? T(0) : minmod(wm[r] - wmm[r], w0[r] - wm[r]);
            fp[r] = k0 == 0 ? ghost[r] : wm[r] + T(0.5) * (T(1) - c[r]) * s;
        } else {
            const T s = z0 ? T(0) : minmod(w0[r] - wm[r], w1[r] - w0[r]);
            fp[r] = w0[r] - T(0.5) * (T(1) + c[r]) * s;
        }
    }
}

// Shared per-tile set-up of both bodies.
template <typename T>
struct Tile2 {
    int i0, k0, k1, nw, lane, wave, W;
    bool jok;
    size_t plane;
    uint32_t pbytes;
    int rb;
};

template <typename T>
__device__ __forceinline__ Tile2<T> tile2(const SweepArgs<T>& a, int it, int kci, int j, int B, int TI)
{
    Tile2<T> t;
    t.i0 = it * TI;
    t.k0 = kci * a.kc;
    t.k1 = min(t.k0 + a.kc, a.nx);
    t.nw = B >> 6;
    t.lane = j & 63;
    t.wave = j >> 6;
    t.W = B + 4;
    t.jok = j < a.nvy;
    t.plane = (size_t)a.nvx * a.nvy;
    t.pbytes = (uint32_t)(t.plane * sizeof(T));
    t.rb = a.nvy * (int)sizeof(T);
    return t;
}

// Emission row of this step below the dielectric (Eq 15) for row i and lane
// j, plus the specular reflection of the wall cell (v_x row nvx-1-i of f^n).
template <typename T>
__device__ __forceinline__ T ghost_value(const SweepArgs<T>& a, int i, int j, bool jok)
{
    double g = 0.0;
    if (jok && i >= 0 && i < a.nvx && 2 * i + 1 > a.nvx) {
        g = a.st->gscale * a.ghat[(size_t)i * a.nvy + j];
        if (a.r_refl != 0.0) g += a.r_refl * (double)a.fin[(size_t)(a.nvx - 1 - i) * a.nvy + j];
    }
    return T(g);
}

// Plane sums of a batch of up to four planes of one wave: lane 16p + q adds
// the row sums of lanes 4q .. 4q + 3 of batch plane p in FP64, a shift-and-
// add inside each row of 16 lanes (by 1, 2, 4, 8) leaves the plane's total
// in lane 16p + 15, which writes it to the block's slot.  kb: the batch's
// first plane, relative to k0; last: the last plane written.
template <typename T>
__device__ __forceinline__ void flush_plane_sums(const Tile2<T>& t, const T* ring, int kb, int last, double* wsum)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int p = t.lane >> 4, q = t.lane & 15;
    const T* src = ring + p * 64 + q * 4;
    double v = ((double)src[0] + (double)src[1]) + ((double)src[2] + (double)src[3]);
    v += dpp_move<0x111, 0xf>(v);   // row_shr:1
    v += dpp_move<0x112, 0xf>(v);   // row_shr:2
    v += dpp_move<0x114, 0xf>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v);   // row_shr:8
    if (q == 15 && kb + p <= last) wsum[(kb + p) * t.nw + t.wave] = v;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Moments of the output plane k for output rows out[0 .. TI): the lane's
// row sum (in T: four or eight values) into the wave's ring of four planes,
// the plane sums every fourth plane and at the chunk's end; wall partials at
// k = 0, top partial at k = nx - 1.
template <typename T, int TI>
__device__ __forceinline__ void plane_moments(const SweepArgs<T>& a, const Tile2<T>& t, int k, const T (&out)[TI],
                                              int j, T* ring, double* wsum, double& spe, double& ssee, double& stop)
{
    T rs = T(0);
#pragma unroll
    for (int r = 0; r < TI; ++r) rs += out[r];
    const int kr = k - t.k0;
    ring[(kr & 3) * 64 + t.lane] = t.jok ? rs : T(0);
    if ((kr & 3) == 3 || k == t.k1 - 1) flush_plane_sums(t, ring, kr & ~3, kr, wsum);
    if (k == 0 && t.jok) {
#pragma unroll
        for (int r = 0; r < TI; ++r) {
            const int i = t.i0 + r;
            if (i < a.nvx && 2 * i + 1 < a.nvx) {
                const double g = -cell_v(i, a.nvx, a.dvx) * (double)out[r];
                spe += g;
                ssee += a.delta[(size_t)i * a.nvy + j] * g;
            }
        }
    }
    if (k == a.nx - 1 && t.jok) {
#pragma unroll
        for (int r = 0; r < TI; ++r) {
            const int i = t.i0 + r;
            if (i < a.nvx && 2 * i + 1 > a.nvx) stop += cell_v(i, a.nvx, a.dvx) * (double)out[r];
        }
    }
}

// End of a tile: plane sums, box loss, wall and top partials (and, for the
// reversed body, the absorbed fluxes) to the tile's slots.
template <typename T>
__device__ __forceinline__ void tile_partials(const SweepArgs<T>& a, const Tile2<T>& t, int it, int kci, int j, int B,
                                              double* wsum, double* red, double lv, double spe, double ssee,
                                              double stop, double abw, double abt, bool rev)
{
    __syncthreads();
    for (int kk = j; kk < t.k1 - t.k0; kk += B) {
        double s = 0.0;
        for (int w = 0; w < t.nw; ++w) s += wsum[kk * t.nw + w];
        a.part_n[(size_t)it * a.nx + t.k0 + kk] = s;
    }
    lv = wave_sum(lv);
    spe = wave_sum(spe);
    ssee = wave_sum(ssee);
    stop = wave_sum(stop);
    if (rev) {
        abw = wave_sum(abw);
        abt = wave_sum(abt);
    }
    if (t.lane == 0) {
        red[t.wave * 6 + 0] = lv;
        red[t.wave * 6 + 1] = spe;
        red[t.wave * 6 + 2] = ssee;
        red[t.wave * 6 + 3] = stop;
        red[t.wave * 6 + 4] = abw;
        red[t.wave * 6 + 5] = abt;
    }
    __syncthreads();
    if (j == 0) {
        double q[6] = {0, 0, 0, 0, 0, 0};
        for (int w = 0; w < t.nw; ++w)
            for (int m = 0; m < 6; ++m) q[m] += red[w * 6 + m];
        a.part_lv[kci * a.n_it + it] = q[0];
        if (t.k0 == 0) {
            a.part_wall[it * 2 + 0] = q[1];
            a.part_wall[it * 2 + 1] = q[2];
            if (rev) a.part_abs[it * 2 + 0] = q[4];
        }
        if (t.k1 == a.nx) {
            a.part_top[it] = q[3];
            if (rev) a.part_abs[it * 2 + 1] = q[5];
        }
    }
}

// ------------------------------------------------------------ forward body
// x -> v_x -> v_y -> source.
template <typename T, int TI>
__device__ __forceinline__ void sweep2_forward(const SweepArgs<T>& a, int it, int kci, double* smem, int j, int B)
{
    constexpr int R = TI + 4;
    const Tile2<T> t = tile2(a, it, kci, j, B, TI);
    T* xb = reinterpret_cast<T*>(smem);                                  // [2][R][W]
    double* wsum = reinterpret_cast<double*>(xb + 2 * R * t.W);          // [kc][nw]
    double* red = wsum + a.kc * t.nw;                                    // [nw][6]
    T* tab = reinterpret_cast<T*>(red + t.nw * 6) + t.wave * 2 * (a.kc + 4);
    T* ring = reinterpret_cast<T*>(red + t.nw * 6) + t.nw * 2 * (a.kc + 4) + t.wave * 256;   // [4][64]
    for (int m = j; m < 2 * R; m += B) {
        xb[m * t.W] = T(0);
        xb[m * t.W + 1] = T(0);
        xb[m * t.W + t.W - 2] = T(0);
        xb[m * t.W + t.W - 1] = T(0);
    }
    // per row (rows i0 - 2 .. i0 + TI + 1): lane offset, Courant number, sign
    int vo[R];
    T c[R];
    bool up[R], edge[R], in_grid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t.i0 - 2 + r;
        in_grid[r] = i >= 0 && i < a.nvx;
        vo[r] = (in_grid[r] && t.jok) ? i * t.rb + j * (int)sizeof(T) : kIdleLaneOffset;
        c[r] = (a.x_on && in_grid[r]) ? T(cell_v(i, a.nvx, a.dvx) * a.dt_dx) : T(0);
        up[r] = 2 * i + 1 > a.nvx;
        edge[r] = i <= 0 || i >= a.nvx - 1;
    }
    const int first_row = -t.i0;               // output row o of v_x row 0 (if in this tile)
    const int last_row = a.nvx - 1 - t.i0;     // output row of v_x row nvx - 1
    auto load_plane = [&](int kk, T (&dst)[R]) {
        const bool in = kk >= 0 && kk < a.nx;
        const rsrc_t pr = make_rsrc(a.fin + (size_t)(in ? kk : 0) * t.plane, in ? t.pbytes : 0u);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r] = bload<T>(pr, vo[r], 0);
    };
    T wmm[R], wm[R], w0[R], w1[R], w2[R], wn[R], fp[R];
    load_plane(t.k0 - 2, wmm);
    load_plane(t.k0 - 1, wm);
    load_plane(t.k0, w0);
    load_plane(t.k0 + 1, w1);
    load_plane(t.k0 + 2, w2);
    {
        T gh[R];
#pragma unroll
        for (int r = 0; r < R; ++r) gh[r] = a.x_on ? ghost_value(a, t.i0 - 2 + r, j, t.jok) : T(0);
        x_first_face<T, R>(wmm, wm, w0, w1, gh, c, up, t.k0, a.nx, fp);
    }
    for (int m = t.lane; m < t.k1 - t.k0; m += 64) {
        tab[m] = T(a.dxk[t.k0 + m]);
        tab[a.kc + 4 + m] = T(a.srck[t.k0 + m]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    double lv = 0.0, spe = 0.0, ssee = 0.0, stop = 0.0;
    const T dy = T(a.dy);
    const rsrc_t psrc = make_rsrc(a.fsrc, t.pbytes);
    for (int k = t.k0; k < t.k1; ++k) {
        const T d_k = tab[k - t.k0];
        const T s_k = tab[a.kc + 4 + k - t.k0];
        load_plane(k + 3, wn);   // reads nothing useful near the end

        // x sweep on all R rows
        T u[R];
        x_update<T, R>(wm, w0, w1, w2, c, up, k <= 0 || k >= a.nx - 1, k + 1 >= a.nx - 1, fp, u);
        // v_x sweep by a_x(x_k)
        T f2[TI];
        lv += vx_update<T, R>(u, edge, in_grid, d_k, f2, first_row, last_row);
        // v_y sweep by a_y
        T f3[TI];
        lv += vy_update<T, TI>(f2, f3, xb + (k & 1) * R * t.W, t.W, j, a.nvy, dy, t.jok, 0, TI);
        // band source (Eq 7)
        if (s_k != T(0)) {
#pragma unroll
            for (int r = 0; r < TI; ++r) f3[r] += s_k * bload<T>(psrc, vo[r + 2], 0);
        }
        {
            const rsrc_t po = make_rsrc(a.fout + (size_t)k * t.plane, t.pbytes);
#pragma unroll
            for (int r = 0; r < TI; ++r) bstore<T>(f3[r], po, vo[r + 2], 0);
        }
        plane_moments<T, TI>(a, t, k, f3, j, ring, wsum, spe, ssee, stop);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            wm[r] = w0[r];
            w0[r] = w1[r];
            w1[r] = w2[r];
            w2[r] = wn[r];
        }
    }
    tile_partials(a, t, it, kci, j, B, wsum, red, lv, spe, ssee, stop, 0.0, 0.0, false);
}

// ----------------------------------------------------------- reversed body
// source -> v_y -> v_x -> x.
template <typename T, int TI>
__device__ __forceinline__ void sweep2_reversed(const SweepArgs<T>& a, int it, int kci, double* smem, int j, int B)
{
    constexpr int R = TI + 4;
    const Tile2<T> t = tile2(a, it, kci, j, B, TI);
    T* xb = reinterpret_cast<T*>(smem);                                  // [2][R][W]
    double* wsum = reinterpret_cast<double*>(xb + 2 * R * t.W);          // [kc][nw]
    double* red = wsum + a.kc * t.nw;                                    // [nw][6]
    T* tab = reinterpret_cast<T*>(red + t.nw * 6) + t.wave * 2 * (a.kc + 4);
    T* ring = reinterpret_cast<T*>(red + t.nw * 6) + t.nw * 2 * (a.kc + 4) + t.wave * 256;   // [4][64]
    for (int m = j; m < 2 * R; m += B) {
        xb[m * t.W] = T(0);
        xb[m * t.W + 1] = T(0);
        xb[m * t.W + t.W - 2] = T(0);
        xb[m * t.W + t.W - 1] = T(0);
    }
    int vo[R];
    bool edge[R], in_grid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t.i0 - 2 + r;
        in_grid[r] = i >= 0 && i < a.nvx;
        vo[r] = (in_grid[r] && t.jok) ? i * t.rb + j * (int)sizeof(T) : kIdleLaneOffset;
        edge[r] = i <= 0 || i >= a.nvx - 1;
    }
    T c[TI];
    bool up[TI];
#pragma unroll
    for (int o = 0; o < TI; ++o) {
        const int i = t.i0 + o;
        c[o] = (a.x_on && i < a.nvx) ? T(cell_v(i, a.nvx, a.dvx) * a.dt_dx) : T(0);
        up[o] = 2 * i + 1 > a.nvx;
    }
    const int first_row = -t.i0;
    const int last_row = a.nvx - 1 - t.i0;
    // per-plane coefficients for planes k0 - 2 .. k1 + 1 (0 outside the grid)
    for (int m = t.lane; m < t.k1 - t.k0 + 4; m += 64) {
        const int kk = t.k0 - 2 + m;
        const bool in = kk >= 0 && kk < a.nx;
        tab[m] = in ? T(a.dxk[kk]) : T(0);
        tab[a.kc + 4 + m] = in ? T(a.srck[kk]) : T(0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    auto load_plane = [&](int kk, T (&dst)[R]) {
        const bool in = kk >= 0 && kk < a.nx;
        const rsrc_t pr = make_rsrc(a.fin + (size_t)(in ? kk : 0) * t.plane, in ? t.pbytes : 0u);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r] = bload<T>(pr, vo[r], 0);
    };
    const rsrc_t psrc = make_rsrc(a.fsrc, t.pbytes);
    const T dy = T(a.dy);
    double lv = 0.0, abw = 0.0, abt = 0.0;
    // the velocity part of plane p (source, v_y, v_x) from its raw rows;
    // the chunk's own planes tally the box loss and the absorbed fluxes
    auto velocity = [&](int p, const T (&raw)[R], T (&h)[TI]) {
        const T d_p = tab[p - t.k0 + 2];
        const T s_p = tab[a.kc + 4 + p - t.k0 + 2];
        T g[R];
#pragma unroll
        for (int r = 0; r < R; ++r) g[r] = raw[r];
        if (s_p != T(0)) {
#pragma unroll
            for (int r = 0; r < R; ++r) g[r] += s_p * bload<T>(psrc, vo[r], 0);
        }
        T y[R];
        const double lvy = vy_update<T, R>(g, y, xb + (p & 1) * R * t.W, t.W, j, a.nvy, dy, t.jok, 2, TI + 2);
        const double lvx = vx_update<T, R>(y, edge, in_grid, d_p, h, first_row, last_row);
        if (p >= t.k0 && p < t.k1) {
            lv += lvy + lvx;
            if (p == 0 && t.jok) {
#pragma unroll
                for (int o = 0; o < TI; ++o)
                    if (t.i0 + o < a.nvx && 2 * (t.i0 + o) + 1 < a.nvx)
                        abw += -cell_v(t.i0 + o, a.nvx, a.dvx) * (double)h[o];
            }
            if (p == a.nx - 1 && t.jok) {
#pragma unroll
                for (int o = 0; o < TI; ++o)
                    if (t.i0 + o < a.nvx && 2 * (t.i0 + o) + 1 > a.nvx)
                        abt += cell_v(t.i0 + o, a.nvx, a.dvx) * (double)h[o];
            }
        }
    };

    // planes k0 - 2 .. k0 + 1 advanced in velocity before the x sweep starts
    T hmm[TI], hm[TI], h0[TI], h1[TI], h2[TI], fp[TI];
    T raw[R], rawn[R];
    load_plane(t.k0 - 2, raw);
    load_plane(t.k0 - 1, rawn);
    velocity(t.k0 - 2, raw, hmm);
    load_plane(t.k0, raw);
    velocity(t.k0 - 1, rawn, hm);
    load_plane(t.k0 + 1, rawn);
    velocity(t.k0, raw, h0);
    load_plane(t.k0 + 2, raw);
    velocity(t.k0 + 1, rawn, h1);
    {
        T gh[TI];
#pragma unroll
        for (int o = 0; o < TI; ++o) gh[o] = a.x_on ? ghost_value(a, t.i0 + o, j, t.jok) : T(0);
        x_first_face<T, TI>(hmm, hm, h0, h1, gh, c, up, t.k0, a.nx, fp);
    }

    double spe = 0.0, ssee = 0.0, stop = 0.0;
    for (int k = t.k0; k < t.k1; ++k) {
        load_plane(k + 3, rawn);               // reads nothing useful near the end
        velocity(k + 2, raw, h2);
        T out[TI];
        x_update<T, TI>(hm, h0, h1, h2, c, up, k <= 0 || k >= a.nx - 1, k + 1 >= a.nx - 1, fp, out);
        {
            const rsrc_t po = make_rsrc(a.fout + (size_t)k * t.plane, t.pbytes);
#pragma unroll
            for (int o = 0; o < TI; ++o) bstore<T>(out[o], po, vo[o + 2], 0);
        }
        plane_moments<T, TI>(a, t, k, out, j, ring, wsum, spe, ssee, stop);
#pragma unroll
        for (int o = 0; o < TI; ++o) {
            hm[o] = h0[o];
            h0[o] = h1[o];
            h1[o] = h2[o];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) raw[r] = rawn[r];
    }
    tile_partials(a, t, it, kci, j, B, wsum, red, lv, spe, ssee, stop, abw, abt, true);
}

// ------------------------------------------------------------ fast bodies
// Tiles whose rows and halo rows lie inside the v_x grid, off its first and
// last cell, and all move the same way in x (UP: v_x > 0; else v_x <= 0):
// no per-row lane masks, edge tests or direction choices, and each row keeps
// only the planes its upwind faces read.  Rows are addressed by one lane
// offset and a scalar row offset.

template <typename T, int TI, bool UP>
__device__ __forceinline__ void sweep2_forward_fast(const SweepArgs<T>& a, int it, int kci, double* smem, int j,
                                                    int B)
{
    constexpr int R = TI + 4;
    const Tile2<T> t = tile2(a, it, kci, j, B, TI);
    T* xb = reinterpret_cast<T*>(smem);                                  // [2][R][W]
    double* wsum = reinterpret_cast<double*>(xb + 2 * R * t.W);          // [kc][nw]
    double* red = wsum + a.kc * t.nw;                                    // [nw][6]
    T* tab = reinterpret_cast<T*>(red + t.nw * 6) + t.wave * 2 * (a.kc + 4);
    T* ring = reinterpret_cast<T*>(red + t.nw * 6) + t.nw * 2 * (a.kc + 4) + t.wave * 256;   // [4][64]
    for (int m = j; m < 2 * R; m += B) {
        xb[m * t.W] = T(0);
        xb[m * t.W + 1] = T(0);
        xb[m * t.W + t.W - 2] = T(0);
        xb[m * t.W + t.W - 1] = T(0);
    }
    const int es = (int)sizeof(T);
    const int vb = t.jok ? (t.i0 - 2) * t.rb + j * es : kIdleLaneOffset;   // row i0 - 2 of this lane
    // Courant number and the face coefficient of each row: (1 - c)/2 for
    // v_x > 0, -(1 + c)/2 for v_x <= 0
    T c[R], hc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        c[r] = a.x_on ? T(cell_v(t.i0 - 2 + r, a.nvx, a.dvx) * a.dt_dx) : T(0);
        hc[r] = UP ? T(0.5) * (T(1) - c[r]) : -(T(0.5) * (T(1) + c[r]));
    }
    auto load_plane = [&](int kk, T (&dst)[R]) {
        const bool in = kk >= 0 && kk < a.nx;
        const rsrc_t pr = make_rsrc(a.fin + (size_t)(in ? kk : 0) * t.plane, in ? t.pbytes : 0u);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r] = bload<T>(pr, vb, r * t.rb);
    };
    // window: UP rows read planes k-1, k, k+1 (prefetch k+2); the others
    // k, k+1, k+2 (prefetch k+3).  q0, q1, q2 hold them in that order.
    T q0[R], q1[R], q2[R], qn[R], fp[R];
    if (UP) {
        T qmm[R];
        load_plane(t.k0 - 2, qmm);
        load_plane(t.k0 - 1, q0);
        load_plane(t.k0, q1);
        load_plane(t.k0 + 1, q2);
        const bool zm = t.k0 - 1 <= 0 || t.k0 - 1 >= a.nx - 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T s = zm ? T(0) : minmod(q0[r] - qmm[r], q1[r] - q0[r]);
            fp[r] = t.k0 == 0 ? (a.x_on ? ghost_value(a, t.i0 - 2 + r, j, t.jok) : T(0)) : q0[r] + hc[r] * s;
        }
    } else {
        load_plane(t.k0 - 1, qn);
        load_plane(t.k0, q0);
        load_plane(t.k0 + 1, q1);
        load_plane(t.k0 + 2, q2);
        const bool z0 = t.k0 <= 0 || t.k0 >= a.nx - 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T s = z0 ? T(0) : minmod(q0[r] - qn[r], q1[r] - q0[r]);
            fp[r] = q0[r] + hc[r] * s;
        }
    }
    for (int m = t.lane; m < t.k1 - t.k0; m += 64) {
        tab[m] = T(a.dxk[t.k0 + m]);
        tab[a.kc + 4 + m] = T(a.srck[t.k0 + m]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    double lv = 0.0, spe = 0.0, ssee = 0.0, stop = 0.0;
    const T dy = T(a.dy);
    const rsrc_t psrc = make_rsrc(a.fsrc, t.pbytes);
    for (int k = t.k0; k < t.k1; ++k) {
        const T d_k = tab[k - t.k0];
        const T s_k = tab[a.kc + 4 + k - t.k0];
        load_plane(UP ? k + 2 : k + 3, qn);   // the next iteration's newest plane

        // x sweep on all R rows: the face right of plane k carries plane k's
        // value (UP) or plane k + 1's (else), moved by the limited slope
        // (one uniform branch: the slope is zero in the first and last plane)
        const bool z = UP ? (k <= 0 || k >= a.nx - 1) : (k + 1 >= a.nx - 1);
        T u[R];
        if (z) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T cur = UP ? q1[r] : q0[r];
                u[r] = cur - c[r] * (q1[r] - fp[r]);
                fp[r] = q1[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T f = q1[r] + hc[r] * minmod(q1[r] - q0[r], q2[r] - q1[r]);
                const T cur = UP ? q1[r] : q0[r];
                u[r] = cur - c[r] * (f - fp[r]);
                fp[r] = f;
            }
        }
        // v_x sweep by a_x(x_k): interior rows, no box edge in the tile
        T f2[TI];
        {
            T sl[R];
#pragma unroll
            for (int r = 1; r < R - 1; ++r) sl[r] = minmod(u[r] - u[r - 1], u[r + 1] - u[r]);
            if (d_k > T(0)) {
                const T h = T(0.5) * (T(1) - d_k);
#pragma unroll
                for (int o = 0; o < TI; ++o)
                    f2[o] = u[o + 2] - d_k * ((u[o + 2] + h * sl[o + 2]) - (u[o + 1] + h * sl[o + 1]));
            } else {
                const T h = T(0.5) * (T(1) + d_k);
#pragma unroll
                for (int o = 0; o < TI; ++o)
                    f2[o] = u[o + 2] - d_k * ((u[o + 3] - h * sl[o + 3]) - (u[o + 2] - h * sl[o + 2]));
            }
        }
        // v_y sweep by a_y
        T f3[TI];
        lv += vy_update<T, TI>(f2, f3, xb + (k & 1) * R * t.W, t.W, j, a.nvy, dy, true, 0, TI);
        // band source (Eq 7)
        if (s_k != T(0)) {
#pragma unroll
            for (int r = 0; r < TI; ++r) f3[r] += s_k * bload<T>(psrc, vb, (r + 2) * t.rb);
        }
        {
            const rsrc_t po = make_rsrc(a.fout + (size_t)k * t.plane, t.pbytes);
            if (a.store_nt) {
#pragma unroll
                for (int r = 0; r < TI; ++r) bstore<T, kCpStream>(f3[r], po, vb, (r + 2) * t.rb);
            } else {
#pragma unroll
                for (int r = 0; r < TI; ++r) bstore<T>(f3[r], po, vb, (r + 2) * t.rb);
            }
        }
        plane_moments<T, TI>(a, t, k, f3, j, ring, wsum, spe, ssee, stop);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            q0[r] = q1[r];
            q1[r] = q2[r];
            q2[r] = qn[r];
        }
    }
    tile_partials(a, t, it, kci, j, B, wsum, red, lv, spe, ssee, stop, 0.0, 0.0, false);
}

template <typename T, int TI, bool UP>
__device__ __forceinline__ void sweep2_reversed_fast(const SweepArgs<T>& a, int it, int kci, double* smem, int j,
                                                     int B)
{
    constexpr int R = TI + 4;
    const Tile2<T> t = tile2(a, it, kci, j, B, TI);
    T* xb = reinterpret_cast<T*>(smem);                                  // [2][R][W]
    double* wsum = reinterpret_cast<double*>(xb + 2 * R * t.W);          // [kc][nw]
    double* red = wsum + a.kc * t.nw;                                    // [nw][6]
    T* tab = reinterpret_cast<T*>(red + t.nw * 6) + t.wave * 2 * (a.kc + 4);
    T* ring = reinterpret_cast<T*>(red + t.nw * 6) + t.nw * 2 * (a.kc + 4) + t.wave * 256;   // [4][64]
    for (int m = j; m < 2 * R; m += B) {
        xb[m * t.W] = T(0);
        xb[m * t.W + 1] = T(0);
        xb[m * t.W + t.W - 2] = T(0);
        xb[m * t.W + t.W - 1] = T(0);
    }
    const int es = (int)sizeof(T);
    const int vb = t.jok ? (t.i0 - 2) * t.rb + j * es : kIdleLaneOffset;
    T c[TI], hc[TI];
#pragma unroll
    for (int o = 0; o < TI; ++o) {
        c[o] = a.x_on ? T(cell_v(t.i0 + o, a.nvx, a.dvx) * a.dt_dx) : T(0);
        hc[o] = UP ? T(0.5) * (T(1) - c[o]) : -(T(0.5) * (T(1) + c[o]));
    }
    for (int m = t.lane; m < t.k1 - t.k0 + 4; m += 64) {
        const int kk = t.k0 - 2 + m;
        const bool in = kk >= 0 && kk < a.nx;
        tab[m] = in ? T(a.dxk[kk]) : T(0);
        tab[a.kc + 4 + m] = in ? T(a.srck[kk]) : T(0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    auto load_plane = [&](int kk, T (&dst)[R]) {
        const bool in = kk >= 0 && kk < a.nx;
        const rsrc_t pr = make_rsrc(a.fin + (size_t)(in ? kk : 0) * t.plane, in ? t.pbytes : 0u);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r] = bload<T>(pr, vb, r * t.rb);
    };
    const rsrc_t psrc = make_rsrc(a.fsrc, t.pbytes);
    const T dy = T(a.dy);
    double lv = 0.0, abw = 0.0, abt = 0.0;
    // the velocity part of plane p (source, v_y, v_x); interior rows, so no
    // box edge in v_x; the chunk's own planes tally the v_y loss and the
    // absorbed fluxes
    auto velocity = [&](int p, const T (&raw)[R], T (&h)[TI]) {
        const T d_p = tab[p - t.k0 + 2];
        const T s_p = tab[a.kc + 4 + p - t.k0 + 2];
        T g[R];
#pragma unroll
        for (int r = 0; r < R; ++r) g[r] = raw[r];
        if (s_p != T(0)) {
#pragma unroll
            for (int r = 0; r < R; ++r) g[r] += s_p * bload<T>(psrc, vb, r * t.rb);
        }
        T y[R];
        const double lvy = vy_update<T, R>(g, y, xb + (p & 1) * R * t.W, t.W, j, a.nvy, dy, true, 2, TI + 2);
        T sl[R];
#pragma unroll
        for (int r = 1; r < R - 1; ++r) sl[r] = minmod(y[r] - y[r - 1], y[r + 1] - y[r]);
        if (d_p > T(0)) {
            const T hh = T(0.5) * (T(1) - d_p);
#pragma unroll
            for (int o = 0; o < TI; ++o)
                h[o] = y[o + 2] - d_p * ((y[o + 2] + hh * sl[o + 2]) - (y[o + 1] + hh * sl[o + 1]));
        } else {
            const T hh = T(0.5) * (T(1) + d_p);
#pragma unroll
            for (int o = 0; o < TI; ++o)
                h[o] = y[o + 2] - d_p * ((y[o + 3] - hh * sl[o + 3]) - (y[o + 2] - hh * sl[o + 2]));
        }
        if (p >= t.k0 && p < t.k1) {
            lv += lvy;
            if (!UP && p == 0 && t.jok) {
#pragma unroll
                for (int o = 0; o < TI; ++o)
                    if (2 * (t.i0 + o) + 1 < a.nvx) abw += -cell_v(t.i0 + o, a.nvx, a.dvx) * (double)h[o];
            }
            if (UP && p == a.nx - 1 && t.jok) {
#pragma unroll
                for (int o = 0; o < TI; ++o) abt += cell_v(t.i0 + o, a.nvx, a.dvx) * (double)h[o];
            }
        }
    };

    // the x window after the velocity part: UP rows read planes k-1, k, k+1
    // (the velocity part runs one plane ahead), the others k, k+1, k+2 (two
    // ahead); g0, g1, g2 hold them in that order
    constexpr int AHEAD = UP ? 1 : 2;
    T g0[TI], g1[TI], g2[TI], fp[TI];
    T raw[R], rawn[R];
    if (UP) {
        T gm[TI];
        load_plane(t.k0 - 2, raw);
        load_plane(t.k0 - 1, rawn);
        velocity(t.k0 - 2, raw, gm);
        load_plane(t.k0, raw);
        velocity(t.k0 - 1, rawn, g0);
        load_plane(t.k0 + 1, rawn);
        velocity(t.k0, raw, g1);
        const bool zm = t.k0 - 1 <= 0 || t.k0 - 1 >= a.nx - 1;
#pragma unroll
        for (int o = 0; o < TI; ++o) {
            const T s = zm ? T(0) : minmod(g0[o] - gm[o], g1[o] - g0[o]);
            fp[o] = t.k0 == 0 ? (a.x_on ? ghost_value(a, t.i0 + o, j, t.jok) : T(0)) : g0[o] + hc[o] * s;
        }
        // rawn holds plane k0 + 1, the loop's first velocity plane
#pragma unroll
        for (int r = 0; r < R; ++r) raw[r] = rawn[r];
    } else {
        T gm[TI];
        load_plane(t.k0 - 1, raw);
        load_plane(t.k0, rawn);
        velocity(t.k0 - 1, raw, gm);
        load_plane(t.k0 + 1, raw);
        velocity(t.k0, rawn, g0);
        load_plane(t.k0 + 2, rawn);
        velocity(t.k0 + 1, raw, g1);
        const bool z0 = t.k0 <= 0 || t.k0 >= a.nx - 1;
#pragma unroll
        for (int o = 0; o < TI; ++o) {
            const T s = z0 ? T(0) : minmod(g0[o] - gm[o], g1[o] - g0[o]);
            fp[o] = g0[o] + hc[o] * s;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) raw[r] = rawn[r];   // plane k0 + 2
    }

    double spe = 0.0, ssee = 0.0, stop = 0.0;
    for (int k = t.k0; k < t.k1; ++k) {
        load_plane(k + AHEAD + 1, rawn);       // reads nothing useful near the end
        velocity(k + AHEAD, raw, g2);
        // UP: window planes k-1 (g0), k (g1), k+1 (g2); else k, k+1, k+2.
        // One uniform branch: the slope is zero in the first and last plane.
        const bool z = UP ? (k <= 0 || k >= a.nx - 1) : (k + 1 >= a.nx - 1);
        T out[TI];
        if (z) {
#pragma unroll
            for (int o = 0; o < TI; ++o) {
                out[o] = (UP ? g1[o] : g0[o]) - c[o] * (g1[o] - fp[o]);
                fp[o] = g1[o];
            }
        } else {
#pragma unroll
            for (int o = 0; o < TI; ++o) {
                const T f = g1[o] + hc[o] * minmod(g1[o] - g0[o], g2[o] - g1[o]);
                out[o] = (UP ? g1[o] : g0[o]) - c[o] * (f - fp[o]);
                fp[o] = f;
            }
        }
        {
            const rsrc_t po = make_rsrc(a.fout + (size_t)k * t.plane, t.pbytes);
            if (a.store_nt) {
#pragma unroll
                for (int o = 0; o < TI; ++o) bstore<T, kCpStream>(out[o], po, vb, (o + 2) * t.rb);
            } else {
#pragma unroll
                for (int o = 0; o < TI; ++o) bstore<T>(out[o], po, vb, (o + 2) * t.rb);
            }
        }
        plane_moments<T, TI>(a, t, k, out, j, ring, wsum, spe, ssee, stop);
#pragma unroll
        for (int o = 0; o < TI; ++o) {
            g0[o] = g1[o];
            g1[o] = g2[o];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) raw[r] = rawn[r];
    }
    tile_partials(a, t, it, kci, j, B, wsum, red, lv, spe, ssee, stop, abw, abt, true);
}

// Main launch: the tiles with a fast body (tile list entries first).
// Waves per SIMD the fast bodies are compiled for (FP32: 4-row tiles 4,
// 8-row tiles 3; FP64: 2), which caps their registers at 512 / waves.
template <typename T, int TI>
constexpr int sweep2_waves()
{
    return sizeof(T) == 4 ? (TI <= 4 ? 4 : 3) : 2;
}

template <typename T, int TI, int MAXB, bool REV>
__global__ void __launch_bounds__(MAXB, (sweep2_waves<T, TI>())) k_sweep2_fast(SweepArgs<T> a)
{
    extern __shared__ double smem[];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int it = a.tile_list[wg % a.n_list];
    const int kci = wg / a.n_list;
    const bool up = tile2_side(it, TI, a.nvx) > 0;
    if (REV) {
        if (up) sweep2_reversed_fast<T, TI, true>(a, it, kci, smem, threadIdx.x, blockDim.x);
        else sweep2_reversed_fast<T, TI, false>(a, it, kci, smem, threadIdx.x, blockDim.x);
    } else {
        if (up) sweep2_forward_fast<T, TI, true>(a, it, kci, smem, threadIdx.x, blockDim.x);
        else sweep2_forward_fast<T, TI, false>(a, it, kci, smem, threadIdx.x, blockDim.x);
    }
}

// Every tile in one launch: workgroups [0, n_gen) (a multiple of 8, the
// last ones idle if needed) take the other tiles with the generic bodies and
// start first; the rest take the fast tiles.  Each part keeps its own
// XCD-aware order (n_gen a multiple of 8 leaves every workgroup on the XCD
// its own part assigns it).
template <typename T, int TI, int MAXB, bool REV>
__global__ void __launch_bounds__(MAXB, (sweep2_waves<T, TI>())) k_sweep2_all(SweepArgs<T> a, const int* tiles,
                                                                            int n_fast, int n_generic, int n_gen,
                                                                            int n_kc)
{
    extern __shared__ double smem[];
    const int b = blockIdx.x;
    if (b < n_gen) {
        const int count = n_generic * n_kc;
        const int wg = xcd_remap(b, n_gen);
        if (wg >= count) return;
        const int it = tiles[n_fast + wg % n_generic];
        const int kci = wg / n_generic;
        if (REV) sweep2_reversed<T, TI>(a, it, kci, smem, threadIdx.x, blockDim.x);
        else sweep2_forward<T, TI>(a, it, kci, smem, threadIdx.x, blockDim.x);
        return;
    }
    const int wg = xcd_remap(b - n_gen, (int)gridDim.x - n_gen);
    const int it = tiles[wg % n_fast];
    const int kci = wg / n_fast;
    const bool up = tile2_side(it, TI, a.nvx) > 0;
    if (REV) {
        if (up) sweep2_reversed_fast<T, TI, true>(a, it, kci, smem, threadIdx.x, blockDim.x);
        else sweep2_reversed_fast<T, TI, false>(a, it, kci, smem, threadIdx.x, blockDim.x);
    } else {
        if (up) sweep2_forward_fast<T, TI, true>(a, it, kci, smem, threadIdx.x, blockDim.x);
        else sweep2_forward_fast<T, TI, false>(a, it, kci, smem, threadIdx.x, blockDim.x);
    }
}

// The other tiles (edge tiles, tiles whose rows straddle v_x = 0): the
// generic bodies with per-row masks.
template <typename T, int TI, int MAXB, bool REV>
__global__ void __launch_bounds__(MAXB) k_sweep2(SweepArgs<T> a)
{
    extern __shared__ double smem[];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int it = a.tile_list[wg % a.n_list];
    const int kci = wg / a.n_list;
    if (REV) sweep2_reversed<T, TI>(a, it, kci, smem, threadIdx.x, blockDim.x);
    else sweep2_forward<T, TI>(a, it, kci, smem, threadIdx.x, blockDim.x);
}

}  // namespace fk
