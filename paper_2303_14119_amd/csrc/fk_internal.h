// fk_internal.h -- definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "flashkin.h"

namespace fk {

// CODATA 2018 (the paper states no values)
constexpr double kE = 1.602176634e-19;     // elementary charge, C
constexpr double kMe = 9.1093837015e-31;   // electron mass, kg
constexpr double kEps0 = 8.8541878128e-12; // vacuum permittivity, F/m
constexpr double kPi = 3.14159265358979323846;

constexpr uint32_t kFlagCfl = 1u;
constexpr uint32_t kFlagNonfinite = 2u;

constexpr int kFieldThreads = 1024;  // one workgroup runs the reduction/field kernel
constexpr size_t kLdsBudget = 64 * 1024;

// Scalars of the current state, in device memory, written only by the
// reduction/field kernel (and by the host through fk_write_state).
struct DevState {
    int64_t step;
    double sigma, sigma_lo;      // Neumaier pair: sigma^n = sigma + sigma_lo
    double g_pe, g_see, g_top;   // fluxes of f^n (Eq 13-14)
    double emitted;              // flux of the emission row built from g_see
    double loss_v, n_total, resid;
    double gscale;               // emission row = gscale * ghat
    double courant_vx_max;       // largest |a_x| dt / dv_x seen
    uint32_t flags;
    uint32_t pad;
};

// Derived grid, step and launch shape of a parameter set (host side).
struct Layout {
    double dx, dvx, dvy, dt;
    double courant_x, courant_vy;
    double dy;                   // signed v_y Courant number a_y dt / dv_y
    int64_t cells;
    int elem;                    // bytes per f element
    int bgk;                     // 1: the collision term (FK_PHYS_BGK) is on
    int scheme;                  // FK_SCHEME_UPWIND or FK_SCHEME_LIMITED2
    int block;                   // threads of the sweep workgroup (one per v_y column)
    int ti;                      // v_x rows per tile
    int kc;                      // x planes per tile
    int n_it, n_kc, nwg;
    int n_fast, n_generic;       // v_x tiles taking the fast / generic sweep body
    int n_it_cap, nwg_cap;       // partial-buffer capacities (any tiling fits)
    size_t lds_sweep, lds_moments;
    uint64_t bytes_device;
};

int derive_layout(const fk_params* p, Layout* L, std::string* why);
size_t sweep_lds(int ti, int block, int kc, int elem, bool bgk);
// LDS of a second-order sweep workgroup: the v_y exchange of TI + 4 rows with
// two halo columns each side (double-buffered), the plane sums, the
// reduction slots and each wave's per-plane coefficients for the chunk and
// two planes on each side
size_t sweep2_lds(int ti, int block, int kc, int elem);

// Number of rows among r = 0..ti+1 of v_x tile `it` (rows i = it*ti - 1 + r)
// with v_x <= 0, i.e. 2 i + 1 <= nvx: the split point of the fast sweep body.
__host__ __device__ inline int tile_split(int it, int ti, int nvx)
{
    int s = 0;
    for (int r = 0; r < ti + 2; ++r)
        if (2 * (it * ti - 1 + r) + 1 <= nvx) ++s;
    return s;
}

// Whether tile `it` takes the main launch's fast body: full and split at
// 0, 1, ti+1 or ti+2.
__host__ __device__ inline bool tile_is_fast(int it, int ti, int nvx)
{
    if ((it + 1) * ti > nvx) return false;
    const int s = tile_split(it, ti, nvx);
    return s == 0 || s == 1 || s == ti + 1 || s == ti + 2;
}

// Of the other tiles, those with a compiled fast body in the second launch:
// tiles of 4 or 8 rows, full (split inside the tile) or ragged at +v_max
// with every row at v_x > 0.
__host__ __device__ inline bool tile_is_special(int it, int ti, int nvx)
{
    if ((ti != 4 && ti != 8) || tile_is_fast(it, ti, nvx)) return false;
    return (it + 1) * ti <= nvx || tile_split(it, ti, nvx) == 0;
}
// Second-order tiles with a compiled fast body: every row of the tile and its
// two halo rows on each side lies inside the v_x grid and off its first and
// last cell, and all of them move the same way in x (v_x > 0 for all, or
// v_x <= 0 for all).  Returns +1 (v_x > 0), -1 (v_x <= 0) or 0 (other).
__host__ __device__ inline int tile2_side(int it, int ti, int nvx)
{
    const int lo = it * ti - 2, hi = it * ti + ti + 1;   // rows i0 - 2 .. i0 + ti + 1
    if (lo < 1 || hi > nvx - 2) return 0;
    if (2 * lo + 1 > nvx) return 1;
    if (2 * hi + 1 <= nvx) return -1;
    return 0;
}

// Whether tile `it` goes to the main sweep launch of its scheme.
__host__ __device__ inline bool tile_main(int it, int ti, int nvx, int scheme)
{
    return scheme == FK_SCHEME_LIMITED2 ? tile2_side(it, ti, nvx) != 0 : tile_is_fast(it, ti, nvx);
}

int set_error(std::string* slot, int code, const std::string& msg);
// error of the calling thread's last failed call that has no object, from a
// message with static storage (no allocation)
int set_static_error(int code, const char* msg);
const char* global_error();

// Block of device buffers of one instance (owned by a context or a batch).
struct Buffers {
    void* f[2];
    double* delta;    // [nvx][nvy]
    double* ghat;     // [nvx][nvy]
    double* fsrc64;   // [nvx][nvy], normalised, FP64
    void* fsrc;       // [nvx][nvy], normalised, element type of f
    double* wband;    // [nx]
    double* srck;     // [nx], dt (J/e) w_k / (x_hi - x_lo) or 0
    double* part_n;   // [n_it][nx]  plane sums of each v_x tile
    double* part_wall;// [n_it][2]
    double* part_top; // [n_it]
    double* part_lv;  // [nwg]
    double* part_abs; // [n_it][2]: absorbed at the wall and at x = L (reversed second-order steps)
    double* plane_sum;// [nx]   plane sums reduced over the v_x tiles (single contexts)
    double* ne;       // [nx]
    double* ex;       // [nx]
    double* dxk;      // [nx], v_x Courant number of each plane
    double* nudt;     // [nx], nu_ee(n_k) dt of each plane (collision term)
    double* nudt_n;   // [nx], nu_ee(n_k) dt n_k
    void* gx;         // [nvx], v_x factor of the normalised equilibrium, element type of f
    void* gy;         // [nvy], v_y factor
    double* consts;   // [4]: zsum, srcnorm, injected per step, emission prefactor
    int* tiles;       // [n_it]: fast v_x tiles, then generic ones
    DevState* st;
    fk_state* ring;   // [trace_cap]
};

}  // namespace fk
