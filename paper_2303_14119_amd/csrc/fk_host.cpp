// fk_host.cpp -- host-only parts of the C-ABI: parameter validation, the
// derived layout, error strings and the saturation test.  Nothing here
// touches the GPU, so these calls work on machines without one.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fk_internal.h"

namespace fk {

static thread_local std::string g_create_error;
static thread_local const char* g_static_error = nullptr;   // set by calls that must not allocate

const char* global_error() { return g_static_error ? g_static_error : g_create_error.c_str(); }

int set_error(std::string* slot, int code, const std::string& msg)
{
    if (slot) {
        *slot = msg;
    } else {
        g_static_error = nullptr;
        g_create_error = msg;
    }
    return code;
}

int set_static_error(int code, const char* msg)
{
    g_static_error = msg;
    return code;
}

// LDS of a sweep workgroup: the v_y exchange rows, the plane sums, the
// reduction slots and each wave's table of per-plane coefficients (2 per
// plane; with the collision term 4 per plane and the tile's rows of the
// v_x factor of the equilibrium)
size_t sweep_lds(int ti, int block, int kc, int elem, bool bgk)
{
    const int waves = (block + 63) / 64;
    const size_t tab = bgk ? (size_t)4 * kc + ti : (size_t)2 * kc;
    return (size_t)2 * ti * (block + 2) * elem + (size_t)kc * waves * 8 + (size_t)waves * 4 * 8 + (size_t)waves * tab * elem;
}

size_t sweep2_lds(int ti, int block, int kc, int elem)
{
    const int waves = (block + 63) / 64;
    return (size_t)2 * (ti + 4) * (block + 4) * elem + (size_t)kc * waves * 8 + (size_t)waves * 6 * 8 +
           (size_t)waves * 2 * (kc + 4) * elem + (size_t)waves * 256 * elem;
}

int derive_layout(const fk_params* p, Layout* L, std::string* why)
{
    auto bad = [&](const char* m) { if (why) *why = m; return FK_E_INVALID; };
    if (!p) return bad("params is NULL");
    if (p->struct_size != sizeof(fk_params)) return bad("params.struct_size != sizeof(fk_params)");
    if (p->abi_version != FK_ABI_VERSION) return bad("params.abi_version does not match FK_ABI_VERSION");
    if (p->nx < 1 || p->nvx < 1 || p->nvy < 1) return bad("nx, nvx and nvy must be >= 1");
    if (p->nvy > 1024) return bad("nvy must be <= 1024 (one v_y column per thread of a workgroup)");
    if (p->dtype != FK_F32 && p->dtype != FK_F64) return bad("dtype must be FK_F32 or FK_F64");
    if (!(p->length_m > 0) || !(p->vmax_x > 0) || !(p->vmax_y > 0)) return bad("length_m, vmax_x, vmax_y must be > 0");
    if (!(p->dt >= 0) || !std::isfinite(p->dt)) return bad("dt must be >= 0 and finite");
    if (p->dt == 0 && !(p->cfl > 0 && p->cfl <= 1)) return bad("cfl must be in (0, 1] when dt = 0");
    if (!std::isfinite(p->ey) || !std::isfinite(p->ex_external)) return bad("fields must be finite");
    if (!(p->delta_max >= 0) || !(p->a_max_ev > 0) || !(p->ks >= 0)) return bad("SEY parameters out of range");
    if (!(p->t_se_ev > 0) || !(p->t_src_ev > 0)) return bad("temperatures must be > 0");
    if (!(p->j_src >= 0) || !std::isfinite(p->j_src)) return bad("j_src must be >= 0");
    if (!(p->x_src_hi >= p->x_src_lo)) return bad("x_src_hi must be >= x_src_lo");
    if (p->emission_norm != FK_EMIT_DISCRETE && p->emission_norm != FK_EMIT_ANALYTIC) return bad("bad emission_norm");
    if (p->physics_mask & ~(uint32_t)(FK_PHYS_ALL | FK_PHYS_BGK | FK_PHYS_NO_SPACE_CHARGE)) return bad("unknown physics_mask bits");
    const bool bgk = (p->physics_mask & FK_PHYS_BGK) != 0;
    if (bgk && !(p->t_e_ev > 0 && std::isfinite(p->t_e_ev))) return bad("t_e_ev must be > 0 and finite with FK_PHYS_BGK");
    if (bgk && !(p->ln_lambda > 0 && std::isfinite(p->ln_lambda))) return bad("ln_lambda must be > 0 and finite with FK_PHYS_BGK");
    if (!(p->r_refl >= 0 && p->r_refl <= 1)) return bad("r_refl must be in [0, 1]");
    if (!(p->r_inel >= 0 && p->r_inel <= 1 - p->r_refl)) return bad("r_inel must be in [0, 1 - r_refl]");
    if (p->scheme != FK_SCHEME_UPWIND && p->scheme != FK_SCHEME_LIMITED2) return bad("scheme must be FK_SCHEME_UPWIND or FK_SCHEME_LIMITED2");
    if (p->scheme == FK_SCHEME_LIMITED2 && bgk) return bad("FK_SCHEME_LIMITED2 does not take FK_PHYS_BGK");
    if (p->reserved0 != 0) return bad("reserved0 must be 0");
    if (p->trace_stride < 1 || p->trace_cap < 1) return bad("trace_stride and trace_cap must be >= 1");
    if (p->tile_rows != 0 && p->tile_rows != 4 && p->tile_rows != 8 && p->tile_rows != 12 && p->tile_rows != 16)
        return bad("tile_rows must be 0, 4, 8, 12 or 16");
    if (p->tile_planes != 0 && (p->tile_planes < 4 || p->tile_planes > 128))
        return bad("tile_planes must be 0 or in [4, 128]");

    const int64_t cells = (int64_t)p->nx * p->nvx * p->nvy;
    if (cells > ((int64_t)1 << 40)) return bad("grid too large");
    // one x plane is addressed through a buffer descriptor with 32-bit offsets
    if ((int64_t)p->nvx * p->nvy * (p->dtype == FK_F32 ? 4 : 8) > ((int64_t)1 << 30))
        return bad("one x plane (nvx * nvy elements) must be at most 1 GiB");

    Layout l{};
    l.cells = cells;
    l.elem = p->dtype == FK_F32 ? 4 : 8;
    l.bgk = bgk ? 1 : 0;
    l.dx = p->length_m / p->nx;
    l.dvx = 2.0 * p->vmax_x / p->nvx;
    l.dvy = 2.0 * p->vmax_y / p->nvy;
    const double ay = -kE * p->ey / kMe;
    if (p->dt > 0) {
        l.dt = p->dt;
    } else {
        double tmin = l.dx / p->vmax_x;
        if (ay != 0) {
            tmin = std::fmin(tmin, l.dvx / std::fabs(ay));
            tmin = std::fmin(tmin, l.dvy / std::fabs(ay));
        }
        l.dt = p->cfl * tmin;
    }
    const double vx_edge = p->vmax_x - 0.5 * l.dvx;   // largest |v_x| of a cell centre
    l.courant_x = (p->physics_mask & FK_PHYS_X) ? vx_edge * l.dt / l.dx : 0.0;
    l.dy = (p->physics_mask & FK_PHYS_VY) ? ay * l.dt / l.dvy : 0.0;
    l.courant_vy = std::fabs(l.dy);
    if (l.courant_x > 1.0) { if (why) *why = "x Courant number exceeds 1"; return FK_E_CFL; }
    if (l.courant_vy > 1.0) { if (why) *why = "v_y Courant number exceeds 1"; return FK_E_CFL; }

    // launch shape: one thread per v_y column; tiles of ti v_x rows and kc x planes
    l.block = ((p->nvy + 63) / 64) * 64;
    l.scheme = p->scheme;
    if (p->scheme == FK_SCHEME_LIMITED2) {
        // second order: 4-row tiles by default (four waves per SIMD; 8-row
        // tiles hold three and ran slower at every chunk length measured);
        // the tiles with a fast body and the rest take one launch each
        int ti = p->tile_rows;
        if (ti == 0) ti = 4;
        if (ti != 4 && ti != 8) return bad("FK_SCHEME_LIMITED2 takes tile_rows 4 or 8");
        if (sweep2_lds(ti, l.block, 4, l.elem) > kLdsBudget)
            return bad("FK_SCHEME_LIMITED2: the v_y exchange does not fit in LDS (nvy up to 768 in FP32 with 4-row tiles, "
                       "512 with 8; 384 in FP64)");
        l.ti = ti;
        l.n_it = (p->nvx + ti - 1) / ti;
        int kc = p->tile_planes;
        if (kc == 0) {
            // short chunks: the sweep is bound by the vector ALU, and many
            // small workgroups balance the slower edge tiles; 32 planes, or
            // 16 where that leaves fewer than 2048 workgroups
            kc = 32;
            if ((int64_t)l.n_it * ((p->nx + 31) / 32) < 2048) kc = 16;
            while (kc > 4 && sweep2_lds(ti, l.block, kc, l.elem) > kLdsBudget) kc /= 2;
        }
        if (kc > p->nx) kc = p->nx;
        l.kc = kc;
        l.n_kc = (p->nx + kc - 1) / kc;
        l.nwg = l.n_it * l.n_kc;
        l.n_fast = 0;
        for (int it = 0; it < l.n_it; ++it) l.n_fast += tile2_side(it, ti, p->nvx) != 0 ? 1 : 0;
        l.n_generic = l.n_it - l.n_fast;
        l.lds_sweep = sweep2_lds(ti, l.block, kc, l.elem);
        l.lds_moments = (size_t)kc * (l.block / 64) * 8 + (size_t)(l.block / 64) * 4 * 8;
        if (l.lds_sweep > kLdsBudget) return bad("tile needs more LDS than a workgroup has; lower tile_planes");
        l.n_it_cap = (p->nvx + 3) / 4;
        l.nwg_cap = l.n_it_cap * ((p->nx + 3) / 4);
        const uint64_t v2 = (uint64_t)p->nvx * p->nvy;
        l.bytes_device = 2ull * cells * l.elem + v2 * (8 * 3 + l.elem) + (uint64_t)p->nx * 8 * 9 +
                         (uint64_t)(p->nvx + p->nvy) * l.elem +
                         (uint64_t)p->nx * l.n_it_cap * 8 + (uint64_t)l.n_it_cap * 44 + (uint64_t)l.nwg_cap * 8 +
                         sizeof(DevState) + (uint64_t)p->trace_cap * sizeof(fk_state) + 4096;
        *L = l;
        return FK_OK;
    }
    int ti = p->tile_rows;
    if (ti == 0) {
        // FP32: 8 rows keep the fast body at four waves per SIMD, best up to
        // 256 v_y lanes; from 320 lanes (5+ waves per workgroup) 16 rows
        // halve the per-plane barrier, exchange and reduction work per row
        // and win (measured 8-12%) as long as the tile fits in LDS.  12 rows
        // fit 3 waves per SIMD (16 rows: 2), so two 6-wave workgroups share
        // a unit; they win (3-4% at 384 lanes) when every 12-row tile is
        // full and meets the v_x sign change at its edge (nvx a multiple of
        // 24); otherwise the generic body on split tiles costs more.
        // FP64: 4 rows.
        ti = l.elem == 4 ? 8 : 4;
        if (l.elem == 4 && l.block >= 320 && l.block <= 512 && sweep_lds(16, l.block, 16, l.elem, bgk) <= kLdsBudget)
            ti = 16;
        if (ti == 16 && p->nvx % 24 == 0 && sweep_lds(12, l.block, 16, l.elem, bgk) <= kLdsBudget) ti = 12;
        while (ti > 4 && sweep_lds(ti, l.block, 16, l.elem, bgk) > kLdsBudget) ti /= 2;
    }
    if (ti == 16 && (l.elem != 4 || l.block > 512)) return bad("tile_rows 16 needs FK_F32 and nvy <= 512");
    if (ti == 12 && (l.elem != 4 || l.block > 512)) return bad("tile_rows 12 needs FK_F32 and nvy <= 512");
    if (ti == 8 && l.elem == 8 && l.block > 512) return bad("tile_rows 8 with FK_F64 needs nvy <= 512");
    l.ti = ti;
    l.n_it = (p->nvx + ti - 1) / ti;
    int kc = p->tile_planes;
    if (kc == 0) {
        // enough workgroups to fill 256 compute units several times over,
        // but long enough x runs that the halo planes stay a small overhead
        const int target = 1024;
        int nkc = (target + l.n_it - 1) / l.n_it;
        kc = (p->nx + nkc - 1) / nkc;
        if (kc < 16) kc = 16;
        if (kc > 128) kc = 128;
        // wide FP64 blocks leave little LDS for the per-plane tables: shorter
        // x runs, down to 4 planes
        while (kc > 4 && sweep_lds(ti, l.block, kc, l.elem, bgk) > kLdsBudget) kc = kc > 16 ? kc - 16 : kc / 2;
    }
    if (kc > p->nx) kc = p->nx;
    l.kc = kc;
    l.n_kc = (p->nx + kc - 1) / kc;
    l.nwg = l.n_it * l.n_kc;
    l.n_fast = 0;
    for (int it = 0; it < l.n_it; ++it) l.n_fast += tile_is_fast(it, ti, p->nvx) ? 1 : 0;
    l.n_generic = l.n_it - l.n_fast;
    l.lds_sweep = sweep_lds(ti, l.block, kc, l.elem, bgk);
    l.lds_moments = (size_t)kc * (l.block / 64) * 8 + (size_t)(l.block / 64) * 4 * 8;
    if (l.lds_sweep > kLdsBudget) return bad("tile needs more LDS than a workgroup has; lower tile_rows or tile_planes");

    // partial buffers are sized for the smallest tile (4 rows, 4 planes) so a
    // context can be retiled without reallocating
    l.n_it_cap = (p->nvx + 3) / 4;
    l.nwg_cap = l.n_it_cap * ((p->nx + 3) / 4);
    const uint64_t v2 = (uint64_t)p->nvx * p->nvy;
    l.bytes_device = 2ull * cells * l.elem + v2 * (8 * 3 + l.elem) + (uint64_t)p->nx * 8 * 9 +
                     (uint64_t)(p->nvx + p->nvy) * l.elem +
                     (uint64_t)p->nx * l.n_it_cap * 8 + (uint64_t)l.n_it_cap * 44 + (uint64_t)l.nwg_cap * 8 +
                     sizeof(DevState) + (uint64_t)p->trace_cap * sizeof(fk_state) + 4096;
    *L = l;
    return FK_OK;
}

}  // namespace fk

using namespace fk;

extern "C" const char* fk_error_string(int code)
{
    switch (code) {
    case FK_OK: return "ok";
    case FK_E_INVALID: return "invalid argument";
    case FK_E_OOM: return "out of memory";
    case FK_E_HIP: return "HIP runtime error";
    case FK_E_CFL: return "Courant number above one";
    case FK_E_NONFINITE: return "non-finite moment or flux";
    case FK_E_STATE: return "call not valid in the current state";
    default: return "unknown error";
    }
}

extern "C" int fk_validate(const fk_params* p, fk_info* out)
{
    Layout L;
    std::string why;
    int rc = derive_layout(p, &L, &why);
    if (rc != FK_OK) return set_error(nullptr, rc, why);
    if (out) {
        out->dx = L.dx; out->dvx = L.dvx; out->dvy = L.dvy; out->dt = L.dt;
        out->courant_x = L.courant_x; out->courant_vy = L.courant_vy;
        out->cells = L.cells; out->tile_rows = L.ti; out->tile_planes = L.kc;
        out->block = L.block; out->n_tiles = L.nwg; out->bytes_device = L.bytes_device;
    }
    return FK_OK;
}

extern "C" int fk_saturation_check(const fk_state* tr, size_t n, double window_s, double rtol, int* out)
{
    if (!out || (!tr && n) || !(window_s > 0) || !(rtol >= 0)) return set_error(nullptr, FK_E_INVALID, "bad arguments to fk_saturation_check");
    *out = 0;
    if (n < 2) return FK_OK;
    const fk_state& last = tr[n - 1];
    // newest record at least one window older than the last one
    long ref = -1;
    for (long m = (long)n - 2; m >= 0; --m)
        if (tr[m].t <= last.t - window_s * (1.0 - 1e-12)) { ref = m; break; }
    if (ref < 0) return FK_OK;
    const fk_state& a = tr[ref];
    if (!(last.g_pe > 0)) return FK_OK;   // no electrons at the wall yet
    const double qa[3] = {a.sigma + a.sigma_lo, a.g_pe, a.g_see};
    const double qb[3] = {last.sigma + last.sigma_lo, last.g_pe, last.g_see};
    for (int q = 0; q < 3; ++q)
        if (!(std::fabs(qb[q] - qa[q]) <= rtol * std::fabs(qb[q]))) return FK_OK;
    *out = 1;
    return FK_OK;
}

