// fk_analysis.cpp -- host-only helpers around a run: the field-emission
// rate of Eq 6 that feeds the band source, and the surface charge along the
// insulator reconstructed from a 1D trace.  No GPU is touched.
#include <cmath>

#include "fk_internal.h"

using namespace fk;

extern "C" int fk_fn_current(double e_field, double phi_ev, double beta, double* j_out)
{
    if (!j_out || !(phi_ev > 0) || !std::isfinite(phi_ev) || !(beta > 0) || !std::isfinite(beta) || !std::isfinite(e_field))
        return set_error(nullptr, FK_E_INVALID, "bad arguments to fk_fn_current");
    constexpr double kPlanck = 6.62607015e-34;   // J s (exact in the 2019 SI)
    const double E = beta * std::fabs(e_field);
    const double phi = phi_ev * kE;                // work function in joules
    *j_out = 0.0;
    if (E == 0.0) return FK_OK;
    // Eq 6: pre-factor e^3 E^2 / (8 pi h phi), barrier term 8 pi sqrt(2 m) phi^1.5 / (3 e h E)
    const double pre = kE * kE * kE * E * E / (8.0 * kPi * kPlanck * phi);
    const double barrier = 8.0 * kPi * std::sqrt(2.0 * kMe) * phi * std::sqrt(phi) / (3.0 * kE * kPlanck * E);
    *j_out = pre * std::exp(-barrier);
    return FK_OK;
}

extern "C" int fk_sigma_along(const fk_state* tr, size_t n, double v_seea, double t, const double* y, size_t ny,
                              double* out)
{
    if (!(v_seea > 0) || !std::isfinite(v_seea) || !std::isfinite(t) || n < 1 || !tr || (ny && (!y || !out)))
        return set_error(nullptr, FK_E_INVALID, "bad arguments to fk_sigma_along");
    for (size_t m = 1; m < n; ++m)
        if (!(tr[m].t > tr[m - 1].t)) return set_error(nullptr, FK_E_INVALID, "trace records must increase in t");
    auto sig = [&](size_t m) { return tr[m].sigma + tr[m].sigma_lo; };
    for (size_t q = 0; q < ny; ++q) {
        const double tau = t - y[q] / v_seea;      // time since the front passed y
        double v;
        if (tau < 0.0) v = 0.0;                    // ahead of the front
        else if (tau <= tr[0].t) v = tr[0].t > 0.0 ? sig(0) * tau / tr[0].t : sig(0);
        else if (tau >= tr[n - 1].t) v = sig(n - 1);
        else {
            size_t lo = 0, hi = n - 1;             // tr[lo].t < tau <= tr[hi].t
            while (hi - lo > 1) {
                const size_t mid = (lo + hi) / 2;
                if (tr[mid].t < tau) lo = mid;
                else hi = mid;
            }
            const double w = (tau - tr[lo].t) / (tr[hi].t - tr[lo].t);
            v = (1.0 - w) * sig(lo) + w * sig(hi);
        }
        out[q] = v;
    }
    return FK_OK;
}
