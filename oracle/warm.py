"""Enclosed-charge profile and warm-start state, plain numpy in FP64.

Test infrastructure only: see ``oracle/__init__.py``.

Neither operation is in the paper; both are stated here from the field
solve of Section 2, whose self field is E_x(x) = sigma / 2 eps0 - (e / eps0)
int_0^x n_e dx'.  The enclosed charge is defined as

    sigma_enc(x) = 2 eps0 E_x^self(x) = sigma - 2 e int_0^x n_e dx'

with n_e constant over each x cell (the cell average the solver keeps), so
sigma_enc is piecewise linear with kinks at the cell faces.  The warm start
inverts it: the density of cell k is the drop of the profile across the cell
over 2 e dx, clamped at zero, spread over velocity as a Maxwellian at the
emission temperature normalised on the discrete velocity grid.
"""
import numpy as np

E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31


def enclosed_profile(sigma, ne, length, npts):
    """sigma_enc at x_p = L p / (npts - 1), p = 0 .. npts - 1."""
    ne = np.asarray(ne, dtype=np.float64)
    nx = ne.size
    dx = length / nx
    out = np.empty(npts)
    for p in range(npts):
        x = length * p / (npts - 1)
        k = min(max(int(np.floor(x / dx)), 0), nx)
        s = sigma - 2.0 * E_CHARGE * dx * float(np.sum(ne[:k]))
        if k < nx:
            s -= 2.0 * E_CHARGE * ne[k] * (x - k * dx)
        out[p] = s
    return out


def cell_centres(n, vmax):
    """v_i = (i + 1/2 - n/2) dv with dv = 2 vmax / n."""
    dv = 2.0 * vmax / n
    return (np.arange(n) + 0.5 - 0.5 * n) * dv, dv


def warm_state(profile, length, nx, nvx, nvy, vmax_x, vmax_y, t_ev):
    """(f, sigma) of the warm start from a profile at uniform points over [0, L]."""
    profile = np.asarray(profile, dtype=np.float64)
    npts = profile.size
    dx = length / nx
    xs = np.linspace(0.0, length, npts)
    faces = np.arange(nx + 1) * dx
    s_faces = np.interp(np.clip(faces, 0.0, length), xs, profile)
    n = np.maximum(0.0, (s_faces[:-1] - s_faces[1:]) / (2.0 * E_CHARGE * dx))
    vx, dvx = cell_centres(nvx, vmax_x)
    vy, dvy = cell_centres(nvy, vmax_y)
    m = np.exp(-M_E * (vx[:, None] ** 2 + vy[None, :] ** 2) / (2.0 * t_ev * E_CHARGE))
    m /= m.sum() * dvx * dvy
    return n[:, None, None] * m[None, :, :], float(profile[0])
