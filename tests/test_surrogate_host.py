"""Host-side helpers of the surrogate pipeline (no GPU): feature scaling,
target encoding, the picosecond trace stride and the error measures."""
import math

import numpy as np
import pytest

S = pytest.importorskip("paper_2303_14119_amd.surrogate")
from paper_2303_14119_amd import workloads as W  # noqa: E402

EPS0 = 8.8541878128e-12


def test_features_map_the_sweep_box_to_unit_cube():
    # the finest sweep grid has the smallest cells, so it sits at -1 with the
    # smallest physical parameters
    lo = W.config(nx=1024, nvx=192, nvy=192, length=0.5e-3, ey=-1e6, delta_max=1.5, a_max_ev=250.0, t_se_ev=1.0)
    hi = W.config(nx=256, nvx=64, nvy=64, length=5e-3, ey=-10e6, delta_max=3.5, a_max_ev=600.0, t_se_ev=5.0)
    f = S.features([lo, hi])
    assert f.shape == (2, S.DIMS[0])
    assert np.allclose(f[0], -1.0) and np.allclose(f[1], 1.0)
    # |E_y| is used, whatever the sign convention of the field
    mid = dict(lo, ey=+5.5e6)
    assert S.features([mid])[0][0] == pytest.approx(0.0, abs=1e-6)
    # grid inputs are linear in the cell size: 1/512 is a third of the way
    # from 1/1024 to 1/256, 1/96 halfway from 1/192 to 1/64
    half = dict(lo, nx=512, nvx=96, nvy=96)
    assert S.features([half])[0][5:] == pytest.approx([-1 / 3, 0.0], abs=1e-6)
    # a grid four times finer than the sweep's coarsest x grid: 1/N_x = 1/1024
    assert S.features([dict(lo, nx=4096)])[0][5] == pytest.approx(-1.5, abs=1e-6)


def test_load_data_rebuilds_inputs_from_raw(tmp_path):
    cfgs = W.c2_instances(seed=3, n=5)
    raw = S._raw(cfgs)
    y = np.zeros((5, S.NPTS + 2), dtype=np.float32)
    sat = np.array([1, 0, 1, 1, 0])
    # stored inputs of another width are ignored
    np.savez(tmp_path / "d.npz", X=np.zeros((5, 3), np.float32), Y=y, sat=sat, raw=raw)
    X, Y, r = S.load_data([str(tmp_path / "d.npz")])
    keep = [c for c, s in zip(cfgs, sat) if s]
    assert np.array_equal(X, S.features(keep)) and len(Y) == 3 and np.array_equal(r, raw[sat.astype(bool)])


def test_encode_decode_round_trip():
    rng = np.random.default_rng(0)
    ey = -6e6
    prof = 2 * EPS0 * abs(ey) * rng.uniform(-0.5, 1.5, S.NPTS)
    y = S.encode(prof, 3.2e24, 1.7e23, ey)
    assert y.shape == (S.NPTS + 2,) and y.dtype == np.float32
    back, gpe, gsee = S.decode(y, ey)
    assert np.allclose(back, prof, rtol=1e-6, atol=1e-6 * np.abs(prof).max())
    assert gpe == pytest.approx(3.2e24, rel=1e-5) and gsee == pytest.approx(1.7e23, rel=1e-5)
    # profiles are in units of 2 eps0 |E_y| (the scale of Eq 20)
    assert S.encode(np.full(S.NPTS, 2 * EPS0 * abs(ey)), 1e24, 1e24, ey)[0] == pytest.approx(1.0)


def test_trace_stride_is_about_a_picosecond():
    assert S.trace_stride(2.343e-14) == 43
    assert S.trace_stride(5e-15) == 200
    assert S.trace_stride(3e-12) == 1          # never zero


def test_profile_errors_measure_relative_l2():
    ey = -5e6
    p = np.linspace(1e-5, 2e-5, S.NPTS)
    yt = S.encode(p, 1e24, 2e24, ey)
    yp = S.encode(1.1 * p, 1.2e24, 2e24, ey)
    e = S.profile_errors(np.array([yp]), np.array([yt]), np.array([[ey]]))[0]
    assert e[0] == pytest.approx(0.1, rel=1e-5)
    assert e[1] == pytest.approx(0.2, rel=1e-4) and e[2] == pytest.approx(0.0, abs=1e-5)


def test_init_params_layout_and_scale():
    dims = [5, 64, 7]
    p = S.init_params(dims, 3)
    assert p.size == 5 * 64 + 64 + 64 * 7 + 7
    w1 = p[:5 * 64].reshape(64, 5)
    assert abs(w1.std() - 1 / math.sqrt(5)) < 0.1
    assert np.all(p[5 * 64:5 * 64 + 64] == 0)


# ------------------------------------------------ cold-start fallback (no GPU)

class _Solver:
    """Records what the warm-start helper asks of a solver."""

    def __init__(self, refuse=False):
        self.calls = []
        self.refuse = refuse

    def warm_start(self, profile, t_ev, step=0):
        if self.refuse:
            from paper_2303_14119_amd import flashkin as fk
            raise fk.FlashkinError(fk.E_INVALID, "refused")
        self.calls.append(("warm", np.asarray(profile).copy()))

    def write_state(self, f=None, sigma=0.0, sigma_lo=0.0, step=0):
        self.calls.append(("cold", sigma, step))


class _Net:
    def __init__(self, y, lo=None, hi=None):
        self.y, self.x_lo, self.x_hi = y, lo, hi

    def predict(self, X):
        return np.repeat(self.y[None, :], len(X), axis=0)


def _inside():
    return W.config(nx=512, nvx=128, nvy=128, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0, t_se_ev=2.0)


def test_warm_start_uses_a_finite_prediction_inside_the_box():
    pytest.importorskip("paper_2303_14119_amd.flashkin")
    y = np.zeros(S.NPTS + 2, dtype=np.float32)
    y[:S.NPTS] = np.linspace(1.0, 0.0, S.NPTS)
    s = _Solver()
    prof, why = S.warm_start(s, _inside(), _Net(y))
    assert why is None and s.calls[0][0] == "warm"
    assert prof[0] == pytest.approx(2 * EPS0 * 5e6, rel=1e-6)


@pytest.mark.parametrize("kw,word", [(dict(ey=-20e6), "|E_y|"), (dict(delta_max=5.0), "delta_max"),
                                     (dict(nx=16), "1/N_x")])
def test_inputs_outside_the_box_cold_start(kw, word):
    pytest.importorskip("paper_2303_14119_amd.flashkin")
    s = _Solver()
    prof, why = S.warm_start(s, dict(_inside(), **kw), _Net(np.zeros(S.NPTS + 2, np.float32)))
    assert prof is None and word in why and "outside the training box" in why
    assert s.calls == [("cold", 0.0, 0)]


def test_the_largest_run_is_inside_the_widened_box():
    """4096 x 384 x 384 encodes its cell sizes to -1.5: within the grid
    inputs' margin of the sweep's box."""
    assert S.trust_inputs(W.c4()) is None
    assert "1/N_x" in S.trust_inputs(dict(W.c4(), nx=8))


def test_non_finite_prediction_cold_starts():
    pytest.importorskip("paper_2303_14119_amd.flashkin")
    y = np.zeros(S.NPTS + 2, dtype=np.float32)
    y[7] = np.nan
    s = _Solver()
    prof, why = S.warm_start(s, _inside(), _Net(y))
    assert prof is None and why == "non-finite prediction" and s.calls == [("cold", 0.0, 0)]
    y = np.zeros(S.NPTS + 2, dtype=np.float32)
    y[S.NPTS] = 1e30                       # decodes to an infinite flux
    s = _Solver()
    prof, why = S.warm_start(s, _inside(), _Net(y))
    assert prof is None and "non-finite" in why


def test_refused_warm_start_cold_starts():
    pytest.importorskip("paper_2303_14119_amd.flashkin")
    s = _Solver(refuse=True)
    prof, why = S.warm_start(s, _inside(), _Net(np.zeros(S.NPTS + 2, np.float32)))
    assert prof is None and why.startswith("warm start refused") and s.calls == [("cold", 0.0, 0)]


def test_training_box_narrows_the_trust():
    """A network that only saw a part of the box trusts only that part (plus
    the margins)."""
    lo = -np.ones(7)
    hi = np.ones(7)
    hi[0] = -0.5                           # trained on |E_y| up to 3.25 MV/m
    assert S.trust_inputs(_inside(), lo, hi) is not None
    assert S.trust_inputs(dict(_inside(), ey=-3.3e6), lo, hi) is None
