"""Pins of the host-side analysis (paper Sec. IV.B figures of merit).

* tau_int of an AR(1) series with coefficient phi is (1+phi)/(2(1-phi));
* the jackknife error of the mean of iid data is sigma/sqrt(n); of a nonlinear f
  it follows the delta method;
* round-trip time and acceptance bookkeeping on constructed inputs.
"""
import numpy as np

from paper_1006_4247_amd import analysis


def _ar1(phi, n, seed):
    from scipy.signal import lfilter
    eps = np.random.default_rng(seed).standard_normal(n)
    return lfilter([1.0], [1.0, -phi], eps)


def test_tau_int_ar1():
    for phi in [0.0, 0.5, 0.8]:
        x = _ar1(phi, 200000, 1)
        tau, tf = analysis.tau_int(x, c=6)
        expect = (1 + phi) / (2 * (1 - phi))
        assert abs(tau - expect) < 0.08 * expect + 0.02, (phi, tau, expect)
        assert tf >= 6 * tau - 1


def test_autocorrelation_of_ar1():
    x = _ar1(0.7, 100000, 2)
    rho = analysis.autocorrelation(x, 5)
    assert np.allclose(rho, 0.7 ** np.arange(6), atol=0.02)


def test_jackknife_iid_mean_and_delta_method():
    r = np.random.default_rng(3)
    x = r.standard_normal(40000) * 2.0 + 1.0
    est, err = analysis.jackknife(x, 40)
    assert abs(est - 1.0) < 5 * 2.0 / np.sqrt(x.size)
    assert abs(err - 2.0 / np.sqrt(x.size)) < 0.3 * 2.0 / np.sqrt(x.size)
    est2, err2 = analysis.jackknife(x, 40, f=lambda m: m ** 2)
    assert abs(err2 - 2 * abs(est) * err) < 0.05 * err2


def test_acceptance_and_round_trips():
    stats = np.zeros((2, 3, 4, 2), dtype=np.int64)
    stats[..., 0] = 10
    stats[..., 1] = [1, 2, 5, 10]
    assert np.allclose(analysis.acceptance(stats), [0.1, 0.2, 0.5, 1.0])
    trips = np.zeros((2, 2, 5), dtype=np.int64)
    trips[0, 0, 1] = 3
    trips[1, 1, 4] = 1
    overall, pc = analysis.round_trip_time(trips, 100)
    assert overall == 100 * 20 / 4
    assert pc[0] == 100 * 5 / 3 and np.isinf(pc[1]) and pc[3] == 500.0
