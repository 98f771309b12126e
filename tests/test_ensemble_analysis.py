"""The host-side ensemble analysis of translocation runs (Sec. III), against distributions
and laws whose answers are known: the mode of skewed distributions, exact and noisy power
laws, the constancy of R_E under static blob scaling, and synthetic event records."""
import numpy as np
import pytest

from paper_0710_1272_amd import ensemble as E


@pytest.mark.parametrize("dist,mode", [
    (lambda rng, n: rng.gamma(4.0, 100.0, n), 300.0),                   # (k - 1) theta
    (lambda rng, n: rng.lognormal(7.0, 0.3, n), np.exp(7.0 - 0.09)),    # exp(mu - s^2)
])
def test_most_probable_time_of_skewed_distributions(dist, mode):
    """Ten samples of 5000 events: the mode estimates scatter (a mode converges slowly) but
    centre on the true mode, well below the mean of the skewed distribution."""
    rng = np.random.default_rng(1)
    est, means = [], []
    for _ in range(10):
        t = dist(rng, 5000)
        est.append(E.most_probable_time(t))
        means.append(t.mean())
    est = np.array(est)
    assert abs(est.mean() / mode - 1) < 0.04, (est, mode)
    assert np.all(np.abs(est / mode - 1) < 0.15)
    assert np.all(est < np.array(means))


def test_scaling_exponent():
    n = np.array([20, 40, 80, 160, 320])
    a, se, A = E.scaling_exponent(n, 3.0 * n ** 1.28)
    assert abs(a - 1.28) < 1e-12 and se < 1e-12 and abs(A - 3.0) < 1e-9
    rng = np.random.default_rng(2)
    alphas = []
    for _ in range(200):
        tau = 3.0 * n ** 1.28 * np.exp(0.05 * rng.standard_normal(len(n)))
        alphas.append(E.scaling_exponent(n, tau))
    a = np.array([x[0] for x in alphas])
    se = np.array([x[1] for x in alphas])
    assert abs(a.mean() - 1.28) < 3 * a.std() / np.sqrt(len(a))
    assert abs(np.median(se) / a.std() - 1) < 0.3  # the standard error is calibrated


def test_effective_radius_is_constant_under_static_scaling():
    """R_I = c N_I^mu for both blobs and N_U + N_T = N give R_E = c N^mu at every split."""
    c, N = 0.7, 200
    nt = np.arange(0, N + 1)
    re = E.effective_radius(c * (N - nt) ** E.FLORY_MU, c * nt ** E.FLORY_MU)
    assert np.allclose(re, c * N ** E.FLORY_MU, rtol=1e-12)
    assert E.effective_radius(np.array([2.0]), np.array([0.0]))[0] == pytest.approx(2.0)


def test_retraction_detection():
    assert E.retracted([0, 1, 3, 8, 12, 6, 2, 0, 0], 50)
    assert not E.retracted([0, 1, 3, 8, 12, 20, 50], 50)
    assert not E.retracted([0, 1, 0, 1, 0], 50)  # never past the threshold
    assert E.retracted([0, 1, 0, 1, 0], 50, threshold=1)


def _synthetic_event(t_done, every, n=40):
    steps = np.arange(every, t_done + 5 * every, every, dtype=float)
    s = steps / t_done
    rows = np.zeros((len(steps), 8))
    rows[:, E.STEP] = steps
    rows[:, E.N_T] = np.clip(np.round(n * s), 0, n)
    rows[:, E.S_H] = 0.02 + 0.0 * s
    rows[:, E.S_E] = 0.01
    rows[:, E.K] = 0.5
    nt = np.clip(n * s, 0, n)
    rows[:, E.R_U2] = (0.7 * (n - nt) ** 0.6) ** 2
    rows[:, E.R_T2] = (0.7 * nt ** 0.6) ** 2
    return rows


def test_event_summary_and_scaled_profile():
    ev = [(_synthetic_event(t, 5), t) for t in (400, 650, 900)]
    s = E.event_summary(ev[0][0], ev[0][1], gamma=0.1)
    assert s["S_H"] == pytest.approx(0.02) and s["S_E"] == pytest.approx(0.01)
    assert s["gammaK"] == pytest.approx(0.05)
    assert s["S_H_positive_fraction"] == 1.0 and s["S_E_negative_fraction"] == 0.0
    assert s["R_T_end_over_R_U_start"] == pytest.approx((40 / (40 - 40 * 5 / 400)) ** 0.6, rel=1e-9)
    prof = E.scaled_profile(ev, gamma=0.1, bins=10)
    assert np.all(prof["rows"] > 0)
    # rows after completion are left out; R_E stays at 0.7 N^mu throughout
    assert np.allclose(prof["R_E"], 0.7 * 40 ** 0.6, rtol=1e-9)
    assert np.all(np.diff(prof["R_T"]) > 0) and np.all(np.diff(prof["R_U"]) < 0)
