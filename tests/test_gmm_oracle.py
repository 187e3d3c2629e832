"""Pins of the oracle's EM fit of a Gaussian mixture (Sec. 2.2, Eq. 20-24).

A single component reduces to the sample mean and variance; EM never lowers the
log-likelihood; well-separated clusters converge to their own sample statistics;
a converged fit is a fixed point of one more iteration; and on draws from the
paper's Tab. 3 mixture the fit recovers the true parameters within their
statistical error.  A dropped weight, a wrong sign in Eq. (21) or the old mean
in Eq. (24) fails at least one of them.
"""
import math

import numpy as np
import pytest

import shale_inputs as si
from oracle import gmm


def test_single_component_is_sample_mean_and_variance():
    x = si.mixture_samples(1, 5000, ((3.0, 2.0, 1.0),))
    phi, mu, var, hist = gmm.fit(x, [1.0], [0.0], [1.0], 1)
    assert phi[0] == 1.0
    assert abs(mu[0] - x.mean()) < 1e-12 * abs(x.mean())
    assert abs(var[0] - x.var()) < 1e-12 * x.var()


def test_log_likelihood_never_decreases():
    x = si.mixture_samples(2, 4000)
    _, _, _, hist = gmm.fit(x, [0.5, 0.5], [8.0, 25.0], [4.0, 25.0], 60)
    d = np.diff(hist)
    assert np.all(d >= -1e-9 * abs(hist[-1]))
    assert hist[-1] > hist[0]


def test_well_separated_clusters_give_their_own_statistics():
    a = si.mixture_samples(3, 3000, ((-50.0, 1.0, 1.0),))
    b = si.mixture_samples(4, 1000, ((50.0, 2.0, 1.0),))
    x = np.concatenate([a, b])
    phi, mu, var, _ = gmm.fit(x, [0.5, 0.5], [-40.0, 40.0], [10.0, 10.0], 20)
    assert np.allclose(phi, [0.75, 0.25], rtol=0, atol=1e-12)
    assert np.allclose(mu, [a.mean(), b.mean()], rtol=1e-12)
    assert np.allclose(var, [a.var(), b.var()], rtol=1e-10)


def test_converged_fit_is_a_fixed_point():
    x = si.mixture_samples(5, 3000)
    phi, mu, var, _ = gmm.fit(x, [0.5, 0.5], [8.0, 25.0], [4.0, 25.0], 2000)
    p2, m2, v2 = gmm.m_step(x, gmm.e_step(x, phi, mu, var))
    assert np.allclose(p2, phi, rtol=1e-9) and np.allclose(m2, mu, rtol=1e-9) and np.allclose(v2, var, rtol=1e-8)


def test_recovers_tab3_mixture_within_sampling_error():
    """Tab. 3: clusters (10, 1, 0.25) and (20, 4, 0.75).  With m = 40000 draws the fitted
    means, standard deviations and fractions lie within 5 standard errors of the truth
    (errors of a single Gaussian's estimators, widened by 1.5 for the overlap).  The
    paper's own fit (9.8848 / 0.9886 / 0.2418 and 19.6846 / 4.0804 / 0.7582) deviates from
    the truth by about 1-2 such errors of a sample of a thousand draws."""
    m = 40000
    x = si.mixture_samples(6, m)
    phi, mu, var, _ = gmm.fit(x, [0.5, 0.5], [8.0, 25.0], [4.0, 25.0], 500)
    o = np.argsort(mu)
    phi, mu, sd = phi[o], mu[o], np.sqrt(var[o])
    for j, (mt, st, ft) in enumerate(si.TAB3_CLUSTERS):
        n = m * ft
        assert abs(mu[j] - mt) < 5 * 1.5 * st / math.sqrt(n)
        assert abs(sd[j] - st) < 5 * 1.5 * st / math.sqrt(2 * n)
        assert abs(phi[j] - ft) < 5 * 1.5 * math.sqrt(ft * (1 - ft) / m)


def test_lognormal_pore_modes_are_recovered_in_log_radius():
    """A two-phase pore-radius sample (organic matter 5 nm, inorganic 20 nm medians, sigma
    0.5 in ln r) fitted in ln r gives back both medians and the shared log-width."""
    r = si.pore_radius_samples(7, 30000)
    phi, mu, var, _ = gmm.fit(np.log(r), [0.5, 0.5], [math.log(3e-9), math.log(30e-9)], [0.5, 0.5], 400)
    o = np.argsort(mu)
    assert np.allclose(np.exp(mu[o]), [5e-9, 20e-9], rtol=0.03)
    assert np.allclose(np.sqrt(var[o]), [0.5, 0.5], rtol=0.05)
    assert np.allclose(phi[o], [0.3, 0.7], atol=0.02)
