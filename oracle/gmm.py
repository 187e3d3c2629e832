"""EM fit of a Gaussian mixture to pore-size samples (the paper's Sec. 2.2, Eq. 20-24).

TEST INFRASTRUCTURE ONLY (oracle): the library's batched GPU fit is checked
against it; the product never imports it.

Samples are scalars (pore size, or its logarithm): the multivariate Gaussian
of Eq. (21) with input length n = 1.  One iteration, in the paper's order:
    E-step (Eq. 20):  w_ij = g_j(x_i) Phi_j / sum_l g_l(x_i) Phi_l,
                      g_j(x) = exp(-(x - mu_j)^2 / (2 var_j)) / sqrt(2 pi var_j)   (Eq. 21)
    M-step:           Phi_j = (1/m) sum_i w_ij                                     (Eq. 22)
                      mu_j  = sum_i w_ij x_i / sum_i w_ij                          (Eq. 23)
                      var_j = sum_i w_ij (x_i - mu_j)^2 / sum_i w_ij                (Eq. 24)
Readings: Eq. (21) is printed without the minus sign of the exponent (a density
must decay); Eq. (24) uses the mean just updated by Eq. (23) (the maximiser of the
expected log-likelihood).  FP64 throughout.
"""
from __future__ import annotations

import math

import numpy as np


def gaussian_pdf(x, mu, var):
    """g(x) of Eq. (21) for one scalar component."""
    x = np.asarray(x, dtype=np.float64)
    return np.exp(-(x - mu) ** 2 / (2.0 * var)) / math.sqrt(2.0 * math.pi * var)


def e_step(x, phi, mu, var):
    """Responsibilities w[i, j] of Eq. (20)."""
    num = np.stack([gaussian_pdf(x, mu[j], var[j]) * phi[j] for j in range(len(phi))], axis=1)
    return num / num.sum(axis=1, keepdims=True)


def m_step(x, w):
    """(Phi, mu, var) of Eq. (22)-(24) from the responsibilities."""
    x = np.asarray(x, dtype=np.float64)
    sw = w.sum(axis=0)
    phi = sw / len(x)
    mu = (w * x[:, None]).sum(axis=0) / sw
    var = (w * (x[:, None] - mu[None, :]) ** 2).sum(axis=0) / sw
    return phi, mu, var


def log_likelihood(x, phi, mu, var):
    """sum_i log sum_j Phi_j g_j(x_i)."""
    dens = sum(phi[j] * gaussian_pdf(x, mu[j], var[j]) for j in range(len(phi)))
    return float(np.log(dens).sum())


def fit(x, phi, mu, var, iters):
    """Run `iters` EM iterations from (phi, mu, var); returns the final parameters and
    the log-likelihood of the starting point and after every iteration."""
    phi, mu, var = (np.array(a, dtype=np.float64) for a in (phi, mu, var))
    hist = [log_likelihood(x, phi, mu, var)]
    for _ in range(iters):
        w = e_step(x, phi, mu, var)
        phi, mu, var = m_step(x, w)
        hist.append(log_likelihood(x, phi, mu, var))
    return phi, mu, var, hist
