"""Imaginary-time / imaginary-frequency grids and fitted transform weights.

The paper uses minimax grids and their weights from an external table; those
tables are not reproduced here.  Instead (an input-preparation choice shared
by both sides of every comparison):

* tau_j: ``n`` log-spaced points in [tau_min, tau_max] (Ha^-1);
* omega_k = 1 / tau_{n-1-k}  (log-spaced, ascending);
* the weights are least-squares fits over ``n_fit`` log-spaced transition
  energies x in [x_lo, x_hi], with an SVD cut ``rcond``:

    cos  c[k, j]:  sum_j c_kj exp(-x tau_j) ~ x / (x^2 + w_k^2)      (relative)
    sin  s[k, j]:  sum_j s_kj exp(-x tau_j) ~ w_k / (x^2 + w_k^2)    (relative)
    icos d[j, k]:  sum_k d_jk x / (x^2 + w_k^2) ~ exp(-x tau_j)      (absolute)
    lapl w[j]:     sum_j w_j exp(-x tau_j) ~ 1 / x                    (relative)

x_lo = max(gap / 2, 1e-3) and x_hi = 3 (eps_max - eps_min) by default.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Grids:
    tau: np.ndarray     # [n_tau]
    omega: np.ndarray   # [n_w]
    cos_w: np.ndarray   # [n_w][n_tau]   c_kj
    sin_w: np.ndarray   # [n_w][n_tau]   s_kj
    icos_w: np.ndarray  # [n_tau][n_w]   d_jk
    lap_w: np.ndarray   # [n_tau]        w_j
    x_lo: float
    x_hi: float


def _lstsq(a, b, rcond):
    sol, *_ = np.linalg.lstsq(a, b, rcond=rcond)
    return sol


def fit_weights(tau, omega, x_lo, x_hi, n_fit=4000, rcond=1e-14) -> Grids:
    tau = np.asarray(tau, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    x = np.geomspace(x_lo, x_hi, n_fit)
    e = np.exp(-np.outer(x, tau))                       # [n_fit, n_tau]
    cos_w = np.empty((len(omega), len(tau)))
    sin_w = np.empty((len(omega), len(tau)))
    for k, w in enumerate(omega):
        tc = x / (x * x + w * w)
        ts = w / (x * x + w * w)
        cos_w[k] = _lstsq(e / tc[:, None], np.ones_like(x), rcond)
        sin_w[k] = _lstsq(e / ts[:, None], np.ones_like(x), rcond)
    lor = x[:, None] / (x[:, None] ** 2 + omega[None, :] ** 2)   # [n_fit, n_w]
    icos_w = np.empty((len(tau), len(omega)))
    for j, t in enumerate(tau):
        icos_w[j] = _lstsq(lor, np.exp(-x * t), rcond)
    lap_w = _lstsq(e * x[:, None], np.ones_like(x), rcond)
    return Grids(tau, omega, cos_w, sin_w, icos_w, lap_w, float(x_lo), float(x_hi))


def make_grids(eps, n_occ, n_tau, n_w=None, tau_min=0.02, tau_max=20.0,
               n_fit=4000, rcond=1e-14, x_lo=None, x_hi=None) -> Grids:
    n_w = n_tau if n_w is None else n_w
    tau = np.geomspace(tau_min, tau_max, n_tau)
    if n_w == n_tau:
        omega = np.sort(1.0 / tau)
    else:
        omega = np.geomspace(1.0 / tau_max, 1.0 / tau_min, n_w)
    eps = np.asarray(eps)
    gap = eps[n_occ] - eps[n_occ - 1]
    if x_lo is None:
        x_lo = max(0.5 * gap, 1e-3)
    if x_hi is None:
        x_hi = 3.0 * (eps[-1] - eps[0])
    return fit_weights(tau, omega, x_lo, x_hi, n_fit, rcond)
