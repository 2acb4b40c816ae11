"""Coulomb matrix of a periodic Gamma-point cell, FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

For periodic cells the paper obtains V of Eq. 8 by Ewald summation.  Reading:
the RI functions are normalized Gaussian charges rho_P (exponent alpha_P,
centre R_P) in an orthorhombic cell of volume Omega with a neutralizing
background (the Gamma-only treatment, G = 0 left out); V is then

  V_PQ = (4 pi / Omega) sum_{G != 0} exp(-G^2/(4 alpha_P)) exp(-G^2/(4 alpha_Q))
                                      cos(G . (R_P - R_Q)) / G^2,

G over the reciprocal lattice.  The Gaussian factors make the sum converge
absolutely; it is taken here as written, over every G whose term can exceed
tol (no Ewald splitting: the oracle is the plain definition the split must
reproduce).  The 3D correction scheme the paper mentions is not defined in
the paper and not included.

Pinned by (tests/test_oracle_periodic.py): the expansion of the cubic-lattice
potential for a pair at small separation R in a large cell of side L,
erf(sqrt(mu) R)/R - alpha_M/L + 2 pi R^2/(3 L^3) + pi/(mu L^3) with the
simple-cubic Madelung constant alpha_M = 2.8372974794806 and
1/mu = 1/alpha_P + 1/alpha_Q; an Ewald split written independently in the
test at two splitting parameters on a non-cubic cell; lattice periodicity.
"""
from __future__ import annotations

import numpy as np


def reciprocal_vectors(cell, g_max):
    """All G != 0 of the orthorhombic cell with |G| <= g_max."""
    cell = np.asarray(cell, dtype=np.float64)
    b = 2.0 * np.pi / cell
    n = np.ceil(g_max / b).astype(int)
    axes = [np.arange(-k, k + 1) * bb for k, bb in zip(n, b)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    g2 = (g * g).sum(1)
    keep = (g2 > 0) & (g2 <= g_max * g_max)
    return g[keep], g2[keep]


def coulomb_periodic(centres, alpha, cell, tol=1e-17, chunk=4096):
    centres = np.asarray(centres, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    omega = float(np.prod(cell))
    # the largest term at |G| is (4 pi/Omega) exp(-G^2/(2 alpha_max)) / G^2
    g_max = np.sqrt(2.0 * alpha.max() * np.log(4.0 * np.pi / omega / tol))
    g, g2 = reciprocal_vectors(cell, g_max)
    n = len(alpha)
    V = np.zeros((n, n))
    for s in range(0, len(g2), chunk):
        gg, gq = g[s:s + chunk], g2[s:s + chunk]
        ph = centres @ gg.T
        damp = np.exp(-gq[None, :] / (4.0 * alpha[:, None]))
        w = 4.0 * np.pi / omega / gq
        c = np.cos(ph) * damp
        si = np.sin(ph) * damp
        V += (c * w) @ c.T + (si * w) @ si.T
    return V


def coulomb_isolated(centres, alpha):
    """erf(sqrt(mu) R)/R of two normalized Gaussian charges (no cell)."""
    from scipy.special import erf
    centres = np.asarray(centres, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    mu = alpha[:, None] * alpha[None, :] / (alpha[:, None] + alpha[None, :])
    d = np.linalg.norm(centres[:, None, :] - centres[None, :, :], axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = erf(np.sqrt(mu) * d) / d
    return np.where(d > 0, v, 2.0 * np.sqrt(mu / np.pi))
