"""The periodic Coulomb oracle (oracle/periodic.py) against fixed points that
do not come from it: the small-separation expansion of the cubic-lattice
potential with the published simple-cubic Madelung constant of a lattice in
a neutralizing background, an Ewald split written here from the textbook
derivation (real-space erf sums plus a damped reciprocal sum plus the
background constant) that must give the same matrix for any splitting
parameter, on a non-cubic cell, and lattice periodicity; the bulk workload's
V is positive definite."""
import numpy as np
import pytest
from scipy.special import erf

from oracle import periodic as oper

MADELUNG_SC = 2.8372974794806


def test_cubic_expansion():
    L = 40.0
    a = np.array([0.8, 0.8, 1.3])
    R = np.array([[0.0, 0.0, 0.0], [1.0, 0.3, -0.2], [-0.4, 0.9, 0.5]])
    V = oper.coulomb_periodic(R, a, np.full(3, L))
    iso = oper.coulomb_isolated(R, a)
    mu = a[:, None] * a[None, :] / (a[:, None] + a[None, :])
    d2 = ((R[:, None, :] - R[None, :, :]) ** 2).sum(-1)
    pred = iso - MADELUNG_SC / L + 2 * np.pi * d2 / (3 * L ** 3) + np.pi / (mu * L ** 3)
    # next term of the cubic expansion is O(R^4 / L^5) ~ 1e-8 here
    np.testing.assert_allclose(V, pred, rtol=0, atol=1e-7)
    np.testing.assert_allclose(np.diag(V), np.diag(pred), rtol=0, atol=1e-12)


def _ewald_split(centres, alpha, cell, eta, tol=1e-17):
    """Textbook Ewald split: [erf(sqrt(mu) r) - erf(eta r)]/r over lattice
    images, + (4 pi/Omega) sum_{G!=0} exp(-G^2/(4 eta^2)) cos(G.R)/G^2,
    - (pi/Omega)(1/eta^2 - 1/mu); valid for eta < sqrt(mu)."""
    cell = np.asarray(cell, float)
    omega = np.prod(cell)
    mu = alpha[:, None] * alpha[None, :] / (alpha[:, None] + alpha[None, :])
    assert eta < np.sqrt(mu.min())
    r_cut = 6.5 / eta
    n = np.ceil(r_cut / cell).astype(int)
    img = np.stack(np.meshgrid(*[np.arange(-k, k + 1) for k in n], indexing="ij"), -1).reshape(-1, 3) * cell
    diff = centres[:, None, :] - centres[None, :, :]
    real = np.zeros(mu.shape)
    for t in img:
        r = np.linalg.norm(diff + t, axis=-1)
        with np.errstate(invalid="ignore", divide="ignore"):
            v = (erf(np.sqrt(mu) * r) - erf(eta * r)) / r
        real += np.where(r > 0, v, 2.0 * (np.sqrt(mu) - eta) / np.sqrt(np.pi))
    g, g2 = oper.reciprocal_vectors(cell, 2.0 * eta * np.sqrt(np.log(1.0 / tol)))
    w = 4 * np.pi / omega * np.exp(-g2 / (4 * eta * eta)) / g2
    ph = centres @ g.T
    rec = (np.cos(ph) * w) @ np.cos(ph).T + (np.sin(ph) * w) @ np.sin(ph).T
    return real + rec - np.pi / omega * (1.0 / eta ** 2 - 1.0 / mu)


def test_ewald_split_agrees_on_a_non_cubic_cell():
    rng = np.random.default_rng(3)
    cell = np.array([6.0, 7.5, 9.0])
    R = rng.uniform(0, 1, (9, 3)) * cell
    a = rng.uniform(0.5, 2.0, 9)
    V = oper.coulomb_periodic(R, a, cell)
    for eta in (0.3, 0.45):
        E = _ewald_split(R, a, cell, eta)
        np.testing.assert_allclose(E, V, rtol=0, atol=1e-12 * np.abs(V).max())


def test_lattice_periodicity_and_bulk_positive_definite():
    from gwinputs import configs
    s = configs.bulk(3, n_ao=5, n_ri=12).system
    R, a = s.ri_charges()
    V = oper.coulomb_periodic(R, a, s.cell)
    R2 = R.copy()
    R2[5] += s.cell * np.array([1, -2, 1])
    V2 = oper.coulomb_periodic(R2, a, s.cell)
    np.testing.assert_allclose(V2, V, rtol=0, atol=1e-12 * np.abs(V).max())
    w = np.linalg.eigvalsh(V)
    assert w.min() > 0 and w.max() / w.min() < 1e10
    # minimum-image distances: the cell is periodic for H and the tensor too
    assert s.dist.max() <= np.linalg.norm(s.cell) / 2 + 1e-12
