"""Pins of the oracle's screening (Eqs. 5-9), self-energy (Eqs. 10-11) and
QP solution (transforms, Pade, Eq. 12)."""
import numpy as np
import pytest

from oracle import gt, chi as ochi, screen, sigma as osig, qp, chain
from conftest import rel_err


@pytest.fixture(scope="module")
def chain12_chi(chain12):
    inp = chain12
    do, dv = gt.density_matrices(inp.C, inp.eps, inp.s.n_occ, inp.mu_f, inp.grids.tau)
    return do, dv, ochi.chi_eq3(inp.t3c, do, dv)


def test_dielectric_and_wc_properties(chain12, chain12_chi):
    inp = chain12
    _, _, chi_tau = chain12_chi
    chi_w = screen.chi_omega(chi_tau, inp.grids.cos_w, 2.0)
    L = screen.cholesky_lower(inp.V)
    assert rel_err(L @ L.T, inp.V) < 1e-14
    for k in (0, 5, 9):
        eps = screen.dielectric(chi_w[k], L)
        assert np.linalg.eigvalsh(0.5 * (eps + eps.T)).min() >= 1.0 - 1e-10
        wc = screen.wc_omega(chi_w[k], L)
        ev = np.linalg.eigvalsh(0.5 * (wc + wc.T))
        assert ev.max() <= 1e-10 * np.abs(ev).max()
        # Cholesky route == V^(1/2) route
        assert rel_err(wc, screen.wc_omega_sqrt(chi_w[k], inp.V)) < 1e-10
    # no polarisation -> no screening
    z = np.zeros_like(chi_tau)
    assert np.abs(screen.screen_w(z, inp.V, inp.grids.cos_w, inp.grids.icos_w, 2.0)).max() == 0.0


def test_sigma_ao_equals_mo_form(chain12, chain12_chi):
    inp = chain12
    do, dv, chi_tau = chain12_chi
    wc = screen.screen_w(chi_tau, inp.V, inp.grids.cos_w, inp.grids.icos_w, 2.0)
    st = np.array([inp.s.n_occ - 2, inp.s.n_occ - 1, inp.s.n_occ, inp.s.n_occ + 3])
    so, sv = osig.sigma_tau(inp.C, inp.t3c, st, do, dv, wc)
    so2, sv2 = osig.sigma_tau_mo(inp.C, inp.eps, inp.s.n_occ, inp.mu_f, inp.t3c, st, wc, inp.grids.tau)
    assert rel_err(so, so2) < 1e-11 and rel_err(sv, sv2) < 1e-11
    d0, _ = gt.density_matrices(inp.C, inp.eps, inp.s.n_occ, inp.mu_f, [0.0])
    sx = osig.sigma_x(inp.C, inp.t3c, st, d0[0], inp.V)
    sx2 = osig.sigma_x_mo(inp.C, inp.s.n_occ, inp.t3c, st, inp.V)
    assert rel_err(sx, sx2) < 1e-12
    assert np.all(sx < 0)


def test_single_pole_sigma_closed_form(chain12):
    """W^c(tau) = -B exp(-Omega |tau|) gives
    Sigma^c_n(i w) = sum_i M_ni / (i w - eb_i + Omega) + sum_a M_na / (i w - eb_a - Omega)."""
    inp = chain12
    g = inp.grids
    rng = np.random.default_rng(3)
    x = rng.standard_normal((inp.s.n_ri, 6))
    B = x @ x.T / 6.0
    Om = 0.4
    wc = np.stack([-B * np.exp(-Om * t) for t in g.tau])
    do, dv = gt.density_matrices(inp.C, inp.eps, inp.s.n_occ, inp.mu_f, g.tau)
    st = inp.states
    so, sv = osig.sigma_tau(inp.C, inp.t3c, st, do, dv, wc)
    siw = qp.sigma_iw(so, sv, g.cos_w, g.sin_w)
    nm = osig.mo_pair_integrals(inp.C, inp.t3c, st)
    M = np.einsum("kip,pq,kiq->ki", nm, B, nm)
    eb = inp.eps - inp.mu_f
    no = inp.s.n_occ
    xo = -eb[:no] + Om
    xv = eb[no:] + Om
    for k, w in enumerate(g.omega):
        ref = ((M[:, :no] / (1j * w - eb[:no] + Om)).sum(1)
               + (M[:, no:] / (1j * w - eb[no:] - Om)).sum(1))
        # exact bound from the transform fit errors at every pole
        ec_o = np.exp(-np.outer(xo, g.tau)) @ g.cos_w[k] - xo / (xo ** 2 + w * w)
        es_o = np.exp(-np.outer(xo, g.tau)) @ g.sin_w[k] - w / (xo ** 2 + w * w)
        ec_v = np.exp(-np.outer(xv, g.tau)) @ g.cos_w[k] - xv / (xv ** 2 + w * w)
        es_v = np.exp(-np.outer(xv, g.tau)) @ g.sin_w[k] - w / (xv ** 2 + w * w)
        bre = np.abs(M[:, :no]) @ np.abs(ec_o) + np.abs(M[:, no:]) @ np.abs(ec_v)
        bim = np.abs(M[:, :no]) @ np.abs(es_o) + np.abs(M[:, no:]) @ np.abs(es_v)
        tol = 1e-10 * np.abs(ref).max()
        assert np.all(np.abs(siw[:, k].real - ref.real) <= bre + tol)
        assert np.all(np.abs(siw[:, k].imag - ref.imag) <= bim + tol)
        assert np.all(bre < 0.5 * np.abs(ref.real) + tol) or k > 7


def test_thiele_reproduces_rational_data():
    rng = np.random.default_rng(1)
    poles = np.array([-0.9, 0.35, 1.7])
    res = np.array([0.4, 1.1, 0.25])
    f = lambda z: (res / (z - poles)).sum()
    for n_nodes in (6, 7):
        zn = 1j * np.geomspace(0.05, 20, n_nodes)
        a = qp.thiele_coeffs(zn, np.array([f(z) for z in zn]))
        for e in (-0.4, 0.05, 0.9, 2.5):
            val, der = qp.thiele_eval(zn, a, e)
            assert abs(val - f(e)) < 1e-10 * max(1, abs(f(e)))
            h = 1e-5
            num = (f(e + h) - f(e - h)) / (2 * h)
            assert abs(der - num) < 1e-6 * max(1, abs(num))


def test_newton_special_cases():
    # Sigma^c = 0 (a single zero node): e_qp = eps - vxc + Sigma^x exactly
    zn = np.array([1j])
    a = qp.thiele_coeffs(zn, np.array([0j]))
    e = qp.solve_qp(-0.3, 0.05, -0.2, 0.0, zn, a)
    assert abs(e - (-0.3 - 0.05 - 0.2)) < 1e-12
    # one pole Sigma^c(z) = m / (z - p): quadratic root
    m, p, mu = 0.3, -0.8, 0.1
    zn = 1j * np.array([0.5, 2.0])
    a = qp.thiele_coeffs(zn, m / (zn - p))
    eps_n, vxc, sx = -0.25, 0.0, -0.1
    e = qp.solve_qp(eps_n, vxc, sx, mu, zn, a)
    A = eps_n - vxc + sx
    roots = np.roots([1.0, -(A + mu + p), A * (mu + p) - m])
    assert np.min(np.abs(roots - e)) < 1e-10
    with pytest.raises(qp.NoConvergence):
        qp.solve_qp(0.0, 0.0, 0.0, 0.0, zn, a, max_iter=1)


def test_full_chain_runs(chain12):
    inp = chain12
    r = chain.g0w0(inp.C, inp.eps, inp.s.n_occ, inp.t3c, inp.V, inp.s.ao_off, inp.s.ri_off,
                   inp.grids, inp.states)
    assert np.all(r.status == 0) and np.all(np.isfinite(r.e_qp))
