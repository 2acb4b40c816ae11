"""The open-shell oracle (oracle/spin.py) against fixed points that do not
come from it: the closed-shell limit (equal channels, spin factor 2 of the
pinned closed-shell chain), the exchange of the channels, and each channel's
chi(tau) against its MO closed form (Eq. 3 summed over occupied-virtual pairs
of that channel).  Input: the 12-atom chain with a spin-dependent potential
of 0.05 Ha per AO (gwinputs System.mean_field_spin): equal occupations (the
broken-symmetry singlet the paper runs its ribbons as) and, with a uniform
0.09 Ha Zeeman split, one electron moved from the down to the up channel."""
import numpy as np
import pytest

from conftest import get_inputs
from oracle import chain as ochain, chi as ochi, spin as ospin

DELTA = 0.05
ZEEMAN = 0.09
CASES = {"singlet": (0.0, 0), "triplet": (ZEEMAN, 1)}


@pytest.fixture(scope="module")
def chain():
    return get_inputs("chain12")


def _run(inp, up, dn, n_up, n_dn, st_up, st_dn):
    s = inp.s
    return ospin.g0w0_spin((up[0], up[1], n_up), (dn[0], dn[1], n_dn), inp.t3c, inp.V, s.ao_off,
                           s.ri_off, inp.grids, st_up, st_dn, s.filter_eps)


def test_closed_shell_limit(chain):
    inp = chain
    s = inp.s
    r = _run(inp, (inp.C, inp.eps), (inp.C, inp.eps), s.n_occ, s.n_occ, inp.states, inp.states)
    ref = ochain.g0w0(inp.C, inp.eps, s.n_occ, inp.t3c, inp.V, s.ao_off, s.ri_off, inp.grids,
                      inp.states, s.filter_eps)
    np.testing.assert_allclose(r.chi_up + r.chi_dn, 2.0 * ref.chi_tau, rtol=0,
                               atol=1e-12 * np.abs(ref.chi_tau).max())
    np.testing.assert_allclose(r.wc_tau, ref.wc_tau, rtol=0, atol=1e-10 * np.abs(ref.wc_tau).max())
    for e in r.e_qp:
        np.testing.assert_allclose(e, ref.e_qp, rtol=0, atol=1e-9)


def test_occupation_check(chain):
    """Without the Zeeman split the moved electron sits above the down
    channel's lowest virtual level: no common Fermi level exists."""
    inp = chain
    s = inp.s
    up, dn = s.mean_field_spin(DELTA)
    with pytest.raises(ValueError):
        _run(inp, up, dn, s.n_occ + 1, s.n_occ - 1, [s.n_occ], [s.n_occ - 1])


@pytest.mark.parametrize("name", list(CASES))
def test_channel_exchange_and_mo_form(chain, name):
    inp = chain
    s = inp.s
    zeeman, moved = CASES[name]
    up, dn = s.mean_field_spin(DELTA, zeeman)
    n_up, n_dn = s.n_occ + moved, s.n_occ - moved
    st_up = np.array([n_up - 1, n_up])
    st_dn = np.array([n_dn - 1, n_dn])
    a = _run(inp, up, dn, n_up, n_dn, st_up, st_dn)
    b = _run(inp, dn, up, n_dn, n_up, st_dn, st_up)
    np.testing.assert_allclose(a.chi_up, b.chi_dn, rtol=0, atol=0)
    np.testing.assert_allclose(a.wc_tau, b.wc_tau, rtol=0, atol=1e-12 * np.abs(a.wc_tau).max())
    np.testing.assert_allclose(a.e_qp[0], b.e_qp[1], rtol=0, atol=1e-9)
    np.testing.assert_allclose(a.e_qp[1], b.e_qp[0], rtol=0, atol=1e-9)
    assert np.all(a.status[0] == 0) and np.all(a.status[1] == 0)
    # each channel's chi(tau) is its MO closed form
    for chi, (C, eps), n_occ in ((a.chi_up, up, n_up), (a.chi_dn, dn, n_dn)):
        iap = ochi.mo_integrals(C, inp.t3c, n_occ).reshape(-1, s.n_ri)
        delta = (eps[None, n_occ:] - eps[:n_occ, None]).ravel()
        for j, tau in enumerate(inp.grids.tau):
            ref = -(iap * np.exp(-delta * tau)[:, None]).T @ iap
            assert np.abs(chi[j] - ref).max() <= 1e-11 * np.abs(ref).max()
    # the two channels differ (the potential splits them)
    assert np.abs(a.e_qp[0] - b.e_qp[0]).max() > 1e-6


def test_with_ri_metric(chain):
    """Equal channels with an RI overlap reproduce the pinned metric chain
    (spin factor 2); S = 1 gives the form without S."""
    from oracle import metric as omet
    inp = chain
    s = inp.s
    S = s.ri_metric()
    r = ospin.g0w0_spin((inp.C, inp.eps, s.n_occ), (inp.C, inp.eps, s.n_occ), inp.t3c, inp.V,
                        s.ao_off, s.ri_off, inp.grids, inp.states, inp.states, s.filter_eps, S=S)
    ref = omet.g0w0_metric(inp.C, inp.eps, s.n_occ, inp.t3c, inp.V, S, s.ao_off, s.ri_off,
                           inp.grids, inp.states, s.filter_eps)
    np.testing.assert_allclose(r.wc_tau, ref.wc_tau, rtol=0, atol=1e-10 * np.abs(ref.wc_tau).max())
    for e in r.e_qp:
        np.testing.assert_allclose(e, ref.e_qp, rtol=0, atol=1e-9)
    up, dn = s.mean_field_spin(DELTA)
    st = np.array([s.n_occ - 1, s.n_occ])
    a = _run(inp, up, dn, s.n_occ, s.n_occ, st, st)
    b = ospin.g0w0_spin((up[0], up[1], s.n_occ), (dn[0], dn[1], s.n_occ), inp.t3c, inp.V,
                        s.ao_off, s.ri_off, inp.grids, st, st, s.filter_eps, S=np.eye(s.n_ri))
    np.testing.assert_allclose(b.wc_tau, a.wc_tau, rtol=0, atol=1e-12 * np.abs(a.wc_tau).max())
    np.testing.assert_allclose(b.e_qp[0], a.e_qp[0], rtol=0, atol=1e-10)
    np.testing.assert_allclose(b.e_qp[1], a.e_qp[1], rtol=0, atol=1e-10)
