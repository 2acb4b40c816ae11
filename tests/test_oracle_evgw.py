"""The evGW oracle (oracle/evgw.py) against fixed points that do not come
from the oracle itself: the update rule on a hand-worked example, weak
coupling (Sigma^c of higher order than Sigma^x), the first step equal to the
pinned G0W0 chain, and the converged energies reproducing themselves (the
definition of self-consistency after the QP equation, Eq. 12).

Input: the 12-atom chain with the three-center tensor scaled by 0.02, so
that the self-energy shifts are of a few eV (the unscaled synthetic tensor
gives keV shifts, for which feeding the energies back is meaningless)."""
import numpy as np
import pytest

from conftest import get_inputs
from oracle import qp as oqp, evgw as oev, chain as ochain

SCALE = 0.02


def test_update_rule_hand_example():
    eps0 = np.array([-3.0, -2.0, -1.0, 1.0, 2.0, 3.0])
    # HOMO-1, HOMO, LUMO computed: occupied corrections -0.5, -0.3 (mean -0.4),
    # virtual +0.6; the others take the mean of their class
    out = oev.update_energies(eps0, 3, np.array([1, 2, 3]), np.array([-2.5, -1.3, 1.6]))
    np.testing.assert_allclose(out, [-3.4, -2.5, -1.3, 1.6, 2.6, 3.6], rtol=0, atol=1e-15)
    # no computed virtual state: virtual levels unchanged
    out = oev.update_energies(eps0, 3, np.array([2]), np.array([-1.5]))
    np.testing.assert_allclose(out, [-3.5, -2.5, -1.5, 1.0, 2.0, 3.0], rtol=0, atol=1e-15)
    # a HOMO pushed above the LUMO is a failure
    assert oev.update_energies(eps0, 3, np.array([2, 3]), np.array([1.5, 1.2])) is None


@pytest.fixture(scope="module")
def chain_scaled():
    inp = get_inputs("chain12")
    return inp, inp.t3c * SCALE


def _run(inp, t3, **kw):
    s = inp.s
    return oev.evgw(inp.C, inp.eps, s.n_occ, t3, inp.V, s.ao_off, s.ri_off, inp.grids, inp.states,
                    s.filter_eps, **kw)


def test_weak_coupling_limit(chain_scaled):
    """Tensor scaled by 1e-3: Sigma^x (O(T^2), independent of the energies)
    shifts the levels, the energy-dependent Sigma^c is O(T^4): evGW must stop
    within a few steps at G0W0 to O(T^4).  (Feeding the updated energies into
    the QP equation itself would make the levels drift by Sigma^x per step.)"""
    inp, t3 = chain_scaled
    s = inp.s
    weak = t3 / SCALE * 1e-3
    r = _run(inp, weak, tol=1e-12, max_iter=6)
    assert r.converged and len(r.history) <= 4
    shift = np.abs(r.e_qp - inp.eps[inp.states]).max()
    assert shift > 1e-6
    assert np.abs(r.e_qp - r.history[0]).max() < 1e-6 * shift


def test_first_step_is_g0w0_and_fixed_point(chain_scaled):
    inp, t3 = chain_scaled
    s = inp.s
    r = _run(inp, t3, tol=1e-8, max_iter=25)
    assert r.converged and len(r.history) >= 3
    ref = ochain.g0w0(inp.C, inp.eps, s.n_occ, t3, inp.V, s.ao_off, s.ri_off, inp.grids,
                      inp.states, s.filter_eps)
    np.testing.assert_allclose(r.history[0], ref.e_qp, rtol=0, atol=1e-12)
    # the steps contract towards the fixed point
    d = [np.abs(r.history[i] - r.history[i - 1]).max() for i in range(1, len(r.history))]
    assert all(d[i + 1] < d[i] for i in range(len(d) - 1))
    # one more step with the Green's function of the converged energies
    # reproduces them
    eps_g = oev.update_energies(inp.eps, s.n_occ, inp.states, r.e_qp)
    again, status = oev.one_step(inp.C, inp.eps, eps_g, s.n_occ, t3, inp.V, s.ao_off, s.ri_off,
                                 inp.grids, inp.states, s.filter_eps, 2.0,
                                 np.zeros(len(inp.states)), oqp.PADE_WINDOW_HA)
    assert np.all(status == 0)
    assert np.abs(again - r.e_qp).max() < 1e-8
    # and evGW moved the energies away from G0W0 (the Green's function changed)
    assert np.abs(r.e_qp - ref.e_qp).max() > 1e-5
