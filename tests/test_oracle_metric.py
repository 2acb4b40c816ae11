"""The non-orthogonal-basis oracle (oracle/metric.py) against fixed points
that do not come from it: S = 1 gives the pinned chain; the QP energies are
invariant under invertible, non-orthogonal changes of the RI basis and of
the AO basis (the method depends on the spans only); the density matrices of
generalized eigenvectors obey the metric forms of idempotency, trace and
completeness.  Input: the 12-atom chain (Gaussian metrics of
gwinputs System.ri_metric / ao_metric), tensor scaled by 0.02 so that the
shifts are of a few eV, filter 0 (a basis change mixes atom blocks)."""
import numpy as np
import pytest

from conftest import get_inputs
from oracle import chain as ochain, gt as ogt, metric as omet

SCALE = 0.02


@pytest.fixture(scope="module")
def chain():
    inp = get_inputs("chain12")
    return inp, inp.s.dense_t3c() * SCALE


def _run(inp, C, eps, t3, V, S):
    s = inp.s
    return omet.g0w0_metric(C, eps, s.n_occ, t3, V, S, s.ao_off, s.ri_off, inp.grids, inp.states)


def _basis_change(n, seed):
    """Invertible, far from orthogonal: I + 0.5 G / sqrt(n), G standard normal."""
    g = np.random.default_rng(seed).standard_normal((n, n))
    a = np.eye(n) + 0.5 * g / np.sqrt(n)
    assert np.linalg.cond(a) < 50 and np.abs(a @ a.T - np.eye(n)).max() > 0.3
    return a


def test_identity_metric_is_the_chain(chain):
    inp, t3 = chain
    s = inp.s
    r = _run(inp, inp.C, inp.eps, t3, inp.V, np.eye(s.n_ri))
    ref = ochain.g0w0(inp.C, inp.eps, s.n_occ, t3, inp.V, s.ao_off, s.ri_off, inp.grids, inp.states)
    np.testing.assert_allclose(r.wc_tau, ref.wc_tau, rtol=0, atol=1e-12 * np.abs(ref.wc_tau).max())
    np.testing.assert_allclose(r.e_qp, ref.e_qp, rtol=0, atol=1e-10)


def test_ri_basis_change_invariance(chain):
    inp, t3 = chain
    s = inp.s
    S = s.ri_metric()
    r = _run(inp, inp.C, inp.eps, t3, inp.V, S)
    assert np.all(r.status == 0)
    A = _basis_change(s.n_ri, 1)
    t3a = np.einsum("mnp,qp->mnq", t3, A, optimize=True)
    ra = _run(inp, inp.C, inp.eps, t3a, A @ inp.V @ A.T, A @ S @ A.T)
    np.testing.assert_allclose(ra.chi_tau, A @ r.chi_tau @ A.T, rtol=0,
                               atol=1e-11 * np.abs(ra.chi_tau).max())
    np.testing.assert_allclose(ra.sig_x, r.sig_x, rtol=0, atol=1e-10)
    np.testing.assert_allclose(ra.e_qp, r.e_qp, rtol=0, atol=1e-9)
    # the metric matters: S = 1 in the changed basis gives other energies
    rb = _run(inp, inp.C, inp.eps, t3a, A @ inp.V @ A.T, np.eye(s.n_ri))
    assert np.abs(rb.e_qp - r.e_qp).max() > 1e-3
    # and S matters in the unchanged basis
    r1 = _run(inp, inp.C, inp.eps, t3, inp.V, np.eye(s.n_ri))
    assert np.abs(r1.e_qp - r.e_qp).max() > 1e-3


def test_ao_basis_change_invariance(chain):
    inp, t3 = chain
    s = inp.s
    S = s.ri_metric()
    Sa = s.ao_metric()
    C, eps = s.mean_field_nonorth(Sa)
    r = _run(inp, C, eps, t3, inp.V, S)
    assert np.all(r.status == 0)
    B = _basis_change(s.n_ao, 2)
    t3b = np.einsum("am,mnp,bn->abp", B, t3, B, optimize=True)
    Cb = np.linalg.solve(B.T, C.T).T                          # C B^-1
    rb = _run(inp, Cb, eps, t3b, inp.V, S)
    np.testing.assert_allclose(rb.chi_tau, r.chi_tau, rtol=0, atol=1e-11 * np.abs(r.chi_tau).max())
    np.testing.assert_allclose(rb.e_qp, r.e_qp, rtol=0, atol=1e-9)


def test_generalized_eigenvector_density(chain):
    inp, _ = chain
    s = inp.s
    Sa = s.ao_metric()
    C, eps = s.mean_field_nonorth(Sa)
    mu = 0.5 * (eps[s.n_occ - 1] + eps[s.n_occ])
    do, dv = ogt.density_matrices(C, eps, s.n_occ, mu, [0.0])
    d = do[0]
    np.testing.assert_allclose(d @ Sa @ d, d, rtol=0, atol=1e-12)
    assert abs(np.trace(d @ Sa) - s.n_occ) < 1e-10
    np.testing.assert_allclose((d + dv[0]) @ Sa, np.eye(s.n_ao), rtol=0, atol=1e-12)
    # the orthonormal-basis forms fail: the AO basis is really non-orthogonal
    assert np.abs(d @ d - d).max() > 1e-2
