"""Periodic Gamma-point cells on the library's calls against the FP64
oracle (oracle/periodic.py, the plain reciprocal-lattice sum): the Coulomb
matrix of Gaussian RI charges from gw_coulomb_periodic (Ewald split) at the
automatic and two given splitting parameters, on the 27-atom cubic cell
(5 AO / 12 RI per atom) and on random charges in a non-cubic cell; then
G0W0 on that cell (minimum-image tensor, filter 1e-4, 8 tau, tensor scaled
by 0.02) with the library's V against the oracle chain with the oracle's V.
Bars: V within 1e-12 of its largest element; chi and W^c within 1e-10; QP
energies within 1e-6 Ha."""
import numpy as np
import pytest

from conftest import Inputs
from oracle import chain as ochain, chi as ochi, periodic as oper

pytestmark = pytest.mark.gpu
SCALE = 0.02


@pytest.fixture(scope="module")
def bulk():
    from gwinputs import configs
    inp = Inputs(configs.bulk(3, filter_eps=1e-4, n_ao=5, n_ri=12, n_tau=8))
    s = inp.s
    R, a = s.ri_charges()
    return inp, R, a, oper.coulomb_periodic(R, a, s.cell)


def test_coulomb_matches_oracle(bulk):
    import torch
    from paper_2104_09857_amd import gw
    inp, R, a, V_ref = bulk
    cell = inp.s.cell
    for eta in (0.0, 0.25, 0.45):
        V, info = gw.coulomb_periodic(R, a, cell, eta=eta)
        torch.cuda.synchronize()
        print("eta", eta, info, flush=True)
        err = np.abs(V.cpu().numpy() - V_ref).max()
        assert err <= 1e-12 * np.abs(V_ref).max(), (eta, err)
    rng = np.random.default_rng(5)
    cell2 = np.array([6.0, 7.5, 9.0])
    R2 = rng.uniform(0, 1, (40, 3)) * cell2
    a2 = rng.uniform(0.5, 2.0, 40)
    V2, info = gw.coulomb_periodic(R2, a2, cell2)
    ref2 = oper.coulomb_periodic(R2, a2, cell2)
    torch.cuda.synchronize()
    assert np.abs(V2.cpu().numpy() - ref2).max() <= 1e-12 * np.abs(ref2).max()


def test_periodic_chain_matches_oracle(bulk):
    import torch
    from paper_2104_09857_amd import gw, pipeline
    inp, R, a, V_ref = bulk
    s, g = inp.s, inp.grids
    t3 = ochi.dense_from_bricks(inp.trip, inp.bricks * SCALE, s.ao_off, s.ri_off, s.n_ao, s.n_ri,
                                s.filter_eps)
    ref = ochain.g0w0(inp.C, inp.eps, s.n_occ, t3, V_ref, s.ao_off, s.ri_off, g, inp.states,
                      s.filter_eps)
    assert np.all(ref.status == 0)
    V, _ = gw.coulomb_periodic(R, a, s.cell)
    t3c = torch.as_tensor(inp.bricks * SCALE, device="cuda")
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, inp.trip, t3c)
    out = pipeline.g0w0(sysd, torch.as_tensor(inp.C, device="cuda"), inp.eps, inp.mu_f, V, g.tau,
                        g.omega, g.cos_w, g.sin_w, g.icos_w, inp.states, s.filter_eps)
    torch.cuda.synchronize()
    chi, wc = out["chi"].cpu().numpy(), out["wc"].cpu().numpy()
    assert np.abs(chi - ref.chi_tau).max() <= 1e-10 * np.abs(ref.chi_tau).max()
    assert np.abs(wc - ref.wc_tau).max() <= 1e-10 * np.abs(ref.wc_tau).max()
    print("dE Ha", np.abs(out["e_qp"] - ref.e_qp).max(), flush=True)
    assert np.all(out["status"] == 0)
    np.testing.assert_allclose(out["e_qp"], ref.e_qp, rtol=0, atol=1e-6)
