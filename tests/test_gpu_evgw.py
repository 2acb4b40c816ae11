"""Eigenvalue self-consistent GW (evGW) on the library's calls against the
FP64 oracle (oracle/evgw.py): the G0W0 chain repeated with the Green's
function of gw_evgw_update's energies until the QP energies stop changing.

Inputs: the 12-atom chain and a 20-atom ribbon with 5 AO / 12 RI per atom
(filter 1e-4, 8 tau), their three-center tensors scaled by 0.02 so that the
self-energy shifts are of 0.4-2 eV (the unscaled synthetic tensors give keV
shifts, for which feeding the energies back is meaningless).  Bar: QP
energies within 1e-6 Ha of the oracle, as for the plain path; the first step
is G0W0."""
import numpy as np
import pytest

from conftest import get_inputs
from oracle import chi as ochi, evgw as oev

pytestmark = pytest.mark.gpu
SCALE = 0.02
TOL = 1e-8


@pytest.fixture(scope="module", params=["chain12", "strip20_small_basis"])
def case(request):
    if request.param == "chain12":
        inp = get_inputs("chain12")
    else:
        inp = get_inputs("strip20", n_ao=5, n_ri=12, filter_eps=1e-4, n_tau=8)
    s = inp.s
    bricks = inp.bricks * SCALE
    t3 = ochi.dense_from_bricks(inp.trip, bricks, s.ao_off, s.ri_off, s.n_ao, s.n_ri, s.filter_eps)
    ref = oev.evgw(inp.C, inp.eps, s.n_occ, t3, inp.V, s.ao_off, s.ri_off, inp.grids, inp.states,
                   s.filter_eps, tol=TOL, max_iter=25)
    assert ref.converged
    return request.param, inp, bricks, ref


def test_evgw_matches_oracle(case):
    import torch
    from paper_2104_09857_amd import gw, pipeline
    name, inp, bricks, ref = case
    s, g = inp.s, inp.grids
    print("case", name, "oracle steps", len(ref.history), flush=True)
    t3c = torch.as_tensor(bricks, device="cuda")
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, inp.trip, t3c)
    out = pipeline.evgw(sysd, torch.as_tensor(inp.C, device="cuda"), inp.eps, inp.mu_f,
                        torch.as_tensor(inp.V, device="cuda"), g.tau, g.omega, g.cos_w, g.sin_w,
                        g.icos_w, inp.states, s.filter_eps, tol=TOL, max_iter=25)
    print("case", name, "gpu steps", out["steps"], "dE Ha", np.abs(out["e_qp"] - ref.e_qp).max(),
          flush=True)
    assert out["converged"]
    assert abs(out["steps"] - len(ref.history)) <= 1
    np.testing.assert_allclose(out["history"][0], ref.history[0], rtol=0, atol=1e-6)
    np.testing.assert_allclose(out["e_qp"], ref.e_qp, rtol=0, atol=1e-6)
    np.testing.assert_allclose(out["eps_g"], oev.update_energies(inp.eps, s.n_occ, inp.states,
                                                                  out["history"][-2]),
                               rtol=0, atol=1e-12)
