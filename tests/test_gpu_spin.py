"""Open-shell G0W0 on the library's calls (gw_screen_w_spins for the common
W) against the FP64 open-shell oracle (oracle/spin.py).  Inputs: the 12-atom
chain with a spin-dependent potential of 0.05 Ha per AO, equal occupations
(broken-symmetry singlet) and, with a 0.09 Ha Zeeman split, one electron
moved to the up channel; a 20-atom ribbon (5 AO / 12 RI per atom, filter
1e-4) as a singlet.  The three-center tensors are scaled by 0.02 so that the
self-energy shifts are of a few eV (the unscaled synthetic tensors give keV
shifts).  Bars as for the closed-shell chain: chi and W^c to
1e-10 of their largest element, QP energies to 1e-6 Ha."""
import numpy as np
import pytest

from conftest import get_inputs
from oracle import chi as ochi, spin as ospin

pytestmark = pytest.mark.gpu
DELTA = 0.05
SCALE = 0.02
CASES = {"chain12_singlet": ("chain12", 0.0, 0), "chain12_triplet": ("chain12", 0.09, 1),
         "strip20_singlet": ("strip20", 0.0, 0)}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    name, zeeman, moved = CASES[request.param]
    if name == "chain12":
        inp = get_inputs("chain12")
    else:
        inp = get_inputs("strip20", n_ao=5, n_ri=12, filter_eps=1e-4, n_tau=8)
    s = inp.s
    up, dn = s.mean_field_spin(DELTA, zeeman)
    n_up, n_dn = s.n_occ + moved, s.n_occ - moved
    st_up = np.array([n_up - 1, n_up], dtype=np.int32)
    st_dn = np.array([n_dn - 1, n_dn], dtype=np.int32)
    # the library filters the scaled bricks: so does the oracle's tensor
    t3 = ochi.dense_from_bricks(inp.trip, inp.bricks * SCALE, s.ao_off, s.ri_off, s.n_ao, s.n_ri,
                                s.filter_eps)
    ref = ospin.g0w0_spin((up[0], up[1], n_up), (dn[0], dn[1], n_dn), t3, inp.V, s.ao_off,
                          s.ri_off, inp.grids, st_up, st_dn, s.filter_eps)
    return request.param, inp, up, dn, n_up, n_dn, st_up, st_dn, ref


def test_open_shell_matches_oracle(case):
    import torch
    from paper_2104_09857_amd import gw, pipeline
    name, inp, up, dn, n_up, n_dn, st_up, st_dn, ref = case
    s, g = inp.s, inp.grids
    print("case", name, flush=True)
    t3c = torch.as_tensor(inp.bricks * SCALE, device="cuda")
    sys_up = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, n_up, inp.trip, t3c)
    sys_dn = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, n_dn, inp.trip, t3c)
    dev = lambda a: torch.as_tensor(a, device="cuda")
    out = pipeline.g0w0_spin(sys_up, sys_dn, dev(up[0]), dev(dn[0]), up[1], dn[1], dev(inp.V),
                             g.tau, g.omega, g.cos_w, g.sin_w, g.icos_w, st_up, st_dn,
                             s.filter_eps)
    torch.cuda.synchronize()
    assert out["mu_f"] == pytest.approx(ref.mu_f, abs=1e-15)
    for got, want in ((out["chi_up"], ref.chi_up), (out["chi_dn"], ref.chi_dn),
                      (out["wc"], ref.wc_tau)):
        got = got.cpu().numpy()
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
    print("case", name, "dE Ha", np.abs(out["e_qp_up"] - ref.e_qp[0]).max(),
          np.abs(out["e_qp_dn"] - ref.e_qp[1]).max(), flush=True)
    assert np.all(out["status_up"] == 0) and np.all(out["status_dn"] == 0)
    assert np.all(ref.status[0] == 0) and np.all(ref.status[1] == 0)
    np.testing.assert_allclose(out["e_qp_up"], ref.e_qp[0], rtol=0, atol=1e-6)
    np.testing.assert_allclose(out["e_qp_dn"], ref.e_qp[1], rtol=0, atol=1e-6)


def test_screen_w_spins_is_screen_w_of_the_sum():
    """gw_screen_w_spins(chi_up, chi_dn) equals gw_screen_w(chi_up + chi_dn,
    spin factor 1) to rounding, and rejects mismatched stacks."""
    import torch
    from paper_2104_09857_amd import gw
    inp = get_inputs("chain12")
    s, g = inp.s, inp.grids
    t3c = torch.as_tensor(inp.bricks, device="cuda")
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, inp.trip, t3c)
    gen = torch.Generator(device="cpu").manual_seed(7)
    n_tau = len(g.tau)
    a = torch.randn((n_tau, s.n_ri, s.n_ri), generator=gen, dtype=torch.float64)
    b = torch.randn((n_tau, s.n_ri, s.n_ri), generator=gen, dtype=torch.float64)
    # negative semidefinite, as a response function
    a = -(a @ a.transpose(1, 2)) * (1e-3 / s.n_ri)
    b = -(b @ b.transpose(1, 2)) * (1e-3 / s.n_ri)
    V = torch.as_tensor(inp.V, device="cuda")
    w2 = gw.screen_w_spins(sysd, a.cuda(), b.cuda(), V, g.cos_w, g.icos_w)
    w1 = gw.screen_w(sysd, (a + b).cuda(), V, g.cos_w, g.icos_w, 1.0)
    torch.cuda.synchronize()
    w1, w2 = w1.cpu().numpy(), w2.cpu().numpy()
    assert np.abs(w1 - w2).max() <= 1e-12 * np.abs(w1).max()
    with pytest.raises(ValueError):
        gw.screen_w_spins(sysd, a.cuda(), b[:-1].cuda(), V, g.cos_w, g.icos_w)


def test_open_shell_with_ri_metric_matches_oracle():
    """The paper's ribbon setting: open-shell singlet with the overlap-metric
    RI (gw_screen_w_spins_metric), chain12, tensor scaled by 0.02."""
    import torch
    from paper_2104_09857_amd import gw, pipeline
    inp = get_inputs("chain12")
    s, g = inp.s, inp.grids
    up, dn = s.mean_field_spin(DELTA)
    S = s.ri_metric()
    st = np.array([s.n_occ - 1, s.n_occ], dtype=np.int32)
    t3 = ochi.dense_from_bricks(inp.trip, inp.bricks * SCALE, s.ao_off, s.ri_off, s.n_ao, s.n_ri,
                                s.filter_eps)
    ref = ospin.g0w0_spin((up[0], up[1], s.n_occ), (dn[0], dn[1], s.n_occ), t3, inp.V, s.ao_off,
                          s.ri_off, g, st, st, s.filter_eps, S=S)
    t3c = torch.as_tensor(inp.bricks * SCALE, device="cuda")
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, inp.trip, t3c)
    dev = lambda a: torch.as_tensor(a, device="cuda")
    out = pipeline.g0w0_spin(sysd, sysd, dev(up[0]), dev(dn[0]), up[1], dn[1], dev(inp.V), g.tau,
                             g.omega, g.cos_w, g.sin_w, g.icos_w, st, st, s.filter_eps,
                             S_ri=dev(S))
    torch.cuda.synchronize()
    wc = out["wc"].cpu().numpy()
    assert np.abs(wc - ref.wc_tau).max() <= 1e-10 * np.abs(ref.wc_tau).max()
    assert np.all(out["status_up"] == 0) and np.all(out["status_dn"] == 0)
    np.testing.assert_allclose(out["e_qp_up"], ref.e_qp[0], rtol=0, atol=1e-6)
    np.testing.assert_allclose(out["e_qp_dn"], ref.e_qp[1], rtol=0, atol=1e-6)
