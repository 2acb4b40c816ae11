"""Non-orthogonal bases on the library's calls (gw_screen_w_metric for W~^c
and V~, generalized eigenvectors through gw_build_gt) against the FP64
oracle (oracle/metric.py).  Inputs: the 12-atom chain and a 20-atom ribbon
with 5 AO / 12 RI per atom (filter 1e-4), Gaussian RI and AO overlaps
(gwinputs System.ri_metric / ao_metric), MOs of H C = S_ao C eps, tensors
scaled by 0.02 (shifts of a few eV).  Bars as for the orthogonal chain: chi
and W~^c within 1e-10 of their largest element, V~ within 1e-12, QP energies
within 1e-6 Ha."""
import numpy as np
import pytest

from conftest import get_inputs
from oracle import chi as ochi, metric as omet

pytestmark = pytest.mark.gpu
SCALE = 0.02


@pytest.fixture(scope="module", params=["chain12", "strip20_small_basis"])
def case(request):
    if request.param == "chain12":
        inp = get_inputs("chain12")
    else:
        inp = get_inputs("strip20", n_ao=5, n_ri=12, filter_eps=1e-4, n_tau=8)
    s = inp.s
    S = s.ri_metric()
    C, eps = s.mean_field_nonorth(s.ao_metric())
    # the library filters the scaled bricks: so does the oracle's tensor
    t3 = ochi.dense_from_bricks(inp.trip, inp.bricks * SCALE, s.ao_off, s.ri_off, s.n_ao, s.n_ri,
                                s.filter_eps)
    ref = omet.g0w0_metric(C, eps, s.n_occ, t3, inp.V, S, s.ao_off, s.ri_off, inp.grids,
                           inp.states, s.filter_eps)
    assert np.all(ref.status == 0)
    return request.param, inp, S, C, eps, ref


def test_metric_chain_matches_oracle(case):
    import torch
    from paper_2104_09857_amd import gw, pipeline
    name, inp, S, C, eps, ref = case
    s, g = inp.s, inp.grids
    print("case", name, flush=True)
    t3c = torch.as_tensor(inp.bricks * SCALE, device="cuda")
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, inp.trip, t3c)
    mu = 0.5 * (eps[s.n_occ - 1] + eps[s.n_occ])
    dev = lambda a: torch.as_tensor(a, device="cuda")
    out = pipeline.g0w0(sysd, dev(C), eps, mu, dev(inp.V), g.tau, g.omega, g.cos_w, g.sin_w,
                        g.icos_w, inp.states, s.filter_eps, S_ri=dev(S))
    torch.cuda.synchronize()
    chi, wc = out["chi"].cpu().numpy(), out["wc"].cpu().numpy()
    assert np.abs(chi - ref.chi_tau).max() <= 1e-10 * np.abs(ref.chi_tau).max()
    assert np.abs(wc - ref.wc_tau).max() <= 1e-10 * np.abs(ref.wc_tau).max()
    np.testing.assert_allclose(out["sig_x"], ref.sig_x, rtol=0, atol=1e-9)
    print("case", name, "dE Ha", np.abs(out["e_qp"] - ref.e_qp).max(), flush=True)
    assert np.all(out["status"] == 0)
    np.testing.assert_allclose(out["e_qp"], ref.e_qp, rtol=0, atol=1e-6)


def test_screen_w_metric_v_tilde_identity_and_errors():
    """V~ against S^-1 V S^-1 of the oracle; S = 1 gives gw_screen_w's W^c
    and V~ = V; a singular S is rejected."""
    import torch
    from paper_2104_09857_amd import gw
    inp = get_inputs("chain12")
    s, g = inp.s, inp.grids
    t3c = torch.as_tensor(inp.bricks, device="cuda")
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, inp.trip, t3c)
    gen = torch.Generator(device="cpu").manual_seed(11)
    a = torch.randn((len(g.tau), s.n_ri, s.n_ri), generator=gen, dtype=torch.float64)
    chi = -(a @ a.transpose(1, 2)) * (1e-3 / s.n_ri)
    V = torch.as_tensor(inp.V, device="cuda")
    S = s.ri_metric()
    wt, vt = gw.screen_w_metric(sysd, chi.cuda(), V, torch.as_tensor(S, device="cuda"), g.cos_w,
                                g.icos_w, 2.0)
    w_ref, v_ref = omet.screen_w_metric(chi.numpy(), inp.V, S, g.cos_w, g.icos_w, 2.0)
    torch.cuda.synchronize()
    assert np.abs(vt.cpu().numpy() - v_ref).max() <= 1e-12 * np.abs(v_ref).max()
    assert np.abs(wt.cpu().numpy() - w_ref).max() <= 1e-10 * np.abs(w_ref).max()
    eye = torch.eye(s.n_ri, dtype=torch.float64, device="cuda")
    w1, v1 = gw.screen_w_metric(sysd, chi.cuda(), V, eye, g.cos_w, g.icos_w, 2.0)
    w0 = gw.screen_w(sysd, chi.cuda(), V, g.cos_w, g.icos_w, 2.0)
    torch.cuda.synchronize()
    w0 = w0.cpu().numpy()
    assert np.abs(w1.cpu().numpy() - w0).max() <= 1e-12 * np.abs(w0).max()
    assert np.abs(v1.cpu().numpy() - inp.V).max() <= 1e-13 * np.abs(inp.V).max()
    bad = eye.clone()
    bad[3, 3] = -1.0
    with pytest.raises(gw.GWError):
        gw.screen_w_metric(sysd, chi.cuda(), V, bad, g.cos_w, g.icos_w, 2.0)
