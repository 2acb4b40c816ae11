"""Three-center overlap integrals of s-type Gaussians (Eq. 4) on the GPU
(gw_t3c_gaussian) against the oracle's closed form, and the G0W0 chain with
those integrals and the overlap metric of the same functions (Eq. 5) against
the FP64 oracle chain on the oracle's own integrals.

Inputs: ribbon geometry (7 wide, 2.5 bohr), 5 AO / 12 RI normalized s
Gaussians per atom (gwinputs System.gaussian_functions: exponents geometric
over [0.25, 1.2] and [0.2, 2.0], centres offset from the atom on spheres of
0.5 and 0.9 bohr), every atom triple enumerated, the filter dropping the
bricks and blocks below 1e-8 (a coarser filter breaks the negative
semidefiniteness of chi by more than the ill-conditioned S^-1 tolerates:
epsilon(i w) turns indefinite); S_ao and S_ri the overlaps of the same
functions (MOs of H C = S_ao C eps); shifts of 30-70 eV.  Bars: bricks within 1e-13 of the
oracle's (relative to the largest), chi and W~^c within 1e-10 of their
largest element, QP energies within 1e-6 Ha."""
import numpy as np
import pytest

from oracle import chi as ochi, integrals as oint, metric as omet

pytestmark = pytest.mark.gpu


def _system(n_atoms, filter_eps=1e-8):
    from gwinputs import configs
    w = configs.strip(n_atoms, filter_eps=filter_eps, n_ao=5, n_ri=12, n_tau=8)
    s = w.system
    return w, s, s.gaussian_functions(), s.all_triples()


def test_t3c_gaussian_matches_oracle():
    import torch
    from paper_2104_09857_amd import gw
    w, s, f, trip = _system(9)
    sysd = gw.System(s.n_atoms, 5, 12, s.n_occ, trip, None, s.xyz)
    print("case strip9 gaussian bricks", len(trip), flush=True)
    got = gw.t3c_gaussian(sysd, f["ao_exp"], f["ao_off"], f["ri_exp"], f["ri_off"])
    torch.cuda.synchronize()
    ref = oint.bricks(s.xyz, trip, f["ao_exp"], f["ao_off"], f["ri_exp"], f["ri_off"])
    got = got.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # and elementwise relative accuracy where the integrals are not tiny
    big = np.abs(ref) > 1e-8 * np.abs(ref).max()
    assert np.abs(got[big] / ref[big] - 1).max() < 1e-12
    # exponents must be positive
    with pytest.raises(gw.GWError):
        gw.t3c_gaussian(sysd, -f["ao_exp"], f["ao_off"], f["ri_exp"], f["ri_off"])


def test_chain_with_gaussian_integrals_matches_oracle():
    import torch
    from gwinputs import configs
    from paper_2104_09857_amd import gw, pipeline
    w, s, f, trip = _system(20)
    S_ao = s.gaussian_overlap(f["ao_exp"], f["ao_off"])
    S_ri = s.gaussian_overlap(f["ri_exp"], f["ri_off"])
    C, eps = s.mean_field_nonorth(S_ao)
    g = configs.grids_for(w, eps)
    states = w.states()
    V = s.coulomb()
    br = oint.bricks(s.xyz, trip, f["ao_exp"], f["ao_off"], f["ri_exp"], f["ri_off"])
    t3 = ochi.dense_from_bricks(trip, br, s.ao_off, s.ri_off, s.n_ao, s.n_ri, s.filter_eps)
    ref = omet.g0w0_metric(C, eps, s.n_occ, t3, V, S_ri, s.ao_off, s.ri_off, g, states,
                           s.filter_eps)
    assert np.all(ref.status == 0)
    print("case strip20 gaussian chain, shifts eV", np.round((ref.e_qp - eps[states]) * 27.2114, 3),
          flush=True)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    sysd = gw.System(s.n_atoms, 5, 12, s.n_occ, trip, None, s.xyz)
    t3c = gw.t3c_gaussian(sysd, f["ao_exp"], f["ao_off"], f["ri_exp"], f["ri_off"])
    sysd = gw.System(s.n_atoms, 5, 12, s.n_occ, trip, t3c, s.xyz)
    mu = 0.5 * (eps[s.n_occ - 1] + eps[s.n_occ])
    out = pipeline.g0w0(sysd, dev(C), eps, mu, dev(V), g.tau, g.omega, g.cos_w, g.sin_w, g.icos_w,
                        states, s.filter_eps, S_ri=dev(S_ri))
    torch.cuda.synchronize()
    chi, wc = out["chi"].cpu().numpy(), out["wc"].cpu().numpy()
    assert np.abs(chi - ref.chi_tau).max() <= 1e-10 * np.abs(ref.chi_tau).max()
    assert np.abs(wc - ref.wc_tau).max() <= 1e-10 * np.abs(ref.wc_tau).max()
    print("case strip20 gaussian chain dE Ha", np.abs(out["e_qp"] - ref.e_qp).max(), flush=True)
    assert np.all(out["status"] == 0)
    np.testing.assert_allclose(out["e_qp"], ref.e_qp, rtol=0, atol=1e-6)
