"""Atoms of two elements (per-atom AO / RI counts, gw_system.ao_off / ri_off)
through the library's chain against the FP64 oracle, which takes the ragged
atom offsets directly.

Inputs: a 14-atom ribbon (two columns of 7, 2.5 bohr) whose edge atoms keep
only their first 5 AO / 12 RI functions (gwinputs System.light_atoms, the
hydrogens of a nanoribbon edge) and the others all 13 / 40; H, V and the
tensor of the uniform generator restricted to the kept functions; bricks in
the padded layout with zeros for the missing functions; MOs of the restricted
H.  The tensor is scaled by 0.02 (self-energy shifts of eV size); filter
1e-5, 12 tau, HOMO-4 .. LUMO+4.  Bars: chi and W^c within 1e-10 of their
largest element, Sigma^x within 1e-9 Ha, QP energies within 1e-6 Ha."""
import numpy as np
import pytest

from oracle import chain as ochain, chi as ochi

pytestmark = pytest.mark.gpu
SCALE = 0.02


def test_mixed_elements_chain_matches_oracle():
    import torch
    from gwinputs import configs
    from paper_2104_09857_amd import gw, pipeline
    w = configs.strip(14, filter_eps=1e-5)
    s = w.system
    light = [k for k in range(s.n_atoms) if k % 7 in (0, 6)]
    m = s.light_atoms(light, 5, 12)
    ao_idx, ri_idx = m["ao_idx"], m["ri_idx"]
    n_ao, n_ri = len(ao_idx), len(ri_idx)
    H = s.hamiltonian()[np.ix_(ao_idx, ao_idx)]
    eps, v = np.linalg.eigh(H)
    C = np.ascontiguousarray(v.T)
    n_occ = n_ao // 2
    V = s.coulomb()[np.ix_(ri_idx, ri_idx)]
    trip = s.triples()
    br = s.bricks(trip).reshape(len(trip), s.n_ao_atom, s.n_ao_atom, s.n_ri_atom) * SCALE
    br = br * m["ao_mask"][trip[:, 0], :, None, None] * m["ao_mask"][trip[:, 1], None, :, None] \
        * m["ri_mask"][trip[:, 2], None, None, :]
    full = ochi.dense_from_bricks(trip, br, s.ao_off, s.ri_off, s.n_ao, s.n_ri, s.filter_eps)
    t3 = np.ascontiguousarray(full[np.ix_(ao_idx, ao_idx, ri_idx)])
    g = configs.grids_for(w, eps)
    states = np.arange(n_occ - 5, n_occ + 5)
    ref = ochain.g0w0(C, eps, n_occ, t3, V, m["ao_off"], m["ri_off"], g, states, s.filter_eps)
    assert np.all(ref.status == 0)
    print("case strip14 mixed", n_ao, "AO", n_ri, "RI, shifts eV",
          np.round((ref.e_qp - eps[states]) * 27.2114, 3), flush=True)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, n_occ, trip, dev(br), s.xyz,
                     ao_off=m["ao_off"], ri_off=m["ri_off"])
    assert sysd.n_ao == n_ao and sysd.n_ri == n_ri
    mu = 0.5 * (eps[n_occ - 1] + eps[n_occ])
    out = pipeline.g0w0(sysd, dev(C), eps, mu, dev(V), g.tau, g.omega, g.cos_w, g.sin_w, g.icos_w,
                        states, s.filter_eps)
    torch.cuda.synchronize()
    chi, wc = out["chi"].cpu().numpy(), out["wc"].cpu().numpy()
    assert chi.shape == ref.chi_tau.shape
    assert np.abs(chi - ref.chi_tau).max() <= 1e-10 * np.abs(ref.chi_tau).max()
    assert np.abs(wc - ref.wc_tau).max() <= 1e-10 * np.abs(ref.wc_tau).max()
    np.testing.assert_allclose(out["sig_x"], ref.sig_x, rtol=0, atol=1e-9)
    print("case strip14 mixed dE Ha", np.abs(out["e_qp"] - ref.e_qp).max(), flush=True)
    assert np.all(out["status"] == 0)
    np.testing.assert_allclose(out["e_qp"], ref.e_qp, rtol=0, atol=1e-6)
    # the batched plans and the block screener take uniform systems only
    with pytest.raises(gw.GWError):
        gw.ChiBatch([sysd], len(g.tau), s.filter_eps)
