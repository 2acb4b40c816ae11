"""One-tau chi plans and per-tau Sigma calls.

Eq. 3 and Eq. 10 are independent per tau point, so a chi plan made for one
tau point (executed once per tau_j) must give chi(tau_j) bit for bit equal
to slice j of the all-tau contraction: such a plan runs stage B (the D^vir
half contraction) for a group of pivot atoms per launch, rows (pivot, tau,
sigma), which changes which tile computes an element of N_b but not the
order of its sum, and stage C adds the pivots in the same order.  Covered on
13 AO / 40 RI strips (twelve pivots per stage-B group) one system at a time
and as a batch of three strips of different lengths (groups cut short at
each system's last atom), in every precision; and Sigma called one tau point
at a time with the exchange term skipped must give the slices of the all-tau
call."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _prep(n_atoms):
    import torch
    from gwinputs import configs
    from paper_2104_09857_amd import gw
    w = configs.strip(n_atoms, filter_eps=1e-9)
    s = w.system
    C, eps = s.mean_field()
    g = configs.grids_for(w, eps)
    mu = configs.mu_fermi(eps, s.n_occ)
    trip = s.triples()
    t3c = torch.as_tensor(s.bricks(trip), device="cuda")
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, trip, t3c)
    Cd = torch.as_tensor(C, device="cuda")
    do, dv = gw.build_gt(sysd, Cd, eps, mu, g.tau)
    return dict(w=w, s=s, sys=sysd, t3c=t3c, C=Cd, eps=eps, mu=mu, g=g, do=do, dv=dv)


@pytest.fixture(scope="module")
def strips():
    return [_prep(n) for n in (22, 15, 9)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_one_tau_plan_equals_all_tau(strips, prec):
    import torch
    from paper_2104_09857_amd import gw
    m = strips[0]
    eps_f = m["s"].filter_eps
    ref, _ = gw.contract_chi(m["sys"], m["do"], m["dv"], eps_f, prec=prec)
    plan = gw.ChiBatch([m["sys"]], 1, eps_f, prec=prec, timing=True)
    out = torch.empty_like(ref[:1])
    n_tau = ref.shape[0]
    for j in range(n_tau):
        print("case one-tau plan", prec, "tau", j, flush=True)
        st = plan.execute([m["do"][j:j + 1]], [m["dv"][j:j + 1]], [out])
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[j]), (prec, j)
        assert st["ms_stage"][1] > 0 and st["flops_c"] > 0
    # fewer stage-B launches than pivots: the pivots are grouped
    assert 0 < st["n_launch"][1] < st["n_launch"][0]
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_one_tau_batch_equals_single_calls(strips, prec):
    import torch
    from paper_2104_09857_amd import gw
    eps_f = strips[0]["s"].filter_eps
    refs = [gw.contract_chi(m["sys"], m["do"], m["dv"], eps_f, prec=prec)[0] for m in strips]
    plan = gw.ChiBatch([m["sys"] for m in strips], 1, eps_f, prec=prec)
    outs = [torch.empty_like(r[:1]) for r in refs]
    for j in (0, 5, 11):
        for pers in (0, 7):
            print("case one-tau batch", prec, "tau", j, "persistent", pers, flush=True)
            plan.set_config(plan.config()[0], pers)
            plan.execute([m["do"][j:j + 1] for m in strips], [m["dv"][j:j + 1] for m in strips],
                         outs)
            torch.cuda.synchronize()
            for m, o, r in zip(strips, outs, refs):
                assert torch.equal(o[0], r[j]), (m["w"].name, j, pers)
    plan.close()


def test_sigma_one_tau_at_a_time(strips):
    import torch
    from paper_2104_09857_amd import gw
    m = strips[1]
    s, g = m["s"], m["g"]
    eps_f = s.filter_eps
    V = torch.as_tensor(s.coulomb(), device="cuda")
    chi, _ = gw.contract_chi(m["sys"], m["do"], m["dv"], eps_f)
    wc = gw.screen_w(m["sys"], chi, V, g.cos_w, g.icos_w)
    d0, _ = gw.build_gt(m["sys"], m["C"], m["eps"], m["mu"], [0.0], d_vir=False)
    states = m["w"].states()
    so, sv, sx, _ = gw.contract_sigma(m["sys"], states, m["C"], m["do"], m["dv"], d0, wc, V, eps_f)
    for j in range(len(g.tau)):
        print("case sigma tau", j, flush=True)
        so1, sv1, sx1, st = gw.contract_sigma(m["sys"], states, m["C"], m["do"][j:j + 1],
                                              m["dv"][j:j + 1], None, wc[j:j + 1], None, eps_f)
        assert sx1 is None and st["flops"] > 0
        np.testing.assert_allclose(so1[:, 0], so[:, j], rtol=1e-13, atol=0)
        np.testing.assert_allclose(sv1[:, 0], sv[:, j], rtol=1e-13, atol=0)
