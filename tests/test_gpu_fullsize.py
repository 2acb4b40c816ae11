"""Full-size parity at the bench workload (300-atom ribbon, 3900 AO, 12000 RI,
12 tau, filter 1e-9), in the launch configuration bench.py times.

The oracle cannot build the whole chi here, so it computes sampled output
blocks one by one (Eq. 3 restricted to the blocks, from bricks drawn by the
host generator and D(tau) from the oracle's own sums over MOs); the rest is
checked through properties that hold at any size: exact symmetry and negative
semidefiniteness of random principal submatrices."""
import numpy as np
import pytest

from gwinputs import configs
from oracle import gt as ogt, chi as ochi

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def full():
    import torch
    from gwinputs import device as gdev
    from paper_2104_09857_amd import gw
    w = configs.by_name("strip300")
    s = w.system
    C, eps = s.mean_field()
    g = configs.grids_for(w, eps)
    mu = configs.mu_fermi(eps, s.n_occ)
    trip = s.triples()
    t3c = gdev.bricks_on_device(s, trip)
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, trip, t3c)
    Cd = torch.as_tensor(C, device="cuda")
    print("full-size inputs ready", flush=True)
    d_occ, d_vir = gw.build_gt(sysd, Cd, eps, mu, g.tau)
    chi, st = gw.contract_chi(sysd, d_occ, d_vir, s.filter_eps)
    torch.cuda.synchronize()
    print("full-size chi done", st["n_trip_kept"], flush=True)
    return dict(w=w, s=s, C=C, eps=eps, g=g, mu=mu, trip=trip, sys=sysd, Cd=Cd, d_occ=d_occ,
                d_vir=d_vir, chi=chi, stats=st)


def test_fullsize_chi_sampled_blocks(full):
    s, trip = full["s"], full["trip"]
    cache = {}

    def brick(a, b, c):
        if (a, b, c) not in cache:
            sel = trip[trip[:, 2] == c]
            vals = s.bricks(sel)
            for t, v in zip(sel, vals):
                cache[tuple(t)] = v.reshape(s.n_ao_atom, s.n_ao_atom, s.n_ri_atom)
        return cache[(a, b, c)]

    j_list = [0, len(full["g"].tau) - 1]
    do, dv = ogt.density_matrices(full["C"], full["eps"], s.n_occ, full["mu"], full["g"].tau[j_list])
    for (c, c2) in [(150, 150), (150, 153), (2, 297)]:
        for jj, j in enumerate(j_list):
            ref = ochi.chi_block(c, c2, trip, brick, do[jj], dv[jj], s.ao_off, s.ri_off, s.filter_eps)
            if np.sqrt((ref * ref).sum()) < s.filter_eps:
                ref = np.zeros_like(ref)
            got = full["chi"][j, s.ri_off[c]:s.ri_off[c + 1], s.ri_off[c2]:s.ri_off[c2 + 1]].cpu().numpy()
            scale = max(np.abs(ref).max(), 1e-300)
            print("block", c, c2, "tau", j, "max|ref|", scale, flush=True)
            assert np.abs(got - ref).max() <= 1e-12 * scale + 1e-14 * np.abs(
                full["chi"][j].diagonal().cpu().numpy()).max()


def test_fullsize_chi_properties(full):
    import torch
    chi = full["chi"]
    n = chi.shape[1]
    rng = np.random.default_rng(1)
    for j in (0, 6, 11):
        x = chi[j]
        assert torch.equal(x, x.T) or float((x - x.T).abs().max()) <= 1e-14 * float(x.abs().max())
        idx = torch.as_tensor(np.sort(rng.choice(n, 600, replace=False)), device="cuda")
        sub = x[idx][:, idx].cpu().numpy()
        ev = np.linalg.eigvalsh(0.5 * (sub + sub.T))
        assert ev.max() <= 1e-12 * np.abs(ev).max()
    st = full["stats"]
    assert st["n_trip_kept"] <= len(full["trip"]) and st["flops_c"] > 0
