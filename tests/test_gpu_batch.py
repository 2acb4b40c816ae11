"""Batched persistent form of the chi contraction (gw_chi_batch_*).

Two molecule sets of uneven size (random 3D packings, as in the batched
workload): 7 molecules of 3-9 atoms with 5 AO / 12 RI per atom and 4 tau
(filter 1e-6), and 5 molecules of 4-12 atoms with the production basis
13 AO / 40 RI per atom and 12 tau (filter 1e-9), plus an empty member (no
bricks).  Every tile variant, both launch modes and graph replay must give
chi bit for bit equal to one gw_contract_chi call per molecule: the tile
shapes change which wave computes an element, never the order of its K sum,
and stage C adds the pivots in the same order.  One member is checked
against the FP64 oracle (1e-12 relative)."""
import numpy as np
import pytest

from gpu_common import rel

pytestmark = pytest.mark.gpu


def _setup(ws):
    import torch
    from paper_2104_09857_amd import gw
    from gwinputs import configs
    out = []
    for w in ws:
        s = w.system
        C, eps = s.mean_field()
        g = configs.grids_for(w, eps)
        mu = configs.mu_fermi(eps, s.n_occ)
        trip = s.triples()
        t3c = torch.as_tensor(s.bricks(trip), device="cuda")
        sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, trip, t3c)
        do, dv = gw.build_gt(sysd, torch.as_tensor(C, device="cuda"), eps, mu, g.tau)
        out.append(dict(w=w, s=s, sys=sysd, t3c=t3c, trip=trip, do=do, dv=dv, C=C, eps=eps, mu=mu,
                        g=g))
    return out


@pytest.fixture(scope="module", params=["small", "production"])
def mols(request):
    from gwinputs import configs
    if request.param == "small":
        ws = configs.molecules(7, seed=3, lo=3, hi=9, filter_eps=1e-6, n_tau=4, n_ao=5, n_ri=12)
    else:
        ws = configs.molecules(5, seed=4, lo=4, hi=12, filter_eps=1e-9, n_tau=12)
    print("molecule set", request.param, [w.system.n_atoms for w in ws], flush=True)
    return request.param, _setup(ws)


def _singles(ms, prec):
    from paper_2104_09857_amd import gw
    return [gw.contract_chi(m["sys"], m["do"], m["dv"], m["s"].filter_eps, prec=prec)[0] for m in ms]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_batch_equals_single_calls(mols, prec):
    import torch
    from paper_2104_09857_amd import gw
    name, ms = mols
    eps_f = ms[0]["s"].filter_eps
    ref = _singles(ms, prec)
    plan = gw.ChiBatch([m["sys"] for m in ms], ms[0]["do"].shape[0], eps_f, prec=prec, timing=True)
    _, _, n_var = plan.config()
    do, dv = [m["do"] for m in ms], [m["dv"] for m in ms]
    for v in range(n_var):
        for pers in (0, 5, 7):
            print("case", name, prec, "variant", v, "persistent", pers, flush=True)
            plan.set_config(v, pers)
            out = plan.outputs()
            st = plan.execute(do, dv, out)
            torch.cuda.synchronize()
            for m, a, b in zip(ms, out, ref):
                assert torch.equal(a, b), (m["w"].name, v, pers)
            assert st["flops_c"] > 0 and st["ms_stage"][2] > 0
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_half_contraction_engines_agree(mols, prec):
    """The register-staged engine of stages A and B (gw_chi_batch_set_engine 1)
    and the direct-to-LDS one (the default where the rows allow it) take the
    same k values in the same order into every sum: chi bit for bit, switching
    back and forth on one plan."""
    import torch
    from paper_2104_09857_amd import gw
    name, ms = mols
    eps_f = ms[0]["s"].filter_eps
    plan = gw.ChiBatch([m["sys"] for m in ms], ms[0]["do"].shape[0], eps_f, prec=prec)
    do, dv = [m["do"] for m in ms], [m["dv"] for m in ms]
    ref = plan.outputs()
    plan.execute(do, dv, ref)
    for engine in (1, 0, 1):
        print("case", name, prec, "half-contraction engine", engine, flush=True)
        plan.set_engine(engine)
        out = plan.outputs()
        plan.execute(do, dv, out)
        torch.cuda.synchronize()
        for m, a, b in zip(ms, out, ref):
            assert torch.equal(a, b), (m["w"].name, engine)
    with pytest.raises(gw.GWError):
        plan.set_engine(2)
    plan.close()


def test_batch_vs_oracle(mols):
    import torch
    from paper_2104_09857_amd import gw
    from oracle import chi as ochi
    name, ms = mols
    m = min(ms, key=lambda x: x["s"].n_atoms)
    s = m["s"]
    print("case", name, m["w"].name, s.n_atoms, flush=True)
    plan = gw.ChiBatch([x["sys"] for x in ms], ms[0]["do"].shape[0], s.filter_eps)
    out = plan.outputs()
    plan.execute([x["do"] for x in ms], [x["dv"] for x in ms], out)
    got = out[ms.index(m)].cpu().numpy()
    t3 = ochi.dense_from_bricks(m["trip"], s.bricks(m["trip"]), s.ao_off, s.ri_off, s.n_ao, s.n_ri,
                                s.filter_eps)
    ref = ochi.chi_filtered(t3, m["do"].cpu().numpy(), m["dv"].cpu().numpy(), s.ao_off, s.ri_off,
                            s.filter_eps)
    assert rel(got, ref) < 1e-12
    plan.close()


def test_graph_replay(mols):
    import torch
    from paper_2104_09857_amd import gw
    name, ms = mols
    eps_f = ms[0]["s"].filter_eps
    n_tau = ms[0]["do"].shape[0]
    ref = _singles(ms, "fp64")
    stream = torch.cuda.Stream()
    plan = gw.ChiBatch([m["sys"] for m in ms], n_tau, eps_f, stream=stream)
    do, dv = [m["do"] for m in ms], [m["dv"] for m in ms]
    for pers in (7, 0):
        plan.set_config(0, pers)
        out = plan.outputs()
        for rep in range(3):
            print("case", name, "graph persistent", pers, "replay", rep, flush=True)
            for o in out:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                plan.execute(do, dv, out, graph=True, stats=False, stream=stream)
            stream.synchronize()
            for a, b in zip(out, ref):
                assert torch.equal(a, b)
            # eager work of the program between replays
            x = torch.randn(256, 256, device="cuda", dtype=torch.float64)
            (x @ x).sum().item()
        # new output pointers: captured again
        out2 = plan.outputs()
        with torch.cuda.stream(stream):
            plan.execute(do, dv, out2, graph=True, stats=False, stream=stream)
        stream.synchronize()
        for a, b in zip(out2, ref):
            assert torch.equal(a, b)
    plan.close()


def test_autotune_cache(mols, tmp_path):
    import torch
    from paper_2104_09857_amd import gw
    name, ms = mols
    eps_f = ms[0]["s"].filter_eps
    n_tau = ms[0]["do"].shape[0]
    cache = tmp_path / "tune.txt"
    do, dv = [m["do"] for m in ms], [m["dv"] for m in ms]
    plan = gw.ChiBatch([m["sys"] for m in ms], n_tau, eps_f)
    out = plan.outputs()
    ms1 = plan.tune(do, dv, out, reps=1, cache_path=cache)
    cfg = plan.config()
    lines = cache.read_text().splitlines()
    print("case", name, "tuned", cfg, ms1, lines, flush=True)
    assert len(lines) == 1 and ms1 > 0
    plan2 = gw.ChiBatch([m["sys"] for m in ms], n_tau, eps_f)
    ms2 = plan2.tune(do, dv, out, reps=1, cache_path=cache)
    assert plan2.config() == cfg and ms2 == pytest.approx(ms1, rel=1e-6)
    assert len(cache.read_text().splitlines()) == 1
    ref = _singles(ms, "fp64")
    plan2.execute(do, dv, out)
    for a, b in zip(out, ref):
        assert torch.equal(a, b)
    plan.close()
    plan2.close()


def test_empty_member():
    import torch
    from paper_2104_09857_amd import gw
    from gwinputs import configs
    ws = configs.molecules(3, seed=5, lo=3, hi=6, filter_eps=1e-6, n_tau=4, n_ao=5, n_ri=12)
    ms = _setup(ws)
    s = ms[1]["s"]
    empty = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, np.zeros((0, 3), np.int32), None)
    systems = [ms[0]["sys"], empty, ms[2]["sys"]]
    plan = gw.ChiBatch(systems, 4, 1e-6)
    out = plan.outputs()
    for o in out:
        o.fill_(1.0)
    print("case empty member", flush=True)
    plan.execute([m["do"] for m in ms], [m["dv"] for m in ms], out)
    assert float(out[1].abs().max()) == 0.0
    ref = _singles([ms[0], ms[2]], "fp64")
    assert torch.equal(out[0], ref[0]) and torch.equal(out[2], ref[1])
    plan.close()


def test_direct_to_lds_variant_needs_aligned_ri_blocks():
    """Variant 3 copies operands into LDS 16 bytes at a time: an FP64 plan
    with an odd RI count per atom rejects it and defaults to variant 2, and
    the default configuration of an FP32 plan with such a count falls back to
    variant 0."""
    import torch
    from paper_2104_09857_amd import gw
    from gwinputs import configs
    ws = configs.molecules(2, seed=6, lo=3, hi=5, filter_eps=1e-6, n_tau=2, n_ao=4, n_ri=13)
    ms = _setup(ws)
    plan = gw.ChiBatch([m["sys"] for m in ms], 2, 1e-6)
    assert plan.config()[0] == 2          # FP64 default without variant 3
    with pytest.raises(gw.GWError):
        plan.set_config(3, 7)
    plan.set_config(2, 7)
    out = plan.outputs()
    plan.execute([m["do"] for m in ms], [m["dv"] for m in ms], out)
    torch.cuda.synchronize()
    plan.close()
    p32 = gw.ChiBatch([m["sys"] for m in ms], 2, 1e-6, prec="fp32")
    assert p32.config()[0] == 0
    p32.close()
