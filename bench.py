"""Benchmark of the low-scaling GW hot path on one GPU.

Default mode: one step = one tau point of the hot path from device-resident
inputs: the density matrices D^occ(tau_j), D^vir(tau_j) (Eq. 2), the
block-sparse polarizability chi(tau_j) (Eq. 3, norms and filter included)
through a one-tau chi plan, and the correlation self-energy pieces of the
computed states at tau_j (Eqs. 10-11), j cycling over the tau grid.
`value` is the chi + Sigma contraction throughput over the timed steps
(algorithmic FLOPs of the executed block products / wall time of the
steps).  Before the steps the whole chain (Eqs. 2-12) runs once:
`time_to_qp_s`.  The dominant kernel (stage C of chi) is timed per launch
with HIP events on the library's stream (`roofline`); the FP64 oracle is
timed on the host cores on a bounded sample (`cpu_baseline`); the precision
forms run their whole chain next to it while the wall budget allows
(`precision_form`: speed-up and QP energy differences in meV).

Default workload strip300: 300-atom ribbon 7 atoms wide, 13 AO / 40 RI per
atom (3900 AO, 12000 RI), half filled, filter 1e-9, 12 tau / 12 omega points,
Sigma for HOMO-4 .. LUMO+4.  Inputs are seeded and synthetic (gwinputs).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload strip300]

--evgw SCALE times eigenvalue self-consistent GW on the workload instead,
its three-center tensor scaled by SCALE (e.g. --workload strip84 --evgw 0.02).

--open-shell DELTA times open-shell G0W0 instead: two spin channels of the
workload's mean field split by a spin-dependent potential of DELTA Ha per AO
(equal occupations, the broken-symmetry singlet), one chi per channel and one
W, next to the closed-shell chain on the same inputs (--t3c-scale scales the
three-center tensor, e.g. 0.02 for eV-sized shifts).

Workload bulk<n> (e.g. bulk5) is a periodic Gamma-point cell: n^3 atoms on
a simple cubic lattice, minimum-image distances, V of Gaussian RI charges by
gw_coulomb_periodic (timed in the setup and reported as periodic_coulomb).

--metric runs the default step with non-orthogonal bases: the Gaussian RI
overlap S (Eq. 5; W~^c and V~ in the self-energies) and MOs of a Gaussian
non-orthogonal AO basis.

Workload ribbon<N> (e.g. ribbon1734, 5 AO / 12 RI per atom, filter 1e-8)
measures the learned block screener: the network is trained on the GPU on
exact runs of ribbon300 and ribbon600, its safety band calibrated on
ribbon900, and chi of ribbon<N> is timed exact and screened in FP64, FP32
and BF16x3, with the skipped blocks audited against an exact run without
the output filter, and the QP energies of the screened FP32 and BF16x3
chains compared with the plain FP64 chain (value: plain FP64 chi time over
screened FP32 chi time).

Workload mol<M> (e.g. mol64) times the batched form instead: one step = one
execution of a gw_chi_batch plan (chi for all tau of M molecules of 10-40
atoms, captured in a hipGraph, tile variant and launch mode autotuned),
next to M one-system gw_contract_chi calls and the eager plan.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chi+Sigma contraction TFLOP/s & time-to-QP; mixed/learned vs FP64 at 1 meV"
# what the paper reports for this path (no contraction timing; its scaling
# figure and its largest run), printed beside the measurement
PAPER_CONTEXT = ("no timing of the chi or Sigma contraction is given; low-scaling G0W0 time "
                 "grows as N^2.1 on a Cray XC40 (CP2K/DBCSR, CPUs); the largest run, a 1734-atom "
                 "7-wide nanoribbon, used 14400 CPU cores")
PEAK_FP64_MFMA_TFLOPS = 78.6
# dense MFMA peaks of MI355X by operand type of the chi contraction
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
DTYPE = {"fp64": "f64", "fp32": "f32 (FP32 MFMA and accumulation in a tile, FP64 across pivots)",
         "bf16x3": "bf16x3 (bf16 hi/lo MFMA, FP32 accumulation in a tile, FP64 across pivots)"}
_C_TILES = {"fp64": ["4,2,5,32", "2,2,5,32", "4,2,5,16", "4,2,5,32,2"],
            "fp32": ["4,2,5,32", "2,2,5,32", "4,2,5,16", "4,2,5,16,3"],
            "bf16x3": ["4,2,4,5,32", "4,2,2,5,32", "2,2,4,5,32", "4,2,4,5,3,0"]}
_C_PROB = {"fp64": "StageC<double>", "fp32": "StageC<float>", "bf16x3": "StageCBf"}


def stage_c_kernel(prec, variant, mask, batched=False):
    """Name of the stage-C kernel a chi run launched (as rocprofv3 lists it);
    variant 3 is the direct-to-LDS engine (tile_dma; tile_bf3_dma in BF16x3)."""
    if prec == "bf16x3":
        eng = "tile_bf3_dma" if variant == 3 else "tile_bf16x3"
    else:
        eng = "tile_dma" if variant == 3 else "tile_gemm"
    prob = _C_PROB[prec]
    if mask & 4:
        return f"{eng}_persistent<{_C_TILES[prec][variant]},Batched<{prob}>>"
    return f"{eng}_kernel<{_C_TILES[prec][variant]},{'Batched<' + prob + '>' if batched else prob}>"


def measured_traffic(path, workload, kernel):
    """HBM bytes per launch of the stage-C kernel from the stored rocprofv3
    FETCH_SIZE / WRITE_SIZE runs, or None when there is no record for this
    workload and kernel or the kernel sources changed since it was taken."""
    import hashlib
    try:
        recs = json.load(open(path)).get(workload) or []
    except (OSError, ValueError):
        return None
    rec = next((r for r in recs if r.get("kernel") == kernel), None)
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(name, seed=0):
    import torch
    from gwinputs import configs, device as gdev
    from paper_2104_09857_amd import gw
    t0 = time.perf_counter()
    w = configs.by_name(name, seed)
    s = w.system
    C, eps = s.mean_field()
    g = configs.grids_for(w, eps)
    mu = configs.mu_fermi(eps, s.n_occ)
    trip = s.triples()
    log(f"[setup] {name}: {s.n_atoms} atoms, {s.n_ao} AO, {s.n_ri} RI, {len(trip)} triples, "
        f"host prep {time.perf_counter() - t0:.1f} s")
    t3c = gdev.bricks_on_device(s, trip)
    coulomb = None
    if s.cell is None:
        V = torch.as_tensor(s.coulomb(), device="cuda")
    else:
        # periodic cell: V of the Gaussian RI charges by the library's Ewald sum
        R, alpha = s.ri_charges()
        gw.coulomb_periodic(R, alpha, s.cell)       # untimed first call
        torch.cuda.synchronize()
        tc = time.perf_counter()
        V, info = gw.coulomb_periodic(R, alpha, s.cell)
        torch.cuda.synchronize()
        coulomb = dict(ms=(time.perf_counter() - tc) * 1e3, cell=[float(x) for x in s.cell], **info)
        log(f"[setup] periodic V by Ewald summation {coulomb['ms']:.1f} ms {info}")
        # V alone for the 512-atom cell (8^3 atoms, 10240 RI charges)
        from gwinputs import configs
        big = configs.bulk(8, n_ao=s.n_ao_atom, n_ri=s.n_ri_atom).system
        Rb, ab = big.ri_charges()
        gw.coulomb_periodic(Rb, ab, big.cell)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        Vb, infob = gw.coulomb_periodic(Rb, ab, big.cell)
        torch.cuda.synchronize()
        coulomb["bulk8_V_only"] = dict(ms=(time.perf_counter() - tc) * 1e3, n_ri=len(ab), **infob)
        log(f"[setup] bulk8 V {coulomb['bulk8_V_only']}")
        del Vb
    Cd = torch.as_tensor(C, device="cuda")
    torch.cuda.synchronize()
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, trip, t3c, s.xyz)
    log(f"[setup] device inputs ready ({t3c.numel() * 8 / 1e9:.1f} GB bricks), "
        f"{time.perf_counter() - t0:.1f} s")
    return dict(w=w, s=s, C=C, eps=eps, g=g, mu=mu, trip=trip, sys=sysd, Cd=Cd, V=V, t3c=t3c,
                coulomb=coulomb)


def use_metric(ctx):
    """Non-orthogonal bases: the Gaussian RI overlap (Eq. 5) on the device
    and the MOs of H C = S_ao C eps with the Gaussian AO overlap."""
    import torch
    from gwinputs import configs
    s = ctx["s"]
    C, eps = s.mean_field_nonorth(s.ao_metric())
    ctx.update(C=C, eps=eps, Cd=torch.as_tensor(C, device="cuda"), mu=configs.mu_fermi(eps, s.n_occ),
               S_ri=torch.as_tensor(s.ri_metric(), device="cuda"))
    torch.cuda.synchronize()


def step(ctx, prec="fp64"):
    from paper_2104_09857_amd import pipeline
    g = ctx["g"]
    return pipeline.g0w0(ctx["sys"], ctx["Cd"], ctx["eps"], ctx["mu"], ctx["V"], g.tau, g.omega,
                         g.cos_w, g.sin_w, g.icos_w, ctx["w"].states(), ctx["s"].filter_eps,
                         events=True, chi_timing=True, prec=prec, S_ri=ctx.get("S_ri"))


def bench_evgw(args):
    """Eigenvalue self-consistent GW (the paper's step after Eq. 12) on the
    workload with its three-center tensor scaled by args.evgw (the synthetic
    tensor gives keV self-energy shifts, for which feeding the energies back
    is meaningless): time-to-QP of the whole evGW loop after one untimed G0W0
    chain."""
    import torch
    from paper_2104_09857_amd import pipeline
    ctx = setup(args.workload)
    ctx["t3c"].mul_(args.evgw)
    torch.cuda.synchronize()
    g, s, states = ctx["g"], ctx["s"], ctx["w"].states()
    t0 = time.perf_counter()
    step(ctx, args.prec)
    torch.cuda.synchronize()
    log(f"[evgw] warm-up G0W0 chain {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    out = pipeline.evgw(ctx["sys"], ctx["Cd"], ctx["eps"], ctx["mu"], ctx["V"], g.tau, g.omega,
                        g.cos_w, g.sin_w, g.icos_w, states, s.filter_eps, tol=1e-6, max_iter=20,
                        prec=args.prec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hist = out["history"]
    ha_ev = 27.211386245988
    homo, lumo = list(states).index(s.n_occ - 1), list(states).index(s.n_occ)
    log(f"[evgw] {out['steps']} steps, converged {out['converged']}, {wall:.1f} s")
    res = {
        "metric": METRIC, "value": wall, "unit": "s (evGW time-to-QP)", "n_gpus": 1,
        "steps": out["steps"], "warmup": 1, "ms_per_step": wall * 1e3 / out["steps"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "paper_context": PAPER_CONTEXT, "dtype": DTYPE[args.prec], "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": s.n_atoms, "n_ao": s.n_ao, "n_ri": s.n_ri,
                   "filter_eps": s.filter_eps, "n_tau": ctx["w"].n_tau, "t3c_scale": args.evgw},
        "evgw": {"converged": bool(out["converged"]), "steps": out["steps"],
                 "shift_eV_g0w0": [round(float(x), 4) for x in (hist[0] - ctx["eps"][states]) * ha_ev],
                 "evgw_minus_g0w0_meV": [round(float(x), 3) for x in (hist[-1] - hist[0]) * ha_ev * 1e3],
                 "gap_eV_g0w0": float((hist[0][lumo] - hist[0][homo]) * ha_ev),
                 "gap_eV_evgw": float((hist[-1][lumo] - hist[-1][homo]) * ha_ev),
                 "max_change_meV_per_step": [float(np.abs(hist[i] - hist[i - 1]).max() * ha_ev * 1e3)
                                             for i in range(1, len(hist))]},
    }
    print(json.dumps(res), flush=True)


def bench_open_shell(args):
    """Open-shell G0W0 (see the module docstring): time-to-QP per step of
    pipeline.g0w0_spin after one untimed chain, and of one closed-shell chain
    on the same inputs."""
    import torch
    from paper_2104_09857_amd import gw, pipeline
    ctx = setup(args.workload)
    ctx["t3c"].mul_(args.t3c_scale)
    g, s, states = ctx["g"], ctx["s"], ctx["w"].states()
    up, dn = s.mean_field_spin(args.open_shell)
    cu = torch.as_tensor(up[0], device="cuda")
    cd = torch.as_tensor(dn[0], device="cuda")
    sys_dn = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, ctx["trip"], ctx["t3c"], s.xyz)
    torch.cuda.synchronize()

    def spin_step():
        return pipeline.g0w0_spin(ctx["sys"], sys_dn, cu, cd, up[1], dn[1], ctx["V"], g.tau, g.omega,
                                  g.cos_w, g.sin_w, g.icos_w, states, states, s.filter_eps,
                                  prec=args.prec)

    t0 = time.perf_counter()
    spin_step()
    torch.cuda.synchronize()
    log(f"[open-shell] warm-up {time.perf_counter() - t0:.1f} s")
    walls = []
    for i in range(args.steps):
        t0 = time.perf_counter()
        out = spin_step()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        log(f"[open-shell] step {i} {walls[-1]:.2f} s")
    t0 = time.perf_counter()
    closed = step(ctx, args.prec)
    torch.cuda.synchronize()
    closed_s = time.perf_counter() - t0
    log(f"[open-shell] closed-shell chain {closed_s:.2f} s")
    ha_ev = 27.211386245988
    wall = float(np.mean(walls))
    res = {
        "metric": METRIC, "value": wall, "unit": "s (open-shell G0W0 time-to-QP)", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": wall * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "paper_context": PAPER_CONTEXT, "dtype": DTYPE[args.prec], "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": s.n_atoms, "n_ao": s.n_ao, "n_ri": s.n_ri,
                   "filter_eps": s.filter_eps, "n_tau": ctx["w"].n_tau, "spin_delta": args.open_shell,
                   "t3c_scale": args.t3c_scale},
        "open_shell": {
            "closed_shell_s": closed_s, "ratio_to_closed_shell": wall / closed_s,
            "status_ok": bool(np.all(out["status_up"] == 0) and np.all(out["status_dn"] == 0)),
            "shift_eV_up": [round(float(x), 4) for x in (out["e_qp_up"] - up[1][states]) * ha_ev],
            "shift_eV_dn": [round(float(x), 4) for x in (out["e_qp_dn"] - dn[1][states]) * ha_ev],
            "shift_eV_closed": [round(float(x), 4)
                                for x in (closed["e_qp"] - ctx["eps"][states]) * ha_ev]},
    }
    print(json.dumps(res), flush=True)


def host_facts():
    """CPU model, logical CPU count and the threads the oracle's BLAS may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", ncpu))
    return {"cpu_model": model, "nproc": ncpu, "blas_threads": min(threads, ncpu)}


def cpu_baseline(ctx, d_occ0, d_vir0, chi_sigma_flops, sample_s=6.0, reps=3):
    """The oracle (FP64 NumPy, host BLAS) timed on the host cores.

    value: its throughput on a bounded sample of the same workload, output
    blocks chi_{cc'}(tau_0) contracted by the oracle's block routine from the
    same bricks and D(tau_0), median of `reps` runs of about `sample_s` s each;
    the strip's whole chi + Sigma contraction at that rate is reported as
    extrapolated.  full_chain_chain12: the oracle's whole chain (Eqs. 2-12)
    on the 12-atom chain, median of `reps`."""
    from oracle import chi as ochi, chain as ochain
    from gwinputs import configs
    s = ctx["s"]
    d_occ = d_occ0.cpu().numpy()
    d_vir = d_vir0.cpu().numpy()
    trip = ctx["trip"]
    rng = np.random.default_rng(0)
    mid = s.n_atoms // 2
    pairs = [(mid, mid), (mid, min(mid + 9, s.n_atoms - 1))] + \
        [tuple(sorted(rng.integers(0, s.n_atoms, 2))) for _ in range(60)]
    cache = {}
    loaded = set()

    def load(c):
        rows = np.nonzero(trip[:, 2] == c)[0]
        vals = ctx["t3c"][rows].cpu().numpy()
        for r, v in zip(rows, vals):
            cache[tuple(trip[r])] = v.reshape(s.n_ao_atom, s.n_ao_atom, s.n_ri_atom)

    nr = s.n_ri_atom

    def block_flops(c, c2):
        n_lam = len({t[0] for t in trip[trip[:, 2] == c]}) * s.n_ao_atom
        n_mu = len({t[0] for t in trip[trip[:, 2] == c2]}) * s.n_ao_atom
        # M: mu x lambda x (sigma P); N: mu x nu x (Q sigma); chi: P x Q x (mu sigma)
        return (2.0 * n_mu * n_lam * n_lam * nr + 2.0 * n_mu * n_mu * nr * n_lam
                + 2.0 * nr * nr * n_mu * n_lam)

    rates, samples = [], []
    for rep in range(reps):
        flops = elapsed = 0.0
        done = []
        for (c, c2) in pairs:
            for cc in (c, c2):
                if cc not in loaded:
                    load(cc)
                    loaded.add(cc)
            t0 = time.perf_counter()
            ochi.chi_block(c, c2, trip, lambda a, b, cc: cache[(a, b, cc)], d_occ, d_vir, s.ao_off,
                           s.ri_off, s.filter_eps)
            elapsed += time.perf_counter() - t0
            flops += block_flops(c, c2)
            done.append((int(c), int(c2)))
            if elapsed > sample_s:
                break
        rates.append(flops / elapsed)
        samples.append(len(done))
    rate = float(np.median(rates))
    # the oracle's whole chain on the 12-atom chain
    w = configs.chain12()
    cs = w.system
    C, eps = cs.mean_field()
    g = configs.grids_for(w, eps)
    tr = cs.triples()
    dense = ochi.dense_from_bricks(tr, cs.bricks(tr), cs.ao_off, cs.ri_off, cs.n_ao, cs.n_ri,
                                   cs.filter_eps)
    Vc = cs.coulomb()
    walls = []
    for rep in range(reps):
        t0 = time.perf_counter()
        ochain.g0w0(C, eps, cs.n_occ, dense, Vc, cs.ao_off, cs.ri_off, g, w.states(), cs.filter_eps)
        walls.append(time.perf_counter() - t0)
    facts = host_facts()
    return {"value": rate / 1e12, "unit": "TFLOP/s", "cores": facts["blas_threads"],
            "kind": "oracle",
            "sample": f"chi blocks (c, c') at tau_0 of {ctx['w'].name} contracted by the oracle's "
                      f"block routine (FP64 NumPy, host BLAS) from the same bricks and D(tau_0); "
                      f"median of {reps} runs of {samples} blocks (~{sample_s:.0f} s each)",
            "rates_tflops": [r / 1e12 for r in rates],
            "extrapolated_chi_sigma_s": chi_sigma_flops / rate,
            "extrapolated_note": "whole chi + Sigma contraction of the workload (all tau) at the "
                                 "sampled rate: extrapolated, not run",
            "full_chain_chain12_s": float(np.median(walls)),
            "full_chain_chain12_runs_s": walls, **facts}


def setup_molecules(name, seed=0):
    import torch
    from gwinputs import configs, device as gdev
    from paper_2104_09857_amd import gw
    t0 = time.perf_counter()
    ws = configs.molecule_set(name, seed)
    ms = []
    for w in ws:
        s = w.system
        C, eps = s.mean_field()
        g = configs.grids_for(w, eps)
        mu = configs.mu_fermi(eps, s.n_occ)
        trip = s.triples()
        t3c = gdev.bricks_on_device(s, trip)
        sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, trip, t3c, s.xyz)
        do, dv = gw.build_gt(sysd, torch.as_tensor(C, device="cuda"), eps, mu, g.tau)
        ms.append(dict(w=w, s=s, sys=sysd, t3c=t3c, trip=trip, do=do, dv=dv))
    torch.cuda.synchronize()
    n = [m["s"].n_atoms for m in ms]
    log(f"[setup] {name}: atoms {min(n)}..{max(n)} (sum {sum(n)}), "
        f"{sum(m['t3c'].numel() for m in ms) * 8 / 1e9:.1f} GB bricks, {time.perf_counter() - t0:.1f} s")
    return ms


def bench_batched(args):
    """The batched form on M molecules (see the module docstring)."""
    import tempfile
    import torch
    from paper_2104_09857_amd import gw
    ms = setup_molecules(args.workload)
    n_mol = len(ms)
    eps_f = ms[0]["s"].filter_eps
    n_tau = ms[0]["do"].shape[0]
    systems = [m["sys"] for m in ms]
    do, dv = [m["do"] for m in ms], [m["dv"] for m in ms]
    stream = torch.cuda.Stream()

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    # reference: one gw_contract_chi call per molecule
    ref = [gw.contract_chi(m["sys"], m["do"], m["dv"], eps_f, prec=args.prec)[0] for m in ms]
    seq_ms = timed(lambda: [gw.contract_chi(m["sys"], m["do"], m["dv"], eps_f, chi=r, prec=args.prec)
                            for m, r in zip(ms, ref)], 1)
    log(f"[batched] sequential one-system calls: {seq_ms:.1f} ms")
    # one-system plans (made beforehand), executed one after another
    singles = [gw.ChiBatch([m["sys"]], n_tau, eps_f, prec=args.prec, stream=stream) for m in ms]

    def run_singles():
        with torch.cuda.stream(stream):
            for p1, m, r in zip(singles, ms, ref):
                p1.execute([m["do"]], [m["dv"]], [r], stats=False, stream=stream)

    run_singles()
    seq_plan_ms = timed(run_singles, 1)
    for p1 in singles:
        p1.close()
    del singles
    log(f"[batched] sequential one-system plans: {seq_plan_ms:.1f} ms")
    plan = gw.ChiBatch(systems, n_tau, eps_f, prec=args.prec, timing=True, stream=stream)
    out = plan.outputs()
    # eager, default configuration, per-stage events
    with torch.cuda.stream(stream):
        st = plan.execute(do, dv, out, stream=stream)
    stream.synchronize()
    eager_ms = st["ms_total"]
    same = all(torch.equal(a, b) for a, b in zip(out, ref))
    cache = args.tune_cache or os.path.join(tempfile.mkdtemp(), "gw_autotune.txt")
    with torch.cuda.stream(stream):
        tune_ms = plan.tune(do, dv, out, reps=1, cache_path=cache, stream=stream)
    variant, persistent, _ = plan.config()
    log(f"[batched] eager default {eager_ms:.1f} ms, tuned variant {variant} persistent {persistent} "
        f"{tune_ms:.1f} ms")
    # per-stage times of the tuned configuration (eager)
    with torch.cuda.stream(stream):
        st = plan.execute(do, dv, out, stream=stream)
    stream.synchronize()

    def run_graph():
        with torch.cuda.stream(stream):
            plan.execute(do, dv, out, graph=True, stats=False, stream=stream)

    for i in range(args.warmup):
        run_graph()
        stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        run_graph()
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph_ms = wall / args.steps * 1e3
    same_graph = all(torch.equal(a, b) for a, b in zip(out, ref))
    flops = st["flops_ab"] + st["flops_c"]
    c_ms, c_n, c_fl = st["ms_stage"][2], st["n_launch"][2], st["flops_stage"][2]
    achieved = (c_fl / max(c_n, 1)) / ((c_ms / max(c_n, 1)) / 1e3) / 1e12
    peak = PEAK[args.prec]
    n = [m["s"].n_atoms for m in ms]
    res = {
        "metric": METRIC, "value": flops / (graph_ms / 1e3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": graph_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "paper_context": PAPER_CONTEXT,
        "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "form": "batched chi (gw_chi_batch, hipGraph)",
                   "n_mol": n_mol, "atoms_min": min(n), "atoms_max": max(n), "atoms_sum": sum(n),
                   "n_tau": n_tau, "filter_eps": eps_f, "ao_per_atom": 13, "ri_per_atom": 40},
        "batched": {"sequential_calls_ms": seq_ms, "sequential_plans_ms": seq_plan_ms,
                    "eager_default_ms": eager_ms, "tuned_ms": tune_ms,
                    "graph_ms": graph_ms, "speedup_vs_sequential_calls": seq_ms / graph_ms,
                    "speedup_vs_sequential_plans": seq_plan_ms / graph_ms,
                    "tuned_variant": variant, "tuned_persistent": persistent,
                    "equal_to_single_calls": bool(same and same_graph),
                    "flops": flops, "stage_ms": [round(x, 2) for x in st["ms_stage"]],
                    "stage_launches": list(st["n_launch"])},
        "roofline": {"kernel": stage_c_kernel(args.prec, st["c_variant"], st["launch_mask"], True)
                               + " (chi outer contraction, batched)", "bound": "mfma",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None, "launches": int(c_n), "avg_launch_ms": c_ms / max(c_n, 1)},
    }
    plan.close()
    print(json.dumps(res), flush=True)


def bench_screened(args):
    """The learned block screener on a long ribbon (see the module docstring)."""
    import torch
    from gwinputs import configs, device as gdev
    from paper_2104_09857_amd import gw, pipeline, screener

    def prepare(name):
        w = configs.by_name(name)
        s = w.system
        C, eps = s.mean_field()
        g = configs.grids_for(w, eps)
        mu = configs.mu_fermi(eps, s.n_occ)
        trip = s.triples()
        t3c = gdev.bricks_on_device(s, trip)
        sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, trip, t3c, s.xyz)
        Cd = torch.as_tensor(C, device="cuda")
        do, dv = gw.build_gt(sysd, Cd, eps, mu, g.tau)
        return dict(w=w, s=s, C=C, Cd=Cd, eps=eps, g=g, mu=mu, sys=sysd, do=do, dv=dv)

    def timed_chi(m, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chi, st = gw.contract_chi(m["sys"], m["do"], m["dv"], m["s"].filter_eps, tau=m["g"].tau, **kw)
        torch.cuda.synchronize()
        return chi, st, (time.perf_counter() - t0) * 1e3

    t_all = time.perf_counter()
    Xs, ts = [], []
    # targets: block norms of the exact contraction without the output filter
    # (continuous through the threshold, unlike the filtered output)
    for name in ("ribbon300", "ribbon600"):
        m = prepare(name)
        chi, _, ms = timed_chi(m, keep_small_blocks=True)
        X, t = screener.samples(m["sys"], m["do"], m["dv"], chi, m["g"].tau, m["s"].filter_eps)
        Xs.append(X)
        ts.append(t)
        log(f"[screen] training data {name}: {X.shape[0]} blocks, exact chi {ms:.0f} ms")
        del chi, m
    eps_f = configs.by_name("ribbon300").system.filter_eps
    sc = screener.BlockScreener(11)
    t0 = time.perf_counter()
    hist = sc.fit(torch.cat(Xs), torch.cat(ts), filter_eps=eps_f, steps=3000, batch=4096, lr=2e-3,
                  alpha=8.0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del Xs, ts
    mv = prepare("ribbon900")
    chi, _, _ = timed_chi(mv, keep_small_blocks=True)
    Xv, tv = screener.samples(mv["sys"], mv["do"], mv["dv"], chi, mv["g"].tau, eps_f)
    margin = sc.calibrate(Xv, tv, eps_f)
    del chi, mv, Xv, tv
    log(f"[screen] trained {train_s:.1f} s (loss {hist[0][1]:.3g} -> {hist[-1][1]:.3g}), "
        f"band {margin:.2f} decades")

    m = prepare(args.workload)
    s = m["s"]
    log(f"[screen] {args.workload} ready ({s.n_atoms} atoms)")
    res = {}
    ref_unf, _, ms_ref = timed_chi(m, keep_small_blocks=True)     # exact, nothing zeroed (warms up)
    lg_ref = gw.chi_block_lognorms(m["sys"], ref_unf)
    del ref_unf
    log(f"[screen] exact unfiltered chi {ms_ref:.0f} ms")
    # audit: the keep mask depends on the features only, so one screened run
    # without the output filter shows every skipped block for all precisions
    scr_unf, _, _ = timed_chi(m, screener=sc.net, screen_margin=margin, keep_small_blocks=True)
    lg_s = gw.chi_block_lognorms(m["sys"], scr_unf)
    del scr_unf
    skipped = (lg_s < -29) & (lg_ref >= -29)
    blk = torch.pow(10.0, lg_ref.double())                           # exact block norms
    audit = {"blocks_skipped_nonzero": int(skipped.sum()),
             "max_skipped_log10_norm": float(lg_ref[skipped].max()) if bool(skipped.any()) else None,
             "skipped_mass_rel": float(torch.sqrt((blk[skipped] ** 2).sum()) / torch.sqrt((blk ** 2).sum()))}
    del lg_s, blk, skipped
    log(f"[screen] audit {audit}")
    for prec in ("fp64", "fp32", "bf16x3"):
        exact, st_e, ms_e = timed_chi(m, prec=prec, timing=True)
        log(f"[screen] {prec} exact {ms_e:.0f} ms")
        scr, st_s, ms_s = timed_chi(m, prec=prec, timing=True, screener=sc.net, screen_margin=margin)
        log(f"[screen] {prec} screened {ms_s:.0f} ms")
        same = bool(torch.equal(scr, exact))
        del exact, scr
        res[prec] = {"chi_ms_exact": ms_e, "chi_ms_screened": ms_s,
                     "stage_ms_exact": st_e["ms_stage"], "stage_ms_screened": st_s["ms_stage"],
                     "flops_c_exact": st_e["flops_c"], "flops_c_screened": st_s["flops_c"],
                     "blocks_screened": int(st_s["n_blocks_screened"]),
                     "blocks_total": int(s.n_atoms * (s.n_atoms + 1) // 2 * m["w"].n_tau),
                     "tiles_screened": int(st_s["n_tiles_screened"]),
                     "equal_to_exact": same}
        torch.cuda.empty_cache()
    # QP: plain FP64 chain vs the screened FP32 and BF16x3 chains
    V = torch.as_tensor(s.coulomb(), device="cuda")
    g = m["g"]
    a = (m["sys"], m["Cd"], m["eps"], m["mu"], V, g.tau, g.omega, g.cos_w, g.sin_w, g.icos_w,
         m["w"].states(), s.filter_eps)
    o64 = pipeline.g0w0(*a, events=True)
    o64 = {k: o64[k] for k in ("e_qp", "status", "ms")}
    log(f"[screen] FP64 chain {sum(o64['ms'].values()) / 1e3:.1f} s")
    shift = np.abs(o64["e_qp"] - m["eps"][m["w"].states()]) * 27211.386245988
    qp = {"shift_meV_fp64": [round(float(x), 1) for x in shift],
          "status_fp64": [int(x) for x in o64["status"]],
          "time_to_qp_s_fp64": sum(o64["ms"].values()) / 1e3}
    for prec in ("fp32", "bf16x3"):
        torch.cuda.empty_cache()
        omx = pipeline.g0w0(*a, events=True, prec=prec, screener=sc.net, screen_margin=margin)
        log(f"[screen] {prec} + screener chain {sum(omx['ms'].values()) / 1e3:.1f} s")
        ok = (o64["status"] == 0) & (omx["status"] == 0)
        de = np.where(ok, np.abs(omx["e_qp"] - o64["e_qp"]) * 27211.386245988, np.nan)
        qp[prec + "_screened"] = {
            "dE_meV_vs_fp64": [round(float(x), 4) for x in de],
            "max_abs_dE_meV": float(np.nanmax(de)) if ok.any() else None,
            "max_dE_over_shift": float(np.nanmax(de / np.maximum(shift, 1e-30))) if ok.any() else None,
            "status": [int(x) for x in omx["status"]],
            "time_to_qp_s": sum(omx["ms"].values()) / 1e3}
    f64, fmx = res["fp64"], res["fp32"]
    out = {
        "metric": METRIC, "value": f64["chi_ms_exact"] / fmx["chi_ms_screened"],
        "unit": "x (chi time, plain FP64 / FP32 + learned screener)", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": fmx["chi_ms_screened"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "paper_context": PAPER_CONTEXT, "dtype": "f32 + fp64 reference", "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": s.n_atoms, "n_ao": s.n_ao, "n_ri": s.n_ri,
                   "filter_eps": s.filter_eps, "n_tau": m["w"].n_tau,
                   "train": ["ribbon300", "ribbon600"], "calibrate": "ribbon900"},
        "screener": {"band_decades": margin, "train_s": train_s, "loss_first_last": [hist[0][1], hist[-1][1]]},
        "audit": audit,
        "chi": res,
        "speedup_vs_fp64_exact": {p + sfx: f64["chi_ms_exact"] / res[p]["chi_ms_" + key]
                                  for p in res for sfx, key in (("", "exact"), ("_screened", "screened"))},
        "qp": qp,
        "wall_s": time.perf_counter() - t_all,
    }
    print(json.dumps(out), flush=True)


def full_chain(ctx, prec):
    """Time-to-QP: the whole chain once from device-resident inputs (a1 -> a10
    of the hot path: the library's chain, chi for all tau in one call)."""
    import torch
    out = step(ctx, prec)
    torch.cuda.synchronize()
    out["wall_s"] = sum(out["ms"].values()) / 1e3
    return out


def bench_chain(args):
    """Default mode: one step = one tau point of the hot path (Eq. 2 for tau_j,
    Eq. 3 through a one-tau plan, Eqs. 10-11 for tau_j), cycling over the
    grid; the whole chain (time-to-QP) runs once before the steps."""
    import torch
    from paper_2104_09857_amd import gw
    t_start = time.perf_counter()
    ctx = setup(args.workload)
    if args.metric:
        use_metric(ctx)
    s, g, w = ctx["s"], ctx["g"], ctx["w"]
    sysd, Cd, eps, mu = ctx["sys"], ctx["Cd"], ctx["eps"], ctx["mu"]
    states = w.states()
    n_tau = len(g.tau)
    chain = full_chain(ctx, args.prec)
    log(f"[chain] time-to-QP {chain['wall_s']:.2f} s " +
        json.dumps({k: round(v, 1) for k, v in chain["ms"].items()}))
    for k in ("chi", "d_occ", "d_vir"):
        chain.pop(k)
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    plan = gw.ChiBatch([sysd], 1, s.filter_eps, prec=args.prec, timing=True)
    if args.c_variant is not None:
        plan.set_config(args.c_variant, plan.config()[1])
    plan_s = time.perf_counter() - t0
    log(f"[plan] one-tau {args.prec} plan {plan_s:.1f} s")
    wc = chain["wc"]
    do1 = torch.empty((1, s.n_ao, s.n_ao), dtype=torch.float64, device="cuda")
    dv1 = torch.empty_like(do1)
    chi1 = torch.empty((1, s.n_ri, s.n_ri), dtype=torch.float64, device="cuda")

    def tau_step(j):
        gw.build_gt(sysd, Cd, eps, mu, g.tau[j:j + 1], d_occ=do1, d_vir=dv1)
        st = plan.execute([do1], [dv1], [chi1])
        _, _, _, sst = gw.contract_sigma(sysd, states, Cd, do1, dv1, None, wc[j:j + 1], None,
                                         s.filter_eps)
        return st, sst

    for i in range(args.warmup):
        ts = time.perf_counter()
        tau_step(i % n_tau)
        torch.cuda.synchronize()
        log(f"[warmup {i}] tau_{i % n_tau} {time.perf_counter() - ts:.2f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flops = c_ms = c_fl = 0.0
    c_n = 0
    stage_ms = np.zeros(3)
    stage_fl = np.zeros(3)
    for i in range(args.steps):
        ts = time.perf_counter()
        st, sst = tau_step((args.warmup + i) % n_tau)
        flops += st["flops_ab"] + st["flops_c"] + sst["flops"]
        stage_ms += st["ms_stage"]
        stage_fl += st["flops_stage"]
        c_ms += st["ms_stage"][2]
        c_n += st["n_launch"][2]
        c_fl += st["flops_stage"][2]
        log(f"[step {i}] tau_{(args.warmup + i) % n_tau} {time.perf_counter() - ts:.2f} s "
            f"stages(ms) {[round(x, 1) for x in st['ms_stage']]}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = flops / wall / 1e12
    # dominant kernel: the outer contraction (stage C), timed per launch with
    # HIP events on the library's stream
    per_launch_ms = c_ms / max(c_n, 1)
    achieved = (c_fl / max(c_n, 1)) / (per_launch_ms / 1e3) / 1e12
    cs = chain["chi_stats"]
    # the kernel of the timed launches: the one-tau plan's (its variant may be set)
    c_kernel = stage_c_kernel(args.prec, st["c_variant"], st["launch_mask"], batched=True)
    traffic = measured_traffic(args.traffic_json, args.workload + ":tau1", c_kernel)
    chain_flops = cs["flops_ab"] + cs["flops_c"] + chain["sig_stats"]["flops"]
    res = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "paper_context": PAPER_CONTEXT,
        "dtype": DTYPE[args.prec], "data": "synthetic",
        "config": {"workload": args.workload, "step": "one tau point: build_gt, chi (one-tau plan), "
                   "Sigma (correlation part) for tau_j, j cycling over the grid",
                   "n_atoms": s.n_atoms, "n_ao": s.n_ao, "n_ri": s.n_ri,
                   "n_occ": s.n_occ, "n_tau": n_tau, "filter_eps": s.filter_eps,
                   "n_gw": len(states), "n_trip": int(len(ctx["trip"])),
                   "n_trip_kept": int(cs["n_trip_kept"]),
                   "bases": "non-orthogonal (Gaussian RI and AO overlaps)" if args.metric
                   else "orthonormal"},
        "time_to_qp_s": chain["wall_s"],
        "chain_stage_ms": {k: round(v, 1) for k, v in chain["ms"].items()},
        "chain_chi_sigma_tflops": chain_flops / ((chain["ms"]["chi"] + chain["ms"]["sigma"]) / 1e3) / 1e12,
        "chain_flops": {"chi_ab": cs["flops_ab"], "chi_c": cs["flops_c"],
                        "sigma": chain["sig_stats"]["flops"]},
        "chain_chi_stage_ms": [round(x, 1) for x in cs["ms_stage"]],
        "step_chi_stage": {"names": ["A (D^occ half)", "B (D^vir half)", "C (outer)"],
                           "ms_per_step": [round(x / args.steps, 1) for x in stage_ms],
                           "tflops": [f / (m / 1e3) / 1e12 if m > 0 else None
                                      for f, m in zip(stage_fl, stage_ms)]},
        "e_qp": [float(x) for x in chain["e_qp"]],
        "qp_status": [int(x) for x in chain["status"]],
        "roofline": {"kernel": c_kernel + " (chi outer contraction)",
                     "bound": "mfma", "achieved": achieved, "peak": PEAK[args.prec],
                     "unit": "TFLOP/s", "frac": achieved / PEAK[args.prec],
                     "traffic": traffic, "launches": int(c_n), "avg_launch_ms": per_launch_ms,
                     "flops_per_launch": c_fl / max(c_n, 1)},
        "before_steps_s": t0 - t_start,
    }
    log(f"[bench] {value:.2f} TFLOP/s, stage C {achieved:.2f} TFLOP/s, "
        f"{time.perf_counter() - t_start:.0f} s so far")
    if not args.no_cpu_baseline:
        t1 = time.perf_counter()
        do0, dv0 = gw.build_gt(sysd, Cd, eps, mu, g.tau[:1])
        res["cpu_baseline"] = cpu_baseline(ctx, do0[0], dv0[0], chain_flops)
        del do0, dv0
        log(f"[cpu] oracle {res['cpu_baseline']['value']:.4f} TFLOP/s ({time.perf_counter() - t1:.0f} s)")
    # precision forms next to the FP64 chain, within the wall budget
    others = [] if args.no_compare or args.compare == "none" else \
        [x for x in args.compare.split(",") if x and x != args.prec]
    forms = {}
    plan.close()
    del chi1, do1, dv1
    del tau_step, wc
    chain.pop("wc")
    for other in others:
        used = time.perf_counter() - t_start
        if used > args.wall_budget:
            forms[other] = {"skipped": f"wall budget ({used:.0f} s used of {args.wall_budget:.0f} s)"}
            continue
        torch.cuda.empty_cache()
        o2 = full_chain(ctx, other)
        log(f"[{other}] chain {o2['wall_s']:.2f} s " +
            json.dumps({k: round(v, 1) for k, v in o2["ms"].items()}))
        c2 = o2["chi_stats"]
        pf = {"chi_ms": o2["ms"]["chi"], "time_to_qp_s": o2["wall_s"],
              "chi_tflops": (c2["flops_ab"] + c2["flops_c"]) / (o2["ms"]["chi"] / 1e3) / 1e12,
              "stage_ms": [round(x, 1) for x in c2["ms_stage"]],
              "chi_speedup_vs_" + args.prec: chain["ms"]["chi"] / o2["ms"]["chi"]}
        ok = (chain["status"] == 0) & (o2["status"] == 0)
        de = np.abs(o2["e_qp"] - chain["e_qp"]) * 27211.386245988
        pf.update({"dE_meV_vs_" + args.prec: [round(float(x), 4) if k else None
                                              for x, k in zip(de, ok)],
                   "max_abs_dE_meV": float(de[ok].max()) if ok.any() else None,
                   "states_within_1meV": int((de[ok] <= 1.0).sum()),
                   "states_compared": int(ok.sum()),
                   "status": [int(x) for x in o2["status"]]})
        forms[other] = pf
        del o2
        torch.cuda.empty_cache()
    if forms:
        res["precision_form"] = forms
    res["wall_s"] = time.perf_counter() - t_start
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="strip300")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the timed chi contraction")
    ap.add_argument("--compare", default="fp32,bf16x3",
                    help="comma list of arithmetics run (untimed) next to the main one, or none")
    ap.add_argument("--no-compare", action="store_true", help="same as --compare none")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--tune-cache", default=None, help="autotune cache file of the batched form")
    ap.add_argument("--c-variant", type=int, default=None,
                    help="stage-C tile variant of the one-tau plan of the steps (default: the plan's)")
    ap.add_argument("--evgw", type=float, default=None, metavar="SCALE",
                    help="time evGW instead, the three-center tensor scaled by SCALE")
    ap.add_argument("--open-shell", type=float, default=None, metavar="DELTA",
                    help="time open-shell G0W0 instead, channels split by DELTA Ha per AO")
    ap.add_argument("--metric", action="store_true",
                    help="non-orthogonal RI and AO bases (Gaussian overlaps)")
    ap.add_argument("--wall-budget", type=float, default=330.0,
                    help="seconds after which the precision-form legs are skipped")
    ap.add_argument("--t3c-scale", type=float, default=1.0,
                    help="scale of the three-center tensor in the --open-shell mode")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU run would shard chi and Sigma by tau point)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload.startswith("mol"):
        bench_batched(args)
        return
    if args.workload.startswith("ribbon"):
        bench_screened(args)
        return
    if args.evgw is not None:
        bench_evgw(args)
        return
    if args.open_shell is not None:
        bench_open_shell(args)
        return
    bench_chain(args)


if __name__ == "__main__":
    main()
