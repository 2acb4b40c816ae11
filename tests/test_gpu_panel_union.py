"""A column panel coupled to more atoms than an LDS table of one entry per
function could hold.

260 atoms with 16 AO and 2 RI functions each and every triple (a, a, c):
each RI atom couples to all 260 AO atoms, so every panel of the outer
contraction (80 RI atoms) has a K union of 260 atoms = 4160 AO functions
(4160 k pairs in the BF16x3 form), beyond 3968 entries.  The stage-C tables
hold one entry per union atom.  FP64 chi against the oracle's block routine
(Eq. 3) on sampled blocks, inside one panel and across two (1e-11 relative:
sums of 4160 and 66560 terms in another order); the register-staged and the
direct-to-LDS stage C give the same chi bit for bit in every precision."""
import numpy as np
import pytest

from gpu_common import rel
from oracle import chi as ochi

pytestmark = pytest.mark.gpu

N_ATOMS, NA, NR = 260, 16, 2
# stage-C variants: direct-to-LDS (FP32 needs NR % 4 == 0: two register-staged tiles)
VARIANTS = {"fp64": (3, 0), "fp32": (2, 0), "bf16x3": (3, 0)}


@pytest.fixture(scope="module")
def big_union():
    import torch
    from paper_2104_09857_amd import gw
    rng = np.random.default_rng(11)
    a = np.repeat(np.arange(N_ATOMS), N_ATOMS)
    c = np.tile(np.arange(N_ATOMS), N_ATOMS)
    trip = np.stack([a, a, c], 1).astype(np.int32)
    x = rng.standard_normal((len(trip), NA, NA, NR))
    bricks = 0.5 * (x + x.transpose(0, 2, 1, 3))            # symmetric in (mu, nu)
    n = N_ATOMS * NA
    do = rng.standard_normal((n, n)) / np.sqrt(n)
    dv = rng.standard_normal((n, n)) / np.sqrt(n)
    do, dv = 0.5 * (do + do.T), 0.5 * (dv + dv.T)
    t3c = torch.as_tensor(bricks, device="cuda")
    sysd = gw.System(N_ATOMS, NA, NR, 10, trip, t3c)
    return trip, bricks, do, dv, sysd


def test_fp64_chi_vs_oracle_blocks(big_union):
    import torch
    from paper_2104_09857_amd import gw
    trip, bricks, do, dv, sysd = big_union
    print("case panel union of 260 atoms, fp64 vs oracle blocks", flush=True)
    chi, _ = gw.contract_chi(sysd, torch.as_tensor(do[None], device="cuda"),
                             torch.as_tensor(dv[None], device="cuda"), 0.0)
    got = chi[0].cpu().numpy()
    index = {(int(p), int(q), int(r)): i for i, (p, q, r) in enumerate(trip)}
    ao_off = np.arange(N_ATOMS + 1) * NA
    ri_off = np.arange(N_ATOMS + 1) * NR
    for c, c2 in ((3, 3), (7, 201)):                        # one panel; across panels
        ref = ochi.chi_block(c, c2, trip, lambda p, q, r: bricks[index[(p, q, r)]], do, dv,
                             ao_off, ri_off, 0.0)
        blk = got[ri_off[c]:ri_off[c + 1], ri_off[c2]:ri_off[c2 + 1]]
        assert rel(blk, ref) < 1e-11, (c, c2)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_stage_c_engines_agree(big_union, prec):
    import torch
    from paper_2104_09857_amd import gw
    _, _, do, dv, sysd = big_union
    d_o = [torch.as_tensor(do[None], device="cuda")]
    d_v = [torch.as_tensor(dv[None], device="cuda")]
    plan = gw.ChiBatch([sysd], 1, 0.0, prec=prec)
    pers = plan.config()[1]
    outs = []
    for variant in VARIANTS[prec]:
        print("case panel union of 260 atoms", prec, "stage-C variant", variant, flush=True)
        plan.set_config(variant, pers)
        out = plan.outputs()
        plan.execute(d_o, d_v, out)
        torch.cuda.synchronize()
        outs.append(out[0])
    plan.close()
    assert torch.isfinite(outs[0]).all()
    assert torch.equal(outs[0], outs[1])
