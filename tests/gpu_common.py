"""Device-side set-up shared by the GPU tests (inputs only; no oracle here)."""
import numpy as np


def device_inputs(inp, bricks_on_device=False):
    """Upload one workload's inputs; returns a dict with the gw.System and tensors."""
    import torch
    from paper_2104_09857_amd import gw
    s = inp.s
    dev = "cuda"
    if bricks_on_device:
        from gwinputs import device as gdev
        t3c = gdev.bricks_on_device(s, inp.trip)
    else:
        t3c = torch.as_tensor(inp.bricks, device=dev)
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, inp.trip, t3c)
    C = torch.as_tensor(inp.C, device=dev)
    V = torch.as_tensor(inp.V, device=dev)
    return dict(sys=sysd, t3c=t3c, C=C, V=V)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
