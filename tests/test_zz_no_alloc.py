"""gw_build_gt_noalloc: the density matrices of Eq. 2 without any allocation
(the per-tau weights staged in the library's per-device array), called
through the C ABI and compared with gw_build_gt bit for bit on two calls in a
row, the second with a smaller system and fewer tau points; a size beyond the
staging array is rejected before anything is launched."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _entry():
    from paper_2104_09857_amd import gw
    f = gw.lib().gw_build_gt_noalloc
    P = ctypes.c_void_p
    f.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int32, P, P, P, P]
    f.restype = ctypes.c_int32
    return f


def _inputs(w, n_tau):
    import torch
    from gwinputs import configs
    from paper_2104_09857_amd import gw
    s = w.system
    C, eps = s.mean_field()
    g = configs.grids_for(w, eps)
    mu = configs.mu_fermi(eps, s.n_occ)
    sysd = gw.System(s.n_atoms, s.n_ao_atom, s.n_ri_atom, s.n_occ, np.zeros((0, 3)), None)
    return sysd, torch.as_tensor(C, device="cuda"), eps, mu, np.ascontiguousarray(g.tau[:n_tau])


def test_noalloc_equals_build_gt():
    import torch
    from gwinputs import configs
    from paper_2104_09857_amd import gw
    f = _entry()
    st = torch.cuda.current_stream()
    for w, n_tau in ((configs.strip(22), 12), (configs.chain12(), 3)):
        sysd, Cd, eps, mu, tau = _inputs(w, n_tau)
        print("case", w.name, "n_tau", n_tau, flush=True)
        ref_o, ref_v = gw.build_gt(sysd, Cd, eps, mu, tau)
        n = sysd.n_ao
        out_o = torch.full((n_tau, n, n), float("nan"), dtype=torch.float64, device="cuda")
        out_v = torch.full_like(out_o, float("nan"))
        e = np.ascontiguousarray(eps, dtype=np.float64)
        rc = f(ctypes.byref(sysd.c), Cd.data_ptr(), e.ctypes.data, float(mu), n_tau,
               tau.ctypes.data, out_o.data_ptr(), out_v.data_ptr(), st.cuda_stream)
        assert rc == gw.GW_OK, gw.lib().gw_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out_o, ref_o) and torch.equal(out_v, ref_v)
        # one branch only
        out_v.fill_(float("nan"))
        rc = f(ctypes.byref(sysd.c), Cd.data_ptr(), e.ctypes.data, float(mu), n_tau,
               tau.ctypes.data, None, out_v.data_ptr(), st.cuda_stream)
        assert rc == gw.GW_OK
        torch.cuda.synchronize()
        assert torch.equal(out_v, ref_v)


def test_noalloc_rejects_sizes_beyond_the_array():
    import torch
    from gwinputs import configs
    from paper_2104_09857_amd import gw
    f = _entry()
    sysd, Cd, eps, mu, _ = _inputs(configs.strip(22), 12)
    tau = np.linspace(0.01, 10.0, 2000)          # 2 * 2000 * 286 weights > 2^20
    dummy = torch.zeros(1, dtype=torch.float64, device="cuda")
    e = np.ascontiguousarray(eps, dtype=np.float64)
    rc = f(ctypes.byref(sysd.c), Cd.data_ptr(), e.ctypes.data, float(mu), len(tau), tau.ctypes.data,
           dummy.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
    assert rc == gw.GW_ERR_ARG and b"staging array" in gw.lib().gw_last_error()
    torch.cuda.synchronize()
    assert float(dummy[0]) == 0.0
