"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments on the host before any launch, and its
host-only QP step agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2104_09857_amd import gw
from oracle import qp as oqp

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "gw.h")


def test_library_exports_every_declared_symbol():
    L = gw.lib()
    decl = re.findall(r"^\w[\w\s\*]*?\b(gw_\w+)\s*\(", open(HEADER).read(), flags=re.M)
    assert set(decl) >= set(gw.EXPORTED)
    for name in decl:
        assert hasattr(L, name), name
    assert b"gfx950" in L.gw_version()


def test_host_validation_rejects_bad_arguments():
    L = gw.lib()
    trip = np.zeros((1, 3), dtype=np.int32)
    sys_ok = gw._System(2, 3, 4, 3, 1, trip.ctypes.data_as(ctypes.c_void_p).value, 1)
    cases = [
        gw._System(0, 3, 4, 3, 0, None, None),      # no atoms
        gw._System(2, 3, 4, 0, 0, None, None),      # no occupied states
        gw._System(2, 3, 4, 6, 0, None, None),      # n_occ == n_ao
    ]
    opts = gw._ChiOpts(0, 0.0)
    for s in cases:
        rc = L.gw_contract_chi(ctypes.byref(s), 1, 1, 1, ctypes.byref(opts), 1, None, None)
        assert rc == gw.GW_ERR_ARG
        assert L.gw_last_error()
    bad_trip = np.array([[0, 5, 0]], dtype=np.int32)
    s = gw._System(2, 3, 4, 3, 1, bad_trip.ctypes.data_as(ctypes.c_void_p).value, 1)
    assert L.gw_contract_chi(ctypes.byref(s), 1, 1, 1, ctypes.byref(opts), 1, None, None) == gw.GW_ERR_ARG
    # null inputs, bad n_tau, negative / NaN filter
    assert L.gw_contract_chi(ctypes.byref(sys_ok), None, 1, 1, ctypes.byref(opts), 1, None, None) == gw.GW_ERR_ARG
    assert L.gw_contract_chi(ctypes.byref(sys_ok), 1, 1, 0, ctypes.byref(opts), 1, None, None) == gw.GW_ERR_ARG
    for f in (-1.0, float("nan")):
        o = gw._ChiOpts(0, f)
        assert L.gw_contract_chi(ctypes.byref(sys_ok), 1, 1, 1, ctypes.byref(o), 1, None, None) == gw.GW_ERR_ARG
    # block features need the atom coordinates (distance feature)
    tau1 = np.array([0.1])
    rc = L.gw_chi_block_features(ctypes.byref(sys_ok), 1, 1, 1, tau1.ctypes.data_as(ctypes.c_void_p),
                                 0.0, 1, None)
    assert rc == gw.GW_ERR_ARG and b"coordinates" in L.gw_last_error()
    # build_gt: an occupied level above mu_f, and a negative tau, are rejected
    eps = np.array([0.3, -0.1, 0.2, 0.5, 0.6, 0.7])
    tau = np.array([0.1])
    rc = L.gw_build_gt(ctypes.byref(sys_ok), 1, eps.ctypes.data_as(ctypes.c_void_p), 0.0, 1,
                       tau.ctypes.data_as(ctypes.c_void_p), 1, 1, None)
    assert rc == gw.GW_ERR_ARG
    eps.sort()
    tau[0] = -1.0                       # levels around mu_f = 0.4 are valid, tau is not
    rc = L.gw_build_gt(ctypes.byref(sys_ok), 1, eps.ctypes.data_as(ctypes.c_void_p), 0.4, 1,
                       tau.ctypes.data_as(ctypes.c_void_p), 1, 1, None)
    assert rc == gw.GW_ERR_ARG and b"tau" in L.gw_last_error()
    # screen_w: too many tau points, non-positive spin
    cw = np.zeros(64 * 64)
    for n_tau, spin in ((40, 2.0), (4, 0.0)):
        rc = L.gw_screen_w(ctypes.byref(sys_ok), 1, 1, n_tau, 4, cw.ctypes.data_as(ctypes.c_void_p),
                           cw.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(spin), 1, None)
        assert rc == gw.GW_ERR_ARG
    # screen_w_metric: null S, too many tau points; screen_w_spins: null chi_dn
    p = cw.ctypes.data_as(ctypes.c_void_p)
    for S, n_tau in ((None, 4), (1, 40)):
        rc = L.gw_screen_w_metric(ctypes.byref(sys_ok), 1, 1, S, n_tau, 4, p, p,
                                  ctypes.c_double(2.0), 1, None, None)
        assert rc == gw.GW_ERR_ARG
    rc = L.gw_screen_w_spins(ctypes.byref(sys_ok), 1, None, 1, 4, 4, p, p, 1, None)
    assert rc == gw.GW_ERR_ARG
    rc = L.gw_screen_w_spins_metric(ctypes.byref(sys_ok), 1, 1, 1, None, 4, 4, p, p, 1, None, None)
    assert rc == gw.GW_ERR_ARG
    # coulomb_periodic: bad cell, non-positive exponent, eta beyond sqrt(min alpha / 2),
    # loose tol, an image box beyond the bound
    cen = np.zeros(6)
    good_a, good_c = np.array([0.5, 1.0]), np.array([5.0, 5.0, 5.0])
    for a_, c_, eta, tol in ((good_a, np.array([5.0, 0.0, 5.0]), 0.0, 1e-17),
                             (np.array([0.5, -1.0]), good_c, 0.0, 1e-17),
                             (good_a, good_c, 0.6, 1e-17), (good_a, good_c, 0.0, 1e-3),
                             (good_a, good_c, 1e-4, 1e-17),
                             (good_a, np.array([1e-12, 5.0, 5.0]), 0.0, 1e-17)):
        rc = L.gw_coulomb_periodic(2, cen.ctypes.data_as(ctypes.c_void_p),
                                   a_.ctypes.data_as(ctypes.c_void_p),
                                   c_.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(eta),
                                   ctypes.c_double(tol), 1, None, None)
        assert rc == gw.GW_ERR_ARG
    # contract_sigma: state out of range
    st = np.array([7], dtype=np.int32)
    so = np.zeros(4)
    rc = L.gw_contract_sigma(ctypes.byref(sys_ok), 1, st.ctypes.data_as(ctypes.c_void_p), 1, 1, 1, 1,
                             1, 1, 1, ctypes.c_double(0.0), so.ctypes.data_as(ctypes.c_void_p),
                             so.ctypes.data_as(ctypes.c_void_p), so.ctypes.data_as(ctypes.c_void_p),
                             None, None)
    assert rc == gw.GW_ERR_ARG


def test_batch_plan_validation():
    L = gw.lib()
    trip = np.zeros((1, 3), dtype=np.int32)
    tp = trip.ctypes.data_as(ctypes.c_void_p).value
    a = gw._System(2, 3, 4, 3, 1, tp, 1)
    b = gw._System(2, 5, 4, 3, 1, tp, 1)          # other AO count per atom
    bad = gw._System(2, 3, 4, 0, 0, None, None)    # no occupied states
    opts = gw._ChiOpts(0, 0.0)
    h = ctypes.c_void_p()

    def create(systems, n_tau=4, o=opts):
        arr = (gw._System * len(systems))(*systems)
        return L.gw_chi_batch_create(len(systems), ctypes.cast(arr, ctypes.c_void_p), n_tau,
                                     ctypes.byref(o), ctypes.byref(h), None)

    assert create([a, b]) == gw.GW_ERR_ARG            # mixed basis sizes
    assert create([a, bad]) == gw.GW_ERR_ARG          # invalid member
    assert create([a], n_tau=0) == gw.GW_ERR_ARG
    assert create([a], o=gw._ChiOpts(5, 0.0)) == gw.GW_ERR_ARG       # unknown precision
    big = gw._System(2, 17, 4, 3, 1, tp, 1)
    assert create([big], o=gw._ChiOpts(2, 0.0)) == gw.GW_ERR_ARG     # BF16x3 beyond 16 AO per atom
    assert create([a], o=gw._ChiOpts(0, 1e-6, 0, 1, 1.0, None)) == gw.GW_ERR_ARG   # screener
    assert L.gw_chi_batch_create(0, None, 4, ctypes.byref(opts), ctypes.byref(h), None) == gw.GW_ERR_ARG
    assert L.gw_chi_batch_create(1, None, 4, ctypes.byref(opts), None, None) == gw.GW_ERR_ARG
    assert h.value is None
    assert L.gw_chi_batch_execute(None, None, None, None, 0, None, None) == gw.GW_ERR_ARG
    assert L.gw_chi_batch_set_config(None, 0, 0) == gw.GW_ERR_ARG
    assert L.gw_chi_batch_set_engine(None, 0) == gw.GW_ERR_ARG
    assert L.gw_chi_batch_tune(None, None, None, None, 1, None, None, None) == gw.GW_ERR_ARG
    assert L.gw_last_error()
    assert L.gw_chi_batch_destroy(None) == gw.GW_OK


def _random_sigma(rng, n_gw, n_tau):
    # a sum of decaying exponentials, like Sigma^occ / Sigma^vir
    t = np.geomspace(0.02, 20, n_tau)
    rates = rng.uniform(0.2, 3.0, (n_gw, 3))
    amps = rng.uniform(-0.5, -0.05, (n_gw, 3))
    return (amps[:, :, None] * np.exp(-rates[:, :, None] * t[None, None, :])).sum(1)


def test_continue_qp_matches_oracle(chain12):
    g = chain12.grids
    rng = np.random.default_rng(11)
    so = _random_sigma(rng, 4, len(g.tau))
    sv = _random_sigma(rng, 4, len(g.tau))
    sx = rng.uniform(-0.8, -0.2, 4)
    eps_n = np.array([-0.4, -0.3, 0.2, 0.35])
    vxc = rng.uniform(-0.3, -0.1, 4)
    is_occ = np.array([1, 1, 0, 0], dtype=np.int32)
    mu = -0.05
    for window in (0.0, 8.0):
        e, st = gw.continue_qp(so, sv, sx, eps_n, vxc, is_occ, mu, g.omega, g.cos_w, g.sin_w, window)
        ref, rst = oqp.qp_energies(so, sv, sx, eps_n, vxc, is_occ, mu, g.omega, g.cos_w, g.sin_w,
                                   window if window > 0 else None)
        assert np.array_equal(st == 0, rst == 0)
        ok = st == 0
        assert np.all(np.abs(e[ok] - ref[ok]) < 1e-9)


def test_continue_qp_reports_non_convergence():
    om = np.array([0.5, 2.0])
    cw = np.zeros((2, 1))
    sw = np.zeros((2, 1))
    so = np.zeros((1, 1))
    e, st = gw.continue_qp(so, so, np.zeros(1), np.zeros(1), np.zeros(1), np.array([0]), 0.0, om,
                           cw, sw, max_iter=1)
    # Sigma^c == 0: the single Newton step converges only if the first step is already < tol
    assert st[0] in (gw.GW_OK, gw.GW_ERR_NO_CONVERGE)
    with pytest.raises(gw.GWError):
        gw.continue_qp(so, so, np.zeros(1), np.zeros(1), np.zeros(1), np.array([0]), 0.0, -om, cw, sw)


def test_evgw_update_matches_oracle():
    """gw_evgw_update (host) against the oracle's update rule on random level
    sets, the crossing failure and invalid arguments."""
    from oracle import evgw as oev
    rng = np.random.default_rng(11)
    for trial in range(20):
        n_mo = int(rng.integers(4, 40))
        n_occ = int(rng.integers(1, n_mo))
        eps0 = np.sort(rng.normal(size=n_mo))
        eps0[n_occ:] += 3.0                       # a gap
        k = int(rng.integers(1, min(n_mo, 8) + 1))
        states = np.sort(rng.choice(n_mo, size=k, replace=False)).astype(np.int32)
        e_qp = eps0[states] + 0.3 * rng.normal(size=k)
        ref = oev.update_energies(eps0, n_occ, states, e_qp)
        if ref is None:
            with pytest.raises(gw.GWError):
                gw.evgw_update(eps0, n_occ, states, e_qp)
            continue
        out, mu = gw.evgw_update(eps0, n_occ, states, e_qp)
        np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14)
        assert mu == pytest.approx(0.5 * (ref[:n_occ].max() + ref[n_occ:].min()), abs=1e-14)
    eps0 = np.array([-2.0, -1.0, 1.0, 2.0])
    with pytest.raises(gw.GWError):            # HOMO pushed above the LUMO
        gw.evgw_update(eps0, 2, [1, 2], [1.5, 1.2])
    with pytest.raises(gw.GWError):            # repeated state
        gw.evgw_update(eps0, 2, [1, 1], [-1.1, -1.2])
    with pytest.raises(gw.GWError):            # state out of range
        gw.evgw_update(eps0, 2, [4], [0.0])
    with pytest.raises(gw.GWError):            # non-finite QP energy
        gw.evgw_update(eps0, 2, [1], [float("nan")])


def test_coulomb_periodic_host_plan():
    """The Ewald plan of gw_coulomb_periodic (filled into gw_coulomb_info on
    the host before any device work; the call then stops at the missing GPU
    here): the reciprocal vectors are the half space of the lattice within
    g_cut, each +-G pair once; the real-space images are those whose distance
    to the box of minimum-image displacements is within r_cut; and the
    split parameter honours eta < sqrt(min alpha / 2)."""
    import math
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("with a GPU the call would go on to launch kernels on the dummy output; "
                    "the device side is covered by tests/test_gpu_periodic.py")
    L = gw.lib()
    cell = np.array([7.5, 8.0, 9.5])
    rng = np.random.default_rng(2)
    cen = rng.uniform(0, 1, (6, 3)) * cell
    alpha = np.array([0.5, 0.8, 1.0, 1.3, 2.0, 0.6])
    for eta in (0.0, 0.3):
        info = gw._CoulombInfo()
        rc = L.gw_coulomb_periodic(6, cen.ctypes.data_as(ctypes.c_void_p),
                                   alpha.ctypes.data_as(ctypes.c_void_p),
                                   cell.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(eta),
                                   ctypes.c_double(1e-17), 1, ctypes.byref(info), None)
        assert rc in (gw.GW_OK, gw.GW_ERR_HIP)
        assert 0 < info.eta < math.sqrt(alpha.min() / 2)
        if eta > 0:
            assert info.eta == eta
        b = 2 * np.pi / cell
        m = np.ceil(info.g_cut / b).astype(int)
        n_g = 0
        for i in range(-m[0], m[0] + 1):
            for j in range(-m[1], m[1] + 1):
                for k in range(-m[2], m[2] + 1):
                    g2 = (i * b[0]) ** 2 + (j * b[1]) ** 2 + (k * b[2]) ** 2
                    if 0 < g2 <= info.g_cut ** 2:
                        n_g += 1
        assert info.n_g * 2 == n_g
        n = np.ceil(info.r_cut / cell + 0.5).astype(int)
        n_img = 0
        for i in range(-n[0], n[0] + 1):
            for j in range(-n[1], n[1] + 1):
                for k in range(-n[2], n[2] + 1):
                    e = np.maximum(0.0, np.abs([i, j, k]) * cell - 0.5 * cell)
                    if (e * e).sum() <= info.r_cut ** 2 * (1 + 1e-12):
                        n_img += 1
        assert info.n_img == n_img
        # the terms left out are below tol
        assert math.erfc(info.eta * info.r_cut) <= 1e-17
        assert 4 * np.pi / np.prod(cell) * math.exp(-info.g_cut ** 2 / (4 * info.eta ** 2)) \
            / info.g_cut ** 2 <= 1e-17


def test_header_is_plain_c(tmp_path):
    """include/gw.h is a C header: a C99 translation unit that includes it and
    names every struct it declares compiles without warnings."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    hdr = open(HEADER).read()
    types = sorted(set(re.findall(r"}\s*(gw_\w+)\s*;", hdr)))
    assert "gw_system" in types and "gw_coulomb_info" in types
    src = tmp_path / "hdr.c"
    src.write_text('#include "gw.h"\nint main(void) {\n'
                   + "".join(f"  {t} v{i}; (void)v{i};\n" for i, t in enumerate(types))
                   + "  return 0;\n}\n")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I" + os.path.dirname(HEADER), "-I/opt/rocm/include", "-c", str(src),
                        "-o", str(tmp_path / "hdr.o")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]


def test_sigma_exchange_arguments_together():
    """gw_contract_sigma: d_occ0, V and sig_x are given together or all null."""
    L = gw.lib()
    trip = np.zeros((1, 3), dtype=np.int32)
    s = gw._System(2, 3, 4, 3, 1, trip.ctypes.data_as(ctypes.c_void_p).value, 1)
    states = np.array([0], dtype=np.int32)
    so, sv, sx = np.zeros(1), np.zeros(1), np.zeros(1)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    for d0, V, x in ((1, None, None), (None, 1, None), (None, None, P(sx)), (1, 1, None)):
        rc = L.gw_contract_sigma(ctypes.byref(s), 1, P(states), 1, 1, 1, d0, 1, V, 1, 0.0, P(so),
                                 P(sv), x, None, None)
        assert rc == gw.GW_ERR_ARG and b"together" in L.gw_last_error()


def test_fermi_level():
    """gw_fermi_level: midpoint of the highest occupied and lowest virtual level
    over the channels; occupations without such a gap are rejected."""
    up = np.array([-0.5, -0.2, 0.1, 0.4])
    dn = np.array([-0.45, -0.3, 0.05, 0.2])
    assert gw.fermi_level([(up, 2)]) == 0.5 * (-0.2 + 0.1)
    assert gw.fermi_level([(up, 2), (dn, 2)]) == 0.5 * (-0.2 + 0.05)
    # one electron moved to the up channel: HOMO 0.1 (up), LUMO -0.3 (dn) -> no gap
    with pytest.raises(gw.GWError) as e:
        gw.fermi_level([(up, 3), (dn, 1)])
    assert e.value.code == gw.GW_ERR_ARG
    with pytest.raises(gw.GWError):
        gw.fermi_level([(np.array([0.0, np.nan]), 1)])
    # levels need not be sorted (an evGW update may reorder them)
    assert gw.fermi_level([(np.array([-0.1, -0.3, 0.5, 0.2]), 2)]) == 0.5 * (-0.1 + 0.2)


def test_binding_checks_device_arguments_before_the_library():
    """The binding rejects a wrong dtype, shape or device before any call into
    libgw.so (a wrong-size buffer would otherwise be read or written past its
    end by the kernels)."""
    import torch
    trip = np.zeros((1, 3), dtype=np.int32)
    with pytest.raises(ValueError):
        gw.System(2, 3, 4, 3, trip, torch.zeros(36, dtype=torch.float32))
    with pytest.raises(ValueError):
        gw.System(2, 3, 4, 3, trip, torch.zeros(35, dtype=torch.float64))
    s = gw.System(2, 3, 4, 3, trip, torch.zeros(36, dtype=torch.float64))
    eps = np.linspace(-1, 1, 6)
    C32 = torch.zeros((6, 6), dtype=torch.float32)
    C64 = torch.zeros((6, 6), dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        gw.build_gt(s, C32, eps, 0.0, [0.1], d_occ=torch.zeros((1, 6, 6), dtype=torch.float64),
                    d_vir=torch.zeros((1, 6, 6), dtype=torch.float64))
    with pytest.raises(ValueError, match="shape"):
        gw.build_gt(s, torch.zeros((6, 5), dtype=torch.float64), eps, 0.0, [0.1],
                    d_occ=torch.zeros((1, 6, 6), dtype=torch.float64), d_vir=False)
    with pytest.raises(ValueError, match="GPU"):
        gw.build_gt(s, C64, eps, 0.0, [0.1], d_occ=torch.zeros((1, 6, 6), dtype=torch.float64),
                    d_vir=False)
    d = torch.zeros((2, 6, 6), dtype=torch.float64)
    with pytest.raises(ValueError, match="d_occ"):
        gw.contract_chi(s, torch.zeros((2, 6, 5), dtype=torch.float64), d,
                        chi=torch.zeros((2, 8, 8), dtype=torch.float64))
    with pytest.raises(ValueError, match="d_occ"):
        gw.contract_chi(s, d.float(), d, chi=torch.zeros((2, 8, 8), dtype=torch.float64))
    cw = np.zeros((2, 2))
    with pytest.raises(ValueError, match="chi"):
        gw.screen_w(s, torch.zeros((2, 8, 7), dtype=torch.float64),
                    torch.zeros((8, 8), dtype=torch.float64), cw, cw,
                    wc=torch.zeros((2, 8, 8), dtype=torch.float64))
    with pytest.raises(ValueError, match="C"):
        gw.contract_sigma(s, [0], C32, d, d, None, torch.zeros((2, 8, 8), dtype=torch.float64), None)
