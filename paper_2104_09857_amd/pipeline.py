"""The five ABI calls chained from device-resident inputs to QP energies.

Only orchestration: each step is one call into libgw.so.  Per-stage wall
times come from HIP events recorded on the stream the library runs on.
"""
from __future__ import annotations

import numpy as np

from . import gw


def g0w0(sys, C, eps, mu_f, V, tau, omega, cos_w, sin_w, icos_w, states, filter_eps,
         spin=2.0, vxc=None, window=gw.PADE_WINDOW_HA, stream=None, events=False,
         chi_timing=False,
         prec="fp64", screener=None, screen_margin=1.0, eps_g=None, mu_g=None,
         sigma_prec="fp64", S_ri=None):
    """The chain of library calls.  prec: arithmetic of the chi contraction;
    sigma_prec: of the Sigma products ("fp64" or "fp32"; FP64 by default: the
    Pade continuation and Newton of the QP step lose a state here and there
    to the last digits of an FP32 Sigma).  eps_g / mu_g (optional): energies
    and energy zero of the Green's function (Eq. 2) when they differ from the
    mean-field eps / mu_f, which the QP equation keeps (an evGW step).  S_ri
    (optional, device [n_ri][n_ri]): RI overlap metric (Eq. 5); the
    self-energies then take W~^c and V~ (gw_screen_w_metric).  C may belong
    to a non-orthogonal AO basis (C S_ao C^T = 1) with no other change."""
    import torch
    st = torch.cuda.current_stream() if stream is None else stream
    ev = {}

    def mark(name):
        if events:
            e = torch.cuda.Event(enable_timing=True)
            e.record(st)
            ev[name] = e

    states = np.asarray(states, dtype=np.int32)
    eps = np.asarray(eps, dtype=np.float64)
    if eps_g is None:
        eps_g, mu_g = eps, mu_f
    eps_g = np.asarray(eps_g, dtype=np.float64)
    mark("start")
    d_occ, d_vir = gw.build_gt(sys, C, eps_g, mu_g, tau, stream=st)
    d0, _ = gw.build_gt(sys, C, eps_g, mu_g, [0.0], d_vir=False, stream=st)
    mark("gt")
    chi, chi_stats = gw.contract_chi(sys, d_occ, d_vir, filter_eps, stream=st, timing=chi_timing,
                                     prec=prec, screener=screener, screen_margin=screen_margin,
                                     tau=tau)
    mark("chi")
    if S_ri is None:
        wc, v_sig = gw.screen_w(sys, chi, V, cos_w, icos_w, spin, stream=st), V
    else:
        wc, v_sig = gw.screen_w_metric(sys, chi, V, S_ri, cos_w, icos_w, spin, stream=st)
    mark("screen")
    so, sv, sx, sig_stats = gw.contract_sigma(sys, states, C, d_occ, d_vir, d0, wc, v_sig,
                                              filter_eps, stream=st, prec=sigma_prec)
    mark("sigma")
    vxc = np.zeros(len(states)) if vxc is None else np.asarray(vxc, dtype=np.float64)
    is_occ = (states < sys.c.n_occ).astype(np.int32)
    e_qp, status = gw.continue_qp(so, sv, sx, eps[states], vxc, is_occ, mu_g, omega, cos_w, sin_w,
                                  window)
    mark("qp")
    out = dict(d_occ=d_occ, d_vir=d_vir, chi=chi, wc=wc, sig_occ=so, sig_vir=sv, sig_x=sx,
               e_qp=e_qp, status=status, chi_stats=chi_stats, sig_stats=sig_stats)
    if events:
        st.synchronize()
        names = list(ev)
        out["ms"] = {names[i]: ev[names[i - 1]].elapsed_time(ev[names[i]]) for i in range(1, len(names))}
    return out


def evgw(sys, C, eps, mu_f, V, tau, omega, cos_w, sin_w, icos_w, states, filter_eps, tol=1e-6,
         max_iter=20, **kw):
    """Eigenvalue self-consistent GW (the paper's step after Eq. 12): G0W0
    chains whose Green's function takes the energies of gw_evgw_update (QP
    energies of the computed states, scissor shift for the others), repeated
    until max |e_qp change| < tol.  The grids stay those of the mean field.
    Returns the last chain's outputs with e_qp history, step count and
    whether it converged."""
    eps = np.asarray(eps, dtype=np.float64)
    states = np.asarray(states, dtype=np.int32)
    n_occ = sys.c.n_occ
    eps_g, mu_g = eps, mu_f
    history, prev, out, converged = [], None, None, False
    for _ in range(max_iter):
        out = g0w0(sys, C, eps, mu_f, V, tau, omega, cos_w, sin_w, icos_w, states, filter_eps,
                   eps_g=eps_g, mu_g=mu_g, **kw)
        e = out["e_qp"]
        history.append(e)
        if np.any(out["status"] != 0):
            break
        if prev is not None and np.abs(e - prev).max() < tol:
            converged = True
            break
        try:
            eps_g, mu_g = gw.evgw_update(eps, n_occ, states, e)
        except gw.GWError:
            break
        prev = e
    out.update(history=history, steps=len(history), converged=converged, eps_g=eps_g, mu_g=mu_g)
    return out


def g0w0_spin(sys_up, sys_dn, C_up, C_dn, eps_up, eps_dn, V, tau, omega, cos_w, sin_w, icos_w,
              states_up, states_dn, filter_eps, vxc_up=None, vxc_dn=None,
              window=gw.PADE_WINDOW_HA, stream=None,
              prec="fp64", sigma_prec="fp64", S_ri=None):
    """Open-shell G0W0: one Green's function and chi per spin channel (sys_up
    and sys_dn share the bricks and differ in n_occ), W from chi_up + chi_dn
    with spin factor 1 (gw_screen_w_spins), Sigma and the QP equation per
    channel.  The energy zero is the midpoint of the highest occupied and the
    lowest virtual level over both channels.  S_ri (optional): RI overlap
    metric, the self-energies then take W~^c and V~.  Returns per-channel
    outputs and the common mu_F."""
    import torch
    st = torch.cuda.current_stream() if stream is None else stream
    chans = ((sys_up, C_up, np.asarray(eps_up, dtype=np.float64), states_up, vxc_up),
             (sys_dn, C_dn, np.asarray(eps_dn, dtype=np.float64), states_dn, vxc_dn))
    mu_f = gw.fermi_level([(e, s.c.n_occ) for s, _, e, _, _ in chans])
    ds, chis = [], []
    for sysc, C, eps, _, _ in chans:
        d_occ, d_vir = gw.build_gt(sysc, C, eps, mu_f, tau, stream=st)
        d0, _ = gw.build_gt(sysc, C, eps, mu_f, [0.0], d_vir=False, stream=st)
        chi, _ = gw.contract_chi(sysc, d_occ, d_vir, filter_eps, stream=st, prec=prec)
        ds.append((d_occ, d_vir, d0))
        chis.append(chi)
    if S_ri is None:
        wc, v_sig = gw.screen_w_spins(sys_up, chis[0], chis[1], V, cos_w, icos_w, stream=st), V
    else:
        wc, v_sig = gw.screen_w_spins_metric(sys_up, chis[0], chis[1], V, S_ri, cos_w, icos_w,
                                             stream=st)
    out = dict(chi_up=chis[0], chi_dn=chis[1], wc=wc, mu_f=mu_f)
    for tag, (sysc, C, eps, states, vxc), (d_occ, d_vir, d0) in zip(("up", "dn"), chans, ds):
        states = np.asarray(states, dtype=np.int32)
        so, sv, sx, _ = gw.contract_sigma(sysc, states, C, d_occ, d_vir, d0, wc, v_sig,
                                          filter_eps, stream=st, prec=sigma_prec)
        vxc = np.zeros(len(states)) if vxc is None else np.asarray(vxc, dtype=np.float64)
        is_occ = (states < sysc.c.n_occ).astype(np.int32)
        e_qp, status = gw.continue_qp(so, sv, sx, eps[states], vxc, is_occ, mu_f, omega, cos_w,
                                      sin_w, window)
        out["e_qp_" + tag] = e_qp
        out["status_" + tag] = status
    return out
