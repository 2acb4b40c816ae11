"""Open-shell (spin-polarized) G0W0 on the oracle pieces, FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

The paper runs its nanoribbons as open-shell singlets (computational
details) and writes the equations for a closed shell.  Readings for two
spin channels s (each with its own orbitals C_s, energies eps_s and
occupation n_occ_s, one shared three-center tensor):

* D^occ_s(tau), D^vir_s(tau) of Eq. 2 per channel;
* chi = chi_up + chi_dn, each channel's Eq. 3 without spin factor; W from
  Eqs. 5-9 with spin factor 1;
* Sigma_{n s} (Eqs. 10-11) from D_s and the common W; Sigma^x from D^occ_s(0);
* one energy zero mu_F, the midpoint of the highest occupied and the lowest
  virtual level over both channels; the QP equation (Eq. 12) per channel;
* with an RI overlap S (the paper's ribbons use the overlap metric and are
  open-shell): the sum chi_up + chi_dn is screened as in oracle/metric.py,
  and both channels take W~^c and V~.

Pinned by (tests/test_oracle_spin.py): equal channels reproduce the
closed-shell chain (spin factor 2); exchanging the channels exchanges the
results; each channel's chi(tau) equals its MO closed form
- sum_{ia} (ia|P)(ia|Q) exp(-(eps_a - eps_i) tau); with S, equal channels
reproduce the pinned metric chain and S = 1 the form without S.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import gt, chi as ochi, screen, sigma as osig, qp, metric


@dataclasses.dataclass
class SpinChain:
    chi_up: np.ndarray
    chi_dn: np.ndarray
    wc_tau: np.ndarray
    e_qp: tuple          # (up, dn)
    status: tuple
    mu_f: float


def mu_common(eps_up, n_up, eps_dn, n_dn):
    """Midpoint of the highest occupied and lowest virtual level of both
    channels; the occupied levels of both must lie below the virtual levels
    of both, else the Green's function of Eq. 2 grows with tau."""
    homo = max(np.max(eps_up[:n_up]), np.max(eps_dn[:n_dn]))
    lumo = min(np.min(eps_up[n_up:]), np.min(eps_dn[n_dn:]))
    if not homo < lumo:
        raise ValueError("an occupied level of one channel lies above a virtual level")
    return 0.5 * (homo + lumo)


def g0w0_spin(chan_up, chan_dn, t3c, V, ao_off, ri_off, grids, states_up, states_dn,
              filter_eps=0.0, window=qp.PADE_WINDOW_HA, S=None):
    """chan_* = (C, eps, n_occ); states_*: computed MOs of each channel; S:
    RI overlap (None: S = 1)."""
    chans = (chan_up, chan_dn)
    states = (np.asarray(states_up), np.asarray(states_dn))
    mu_f = mu_common(chan_up[1], chan_up[2], chan_dn[1], chan_dn[2])
    ds, chis = [], []
    for C, eps, n_occ in chans:
        d_occ, d_vir = gt.density_matrices(C, eps, n_occ, mu_f, grids.tau)
        ds.append((d_occ, d_vir))
        chis.append(ochi.chi_filtered(t3c, d_occ, d_vir, ao_off, ri_off, filter_eps))
    if S is None:
        wc_tau = screen.screen_w(chis[0] + chis[1], V, grids.cos_w, grids.icos_w, 1.0)
        v_x = V
    else:
        wc_tau, v_x = metric.screen_w_metric(chis[0] + chis[1], V, S, grids.cos_w, grids.icos_w,
                                             1.0)
    e_out, st_out = [], []
    for (C, eps, n_occ), (d_occ, d_vir), stt in zip(chans, ds, states):
        dof = np.stack([ochi.filter_blocks(d, ao_off, ao_off, filter_eps) for d in d_occ])
        dvf = np.stack([ochi.filter_blocks(d, ao_off, ao_off, filter_eps) for d in d_vir])
        so, sv = osig.sigma_tau(C, t3c, stt, dof, dvf, wc_tau)
        d0, _ = gt.density_matrices(C, eps, n_occ, mu_f, [0.0])
        d0 = ochi.filter_blocks(d0[0], ao_off, ao_off, filter_eps)
        sx = osig.sigma_x(C, t3c, stt, d0, v_x)
        is_occ = (stt < n_occ).astype(np.int32)
        e, s = qp.qp_energies(so, sv, sx, eps[stt], np.zeros(len(stt)), is_occ, mu_f, grids.omega,
                              grids.cos_w, grids.sin_w, window)
        e_out.append(e)
        st_out.append(s)
    return SpinChain(chis[0], chis[1], wc_tau, tuple(e_out), tuple(st_out), mu_f)
