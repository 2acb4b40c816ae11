"""Eigenvalue self-consistent GW (evGW) on the oracle chain, FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

evGW as the paper defines it right after the QP equation (Eq. 12; the dashed
arrow of its workflow figure): the QP energies replace the mean-field levels
in the Green's function (Eq. 2), and the cycle (Eq. 3, Eqs. 5-9, Eqs. 10-11,
Eq. 12) is repeated until the QP energies are self-consistent; the orbitals
stay those of the mean field (no orbital updates, as the paper restricts
itself to).  The paper is silent on the states
outside the computed set, on the energy zero and on the grids.  Readings:

* a computed state takes its QP energy; every other occupied (virtual) state
  is shifted by the mean correction e_qp - eps of the computed occupied
  (virtual) states (a scissor shift; no shift for a class without a computed
  state);
* occupations stay those of the mean field (the first n_occ states); an update
  that puts an occupied level at or above mu_F or a virtual one at or below it
  is a failure (the Green's function of Eq. 2 would not decay in tau);
* mu_F is the midpoint of the updated highest occupied and lowest virtual
  levels;
* the tau / omega grids and the transform weights stay those of the mean
  field;
* the QP equation (Eq. 12) keeps the mean-field eps_n and v^xc: only the
  Green's function, hence chi, W and Sigma, sees the updated energies.

The iteration stops when max |e_qp - previous e_qp| < tol (converged), or
when a computed state has no QP solution, the update fails, or max_iter
passes (not converged).

Pinned by (tests/test_oracle_evgw.py): the update rule on a hand example;
the weak-coupling limit (evGW within O(T^4) of G0W0 after a few steps, the
levels shifted by the O(T^2) exchange term); the first step reproducing the
pinned G0W0 chain; the fixed point reproducing itself.  The choice of the
readings above is not pinned (the paper fixes none of them).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import gt, chi as ochi, screen, sigma as osig, qp


def update_energies(eps0, n_occ, states, e_qp):
    """Energies of the next Green's function (readings above); None if the
    occupied levels do not stay below the virtual ones."""
    eps0 = np.asarray(eps0, dtype=np.float64)
    states = np.asarray(states)
    d = np.asarray(e_qp, dtype=np.float64) - eps0[states]
    occ = states < n_occ
    d_occ = d[occ].mean() if occ.any() else 0.0
    d_vir = d[~occ].mean() if (~occ).any() else 0.0
    out = eps0.copy()
    out[:n_occ] += d_occ
    out[n_occ:] += d_vir
    out[states] = e_qp
    if not (out[:n_occ].max() < out[n_occ:].min()):
        return None
    return out


def one_step(C, eps0, eps_g, n_occ, t3c, V, ao_off, ri_off, grids, states, filter_eps, spin,
             vxc, window):
    """QP energies with the Green's function built from eps_g (Eqs. 2-12)."""
    mu_f = 0.5 * (eps_g[:n_occ].max() + eps_g[n_occ:].min())
    d_occ, d_vir = gt.density_matrices(C, eps_g, n_occ, mu_f, grids.tau)
    chi_tau = ochi.chi_filtered(t3c, d_occ, d_vir, ao_off, ri_off, filter_eps)
    wc_tau = screen.screen_w(chi_tau, V, grids.cos_w, grids.icos_w, spin)
    dof = np.stack([ochi.filter_blocks(d, ao_off, ao_off, filter_eps) for d in d_occ])
    dvf = np.stack([ochi.filter_blocks(d, ao_off, ao_off, filter_eps) for d in d_vir])
    so, sv = osig.sigma_tau(C, t3c, states, dof, dvf, wc_tau)
    d0, _ = gt.density_matrices(C, eps_g, n_occ, mu_f, [0.0])
    d0 = ochi.filter_blocks(d0[0], ao_off, ao_off, filter_eps)
    sx = osig.sigma_x(C, t3c, states, d0, V)
    is_occ = (states < n_occ).astype(np.int32)
    return qp.qp_energies(so, sv, sx, eps0[states], vxc, is_occ, mu_f, grids.omega, grids.cos_w,
                          grids.sin_w, window)


@dataclasses.dataclass
class EvGW:
    e_qp: np.ndarray          # last QP energies of the computed states
    status: np.ndarray        # per state, 0 ok (last step)
    eps_g: np.ndarray         # energies of the last Green's function
    history: list             # e_qp of every step
    converged: bool


def evgw(C, eps, n_occ, t3c, V, ao_off, ri_off, grids, states, filter_eps=0.0, spin=2.0,
         vxc=None, window=qp.PADE_WINDOW_HA, tol=1e-6, max_iter=20):
    eps0 = np.asarray(eps, dtype=np.float64)
    states = np.asarray(states)
    vxc = np.zeros(len(states)) if vxc is None else np.asarray(vxc, dtype=np.float64)
    eps_g = eps0.copy()
    history = []
    prev = None
    for _ in range(max_iter):
        e_qp, status = one_step(C, eps0, eps_g, n_occ, t3c, V, ao_off, ri_off, grids, states,
                                filter_eps, spin, vxc, window)
        history.append(e_qp)
        if np.any(status != 0):
            return EvGW(e_qp, status, eps_g, history, False)
        if prev is not None and np.abs(e_qp - prev).max() < tol:
            return EvGW(e_qp, status, eps_g, history, True)
        nxt = update_energies(eps0, n_occ, states, e_qp)
        if nxt is None:
            return EvGW(e_qp, status, eps_g, history, False)
        eps_g, prev = nxt, e_qp
    return EvGW(e_qp, status, eps_g, history, False)
