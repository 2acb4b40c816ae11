"""The whole G0W0 chain on dense arrays, plus the canonical O(N^4) forms.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

``g0w0`` runs every step of the oracle in the paper's order (Eq. 2 -> Eq. 3
-> Eqs. 5-9 -> Eqs. 10-11 -> transforms, Pade, Eq. 12) and returns every
intermediate, so that each piece of the HIP path can be compared with it.

``chi_omega_canonical`` is the canonical (O(N^4)) polarizability on the
imaginary-frequency axis from MO-basis integrals,
    chi_PQ(i w) = - s sum_{ia} (ia|P)(ia|Q) 2 D_ia / (D_ia^2 + w^2),
and ``chi_static_laplace`` its zero-frequency half,
    - s sum_{ia} (ia|P)(ia|Q) / D_ia,
the two closed forms the time-domain route is checked against.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import gt, chi as ochi, screen, sigma as osig, qp


@dataclasses.dataclass
class Chain:
    d_occ: np.ndarray
    d_vir: np.ndarray
    chi_tau: np.ndarray
    wc_tau: np.ndarray
    sig_occ: np.ndarray
    sig_vir: np.ndarray
    sig_x: np.ndarray
    e_qp: np.ndarray
    status: np.ndarray


def g0w0(C, eps, n_occ, t3c, V, ao_off, ri_off, grids, states, filter_eps=0.0,
         spin=2.0, vxc=None, window=qp.PADE_WINDOW_HA):
    """Full chain; ``t3c`` is the dense tensor with its bricks already filtered."""
    mu_f = 0.5 * (eps[n_occ - 1] + eps[n_occ])
    states = np.asarray(states)
    d_occ, d_vir = gt.density_matrices(C, eps, n_occ, mu_f, grids.tau)
    chi_tau = ochi.chi_filtered(t3c, d_occ, d_vir, ao_off, ri_off, filter_eps)
    wc_tau = screen.screen_w(chi_tau, V, grids.cos_w, grids.icos_w, spin)
    dof = np.stack([ochi.filter_blocks(d, ao_off, ao_off, filter_eps) for d in d_occ])
    dvf = np.stack([ochi.filter_blocks(d, ao_off, ao_off, filter_eps) for d in d_vir])
    so, sv = osig.sigma_tau(C, t3c, states, dof, dvf, wc_tau)
    d0, _ = gt.density_matrices(C, eps, n_occ, mu_f, [0.0])
    d0 = ochi.filter_blocks(d0[0], ao_off, ao_off, filter_eps)
    sx = osig.sigma_x(C, t3c, states, d0, V)
    vxc = np.zeros(len(states)) if vxc is None else np.asarray(vxc)
    is_occ = (states < n_occ).astype(np.int32)
    e_qp, status = qp.qp_energies(so, sv, sx, eps[states], vxc, is_occ, mu_f,
                                  grids.omega, grids.cos_w, grids.sin_w, window)
    return Chain(d_occ, d_vir, chi_tau, wc_tau, so, sv, sx, e_qp, status)


def chi_omega_canonical(C, eps, n_occ, t3c, omega, spin=2.0):
    iap = ochi.mo_integrals(C, t3c, n_occ)
    delta = (eps[None, n_occ:] - eps[:n_occ, None]).ravel()
    flat = iap.reshape(-1, t3c.shape[2])
    out = np.empty((len(omega), t3c.shape[2], t3c.shape[2]))
    for k, w in enumerate(omega):
        f = 2.0 * delta / (delta * delta + w * w)
        out[k] = -spin * (flat * f[:, None]).T @ flat
    return out


def chi_static_laplace(C, eps, n_occ, t3c, spin=2.0):
    iap = ochi.mo_integrals(C, t3c, n_occ)
    delta = (eps[None, n_occ:] - eps[:n_occ, None]).ravel()
    flat = iap.reshape(-1, t3c.shape[2])
    return -spin * (flat / delta[:, None]).T @ flat
