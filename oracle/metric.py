"""G0W0 with non-orthogonal bases, FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

RI overlap metric (Eq. 5 and the definitions after Eqs. 10 and 11): with the
RI overlap S_PQ, the polarizability entering the dielectric function is
chi~ = S^-1 chi S^-1; the correlation self-energy takes W~^c = S^-1 W^c S^-1
and the exchange self-energy V~ = S^-1 V S^-1.  Step by step, in the paper's
order:

  chi(i w_k)     cosine transform of chi(tau_j)          (as for S = 1)
  chi~(i w_k)  = S^-1 chi(i w_k) S^-1                    (Eq. 5)
  eps(i w_k)   = 1 - L^T chi~(i w_k) L,  V = L L^T       (Eqs. 7-8)
  W^c(i w_k)   = L [eps^-1 - 1] L^T                      (Eq. 9)
  W^c(tau_j)     inverse cosine transform
  W~^c(tau_j)  = S^-1 W^c(tau_j) S^-1,  V~ = S^-1 V S^-1  (Eqs. 10-11)

Non-orthogonal AO basis: the Green's function of Eq. 2 is built from the MO
coefficients as given (C S_ao C^T = 1 instead of C C^T = 1); no step of the
chain assumes orthonormal AOs, so nothing else changes.

Pinned by (tests/test_oracle_metric.py): S = 1 reproduces the pinned chain;
the QP energies do not change under an invertible non-orthogonal change of
the RI basis (T -> T A^T on the RI index, S -> A S A^T, V -> A V A^T), nor
under one of the AO basis (C -> C B^-1, T -> B T B^T on the AO indices);
D^occ(0) S_ao D^occ(0) = D^occ(0), tr(D^occ(0) S_ao) = n_occ and
(D^occ(0) + D^vir(0)) S_ao = 1 for the generalized eigenvectors.
"""
from __future__ import annotations

import numpy as np

from . import gt, chi as ochi, screen, sigma as osig, qp
from .chain import Chain


def sandwich_inv(S, a):
    """S^-1 a S^-1 for symmetric S and a."""
    x = np.linalg.solve(S, a)
    return np.linalg.solve(S, x.T).T


def screen_w_metric(chi_tau, V, S, cos_w, icos_w, spin):
    """(W~^c(tau_j) stack, V~) for the RI overlap S."""
    L = screen.cholesky_lower(V)
    chi_w = screen.chi_omega(chi_tau, cos_w, spin)
    wcw = np.stack([screen.wc_omega(sandwich_inv(S, chi_w[k]), L) for k in range(chi_w.shape[0])])
    wc_tau = 0.5 * np.einsum("jk,kpq->jpq", icos_w, wcw, optimize=True)
    return np.stack([sandwich_inv(S, w) for w in wc_tau]), sandwich_inv(S, V)


def g0w0_metric(C, eps, n_occ, t3c, V, S, ao_off, ri_off, grids, states, filter_eps=0.0,
                spin=2.0, vxc=None, window=qp.PADE_WINDOW_HA):
    """The chain with the RI overlap S (C may be non-orthogonal in the AOs);
    Chain.wc_tau holds W~^c."""
    mu_f = 0.5 * (eps[n_occ - 1] + eps[n_occ])
    states = np.asarray(states)
    d_occ, d_vir = gt.density_matrices(C, eps, n_occ, mu_f, grids.tau)
    chi_tau = ochi.chi_filtered(t3c, d_occ, d_vir, ao_off, ri_off, filter_eps)
    wct, vt = screen_w_metric(chi_tau, V, S, grids.cos_w, grids.icos_w, spin)
    dof = np.stack([ochi.filter_blocks(d, ao_off, ao_off, filter_eps) for d in d_occ])
    dvf = np.stack([ochi.filter_blocks(d, ao_off, ao_off, filter_eps) for d in d_vir])
    so, sv = osig.sigma_tau(C, t3c, states, dof, dvf, wct)
    d0, _ = gt.density_matrices(C, eps, n_occ, mu_f, [0.0])
    d0 = ochi.filter_blocks(d0[0], ao_off, ao_off, filter_eps)
    sx = osig.sigma_x(C, t3c, states, d0, vt)
    vxc = np.zeros(len(states)) if vxc is None else np.asarray(vxc)
    is_occ = (states < n_occ).astype(np.int32)
    e_qp, status = qp.qp_energies(so, sv, sx, eps[states], vxc, is_occ, mu_f, grids.omega,
                                  grids.cos_w, grids.sin_w, window)
    return Chain(d_occ, d_vir, chi_tau, wct, so, sv, sx, e_qp, status)
