"""Diagonal self-energy pieces (Eqs. 10-11), FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

  B^n_{mu P}     = sum_nu C_{n nu} (nu mu P)                 half transform
  Z^n_{P nu}     = sum_Q W_PQ B^n_{nu Q}                      inner sum of Eq. 10
  S^occ_n(tau)   = sum_{mu nu} D^occ_{mu nu}(tau) sum_P B^n_{mu P} Z^n_{P nu}
  S^vir_n(tau)   = the same with D^vir(tau)
  Sigma^x_n      = - the same with W := V and D := D^occ(0)   (Eq. 11)

Pinned by: AO contraction == MO form (brute force),
S^occ_n(tau) = sum_i exp(eps_bar_i tau) sum_PQ (ni|P) W_PQ (Q|in), likewise
for the virtual part, Sigma^x_n = -sum_i (ni|P) V_PQ (Q|in) <= 0, and the
single-pole closed form of Sigma^c(i w) (tests/test_oracle_screen_sigma_qp.py).
"""
from __future__ import annotations

import numpy as np


def half_transform(C, t3c, states):
    """B[n][mu][P] for the listed states."""
    return np.ascontiguousarray(np.einsum("kn,nmp->kmp", C[states], t3c, optimize=True))


def sigma_pieces(b, d, w):
    """<D, B W B^T>_F for each state: b [n_gw][n_ao][n_ri], d [n_ao][n_ao],
    w [n_ri][n_ri] -> [n_gw], in the order of Eq. 10."""
    out = np.empty(b.shape[0])
    d = np.ascontiguousarray(d)
    w = np.ascontiguousarray(w)
    for k in range(b.shape[0]):
        z = w @ b[k].T                      # Z_{P nu} = sum_Q W_PQ B_{nu Q}
        y = b[k] @ z                        # Y_{mu nu} = sum_P B_{mu P} Z_{P nu}
        out[k] = np.sum(d * y)
    return out


def sigma_tau(C, t3c, states, d_occ, d_vir, wc_tau):
    """S^occ, S^vir as [n_gw][n_tau]."""
    b = half_transform(C, t3c, states)
    n_tau = d_occ.shape[0]
    so = np.empty((len(states), n_tau))
    sv = np.empty((len(states), n_tau))
    for j in range(n_tau):
        so[:, j] = sigma_pieces(b, d_occ[j], wc_tau[j])
        sv[:, j] = sigma_pieces(b, d_vir[j], wc_tau[j])
    return so, sv


def sigma_x(C, t3c, states, d_occ0, V):
    b = half_transform(C, t3c, states)
    return -sigma_pieces(b, d_occ0, V)


# ------------------------------------------------------------- MO forms
def mo_pair_integrals(C, t3c, states):
    """(n m|P) for n in states, all m: [n_gw][n_mo][n_ri]."""
    half = np.einsum("kn,nmp->kmp", C[states], t3c, optimize=True)
    return np.einsum("jm,kmp->kjp", C, half, optimize=True)


def sigma_tau_mo(C, eps, n_occ, mu_f, t3c, states, wc_tau, tau):
    nm = mo_pair_integrals(C, t3c, states)
    eb = eps - mu_f
    so = np.empty((len(states), len(tau)))
    sv = np.empty((len(states), len(tau)))
    for j, t in enumerate(tau):
        m = np.einsum("kip,pq,kiq->ki", nm, wc_tau[j], nm, optimize=True)
        so[:, j] = (m[:, :n_occ] * np.exp(eb[:n_occ] * t)).sum(1)
        sv[:, j] = (m[:, n_occ:] * np.exp(-eb[n_occ:] * t)).sum(1)
    return so, sv


def sigma_x_mo(C, n_occ, t3c, states, V):
    nm = mo_pair_integrals(C, t3c, states)
    m = np.einsum("kip,pq,kiq->ki", nm[:, :n_occ], V, nm[:, :n_occ], optimize=True)
    return -m.sum(1)
