"""Polarizability chi_PQ(tau) (Eq. 3), FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

* ``chi_eq3``: the printed contraction order of Eq. 3 on dense arrays:
  first the two inner sums (over lambda with D^occ, over nu with D^vir), then
  the outer sum over mu and sigma.  Returns the per-spin chi (negative
  semidefinite).
* ``chi_mo``: the same quantity from the MO-basis three-center integrals,
  chi_PQ(tau) = - sum_{ia} (ia|P)(ia|Q) exp(-(eps_a - eps_i) tau).
* ``filtered_inputs`` / ``filter_blocks``: the atom-block filter
  (drop blocks whose Frobenius norm is below the threshold), applied to the
  tensor, to D(tau) and to the chi output blocks.
* ``chi_block``: one (c, c') output block of chi from bricks only, for
  sampled checks at sizes where the dense arrays do not fit.

Pinned by: chi_eq3 == chi_mo (brute force on small systems), symmetry,
negative semidefiniteness, mu_F invariance, MO sign-flip invariance, the
cosine-transform closed form and the Laplace closed form (tests/test_oracle_gt_chi.py).
"""
from __future__ import annotations

import numpy as np


def chi_eq3(t3c, d_occ, d_vir):
    """chi[j] for each tau_j from a dense tensor t3c[mu][nu][P] and D stacks."""
    if d_occ.ndim == 2:
        d_occ, d_vir = d_occ[None], d_vir[None]
    n_ri = t3c.shape[2]
    out = np.empty((d_occ.shape[0], n_ri, n_ri))
    for j in range(d_occ.shape[0]):
        # M_{mu sigma P} = sum_lambda (lambda sigma P) G_{mu lambda}
        m = np.ascontiguousarray(np.einsum("ml,lsp->msp", d_occ[j], t3c, optimize=True))
        # N_{mu sigma Q} = sum_nu (mu nu Q) G_{nu sigma}
        n = np.ascontiguousarray(np.einsum("mnq,ns->msq", t3c, d_vir[j], optimize=True))
        # chi_PQ = - sum_{mu sigma} M N
        out[j] = -np.einsum("msp,msq->pq", m, n, optimize=True)
    return out


def mo_integrals(C, t3c, n_occ):
    """(ia|P) = sum_{mu nu} C_{i mu} C_{a nu} (mu nu P), [n_occ][n_vir][n_ri]."""
    co, cv = C[:n_occ], C[n_occ:]
    half = np.einsum("im,mnp->inp", co, t3c, optimize=True)
    return np.einsum("an,inp->iap", cv, half, optimize=True)


def chi_mo(C, eps, n_occ, t3c, tau):
    iap = mo_integrals(C, t3c, n_occ)
    delta = eps[None, n_occ:] - eps[:n_occ, None]          # [occ][vir] > 0
    tau = np.atleast_1d(tau)
    out = np.empty((len(tau), t3c.shape[2], t3c.shape[2]))
    flat = iap.reshape(-1, t3c.shape[2])
    for j, t in enumerate(tau):
        w = np.exp(-delta * t).ravel()
        out[j] = -(flat * w[:, None]).T @ flat
    return out


# ------------------------------------------------------------------ filters
def block_norms(x, row_off, col_off):
    """Frobenius norms of the atom blocks of a 2D matrix."""
    nr, nc = len(row_off) - 1, len(col_off) - 1
    out = np.empty((nr, nc))
    for i in range(nr):
        for k in range(nc):
            blk = x[row_off[i]:row_off[i + 1], col_off[k]:col_off[k + 1]]
            out[i, k] = np.sqrt(np.sum(blk * blk))
    return out


def filter_blocks(x, row_off, col_off, eps_f):
    """Copy of x with every atom block of Frobenius norm < eps_f set to 0."""
    y = np.array(x, dtype=np.float64, copy=True)
    if eps_f <= 0:
        return y
    nrm = block_norms(y, row_off, col_off)
    for i, k in zip(*np.nonzero(nrm < eps_f)):
        y[row_off[i]:row_off[i + 1], col_off[k]:col_off[k + 1]] = 0.0
    return y


def filter_t3c(t3c, ao_off, ri_off, eps_f):
    """Dense tensor with every atom-triple brick of norm < eps_f set to 0."""
    y = np.array(t3c, dtype=np.float64, copy=True)
    if eps_f <= 0:
        return y
    na = len(ao_off) - 1
    for a in range(na):
        for b in range(na):
            for c in range(len(ri_off) - 1):
                blk = y[ao_off[a]:ao_off[a + 1], ao_off[b]:ao_off[b + 1], ri_off[c]:ri_off[c + 1]]
                if np.sqrt(np.sum(blk * blk)) < eps_f:
                    blk[...] = 0.0
    return y


def dense_from_bricks(trip, bricks, ao_off, ri_off, n_ao, n_ri, eps_f=0.0):
    """Dense tensor assembled from atom-triple bricks; bricks of norm < eps_f
    are dropped (the tensor filter)."""
    t = np.zeros((n_ao, n_ao, n_ri))
    for (a, b, c), v in zip(trip, bricks):
        if eps_f > 0 and np.sqrt(np.sum(v * v)) < eps_f:
            continue
        t[ao_off[a]:ao_off[a + 1], ao_off[b]:ao_off[b + 1], ri_off[c]:ri_off[c + 1]] = v.reshape(
            ao_off[a + 1] - ao_off[a], ao_off[b + 1] - ao_off[b], ri_off[c + 1] - ri_off[c])
    return t


def chi_filtered(t3c, d_occ, d_vir, ao_off, ri_off, eps_f):
    """chi with the three filters: tensor bricks and D(tau) blocks below eps_f
    dropped, then chi output blocks below eps_f zeroed.  ``t3c`` must already
    have its bricks filtered (dense_from_bricks / filter_t3c)."""
    out = np.empty((d_occ.shape[0], t3c.shape[2], t3c.shape[2]))
    for j in range(d_occ.shape[0]):
        do = filter_blocks(d_occ[j], ao_off, ao_off, eps_f)
        dv = filter_blocks(d_vir[j], ao_off, ao_off, eps_f)
        x = chi_eq3(t3c, do[None], dv[None])[0]
        out[j] = filter_blocks(x, ri_off, ri_off, eps_f)
    return out


# ---------------------------------------------------------- sampled blocks
def chi_block(c, c2, trip, brick_fn, d_occ, d_vir, ao_off, ri_off, eps_f):
    """One output block chi[c][c2] (before the output filter) from bricks.

    ``brick_fn(a, b, c)`` returns brick (a, b, c) as [n_ao(a)][n_ao(b)][n_ri(c)];
    ``trip`` lists the enumerated triples.  D blocks below eps_f are dropped,
    bricks below eps_f are dropped.  Follows Eq. 3 restricted to the
    (mu, sigma) pairs that can contribute: sigma on atoms b with a brick
    (., b, c), mu on atoms a' with a brick (a', ., c2).
    """
    def ao_range(atoms):
        return np.concatenate([np.arange(ao_off[a], ao_off[a + 1]) for a in atoms])

    def tensor_for(cc):
        """Bricks (a, b, cc) on the restricted index sets: (first atoms,
        second atoms, t[lambda][sigma][P])."""
        sel = [(int(a), int(b)) for a, b, c3 in trip if c3 == cc]
        first = sorted({a for a, _ in sel})
        second = sorted({b for _, b in sel})
        fpos = {a: i for i, a in enumerate(first)}
        spos = {b: i for i, b in enumerate(second)}
        na = ao_off[1] - ao_off[0]
        nr = ri_off[cc + 1] - ri_off[cc]
        t = np.zeros((len(first) * na, len(second) * na, nr))
        for a, b in sel:
            v = brick_fn(a, b, cc)
            if eps_f > 0 and np.sqrt(np.sum(v * v)) < eps_f:
                continue
            i, k = fpos[a] * na, spos[b] * na
            t[i:i + na, k:k + na, :] = v
        return first, second, t

    do = filter_blocks(d_occ, ao_off, ao_off, eps_f)
    dv = filter_blocks(d_vir, ao_off, ao_off, eps_f)
    f_p, s_p, tp = tensor_for(c)            # (lambda sigma P): lambda on f_p, sigma on s_p
    f_q, s_q, tq = (f_p, s_p, tp) if c2 == c else tensor_for(c2)   # (mu nu Q)
    lam, sig = ao_range(f_p), ao_range(s_p)
    mus, nus = ao_range(f_q), ao_range(s_q)
    # M_{mu sigma P} = sum_lambda (lambda sigma P) D^occ_{mu lambda}
    m = np.einsum("ml,lsp->msp", do[np.ix_(mus, lam)], tp, optimize=True)
    # N_{mu sigma Q} = sum_nu (mu nu Q) D^vir_{nu sigma}
    n = np.einsum("mnq,ns->msq", tq, dv[np.ix_(nus, sig)], optimize=True)
    return -np.einsum("msp,msq->pq", m, n, optimize=True)
