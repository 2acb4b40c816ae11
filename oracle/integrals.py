"""Three-center overlap integrals of s-type Gaussians (Eq. 4), FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

Every basis function is a normalized s-type Gaussian
    g(r) = (2 a / pi)^(3/4) exp(-a |r - R|^2),     int g^2 dr = 1,
so the overlap-metric tensor of Eq. 4, (mu nu P) = int phi_mu phi_nu phi_P dr,
is the integral of a product of three Gaussians.  The product of Gaussians
of exponents a, b, c centred at A, B, C is a Gaussian of exponent
s = a + b + c times exp(-(ab |A-B|^2 + ac |A-C|^2 + bc |B-C|^2) / s), and a
Gaussian of exponent s integrates to (pi / s)^(3/2), hence
    (mu nu P) = N_a N_b N_c (pi / s)^(3/2)
                exp(-(ab |A-B|^2 + ac |A-C|^2 + bc |B-C|^2) / s),
N = (2 a / pi)^(3/4).  The two-center overlap (the metric S of Eq. 5) is the
same with two functions.

A function is given by its atom's position plus an offset and its exponent:
function i of an atom a sits at xyz[a] + off[i] with exponent exp[i].

Pinned by: numerical quadrature of the integrals on a grid (the integrand is
a product of one-dimensional Gaussians along x, y and z), the normalization
int g^2 = 1, symmetry in mu and nu, and the limit of a very diffuse third
function (tests/test_oracle_integrals.py).
"""
from __future__ import annotations

import numpy as np


def _norm(a):
    return (2.0 * a / np.pi) ** 0.75


def three_center(ra, a, rb, b, rc, c):
    """(mu nu P) of single functions: centres ra, rb, rc [3], exponents a, b, c."""
    s = a + b + c
    e = (a * b * np.sum((ra - rb) ** 2) + a * c * np.sum((ra - rc) ** 2)
         + b * c * np.sum((rb - rc) ** 2)) / s
    return _norm(a) * _norm(b) * _norm(c) * (np.pi / s) ** 1.5 * np.exp(-e)


def bricks(xyz, trip, ao_exp, ao_off, ri_exp, ri_off):
    """Brick of every triple (a, b, c): [n_trip][n_ao][n_ao][n_ri], element
    (mu, nu, P) = (mu nu P) of AO function mu of atom a, nu of atom b and RI
    function P of atom c (the formula above, broadcast over mu, nu, P)."""
    ao_e = np.asarray(ao_exp, dtype=np.float64)
    ri_e = np.asarray(ri_exp, dtype=np.float64)
    a = ao_e[:, None, None]
    b = ao_e[None, :, None]
    c = ri_e[None, None, :]
    s = a + b + c
    pref = _norm(a) * _norm(b) * _norm(c) * (np.pi / s) ** 1.5
    out = np.empty((len(trip), len(ao_e), len(ao_e), len(ri_e)))
    for t, (ia, ib, ic) in enumerate(trip):
        ra = (xyz[ia] + np.asarray(ao_off))[:, None, None, :]
        rb = (xyz[ib] + np.asarray(ao_off))[None, :, None, :]
        rc = (xyz[ic] + np.asarray(ri_off))[None, None, :, :]
        e = (a * b * np.sum((ra - rb) ** 2, -1) + a * c * np.sum((ra - rc) ** 2, -1)
             + b * c * np.sum((rb - rc) ** 2, -1)) / s
        out[t] = pref * np.exp(-e)
    return out


def overlap(xyz, exps, offs):
    """Two-center overlap S of the functions (atom-major, function i of each
    atom at xyz[a] + offs[i] with exponent exps[i]):
        S_ij = N_i N_j (pi / (a_i + a_j))^(3/2) exp(-a_i a_j |R_i - R_j|^2 / (a_i + a_j))."""
    n = len(exps)
    centres = (xyz[:, None, :] + np.asarray(offs)[None, :, :]).reshape(-1, 3)
    a = np.tile(np.asarray(exps, dtype=np.float64), len(xyz))
    out = np.empty((len(a), len(a)))
    for i in range(len(a)):
        for j in range(len(a)):
            s = a[i] + a[j]
            d2 = np.sum((centres[i] - centres[j]) ** 2)
            out[i, j] = _norm(a[i]) * _norm(a[j]) * (np.pi / s) ** 1.5 * np.exp(-a[i] * a[j] * d2 / s)
    return out
