"""Synthetic GW inputs: geometry, basis layout, H, V, the three-center tensor.

The inputs stand in for the mean-field run and the Gaussian integrals that
feed the paper's method (Eqs. 1, 4 and 8): atoms on a chain, a ribbon-shaped
strip or a random 3D packing; every atom carries ``n_ao`` primary and
``n_ri`` auxiliary functions.  With d the distance between the atoms that
carry two functions:

  H_{mu nu}   = z * exp(-k_H d_{mu nu})  (mu < nu, mirrored);
  H_{mu mu}   = z + (2u - 1)             (u uniform in [0,1))
  (mu nu|P)   = z * exp(-k_T (d_{mu nu} + d_{mu P} + d_{nu P})), symmetric in mu nu
  V_PQ        = exp(-k_V d_PQ) + delta_PQ
with z a Philox/Box-Muller normal keyed by the global element index.  The
mean-field orbitals C and energies eps come from LAPACK ``eigh`` of H
(orthonormal AO basis, S = 1).

This module holds no arithmetic of the GW method itself; it only produces
inputs.  The tensor is stored as dense atom-triple "bricks" (a, b, c), each
``[n_ao(a)][n_ao(b)][n_ri(c)]`` row-major; only the triples whose exact norm
bound ``Z_MAX * sqrt(n_a n_b n_c) * exp(-k_T s_abc)`` reaches the filter are
enumerated (the others are below the filter whatever the draws are).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import philox

STREAM_H = 1
STREAM_H_DIAG = 2
STREAM_T = 3
STREAM_SPIN = 4
SPACING = 2.5          # bohr
STRIP_WIDTH = 7


def stream_id(tensor: int, sys_id: int = 0) -> int:
    return tensor + 16 * sys_id


# ----------------------------------------------------------------- geometry
def chain(n_atoms: int, spacing: float = SPACING) -> np.ndarray:
    xyz = np.zeros((n_atoms, 3))
    xyz[:, 0] = spacing * np.arange(n_atoms)
    return xyz


def strip(n_atoms: int, width: int = STRIP_WIDTH, spacing: float = SPACING) -> np.ndarray:
    """Rectangular ribbon: atom k at (s*floor(k/w), s*(k mod w), 0)."""
    k = np.arange(n_atoms)
    xyz = np.zeros((n_atoms, 3))
    xyz[:, 0] = spacing * (k // width)
    xyz[:, 1] = spacing * (k % width)
    return xyz


def cubic_lattice(n: int, spacing: float = SPACING) -> np.ndarray:
    """n^3 atoms on a simple cubic lattice, atom (i, j, k) at spacing*(i, j, k),
    i slowest; the periodic cell of the bulk workloads is the cube of side
    n*spacing."""
    k = np.arange(n)
    return np.stack(np.meshgrid(k, k, k, indexing="ij"), -1).reshape(-1, 3) * float(spacing)


def fibonacci_sphere(n: int, radius: float) -> np.ndarray:
    """n nearly uniform points on a sphere (golden-angle spiral)."""
    i = np.arange(n) + 0.5
    polar = np.arccos(1.0 - 2.0 * i / n)
    azim = np.pi * (1.0 + 5.0 ** 0.5) * i
    return radius * np.stack([np.cos(azim) * np.sin(polar), np.sin(azim) * np.sin(polar),
                              np.cos(polar)], axis=1)


def packing(n_atoms: int, seed: int, stream: int, density: float = 0.0148,
            d_min: float = SPACING, max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition in a cube of the given number density."""
    side = (n_atoms / density) ** (1.0 / 3.0)
    pts = []
    i = 0
    while len(pts) < n_atoms:
        if i >= max_tries:
            raise RuntimeError("packing did not converge")
        u = philox.uniform(seed, stream, np.arange(3 * i, 3 * i + 3))
        p = side * u
        if all(np.linalg.norm(p - q) >= d_min for q in pts):
            pts.append(p)
        i += 1
    return np.array(pts)


def atom_distances(xyz: np.ndarray) -> np.ndarray:
    diff = xyz[:, None, :] - xyz[None, :, :]
    return np.sqrt((diff * diff).sum(-1))


# ----------------------------------------------------------------- system
@dataclasses.dataclass
class System:
    """One synthetic molecule/strip with its inputs (all float64)."""
    xyz: np.ndarray            # [n_atoms, 3] bohr
    n_ao_atom: int
    n_ri_atom: int
    k_h: float
    k_t: float
    k_v: float
    filter_eps: float
    seed: int = 0
    sys_id: int = 0
    n_occ: Optional[int] = None
    cell: Optional[np.ndarray] = None   # orthorhombic periodic cell (box lengths), or None

    def __post_init__(self):
        self.n_atoms = self.xyz.shape[0]
        self.n_ao = self.n_atoms * self.n_ao_atom
        self.n_ri = self.n_atoms * self.n_ri_atom
        if self.n_occ is None:
            self.n_occ = self.n_ao // 2
        self.ao_off = np.arange(self.n_atoms + 1, dtype=np.int32) * self.n_ao_atom
        self.ri_off = np.arange(self.n_atoms + 1, dtype=np.int32) * self.n_ri_atom
        if self.cell is None:
            self.dist = atom_distances(self.xyz)
        else:
            # minimum-image distances of the periodic cell
            self.cell = np.asarray(self.cell, dtype=np.float64)
            diff = self.xyz[:, None, :] - self.xyz[None, :, :]
            diff -= self.cell * np.round(diff / self.cell)
            self.dist = np.sqrt((diff * diff).sum(-1))
        self.ao_atom = np.repeat(np.arange(self.n_atoms), self.n_ao_atom)
        self.ri_atom = np.repeat(np.arange(self.n_atoms), self.n_ri_atom)

    # ---- H, eigenpairs
    def hamiltonian(self) -> np.ndarray:
        n = self.n_ao
        iu, ju = np.triu_indices(n)
        tri = (ju.astype(np.uint64) * (ju.astype(np.uint64) + np.uint64(1)) // np.uint64(2)
               + iu.astype(np.uint64))
        z = philox.normal(self.seed, stream_id(STREAM_H, self.sys_id), tri)
        d = self.dist[self.ao_atom[iu], self.ao_atom[ju]]
        h = np.zeros((n, n))
        h[iu, ju] = z * np.exp(-self.k_h * d)
        h = h + np.triu(h, 1).T
        u = philox.uniform(self.seed, stream_id(STREAM_H_DIAG, self.sys_id), np.arange(n))
        h[np.arange(n), np.arange(n)] += 2.0 * u - 1.0
        return h

    def mean_field(self):
        """(C [n_mo][n_ao] row per MO, eps ascending) from eigh(H)."""
        w, v = np.linalg.eigh(self.hamiltonian())
        return np.ascontiguousarray(v.T), w

    def mean_field_spin(self, delta: float, zeeman: float = 0.0):
        """Spin-polarized mean field: H_up/dn = H +/- (delta * diag(z) - zeeman),
        z a normal draw per AO function (stream STREAM_SPIN): delta splits the
        orbitals of the channels, zeeman shifts the up levels down and the
        down levels up uniformly.  Returns ((C_up, eps_up), (C_dn, eps_dn));
        delta = zeeman = 0 gives the closed shell."""
        h = self.hamiltonian()
        z = philox.normal(self.seed, stream_id(STREAM_SPIN, self.sys_id), np.arange(self.n_ao))
        out = []
        for sgn in (1.0, -1.0):
            w, v = np.linalg.eigh(h + sgn * (delta * np.diag(z) - zeeman * np.eye(self.n_ao)))
            out.append((np.ascontiguousarray(v.T), w))
        return tuple(out)

    # ---- non-orthogonal bases
    def gaussian_metric(self, n_per_atom: int, atom_of: np.ndarray, ov_max: float = 0.4,
                        ov_min: float = 0.05) -> np.ndarray:
        """Overlap matrix of normalized s-type Gaussians, n_per_atom of them on
        every atom: function p of an atom has exponent alpha_p, geometric from
        the value whose overlap with its copy on a neighbour at SPACING is
        ov_max down to the value where it is ov_min.  Functions of different
        p are taken as orthogonal (as components of different angular
        momentum would be on one centre), so
        S[(a, p), (b, q)] = delta_pq exp(-alpha_p d_ab^2 / 2):
        symmetric positive definite (a Gaussian kernel per p), unit diagonal."""
        lo, hi = -2.0 * np.log(ov_max) / SPACING ** 2, -2.0 * np.log(ov_min) / SPACING ** 2
        alpha = lo * (hi / lo) ** (np.arange(n_per_atom) / max(n_per_atom - 1, 1))
        p = np.tile(np.arange(n_per_atom), self.n_atoms)
        d = self.dist[atom_of[:, None], atom_of[None, :]]
        return np.where(p[:, None] == p[None, :], np.exp(-0.5 * alpha[p][:, None] * d * d), 0.0)

    def ri_metric(self) -> np.ndarray:
        """RI overlap S_PQ (Eq. 5): the Gaussian metric over the RI functions."""
        return self.gaussian_metric(self.n_ri_atom, self.ri_atom)

    def ao_metric(self) -> np.ndarray:
        """AO overlap: the Gaussian metric over the AO functions."""
        return self.gaussian_metric(self.n_ao_atom, self.ao_atom, ov_max=0.3)

    def mean_field_nonorth(self, s_ao: np.ndarray):
        """(C, eps) of H C = S C eps in the non-orthogonal AO basis of overlap
        s_ao: rows of C are the MOs, C s_ao C^T = 1."""
        lc = np.linalg.cholesky(s_ao)
        linv = np.linalg.inv(lc)
        w, v = np.linalg.eigh(linv @ self.hamiltonian() @ linv.T)
        return np.ascontiguousarray((linv.T @ v).T), w

    # ---- atoms of two elements
    def light_atoms(self, light: np.ndarray, n_ao_light: int, n_ri_light: int) -> dict:
        """Per-atom sizes: the atoms listed in `light` keep only their first
        n_ao_light AO and n_ri_light RI functions (the hydrogens at the edge of
        a nanoribbon beside its carbons), the others all of theirs.  Returns
        dict(ao_off, ri_off [n_atoms + 1], ao_idx, ri_idx: the kept functions
        as indices into this system's uniform numbering, ao_mask [n_atoms]
        [n_ao_atom], ri_mask [n_atoms][n_ri_atom]: 1 for kept functions)."""
        is_light = np.zeros(self.n_atoms, dtype=bool)
        is_light[np.asarray(light, dtype=np.int64)] = True
        na = np.where(is_light, n_ao_light, self.n_ao_atom)
        nr = np.where(is_light, n_ri_light, self.n_ri_atom)
        ao_mask = (np.arange(self.n_ao_atom)[None, :] < na[:, None]).astype(np.float64)
        ri_mask = (np.arange(self.n_ri_atom)[None, :] < nr[:, None]).astype(np.float64)
        return dict(ao_off=np.concatenate([[0], np.cumsum(na)]).astype(np.int32),
                    ri_off=np.concatenate([[0], np.cumsum(nr)]).astype(np.int32),
                    ao_idx=np.nonzero(ao_mask.ravel())[0], ri_idx=np.nonzero(ri_mask.ravel())[0],
                    ao_mask=ao_mask, ri_mask=ri_mask)

    # ---- s-type Gaussian functions for the three-center integrals of Eq. 4
    def gaussian_functions(self, ao_alpha=(0.25, 1.2), ao_radius=0.5, ri_alpha=(0.2, 2.0),
                           ri_radius=0.9):
        """Normalized s-type Gaussian AO and RI functions, the same set on every
        atom: function i of an atom sits at the atom plus an offset on a
        Fibonacci sphere of the given radius (standing in for the angular
        structure of a real basis; concentric s functions of close exponents
        are nearly dependent) with an exponent geometric over the given range.
        Returns dict(ao_exp [n_ao_atom], ao_off [n_ao_atom][3],
        ri_exp [n_ri_atom], ri_off [n_ri_atom][3])."""
        def geo(lo_hi, n):
            lo, hi = lo_hi
            return lo * (hi / lo) ** (np.arange(n) / max(n - 1, 1))
        return dict(ao_exp=geo(ao_alpha, self.n_ao_atom),
                    ao_off=fibonacci_sphere(self.n_ao_atom, ao_radius),
                    ri_exp=geo(ri_alpha, self.n_ri_atom),
                    ri_off=fibonacci_sphere(self.n_ri_atom, ri_radius))

    def gaussian_overlap(self, exps: np.ndarray, offs: np.ndarray) -> np.ndarray:
        """Overlap matrix of normalized s Gaussians (exponents exps, offsets
        offs, the same on every atom; atom-major order):
        S_ij = (2 sqrt(a_i a_j) / (a_i + a_j))^(3/2) exp(-a_i a_j d_ij^2 / (a_i + a_j))."""
        cen = (self.xyz[:, None, :] + np.asarray(offs)[None, :, :]).reshape(-1, 3)
        a = np.tile(np.asarray(exps, dtype=np.float64), self.n_atoms)
        d2 = ((cen[:, None, :] - cen[None, :, :]) ** 2).sum(-1)
        sa = a[:, None] + a[None, :]
        pa = a[:, None] * a[None, :]
        return (2.0 * np.sqrt(pa) / sa) ** 1.5 * np.exp(-pa * d2 / sa)

    def all_triples(self) -> np.ndarray:
        """Every ordered atom triple (a, b, c), sorted by (c, b, a), int32 [n^3, 3]."""
        n = self.n_atoms
        c, b, a = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        return np.ascontiguousarray(np.stack([a.ravel(), b.ravel(), c.ravel()], 1).astype(np.int32))

    def ri_charges(self, radius: float = 0.8, alpha_lo: float = 0.5, alpha_hi: float = 2.0):
        """RI functions as normalized Gaussian charges for the periodic
        Coulomb matrix: function p of atom a centred at xyz[a] + o_p (o_p on a
        sphere of the given radius, standing in for the angular structure of a
        real RI basis) with exponent alpha_p geometric in [alpha_lo, alpha_hi].
        Returns (centres [n_ri][3], alpha [n_ri])."""
        nr = self.n_ri_atom
        alpha = alpha_lo * (alpha_hi / alpha_lo) ** (np.arange(nr) / max(nr - 1, 1))
        off = fibonacci_sphere(nr, radius)
        centres = (self.xyz[:, None, :] + off[None, :, :]).reshape(-1, 3)
        return np.ascontiguousarray(centres), np.tile(alpha, self.n_atoms)

    # ---- V
    def coulomb(self) -> np.ndarray:
        d = self.dist[self.ri_atom[:, None], self.ri_atom[None, :]]
        return np.exp(-self.k_v * d) + np.eye(self.n_ri)

    # ---- three-center tensor
    def perimeter(self) -> np.ndarray:
        """s[a, b, c] = d_ab + (d_ac + d_bc), summed in this order so that
        s[a, b, c] == s[b, a, c] exactly."""
        d = self.dist
        return d[:, :, None] + (d[:, None, :] + d[None, :, :])

    def triples(self) -> np.ndarray:
        """Kept ordered atom triples (a, b, c), sorted by (c, b, a), int32 [n, 3].

        A triple is enumerated when the norm bound of its brick reaches the
        filter threshold (all triples when the filter is 0).
        """
        na = self.n_atoms
        size = np.sqrt(float(self.n_ao_atom * self.n_ao_atom * self.n_ri_atom))
        # the perimeter s is at least 2 d_ac and 2 d_bc, so only atoms within
        # s_max / 2 of c can take part (s_max: the largest perimeter whose bound
        # reaches the filter; a relative slack keeps rounding on the safe side)
        if self.filter_eps > 0.0:
            s_max = np.log(philox.Z_MAX * size / self.filter_eps) / self.k_t
            reach = 0.5 * s_max * (1.0 + 1e-9) + 1e-9
        else:
            reach = np.inf
        out = []
        for c in range(na):
            idx = np.nonzero(self.dist[:, c] <= reach)[0]
            d = self.dist[np.ix_(idx, idx)]
            dc = self.dist[idx, c]
            s = d + (dc[:, None] + dc[None, :])
            bound = philox.Z_MAX * size * np.exp(-self.k_t * s)
            b_sub, a_sub = np.nonzero((bound >= self.filter_eps).T)
            a_idx, b_idx = idx[a_sub], idx[b_sub]
            trip = np.stack([a_idx, b_idx, np.full_like(a_idx, c)], axis=1)
            out.append(trip)
        return np.ascontiguousarray(np.concatenate(out).astype(np.int32))

    def brick_size(self) -> int:
        return self.n_ao_atom * self.n_ao_atom * self.n_ri_atom

    def brick(self, a: int, b: int, c: int) -> np.ndarray:
        """Brick (a, b, c) as [n_ao(a)][n_ao(b)][n_ri(c)] float64."""
        mu = np.arange(self.ao_off[a], self.ao_off[a + 1]).astype(np.uint64)
        nu = np.arange(self.ao_off[b], self.ao_off[b + 1]).astype(np.uint64)
        p = np.arange(self.ri_off[c], self.ri_off[c + 1]).astype(np.uint64)
        lo = np.minimum(mu[:, None], nu[None, :])
        hi = np.maximum(mu[:, None], nu[None, :])
        tri = hi * (hi + np.uint64(1)) // np.uint64(2) + lo
        idx = tri[:, :, None] * np.uint64(self.n_ri) + p[None, None, :]
        z = philox.normal(self.seed, stream_id(STREAM_T, self.sys_id), idx)
        s = self.dist[a, b] + (self.dist[a, c] + self.dist[b, c])
        return z * np.exp(-self.k_t * s)

    def bricks(self, trip: np.ndarray, chunk: int = 256) -> np.ndarray:
        """All bricks of a triple list, shape [n_trip, bs] (vectorised)."""
        trip = np.asarray(trip)
        na, nr = self.n_ao_atom, self.n_ri_atom
        out = np.empty((len(trip), self.brick_size()))
        li = np.arange(na, dtype=np.uint64)
        lp = np.arange(nr, dtype=np.uint64)
        for s0 in range(0, len(trip), chunk):
            t = trip[s0:s0 + chunk]
            a, b, c = t[:, 0], t[:, 1], t[:, 2]
            mu = self.ao_off[a].astype(np.uint64)[:, None] + li[None, :]
            nu = self.ao_off[b].astype(np.uint64)[:, None] + li[None, :]
            p = self.ri_off[c].astype(np.uint64)[:, None] + lp[None, :]
            lo = np.minimum(mu[:, :, None], nu[:, None, :])
            hi = np.maximum(mu[:, :, None], nu[:, None, :])
            tri = hi * (hi + np.uint64(1)) // np.uint64(2) + lo
            idx = tri[:, :, :, None] * np.uint64(self.n_ri) + p[:, None, None, :]
            z = philox.normal(self.seed, stream_id(STREAM_T, self.sys_id), idx)
            s = self.dist[a, b] + (self.dist[a, c] + self.dist[b, c])
            out[s0:s0 + len(t)] = (z * np.exp(-self.k_t * s)[:, None, None, None]).reshape(len(t), -1)
        return out

    def dense_t3c(self) -> np.ndarray:
        """The full tensor (mu nu|P) as a dense [n_ao][n_ao][n_ri] array
        (small systems only; every triple, no enumeration cut)."""
        n, m = self.n_ao, self.n_ri
        mu = np.arange(n, dtype=np.uint64)
        lo = np.minimum(mu[:, None], mu[None, :])
        hi = np.maximum(mu[:, None], mu[None, :])
        tri = hi * (hi + np.uint64(1)) // np.uint64(2) + lo
        idx = tri[:, :, None] * np.uint64(m) + np.arange(m, dtype=np.uint64)[None, None, :]
        z = philox.normal(self.seed, stream_id(STREAM_T, self.sys_id), idx)
        aa = self.ao_atom
        cc = self.ri_atom
        s = (self.dist[aa[:, None], aa[None, :]][:, :, None]
             + (self.dist[aa[:, None], cc[None, :]][:, None, :]
                + self.dist[aa[:, None], cc[None, :]][None, :, :]))
        return z * np.exp(-self.k_t * s)

    def states_around_gap(self, n_below: int, n_above: int) -> np.ndarray:
        h = self.n_occ - 1
        return np.arange(h - n_below + 1, self.n_occ + n_above, dtype=np.int32)
