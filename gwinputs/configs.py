"""The synthetic workloads, by name, with their sizes.

  chain12      12-atom chain at 2.5 bohr, 8 AO / 20 RI per atom (96 / 240),
               48 occupied, decays H 0.5 / T 0.3 / V 0.2, no filter,
               10 tau / 10 omega, HOMO and LUMO.
  strip300     300-atom ribbon 7 atoms wide, 13 AO / 40 RI per atom
               (3900 / 12000), half filled, decays 0.8 / 0.8 / 0.2,
               filter 1e-9, 12 tau / 12 omega, HOMO-4 .. LUMO+4.
  strip1000    the same generator at 1000 atoms (13000 / 40000).
  strip1734    the same generator at 1734 atoms, filter 1e-8.
  strip<N>     any other atom count with the strip generator (tests).
  wire<N>      the strip generator on a ribbon one atom wide (a chain of N
               atoms at 2.5 bohr), filter 1e-8: a long quasi-1D system whose
               far output blocks fall below the filter.
  ribbon<N>    the 7-wide strip with 5 AO / 12 RI per atom, filter 1e-8: the
               long-ribbon geometry (e.g. ribbon1734, 620 bohr long) for the
               learned-screener measurement at a basis that allows exact runs.
  mol<M>       M independent molecules for the batched form: atom counts
               drawn uniformly from [10, 40] (mol<M>:<lo>-<hi> for another
               range; Philox uniform, stream 7),
               3D random sequential packings of number density 0.0148 / bohr^3
               with minimum distance 2.5 bohr, 13 AO / 40 RI per atom,
               decays 0.8 / 0.8 / 0.2, filter 1e-9, 12 tau, HOMO / LUMO.
               Molecule m uses sys_id m (its own random streams).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import system as gsys
from . import grids as ggrids


@dataclasses.dataclass
class Workload:
    name: str
    system: gsys.System
    n_tau: int
    n_w: int
    n_below: int        # states: HOMO-(n_below-1) .. LUMO+(n_above-1)
    n_above: int

    def states(self):
        return self.system.states_around_gap(self.n_below, self.n_above)


def chain12(seed=0) -> Workload:
    s = gsys.System(gsys.chain(12), 8, 20, 0.5, 0.3, 0.2, 0.0, seed=seed, n_occ=48)
    return Workload("chain12", s, 10, 10, 1, 1)


def strip(n_atoms: int, seed=0, filter_eps=1e-9, n_ao=13, n_ri=40, n_tau=12,
          n_below=5, n_above=5) -> Workload:
    s = gsys.System(gsys.strip(n_atoms), n_ao, n_ri, 0.8, 0.8, 0.2, filter_eps, seed=seed)
    return Workload(f"strip{n_atoms}", s, n_tau, n_tau, n_below, n_above)


def ribbon(n_atoms: int, seed=0, filter_eps=1e-8, n_tau=12) -> Workload:
    """The 7-wide strip generator with 5 AO / 12 RI per atom and filter 1e-8:
    the geometry of the long-ribbon (1734-atom) screening workload at a basis
    small enough for exact reference runs on one GPU."""
    s = gsys.System(gsys.strip(n_atoms), 5, 12, 0.8, 0.8, 0.2, filter_eps, seed=seed)
    return Workload(f"ribbon{n_atoms}", s, n_tau, n_tau, 5, 5)


def wire(n_atoms: int, seed=0, filter_eps=1e-8, n_tau=12) -> Workload:
    s = gsys.System(gsys.strip(n_atoms, width=1), 13, 40, 0.8, 0.8, 0.2, filter_eps, seed=seed)
    return Workload(f"wire{n_atoms}", s, n_tau, n_tau, 5, 5)


def bulk(n: int, seed=0, filter_eps=1e-9, n_ao=8, n_ri=20, n_tau=12) -> Workload:
    """Periodic Gamma-point cell: n^3 atoms on the simple cubic lattice in a
    cube of side n * SPACING, minimum-image distances for H and the tensor; V
    is the periodic Coulomb matrix of the RI charges (System.ri_charges)."""
    xyz = gsys.cubic_lattice(n)
    s = gsys.System(xyz, n_ao, n_ri, 0.8, 0.8, 0.2, filter_eps, seed=seed,
                    cell=np.full(3, n * gsys.SPACING))
    return Workload(f"bulk{n}", s, n_tau, n_tau, 5, 5)


STREAM_SIZES = 7
STREAM_PACKING = 8


def molecules(n_mol: int, seed=0, lo=10, hi=40, filter_eps=1e-9, n_tau=12, n_ao=13,
              n_ri=40) -> list:
    """The molecule set of the batched form (see the module docstring)."""
    from . import philox
    u = philox.uniform(seed, STREAM_SIZES, np.arange(n_mol))
    sizes = lo + np.minimum((u * (hi - lo + 1)).astype(np.int64), hi - lo)
    out = []
    for m, n in enumerate(sizes):
        xyz = gsys.packing(int(n), seed, STREAM_PACKING + 16 * m)
        s = gsys.System(xyz, n_ao, n_ri, 0.8, 0.8, 0.2, filter_eps, seed=seed, sys_id=m)
        out.append(Workload(f"mol{n_mol}[{m}]", s, n_tau, n_tau, 1, 1))
    return out


def by_name(name: str, seed=0) -> Workload:
    if name == "chain12":
        return chain12(seed)
    if name == "strip1734":
        return strip(1734, seed, filter_eps=1e-8)
    if name.startswith("strip"):
        return strip(int(name[5:]), seed)
    if name.startswith("wire"):
        return wire(int(name[4:]), seed)
    if name.startswith("ribbon"):
        return ribbon(int(name[6:]), seed)
    if name.startswith("bulk"):
        return bulk(int(name[4:]), seed)
    raise KeyError(name)


def molecule_set(name: str, seed=0) -> list:
    """mol<M> (atom counts in [10, 40]) or mol<M>:<lo>-<hi>."""
    head, _, rng = name.partition(":")
    lo, hi = (10, 40) if not rng else (int(x) for x in rng.split("-"))
    return molecules(int(head[3:]), seed, lo=lo, hi=hi)


def grids_for(w: Workload, eps) -> ggrids.Grids:
    return ggrids.make_grids(eps, w.system.n_occ, w.n_tau, w.n_w)


def mu_fermi(eps, n_occ) -> float:
    eps = np.asarray(eps)
    return 0.5 * float(eps[n_occ - 1] + eps[n_occ])
