import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running (full-size) test")


class Inputs:
    """Seeded synthetic inputs of one workload, generated once per session."""

    def __init__(self, workload, dense=True):
        from gwinputs import configs
        self.w = workload
        s = self.s = workload.system
        self.C, self.eps = s.mean_field()
        self.grids = configs.grids_for(workload, self.eps)
        self.mu_f = configs.mu_fermi(self.eps, s.n_occ)
        self.V = s.coulomb()
        self.trip = s.triples()
        self.bricks = s.bricks(self.trip)
        self.states = workload.states()
        self._dense = None

    @property
    def t3c(self):
        """Dense tensor from the enumerated bricks, bricks below the filter dropped."""
        if self._dense is None:
            from oracle import chi as ochi
            s = self.s
            self._dense = ochi.dense_from_bricks(self.trip, self.bricks, s.ao_off, s.ri_off,
                                                 s.n_ao, s.n_ri, s.filter_eps)
        return self._dense


_CACHE = {}


def get_inputs(name, **kw):
    from gwinputs import configs
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        if name == "chain12":
            w = configs.chain12()
        else:
            w = configs.strip(int(name[5:]), **kw)
        _CACHE[key] = Inputs(w)
    return _CACHE[key]


@pytest.fixture(scope="session")
def chain12():
    return get_inputs("chain12")


@pytest.fixture(scope="session")
def strip_small():
    """A 21-atom ribbon (3 columns) with 5 AO / 12 RI per atom and a filter
    that drops part of the tensor."""
    return get_inputs("strip21", n_ao=5, n_ri=12, filter_eps=1e-4, n_tau=6)


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / den)
