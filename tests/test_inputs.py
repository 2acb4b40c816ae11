"""Seeded input generator: Philox definition, ranges, symmetry, enumeration."""
import os

import numpy as np
import pytest

from gwinputs import philox, system as gsys, configs, grids as ggrids

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*v[:4], v[4], v[5])
        assert [int(o) for o in out] == v[6:]


def test_normal_range_and_moments():
    z = philox.normal(0, 3, np.arange(400000))
    assert np.abs(z).max() <= philox.Z_MAX
    assert abs(z.mean()) < 5e-3 and abs(z.std() - 1) < 5e-3
    # counter-based: any subrange reproduces the same values
    assert np.array_equal(z[1234:1300], philox.normal(0, 3, np.arange(1234, 1300)))
    assert not np.array_equal(z[:100], philox.normal(1, 3, np.arange(100)))


def test_brick_symmetry_and_dense_agree():
    w = configs.strip(9, n_ao=3, n_ri=4, filter_eps=0.0)
    s = w.system
    t = s.dense_t3c()
    assert np.array_equal(t, t.transpose(1, 0, 2))
    trip = s.triples()
    assert len(trip) == s.n_atoms ** 3
    b = s.bricks(trip)
    for (a, bb, c), v in zip(trip[::37], b[::37]):
        ref = t[s.ao_off[a]:s.ao_off[a + 1], s.ao_off[bb]:s.ao_off[bb + 1], s.ri_off[c]:s.ri_off[c + 1]]
        assert np.array_equal(v.reshape(ref.shape), ref)
        assert np.array_equal(s.brick(a, bb, c), ref)


def test_enumeration_drops_only_subfilter_bricks():
    w = configs.strip(21, n_ao=3, n_ri=4, filter_eps=1e-3)
    s = w.system
    trip = set(map(tuple, s.triples()))
    assert len(trip) < s.n_atoms ** 3
    for (a, b, c) in trip:
        assert (b, a, c) in trip
    rng = np.random.default_rng(0)
    dropped = [(a, b, c) for a in range(s.n_atoms) for b in range(s.n_atoms)
               for c in range(s.n_atoms) if (a, b, c) not in trip]
    for k in rng.choice(len(dropped), 200, replace=False):
        v = s.brick(*dropped[k])
        assert np.sqrt((v * v).sum()) < s.filter_eps


def test_h_and_v():
    s = configs.chain12().system
    h = s.hamiltonian()
    assert np.array_equal(h, h.T)
    v = s.coulomb()
    assert np.linalg.eigvalsh(v).min() > 0.5
    C, eps = s.mean_field()
    assert np.all(np.diff(eps) >= 0)
    assert np.allclose(C @ C.T, np.eye(s.n_ao), atol=1e-12)


def test_grid_weights_fit_their_targets(chain12):
    g = chain12.grids
    assert np.all(np.diff(g.tau) > 0) and np.all(np.diff(g.omega) > 0)
    x = np.geomspace(g.x_lo, g.x_hi, 997)
    e = np.exp(-np.outer(x, g.tau))
    for k, wk in enumerate(g.omega):
        fit = e @ g.cos_w[k]
        true = x / (x * x + wk * wk)
        assert np.all(fit > 0)                      # keeps chi(i w) negative definite
        assert np.max(np.abs(fit / true - 1)) < 0.5
    lap = (e @ g.lap_w) * x
    assert np.max(np.abs(lap - 1)) < 0.5


def test_non_orthogonal_and_periodic_inputs():
    """Gaussian metrics are SPD with unit diagonal; the generalized
    eigenvectors are S_ao-orthonormal; a periodic cell has symmetric
    minimum-image distances no longer than half its diagonal; the RI charges
    sit off the atoms on their sphere."""
    from gwinputs import configs
    s = configs.chain12().system
    for S in (s.ri_metric(), s.ao_metric()):
        np.testing.assert_allclose(S, S.T, rtol=0, atol=0)
        np.testing.assert_allclose(np.diag(S), 1.0, rtol=0, atol=0)
        assert np.linalg.eigvalsh(S).min() > 0.05
    Sa = s.ao_metric()
    C, eps = s.mean_field_nonorth(Sa)
    np.testing.assert_allclose(C @ Sa @ C.T, np.eye(s.n_ao), rtol=0, atol=1e-12)
    assert np.all(np.diff(eps) >= 0)
    b = configs.bulk(3, n_ao=5, n_ri=12).system
    np.testing.assert_allclose(b.dist, b.dist.T, rtol=0, atol=0)
    assert b.dist.max() <= 0.5 * np.linalg.norm(b.cell) + 1e-12
    # atoms (0, 0, 0) and (2, 0, 0) are neighbours through the cell boundary
    assert abs(b.dist[0, 18] - 2.5) < 1e-12
    R, a = b.ri_charges()
    assert R.shape == (b.n_ri, 3) and a.shape == (b.n_ri,)
    off = R.reshape(b.n_atoms, b.n_ri_atom, 3) - b.xyz[:, None, :]
    np.testing.assert_allclose(np.linalg.norm(off, axis=-1), 0.8, rtol=0, atol=1e-12)
    assert a.min() == 0.5 and abs(a.max() - 2.0) < 1e-12
    # open-shell inputs: delta = zeeman = 0 gives the closed shell
    (cu, eu), (cd, ed) = s.mean_field_spin(0.0)
    C0, e0 = s.mean_field()
    np.testing.assert_allclose(eu, e0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ed, e0, rtol=0, atol=1e-12)
