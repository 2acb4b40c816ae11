"""Pins of the oracle's Gaussian integrals (oracle/integrals.py, Eq. 4 and
the overlap metric of Eq. 5) by numerical quadrature and limits."""
import numpy as np

from oracle import integrals as oint


def _quad3(fs, lo=-14.0, hi=14.0, n=4001):
    """Integral over R^3 of a product of s Gaussians [(centre, exponent, norm)]:
    the integrand factorizes along x, y and z, each factor integrated by the
    trapezoidal rule on a uniform grid (spectrally accurate for Gaussians)."""
    x = np.linspace(lo, hi, n)
    h = x[1] - x[0]
    total = 1.0
    for ax in range(3):
        f = np.ones_like(x)
        for r, a, _ in fs:
            f = f * np.exp(-a * (x - r[ax]) ** 2)
        total *= h * (f.sum() - 0.5 * (f[0] + f[-1]))
    for _, a, _ in fs:
        total *= (2.0 * a / np.pi) ** 0.75
    return total


def test_three_center_by_quadrature():
    rng = np.random.default_rng(5)
    for _ in range(12):
        r = rng.uniform(-2.0, 2.0, (3, 3))
        e = rng.uniform(0.1, 3.0, 3)
        want = _quad3([(r[0], e[0], 0), (r[1], e[1], 0), (r[2], e[2], 0)])
        got = oint.three_center(r[0], e[0], r[1], e[1], r[2], e[2])
        assert abs(got - want) <= 1e-12 * max(abs(want), 1e-300) + 1e-16, (got, want)


def test_overlap_by_quadrature_and_normalization():
    xyz = np.array([[0.0, 0.0, 0.0], [1.3, -0.4, 0.7]])
    exps = np.array([0.3, 1.1])
    offs = np.array([[0.0, 0.0, 0.0], [0.2, 0.1, -0.3]])
    S = oint.overlap(xyz, exps, offs)
    centres = (xyz[:, None, :] + offs[None]).reshape(-1, 3)
    a = np.tile(exps, 2)
    for i in range(4):
        for j in range(4):
            want = _quad3([(centres[i], a[i], 0), (centres[j], a[j], 0)])
            assert abs(S[i, j] - want) <= 1e-12
    np.testing.assert_allclose(np.diag(S), 1.0, rtol=1e-14)
    assert np.allclose(S, S.T) and np.linalg.eigvalsh(S).min() > 0


def test_bricks_layout_symmetry_and_diffuse_limit():
    xyz = np.array([[0.0, 0.0, 0.0], [2.5, 0.0, 0.0], [0.0, 2.5, 0.0]])
    ao_e, ao_o = np.array([0.4, 1.5]), np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.2]])
    ri_e, ri_o = np.array([0.2, 0.9, 2.0]), np.array([[0.0, 0.0, 0.0], [0.0, 0.3, 0.0],
                                                      [-0.2, 0.0, 0.1]])
    trip = np.array([[0, 1, 2], [1, 0, 2], [2, 2, 0]])
    b = oint.bricks(xyz, trip, ao_e, ao_o, ri_e, ri_o)
    assert b.shape == (3, 2, 2, 3)
    # (a, b, c) and (b, a, c) are transposes in (mu, nu)
    np.testing.assert_allclose(b[0], b[1].transpose(1, 0, 2), rtol=1e-14, atol=0)
    # every element equals the single-function formula
    for t, (ia, ib, ic) in enumerate(trip):
        for m in range(2):
            for n in range(2):
                for p in range(3):
                    one = oint.three_center(xyz[ia] + ao_o[m], ao_e[m], xyz[ib] + ao_o[n], ao_e[n],
                                            xyz[ic] + ri_o[p], ri_e[p])
                    assert abs(b[t, m, n, p] - one) <= 1e-15 * one
    # element (mu, nu, P) of brick (a, b, c) by quadrature
    want = _quad3([(xyz[0] + ao_o[1], ao_e[1], 0), (xyz[1] + ao_o[0], ao_e[0], 0),
                   (xyz[2] + ri_o[2], ri_e[2], 0)])
    assert abs(b[0, 1, 0, 2] - want) <= 1e-12 * want
    # a very diffuse third function c -> 0 is nearly constant over the
    # product of the first two: (mu nu P) -> N_c (pi/...) ... = N_c S_mu nu
    c = 1e-8
    s_mn = oint.overlap(xyz[:2], np.array([0.7]), np.zeros((1, 3)))[0, 1]
    got = oint.three_center(xyz[0], 0.7, xyz[1], 0.7, np.array([0.3, 0.1, 0.0]), c)
    assert abs(got / ((2 * c / np.pi) ** 0.75) - s_mn) <= 1e-6 * s_mn
