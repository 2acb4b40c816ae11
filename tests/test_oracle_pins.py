"""Pins of oracle functions that the invariant tests leave open: the block
filter (its norm and its strict < rule, and the error bound of the three
filters of the computational details at a non-zero threshold), the screener
network's forward pass and loss (computed by hand), and the occupied branch
of the Pade nodes (told apart from the virtual one on data that is not
symmetric under conjugation)."""
import numpy as np
import pytest

from oracle import chi as ochi, gt, mlp, qp


# ------------------------------------------------------------ block filter
def _hand_matrix():
    """4 x 4 matrix of 2 x 2 atom blocks with known norms:
    (0,0) = identity: Frobenius sqrt 2 (max-abs 1, spectral 1, sum of |x| 2)
    (0,1) = all 0.6: Frobenius 1.2 (sum of |x| 2.4)
    (1,0) = [[3, 4], [0, 0]]: Frobenius 5 exactly
    (1,1) = zero."""
    x = np.zeros((4, 4))
    x[0:2, 0:2] = np.eye(2)
    x[0:2, 2:4] = 0.6
    x[2, 0], x[2, 1] = 3.0, 4.0
    return x


def test_block_norms_are_frobenius():
    off = [0, 2, 4]
    nrm = ochi.block_norms(_hand_matrix(), off, off)
    np.testing.assert_allclose(nrm, [[np.sqrt(2.0), 1.2], [5.0, 0.0]], rtol=1e-15, atol=0)
    # ragged blocks: rows [0,1), [1,3); columns [0,2), [2,3)
    y = np.arange(1.0, 10.0).reshape(3, 3)
    nrm = ochi.block_norms(y, [0, 1, 3], [0, 2, 3])
    # by hand: (1^2+2^2), 3^2, (4^2+5^2+7^2+8^2), (6^2+9^2)
    np.testing.assert_allclose(nrm, np.sqrt([[5.0, 9.0], [154.0, 117.0]]), rtol=1e-15)


def test_filter_blocks_rule():
    off = [0, 2, 4]
    x = _hand_matrix()
    # eps 1.3: the Frobenius rule keeps (0,0) (sqrt 2) and drops (0,1) (1.2);
    # a max-abs or spectral rule would drop (0,0), a sum-of-|x| rule keep (0,1)
    y = ochi.filter_blocks(x, off, off, 1.3)
    np.testing.assert_array_equal(y[0:2, 0:2], np.eye(2))
    np.testing.assert_array_equal(y[0:2, 2:4], 0.0)
    np.testing.assert_array_equal(y[2:4, 0:2], x[2:4, 0:2])
    # strict <: a block of norm exactly eps is kept, one ulp above drops it
    np.testing.assert_array_equal(ochi.filter_blocks(x, off, off, 5.0)[2:4, 0:2], x[2:4, 0:2])
    np.testing.assert_array_equal(ochi.filter_blocks(x, off, off, np.nextafter(5.0, 6.0))[2:4, 0:2], 0.0)
    # the input is not modified, eps 0 keeps everything
    np.testing.assert_array_equal(ochi.filter_blocks(x, off, off, 0.0), _hand_matrix())
    np.testing.assert_array_equal(x, _hand_matrix())


def test_tensor_filter_rule():
    # two atoms of 1 AO, one RI atom of 2 functions: bricks (a, b, 0) of norm
    # 5 (3, 4), 1 (1, 0), 0.5 (0.3, 0.4) and 2 (0, 2)
    ao_off, ri_off = [0, 1, 2], [0, 2]
    t = np.zeros((2, 2, 2))
    t[0, 0] = (3.0, 4.0)
    t[0, 1] = (1.0, 0.0)
    t[1, 0] = (0.3, 0.4)
    t[1, 1] = (0.0, 2.0)
    y = ochi.filter_t3c(t, ao_off, ri_off, 1.0)
    np.testing.assert_array_equal(y[0, 0], t[0, 0])
    np.testing.assert_array_equal(y[0, 1], t[0, 1])        # norm == eps: kept
    np.testing.assert_array_equal(y[1, 0], 0.0)            # 0.5 < 1: dropped
    np.testing.assert_array_equal(y[1, 1], t[1, 1])
    trip = np.array([[0, 0, 0], [0, 1, 0], [1, 0, 0], [1, 1, 0]])
    bricks = np.stack([t[0, 0], t[0, 1], t[1, 0], t[1, 1]]).reshape(4, 1, 1, 2)
    np.testing.assert_array_equal(ochi.dense_from_bricks(trip, bricks, ao_off, ri_off, 2, 2, 1.0), y)


def test_filter_error_bound():
    """At eps_f > 0 the filtered chi stays within the bound of the multilinear
    expansion of Eq. 3 around the kept blocks.  chi_PQ = -<D^occ T^P, T^Q D^vir>_F
    gives ||chi(D^o, A, B, D^v)||_F <= ||D^o||_2 ||A||_F ||B||_F ||D^v||_2; with
    every input split into kept + dropped parts (the test's own split at eps),
    chi_full - chi_kept is the sum of the terms with at least one dropped part:
        ||chi_kept - chi_full|| <= prod(k_i + d_i) - prod(k_i),
    and the output filter moves chi_kept by less than eps per zeroed block."""
    from gwinputs import configs
    w = configs.strip(8, filter_eps=0.0)
    s = w.system
    C, eps = s.mean_field()
    g = configs.grids_for(w, eps)
    trip = s.triples()
    br = s.bricks(trip)
    full = ochi.dense_from_bricks(trip, br, s.ao_off, s.ri_off, s.n_ao, s.n_ri, 0.0)
    mu = 0.5 * (eps[s.n_occ - 1] + eps[s.n_occ])
    d_occ, d_vir = gt.density_matrices(C, eps, s.n_occ, mu, g.tau)
    eps_f = 1e-4

    def split(x, row_off, col_off):
        k = np.array(x, copy=True)
        for i in range(len(row_off) - 1):
            for j in range(len(col_off) - 1):
                b = k[row_off[i]:row_off[i + 1], col_off[j]:col_off[j + 1]]
                if np.sqrt((b * b).sum()) < eps_f:
                    b[...] = 0.0
        return k, x - k

    tk = np.zeros_like(full)
    for (a, b, c), v in zip(trip, br):
        if np.sqrt((v * v).sum()) >= eps_f:
            tk[s.ao_off[a]:s.ao_off[a + 1], s.ao_off[b]:s.ao_off[b + 1],
               s.ri_off[c]:s.ri_off[c + 1]] = v.reshape(s.n_ao_atom, s.n_ao_atom, s.n_ri_atom)
    td = full - tk
    assert np.count_nonzero(td) > 0 and np.count_nonzero(tk) > 0
    t_k, t_d = np.linalg.norm(tk), np.linalg.norm(td)
    kept_t = ochi.dense_from_bricks(trip, br, s.ao_off, s.ri_off, s.n_ao, s.n_ri, eps_f)
    np.testing.assert_array_equal(kept_t, tk)
    n_blk = (len(s.ri_off) - 1) ** 2
    d_dropped = tight = 0
    for j in range(len(g.tau)):
        dok, dod = split(d_occ[j], s.ao_off, s.ao_off)
        dvk, dvd = split(d_vir[j], s.ao_off, s.ao_off)
        nk = [np.linalg.norm(dok, 2), t_k, t_k, np.linalg.norm(dvk, 2)]
        nd = [np.linalg.norm(dod, 2), t_d, t_d, np.linalg.norm(dvd, 2)]
        bound = np.prod(np.add(nk, nd)) - np.prod(nk) + eps_f * np.sqrt(n_blk)
        dense = ochi.chi_eq3(full, d_occ[j:j + 1], d_vir[j:j + 1])[0]
        filt = ochi.chi_filtered(kept_t, d_occ[j:j + 1], d_vir[j:j + 1], s.ao_off, s.ri_off, eps_f)[0]
        diff = np.linalg.norm(filt - dense)
        assert 0 < diff <= bound * (1 + 1e-12), (j, diff, bound)
        if np.count_nonzero(dod) + np.count_nonzero(dvd) == 0:
            # only bricks and output blocks dropped: the bound is tight enough
            # to mean something (about 1e-4 of chi here)
            tight += 1
            assert bound < 0.02 * np.linalg.norm(dense), (j, bound, np.linalg.norm(dense))
        else:
            d_dropped += 1
    assert d_dropped > 0 and tight > 0


def test_filter_error_bound_sees_a_wrong_rule(monkeypatch):
    """The bound test fails for a filter that drops the wrong blocks (norm >= eps)."""
    from gwinputs import configs
    w = configs.strip(6, filter_eps=0.0)
    s = w.system
    C, eps = s.mean_field()
    g = configs.grids_for(w, eps)
    trip = s.triples()
    full = ochi.dense_from_bricks(trip, s.bricks(trip), s.ao_off, s.ri_off, s.n_ao, s.n_ri, 0.0)
    mu = 0.5 * (eps[s.n_occ - 1] + eps[s.n_occ])
    d_occ, d_vir = gt.density_matrices(C, eps, s.n_occ, mu, g.tau[:1])
    right = ochi.chi_filtered(full, d_occ, d_vir, s.ao_off, s.ri_off, 5e-3)[0]
    orig = ochi.block_norms
    monkeypatch.setattr(ochi, "block_norms", lambda x, r, c: 1.0 / (orig(x, r, c) + 1e-300))
    wrong = ochi.chi_filtered(full, d_occ, d_vir, s.ao_off, s.ri_off, 5e-3)[0]
    dense = ochi.chi_eq3(full, d_occ, d_vir)[0]
    assert np.linalg.norm(right - dense) < 0.05 * np.linalg.norm(dense)
    assert np.linalg.norm(wrong - dense) > 0.5 * np.linalg.norm(dense)


# ------------------------------------------------------- screener network
def _hand_net():
    return {"w1": np.array([[1.0, -1.0], [2.0, 1.0], [0.5, 0.0]]), "b1": np.array([0.0, -1.0, 0.25]),
            "w2": np.array([[1.0, 0.0, 4.0], [-1.0, 1.0, 0.0], [0.0, -2.0, 1.0]]),
            "b2": np.array([0.0, 0.5, 0.0]),
            "w3": np.array([[2.0, -1.0, 7.0]]), "b3": np.array([0.125])}


def test_mlp_forward_by_hand():
    """x = (1, 2): a1 = (-1, 3, 0.75), h1 = (0, 3, 0.75); a2 = (3, 3.5, -5.25),
    h2 = (3, 3.5, 0); y = 6 - 3.5 + 0.125 = 2.625.
    x = (-1, 0): a1 = (-1, -3, -0.25), h1 = 0; h2 = relu(b2) = (0, 0.5, 0);
    y = -0.5 + 0.125 = -0.375."""
    p = _hand_net()
    y, (x, a1, h1, a2, h2) = mlp.forward(p, np.array([[1.0, 2.0], [-1.0, 0.0]]))
    np.testing.assert_array_equal(a1, [[-1.0, 3.0, 0.75], [-1.0, -3.0, -0.25]])
    np.testing.assert_array_equal(h1, [[0.0, 3.0, 0.75], [0.0, 0.0, 0.0]])
    np.testing.assert_array_equal(a2, [[3.0, 3.5, -5.25], [0.0, 0.5, 0.0]])
    np.testing.assert_array_equal(h2, [[3.0, 3.5, 0.0], [0.0, 0.5, 0.0]])
    np.testing.assert_array_equal(y, [2.625, -0.375])


def test_mlp_loss_by_hand():
    """Targets (2, 0): r = (0.625, -0.375); the under-prediction weighs alpha
    = 8: L = (0.390625 + 8 * 0.140625) / 2 = 0.7578125."""
    x = np.array([[1.0, 2.0], [-1.0, 0.0]])
    assert mlp.loss(_hand_net(), x, np.array([2.0, 0.0]), 8.0) == 0.7578125
    # alpha = 1 is the plain mean squared error
    assert mlp.loss(_hand_net(), x, np.array([2.0, 0.0]), 1.0) == (0.390625 + 0.140625) / 2


# --------------------------------------------------------- Pade branches
def test_pade_occupied_branch_conjugates():
    """On data that is not symmetric under conjugation, f(z) = a/(z - b) + c
    with complex a, b, c, the virtual branch (nodes +i w, values f(i w))
    reproduces f on the real axis and the occupied branch (nodes -i w, values
    conj f(i w)) reproduces conj f: f(i w)* is the value at -i w of
    f*(z) = conj(a)/(z - conj(b)) + conj(c), whose real-axis value is conj f(E).
    Nodes -i w with unconjugated values, or +i w with conjugated ones, are not
    a rational of this degree and miss both."""
    a, b, c = 0.3 + 0.2j, 0.5 - 0.4j, -0.1 + 0.05j
    f = lambda z: a / (z - b) + c
    omega = np.geomspace(0.05, 50.0, 12)
    fiw = f(1j * omega)
    E = np.array([-0.7, -0.2, 0.1, 0.45, 0.9])
    for occupied in (False, True):
        zn, fv = qp.pade_nodes(omega, fiw, occupied)
        if occupied:
            np.testing.assert_allclose(zn, -1j * omega, rtol=0, atol=0)
            np.testing.assert_allclose(fv, np.conj(fiw), rtol=0, atol=0)
        coef = qp.thiele_coeffs(zn, fv)
        got = np.array([qp.thiele_eval(zn, coef, e)[0] for e in E])
        want = np.conj(f(E)) if occupied else f(E)
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)
    for zn, fv in ((-1j * omega, fiw), (1j * omega, np.conj(fiw))):
        coef = qp.thiele_coeffs(zn, fv)
        got = np.array([qp.thiele_eval(zn, coef, e)[0] for e in E])
        assert np.abs(got - f(E)).max() > 1e-3 and np.abs(got - np.conj(f(E))).max() > 1e-3
    # the window keeps the nodes with w <= window in both branches
    zn, _ = qp.pade_nodes(omega, fiw, True, window=1.0)
    np.testing.assert_array_equal(zn, -1j * omega[omega <= 1.0])
