"""Pins of the FP64 oracle's adjoints of L = sum_i w_i . a_i against central
finite differences of the oracle's own forward sums (which are pinned
against the paper in the other oracle tests)."""
import numpy as np
import pytest

import oracle
import synth


def _loss_newton(xi, yi, zi, e2, xj, yj, zj, mj, w):
    ax, ay, az, _ = oracle.newton(xi, yi, zi, e2, xj, yj, zj, mj)
    return float(np.sum(w[0] * ax + w[1] * ay + w[2] * az))


def _setup(ni=7, nj=9, seed=3):
    rng = np.random.default_rng(seed)
    xi = [a.astype(np.float64) for a in synth.plummer(ni, seed)]
    xj = [a.astype(np.float64) for a in synth.plummer(nj, seed + 1)]
    mj = rng.uniform(0.2, 1.0, nj)
    e2 = rng.uniform(0.01, 0.04, ni)
    w = [rng.standard_normal(ni) for _ in range(3)]
    return xi, xj, mj, e2, w


def test_newton_position_gradients_match_central_differences():
    xi, xj, mj, e2, w = _setup()
    g = oracle.newton_bwd(*xi, e2, *xj, mj, *w)
    gxi, gxj = np.stack(g[0:3]), np.stack(g[3:6])
    h = 1e-5
    for ax in range(3):
        for i in range(len(xi[0])):
            p = [a.copy() for a in xi]; m = [a.copy() for a in xi]
            p[ax][i] += h; m[ax][i] -= h
            fd = (_loss_newton(*p, e2, *xj, mj, w) - _loss_newton(*m, e2, *xj, mj, w)) / (2 * h)
            assert fd == pytest.approx(gxi[ax, i], rel=1e-7, abs=1e-7 * np.abs(gxi).max())
        for j in range(len(xj[0])):
            p = [a.copy() for a in xj]; m = [a.copy() for a in xj]
            p[ax][j] += h; m[ax][j] -= h
            fd = (_loss_newton(*xi, e2, *p, mj, w) - _loss_newton(*xi, e2, *m, mj, w)) / (2 * h)
            assert fd == pytest.approx(gxj[ax, j], rel=1e-7, abs=1e-7 * np.abs(gxj).max())


def test_newton_mass_gradient_is_exact_for_a_linear_loss():
    xi, xj, mj, e2, w = _setup(5, 6, 11)
    gmj = oracle.newton_bwd(*xi, e2, *xj, mj, *w)[6]
    for j in range(len(mj)):
        p = mj.copy(); p[j] += 0.5
        m = mj.copy(); m[j] -= 0.5
        fd = (_loss_newton(*xi, e2, *xj, p, w) - _loss_newton(*xi, e2, *xj, m, w)) / 1.0
        assert fd == pytest.approx(gmj[j], rel=1e-11, abs=1e-12 * np.abs(gmj).max())


def test_shared_set_gradient_is_sum_of_both_roles():
    """With i-set = j-set (all pairs, one eps) moving particle k moves it as a
    target and as a source: dL/dx_k = gxi_k + gxj_k (the quantity the fused
    all-pairs adjoint computes)."""
    n = 8
    x = [a.astype(np.float64) for a in synth.plummer(n, 5)]
    m = np.linspace(0.3, 1.1, n)
    e2 = np.full(n, 0.02)
    w = [np.random.default_rng(2).standard_normal(n) for _ in range(3)]
    g = oracle.newton_bwd(*x, e2, *x, m, *w)
    tot = np.stack(g[0:3]) + np.stack(g[3:6])
    h = 1e-5
    for ax in range(3):
        for k in range(n):
            p = [a.copy() for a in x]; q = [a.copy() for a in x]
            p[ax][k] += h; q[ax][k] -= h
            fd = (_loss_newton(*p, e2, *p, m, w) - _loss_newton(*q, e2, *q, m, w)) / (2 * h)
            assert fd == pytest.approx(tot[ax, k], rel=1e-7, abs=1e-7 * np.abs(tot).max())


def test_table_gradients_are_exact_for_a_linear_loss():
    E, F, rcut, eps = 3, 3, 0.3, 0.02
    t = oracle.table_build(E, F, rcut, oracle.SHAPE_S2PP, eps).astype(np.float64)
    n = 40
    x, y, z = [a.astype(np.float64) for a in synth.uniform_box(n, 8, box=0.5)]
    mj = np.linspace(0.5, 1.5, n)
    w = [np.random.default_rng(4).standard_normal(n) for _ in range(3)]
    items = np.array([[0, 20, 0, 40], [20, 20, 10, 25]], np.int32)
    gt, gm = oracle.lut_bwd_items(items, x, y, z, x, y, z, mj, *w, E, F, rcut, t)

    def loss(tab, m):
        ax, ay, az, _ = oracle.lut_items(items, x, y, z, x, y, z, m, E, F, rcut, tab)
        return float(np.sum(w[0] * ax + w[1] * ay + w[2] * az))

    scale_t = np.abs(gt).max()
    for k in range(t.size):
        p = t.copy(); p[k] += 1.0
        q = t.copy(); q[k] -= 1.0
        fd = (loss(p, mj) - loss(q, mj)) / 2.0
        assert fd == pytest.approx(gt[k], rel=1e-9, abs=1e-12 * scale_t)
    assert np.any(gt[0::2] != 0) and np.any(gt[1::2] != 0)
    for j in range(n):
        p = mj.copy(); p[j] += 0.25
        q = mj.copy(); q[j] -= 0.25
        fd = (loss(t, p) - loss(t, q)) / 0.5
        assert fd == pytest.approx(gm[j], rel=1e-9, abs=1e-12 * np.abs(gm).max())


def test_error_scales_bound_the_sums_and_see_inside_the_dot_product():
    """The absolute-term scales used by the GPU error gates bound their sums
    (triangle inequality), and they stay of the size of the products even
    when w_i . d cancels: a weight perpendicular to d gives w . d = 0 but a
    scale of |w_x d_x| + |w_y d_y| + |w_z d_z|."""
    xi, xj, mj, e2, w = _setup(ni=6, nj=8, seed=11)
    r = oracle.newton_bwd(*xi, e2, *xj, mj, *w, scales=True)
    gi, gj, gm, si, sj, sm = np.stack(r[0:3]), np.stack(r[3:6]), r[6], r[7], r[8], r[9]
    assert np.all(np.linalg.norm(gi, axis=0) <= si * (1 + 1e-12))
    assert np.all(np.linalg.norm(gj, axis=0) <= sj * (1 + 1e-12))
    assert np.all(np.abs(gm) <= sm * (1 + 1e-12))
    # one i, one j; w perpendicular to d = (1, 1, 0): w = (1, -1, 0)
    one = [np.array([0.0]) for _ in range(3)]
    r = oracle.newton_bwd(*one, np.array([0.0]), np.array([1.0]), np.array([1.0]),
                          np.array([0.0]), np.array([2.0]), np.array([1.0]), np.array([-1.0]),
                          np.array([0.0]), scales=True)
    rho3 = 2.0 ** -1.5
    assert r[6][0] == 0.0 and r[9][0] == pytest.approx(2 * rho3, rel=1e-14)
    # table adjoint
    E, F, rcut, eps = 3, 3, 0.3, 0.02
    t = oracle.table_build(E, F, rcut, oracle.SHAPE_S2PP, eps).astype(np.float64)
    n = 40
    x, y, z = [a.astype(np.float64) for a in synth.uniform_box(n, 8, box=0.5)]
    m = np.linspace(0.5, 1.5, n)
    wt = [np.random.default_rng(4).standard_normal(n) for _ in range(3)]
    items = np.array([[0, 20, 0, 40], [20, 20, 10, 25]], np.int32)
    gt, gmj, at, am = oracle.lut_bwd_items(items, x, y, z, x, y, z, m, *wt, E, F, rcut, t,
                                           scales=True)
    assert np.all(np.abs(gt) <= at * (1 + 1e-12))
    assert np.all(np.abs(gmj) <= am * (1 + 1e-12))


def test_table_gradient_chain_to_node_values_matches_central_differences():
    """A table parametrised by its node values G0_k, slopes G1_k = chord to
    the next node (Sec. 3.4.1) and G1_{K-1} = 0: the loss is linear in G0,
    so central differences through oracle.lut_items are exact, and they must
    equal table_grad_chain applied to the (G0, G1) gradient."""
    E, F, rcut = 2, 2, 0.4
    K = 1 << (E + F)
    nodes = np.array([oracle.node_s(E, F, k) for k in range(K)])
    rng = np.random.default_rng(12)
    g0 = rng.uniform(-1.0, 1.0, K)

    def table_of(v):
        t = np.zeros(2 * K)
        t[0::2] = v
        t[1:2 * K - 2:2] = (v[1:] - v[:-1]) / (nodes[1:] - nodes[:-1])
        return t

    n = 30
    x, y, z = [a.astype(np.float64) for a in synth.uniform_box(n, 13, box=0.6)]
    m = np.linspace(0.5, 1.5, n)
    w = [rng.standard_normal(n) for _ in range(3)]
    items = np.array([[0, 15, 0, 30], [15, 15, 5, 20]], np.int32)

    def loss(v):
        ax, ay, az, _ = oracle.lut_items(items, x, y, z, x, y, z, m, E, F, rcut, table_of(v))
        return float(np.sum(w[0] * ax + w[1] * ay + w[2] * az))

    gt, _ = oracle.lut_bwd_items(items, x, y, z, x, y, z, m, *w, E, F, rcut, table_of(g0))
    chained = oracle.table_grad_chain(E, F, gt)
    fd = np.zeros(K)
    for k in range(K):
        p = g0.copy(); p[k] += 0.5
        q = g0.copy(); q[k] -= 0.5
        fd[k] = loss(p) - loss(q)
    assert np.allclose(chained, fd, rtol=1e-9, atol=1e-12 * np.abs(fd).max())
    assert np.any(gt[1::2] != 0)  # the slope terms take part


def test_table_position_gradients_match_central_differences():
    """The table force is piecewise smooth in the positions (g is linear in
    s inside a bin, s = c |d|^2 + 2): central differences of the oracle's
    forward sum, with h small enough that no pair crosses a node, equal
    gxi + gxj of a particle that is both an i- and a j-particle."""
    E, F, rcut, eps = 3, 3, 0.3, 0.02
    t = oracle.table_build(E, F, rcut, oracle.SHAPE_S2PP, eps).astype(np.float64)
    n = 40
    x, y, z = [a.astype(np.float64) for a in synth.uniform_box(n, 8, box=0.5)]
    m = np.linspace(0.5, 1.5, n)
    w = [np.random.default_rng(4).standard_normal(n) for _ in range(3)]
    items = np.array([[0, 20, 0, 40], [20, 20, 10, 25]], np.int32)
    g = oracle.lut_bwd_pos_items(items, x, y, z, x, y, z, m, *w, E, F, rcut, t, scales=True)
    tot = np.stack(g[0:3]) + np.stack(g[3:6])
    scale = g[6] + g[7]

    def loss(P):
        ax, ay, az, _ = oracle.lut_items(items, *P, *P, m, E, F, rcut, t)
        return float(np.sum(w[0] * ax + w[1] * ay + w[2] * az))

    h = 1e-8
    X = [x, y, z]
    for ax_ in range(3):
        for k in range(n):
            p = [a.copy() for a in X]; q = [a.copy() for a in X]
            p[ax_][k] += h; q[ax_][k] -= h
            fd = (loss(p) - loss(q)) / (2 * h)
            assert abs(fd - tot[ax_, k]) <= 1e-6 * max(scale[k], 1e-12), (ax_, k, fd, tot[ax_, k])
    assert np.abs(tot).max() > 0
    assert np.all(np.linalg.norm(np.stack(g[0:3]), axis=0) <= g[6] * (1 + 1e-12))
