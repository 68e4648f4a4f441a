"""Pins of the FP64 oracle's Newton force against facts the paper and the
mathematics fix (Eq. newton_force, Sec. 3; the potential sign of the kernel in
Sec. 3.3; the self-interaction handling of Sec. 4.1)."""
import numpy as np
import pytest

import oracle
import synth


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def test_two_body_closed_form():
    # a_1 = m_2 d / (|d|^2+eps^2)^{3/2} pointing from 1 to 2; phi_1 = -m_2/(|d|^2+eps^2)^{1/2}
    xi = np.array([0.25], np.float32); yi = np.array([-0.5], np.float32); zi = np.array([1.0], np.float32)
    xj = np.array([1.25], np.float32); yj = np.array([1.5], np.float32); zj = np.array([-1.0], np.float32)
    m = np.array([3.0], np.float32)
    eps2 = np.array([0.0625], np.float32)
    ax, ay, az, phi = oracle.newton(xi, yi, zi, eps2, xj, yj, zj, m)
    d = np.array([1.0, 2.0, -2.0])
    q = 9.0 + 0.0625
    assert np.allclose([ax[0], ay[0], az[0]], 3.0 * d / q ** 1.5, rtol=1e-15, atol=0)
    assert phi[0] == pytest.approx(-3.0 / np.sqrt(q), rel=1e-15)
    # the force points towards the source
    assert ax[0] > 0 and ay[0] > 0 and az[0] < 0


def test_superposition_of_two_sources():
    xi = np.zeros(1, np.float32)
    xj = np.array([1.0, -2.0], np.float32)
    z = np.zeros(2, np.float32)
    m = np.array([1.0, 4.0], np.float32)
    e = np.zeros(1, np.float32)
    ax, ay, az, phi = oracle.newton(xi, xi, xi, e, xj, z, z, m)
    assert ax[0] == pytest.approx(1.0 - 1.0, abs=1e-15)   # 1/1^2 - 4/2^2 = 0
    assert phi[0] == pytest.approx(-(1.0 + 2.0), rel=1e-15)


@pytest.mark.parametrize("n", [7, 64])
def test_third_law_uniform_softening(n):
    # sum_i m_i a_i = 0 for all-pairs with a common eps (the self pair adds no force)
    x, y, z = synth.plummer(n, 11)
    m = (np.arange(1, n + 1) / n).astype(np.float32)
    e = np.full(n, 0.01, np.float32)
    ax, ay, az, _ = oracle.newton(x, y, z, e, x, y, z, m)
    scale = np.sum(m * np.sqrt(ax ** 2 + ay ** 2 + az ** 2))
    for a in (ax, ay, az):
        assert abs(np.sum(m.astype(np.float64) * a)) < 1e-13 * scale


def test_acceleration_is_minus_gradient_of_potential():
    # a_i = -grad_{x_i} phi_i with phi_i the potential from all j != i
    n = 24
    x, y, z = synth.plummer(n, 5)
    m = synth.equal_masses(n)
    eps = 0.05
    e = np.full(n, eps * eps)
    sj = np.arange(n)
    ax, ay, az, _ = oracle.newton(x, y, z, e, x, y, z, m, self_j=sj)
    h = 1e-5 * eps
    for i in range(0, n, 5):
        g = []
        for axis in range(3):
            pos = [np.array([x[i]], np.float64), np.array([y[i]], np.float64), np.array([z[i]], np.float64)]
            plus = [p.copy() for p in pos]; minus = [p.copy() for p in pos]
            plus[axis] += h; minus[axis] -= h
            pp = oracle.newton(*plus, e[:1], x, y, z, m, self_j=[i])[3][0]
            pm = oracle.newton(*minus, e[:1], x, y, z, m, self_j=[i])[3][0]
            g.append(-(pp - pm) / (2 * h))
        a = np.array([ax[i], ay[i], az[i]])
        assert np.allclose(g, a, rtol=1e-7, atol=1e-9 * np.linalg.norm(a))


def test_self_term_identity():
    # raw phi_i (self pair summed) = physical phi_i - m_i/eps_i  (Sec. 4.1)
    n = 33
    x, y, z = synth.plummer(n, 3)
    m = (0.5 + np.arange(n) / n).astype(np.float32)
    e2 = np.full(n, np.float32(0.02) ** 2, np.float32)
    raw = oracle.newton(x, y, z, e2, x, y, z, m)
    phys = oracle.newton(x, y, z, e2, x, y, z, m, self_j=np.arange(n))
    self_term = -m.astype(np.float64) / np.sqrt(e2.astype(np.float64))
    assert np.allclose(raw[3], phys[3] + self_term, rtol=1e-14, atol=0)
    for k in range(3):  # the self pair has d = 0 and adds no force
        assert np.array_equal(raw[k], phys[k])


def test_zero_distance_pair_is_skipped():
    # eps = 0 and a coincident pair: the contribution is defined as 0
    x = np.array([0.0, 1.0], np.float32); z = np.zeros(2, np.float32)
    m = np.ones(2, np.float32); e = np.zeros(2, np.float32)
    ax, ay, az, phi = oracle.newton(x, z, z, e, x, z, z, m)
    assert np.all(np.isfinite(ax)) and np.all(np.isfinite(phi))
    assert ax[0] == pytest.approx(1.0) and phi[0] == pytest.approx(-1.0)


def test_translation_and_permutation_invariance():
    # positions on a dyadic grid so that a shift by 8 is exact in FP32
    rng = np.random.default_rng(0)
    n = 50
    p = (rng.integers(-2048, 2048, size=(3, n)) / 1024.0).astype(np.float32)
    m = rng.random(n).astype(np.float32)
    e = np.full(n, 0.01, np.float32)
    base = oracle.newton(*p, e, *p, m)
    q = p + np.float32(8.0)
    moved = oracle.newton(*q, e, *q, m)
    for a, b in zip(base, moved):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * np.max(np.abs(b)))
    perm = rng.permutation(n)
    pp = p[:, perm]
    permuted = oracle.newton(*pp, e, *pp, m[perm])
    for a, b in zip(base, permuted):
        assert np.allclose(a[perm], b, rtol=1e-12, atol=1e-13 * np.max(np.abs(b)))


def test_brute_force_tiny():
    # an independent pairwise loop in Python (math module, one pair at a time)
    import math
    n = 9
    x, y, z = synth.plummer(n, 21)
    m = (1.0 + np.arange(n)).astype(np.float32)
    e = (0.001 * (1 + np.arange(n))).astype(np.float32)
    ax, ay, az, phi = oracle.newton(x, y, z, e, x, y, z, m)
    for i in range(n):
        acc = [0.0, 0.0, 0.0]; pot = 0.0
        for j in range(n):
            d = [float(x[j]) - float(x[i]), float(y[j]) - float(y[i]), float(z[j]) - float(z[i])]
            r = math.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + float(e[i]))
            for k in range(3):
                acc[k] += float(m[j]) * d[k] / r ** 3
            pot -= float(m[j]) / r
        assert np.allclose([ax[i], ay[i], az[i]], acc, rtol=1e-12)
        assert phi[i] == pytest.approx(pot, rel=1e-12)


def test_items_match_per_group_calls():
    rng = np.random.default_rng(1)
    n = 200
    x, y, z = synth.plummer(n, 2)
    m = synth.equal_masses(n)
    e = np.full(n, 1e-4, np.float32)
    items = np.array([[0, 40, 10, 90], [40, 1, 0, 200], [41, 59, 150, 50]], np.int32)
    got = oracle.newton_items(items, x, y, z, e, x, y, z, m)
    for i0, ni, j0, nj in items:
        ref = oracle.newton(x[i0:i0 + ni], y[i0:i0 + ni], z[i0:i0 + ni], e[i0:i0 + ni],
                            x[j0:j0 + nj], y[j0:j0 + nj], z[j0:j0 + nj], m[j0:j0 + nj])
        for a, b in zip(got, ref):
            assert np.array_equal(a[i0:i0 + ni], b)
    assert np.all(np.isnan(got[0][100:]))  # rows outside every item stay untouched
    del rng


def test_plummer_generator_statistics():
    # the half-mass radius of a Plummer sphere is b / sqrt(2^{2/3} - 1) = 1.3048 b
    x, y, z = synth.plummer(200000, 7)
    r = np.sqrt(x.astype(np.float64) ** 2 + y ** 2 + z ** 2)
    assert np.median(r) == pytest.approx(1.0 / np.sqrt(2 ** (2 / 3) - 1), rel=0.01)
    assert abs(np.mean(x)) < 0.05 and abs(np.mean(z)) < 0.05
