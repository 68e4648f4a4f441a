"""Pins of the FP64 oracle's bit-binned look-up table and table force
(Sec. 3.4.1-3.4.2, Table 4, Eqs. s2 and s2pp, the accuracy test of Sec. 4.2)."""
import json
import math
import os
import struct

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table4_E4F6.json")


def _bits(s):
    u = struct.unpack("<I", struct.pack("<f", s))[0]
    return u


def _bit_index(s, E, F):
    """The paper's definition of the index, written as bit extraction: the
    lower E bits of the exponent followed by the upper F bits of the fraction
    of the FP32 number s."""
    u = _bits(s)
    exp = (u >> 23) & 0xFF
    frac = u & ((1 << 23) - 1)
    return ((exp & ((1 << E) - 1)) << F) | (frac >> (23 - F))


def test_table4_worked_example():
    g = json.load(open(GOLDEN))
    E, F = g["E"], g["F"]
    assert oracle.smax(E, F) == 130048.0
    rcut = 0.046875
    c = (oracle.smax(E, F) - 2.0) / rcut ** 2
    for row in g["rows"]:
        s = c * (row["r_over_rcut"] * rcut) ** 2 + 2.0
        assert s == pytest.approx(row["s_exact"], rel=1e-12)
        assert s == pytest.approx(row["s_printed"], rel=5e-5)
        u = _bits(np.float32(row["s_exact"]))
        assert format((u >> 23) & 0xFF, "08b") == row["exponent_bits"]
        assert format(u & ((1 << 23) - 1), "023b") == row["fraction_bits"]
        k, _ = oracle.lut_index(row["s_exact"], E, F)
        assert k == row["index"]


@pytest.mark.parametrize("E,F", [(4, 6), (4, 5), (4, 2), (0, 3), (3, 0), (6, 8), (1, 1)])
def test_floor_index_equals_bit_extraction(E, F):
    rng = np.random.default_rng(E * 100 + F)
    smax = oracle.smax(E, F)
    s = np.exp(rng.uniform(np.log(2.0), np.log(smax), 3000)).astype(np.float32)
    s = np.concatenate([s, np.float32([2.0, smax])])
    for v in s:
        k, sk = oracle.lut_index(float(v), E, F)
        assert k == _bit_index(float(v), E, F)
        # s_k is s with the low 23-F fraction bits cleared
        assert _bits(np.float32(sk)) == _bits(v) & ~((1 << (23 - F)) - 1)


@pytest.mark.parametrize("E,F", [(4, 6), (4, 5), (2, 3)])
def test_node_round_trip(E, F):
    K = 1 << (E + F)
    for k in range(K):
        sk = oracle.node_s(E, F, k)
        assert oracle.lut_index(sk, E, F) == (k, sk)
        assert (_bits(np.float32(sk)) & ((1 << (23 - F)) - 1)) == 0
        if k + 1 < K:
            below = np.nextafter(oracle.node_s(E, F, k + 1), 0.0)
            assert oracle.lut_index(below, E, F)[0] == k
    assert oracle.node_s(E, F, 0) == 2.0
    assert oracle.node_s(E, F, K - 1) == oracle.smax(E, F)
    assert oracle.node_r(E, F, 0.3, K - 1) == 0.3


def test_node_spacing_asymptotics():
    # Eq. comp_e: r_{bE+1,bF}/r_{bE,bF} -> sqrt(2) for bE >> 1;
    # Eq. comp_f: r_{bE,bF+1} - r_{bE,bF} ~ (2^F+bF)^{-1/2} ((2^{bE+1}/2^{F+2})/(s_max-2))^{1/2}
    E, F, rcut = 6, 8, 1.0
    smax = oracle.smax(E, F)
    for bE in (40, 55):
        for bF in (0, 100, 255):
            k = bE * (1 << F) + bF
            ratio = oracle.node_r(E, F, rcut, k + (1 << F)) / oracle.node_r(E, F, rcut, k)
            assert ratio == pytest.approx(math.sqrt(2.0), rel=1e-9)
    for bE, bF in ((50, 10), (60, 200)):
        k = bE * (1 << F) + bF
        dr = oracle.node_r(E, F, rcut, k + 1) - oracle.node_r(E, F, rcut, k)
        pred = (2 ** F + bF) ** -0.5 * math.sqrt((2.0 ** (bE + 1) / 2.0 ** (F + 2)) / (smax - 2.0))
        assert dr == pytest.approx(pred, rel=5e-3)


def test_s2_profile_continuity_and_limits():
    a = 0.37
    # xi = 1 at r = a/2: both polynomial branches give 97/(35 a^2)
    lo = oracle.s2_R(np.nextafter(a / 2, 0), a)
    hi = oracle.s2_R(a / 2, a)
    assert lo == pytest.approx(97.0 / (35 * a * a), rel=1e-12)
    assert hi == pytest.approx(97.0 / (35 * a * a), rel=1e-12)
    # xi = 2 at r = a: the second branch reaches 1/a^2 = 1/r^2
    assert oracle.s2_R(np.nextafter(a, 0), a) == pytest.approx(1.0 / a ** 2, rel=1e-10)
    assert oracle.s2_R(a, a) == pytest.approx(1.0 / a ** 2, rel=1e-15)
    # small r: R ~ 224 xi/(35 a^2) = 448 r/(35 a^3)
    r = 1e-7 * a
    assert oracle.s2_R(r, a) == pytest.approx(448 * r / (35 * a ** 3), rel=1e-6)
    # the PP shape vanishes at and beyond the cutoff and h(0) is its limit
    eps, rcut = 3.125e-3, 4.6875e-2
    assert oracle.s2pp_f(rcut, eps, rcut) == 0.0
    assert oracle.s2pp_f(2 * rcut, eps, rcut) == 0.0
    h0 = oracle.shape_h(oracle.SHAPE_S2PP, 0.0, eps, rcut)
    assert oracle.shape_h(oracle.SHAPE_S2PP, 1e-6 * eps, eps, rcut) == pytest.approx(h0, rel=1e-8)


@pytest.mark.parametrize("E,F", [(4, 6), (4, 5)])
def test_table_values_at_nodes_and_continuity(E, F):
    eps, rcut = 3.125e-3, 4.6875e-2
    t = oracle.table_build(E, F, rcut, oracle.SHAPE_S2PP, eps)
    K = 1 << (E + F)
    G0, G1 = t[0::2].astype(np.float64), t[1::2].astype(np.float64)
    for k in range(K - 1):
        r = oracle.node_r(E, F, rcut, k)
        exact = oracle.shape_h(oracle.SHAPE_S2PP, r, eps, rcut)
        assert G0[k] == np.float32(exact)
        assert oracle.lut_eval(oracle.node_s(E, F, k), E, F, t) == G0[k]
        # the interpolant is continuous at the next node (to a couple of ulp)
        ds = oracle.node_s(E, F, k + 1) - oracle.node_s(E, F, k)
        end = G0[k] + G1[k] * ds
        assert abs(end - G0[k + 1]) <= 4 * np.spacing(np.float32(max(abs(G0[k]), abs(G0[k + 1]))))
    assert G0[K - 1] == 0.0 and G1[K - 1] == 0.0


def test_paper_table_accuracy_s2():
    """Sec. 4.2 (Fig. 8): 4096 pairs log-uniform in r/rcut on (5e-3, 1),
    eps = 3.125e-3, rcut = 4.6875e-2, m = 1, E = 4, F = 5: the PP force from
    the table plus the exact PM part R(r, rcut) matches R(r, eps) to < 1e-3."""
    eps, rcut = 3.125e-3, 4.6875e-2
    for E, F in ((4, 5), (4, 6)):
        t = oracle.table_build(E, F, rcut, oracle.SHAPE_S2PP, eps)
        dx, dy, dz, r = synth.log_uniform_pairs(4096, 2012, 5e-3 * rcut, rcut)
        n = dx.size
        z = np.zeros(1, np.float32)
        items = np.stack([np.arange(n), np.ones(n), np.arange(n), np.ones(n)], 1).astype(np.int32)
        ax, ay, az, _ = oracle.lut_items(items, np.zeros(n, np.float32), np.zeros(n, np.float32),
                                         np.zeros(n, np.float32), dx, dy, dz,
                                         np.ones(n, np.float32), E, F, rcut, t)
        rr = np.sqrt(dx.astype(np.float64) ** 2 + dy.astype(np.float64) ** 2 + dz.astype(np.float64) ** 2)
        pp = np.sqrt(ax ** 2 + ay ** 2 + az ** 2)
        total = pp + np.array([oracle.s2_R(v, rcut) for v in rr])
        exact = np.array([oracle.s2_R(v, eps) for v in rr])
        err = np.abs(total - exact) / exact
        assert err.max() < 1e-3, (E, F, err.max())
        del z


def test_cutoff_gives_exact_zero():
    eps, rcut, E, F = 1e-3, 0.05, 4, 6
    t = oracle.table_build(E, F, rcut, oracle.SHAPE_S2PP, eps)
    dx = np.array([rcut, 1.0001 * rcut, 3 * rcut, 0.999 * rcut], np.float32)
    n = dx.size
    z = np.zeros(n, np.float32)
    items = np.stack([np.arange(n), np.ones(n), np.arange(n), np.ones(n)], 1).astype(np.int32)
    ax, ay, az, _ = oracle.lut_items(items, z, z, z, dx, z, z, np.ones(n, np.float32), E, F, rcut, t)
    assert np.all(ax[:3] == 0.0)
    assert ax[3] > 0.0


def test_table_of_plummer_shape_matches_newton_inside_half_cutoff():
    """A table of the softened Newtonian f/r (tapered to 0 beyond rcut/2)
    reproduces Eq. newton_force for pairs inside rcut/2 within the table's
    interpolation error."""
    eps, rcut, E, F = 0.01, 0.2, 4, 6
    t = oracle.table_build(E, F, rcut, oracle.SHAPE_PLUMMER_TAPER, eps)
    dx, dy, dz, r = synth.log_uniform_pairs(2000, 9, 1e-3 * rcut, 0.5 * rcut)
    n = dx.size
    z = np.zeros(n, np.float32)
    m = np.ones(n, np.float32)
    items = np.stack([np.arange(n), np.ones(n), np.arange(n), np.ones(n)], 1).astype(np.int32)
    ax, ay, az, _ = oracle.lut_items(items, z, z, z, dx, dy, dz, m, E, F, rcut, t)
    e2 = np.full(1, eps * eps)
    for k in range(0, n, 97):
        ref = oracle.newton(z[:1], z[:1], z[:1], e2, dx[k:k + 1], dy[k:k + 1], dz[k:k + 1], m[:1])
        a = np.array([ax[k], ay[k], az[k]])
        b = np.array([ref[0][0], ref[1][0], ref[2][0]])
        assert np.linalg.norm(a - b) <= 2e-3 * np.linalg.norm(b)


def test_lut_items_match_exact_shape_within_table_error():
    eps, rcut, E, F = 1.0 / 1280, 3.0 / 256, 4, 6
    x, y, z = synth.uniform_box(3000, 4, box=0.05)
    m = synth.equal_masses(3000)
    items = np.array([[0, 3000, 0, 3000]], np.int32)
    t = oracle.table_build(E, F, rcut, oracle.SHAPE_S2PP, eps)
    a_tab = oracle.lut_items(items, x, y, z, x, y, z, m, E, F, rcut, t)
    a_ex = oracle.central_items(items, x, y, z, x, y, z, m, oracle.SHAPE_S2PP, eps, rcut)
    # the paper's measure: error relative to the whole (PP + PM) force
    scale = np.maximum(a_ex[4], 1e-300)
    for k in range(3):
        err = np.abs(a_tab[k] - a_ex[k]) / scale
        assert np.max(err[a_ex[4] > 0]) < 1e-3
    # particles with no neighbour inside rcut feel exactly zero
    lonely = a_ex[3] == 0
    assert np.all(a_tab[0][lonely] == 0) and np.all(a_tab[1][lonely] == 0)


# ---- potential tables (a second table on the force table's bins) ----

def test_soft_cut_shape_pair_is_consistent():
    """h = p'(r)/r for the soft-cut shape (central differences of p in FP64),
    p and h vanish at rcut, and the small-r limits are finite."""
    eps, rcut = 0.01, 0.2
    rng = np.random.default_rng(21)
    for r in np.concatenate([rng.uniform(1e-3, rcut * 0.999, 200), [1e-6, 0.5 * rcut]]):
        d = 1e-5 * max(r, 1e-2)
        dp = (oracle.shape_p(2, r + d, eps, rcut) - oracle.shape_p(2, r - d, eps, rcut)) / (2 * d)
        hr = oracle.shape_h(2, r, eps, rcut) * r
        assert abs(dp - hr) <= 1e-6 * abs(oracle.shape_h(2, 0.0, eps, rcut) * r) + 1e-9, (r, dp, hr)
    assert oracle.shape_p(2, rcut, eps, rcut) == 0.0 and oracle.shape_h(2, rcut, eps, rcut) == 0.0
    assert oracle.shape_p(2, 0.0, eps, rcut) == pytest.approx(-1.0 / eps, rel=1e-15)


@pytest.mark.parametrize("E,F", [(4, 6), (3, 5)])
def test_potential_table_nodes_continuity_and_accuracy(E, F):
    """The potential table holds fl32(p(r_k)) at the nodes, is continuous
    (P0_k + P1_k ds_k = P0_{k+1}), gives 0 beyond rcut, and its
    interpolation over 4096 log-uniform single pairs stays within 1e-3 of
    the exact potential, measured against the whole softened potential
    1/sqrt(r^2 + eps^2) the cut one is part of (near rcut the cut potential
    itself goes to 0, as the force does in the paper's error measure)."""
    eps, rcut = 0.01, 0.2
    K = 1 << (E + F)
    t = oracle.pot_table_build(E, F, rcut, oracle.SHAPE_SOFT_CUT, eps)
    for k in range(0, K - 1, 37):
        rk = oracle.node_r(E, F, rcut, k)
        assert t[2 * k] == np.float32(oracle.shape_p(2, rk, eps, rcut))
    nodes = np.array([oracle.node_s(E, F, k) for k in range(K)])
    cont = t[0:-2:2].astype(np.float64) + t[1:-2:2] * np.diff(nodes)
    assert np.allclose(cont, t[2::2], rtol=3e-7, atol=3e-7 * abs(t[0]))
    rng = np.random.default_rng(22)
    r = rcut * 10.0 ** rng.uniform(-2.5, 0.0, 4096)
    n = r.size
    xi = np.zeros(n); yi = np.zeros(n); zi = np.zeros(n)
    items = np.array([[k, 1, k, 1] for k in range(n)], np.int32)
    phi, _ = oracle.lut_pot_items(items, xi, yi, zi, r, np.zeros(n), np.zeros(n), np.ones(n),
                                  E, F, rcut, t)
    exact = np.array([oracle.shape_p(2, rr, eps, rcut) for rr in r])
    err = np.abs(phi - exact) * np.sqrt(r * r + eps * eps)
    assert err.max() < 1e-3, err.max()
    far, _ = oracle.lut_pot_items(np.array([[0, 1, 0, 1]], np.int32), [0.0], [0.0], [0.0],
                                  [1.5 * rcut], [0.0], [0.0], [2.0], E, F, rcut, t)
    assert far[0] == 0.0


def test_ht_form_is_one_rounding_of_the_paper_form():
    """The (H, G1) form of the table (the "htab" kernel variants): g =
    H_k + G1_k s with H_k = G0_k - G1_k s_k rounded once to FP32.  For the
    S2 table (E = 4, F = 6): every H_k is an FP32 number, it equals the
    rounding computed independently in extended precision, it lies within
    half an ulp of the exact G0_k - G1_k s_k, the last node stays zero, and
    the form still meets the accuracy measure of Sec. 4.2 (1e-3 of the
    softened force, over 4096 log-uniform pairs)."""
    from fractions import Fraction
    E, F, eps, rcut = 4, 6, 3.125e-3, 4.6875e-2
    K = 1 << (E + F)
    t = oracle.table_build(E, F, rcut, oracle.SHAPE_S2PP, eps)
    h = oracle.table_ht(t, E, F)
    g0, g1 = t[0::2], t[1::2]
    sk = [oracle.node_s(E, F, k) for k in range(K)]
    for k in range(K):
        H = Fraction(float(h[2 * k])) - Fraction(float(g1[k])) * Fraction(sk[k])
        assert float(H) == float(np.float32(float(H))) and Fraction(float(H)) == H, k
        exact = Fraction(float(g0[k])) - Fraction(float(g1[k])) * Fraction(sk[k])
        half_ulp = Fraction(abs(float(np.spacing(np.float32(float(H)))))) / 2
        assert abs(H - exact) <= half_ulp, k
        ld = np.float32(np.longdouble(g0[k]) - np.longdouble(g1[k]) * np.longdouble(sk[k]))
        assert ld == np.float32(float(H)), k
        assert h[2 * k + 1] == g1[k]
    assert h[-2] == 0.0 and h[-1] == 0.0
    dx, dy, dz, r = synth.log_uniform_pairs(4096, 2012, 5e-3 * rcut, rcut)
    n = r.size
    items = np.array([[k, 1, 0, 1] for k in range(n)], np.int32)
    o = np.zeros(1)
    a = oracle.lut_items(items, dx, dy, dz, o, o, o, np.ones(1), E, F, rcut, h)
    rr = np.sqrt(dx.astype(np.float64) ** 2 + dy.astype(np.float64) ** 2
                 + dz.astype(np.float64) ** 2)
    pp = np.sqrt(a[0] ** 2 + a[1] ** 2 + a[2] ** 2)
    total = pp + np.array([oracle.s2_R(v, rcut) for v in rr])
    exact = np.array([oracle.s2_R(v, eps) for v in rr])
    assert np.max(np.abs(total - exact) / exact) < 1e-3


def _nearest_f32(fr):
    """The FP32 number nearest to the rational fr, ties to an even last bit
    (one correctly rounded operation, as IEEE arithmetic gives)."""
    from fractions import Fraction
    f = np.float32(float(fr))
    best = None
    for c in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        key = (abs(Fraction(float(c)) - fr), _bits(c) & 1)
        if best is None or key < best[0]:
            best = (key, c)
    return best[1]


@pytest.mark.parametrize("E,F,rcut", [(4, 6, 3.0 / 256), (4, 5, 4.6875e-2), (3, 8, 0.2),
                                      (6, 7, 1.0 / 32), (2, 10, 0.06)])
def test_fp32_scale_is_the_smallest_float_reaching_smax(E, F, rcut):
    """The oracle's FP32 scale c_f: fl(fl(rcut^2) c_f + 2) reaches s_max and
    the next smaller float does not (one rounding, from exact rationals),
    and c_f lies within a few ulps of (s_max - 2)/rcut^2."""
    from fractions import Fraction
    r = np.float32(rcut)
    r2 = _nearest_f32(Fraction(float(r)) ** 2)
    smaxf = np.float32(oracle.smax(E, F))
    c = np.float32(oracle.scale_f32(E, F, float(r)))

    def s_of(cv):
        return _nearest_f32(Fraction(float(r2)) * Fraction(float(cv)) + 2)

    assert s_of(c) >= smaxf
    assert s_of(np.nextafter(c, np.float32(0))) < smaxf
    exact = (Fraction(oracle.smax(E, F)) - 2) / Fraction(float(r)) ** 2
    assert abs(Fraction(float(c)) - exact) <= 4 * Fraction(float(np.spacing(c)))


@pytest.mark.parametrize("E,F,rcut", [(4, 6, 3.0 / 256), (3, 8, 0.2)])
def test_pair_bin_is_the_fp32_decision(E, F, rcut):
    """The bin every table function of the oracle uses is the bit index of
    the FP32 s (Sec. 3.4.2 reads it off the bits): d by FP32 subtractions,
    |d|^2 and s by single-rounding fused multiply-adds (emulated here from
    exact rationals), clamped at s_max.  Random pairs, and pairs placed at
    node radii, where the FP32 and the double s can fall on either side of a
    node: there the two decisions differ, and only there (s within a few FP32
    roundings of the node)."""
    from fractions import Fraction
    rng = np.random.default_rng(11 + F)
    r = np.float32(rcut)
    c = np.float32(oracle.scale_f32(E, F, float(r)))
    smax = oracle.smax(E, F)
    smaxf = np.float32(smax)
    K = 1 << (E + F)
    pairs = [rng.random(6).astype(np.float32) * np.float32(0.8 * rcut) for _ in range(1500)]
    for k in range(1, K, max(1, K // 300)):  # along x at the radius of node k
        xj = np.float32(oracle.node_r(E, F, float(r), k))
        pairs.append(np.array([0, 0, 0, xj, 0, 0], np.float32))
    pairs.append(np.array([0, 0, 0, r, 0, 0], np.float32))          # exactly rcut
    pairs.append(np.array([0, 0, 0, r * np.float32(1.5), 0, 0], np.float32))
    flips = 0
    for p in pairs:
        d = [np.float32(p[3 + a] - p[a]) for a in range(3)]
        r2 = _nearest_f32(Fraction(float(d[0])) ** 2)
        r2 = _nearest_f32(Fraction(float(d[1])) ** 2 + Fraction(float(r2)))
        r2 = _nearest_f32(Fraction(float(d[2])) ** 2 + Fraction(float(r2)))
        s = _nearest_f32(Fraction(float(r2)) * Fraction(float(c)) + 2)
        clamped = bool(s >= smaxf)
        s = min(s, smaxf)
        want = _bit_index(s, E, F)
        k, sk, cl = oracle.pair_bin(*[float(v) for v in p], E, F, float(r))
        assert (k, cl) == (want, clamped), (p, k, want)
        assert sk == oracle.node_s(E, F, k)
        # the decision from s in double (the pair's own d, the exact scale)
        sd = (smax - 2.0) / float(r) ** 2 * sum(float(v) ** 2 for v in d) + 2.0
        kd, _ = oracle.lut_index(min(sd, smax), E, F)
        if kd != k:
            flips += 1
            edge = oracle.node_s(E, F, max(k, kd))
            assert abs(sd - edge) <= 4 * float(np.spacing(np.float32(edge))), (p, k, kd)
    assert flips > 0  # the node-radius pairs reach both sides
