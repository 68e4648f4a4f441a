"""Pins of the FP64 tree oracle (the Barnes-Hut tree of the paper's tree-code
experiment, Sec. 5) against definitions and facts outside it: an independent
recursive build of the octree, numpy's weighted moments and symmetric
eigen-solver, the multipole orders of the pseudo-particle sets, the covering
and opening properties every interaction list must have, the theta = 0 limit
(the direct sum) and the ordering of the tree-force errors."""
import numpy as np
import pytest

import oracle
import synth


def _sorted_inputs(n, seed, n_leaf=8, quad=False):
    x, y, z = synth.plummer(n, seed)
    m = synth.equal_masses(n)
    return (x, y, z, m), oracle.tree_build(x, y, z, m, n_leaf=n_leaf, quad=quad)


def _morton_python(kx, ky, kz):
    """Bit interleave written independently: bit b of x goes to 3b + 2."""
    k = 0
    for b in range(21):
        k |= ((kx >> b) & 1) << (3 * b + 2)
        k |= ((ky >> b) & 1) << (3 * b + 1)
        k |= ((kz >> b) & 1) << (3 * b)
    return k


def test_keys_and_order():
    (x, y, z, m), t = _sorted_inputs(500, 1)
    lo = np.array([x.min(), y.min(), z.min()], np.float32)
    ext = np.float32(max(x.max() - x.min(), y.max() - y.min(), z.max() - z.min()))
    assert np.all(t.frame[:3] == lo) and t.frame[3] == ext
    scale = np.float32(2.0 ** 21) / ext
    assert t.frame[4] == scale
    for r in range(0, 500, 37):
        i = t.perm[r]
        ks = []
        for v, l in ((x[i], lo[0]), (y[i], lo[1]), (z[i], lo[2])):
            c = int(np.floor(np.float32(np.float32(v - l) * scale)))
            ks.append(min(max(c, 0), 2 ** 21 - 1))
        assert int(t.keys[r]) == _morton_python(*ks)
    # sorted by (key, index)
    pairs = list(zip(t.keys.tolist(), t.perm.tolist()))
    assert pairs == sorted(pairs)
    assert sorted(t.perm.tolist()) == list(range(500))


def _recursive_tree(keys, n_leaf):
    """(begin, count, level) of every node, breadth first by level then key."""
    out = []

    def rec(b, c, L):
        out.append((L, b, c))
        if c <= n_leaf or L == 21:
            return
        shift = 3 * (21 - (L + 1))
        for dg in range(8):
            idx = [r for r in range(b, b + c) if (int(keys[r]) >> shift) & 7 == dg]
            if idx:
                assert idx == list(range(idx[0], idx[-1] + 1))
                rec(idx[0], len(idx), L + 1)

    rec(0, len(keys), 0)
    return sorted(out)


@pytest.mark.parametrize("n_leaf", [1, 4, 16])
def test_octree_matches_recursive_definition(n_leaf):
    _, t = _sorted_inputs(700, 2, n_leaf=n_leaf)
    mine = sorted(zip(t.level.tolist(), t.begin.tolist(), t.count.tolist()))
    assert mine == _recursive_tree(t.keys, n_leaf)
    # breadth-first numbering: levels non-decreasing, begin increasing per level
    assert np.all(np.diff(t.level) >= 0)
    for L in np.unique(t.level):
        b = t.begin[t.level == L]
        assert np.all(np.diff(b) > 0)
    # children partition their parent; leaves are small or at level 21
    for p in range(t.n_nodes):
        k = t.n_child[p]
        if k == 0:
            assert t.count[p] <= n_leaf or t.level[p] == 21
            continue
        ch = np.arange(t.first_child[p], t.first_child[p] + k)
        assert np.all(t.parent[ch] == p)
        assert t.begin[ch[0]] == t.begin[p]
        assert t.count[ch].sum() == t.count[p]
        assert np.all(t.begin[ch[1:]] == t.begin[ch[:-1]] + t.count[ch[:-1]])


def test_coincident_keys_stop_at_level_21():
    n = 40
    x = np.full(n, 0.5, np.float32)
    y = np.full(n, 0.25, np.float32)
    z = np.full(n, 0.125, np.float32)
    x[0] = 0.0  # a second point sets the extent
    t = oracle.tree_build(x, y, z, synth.equal_masses(n), n_leaf=4)
    assert t.level.max() == 21
    leaf = np.where(t.n_child == 0)[0]
    assert t.count[leaf].max() == n - 1  # the 39 coincident particles share one leaf


def test_moments_against_numpy():
    (x, y, z, m), t = _sorted_inputs(2000, 3)
    rng = np.random.default_rng(4)
    mm = rng.uniform(0.5, 2.0, 2000).astype(np.float32)
    t2 = oracle.tree_build(x, y, z, mm, n_leaf=8)
    for tt in (t, t2):
        for p in list(range(0, tt.n_nodes, 29)) + [0]:
            b, c = tt.begin[p], tt.count[p]
            P = np.stack([tt.x[b:b + c], tt.y[b:b + c], tt.z[b:b + c]], 1)
            w = tt.m[b:b + c]
            M = w.sum()
            com = (w[:, None] * P).sum(0) / M
            C = np.cov(P.T, aweights=w, bias=True) * M if c > 1 else np.zeros((3, 3))
            assert np.isclose(tt.mass[p], M, rtol=1e-13)
            assert np.allclose(tt.com[p], com, rtol=1e-12, atol=1e-12 * np.abs(P).max())
            S = tt.S[p]
            Sm = np.array([[S[0], S[3], S[4]], [S[3], S[1], S[5]], [S[4], S[5], S[2]]])
            assert np.allclose(Sm, C, rtol=1e-9, atol=1e-12 * (np.abs(C).max() + 1e-300))


def test_moments_parallel_axis_over_children():
    """The parent's second moment is the children's, each moved to the
    parent's centre of mass (the parallel-axis theorem)."""
    _, t = _sorted_inputs(3000, 5)
    for p in np.where(t.n_child > 0)[0][:200]:
        ch = np.arange(t.first_child[p], t.first_child[p] + t.n_child[p])
        S = np.zeros(6)
        for c in ch:
            d = t.com[c] - t.com[p]
            S += t.S[c] + t.mass[c] * np.array([d[0] * d[0], d[1] * d[1], d[2] * d[2],
                                                d[0] * d[1], d[0] * d[2], d[1] * d[2]])
        assert np.allclose(S, t.S[p], rtol=1e-9, atol=1e-12 * np.abs(t.S[p]).max())
        assert np.isclose(t.mass[ch].sum(), t.mass[p], rtol=1e-14)


@pytest.mark.parametrize("seed", range(6))
def test_sym3_eigen_against_eigh(seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3))
    A = A @ A.T if seed % 2 else A + A.T
    if seed == 4:
        A = np.diag([2.0, 2.0, 1.0])  # degenerate
    S6 = [A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]]
    w, V = oracle.sym3_eigen(S6)
    ref = np.linalg.eigh(A)[0][::-1]
    assert np.allclose(w, ref, rtol=1e-12, atol=1e-13)
    assert np.all(np.diff(w) <= 0)
    assert np.allclose(V.T @ V, np.eye(3), atol=1e-12)
    assert np.allclose(A @ V, V * w, atol=1e-11)


def _pp_of(t, p):
    q = slice(t.npp * p, t.npp * p + t.npp)
    return np.stack([t.px[q], t.py[q], t.pz[q]], 1), t.pm[q]


def test_pseudo_particles_reproduce_moments():
    """Monopole, zero dipole and the traceless quadrupole of every node's
    three pseudo-particles equal those of its particles."""
    _, t = _sorted_inputs(3000, 6, quad=True)
    for p in range(0, t.n_nodes, 7):
        P, w = _pp_of(t, p)
        assert np.isclose(w.sum(), t.mass[p], rtol=1e-14)
        d = P - t.com[p]
        scale = np.sqrt(max(t.S[p][:3].sum() / t.mass[p], 1e-300))
        assert np.allclose((w[:, None] * d).sum(0) / t.mass[p], 0.0, atol=1e-12 * scale + 1e-15)
        Spp = (w[:, None, None] * d[:, :, None] * d[:, None, :]).sum(0)
        S = t.S[p]
        Sm = np.array([[S[0], S[3], S[4]], [S[3], S[1], S[5]], [S[4], S[5], S[2]]])
        tl = lambda A: A - np.trace(A) / 3.0 * np.eye(3)
        assert np.allclose(tl(Spp), tl(Sm), atol=1e-10 * (np.abs(Sm).max() + 1e-300))


def test_pseudo_particle_far_field_orders():
    """The potential of a clump at distance D: the monopole's error falls as
    D^-3 (the quadrupole term it misses), the three pseudo-particles' as D^-4
    (they carry the quadrupole; the octupole is the first missing term)."""
    rng = np.random.default_rng(7)
    n = 50
    P = rng.standard_normal((n, 3)) * np.array([1.0, 0.5, 0.2])
    P = P.astype(np.float32)
    m = rng.uniform(0.5, 1.5, n).astype(np.float32)
    errs = {}
    for quad in (False, True):
        t = oracle.tree_build(P[:, 0], P[:, 1], P[:, 2], m, n_leaf=n, quad=quad)
        pp, pw = _pp_of(t, 0)
        e = []
        u = np.array([0.48, -0.6, 0.64])
        for D in (40.0, 80.0, 160.0):
            X = t.com[0] + D * u
            exact = -(t.m / np.linalg.norm(np.stack([t.x, t.y, t.z], 1) - X, axis=1)).sum()
            approx = -(pw / np.linalg.norm(pp - X, axis=1)).sum()
            e.append(abs(approx - exact))
        errs[quad] = e
    r_mono = [errs[False][k] / errs[False][k + 1] for k in range(2)]
    r_quad = [errs[True][k] / errs[True][k + 1] for k in range(2)]
    assert all(7.0 < r < 9.0 for r in r_mono), r_mono
    assert all(14.0 < r < 18.0 for r in r_quad), r_quad


def test_groups_partition_particles():
    _, t = _sorted_inputs(5000, 8)
    for n_crit in (16, 64, 256):
        g = t.find_groups(n_crit)
        b, c = t.begin[g], t.count[g]
        assert b[0] == 0 and np.all(b[1:] == b[:-1] + c[:-1]) and b[-1] + c[-1] == t.n
        for p in g:
            assert t.count[p] <= n_crit or t.n_child[p] == 0
            assert t.parent[p] < 0 or t.count[t.parent[p]] > n_crit


def _node_ranges(t):
    return t.begin, t.count


@pytest.mark.parametrize("quad", [False, True])
def test_lists_cover_every_particle_and_obey_the_criterion(quad):
    theta = 0.75
    _, t = _sorted_inputs(4000, 9, quad=quad)
    g = t.find_groups(64)
    for gi in list(range(0, len(g), 5)):
        gn = g[gi]
        src, _ = t.walk(gn, theta)
        cover = np.zeros(t.n, np.int64)
        part = src[src >= 0]
        cover[part] += 1
        nodes = np.unique((-1 - src[src < 0]) // t.npp)
        assert np.all(np.bincount((-1 - src[src < 0]) // t.npp) % t.npp == 0)
        b, c = t.begin[gn], t.count[gn]
        P = np.stack([t.x[b:b + c], t.y[b:b + c], t.z[b:b + c]], 1)
        lo, hi = P.min(0), P.max(0)
        for nd in nodes:
            cover[t.begin[nd]:t.begin[nd] + t.count[nd]] += 1
            d = np.linalg.norm(np.maximum(0, np.maximum(lo - t.com[nd], t.com[nd] - hi)))
            assert t.extent / 2.0 ** t.level[nd] < theta * d
            # its parent was opened: it failed the criterion or is an ancestor
            pa = t.parent[nd]
            dp = np.linalg.norm(np.maximum(0, np.maximum(lo - t.com[pa], t.com[pa] - hi)))
            anc = t.begin[pa] <= b < t.begin[pa] + t.count[pa] and t.level[pa] <= t.level[gn]
            assert anc or not (t.extent / 2.0 ** t.level[pa] < theta * dp)
        assert np.all(cover == 1)
        # the group's own particles come as particles (in visit order)
        own = part[(part >= b) & (part < b + c)]
        assert np.array_equal(np.sort(own), np.arange(b, b + c))


def test_theta_zero_is_the_direct_sum():
    (x, y, z, m), t = _sorted_inputs(1500, 10, quad=True)
    eps = 0.01
    items, src, _, ax, ay, az, phi = oracle.tree_force(t, 0.0, 32, eps)
    assert np.all(items[:, 3] == t.n)
    e2 = np.full(t.n, float(np.float32(eps)) ** 2)
    ref = oracle.newton(t.x, t.y, t.z, e2, t.x, t.y, t.z, t.m)
    for a, r in zip((ax, ay, az, phi), ref):
        assert np.allclose(a, r, rtol=1e-12, atol=1e-12 * np.abs(r).max())


def test_tree_force_error_ordering():
    """Against the direct sum: the error grows with theta and the
    quadrupole pseudo-particles beat the monopole at every theta."""
    (x, y, z, m), tm = _sorted_inputs(6000, 11, quad=False)
    tq = oracle.tree_build(x, y, z, m, n_leaf=8, quad=True)
    eps = 1.0 / 256
    e2 = np.full(tm.n, float(np.float32(eps)) ** 2)
    ref = oracle.newton(tm.x, tm.y, tm.z, e2, tm.x, tm.y, tm.z, tm.m)
    R = np.stack(ref[:3])
    amag = np.linalg.norm(R, axis=0)
    res = {}
    for quad, t in ((False, tm), (True, tq)):
        for th in (0.3, 0.5, 0.75):
            _, _, _, ax, ay, az, _ = oracle.tree_force(t, th, 64, eps)
            err = np.linalg.norm(np.stack([ax, ay, az]) - R, axis=0) / amag
            res[quad, th] = np.sqrt(np.mean(err ** 2))
    for quad in (False, True):
        assert res[quad, 0.3] < res[quad, 0.5] < res[quad, 0.75]
    for th in (0.3, 0.5, 0.75):
        assert res[True, th] < res[False, th]
    assert res[False, 0.75] < 2e-2 and res[True, 0.75] < 5e-3, res
