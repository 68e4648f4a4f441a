"""GPU parity of the device Barnes-Hut tree (the tree code of Sec. 5: shared
lists for groups of i-particles, theta = 0.75, monopole or three-particle
quadrupole pseudo-particles) against the FP64 tree oracle, through the C ABI.

Integer work is compared bit for bit: the frame, keys and order, every node
array and the groups.  FP64 moments are compared to rounding; pseudo-particles
through what is unique about them (mass, dipole, traceless quadrupole); the
lists entry by entry wherever no opening decision lies within rounding of its
threshold (the oracle reports each group's margin), and for every group
through the properties every valid list has; forces against the oracle's sum
over the GPU's own lists and over the oracle's lists, to the Newton gate."""
import numpy as np
import pytest

import oracle
import synth
from _helpers import rel_vec_err, rms, to_dev, to_host

pytestmark = pytest.mark.gpu

BORDER = 1e-5  # decisions nearer than this (relative to the coordinates) may flip


@pytest.fixture(scope="module")
def pgh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1203_4037_amd as p
    return p


@pytest.fixture()
def ctx(pgh):
    c = pgh.Context(0)
    yield c
    c.close()


def _build(ctx, x, y, z, m, n_leaf=8, n_crit=64, quad=False):
    t = ctx.tree()
    d = to_dev(x, y, z, m)
    t.build(*d, n_leaf=n_leaf, n_crit=n_crit, quad=quad)
    return t, d


def _S3(S):
    return np.array([[S[0], S[3], S[4]], [S[3], S[1], S[5]], [S[4], S[5], S[2]]])


@pytest.mark.parametrize("quad", [False, True])
@pytest.mark.parametrize("n,n_leaf,n_crit", [(20000, 8, 64), (3000, 1, 16), (777, 16, 16)])
def test_structure_matches_oracle(pgh, ctx, quad, n, n_leaf, n_crit):
    x, y, z = synth.plummer(n, 200 + n)
    m = synth.equal_masses(n) * np.float32(1.0 + 0.5 * np.sin(np.arange(n))).astype(np.float32)
    t, _ = _build(ctx, x, y, z, m, n_leaf, n_crit, quad)
    o = oracle.tree_build(x, y, z, m, n_leaf=n_leaf, quad=quad)
    g_ref = o.find_groups(n_crit)
    st = t.stats()
    assert np.array_equal(st["frame"], o.frame)
    assert np.array_equal(t.get("perm"), o.perm)
    assert np.array_equal(t.get("keys"), o.keys)
    for f in ("x", "y", "z", "m"):
        assert np.array_equal(t.get(f).astype(np.float64), getattr(o, f))
    assert st["n_nodes"] == o.n_nodes and st["depth"] == o.level.max()
    assert st["n_leaves"] == int((o.n_child == 0).sum())
    for f, ref in (("node_begin", o.begin), ("node_count", o.count), ("node_level", o.level),
                   ("node_first_child", o.first_child), ("node_n_child", o.n_child),
                   ("node_parent", o.parent)):
        assert np.array_equal(t.get(f), ref), f
    assert np.array_equal(t.get("groups"), g_ref)
    mom = t.get("moments")
    assert np.allclose(mom[:, 0], o.mass, rtol=1e-12)
    scale = np.abs(o.com).max()
    assert np.allclose(mom[:, 1:4], o.com, rtol=0, atol=1e-12 * scale)
    Smax = np.abs(o.S).max(axis=1, keepdims=True)
    assert np.all(np.abs(mom[:, 4:] - o.S) <= 1e-9 * Smax + 1e-300)
    pp = t.get("pseudo").astype(np.float64)
    if not quad:  # the FP64 values rounded once (1 ulp where they straddle a tie)
        assert np.all(np.abs(pp[:, :3] - o.com) <= 2.0 ** -23 * np.abs(o.com))
        assert np.all(np.abs(pp[:, 3] - o.mass) <= 2.0 ** -23 * o.mass)
        return
    # the three pseudo-particles: mass, zero dipole, traceless quadrupole
    P = pp.reshape(-1, 3, 4)
    u = 2.0 ** -24
    for k in range(0, o.n_nodes, max(1, o.n_nodes // 4000)):
        w = P[k, :, 3]
        M = o.mass[k]
        assert abs(w.sum() - M) <= 4 * u * M
        d = P[k, :, :3] - o.com[k]
        pos = np.abs(P[k, :, :3]).max()
        assert np.all(np.abs((w[:, None] * d).sum(0)) <= 8 * u * pos * M + 1e-300)
        Q = (w[:, None, None] * d[:, :, None] * d[:, None, :]).sum(0)
        S = _S3(o.S[k])
        tl = lambda A: A - np.trace(A) / 3 * np.eye(3)
        spread = np.sqrt(max(np.trace(S) / M, 0.0))
        tol = 16 * u * pos * (spread + u * pos) * M + 1e-12 * np.abs(S).max() + 1e-300
        assert np.all(np.abs(tl(Q) - tl(S)) <= tol), k


def _list_case(pgh, ctx, n, seed, quad, theta=0.75, n_leaf=8, n_crit=64):
    x, y, z = synth.plummer(n, seed)
    m = synth.equal_masses(n)
    t, d = _build(ctx, x, y, z, m, n_leaf, n_crit, quad)
    t.walk(theta, record_src=True)
    o = oracle.tree_build(x, y, z, m, n_leaf=n_leaf, quad=quad)
    o.find_groups(n_crit)
    return t, d, o, (x, y, z, m)


@pytest.mark.parametrize("quad", [False, True])
def test_lists_match_oracle(pgh, ctx, quad):
    n = 30000
    t, d, o, _ = _list_case(pgh, ctx, n, 301, quad)
    items = t.get("items")
    src = t.get("list_src").astype(np.int64)
    lx = t.get("list_x")
    st = t.stats()
    assert st["n_entries"] == src.size == items[:, 3].sum()
    assert st["interactions"] == int((items[:, 1].astype(np.int64) * items[:, 3]).sum())
    g = o.groups
    assert np.array_equal(items[:, 0], o.begin[g]) and np.array_equal(items[:, 1], o.count[g])
    assert np.array_equal(items[:, 2][1:], np.cumsum(items[:, 3])[:-1]) and items[0, 2] == 0
    pp = t.get("pseudo")
    xs = t.get("x")
    leaf_of = _leaf_of(o)
    exact = border = 0
    for k, gn in enumerate(g):
        s_gpu = src[items[k, 2]:items[k, 2] + items[k, 3]]
        # entries carry their source's values
        part = s_gpu >= 0
        vals = np.where(part, xs[np.where(part, s_gpu, 0)], pp[np.where(part, 0, -1 - s_gpu), 0])
        assert np.array_equal(lx[items[k, 2]:items[k, 2] + items[k, 3]], vals)
        ref, margin = o.walk(gn, 0.75)
        if margin > BORDER:
            assert np.array_equal(s_gpu, ref), k
            exact += 1
            continue
        border += 1
        # a list near a decision threshold: still a valid cover of the particles
        cover = np.zeros(n, np.int64)
        np.add.at(cover, s_gpu[part], 1)
        nodes = (-1 - s_gpu[~part]) // o.npp
        for nd in np.unique(nodes):
            cover[o.begin[nd]:o.begin[nd] + o.count[nd]] += 1
        assert np.all(cover == 1), k
        _check_decisions(o, gn, np.unique(nodes), s_gpu[part], 0.75, leaf_of, k)
    assert exact >= 0.9 * len(g), (exact, border)
    assert border > 0  # the borderline branch is exercised


def _leaf_of(o):
    """The leaf holding each sorted particle rank."""
    leaf = np.full(o.x.size, -1, np.int64)
    for t in np.nonzero(o.n_child == 0)[0]:
        leaf[o.begin[t]:o.begin[t] + o.count[t]] = t
    assert np.all(leaf >= 0)
    return leaf


def _check_decisions(o, g, accepted, particles, theta, leaf_of, what):
    """Every decision behind a GPU list taken near a threshold agrees with the
    criterion of the FP64 oracle to within BORDER: with crit(t) = (d - l /
    theta) / s (d the distance from the node's FP64 centre of mass to the
    group's box, l the node size, s the largest magnitude among the
    coordinates involved, as the oracle's margin is measured), each accepted
    node has crit > -BORDER, and each opened node that is neither the group
    nor one of its ancestors (the nodes above an accepted node, and the
    leaves of the particle entries with the nodes above them) has
    crit < +BORDER."""
    b0, b1 = o.begin[g], o.begin[g] + o.count[g]
    lo = np.array([o.x[b0:b1].min(), o.y[b0:b1].min(), o.z[b0:b1].min()])
    hi = np.array([o.x[b0:b1].max(), o.y[b0:b1].max(), o.z[b0:b1].max()])

    def crit(t):
        c = o.com[t]
        e = np.where(c < lo, lo - c, np.where(c > hi, c - hi, 0.0))
        d = np.sqrt((e * e).sum(-1))
        sc = np.maximum(1.0, np.maximum(np.abs(c).max(-1), max(np.abs(lo).max(), np.abs(hi).max())))
        l = o.extent / 2.0 ** o.level[t]
        return (d - l / theta) / sc

    def is_anc(t):  # the group and its ancestors: opened without a test
        return (o.level[t] <= o.level[g]) & (o.begin[t] <= b0) & (b0 < o.begin[t] + o.count[t])

    accepted = np.asarray(accepted, np.int64)
    assert not np.any(is_anc(accepted)), what
    assert np.all(crit(accepted) > -BORDER), what
    opened = set()
    for t in list(accepted) + list(np.unique(leaf_of[particles])):
        u = int(o.parent[t]) if t in accepted else int(t)
        while u >= 0 and u not in opened:
            opened.add(u)
            u = int(o.parent[u])
    opened = np.array(sorted(opened), np.int64)
    opened = opened[~is_anc(opened)]
    assert np.all(crit(opened) < BORDER), what


@pytest.mark.parametrize("quad", [False, True])
def test_tree_force_parity(pgh, ctx, quad):
    """Force and potential on every particle, in input order: against the
    oracle's sum over the GPU's lists (every group) and against the oracle's
    own tree force (groups without borderline decisions)."""
    n, eps = 30000, 1.0 / 256
    t, d, o, (x, y, z, m) = _list_case(pgh, ctx, n, 302, quad)
    ctx.set_eps_to_all(eps)
    got = np.stack(to_host(*t.newton()))
    perm = t.get("perm")
    got_s = got[:, perm]  # key order
    items = t.get("items")
    lists = [t.get(f).astype(np.float64) for f in ("list_x", "list_y", "list_z", "list_m")]
    e2 = np.full(n, float(np.float32(eps)) ** 2)
    ref = np.stack(oracle.newton_items(items, o.x, o.y, o.z, e2, *lists))
    ea = rel_vec_err(got_s[:3], ref[:3])
    ep = np.abs(got_s[3] - ref[3]) / np.abs(ref[3])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (rms(ea), ea.max())
    assert rms(ep) <= 1e-5 and ep.max() <= 1e-3, (rms(ep), ep.max())
    _, _, margins, ax, ay, az, phi = oracle.tree_force(o, 0.75, 64, eps)
    ok = np.zeros(n, bool)
    for k, gn in enumerate(o.groups):
        if margins[k] > BORDER:
            ok[o.begin[gn]:o.begin[gn] + o.count[gn]] = True
    assert ok.mean() > 0.9
    eo = rel_vec_err(got_s[:3, ok], np.stack([ax, ay, az])[:, ok])
    assert rms(eo) <= 1e-5 and eo.max() <= 1e-3, (rms(eo), eo.max())
    # and the tree approximates the direct sum as the oracle's tree does
    full = np.stack(oracle.newton(o.x, o.y, o.z, e2, o.x, o.y, o.z, o.m)[:3])
    err = rel_vec_err(got_s[:3], full)
    assert rms(err) < (3e-3 if quad else 8e-3), rms(err)


def test_theta_zero_is_the_direct_sum(pgh, ctx):
    n, eps = 2500, 0.01
    x, y, z = synth.plummer(n, 303)
    m = synth.equal_masses(n)
    t, d = _build(ctx, x, y, z, m, 8, 32, True)
    t.walk(0.0)
    assert t.stats()["n_entries"] == n * t.stats()["n_groups"]
    ctx.set_eps_to_all(eps)
    got = np.stack(to_host(*t.newton()))
    e2 = np.full(n, np.float32(eps) ** 2, np.float32)
    ref = np.stack(oracle.newton(x, y, z, e2, x, y, z, m))
    ea = rel_vec_err(got[:3], ref[:3])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3
    ep = np.abs(got[3] - ref[3]) / np.abs(ref[3])
    assert rms(ep) <= 1e-5 and ep.max() <= 1e-3


def test_degenerate_inputs(pgh, ctx):
    import torch
    t = ctx.tree()
    e = torch.zeros(0, device="cuda")
    t.build(e, e, e, e)
    t.walk(0.75)
    st = t.stats()
    assert st["n_nodes"] == 0 and st["n_groups"] == 0 and st["n_entries"] == 0
    t.newton(out=[e, e, e, e])
    ctx.set_eps_to_all(0.1)
    # one particle: no force, the self term in the potential
    one = to_dev(np.array([0.3], np.float32), np.array([-0.2], np.float32),
                 np.array([0.1], np.float32), np.array([2.0], np.float32))
    t.build(*one)
    t.walk(0.75)
    a = to_host(*t.newton())
    assert a[0][0] == 0 and a[1][0] == 0 and a[2][0] == 0
    assert np.isclose(a[3][0], -2.0 / np.float32(0.1), rtol=1e-6)
    # coincident particles: a chain of nodes down to level 21, one leaf group
    n = 100
    c = [np.full(n, v, np.float32) for v in (0.5, 0.25, -0.125)] + [synth.equal_masses(n)]
    t.build(*to_dev(*c), n_leaf=8, n_crit=64)
    st = t.stats()
    assert st["depth"] == 21 and st["n_groups"] == 1 and st["frame"][3] == 0
    t.walk(0.75)
    assert t.stats()["n_entries"] == n
    a = to_host(*t.newton())
    assert np.all(a[0] == 0) and np.all(a[1] == 0) and np.all(a[2] == 0)
    assert np.allclose(a[3], -1.0 / np.float32(0.1), rtol=1e-5)
    # massless particles: zero forces, the walk still covers every particle
    x, y, z = synth.plummer(3000, 304)
    z0 = np.zeros(3000, np.float32)
    t.build(*to_dev(x, y, z, z0), quad=True)
    t.walk(0.75)
    a = to_host(*t.newton())
    assert all(np.all(v == 0) for v in a)
    # groups of single particles
    x, y, z = synth.plummer(500, 305)
    m = synth.equal_masses(500)
    t.build(*to_dev(x, y, z, m), n_leaf=1, n_crit=1)
    assert t.stats()["n_groups"] == 500
    t.walk(0.75)
    o = oracle.tree_build(x, y, z, m, n_leaf=1)
    o.find_groups(1)
    _, _, mg, ax, ay, az, ph = oracle.tree_force(o, 0.75, 1, 0.1)
    got = np.stack(to_host(*t.newton()))[:, o.perm]
    ok = np.repeat(mg > BORDER, 1)
    ea = rel_vec_err(got[:3, ok], np.stack([ax, ay, az])[:, ok])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3
    t.free()


def test_rebuild_smaller_and_larger(pgh, ctx):
    """One tree object rebuilt on growing and shrinking inputs matches fresh
    oracle trees each time (buffers are reused or grown)."""
    t = ctx.tree()
    ctx.set_eps_to_all(0.02)
    for n in (5000, 1200, 40000, 9000):
        x, y, z = synth.plummer(n, 310 + n)
        m = synth.equal_masses(n)
        t.build(*to_dev(x, y, z, m), n_leaf=8, n_crit=64, quad=n % 2 == 0)
        t.walk(0.75)
        o = oracle.tree_build(x, y, z, m, n_leaf=8, quad=n % 2 == 0)
        o.find_groups(64)
        assert np.array_equal(t.get("node_count"), o.count)
        assert np.array_equal(t.get("groups"), o.groups)
        got = np.stack(to_host(*t.newton()))[:, o.perm]
        items = t.get("items")
        lists = [t.get(f).astype(np.float64) for f in ("list_x", "list_y", "list_z", "list_m")]
        e2 = np.full(n, float(np.float32(0.02)) ** 2)
        ref = np.stack(oracle.newton_items(items, o.x, o.y, o.z, e2, *lists))
        ea = rel_vec_err(got[:3], ref[:3])
        assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, n
    t.free()


def test_rewalk_refills_the_plan(pgh, ctx):
    """Walks of one build with a wider and a narrower opening angle write
    their plans into the same plan object (grown, then reused); a build
    hides the plan until the next walk.  Each walk's force matches the
    oracle's sum over the lists it wrote."""
    n = 20000
    x, y, z = synth.plummer(n, 340)
    m = synth.equal_masses(n)
    ctx.set_eps_to_all(0.02)
    t = ctx.tree().build(*to_dev(x, y, z, m), n_leaf=8, n_crit=64)
    o = oracle.tree_build(x, y, z, m, n_leaf=8)
    plan = None
    for theta in (0.9, 0.3, 0.75):
        t.walk(theta)
        p = pgh.lib.pgh_tree_plan(t.h)
        assert p is not None and (plan is None or p == plan)
        plan = p
        got = np.stack(to_host(*t.newton()))[:, o.perm]
        items = t.get("items")
        lists = [t.get(f).astype(np.float64) for f in ("list_x", "list_y", "list_z", "list_m")]
        e2 = np.full(n, float(np.float32(0.02)) ** 2)
        ref = np.stack(oracle.newton_items(items, o.x, o.y, o.z, e2, *lists))
        ea = rel_vec_err(got[:3], ref[:3])
        assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, theta
    # the walk's plan belongs to the tree: pgh_plan_free refuses it, and the
    # tree's next walk and force still use it
    assert pgh.lib.pgh_plan_free(ctx.h, plan) == pgh.PGH_EINVAL
    t.walk(0.75)
    assert pgh.lib.pgh_tree_plan(t.h) == plan
    again = np.stack(to_host(*t.newton()))[:, o.perm]
    ea = rel_vec_err(again[:3], ref[:3])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3
    t.build(*to_dev(x, y, z, m), n_leaf=8, n_crit=64)
    assert pgh.lib.pgh_tree_plan(t.h) is None
    t.free()


def test_errors(pgh, ctx):
    import torch
    t = ctx.tree()
    with pytest.raises(pgh.PGHError) as e:
        t.walk(0.75)
    assert e.value.code == pgh.PGH_ESTATE
    x, y, z = synth.plummer(20000, 320)
    m = synth.equal_masses(20000)
    d = to_dev(x, y, z, m)
    for kw in ({"n_leaf": 0}, {"n_leaf": 65, "n_crit": 100}, {"n_leaf": 8, "n_crit": 4}):
        with pytest.raises(pgh.PGHError) as e:
            t.build(*d, **kw)
        assert e.value.code == pgh.PGH_ERANGE
    t.build(*d, n_leaf=1, n_crit=1)
    with pytest.raises(pgh.PGHError) as e:
        t.newton()
    assert e.value.code == pgh.PGH_ESTATE
    with pytest.raises(pgh.PGHError) as e:
        t.get("list_x")
    assert e.value.code == pgh.PGH_ESTATE
    with pytest.raises(pgh.PGHError) as e:
        t.walk(-1.0)
    assert e.value.code == pgh.PGH_ERANGE
    # theta = 0 on 20000 single-particle leaves: a frontier level exceeds the
    # walk's capacity, reported as an error (every wave still exits)
    assert t.stats()["max_level_nodes"] > 4096
    with pytest.raises(pgh.PGHError) as e:
        t.walk(0.0)
    assert e.value.code == pgh.PGH_ERANGE
    t.walk(0.75)
    with pytest.raises(pgh.PGHError) as e:
        t.get("list_src")  # walked without record_src
    assert e.value.code == pgh.PGH_ESTATE
    cnt = pgh.ctypes.c_longlong()
    small = np.zeros(10, np.float32)
    rc = pgh.lib.pgh_tree_get(ctx.h, t.h, 2, small.ctypes.data, 10, pgh.ctypes.byref(cnt))
    assert rc == pgh.PGH_ERANGE and cnt.value == 20000
    inf = d[0].clone()
    inf[3] = float("inf")
    with pytest.raises(pgh.PGHError) as e:
        t.build(inf, d[1], d[2], d[3])
    assert e.value.code == pgh.PGH_ERANGE
    with pytest.raises(pgh.PGHError) as e:  # the failed build left no tree
        t.walk(0.75)
    assert e.value.code == pgh.PGH_ESTATE
    t.free()
    assert torch.cuda.is_available()


def test_full_size_plummer_sampled(pgh, ctx):
    """N = 2^20 Plummer sphere, theta = 0.75, n_leaf = 8, n_crit = 64, both
    moment orders: 64 sampled groups against the oracle's tree force (those
    without borderline decisions) and every particle's list length against
    the oracle's count of its group's walk."""
    n, eps = 1 << 20, 1.0 / 512
    x, y, z = synth.plummer(n, 330)
    m = synth.equal_masses(n)
    d = to_dev(x, y, z, m)
    ctx.set_eps_to_all(eps)
    for quad in (False, True):
        t = ctx.tree()
        t.build(*d, n_leaf=8, n_crit=64, quad=quad)
        t.walk(0.75)
        got = np.stack(to_host(*t.newton()))
        o = oracle.tree_build(x, y, z, m, n_leaf=8, quad=quad)
        g = o.find_groups(64)
        assert np.array_equal(t.get("groups"), g)
        items = t.get("items")
        rng = np.random.default_rng(5)
        pick = np.unique(np.concatenate([[0, len(g) - 1, np.argmax(items[:, 3])],
                                         rng.integers(0, len(g), 61)]))
        _, _, mg, ax, ay, az, phi = oracle.tree_force(o, 0.75, 64, eps, groups=g[pick])
        checked = 0
        for k, gi in enumerate(pick):
            gn = g[gi]
            ref_src, margin = o.walk(gn, 0.75)
            if margin <= BORDER:
                continue
            assert items[gi, 3] == ref_src.size
            r = np.arange(o.begin[gn], o.begin[gn] + o.count[gn])
            ea = rel_vec_err(got[:3, o.perm[r]], np.stack([ax[r], ay[r], az[r]]))
            assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (quad, gi, rms(ea), ea.max())
            checked += 1
        assert checked >= 48
        t.free()


@pytest.mark.parametrize("n,n_crit,thetas,quad", [(1 << 19, 64, (0.75, 0.4), False),
                                                   (1 << 20, 1024, (0.5,), True)])
def test_device_expanded_plan_matches_host_plan(pgh, ctx, n, n_crit, thetas, quad):
    """A walk's plan is expanded on the device from its compact form; a plan
    of the same lists made on the host (pgh_plan_create) holds the same tasks,
    so the batched force over the tree's key-ordered arrays with it gives the
    tree force bit for bit (groups of 64 pair their partly filled chunks,
    groups of 1024 with theta = 0.5 cut their long lists into parts; a second
    walk of one build writes a larger plan into the same plan object)."""
    x, y, z = synth.plummer(n, 345)
    m = synth.equal_masses(n)
    ctx.set_eps_to_all(1.0 / 512)
    t = ctx.tree().build(*to_dev(x, y, z, m), n_leaf=8, n_crit=n_crit, quad=quad)
    perm = t.get("perm")
    keyed = to_dev(*(t.get(f) for f in ("x", "y", "z")))
    for theta in thetas:
        t.walk(theta)
        got = np.stack(to_host(*t.newton()))
        items = t.get("items")
        lists = to_dev(*(t.get(f) for f in ("list_x", "list_y", "list_z", "list_m")))
        ctx.set_plan_expansion(False)  # every task written on the host
        plan = ctx.plan(items, n, int((items[:, 2].astype(np.int64) + items[:, 3]).max()))
        ctx.set_plan_expansion(True)
        ref = np.stack(to_host(*plan.newton(*keyed, *lists)))
        assert plan.interactions == int((items[:, 1].astype(np.int64) * items[:, 3]).sum())
        assert np.array_equal(got[:, perm], ref), theta
        plan.free()
    t.free()


def test_king_model_sampled(pgh, ctx):
    """King model with W0 = 9 (the paper's second tree-code distribution),
    N = 2^18, groups of at most 256: sampled groups against the oracle's tree
    force, both moment orders."""
    n, eps = 1 << 18, 1.0 / 512
    x, y, z = synth.king(n, 331, 9.0)
    m = synth.equal_masses(n)
    d = to_dev(x, y, z, m)
    ctx.set_eps_to_all(eps)
    for quad in (False, True):
        t = ctx.tree()
        t.build(*d, n_leaf=8, n_crit=256, quad=quad)
        t.walk(0.75)
        got = np.stack(to_host(*t.newton()))
        o = oracle.tree_build(x, y, z, m, n_leaf=8, quad=quad)
        g = o.find_groups(256)
        assert np.array_equal(t.get("groups"), g)
        assert np.array_equal(t.get("node_count"), o.count)
        rng = np.random.default_rng(9)
        pick = np.unique(rng.integers(0, len(g), 40))
        _, _, mg, ax, ay, az, _ = oracle.tree_force(o, 0.75, 256, eps, groups=g[pick])
        checked = 0
        for k, gi in enumerate(pick):
            if mg[k] <= BORDER:
                continue
            gn = g[gi]
            r = np.arange(o.begin[gn], o.begin[gn] + o.count[gn])
            ea = rel_vec_err(got[:3, o.perm[r]], np.stack([ax[r], ay[r], az[r]]))
            assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (quad, gi, rms(ea), ea.max())
            checked += 1
        assert checked >= 30
        t.free()


@pytest.mark.parametrize("theta,n_leaf,quad", [(0.3, 16, False), (0.5, 4, True), (1.0, 1, False),
                                               (0.75, 64, True)])
def test_theta_and_leaf_variants(pgh, ctx, theta, n_leaf, quad):
    """Other opening angles and leaf sizes: lists entry by entry against the
    oracle (groups without borderline decisions), forces against the
    oracle's sum over the GPU's lists."""
    n, eps = 20000, 1.0 / 256
    x, y, z = synth.plummer(n, 340)
    m = synth.equal_masses(n)
    t, _ = _build(ctx, x, y, z, m, n_leaf, max(64, n_leaf), quad)
    t.walk(theta, record_src=True)
    o = oracle.tree_build(x, y, z, m, n_leaf=n_leaf, quad=quad)
    g = o.find_groups(max(64, n_leaf))
    items = t.get("items")
    src = t.get("list_src").astype(np.int64)
    exact = 0
    for k, gn in enumerate(g):
        ref, margin = o.walk(gn, theta)
        if margin > BORDER:
            assert np.array_equal(src[items[k, 2]:items[k, 2] + items[k, 3]], ref), k
            exact += 1
    assert exact >= 0.9 * len(g)
    ctx.set_eps_to_all(eps)
    got = np.stack(to_host(*t.newton()))[:, o.perm]
    lists = [t.get(f).astype(np.float64) for f in ("list_x", "list_y", "list_z", "list_m")]
    e2 = np.full(n, float(np.float32(eps)) ** 2)
    ref = np.stack(oracle.newton_items(items, o.x, o.y, o.z, e2, *lists))
    ea = rel_vec_err(got[:3], ref[:3])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (rms(ea), ea.max())
    t.free()


def test_lists_beyond_int32_are_an_error(pgh, ctx):
    """2^24 particles in groups of at most 8 with quadrupole pseudo-particles
    need more than 2^31 - 1 list entries: the walk reports PGH_ERANGE after its
    counting pass (no list memory is allocated), and a coarser walk of the
    same tree still works."""
    n = 1 << 24
    x, y, z = synth.plummer(n, 350)
    d = to_dev(x, y, z, synth.equal_masses(n))
    t = ctx.tree()
    t.build(*d, n_leaf=8, n_crit=8, quad=True)
    with pytest.raises(pgh.PGHError) as e:
        t.walk(0.75)
    assert e.value.code == pgh.PGH_ERANGE and "2^31" in str(e.value)
    t.build(*d, n_leaf=8, n_crit=256, quad=False)
    t.walk(0.75)
    assert 0 < t.stats()["n_entries"] < 2 ** 31
    t.free()


def test_deep_chains_grow_the_node_arrays(pgh, ctx):
    """500 tight pairs with leaves of one particle: every pair hangs from a
    chain of single-child nodes down to level 20 or 21, some 10^4 nodes for
    10^3 particles, more than the node arrays first hold (2n), so the build
    runs again with more room; the tree still matches the oracle's."""
    rng = np.random.default_rng(360)
    c = rng.random((500, 3))
    off = rng.standard_normal((500, 3)) * 1e-6
    p = np.concatenate([c, c + off]).astype(np.float32)
    x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
    m = synth.equal_masses(1000)
    t, _ = _build(ctx, x, y, z, m, 1, 1, False)
    o = oracle.tree_build(x, y, z, m, n_leaf=1)
    assert o.n_nodes > 2 * 1000 + 64
    assert t.stats()["n_nodes"] == o.n_nodes
    for f, ref in (("node_begin", o.begin), ("node_count", o.count), ("node_level", o.level),
                   ("node_first_child", o.first_child), ("node_parent", o.parent)):
        assert np.array_equal(t.get(f), ref), f
    assert np.array_equal(t.get("groups"), o.find_groups(1))
    ctx.set_eps_to_all(1e-3)
    t.walk(0.75)
    got = np.stack(to_host(*t.newton()))[:, o.perm]
    items = t.get("items")
    lists = [t.get(f).astype(np.float64) for f in ("list_x", "list_y", "list_z", "list_m")]
    e2 = np.full(1000, float(np.float32(1e-3)) ** 2)
    ref = np.stack(oracle.newton_items(items, o.x, o.y, o.z, e2, *lists))
    ea = rel_vec_err(got[:3], ref[:3])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3
    t.free()


def test_handle_errors(pgh, ctx):
    """A tree is used only with its own context; unknown fields, NULL
    arguments and a second free are errors, not crashes."""
    other = pgh.Context(0)
    t = ctx.tree()
    x, y, z = synth.plummer(1000, 370)
    d = to_dev(x, y, z, synth.equal_masses(1000))
    with pytest.raises(pgh.PGHError) as e:
        pgh.pgh_tree_build(other.h, t.h, 1000, *d)
    assert e.value.code == pgh.PGH_EINVAL
    t.build(*d)
    with pytest.raises(pgh.PGHError) as e:
        pgh.pgh_tree_walk(other.h, t.h, 0.75)
    assert e.value.code == pgh.PGH_EINVAL
    cnt = pgh.ctypes.c_longlong()
    assert pgh.lib.pgh_tree_get(ctx.h, t.h, 99, None, 0, pgh.ctypes.byref(cnt)) == pgh.PGH_ERANGE
    assert pgh.lib.pgh_tree_build(ctx.h, None, 10, None, None, None, None, 8, 64, 0) == pgh.PGH_EINVAL
    assert pgh.lib.pgh_tree_build(ctx.h, t.h, 10, None, None, None, None, 8, 64, 0) == pgh.PGH_EINVAL
    assert pgh.lib.pgh_tree_stats_get(None, None) == pgh.PGH_EINVAL
    assert pgh.lib.pgh_tree_plan(None) is None
    assert pgh.lib.pgh_tree_free(other.h, t.h) == pgh.PGH_EINVAL  # not other's tree
    t.free()
    assert pgh.lib.pgh_tree_free(ctx.h, None) == pgh.PGH_OK
    # a tree left alive is freed with its context
    t2 = other.tree().build(*d).walk(0.75)
    assert t2.stats()["walked"] == 1
    other.close()
