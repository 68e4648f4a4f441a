"""GPU parity of the persistent batched kernels (interaction lists of tree /
TreePM codes, Sec. 5.1) against the FP64 oracle, through the C ABI; plan
validation; replays and graph capture."""
import numpy as np
import pytest

import oracle
import synth
from _helpers import oracle_table, norm_vec_err, rel_vec_err, rms, to_dev, to_host

pytestmark = pytest.mark.gpu

# tile shapes of the batched table kernel (each is run by the cell-list test)
TABLE_BATCH_VARIANTS = 9
# tile shapes of the batched Newton kernel
NEWTON_BATCH_VARIANTS = 5


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


def _dev_set(s, eps2=None):
    di = to_dev(s.xi, s.yi, s.zi)
    dj = to_dev(s.xj, s.yj, s.zj, s.mj)
    return di, dj


def _newton_case(pgh, ctx, s, eps, sample_items=None):
    import torch
    di, dj = _dev_set(s)
    ctx.set_eps_to_all(eps)
    plan = ctx.plan(s.items, s.xi.size, s.xj.size)
    n = s.xi.size
    out = [torch.full((n,), 12345.0, device="cuda") for _ in range(4)]
    plan.newton(*di, *dj, out=out)
    got = to_host(*out)
    items = s.items if sample_items is None else s.items[sample_items]
    e2 = np.full(n, np.float32(eps) ** 2, np.float32)
    ref = oracle.newton_items(items, s.xi, s.yi, s.zi, e2, s.xj, s.yj, s.zj, s.mj)
    rows = np.concatenate([np.arange(i0, i0 + ni) for i0, ni, _, _ in items]) if len(items) else \
        np.zeros(0, np.int64)
    a = np.stack(got[:3])[:, rows]
    ea = rel_vec_err(a, np.stack(ref[:3])[:, rows])
    rp = ref[3][rows]
    ep = np.abs(got[3][rows] - rp) / np.maximum(np.abs(rp), 1e-300)
    assert np.all(got[3][rows][rp == 0] == 0)  # empty j-lists give exact zeros
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (rms(ea), ea.max())
    assert rms(ep) <= 1e-5 and ep.max() <= 1e-3, (rms(ep), ep.max())
    return plan, di, dj, out, got


@pytest.mark.parametrize("variant", range(NEWTON_BATCH_VARIANTS))
@pytest.mark.parametrize("refine", [1, 0])
def test_tree_style_small(pgh, ctx, variant, refine):
    """A small instance of the batched tree workload: Morton-sorted Plummer
    sphere, i-groups of 32..256, log-normal j-list lengths; every variant of
    the batched Newton kernel, with and without the Newton step."""
    s = synth.tree_style_items(1 << 16, 400, 104, nj_median=600, nj_lo=50, nj_hi=6000)
    ctx.set_variant(pgh.PGH_FAMILY_NEWTON_BATCH, variant)
    ctx.set_rsqrt_refine(refine)
    _newton_case(pgh, ctx, s, 1e-3)


@pytest.mark.parametrize("variant", range(NEWTON_BATCH_VARIANTS))
def test_group_size_edges_and_split_lists(pgh, ctx, variant):
    """Group sizes around the lane-sharing thresholds (16, 32, 64) and j-lists
    of 0, 1, 63, 64, 65 and long ones that the plan cuts into parts."""
    ctx.set_variant(pgh.PGH_FAMILY_NEWTON_BATCH, variant)
    rng = np.random.default_rng(8)
    n = 20000
    x, y, z = synth.plummer(n, 44)
    m = synth.equal_masses(n)
    sizes_i = [1, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129, 200]
    sizes_j = [0, 1, 63, 64, 65, 700, 5000, 12000]
    items, i_off, jx, jy, jz, jm, j_off = [], 0, [], [], [], [], 0
    for a in sizes_i:
        for b in sizes_j:
            src = rng.integers(0, n, b)
            jx.append(x[src]); jy.append(y[src]); jz.append(z[src]); jm.append(m[src])
            items.append((i_off, a, j_off, b))
            i_off += a + 3  # leave gaps: rows in no item must stay untouched
            j_off += b
    assert i_off <= n
    s = synth.ItemSet(items=np.array(items, np.int32), xi=x, yi=y, zi=z,
                      xj=np.concatenate(jx), yj=np.concatenate(jy), zj=np.concatenate(jz),
                      mj=np.concatenate(jm), jsrc=None, iperm=None)
    plan, di, dj, out, got = _newton_case(pgh, ctx, s, 1e-2)
    covered = np.zeros(n, bool)
    for i0, ni, _, _ in items:
        covered[i0:i0 + ni] = True
    for g in got:
        assert np.all(g[~covered] == 12345.0)
    # replaying the plan gives the same bits (the queue resets itself)
    import torch
    out2 = [torch.full((n,), 12345.0, device="cuda") for _ in range(4)]
    plan.newton(*di, *dj, out=out2)
    for a, b in zip(got, to_host(*out2)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n_items", [1, 3, 17, 40])
def test_few_tasks_and_repeats(pgh, ctx, n_items):
    """Plans with fewer tasks than task sublists, and a few more; each run
    twice on the same plan with identical bits (every sublist counter puts
    itself back to zero)."""
    import torch
    n = 4000
    x, y, z = synth.plummer(n, 61)
    m = synth.equal_masses(n)
    rng = np.random.default_rng(n_items)
    items, i_off = [], 0
    for k in range(n_items):
        ni = int(rng.integers(1, 90))
        items.append((i_off, ni, int(rng.integers(0, n - 3000)), int(rng.integers(0, 3000))))
        i_off += ni
    s = synth.ItemSet(items=np.array(items, np.int32), xi=x, yi=y, zi=z, xj=x, yj=y, zj=z, mj=m,
                      jsrc=None, iperm=None)
    plan, di, dj, out, got = _newton_case(pgh, ctx, s, 1e-2)
    out2 = [torch.full((n,), 12345.0, device="cuda") for _ in range(4)]
    plan.newton(*di, *dj, out=out2)
    for a, b in zip(got, to_host(*out2)):
        assert np.array_equal(a, b)


def test_plan_validation(pgh, ctx):
    with pytest.raises(pgh.PGHError) as e:
        ctx.plan([[0, 10, 0, 5], [5, 10, 0, 5]], 100, 100)  # overlapping i-ranges
    assert e.value.code == pgh.PGH_EINVAL
    with pytest.raises(pgh.PGHError) as e:
        ctx.plan([[95, 10, 0, 5]], 100, 100)
    assert e.value.code == pgh.PGH_ERANGE
    with pytest.raises(pgh.PGHError) as e:
        ctx.plan([[0, 10, 98, 5]], 100, 100)
    assert e.value.code == pgh.PGH_ERANGE
    with pytest.raises(pgh.PGHError) as e:
        ctx.plan([[0, -1, 0, 5]], 100, 100)
    assert e.value.code == pgh.PGH_EINVAL
    p = ctx.plan(np.zeros((0, 4), np.int32), 0, 0)  # an empty plan launches nothing
    assert p.interactions == 0
    p.free()


def test_graph_capture_replays(pgh, ctx):
    """The batched launch captured in a graph and replayed several times,
    with eager work in between, matches the eager result every time."""
    import torch
    s = synth.tree_style_items(1 << 15, 150, 7, nj_median=400, nj_lo=50, nj_hi=4000)
    plan, di, dj, out, got = _newton_case(pgh, ctx, s, 1e-3)
    n = s.xi.size
    gout = [torch.zeros(n, device="cuda") for _ in range(4)]
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        plan.newton(*di, *dj, out=gout)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.newton(*di, *dj, out=gout)
    for rep in range(4):
        for t in gout:
            t.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(got, to_host(*gout)):
            rows = np.concatenate([np.arange(i0, i0 + ni) for i0, ni, _, _ in s.items])
            assert np.array_equal(a[rows], b[rows]), rep
        plan.newton(*di, *dj, out=out)  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("variant", range(TABLE_BATCH_VARIANTS))
def test_cell_list_table_force(pgh, ctx, variant):
    """Cell-grid neighbour lists in a periodic unit box (the PP part of a
    TreePM step) with the S2 table: N = 32768, 32^3 cells, 4^3-cell groups;
    every tile shape of the batched kernel."""
    assert pgh.pgh_variant_count(pgh.PGH_FAMILY_TABLE_BATCH) == TABLE_BATCH_VARIANTS
    ctx.set_variant(pgh.PGH_FAMILY_TABLE_BATCH, variant)
    n = 32768
    x, y, z = synth.uniform_box(n, 103)
    m = synth.equal_masses(n)
    rcut, eps = 1.0 / 32, 1.0 / 32 / 15
    s = synth.cell_grid_items(x, y, z, m, ncell=32, block=4)
    table = ctx.build_table(4, 6, rcut, eps=eps)
    di, dj = _dev_set(s)
    plan = ctx.plan(s.items, n, s.xj.size)
    a = np.stack(to_host(*plan.table(*di, *dj)))
    rt = oracle.lut_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, 4, 6,
                          float(np.float32(rcut)),
                          oracle_table(pgh, pgh.PGH_FAMILY_TABLE_BATCH, variant, table, 4, 6))
    rx = oracle.central_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj,
                              oracle.SHAPE_S2PP, eps, float(np.float32(rcut)))
    has = rt[3] > 0
    e1 = norm_vec_err(a[:, has], np.stack(rt[:3])[:, has], rt[3][has])
    assert rms(e1) <= 1e-5 and e1.max() <= 1e-3, (rms(e1), e1.max())
    hx = rx[4] > 0
    e2 = norm_vec_err(a[:, hx], np.stack(rx[:3])[:, hx], rx[4][hx])
    assert e2.max() <= 1e-3
    assert np.all(a[:, ~has] == 0.0)
    # the cell lists see every pair inside rcut: same result as all-pairs with
    # minimum-image separations is implied by the oracle's exact companion


def test_cell_list_table_config_full(pgh, ctx):
    """Full-size table workload: N = 262144 uniform in the unit periodic box,
    64^3 cells, 4^3-cell groups (4096 lists), S2 PP shape with rcut = 3/256,
    eps = rcut/15, E = 4, F = 6.  The oracle recomputes 96 sampled lists,
    for every variant on the default plan and for the configurations the
    bench's tuner picks among (plans for 0.5 and 1 times the resident waves,
    plain and packed, with the two-wave (H, G1) variant)."""
    n = 262144
    x, y, z = synth.uniform_box(n, 103)
    m = synth.equal_masses(n)
    rcut, eps = 3.0 / 256, 1.0 / 1280
    s = synth.cell_grid_items(x, y, z, m, ncell=64, block=4)
    table = ctx.build_table(4, 6, rcut, eps=eps)
    di, dj = _dev_set(s)
    plan = ctx.plan(s.items, n, s.xj.size)
    rng = np.random.default_rng(0)
    pick = np.unique(np.concatenate([[0, len(s.items) - 1], rng.integers(0, len(s.items), 94)]))
    items = s.items[pick]
    rows = np.concatenate([np.arange(i0, i0 + ni) for i0, ni, _, _ in items])
    fam = pgh.PGH_FAMILY_TABLE_BATCH
    for v in range(pgh.pgh_variant_count(fam)):
        ctx.set_variant(fam, v)
        rt = oracle.lut_items(items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, 4, 6,
                              float(np.float32(rcut)), oracle_table(pgh, fam, v, table, 4, 6))
        has = rt[3][rows] > 0
        a = np.stack(to_host(*plan.table(*di, *dj)))
        e1 = norm_vec_err(a[:, rows][:, has], np.stack(rt[:3])[:, rows][:, has], rt[3][rows][has])
        assert rms(e1) <= 1e-5 and e1.max() <= 1e-3, (v, rms(e1), e1.max())
        assert np.all(a[:, rows][:, ~has] == 0.0)
        assert np.all(np.isfinite(a))
    plan.free()
    names = [pgh.pgh_variant_name(fam, k) for k in range(pgh.pgh_variant_count(fam))]
    v = names.index("ki=2 tw=2 wg=2 htab")
    ctx.set_variant(fam, v)
    rt = oracle.lut_items(items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, 4, 6,
                          float(np.float32(rcut)), oracle_table(pgh, fam, v, table, 4, 6))
    has = rt[3][rows] > 0
    base = pgh.pgh_get_plan_waves(ctx.h)
    try:
        for scale, pack in ((0.5, True), (1.0, True), (0.5, False)):
            ctx.set_plan_waves(max(1, int(round(base * scale))))
            ctx.set_plan_packing(pack)
            plan = ctx.plan(s.items, n, s.xj.size)
            a = np.stack(to_host(*plan.table(*di, *dj)))
            plan.free()
            e1 = norm_vec_err(a[:, rows][:, has], np.stack(rt[:3])[:, rows][:, has],
                              rt[3][rows][has])
            assert rms(e1) <= 1e-5 and e1.max() <= 1e-3, (scale, pack, rms(e1), e1.max())
            assert np.all(a[:, rows][:, ~has] == 0.0) and np.all(np.isfinite(a))
    finally:
        ctx.set_plan_waves(0)
        ctx.set_plan_packing(False)


def test_tree_style_config_full(pgh, ctx):
    """Full-size batched Newton workload: 16384 lists over a Morton-sorted
    Plummer sphere of 2^22 particles, eps = 1e-3, i-groups of 32..256,
    j-lists log-normal (median 2000, clipped to [200, 20000]).  The oracle
    recomputes 48 lists: the longest, the shortest and random ones; every
    variant on the default plan, and the last one on a packed plan."""
    s = synth.tree_style_items(1 << 22, 16384, 104)
    cost = s.items[:, 1].astype(np.int64) * s.items[:, 3]
    rng = np.random.default_rng(1)
    pick = np.unique(np.concatenate([[np.argmax(cost), np.argmin(cost), np.argmax(s.items[:, 3])],
                                     rng.integers(0, len(s.items), 45)]))
    for v in range(pgh.pgh_variant_count(pgh.PGH_FAMILY_NEWTON_BATCH)):
        ctx.set_variant(pgh.PGH_FAMILY_NEWTON_BATCH, v)
        _newton_case(pgh, ctx, s, 1e-3, sample_items=pick)
    # a packed plan (a tuning choice of the bench's tuner)
    ctx.set_plan_packing(True)
    try:
        _newton_case(pgh, ctx, s, 1e-3, sample_items=pick)
    finally:
        ctx.set_plan_packing(False)


def test_plan_autotuner(pgh, ctx):
    """pgh_autotune_plan times both batched variants on a plan, keeps the
    fastest, and the chosen kernel still meets the parity gate."""
    s = synth.tree_style_items(1 << 15, 200, 11, nj_median=500, nj_lo=50, nj_hi=5000)
    di, dj = _dev_set(s)
    ctx.set_eps_to_all(1e-3)
    plan = ctx.plan(s.items, s.xi.size, s.xj.size)
    v = plan.autotune(pgh.PGH_FAMILY_NEWTON_BATCH, *di, *dj, reps=2)
    assert 0 <= v < pgh.pgh_variant_count(pgh.PGH_FAMILY_NEWTON_BATCH)
    assert pgh.pgh_get_variant(ctx.h, pgh.PGH_FAMILY_NEWTON_BATCH) == v
    _newton_case(pgh, ctx, s, 1e-3)
    with pytest.raises(pgh.PGHError) as e:  # the table family needs a table
        plan.autotune(pgh.PGH_FAMILY_TABLE_BATCH, *di, *dj)
    assert e.value.code == pgh.PGH_ESTATE
    with pytest.raises(pgh.PGHError) as e:
        plan.autotune(pgh.PGH_FAMILY_NEWTON_ALLPAIRS, *di, *dj)
    assert e.value.code == pgh.PGH_ERANGE


def test_plan_autotuner_table_family(pgh, ctx):
    """pgh_autotune_plan on the table family picks one of its variants, and
    the chosen kernel meets the gate against the oracle."""
    n = 16384
    x, y, z = synth.uniform_box(n, 91)
    m = synth.equal_masses(n)
    rcut = 1.0 / 32
    s = synth.cell_grid_items(x, y, z, m, ncell=32, block=4)
    table = ctx.build_table(4, 6, rcut, eps=rcut / 15)
    di, dj = _dev_set(s)
    plan = ctx.plan(s.items, n, s.xj.size)
    v = plan.autotune(pgh.PGH_FAMILY_TABLE_BATCH, *di, *dj, reps=2)
    assert pgh.pgh_get_variant(ctx.h, pgh.PGH_FAMILY_TABLE_BATCH) == v
    a = np.stack(to_host(*plan.table(*di, *dj)))
    rt = oracle.lut_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, 4, 6,
                          float(np.float32(rcut)),
                          oracle_table(pgh, pgh.PGH_FAMILY_TABLE_BATCH, v, table, 4, 6))
    has = rt[3] > 0
    e = norm_vec_err(a[:, has], np.stack(rt[:3])[:, has], rt[3][has])
    assert rms(e) <= 1e-5 and e.max() <= 1e-3, (v, rms(e), e.max())


def test_plan_autotuner_cache(pgh, ctx, tmp_path):
    """The plan autotuner's JSON cache: the first plan is timed and its
    choice stored by variant name under its shape class; a second plan of the
    same class (another seed) takes the stored variant without timing, and a
    plan of another class is timed again."""
    import json
    fam = pgh.PGH_FAMILY_TABLE_BATCH
    cache = str(tmp_path / "tune.json")
    rcut = 1.0 / 32
    ctx.build_table(4, 6, rcut, eps=rcut / 15)
    plans = []
    for seed, block in ((91, 4), (92, 4), (93, 8)):
        x, y, z = synth.uniform_box(16384, seed)
        s = synth.cell_grid_items(x, y, z, synth.equal_masses(16384), ncell=32, block=block)
        di, dj = _dev_set(s)
        plans.append((ctx.plan(s.items, 16384, s.xj.size), di, dj))
    p0, p1, p2 = plans
    assert p0[0].shape_class == p1[0].shape_class != p2[0].shape_class
    v0 = p0[0].autotune(fam, *p0[1], *p0[2], reps=2, cache=cache)
    with open(cache) as f:
        stored = json.load(f)
    assert list(stored.values()) == [pgh.pgh_variant_name(fam, v0)]
    # a stored choice is taken as is: mark it with another variant and see it come back
    other = (v0 + 1) % pgh.pgh_variant_count(fam)
    key = next(iter(stored))
    stored[key] = pgh.pgh_variant_name(fam, other)
    with open(cache, "w") as f:
        json.dump(stored, f)
    assert p1[0].autotune(fam, *p1[1], *p1[2], cache=cache) == other
    assert pgh.pgh_get_variant(ctx.h, fam) == other
    p2[0].autotune(fam, *p2[1], *p2[2], reps=2, cache=cache)
    with open(cache) as f:
        assert len(json.load(f)) == 2


def test_two_contexts_on_two_streams(pgh):
    """Two contexts, each on its own stream with its own j-memory, table and
    plans, launched interleaved: no state leaks from one to the other."""
    import torch
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ca, cb = pgh.Context(0), pgh.Context(0)
    n = 4096
    xa = synth.plummer(n, 93)
    xb = synth.plummer(n, 94)
    m = synth.equal_masses(n)
    da, db = to_dev(*xa, m), to_dev(*xb, m)
    torch.cuda.synchronize()
    outs = {}
    for rep in range(3):
        with torch.cuda.stream(sa):
            ca.set_eps_to_all(0.01)
            ca.set_j(*da)
            outs["a"] = ca.newton(da[0], da[1], da[2])
        with torch.cuda.stream(sb):
            cb.set_eps_to_all(0.05)
            cb.set_j(*db)
            outs["b"] = cb.newton(db[0], db[1], db[2])
    torch.cuda.synchronize()
    for key, x, eps in (("a", xa, 0.01), ("b", xb, 0.05)):
        ref = oracle.newton(*x, np.full(n, np.float32(eps) ** 2, np.float32), *x, m)
        a = np.stack(to_host(*outs[key][:3]))
        ea = rel_vec_err(a, np.stack(ref[:3]))
        assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (key, rms(ea), ea.max())
    ca.close()
    cb.close()


def _random_items(rng, n_items, ni_max, nj_max, long_frac):
    """Items in random order over disjoint i-ranges with gaps, j-ranges
    anywhere in the j-arrays (lists may share entries), some empty groups
    and empty lists, a fraction of long lists (split into parts)."""
    items, i_at = [], 0
    for _ in range(n_items):
        i_at += int(rng.integers(0, 3))
        ni = 0 if rng.random() < 0.05 else int(rng.integers(1, ni_max + 1))
        nj = 0 if rng.random() < 0.05 else int(rng.integers(1, nj_max + 1))
        if rng.random() < long_frac:
            nj = int(rng.integers(4 * nj_max, 12 * nj_max))
        items.append((i_at, ni, 0, nj))
        i_at += ni
    ni_total = i_at + 5
    nj_total = max(1, max(it[3] for it in items) + 100)
    items = [(a, b, int(rng.integers(0, nj_total - d + 1)), d) for a, b, _, d in items]
    order = rng.permutation(len(items))
    return np.array(items, dtype=np.int32)[order], ni_total, nj_total


@pytest.mark.parametrize("seed", range(2))
def test_device_and_host_plans_agree(pgh, ctx, seed):
    """Plans large enough for chunks of 64 (12000 random lists, empty groups
    and lists, long lists cut into parts, shared j-entries) get their tasks
    written on the device from compact entries; the same items planned on
    the host hold the same tasks, so both plans give bit-identical Newton and
    table forces, and the device plan's forces match the oracle on sampled
    rows."""
    import torch
    rng = np.random.default_rng(2000 + seed)
    items, ni_total, nj_total = _random_items(rng, 12000, 140, 700, 0.03)
    xi, yi, zi = (rng.random(ni_total).astype(np.float32) for _ in range(3))
    xj, yj, zj = (rng.random(nj_total).astype(np.float32) for _ in range(3))
    mj = rng.uniform(0.5, 1.5, nj_total).astype(np.float32) / nj_total
    di, dj = to_dev(xi, yi, zi), to_dev(xj, yj, zj, mj)
    ctx.set_eps_to_all(0.01)
    ctx.build_table(4, 6, rcut=0.05, eps=0.005)
    res = {}
    for on_device in (True, False):
        ctx.set_plan_expansion(on_device)
        plan = ctx.plan(items, ni_total, nj_total)
        outs = []
        for kind in ("newton", "table"):
            out = [torch.full((ni_total,), 777.0, device="cuda") for _ in range(4 if kind == "newton" else 3)]
            getattr(plan, kind)(*di, *dj, out=out)
            outs.append(np.stack(to_host(*out)))
        res[on_device] = outs
        plan.free()
    ctx.set_plan_expansion(True)
    for a, b in zip(res[True], res[False]):
        assert np.array_equal(a, b)
    # sampled rows of the device plan against the oracle
    pick = items[rng.choice(len(items), 40, replace=False)]
    pick = pick[(pick[:, 1] > 0)]
    e2 = np.full(ni_total, np.float32(0.01) ** 2, np.float32)
    ref = np.stack(oracle.newton_items(pick, xi, yi, zi, e2, xj, yj, zj, mj))
    rows = np.concatenate([np.arange(a, a + b) for a, b, _, _ in pick])
    rows = rows[ref[3, rows] != 0]
    got = res[True][0]
    ea = rel_vec_err(got[:3, rows], ref[:3, rows])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (rms(ea), ea.max())


@pytest.mark.parametrize("seed", range(8))
def test_random_item_sets(pgh, ctx, seed):
    """Random plans (group sizes 1..200, list lengths up to ~10^4, empty
    groups and lists, shared j-entries, long lists cut into parts, several
    device fill levels): Newton and table forces of every covered row against
    the oracle, and uncovered rows left untouched."""
    import torch
    rng = np.random.default_rng(1000 + seed)
    n_items = [3, 40, 300, 1500][seed % 4]
    items, ni_total, nj_total = _random_items(rng, n_items, 200, 900, 0.05)
    xi, yi, zi = (rng.random(ni_total).astype(np.float32) for _ in range(3))
    xj, yj, zj = (rng.random(nj_total).astype(np.float32) for _ in range(3))
    mj = rng.uniform(0.5, 1.5, nj_total).astype(np.float32) / nj_total
    di, dj = to_dev(xi, yi, zi), to_dev(xj, yj, zj, mj)
    eps = 0.01
    ctx.set_eps_to_all(eps)
    plan = ctx.plan(items, ni_total, nj_total)
    out = [torch.full((ni_total,), 777.0, device="cuda") for _ in range(4)]
    plan.newton(*di, *dj, out=out)
    got = np.stack(to_host(*out))
    e2 = np.full(ni_total, np.float32(eps) ** 2, np.float32)
    ref = np.stack(oracle.newton_items(items, xi, yi, zi, e2, xj, yj, zj, mj))
    covered = np.zeros(ni_total, bool)
    for a, b, _, _ in items:
        covered[a:a + b] = True
    assert np.all(got[:, ~covered] == 777.0)
    rows = covered & (ref[3] != 0)
    ea = rel_vec_err(got[:3, rows], ref[:3, rows])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (seed, rms(ea), ea.max())
    ep = np.abs(got[3, rows] - ref[3, rows]) / np.abs(ref[3, rows])
    assert rms(ep) <= 1e-5 and ep.max() <= 1e-3
    assert np.all(got[:, covered & (ref[3] == 0)] == 0)  # empty lists give zeros
    rcut = 0.2
    table = ctx.build_table(4, 6, rcut, eps=rcut / 15)
    # every tile shape of the batched table kernel
    fam = pgh.PGH_FAMILY_TABLE_BATCH
    for v in range(pgh.pgh_variant_count(fam)):
        ctx.set_variant(fam, v)
        rt = oracle.lut_items(items, xi, yi, zi, xj, yj, zj, mj, 4, 6, float(np.float32(rcut)),
                              oracle_table(pgh, fam, v, table, 4, 6))
        has = covered & (rt[3] > 0)
        out_t = [torch.full((ni_total,), 777.0, device="cuda") for _ in range(3)]
        plan.table(*di, *dj, out=out_t)
        a = np.stack(to_host(*out_t))
        e1 = norm_vec_err(a[:, has], np.stack(rt[:3])[:, has], rt[3][has])
        assert rms(e1) <= 1e-5 and e1.max() <= 1e-3, (seed, v, rms(e1), e1.max())
        assert np.all(a[:, ~covered] == 777.0)
        assert np.all(a[:, covered & (rt[3] == 0)] == 0)
    plan.free()


@pytest.mark.parametrize("kind", ["cells", "tree"])
def test_packed_plans(pgh, ctx, kind):
    """pgh_set_plan_packing: the rows an item leaves empty in its last chunk
    of 64 take the next item's first i-particles (a paired task).  Cell
    lists of groups of ~64 (Poisson) and tree-style lists, at wave targets
    that give chunks of 64: every row's Newton and table forces meet the
    oracle gate, rows in no item are left alone, and with device expansion
    on the packed plan is made on the host and gives the same bits."""
    import torch
    if kind == "cells":
        n = 1 << 16
        x, y, z = synth.uniform_box(n, 93)
        s = synth.cell_grid_items(x, y, z, synth.equal_masses(n), ncell=40, block=4)
    else:
        s = synth.tree_style_items(1 << 16, 180, 13, nj_median=300, nj_lo=40, nj_hi=2000)
    di, dj = _dev_set(s)
    ni_total = s.xi.size
    rcut = 0.05
    table = ctx.build_table(4, 6, rcut, eps=rcut / 15)
    ctx.set_eps_to_all(1e-3)
    rows = np.zeros(ni_total, bool)
    for i0, k, _, _ in s.items:
        rows[i0:i0 + k] = True
    assert not rows.all() or kind == "cells"
    fam = pgh.PGH_FAMILY_TABLE_BATCH
    names = [pgh.pgh_variant_name(fam, k) for k in range(pgh.pgh_variant_count(fam))]
    v = names.index("ki=2 tw=2 wg=2 htab")
    ctx.set_variant(fam, v)
    ctx.set_plan_waves(64)  # chunks of 64
    ctx.set_plan_packing(True)
    assert pgh.pgh_get_plan_packing(ctx.h) == 1
    try:
        got = {}
        for on_device in (False, True):
            ctx.set_plan_expansion(on_device)
            plan = ctx.plan(s.items, ni_total, s.xj.size)
            assert plan.packed
            outs = []
            for kind_f in ("newton", "table"):
                out = [torch.full((ni_total,), 777.0, device="cuda")
                       for _ in range(4 if kind_f == "newton" else 3)]
                getattr(plan, kind_f)(*di, *dj, out=out)
                outs.append(np.stack(to_host(*out)))
            got[on_device] = outs
            plan.free()
    finally:
        ctx.set_plan_packing(False)
        ctx.set_plan_expansion(True)
        ctx.set_plan_waves(0)
    for a, b in zip(got[False], got[True]):
        assert np.array_equal(a, b)
    newton, tab = got[False]
    assert np.all(newton[:, ~rows] == 777.0) and np.all(tab[:, ~rows] == 777.0)
    e2 = np.full(ni_total, np.float32(1e-3) ** 2, np.float32)
    ref = np.stack(oracle.newton_items(s.items, s.xi, s.yi, s.zi, e2, s.xj, s.yj, s.zj, s.mj))
    ea = rel_vec_err(newton[:3, rows], ref[:3, rows])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (rms(ea), ea.max())
    rt = oracle.lut_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, 4, 6,
                          float(np.float32(rcut)), oracle_table(pgh, fam, v, table, 4, 6))
    has = rows & (rt[3] > 0)
    e1 = norm_vec_err(tab[:, has], np.stack(rt[:3])[:, has], rt[3][has])
    assert rms(e1) <= 1e-5 and e1.max() <= 1e-3, (rms(e1), e1.max())


def test_plan_wave_targets_and_tuned_plan(pgh, ctx, tmp_path):
    """Plans cut for other wave counts (pgh_set_plan_waves: chunk sizes and
    list parts follow the target) give the same forces up to FP32 summation
    order (the oracle gate); Context.plan_tuned times plans of three wave
    targets with every variant, returns the fastest pair, and takes it from
    its JSON cache the second time.  Cell lists of 16384 particles (table
    family) and tree-style lists (Newton family)."""
    import json
    n = 16384
    x, y, z = synth.uniform_box(n, 92)
    m = synth.equal_masses(n)
    rcut = 1.0 / 32
    s = synth.cell_grid_items(x, y, z, m, ncell=32, block=4)
    table = ctx.build_table(4, 6, rcut, eps=rcut / 15)
    di, dj = _dev_set(s)
    fam = pgh.PGH_FAMILY_TABLE_BATCH
    base = pgh.pgh_get_plan_waves(ctx.h)
    assert base > 0
    with pytest.raises(pgh.PGHError) as e:
        pgh.pgh_set_plan_waves(ctx.h, -1)
    assert e.value.code == pgh.PGH_EINVAL

    def table_gate(a, v):
        rt = oracle.lut_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, 4, 6,
                              float(np.float32(rcut)), oracle_table(pgh, fam, v, table, 4, 6))
        has = rt[3] > 0
        e1 = norm_vec_err(a[:, has], np.stack(rt[:3])[:, has], rt[3][has])
        assert rms(e1) <= 1e-5 and e1.max() <= 1e-3, (v, rms(e1), e1.max())
        assert np.all(a[:, ~has] == 0.0)

    ctx.set_variant(fam, 2)
    tasks = []
    for w in (max(1, base // 4), base, 4 * base):
        ctx.set_plan_waves(w)
        assert pgh.pgh_get_plan_waves(ctx.h) == w
        plan = ctx.plan(s.items, n, s.xj.size)
        assert plan.waves == w
        table_gate(np.stack(to_host(*plan.table(*di, *dj))), 2)
        tasks.append(plan)
    for plan in tasks:
        plan.free()
    ctx.set_plan_waves(0)
    assert pgh.pgh_get_plan_waves(ctx.h) == base

    cache = str(tmp_path / "tuned.json")
    p, v, sc = ctx.plan_tuned(s.items, n, s.xj.size, fam, *di, *dj, reps=1, cache=cache)
    assert sc in (0.5, 1.0, 2.0) and pgh.pgh_get_variant(ctx.h, fam) == v
    assert p.waves == max(1, int(round(base * sc)))
    table_gate(np.stack(to_host(*p.table(*di, *dj))), v)
    p.free()
    with open(cache) as f:
        stored = json.load(f)
    assert list(stored.values()) == [{"scale": sc, "variant": pgh.pgh_variant_name(fam, v),
                                      "packing": p.packed}]
    assert pgh.pgh_get_plan_packing(ctx.h) == 0  # the context's setting is left alone
    ctx.set_variant(fam, 0)
    p2, v2, sc2 = ctx.plan_tuned(s.items, n, s.xj.size, fam, *di, *dj, reps=1, cache=cache)
    assert (v2, sc2) == (v, sc) and pgh.pgh_get_variant(ctx.h, fam) == v
    p2.free()

    st = synth.tree_style_items(1 << 15, 150, 12, nj_median=400, nj_lo=50, nj_hi=3000)
    ti, tj = _dev_set(st)
    ctx.set_eps_to_all(1e-3)
    p3, v3, _ = ctx.plan_tuned(st.items, st.xi.size, st.xj.size, pgh.PGH_FAMILY_NEWTON_BATCH,
                               *ti, *tj, reps=1)
    got = np.stack(to_host(*p3.newton(*ti, *tj)))
    rows = np.concatenate([np.arange(i0, i0 + k) for i0, k, _, _ in st.items])
    e2 = np.full(st.xi.size, np.float32(1e-3) ** 2, np.float32)
    ref = np.stack(oracle.newton_items(st.items, st.xi, st.yi, st.zi, e2, st.xj, st.yj, st.zj,
                                       st.mj))
    ea = rel_vec_err(got[:3, rows], ref[:3, rows])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (v3, rms(ea), ea.max())
    p3.free()
