"""GPU parity of the adjoint kernels (L = sum_i w_i . a_i) against the FP64
oracle's gradients and against FP64 central finite differences, through the
C ABI and through torch.autograd.

Gate (per particle or per table bin, normalised by the sum of absolute pair
terms, with s - s_k bounded by the bin width for the G1 bins): rms <= 1e-5,
max <= 1e-3."""
import numpy as np
import pytest

import oracle
import synth
from _helpers import norm_vec_err, rms, to_dev, to_host

pytestmark = pytest.mark.gpu


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


def _gate(got, ref, scale, what):
    got = np.atleast_2d(got)
    ref = np.atleast_2d(ref)
    err = np.sqrt(np.sum((got - ref) ** 2, axis=0)) / np.maximum(scale, 1e-300)
    err = err[scale > 0]
    assert rms(err) <= 1e-5 and err.max() <= 1e-3, (what, rms(err), err.max())
    return err


def _table_gate(gt, rt, at, E, F, what):
    """G0 bins against their absolute-term sums; G1 bins against the bin
    width times the G0 scale: s is an FP32 number in the method (its bits
    pick the bin), so s - s_k carries an FP32 rounding of s that the FP64
    reference does not have, and |s - s_k| < s_{k+1} - s_k bounds each term."""
    K = 1 << (E + F)
    sk = np.array([oracle.node_s(E, F, k) for k in range(K)] + [oracle.smax(E, F)])
    width = np.maximum(np.diff(sk), 1.0)  # the last bin (s = s_max) has no width
    _gate(gt[0::2], rt[0::2], at[0::2], what + " G0")
    _gate(gt[1::2], rt[1::2], at[0::2] * width, what + " G1")


def _allpairs_gpu(pgh, ctx, x, y, z, m, eps2, w):
    import torch
    n = x.size
    d = to_dev(x, y, z, m, *w)
    out = [torch.empty(n, device="cuda") for _ in range(4)]
    pgh.pgh_newton_allpairs_bwd(ctx.h, n, d[0], d[1], d[2], d[3], eps2, d[4], d[5], d[6], *out)
    return to_host(*out)


@pytest.mark.parametrize("refine", [1, 0])
def test_allpairs_adjoint_vs_oracle(pgh, ctx, refine):
    n = 2048
    x, y, z = synth.plummer(n, 105)
    m = synth.equal_masses(n)
    eps2 = np.float32(0.01) ** 2
    w = synth.weights(n, 205)
    ctx.set_rsqrt_refine(refine)
    gx, gy, gz, gm = _allpairs_gpu(pgh, ctx, x, y, z, m, eps2, w)
    e2 = np.full(n, eps2, np.float32)
    r = oracle.newton_bwd(x, y, z, e2, x, y, z, m, *w, scales=True)
    gref = np.stack(r[0:3]) + np.stack(r[3:6])
    _gate(np.stack([gx, gy, gz]), gref, r[7] + r[8], "gx")
    _gate(gm, r[6], r[9], "gm")


def test_allpairs_adjoint_full_size_sampled(pgh, ctx):
    """N = 65536 Plummer sphere (seed 105), eps = 0.01: full GPU launch; the
    oracle recomputes both roles of 256 sampled particles."""
    n = 65536
    x, y, z = synth.plummer(n, 105)
    m = synth.equal_masses(n)
    eps2 = np.float32(0.01) ** 2
    w = synth.weights(n, 205)
    gx, gy, gz, gm = _allpairs_gpu(pgh, ctx, x, y, z, m, eps2, w)
    rng = np.random.default_rng(3)
    k = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 254)]))
    e2 = np.full(n, eps2, np.float32)
    ri = oracle.newton_bwd(x[k], y[k], z[k], e2[k], x, y, z, m, w[0][k], w[1][k], w[2][k], scales=True)
    rj = oracle.newton_bwd(x, y, z, e2, x[k], y[k], z[k], m[k], *w, scales=True)
    gref = np.stack(ri[0:3]) + np.stack(rj[3:6])
    _gate(np.stack([gx[k], gy[k], gz[k]]), gref, ri[7] + rj[8], "gx")
    _gate(gm[k], rj[6], rj[9], "gm")


@pytest.mark.parametrize("ni,nj", [(1, 1), (65, 257), (1000, 777), (300, 4100)])
def test_ij_adjoint_vs_oracle(pgh, ctx, ni, nj):
    import torch
    xi, yi, zi = synth.plummer(ni, 500 + ni)
    xj, yj, zj = synth.plummer(nj, 600 + nj)
    rng = np.random.default_rng(ni + nj)
    mj = rng.uniform(0.1, 1.0, nj).astype(np.float32)
    eps2 = rng.uniform(1e-4, 1e-2, ni).astype(np.float32)
    w = synth.weights(ni, 7)
    di = to_dev(xi, yi, zi, eps2, *w)
    dj = to_dev(xj, yj, zj, mj)
    gi = [torch.empty(ni, device="cuda") for _ in range(3)]
    gj = [torch.empty(nj, device="cuda") for _ in range(4)]
    pgh.pgh_newton_ij_bwd(ctx.h, ni, di[0], di[1], di[2], di[3], nj, *dj, di[4], di[5], di[6],
                          *gi, *gj)
    r = oracle.newton_bwd(xi, yi, zi, eps2, xj, yj, zj, mj, *w, scales=True)
    _gate(np.stack(to_host(*gi)), np.stack(r[0:3]), r[7], "gxi")
    _gate(np.stack(to_host(*gj[:3])), np.stack(r[3:6]), r[8], "gxj")
    _gate(to_host(gj[3])[0], r[6], r[9], "gmj")


def test_autograd_newton_vs_finite_differences(pgh):
    """torch.autograd through the library's adjoint against FP64 central
    differences of the oracle's forward sum."""
    import torch
    n = 96
    x, y, z = synth.plummer(n, 42)
    m = np.linspace(0.5, 1.5, n).astype(np.float32) / n
    eps = np.float32(0.05)
    w = synth.weights(n, 43)
    t = [torch.tensor(a, device="cuda", requires_grad=True) for a in (x, y, z, m)]
    ax, ay, az, phi = pgh.newton_allpairs(*t, float(eps))
    wt = to_dev(*w)
    loss = (ax * wt[0] + ay * wt[1] + az * wt[2]).sum()
    loss.backward()
    g = np.stack([to_host(tt.grad)[0] for tt in t])

    X = [a.astype(np.float64) for a in (x, y, z)]
    e2 = np.full(n, np.float64(eps) ** 2)

    def L(P, M):
        a = oracle.newton(*P, e2, *P, M)
        return float(sum(np.sum(w[k] * a[k]) for k in range(3)))

    h = 1e-6
    fd = np.zeros((4, n))
    for ax_ in range(3):
        for k in range(n):
            p = [a.copy() for a in X]; q = [a.copy() for a in X]
            p[ax_][k] += h; q[ax_][k] -= h
            fd[ax_, k] = (L(p, m) - L(q, m)) / (2 * h)
    M = m.astype(np.float64)
    for k in range(n):
        p = M.copy(); p[k] += 1e-3
        q = M.copy(); q[k] -= 1e-3
        fd[3, k] = (L(X, p) - L(X, q)) / 2e-3
    for r in range(4):
        err = np.abs(g[r] - fd[r]) / np.abs(fd[r]).max()
        assert err.max() < 1e-4, (r, err.max())


def test_table_adjoint_cell_lists(pgh, ctx):
    """The table-force adjoint on cell lists: N = 65536 uniform in the unit
    periodic box, 64^3 cells, 8^3-cell groups, S2 PP shape (rcut = 3/256,
    eps = 1/1280, E = 4, F = 6); gradients with respect to every (G0, G1)
    entry and to the j masses."""
    import torch
    n = 65536
    x, y, z = synth.uniform_box(n, 105)
    m = synth.equal_masses(n)
    rcut, eps = 3.0 / 256, 1.0 / 1280
    s = synth.cell_grid_items(x, y, z, m, ncell=64, block=8)
    table = ctx.build_table(4, 6, rcut, eps=eps)
    w = synth.weights(n, 305)
    plan = ctx.plan(s.items, n, s.xj.size)
    di = to_dev(s.xi, s.yi, s.zi, *w)
    dj = to_dev(s.xj, s.yj, s.zj, s.mj)
    gt = torch.empty(table.size, device="cuda")
    gm = torch.empty(s.xj.size, device="cuda")
    pgh.pgh_batch_table_bwd(ctx.h, plan.h, di[0], di[1], di[2], *dj, di[3], di[4], di[5], gt, gm)
    rt, rm, at, am = oracle.lut_bwd_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, *w,
                                          4, 6, float(np.float32(rcut)), table, scales=True)
    _table_gate(to_host(gt)[0], rt, at, 4, 6, "gtable")
    _gate(to_host(gm)[0], rm, am, "gmj")


def test_autograd_table_force(pgh, ctx):
    """TableForceBatch: gradients of the table, the masses and the i- and
    j-positions against the oracle."""
    import torch
    n = 8192
    x, y, z = synth.uniform_box(n, 9)
    m = synth.equal_masses(n)
    rcut, eps, E, F = 1.0 / 16, 1.0 / 16 / 15, 4, 5
    s = synth.cell_grid_items(x, y, z, m, ncell=16, block=4)
    table = ctx.build_table(E, F, rcut, eps=eps)
    plan = ctx.plan(s.items, n, s.xj.size)
    tab = torch.tensor(table, device="cuda", requires_grad=True)
    mj = torch.tensor(s.mj, device="cuda", requires_grad=True)
    di = to_dev(s.xi, s.yi, s.zi)
    dj = to_dev(s.xj, s.yj, s.zj)
    w = to_dev(*synth.weights(n, 1))
    ax, ay, az = pgh.table_force_batch(plan, E, F, rcut, tab, *di, *dj, mj)
    (ax * w[0] + ay * w[1] + az * w[2]).sum().backward()
    rt, rm, at, am = oracle.lut_bwd_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj,
                                          *[to_host(t)[0] for t in w], E, F,
                                          float(np.float32(rcut)), table, scales=True)
    _table_gate(to_host(tab.grad)[0], rt, at, E, F, "gtable")
    _gate(to_host(mj.grad)[0], rm, am, "gmj")
    # position gradients through autograd
    xi_ = [t.clone().requires_grad_(True) for t in di]
    xj_ = [t.clone().requires_grad_(True) for t in dj]
    ax, ay, az = pgh.table_force_batch(plan, E, F, rcut, tab.detach(), *xi_, *xj_, mj.detach())
    (ax * w[0] + ay * w[1] + az * w[2]).sum().backward()
    r = oracle.lut_bwd_pos_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj,
                                 *[to_host(t)[0] for t in w], E, F, float(np.float32(rcut)), table,
                                 scales=True)
    _gate(np.stack([to_host(t.grad)[0] for t in xi_]), np.stack(r[0:3]), r[6], "gxi")
    _gate(np.stack([to_host(t.grad)[0] for t in xj_]), np.stack(r[3:6]), r[7], "gxj")


def test_table_adjoint_partial_outputs_and_repeats(pgh, ctx):
    """Asking for only the table gradient, or only the mass gradient, gives
    what the combined call gives (up to the order of float atomics), and
    repeated calls on one plan restart from zero."""
    import torch
    n = 16384
    x, y, z = synth.uniform_box(n, 21)
    m = synth.equal_masses(n)
    rcut, eps, E, F = 1.0 / 32, 1.0 / 32 / 15, 4, 6
    s = synth.cell_grid_items(x, y, z, m, ncell=32, block=4)
    table = ctx.build_table(E, F, rcut, eps=eps)
    w = synth.weights(n, 22)
    plan = ctx.plan(s.items, n, s.xj.size)
    di = to_dev(s.xi, s.yi, s.zi, *w)
    dj = to_dev(s.xj, s.yj, s.zj, s.mj)
    gt = torch.empty(table.size, device="cuda")
    gm = torch.empty(s.xj.size, device="cuda")
    both = []
    for _ in range(2):
        pgh.pgh_batch_table_bwd(ctx.h, plan.h, di[0], di[1], di[2], *dj, di[3], di[4], di[5], gt, gm)
        both.append((to_host(gt)[0], to_host(gm)[0]))
    gt2 = torch.full((table.size,), 7.0, device="cuda")
    gm2 = torch.full((s.xj.size,), 7.0, device="cuda")
    pgh.pgh_batch_table_bwd(ctx.h, plan.h, di[0], di[1], di[2], *dj, di[3], di[4], di[5], gt2, None)
    pgh.pgh_batch_table_bwd(ctx.h, plan.h, di[0], di[1], di[2], *dj, di[3], di[4], di[5], None, gm2)
    rt, rm, at, am = oracle.lut_bwd_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, *w,
                                          E, F, float(np.float32(rcut)), table, scales=True)
    for g_t, g_m in both + [(to_host(gt2)[0], to_host(gm2)[0])]:
        _table_gate(g_t, rt, at, E, F, "gtable")
        _gate(g_m, rm, am, "gmj")


@pytest.mark.parametrize("E,F", [(4, 6), (2, 3), (0, 4)])
def test_table_grad_chain_kernel(pgh, ctx, E, F):
    """pgh_table_grad_chain against the oracle's chain rule on the same
    gradient entries (and, for E = 4, F = 6, on the adjoint's own output)."""
    import torch
    K = 1 << (E + F)
    g = np.random.default_rng(E * 16 + F).standard_normal(2 * K).astype(np.float32)
    out = torch.empty(K, device="cuda")
    pgh.pgh_table_grad_chain(ctx.h, E, F, to_dev(g)[0], out)
    ref = oracle.table_grad_chain(E, F, g)
    nodes = np.array([oracle.node_s(E, F, k) for k in range(K)])
    ds = np.diff(nodes)
    scale = np.abs(g[0::2]).astype(np.float64)
    scale[1:] += np.abs(g[1:2 * K - 2:2]) / ds
    scale[:-1] += np.abs(g[1:2 * K - 2:2]) / ds
    err = np.abs(to_host(out)[0] - ref) / scale
    assert err.max() < 4e-7, err.max()


def test_self_potential_correction(pgh, ctx):
    """Raw potentials plus pgh_correct_self_potential equal the oracle's
    potential with the self pair skipped (Sec. 4.1), for one eps and for
    per-particle eps^2."""
    import torch
    n = 2048
    x, y, z = synth.plummer(n, 31)
    m = np.linspace(0.5, 1.5, n).astype(np.float32) / n
    d = to_dev(x, y, z, m)
    ctx.set_j(*d)
    for e2 in (None, np.random.default_rng(3).uniform(1e-4, 4e-4, n).astype(np.float32)):
        if e2 is None:
            ctx.set_eps_to_all(0.01)
            e2h = np.full(n, np.float32(0.01) ** 2, np.float32)
            e2d = None
        else:
            e2h, e2d = e2, to_dev(e2)[0]
        ax, ay, az, phi = ctx.newton(d[0], d[1], d[2], eps2=e2d)
        pgh.pgh_correct_self_potential(ctx.h, n, d[3], e2d, phi)
        ref = oracle.newton(x, y, z, e2h, x, y, z, m, self_j=np.arange(n))
        ep = np.abs(to_host(phi)[0] - ref[3]) / np.abs(ref[3])
        assert rms(ep) <= 1e-5 and ep.max() <= 1e-3, (rms(ep), ep.max())
    phi2 = pgh.correct_self_potential(torch.zeros(n, device="cuda"), d[3], eps=0.5, lib_ctx=ctx)
    assert np.allclose(to_host(phi2)[0], m / np.float32(0.5), rtol=1e-6)


@pytest.mark.parametrize("block", [4, 8])
def test_table_position_gradients_cell_lists(pgh, ctx, block):
    """i- and j-side position gradients of the table force on cell lists
    (N = 16384 uniform in the unit periodic box, 32^3 cells, S2 table with
    rcut = 1/32, E = 4, F = 6), alone and together with the table and mass
    gradients, against the oracle."""
    import torch
    n = 16384
    x, y, z = synth.uniform_box(n, 41)
    m = synth.equal_masses(n)
    rcut, eps, E, F = 1.0 / 32, 1.0 / 32 / 15, 4, 6
    s = synth.cell_grid_items(x, y, z, m, ncell=32, block=block)
    table = ctx.build_table(E, F, rcut, eps=eps)
    w = synth.weights(n, 42)
    plan = ctx.plan(s.items, n, s.xj.size)
    di = to_dev(s.xi, s.yi, s.zi, *w)
    dj = to_dev(s.xj, s.yj, s.zj, s.mj)
    r = oracle.lut_bwd_pos_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, *w, E, F,
                                 float(np.float32(rcut)), table, scales=True)
    rt, rm, at, am = oracle.lut_bwd_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, *w,
                                          E, F, float(np.float32(rcut)), table, scales=True)
    for with_rest in (False, True):
        gi = [torch.full((n,), 7.0, device="cuda") for _ in range(3)]
        gj = [torch.full((s.xj.size,), 7.0, device="cuda") for _ in range(3)]
        gt = torch.empty(table.size, device="cuda") if with_rest else None
        gm = torch.empty(s.xj.size, device="cuda") if with_rest else None
        pgh.pgh_batch_table_bwd(ctx.h, plan.h, di[0], di[1], di[2], *dj, di[3], di[4], di[5],
                                gt, gm, *gi, *gj)
        _gate(np.stack(to_host(*gi)), np.stack(r[0:3]), r[6], "gxi")
        _gate(np.stack(to_host(*gj)), np.stack(r[3:6]), r[7], "gxj")
        assert np.all(np.isfinite(np.stack(to_host(*gi))))
        if with_rest:
            _table_gate(to_host(gt)[0], rt, at, E, F, "gtable")
            _gate(to_host(gm)[0], rm, am, "gmj")
    with pytest.raises(pgh.PGHError):  # triples only
        pgh.pgh_batch_table_bwd(ctx.h, plan.h, di[0], di[1], di[2], *dj, di[3], di[4], di[5],
                                None, None, gi[0], None, None)


def test_table_adjoint_largest_table(pgh, ctx):
    """E + F = 13, the largest table the adjoint holds in LDS (8192 nodes and
    their gradient sums, 128 KiB: one workgroup per CU): table, mass and
    both position gradients, and the moments path, on cell lists (N = 16384
    uniform in the unit periodic box, 32^3 cells, S2 table with rcut = 1/32,
    E = 5, F = 8) against the oracle."""
    import torch
    n = 16384
    x, y, z = synth.uniform_box(n, 46)
    m = synth.equal_masses(n)
    rcut, eps, E, F = 1.0 / 32, 1.0 / 32 / 15, 5, 8
    rc = float(np.float32(rcut))
    s = synth.cell_grid_items(x, y, z, m, ncell=32, block=4)
    table = ctx.build_table(E, F, rcut, eps=eps)
    w = synth.weights(n, 47)
    plan = ctx.plan(s.items, n, s.xj.size)
    di = to_dev(s.xi, s.yi, s.zi, *w)
    dj = to_dev(s.xj, s.yj, s.zj, s.mj)
    r = oracle.lut_bwd_pos_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, *w, E, F,
                                 rc, table, scales=True)
    rt, rm, at, am = oracle.lut_bwd_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, *w,
                                          E, F, rc, table, scales=True)
    gi = [torch.full((n,), 7.0, device="cuda") for _ in range(3)]
    gj = [torch.full((s.xj.size,), 7.0, device="cuda") for _ in range(3)]
    gt = torch.empty(table.size, device="cuda")
    gm = torch.empty(s.xj.size, device="cuda")
    pgh.pgh_batch_table_bwd(ctx.h, plan.h, di[0], di[1], di[2], *dj, di[3], di[4], di[5],
                            gt, gm, *gi, *gj)
    _gate(np.stack(to_host(*gi)), np.stack(r[0:3]), r[6], "gxi")
    _gate(np.stack(to_host(*gj)), np.stack(r[3:6]), r[7], "gxj")
    _table_gate(to_host(gt)[0], rt, at, E, F, "gtable")
    _gate(to_host(gm)[0], rm, am, "gmj")
    # the moments path: its forward meets the force gate, its i-side
    # gradient the adjoint's
    out = [torch.empty(n, device="cuda") for _ in range(3)]
    mom = torch.empty(7 * n, device="cuda")
    pgh.pgh_batch_table_moments(ctx.h, plan.h, *di[:3], *dj, *out, mom)
    ra = oracle.lut_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, E, F, rc, table)
    e1 = norm_vec_err(np.stack(to_host(*out)), np.stack(ra[:3]), ra[3])
    assert rms(e1) <= 1e-5 and e1.max() <= 1e-3, (rms(e1), e1.max())
    gi2 = [torch.full((n,), 7.0, device="cuda") for _ in range(3)]
    pgh.pgh_batch_table_bwd_moments(ctx.h, plan.h, *di[:3], *dj, *di[3:], mom, None, None,
                                    *gi2, None, None, None)
    _gate(np.stack(to_host(*gi2)), np.stack(r[0:3]), r[6], "gxi (moments)")
    plan.free()


@pytest.mark.parametrize("E,F", [(4, 6), (4, 7), (5, 8)])
def test_table_adjoint_many_small_lists(pgh, ctx, E, F):
    """40000 short lists (1..8 rows against 1..24 shared j-entries): about
    80000 adjoint tasks, more than four per resident wave, so the waves of
    each workgroup take their tasks from its LDS counter; for E + F = 10, 11
    and 13 (four, two and one workgroup per CU).  Every gradient, and the
    i-side gradient from the moments, against the oracle."""
    import torch
    rng = np.random.default_rng(48 + F)
    items, i_at = [], 0
    for _ in range(40000):
        i_at += int(rng.integers(0, 2))
        ni, nj = int(rng.integers(1, 9)), int(rng.integers(1, 25))
        items.append((i_at, ni, 0, nj))
        i_at += ni
    ni_total, nj_total = i_at, 20000
    items = np.array([(a, b, int(rng.integers(0, nj_total - d + 1)), d) for a, b, _, d in items],
                     np.int32)[rng.permutation(len(items))]
    xi, yi, zi = (rng.random(ni_total).astype(np.float32) * 0.1 for _ in range(3))
    xj, yj, zj = (rng.random(nj_total).astype(np.float32) * 0.1 for _ in range(3))
    mj = rng.uniform(0.5, 1.5, nj_total).astype(np.float32) / nj_total
    w = [rng.standard_normal(ni_total).astype(np.float32) for _ in range(3)]
    rcut, eps = 0.06, 0.004
    rc = float(np.float32(rcut))
    table = ctx.build_table(E, F, rcut, eps=eps)
    plan = ctx.plan(items, ni_total, nj_total)
    di = to_dev(xi, yi, zi, *w)
    dj = to_dev(xj, yj, zj, mj)
    gi = [torch.full((ni_total,), 7.0, device="cuda") for _ in range(3)]
    gj = [torch.full((nj_total,), 7.0, device="cuda") for _ in range(3)]
    gt = torch.empty(table.size, device="cuda")
    gm = torch.empty(nj_total, device="cuda")
    pgh.pgh_batch_table_bwd(ctx.h, plan.h, *di[:3], *dj, *di[3:], gt, gm, *gi, *gj)
    r = oracle.lut_bwd_pos_items(items, xi, yi, zi, xj, yj, zj, mj, *w, E, F, rc, table,
                                 scales=True)
    rt, rm, at, am = oracle.lut_bwd_items(items, xi, yi, zi, xj, yj, zj, mj, *w, E, F, rc, table,
                                          scales=True)
    _gate(np.stack(to_host(*gi)), np.stack(r[0:3]), r[6], "gxi")
    _gate(np.stack(to_host(*gj)), np.stack(r[3:6]), r[7], "gxj")
    _table_gate(to_host(gt)[0], rt, at, E, F, "gtable")
    _gate(to_host(gm)[0], rm, am, "gmj")
    out = [torch.empty(ni_total, device="cuda") for _ in range(3)]
    mom = torch.empty(7 * ni_total, device="cuda")
    pgh.pgh_batch_table_moments(ctx.h, plan.h, *di[:3], *dj, *out, mom)
    gi2 = [torch.full((ni_total,), 7.0, device="cuda") for _ in range(3)]
    pgh.pgh_batch_table_bwd_moments(ctx.h, plan.h, *di[:3], *dj, *di[3:], mom, gt, gm, *gi2,
                                    None, None, None)
    _gate(np.stack(to_host(*gi2)), np.stack(r[0:3]), r[6], "gxi (moments)")
    _table_gate(to_host(gt)[0], rt, at, E, F, "gtable (moments call)")
    _gate(to_host(gm)[0], rm, am, "gmj (moments call)")
    plan.free()


def test_table_adjoint_graph_replays(pgh, ctx):
    """The table adjoint (zeroing prologue, persistent kernel, summing kernel)
    captured in a graph and replayed several times with eager work in
    between: every replay matches the eager call (float atomics: to rounding)."""
    import torch
    n = 16384
    x, y, z = synth.uniform_box(n, 81)
    m = synth.equal_masses(n)
    s = synth.cell_grid_items(x, y, z, m, ncell=32, block=4)
    table = ctx.build_table(4, 6, 1.0 / 32, eps=1.0 / 480)
    plan = ctx.plan(s.items, n, s.xj.size)
    di = to_dev(s.xi, s.yi, s.zi, *synth.weights(n, 82))
    dj = to_dev(s.xj, s.yj, s.zj, s.mj)
    gt = torch.empty(table.size, device="cuda")
    gm = torch.empty(s.xj.size, device="cuda")
    gi = [torch.empty(n, device="cuda") for _ in range(3)]

    def call():
        pgh.pgh_batch_table_bwd(ctx.h, plan.h, di[0], di[1], di[2], *dj, di[3], di[4], di[5],
                                gt, gm, *gi)

    ctx._sync_stream()
    call()
    torch.cuda.synchronize()
    ref = [to_host(t)[0].copy() for t in (gt, gm, *gi)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx._sync_stream()
        call()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx._sync_stream()
        call()
    for rep in range(3):
        for t in (gt, gm, *gi):
            t.fill_(123.0)
        g.replay()
        torch.cuda.synchronize()
        for r, t in zip(ref, (gt, gm, *gi)):
            got = to_host(t)[0]
            tol = 1e-4 * (np.abs(r) + np.abs(r).max())  # float atomics add in any order
            assert np.all(np.abs(got - r) <= tol), rep
        ctx._sync_stream()
        call()  # eager work between replays
        torch.cuda.synchronize()


def test_table_moments_path(pgh, ctx):
    """pgh_batch_table_moments and pgh_batch_table_bwd_moments through the C
    ABI: the forward's force meets the table gate; the i-side gradient formed
    from the saved moments meets the same gate against the oracle's adjoint
    as the two-pass one does, with the other gradients unchanged; rows in no
    item get a zero gradient and keep their moment entries; and lists long
    enough to be cut into parts (their moments added by the combine kernel)
    give the same; so do lists with disjoint j-ranges that leave entries out,
    whose per-entry gradients are stored rather than added."""
    import torch
    rcut, eps, E, F = 1.0 / 32, 1.0 / 32 / 15, 4, 6
    table = ctx.build_table(E, F, rcut, eps=eps)
    rc = float(np.float32(rcut))

    def check(items, xi, yi, zi, xj, yj, zj, mj, w, what, rest=True):
        ni, nj = xi.size, xj.size
        plan = ctx.plan(items, ni, nj)
        di = to_dev(xi, yi, zi, *w)
        dj = to_dev(xj, yj, zj, mj)
        out = [torch.full((ni,), 7.0, device="cuda") for _ in range(3)]
        mom = torch.full((7 * ni,), 5.0, device="cuda")
        pgh.pgh_batch_table_moments(ctx.h, plan.h, *di[:3], *dj, *out, mom)
        rows = np.zeros(ni, bool)
        for i0, k, _, _ in items:
            rows[i0:i0 + k] = True
        a = np.stack(to_host(*out))
        rt = oracle.lut_items(items, xi, yi, zi, xj, yj, zj, mj, E, F, rc, table)
        has = rows & (rt[3] > 0)
        e1 = norm_vec_err(a[:, has], np.stack(rt[:3])[:, has], rt[3][has])
        assert rms(e1) <= 1e-5 and e1.max() <= 1e-3, (what, rms(e1), e1.max())
        assert np.all(a[:, ~rows] == 7.0)
        mh = to_host(mom)[0].reshape(7, ni)
        assert np.all(mh[:, ~rows] == 5.0) and np.all(np.isfinite(mh[:, rows]))
        gi = [torch.full((ni,), 3.0, device="cuda") for _ in range(3)]
        gj = [torch.full((nj,), 3.0, device="cuda") for _ in range(3)]
        gt = torch.full((table.size,), 3.0, device="cuda")
        gm = torch.full((nj,), 3.0, device="cuda")
        pgh.pgh_batch_table_bwd_moments(ctx.h, plan.h, *di[:3], *dj, *di[3:], mom, gt, gm, *gi,
                                        *gj)
        r = oracle.lut_bwd_pos_items(items, xi, yi, zi, xj, yj, zj, mj, *w, E, F, rc, table,
                                     scales=True)
        rtab, rm, at, am = oracle.lut_bwd_items(items, xi, yi, zi, xj, yj, zj, mj, *w, E, F, rc,
                                                table, scales=True)
        g = np.stack(to_host(*gi))
        _gate(g[:, rows], np.stack(r[0:3])[:, rows], r[6][rows], what + " gxi")
        assert np.all(g[:, ~rows] == 0.0)
        _gate(np.stack(to_host(*gj)), np.stack(r[3:6]), r[7], what + " gxj")
        jrows = np.zeros(nj, bool)
        for i0, k, j0, kj in items:
            if k > 0:
                jrows[j0:j0 + kj] = True
        assert np.all(np.stack(to_host(*gj))[:, ~jrows] == 0.0)
        assert np.all(to_host(gm)[0][~jrows] == 0.0)
        if rest:
            _table_gate(to_host(gt)[0], rtab, at, E, F, what + " gtable")
            _gate(to_host(gm)[0], rm, am, what + " gmj")
        with pytest.raises(pgh.PGHError):
            pgh.pgh_batch_table_bwd_moments(ctx.h, plan.h, *di[:3], *dj, *di[3:], None, gt, gm,
                                            *gi, *gj)
        plan.free()

    # cell lists with every row in a list
    n = 16384
    x, y, z = synth.uniform_box(n, 43)
    m = synth.equal_masses(n)
    s = synth.cell_grid_items(x, y, z, m, ncell=32, block=4)
    check(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, synth.weights(n, 44), "cells")
    # rows in no list, and long lists cut into parts
    n = 6000
    x, y, z = synth.uniform_box(n, 45, box=0.1)
    m = synth.equal_masses(n)
    items = np.array([[0, 1500, 0, n], [1700, 2000, 0, n], [4000, 37, 100, 3000],
                      [5000, 900, 2500, n - 2500]], np.int32)
    # (the table and mass gradients come from the j-major pass that
    # pgh_batch_table_bwd runs too; in this dense box a bin gathers ~1e5 float
    # atomics, whose FP32 sum errs by more than the rms gate allows, so they
    # are checked on the cell lists above only)
    check(items, x, y, z, x, y, z, m, synth.weights(n, 46), "gaps and parts", rest=False)
    # disjoint j-ranges that leave j-entries out (their gradients are stored,
    # the entries outside set to zero), twice in a row (the second call finds
    # the gradient copies cleared by the first)
    items = np.array([[0, 1500, 0, 2000], [1700, 2000, 2500, 1500], [4000, 37, 4100, 900]],
                     np.int32)
    for rep in range(2):
        check(items, x, y, z, x, y, z, m, synth.weights(n, 47 + rep), f"disjoint j {rep}",
              rest=False)
