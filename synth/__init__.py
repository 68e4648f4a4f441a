"""Seeded synthetic inputs for the direct-summation force path.

Both the library's tests/benchmark and the FP64 oracle consume these arrays;
this module holds none of the force arithmetic.  It draws particle
distributions (Plummer sphere, King model, uniform periodic box), builds interaction lists
(cell-grid neighbour lists, tree-style batched groups) and loss weights.

All generators use numpy's PCG64 (``default_rng(seed)``), draw in float64 and
return float32 arrays, so inputs are bit-reproducible for a given seed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def plummer(n: int, seed: int, b: float = 1.0):
    """Plummer sphere positions (scale radius b, G = M = 1), the paper's test
    distribution (Sec. 4.1, Sec. 5.1).

    Radius by inverting the cumulative mass M(<r) = r^3/(r^2+b^2)^{3/2}:
    with X ~ U(0,1), r = b (X^{-2/3} - 1)^{-1/2}; direction isotropic.
    No truncation and no re-centring.  Returns float32 (x, y, z).
    """
    rng = np.random.default_rng(seed)
    X = rng.random(n)
    X = np.where(X == 0.0, np.finfo(np.float64).tiny, X)
    r = b / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    cth = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    x = r * sth * np.cos(ph)
    y = r * sth * np.sin(ph)
    z = r * cth
    return x.astype(np.float32), y.astype(np.float32), z.astype(np.float32)


def plummer_virial_radius(b: float = 1.0) -> float:
    """r_v = 16 b / (3 pi) for the Plummer model (G = M = 1)."""
    return 16.0 * b / (3.0 * np.pi)


def king_density(W):
    """Density of the King (1966) model at dimensionless potential W =
    Psi/sigma^2, in units of rho_1 (the DF f(E) = rho_1 (2 pi sigma^2)^{-3/2}
    (e^{E/sigma^2} - 1) integrated over velocities; Binney & Tremaine 2008,
    Eq. 4.114): e^W erf(sqrt W) - sqrt(4W/pi) (1 + 2W/3), zero for W <= 0."""
    from scipy.special import erf
    W = np.maximum(np.asarray(W, dtype=np.float64), 0.0)
    return np.exp(W) * erf(np.sqrt(W)) - np.sqrt(4.0 * W / np.pi) * (1.0 + 2.0 * W / 3.0)


def king_profile(W0: float):
    """Radial profile of a King model of central potential W0 in units of the
    King radius r_0 = sqrt(9 sigma^2 / (4 pi G rho_0)): Poisson's equation
    W'' + (2/r) W' = -9 rho(W)/rho(W0), W(0) = W0, W'(0) = 0, integrated out
    to the tidal radius r_t where W = 0.  Returns (r grid, enclosed mass
    fraction M(<r)/M, r_t); M(<r) is proportional to -r^2 W'(r)."""
    from scipy.integrate import solve_ivp
    rho0 = float(king_density(W0))

    def rhs(r, y):
        return [y[1], -9.0 * float(king_density(y[0])) / rho0 - 2.0 * y[1] / r]

    def edge(r, y):
        return y[0]

    edge.terminal = True
    edge.direction = -1
    r_start = 1e-6  # series start: W = W0 - (3/2) r^2 near the centre
    grid = np.concatenate([[r_start], np.logspace(-5.5, 6, 4000)])
    sol = solve_ivp(rhs, [r_start, 1e6], [W0 - 1.5 * r_start ** 2, -3.0 * r_start],
                    events=edge, dense_output=True, rtol=1e-11, atol=1e-13, method="DOP853")
    rt = float(sol.t_events[0][0])
    r = np.concatenate([grid[grid < rt], [rt]])
    dW = sol.sol(r)[1]
    mass = np.maximum.accumulate(-r * r * dW)  # the interpolant may dip by 1e-12 at r_t
    return r, mass / mass[-1], rt


def king(n: int, seed: int, W0: float = 9.0):
    """King-model positions (the paper's second tree-code distribution,
    Sec. 5, with W0 = 9) in units of the King radius: radii by inverting the
    enclosed-mass profile of king_profile(W0), directions isotropic.  Returns
    float32 (x, y, z)."""
    r_grid, frac, _ = king_profile(W0)
    rng = np.random.default_rng(seed)
    X = rng.random(n)
    r = np.interp(X, frac, r_grid)
    cth = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    return ((r * sth * np.cos(ph)).astype(np.float32), (r * sth * np.sin(ph)).astype(np.float32),
            (r * cth).astype(np.float32))


def uniform_box(n: int, seed: int, box: float = 1.0):
    """Uniform positions in [0, box)^3, float32."""
    rng = np.random.default_rng(seed)
    p = rng.random((3, n)) * box
    p = p.astype(np.float32)
    p[p >= np.float32(box)] = np.float32(0.0)
    return p[0].copy(), p[1].copy(), p[2].copy()


def equal_masses(n: int):
    return np.full(n, 1.0 / n, dtype=np.float32)


def weights(n: int, seed: int):
    """Loss weights w_i ~ N(0,1)^3 (float32)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((3, n)).astype(np.float32)
    return w[0].copy(), w[1].copy(), w[2].copy()


def log_uniform_pairs(n: int, seed: int, lo: float, hi: float):
    """Pair separations uniform in ln r on (lo, hi) with isotropic directions:
    the paper's table-accuracy workload (Sec. 4.2).  Returns float32
    separation vectors (dx, dy, dz) and float64 r."""
    rng = np.random.default_rng(seed)
    r = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    cth = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    d = np.stack([r * sth * np.cos(ph), r * sth * np.sin(ph), r * cth])
    return d[0].astype(np.float32), d[1].astype(np.float32), d[2].astype(np.float32), r


# --------------------------------------------------------------------------
# Interaction lists
# --------------------------------------------------------------------------

@dataclass
class ItemSet:
    """Interaction lists in the library's layout.

    items: int32 [n_items, 4] = (i_off, n_i, j_off, n_j) into the i-arrays
    and the materialised j-arrays; i-ranges are disjoint.
    xi, yi, zi: i-particle positions (sorted so every group is contiguous).
    xj, yj, zj, mj: materialised j entries (periodic images already shifted).
    jsrc: int64, for every j entry the index of the i-particle it copies.
    iperm: int64, xi[k] is particle iperm[k] of the original ordering.
    """
    items: np.ndarray
    xi: np.ndarray
    yi: np.ndarray
    zi: np.ndarray
    xj: np.ndarray
    yj: np.ndarray
    zj: np.ndarray
    mj: np.ndarray
    jsrc: np.ndarray
    iperm: np.ndarray

    @property
    def interactions(self) -> int:
        return int(np.sum(self.items[:, 1].astype(np.int64) * self.items[:, 3].astype(np.int64)))


def cell_grid_items(x, y, z, m, box: float = 1.0, ncell: int = 64, block: int = 4,
                    halo: int = 1) -> ItemSet:
    """Cell-grid neighbour lists in a periodic box (the PP part of PPPM/TreePM).

    The box is cut into ncell^3 cells.  An i-group is a block^3 cube of cells;
    its j-list holds every particle of the (block+2 halo)^3 cells around it,
    with periodic images shifted by +-box so that plain differences give the
    minimum-image separation.  Any pair closer than halo * box / ncell is in
    the list.
    """
    x = np.asarray(x, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    z = np.asarray(z, dtype=np.float32)
    m = np.asarray(m, dtype=np.float32)
    n = x.size
    h = box / ncell
    cx = np.minimum((x / h).astype(np.int64), ncell - 1)
    cy = np.minimum((y / h).astype(np.int64), ncell - 1)
    cz = np.minimum((z / h).astype(np.int64), ncell - 1)
    nb = ncell // block
    assert nb * block == ncell
    # sort particles by (block, cell) so each i-group is contiguous
    bx, by, bz = cx // block, cy // block, cz // block
    bid = (bx * nb + by) * nb + bz
    cid = (cx * ncell + cy) * ncell + cz
    order = np.lexsort((cid, bid))
    cid_sorted = cid[order]
    bid_sorted = bid[order]
    xs, ys, zs, ms = x[order], y[order], z[order], m[order]
    # cell start offsets in the sorted order
    cell_count = np.bincount(cid_sorted, minlength=ncell ** 3)
    # cells are not contiguous in sorted order across blocks; build per-cell lists
    cell_order = np.argsort(cid_sorted, kind="stable")
    cell_start = np.zeros(ncell ** 3 + 1, dtype=np.int64)
    cell_start[1:] = np.cumsum(cell_count)
    block_count = np.bincount(bid_sorted, minlength=nb ** 3)
    block_start = np.zeros(nb ** 3 + 1, dtype=np.int64)
    block_start[1:] = np.cumsum(block_count)

    w = block + 2 * halo
    offs = np.arange(-halo, block + halo)
    items = np.zeros((nb ** 3, 4), dtype=np.int64)
    jx, jy, jz, jm, js = [], [], [], [], []
    j_off = 0
    for b in range(nb ** 3):
        bxx, byy, bzz = b // (nb * nb), (b // nb) % nb, b % nb
        gx = bxx * block + offs
        gy = byy * block + offs
        gz = bzz * block + offs
        sx = np.where(gx < 0, -box, np.where(gx >= ncell, box, 0.0))
        sy = np.where(gy < 0, -box, np.where(gy >= ncell, box, 0.0))
        sz = np.where(gz < 0, -box, np.where(gz >= ncell, box, 0.0))
        gx %= ncell
        gy %= ncell
        gz %= ncell
        idx_list, shx, shy, shz = [], [], [], []
        for a in range(w):
            for c in range(w):
                for d in range(w):
                    cc = (gx[a] * ncell + gy[c]) * ncell + gz[d]
                    lo, hi = cell_start[cc], cell_start[cc + 1]
                    if hi > lo:
                        ids = cell_order[lo:hi]
                        idx_list.append(ids)
                        k = hi - lo
                        shx.append(np.full(k, sx[a]))
                        shy.append(np.full(k, sy[c]))
                        shz.append(np.full(k, sz[d]))
        if idx_list:
            ids = np.concatenate(idx_list)
            ox = np.concatenate(shx)
            oy = np.concatenate(shy)
            oz = np.concatenate(shz)
        else:
            ids = np.zeros(0, dtype=np.int64)
            ox = oy = oz = np.zeros(0)
        nj_b = ids.size
        jx.append((xs[ids].astype(np.float64) + ox).astype(np.float32))
        jy.append((ys[ids].astype(np.float64) + oy).astype(np.float32))
        jz.append((zs[ids].astype(np.float64) + oz).astype(np.float32))
        jm.append(ms[ids])
        js.append(ids)
        items[b] = (block_start[b], block_count[b], j_off, nj_b)
        j_off += nj_b
    items = items[items[:, 1] > 0]
    return ItemSet(items=items.astype(np.int32), xi=xs, yi=ys, zi=zs,
                   xj=np.concatenate(jx), yj=np.concatenate(jy), zj=np.concatenate(jz),
                   mj=np.concatenate(jm), jsrc=np.concatenate(js), iperm=order)


def morton_order(x, y, z, bits: int = 10):
    """Permutation sorting points along a Morton (Z-order) curve of their
    bounding box."""
    p = np.stack([x, y, z]).astype(np.float64)
    lo = p.min(axis=1, keepdims=True)
    hi = p.max(axis=1, keepdims=True)
    q = ((p - lo) / np.maximum(hi - lo, 1e-30) * ((1 << bits) - 1)).astype(np.uint64)
    code = np.zeros(q.shape[1], dtype=np.uint64)
    for bit in range(bits):
        for ax in range(3):
            code |= ((q[ax] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + ax)
    return np.argsort(code, kind="stable")


def tree_style_items(n: int, n_items: int, seed: int, ni_lo: int = 32, ni_hi: int = 256,
                     nj_median: float = 2000.0, nj_sigma: float = np.log(10.0) / 2.0,
                     nj_lo: int = 200, nj_hi: int = 20000) -> ItemSet:
    """Batched tree-style workload: a Morton-sorted Plummer sphere of n
    particles; i-groups are consecutive disjoint ranges with sizes uniform in
    [ni_lo, ni_hi]; each j-list draws n_j = clip(round(LogNormal(ln median,
    sigma)), nj_lo, nj_hi) particle indices uniformly with replacement and is
    materialised into one j-buffer at prefix offsets."""
    x, y, z = plummer(n, seed)
    rng = np.random.default_rng((seed, 1))  # a stream independent of the positions
    order = morton_order(x, y, z)
    x, y, z = x[order], y[order], z[order]
    m = equal_masses(n)
    n_i = rng.integers(ni_lo, ni_hi + 1, size=n_items)
    tot = int(n_i.sum())
    if tot > n:
        raise ValueError("i-groups do not fit in the particle set")
    i_off = np.zeros(n_items, dtype=np.int64)
    i_off[1:] = np.cumsum(n_i)[:-1]
    n_j = np.clip(np.rint(rng.lognormal(np.log(nj_median), nj_sigma, size=n_items)),
                  nj_lo, nj_hi).astype(np.int64)
    j_off = np.zeros(n_items, dtype=np.int64)
    j_off[1:] = np.cumsum(n_j)[:-1]
    total_j = int(n_j.sum())
    jsrc = rng.integers(0, n, size=total_j)
    items = np.stack([i_off, n_i, j_off, n_j], axis=1).astype(np.int32)
    return ItemSet(items=items, xi=x, yi=y, zi=z, xj=x[jsrc], yj=y[jsrc], zj=z[jsrc],
                   mj=m[jsrc], jsrc=jsrc, iperm=order)
