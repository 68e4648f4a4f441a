"""FP64 CPU oracle for the direct-summation force path of Phantom-GRAPE
(arXiv:1203.4037).

TEST INFRASTRUCTURE ONLY: only the test-suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The library
package never does, and the two share no code: the arithmetic lives in
``pgh_oracle.c`` (plain C, double precision, OpenMP over i-particles as in the
paper's Sec. 3.5) and is wrapped here with ctypes and numpy.

Every function takes the same FP32 arrays the GPU path receives and widens
them to float64 (exactly) before the C code runs in double precision;
finite-difference checks may pass float64 arrays directly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pgh_oracle.c")
_SRCS = (_SRC, os.path.join(_HERE, "tree_oracle.c"))
_LIB = os.path.join(_HERE, "libpgh_oracle.so")

SHAPE_S2PP = 0
SHAPE_PLUMMER_TAPER = 1
SHAPE_SOFT_CUT = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp, no fast-math)."""
    stale = not os.path.exists(_LIB) or any(
        os.path.getmtime(_LIB) < os.path.getmtime(src) for src in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-Wall", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        l, i, d = ctypes.c_long, ctypes.c_int, ctypes.c_double
        sig = {
            "pgo_newton": [l, P, P, P, P, l, P, P, P, P, P, P, P, P, P],
            "pgo_newton_items": [l, P, P, P, P, P, P, P, P, P, P, P, P, P],
            "pgo_s2_R": [d, d],
            "pgo_s2pp_f": [d, d, d],
            "pgo_shape_h": [i, d, P],
            "pgo_smax": [i, i],
            "pgo_node_s": [i, i, l],
            "pgo_node_r": [i, i, d, l],
            "pgo_lut_index": [d, i, i, P],
            "pgo_scale_f32": [i, i, d],
            "pgo_pair_bin": [d, d, d, d, d, d, ctypes.c_float, i, i, P, P],
            "pgo_table_build": [i, i, d, i, P, P],
            "pgo_lut_eval": [d, i, i, P],
            "pgo_lut_items": [l, P, P, P, P, P, P, P, P, i, i, d, P, P, P, P, P],
            "pgo_central_items": [l, P, P, P, P, P, P, P, P, i, P, P, P, P, P, P],
            "pgo_newton_bwd": [l, P, P, P, P, l, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P],
            "pgo_lut_bwd_items": [l, P, P, P, P, P, P, P, P, P, P, P, i, i, d, P, P, P, l, P, P],
            "pgo_table_grad_chain": [i, i, P, P],
            "pgo_shape_p": [i, d, P],
            "pgo_pot_table_build": [i, i, d, i, P, P],
            "pgo_lut_pot_items": [l, P, P, P, P, P, P, P, P, i, i, d, P, l, P, P],
            "pgo_lut_bwd_pos_items": [l, P, P, P, P, P, P, P, P, P, P, P, i, i, d, P, l, l,
                                      P, P, P, P, P, P, P, P],
            "pgo_tree_frame": [l, P, P, P, P],
            "pgo_tree_keys": [l, P, P, P, P, P],
            "pgo_tree_sort": [l, P, P],
            "pgo_tree_build": [l, P, i, l, P, P, P, P, P, P],
            "pgo_tree_moments": [l, P, P, P, P, P, P, P, P, P],
            "pgo_sym3_eigen": [P, P, P],
            "pgo_tree_pseudo": [l, P, P, P, i, P, P, P, P],
            "pgo_tree_groups": [l, P, P, P, P, i, P],
            "pgo_tree_walk": [l, P, P, P, P, P, P, d, P, P, P, l, d, i, l, P, P],
        }
        ret = {"pgo_s2_R": d, "pgo_s2pp_f": d, "pgo_shape_h": d, "pgo_shape_p": d, "pgo_smax": d,
               "pgo_node_s": d, "pgo_node_r": d, "pgo_lut_index": l, "pgo_lut_eval": d,
               "pgo_scale_f32": ctypes.c_float, "pgo_pair_bin": l,
               "pgo_tree_build": l, "pgo_tree_groups": l, "pgo_tree_walk": l}
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ret.get(name, None)
        _lib = L
    return _lib


def _f64(a):
    """Widen to float64 (exact for the FP32 inputs the GPU receives)."""
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _items32(items):
    return np.ascontiguousarray(np.asarray(items, dtype=np.int32).reshape(-1, 4))


# --------------------------------------------------------------------------
# Newton's force (Eq. newton_force)
# --------------------------------------------------------------------------

def newton(xi, yi, zi, eps2i, xj, yj, zj, mj, self_j=None):
    """a_i = sum_j m_j d/(|d|^2+eps_i^2)^{3/2}, phi_i = -sum_j m_j/(|d|^2+eps_i^2)^{1/2}.

    ``self_j``: optional int array, per i the j index to skip (-1 none).
    Returns (ax, ay, az, phi) as float64 arrays.
    """
    xi, yi, zi, eps2i = map(_f64, (xi, yi, zi, eps2i))
    xj, yj, zj, mj = map(_f64, (xj, yj, zj, mj))
    ni, nj = xi.size, xj.size
    out = [np.zeros(ni) for _ in range(4)]
    sj = None if self_j is None else np.ascontiguousarray(self_j, dtype=np.int64)
    lib().pgo_newton(ni, _ptr(xi), _ptr(yi), _ptr(zi), _ptr(eps2i), nj, _ptr(xj), _ptr(yj),
                     _ptr(zj), _ptr(mj), _ptr(sj), *[_ptr(o) for o in out])
    return tuple(out)


def newton_items(items, xi, yi, zi, eps2i, xj, yj, zj, mj, with_phi=True):
    it = _items32(items)
    xi, yi, zi, eps2i = map(_f64, (xi, yi, zi, eps2i))
    xj, yj, zj, mj = map(_f64, (xj, yj, zj, mj))
    ni = xi.size
    out = [np.full(ni, np.nan) for _ in range(4)]
    lib().pgo_newton_items(it.shape[0], _ptr(it), _ptr(xi), _ptr(yi), _ptr(zi), _ptr(eps2i),
                           _ptr(xj), _ptr(yj), _ptr(zj), _ptr(mj), _ptr(out[0]), _ptr(out[1]),
                           _ptr(out[2]), _ptr(out[3]) if with_phi else None)
    return tuple(out)


# --------------------------------------------------------------------------
# Force shapes and the bit-binned table (Sec. 3.4, Sec. 4.2)
# --------------------------------------------------------------------------

def s2_R(r, a):
    return lib().pgo_s2_R(float(r), float(a))


def s2pp_f(r, eps, rcut):
    return lib().pgo_s2pp_f(float(r), float(eps), float(rcut))


def shape_h(shape, r, eps, rcut):
    p = np.array([eps, rcut], dtype=np.float64)
    return lib().pgo_shape_h(int(shape), float(r), _ptr(p))


def smax(E, F):
    return lib().pgo_smax(E, F)


def node_s(E, F, k):
    return lib().pgo_node_s(E, F, int(k))


def node_r(E, F, rcut, k):
    return lib().pgo_node_r(E, F, float(rcut), int(k))


def lut_index(s, E, F):
    sk = ctypes.c_double()
    k = lib().pgo_lut_index(float(s), E, F, ctypes.byref(sk))
    return int(k), sk.value


def scale_f32(E, F, rcut):
    """The FP32 scale c_f of the pair's s: the smallest float with
    fl(fl(rcut^2) c_f + 2) >= s_max."""
    return float(np.float32(lib().pgo_scale_f32(E, F, float(rcut))))


def pair_bin(xi, yi, zi, xj, yj, zj, E, F, rcut):
    """(k, s_k, clamped) of a pair, the bin taken from its FP32 s (the
    decision every table function of the oracle makes)."""
    sk, cl = ctypes.c_double(), ctypes.c_int()
    k = lib().pgo_pair_bin(float(xi), float(yi), float(zi), float(xj), float(yj), float(zj),
                           ctypes.c_float(scale_f32(E, F, rcut)), E, F, ctypes.byref(sk),
                           ctypes.byref(cl))
    return int(k), sk.value, bool(cl.value)


def table_build(E, F, rcut, shape, eps):
    """Returns the interleaved FP32 table (G0_0, G1_0, G0_1, ...) of length 2^(E+F+1)."""
    K = 1 << (E + F)
    t = np.zeros(2 * K, dtype=np.float32)
    p = np.array([eps, rcut], dtype=np.float64)
    lib().pgo_table_build(E, F, float(rcut), int(shape), _ptr(p), _ptr(t))
    return t


def lut_eval(s, E, F, table):
    t = _f64(table)
    return lib().pgo_lut_eval(float(s), E, F, _ptr(t))


def _round_f32(fr):
    """The FP32 number nearest to the rational fr (ties to an even last bit)."""
    from fractions import Fraction
    f = np.float32(float(fr))
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
    return min(cands, key=lambda c: (abs(Fraction(float(c)) - fr),
                                     int(np.array(c, np.float32).view(np.uint32)) & 1))


def table_ht(table, E, F):
    """The (H, G1) form of an interleaved FP32 table (force or potential):
    the interpolant G0_k + G1_k (s - s_k) of Sec. 3.4.2 rewritten as
    H_k + G1_k s, with H_k = G0_k - G1_k s_k rounded once to FP32 (the form
    the "htab" kernel variants keep in LDS).  Returned as a float64 table in
    the paper's form, (H_k + G1_k s_k, G1_k), so the paper-form evaluators
    (lut_items, lut_pot_items) interpolate H_k + G1_k s with it."""
    from fractions import Fraction
    K = 1 << (E + F)
    t = np.asarray(table, dtype=np.float32).reshape(K, 2)
    out = np.zeros((K, 2), dtype=np.float64)
    for k in range(K):
        g0, g1 = Fraction(float(t[k, 0])), Fraction(float(t[k, 1]))
        sk = Fraction(node_s(E, F, k))
        h = _round_f32(g0 - g1 * sk)
        out[k, 0] = float(Fraction(float(h)) + g1 * sk)
        out[k, 1] = float(g1)
    return out.reshape(-1)


def lut_items(items, xi, yi, zi, xj, yj, zj, mj, E, F, rcut, table):
    """Table force over interaction lists. Returns (ax, ay, az, absum)."""
    it = _items32(items)
    xi, yi, zi = map(_f64, (xi, yi, zi))
    xj, yj, zj, mj = map(_f64, (xj, yj, zj, mj))
    t = _f64(table)
    ni = xi.size
    out = [np.full(ni, np.nan) for _ in range(4)]
    lib().pgo_lut_items(it.shape[0], _ptr(it), _ptr(xi), _ptr(yi), _ptr(zi), _ptr(xj),
                        _ptr(yj), _ptr(zj), _ptr(mj), E, F, float(rcut), _ptr(t),
                        *[_ptr(o) for o in out])
    return tuple(out)


def central_items(items, xi, yi, zi, xj, yj, zj, mj, shape, eps, rcut):
    """Exact central force with the analytic h = f/r.  Returns (ax, ay, az,
    absum, fullsum): absum = sum m|h|r, fullsum = sum over 0 < r < rcut of
    m F(r) with F the whole force of the split (R(r, eps) for S2)."""
    it = _items32(items)
    xi, yi, zi = map(_f64, (xi, yi, zi))
    xj, yj, zj, mj = map(_f64, (xj, yj, zj, mj))
    p = np.array([eps, rcut], dtype=np.float64)
    ni = xi.size
    out = [np.full(ni, np.nan) for _ in range(5)]
    lib().pgo_central_items(it.shape[0], _ptr(it), _ptr(xi), _ptr(yi), _ptr(zi), _ptr(xj),
                            _ptr(yj), _ptr(zj), _ptr(mj), int(shape), _ptr(p),
                            *[_ptr(o) for o in out])
    return tuple(out)


# --------------------------------------------------------------------------
# Adjoints of L = sum_i w_i . a_i
# --------------------------------------------------------------------------

def newton_bwd(xi, yi, zi, eps2i, xj, yj, zj, mj, wx, wy, wz, scales=False):
    """Adjoint of L = sum_i w_i . a_i.  Returns (gxi, gyi, gzi, gxj, gyj, gzj,
    gmj), plus (absi, absj, absm) when scales: the sums of the absolute pair
    terms of the i-side, j-side and mass gradients."""
    xi, yi, zi, eps2i = map(_f64, (xi, yi, zi, eps2i))
    xj, yj, zj, mj = map(_f64, (xj, yj, zj, mj))
    wx, wy, wz = map(_f64, (wx, wy, wz))
    ni, nj = xi.size, xj.size
    gi = [np.zeros(ni) for _ in range(3)]
    gj = [np.zeros(nj) for _ in range(4)]
    sc = [np.zeros(ni), np.zeros(nj), np.zeros(nj)]
    lib().pgo_newton_bwd(ni, _ptr(xi), _ptr(yi), _ptr(zi), _ptr(eps2i), nj, _ptr(xj),
                         _ptr(yj), _ptr(zj), _ptr(mj), _ptr(wx), _ptr(wy), _ptr(wz),
                         *[_ptr(o) for o in gi], *[_ptr(o) for o in gj],
                         *[_ptr(o) for o in sc])
    out = tuple(gi) + tuple(gj)
    return out + tuple(sc) if scales else out


def lut_bwd_items(items, xi, yi, zi, xj, yj, zj, mj, wx, wy, wz, E, F, rcut, table, scales=False):
    """Returns (gtable float64[2K] interleaved like the table, gmj float64[nj]),
    plus their absolute-term sums when scales."""
    it = _items32(items)
    xi, yi, zi = map(_f64, (xi, yi, zi))
    xj, yj, zj, mj = map(_f64, (xj, yj, zj, mj))
    wx, wy, wz = map(_f64, (wx, wy, wz))
    t = _f64(table)
    K = 1 << (E + F)
    gt = np.zeros(2 * K)
    gm = np.zeros(xj.size)
    ga = np.zeros(2 * K)
    gma = np.zeros(xj.size)
    lib().pgo_lut_bwd_items(it.shape[0], _ptr(it), _ptr(xi), _ptr(yi), _ptr(zi), _ptr(xj),
                            _ptr(yj), _ptr(zj), _ptr(mj), _ptr(wx), _ptr(wy), _ptr(wz), E, F,
                            float(rcut), _ptr(t), _ptr(gt), _ptr(gm), xj.size, _ptr(ga), _ptr(gma))
    return (gt, gm, ga, gma) if scales else (gt, gm)


def table_grad_chain(E, F, gtab):
    """dL/dG0 (total) for a table whose slopes follow its node values, from
    the gradient of the interleaved (G0, G1) entries."""
    g = _f64(gtab)
    out = np.zeros(1 << (E + F))
    lib().pgo_table_grad_chain(E, F, _ptr(g), _ptr(out))
    return out


def lut_bwd_pos_items(items, xi, yi, zi, xj, yj, zj, mj, wx, wy, wz, E, F, rcut, table,
                      scales=False):
    """Position gradients of L = sum_i w_i . a_i for the table force:
    (gxi, gyi, gzi, gxj, gyj, gzj), plus (absi, absj) when scales."""
    it = _items32(items)
    xi, yi, zi = map(_f64, (xi, yi, zi))
    xj, yj, zj, mj = map(_f64, (xj, yj, zj, mj))
    wx, wy, wz = map(_f64, (wx, wy, wz))
    t = _f64(table)
    out = [np.zeros(xi.size) for _ in range(3)] + [np.zeros(xj.size) for _ in range(3)]
    sc = [np.zeros(xi.size), np.zeros(xj.size)]
    lib().pgo_lut_bwd_pos_items(it.shape[0], _ptr(it), _ptr(xi), _ptr(yi), _ptr(zi), _ptr(xj),
                                _ptr(yj), _ptr(zj), _ptr(mj), _ptr(wx), _ptr(wy), _ptr(wz), E, F,
                                float(rcut), _ptr(t), xi.size, xj.size, *[_ptr(a) for a in out],
                                _ptr(sc[0]), _ptr(sc[1]))
    return tuple(out) + (tuple(sc) if scales else ())



def shape_p(shape, r, eps, rcut):
    p = np.array([eps, rcut], dtype=np.float64)
    return lib().pgo_shape_p(int(shape), float(r), _ptr(p))


def pot_table_build(E, F, rcut, shape, eps):
    """Interleaved FP32 potential table (P0_0, P1_0, ...) of length 2^(E+F+1)."""
    K = 1 << (E + F)
    t = np.zeros(2 * K, dtype=np.float32)
    p = np.array([eps, rcut], dtype=np.float64)
    lib().pgo_pot_table_build(E, F, float(rcut), int(shape), _ptr(p), _ptr(t))
    return t


def lut_pot_items(items, xi, yi, zi, xj, yj, zj, mj, E, F, rcut, ptable):
    """(phi, absum) over the lists from a potential table."""
    it = _items32(items)
    xi, yi, zi = map(_f64, (xi, yi, zi))
    xj, yj, zj, mj = map(_f64, (xj, yj, zj, mj))
    t = _f64(ptable)
    phi = np.zeros(xi.size)
    sa = np.zeros(xi.size)
    lib().pgo_lut_pot_items(it.shape[0], _ptr(it), _ptr(xi), _ptr(yi), _ptr(zi), _ptr(xj),
                            _ptr(yj), _ptr(zj), _ptr(mj), E, F, float(rcut), _ptr(t), xi.size,
                            _ptr(phi), _ptr(sa))
    return phi, sa


# --------------------------------------------------------------------------
# Barnes-Hut tree and its interaction lists (the tree code of Sec. 5);
# the definitions are stated in tree_oracle.c.
# --------------------------------------------------------------------------

class Tree:
    """Octree of one particle set with its node moments and pseudo-particles.

    Fields: frame (lo[3], extent, scale in FP32), keys (sorted), perm (rank ->
    original index), x, y, z, m (sorted, float64 holding the FP32 inputs),
    node arrays begin, count, level, first_child, n_child, parent, moments
    mass, com [n, 3], S [n, 6] (xx, yy, zz, xy, xz, yz), pseudo-particles px,
    py, pz, pm (n_pp per node, node-major), and groups (node ids in key
    order) once ``groups(n_crit)`` has run.
    """

    def __init__(self, x, y, z, m, n_leaf, quad):
        x, y, z = (np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, z))
        n = x.size
        self.n, self.n_leaf, self.quad = n, int(n_leaf), bool(quad)
        self.npp = 3 if quad else 1
        L = lib()
        self.frame = np.zeros(5, np.float32)
        L.pgo_tree_frame(n, _ptr(x), _ptr(y), _ptr(z), _ptr(self.frame))
        keys = np.zeros(n, np.uint64)
        L.pgo_tree_keys(n, _ptr(x), _ptr(y), _ptr(z), _ptr(self.frame), _ptr(keys))
        self.perm = np.zeros(n, np.int64)
        L.pgo_tree_sort(n, _ptr(keys), _ptr(self.perm))
        self.keys = np.ascontiguousarray(keys[self.perm])
        self.x, self.y, self.z = (_f64(a[self.perm]) for a in (x, y, z))
        self.m = _f64(np.asarray(m, dtype=np.float32)[self.perm])
        cap = max(16, 2 * n + 16)
        while True:
            arrs = [np.zeros(cap, np.int64), np.zeros(cap, np.int64), np.zeros(cap, np.int32),
                    np.zeros(cap, np.int64), np.zeros(cap, np.int32), np.zeros(cap, np.int64)]
            nn = L.pgo_tree_build(n, _ptr(self.keys), self.n_leaf, cap, *[_ptr(a) for a in arrs])
            if nn >= 0:
                break
            cap *= 2
        (self.begin, self.count, self.level, self.first_child, self.n_child,
         self.parent) = (a[:nn].copy() for a in arrs)
        self.n_nodes = nn
        self.mass = np.zeros(nn)
        self.com = np.zeros((nn, 3))
        self.S = np.zeros((nn, 6))
        L.pgo_tree_moments(nn, _ptr(self.begin), _ptr(self.count), _ptr(self.x), _ptr(self.y),
                           _ptr(self.z), _ptr(self.m), _ptr(self.mass), _ptr(self.com),
                           _ptr(self.S))
        k = nn * self.npp
        self.px, self.py, self.pz, self.pm = (np.zeros(k) for _ in range(4))
        L.pgo_tree_pseudo(nn, _ptr(self.mass), _ptr(self.com), _ptr(self.S), int(self.quad),
                          _ptr(self.px), _ptr(self.py), _ptr(self.pz), _ptr(self.pm))
        self.groups = None

    @property
    def extent(self):
        return float(self.frame[3])

    def find_groups(self, n_crit):
        g = np.zeros(max(1, self.n_nodes), np.int64)
        ng = lib().pgo_tree_groups(self.n_nodes, _ptr(self.begin), _ptr(self.count),
                                   _ptr(self.n_child), _ptr(self.parent), int(n_crit), _ptr(g))
        self.groups = g[:ng].copy()
        return self.groups

    def walk(self, g, theta):
        """(src, margin) of group node g: src as in pgo_tree_walk."""
        args = (self.n_nodes, _ptr(self.begin), _ptr(self.count), _ptr(self.level),
                _ptr(self.first_child), _ptr(self.n_child), _ptr(self.com), self.extent,
                _ptr(self.x), _ptr(self.y), _ptr(self.z), int(g), float(theta), int(self.quad))
        L = lib()
        n = L.pgo_tree_walk(*args, 0, None, None)
        src = np.zeros(max(1, n), np.int64)
        mg = ctypes.c_double(0.0)
        L.pgo_tree_walk(*args, n, _ptr(src), ctypes.byref(mg))
        return src[:n], mg.value

    def list_arrays(self, src):
        """(xj, yj, zj, mj) float64 of a list given by its src entries."""
        part = src >= 0
        q = np.where(part, 0, -1 - src)
        r = np.where(part, src, 0)
        xj = np.where(part, self.x[r], self.px[q])
        yj = np.where(part, self.y[r], self.py[q])
        zj = np.where(part, self.z[r], self.pz[q])
        mj = np.where(part, self.m[r], self.pm[q])
        return xj, yj, zj, mj

    def lists(self, groups, theta):
        """Lists of the given group nodes: (items [k, 4] int64 in sorted
        particle ranks, src, xj, yj, zj, mj, margins)."""
        items, srcs, margins = [], [], []
        off = 0
        for g in groups:
            src, mg = self.walk(g, theta)
            items.append((self.begin[g], self.count[g], off, src.size))
            srcs.append(src)
            margins.append(mg)
            off += src.size
        src = np.concatenate(srcs) if srcs else np.zeros(0, np.int64)
        xj, yj, zj, mj = self.list_arrays(src)
        return (np.array(items, dtype=np.int64).reshape(-1, 4), src, xj, yj, zj, mj,
                np.array(margins))


def tree_build(x, y, z, m, n_leaf=8, quad=False):
    """Octree, moments and pseudo-particles of FP32 positions x, y, z."""
    return Tree(x, y, z, m, n_leaf, quad)


def sym3_eigen(S6):
    """Eigenvalues (descending) and eigenvectors (columns) of a symmetric 3x3
    given as (xx, yy, zz, xy, xz, yz)."""
    s = _f64(S6)
    w = np.zeros(3)
    V = np.zeros(9)
    lib().pgo_sym3_eigen(_ptr(s), _ptr(w), _ptr(V))
    return w, V.reshape(3, 3)


def tree_force(tree, theta, n_crit, eps, groups=None):
    """Tree force and potential on the sorted particles of the chosen groups
    (all by default): the direct sum over each group's list with softening
    eps (Eq. newton_force).  Returns (items, src, margins, ax, ay, az, phi)
    with rows in sorted order (rows outside the groups are zero)."""
    if tree.groups is None or groups is None:
        tree.find_groups(n_crit)
    gs = tree.groups if groups is None else np.asarray(groups)
    items, src, xj, yj, zj, mj, margins = tree.lists(gs, theta)
    e2 = np.full(tree.n, float(np.float32(eps)) ** 2)
    ax, ay, az, phi = newton_items(items, tree.x, tree.y, tree.z, e2, xj, yj, zj, mj)
    return items, src, margins, ax, ay, az, phi
