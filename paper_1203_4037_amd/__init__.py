"""Python binding of libpgh, an MI355X (gfx950) direct-summation force library
in the shape of Phantom-GRAPE (Tanikawa et al., arXiv:1203.4037).

The binding only marshals arguments: every step of the force path runs in the
HIP kernels of ``libpgh.so`` (built by ``paper_1203_4037_amd/build.py``).  PyTorch
provides device memory and streams: tensors are passed as device pointers and
every call runs on torch's current stream.  Importing this package on a
machine where the library has not been built raises immediately; there is no
CPU fallback.

Two layers:
  * ``pgh_*`` functions with the names and argument order of include/pgh.h,
    taking torch tensors where the C ABI takes device pointers;
  * ``Context``, a small object-oriented wrapper that allocates outputs.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # first, so that libpgh binds to the HIP runtime torch has loaded

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpgh.so")

PGH_OK, PGH_EINVAL, PGH_ESTATE, PGH_ENOMEM, PGH_EHIP, PGH_ERANGE = 0, -1, -2, -3, -4, -5
PGH_KIND_NEWTON, PGH_KIND_TABLE = 0, 1
PGH_FAMILY_NEWTON_ALLPAIRS, PGH_FAMILY_TABLE_ALLPAIRS = 0, 1
PGH_FAMILY_NEWTON_BATCH, PGH_FAMILY_TABLE_BATCH = 2, 3

_STATUS = {PGH_EINVAL: "PGH_EINVAL", PGH_ESTATE: "PGH_ESTATE", PGH_ENOMEM: "PGH_ENOMEM",
           PGH_EHIP: "PGH_EHIP", PGH_ERANGE: "PGH_ERANGE"}

F_OVER_R = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_double, ctypes.c_void_p)


class PGHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class PghTreeStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("n_nodes", ctypes.c_int), ("n_leaves", ctypes.c_int),
                ("depth", ctypes.c_int), ("n_groups", ctypes.c_int),
                ("max_level_nodes", ctypes.c_int), ("max_frontier", ctypes.c_int),
                ("n_leaf", ctypes.c_int),
                ("n_crit", ctypes.c_int), ("quad", ctypes.c_int), ("walked", ctypes.c_int),
                ("theta", ctypes.c_float), ("frame", ctypes.c_float * 5),
                ("n_entries", ctypes.c_longlong), ("interactions", ctypes.c_longlong)]


# Tree fields of pgh_tree_get: (enum value, numpy dtype, trailing shape)
PGH_TREE_FIELDS = {
    "perm": (0, np.int32, ()), "keys": (1, np.uint64, ()),
    "x": (2, np.float32, ()), "y": (3, np.float32, ()), "z": (4, np.float32, ()),
    "m": (5, np.float32, ()),
    "node_begin": (6, np.int32, ()), "node_count": (7, np.int32, ()),
    "node_level": (8, np.int32, ()), "node_first_child": (9, np.int32, ()),
    "node_n_child": (10, np.int32, ()), "node_parent": (11, np.int32, ()),
    "moments": (12, np.float64, (10,)), "pseudo": (13, np.float32, (4,)),
    "groups": (14, np.int32, ()), "items": (15, np.int32, (4,)),
    "list_x": (16, np.float32, ()), "list_y": (17, np.float32, ()),
    "list_z": (18, np.float32, ()), "list_m": (19, np.float32, ()),
    "list_src": (20, np.int32, ()),
}


class PghItem(ctypes.Structure):
    _fields_ = [("i_off", ctypes.c_int), ("n_i", ctypes.c_int), ("j_off", ctypes.c_int),
                ("n_j", ctypes.c_int)]


# The exported symbols of libpgh and their C signatures.
_P, _I, _F, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
SIGNATURES = {
    "pgh_open": (_I, [ctypes.POINTER(_P), _I, _P]),
    "pgh_close": (_I, [_P]),
    "pgh_last_error": (ctypes.c_char_p, [_P]),
    "pgh_version": (_I, []),
    "pgh_set_stream": (_I, [_P, _P]),
    "pgh_set_eps_to_all": (_I, [_P, _F]),
    "pgh_set_n": (_I, [_P, _I]),
    "pgh_set_xmj": (_I, [_P, _I, _I, _P, _P, _P, _P]),
    "pgh_set_rsqrt_refine": (_I, [_P, _I]),
    "pgh_set_plan_expansion": (_I, [_P, _I]),
    "pgh_set_plan_waves": (_I, [_P, _I]),
    "pgh_get_plan_waves": (_I, [_P]),
    "pgh_set_plan_packing": (_I, [_P, _I]),
    "pgh_get_plan_packing": (_I, [_P]),
    "pgh_calc_newton": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pgh_calc_newton_noalloc": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pgh_build_table": (_I, [_P, _I, _I, _F, _P, _P, _P]),
    "pgh_table_compute": (_I, [_I, _I, _F, _P, _P, _P]),
    "pgh_set_table": (_I, [_P, _I, _I, _F, _P]),
    "pgh_s2pp_f_over_r": (_D, [_D, _P]),
    "pgh_calc_table": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P]),
    "pgh_build_pot_table": (_I, [_P, _P, _P, _P]),
    "pgh_set_pot_table": (_I, [_P, _P]),
    "pgh_plan_create": (_I, [_P, _I, _P, _I, _I, ctypes.POINTER(_P)]),
    "pgh_plan_free": (_I, [_P, _P]),
    "pgh_plan_interactions": (ctypes.c_longlong, [_P]),
    "pgh_batch_newton": (_I, [_P, _P] + [_P] * 12),
    "pgh_batch_table": (_I, [_P, _P] + [_P] * 11),
    "pgh_newton_allpairs_bwd": (_I, [_P, _I, _P, _P, _P, _P, _F, _P, _P, _P, _P, _P, _P, _P]),
    "pgh_newton_ij_bwd": (_I, [_P, _I, _P, _P, _P, _P, _I] + [_P] * 14),
    "pgh_batch_table_bwd": (_I, [_P, _P] + [_P] * 18),
    "pgh_batch_table_moments": (_I, [_P, _P] + [_P] * 11),
    "pgh_batch_table_bwd_moments": (_I, [_P, _P] + [_P] * 19),
    "pgh_variant_count": (_I, [_I]),
    "pgh_variant_name": (ctypes.c_char_p, [_I, _I]),
    "pgh_set_variant": (_I, [_P, _I, _I]),
    "pgh_get_variant": (_I, [_P, _I]),
    "pgh_autotune": (_I, [_P, _I, _I, _P, _P, _P, _I, ctypes.POINTER(_F)]),
    "pgh_autotune_plan": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P, _I, ctypes.POINTER(_F)]),
    "pgh_correct_self_potential": (_I, [_P, _I, _P, _P, _P]),
    "pgh_table_grad_chain": (_I, [_P, _I, _I, _P, _P]),
    "pgh_tree_create": (_I, [_P, ctypes.POINTER(_P)]),
    "pgh_tree_free": (_I, [_P, _P]),
    "pgh_tree_build": (_I, [_P, _P, _I, _P, _P, _P, _P, _I, _I, _I]),
    "pgh_tree_walk": (_I, [_P, _P, _F, _I]),
    "pgh_tree_newton": (_I, [_P, _P, _P, _P, _P, _P]),
    "pgh_tree_stats_get": (_I, [_P, _P]),
    "pgh_tree_plan": (_P, [_P]),
    "pgh_tree_get": (_I, [_P, _P, _I, _P, ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]),
    # GRAPE-5-compatible host interface (include/grape5.h)
    "g5_open": (None, []),
    "g5_close": (None, []),
    "g5_set_eps_to_all": (None, [ctypes.c_double]),
    "g5_set_n": (None, [_I]),
    "g5_set_xmj": (None, [_I, _I, _P, _P]),
    "g5_calculate_force_on_x": (None, [_P, _P, _P, _I]),
    "g5_set_force_table": (_I, [_I, _I, ctypes.c_double, _P]),
    "g5_use_newton": (None, []),
    "g5_last_error": (ctypes.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1203_4037_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


# --------------------------------------------------------------------------
# argument marshalling
# --------------------------------------------------------------------------

def _ptr(t, n=None, what="array", device=None):
    """Device pointer of a float32 contiguous GPU tensor with at least n elements."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{what} must be float32, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{what} must be on the GPU")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what} is on device {t.device.index}, the context on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{what} has {t.numel()} elements, {n} needed")
    return t.data_ptr()


def _check(ctx, st):
    if st != PGH_OK:
        raise PGHError(st, lib.pgh_last_error(ctx).decode())


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


# --------------------------------------------------------------------------
# C-ABI functions (same names and argument order as include/pgh.h)
# --------------------------------------------------------------------------

def pgh_open(device=0):
    h = ctypes.c_void_p()
    _check(None, lib.pgh_open(ctypes.byref(h), device, _stream(device)))
    return h.value


def pgh_close(ctx):
    _check(ctx, lib.pgh_close(ctx))


def pgh_last_error(ctx):
    return lib.pgh_last_error(ctx).decode()


def pgh_version():
    return lib.pgh_version()


def pgh_set_stream(ctx, stream):
    _check(ctx, lib.pgh_set_stream(ctx, stream))


def pgh_set_eps_to_all(ctx, eps):
    _check(ctx, lib.pgh_set_eps_to_all(ctx, float(eps)))


def pgh_set_n(ctx, nj):
    _check(ctx, lib.pgh_set_n(ctx, int(nj)))


def pgh_set_rsqrt_refine(ctx, on):
    _check(ctx, lib.pgh_set_rsqrt_refine(ctx, int(bool(on))))


def pgh_set_plan_expansion(ctx, on_device):
    _check(ctx, lib.pgh_set_plan_expansion(ctx, int(bool(on_device))))


def pgh_set_plan_waves(ctx, waves):
    _check(ctx, lib.pgh_set_plan_waves(ctx, int(waves)))


def pgh_get_plan_waves(ctx):
    v = lib.pgh_get_plan_waves(ctx)
    if v < 0:
        _check(ctx, v)
    return v


def pgh_set_plan_packing(ctx, on):
    _check(ctx, lib.pgh_set_plan_packing(ctx, int(bool(on))))


def pgh_get_plan_packing(ctx):
    v = lib.pgh_get_plan_packing(ctx)
    if v < 0:
        _check(ctx, v)
    return v


def pgh_set_xmj(ctx, adr, nj, x, y, z, m):
    _check(ctx, lib.pgh_set_xmj(ctx, adr, nj, _ptr(x, nj, "x"), _ptr(y, nj, "y"),
                                _ptr(z, nj, "z"), _ptr(m, nj, "m")))


def pgh_calc_newton(ctx, ni, xi, yi, zi, eps2_i, ax, ay, az, phi):
    _check(ctx, lib.pgh_calc_newton(ctx, ni, _ptr(xi, ni, "xi"), _ptr(yi, ni, "yi"),
                                    _ptr(zi, ni, "zi"), _ptr(eps2_i, ni, "eps2_i"),
                                    _ptr(ax, ni, "ax"), _ptr(ay, ni, "ay"), _ptr(az, ni, "az"),
                                    _ptr(phi, ni, "phi")))


def pgh_calc_newton_noalloc(ctx, ni, xi, yi, zi, eps2_i, ax, ay, az, phi):
    _check(ctx, lib.pgh_calc_newton_noalloc(ctx, ni, _ptr(xi, ni, "xi"), _ptr(yi, ni, "yi"),
                                    _ptr(zi, ni, "zi"), _ptr(eps2_i, ni, "eps2_i"),
                                    _ptr(ax, ni, "ax"), _ptr(ay, ni, "ay"), _ptr(az, ni, "az"),
                                    _ptr(phi, ni, "phi")))


def pgh_build_table(ctx, E, F, rcut, f_over_r, user=None, table_out=None):
    """f_over_r: a ctypes function pointer (F_OVER_R or the library's
    pgh_s2pp_f_over_r) or a Python callable h(r) -> float.  table_out: an
    optional host float32 numpy array of 2 * 2^(E+F) entries."""
    cb = _callback(f_over_r)
    out = None if table_out is None else table_out.ctypes.data
    _check(ctx, lib.pgh_build_table(ctx, E, F, float(rcut), ctypes.cast(cb, ctypes.c_void_p),
                                    user, out))


def _callback(f_over_r):
    if isinstance(f_over_r, F_OVER_R):
        return f_over_r
    if callable(f_over_r) and not isinstance(f_over_r, ctypes._CFuncPtr):
        return F_OVER_R(lambda r, _u: float(f_over_r(r)))
    return ctypes.cast(f_over_r, ctypes.c_void_p)


def pgh_table_compute(E, F, rcut, f_over_r, user, table_out):
    """Host-only table computation into a float32 numpy array of 2 * 2^(E+F)."""
    cb = _callback(f_over_r)
    _check(None, lib.pgh_table_compute(E, F, float(rcut), ctypes.cast(cb, ctypes.c_void_p), user,
                                       table_out.ctypes.data))


def pgh_set_table(ctx, E, F, rcut, table):
    _check(ctx, lib.pgh_set_table(ctx, E, F, float(rcut), _ptr(table, 2 << (E + F), "table")))


def pgh_build_pot_table(ctx, pot, user=None, table_out=None):
    """Potential table from a callable p(r) (or an F_OVER_R callback) on the
    bins of the context's force table."""
    cb = _callback(pot)
    out = None if table_out is None else table_out.ctypes.data
    _check(ctx, lib.pgh_build_pot_table(ctx, ctypes.cast(cb, ctypes.c_void_p), user, out))


def pgh_set_pot_table(ctx, table):
    _check(ctx, lib.pgh_set_pot_table(ctx, _ptr(table, None, "table")))


def pgh_calc_table(ctx, ni, xi, yi, zi, ax, ay, az, phi=None):
    _check(ctx, lib.pgh_calc_table(ctx, ni, _ptr(xi, ni, "xi"), _ptr(yi, ni, "yi"),
                                   _ptr(zi, ni, "zi"), _ptr(ax, ni, "ax"), _ptr(ay, ni, "ay"),
                                   _ptr(az, ni, "az"), _ptr(phi, ni, "phi")))


def _items_array(items):
    a = np.ascontiguousarray(np.asarray(items, dtype=np.int32).reshape(-1, 4))
    return a


def pgh_plan_create(ctx, n_items, items, ni_total, nj_total):
    """items: host int32 array [n_items, 4] of (i_off, n_i, j_off, n_j)."""
    a = _items_array(items)
    if a.shape[0] < n_items:
        raise ValueError("fewer items than n_items")
    h = ctypes.c_void_p()
    _check(ctx, lib.pgh_plan_create(ctx, int(n_items), a.ctypes.data if a.size else None,
                                    int(ni_total), int(nj_total), ctypes.byref(h)))
    return h.value


def pgh_plan_free(ctx, plan):
    _check(ctx, lib.pgh_plan_free(ctx, plan))


def pgh_plan_interactions(plan):
    return lib.pgh_plan_interactions(plan)


def pgh_batch_newton(ctx, plan, xi, yi, zi, eps2_i, xj, yj, zj, mj, ax, ay, az, phi):
    _check(ctx, lib.pgh_batch_newton(ctx, plan, _ptr(xi, None, "xi"), _ptr(yi, None, "yi"),
                                     _ptr(zi, None, "zi"), _ptr(eps2_i, None, "eps2_i"),
                                     _ptr(xj, None, "xj"), _ptr(yj, None, "yj"),
                                     _ptr(zj, None, "zj"), _ptr(mj, None, "mj"),
                                     _ptr(ax, None, "ax"), _ptr(ay, None, "ay"),
                                     _ptr(az, None, "az"), _ptr(phi, None, "phi")))


def pgh_batch_table(ctx, plan, xi, yi, zi, xj, yj, zj, mj, ax, ay, az, phi=None):
    _check(ctx, lib.pgh_batch_table(ctx, plan, _ptr(xi, None, "xi"), _ptr(yi, None, "yi"),
                                    _ptr(zi, None, "zi"), _ptr(xj, None, "xj"), _ptr(yj, None, "yj"),
                                    _ptr(zj, None, "zj"), _ptr(mj, None, "mj"), _ptr(ax, None, "ax"),
                                    _ptr(ay, None, "ay"), _ptr(az, None, "az"),
                                    _ptr(phi, None, "phi")))


def pgh_newton_allpairs_bwd(ctx, n, x, y, z, m, eps2, wx, wy, wz, gx, gy, gz, gm):
    _check(ctx, lib.pgh_newton_allpairs_bwd(ctx, n, _ptr(x, n, "x"), _ptr(y, n, "y"),
                                            _ptr(z, n, "z"), _ptr(m, n, "m"), float(eps2),
                                            _ptr(wx, n, "wx"), _ptr(wy, n, "wy"),
                                            _ptr(wz, n, "wz"), _ptr(gx, n, "gx"),
                                            _ptr(gy, n, "gy"), _ptr(gz, n, "gz"),
                                            _ptr(gm, n, "gm")))


def pgh_newton_ij_bwd(ctx, ni, xi, yi, zi, eps2_i, nj, xj, yj, zj, mj, wx, wy, wz,
                      gxi, gyi, gzi, gxj, gyj, gzj, gmj):
    _check(ctx, lib.pgh_newton_ij_bwd(
        ctx, ni, _ptr(xi, ni, "xi"), _ptr(yi, ni, "yi"), _ptr(zi, ni, "zi"),
        _ptr(eps2_i, ni, "eps2_i"), nj, _ptr(xj, nj, "xj"), _ptr(yj, nj, "yj"),
        _ptr(zj, nj, "zj"), _ptr(mj, nj, "mj"), _ptr(wx, ni, "wx"), _ptr(wy, ni, "wy"),
        _ptr(wz, ni, "wz"), _ptr(gxi, ni, "gxi"), _ptr(gyi, ni, "gyi"), _ptr(gzi, ni, "gzi"),
        _ptr(gxj, nj, "gxj"), _ptr(gyj, nj, "gyj"), _ptr(gzj, nj, "gzj"), _ptr(gmj, nj, "gmj")))


def pgh_batch_table_bwd(ctx, plan, xi, yi, zi, xj, yj, zj, mj, wx, wy, wz, gtable, gmj,
                        gxi=None, gyi=None, gzi=None, gxj=None, gyj=None, gzj=None):
    _check(ctx, lib.pgh_batch_table_bwd(
        ctx, plan, _ptr(xi, None, "xi"), _ptr(yi, None, "yi"), _ptr(zi, None, "zi"),
        _ptr(xj, None, "xj"), _ptr(yj, None, "yj"), _ptr(zj, None, "zj"), _ptr(mj, None, "mj"),
        _ptr(wx, None, "wx"), _ptr(wy, None, "wy"), _ptr(wz, None, "wz"),
        _ptr(gtable, None, "gtable"), _ptr(gmj, None, "gmj"),
        _ptr(gxi, None, "gxi"), _ptr(gyi, None, "gyi"), _ptr(gzi, None, "gzi"),
        _ptr(gxj, None, "gxj"), _ptr(gyj, None, "gyj"), _ptr(gzj, None, "gzj")))


def pgh_batch_table_moments(ctx, plan, xi, yi, zi, xj, yj, zj, mj, ax, ay, az, mom):
    _check(ctx, lib.pgh_batch_table_moments(
        ctx, plan, _ptr(xi, None, "xi"), _ptr(yi, None, "yi"), _ptr(zi, None, "zi"),
        _ptr(xj, None, "xj"), _ptr(yj, None, "yj"), _ptr(zj, None, "zj"), _ptr(mj, None, "mj"),
        _ptr(ax, None, "ax"), _ptr(ay, None, "ay"), _ptr(az, None, "az"),
        _ptr(mom, None, "mom")))


def pgh_batch_table_bwd_moments(ctx, plan, xi, yi, zi, xj, yj, zj, mj, wx, wy, wz, mom, gtable,
                                gmj, gxi=None, gyi=None, gzi=None, gxj=None, gyj=None,
                                gzj=None):
    _check(ctx, lib.pgh_batch_table_bwd_moments(
        ctx, plan, _ptr(xi, None, "xi"), _ptr(yi, None, "yi"), _ptr(zi, None, "zi"),
        _ptr(xj, None, "xj"), _ptr(yj, None, "yj"), _ptr(zj, None, "zj"), _ptr(mj, None, "mj"),
        _ptr(wx, None, "wx"), _ptr(wy, None, "wy"), _ptr(wz, None, "wz"),
        _ptr(mom, None, "mom"), _ptr(gtable, None, "gtable"), _ptr(gmj, None, "gmj"),
        _ptr(gxi, None, "gxi"), _ptr(gyi, None, "gyi"), _ptr(gzi, None, "gzi"),
        _ptr(gxj, None, "gxj"), _ptr(gyj, None, "gyj"), _ptr(gzj, None, "gzj")))


def pgh_correct_self_potential(ctx, n, m, eps2_i, phi):
    _check(ctx, lib.pgh_correct_self_potential(ctx, n, _ptr(m, n, "m"), _ptr(eps2_i, n, "eps2_i"),
                                               _ptr(phi, n, "phi")))


def pgh_table_grad_chain(ctx, E, F, gtable, g0):
    K = 1 << (E + F)
    _check(ctx, lib.pgh_table_grad_chain(ctx, E, F, _ptr(gtable, 2 * K, "gtable"),
                                         _ptr(g0, K, "g0")))


def correct_self_potential(phi, m, eps=None, eps2=None, lib_ctx=None):
    """Adds m_i/eps_i to raw potentials in place (pgh_correct_self_potential):
    the physical potential of i-particles that are also j-particles.  eps is
    a scalar softening (or eps2 a per-particle eps^2 tensor)."""
    c = lib_ctx or default_context(phi.device.index)
    c._sync_stream()
    if eps2 is None:
        c.set_eps_to_all(eps)
    pgh_correct_self_potential(c.h, phi.numel(), m, eps2, phi)
    return phi


def pgh_variant_count(family):
    return lib.pgh_variant_count(family)


def pgh_variant_name(family, v):
    s = lib.pgh_variant_name(family, v)
    return None if s is None else s.decode()


def pgh_set_variant(ctx, family, v):
    _check(ctx, lib.pgh_set_variant(ctx, family, v))


def pgh_get_variant(ctx, family):
    return lib.pgh_get_variant(ctx, family)


def pgh_autotune(ctx, family, ni, xi, yi, zi, reps=3):
    """Returns (best variant, ms per call); the context keeps the choice."""
    ms = ctypes.c_float()
    v = lib.pgh_autotune(ctx, family, ni, _ptr(xi, ni, "xi"), _ptr(yi, ni, "yi"),
                         _ptr(zi, ni, "zi"), int(reps), ctypes.byref(ms))
    if v < 0:
        _check(ctx, v)
    return v, ms.value


def pgh_autotune_plan(ctx, family, plan, xi, yi, zi, xj, yj, zj, mj, reps=3):
    """Returns (best variant, ms per call) of a batched family on a plan."""
    ms = ctypes.c_float()
    v = lib.pgh_autotune_plan(ctx, family, plan, _ptr(xi, None, "xi"), _ptr(yi, None, "yi"),
                              _ptr(zi, None, "zi"), _ptr(xj, None, "xj"), _ptr(yj, None, "yj"),
                              _ptr(zj, None, "zj"), _ptr(mj, None, "mj"), int(reps),
                              ctypes.byref(ms))
    if v < 0:
        _check(ctx, v)
    return v, ms.value


# --------------------------------------------------------------------------
# Barnes-Hut tree (pgh_tree_*): lists of the tree code built on the device
# --------------------------------------------------------------------------

def pgh_tree_create(ctx):
    h = ctypes.c_void_p()
    _check(ctx, lib.pgh_tree_create(ctx, ctypes.byref(h)))
    return h.value


def pgh_tree_free(ctx, tree):
    _check(ctx, lib.pgh_tree_free(ctx, tree))


def pgh_tree_build(ctx, tree, n, x, y, z, m, n_leaf=8, n_crit=64, quad=0):
    _check(ctx, lib.pgh_tree_build(ctx, tree, int(n), _ptr(x, n, "x"), _ptr(y, n, "y"),
                                   _ptr(z, n, "z"), _ptr(m, n, "m"), int(n_leaf), int(n_crit),
                                   int(quad)))


def pgh_tree_walk(ctx, tree, theta, record_src=0):
    _check(ctx, lib.pgh_tree_walk(ctx, tree, float(theta), int(record_src)))


def pgh_tree_newton(ctx, tree, ax, ay, az, phi=None):
    _check(ctx, lib.pgh_tree_newton(ctx, tree, _ptr(ax, None, "ax"), _ptr(ay, None, "ay"),
                                    _ptr(az, None, "az"), _ptr(phi, None, "phi")))


def pgh_tree_stats_get(tree):
    st = PghTreeStats()
    rc = lib.pgh_tree_stats_get(tree, ctypes.byref(st))
    if rc != PGH_OK:
        raise PGHError(rc, "pgh_tree_stats_get failed")
    d = {k: getattr(st, k) for k, _ in PghTreeStats._fields_}
    d["frame"] = np.array(list(st.frame), dtype=np.float32)
    return d


def pgh_tree_plan(tree):
    return lib.pgh_tree_plan(tree)


def pgh_tree_get(ctx, tree, field):
    """Host numpy copy of a tree field (a name of PGH_TREE_FIELDS)."""
    code, dtype, tail = PGH_TREE_FIELDS[field]
    cnt = ctypes.c_longlong()
    _check(ctx, lib.pgh_tree_get(ctx, tree, code, None, 0, ctypes.byref(cnt)))
    out = np.empty((cnt.value,) + tail, dtype=dtype)
    if cnt.value:
        _check(ctx, lib.pgh_tree_get(ctx, tree, code, out.ctypes.data, cnt.value,
                                     ctypes.byref(cnt)))
    return out


class Tree:
    """A device Barnes-Hut tree of one context (pgh_tree_*)."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.h = pgh_tree_create(ctx.h)
        self.n = 0

    def free(self):
        if self.h and self.ctx.h:
            pgh_tree_free(self.ctx.h, self.h)
        self.h = None

    def build(self, x, y, z, m, n_leaf=8, n_crit=64, quad=False):
        self.ctx._sync_stream()
        self.n = x.numel()
        pgh_tree_build(self.ctx.h, self.h, self.n, x, y, z, m, n_leaf, n_crit, int(bool(quad)))
        return self

    def walk(self, theta=0.75, record_src=False):
        self.ctx._sync_stream()
        pgh_tree_walk(self.ctx.h, self.h, theta, int(bool(record_src)))
        return self

    def newton(self, out=None, with_phi=True):
        """Tree force (and raw potential) on every particle, input order."""
        c = self.ctx
        c._sync_stream()
        if out is None:
            out = [c._empty(self.n) for _ in range(4 if with_phi else 3)]
        for o in out[:4 if with_phi else 3]:
            _ptr(o, self.n, "output")
        pgh_tree_newton(c.h, self.h, out[0], out[1], out[2], out[3] if with_phi else None)
        return out

    def stats(self):
        return pgh_tree_stats_get(self.h)

    def get(self, field):
        self.ctx._sync_stream()
        return pgh_tree_get(self.ctx.h, self.h, field)


# --------------------------------------------------------------------------
# GRAPE-5-compatible host interface (host numpy arrays in double precision)
# --------------------------------------------------------------------------

G5_F_OVER_R = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_double)


def _host_f64(a, shape_tail, what):
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError(f"{what} must be a C-contiguous float64 numpy array")
    if a.shape[1:] != shape_tail:
        raise ValueError(f"{what} has shape {a.shape}")
    return a.ctypes.data


def _g5_check():
    e = lib.g5_last_error()
    if e:
        raise PGHError(PGH_EHIP, e.decode())


def g5_open():
    lib.g5_open()
    _g5_check()


def g5_close():
    lib.g5_close()


def g5_set_eps_to_all(eps):
    lib.g5_set_eps_to_all(float(eps))
    _g5_check()


def g5_set_n(nj):
    lib.g5_set_n(int(nj))
    _g5_check()


def g5_set_xmj(adr, nj, xj, mj):
    """xj: float64 (n, 3), mj: float64 (n,), host arrays."""
    if xj.shape[0] < nj or mj.shape[0] < nj:
        raise ValueError("arrays shorter than nj")
    lib.g5_set_xmj(int(adr), int(nj), _host_f64(xj, (3,), "xj"), _host_f64(mj, (), "mj"))
    _g5_check()


def g5_calculate_force_on_x(xi, ai, pi, ni):
    """xi, ai: float64 (n, 3); pi: float64 (n,) or None; host arrays."""
    if xi.shape[0] < ni or ai.shape[0] < ni or (pi is not None and pi.shape[0] < ni):
        raise ValueError("arrays shorter than ni")
    lib.g5_calculate_force_on_x(_host_f64(xi, (3,), "xi"), _host_f64(ai, (3,), "ai"),
                                None if pi is None else _host_f64(pi, (), "pi"), int(ni))
    _g5_check()


def g5_set_force_table(E, F, rcut, f_over_r):
    """f_over_r: a G5_F_OVER_R (keep a reference while the table is built)."""
    st = lib.g5_set_force_table(int(E), int(F), float(rcut), ctypes.cast(f_over_r, ctypes.c_void_p))
    if st != PGH_OK:
        raise PGHError(st, (lib.g5_last_error() or b"").decode())


def g5_use_newton():
    lib.g5_use_newton()


def s2pp_callback():
    """The library's built-in h(r) of the S2 particle-particle force shape
    (Eqs. s2pp and s2); pass user = ctypes pointer to double[2] {eps, rcut}."""
    return ctypes.cast(lib.pgh_s2pp_f_over_r, ctypes.c_void_p)


# --------------------------------------------------------------------------
# Object wrapper
# --------------------------------------------------------------------------

class Context:
    """One library context on one GPU; calls run on torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device).index
        self.h = pgh_open(self.device)
        self.nj = 0
        self.table = None
        self.refine = 0
        self.plan_waves = 0
        self.plan_packing = False

    def close(self):
        if self.h:
            pgh_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        pgh_set_stream(self.h, _stream(self.device))

    def _empty(self, n):
        return torch.empty(n, dtype=torch.float32, device=torch.device("cuda", self.device))

    def set_eps_to_all(self, eps):
        pgh_set_eps_to_all(self.h, eps)

    def set_rsqrt_refine(self, on):
        pgh_set_rsqrt_refine(self.h, on)
        self.refine = int(bool(on))

    def set_plan_expansion(self, on_device):
        """Plans' task lists written on the device (True, default) or the host."""
        pgh_set_plan_expansion(self.h, on_device)

    def set_j(self, x, y, z, m, adr=0):
        """Copies j-particles into the j-memory at adr and sets n to adr + len."""
        self._sync_stream()
        n = x.numel()
        pgh_set_xmj(self.h, adr, n, x, y, z, m)
        pgh_set_n(self.h, adr + n)
        self.nj = adr + n

    def newton(self, x, y, z, eps2=None, with_phi=True):
        """Accelerations (and raw potentials) of the i-particles x, y, z."""
        self._sync_stream()
        n = x.numel()
        ax, ay, az = self._empty(n), self._empty(n), self._empty(n)
        phi = self._empty(n) if with_phi else None
        pgh_calc_newton(self.h, n, x, y, z, eps2, ax, ay, az, phi)
        return ax, ay, az, phi

    def build_table(self, E, F, rcut, f_over_r=None, eps=None):
        """Builds the table from a Python callable h(r) = f(r)/r, or from the
        built-in S2 particle-particle shape when f_over_r is None (needs eps)."""
        out = np.zeros(2 << (E + F), dtype=np.float32)
        if f_over_r is None:
            params = (ctypes.c_double * 2)(float(eps), float(rcut))
            pgh_build_table(self.h, E, F, rcut, s2pp_callback(), ctypes.cast(params, ctypes.c_void_p), out)
        else:
            pgh_build_table(self.h, E, F, rcut, f_over_r, None, out)
        self.table = (E, F, float(rcut))
        return out

    def set_table(self, E, F, rcut, table):
        self._sync_stream()
        pgh_set_table(self.h, E, F, rcut, table)
        self.table = (E, F, float(rcut))

    def build_pot_table(self, pot):
        """Potential table of a callable p(r) on the force table's bins; returns
        the host copy (float32, interleaved P0, P1)."""
        E, F, _ = self.table
        out = np.zeros(2 << (E + F), dtype=np.float32)
        pgh_build_pot_table(self.h, pot, None, out)
        return out

    def table_force(self, x, y, z, with_phi=False):
        self._sync_stream()
        n = x.numel()
        ax, ay, az = self._empty(n), self._empty(n), self._empty(n)
        phi = self._empty(n) if with_phi else None
        pgh_calc_table(self.h, n, x, y, z, ax, ay, az, phi)
        return (ax, ay, az, phi) if with_phi else (ax, ay, az)

    def set_variant(self, family, v):
        pgh_set_variant(self.h, family, v)

    def autotune(self, family, x, y, z, reps=3, cache=None):
        """Chooses the fastest variant of an all-pairs family for the i-particles
        x, y, z against the current j-memory (and table).  With a cache path
        (JSON) a previous choice for the same device, family and shape is
        reused without timing.  Returns the variant index."""
        self._sync_stream()
        key = ("allpairs", family, x.numel(), self.nj,
               self.table if family == PGH_FAMILY_TABLE_ALLPAIRS else "", self.refine)
        return _cached_tune(self, family, key, cache,
                            lambda: pgh_autotune(self.h, family, x.numel(), x, y, z, reps)[0])

    # interaction lists ------------------------------------------------------

    def set_plan_waves(self, waves):
        """The wave count later plans are cut for (0: the device's)."""
        pgh_set_plan_waves(self.h, waves)
        self.plan_waves = int(waves)

    def set_plan_packing(self, on):
        """Whether later plans pack the rows an item leaves empty with the
        next item's first i-particles (pgh_set_plan_packing)."""
        pgh_set_plan_packing(self.h, on)
        self.plan_packing = bool(on)

    def plan(self, items, ni_total, nj_total):
        """A Plan for host items [n, 4] = (i_off, n_i, j_off, n_j)."""
        return Plan(self, items, ni_total, nj_total)

    def plan_tuned(self, items, ni_total, nj_total, family, xi, yi, zi, xj, yj, zj, mj,
                   scales=(0.5, 1.0, 2.0), packings=(False, True), reps=3, cache=None):
        """A Plan whose schedule and kernel variant are chosen by timing: for
        each wave target (the device's resident waves times each scale) and
        each packing setting a plan is made and every variant of the batched
        family is timed on it (pgh_autotune_plan); the fastest is kept and its
        variant selected (the plan's `packed` says whether it is packed).
        With a cache path (JSON) a previous choice for lists of the same
        shape class on the same device is made without timing.  The context's
        own wave target and packing setting are left as they were.
        Returns (plan, variant index, scale)."""
        import json
        a = _items_array(items)
        for t in (xi, yi, zi):
            if t.numel() < ni_total:
                raise ValueError("an i-array is shorter than ni_total")
        for t in (xj, yj, zj, mj):
            if t.numel() < nj_total:
                raise ValueError("a j-array is shorter than nj_total")
        self._sync_stream()
        user_waves, user_pack = self.plan_waves, self.plan_packing
        pgh_set_plan_waves(self.h, 0)
        base = pgh_get_plan_waves(self.h)
        packings = tuple(bool(k) for k in packings)
        names = [pgh_variant_name(family, v) for v in range(pgh_variant_count(family))]
        key = None
        if cache:
            props = torch.cuda.get_device_properties(self.device)
            key = "|".join(str(x) for x in (props.name, "plan_tuned", family) + _shape_class(a)
                           + (self.table if family == PGH_FAMILY_TABLE_BATCH else "",
                              self.refine, tuple(scales), packings))
            try:
                with open(cache) as f:
                    stored = json.load(f)
            except (OSError, ValueError):
                stored = {}
            hit = stored.get(key)
            if (hit and hit.get("variant") in names and hit.get("scale") in scales
                    and hit.get("packing", False) in packings):
                pgh_set_plan_waves(self.h, max(1, int(round(base * hit["scale"]))))
                pgh_set_plan_packing(self.h, hit.get("packing", False))
                try:
                    p = Plan(self, a, ni_total, nj_total)
                finally:
                    pgh_set_plan_waves(self.h, user_waves)
                    pgh_set_plan_packing(self.h, user_pack)
                v = names.index(hit["variant"])
                pgh_set_variant(self.h, family, v)
                return p, v, hit["scale"]
        best = None
        try:
            for sc, pk in [(sc, pk) for sc in scales for pk in packings]:
                pgh_set_plan_waves(self.h, max(1, int(round(base * sc))))
                pgh_set_plan_packing(self.h, pk)
                p = Plan(self, a, ni_total, nj_total)
                try:
                    v, ms = pgh_autotune_plan(self.h, family, p.h, xi, yi, zi, xj, yj, zj, mj,
                                              reps)
                except Exception:
                    p.free()
                    raise
                if best is None or ms < best[2]:
                    if best is not None:
                        best[0].free()
                    best = (p, v, ms, sc)
                else:
                    p.free()
        except Exception:
            if best is not None:
                best[0].free()
            raise
        finally:
            pgh_set_plan_waves(self.h, user_waves)
            pgh_set_plan_packing(self.h, user_pack)
        p, v, _, sc = best
        pgh_set_variant(self.h, family, v)
        if cache:
            stored[key] = {"scale": sc, "variant": names[v], "packing": p.packed}
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(stored, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return p, v, sc

    def tree(self):
        """An empty device Barnes-Hut tree of this context."""
        return Tree(self)


def _cached_tune(ctx, family, key, cache, tune):
    """Runs tune() (which times the variants and selects the fastest), or,
    with a JSON cache path holding a choice for this device and key, selects
    that variant without timing.  Choices are stored by variant name, so a
    library with other variants re-tunes instead of misreading an index."""
    import json
    if not cache:
        return tune()
    props = torch.cuda.get_device_properties(ctx.device)
    k = "|".join(str(x) for x in (props.name,) + tuple(key))
    try:
        with open(cache) as f:
            table = json.load(f)
    except (OSError, ValueError):
        table = {}
    names = [pgh_variant_name(family, v) for v in range(pgh_variant_count(family))]
    if k in table and table[k] in names:
        v = names.index(table[k])
        pgh_set_variant(ctx.h, family, v)
        return v
    v = tune()
    table[k] = names[v]
    tmp = cache + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, cache)
    return v


def _shape_class(a):
    """A plan's shape class: its number of lists and its median group size
    and list length, each rounded to a power of two."""
    def pow2(v):
        return 1 << max(0, int(round(np.log2(max(1.0, float(v))))))
    live = a[a[:, 1] > 0] if a.shape[0] else a
    return (pow2(live.shape[0]),
            pow2(np.median(live[:, 1])) if live.shape[0] else 0,
            pow2(np.median(live[:, 3])) if live.shape[0] else 0)


class Plan:
    """Execution plan of a set of interaction lists (pgh_plan_create)."""

    def __init__(self, ctx, items, ni_total, nj_total):
        a = _items_array(items)
        self.ctx = ctx
        self.ni_total, self.nj_total = int(ni_total), int(nj_total)
        self.h = pgh_plan_create(ctx.h, a.shape[0], a, ni_total, nj_total)
        self.interactions = pgh_plan_interactions(self.h)

        self.shape_class = _shape_class(a)
        self.waves = pgh_get_plan_waves(ctx.h)
        self.packed = bool(pgh_get_plan_packing(ctx.h))

    def free(self):
        if self.h and self.ctx.h:
            pgh_plan_free(self.ctx.h, self.h)
        self.h = None

    def _check_sizes(self, i_arrays, j_arrays):
        for t in i_arrays:
            if t is not None and t.numel() < self.ni_total:
                raise ValueError("an i-array is shorter than the plan's ni_total")
        for t in j_arrays:
            if t is not None and t.numel() < self.nj_total:
                raise ValueError("a j-array is shorter than the plan's nj_total")

    def newton(self, xi, yi, zi, xj, yj, zj, mj, eps2=None, out=None, with_phi=True):
        """Newton force of every list; rows outside every item keep the
        values of `out` (allocated uninitialised when out is None)."""
        c = self.ctx
        c._sync_stream()
        self._check_sizes((xi, yi, zi, eps2), (xj, yj, zj, mj))
        n = self.ni_total
        if out is None:
            out = [c._empty(n) for _ in range(4 if with_phi else 3)]
        phi = out[3] if with_phi else None
        pgh_batch_newton(c.h, self.h, xi, yi, zi, eps2, xj, yj, zj, mj, out[0], out[1], out[2], phi)
        return out

    def table(self, xi, yi, zi, xj, yj, zj, mj, out=None, with_phi=False):
        """Table force (and the potential from the potential table when
        with_phi, out then holding 4 arrays)."""
        c = self.ctx
        c._sync_stream()
        self._check_sizes((xi, yi, zi), (xj, yj, zj, mj))
        if out is None:
            out = [c._empty(self.ni_total) for _ in range(4 if with_phi else 3)]
        phi = out[3] if with_phi else None
        pgh_batch_table(c.h, self.h, xi, yi, zi, xj, yj, zj, mj, out[0], out[1], out[2], phi)
        return out

    def table_moments(self, xi, yi, zi, xj, yj, zj, mj, out=None, mom=None):
        """Table force with the i-side moments of its adjoint
        (pgh_batch_table_moments): returns [ax, ay, az] and mom [7 * ni_total]
        (S, Mxx, Mxy, Mxz, Myy, Myz, Mzz, each a row of ni_total)."""
        c = self.ctx
        c._sync_stream()
        self._check_sizes((xi, yi, zi), (xj, yj, zj, mj))
        if out is None:
            out = [c._empty(self.ni_total) for _ in range(3)]
        if mom is None:
            mom = c._empty(7 * self.ni_total)
        pgh_batch_table_moments(c.h, self.h, xi, yi, zi, xj, yj, zj, mj, out[0], out[1], out[2],
                                mom)
        return out, mom

    def autotune(self, family, xi, yi, zi, xj, yj, zj, mj, reps=3, cache=None):
        """Selects the fastest variant (tile shape) of a batched family on this
        plan (PGH_FAMILY_NEWTON_BATCH uses the context's eps_to_all) and
        returns its index.  With a cache path (JSON) a previous choice for a
        plan of the same shape class on the same device is reused without
        timing: the class is the number of lists and the median group size
        and list length, each rounded to a power of two, with the table and
        the rsqrt mode."""
        c = self.ctx
        c._sync_stream()
        self._check_sizes((xi, yi, zi), (xj, yj, zj, mj))
        key = ("plan", family) + self.shape_class + (
            c.table if family == PGH_FAMILY_TABLE_BATCH else "", c.refine)
        return _cached_tune(c, family, key, cache, lambda: pgh_autotune_plan(
            c.h, family, self.h, xi, yi, zi, xj, yj, zj, mj, reps)[0])


# --------------------------------------------------------------------------
# Differentiable forces (the adjoint kernels behind torch.autograd)
# --------------------------------------------------------------------------

_default_contexts = {}


def default_context(device=None) -> Context:
    """One library context per device, created on first use."""
    d = torch.cuda.current_device() if device is None else torch.device("cuda", device).index
    if d not in _default_contexts:
        _default_contexts[d] = Context(d)
    return _default_contexts[d]


def _zeros_if_none(g, like):
    return torch.zeros_like(like) if g is None else g.contiguous()


class NewtonAllPairs(torch.autograd.Function):
    """Accelerations and raw potentials of N particles on each other (i-set =
    j-set), softening eps.  Gradients flow from the accelerations to the
    positions and masses through pgh_newton_allpairs_bwd; the potential is
    returned as a non-differentiable output."""

    @staticmethod
    def forward(fctx, x, y, z, m, eps, lib_ctx=None):
        c = lib_ctx or default_context(x.device.index)
        c.set_eps_to_all(eps)
        c.set_j(x, y, z, m)
        ax, ay, az, phi = c.newton(x, y, z)
        fctx.save_for_backward(x, y, z, m)
        fctx.eps2 = float(torch.tensor(eps, dtype=torch.float32) ** 2)
        fctx.lib_ctx = c
        fctx.mark_non_differentiable(phi)
        return ax, ay, az, phi

    @staticmethod
    def backward(fctx, gax, gay, gaz, gphi):
        x, y, z, m = fctx.saved_tensors
        c = fctx.lib_ctx
        c._sync_stream()
        wx, wy, wz = (_zeros_if_none(g, x) for g in (gax, gay, gaz))
        n = x.numel()
        gx, gy, gz, gm = (c._empty(n) for _ in range(4))
        pgh_newton_allpairs_bwd(c.h, n, x, y, z, m, fctx.eps2, wx, wy, wz, gx, gy, gz, gm)
        return gx, gy, gz, gm, None, None


class NewtonIJ(torch.autograd.Function):
    """Accelerations of the i-particles from separate j-particles, with
    gradients to both position sets and the j masses (pgh_newton_ij_bwd)."""

    @staticmethod
    def forward(fctx, xi, yi, zi, xj, yj, zj, mj, eps, lib_ctx=None):
        c = lib_ctx or default_context(xi.device.index)
        c.set_eps_to_all(eps)
        c.set_j(xj, yj, zj, mj)
        ax, ay, az, _ = c.newton(xi, yi, zi, with_phi=False)
        fctx.save_for_backward(xi, yi, zi, xj, yj, zj, mj)
        fctx.lib_ctx = c
        fctx.eps = eps
        return ax, ay, az

    @staticmethod
    def backward(fctx, gax, gay, gaz):
        xi, yi, zi, xj, yj, zj, mj = fctx.saved_tensors
        c = fctx.lib_ctx
        c.set_eps_to_all(fctx.eps)
        c._sync_stream()
        wx, wy, wz = (_zeros_if_none(g, xi) for g in (gax, gay, gaz))
        ni, nj = xi.numel(), xj.numel()
        gi = [c._empty(ni) for _ in range(3)]
        gj = [c._empty(nj) for _ in range(4)]
        pgh_newton_ij_bwd(c.h, ni, xi, yi, zi, None, nj, xj, yj, zj, mj, wx, wy, wz, *gi, *gj)
        return (*gi, *gj, None, None)


class TableForceBatch(torch.autograd.Function):
    """Table force of every list of a Plan, differentiable with respect to the
    table entries (G0 and G1 as independent leaves, interleaved like the
    table), the j masses and the i- and j-positions through
    pgh_batch_table_bwd (the interpolant is linear in s inside a bin, so its
    s-derivative is the bin's G1; zero beyond the cutoff).  When the
    i-positions need a gradient the forward also keeps the i-side moments
    (pgh_batch_table_moments) and the backward forms that gradient from them
    (pgh_batch_table_bwd_moments) instead of a second pass over the pairs."""

    @staticmethod
    def forward(fctx, plan, E, F, rcut, table, xi, yi, zi, xj, yj, zj, mj):
        c = plan.ctx
        c.set_table(E, F, rcut, table)
        if any(fctx.needs_input_grad[5:8]):
            out, mom = plan.table_moments(xi, yi, zi, xj, yj, zj, mj)
        else:
            out, mom = plan.table(xi, yi, zi, xj, yj, zj, mj), None
        fctx.save_for_backward(table, xi, yi, zi, xj, yj, zj, mj)
        fctx.mom = mom
        fctx.plan = plan
        fctx.shape = (E, F, float(rcut))
        return tuple(out)

    @staticmethod
    def backward(fctx, gax, gay, gaz):
        table, xi, yi, zi, xj, yj, zj, mj = fctx.saved_tensors
        plan = fctx.plan
        c = plan.ctx
        E, F, rcut = fctx.shape
        c.set_table(E, F, rcut, table)
        wx, wy, wz = (_zeros_if_none(g, xi) for g in (gax, gay, gaz))
        need = fctx.needs_input_grad
        gt = c._empty(table.numel()) if need[4] else None
        gm = c._empty(plan.nj_total) if need[11] else None
        gi = [c._empty(plan.ni_total) for _ in range(3)] if any(need[5:8]) else [None] * 3
        gj = [c._empty(plan.nj_total) for _ in range(3)] if any(need[8:11]) else [None] * 3
        if fctx.mom is not None:
            pgh_batch_table_bwd_moments(c.h, plan.h, xi, yi, zi, xj, yj, zj, mj, wx, wy, wz,
                                        fctx.mom, gt, gm, *gi, *gj)
        else:
            pgh_batch_table_bwd(c.h, plan.h, xi, yi, zi, xj, yj, zj, mj, wx, wy, wz, gt, gm, *gi,
                                *gj)
        fctx.mom = None
        return (None, None, None, None, gt, *gi, *gj, gm)


def newton_allpairs(x, y, z, m, eps, lib_ctx=None):
    return NewtonAllPairs.apply(x, y, z, m, eps, lib_ctx)


def newton_ij(xi, yi, zi, xj, yj, zj, mj, eps, lib_ctx=None):
    return NewtonIJ.apply(xi, yi, zi, xj, yj, zj, mj, eps, lib_ctx)


def table_force_batch(plan, E, F, rcut, table, xi, yi, zi, xj, yj, zj, mj):
    return TableForceBatch.apply(plan, E, F, rcut, table, xi, yi, zi, xj, yj, zj, mj)
