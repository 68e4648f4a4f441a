"""Shared helpers of the GPU parity tests (comparison metrics, tensor moves)."""
import numpy as np


def rel_vec_err(got, ref):
    """Per-particle |a_got - a_ref| / |a_ref| for (3, n) arrays."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.sqrt(np.sum((got - ref) ** 2, axis=0))
    den = np.sqrt(np.sum(ref ** 2, axis=0))
    return num / np.maximum(den, 1e-300)


def norm_vec_err(got, ref, scale):
    """Per-particle |a_got - a_ref| / scale (scale: sum of |terms|, for sums
    with cancellation)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.sqrt(np.sum((got - ref) ** 2, axis=0))
    return num / np.maximum(np.asarray(scale, dtype=np.float64), 1e-300)


def rms(e):
    e = np.asarray(e, dtype=np.float64)
    return float(np.sqrt(np.mean(e ** 2))) if e.size else 0.0


def to_dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrays]


def to_host(*tensors):
    return [t.detach().cpu().numpy().astype(np.float64) for t in tensors]


def oracle_table(pgh, family, variant, table, E, F):
    """The table the oracle interpolates to check a table-kernel variant: the
    (H, G1) form (oracle.table_ht) for the "htab" variants, whose LDS copy
    holds H_k = fl32(G0_k - G1_k s_k); the table itself for the others."""
    import oracle
    name = pgh.pgh_variant_name(family, variant)
    return oracle.table_ht(table, E, F) if "htab" in name else table
