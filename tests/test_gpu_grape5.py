"""The GRAPE-5-compatible host interface (include/grape5.h, Sec. 3.6): the
paper's sample call sequence with host double arrays, against the FP64
oracle on the same (FP32-representable) inputs."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from _helpers import rel_vec_err, rms, norm_vec_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pgh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1203_4037_amd as p
    p.g5_open()
    yield p
    p.g5_close()


def test_sample_code_sequence_newton(pgh):
    """g5_open, g5_set_eps_to_all, g5_set_n, g5_set_xmj (in two pieces at
    adr 0 and n/2), g5_calculate_force_on_x: accelerations and raw
    potentials of a Plummer sphere of 4096 on itself."""
    n = 4096
    x32 = np.stack(synth.plummer(n, 55), axis=1)
    m32 = synth.equal_masses(n)
    x = x32.astype(np.float64)
    m = m32.astype(np.float64)
    eps = 0.015625  # exact in FP32
    pgh.g5_use_newton()
    pgh.g5_set_eps_to_all(eps)
    pgh.g5_set_n(n)
    h = n // 2
    pgh.g5_set_xmj(0, h, np.ascontiguousarray(x[:h]), np.ascontiguousarray(m[:h]))
    pgh.g5_set_xmj(h, n - h, np.ascontiguousarray(x[h:]), np.ascontiguousarray(m[h:]))
    a = np.zeros((n, 3))
    p = np.zeros(n)
    pgh.g5_calculate_force_on_x(x, a, p, n)
    e2 = np.full(n, np.float32(eps) ** 2, np.float32)
    ref = oracle.newton(x32[:, 0], x32[:, 1], x32[:, 2], e2, x32[:, 0], x32[:, 1], x32[:, 2], m32)
    ea = rel_vec_err(a.T, np.stack(ref[:3]))
    ep = np.abs(p - ref[3]) / np.abs(ref[3])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (rms(ea), ea.max())
    assert rms(ep) <= 1e-5 and ep.max() <= 1e-3, (rms(ep), ep.max())
    # a subset of i-particles, and no potential array: the same sums (the
    # j-range is split into shares by the size of the i-set, so the order of
    # the additions, and the last bits, may differ from the call above)
    a2 = np.zeros((100, 3))
    pgh.g5_calculate_force_on_x(np.ascontiguousarray(x[:100]), a2, None, 100)
    ea2 = rel_vec_err(a2.T, np.stack(ref[:3])[:, :100])
    assert rms(ea2) <= 1e-5 and ea2.max() <= 1e-3, (rms(ea2), ea2.max())
    pgh.g5_calculate_force_on_x(x, a2, None, 0)  # ni = 0 is a no-op


def test_force_table_by_function_pointer(pgh):
    """g5_set_force_table with a host h(r) = f(r)/r (a softened Newtonian
    shape with a smooth taper to zero at rcut), then the table force of a
    uniform box on itself against the oracle's evaluation of the same table
    (the library's host builder, pinned against the oracle's elsewhere)."""
    n = 2048
    rcut, epsl = 0.2, 0.01
    x32 = np.stack(synth.uniform_box(n, 56, box=0.5), axis=1)
    m32 = np.linspace(0.5, 1.5, n).astype(np.float32) / n

    def h(r):
        t = 1.0 - (r / rcut) ** 2 if r < rcut else 0.0
        return (r * r + epsl * epsl) ** -1.5 * t * t

    cb = pgh.G5_F_OVER_R(h)
    pgh.g5_set_force_table(4, 6, rcut, cb)
    x = x32.astype(np.float64)
    pgh.g5_set_n(n)
    pgh.g5_set_xmj(0, n, x, m32.astype(np.float64))
    a = np.zeros((n, 3))
    p = np.full(n, 9.0)
    pgh.g5_calculate_force_on_x(x, a, p, n)
    assert np.all(p == 0.0)
    table = np.zeros(2 << 10, np.float32)
    ucb = pgh.F_OVER_R(lambda r, user: h(r))
    pgh.pgh_table_compute(4, 6, rcut, ucb, None, table)
    items = np.array([[0, n, 0, n]], np.int32)
    ref = oracle.lut_items(items, x32[:, 0], x32[:, 1], x32[:, 2], x32[:, 0], x32[:, 1], x32[:, 2],
                           m32, 4, 6, float(np.float32(rcut)), table)
    has = ref[3] > 0
    e = norm_vec_err(a.T[:, has], np.stack(ref[:3])[:, has], ref[3][has])
    assert rms(e) <= 1e-5 and e.max() <= 1e-3, (rms(e), e.max())
    pgh.g5_use_newton()
