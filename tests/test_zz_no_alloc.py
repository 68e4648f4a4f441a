"""The allocation-free Newton entry point (pgh_calc_newton_noalloc) through
the C ABI: two calls in a row (the second with fewer particles) against
pgh_calc_newton on the same context, bit for bit where both split the
j-range the same way (else to the Newton gate), and against the FP64
oracle at the Newton gate
(rms <= 1e-5, max <= 1e-3 relative acceleration and potential error)."""
import numpy as np
import pytest

import oracle
import synth
from _helpers import rel_vec_err, rms, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pgh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1203_4037_amd as p
    return p


def _call(pgh, ctx, fn, ni, di):
    import torch
    out = [torch.full((ni,), 12345.0, device="cuda") for _ in range(4)]
    fn(ctx.h, ni, di[0], di[1], di[2], None, *out)
    return np.stack(to_host(*out))


def _oracle(xi, yi, zi, eps, xj, yj, zj, mj):
    e2 = np.full(xi.size, np.float32(eps) ** 2, np.float32)
    return np.stack(oracle.newton(xi, yi, zi, e2, xj, yj, zj, mj))


def _gate(got, ref, what):
    ea = rel_vec_err(got[:3], ref[:3])
    ep = np.abs(got[3] - ref[3]) / np.abs(ref[3])
    assert rms(ea) <= 1e-5 and ea.max() <= 1e-3, (what, rms(ea), ea.max())
    assert rms(ep) <= 1e-5 and ep.max() <= 1e-3, (what, rms(ep), ep.max())


def test_noalloc_matches_calc_newton(pgh):
    ctx = pgh.Context(0)
    try:
        cases = [
            # (ni, nj, eps, seed): all-pairs of 1024 (j-split into shares of
            # 64 records, partial sums in the scratch array), then a smaller,
            # ragged call that reuses the array
            (1024, 1024, 1.0 / 64, 101),
            (300, 777, 0.02, 7),
        ]
        for ni, nj, eps, seed in cases:
            x, y, z = synth.plummer(max(ni, nj), seed)
            m = synth.equal_masses(nj)
            dj = to_dev(x[:nj], y[:nj], z[:nj], m)
            di = to_dev(x[:ni], y[:ni], z[:ni])
            ctx.set_eps_to_all(eps)
            ctx.set_j(*dj)
            ref_lib = _call(pgh, ctx, pgh.pgh_calc_newton, ni, di)
            got = _call(pgh, ctx, pgh.pgh_calc_newton_noalloc, ni, di)
            # the same split (both caps hold these partial sums): same bits
            assert np.array_equal(got, ref_lib), (ni, nj)
            ref = _oracle(x[:ni], y[:ni], z[:ni], eps, x[:nj], y[:nj], z[:nj], m)
            _gate(got, ref, f"noalloc ni={ni} nj={nj}")
    finally:
        ctx.close()


def test_noalloc_large_split(pgh):
    """Larger i-sets whose j-split is bounded by the array: 40000 i-particles
    (pgh_calc_newton aims for 8 waves per SIMD and splits the j-range in 14
    shares; the allocation-free call splits it in the 6 whose partial sums
    fit in the array, 960000 floats), then a smaller one (20000: 27 and 13
    shares) reusing it.  The two entry points differ only in the order of
    the FP32 sums: equal to the Newton gate, and a sample of rows against the
    oracle."""
    ctx = pgh.Context(0)
    try:
        x, y, z = synth.plummer(40000, 55)
        nj = 30000
        m = synth.equal_masses(nj)
        ctx.set_eps_to_all(0.01)
        ctx.set_j(*to_dev(x[:nj], y[:nj], z[:nj], m))
        for ni in (40000, 20000):
            di = to_dev(x[:ni], y[:ni], z[:ni])
            a = _call(pgh, ctx, pgh.pgh_calc_newton, ni, di)
            b = _call(pgh, ctx, pgh.pgh_calc_newton_noalloc, ni, di)
            _gate(b, a, f"noalloc vs calc_newton ni={ni}")
            rows = np.unique(np.random.default_rng(ni).integers(0, ni, 512))
            ref = _oracle(x[rows], y[rows], z[rows], 0.01, x[:nj], y[:nj], z[:nj], m)
            _gate(b[:, rows], ref, f"noalloc ni={ni}")
    finally:
        ctx.close()
