"""Pins of the King-model generator (the second particle distribution of the
paper's tree-code experiment, Sec. 5, W0 = 9): its closed-form density
against a direct integration of the King distribution function, its
concentrations c = log10(r_t / r_0) against the values of King's (1966) model
sequence, and the sampled radii against the enclosed-mass profile."""
import numpy as np
import pytest
from scipy.integrate import quad

import synth


@pytest.mark.parametrize("W", [0.05, 0.3, 2.0, 9.0])
def test_density_is_the_integrated_distribution_function(W):
    # sigma = 1: rho = 4 pi (2 pi)^{-3/2} int_0^{sqrt(2W)} (e^{W - v^2/2} - 1) v^2 dv
    num = 4 * np.pi * (2 * np.pi) ** -1.5 * quad(
        lambda v: (np.exp(W - v * v / 2) - 1) * v * v, 0, np.sqrt(2 * W), epsabs=0, epsrel=1e-13)[0]
    assert np.isclose(synth.king_density(W), num, rtol=1e-10)
    assert synth.king_density(-1.0) == 0.0


@pytest.mark.parametrize("W0,c", [(3.0, 0.67), (7.0, 1.53), (9.0, 2.12), (12.0, 2.74)])
def test_concentrations_of_the_king_sequence(W0, c):
    _, frac, rt = synth.king_profile(W0)
    assert abs(np.log10(rt) - c) < 0.01
    assert frac[-1] == 1.0 and np.all(np.diff(frac) >= 0)


def test_sampled_radii_follow_the_profile():
    n = 200000
    x, y, z = synth.king(n, 7, 9.0)
    r = np.sqrt(x.astype(np.float64) ** 2 + y.astype(np.float64) ** 2 + z.astype(np.float64) ** 2)
    grid, frac, rt = synth.king_profile(9.0)
    assert r.max() <= rt * (1 + 1e-6)
    for q in (1.0, 10.0, 30.0):
        p = np.interp(q, grid, frac)
        got = np.mean(r < q)
        assert abs(got - p) < 5 * np.sqrt(p * (1 - p) / n) + 1e-4, (q, got, p)
    # isotropy: the mean position is zero to the sampling error
    for v in (x, y, z):
        assert abs(np.mean(np.sign(v))) < 5 / np.sqrt(n)
