"""Pins of the oracle's detector response (long-wavelength L-shaped detector, the
paper's three-detector network) against geometric identities."""
import math

import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(7)


def _rand_geom():
    return np.array([math.asin(RNG.uniform(-1, 1)), RNG.uniform(0, 2 * math.pi), RNG.uniform(0, 2 * math.pi)])


@pytest.mark.parametrize("i", range(5))
def test_overhead_source_with_axes_on_the_arms(i):
    geom = _rand_geom()
    lat, lon, az = geom
    ra, dec = lon, lat  # overhead with gmst = 0
    psi = math.pi / 2 - az  # polarisation x-axis along the x arm
    fp, fc, dt = oracle.antenna(geom, ra, dec, psi)
    assert abs(abs(fp) - 1) < 1e-13 and abs(fc) < 1e-13
    fp2, fc2, _ = oracle.antenna(geom, ra, dec, psi + math.pi / 4)
    assert abs(fp2) < 1e-13 and abs(abs(fc2) - 1) < 1e-13
    assert dt == pytest.approx(-oracle.r_earth() / oracle.c_si(), rel=1e-14)


def test_response_bounds_and_polarisation_symmetry():
    for _ in range(200):
        geom = _rand_geom()
        ra, dec, psi = RNG.uniform(0, 2 * math.pi), math.asin(RNG.uniform(-1, 1)), RNG.uniform(0, math.pi)
        fp, fc, dt = oracle.antenna(geom, ra, dec, psi)
        assert fp * fp + fc * fc <= 1 + 1e-12
        assert abs(dt) <= oracle.r_earth() / oracle.c_si() * (1 + 1e-14)
        fp2, fc2, dt2 = oracle.antenna(geom, ra, dec, psi + math.pi / 2)
        assert fp2 == pytest.approx(-fp, abs=1e-13) and fc2 == pytest.approx(-fc, abs=1e-13)
        fp3, fc3, _ = oracle.antenna(geom, ra, dec, psi + math.pi)
        assert fp3 == pytest.approx(fp, abs=1e-13) and fc3 == pytest.approx(fc, abs=1e-13)
        assert dt2 == dt


def test_rotation_about_the_axis_and_gmst():
    for _ in range(50):
        geom = _rand_geom()
        ra, dec, psi = RNG.uniform(0, 2 * math.pi), math.asin(RNG.uniform(-1, 1)), RNG.uniform(0, math.pi)
        alpha = RNG.uniform(0, 2 * math.pi)
        a = oracle.antenna(geom, ra, dec, psi)
        g2 = geom.copy()
        g2[1] += alpha
        b = oracle.antenna(g2, ra + alpha, dec, psi)
        c = oracle.antenna(geom, ra + alpha, dec, psi, gmst=alpha)
        np.testing.assert_allclose(a, b, atol=1e-12)
        np.testing.assert_allclose(a, c, atol=1e-12)


def test_sky_averaged_response():
    """<F+^2 + Fx^2> over the sky and polarisation = 2/5 for an L-shaped interferometer."""
    geom = _rand_geom()
    n = 20000
    acc = 0.0
    for _ in range(n):
        ra, dec, psi = RNG.uniform(0, 2 * math.pi), math.asin(RNG.uniform(-1, 1)), RNG.uniform(0, math.pi)
        fp, fc, _ = oracle.antenna(geom, ra, dec, psi)
        acc += fp * fp + fc * fc
    assert acc / n == pytest.approx(0.4, abs=0.01)
