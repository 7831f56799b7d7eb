"""Pins of the oracle's TaylorF2 phase (the waveform model; the paper's own models are
IMRPhenom, which are not available).

The TaylorF2 coefficients are re-derived here from a different pair of PN quantities,
the binding energy E(v) and the GW flux F(v) (Blanchet, Living Rev. Rel. 17, 2 (2014),
energy and flux of circular orbits, with the leading spin-orbit terms; same
normalisation as Kidder 1995), through the stationary-phase integral

    Psi(v) = 2 v^3 t_c / M - phi_c - pi/4 + (2/M) int_v (v^3 - u^3) E'(u) / F(u) du,

re-expanded in v. A dropped term, a wrong sign or a transposed mass ratio in the oracle's
coefficients fails here.

The 2PN spin-spin pieces of E and F are not taken from a table: they are derived below
from the leading-order physics of a circular orbit with spins along the orbital angular
momentum (Kidder, Phys. Rev. D 52, 821 (1995): the spin-spin interaction energy
(3 (S1.n)(S2.n) - S1.S2)/r^3 and the spin part 3/2 x^<i S^j> of the current quadrupole;
Poisson, Phys. Rev. D 57, 5287 (1998): the quadrupole-monopole interaction of a spinning
body whose quadrupole is that of a Kerr black hole, Q = -chi^2 m^3): Kepler's law and the
energy of the orbit in that potential, and the flux of the mass and current quadrupoles,
(1/5) |d^3 I/dt^3|^2 + (16/45) |d^3 J/dt^3|^2.
"""
import math
from functools import lru_cache

import numpy as np
import pytest

import oracle

sp = pytest.importorskip("sympy")


@lru_cache(maxsize=1)
def _spin_spin_energy_flux():
    """2PN spin-spin coefficients e4, f4 of E = -(eta v^2/2)(1 + ... + e4 v^4) and
    F = (32/5) eta^2 v^10 (1 + ... + f4 v^4), in units M = 1, as sympy expressions in the mass
    fractions x1, x2 and the aligned spins chi1, chi2. lam marks the spin-spin order; only
    its first power is kept (the square is 4PN)."""
    r, t, w, v, lam, a = sp.symbols("r t omega v lam a", positive=True)
    x1, x2, c1, c2 = sp.symbols("x1 x2 chi1 chi2", real=True)
    eta = x1 * x2
    S1, S2 = x1 ** 2 * c1, x2 ** 2 * c2
    # potential energy of the relative orbit (reduced mass eta), separation n in the plane
    # orthogonal to the spins: Newtonian, spin-spin (S.n = 0), and each body's Kerr
    # quadrupole acting on the companion at its equator (P2(0) = -1/2; m_j m_i^3 = eta x_i^2)
    U = -eta / r + lam * (-S1 * S2 / r ** 3 - eta * x1 ** 2 * c1 ** 2 / (2 * r ** 3)
                          - eta * x2 ** 2 * c2 ** 2 / (2 * r ** 3))
    w2 = sp.diff(U, r) / (eta * r)            # circular orbit: eta omega^2 r = dU/dr
    E = eta * w2 * r ** 2 / 2 + U
    # r as a function of v = omega^(1/3): r = v^-2 / (1 + lam a v^4), a fixed by Kepler's law
    rv = 1 / (v ** 2 * (1 + lam * a * v ** 4))
    kepler = sp.series(sp.simplify(w2.subs(r, rv)) - v ** 6, lam, 0, 2).removeO()
    a_sol = sp.solve(sp.expand(kepler.coeff(lam, 1)), a)[0]
    Ev = sp.series(E.subs(r, rv).subs(a, a_sol), lam, 0, 2).removeO()
    e_norm = sp.expand(Ev / (-eta * v ** 2 / 2))
    assert sp.simplify(e_norm.coeff(lam, 0)) == 1
    e4 = sp.simplify(e_norm.coeff(lam, 1) / v ** 4)
    # flux: mass quadrupole eta x^<i x^j> of the relative orbit, and the spin part of the
    # current quadrupole sum_A 3/2 x_A^<i S_A^j> with x_1 = x2 X, x_2 = -x1 X (centre of mass)
    X = sp.Matrix([r * sp.cos(w * t), r * sp.sin(w * t), 0])
    zhat = sp.Matrix([0, 0, 1])

    def stf(m):
        m = (m + m.T) / 2
        return m - sp.eye(3) * m.trace() / 3

    I = eta * stf(X * X.T)
    J = sp.Rational(3, 2) * stf((x2 * X) * (S1 * zhat).T + (-x1 * X) * (S2 * zhat).T)
    I3, J3 = I.diff(t, 3), J.diff(t, 3)
    F_I = sp.simplify(sum(I3[i, j] ** 2 for i in range(3) for j in range(3)) / 5)
    F_J = sp.simplify(sp.Rational(16, 45) * sum(J3[i, j] ** 2 for i in range(3) for j in range(3)))
    F = (F_I + lam * F_J).subs(w, sp.sqrt(w2))
    Fv = sp.series(sp.simplify(F.subs(r, rv).subs(a, a_sol)), lam, 0, 2).removeO()
    f_norm = sp.expand(sp.simplify(Fv / (sp.Rational(32, 5) * eta ** 2 * v ** 10)))
    assert sp.simplify(f_norm.coeff(lam, 0)) == 1
    f4 = sp.simplify(f_norm.coeff(lam, 1) / v ** 4)
    return (x1, x2, c1, c2), e4, f4


@lru_cache(maxsize=1)
def _derived():
    v, eta, delta, s, sg, L = sp.symbols("v eta delta s sg L")
    c1, c2 = sp.symbols("c1 c2")
    R = sp.Rational
    pi = sp.pi
    (x1, x2, chi1, chi2), e4ss, f4ss = _spin_spin_energy_flux()
    xs = {x1: (1 + delta) / 2, x2: (1 - delta) / 2, chi1: c1, chi2: c2}
    e4ss, f4ss = e4ss.subs(xs), f4ss.subs(xs)
    # E = -(M eta v^2 / 2) (1 + sum_k E_k v^k); s = S_l/M^2, sg = Sigma_l/M^2
    E = {2: -R(3, 4) - eta / 12,
         3: R(14, 3) * s + 2 * delta * sg,
         4: -R(27, 8) + R(19, 8) * eta - eta ** 2 / 24 + e4ss,
         5: (11 - R(61, 9) * eta) * s + delta * (3 - R(10, 3) * eta) * sg,
         6: -R(675, 64) + (R(34445, 576) - R(205, 96) * pi ** 2) * eta - R(155, 96) * eta ** 2
            - R(35, 5184) * eta ** 3,
         7: (R(135, 4) - R(367, 4) * eta + R(29, 12) * eta ** 2) * s
            + delta * (R(27, 4) - 39 * eta + R(5, 4) * eta ** 2) * sg}
    # F = (32/5) eta^2 v^10 (1 + sum_k F_k v^k + F6l v^6 ln v)
    F = {2: -R(1247, 336) - R(35, 12) * eta,
         3: 4 * pi - 4 * s - R(5, 4) * delta * sg,
         4: -R(44711, 9072) + R(9271, 504) * eta + R(65, 18) * eta ** 2 + f4ss,
         5: -(R(8191, 672) + R(583, 24) * eta) * pi + (-R(9, 2) + R(272, 9) * eta) * s
            + (-R(13, 16) + R(43, 4) * eta) * delta * sg,
         6: R(6643739519, 69854400) + R(16, 3) * pi ** 2 - R(1712, 105) * sp.EulerGamma
            - R(856, 105) * sp.log(16) + (-R(134543, 7776) + R(41, 48) * pi ** 2) * eta
            - R(94403, 3024) * eta ** 2 - R(775, 324) * eta ** 3 - 16 * pi * s - R(31, 6) * pi * delta * sg,
         7: (-R(16285, 504) + R(214745, 1728) * eta + R(193385, 3024) * eta ** 2) * pi
            + (R(476645, 6804) + R(6172, 189) * eta - R(2810, 27) * eta ** 2) * s
            + (R(9535, 336) + R(1849, 126) * eta - R(1501, 36) * eta ** 2) * delta * sg}
    F6l = -R(1712, 105)
    # E'(v)/F(v) = -(5 M / (32 eta)) v^-9 * ratio(v)
    num = 1 + sum(R(k + 2, 2) * E[k] * v ** k for k in E)
    den = 1 + sum(F[k] * v ** k for k in F) + F6l * v ** 6 * L
    ser = sp.expand(sp.series(num / den, v, 0, 8).removeO())
    c = {k: sp.expand(ser.coeff(v, k)) for k in range(8)}
    c6l = c[6].coeff(L, 1)
    c6 = c[6].coeff(L, 0)
    # term c_k u^k integrates to -3 v^(k-5) / ((8-k)(5-k)); Psi_PN = 3/(128 eta v^5) sum phi_k v^k
    phi = {}
    for k in (0, 1, 2, 3, 4, 7):
        phi[k] = sp.expand(R(40, (8 - k) * (5 - k)) * c[k])
    phi[5] = sp.expand(-R(40, 9) * c[5])          # (1/3 + ln v) -> (1 + 3 ln v)/3
    phi[6] = sp.expand(-20 * c6 + 10 * c6l)        # v ln v and v terms of the log integral
    phi6l = sp.expand(-20 * c6l)
    funcs = {k: sp.lambdify((eta, delta, s, sg, c1, c2), phi[k], "mpmath") for k in phi}
    return funcs, float(phi6l)


def _derived_vals(eta, delta, chi1, chi2, spin_spin=True):
    """Derived coefficients; spin_spin=False leaves the spin-spin pieces of E and F out (their
    products with the spin-orbit terms are cubic in the spins at 3.5PN, which the model omits)."""
    funcs, phi6l = _derived()
    x1, x2 = 0.5 * (1 + delta), 0.5 * (1 - delta)
    s = x1 * x1 * chi1 + x2 * x2 * chi2
    sg = x2 * chi2 - x1 * chi1
    c1, c2 = (chi1, chi2) if spin_spin else (0.0, 0.0)
    return np.array([float(funcs[k](eta, delta, s, sg, c1, c2)) for k in range(8)]), phi6l


ETAS = [0.25, 0.2475, 0.22, 0.2, 0.16, 0.1, 0.05]


@pytest.mark.parametrize("eta", ETAS)
def test_nonspinning_coefficients_match_energy_flux_derivation(eta):
    delta = math.sqrt(1 - 4 * eta)
    phi, phil = oracle.pn_coeffs(eta, delta, 0.0, 0.0)
    want, phi6l = _derived_vals(eta, delta, 0.0, 0.0)
    np.testing.assert_allclose(phi, want, rtol=1e-13, atol=1e-12)
    assert phil[5] == pytest.approx(3 * phi[5], rel=1e-15)
    assert phil[6] == pytest.approx(phi6l, rel=1e-15)
    assert np.all(phil[[0, 1, 2, 3, 4, 7]] == 0)


@pytest.mark.parametrize("eta,chi1,chi2", [(0.25, 0.3, -0.2), (0.2, 0.5, 0.7), (0.1, -0.8, 0.4),
                                           (0.16, 0.05, -0.05), (0.2475, 0.0, 0.85)])
def test_spin_orbit_terms_match_energy_flux_derivation(eta, chi1, chi2):
    """Odd part in the spins = spin-orbit terms at 1.5, 2.5, 3 and 3.5PN."""
    delta = math.sqrt(1 - 4 * eta)
    p_plus, _ = oracle.pn_coeffs(eta, delta, chi1, chi2)
    p_minus, _ = oracle.pn_coeffs(eta, delta, -chi1, -chi2)
    odd = 0.5 * (p_plus - p_minus)
    w_plus, _ = _derived_vals(eta, delta, chi1, chi2, spin_spin=False)
    # the derivation is linear in the spins except through products of 1.5PN terms (v^6 and up)
    w_minus, _ = _derived_vals(eta, delta, -chi1, -chi2, spin_spin=False)
    want = 0.5 * (w_plus - w_minus)
    np.testing.assert_allclose(odd, want, rtol=1e-12, atol=1e-10)
    assert abs(odd[3]) > 0 and abs(odd[5]) > 0


def test_spin_spin_term_structure():
    """2PN spin-spin: even in the spins, only in the 2PN coefficient, exchange symmetric,
    quadratic."""
    eta, delta = 0.2, math.sqrt(1 - 0.8)
    base, _ = oracle.pn_coeffs(eta, delta, 0.0, 0.0)
    a, _ = oracle.pn_coeffs(eta, delta, 0.3, -0.1)
    b, _ = oracle.pn_coeffs(eta, delta, -0.3, 0.1)
    c, _ = oracle.pn_coeffs(eta, delta, 0.6, -0.2)
    even_a = 0.5 * (a + b) - base
    even_c = 0.5 * (c + oracle.pn_coeffs(eta, delta, -0.6, 0.2)[0]) - base
    assert np.all(np.abs(np.delete(even_a, 4)) < 1e-12 * np.maximum(1, np.abs(np.delete(base, 4))))
    assert even_a[4] != 0
    assert even_c[4] == pytest.approx(4 * even_a[4], rel=1e-12)


@pytest.mark.parametrize("eta,chi1,chi2", [(0.25, 0.3, -0.2), (0.2, 0.5, 0.7), (0.1, -0.8, 0.4),
                                           (0.16, 0.05, -0.05), (0.2475, 0.0, 0.85), (0.1875, 0.8, 0.0),
                                           (0.09, -0.6, -0.7)])
def test_spin_spin_terms_match_energy_flux_derivation(eta, chi1, chi2):
    """Even part in the spins of the 2PN coefficient = the spin-spin term, against the one
    the derived spin-spin energy and flux give (S1 S2 coupling, each body's quadrupole-monopole
    term, and the square of the spin part of the current quadrupole). Cases with one spin zero
    isolate the self terms; spins of both signs weigh the S1 S2 coupling."""
    delta = math.sqrt(1 - 4 * eta)
    p0, _ = oracle.pn_coeffs(eta, delta, 0.0, 0.0)
    p_plus, _ = oracle.pn_coeffs(eta, delta, chi1, chi2)
    p_minus, _ = oracle.pn_coeffs(eta, delta, -chi1, -chi2)
    even = 0.5 * (p_plus + p_minus) - p0
    w0, _ = _derived_vals(eta, delta, 0.0, 0.0)
    w_plus, _ = _derived_vals(eta, delta, chi1, chi2)
    w_minus, _ = _derived_vals(eta, delta, -chi1, -chi2)
    want = 0.5 * (w_plus + w_minus) - w0
    assert abs(want[4]) > 1e-3
    assert even[4] == pytest.approx(want[4], rel=1e-12, abs=1e-12)


def test_spin_spin_derivation_limits():
    """The derived spin-spin pieces of E and F: for a single spinning body with a test mass
    (x2 -> 0) the energy term is -chi1^2 (the Kerr quadrupole alone), and both pieces are
    symmetric under the exchange of the bodies."""
    (x1, x2, c1, c2), e4, f4 = _spin_spin_energy_flux()
    assert sp.simplify(e4.subs({x1: 1, x2: 0}) + c1 ** 2) == 0
    swap = {x1: x2, x2: x1, c1: c2, c2: c1}
    assert sp.simplify(e4 - e4.subs(swap, simultaneous=True)) == 0
    assert sp.simplify(f4 - f4.subs(swap, simultaneous=True)) == 0


@pytest.mark.parametrize("eta,chi1,chi2", [(0.2, 0.3, -0.6), (0.1, 0.8, 0.1), (0.24, -0.05, 0.02)])
def test_label_exchange_symmetry(eta, chi1, chi2):
    """Psi(m1, m2, chi1, chi2) = Psi(m2, m1, chi2, chi1): delta -> -delta with the spins swapped."""
    delta = math.sqrt(1 - 4 * eta)
    a, al = oracle.pn_coeffs(eta, delta, chi1, chi2)
    b, bl = oracle.pn_coeffs(eta, -delta, chi2, chi1)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-11)
    np.testing.assert_allclose(al, bl, rtol=1e-13, atol=1e-11)


def _ev11(f_lo=20.0, df=0.25, K=8):
    return oracle.Event(1, K, f_lo, df, params=oracle.PARAMS_11D, phase=oracle.PHASE_EXPLICIT,
                        det_geom=[[0.3, 0.2, 0.1]])


def test_newtonian_limit():
    """3/(128 eta v^5) is the whole phase as v -> 0: Psi_PN * 128 eta v^5 / 3 -> 1 with a v^2 correction."""
    ev = _ev11()
    th = np.array([1.2, 0.8, 0.02, -0.03, 1.0, 0.2, 0.5, 0.3, 100.0, 0.0, 0.0])
    ok, src = ev.source(th)
    for f in (1e-4, 1e-3, 1e-2):
        v = (math.pi * src.M * oracle.t_sun() * f) ** (1 / 3)
        psi_pn = ev.psi(th, f)[0] + math.pi / 4
        ratio = psi_pn * 128 * src.eta * v ** 5 / 3
        assert abs(ratio - 1) < 10 * v ** 2


def test_stationary_phase_time():
    """dPsi/df = 2 pi t(f): at low frequency t_c - t(f) is the Newtonian chirp time
    tau0 = (5/256) Mc^(-5/3) (pi f)^(-8/3) (quadrupole formula), up to O(v^2)."""
    ev = _ev11()
    tc = 0.123
    th = np.array([1.3, 0.9, 0.0, 0.0, 1.0, 0.2, 0.5, 0.3, 100.0, tc, 0.0])
    ok, src = ev.source(th)
    mc_s = 1.3 * oracle.t_sun()
    for f in (0.5, 2.0, 5.0):
        h = 1e-4 * f
        dpsi = (ev.psi(th, f + h)[0] - ev.psi(th, f - h)[0]) / (2 * h)
        t_f = dpsi / (2 * math.pi)
        tau0 = 5.0 / 256.0 * mc_s ** (-5.0 / 3.0) * (math.pi * f) ** (-8.0 / 3.0)
        v = (math.pi * src.M * oracle.t_sun() * f) ** (1 / 3)
        assert abs((tc - t_f) / tau0 - 1) < 10 * v ** 2
