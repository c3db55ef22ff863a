"""Pins of the oracle's second-order (Bezier) formal solution, section 3.3 eq. rtdisc
with the clamped control point: segment coefficients against high-precision integrals,
reduction to the first-order form for a source linear in optical depth, exactness for a
quadratic source, the control point's clamping, an independent 1D two-stream solver,
uniform-field and symmetry identities, and higher accuracy than the first-order form
against the paper's eq. jana."""
import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")
mpmath.mp.dps = 50


def _bezier_integrals(dt):
    """alpha, beta, gamma = int_0^dt basis(t/dt) e^-t dt for the quadratic Bezier basis
    u^2 (S-), (1-u)^2 (S0), 2u(1-u) (Sc), at 50 digits."""
    d = mpmath.mpf(dt)
    f = lambda g: mpmath.quad(lambda t: g(t / d) * mpmath.e ** (-t), [0, d])
    return (float(f(lambda u: u * u)), float(f(lambda u: (1 - u) ** 2)), float(f(lambda u: 2 * u * (1 - u))))


@pytest.mark.parametrize("dt", [1e-7, 1e-4, 0.03, 0.3, 0.4999, 0.5, 0.7, 2.0, 9.0, 40.0])
def test_bezier_coefficients_against_integrals(oracle_mod, dt):
    E, a, b, g = oracle_mod.bezier_coeffs(dt)
    ra, rb, rg = _bezier_integrals(dt)
    assert E == pytest.approx(float(mpmath.e ** (-mpmath.mpf(dt))), rel=1e-15)
    for x, r in ((a, ra), (b, rb), (g, rg)):
        assert abs(x - r) <= 1e-14 * abs(r) + 1e-300
    # E + alpha + beta + gamma = 1 (a constant source passes unchanged)
    assert abs(E + a + b + g - 1.0) <= 4e-16


@pytest.mark.parametrize("dt", [1e-5, 0.01, 0.2, 0.5, 1.5, 12.0])
def test_bezier_reduces_to_linear_at_midpoint_control(oracle_mod, dt):
    """A control point halfway between S- and S0 makes the Bezier curve the straight
    line, so the weights of S- and S0 become psi- and psi0 of the first-order form."""
    E, a, b, g = oracle_mod.bezier_coeffs(dt)
    E1, pm, p0 = oracle_mod.coeffs(dt)
    assert abs((a + 0.5 * g) - pm) <= 1e-14 * max(pm, p0)
    assert abs((b + 0.5 * g) - p0) <= 1e-14 * max(pm, p0)


@pytest.mark.parametrize("h1,h2", [(0.3, 0.3), (1.0, 2.5), (4.0, 0.7), (0.02, 0.05)])
def test_quadratic_source_is_integrated_exactly(oracle_mod, h1, h2):
    """For S quadratic in optical depth (and monotone over the upwind segment) the
    parabola through S-, S0, S+ is S itself, the control point reproduces it, and the
    segment integral int_0^h1 S(-t) e^-t dt is exact."""
    c0, c1, c2 = 1.3, 0.4, 0.05        # S(tau) = c0 + c1 tau + c2 tau^2, tau along the ray
    S = lambda tau: c0 + c1 * tau + c2 * tau * tau
    Sm, S0, Sp = S(-h1), S(0.0), S(h2)
    Sc = oracle_mod.control_point(Sm, S0, Sp, h1, h2)
    E, a, b, g = oracle_mod.bezier_coeffs(h1)
    got = a * Sm + b * S0 + g * Sc
    ref = mpmath.quad(lambda t: (c0 - c1 * t + c2 * t * t) * mpmath.e ** (-t), [0, h1])
    assert got == pytest.approx(float(ref), rel=1e-13)


def test_control_point_rules(oracle_mod):
    cp = oracle_mod.control_point
    # linear data: the midpoint
    assert cp(1.0, 2.0, 3.0, 1.0, 1.0) == pytest.approx(1.5, rel=1e-15)
    # S' = (1 + 8)/2 = 4.5, Sc = 2 - 2.25 < min(S-, S0): clamped to the minimum
    assert cp(1.0, 2.0, 10.0, 1.0, 1.0) == 1.0
    # S' = (-1 + 9)/2 = 4, Sc = 1 - 2 < min(2, 1): clamped to the minimum
    assert cp(2.0, 1.0, 10.0, 1.0, 1.0) == 1.0
    # S' = (1 - 12)/2 = -5.5, Sc = 2 + 2.75 > max(1, 2): clamped to the maximum
    assert cp(1.0, 2.0, -10.0, 1.0, 1.0) == 2.0
    # no downwind interval: one-sided slope
    assert cp(1.0, 2.0, 99.0, 2.0, 0.0) == pytest.approx(1.5, rel=1e-15)
    # no upwind interval: S0
    assert cp(1.0, 2.0, 3.0, 0.0, 1.0) == 2.0


def _bez_1d(dt):
    """E, alpha, beta, gamma written out independently (expm1 closed forms, series for
    small dt)."""
    dt = float(dt)
    E = np.exp(-dt)
    if dt < 0.05:
        # leading terms of the three series (error below dt^8)
        a = dt / 3 - dt ** 2 / 4 + dt ** 3 / 10 - dt ** 4 / 36 + dt ** 5 / 168 - dt ** 6 / 960 + dt ** 7 / 6480
        g = dt / 3 - dt ** 2 / 6 + dt ** 3 / 20 - dt ** 4 / 90 + dt ** 5 / 504 - dt ** 6 / 3360 + dt ** 7 / 25920
        b = dt / 3 - dt ** 2 / 12 + dt ** 3 / 60 - dt ** 4 / 360 + dt ** 5 / 2520 - dt ** 6 / 20160 \
            + dt ** 7 / 181440
        return E, a, b, g
    e0 = -np.expm1(-dt)
    e1 = e0 - dt * E
    e2 = 2.0 * e1 - dt * dt * E
    a = e2 / dt ** 2
    g = 2.0 * e1 / dt - 2.0 * e2 / dt ** 2
    return E, a, e0 - a - g, g


def _cp_1d(Sm, S0, Sp, h1, h2):
    if h1 <= 0.0:
        return S0
    dm = (S0 - Sm) / h1
    Sd = dm if h2 <= 0.0 else (h2 * dm + h1 * (Sp - S0) / h2) / (h1 + h2)
    return min(max(S0 - 0.5 * h1 * Sd, min(Sm, S0)), max(Sm, S0))


def _two_stream_bezier_1d(chi, S, B0):
    """J of the 1D two-stream problem (mu = 1/sqrt 3, unit spacing) by the second-order
    Bezier scheme: thermal ghost below (I = B0, chi and S of level 0), vacuum above;
    ghosts beyond the ends copy chi and S of the end levels."""
    n = len(chi)
    s = np.sqrt(3.0)
    idx = lambda k: min(max(k, 0), n - 1)
    up, dn = np.zeros(n), np.zeros(n)
    I = B0
    for k in range(n):
        km, kp = idx(k - 1), idx(k + 1)
        h1 = s * (chi[km] + chi[k]) / 2
        h2 = s * (chi[k] + chi[kp]) / 2
        E, a, b, g = _bez_1d(h1)
        I = I * E + a * S[km] + b * S[k] + g * _cp_1d(S[km], S[k], S[kp], h1, h2)
        up[k] = I
    I = 0.0
    for k in range(n - 1, -1, -1):
        km, kp = idx(k + 1), idx(k - 1)
        h1 = s * (chi[km] + chi[k]) / 2
        h2 = s * (chi[k] + chi[kp]) / 2
        E, a, b, g = _bez_1d(h1)
        I = I * E + a * S[km] + b * S[k] + g * _cp_1d(S[km], S[k], S[kp], h1, h2)
        dn[k] = I
    return 0.5 * (up + dn)


def test_two_stream_bezier_3d_equals_independent_1d(oracle_mod):
    """n_mu = 2 on cubic cells: every ray meets corner vertices upwind and downwind,
    so a horizontally uniform 3D formal solution (periodic ghosts converged) is the
    1D two-stream one."""
    o = oracle_mod
    rng = np.random.default_rng(5)
    nz, nx, ny = 40, 2, 3
    chi_z = np.exp(rng.normal(0.0, 1.0, nz)) * 0.7
    S_z = 1.0 + np.cumsum(rng.normal(0.0, 0.2, nz)) ** 2 * 0.1 + rng.uniform(0, 0.3, nz)
    B_z = 1.0 + 0.1 * rng.random(nz)
    bc = lambda a: np.broadcast_to(a[:, None, None], (nz, ny, nx)).copy()
    p = o.Problem((nx, ny, nz), bc(chi_z), 1.0, bc(B_z), n_mu=2, order=1,
                  bc_lo=(o.PERIODIC, o.PERIODIC, o.THERMAL), bc_hi=(o.PERIODIC, o.PERIODIC, o.VACUUM))
    # the lagged periodic ghosts iterated to convergence (section 3) on the fixed S
    J3 = p.formal_solve(bc(S_z), converge_periodic=1e-15, max_sweeps=400)["J"][0]
    J1 = _two_stream_bezier_1d(chi_z, S_z, B_z[0])
    assert np.max(np.abs(J3 - J1[:, None, None]) / J1[:, None, None]) <= 1e-13


def test_bezier_uniform_field_and_enclosure(oracle_mod):
    """Uniform S with every face periodic gives I = S on every ray (J = S); a thermal
    enclosure with S = B uniform gives J = B for any chi."""
    o = oracle_mod
    rng = np.random.default_rng(2)
    shape = (6, 5, 7)
    chi = np.exp(rng.normal(0, 1, (7, 5, 6)))
    p = o.Problem(shape, chi, 0.5, np.full((7, 5, 6), 2.0), n_mu=4, order=1,
                  bc_lo=(o.PERIODIC,) * 3, bc_hi=(o.PERIODIC,) * 3)
    for _ in range(3):   # periodic memory converges to the uniform field
        J = p.sweep(np.full((7, 5, 6), 1.25))["J"]
    assert np.allclose(J, 1.25, rtol=1e-13)
    q = o.Problem(shape, chi, 1.0, np.full((7, 5, 6), 3.0), n_mu=4, order=1,
                  bc_lo=(o.THERMAL,) * 3, bc_hi=(o.THERMAL,) * 3)
    assert np.allclose(q.sweep(np.full((7, 5, 6), 3.0))["J"], 3.0, rtol=1e-13)


def test_bezier_reflection_symmetry(oracle_mod):
    """Reflecting the problem in x reflects J (the angle set is symmetric)."""
    o = oracle_mod
    rng = np.random.default_rng(9)
    nx, ny, nz = 7, 5, 6
    chi = np.exp(rng.normal(0, 1, (nz, ny, nx)))
    S = 1.0 + rng.random((nz, ny, nx))
    B = 1.0 + rng.random((nz, ny, nx))
    kw = dict(n_mu=4, order=1, bc_lo=(o.VACUUM, o.PERIODIC, o.THERMAL), bc_hi=(o.VACUUM, o.PERIODIC, o.VACUUM))
    J = o.Problem((nx, ny, nz), chi, 0.5, B, **kw).sweep(S)["J"][0]
    Jr = o.Problem((nx, ny, nz), chi[:, :, ::-1], 0.5, B[:, :, ::-1], **kw).sweep(S[:, :, ::-1])["J"][0]
    assert np.allclose(Jr[:, :, ::-1], J, rtol=1e-13)


def test_bezier_more_accurate_than_linear_against_eq_jana(oracle_mod):
    """Section 3.3 prefers the second-order form; on the scattering atmosphere of the
    paper's eq. jana (Eddington limit J = B (1 - e^{-sqrt(3 eps) tau}/(1 + sqrt eps)))
    the converged Bezier two-stream solution is much closer than the first-order one on
    the same grid (9 levels per decade of an exponential atmosphere, tau 1e-4..1e4,
    eps = 1e-2), and the Jacobi iteration with Lambda* = sum w beta converges."""
    o = oracle_mod
    eps = 1e-2
    per = 9
    n = per * 8 + 1
    tau = np.logspace(4, -4, n)                   # bottom -> top
    chi = tau / (per / np.log(10.0))              # exponential: chi = tau / scale height
    Jana = 1.0 - np.exp(-np.sqrt(3 * eps) * tau) / (1 + np.sqrt(eps))
    nx = ny = 2
    bc = lambda a: np.broadcast_to(a[:, None, None], (n, ny, nx)).copy()
    errs = {}
    for order in (0, 1):
        p = o.Problem((nx, ny, n), bc(chi), eps, np.ones((n, ny, nx)), n_mu=2, order=order,
                      bc_lo=(o.PERIODIC, o.PERIODIC, o.THERMAL), bc_hi=(o.PERIODIC, o.PERIODIC, o.VACUUM))
        res = p.ali(delta_c=1e-10, max_iter=20000)
        assert res["converged"]
        J = res["J"][0][:, 0, 0]
        errs[order] = np.max(np.abs(J - Jana) / Jana)
    assert errs[1] < 0.1 * errs[0]
    assert errs[1] < 0.01
