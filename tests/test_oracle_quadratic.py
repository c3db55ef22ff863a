"""Pins of the oracle's monotone quadratic interpolation of the upwind intensity
(section 3.3: a monotonic second-order scheme that neither overshoots nor loses
positivity, swept plane by plane so that the whole upwind plane is known).

The interpolant is pinned by its algebra (exact for parabolas while the control point
is inside the interval, bounded by the bracketing values, linear for collinear data);
the sweep by fields it must reproduce exactly, by the n_mu = 2 set (every ray hits a
vertex, so it must equal the bilinear sweep), by the exact solution of a sinusoidal
incident intensity advected through vacuum (against which it must converge faster
than bilinear interpolation), by positivity and the maximum principle on a sharp
beam, and by reflection symmetry."""
import numpy as np
import pytest

P_ = 2


def test_interpolant_endpoints_and_linear_reduction(oracle_mod):
    o = oracle_mod
    rng = np.random.default_rng(1)
    for _ in range(200):
        fm, f0, f1 = rng.normal(size=3)
        assert o.quad_interp(fm, f0, f1, 0.0) == f0
        assert o.quad_interp(fm, f0, f1, 1.0) == f1
        # collinear data: the interpolant is the straight line
        a, b = rng.normal(size=2)
        t = rng.random()
        assert abs(o.quad_interp(a - b, a, a + b, t) - (a + b * t)) <= 1e-14 * (abs(a) + abs(b) + 1)


def test_interpolant_exact_for_parabolas_inside_the_bracket(oracle_mod):
    """For q(u) = a + b u + c u^2 sampled at u = -1, 0, 1 the result is q(t) whenever the
    Bezier control point a + b/2 lies between q(0) and q(1)."""
    o = oracle_mod
    rng = np.random.default_rng(2)
    n = 0
    while n < 300:
        a, b, c = rng.normal(size=3)
        q = lambda u: a + b * u + c * u * u
        ctrl = a + b / 2
        if not (min(q(0), q(1)) <= ctrl <= max(q(0), q(1))):
            continue
        for t in rng.random(4):
            assert abs(o.quad_interp(q(-1), q(0), q(1), t) - q(t)) <= 1e-13 * (1 + abs(a) + abs(b) + abs(c))
        n += 1


def test_interpolant_is_bounded_and_monotone(oracle_mod):
    """No overshoot: the value stays between f0 and f1 and moves monotonically from f0
    to f1 as t runs over [0, 1] (positivity follows)."""
    o = oracle_mod
    rng = np.random.default_rng(3)
    ts = np.linspace(0.0, 1.0, 21)
    for _ in range(300):
        fm, f0, f1 = rng.normal(size=3) * rng.choice([1e-3, 1.0, 1e3])
        v = np.array([o.quad_interp(fm, f0, f1, t) for t in ts])
        lo, hi = min(f0, f1), max(f0, f1)
        tol = 1e-14 * max(abs(lo), abs(hi), 1e-300)
        assert np.all(v >= lo - tol) and np.all(v <= hi + tol)
        d = np.diff(v) * np.sign(f1 - f0)
        assert np.all(d >= -tol)


def _uniform_problem(o, interp, shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    chi = np.exp(rng.normal(0.0, 1.0, n)) * 2.0
    B = np.full(n, 1.7)
    return o.Problem(shape, chi, 1.0, B, n_mu=6, interp=interp,
                     bc_lo=(o.THERMAL, o.THERMAL, o.THERMAL), bc_hi=(o.THERMAL, o.THERMAL, o.THERMAL)), B


def test_thermal_enclosure_exact(oracle_mod):
    """Thermal walls and S = B uniform: I = B on every ray for any opacity."""
    o = oracle_mod
    p, B = _uniform_problem(o, 1, (7, 6, 8), 5)
    out = p.sweep(B, want_hk=True)
    assert np.max(np.abs(out["J"] - 1.7)) <= 1e-14
    assert np.max(np.abs(out["H"])) <= 1e-14


def test_nmu2_matches_bilinear(oracle_mod):
    """With n_mu = 2 on cubic cells every short characteristic ends on a vertex (the
    interpolation weight is 1 on one point), so once the lagged periodic ghosts have
    converged the quadratic and the bilinear sweeps must agree."""
    o = oracle_mod
    rng = np.random.default_rng(8)
    shape = (7, 6, 9)
    n = int(np.prod(shape))
    chi = np.exp(rng.normal(0.0, 1.0, n))
    S = 0.5 + rng.random(n)
    kw = dict(n_mu=2, bc_lo=(o.PERIODIC, o.PERIODIC, o.THERMAL), bc_hi=(o.PERIODIC, o.PERIODIC, o.VACUUM))
    lin = o.Problem(shape, chi, 1.0, S, **kw).formal_solve(S, converge_periodic=1e-15, max_sweeps=500)
    quad = o.Problem(shape, chi, 1.0, S, interp=1, **kw).formal_solve(S, converge_periodic=1e-15, max_sweeps=500)
    assert np.max(np.abs(quad["J"] - lin["J"]) / lin["J"]) <= 1e-13


def _octant_rays(d):
    d = np.asarray(d, float)
    d /= np.linalg.norm(d)
    mu = np.array([[sx * d[0], sy * d[1], sz * d[2]] for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)])
    return mu, np.full(8, 1.0 / 8.0)


def _advect_error(o, N, interp, mu, w):
    """chi = S = 0, periodic x/y, incident I0(x, y) = 1 + sin(2 pi x/N + 0.3) cos(2 pi y/N)/2
    on the bottom ghost plane: the exact J at (x, y, z) is the sum over upward rays of
    w I0 at the point where the ray crosses that plane.  Returns max |J - J_exact| / 0.5."""
    nx = ny = nz = N
    n = nx * ny * nz
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    I0 = lambda x, y: 1.0 + 0.5 * np.sin(2 * np.pi * x / nx + 0.3) * np.cos(2 * np.pi * y / ny)
    bottom = np.zeros((1, len(w), nx * ny))
    bottom[0, :] = I0(X, Y).ravel()
    top = np.zeros((1, len(w), nx * ny))
    p = o.Problem((nx, ny, nz), np.zeros(n), 1.0, np.zeros(n), mu=mu, w=w, interp=interp,
                  bc_lo=(o.PERIODIC, o.PERIODIC, o.FIXED), bc_hi=(o.PERIODIC, o.PERIODIC, o.FIXED),
                  fixed=[None, None, None, None, bottom, top])
    J = p.formal_solve(np.zeros(n), converge_periodic=1e-14, max_sweeps=400)["J"][0]
    Z = np.arange(nz)[:, None, None]
    Je = np.zeros((nz, ny, nx))
    for k in range(len(w)):
        if mu[k, 2] > 0:
            tx, ty = mu[k, 0] / mu[k, 2], mu[k, 1] / mu[k, 2]
            Je += w[k] * I0(X[None] - (Z + 1) * tx, Y[None] - (Z + 1) * ty)
    return float(np.max(np.abs(J - Je)) / 0.5)


def test_advected_sinusoid_converges_faster_than_bilinear(oracle_mod):
    """Rays crossing z planes first: the bilinear error falls about linearly with the
    cell size, the quadratic one faster, and it is several times smaller."""
    o = oracle_mod
    mu, w = _octant_rays((0.3, 0.4, 0.866))
    assert o.ray_info(mu[0])[0] == 2
    lin = [_advect_error(o, N, 0, mu, w) for N in (16, 32)]
    quad = [_advect_error(o, N, 1, mu, w) for N in (16, 32)]
    assert lin[0] / lin[1] < 2.0
    assert quad[0] / quad[1] > 2.5
    assert quad[1] < 0.3 * lin[1]


def test_advected_sinusoid_shallow_rays(oracle_mod):
    """Rays crossing x planes first travel through the periodic x boundary several
    times before reaching the top; the quadratic scheme still diffuses less."""
    o = oracle_mod
    mu, w = _octant_rays((0.866, 0.3, 0.4))
    assert o.ray_info(mu[0])[0] == 0
    assert _advect_error(o, 32, 1, mu, w) < 0.7 * _advect_error(o, 32, 0, mu, w)


def test_sharp_beam_positive_bounded_and_less_diffused(oracle_mod):
    """A narrow beam (one bright ghost vertex) through vacuum: J stays in
    [0, max incident x sum of weights] (no overshoot, positivity), and the quadratic
    sweep keeps more of the beam's peak than the bilinear one."""
    o = oracle_mod
    N = 16
    n = N ** 3
    mu, w = _octant_rays((0.3, 0.4, 0.866))
    bottom = np.zeros((1, 8, N * N))
    bottom[0, :, 5 + N * 6] = 1.0
    top = np.zeros((1, 8, N * N))
    peaks = []
    for interp in (0, 1):
        p = o.Problem((N, N, N), np.zeros(n), 1.0, np.zeros(n), mu=mu, w=w, interp=interp,
                      bc_lo=(o.PERIODIC, o.PERIODIC, o.FIXED), bc_hi=(o.PERIODIC, o.PERIODIC, o.FIXED),
                      fixed=[None, None, None, None, bottom, top])
        J = p.formal_solve(np.zeros(n), converge_periodic=1e-14, max_sweeps=200)["J"][0]
        assert np.min(J) >= 0.0
        assert np.max(J) <= 0.5 + 1e-15
        peaks.append(np.max(J[N - 1]))
    assert peaks[1] > 1.2 * peaks[0]


def test_reflection_symmetry(oracle_mod):
    o = oracle_mod
    nx, ny, nz = 6, 5, 7
    rng = np.random.default_rng(23)
    chi = np.exp(rng.normal(0, 1, (nz, ny, nx)))
    S = 1 + rng.random((nz, ny, nx))
    kw = dict(n_mu=4, interp=1, bc_lo=(o.PERIODIC, o.PERIODIC, o.THERMAL), bc_hi=(o.PERIODIC, o.PERIODIC, o.VACUUM))
    base = o.Problem((nx, ny, nz), chi, 1.0, S, **kw).sweep(S, want_hk=True)
    chi_r, S_r = chi[:, :, ::-1].copy(), S[:, :, ::-1].copy()
    ref = o.Problem((nx, ny, nz), chi_r, 1.0, S_r, **kw).sweep(S_r, want_hk=True)
    assert np.allclose(ref["J"][0], base["J"][0][:, :, ::-1], rtol=1e-13)
    assert np.allclose(ref["H"][0, 0], -base["H"][0, 0][:, :, ::-1], rtol=1e-11, atol=1e-14)


def test_ali_converges_to_a_fixed_point(oracle_mod):
    """Jacobi ALI with the quadratic upwind intensity converges, and its S satisfies
    S = (1 - eps) Lambda[S] + eps B to the stopping tolerance (Lambda* = sum w psi0
    is unchanged: S is still linear along the segment)."""
    o = oracle_mod
    rng = np.random.default_rng(31)
    shape = (9, 8, 10)
    n = int(np.prod(shape))
    chi = np.exp(rng.normal(0, 1, n)) * 3.0
    eps = 10 ** rng.uniform(-2, 0, n)
    B = rng.uniform(0.5, 1.5, n) ** 4
    p = o.Problem(shape, chi, eps, B, n_mu=4, interp=1)
    out = p.ali(delta_c=1e-10, max_iter=5000)
    S = out["S"]
    J = p.sweep(S)["J"]
    resid = np.max(np.abs((1 - eps.reshape(S.shape)) * J + eps.reshape(S.shape) * B.reshape(S.shape) - S) / S)
    assert resid <= 1e-8


def _crossing_beams(o, interp, N=32, beams=(True, True)):
    """Two narrow beams through vacuum that cross: beam A rides the ray (+, +, +) in from
    one vertex of the x-lo face, beam B the ray (-, +, +) in from the mirror vertex of the
    x-hi face; both climb in y and z, A towards +x and B towards -x, and they cross half
    way.  Returns J."""
    mu, w = _octant_rays((0.5, 0.45, 0.74))
    assert tuple(np.sign(mu[0])) == (1, 1, 1) and tuple(np.sign(mu[1])) == (-1, 1, 1)
    n = N ** 3
    na = len(w)
    fxl = np.zeros((1, na, N * N))
    fxh = np.zeros((1, na, N * N))
    if beams[0]:
        fxl[0, 0, 3 * N + 4] = 1.0     # x-lo face, (y, z) = (4, 3), ray (+, +, +)
    if beams[1]:
        fxh[0, 1, 3 * N + 4] = 1.0     # x-hi face, (y, z) = (4, 3), ray (-, +, +)
    p = o.Problem((N, N, N), np.zeros(n), 1.0, np.zeros(n), mu=mu, w=w, interp=interp,
                  bc_lo=(o.FIXED, o.VACUUM, o.VACUUM), bc_hi=(o.FIXED, o.VACUUM, o.VACUUM),
                  fixed=[fxl, fxh, None, None, None, None])
    return p.sweep(np.zeros(n))["J"][0]


def _spot(plane):
    """Total, centre along x and second moment about the centre of a 2D intensity spot."""
    Y, X = np.mgrid[0:plane.shape[0], 0:plane.shape[1]]
    tot = plane.sum()
    cx, cy = (plane * X).sum() / tot, (plane * Y).sum() / tot
    return tot, cx, float((plane * ((X - cx) ** 2 + (Y - cy) ** 2)).sum() / tot)


def test_crossing_beams_stay_narrow_and_bounded(oracle_mod):
    """The crossing-beam test of section 3.3: linear interpolation of I- spreads a beam
    over neighbouring vertices at every step; the monotone quadratic scheme keeps a beam
    narrower after the crossing (second moment of its spot on a plane near the top)
    and keeps more of its peak, while J stays non-negative and bounded by the incident
    intensity.  In vacuum each ray is transported on its own, so J of the crossing pair
    is exactly the sum of the two beams alone, for either interpolation, and the two
    beams are mirror images in x."""
    o = oracle_mod
    N = 32
    widths, peaks = [], []
    for interp in (0, 1):
        J = _crossing_beams(o, interp, N)
        JA = _crossing_beams(o, interp, N, (True, False))
        JB = _crossing_beams(o, interp, N, (False, True))
        assert np.max(np.abs(J - (JA + JB))) <= 1e-16
        assert np.min(J) >= 0.0
        assert np.max(J) <= 1.0 / 8.0 + 1e-15
        assert np.max(np.abs(JA - JB[:, :, ::-1])) <= 1e-16     # mirror images in x
        tot, cx, width = _spot(JA[N - 3])
        assert cx > (N - 1) / 2                                   # beam A has crossed the middle
        widths.append(width)
        peaks.append(float(JA[N - 3].max()))
    assert widths[1] < 0.7 * widths[0]
    assert peaks[1] > 1.2 * peaks[0]
