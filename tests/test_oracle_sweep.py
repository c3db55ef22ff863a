"""Pins of the oracle's formal solution (paper section 3.3) against mathematics that
does not come from the oracle: high-precision integrals, exact discrete solutions of
horizontally uniform slabs derived by hand, a dense brute-force Lambda operator,
invariants (isotropy, beam conservation) and symmetries."""
import mpmath
import numpy as np
import pytest

mpmath.mp.dps = 50


def _mp_coeffs(dt):
    """Integrals of a source linear in tau over one segment, to 50 digits:
    psi_minus = int_0^dt (1 - t/dt) e^-(dt-t) dt, psi_0 = int_0^dt (t/dt) e^-(dt-t) dt."""
    x = mpmath.mpf(dt)
    E = mpmath.e ** (-x)
    psi_m = mpmath.quad(lambda t: (1 - t / x) * mpmath.e ** (-(x - t)), [0, x])
    psi_0 = mpmath.quad(lambda t: (t / x) * mpmath.e ** (-(x - t)), [0, x])
    return E, psi_m, psi_0


@pytest.mark.parametrize("dt", [1e-9, 1e-5, 1e-3, 0.03, 0.0999, 0.1, 0.1001, 0.5, 1.0, 3.7, 40.0, 700.0])
def test_coefficients_against_integrals(oracle_mod, dt):
    E, pm, p0 = oracle_mod.coeffs(dt)
    Em, pmm, p0m = _mp_coeffs(dt)
    assert abs(E - float(Em)) <= 1e-15 * float(Em) + 1e-300
    assert abs(p0 - float(p0m)) <= 1e-14 * float(p0m)
    # psi_minus = e0 - psi_0 cancels for large dt; its error is judged against the
    # larger of the two weights it is summed with
    assert abs(pm - float(pmm)) <= 1e-14 * max(float(pmm), float(p0m))


def test_coefficients_partition_of_unity(oracle_mod):
    """A constant source reproduces itself: E + psi_minus + psi_0 = 1."""
    for dt in np.logspace(-12, 3, 200):
        E, pm, p0 = oracle_mod.coeffs(dt)
        assert abs(E + pm + p0 - 1.0) < 3e-16
    E, pm, p0 = oracle_mod.coeffs(0.0)
    assert (E, pm, p0) == (1.0, 0.0, 0.0)


def test_geometry_lq4(oracle_mod):
    """Cubic cells: the upwind segment crosses the plane of the largest |mu| first,
    s = dx/|mu_d| and the face offsets are |mu_b|/|mu_d|."""
    mu, w = oracle_mod.quadrature(4)
    for m in mu:
        d, a, b, sg, s, fa, fb = oracle_mod.ray_info(m)
        am = np.abs(m)
        assert d == int(np.argmax(am))
        assert {a, b} == {0, 1, 2} - {d} and a < b
        assert sg == tuple(int(np.sign(x)) for x in m)
        assert abs(s - 1.0 / am[d]) < 1e-15
        assert abs(fa - am[a] / am[d]) < 1e-15 and abs(fb - am[b] / am[d]) < 1e-15


def test_geometry_ties_and_aspect(oracle_mod):
    # the cube diagonal hits the corner: tie broken towards z, both offsets 1
    d, a, b, sg, s, fa, fb = oracle_mod.ray_info(np.array([1, -1, 1]) / np.sqrt(3))
    assert (d, a, b, sg) == (2, 0, 1, (1, -1, 1)) and fa == 1.0 and fb == 1.0
    assert abs(s - np.sqrt(3)) < 1e-15
    # equal |mu_x| = |mu_y| > |mu_z|: y wins the x/y tie
    d, *_ = oracle_mod.ray_info(np.array([0.6, 0.6, np.sqrt(0.28)]))
    assert d == 1
    # elongated cells change which plane is crossed first: dx = 4 makes z first
    m = np.array([0.8, 0.36, 0.48])
    d, a, b, sg, s, fa, fb = oracle_mod.ray_info(m, h=(4.0, 1.0, 1.0))
    assert d == 2 and abs(s - 1.0 / 0.48) < 1e-15
    assert abs(fa - s * 0.8 / 4.0) < 1e-15 and abs(fb - s * 0.36) < 1e-15
    # a zero cosine never selects its axis; its offset is 0 and its sign +1
    d, a, b, sg, s, fa, fb = oracle_mod.ray_info(np.array([0.0, -0.6, 0.8]))
    assert d == 2 and sg == (1, -1, 1) and fa == 0.0 and abs(fb - 0.75) < 1e-15


# ----------------------------------------------------------------------------------
# exact discrete solution of a horizontally uniform slab, derived by hand
# ----------------------------------------------------------------------------------

def _slab_exact(mu, h, chi_z, S_z, I_bot, I_top):
    """Per ray, the heights k of a horizontally uniform slab (chi, S depend on z only).
    Every face vertex at height k has the intensity of the cell at height k, so for a
    ray whose first crossed plane is z:
        I_k = I_{k-1} E + psi_m S_{k-1} + psi_0 S_k,
    and for a ray that crosses an x or y plane first, with fractional z offset f_z:
        I_k = [(1-f_z) I_k + f_z I_{k-1}] E + psi_m S^- + psi_0 S_k,
        S^- = (1-f_z) S_k + f_z S_{k-1},  chi^- likewise,
    i.e. I_k = (f_z I_{k-1} E + psi_m S^- + psi_0 S_k) / (1 - (1-f_z) E).
    Heights are numbered along the ray's travel; the ghost below the first level
    carries I_bot (upward rays) or I_top (downward rays) and the boundary S, chi.
    Coefficients from closed forms evaluated with mpmath."""
    nz = len(chi_z)
    out = np.zeros((len(mu), nz))
    for r, m in enumerate(mu):
        am = np.abs(m)
        lens = [h[q] / am[q] if am[q] > 0 else np.inf for q in range(3)]
        d = 2
        if lens[1] < lens[d]:
            d = 1
        if lens[0] < lens[d]:
            d = 0
        s = lens[d]
        order = range(nz) if m[2] > 0 else range(nz - 1, -1, -1)
        prev_k = None
        Iprev = I_bot if m[2] > 0 else I_top
        for k in order:
            kp = prev_k if prev_k is not None else k  # ghost copies the boundary vertex
            if d == 2:
                Sm, Cm = S_z[kp], chi_z[kp]
            else:
                fz = min(s * am[2] / h[2], 1.0)
                Sm = (1 - fz) * S_z[k] + fz * S_z[kp]
                Cm = (1 - fz) * chi_z[k] + fz * chi_z[kp]
            dt = s * (Cm + chi_z[k]) / 2
            E, pmm, p0m = (float(x) for x in _mp_coeffs(dt)) if dt > 0 else (1.0, 0.0, 0.0)
            if d == 2:
                I = Iprev * E + pmm * Sm + p0m * S_z[k]
            else:
                I = (fz * Iprev * E + pmm * Sm + p0m * S_z[k]) / (1 - (1 - fz) * E)
            out[r, k] = I
            Iprev, prev_k = I, k
    return out


def _seed_from_levels(p, I_rk):
    """Periodic memory holding the horizontally uniform intensity of each ray."""
    nx, ny, nz = p.n
    planes = []
    for q in range(3):
        if p.prev[q] is None:
            planes.append(None)
            continue
        n1 = ny if q == 0 else nx
        arr = np.repeat(I_rk[:, :, None], n1, axis=2).reshape(1, p.na, -1)
        planes.append(np.repeat(arr, p.nf, axis=0))
    return planes


@pytest.mark.parametrize("n_mu,h", [(4, (1.0, 1.0, 1.0)), (6, (1.0, 1.0, 1.0)),
                                    (4, (1.5, 0.7, 1.0)), (8, (1.0, 1.0, 0.5))])
def test_uniform_slab_exact(oracle_mod, n_mu, h):
    """Horizontally uniform, vertically varying slab with periodic x/y, thermal bottom
    and vacuum top: one sweep with exact periodic memory reproduces the hand-derived
    discrete solution for every ray class."""
    o = oracle_mod
    nx, ny, nz = 5, 4, 9
    rng = np.random.default_rng(7)
    chi_z = np.exp(rng.normal(0, 1, nz))
    S_z = 1.0 + rng.random(nz)
    chi = np.broadcast_to(chi_z[:, None, None], (nz, ny, nx)).copy()
    S = np.broadcast_to(S_z[:, None, None], (nz, ny, nx)).copy()
    B = S.copy()
    p = o.Problem((nx, ny, nz), chi, 1.0, B, n_mu=n_mu, h=h,
                  bc_lo=(o.PERIODIC, o.PERIODIC, o.THERMAL), bc_hi=(o.PERIODIC, o.PERIODIC, o.VACUUM))
    I_rk = _slab_exact(p.mu, h, chi_z, S_z, I_bot=S_z[0], I_top=0.0)
    p.seed_periodic(_seed_from_levels(p, I_rk))
    out = p.sweep(S, want_hk=True)
    J = (p.w[:, None] * I_rk).sum(0)
    Hz = (p.w[:, None] * p.mu[:, 2:3] * I_rk).sum(0)
    Kzz = (p.w[:, None] * p.mu[:, 2:3] ** 2 * I_rk).sum(0)
    assert np.allclose(out["J"][0], J[:, None, None], rtol=1e-13, atol=0)
    assert np.allclose(out["H"][2, 0], Hz[:, None, None], rtol=1e-12, atol=1e-14)
    assert np.allclose(out["K"][2, 0], Kzz[:, None, None], rtol=1e-13, atol=0)
    # horizontal fluxes vanish by symmetry of the angle set
    assert np.max(np.abs(out["H"][0])) < 1e-14 and np.max(np.abs(out["H"][1])) < 1e-14
    # after the sweep the periodic memory holds the same uniform solution
    p2 = _seed_from_levels(p, I_rk)
    for q in range(2):
        assert np.allclose(p.prev[q], p2[q], rtol=1e-13)


def test_uniform_slab_periodic_iteration_converges(oracle_mod):
    """Starting from cold periodic ghosts (I = S), repeated sweeps on a fixed S converge
    to the same exact slab solution (the periodic iteration of section 3)."""
    o = oracle_mod
    nx, ny, nz = 4, 4, 6
    chi_z = np.array([0.3, 0.5, 0.9, 1.4, 2.0, 3.1])
    S_z = np.array([2.0, 1.8, 1.5, 1.3, 1.2, 1.1])
    chi = np.broadcast_to(chi_z[:, None, None], (nz, ny, nx)).copy()
    S = np.broadcast_to(S_z[:, None, None], (nz, ny, nx)).copy()
    p = o.Problem((nx, ny, nz), chi, 1.0, S, n_mu=4,
                  bc_lo=(o.PERIODIC, o.PERIODIC, o.VACUUM), bc_hi=(o.PERIODIC, o.PERIODIC, o.VACUUM))
    out = p.formal_solve(S, converge_periodic=1e-15, max_sweeps=400)
    I_rk = _slab_exact(p.mu, (1, 1, 1), chi_z, S_z, I_bot=0.0, I_top=0.0)
    J = (p.w[:, None] * I_rk).sum(0)
    assert out["sweeps"] > 2
    assert np.allclose(out["J"][0], J[:, None, None], rtol=1e-13)


def test_isotropic_field(oracle_mod):
    """Uniform S with every face periodic: I = S on every ray from the first sweep
    (cold ghosts are S), so J = S, H = 0, K_ij = delta_ij S/3 for any opacity field."""
    o = oracle_mod
    nx, ny, nz = 4, 5, 3
    rng = np.random.default_rng(3)
    chi = np.exp(rng.normal(0, 1.5, nz * ny * nx))
    S = np.full(nx * ny * nz, 2.5)
    p = o.Problem((nx, ny, nz), chi, 1.0, S, n_mu=6,
                  bc_lo=(o.PERIODIC,) * 3, bc_hi=(o.PERIODIC,) * 3)
    out = p.sweep(S, want_hk=True)
    assert np.allclose(out["J"], 2.5, rtol=1e-15)
    assert np.max(np.abs(out["H"])) < 1e-15
    for c in range(3):
        assert np.allclose(out["K"][c], 2.5 / 3, rtol=1e-14)
    for c in range(3, 6):
        assert np.max(np.abs(out["K"][c])) < 1e-15
    lam = out["lam"][0]
    assert np.all(lam > 0) and np.all(lam < 1)


def test_thermal_enclosure_exact(oracle_mod):
    """S = B = const with thermal faces everywhere: I = B exactly for a random opacity
    field (the thick-limit equilibrium J = B)."""
    o = oracle_mod
    nx, ny, nz = 5, 3, 4
    rng = np.random.default_rng(11)
    chi = np.exp(rng.normal(0, 2, nx * ny * nz))
    B = np.full(nx * ny * nz, 3.0)
    p = o.Problem((nx, ny, nz), chi, 1.0, B, n_mu=4, bc_lo=(o.THERMAL,) * 3, bc_hi=(o.THERMAL,) * 3)
    out = p.sweep(B)
    assert np.allclose(out["J"], 3.0, rtol=2e-15)


def test_lambda_star_is_diagonal_of_dense_lambda(oracle_mod):
    """Brute force: with vacuum faces J = Lambda S is linear; build Lambda column by
    column and compare its diagonal with the oracle's Lambda* = sum_k w_k psi0_k
    (section 3.4, diagonal operator of eq. dsjacobi).  Equality holds for interior
    cells; a boundary cell's ghost vertices copy its own S, which adds psi_minus terms
    to the true diagonal there, so Lambda* is a lower bound on the boundary."""
    o = oracle_mod
    nx, ny, nz = 5, 4, 5
    n = nx * ny * nz
    rng = np.random.default_rng(5)
    chi = np.exp(rng.normal(0, 1, n))
    p = o.Problem((nx, ny, nz), chi, 1.0, np.zeros(n), n_mu=4,
                  bc_lo=(o.VACUUM,) * 3, bc_hi=(o.VACUUM,) * 3)
    L = np.zeros((n, n))
    lam = None
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        out = p.sweep(e)
        L[:, c] = out["J"].ravel()
        lam = out["lam"].ravel()
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inner = ((i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)).ravel()
    assert inner.sum() == 18
    assert np.allclose(np.diag(L)[inner], lam[inner], rtol=1e-14, atol=0)
    assert np.all(np.diag(L)[~inner] >= lam[~inner] * (1 - 1e-14))
    # linearity: Lambda applied to a random S equals the matrix product
    S = rng.random(n)
    assert np.allclose(p.sweep(S)["J"].ravel(), L @ S, rtol=1e-13)
    # every coefficient is a product of non-negative weights
    assert np.all(L >= 0)


@pytest.mark.parametrize("bottom", ["vacuum", "thermal"])
def test_ali_fixed_point_dense_solve(oracle_mod, bottom):
    """The Jacobi ALI converges to the solution of eq. sourcefunc3,
    [1 - (1-eps) Lambda] S = eps B + (1-eps) j_b, solved densely (j_b = J of S = 0
    holds the thermal boundary's contribution)."""
    o = oracle_mod
    nx, ny, nz = 3, 3, 4
    n = nx * ny * nz
    rng = np.random.default_rng(9)
    chi = np.exp(rng.normal(0.5, 1, n))
    eps = 10 ** rng.uniform(-2, 0, n)
    B = 1.0 + rng.random(n)
    bot = o.THERMAL if bottom == "thermal" else o.VACUUM
    mk = lambda: o.Problem((nx, ny, nz), chi, eps, B, n_mu=4,
                           bc_lo=(o.VACUUM, o.VACUUM, bot), bc_hi=(o.VACUUM,) * 3)
    p = mk()
    jb = p.sweep(np.zeros(n))["J"].ravel()
    L = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        L[:, c] = p.sweep(e)["J"].ravel() - jb
    S_star = np.linalg.solve(np.eye(n) - (1 - eps)[:, None] * L, eps * B + (1 - eps) * jb)
    res = mk().ali(delta_c=1e-14, max_iter=5000)
    assert res["converged"]
    assert np.allclose(res["S"].ravel(), S_star, rtol=1e-11)
    # the returned J is Lambda[S^n] one update behind; at convergence S = (1-eps)J + eps B
    assert np.allclose(res["J"].ravel(), L @ S_star + jb, rtol=1e-11)


def test_beam_conservation(oracle_mod):
    """chi = S = 0 (section 5.2's rarefied beam domain): dtau = 0 and the intensity is
    only interpolated.  One ray enters through fixed-intensity cells at the bottom; with
    periodic x/y, once the lagged ghosts have caught up the plane sum of I is the same
    on every level for a ray that crosses z planes first (bilinear weights sum to 1)."""
    o = oracle_mod
    nx, ny, nz = 6, 5, 7
    n = nx * ny * nz
    mu, w = o.quadrature(4)
    ray = next(r for r in range(len(w)) if mu[r, 2] > 0 and np.argmax(np.abs(mu[r])) == 2)
    fixed_bot = np.zeros((1, len(w), nx * ny))
    fixed_bot[0, ray, 2 + nx * 1] = 5.0
    fixed_bot[0, ray, 3 + nx * 3] = 2.0
    fixed_top = np.zeros((1, len(w), nx * ny))
    p = o.Problem((nx, ny, nz), np.zeros(n), 1.0, np.zeros(n), mu=mu, w=w,
                  bc_lo=(o.PERIODIC, o.PERIODIC, o.FIXED), bc_hi=(o.PERIODIC, o.PERIODIC, o.FIXED),
                  fixed=[None, None, None, None, fixed_bot, fixed_top])
    for _ in range(nz + 3):
        J = p.sweep(np.zeros(n))["J"][0]
    sums = J.sum(axis=(1, 2)) / w[ray]
    assert np.allclose(sums, 7.0, rtol=1e-14)
    assert np.min(J) >= 0.0


def _mirror_x(a, nx, ny, nz):
    return a.reshape(-1, nz, ny, nx)[..., ::-1]


def test_reflection_and_rotation_symmetry(oracle_mod):
    """Reflecting the fields in x, or rotating them by 90 degrees about z, transforms
    J, H and K accordingly (the angle set is invariant under both)."""
    o = oracle_mod
    nx = ny = 5
    nz = 4
    n = nx * ny * nz
    rng = np.random.default_rng(21)
    chi = np.exp(rng.normal(0, 1, (nz, ny, nx)))
    S = 1 + rng.random((nz, ny, nx))
    kw = dict(n_mu=6, bc_lo=(o.PERIODIC, o.PERIODIC, o.THERMAL), bc_hi=(o.PERIODIC, o.PERIODIC, o.VACUUM))
    base = o.Problem((nx, ny, nz), chi, 1.0, S, **kw).sweep(S, want_hk=True)
    # reflection x -> -x
    chi_r, S_r = chi[:, :, ::-1].copy(), S[:, :, ::-1].copy()
    ref = o.Problem((nx, ny, nz), chi_r, 1.0, S_r, **kw).sweep(S_r, want_hk=True)
    assert np.allclose(ref["J"][0], base["J"][0][:, :, ::-1], rtol=1e-13)
    assert np.allclose(ref["H"][0, 0], -base["H"][0, 0][:, :, ::-1], rtol=1e-11, atol=1e-14)
    assert np.allclose(ref["K"][3, 0], -base["K"][3, 0][:, :, ::-1], rtol=1e-11, atol=1e-14)
    # rotation: new[k, j, i] = old[k, i, n-1-j], i.e. a point (x, y) moves to
    # (y, n-1-x) and a vector (v_x, v_y) turns into (v_y, -v_x)
    rot = lambda a: np.transpose(a, (0, 2, 1))[:, ::-1, :]
    chi_t, S_t = rot(chi).copy(), rot(S).copy()
    tr = o.Problem((nx, ny, nz), chi_t, 1.0, S_t, **kw).sweep(S_t, want_hk=True)
    assert np.allclose(tr["J"][0], rot(base["J"][0]), rtol=1e-12)
    assert np.allclose(tr["H"][0, 0], rot(base["H"][1, 0]), rtol=1e-10, atol=1e-13)
    assert np.allclose(tr["H"][1, 0], -rot(base["H"][0, 0]), rtol=1e-10, atol=1e-13)
    assert np.allclose(tr["K"][3, 0], -rot(base["K"][3, 0]), rtol=1e-10, atol=1e-13)
    assert np.allclose(tr["K"][0, 0], rot(base["K"][1, 0]), rtol=1e-12)
    assert np.allclose(tr["H"][2, 0], rot(base["H"][2, 0]), rtol=1e-10, atol=1e-13)
