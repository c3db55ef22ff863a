"""Pins of the oracle's Gauss-Seidel ALI (section 3.4: S updated as soon as J is
complete, the scheme of Trujillo Bueno & Fabiani Bendicho generalised to 3D with
bilinear interpolation) in its two orderings:

* "zone", the paper's: zones updated one at a time in the backward sweep of Fig.
  f:sweep (from the top corner, i the fastest index), each with J from the current S;
* "plane", the variant the GPU runs: horizontal planes from the top down as the
  blocks, Jacobi inside a plane.

Each is pinned by its definition written out the slow way (a full formal solution
with the current S before every zone, or every plane, update), by textbook point or
block Gauss-Seidel on the Lambda matrix assembled column by column from formal
solutions, by the paper's result that Gauss-Seidel needs about half the iterations
of Jacobi (the zone order; the plane blocks gain less with shallow rays), by the
common fixed point of the iterations, and by the eps = 1 case (S = B after one
iteration)."""
import numpy as np
import pytest

P_, V_, T_, F_ = 2, 0, 1, 3


def _problem(o, shape, seed, nf=1, n_mu=4, bc_lo=(P_, P_, T_), bc_hi=(P_, P_, V_), fixed=None, eps_range=(1e-2, 1.0)):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    chi = np.exp(rng.normal(0.0, 1.0, (nf, n))) * 1.5
    eps = 10 ** rng.uniform(np.log10(eps_range[0]), np.log10(eps_range[1]), (nf, n))
    B = rng.uniform(0.5, 1.5, (nf, n)) ** 4
    return o.Problem(shape, chi, eps, B, n_mu=n_mu, bc_lo=bc_lo, bc_hi=bc_hi, fixed=fixed)


def _planes_from(o, p, S):
    """Periodic memory holding S of the wrapped vertex (the cold ghosts) for S."""
    nx, ny, nz = p.n
    S = S.reshape(p.chi.shape)
    planes = [None, None, None]
    for q in range(2):
        if p.bc_lo[q] != P_:
            continue
        arr = np.zeros((p.nf, p.na, p._plane(q)))
        for r in range(p.na):
            sg = o.ray_info(p.mu[r], p.h)[3][q]
            outc = p.n[q] - 1 if sg > 0 else 0
            arr[:, r] = (S[:, :, :, outc] if q == 0 else S[:, :, outc, :]).reshape(p.nf, -1)
        planes[q] = arr
    return planes


def _brute_force_iteration(o, p, S, memory):
    """Gauss-Seidel by definition: for k from the top down, J on plane k is that of a
    full formal solution with the current S (periodic ghosts from ``memory``); plane
    k is then updated with eq. dsjacobi.  Returns S, J, the new periodic memory (rays
    going up from the solution with the old S, rays going down from the one with the
    new S)."""
    nz = p.n[2]
    S_cur = S.reshape(p.chi.shape).copy()
    J = np.zeros_like(S_cur)
    for k in range(nz - 1, -1, -1):
        p.seed_periodic(memory)
        out = p.sweep(S_cur)
        e, lam = p.eps[:, k], out["lam"][:, k]
        J[:, k] = out["J"][:, k]
        S_cur[:, k] += ((1.0 - e) * J[:, k] + e * p.B[:, k] - S_cur[:, k]) / (1.0 - (1.0 - e) * lam)
    p.seed_periodic(memory)
    p.sweep(S.reshape(p.chi.shape))
    up = [None if a is None else a.copy() for a in p.prev]
    p.seed_periodic(memory)
    p.sweep(S_cur)
    new = [None if a is None else a.copy() for a in p.prev]
    down = p.mu[:, 2] < 0.0
    for q in range(3):
        if new[q] is not None:
            new[q][:, ~down] = up[q][:, ~down]
    return S_cur, J, new


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


@pytest.mark.parametrize("case", ["periodic", "fixed_faces", "cold"])
def test_iteration_matches_its_definition(oracle_mod, case):
    o = oracle_mod
    if case == "fixed_faces":
        shape, lo, hi = (5, 4, 6), (F_, V_, T_), (T_, F_, V_)
        rng = np.random.default_rng(4)
        fixed = [None] * 6
        fixed[0] = rng.uniform(0, 2, (2, 24, 4 * 6))
        fixed[3] = rng.uniform(0, 2, (2, 24, 5 * 6))
    else:
        shape, lo, hi, fixed = (5, 4, 6), (P_, P_, T_), (P_, P_, V_), None
    p_gs = _problem(o, shape, 11, nf=2, bc_lo=lo, bc_hi=hi, fixed=fixed)
    p_bf = _problem(o, shape, 11, nf=2, bc_lo=lo, bc_hi=hi, fixed=fixed)
    rng = np.random.default_rng(12)
    S = (0.5 + rng.random(p_gs.chi.shape)) * p_gs.B
    if case == "cold":
        memory = _planes_from(o, p_gs, S)
        p_gs.reset_periodic()
    else:
        memory = [None if a is None else rng.uniform(0.5, 2.0, a.shape) for a in p_gs.prev]
        p_gs.seed_periodic(memory)
    out = p_gs.gs_iteration(S)
    S_bf, J_bf, mem_bf = _brute_force_iteration(o, p_bf, S, memory)
    assert _rel(out["S"], S_bf) <= 1e-13
    assert _rel(out["J"], J_bf) <= 1e-13
    for q in range(3):
        if mem_bf[q] is not None:
            assert _rel(p_gs.prev[q], mem_bf[q]) <= 1e-13


def _lambda_matrix(p):
    """Lambda as an affine map S -> J assembled from formal solutions (no periodic
    axis, so no memory between sweeps): J = A S + c."""
    n = p.chi.size
    c = p.sweep(np.zeros(n))["J"].ravel()
    A = np.zeros((n, n))
    for m in range(n):
        e = np.zeros(n)
        e[m] = 1.0
        A[:, m] = p.sweep(e)["J"].ravel() - c
    return A, c


def test_textbook_block_gauss_seidel_on_the_lambda_matrix(oracle_mod):
    o = oracle_mod
    shape = (4, 3, 5)
    kw = dict(bc_lo=(T_, V_, T_), bc_hi=(V_, T_, V_))
    p = _problem(o, shape, 21, **kw)
    A, c = _lambda_matrix(_problem(o, shape, 21, **kw))
    lam = p.sweep(p.B)["lam"].ravel()
    # Lambda* is the diagonal of Lambda away from the faces, where no ghost vertex
    # copies the vertex's own S into its upwind interpolation
    inner = np.zeros(shape[::-1], dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    inner = inner.ravel()
    assert inner.sum() == 6
    assert np.max(np.abs(np.diag(A)[inner] - lam[inner])) <= 1e-14
    eps, B = p.eps.ravel(), p.B.ravel()
    S = B.copy()
    nxy = shape[0] * shape[1]
    for _ in range(4):
        for k in range(shape[2] - 1, -1, -1):
            sl = slice(k * nxy, (k + 1) * nxy)
            J = A[sl] @ S + c[sl]
            S[sl] = S[sl] + ((1.0 - eps[sl]) * J + eps[sl] * B[sl] - S[sl]) / (1.0 - (1.0 - eps[sl]) * lam[sl])
    out = p.ali_gs(fixed_iters=4)
    assert _rel(out["S"].ravel(), S) <= 1e-12


def _stratified(o, shape, eps, n_mu):
    """A plane-parallel scattering atmosphere (chi falling off with height, periodic
    x and y, thermal bottom, vacuum top) with a horizontally varying B."""
    nx, ny, nz = shape
    k = np.arange(nz)
    prof = np.exp(-k / (nz / 6.0))
    prof *= 1e3 / prof.sum()
    chi = np.broadcast_to(prof[:, None, None], (nz, ny, nx)).copy()
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    T = 1.0 + 0.1 * np.sin(2 * np.pi * X / nx) * np.cos(2 * np.pi * Y / ny)
    B = np.broadcast_to((T ** 4)[None], (nz, ny, nx)).copy()
    return o.Problem(shape, chi, eps, B, n_mu=n_mu)


@pytest.mark.parametrize("n_mu, lo, hi", [(2, 1.7, 2.1), (4, 1.25, 1.7)])
def test_fewer_iterations_than_jacobi_and_the_same_fixed_point(oracle_mod, n_mu, lo, hi):
    """The paper (after TF95) finds Gauss-Seidel converging nearly twice as fast as
    Jacobi.  With n_mu = 2 every ray crosses a z face first, no vertex of a plane
    depends on another of the same plane, and the plane-block ordering is point
    Gauss-Seidel: the factor is close to 2.  With shallow rays (n_mu = 4) the
    couplings inside a plane stay Jacobi and the gain is smaller.  Both iterations
    stop near the same S."""
    o = oracle_mod
    shape = (4, 4, 24)
    jac = _stratified(o, shape, 1e-3, n_mu).ali(delta_c=1e-9, max_iter=20000)
    gs = _stratified(o, shape, 1e-3, n_mu).ali_gs(delta_c=1e-9, max_iter=20000)
    assert jac["converged"] and gs["converged"]
    ratio = jac["iters"][0] / gs["iters"][0]
    assert lo <= ratio <= hi, (jac["iters"], gs["iters"])
    assert _rel(gs["S"], jac["S"]) <= 1e-5


def test_fixed_point_satisfies_the_equation(oracle_mod):
    o = oracle_mod
    p = _problem(o, (6, 5, 8), 31, eps_range=(1e-2, 1.0))
    out = p.ali_gs(delta_c=1e-11, max_iter=5000)
    S = out["S"]
    J = p.formal_solve(S, converge_periodic=1e-15, max_sweeps=200)["J"]
    # a second formal solution on the same S converges the lagged periodic ghosts
    resid = np.max(np.abs((1 - p.eps) * J + p.eps * p.B - S) / S)
    assert resid <= 1e-8


def test_lte_is_exact_after_one_iteration(oracle_mod):
    o = oracle_mod
    p = _problem(o, (5, 4, 6), 41, eps_range=(1.0, 1.0))
    out = p.ali_gs(fixed_iters=1, S0=np.full(p.chi.shape, 3.0))
    assert np.max(np.abs(out["S"] - p.B)) <= 1e-15 * np.max(p.B)


def test_unsupported_configurations(oracle_mod):
    o = oracle_mod
    rng = np.random.default_rng(0)
    n = 4 * 4 * 4
    args = ((4, 4, 4), np.ones(n), 0.5, np.ones(n))
    with pytest.raises(ValueError):
        o.Problem(*args, bc_lo=(P_, P_, P_), bc_hi=(P_, P_, P_)).gs_iteration(rng.random(n))
    with pytest.raises(ValueError):
        o.Problem(*args, order=1).gs_iteration(rng.random(n))
    with pytest.raises(ValueError):
        o.Problem(*args, interp=1).gs_iteration(rng.random(n))


# ---- the paper's zone order ------------------------------------------------------------

def _zone_order(shape):
    """Flat cell indices in the backward sweep's update order: planes from the top,
    rows from the back, i descending (the reverse of row-major order)."""
    return list(range(int(np.prod(shape)) - 1, -1, -1))


def _brute_force_zone_iteration(o, p, S, memory):
    """Zone-order Gauss-Seidel by definition: before each zone's update a full formal
    solution with the current S (periodic ghosts from ``memory``) gives its J.  Returns
    S, J and the new periodic memory (rays going up from the solution with the old S,
    rays going down from the one with the new S)."""
    S_cur = S.reshape(p.nf, -1).copy()
    J = np.zeros_like(S_cur)
    eps, B = p.eps.reshape(p.nf, -1), p.B.reshape(p.nf, -1)
    for z in _zone_order(p.n):
        p.seed_periodic(memory)
        out = p.sweep(S_cur)
        Jz, lam = out["J"].reshape(p.nf, -1)[:, z], out["lam"].reshape(p.nf, -1)[:, z]
        J[:, z] = Jz
        S_cur[:, z] += ((1.0 - eps[:, z]) * Jz + eps[:, z] * B[:, z] - S_cur[:, z]) / (1.0 - (1.0 - eps[:, z]) * lam)
    p.seed_periodic(memory)
    p.sweep(S.reshape(p.chi.shape))
    up = [None if a is None else a.copy() for a in p.prev]
    p.seed_periodic(memory)
    p.sweep(S_cur)
    new = [None if a is None else a.copy() for a in p.prev]
    down = p.mu[:, 2] < 0.0
    for q in range(3):
        if new[q] is not None:
            new[q][:, ~down] = up[q][:, ~down]
    return S_cur.reshape(p.chi.shape), J.reshape(p.chi.shape), new


@pytest.mark.parametrize("case", ["periodic", "fixed_faces", "cold"])
def test_zone_iteration_matches_its_definition(oracle_mod, case):
    o = oracle_mod
    if case == "fixed_faces":
        shape, lo, hi = (4, 3, 4), (F_, V_, T_), (T_, F_, V_)
        rng = np.random.default_rng(5)
        fixed = [None] * 6
        fixed[0] = rng.uniform(0, 2, (2, 24, 3 * 4))
        fixed[3] = rng.uniform(0, 2, (2, 24, 4 * 4))
    else:
        shape, lo, hi, fixed = (4, 3, 4), (P_, P_, T_), (P_, P_, V_), None
    p_gs = _problem(o, shape, 13, nf=2, bc_lo=lo, bc_hi=hi, fixed=fixed)
    p_bf = _problem(o, shape, 13, nf=2, bc_lo=lo, bc_hi=hi, fixed=fixed)
    rng = np.random.default_rng(14)
    S = (0.5 + rng.random(p_gs.chi.shape)) * p_gs.B
    if case == "cold":
        memory = _planes_from(o, p_gs, S)
        p_gs.reset_periodic()
    else:
        memory = [None if a is None else rng.uniform(0.5, 2.0, a.shape) for a in p_gs.prev]
        p_gs.seed_periodic(memory)
    out = p_gs.gs_iteration(S, ordering="zone")
    S_bf, J_bf, mem_bf = _brute_force_zone_iteration(o, p_bf, S, memory)
    assert _rel(out["S"], S_bf) <= 1e-13
    assert _rel(out["J"], J_bf) <= 1e-13
    for q in range(3):
        if mem_bf[q] is not None:
            assert _rel(p_gs.prev[q], mem_bf[q]) <= 1e-13


@pytest.mark.parametrize("n_mu", [4, 6])
def test_textbook_point_gauss_seidel_on_the_lambda_matrix(oracle_mod, n_mu):
    """Four iterations against point Gauss-Seidel on the assembled Lambda, the zones
    taken in the reverse of row-major order; shallow rays couple the zones of a plane,
    so this differs from the plane blocks."""
    o = oracle_mod
    shape = (4, 3, 4)
    kw = dict(bc_lo=(T_, V_, T_), bc_hi=(V_, T_, V_), n_mu=n_mu)
    p = _problem(o, shape, 22, **kw)
    A, c = _lambda_matrix(_problem(o, shape, 22, **kw))
    lam = p.sweep(p.B)["lam"].ravel()
    eps, B = p.eps.ravel(), p.B.ravel()
    S = B.copy()
    for _ in range(4):
        for z in _zone_order(shape):
            J = A[z] @ S + c[z]
            S[z] = S[z] + ((1.0 - eps[z]) * J + eps[z] * B[z] - S[z]) / (1.0 - (1.0 - eps[z]) * lam[z])
    out = p.ali_gs(fixed_iters=4, ordering="zone")
    assert _rel(out["S"].ravel(), S) <= 1e-12
    blocks = _problem(o, shape, 22, **kw).ali_gs(fixed_iters=4, ordering="plane")
    assert _rel(blocks["S"].ravel(), S) > 1e-6


@pytest.mark.parametrize("n_mu", [2, 4, 6])
def test_zone_order_halves_the_iterations(oracle_mod, n_mu):
    """Section 3.4 (after TF95): Gauss-Seidel converges nearly twice as fast as Jacobi.
    In the zone order the gain holds for every angle set (measured 1.85-1.86 on this
    atmosphere); the plane blocks keep Jacobi inside a plane and gain 1.40-1.43 with
    the shallow rays of n_mu = 4 and 6.  All three stop near the same S."""
    o = oracle_mod
    shape = (4, 4, 24)
    jac = _stratified(o, shape, 1e-3, n_mu).ali(delta_c=1e-9, max_iter=20000)
    zone = _stratified(o, shape, 1e-3, n_mu).ali_gs(delta_c=1e-9, max_iter=20000, ordering="zone")
    plane = _stratified(o, shape, 1e-3, n_mu).ali_gs(delta_c=1e-9, max_iter=20000, ordering="plane")
    assert jac["converged"] and zone["converged"] and plane["converged"]
    rz = jac["iters"][0] / zone["iters"][0]
    rp = jac["iters"][0] / plane["iters"][0]
    assert 1.75 <= rz <= 2.0, (jac["iters"], zone["iters"])
    if n_mu > 2:
        assert rz > rp + 0.3, (zone["iters"], plane["iters"])
    assert _rel(zone["S"], jac["S"]) <= 1e-5


def test_zone_fixed_point_and_lte(oracle_mod):
    o = oracle_mod
    p = _problem(o, (4, 4, 5), 32, eps_range=(1e-2, 1.0))
    out = p.ali_gs(delta_c=1e-11, max_iter=5000, ordering="zone")
    S = out["S"]
    J = p.formal_solve(S, converge_periodic=1e-15, max_sweeps=200)["J"]
    assert np.max(np.abs((1 - p.eps) * J + p.eps * p.B - S) / S) <= 1e-8
    q = _problem(o, (4, 3, 4), 42, eps_range=(1.0, 1.0))
    out = q.ali_gs(fixed_iters=1, S0=np.full(q.chi.shape, 3.0), ordering="zone")
    assert np.max(np.abs(out["S"] - q.B)) <= 1e-15 * np.max(q.B)
    with pytest.raises(ValueError):
        q.gs_iteration(q.B, ordering="diagonal")
