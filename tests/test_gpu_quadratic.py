"""Parity of the plane-ordered sweep with monotone quadratic interpolation of the
upwind intensity (section 3.3) on the HIP path with the FP64 oracle's quadratic sweep
on identical seeded inputs: FP64 within 1e-12 relative on J, FP32 difference form
within 2e-5; Lambda* (unchanged, sum of w psi0) within 1e-13."""
import numpy as np
import pytest

from paper_1201_2222_amd import workloads as W

pytestmark = pytest.mark.gpu

P, V, T, F = W.PERIODIC, W.VACUUM, W.THERMAL, W.FIXED
TOL64 = 1e-12
TOL32 = 2e-5
_REF = {}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1201_2222_amd as rt
    assert torch.cuda.is_available(), "GPU tests need a device"
    rt.load()
    return rt, torch


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _fixed_faces(wl, seed=3):
    rng = np.random.default_rng(seed)
    nx, ny, nz = wl.shape
    planes = [ny * nz, ny * nz, nx * nz, nx * nz, nx * ny, nx * ny]
    faces = [None] * 6
    for q in range(3):
        for hi in range(2):
            if (wl.bc_hi if hi else wl.bc_lo)[q] == F:
                faces[2 * q + hi] = rng.uniform(0.0, 2.0, (wl.nf, wl.na, planes[2 * q + hi]))
    return faces


def _pair(env, oracle_mod, wl, precision, fixed=None, mu=None, w=None):
    rt, torch = env
    op = oracle_mod.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, mu=mu, w=w, h=wl.h, bc_lo=wl.bc_lo,
                            bc_hi=wl.bc_hi, w_nu=wl.w_nu, fixed=fixed, interp=1)
    dfix = None if fixed is None else [None if a is None else _dev(torch, a) for a in fixed]
    gp = rt.Problem(wl.shape, nf=wl.nf, h=wl.h, n_mu=wl.n_mu, mu=mu, w=w, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi,
                    precision=precision, w_nu=wl.w_nu, I_fixed=dfix, interp=rt.RT_INTERP_QUADRATIC)
    gp._dfix = dfix
    gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    return op, gp


CASES = [
    # shape, n_mu, bc_lo, bc_hi, h, nf
    ((19, 13, 11), 4, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 2),       # ragged in-plane tiles
    ((32, 16, 17), 6, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 1),       # two tiles along x, one along y
    ((5, 3, 7), 4, (V, T, V), (T, V, T), (1.0, 1.0, 1.0), 1),          # smaller than one tile, no periodic axis
    ((10, 9, 17), 8, (P, V, T), (P, T, V), (1.3, 0.8, 1.1), 2),        # non-cubic cells, LQ8, mixed faces
    ((12, 1, 20), 2, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 1),        # degenerate axis
    ((9, 11, 10), 4, (F, P, F), (F, P, T), (1.0, 1.0, 1.0), 1),        # fixed incident intensity
    ((9, 9, 9), 6, (P, P, P), (P, P, P), (1.0, 1.0, 1.0), 1),          # all periodic
    ((18, 17, 20), 10, (V, V, T), (V, V, V), (1.0, 1.0, 1.0), 1),      # closed box, many rays per class
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_quadratic_formal_solve_parity(env, oracle_mod, case, precision):
    """Two consecutive formal solutions (the second reads the first one's last planes
    on periodic axes) on random S; J and Lambda* against the oracle."""
    rt, torch = env
    shape, n_mu, lo, hi, h, nf = CASES[case]
    wl = W.random_problem(shape, nf=nf, seed=700 + case, n_mu=n_mu, bc_lo=lo, bc_hi=hi, h=h)
    fixed = _fixed_faces(wl) if F in lo + hi else None
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec, fixed)
    rng = np.random.default_rng(27 + case)
    tol = TOL64 if precision == "f64" else TOL32
    n = wl.chi.size
    for sweep in range(2):
        S = (0.5 + rng.random(wl.chi.shape)) * wl.B
        ref = op.sweep(S)
        J = torch.empty(n, dtype=torch.float64, device="cuda")
        lam = torch.empty(n, dtype=torch.float64, device="cuda")
        gp.formal_solve(_dev(torch, S), J, lam)
        torch.cuda.synchronize()
        Jg = J.cpu().numpy().reshape(ref["J"].shape)
        assert _rel(Jg, ref["J"]) <= tol, (sweep, _rel(Jg, ref["J"]))
        assert _rel(lam.cpu().numpy().reshape(ref["lam"].shape), ref["lam"]) <= 1e-13
    gp.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_quadratic_advected_beam(env, oracle_mod, precision):
    """chi = S = 0 with a sinusoidal incident intensity on the bottom face and periodic
    x, y (the advection case of the oracle's pins): the GPU sweep follows the oracle
    sweep by sweep while the lagged planes catch up."""
    rt, torch = env
    N = 24
    n = N ** 3
    mu, w = oracle_mod.quadrature(4)
    X, Y = np.meshgrid(np.arange(N), np.arange(N))
    I0 = 1.0 + 0.5 * np.sin(2 * np.pi * X / N + 0.3) * np.cos(2 * np.pi * Y / N)
    bottom = np.zeros((1, len(w), N * N))
    bottom[0, :] = I0.ravel()
    top = np.zeros((1, len(w), N * N))
    wl = W.Workload("beam", (N, N, N), 4, np.zeros((1, N, N, N)), np.ones((1, N, N, N)), np.zeros((1, N, N, N)),
                    np.ones(1), bc_lo=(P, P, F), bc_hi=(P, P, F), h=(1.0, 1.0, 1.0))
    fixed = [None, None, None, None, bottom, top]
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec, fixed, mu=mu, w=w)
    S = np.zeros(n)
    for sweep in range(6):
        ref = op.sweep(S)
        J = torch.empty(n, dtype=torch.float64, device="cuda")
        gp.formal_solve(_dev(torch, S), J)
        torch.cuda.synchronize()
        Jg = J.cpu().numpy().reshape(ref["J"].shape)
        # J vanishes nowhere here (every upward ray carries I0 >= 0.5)
        assert _rel(Jg, ref["J"]) <= (TOL64 if precision == "f64" else TOL32), sweep
    gp.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_quadratic_ali_fixed_iterations_parity(env, oracle_mod, precision):
    rt, torch = env
    wl = W.random_problem((17, 10, 12), nf=3, seed=711, n_mu=4, eps_range=(1e-3, 1.0))
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec)
    ref = op.ali(fixed_iters=3)
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    st, stats = gp.ali_solve(S, J, fixed_iters=3)
    torch.cuda.synchronize()
    tol = TOL64 if precision == "f64" else TOL32
    assert stats["iterations"] == 3
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= tol
    assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= tol
    gp.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_quadratic_ali_converged_parity(env, oracle_mod, precision):
    """The scattering atmosphere at 24^3 to max|dS/S| <= 1e-6: FP64 takes the oracle's
    iteration count and agrees to 1e-12; FP32 agrees to 2e-5."""
    rt, torch = env
    wl = W.scattering(24, eps=1e-2, tau_bottom=1e3)
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec)
    if "scattering24" not in _REF:
        _REF["scattering24"] = op.ali(delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    ref = _REF["scattering24"]
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    status, stats = gp.ali_solve(S, J, delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    torch.cuda.synchronize()
    assert status == rt.RT_OK
    it, _ = rt.rt_ali_bin_stats(gp.handle, wl.nf)
    Jg = J.cpu().numpy().reshape(ref["J"].shape)
    if precision == "f64":
        assert list(it) == list(ref["iters"])
        assert _rel(Jg, ref["J"]) <= TOL64
        assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= TOL64
    else:
        assert np.all(np.abs(it - ref["iters"]) <= max(3, 0.02 * ref["iters"].max()))
        assert _rel(Jg, ref["J"]) <= TOL32
    gp.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_quadratic_workload_scattering_full_size(env, oracle_mod, precision):
    """The 128^3 scattering workload at full size with the quadratic upwind intensity,
    in the launch configuration the benchmark times: two Jacobi iterations from S = B."""
    rt, torch = env
    wl = W.scattering()
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec)
    if "full" not in _REF:   # the oracle's two sweeps (~25 s) serve both precisions
        _REF["full"] = op.ali(fixed_iters=2)
    ref = _REF["full"]
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    gp.ali_solve(S, J, fixed_iters=2)
    torch.cuda.synchronize()
    tol = TOL64 if precision == "f64" else TOL32
    assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= tol
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= tol
    gp.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_quadratic_moments_parity(env, oracle_mod, precision):
    """The moments epilogue on the quadratic sweep: per-bin J, H, K and the frequency-
    integrated J, H, K, f, Q and heating against the oracle's moments with the same
    upwind interpolation (two bins, fixed faces, non-cubic cells)."""
    rt, torch = env
    wl = W.random_problem((15, 12, 11), nf=2, seed=730, n_mu=4, bc_lo=(P, F, T), bc_hi=(P, V, V),
                          h=(1.2, 0.9, 1.0))
    fixed = _fixed_faces(wl)
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec, fixed)
    rng = np.random.default_rng(731)
    S = (0.5 + rng.random(wl.chi.shape)) * wl.B
    ref = op.moments(S)
    n = wl.chi.size
    c = n // wl.nf
    out = {k: torch.empty(m, dtype=torch.float64, device="cuda")
           for k, m in (("J", n), ("H", 3 * n), ("K", 6 * n), ("J_int", c), ("H_int", 3 * c), ("K_int", 6 * c),
                        ("f_int", 6 * c), ("Q_int", c))}
    heat = gp.moments(_dev(torch, S), want_heating=True, **out)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    tol = TOL64 if precision == "f64" else TOL32
    Jref = ref["J"]
    scale = np.max(np.abs(Jref))
    assert _rel(g["J"].reshape(Jref.shape), Jref) <= tol
    # H and K carry no scale of their own: compared against that of J
    assert np.max(np.abs(g["H"].reshape(ref["H"].shape) - ref["H"])) <= tol * scale
    assert np.max(np.abs(g["K"].reshape(ref["K"].shape) - ref["K"])) <= tol * scale
    Jint = ref["J_int"]
    assert _rel(g["J_int"].reshape(Jint.shape), Jint) <= 2 * tol
    iscale = np.max(np.abs(Jint))
    assert np.max(np.abs(g["H_int"].reshape(ref["H_int"].shape) - ref["H_int"])) <= 2 * tol * iscale
    assert np.max(np.abs(g["K_int"].reshape(ref["K_int"].shape) - ref["K_int"])) <= 2 * tol * iscale
    assert np.max(np.abs(g["f_int"].reshape(ref["f_int"].shape) - ref["f_int"])) <= 6 * tol
    h = wl.h
    qtol = 4 * np.pi * tol * scale * np.sum(np.abs(wl.w_nu)) * (np.max(wl.chi) + 6.0 / min(h)) * 2
    assert np.max(np.abs(g["Q_int"].reshape(ref["Q_int"].shape) - ref["Q_int"])) <= qtol
    assert abs(heat - ref["heating"]) <= qtol * c * h[0] * h[1] * h[2]
    gp.close()


def test_quadratic_in_a_batch_equals_its_single_solve(env):
    """A plane-ordered problem in a batch with tile-wavefront problems (it runs its own
    launches within the batch's iterations) gives bitwise its single solve; so do the
    others."""
    rt, torch = env
    specs = [((14, 12, 10), 4, rt.RT_INTERP_QUADRATIC, rt.RT_F32, 740),
             ((12, 10, 9), 4, rt.RT_INTERP_BILINEAR, rt.RT_F32, 741),
             ((10, 9, 8), 6, rt.RT_INTERP_QUADRATIC, rt.RT_F64, 742)]
    probs, single = [], []
    for shape, n_mu, interp, prec, seed in specs:
        wl = W.random_problem(shape, nf=2, seed=seed, n_mu=n_mu, eps_range=(1e-2, 1.0))
        out = []
        for _ in range(2):
            gp = rt.Problem(wl.shape, nf=2, n_mu=n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=prec, interp=interp)
            gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
            S = torch.empty(wl.chi.size, dtype=torch.float64, device="cuda")
            J = torch.empty_like(S)
            out.append((gp, S, J))
        probs.append(out[0])
        gp, S, J = out[1]
        gp.ali_solve(S, J, delta_c=1e-7, max_iter=2000)
        torch.cuda.synchronize()
        single.append((S.cpu().numpy(), J.cpu().numpy()))
        gp.close()
    status, per, stats = rt.rt_ali_solve_batch([p[0].handle for p in probs], [p[1] for p in probs],
                                               [p[2] for p in probs], delta_c=1e-7, max_iter=2000)
    torch.cuda.synchronize()
    assert status == rt.RT_OK
    for (gp, S, J), (S1, J1) in zip(probs, single):
        assert np.array_equal(S.cpu().numpy(), S1)
        assert np.array_equal(J.cpu().numpy(), J1)
        gp.close()


@pytest.mark.parametrize("interp", [0, 1])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_crossing_beams(env, oracle_mod, interp, precision):
    """Two narrow beams crossing in vacuum (the oracle's crossing-beam pin): the GPU
    sweep with either upwind interpolation follows the oracle (compared against the
    beam's peak: J vanishes in most of the box)."""
    rt, torch = env
    N = 32
    d = np.array([0.5, 0.45, 0.74])
    d /= np.linalg.norm(d)
    mu = np.array([[sx * d[0], sy * d[1], sz * d[2]] for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)])
    w = np.full(8, 1.0 / 8.0)
    fxl = np.zeros((1, 8, N * N))
    fxh = np.zeros((1, 8, N * N))
    fxl[0, 0, 3 * N + 4] = 1.0
    fxh[0, 1, 3 * N + 4] = 1.0
    fixed = [fxl, fxh, None, None, None, None]
    n = N ** 3
    op = oracle_mod.Problem((N, N, N), np.zeros(n), 1.0, np.zeros(n), mu=mu, w=w, interp=interp,
                            bc_lo=(F, V, V), bc_hi=(F, V, V), fixed=fixed)
    ref = op.sweep(np.zeros(n))["J"][0]
    dfix = [None if a is None else _dev(torch, a) for a in fixed]
    gp = rt.Problem((N, N, N), nf=1, mu=mu, w=w, bc_lo=(F, V, V), bc_hi=(F, V, V), I_fixed=dfix,
                    precision=rt.RT_F64 if precision == "f64" else rt.RT_F32,
                    interp=rt.RT_INTERP_QUADRATIC if interp else rt.RT_INTERP_BILINEAR)
    z = _dev(torch, np.zeros(n))
    gp.set_fields(_dev(torch, np.full(n, 1e-30)), _dev(torch, np.ones(n)), z)
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    gp.formal_solve(z, J)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy().reshape(ref.shape)
    tol = TOL64 if precision == "f64" else TOL32
    assert np.max(np.abs(Jg - ref)) <= tol * np.max(ref)
    gp.close()


def test_quadratic_through_the_server(env):
    """A plane-ordered request and a tile-wavefront request through the serving loop
    give their single solves bitwise."""
    import time
    rt, torch = env
    srv = rt.rt_server_create(1 << 32, check_every=8)
    jobs = []
    for shape, interp, seed in (((13, 11, 9), rt.RT_INTERP_QUADRATIC, 750), ((12, 12, 8), rt.RT_INTERP_BILINEAR, 751)):
        wl = W.random_problem(shape, nf=1, seed=seed, n_mu=4, eps_range=(1e-2, 1.0))
        ref = rt.Problem(wl.shape, nf=1, n_mu=4, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F32, interp=interp)
        ref.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
        S1 = torch.empty(wl.chi.size, dtype=torch.float64, device="cuda")
        J1 = torch.empty_like(S1)
        ref.ali_solve(S1, J1, delta_c=1e-7, max_iter=2000)
        torch.cuda.synchronize()
        gp = rt.Problem(wl.shape, nf=1, n_mu=4, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F32, interp=interp)
        gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
        torch.cuda.synchronize()
        S = torch.empty_like(S1)
        J = torch.empty_like(S1)
        t = rt.rt_server_submit(srv, gp.handle, S, J, delta_c=1e-7, max_iter=2000)
        jobs.append((t, gp, ref, S, J, S1.cpu().numpy(), J1.cpu().numpy()))
    for t, gp, ref, S, J, S1, J1 in jobs:
        t0 = time.time()
        r = None
        while r is None and time.time() - t0 < 120:
            r = rt.rt_server_poll(srv, t)
            if r is None:
                time.sleep(0.01)
        assert r is not None and r[0] == rt.RT_OK
        torch.cuda.synchronize()
        assert np.array_equal(S.cpu().numpy(), S1)
        assert np.array_equal(J.cpu().numpy(), J1)
        rt.rt_server_release(srv, t)
        gp.close()
        ref.close()
    rt.rt_server_destroy(srv)
