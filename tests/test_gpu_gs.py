"""Parity of the Gauss-Seidel ALI (section 3.4, horizontal planes from the top down as
the blocks) on the HIP path with the FP64 oracle's Gauss-Seidel iteration on identical
seeded inputs: FP64 within 1e-12 relative on S and J, FP32 difference form within
2e-5."""
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


def _pair(env, oracle_mod, wl, precision, fixed=None):
    rt, torch = env
    op = oracle_mod.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, h=wl.h, bc_lo=wl.bc_lo,
                            bc_hi=wl.bc_hi, w_nu=wl.w_nu, fixed=fixed)
    dfix = None if fixed is None else [None if a is None else _dev(torch, a) for a in fixed]
    gp = rt.Problem(wl.shape, nf=wl.nf, h=wl.h, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi,
                    precision=precision, w_nu=wl.w_nu, I_fixed=dfix)
    gp._dfix = dfix
    gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    return op, gp


CASES = [
    # shape, n_mu, bc_lo, bc_hi, h, nf
    ((19, 13, 11), 4, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 2),       # ragged tiles
    ((32, 16, 17), 6, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 1),       # LQ6: shallow rays along x and y
    ((5, 3, 7), 4, (V, T, V), (T, V, T), (1.0, 1.0, 1.0), 1),          # smaller than a tile, no periodic axis
    ((10, 9, 17), 8, (P, V, T), (P, T, V), (1.3, 0.8, 1.1), 2),        # non-cubic cells, LQ8, mixed faces
    ((12, 1, 20), 2, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 1),        # every ray steep, degenerate y
    ((9, 11, 10), 4, (F, P, F), (F, P, F), (1.0, 1.0, 1.0), 1),        # fixed incident intensity, top too
    ((70, 65, 9), 4, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 1),        # chains of two vertices per lane
    ((130, 20, 6), 4, (P, V, T), (P, V, V), (1.0, 1.0, 1.0), 1),       # chains of four vertices per lane
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gs_fixed_iterations_parity(env, oracle_mod, case, precision):
    """Three Gauss-Seidel iterations from S = B (the second and third read the periodic
    memory the first wrote): S and J against the oracle."""
    rt, torch = env
    shape, n_mu, lo, hi, h, nf = CASES[case]
    wl = W.random_problem(shape, nf=nf, seed=900 + case, n_mu=n_mu, bc_lo=lo, bc_hi=hi, h=h,
                          eps_range=(1e-3, 1.0))
    fixed = _fixed_faces(wl) if F in lo + hi else None
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec, fixed)
    ref = op.ali_gs(fixed_iters=3)
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    st, stats = gp.ali_solve_gs(S, J, fixed_iters=3)
    torch.cuda.synchronize()
    tol = TOL64 if precision == "f64" else TOL32
    assert stats["iterations"] == 3
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= tol
    assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= tol
    gp.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gs_converged_parity(env, oracle_mod, precision):
    """The scattering atmosphere at 24^3 to max|dS/S| <= 1e-6: FP64 takes the oracle's
    iteration count and agrees to 1e-12; FP32 agrees to 2e-5."""
    rt, torch = env
    wl = W.scattering(24, eps=1e-2, tau_bottom=1e3)
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec)
    if "scattering24" not in _REF:
        _REF["scattering24"] = op.ali_gs(delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    ref = _REF["scattering24"]
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    status, stats = gp.ali_solve_gs(S, J, delta_c=1e-6, max_iter=5000, per_bin_stop=True)
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
def test_gs_workload_scattering_full_size(env, oracle_mod, precision):
    """The 128^3 scattering workload at full size: two Gauss-Seidel iterations from S = B."""
    rt, torch = env
    wl = W.scattering()
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec)
    if "full" not in _REF:   # the oracle's two iterations serve both precisions
        _REF["full"] = op.ali_gs(fixed_iters=2)
    ref = _REF["full"]
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    gp.ali_solve_gs(S, J, fixed_iters=2)
    torch.cuda.synchronize()
    tol = TOL64 if precision == "f64" else TOL32
    assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= tol
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= tol
    gp.close()


def test_gs_then_jacobi_share_the_periodic_memory(env, oracle_mod):
    """A Jacobi solve after a Gauss-Seidel solve on the same problem reads the periodic
    memory the Gauss-Seidel iterations wrote (warm start from S): the oracle does the same."""
    rt, torch = env
    wl = W.random_problem((14, 12, 10), nf=1, seed=950, n_mu=4, eps_range=(1e-2, 1.0))
    op, gp = _pair(env, oracle_mod, wl, rt.RT_F64)
    ref_gs = op.ali_gs(fixed_iters=2)
    ref = op.ali(fixed_iters=2, S0=ref_gs["S"])
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    gp.ali_solve_gs(S, J, fixed_iters=2)
    gp.ali_solve(S, J, fixed_iters=2, warm_start=1)
    torch.cuda.synchronize()
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= TOL64
    assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= TOL64
    gp.close()


def test_gs_unsupported_configurations(env):
    """Periodic z, second-order segments and the quadratic upwind intensity are refused
    before any work."""
    rt, torch = env
    for kw in (dict(bc_lo=(P, P, P), bc_hi=(P, P, P)), dict(order=rt.RT_SC_BEZIER),
               dict(interp=rt.RT_INTERP_QUADRATIC)):
        wl = W.random_problem((8, 8, 8), nf=1, seed=960, n_mu=4)
        gp = rt.Problem(wl.shape, nf=1, n_mu=4, **({"bc_lo": wl.bc_lo, "bc_hi": wl.bc_hi} | kw))
        gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
        S = _dev(torch, wl.B)
        J = torch.empty_like(S)
        with pytest.raises(rt.RtError):
            gp.ali_solve_gs(S, J, fixed_iters=1)
        gp.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gs_bins_stop_at_different_iterations(env, oracle_mod, precision):
    """Two bins of very different eps converge after different numbers of iterations:
    the first one frozen stays untouched while the other goes on (every Gauss-Seidel
    kernel skips frozen bins), as in the oracle."""
    rt, torch = env
    wl = W.scattering(20, eps=1e-2, tau_bottom=1e3)
    chi = np.concatenate([wl.chi, wl.chi * 0.5])
    eps = np.concatenate([np.full_like(wl.eps, 0.3), np.full_like(wl.eps, 3e-3)])
    B = np.concatenate([wl.B, wl.B * 1.3])
    wl2 = W.Workload("two-bin", wl.shape, wl.n_mu, chi, eps, B, np.array([1.0, 0.5]), bc_lo=wl.bc_lo,
                     bc_hi=wl.bc_hi, h=wl.h)
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl2, prec)
    ref = op.ali_gs(delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    assert ref["iters"][0] < ref["iters"][1] // 2
    n = wl2.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    status, stats = gp.ali_solve_gs(S, J, delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    torch.cuda.synchronize()
    assert status == rt.RT_OK
    it, _ = rt.rt_ali_bin_stats(gp.handle, wl2.nf)
    tol = TOL64 if precision == "f64" else TOL32
    if precision == "f64":
        assert list(it) == list(ref["iters"])
    else:
        assert np.all(np.abs(it - ref["iters"]) <= np.maximum(3, 0.02 * ref["iters"]))
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= tol
    assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= tol
    gp.close()


def test_gs_chain_launch_timing(env):
    """rt_problem_profile times the chain launches of steps 1 .. nz-1 in the first
    iteration of every check interval (the benchmark's roofline for Gauss-Seidel); the
    counts follow the rays crossing an x or y face first, and timing leaves the results
    as they are."""
    rt, torch = env
    wl = W.random_problem((20, 14, 12), nf=2, seed=1600, n_mu=4)
    mu, _ = rt.rt_quadrature(4)
    shallow = int(np.sum((mu[:, 2] < 0) & (np.argmax(np.abs(mu), axis=1) != 2)))
    assert shallow == 8
    out = []
    for prof in (False, True):
        gp = rt.Problem(wl.shape, nf=wl.nf, n_mu=4, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F32)
        gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
        gp.use_graphs(False)
        rt.rt_problem_profile(gp.handle, prof)
        S = torch.empty(wl.chi.size, dtype=torch.float64, device="cuda")
        J = torch.empty_like(S)
        gp.ali_solve_gs(S, J, fixed_iters=8, check_every=4)
        torch.cuda.synchronize()
        p = rt.rt_problem_profile_read(gp.handle)
        nz = wl.shape[2]
        if prof:
            assert p["chain_launches"] == 2 * (nz - 1)
            assert p["chain_updates"] == 2 * (nz - 1) * shallow * 20 * 14 * wl.nf
            assert p["chain_ms"] > 0.0
        else:
            assert p["chain_launches"] == 0 and p["chain_ms"] == 0.0
        out.append((S.cpu().numpy(), J.cpu().numpy()))
        gp.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
