"""Parity of the HIP path (through the C ABI) with the FP64 oracle on identical seeded
inputs.  FP64 sweeps: max relative error <= 1e-12 on J; FP32 difference-form sweeps:
<= 2e-5 relative on J (the tolerance fixed for the FP32 solver)."""
import numpy as np
import pytest

from paper_1201_2222_amd import workloads as W

pytestmark = pytest.mark.gpu

P, V, T, F = W.PERIODIC, W.VACUUM, W.THERMAL, W.FIXED
TOL64 = 1e-12
TOL32 = 2e-5


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
    """Random incident intensity on every FIXED face ([nf][na][n2][n1])."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = wl.shape
    planes = [ny * nz, ny * nz, nx * nz, nx * nz, nx * ny, nx * ny]
    faces = [None] * 6
    for q in range(3):
        for hi in range(2):
            kind = (wl.bc_hi if hi else wl.bc_lo)[q]
            if kind == F:
                faces[2 * q + hi] = rng.uniform(0.0, 2.0, (wl.nf, wl.na, planes[2 * q + hi]))
    return faces


def _pair(env, oracle_mod, wl, precision, fixed=None, schedule=0):
    rt, torch = env
    o = oracle_mod
    op = o.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, h=wl.h, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi,
                   w_nu=wl.w_nu, fixed=fixed)
    dfix = None if fixed is None else [None if a is None else _dev(torch, a) for a in fixed]
    gp = rt.Problem(wl.shape, nf=wl.nf, h=wl.h, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi,
                    precision=precision, w_nu=wl.w_nu, I_fixed=dfix, schedule=schedule)
    gp._dfix = dfix
    gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    return op, gp


CASES = [
    # shape, n_mu, bc_lo, bc_hi, h, nf
    ((19, 13, 11), 4, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 2),       # several tiles, ragged tails
    ((16, 16, 16), 6, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 1),       # exact tile multiple
    ((5, 3, 7), 4, (V, T, V), (T, V, T), (1.0, 1.0, 1.0), 1),          # smaller than one tile
    ((10, 9, 17), 8, (P, V, T), (P, T, V), (1.3, 0.8, 1.1), 2),        # non-cubic cells, LQ8
    ((12, 1, 20), 2, (P, P, T), (P, P, V), (1.0, 1.0, 1.0), 1),        # degenerate axis, corner rays
    ((9, 11, 10), 4, (F, P, F), (F, P, T), (1.0, 1.0, 1.0), 1),        # fixed incident intensity
    ((9, 9, 9), 6, (P, P, P), (P, P, P), (1.0, 1.0, 1.0), 1),          # all periodic
]


SCHEDULES = {"stages": 1, "persistent": 2}


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("schedule", ["stages", "persistent"])
def test_formal_solve_parity(env, oracle_mod, case, precision, schedule):
    """Two consecutive formal solutions (the second reads the first one's periodic
    memory) on random S; J and Lambda* against the oracle."""
    rt, torch = env
    shape, n_mu, lo, hi, h, nf = CASES[case]
    wl = W.random_problem(shape, nf=nf, seed=100 + case, n_mu=n_mu, bc_lo=lo, bc_hi=hi, h=h)
    fixed = _fixed_faces(wl) if F in lo + hi else None
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec, fixed, schedule=SCHEDULES[schedule])
    rng = np.random.default_rng(7 + case)
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
@pytest.mark.parametrize("schedule", ["stages", "persistent"])
def test_ali_fixed_iterations_parity(env, oracle_mod, precision, schedule):
    """Three Jacobi iterations from S = B on a multi-bin random problem."""
    rt, torch = env
    wl = W.random_problem((17, 10, 12), nf=3, seed=11, n_mu=4, eps_range=(1e-3, 1.0))
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec, schedule=SCHEDULES[schedule])
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
@pytest.mark.parametrize("schedule", ["stages", "persistent"])
def test_ali_converged_parity(env, oracle_mod, precision, schedule):
    """Scattering atmosphere (the 128^3 workload's structure at 24^3, two bins with
    different eps): Jacobi ALI to max|dS/S| <= 1e-6 with per-bin stopping.  FP64 must
    take the same iteration counts and agree to 1e-12; FP32 must agree to 2e-5."""
    rt, torch = env
    base = W.scattering(24, eps=1e-2, tau_bottom=1e3)
    wl2 = W.scattering(24, seed=77, eps=1e-1, tau_bottom=1e3)
    chi = np.concatenate([base.chi, wl2.chi])
    eps = np.concatenate([base.eps, wl2.eps])
    B = np.concatenate([base.B, wl2.B])
    wl = W.Workload("scat2", base.shape, 4, chi, eps, B, np.ones(2), delta_c=1e-6)
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec, schedule=SCHEDULES[schedule])
    ref = op.ali(delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    status, stats = gp.ali_solve(S, J, delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    torch.cuda.synchronize()
    assert status == rt.RT_OK
    it, resid = rt.rt_ali_bin_stats(gp.handle, wl.nf)
    Jg = J.cpu().numpy().reshape(ref["J"].shape)
    if precision == "f64":
        assert list(it) == list(ref["iters"])
        assert _rel(Jg, ref["J"]) <= TOL64
        assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= TOL64
    else:
        assert np.all(np.abs(it - ref["iters"]) <= max(3, 0.02 * ref["iters"].max()))
        assert _rel(Jg, ref["J"]) <= TOL32
    gp.close()


_REF40 = {}


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_ali_converged_parity_40(env, oracle_mod, precision):
    """The scattering atmosphere at 40^3 (48 rays, eps = 0.03, tau_bottom = 1e3; 5^3 tiles in
    13 stages, face planes of 5 x 5 blocks): Jacobi ALI
    to max|dS/S| <= 1e-6 against the oracle's converged solve (about 40 s of CPU, shared
    by both precisions).  FP64: the oracle's iteration count and J, S within 1e-12;
    FP32: within 2% of the count and 2e-5."""
    rt, torch = env
    wl = W.scattering(40, eps=3e-2, tau_bottom=1e3)
    if "ref" not in _REF40:
        op = oracle_mod.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, h=wl.h, bc_lo=wl.bc_lo,
                                bc_hi=wl.bc_hi, w_nu=wl.w_nu)
        _REF40["ref"] = op.ali(delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    ref = _REF40["ref"]
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    gp = rt.Problem(wl.shape, nf=wl.nf, h=wl.h, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=prec,
                    w_nu=wl.w_nu)
    gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    status, stats = gp.ali_solve(S, J, delta_c=1e-6, max_iter=5000, per_bin_stop=True)
    torch.cuda.synchronize()
    assert status == rt.RT_OK
    Jg = J.cpu().numpy().reshape(ref["J"].shape)
    Sg = S.cpu().numpy().reshape(ref["S"].shape)
    if precision == "f64":
        assert stats["iterations"] == int(ref["iters"][0])
        assert _rel(Jg, ref["J"]) <= TOL64 and _rel(Sg, ref["S"]) <= TOL64
    else:
        assert abs(stats["iterations"] - int(ref["iters"][0])) <= max(3, 0.02 * int(ref["iters"][0]))
        assert _rel(Jg, ref["J"]) <= TOL32 and _rel(Sg, ref["S"]) <= TOL32
    gp.close()


def test_workload_plain_full_size(env, oracle_mod):
    """The 32^3 grey LTE workload (24 rays, FP64): one formal solution plus a second
    with warm periodic memory, full size."""
    rt, torch = env
    wl = W.plain()
    op, gp = _pair(env, oracle_mod, wl, rt.RT_F64)
    n = wl.chi.size
    for _ in range(2):
        ref = op.sweep(wl.B)
        J = torch.empty(n, dtype=torch.float64, device="cuda")
        gp.formal_solve(_dev(torch, wl.B), J)
        torch.cuda.synchronize()
        assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= TOL64
    gp.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("schedule", ["stages", "persistent"])
def test_workload_scattering_full_size(env, oracle_mod, precision, schedule):
    """The 128^3 scattering workload at full size, in the launch configurations the
    benchmark times: two Jacobi iterations from S = B against the oracle."""
    rt, torch = env
    wl = W.scattering()
    prec = rt.RT_F64 if precision == "f64" else rt.RT_F32
    op, gp = _pair(env, oracle_mod, wl, prec, schedule=SCHEDULES[schedule])
    ref = op.ali(fixed_iters=2)
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    gp.ali_solve(S, J, fixed_iters=2)
    torch.cuda.synchronize()
    tol = TOL64 if precision == "f64" else TOL32
    assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= tol
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= tol
    gp.close()
