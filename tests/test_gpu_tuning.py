"""Every wave count of the sweep workgroup (fewer waves than rays: each wave runs several
rays) keeps parity with the oracle, also with the persistent schedule (whose grid follows
the wave count), and the autotuner picks one of them without disturbing the next solve."""
import numpy as np
import pytest

from paper_1201_2222_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1201_2222_amd as rt
    assert torch.cuda.is_available(), "GPU tests need a device"
    rt.load()
    return rt, torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _problem(env, wl, prec, **kw):
    rt, torch = env
    gp = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=prec, **kw)
    gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    return gp


@pytest.mark.parametrize("waves", [1, 2, 4, 6])
@pytest.mark.parametrize("variant", ["f64", "f32", "bezier32", "gs64", "persistent32"])
def test_wave_counts_keep_parity(env, oracle_mod, waves, variant):
    rt, torch = env
    wl = W.random_problem((19, 17, 12), nf=2, seed=1300, n_mu=6, eps_range=(1e-2, 1.0))
    order = 1 if variant == "bezier32" else 0
    prec = rt.RT_F64 if variant in ("f64", "gs64") else rt.RT_F32
    gs = variant == "gs64"
    sched = rt.RT_SCHED_PERSISTENT if variant == "persistent32" else rt.RT_SCHED_STAGES
    op = oracle_mod.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, order=order)
    ref = op.ali_gs(fixed_iters=3) if gs else op.ali(fixed_iters=3)
    gp = _problem(env, wl, prec, order=order, schedule=sched)
    gp.set_waves(waves)
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    (gp.ali_solve_gs if gs else gp.ali_solve)(S, J, fixed_iters=3)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == rt.RT_F64 else 2e-5
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= tol
    assert _rel(J.cpu().numpy().reshape(ref["J"].shape), ref["J"]) <= tol
    gp.close()


@pytest.mark.parametrize("schedule", ["stages", "persistent"])
def test_tune_picks_a_count_and_leaves_the_solve_alone(env, oracle_mod, schedule):
    rt, torch = env
    wl = W.random_problem((24, 20, 16), nf=1, seed=1310, n_mu=6, eps_range=(1e-2, 1.0))
    op = oracle_mod.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi)
    ref = op.ali(fixed_iters=4)
    gp = _problem(env, wl, rt.RT_F32,
                  schedule=rt.RT_SCHED_PERSISTENT if schedule == "persistent" else rt.RT_SCHED_STAGES)
    best, ms = gp.tune(_dev(torch, wl.B), reps=2)     # cold problem: stays cold
    assert 1 <= best <= 6 and set(ms) == {1, 2, 3, 4, 5, 6}
    assert ms[best] == min(ms.values())
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    gp.ali_solve(S, J, fixed_iters=4)
    torch.cuda.synchronize()
    assert _rel(S.cpu().numpy().reshape(ref["S"].shape), ref["S"]) <= 2e-5
    gp.close()


def test_autotune_cache(env, tmp_path):
    rt, torch = env
    from paper_1201_2222_amd import tuning
    wl = W.random_problem((16, 16, 16), nf=1, seed=1320, n_mu=4)
    path = str(tmp_path / "tune.json")
    gp = _problem(env, wl, rt.RT_F32)
    e = tuning.autotune(gp, _dev(torch, wl.B), path=path, reps=1)
    gp2 = _problem(env, wl, rt.RT_F32)
    e2 = tuning.autotune(gp2, _dev(torch, wl.B), path=path)
    assert e2["waves"] == e["waves"]
    gp.close()
    gp2.close()


def test_invalid_wave_counts(env):
    rt, torch = env
    wl = W.random_problem((8, 8, 8), nf=1, seed=1330, n_mu=4)
    gp = _problem(env, wl, rt.RT_F64)
    for w in (0, 4, 11):        # LQ4: 3 rays per octant
        with pytest.raises(rt.RtError):
            gp.set_waves(w)
    gp.close()
    gq = _problem(env, wl, rt.RT_F32, interp=rt.RT_INTERP_QUADRATIC)
    with pytest.raises(rt.RtError):
        gq.set_waves(1)
    gq.close()
