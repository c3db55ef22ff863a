"""Batched ALI (rt_ali_solve_batch) through the C ABI: every problem of an uneven batch
(grids, rays, bins, boundaries and precisions all differ) must give exactly what
rt_ali_solve gives for it alone, and problems must retire independently.  The same
holds when the members use the persistent schedule: then each batch class sweeps all
of its members in one launch per formal solution."""
import numpy as np
import pytest

from paper_1201_2222_amd import workloads as W

pytestmark = pytest.mark.gpu

P, V, T = W.PERIODIC, W.VACUUM, W.THERMAL


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1201_2222_amd as rt
    assert torch.cuda.is_available()
    rt.load()
    return rt, torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


# shape, nf, n_mu, bc_lo, bc_hi, precision, eps_range
BATCH = [
    ((19, 13, 11), 2, 4, (P, P, T), (P, P, V), "f32", (1e-2, 1.0)),
    ((16, 16, 16), 1, 6, (P, P, T), (P, P, V), "f32", (1e-3, 1e-1)),
    ((5, 3, 7), 1, 4, (V, T, V), (T, V, T), "f32", (0.1, 1.0)),
    ((12, 9, 20), 3, 2, (P, V, T), (P, T, V), "f64", (1e-2, 1.0)),
    ((9, 9, 9), 1, 6, (P, P, P), (P, P, P), "f64", (0.05, 0.5)),
    ((24, 10, 8), 2, 4, (P, P, T), (P, P, V), "f32", (0.3, 1.0)),
]


def _make(rt, torch, k, spec, schedule=0):
    shape, nf, n_mu, lo, hi, prec, er = spec
    wl = W.random_problem(shape, nf=nf, seed=500 + k, n_mu=n_mu, bc_lo=lo, bc_hi=hi, eps_range=er)
    p = rt.Problem(shape, nf=nf, n_mu=n_mu, bc_lo=lo, bc_hi=hi, w_nu=wl.w_nu,
                   precision=rt.RT_F32 if prec == "f32" else rt.RT_F64, schedule=schedule)
    p.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    return wl, p, S, J


def _run_both(env, schedules=None, **opts):
    rt, torch = env
    schedules = schedules or [0] * len(BATCH)
    batch = [_make(rt, torch, k, spec, sc) for k, (spec, sc) in enumerate(zip(BATCH, schedules))]
    status, res, stats = rt.rt_ali_solve_batch([b[1].handle for b in batch], [b[2] for b in batch],
                                               [b[3] for b in batch], **opts)
    torch.cuda.synchronize()
    alone = []
    for k, (spec, sc) in enumerate(zip(BATCH, schedules)):
        _, p, S, J = _make(rt, torch, k, spec, sc)
        st, sd = p.ali_solve(S, J, **opts)
        torch.cuda.synchronize()
        alone.append((st, sd, S.cpu().numpy(), J.cpu().numpy(), rt.rt_ali_bin_stats(p.handle, p.desc.nf)[0]))
        p.close()
    return batch, status, res, stats, alone


def test_batch_fixed_iterations_equal_single(env):
    rt, torch = env
    batch, status, res, stats, alone = _run_both(env, fixed_iters=3)
    assert status == rt.RT_OK and all(r == rt.RT_OK for r in res)
    for (wl, p, S, J), st, (_, sd, Sa, Ja, _) in zip(batch, stats, alone):
        assert st["iterations"] == 3 == sd["iterations"]
        assert np.array_equal(S.cpu().numpy(), Sa)
        assert np.array_equal(J.cpu().numpy(), Ja)
        p.close()


def test_batch_converged_equal_single_and_retire(env):
    """Per-bin stopping: each problem (and bin) takes the iteration count it takes alone;
    problems with fewer iterations leave the batch earlier."""
    rt, torch = env
    batch, status, res, stats, alone = _run_both(env, delta_c=1e-6, max_iter=3000, per_bin_stop=True,
                                                 check_every=8)
    assert status == rt.RT_OK
    iters = []
    for (wl, p, S, J), st, (sa, sd, Sa, Ja, ita) in zip(batch, stats, alone):
        assert sa == rt.RT_OK
        itb = rt.rt_ali_bin_stats(p.handle, p.desc.nf)[0]
        assert list(itb) == list(ita)
        assert st["iterations"] == sd["iterations"]
        assert np.array_equal(S.cpu().numpy(), Sa)
        assert np.array_equal(J.cpu().numpy(), Ja)
        iters.append(st["iterations"])
        p.close()
    # retirement at the check after convergence: fewer iterations never retire later
    order = np.argsort(iters)
    secs = [stats[i]["seconds"] for i in order]
    assert all(secs[i] <= secs[i + 1] + 1e-9 for i in range(len(secs) - 1))
    assert len(set(iters)) > 1


def test_persistent_batch_fixed_iterations_equal_single(env):
    """Every member with the persistent schedule: one launch per formal solution of each
    class (FP32 and FP64), each member bitwise equal to its persistent solve alone."""
    rt, torch = env
    sched = [rt.RT_SCHED_PERSISTENT] * len(BATCH)
    batch, status, res, stats, alone = _run_both(env, schedules=sched, fixed_iters=4)
    assert status == rt.RT_OK and all(r == rt.RT_OK for r in res)
    for (wl, p, S, J), st, (_, sd, Sa, Ja, _) in zip(batch, stats, alone):
        assert st["iterations"] == 4 == sd["iterations"]
        assert np.array_equal(S.cpu().numpy(), Sa)
        assert np.array_equal(J.cpu().numpy(), Ja)
        p.close()


def test_persistent_batch_converged_mixed_schedules(env):
    """Members of both schedules in one batch, to convergence with per-bin stopping:
    bins freeze and members retire while the persistent classes keep sweeping the rest."""
    rt, torch = env
    sched = [rt.RT_SCHED_PERSISTENT if k % 2 == 0 else rt.RT_SCHED_STAGES for k in range(len(BATCH))]
    batch, status, res, stats, alone = _run_both(env, schedules=sched, delta_c=1e-6, max_iter=3000,
                                                 per_bin_stop=True, check_every=8)
    assert status == rt.RT_OK
    for (wl, p, S, J), st, (sa, sd, Sa, Ja, ita) in zip(batch, stats, alone):
        assert sa == rt.RT_OK
        assert list(rt.rt_ali_bin_stats(p.handle, p.desc.nf)[0]) == list(ita)
        assert st["iterations"] == sd["iterations"]
        assert np.array_equal(S.cpu().numpy(), Sa)
        assert np.array_equal(J.cpu().numpy(), Ja)
        p.close()


@pytest.mark.parametrize("k", [0, 3])
def test_persistent_batch_matches_oracle(env, oracle_mod, k):
    """Members of the persistent batch against the FP64 oracle (3 fixed iterations):
    an FP32 member with periodic x and y, and the FP64 member with three bins."""
    rt, torch = env
    shape, nf, n_mu, lo, hi, prec, er = BATCH[k]
    batch = [_make(rt, torch, j, spec, rt.RT_SCHED_PERSISTENT) for j, spec in enumerate(BATCH)]
    status, res, stats = rt.rt_ali_solve_batch([b[1].handle for b in batch], [b[2] for b in batch],
                                               [b[3] for b in batch], fixed_iters=3)
    torch.cuda.synchronize()
    assert status == rt.RT_OK
    wl = batch[k][0]
    op = oracle_mod.Problem(shape, wl.chi, wl.eps, wl.B, n_mu=n_mu, bc_lo=lo, bc_hi=hi, w_nu=wl.w_nu)
    ref = op.ali(fixed_iters=3)
    Sg = batch[k][2].cpu().numpy().reshape(ref["S"].shape)
    Jg = batch[k][3].cpu().numpy().reshape(ref["J"].shape)
    tol = 1e-12 if prec == "f64" else 2e-5
    assert np.max(np.abs(Sg - ref["S"]) / np.abs(ref["S"])) <= tol
    assert np.max(np.abs(Jg - ref["J"]) / np.abs(ref["J"])) <= tol
    for b in batch:
        b[1].close()


def test_batch_matches_oracle(env, oracle_mod):
    """One batch member against the FP64 oracle (3 fixed iterations)."""
    rt, torch = env
    k = 3   # the FP64 member with three bins and n_mu = 2
    shape, nf, n_mu, lo, hi, prec, er = BATCH[k]
    batch = [_make(rt, torch, j, spec) for j, spec in enumerate(BATCH)]
    status, res, stats = rt.rt_ali_solve_batch([b[1].handle for b in batch], [b[2] for b in batch],
                                               [b[3] for b in batch], fixed_iters=3)
    torch.cuda.synchronize()
    wl = batch[k][0]
    op = oracle_mod.Problem(shape, wl.chi, wl.eps, wl.B, n_mu=n_mu, bc_lo=lo, bc_hi=hi, w_nu=wl.w_nu)
    ref = op.ali(fixed_iters=3)
    Sg = batch[k][2].cpu().numpy().reshape(ref["S"].shape)
    Jg = batch[k][3].cpu().numpy().reshape(ref["J"].shape)
    assert np.max(np.abs(Sg - ref["S"]) / np.abs(ref["S"])) <= 1e-12
    assert np.max(np.abs(Jg - ref["J"]) / np.abs(ref["J"])) <= 1e-12
    for b in batch:
        b[1].close()


def test_batch_rejects_bad_arguments(env):
    rt, torch = env
    wl, p, S, J = _make(rt, torch, 0, BATCH[0])
    with pytest.raises(rt.RtError):
        rt.rt_ali_solve_batch([p.handle, p.handle], [S, S], [J, J], fixed_iters=1)   # same problem twice
    with pytest.raises(rt.RtError):
        rt.rt_ali_solve_batch([p.handle], [S], [J], fixed_iters=-1)
    p.close()
