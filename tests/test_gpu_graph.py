"""The ALI chunks captured as HIP graphs give bitwise the results of the same launches
issued from the host, over several replays with the program's own eager work (formal
solutions, warm-started solves, a moments pass) between them: Jacobi in both
precisions, second order, the quadratic upwind intensity and Gauss-Seidel."""
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


def _sequence(env, wl, graphs, precision, gs=False, **kw):
    """A solve to convergence, a formal solution, a warm-started solve of a fixed number
    of iterations (shorter last chunk), and a second converged solve: returns every
    output along the way."""
    rt, torch = env
    gp = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=precision, **kw)
    gp.use_graphs(graphs)
    gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    solve = gp.ali_solve_gs if gs else gp.ali_solve
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    out = []
    st, stats = solve(S, J, delta_c=1e-8, max_iter=3000, check_every=8)
    torch.cuda.synchronize()
    out += [S.cpu().numpy().copy(), J.cpu().numpy().copy(), stats["iterations"]]
    J2 = torch.empty_like(J)
    gp.formal_solve(S, J2)
    torch.cuda.synchronize()
    out.append(J2.cpu().numpy().copy())
    solve(S, J, fixed_iters=21, warm_start=1, check_every=8)
    torch.cuda.synchronize()
    out += [S.cpu().numpy().copy(), J.cpu().numpy().copy()]
    st, stats = solve(S, J, delta_c=1e-9, max_iter=3000, warm_start=2, check_every=8)
    torch.cuda.synchronize()
    out += [S.cpu().numpy().copy(), J.cpu().numpy().copy(), stats["iterations"]]
    gp.close()
    return out


@pytest.mark.parametrize("variant", ["f64", "f32", "bezier", "quadratic", "gs64", "gs32", "persistent64",
                                     "persistent32"])
def test_graph_replays_match_eager(env, variant):
    rt, torch = env
    wl = W.random_problem((20, 14, 12), nf=2, seed=1200, n_mu=4, eps_range=(1e-2, 1.0))
    prec = rt.RT_F32 if variant in ("f32", "bezier", "quadratic", "gs32", "persistent32") else rt.RT_F64
    kw = {}
    if variant.startswith("persistent"):
        kw["schedule"] = rt.RT_SCHED_PERSISTENT
    if variant == "bezier":
        kw["order"] = rt.RT_SC_BEZIER
    if variant == "quadratic":
        kw["interp"] = rt.RT_INTERP_QUADRATIC
    gs = variant.startswith("gs")
    eager = _sequence(env, wl, False, prec, gs=gs, **kw)
    graph = _sequence(env, wl, True, prec, gs=gs, **kw)
    assert len(eager) == len(graph)
    for a, b in zip(eager, graph):
        if isinstance(a, np.ndarray):
            assert np.array_equal(a, b)
        else:
            assert a == b


def test_persistent_graph_of_one_iteration(env):
    """The persistent schedule replayed from a one-iteration graph many times in a row
    (every replay needs its own epoch and fresh ticket counters, set on the device)
    gives bitwise the host-issued iterations."""
    rt, torch = env
    wl = W.random_problem((26, 17, 21), nf=2, seed=1300, n_mu=6, eps_range=(1e-2, 1.0))
    out = []
    for graphs in (False, True):
        gp = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F32,
                        schedule=rt.RT_SCHED_PERSISTENT)
        gp.use_graphs(graphs)
        gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
        n = wl.chi.size
        S = torch.empty(n, dtype=torch.float64, device="cuda")
        J = torch.empty(n, dtype=torch.float64, device="cuda")
        st, stats = gp.ali_solve(S, J, fixed_iters=40, check_every=1)
        torch.cuda.synchronize()
        assert st == rt.RT_OK and stats["iterations"] == 40
        out.append((S.cpu().numpy(), J.cpu().numpy()))
        gp.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_graph_cache_follows_the_buffers(env, oracle_mod):
    """A solve into other S and J buffers captures again (the chunk's arguments differ);
    results still match the oracle."""
    rt, torch = env
    wl = W.random_problem((16, 12, 10), nf=1, seed=1210, n_mu=4, eps_range=(1e-2, 1.0))
    op = oracle_mod.Problem(wl.shape, wl.chi, wl.eps, wl.B, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi)
    ref = op.ali(fixed_iters=5)
    gp = rt.Problem(wl.shape, nf=1, n_mu=4, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi)
    gp.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    n = wl.chi.size
    for _ in range(3):
        S = torch.empty(n, dtype=torch.float64, device="cuda")
        J = torch.empty(n, dtype=torch.float64, device="cuda")
        gp.reset_periodic()
        gp.ali_solve(S, J, fixed_iters=5, check_every=2)
        torch.cuda.synchronize()
        Sg = S.cpu().numpy().reshape(ref["S"].shape)
        assert np.max(np.abs(Sg - ref["S"]) / ref["S"]) <= 1e-12
    gp.close()
