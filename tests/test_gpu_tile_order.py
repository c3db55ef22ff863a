"""Race check of the tile wavefront: with RTSC_TILE_ORDER_SEED set when a problem is
created, the tiles of every stage go to the workgroups of that stage's launch in a
shuffled order, which changes which workgroup (and which XCD) sweeps which tile and
when.  Tiles of one stage only read faces written by earlier stages, so the formal
solution, Lambda*, the ALI (Jacobi and the upward sweeps of Gauss-Seidel), the
moments and a batched solve are bitwise the same for every seed."""
import numpy as np
import pytest

from paper_1201_2222_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPE = (40, 36, 28)   # 5 x 5 x 4 tiles of 8^3: stages of up to 18 tiles
SEEDS = (1, 7, 982451653)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1201_2222_amd as rt
    assert torch.cuda.is_available(), "GPU tests need a device"
    rt.load()
    return rt, torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _make(env, wl, variant):
    rt, torch = env
    kw = {"precision": rt.RT_F64 if variant == "f64" else rt.RT_F32}
    if variant == "bezier":
        kw["order"] = rt.RT_SC_BEZIER
    p = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, w_nu=wl.w_nu, **kw)
    p.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    return p


def _outputs(env, wl, variant):
    rt, torch = env
    p = _make(env, wl, variant)
    n = wl.chi.size
    S0 = _dev(torch, wl.B.ravel() * 1.2)
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    lam = torch.empty_like(J)
    p.formal_solve(S0, J, lam)
    out = [J, lam]
    S = torch.empty_like(J)
    J2 = torch.empty_like(J)
    (p.ali_solve_gs if variant == "gs32" else p.ali_solve)(S, J2, fixed_iters=12, check_every=4)
    out += [S, J2]
    if variant != "gs32":
        H = torch.empty(3 * n, dtype=torch.float64, device="cuda")
        K = torch.empty(6 * n, dtype=torch.float64, device="cuda")
        heat = p.moments(S, H=H, K=K, want_heating=True)
        out += [H, K]
    torch.cuda.synchronize()
    res = [t.cpu().numpy().copy() for t in out]
    if variant != "gs32":
        res.append(np.array([heat]))
    p.close()
    return res


@pytest.mark.parametrize("variant", ["f64", "f32", "bezier", "gs32"])
def test_shuffled_tile_order_is_bitwise_the_same(env, variant, monkeypatch):
    wl = W.random_problem(SHAPE, nf=2, seed=1400, n_mu=4, eps_range=(1e-2, 1.0))
    monkeypatch.delenv("RTSC_TILE_ORDER_SEED", raising=False)
    ref = _outputs(env, wl, variant)
    for seed in SEEDS:
        monkeypatch.setenv("RTSC_TILE_ORDER_SEED", str(seed))
        got = _outputs(env, wl, variant)
        assert len(got) == len(ref)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), f"seed {seed}"


def test_shuffled_batch_is_bitwise_the_same(env, monkeypatch):
    rt, torch = env
    wls = [W.random_problem(SHAPE, nf=2, seed=1410, n_mu=4),
           W.random_problem((24, 17, 33), nf=1, seed=1411, n_mu=6),
           W.random_problem((16, 40, 9), nf=3, seed=1412, n_mu=2)]

    def run():
        ps = [_make(env, wl, "f32") for wl in wls]
        S = [torch.empty(wl.chi.size, dtype=torch.float64, device="cuda") for wl in wls]
        J = [torch.empty_like(s) for s in S]
        rt.rt_ali_solve_batch([p.handle for p in ps], S, J, fixed_iters=9, check_every=3)
        torch.cuda.synchronize()
        for p in ps:
            p.close()
        return [t.cpu().numpy() for t in S + J]

    monkeypatch.delenv("RTSC_TILE_ORDER_SEED", raising=False)
    ref = run()
    monkeypatch.setenv("RTSC_TILE_ORDER_SEED", "31337")
    got = run()
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
