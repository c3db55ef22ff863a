"""Checkpoint and resume: a problem's periodic memory saved after some iterations and
loaded into a new problem of the same description, with S, continues the ALI with
bitwise the results of the uninterrupted run (Jacobi in both precisions, second order,
the quadratic upwind intensity, Gauss-Seidel), to host or device buffers.  Without the
saved memory the continuation differs, so the test sees the state that matters.  A
state of another problem, a short buffer or a buffer that is no state is refused and
leaves the problem as it was."""
import numpy as np
import pytest

from paper_1201_2222_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPE = (20, 14, 12)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1201_2222_amd as rt
    assert torch.cuda.is_available(), "GPU tests need a device"
    rt.load()
    return rt, torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _kw(rt, variant):
    kw = {"precision": rt.RT_F64 if variant in ("f64", "quadratic64", "gs64") else rt.RT_F32}
    if variant == "bezier":
        kw["order"] = rt.RT_SC_BEZIER
    if variant.startswith("quadratic"):
        kw["interp"] = rt.RT_INTERP_QUADRATIC
    return kw


def _problem(env, wl, **kw):
    rt, torch = env
    p = rt.Problem(wl.shape, nf=wl.nf, n_mu=wl.n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, **kw)
    p.set_fields(_dev(torch, wl.chi), _dev(torch, wl.eps), _dev(torch, wl.B))
    return p


def _continue(env, p, S, gs, iters):
    rt, torch = env
    S = S.clone()
    J = torch.empty_like(S)
    (p.ali_solve_gs if gs else p.ali_solve)(S, J, fixed_iters=iters, warm_start=1, check_every=8)
    torch.cuda.synchronize()
    return S.cpu().numpy(), J.cpu().numpy()


@pytest.mark.parametrize("where", ["host", "device"])
@pytest.mark.parametrize("variant", ["f64", "f32", "bezier", "quadratic", "quadratic64", "gs32", "gs64"])
def test_resume_continues_bitwise(env, variant, where):
    rt, torch = env
    wl = W.random_problem(SHAPE, nf=2, seed=1300, n_mu=4, eps_range=(1e-2, 1.0))
    kw = _kw(rt, variant)
    gs = variant.startswith("gs")
    a = _problem(env, wl, **kw)
    n = wl.chi.size
    S = torch.empty(n, dtype=torch.float64, device="cuda")
    J = torch.empty_like(S)
    (a.ali_solve_gs if gs else a.ali_solve)(S, J, fixed_iters=13, check_every=8)
    nb = a.state_bytes()
    if where == "host":
        state = a.save_state()
    else:
        state = a.save_state(torch.zeros(nb, dtype=torch.uint8, device="cuda"))
    S_ref, J_ref = _continue(env, a, S, gs, 17)

    b = _problem(env, wl, **kw)
    b.load_state(state)
    S_b, J_b = _continue(env, b, S, gs, 17)
    assert np.array_equal(S_b, S_ref)
    assert np.array_equal(J_b, J_ref)

    c = _problem(env, wl, **kw)   # cold: periodic ghosts from S instead of the memory
    S_c, _ = _continue(env, c, S, gs, 17)
    assert not np.array_equal(S_c, S_ref)
    for p in (a, b, c):
        p.close()


def test_state_size_follows_the_periodic_faces(env):
    rt, torch = env
    nx, ny, nz = SHAPE
    wl = W.random_problem(SHAPE, nf=2, seed=1310, n_mu=4)
    p = _problem(env, wl, precision=rt.RT_F32)
    na = 24
    pad = lambda b: (b + 255) // 256 * 256
    expect = pad(56) + pad(4 * 2) + pad(2 * na * 2 * ny * nz * 8) + pad(2 * na * 2 * nx * nz * 8)
    assert p.state_bytes() == expect
    p.close()
    closed = W.random_problem(SHAPE, nf=2, seed=1310, n_mu=4, bc_lo=(W.VACUUM, W.VACUUM, W.THERMAL),
                              bc_hi=(W.VACUUM, W.VACUUM, W.VACUUM))
    q = _problem(env, closed, precision=rt.RT_F32)
    assert q.state_bytes() == pad(56) + pad(4 * 2)
    q.close()


def test_cold_state_round_trip(env):
    """The state of a problem that has not swept yet is the cold flag: loading it into
    a problem that has swept makes its next solve that of a fresh problem."""
    rt, torch = env
    wl = W.random_problem(SHAPE, nf=2, seed=1320, n_mu=4)
    fresh = _problem(env, wl, precision=rt.RT_F32)
    cold = fresh.save_state()
    n = wl.chi.size
    S0 = _dev(torch, wl.B.ravel() * 1.1)
    S_f, J_f = _continue(env, fresh, S0, False, 9)
    used = _problem(env, wl, precision=rt.RT_F32)
    _continue(env, used, S0, False, 5)
    used.load_state(cold)
    S_u, J_u = _continue(env, used, S0, False, 9)
    assert np.array_equal(S_u, S_f) and np.array_equal(J_u, J_f)
    assert S_u.shape == (n,)
    for p in (fresh, used):
        p.close()


def test_foreign_or_damaged_states_are_refused(env):
    rt, torch = env
    wl = W.random_problem(SHAPE, nf=2, seed=1330, n_mu=4)
    p = _problem(env, wl, precision=rt.RT_F32)
    n = wl.chi.size
    S0 = _dev(torch, wl.B.ravel())
    _continue(env, p, S0, False, 6)
    good = p.save_state()
    S_ref, J_ref = _continue(env, p, S0, False, 7)
    p.load_state(good)

    others = [
        (W.random_problem(SHAPE, nf=1, seed=1331, n_mu=4), {"precision": rt.RT_F32}),
        (wl, {"precision": rt.RT_F64}),
        (W.random_problem(SHAPE, nf=2, seed=1332, n_mu=6), {"precision": rt.RT_F32}),
        (W.random_problem((20, 14, 13), nf=2, seed=1333, n_mu=4), {"precision": rt.RT_F32}),
        (wl, {"precision": rt.RT_F32, "interp": rt.RT_INTERP_QUADRATIC}),
    ]
    # the same 24 directions with other weights: another angle set of the same size
    mu, w = rt.rt_quadrature(4)
    w2 = w * (1.0 + 0.01 * (np.arange(w.size) % 2))
    others.append((wl, {"precision": rt.RT_F32, "mu": mu, "w": w2 / w2.sum()}))
    for owl, kw in others:
        o = _problem(env, owl, **kw)
        with pytest.raises(rt.RtError) as e:
            p.load_state(o.save_state())
        assert e.value.status == rt.RT_E_INVALID
        o.close()
    with pytest.raises(rt.RtError):
        p.load_state(good[: good.size // 2].copy())
    junk = good.copy()
    junk[0] ^= 0xFF
    with pytest.raises(rt.RtError):
        p.load_state(junk)
    with pytest.raises(rt.RtError):
        p.save_state(np.zeros(good.size - 1, dtype=np.uint8))
    # the refusals left the loaded state in place
    S_p, J_p = _continue(env, p, S0, False, 7)
    assert np.array_equal(S_p, S_ref) and np.array_equal(J_p, J_ref)
    p.close()
