"""The C ABI's context object and FP32 caller arrays, and the serving loop's ordering
against the caller's stream, through the binding.

* A context names a device: problems, batches and servers made with it run there,
  and failures of calls on them are recorded in it as well as per thread.
* FP32 caller arrays (rt_problem_desc.in_dtype = RT_DTYPE_F32): the library widens the
  fields and S (and J for warm starts) to FP64, computes exactly as for FP64 arrays of
  the same values, and rounds its FP64 results once.  So every output equals the
  FP64-array problem's output on the widened inputs, rounded to FP32, bit for bit:
  formal solution with Lambda*, ALI from each start, moments with the heating sum,
  a batch that mixes both kinds, and a server request.
* rt_server_submit waits for the work queued on the caller's stream before the
  request: fields and a warm-start S written on a side stream behind a long kernel,
  submitted without synchronising, give the synchronous result."""
import time

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


def _pair(rt, torch, shape=(13, 10, 9), nf=2, n_mu=4, seed=31, precision=None, order=0):
    """The same problem twice: FP32 caller arrays, and FP64 arrays holding the widened
    FP32 values."""
    wl = W.random_problem(shape, nf=nf, seed=seed, n_mu=n_mu, eps_range=(1e-2, 1.0))
    prec = rt.RT_F32 if precision is None else precision
    f32 = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).ravel()).cuda() for a in (wl.chi, wl.eps, wl.B)]
    f64 = [a.double() for a in f32]
    kw = dict(nf=nf, n_mu=n_mu, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, w_nu=wl.w_nu, precision=prec, order=order)
    a = rt.Problem(shape, in_dtype=rt.RT_DTYPE_F32, **kw)
    a.set_fields(*f32)
    b = rt.Problem(shape, **kw)
    b.set_fields(*f64)
    return wl, a, b


def _same(x32, x64):
    assert x32.dtype.itemsize == 4
    np.testing.assert_array_equal(x32.cpu().numpy(), x64.float().cpu().numpy())


def test_context_device_and_errors(env):
    rt, torch = env
    ctx = rt.rt_context_create(0)
    try:
        with pytest.raises(rt.RtError):
            rt.rt_context_create(torch.cuda.device_count())
        wl = W.random_problem((9, 8, 7), nf=1, seed=3, n_mu=4)
        p = rt.Problem(wl.shape, nf=1, n_mu=4, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, precision=rt.RT_F32, ctx=ctx)
        dev = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64).ravel()).cuda()
        p.set_fields(dev(wl.chi), dev(wl.eps), dev(wl.B))
        S = torch.empty(wl.chi.size, dtype=torch.float64, device="cuda")
        J = torch.empty_like(S)
        status, st = p.ali_solve(S, J, fixed_iters=3)
        assert status == rt.RT_OK and st["iterations"] == 3
        # a failing call on the problem: the message is in the context and on the thread
        with pytest.raises(rt.RtError):
            p.ali_solve(S, J, fixed_iters=-1)
        assert "fixed_iters" in rt.rt_last_error(ctx)
        assert "fixed_iters" in rt.rt_last_error()
        # a batch and a server made with the context run its problems
        status, res, stats = rt.rt_ali_solve_batch([p.handle], [S], [J], fixed_iters=2, ctx=ctx)
        assert status == rt.RT_OK and stats[0]["iterations"] == 2
        srv = rt.rt_server_create(1 << 34, ctx=ctx)
        t = rt.rt_server_submit(srv, p.handle, S, J, fixed_iters=2)
        t0 = time.time()
        while rt.rt_server_poll(srv, t) is None:
            assert time.time() - t0 < 60
            time.sleep(0.001)
        rt.rt_server_release(srv, t)
        rt.rt_server_destroy(srv)
        p.close()
    finally:
        rt.rt_context_destroy(ctx)


@pytest.mark.parametrize("precision, order", [("f32", 0), ("f64", 0), ("f32", 1)])
def test_fp32_arrays_formal_solve_and_ali(env, precision, order):
    rt, torch = env
    prec = rt.RT_F32 if precision == "f32" else rt.RT_F64
    wl, a, b = _pair(rt, torch, precision=prec, order=order)
    n = wl.chi.size
    rng = np.random.default_rng(5)
    S32 = torch.from_numpy((wl.B * (0.5 + rng.random(wl.B.shape))).astype(np.float32).ravel()).cuda()
    J32, L32 = torch.empty_like(S32), torch.empty_like(S32)
    J64 = torch.empty(n, dtype=torch.float64, device="cuda")
    L64 = torch.empty_like(J64)
    a.formal_solve(S32, J32, L32)
    b.formal_solve(S32.double(), J64, L64)
    torch.cuda.synchronize()
    _same(J32, J64)
    _same(L32, L64)
    for warm in (0, 1, 2):
        Sa, Ja = S32.clone(), J32.clone()
        Sb, Jb = Sa.double(), Ja.double()
        sa, sta = a.ali_solve(Sa, Ja, fixed_iters=5, warm_start=warm)
        sb, stb = b.ali_solve(Sb, Jb, fixed_iters=5, warm_start=warm)
        torch.cuda.synchronize()
        assert sa == sb == rt.RT_OK
        _same(Sa, Sb)
        _same(Ja, Jb)
    a.close()
    b.close()


def test_fp32_arrays_moments(env):
    rt, torch = env
    wl, a, b = _pair(rt, torch, shape=(12, 11, 10), nf=3)
    n, c = wl.chi.size, wl.cells
    S32 = torch.from_numpy(wl.B.astype(np.float32).ravel()).cuda()
    sizes = {"J": n, "H": 3 * n, "K": 6 * n, "J_int": c, "H_int": 3 * c, "K_int": 6 * c, "f_int": 6 * c, "Q_int": c}
    o32 = {k: torch.empty(v, dtype=torch.float32, device="cuda") for k, v in sizes.items()}
    o64 = {k: torch.empty(v, dtype=torch.float64, device="cuda") for k, v in sizes.items()}
    h32 = a.moments(S32, want_heating=True, **o32)
    h64 = b.moments(S32.double(), want_heating=True, **o64)
    torch.cuda.synchronize()
    assert h32 == h64
    for k in sizes:
        _same(o32[k], o64[k])
    a.close()
    b.close()


def test_fp32_arrays_batch_and_server(env):
    rt, torch = env
    pairs = [_pair(rt, torch, shape=s, nf=nf, seed=50 + k) for k, (s, nf) in
             enumerate((((11, 9, 8), 2), ((9, 12, 10), 1), ((10, 10, 7), 3)))]
    # a batch mixing FP32-array and FP64-array problems, each to convergence
    batch = [pairs[0][1], pairs[1][1], pairs[2][2]]
    Ss = [torch.empty(p.nf * p.cells, dtype=torch.float32 if i < 2 else torch.float64, device="cuda")
          for i, p in enumerate(batch)]
    Js = [torch.empty_like(x) for x in Ss]
    status, res, stats = rt.rt_ali_solve_batch([p.handle for p in batch], Ss, Js, delta_c=1e-6, max_iter=3000)
    assert status == rt.RT_OK
    for i, (wl, a, b) in enumerate(pairs[:2]):
        S64 = torch.empty(a.nf * a.cells, dtype=torch.float64, device="cuda")
        J64 = torch.empty_like(S64)
        b.ali_solve(S64, J64, delta_c=1e-6, max_iter=3000)
        torch.cuda.synchronize()
        _same(Ss[i], S64)
        _same(Js[i], J64)
    # a server request with FP32 arrays
    wl, a, b = pairs[2]
    S32 = torch.empty(a.nf * a.cells, dtype=torch.float32, device="cuda")
    J32 = torch.empty_like(S32)
    srv = rt.rt_server_create(1 << 34, check_every=8)
    t = rt.rt_server_submit(srv, a.handle, S32, J32, delta_c=1e-6, max_iter=3000)
    t0 = time.time()
    while (r := rt.rt_server_poll(srv, t)) is None:
        assert time.time() - t0 < 60
        time.sleep(0.001)
    assert r[0] == rt.RT_OK
    rt.rt_server_release(srv, t)
    rt.rt_server_destroy(srv)
    torch.cuda.synchronize()
    _same(S32, Ss[2])
    _same(J32, Js[2])
    for _, a, b in pairs:
        a.close()
        b.close()


def test_server_waits_for_the_callers_stream(env):
    """Fields and a warm-start S are written on a side stream behind a kernel that spins
    for tens of milliseconds, and the request is submitted right away with that stream:
    the result is the one of the same inputs submitted after a full synchronisation."""
    rt, torch = env
    wl = W.random_problem((14, 12, 10), nf=2, seed=61, n_mu=4, eps_range=(1e-2, 1.0))
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64).ravel()).cuda()
    chi, eps, B = dev(wl.chi), dev(wl.eps), dev(wl.B)
    start = (B * 1.5).contiguous()
    results = []
    for synchronous in (True, False):
        p = rt.Problem(wl.shape, nf=2, n_mu=4, bc_lo=wl.bc_lo, bc_hi=wl.bc_hi, w_nu=wl.w_nu, precision=rt.RT_F32)
        S = torch.zeros_like(B)
        J = torch.zeros_like(B)
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        srv = rt.rt_server_create(1 << 34, check_every=4)
        with torch.cuda.stream(side):
            torch.cuda._sleep(50_000_000)          # about 20 ms of spinning on the side stream
            p.set_fields(chi, eps, B, stream=side)
            S.copy_(start)
        if synchronous:
            torch.cuda.synchronize()
        t = rt.rt_server_submit(srv, p.handle, S, J, fixed_iters=6, warm_start=1, stream=side)
        t0 = time.time()
        while (r := rt.rt_server_poll(srv, t)) is None:
            assert time.time() - t0 < 60
            time.sleep(0.001)
        assert r[0] == rt.RT_OK
        rt.rt_server_release(srv, t)
        rt.rt_server_destroy(srv)
        torch.cuda.synchronize()
        results.append((S.cpu().numpy(), J.cpu().numpy()))
        p.close()
    np.testing.assert_array_equal(results[0][0], results[1][0])
    np.testing.assert_array_equal(results[0][1], results[1][1])
