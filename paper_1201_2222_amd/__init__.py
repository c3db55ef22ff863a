"""MI355X-native short-characteristics radiative transfer (Davis, Stone & Jiang 2012).

Thin Python binding of the C ABI in ``include/rt.h`` (``librtsc.so``).  The
functions here only marshal arguments: every step of the formal solution, the
Lambda iteration and the moments runs in the library's HIP kernels.  PyTorch is
used for device memory and streams only.  If the library is missing the calls
raise; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtsc.so")

RT_OK, RT_NOT_CONVERGED = 0, 1
RT_E_INVALID, RT_E_OOM, RT_E_HIP, RT_E_NONFINITE, RT_E_UNSUPPORTED, RT_E_BUSY = -1, -2, -3, -4, -5, -6
RT_F64, RT_F32 = 0, 1
RT_BC_VACUUM, RT_BC_THERMAL, RT_BC_PERIODIC, RT_BC_FIXED = 0, 1, 2, 3
RT_SCHED_DEFAULT, RT_SCHED_STAGES, RT_SCHED_PERSISTENT = 0, 1, 2
RT_SC_LINEAR, RT_SC_BEZIER = 0, 1
RT_INTERP_BILINEAR, RT_INTERP_QUADRATIC = 0, 1
RT_DTYPE_F64, RT_DTYPE_F32 = 0, 1

# names of the C entry points (include/rt.h); every one is looked up at load time
EXPORTS = ("rt_status_string", "rt_last_error", "rt_context_create", "rt_context_destroy", "rt_quadrature", "rt_problem_bytes", "rt_problem_create",
           "rt_problem_destroy", "rt_problem_set_fields", "rt_problem_reset_periodic", "rt_problem_state_bytes",
           "rt_problem_save_state", "rt_problem_load_state", "rt_formal_solve",
           "rt_ali_solve", "rt_ali_solve_gs", "rt_problem_use_graphs", "rt_problem_set_waves", "rt_problem_set_wait_limit",
           "rt_problem_tune", "rt_ali_bin_stats", "rt_moments", "rt_problem_profile", "rt_problem_profile_read",
           "rt_ali_solve_batch", "rt_server_create", "rt_server_submit", "rt_server_poll", "rt_server_release",
           "rt_server_load", "rt_server_destroy", "rt_formal_solve_noalloc")


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class ProblemDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("nf", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("n_mu", ctypes.c_int32), ("na", ctypes.c_int32),
                ("mu", ctypes.c_void_p), ("w", ctypes.c_void_p), ("w_nu", ctypes.c_void_p),
                ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
                ("I_fixed", ctypes.c_void_p * 6),
                ("precision", ctypes.c_int32), ("tile", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("order", ctypes.c_int32), ("interp", ctypes.c_int32), ("in_dtype", ctypes.c_int32)]


class AliOpts(ctypes.Structure):
    _fields_ = [("delta_c", ctypes.c_double), ("max_iter", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("per_bin_stop", ctypes.c_int32), ("warm_start", ctypes.c_int32), ("check_every", ctypes.c_int32)]


class AliStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("bins_converged", ctypes.c_int32),
                ("max_rel_dS", ctypes.c_double), ("seconds", ctypes.c_double)]


class MomentsOut(ctypes.Structure):
    _fields_ = [("J", ctypes.c_void_p), ("H", ctypes.c_void_p), ("K", ctypes.c_void_p),
                ("J_int", ctypes.c_void_p), ("H_int", ctypes.c_void_p), ("K_int", ctypes.c_void_p),
                ("f_int", ctypes.c_void_p), ("Q_int", ctypes.c_void_p), ("heating", ctypes.c_void_p)]


class Profile(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("launches", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("updates", ctypes.c_double), ("stages", ctypes.c_int32), ("chain_ms", ctypes.c_double),
                ("chain_launches", ctypes.c_int64), ("chain_updates", ctypes.c_double)]


_lib = None


def load():
    """Load librtsc.so from the package directory (built by ``build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"librtsc.so is not built ({LIB_PATH}); run paper_1201_2222_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    lib.rt_status_string.restype = ctypes.c_char_p
    lib.rt_status_string.argtypes = [ctypes.c_int]
    lib.rt_last_error.restype = ctypes.c_char_p
    lib.rt_last_error.argtypes = [P]
    lib.rt_context_create.argtypes = [I32, ctypes.POINTER(P)]
    lib.rt_context_destroy.argtypes = [P]
    lib.rt_quadrature.argtypes = [I32, P, P, P]
    lib.rt_problem_bytes.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(ctypes.c_size_t)]
    lib.rt_problem_create.argtypes = [P, ctypes.POINTER(ProblemDesc), ctypes.POINTER(P)]
    lib.rt_problem_destroy.argtypes = [P]
    lib.rt_problem_set_fields.argtypes = [P, P, P, P, P]
    lib.rt_problem_reset_periodic.argtypes = [P, P]
    lib.rt_problem_state_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.rt_problem_save_state.argtypes = [P, P, ctypes.c_size_t, P]
    lib.rt_problem_load_state.argtypes = [P, P, ctypes.c_size_t, P]
    lib.rt_formal_solve.argtypes = [P, P, P, P, P]
    lib.rt_ali_solve.argtypes = [P, ctypes.POINTER(AliOpts), P, P, ctypes.POINTER(AliStats), P]
    lib.rt_ali_solve_gs.argtypes = [P, ctypes.POINTER(AliOpts), P, P, ctypes.POINTER(AliStats), P]
    lib.rt_problem_use_graphs.argtypes = [P, I32]
    lib.rt_problem_set_waves.argtypes = [P, I32]
    lib.rt_problem_set_wait_limit.argtypes = [P, ctypes.c_double]
    lib.rt_problem_tune.argtypes = [P, P, I32, ctypes.POINTER(I32), P, P]
    lib.rt_ali_bin_stats.argtypes = [P, P, P, P]
    lib.rt_moments.argtypes = [P, P, ctypes.POINTER(MomentsOut), P]
    lib.rt_problem_profile.argtypes = [P, I32]
    lib.rt_problem_profile_read.argtypes = [P, ctypes.POINTER(Profile)]
    lib.rt_ali_solve_batch.argtypes = [P, P, I32, ctypes.POINTER(AliOpts), P, P, P, P, P]
    lib.rt_server_create.argtypes = [P, ctypes.c_size_t, I32, ctypes.POINTER(P)]
    lib.rt_server_submit.argtypes = [P, P, ctypes.POINTER(AliOpts), P, P, P, ctypes.POINTER(ctypes.c_uint64)]
    lib.rt_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(AliStats), ctypes.POINTER(ctypes.c_int)]
    lib.rt_server_release.argtypes = [P, ctypes.c_uint64]
    lib.rt_server_load.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_size_t)]
    lib.rt_server_destroy.argtypes = [P]
    lib.rt_formal_solve_noalloc.argtypes = [ctypes.POINTER(ProblemDesc), P, P, P, P, P, P]
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype or ctypes.c_int
    _lib = lib
    return lib


def _check(status, allow=(RT_OK,)):
    if status not in allow:
        lib = load()
        raise RtError(status, lib.rt_last_error(None).decode())
    return status


def _hval(h):
    """Integer value of a library handle (ctypes.c_void_p or int)."""
    return h.value if isinstance(h, ctypes.c_void_p) else int(h)


# Shape of every live problem handle, for the size checks of the marshalling:
# handle value -> (cells, nf, in_dtype, na)
_SHAPES = {}


def _shape(p):
    try:
        return _SHAPES[_hval(p)]
    except KeyError:
        raise ValueError("unknown or destroyed problem handle") from None


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, n=None, name="tensor", dtype=RT_DTYPE_F64):
    """Device pointer of a contiguous CUDA tensor of the given element type (float64, or
    float32 for RT_DTYPE_F32) with n elements; refuses any other tensor before the
    library sees it, so a short buffer never reaches a kernel."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a device tensor")
    want = torch.float32 if dtype == RT_DTYPE_F32 else torch.float64
    if t.dtype != want or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous {str(want).replace('torch.', '')}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _field(p, t, name, per=1):
    """Pointer of a field array of problem p: per * nf * cells elements in its in_dtype."""
    cells, nf, dt, _ = _shape(p)
    return _dptr(t, per * nf * cells, name, dt)


def _cellfield(p, t, name, per=1):
    """Pointer of a frequency-integrated array of problem p: per * cells elements."""
    cells, _, dt, _ = _shape(p)
    return _dptr(t, per * cells, name, dt)


def rt_quadrature(n_mu: int):
    """Level-symmetric angle set (mu [na, 3], w [na]) generated by the library."""
    lib = load()
    na = ctypes.c_int32()
    _check(lib.rt_quadrature(n_mu, None, None, ctypes.byref(na)))
    mu = np.zeros((na.value, 3))
    w = np.zeros(na.value)
    _check(lib.rt_quadrature(n_mu, mu.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                             ctypes.byref(na)))
    return mu, w


def make_desc(shape, nf=1, h=(1.0, 1.0, 1.0), n_mu=4, bc_lo=(2, 2, 1), bc_hi=(2, 2, 0), precision=RT_F64,
              mu=None, w=None, w_nu=None, I_fixed=None, tile=0, schedule=RT_SCHED_DEFAULT, order=RT_SC_LINEAR,
              interp=RT_INTERP_BILINEAR, in_dtype=RT_DTYPE_F64):
    d = ProblemDesc()
    d.nx, d.ny, d.nz = (int(x) for x in shape)
    d.nf = int(nf)
    d.dx, d.dy, d.dz = (float(x) for x in h)
    d.n_mu = int(n_mu)
    keep = []
    if mu is not None:
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        keep += [mu, w]
        d.na = len(w)
        d.mu = mu.ctypes.data
        d.w = w.ctypes.data
    if w_nu is not None:
        w_nu = np.ascontiguousarray(w_nu, dtype=np.float64)
        keep.append(w_nu)
        d.w_nu = w_nu.ctypes.data
    d.bc_lo[:] = [int(x) for x in bc_lo]
    d.bc_hi[:] = [int(x) for x in bc_hi]
    if I_fixed is not None:
        na = d.na if mu is not None else d.n_mu * (d.n_mu + 2)
        n3 = (d.nx, d.ny, d.nz)
        for k, t in enumerate(I_fixed):
            if t is not None:
                q = k // 2
                face = int(np.prod([n3[a] for a in range(3) if a != q]))
                d.I_fixed[k] = _dptr(t, d.nf * na * face, name="I_fixed").value
                keep.append(t)
    d.precision = int(precision)
    d.tile = int(tile)
    d.schedule = int(schedule)
    d.order = int(order)
    d.interp = int(interp)
    d.in_dtype = int(in_dtype)
    d._keep = keep
    return d


def rt_problem_bytes(desc: ProblemDesc) -> int:
    lib = load()
    b = ctypes.c_size_t()
    _check(lib.rt_problem_bytes(ctypes.byref(desc), ctypes.byref(b)))
    return b.value


def rt_context_create(device=0):
    """A context on HIP device ``device`` (rt_context_create)."""
    h = ctypes.c_void_p()
    _check(load().rt_context_create(int(device), ctypes.byref(h)))
    return h


def rt_context_destroy(ctx):
    return _check(load().rt_context_destroy(ctx))


def rt_last_error(ctx=None):
    """The last failure recorded in a context, or on this thread (ctx None)."""
    return load().rt_last_error(ctx).decode()


def rt_problem_create(desc: ProblemDesc, ctx=None):
    lib = load()
    h = ctypes.c_void_p()
    _check(lib.rt_problem_create(ctx, ctypes.byref(desc), ctypes.byref(h)))
    na = desc.na if desc.mu else desc.n_mu * (desc.n_mu + 2)
    _SHAPES[h.value] = (int(desc.nx) * int(desc.ny) * int(desc.nz), int(desc.nf), int(desc.in_dtype), int(na))
    return h


def rt_problem_destroy(p):
    st = _check(load().rt_problem_destroy(p))
    _SHAPES.pop(_hval(p), None)
    return st


def rt_problem_set_fields(p, chi, eps, B, stream=None):
    return _check(load().rt_problem_set_fields(p, _field(p, chi, "chi"), _field(p, eps, "eps"), _field(p, B, "B"),
                                               _stream(stream)))


def rt_problem_reset_periodic(p, stream=None):
    return _check(load().rt_problem_reset_periodic(p, _stream(stream)))


def _raw(buf):
    """Address and size in bytes of a contiguous numpy array or torch tensor."""
    if isinstance(buf, np.ndarray):
        if not buf.flags["C_CONTIGUOUS"]:
            raise ValueError("state buffer must be contiguous")
        return ctypes.c_void_p(buf.ctypes.data), buf.nbytes
    if not buf.is_contiguous():
        raise ValueError("state buffer must be contiguous")
    return ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()


def rt_problem_state_bytes(p):
    b = ctypes.c_size_t()
    _check(load().rt_problem_state_bytes(p, ctypes.byref(b)))
    return b.value


def rt_problem_save_state(p, dst=None, stream=None):
    """Save the periodic memory into ``dst`` (numpy array or torch tensor, host or
    device) or, if None, into a new host uint8 array, which is returned."""
    if dst is None:
        dst = np.zeros(rt_problem_state_bytes(p), dtype=np.uint8)
    ptr, nb = _raw(dst)
    _check(load().rt_problem_save_state(p, ptr, nb, _stream(stream)))
    return dst


def rt_problem_load_state(p, src, stream=None):
    ptr, nb = _raw(src)
    return _check(load().rt_problem_load_state(p, ptr, nb, _stream(stream)))


def rt_formal_solve(p, S, J, lambda_star=None, stream=None):
    return _check(load().rt_formal_solve(p, _field(p, S, "S"), _field(p, J, "J"),
                                         _field(p, lambda_star, "lambda_star"), _stream(stream)))


def rt_ali_solve(p, S, J, delta_c=1e-6, max_iter=10000, fixed_iters=0, per_bin_stop=True, warm_start=0,
                 check_every=0, stream=None, gauss_seidel=False):
    """Returns (status, stats dict); status is RT_OK or RT_NOT_CONVERGED, errors raise.
    ``gauss_seidel`` calls rt_ali_solve_gs instead of the Jacobi rt_ali_solve."""
    o = AliOpts(float(delta_c), int(max_iter), int(fixed_iters), 1 if per_bin_stop else 0, int(warm_start),
                int(check_every))
    st = AliStats()
    fn = load().rt_ali_solve_gs if gauss_seidel else load().rt_ali_solve
    status = fn(p, ctypes.byref(o), _field(p, S, "S"), _field(p, J, "J"), ctypes.byref(st), _stream(stream))
    _check(status, allow=(RT_OK, RT_NOT_CONVERGED))
    return status, {"iterations": st.iterations, "bins_converged": st.bins_converged,
                    "max_rel_dS": st.max_rel_dS, "seconds": st.seconds}


def rt_ali_solve_batch(problems, S_list, J_list, delta_c=1e-6, max_iter=10000, fixed_iters=0, per_bin_stop=True,
                       warm_start=0, check_every=0, stream=None, ctx=None):
    """Batched ALI over independent problems (handles); returns (status, [per-problem status],
    [per-problem stats dict]).  RT_E_NONFINITE is returned, not raised, so the per-problem
    results can be inspected; other errors raise."""
    n = len(problems)
    if len(S_list) != n or len(J_list) != n:
        raise ValueError("problems, S_list and J_list must have the same length")
    o = AliOpts(float(delta_c), int(max_iter), int(fixed_iters), 1 if per_bin_stop else 0, int(warm_start),
                int(check_every))
    probs = (ctypes.c_void_p * n)(*[ctypes.c_void_p(h.value if isinstance(h, ctypes.c_void_p) else h)
                                    for h in problems])
    Sp = (ctypes.c_void_p * n)(*[_field(p, S, "S").value for p, S in zip(problems, S_list)])
    Jp = (ctypes.c_void_p * n)(*[_field(p, J, "J").value for p, J in zip(problems, J_list)])
    st = (AliStats * n)()
    res = (ctypes.c_int * n)()
    status = load().rt_ali_solve_batch(ctx, probs, n, ctypes.byref(o), Sp, Jp, st, res, _stream(stream))
    _check(status, allow=(RT_OK, RT_NOT_CONVERGED, RT_E_NONFINITE))
    stats = [{"iterations": x.iterations, "bins_converged": x.bins_converged, "max_rel_dS": x.max_rel_dS,
              "seconds": x.seconds} for x in st]
    return status, list(res), stats


# S and J of every unfinished server request, held until its release: the worker
# keeps only the pointers.  server handle value -> {ticket: (S, J)}
_PENDING = {}


def rt_server_create(hbm_budget, check_every=0, ctx=None):
    h = ctypes.c_void_p()
    _check(load().rt_server_create(ctx, int(hbm_budget), int(check_every), ctypes.byref(h)))
    _PENDING[h.value] = {}
    return h


def rt_server_submit(srv, p, S, J, delta_c=1e-6, max_iter=10000, fixed_iters=0, per_bin_stop=True, warm_start=0,
                     check_every=0, stream=None):
    """Queue a solve; the server's stream waits for the work queued on ``stream`` (the
    current stream when None) before the request's first kernel.  S and J are held here
    until rt_server_release."""
    o = AliOpts(float(delta_c), int(max_iter), int(fixed_iters), 1 if per_bin_stop else 0, int(warm_start),
                int(check_every))
    t = ctypes.c_uint64()
    _check(load().rt_server_submit(srv, p, ctypes.byref(o), _field(p, S, "S"), _field(p, J, "J"), _stream(stream),
                                   ctypes.byref(t)))
    _PENDING.setdefault(_hval(srv), {})[t.value] = (S, J)
    return t.value


def rt_server_poll(srv, ticket):
    """None while the request is queued or running, else (result status, stats dict)."""
    st = AliStats()
    res = ctypes.c_int()
    status = load().rt_server_poll(srv, ctypes.c_uint64(ticket), ctypes.byref(st), ctypes.byref(res))
    if status == RT_E_BUSY:
        return None
    _check(status)
    return res.value, {"iterations": st.iterations, "bins_converged": st.bins_converged,
                       "max_rel_dS": st.max_rel_dS, "seconds": st.seconds}


def rt_server_release(srv, ticket):
    st = _check(load().rt_server_release(srv, ctypes.c_uint64(ticket)))
    _PENDING.get(_hval(srv), {}).pop(ticket, None)
    return st


def rt_server_load(srv, with_bytes=False):
    """(queued, running) requests, and with_bytes: also the summed rt_problem_bytes of
    the running ones."""
    q, r, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    _check(load().rt_server_load(srv, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b)))
    return (q.value, r.value, b.value) if with_bytes else (q.value, r.value)


def rt_formal_solve_noalloc(desc, chi, B, S, J, lambda_star=None, stream=None):
    """One formal solution with the library's fixed workspace (no device allocation):
    desc as for a problem, chi, B, S, J (and lambda_star) device FP64 [nf][cells]."""
    nc = int(desc.nx) * int(desc.ny) * int(desc.nz) * int(desc.nf)
    return _check(load().rt_formal_solve_noalloc(ctypes.byref(desc), _dptr(chi, nc, "chi"), _dptr(B, nc, "B"),
                                                 _dptr(S, nc, "S"), _dptr(J, nc, "J"),
                                                 _dptr(lambda_star, nc, "lambda_star"), _stream(stream)))


def rt_server_destroy(srv):
    st = _check(load().rt_server_destroy(srv))   # finishes every request first
    _PENDING.pop(_hval(srv), None)
    return st


def rt_ali_bin_stats(p, nf, stream=None):
    it = np.zeros(nf, dtype=np.int32)
    rs = np.zeros(nf)
    _check(load().rt_ali_bin_stats(p, it.ctypes.data_as(ctypes.c_void_p), rs.ctypes.data_as(ctypes.c_void_p),
                                   _stream(stream)))
    return it, rs


def rt_moments(p, S, J=None, H=None, K=None, J_int=None, H_int=None, K_int=None, f_int=None, Q_int=None,
               want_heating=False, stream=None):
    heat = ctypes.c_double(0.0)
    ptrs = [_field(p, J, "J"), _field(p, H, "H", 3), _field(p, K, "K", 6), _cellfield(p, J_int, "J_int"),
            _cellfield(p, H_int, "H_int", 3), _cellfield(p, K_int, "K_int", 6), _cellfield(p, f_int, "f_int", 6),
            _cellfield(p, Q_int, "Q_int")]
    out = MomentsOut(*[(x.value if x is not None else None) for x in ptrs],
                     ctypes.addressof(heat) if want_heating else None)
    _check(load().rt_moments(p, _field(p, S, "S"), ctypes.byref(out), _stream(stream)))
    return heat.value if want_heating else None


def rt_problem_profile(p, enable=True):
    return _check(load().rt_problem_profile(p, 1 if enable else 0))


def rt_problem_profile_read(p):
    out = Profile()
    _check(load().rt_problem_profile_read(p, ctypes.byref(out)))
    return {"kernel_ms": out.kernel_ms, "launches": out.launches, "sweeps": out.sweeps, "updates": out.updates,
            "stages": out.stages, "chain_ms": out.chain_ms, "chain_launches": out.chain_launches,
            "chain_updates": out.chain_updates}


class Problem:
    """Owner of one ``rt_problem`` handle (marshalling only)."""

    def __init__(self, shape, nf=1, ctx=None, **kw):
        self.shape = tuple(int(x) for x in shape)
        self.nf = int(nf)
        self.desc = make_desc(shape, nf=nf, **kw)
        self.handle = rt_problem_create(self.desc, ctx)
        self.cells = int(np.prod(self.shape))

    def set_fields(self, chi, eps, B, stream=None):
        rt_problem_set_fields(self.handle, chi, eps, B, stream)

    def reset_periodic(self, stream=None):
        rt_problem_reset_periodic(self.handle, stream)

    def state_bytes(self):
        return rt_problem_state_bytes(self.handle)

    def save_state(self, dst=None, stream=None):
        return rt_problem_save_state(self.handle, dst, stream)

    def load_state(self, src, stream=None):
        rt_problem_load_state(self.handle, src, stream)

    def formal_solve(self, S, J, lambda_star=None, stream=None):
        rt_formal_solve(self.handle, S, J, lambda_star, stream)

    def ali_solve(self, S, J, **kw):
        return rt_ali_solve(self.handle, S, J, **kw)

    def ali_solve_gs(self, S, J, **kw):
        return rt_ali_solve(self.handle, S, J, gauss_seidel=True, **kw)

    def use_graphs(self, enable=True):
        _check(load().rt_problem_use_graphs(self.handle, 1 if enable else 0))

    def set_waves(self, waves):
        _check(load().rt_problem_set_waves(self.handle, int(waves)))

    def set_wait_limit(self, microseconds):
        _check(load().rt_problem_set_wait_limit(self.handle, float(microseconds)))

    def tune(self, S, reps=3, stream=None):
        """Time the sweep for every wave count, keep the fastest: (waves, {waves: ms})."""
        best = ctypes.c_int32()
        ms = (ctypes.c_float * 10)(*([-1.0] * 10))
        _check(load().rt_problem_tune(self.handle, _field(self.handle, S, "S"), int(reps), ctypes.byref(best), ms,
                                      _stream(stream)))
        return best.value, {w + 1: ms[w] for w in range(10) if ms[w] >= 0.0}

    def moments(self, S, **kw):
        return rt_moments(self.handle, S, **kw)

    def close(self):
        if self.handle:
            rt_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
