"""Plain FP64 CPU oracle for the short-characteristics radiative transfer hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_1201_2222_amd``: its own angle-set generator,
its own ray geometry and sweep (``rt_oracle.c``), its own Lambda-iteration and
moment steps (this file).

Paper: Davis, Stone & Jiang (2012), arXiv:1201.2222.
  * angle set ........ section 3.2 (n_a = n_mu (n_mu + 2), identical octants)
  * formal solution .. section 3.3, eq. rtdisc, first-order form, the second-order
                       (Bezier) form, and the monotone quadratic upwind intensity
                       with plane-ordered sweeps (``rt_oracle.c``)
  * Jacobi ALI ....... section 3.4, eqs. sourcefunc2 and dsjacobi, criterion eq. conv
  * Gauss-Seidel ALI . section 3.4: the paper's zone order (the backward sweep of
                       Fig. f:sweep, zones updated one at a time from the top corner;
                       ``orc_gs_point_iteration``, ``Problem.ali_gs(ordering="zone")``)
                       and the variant with horizontal planes from the top down as the
                       blocks that the GPU runs (``orc_gs_iteration``,
                       ``ordering="plane"``)
  * boundaries ....... section 3.5 and the periodic iteration of section 3
  * moments .......... eqs. Jsum/Hsum/Ksum, VET f = K/J and Q_rad (section 4)
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt_oracle.c")
_LIB = os.path.join(_HERE, "_rt_oracle.so")

VACUUM, THERMAL, PERIODIC, FIXED = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the C sweep with plain FP64 semantics (no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("nf", ctypes.c_int32), ("na", ctypes.c_int32),
                ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
                ("want_hk", ctypes.c_int32), ("h", ctypes.c_double * 3), ("order", ctypes.c_int32),
                ("interp", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("RTSC_ORACLE_LIB")   # another build of rt_oracle.c (sanitizers)
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.orc_sweep.argtypes = [ctypes.POINTER(_Grid), P, P, P, P, P, P, P, ctypes.c_int, P, P,
                                  P, P, P, P]
        lib.orc_sweep.restype = ctypes.c_int
        lib.orc_coeffs.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        lib.orc_ray_info.argtypes = [P, P, P, P]
        D = ctypes.POINTER(ctypes.c_double)
        lib.orc_bezier_coeffs.argtypes = [ctypes.c_double, D, D, D, D]
        lib.orc_control_point.argtypes = [ctypes.c_double] * 5
        lib.orc_control_point.restype = ctypes.c_double
        lib.orc_quad_interp.argtypes = [ctypes.c_double] * 4
        lib.orc_quad_interp.restype = ctypes.c_double
        lib.orc_gs_iteration.argtypes = [ctypes.POINTER(_Grid), P, P, P, P, P, P, P, P, ctypes.c_int, P, P,
                                         P, P, P]
        lib.orc_gs_iteration.restype = ctypes.c_int
        lib.orc_gs_point_iteration.argtypes = lib.orc_gs_iteration.argtypes
        lib.orc_gs_point_iteration.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Angle set (section 3.2).  The paper takes its rays from Bruls et al. (1999),
# App. B, which is not reproduced in the paper.  This oracle builds the
# level-symmetric set of that family: per octant the directions
# (mu_i, mu_j, mu_k) with i + j + k = n_mu/2 + 2, levels
# mu_i^2 = mu_1^2 + (i-1) * 2 (1 - 3 mu_1^2) / (n_mu - 2), one weight per
# permutation class, and mu_1 and the weights fixed by requiring the even
# moments sum_k w_k mu_x^(2p) = 1/(2p+1) for p = 0, 2, 3, ..., n_mu/2.  For
# n_mu <= 12 the number of classes is n_mu/2 - 1, so these n_mu/2 conditions fix
# the n_mu/2 unknowns -- the paper's statement that the set is unique only for
# n_mu <= 12.
# ---------------------------------------------------------------------------

def _classes(m):
    """Permutation classes (i <= j <= k, i + j + k = m + 2) of the level indices."""
    return [(i, j, k) for i in range(1, m + 1) for j in range(i, m + 1) for k in range(j, m + 1)
            if i + j + k == m + 2]


def _perms(c):
    return sorted(set(itertools.permutations(c)))


def _levels(a, n_mu):
    m = n_mu // 2
    step = 2.0 * (1.0 - 3.0 * a) / (n_mu - 2)
    return np.array([a + i * step for i in range(m)])  # mu_i^2, i = 1..m


def _class_moment(c, p, lev):
    """sum over the class's permutations of mu_x^(2p)"""
    return sum(lev[t[0] - 1] ** p for t in _perms(c))


def _weights_for(a, n_mu):
    m = n_mu // 2
    cls = _classes(m)
    lev = _levels(a, n_mu)
    ps = [0] + list(range(2, m))  # conditions used for the weights
    A = np.array([[_class_moment(c, p, lev) for c in cls] for p in ps], dtype=np.float64)
    rhs = np.array([1.0 / (2 * p + 1) for p in ps])
    try:
        wc = np.linalg.solve(A, rhs)
    except np.linalg.LinAlgError:
        return cls, np.full(len(cls), np.nan), np.nan
    resid = sum(wc[ci] * _class_moment(c, m, lev) for ci, c in enumerate(cls)) - 1.0 / (2 * m + 1)
    return cls, wc, resid


def _solve_mu1sq(n_mu):
    """Smallest mu_1^2 in (0, 1/3) that satisfies the highest moment condition with all
    class weights positive."""
    grid = np.linspace(1e-6, 1.0 / 3.0 - 1e-6, 4001)
    vals = [_weights_for(a, n_mu)[2] for a in grid]
    for lo, hi, flo, fhi in zip(grid[:-1], grid[1:], vals[:-1], vals[1:]):
        if not (np.isfinite(flo) and np.isfinite(fhi)):
            continue
        if flo == 0.0:
            root = lo
        elif flo * fhi < 0.0:
            for _ in range(200):  # bisection to the last bit
                mid = 0.5 * (lo + hi)
                fm = _weights_for(mid, n_mu)[2]
                if fm == 0.0 or mid in (lo, hi):
                    break
                if (fm < 0.0) == (flo < 0.0):
                    lo, flo = mid, fm
                else:
                    hi = mid
            root = mid
        else:
            continue
        if np.all(_weights_for(root, n_mu)[1] > 0.0):
            return root
    raise ValueError(f"no level-symmetric set with positive weights for n_mu={n_mu}")


def quadrature(n_mu: int):
    """Return (mu [na,3], w [na]) with sum(w) = 1, octant-major.

    Octant o has signs (-1)^(o&1), (-1)^((o>>1)&1), (-1)^((o>>2)&1) for x, y, z; within an
    octant the directions follow the lexicographic order of their level-index triples."""
    if n_mu == 2:
        pts = [((1, 1, 1), 1.0)]
        lev = np.array([1.0 / 3.0])
    elif n_mu in (4, 6, 8, 10, 12):
        a = _solve_mu1sq(n_mu)
        cls, wc, _ = _weights_for(a, n_mu)
        lev = _levels(a, n_mu)
        pts = []
        for ci, c in enumerate(cls):
            for t in _perms(c):
                pts.append((t, wc[ci]))
        pts.sort(key=lambda pw: pw[0])
    else:
        raise ValueError("n_mu must be one of 2, 4, 6, 8, 10, 12")
    mu_oct = np.array([[np.sqrt(lev[t[0] - 1]), np.sqrt(lev[t[1] - 1]), np.sqrt(lev[t[2] - 1])]
                       for t, _ in pts])
    w_oct = np.array([wt for _, wt in pts])
    mus, ws = [], []
    for o in range(8):
        sg = np.array([-1.0 if (o >> q) & 1 else 1.0 for q in range(3)])
        mus.append(mu_oct * sg)
        ws.append(w_oct / 8.0)
    return np.concatenate(mus), np.concatenate(ws)


# ---------------------------------------------------------------------------
# Small exported pieces of the C sweep, for pinning
# ---------------------------------------------------------------------------

def coeffs(dt: float):
    """(E, psi_minus, psi_0) of the first-order segment integration (section 3.3)."""
    lib = _load()
    E, pm, p0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.orc_coeffs(float(dt), ctypes.byref(E), ctypes.byref(pm), ctypes.byref(p0))
    return E.value, pm.value, p0.value


def bezier_coeffs(dt: float):
    """(E, alpha, beta, gamma) of the second-order Bezier segment integration."""
    lib = _load()
    v = [ctypes.c_double() for _ in range(4)]
    lib.orc_bezier_coeffs(float(dt), *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v)


def control_point(Sm, S0, Sp, h1, h2):
    """Clamped Bezier control point of the source function at the vertex."""
    return _load().orc_control_point(float(Sm), float(S0), float(Sp), float(h1), float(h2))


def quad_interp(fm, f0, f1, t):
    """Monotone quadratic interpolant between f0 (t = 0) and f1 (t = 1) with the third
    point fm at t = -1 (upwind intensity of the quadratic scheme)."""
    return _load().orc_quad_interp(float(fm), float(f0), float(f1), float(t))


def ray_info(mu, h=(1.0, 1.0, 1.0)):
    """(d, a, b, signs, s, fa, fb) of the short characteristic of one ray."""
    lib = _load()
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    io = np.zeros(6, dtype=np.int32)
    do = np.zeros(3, dtype=np.float64)
    lib.orc_ray_info(_ptr(mu), _ptr(h), _ptr(io), _ptr(do))
    return int(io[0]), int(io[1]), int(io[2]), tuple(int(x) for x in io[3:6]), do[0], do[1], do[2]


# ---------------------------------------------------------------------------
# Problem: fields + periodic memory, formal solution, Jacobi ALI, moments
# ---------------------------------------------------------------------------

class Problem:
    """One radiative transfer problem on an nx*ny*nz grid with nf bins.

    Arrays use the layout [nf][nz][ny][nx] (x fastest).  ``chi`` is the total
    opacity chi_abs + chi_sc, ``eps`` the photon destruction probability
    chi_abs/chi_tot and ``B`` the thermal source function (section 2, eq.
    sourcefunc).  ``bc_lo``/``bc_hi`` give VACUUM, THERMAL, PERIODIC or FIXED per axis
    (x, y, z); periodic axes must be periodic on both sides."""

    def __init__(self, shape, chi, eps, B, n_mu=4, mu=None, w=None, h=(1.0, 1.0, 1.0),
                 bc_lo=(PERIODIC, PERIODIC, THERMAL), bc_hi=(PERIODIC, PERIODIC, VACUUM),
                 w_nu=None, fixed=None, order=0, interp=0):
        nx, ny, nz = shape
        if order not in (0, 1):
            raise ValueError("order is 0 (first order) or 1 (second order, Bezier)")
        if interp not in (0, 1):
            raise ValueError("interp is 0 (bilinear I-) or 1 (monotone quadratic I-)")
        if interp == 1 and order != 0:
            raise ValueError("the quadratic upwind intensity is built with first-order segments only")
        self.order = int(order)
        self.interp = int(interp)
        self.n = (int(nx), int(ny), int(nz))
        chi = np.asarray(chi, dtype=np.float64)
        self.nf = chi.size // (nx * ny * nz)
        fs = (self.nf, nz, ny, nx)
        self.chi = np.ascontiguousarray(chi.reshape(fs))
        eps = np.asarray(eps, dtype=np.float64)
        self.eps = np.ascontiguousarray(np.broadcast_to(eps if eps.ndim == 0 else eps.reshape(fs), fs))
        self.B = np.ascontiguousarray(np.asarray(B, dtype=np.float64).reshape(fs))
        if mu is None:
            mu, w = quadrature(n_mu)
        self.mu = np.ascontiguousarray(mu, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.na = len(self.w)
        self.h = tuple(float(x) for x in h)
        self.bc_lo, self.bc_hi = tuple(bc_lo), tuple(bc_hi)
        for q in range(3):
            if (self.bc_lo[q] == PERIODIC) != (self.bc_hi[q] == PERIODIC):
                raise ValueError("a periodic axis must be periodic on both faces")
        self.w_nu = np.ones(self.nf) if w_nu is None else np.asarray(w_nu, dtype=np.float64)
        self._fixed = [None] * 6
        if fixed is not None:
            for i, a in enumerate(fixed):
                if a is not None:
                    self._fixed[i] = np.ascontiguousarray(a, dtype=np.float64)
        for q in range(3):
            for hi in range(2):
                kind = (self.bc_hi if hi else self.bc_lo)[q]
                if kind == FIXED and self._fixed[2 * q + hi] is None:
                    raise ValueError("FIXED face without an intensity array")
        self.reset_periodic()

    # -- periodic memory (one plane per periodic axis and ray) -----------------
    def _plane(self, q):
        nx, ny, nz = self.n
        return {0: ny * nz, 1: nx * nz, 2: nx * ny}[q]

    def reset_periodic(self):
        """Forget the previous sweep: periodic ghosts fall back to S (cold start)."""
        self.have_prev = 0
        self.prev = [np.zeros((self.nf, self.na, self._plane(q))) if self.bc_lo[q] == PERIODIC else None
                     for q in range(3)]

    def seed_periodic(self, planes):
        """Set the periodic memory explicitly: ``planes[q]`` is [nf][na][plane] or None."""
        for q in range(3):
            if self.prev[q] is not None:
                self.prev[q][...] = np.asarray(planes[q]).reshape(self.prev[q].shape)
        self.have_prev = 1

    # -- one formal solution ---------------------------------------------------
    def _grid(self, want_hk=False):
        g = _Grid()
        g.n[:] = list(self.n)
        g.nf, g.na = self.nf, self.na
        g.bc_lo[:] = list(self.bc_lo)
        g.bc_hi[:] = list(self.bc_hi)
        g.want_hk = 1 if want_hk else 0
        g.h[:] = list(self.h)
        g.order = self.order
        g.interp = self.interp
        return g

    def sweep(self, S, want_hk=False, bin_active=None):
        """J = Lambda[S] for every bin (plus H, K and the diagonal Lambda*).

        Periodic ghosts come from the previous sweep of this problem (or from S
        before the first one); afterwards the memory holds this sweep's planes."""
        lib = _load()
        S = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(self.chi.shape))
        g = self._grid(want_hk)
        shp = self.chi.shape
        J = np.zeros(shp)
        lam = np.zeros(shp)
        H = np.zeros((3,) + shp) if want_hk else None
        K = np.zeros((6,) + shp) if want_hk else None
        fixed = (ctypes.c_void_p * 6)(*[a.ctypes.data if a is not None else None for a in self._fixed])
        prev_in = (ctypes.c_void_p * 3)(*[a.ctypes.data if a is not None else None for a in self.prev])
        new = [np.zeros_like(a) if a is not None else None for a in self.prev]
        if bin_active is not None:
            for q in range(3):
                if new[q] is not None:
                    new[q][...] = self.prev[q]
        prev_out = (ctypes.c_void_p * 3)(*[a.ctypes.data if a is not None else None for a in new])
        act = None if bin_active is None else np.ascontiguousarray(bin_active, dtype=np.int32)
        rc = lib.orc_sweep(ctypes.byref(g), _ptr(self.mu), _ptr(self.w), _ptr(self.chi), _ptr(self.B),
                           _ptr(S), fixed, prev_in, int(self.have_prev), prev_out, _ptr(act),
                           _ptr(J), _ptr(H), _ptr(K), _ptr(lam))
        if rc != 0:
            raise MemoryError("oracle sweep ran out of memory")
        self.prev = new
        self.have_prev = 1
        return {"J": J, "H": H, "K": K, "lam": lam}

    def formal_solve(self, S, want_hk=False, converge_periodic=None, max_sweeps=10000):
        """One sweep; with ``converge_periodic=delta`` repeat sweeps on the same S
        until max |Delta J|/J <= delta (the LTE form of eq. conv), which iterates the
        lagged periodic ghosts to convergence (section 3)."""
        out = self.sweep(S, want_hk=want_hk)
        out["sweeps"] = 1
        if converge_periodic is None:
            return out
        for extra in range(max_sweeps - 1):
            J_old = out["J"]
            out = self.sweep(S, want_hk=want_hk)
            out["sweeps"] = extra + 2
            m = J_old != 0.0
            r = np.max(np.abs(out["J"][m] - J_old[m]) / np.abs(J_old[m])) if m.any() else 0.0
            if r <= converge_periodic:
                break
        return out

    def ali(self, delta_c=1e-6, max_iter=10000, fixed_iters=0, S0=None, J_prev=None,
            per_bin_stop=True):
        """Jacobi accelerated Lambda iteration with the diagonal Lambda* (section 3.4).

        Start: S0 = B (cold, the J = B start of section 5.1), or the given S0, or
        S0 = eps B + (1-eps) J_prev (warm start from a previous J, section 4).
        Iteration n:  J^n = Lambda[S^n];
            Delta S = ((1-eps) J^n + eps B - S^n) / (1 - (1-eps) Lambda*)   (eq. dsjacobi)
            S^{n+1} = S^n + Delta S;  r = max |Delta S| / S^{n+1}  (eq. conv, per bin)
        A bin stops once r <= delta_c (all bins together when per_bin_stop is
        false).  ``fixed_iters > 0`` runs exactly that many iterations.
        Returns S^{n+1}, J^n of each bin's last iteration, iteration counts, residuals."""
        eps, B = self.eps, self.B
        if S0 is not None:
            S = np.array(S0, dtype=np.float64).reshape(B.shape)
        elif J_prev is not None:
            S = eps * B + (1.0 - eps) * np.asarray(J_prev, dtype=np.float64).reshape(B.shape)
        else:
            S = B.copy()
        nf = self.nf
        active = np.ones(nf, dtype=bool)
        iters = np.zeros(nf, dtype=np.int64)
        resid = np.full(nf, np.inf)
        J = np.zeros_like(S)
        lam = None
        n_total = fixed_iters if fixed_iters > 0 else max_iter
        for n in range(n_total):
            out = self.sweep(S, bin_active=active.astype(np.int32))
            if lam is None:
                lam = out["lam"].copy()
            for f in np.nonzero(active)[0]:
                Jn = out["J"][f]
                dS = ((1.0 - eps[f]) * Jn + eps[f] * B[f] - S[f]) / (1.0 - (1.0 - eps[f]) * lam[f])
                Snew = S[f] + dS
                m = Snew != 0.0
                r = float(np.max(np.abs(dS[m]) / np.abs(Snew[m]))) if m.any() else 0.0
                S[f] = Snew
                J[f] = Jn
                iters[f] = n + 1
                resid[f] = r
            if fixed_iters > 0:
                continue
            conv = resid <= delta_c
            if per_bin_stop:
                active &= ~conv
                if not active.any():
                    break
            elif conv[active].all():
                break
        converged = bool(np.all(resid <= delta_c))
        return {"S": S, "J": J, "iters": iters, "resid": resid, "lam": lam, "converged": converged}

    def gs_iteration(self, S, bin_active=None, ordering="plane"):
        """One Gauss-Seidel iteration (section 3.4): returns S^{n+1}, the J each vertex
        was updated with, Lambda* and the update dS.

        ordering="zone": the paper's order, zones updated one at a time in the
        backward sweep of Fig. f:sweep (from the top corner, i fastest), each with J
        from the current S (orc_gs_point_iteration).  ordering="plane": horizontal
        planes from the top down as the blocks, Jacobi inside a plane (the variant the
        GPU runs; orc_gs_iteration).  Periodic ghosts read this problem's memory (S at
        the iteration's start before any sweep); afterwards the memory holds the
        iteration's outgoing planes."""
        if ordering not in ("plane", "zone"):
            raise ValueError("ordering is 'zone' (the paper's) or 'plane' (horizontal planes as blocks)")
        if self.order != 0 or self.interp != 0:
            raise ValueError("Gauss-Seidel is built with first-order segments and bilinear I- only")
        if self.bc_lo[2] == PERIODIC:
            raise ValueError("Gauss-Seidel orders the planes along a non-periodic z axis")
        lib = _load()
        shp = self.chi.shape
        S = np.array(np.asarray(S, dtype=np.float64).reshape(shp), order="C")
        J = np.zeros(shp)
        lam = np.zeros(shp)
        dS = np.zeros(shp)
        fixed = (ctypes.c_void_p * 6)(*[a.ctypes.data if a is not None else None for a in self._fixed])
        prev_in = (ctypes.c_void_p * 3)(*[a.ctypes.data if a is not None else None for a in self.prev])
        new = [a.copy() if a is not None else None for a in self.prev]
        prev_out = (ctypes.c_void_p * 3)(*[a.ctypes.data if a is not None else None for a in new])
        act = None if bin_active is None else np.ascontiguousarray(bin_active, dtype=np.int32)
        fn = lib.orc_gs_point_iteration if ordering == "zone" else lib.orc_gs_iteration
        rc = fn(ctypes.byref(self._grid()), _ptr(self.mu), _ptr(self.w), _ptr(self.chi),
                _ptr(self.B), _ptr(self.eps), _ptr(S), fixed, prev_in, int(self.have_prev),
                prev_out, _ptr(act), _ptr(J), _ptr(lam), _ptr(dS))
        if rc == -1:
            raise MemoryError("oracle Gauss-Seidel iteration ran out of memory")
        if rc != 0:
            raise ValueError("unsupported problem for the Gauss-Seidel iteration")
        self.prev = new
        self.have_prev = 1
        return {"S": S, "J": J, "lam": lam, "dS": dS}

    def ali_gs(self, delta_c=1e-6, max_iter=10000, fixed_iters=0, S0=None, J_prev=None, per_bin_stop=True,
               ordering="plane"):
        """Gauss-Seidel accelerated Lambda iteration (section 3.4): as ``ali`` with
        each iteration a Gauss-Seidel pass (gs_iteration with the given ordering:
        "zone", the paper's, or "plane", the GPU's blocks).  r = max |dS| / S^{n+1} per
        bin (eq. conv); J is the J of each bin's last iteration."""
        eps, B = self.eps, self.B
        if S0 is not None:
            S = np.array(S0, dtype=np.float64).reshape(B.shape)
        elif J_prev is not None:
            S = eps * B + (1.0 - eps) * np.asarray(J_prev, dtype=np.float64).reshape(B.shape)
        else:
            S = B.copy()
        nf = self.nf
        active = np.ones(nf, dtype=bool)
        iters = np.zeros(nf, dtype=np.int64)
        resid = np.full(nf, np.inf)
        J = np.zeros_like(S)
        lam = None
        n_total = fixed_iters if fixed_iters > 0 else max_iter
        for n in range(n_total):
            out = self.gs_iteration(S, bin_active=active.astype(np.int32), ordering=ordering)
            if lam is None:
                lam = out["lam"].copy()
            for f in np.nonzero(active)[0]:
                Snew = out["S"][f]
                dS = out["dS"][f]
                m = Snew != 0.0
                r = float(np.max(np.abs(dS[m]) / np.abs(Snew[m]))) if m.any() else 0.0
                S[f] = Snew
                J[f] = out["J"][f]
                iters[f] = n + 1
                resid[f] = r
            if fixed_iters > 0:
                continue
            conv = resid <= delta_c
            if per_bin_stop:
                active &= ~conv
                if not active.any():
                    break
            elif conv[active].all():
                break
        converged = bool(np.all(resid <= delta_c))
        return {"S": S, "J": J, "iters": iters, "resid": resid, "lam": lam, "converged": converged}

    def moments(self, S, converge_periodic=None):
        """Moments epilogue (section 3.2 eqs. Jsum/Hsum/Ksum, section 4):
        per bin J, H, K; f = K/J; Q_int = 4 pi eps chi (J - B); Q_dif = -4 pi div H;
        Q = Q_int where chi dx_min <= 1 else Q_dif; frequency-integrated
        sum_nu w_nu X_nu; heating = sum over cells of Q dV."""
        out = self.formal_solve(S, want_hk=True, converge_periodic=converge_periodic)
        return moments_from(self, out["J"], out["H"], out["K"])


def divergence(H, h, periodic):
    """Second-order differences of a [3][nz][ny][nx] field: central inside, wrapped on
    periodic axes, second-order one-sided at other faces (two-point with only two
    cells, zero with one)."""
    div = np.zeros(H.shape[1:])
    for q in range(3):
        ax = 2 - q  # array axis of coordinate q in [nz][ny][nx]
        F = H[q]
        n = F.shape[ax]
        if n == 1:
            continue
        if periodic[q]:
            d = (np.roll(F, -1, axis=ax) - np.roll(F, 1, axis=ax)) / (2.0 * h[q])
        else:
            d = np.empty_like(F)
            sl = lambda a, b: tuple(slice(a, b) if i == ax else slice(None) for i in range(3))
            if n >= 3:
                d[sl(1, n - 1)] = (F[sl(2, n)] - F[sl(0, n - 2)]) / (2.0 * h[q])
                d[sl(0, 1)] = (-3.0 * F[sl(0, 1)] + 4.0 * F[sl(1, 2)] - F[sl(2, 3)]) / (2.0 * h[q])
                d[sl(n - 1, n)] = (3.0 * F[sl(n - 1, n)] - 4.0 * F[sl(n - 2, n - 1)]
                                   + F[sl(n - 3, n - 2)]) / (2.0 * h[q])
            else:
                d[...] = (F[sl(1, 2)] - F[sl(0, 1)]) / h[q]
        div += d
    return div


def moments_from(p: Problem, J, H, K):
    fourpi = 4.0 * np.pi
    periodic = [p.bc_lo[q] == PERIODIC for q in range(3)]
    hmin = min(p.h)
    Q = np.zeros_like(J)
    for f in range(p.nf):
        q_int = fourpi * p.eps[f] * p.chi[f] * (J[f] - p.B[f])
        q_dif = -fourpi * divergence(H[:, f], p.h, periodic)
        Q[f] = np.where(p.chi[f] * hmin <= 1.0, q_int, q_dif)
    wn = p.w_nu
    Jt = np.tensordot(wn, J, axes=(0, 0))
    Ht = np.tensordot(wn, H, axes=(0, 1))
    Kt = np.tensordot(wn, K, axes=(0, 1))
    Qt = np.tensordot(wn, Q, axes=(0, 0))
    with np.errstate(divide="ignore", invalid="ignore"):
        ft = np.where(Jt != 0.0, Kt / Jt, 0.0)
    dV = p.h[0] * p.h[1] * p.h[2]
    heating = float(np.sum(Qt) * dV)
    return {"J": J, "H": H, "K": K, "Q": Q, "J_int": Jt, "H_int": Ht, "K_int": Kt,
            "f_int": ft, "Q_int": Qt, "heating": heating}
