"""CPU FP64 oracle for the AdS4 Einstein-Klein-Gordon method of lines.

TEST INFRASTRUCTURE ONLY.  This package wraps ``liboracle.so`` (plain sequential
C, see ``adscl_oracle.c``) with numpy.  Only ``tests/``, the package smoke check
and the CPU-baseline leg of ``bench.py`` may import it.  The product library
(``paper_1706_07413_amd``) never imports it and shares no code with it.

All arrays are float64; one instance at a time.  Citations refer to Liebling &
Khanna, arXiv:1706.07413 (Sec. II equations numbered as in the paper).
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

GAUGE_BOUNDARY = 0
GAUGE_ORIGIN = 1
RUNNING, COLLAPSED, NONFINITE, DONE = 0, 1, 2, 3

_d = ctypes.c_double
_i = ctypes.c_int
_i64 = ctypes.c_int64
_p = ctypes.POINTER(ctypes.c_double)


_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_BATCH_SIG = {
    "ora_threads": (_i, []),
    "ora_evolve_gaussian_batch": (None, [_i, _i32p, _p, _p, _i, _d, _d, _d, _i64p, _i64p, _i32p]),
    "ora_objective_batch": (None, [_i, _i32p, _i, _d, _d, _d, _p, _i, _p, _i, _i64p, _i64, _p, _p, _i32p]),
}


_SIG = {
    "ora_tables": (None, [_i, _p, _p, _p, _p, _p]),
    "ora_op_D": (None, [_i, _d, _p, _i, _i, _p]),
    "ora_op_KO": (None, [_i, _d, _d, _p, _i, _i, _p]),
    "ora_op_cell4": (None, [_i, _d, _p, _i, _i, _p]),
    "ora_constraints": (None, [_i, _i, _p, _p, _p, _p, _p, _p]),
    "ora_rhs": (None, [_i, _d, _i, _p, _p, _p, _p, _p, _p]),
    "ora_evolve": (_i, [_i, _i, _i, _d, _d, _d, _p, _p, _i64, _i64, ctypes.c_int32, _i64, _p,
                        _p, _p, _p, ctypes.POINTER(_i64), _p, _p]),
    "ora_evolve_scheme": (_i, [_i, _i, _i, _d, _d, _d, _i, _i, _p, _p, _p, _i64, _i64, ctypes.c_int32, _i64,
                               _p, _p, _p, ctypes.POINTER(_i64), _p, _p]),
    "ora_mass_paper": (_d, [_i, _p, _p, _p]),
    "ora_residuals": (None, [_i, _p, _p, _p, _p, _p, _p]),
    "ora_adot_residual": (None, [_i, _i, _d, _p, _p, _p, _p]),
    "ora_jacobi": (_d, [_i, _d, _d, _d]),
    "ora_modes": (None, [_i, _i, _p, _p]),
    "ora_spectrum": (None, [_i, _i, _p, _p, _p, _p, _p, _p]),
    "ora_init_gaussian": (None, [_i, _d, _d, _p, _p]),
    "ora_init_modes": (None, [_i, _d, _i, _p, _p, _p]),
    "ora_objective": (_i, [_i, _i, _d, _d, _d, _d, _i, _p, _i, _i64, _i64, _p, _p, _p, _p]),
    "ora_constraints_vjp": (None, [_i, _i, _p, _p, _p, _p, _p, _p]),
    "ora_rhs_vjp": (None, [_i, _d, _i, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]),
    "ora_step": (None, [_i, _i, _d, _d, _p, _p]),
    "ora_step_vjp": (None, [_i, _i, _d, _d, _p, _p, _p, _p]),
    "ora_spectrum_vjp": (None, [_i, _i, _p, _p, _p, _p, _p, _p, _p]),
}


def _bind(lib, sig):
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: F401  (build on first use in a checkout)
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    _bind(lib, _BATCH_SIG)
    _bind(lib, _SIG)
    _lib = lib
    return lib


def load_library(path):
    """Another build of the oracle's sources at `path` (say with other compiler
    flags), with every function bound; pass it as ``lib=`` to :func:`evolve`."""
    lib = ctypes.CDLL(path)
    _bind(lib, _BATCH_SIG)
    _bind(lib, _SIG)
    return lib


def _ptr(a):
    return a.ctypes.data_as(_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def grid(N):
    """x_i = i h, h = (pi/2)/(N-1)."""
    h = (math.pi / 2) / (N - 1)
    return np.arange(N) * h, h


def dt_of(N, cfl=0.25):
    return cfl * (math.pi / 2) / (N - 1)


def n_steps_for(T, N, cfl=0.25):
    """Number of steps to reach t >= T: ceil(T/dt - 1e-9); t_n = n dt is not clamped."""
    return int(math.ceil(T / dt_of(N, cfl) - 1e-9))


def tables(N):
    lib = _load()
    out = [np.empty(N) for _ in range(5)]
    lib.ora_tables(N, *[_ptr(o) for o in out])
    return dict(zip(["x", "sc", "t2", "ct2", "c3s"], out))


def op_D(u, h, p0, p1):
    lib = _load()
    u = _f64(u)
    out = np.empty_like(u)
    lib.ora_op_D(len(u), h, _ptr(u), p0, p1, _ptr(out))
    return out


def op_KO(u, h, sig, p0, p1):
    lib = _load()
    u = _f64(u)
    out = np.empty_like(u)
    lib.ora_op_KO(len(u), h, sig, _ptr(u), p0, p1, _ptr(out))
    return out


def op_cell4(u, h, p0, p1):
    lib = _load()
    u = _f64(u)
    out = np.empty(len(u) - 1)
    lib.ora_op_cell4(len(u), h, _ptr(u), p0, p1, _ptr(out))
    return out


def constraints(Phi, Pi, gauge=GAUGE_BOUNDARY):
    """Solve Eqs. (5)-(6) for one state; returns dict A, delta, m, dtil."""
    lib = _load()
    Phi, Pi = _f64(Phi), _f64(Pi)
    N = len(Phi)
    A, delta, m, dtil = (np.empty(N) for _ in range(4))
    lib.ora_constraints(N, gauge, _ptr(Phi), _ptr(Pi), _ptr(A), _ptr(delta), _ptr(m), _ptr(dtil))
    return dict(A=A, delta=delta, m=m, dtil=dtil)


def rhs(Phi, Pi, A, delta, ko=0.5, frozen=False):
    lib = _load()
    Phi, Pi, A, delta = map(_f64, (Phi, Pi, A, delta))
    N = len(Phi)
    dPhi, dPi = np.empty(N), np.empty(N)
    lib.ora_rhs(N, ko, int(frozen), _ptr(Phi), _ptr(Pi), _ptr(A), _ptr(delta), _ptr(dPhi), _ptr(dPi))
    return dPhi, dPi


def evolve(Phi, Pi, n_stop, n0=0, gauge=GAUGE_BOUNDARY, frozen=False, cfl=0.25, ko=0.5,
           a_collapse=0.0, snap_every=0, n_slots=0, n_final=None, lib=None):
    """Evolve one instance from step n0 to n_stop (classical RK4, dt = cfl h).

    Returns dict with Phi, Pi (state U^n at exit), A, delta, m (its metric),
    steps (n at exit), state, minA, t, t_c and snaps [n_slots, 5, N] when
    snap_every > 0.  State is DONE when n reaches ``n_final`` (default n_stop).
    ``lib``: another build of the sources (:func:`load_library`).
    """
    lib = lib or _load()
    Phi, Pi = _f64(Phi).copy(), _f64(Pi).copy()
    N = len(Phi)
    A, delta, m = np.empty(N), np.empty(N), np.empty(N)
    snaps = np.zeros((max(n_slots, 1), 5, N))
    n_out = _i64(0)
    minA, tc = _d(0), _d(0)
    st = lib.ora_evolve(N, gauge, int(frozen), cfl, ko, a_collapse, _ptr(Phi), _ptr(Pi),
                        n0, n_stop, snap_every, n_slots, _ptr(snaps), _ptr(A), _ptr(delta), _ptr(m),
                        ctypes.byref(n_out), ctypes.byref(minA), ctypes.byref(tc))
    n_final = n_stop if n_final is None else n_final
    if st == RUNNING and n_out.value >= n_final:
        st = DONE
    dt = dt_of(N, cfl)
    return dict(Phi=Phi, Pi=Pi, A=A, delta=delta, m=m, steps=n_out.value, state=st,
                minA=minA.value, t=n_out.value * dt, t_c=tc.value,
                snaps=snaps[:n_slots] if n_slots > 0 else None)


def evolve_scheme(Phi, Pi, n_stop, rk=4, a_reint=0, A=None, n0=0, gauge=GAUGE_BOUNDARY, frozen=False, cfl=0.25,
                  ko=0.5, a_collapse=0.0, snap_every=0, n_slots=0, n_final=None):
    """``evolve`` with the scheme options of Sec. II: Runge-Kutta order ``rk``
    (2 and 3: the Shu-Osher SSP methods; 4: classical) and ``a_reint`` (0: A
    from Eq. (5) at every stage; K >= 1: A evolved with Eq. (4) and replaced
    by Eq. (5)'s at every step that is a multiple of K).  ``A``: the state's
    evolved A at n0 (needed only when A is evolved and n0 is not a multiple of
    K).  Returns the dict of ``evolve`` (A the state's A)."""
    lib = _load()
    Phi, Pi = _f64(Phi).copy(), _f64(Pi).copy()
    N = len(Phi)
    A = np.ones(N) if A is None else _f64(A).copy()
    delta, m = np.empty(N), np.empty(N)
    snaps = np.zeros((max(n_slots, 1), 5, N))
    n_out = _i64(0)
    minA, tc = _d(0), _d(0)
    st = lib.ora_evolve_scheme(N, gauge, int(frozen), cfl, ko, a_collapse, int(rk), int(a_reint), _ptr(Phi), _ptr(Pi),
                               _ptr(A), n0, n_stop, snap_every, n_slots, _ptr(snaps), _ptr(delta), _ptr(m),
                               ctypes.byref(n_out), ctypes.byref(minA), ctypes.byref(tc))
    if st < 0:
        raise ValueError("invalid scheme option")
    n_final = n_stop if n_final is None else n_final
    if st == RUNNING and n_out.value >= n_final:
        st = DONE
    return dict(Phi=Phi, Pi=Pi, A=A, delta=delta, m=m, steps=n_out.value, state=st, minA=minA.value,
                t=n_out.value * dt_of(N, cfl), t_c=tc.value, snaps=snaps[:n_slots] if n_slots > 0 else None)


def mass_paper(Phi, Pi, A):
    lib = _load()
    Phi, Pi, A = map(_f64, (Phi, Pi, A))
    return lib.ora_mass_paper(len(Phi), _ptr(Phi), _ptr(Pi), _ptr(A))


def residuals(Phi, Pi, A, delta):
    lib = _load()
    Phi, Pi, A, delta = map(_f64, (Phi, Pi, A, delta))
    N = len(Phi)
    RA, Rd = np.empty(N), np.empty(N)
    lib.ora_residuals(N, _ptr(Phi), _ptr(Pi), _ptr(A), _ptr(delta), _ptr(RA), _ptr(Rd))
    return RA, Rd


def adot_residual(Phi, Pi, gauge=GAUGE_BOUNDARY, ko=0.5):
    """Eq. (4) residual of one state: the metric is solved from (Phi, Pi), A_t is
    the derivative of that solve along the right-hand sides (Phi_t, Pi_t).
    Returns (Adot, R), R = A_t + 2 sin x cos x A^2 e^-delta Phi Pi (0 at the ends)."""
    lib = _load()
    Phi, Pi = _f64(Phi), _f64(Pi)
    N = len(Phi)
    Ad, R = np.empty(N), np.empty(N)
    lib.ora_adot_residual(N, gauge, ko, _ptr(Phi), _ptr(Pi), _ptr(Ad), _ptr(R))
    return Ad, R


def jacobi(n, a, b, z):
    return _load().ora_jacobi(n, a, b, z)


def modes(N, J):
    lib = _load()
    e, de = np.empty((J, N)), np.empty((J, N))
    lib.ora_modes(N, J, _ptr(e), _ptr(de))
    return e, de


def spectrum(Phi, Pi, A, J):
    lib = _load()
    Phi, Pi, A = map(_f64, (Phi, Pi, A))
    N = len(Phi)
    E, Ph, Fh = np.empty(J), np.empty(J), np.empty(J)
    lib.ora_spectrum(N, J, _ptr(Phi), _ptr(Pi), _ptr(A), _ptr(E), _ptr(Ph), _ptr(Fh))
    return E, Ph, Fh


def init_gaussian(N, eps, sigma):
    lib = _load()
    Phi, Pi = np.empty(N), np.empty(N)
    lib.ora_init_gaussian(N, eps, sigma, _ptr(Phi), _ptr(Pi))
    return Phi, Pi


def init_modes(N, eps, c):
    lib = _load()
    c = _f64(c)
    Phi, Pi = np.empty(N), np.empty(N)
    lib.ora_init_modes(N, eps, len(c), _ptr(c), _ptr(Phi), _ptr(Pi))
    return Phi, Pi


# ---------------------------------------------------------------------------
# Batches: independent instances over the host's cores (adscl_oracle_batch.c)
# ---------------------------------------------------------------------------

def timing_lib(path):
    """The -O3 -march=native timing build at `path` (see build.build_timing),
    with the batch drivers bound; pass it as ``lib=`` to the batch functions."""
    lib = ctypes.CDLL(path)
    _bind(lib, _BATCH_SIG)
    return lib


def threads(lib=None):
    """OpenMP threads the batch drivers of `lib` (default: the parity build) use."""
    return (lib or _load()).ora_threads()


def evolve_gaussian_batch(Ns, eps, sigma, n_stop, gauge=GAUGE_BOUNDARY, cfl=0.25, ko=0.5, a_collapse=0.0,
                          lib=None):
    """Gaussian data for every instance evolved to n_stop[b] steps or collapse,
    one instance per thread; returns (steps, state) arrays."""
    L = lib or _load()
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    n = len(Ns)
    eps, sigma = _f64(eps), _f64(sigma)
    ns = np.ascontiguousarray(np.broadcast_to(np.asarray(n_stop, np.int64), (n,)))
    steps = np.zeros(n, np.int64)
    state = np.zeros(n, np.int32)
    L.ora_evolve_gaussian_batch(n, Ns.ctypes.data_as(_i32p), _ptr(eps), _ptr(sigma), gauge, cfl, ko, a_collapse,
                                ns.ctypes.data_as(_i64p), steps.ctypes.data_as(_i64p), state.ctypes.data_as(_i32p))
    return steps, state


def objective_batch(Ns, eps, c, J, n_steps, K, gauge=GAUGE_BOUNDARY, cfl=0.25, ko=0.5, a_collapse=0.0, lib=None):
    """``objective`` for every instance, one instance per thread; returns
    (L [n], grad [n, Jc], valid [n])."""
    L_ = lib or _load()
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    n = len(Ns)
    c = np.ascontiguousarray(c, dtype=np.float64)
    eps = _f64(eps)
    ns = np.ascontiguousarray(np.broadcast_to(np.asarray(n_steps, np.int64), (n,)))
    Lv, g = np.zeros(n), np.zeros((n, c.shape[1]))
    valid = np.zeros(n, np.int32)
    L_.ora_objective_batch(n, Ns.ctypes.data_as(_i32p), gauge, cfl, ko, a_collapse, _ptr(eps), c.shape[1], _ptr(c),
                           int(J), ns.ctypes.data_as(_i64p), int(K), _ptr(Lv), _ptr(g), valid.ctypes.data_as(_i32p))
    return Lv, g, valid


# ---------------------------------------------------------------------------
# Reverse-mode derivative (adscl_oracle_adj.c)
# ---------------------------------------------------------------------------

def objective(N, eps, c, T=None, n_steps=None, J=16, K=512, gauge=GAUGE_BOUNDARY, cfl=0.25, ko=0.5,
              a_collapse=0.0, grad=True):
    """L = sum_{j<J} (E_j(t_n) - E_j(0))^2 for Pi(x,0) = eps sum_k c_k e_k(x),
    Phi(x,0) = 0, and dL/dc by the discrete adjoint with checkpoints every K
    steps.  Returns dict L, grad (None if not asked or invalid), valid, E0, ET."""
    lib = _load()
    c = _f64(c)
    if n_steps is None:
        n_steps = n_steps_for(T, N, cfl)
    Lv = _d(0)
    g = np.zeros(len(c))
    E0, ET = np.zeros(J), np.zeros(J)
    valid = lib.ora_objective(N, gauge, cfl, ko, a_collapse, eps, len(c), _ptr(c), J, int(n_steps), int(K),
                              ctypes.byref(Lv), _ptr(g) if grad else None, _ptr(E0), _ptr(ET))
    return dict(L=Lv.value, grad=(g if (grad and valid) else None), valid=bool(valid), E0=E0, ET=ET,
                n_steps=int(n_steps))


def descend(Ns, eps, c, J, T, K, iters, step0, gauge=GAUGE_BOUNDARY, a_collapse=0.0):
    """Batched gradient descent on the drift objective (the scheme's objective
    has no descent rule in the paper; this is the rule the library documents):
    per instance, step fraction s = step0; each iteration takes (L, g) from
    ``objective``; an instance whose evolution collapses is masked from then on
    (c kept, later L entries NaN); otherwise s halves when L grew since the
    previous iteration and c <- c - s |c| / |g| g.  Plain loops, sums in index
    order.  Returns (c, L_hist [iters x n], active [n])."""
    c = np.array(c, dtype=np.float64, copy=True)
    n = len(Ns)
    s = [float(step0)] * n
    Lprev = [math.inf] * n
    active = [1] * n
    hist = np.full((iters, n), np.nan)
    for it in range(iters):
        for b in range(n):
            if not active[b]:
                continue
            r = objective(int(Ns[b]), float(eps[b]), c[b], T=T, J=J, K=K, gauge=gauge, a_collapse=a_collapse)
            hist[it, b] = r["L"]
            if not r["valid"]:
                active[b] = 0
                continue
            if r["L"] > Lprev[b]:
                s[b] *= 0.5
            Lprev[b] = r["L"]
            g = r["grad"]
            cn = 0.0
            gn = 0.0
            for k in range(c.shape[1]):
                cn += c[b, k] * c[b, k]
                gn += g[k] * g[k]
            if gn > 0.0:
                f = s[b] * math.sqrt(cn) / math.sqrt(gn)
                for k in range(c.shape[1]):
                    c[b, k] -= f * g[k]
    return c, hist, np.array(active, np.int32)


def constraints_vjp(Phi, Pi, Abar, dbar, gauge=GAUGE_BOUNDARY):
    lib = _load()
    Phi, Pi, Abar, dbar = map(_f64, (Phi, Pi, Abar, dbar))
    N = len(Phi)
    Pb, Qb = np.zeros(N), np.zeros(N)
    lib.ora_constraints_vjp(N, gauge, _ptr(Phi), _ptr(Pi), _ptr(Abar), _ptr(dbar), _ptr(Pb), _ptr(Qb))
    return Pb, Qb


def rhs_vjp(Phi, Pi, A, delta, kbar0, kbar1, ko=0.5, frozen=False):
    lib = _load()
    Phi, Pi, A, delta, kbar0, kbar1 = map(_f64, (Phi, Pi, A, delta, kbar0, kbar1))
    N = len(Phi)
    out = [np.zeros(N) for _ in range(4)]
    lib.ora_rhs_vjp(N, ko, int(frozen), _ptr(Phi), _ptr(Pi), _ptr(A), _ptr(delta), _ptr(kbar0), _ptr(kbar1),
                    *[_ptr(o) for o in out])
    return out


def step(Phi, Pi, gauge=GAUGE_BOUNDARY, cfl=0.25, ko=0.5):
    lib = _load()
    Phi, Pi = _f64(Phi).copy(), _f64(Pi).copy()
    lib.ora_step(len(Phi), gauge, cfl, ko, _ptr(Phi), _ptr(Pi))
    return Phi, Pi


def step_vjp(Phi, Pi, Phibar, Pibar, gauge=GAUGE_BOUNDARY, cfl=0.25, ko=0.5):
    lib = _load()
    Phi, Pi = _f64(Phi), _f64(Pi)
    Pb, Qb = _f64(Phibar).copy(), _f64(Pibar).copy()
    lib.ora_step_vjp(len(Phi), gauge, cfl, ko, _ptr(Phi), _ptr(Pi), _ptr(Pb), _ptr(Qb))
    return Pb, Qb


def spectrum_vjp(Phi, Pi, A, Ebar):
    lib = _load()
    Phi, Pi, A, Ebar = map(_f64, (Phi, Pi, A, Ebar))
    N = len(Phi)
    out = [np.zeros(N) for _ in range(3)]
    lib.ora_spectrum_vjp(N, len(Ebar), _ptr(Phi), _ptr(Pi), _ptr(A), _ptr(Ebar), *[_ptr(o) for o in out])
    return out
