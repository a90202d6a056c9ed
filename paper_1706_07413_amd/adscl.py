"""Thin ctypes binding of libadscl.so (include/adscl.h).

Argument marshalling only: every step of the evolution runs in the HIP kernels
of the library.  Device arrays are torch tensors on the context's GPU (their
data pointers go straight through the ABI); host arrays are numpy arrays.  The
module refuses to work without the built library.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadscl.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GAUGE_BOUNDARY, GAUGE_ORIGIN = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
FROZEN_METRIC = 1
TIME_KERNELS = 2
DESCEND_EAGER = 1
RUNNING, COLLAPSED, NONFINITE, DONE = 0, 1, 2, 3

# Every function include/adscl.h declares.
EXPORTS = ("adscl_create", "adscl_destroy", "adscl_init", "adscl_init_gaussian", "adscl_init_modes",
           "adscl_step", "adscl_get_state", "adscl_status", "adscl_constraints", "adscl_constraints_noalloc",
           "adscl_spectrum", "adscl_spectrum_snaps",
           "adscl_adjoint", "adscl_descend", "adscl_sync", "adscl_layout", "adscl_kernel_stats", "adscl_last_error",
           "adscl_autotune", "adscl_autotune_clear")


class AdsclError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("adscl error %d: %s" % (code, msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("n_grid", ctypes.POINTER(ctypes.c_int32)),
                ("cfl", ctypes.c_double), ("ko_sigma", ctypes.c_double), ("a_collapse", ctypes.c_double),
                ("gauge", ctypes.c_int32), ("n_modes", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("rk_order", ctypes.c_int32), ("a_reint", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double


def lib():
    """Load libadscl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libadscl.so is not built (%s); run python -m paper_1706_07413_amd.build" % LIB_PATH)
    # torch ships a HIP runtime under the same soname as the system one the
    # library links; loading torch first makes the library bind to that one
    # instance, the only process layout in which device pointers and streams
    # are shared with torch.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "adscl_create": (ctypes.c_int, [ctypes.POINTER(Config), _vp, ctypes.POINTER(_vp)]),
        "adscl_destroy": (None, [_vp]),
        "adscl_init": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
        "adscl_init_gaussian": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
        "adscl_init_modes": (ctypes.c_int, [_vp, _vp, _vp, _i32, ctypes.c_int]),
        "adscl_step": (ctypes.c_int, [_vp, _i64, _d, _i32, _i32, _vp, ctypes.c_int]),
        "adscl_get_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int]),
        "adscl_status": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "adscl_constraints": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
        "adscl_constraints_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
        "adscl_spectrum": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, ctypes.c_int]),
        "adscl_spectrum_snaps": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, ctypes.c_int]),
        "adscl_adjoint": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _d, _i32, _vp, _vp, _vp, ctypes.c_int]),
        "adscl_descend": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _d, _i32, _i32, _d, _i32, _vp, _vp,
                                         ctypes.c_int]),
        "adscl_sync": (ctypes.c_int, [_vp]),
        "adscl_layout": (ctypes.c_int, [_vp, _vp, _vp]),
        "adscl_kernel_stats": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
        "adscl_last_error": (ctypes.c_char_p, [_vp]),
        "adscl_autotune": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp]),
        "adscl_autotune_clear": (None, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def autotune(n_grid, steps=256, apply=True):
    """Time every compiled kernel configuration for each grid size on a full
    batch of weak data and return {N: (P, W, pt-steps/s)} of the fastest; with
    ``apply`` the choices hold for every later Batch in this process (see
    adscl_autotune in include/adscl.h)."""
    L = lib()
    Ns = np.ascontiguousarray(np.asarray(n_grid, dtype=np.int32))
    n = len(Ns)
    P, W = np.zeros(n, np.int32), np.zeros(n, np.int32)
    rate = np.zeros(n)
    rc = L.adscl_autotune(Ns.ctypes.data, n, int(steps), 1 if apply else 0, P.ctypes.data, W.ctypes.data,
                          rate.ctypes.data)
    if rc:
        raise AdsclError(rc, L.adscl_last_error(None).decode())
    return {int(Ns[i]): (int(P[i]), int(W[i]), float(rate[i])) for i in range(n)}


def autotune_clear():
    """Forget the autotuner's choices (later Batches use the default rule)."""
    lib().adscl_autotune_clear()


def _ptr_mem(a):
    """(pointer, mem) of a torch tensor (device) or numpy array (host)."""
    if a is None:
        return None, None
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
            raise TypeError("host arrays must be C-contiguous float64")
        return a.ctypes.data, MEM_HOST
    import torch
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError("tensors must be contiguous float64")
        if a.is_cuda:
            # the context's stream is not ordered after torch's streams: work
            # torch has queued that writes this tensor must be done before the
            # library reads it
            torch.cuda.current_stream(a.device).synchronize()
            return a.data_ptr(), MEM_DEVICE
        return a.data_ptr(), MEM_HOST
    raise TypeError("expected numpy array or torch tensor")


# Contexts still open at interpreter exit are destroyed by an exit handler,
# while the HIP runtime is still intact, rather than by __del__ during the
# interpreter's final teardown (when the runtime's own state may be gone).
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for b in list(_live):
        try:
            b.close()
        except Exception:
            pass


class Batch:
    """A batch of independent instances with grid sizes ``n_grid`` on one GPU."""

    def __init__(self, n_grid, cfl=0.25, ko_sigma=0.5, a_collapse=0.01, gauge=GAUGE_BOUNDARY, n_modes=0,
                 flags=0, stream=None, rk_order=4, a_reint=0):
        """``rk_order`` (4, 3 or 2) and ``a_reint`` (0: A from Eq. (5) at every
        stage; K: A evolved by Eq. (4), re-integrated every K steps) select the
        scheme options of adscl_config."""
        L = lib()
        self._N = np.ascontiguousarray(np.asarray(n_grid, dtype=np.int32))
        cfg = Config(len(self._N), self._N.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cfl, ko_sigma,
                     a_collapse, gauge, n_modes, flags, rk_order, a_reint)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = _vp()
        rc = L.adscl_create(ctypes.byref(cfg), _vp(stream), ctypes.byref(h))
        if rc != OK:
            raise AdsclError(rc, L.adscl_last_error(None).decode())
        self._h = h
        _live.add(self)
        self.n_inst = len(self._N)
        self.cfl = cfl
        off = np.zeros(self.n_inst, np.int64)
        tot = _i64(0)
        L.adscl_layout(self._h, off.ctypes.data, ctypes.byref(tot))
        self.off = off
        self.total = tot.value
        self.n_grid = self._N

    def _check(self, rc):
        if rc != OK:
            raise AdsclError(rc, lib().adscl_last_error(self._h).decode())

    def close(self):
        """Synchronise the context's stream and free everything it holds."""
        if getattr(self, "_h", None):
            lib().adscl_sync(self._h)
            lib().adscl_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- initial data ----
    def init(self, Phi0, Pi0):
        p1, m1 = _ptr_mem(Phi0)
        p2, m2 = _ptr_mem(Pi0)
        assert m1 == m2
        self._check(lib().adscl_init(self._h, p1, p2, m1))

    def init_gaussian(self, eps, sigma):
        p1, m1 = _ptr_mem(eps)
        p2, m2 = _ptr_mem(sigma)
        assert m1 == m2
        self._check(lib().adscl_init_gaussian(self._h, p1, p2, m1))

    def init_modes(self, eps, c):
        p1, m1 = _ptr_mem(eps)
        p2, m2 = _ptr_mem(c)
        assert m1 == m2
        self._check(lib().adscl_init_modes(self._h, p1, p2, int(c.shape[1]), m1))

    # ---- evolution ----
    def step(self, max_steps, t_end, snap_every=0, snaps=None):
        """Advance; ``snaps`` (optional) is a [slots, 5, total] float64 array/tensor."""
        if snaps is not None:
            p, m = _ptr_mem(snaps)
            slots = int(snaps.shape[0])
        else:
            p, m, slots = None, MEM_DEVICE, 0
        self._check(lib().adscl_step(self._h, int(max_steps), float(t_end), int(snap_every), slots, p, m))
        if snaps is not None and m == MEM_DEVICE:
            self.sync()

    def sync(self):
        self._check(lib().adscl_sync(self._h))

    # ---- outputs ----
    def get_state(self, out=None):
        """Dict of packed Phi, Pi, A, delta, m (torch tensors on the GPU unless
        ``out`` holds numpy arrays)."""
        if out is None:
            import torch
            out = {k: torch.empty(self.total, dtype=torch.float64, device="cuda")
                   for k in ("Phi", "Pi", "A", "delta", "m")}
        ptrs = [_ptr_mem(out[k]) for k in ("Phi", "Pi", "A", "delta", "m")]
        mem = ptrs[0][1]
        self._check(lib().adscl_get_state(self._h, *[p for p, _ in ptrs], mem))
        if mem == MEM_DEVICE:
            # the context's stream is not ordered with torch's streams
            self.sync()
        return out

    def status(self):
        n = self.n_inst
        t, tc, mA = np.zeros(n), np.zeros(n), np.zeros(n)
        steps = np.zeros(n, np.int64)
        state = np.zeros(n, np.int32)
        self._check(lib().adscl_status(self._h, t.ctypes.data, steps.ctypes.data, state.ctypes.data,
                                       tc.ctypes.data, mA.ctypes.data))
        return dict(t=t, steps=steps, state=state, t_c=tc, minA=mA)

    def constraints(self):
        """[n_inst, 5]: max |R_A'|, max |R_delta'|, max |R_A_t| (Eqs. (5), (6), (4)),
        the mass m(pi/2) and the mass integral (adscl_constraints)."""
        out = np.zeros((self.n_inst, 5))
        self._check(lib().adscl_constraints(self._h, out.ctypes.data, MEM_HOST))
        return out

    def constraints_noalloc(self, out=None):
        """adscl_constraints_noalloc into `out` ([n_inst, 5] numpy or torch float64),
        a new numpy array by default."""
        if out is None:
            out = np.zeros((self.n_inst, 5))
        p, m = _ptr_mem(out)
        self._check(lib().adscl_constraints_noalloc(self._h, p, m))
        if m == MEM_DEVICE:
            self.sync()
        return out

    def spectrum(self, J):
        E, P, F = (np.zeros((self.n_inst, J)) for _ in range(3))
        self._check(lib().adscl_spectrum(self._h, int(J), E.ctypes.data, P.ctypes.data, F.ctypes.data, MEM_HOST))
        return E, P, F

    def spectrum_snaps(self, J, snaps):
        """Mode energies of stored states snaps [slots, 5, total] (numpy or
        torch); returns E, Pihat, Phihat [slots, n_inst, J] of the same kind."""
        p, m = _ptr_mem(snaps)
        S = int(snaps.shape[0])
        if m == MEM_DEVICE:
            import torch
            outs = [torch.empty((S, self.n_inst, J), dtype=torch.float64, device=snaps.device) for _ in range(3)]
        else:
            outs = [np.zeros((S, self.n_inst, J)) for _ in range(3)]
        self._check(lib().adscl_spectrum_snaps(self._h, int(J), S, p, *[_ptr_mem(o)[0] for o in outs], m))
        if m == MEM_DEVICE:
            self.sync()
        return tuple(outs)

    def adjoint(self, eps, c, J, T, ckpt_every=512):
        """Drift objective L_b = sum_{j<J} (E_j(T) - E_j(0))^2 of mode-sum data
        eps_b sum_k c_bk e_k and its gradient dL_b/dc_b (adscl_adjoint).  Host
        (numpy) or device (torch) inputs; returns (L, dLdc, valid) of the same
        kind.  Leaves the batch at the final state."""
        pe, me = _ptr_mem(eps)
        pc, mc = _ptr_mem(c)
        assert me == mc
        n, Jc = self.n_inst, int(c.shape[1])
        if me == MEM_DEVICE:
            import torch
            L = torch.empty(n, dtype=torch.float64, device=c.device)
            g = torch.empty((n, Jc), dtype=torch.float64, device=c.device)
            v = torch.empty(n, dtype=torch.int32, device=c.device)
            pv = v.data_ptr()
        else:
            L, g = np.zeros(n), np.zeros((n, Jc))
            v = np.zeros(n, np.int32)
            pv = v.ctypes.data
        self._check(lib().adscl_adjoint(self._h, pe, pc, Jc, int(J), float(T), int(ckpt_every), _ptr_mem(L)[0],
                                        _ptr_mem(g)[0], pv, me))
        if me == MEM_DEVICE:
            self.sync()
        return L, g, v

    def descend(self, eps, c, J, T, iters, step0=0.05, ckpt_every=512, eager=False):
        """Batched gradient descent on the drift objective (adscl_descend).
        Returns (c_final, L_hist [iters x n_inst], active) of the kind of c
        (numpy on the host, torch on the device); c itself is not modified."""
        n, Jc = self.n_inst, int(c.shape[1])
        pe, me = _ptr_mem(eps)
        if me == MEM_DEVICE:
            import torch
            cw = c.clone()
            hist = torch.empty((iters, n), dtype=torch.float64, device=c.device)
            act = torch.empty(n, dtype=torch.int32, device=c.device)
            pa = act.data_ptr()
        else:
            cw = np.array(c, dtype=np.float64, copy=True)
            hist = np.zeros((iters, n))
            act = np.zeros(n, np.int32)
            pa = act.ctypes.data
        self._check(lib().adscl_descend(self._h, pe, _ptr_mem(cw)[0], Jc, int(J), float(T), int(ckpt_every),
                                        int(iters), float(step0), DESCEND_EAGER if eager else 0,
                                        _ptr_mem(hist)[0], pa, me))
        if me == MEM_DEVICE:
            self.sync()
        return cw, hist, act

    def kernel_stats(self):
        """Launch classes: list of dicts (P, W, members, last_ms) and the class
        index of every instance."""
        n = ctypes.c_int32(0)
        self._check(lib().adscl_kernel_stats(self._h, 0, ctypes.addressof(n), None, None, None, None, None))
        k = n.value
        P, W, M = (np.zeros(k, np.int32) for _ in range(3))
        ms = np.zeros(k)
        cls = np.zeros(self.n_inst, np.int32)
        self._check(lib().adscl_kernel_stats(self._h, k, ctypes.addressof(n), P.ctypes.data, W.ctypes.data,
                                             M.ctypes.data, ms.ctypes.data, cls.ctypes.data))
        return [dict(P=int(P[i]), W=int(W[i]), members=int(M[i]), last_ms=float(ms[i])) for i in range(k)], cls

    def split(self, packed):
        """List of per-instance views of a packed array."""
        return [packed[o:o + n] for o, n in zip(self.off, self.n_grid)]
