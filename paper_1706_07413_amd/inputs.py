"""Seeded synthetic workloads for the AdS4 scalar-collapse evolution.

This module only draws parameters (grid sizes, amplitudes, widths, mode
coefficients) with numpy's PCG64 and holds none of the method's arithmetic: both
the HIP library and the CPU oracle turn these parameters into initial data with
their own code.  Seeds are ``SEED_BASE + k`` for workload k.

Workloads (the initial-data families follow Sec. II of Liebling & Khanna,
arXiv:1706.07413: Phi(x,0) = 0 and Pi(x,0) given, constraints solved at t = 0):

0. single instance, N=513, Gaussian Pi with eps=10, sigma=1/16, origin gauge,
   t = 2 pi, snapshots every 256 steps;
1. single instance, N=16385, two-mode data eps*(e_0 + 0.6 e_1), eps=0.05,
   t = 200, spectrum (64 modes) every 1024 steps;
2. 1024 instances, Gaussian data, sigma ~ U[1/16, 1/4], eps log-uniform in
   [1, 40], N uniform in {1025, 2049, 4097}, t = 50 or collapse (min A < 0.02);
3. single instance, N=4097, Pi = eps sum_{j<32} c_j e_j with
   c_j ~ N(0,1) exp(-j/4), eps=0.1, T = 100, checkpoints every 512 steps;
4. 256 instances of 3 with eps log-uniform in [0.02, 0.2], N in {2049, 4097}.
"""
import math

import numpy as np

SEED_BASE = 170607413
GAUGE_BOUNDARY = 0
GAUGE_ORIGIN = 1


def rng_for(k):
    return np.random.default_rng(SEED_BASE + k)


def config0():
    return dict(name="single_gaussian_N513", N=np.array([513], np.int32), eps=np.array([10.0]),
                sigma=np.array([1.0 / 16.0]), T=2.0 * math.pi, gauge=GAUGE_ORIGIN, snap_every=256,
                a_collapse=0.01)


def config1():
    return dict(name="single_twomode_N16385", N=np.array([16385], np.int32), eps=np.array([0.05]),
                c=np.array([[1.0, 0.6]]), T=200.0, gauge=GAUGE_BOUNDARY, n_modes=64,
                spec_every=1024, a_collapse=0.01)


def config2(B=1024):
    """The 1024-instance draw; B < 1024 returns its first B instances."""
    r = rng_for(2)
    n = 1024
    N = r.choice(np.array([1025, 2049, 4097], np.int32), size=n)
    sigma = r.uniform(1.0 / 16.0, 1.0 / 4.0, size=n)
    eps = np.exp(r.uniform(0.0, math.log(40.0), size=n))
    return dict(name="batched_gaussian_1024", N=N[:B].astype(np.int32), eps=eps[:B], sigma=sigma[:B],
                T=50.0, gauge=GAUGE_BOUNDARY, a_collapse=0.02)


def mode_coefficients(r, n, J=32):
    return r.standard_normal((n, J)) * np.exp(-np.arange(J) / 4.0)[None, :]


def config3():
    r = rng_for(3)
    return dict(name="adjoint_N4097", N=np.array([4097], np.int32), eps=np.array([0.1]),
                c=mode_coefficients(r, 1), T=100.0, J_obj=16, ckpt_every=512, gauge=GAUGE_BOUNDARY,
                a_collapse=0.01, fd_h=1e-6)


def config4(B=256):
    """The 256-instance draw; B < 256 returns its first B instances."""
    r = rng_for(4)
    n = 256
    N = r.choice(np.array([2049, 4097], np.int32), size=n)
    eps = np.exp(r.uniform(math.log(0.02), math.log(0.2), size=n))
    c = mode_coefficients(r, n)
    return dict(name="batched_adjoint_gd_256", N=N[:B].astype(np.int32), eps=eps[:B], c=c[:B],
                T=100.0, J_obj=16, ckpt_every=512, gd_iters=50, gauge=GAUGE_BOUNDARY, a_collapse=0.01)


def qp_family(kd, mu, J=40):
    """Mode-sum coefficients of the paper's approximate quasi-periodic families
    (Sec. II, Eq. (13)): amplitudes A_k = eps exp(-mu |k - k_d|) of phi in mode
    k, i.e. Pi(x,0) = eps sum_{k<J} omega_k exp(-mu |k - k_d|) e_k(x) with
    omega_k = 3 + 2k, Phi(x,0) = 0.  Returns the J coefficients of e_k (eps
    applied separately, as adscl_init_modes takes it)."""
    k = np.arange(J)
    return (3.0 + 2.0 * k) * np.exp(-mu * np.abs(k - kd))


# the four families the paper evolves: (k_d, mu)
QP_FAMILIES = ((3, 1.0), (3, 1.75), (5, 1.0), (5, 1.75))


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}
