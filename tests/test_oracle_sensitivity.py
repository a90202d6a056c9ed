"""Self-sensitivity of the method to rounding: the oracle's sources built a
second time with FMA contraction on (``oracle.build.build_contract``) and run
beside the parity build on the parity tests' longest windows.

Two correct evaluations of the same arithmetic that round differently drift
apart at the rate the scheme amplifies rounding; the GPU kernels differ from
the oracle in the same way (other FMA contractions, their own exponential,
another summation order), so this drift is the floor under any parity
tolerance.  Measured: within 3.4e-12 (relative max-norm over the five fields)
at every snapshot of the 513-point Gaussian run to t = 2 pi (8192 steps), the
worst at t = pi/2 and 3 pi/2, when the pulse reflects off the boundary and the
max-norm of Pi is at its smallest; 1e-13 to 7e-13 on a 1025-point run of 8192
steps.  The 1e-11 bar of the parity tests therefore keeps a margin of 3 or
more over the windows they use (at most 8192 steps; the full-length GPU checks
measure the longer runs directly).  CPU only.
"""
import shutil

import numpy as np
import pytest

import oracle as O
from oracle import build as B


def rel(a, b):
    n = np.max(np.abs(b))
    d = np.max(np.abs(a - b))
    return d / n if n > 1e-12 else d / 1e-12 * 1e-13


@pytest.fixture(scope="module")
def contract_lib(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    out = str(tmp_path_factory.mktemp("oracle_contract") / "liboracle_contract.so")
    B.build_contract(out)
    return O.load_library(out)


@pytest.mark.parametrize("N,eps,sig,gauge,n,every,bound_each,bound_end", [
    (513, 10.0, 1 / 16, O.GAUGE_ORIGIN, 8192, 256, 5e-12, 2e-13),
    (1025, 20.0, 0.1, O.GAUGE_BOUNDARY, 8192, 512, 2e-12, 5e-13),
])
def test_rounding_drift_stays_inside_the_parity_tolerance(contract_lib, N, eps, sig, gauge, n, every, bound_each,
                                                          bound_end):
    Phi, Pi = O.init_gaussian(N, eps, sig)
    slots = n // every + 1
    a = O.evolve(Phi, Pi, n, gauge=gauge, snap_every=every, n_slots=slots)
    b = O.evolve(Phi, Pi, n, gauge=gauge, snap_every=every, n_slots=slots, lib=contract_lib)
    assert a["steps"] == b["steps"] == n
    drift = [max(rel(b["snaps"][k, f], a["snaps"][k, f]) for f in range(5)) for k in range(slots)]
    # the two builds do round differently (otherwise the check measures nothing)
    assert max(drift) > 1e-15
    assert max(drift) <= bound_each, ["%.1e" % d for d in drift]
    assert drift[-1] <= bound_end
