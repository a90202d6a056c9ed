"""Parity of the library's discrete adjoint (adscl_adjoint) with the oracle's.

Both sides compute L = sum_{j<J} (E_j(t_n) - E_j(0))^2 for mode-sum data and
dL/dc as the exact derivative of their own discrete computation; the two
computations agree to rounding, so the gradients must too.  Tolerances: the
gradient within 1e-9 in relative max-norm (a reverse sweep accumulates
rounding over every step, and each entry is a sum over the whole grid and run);
L within 1e-9 relative (L is a square of a drift E_j(t_n) - E_j(0) that cancels
most of E_j, so the relative rounding of E_j ~ 1e-14 is amplified by
E_j / |E_j(t_n) - E_j(0)|, up to ~1e4 here).  Validity flags must match
exactly, and results that must not depend on the checkpoint interval or on
the batch composition must be bitwise equal.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1706_07413_amd import adscl
from paper_1706_07413_amd import inputs as I

pytestmark = pytest.mark.gpu

GTOL = 1e-9
LTOL = 1e-9

# The reverse sweep reads each step's stages from the record the forward
# recompute of the segment kept, or (when the records would exceed a quarter of
# the device memory, or with ADSCL_ADJOINT_RECOMPUTE=1) recomputes them itself.
MODES = ["stored", "recompute"]


def set_mode(monkeypatch, mode):
    if mode == "recompute":
        monkeypatch.setenv("ADSCL_ADJOINT_RECOMPUTE", "1")
    else:
        monkeypatch.delenv("ADSCL_ADJOINT_RECOMPUTE", raising=False)


def relmax(g, o):
    g, o = np.asarray(g), np.asarray(o)
    return np.max(np.abs(g - o)) / max(np.max(np.abs(o)), 1e-300)


def coeffs(seed, n, Jc):
    r = np.random.default_rng(seed)
    return np.ascontiguousarray(r.standard_normal((n, Jc)) * np.exp(-np.arange(Jc) / 4.0))


def run_gpu(Ns, eps, c, J, T, K, gauge=O.GAUGE_BOUNDARY, thr=0.0, n_modes=None):
    b = adscl.Batch(Ns, gauge=gauge, a_collapse=thr, n_modes=n_modes or max(J, c.shape[1]))
    L, g, v = b.adjoint(np.ascontiguousarray(eps, dtype=np.float64), c, J, T, K)
    return b, L, g, v


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("gauge", [O.GAUGE_BOUNDARY, O.GAUGE_ORIGIN])
def test_adjoint_ragged_batch_matches_oracle(monkeypatch, gauge, mode):
    """Five instances of four grid sizes (17 to 131 steps each), 8 modes in,
    drift of 4 modes, checkpoints every 7 steps.  In origin time the N=257
    instance runs unstable on both sides (its boundary speed A e^-delta grows
    past what RK4 at dt = h/4 tolerates) and must come back invalid with a zero
    gradient; the others are compared."""
    Ns = np.array([33, 65, 129, 257, 65], np.int32)
    eps = np.array([0.5, 0.3, 0.8, 0.4, 1.0])
    Jc, J, T, K = 8, 4, 0.2, 7
    c = coeffs(11, len(Ns), Jc)
    set_mode(monkeypatch, mode)
    print("adjoint ragged gauge", gauge, mode, flush=True)
    _, L, g, v = run_gpu(Ns, eps, c, J, T, K, gauge=gauge)
    n_valid = 0
    for b, N in enumerate(Ns):
        ref = O.objective(int(N), float(eps[b]), c[b], T=T, J=J, K=K, gauge=gauge)
        assert v[b] == int(ref["valid"]), (b, v[b], ref["valid"])
        if not ref["valid"]:
            assert np.all(g[b] == 0.0)
            continue
        n_valid += 1
        assert abs(L[b] - ref["L"]) <= LTOL * ref["L"], (b, L[b], ref["L"])
        e = relmax(g[b], ref["grad"])
        assert e <= GTOL, "instance %d (N=%d): gradient error %.3e" % (b, N, e)
    assert n_valid >= 4


def test_adjoint_stored_and_recomputed_stages_agree(monkeypatch):
    """The two ways of obtaining each step's stages in the reverse sweep (read
    from the record of the segment's forward recompute, or recomputed by the
    reverse kernel from the step's state) give the same gradient: the same
    arithmetic in two compiled kernels, so equal to rounding."""
    Ns = np.array([33, 65, 129, 257, 65, 1025], np.int32)
    eps = np.array([0.5, 0.3, 0.8, 0.4, 1.0, 0.6])
    c = coeffs(21, len(Ns), 8)
    print("adjoint stored vs recomputed", flush=True)
    out = {}
    for mode in MODES:
        set_mode(monkeypatch, mode)
        _, L, g, v = run_gpu(Ns, eps, c, 4, 0.2, 7)
        out[mode] = (L, g, v)
    (L1, g1, v1), (L2, g2, v2) = out["stored"], out["recompute"]
    assert np.array_equal(v1, v2) and np.all(v1 == 1)
    assert np.max(np.abs(L1 - L2) / np.abs(L2)) <= 1e-12
    for b in range(len(Ns)):
        assert relmax(g1[b], g2[b]) <= 1e-12, b


def test_adjoint_checkpoint_interval_is_bitwise_irrelevant():
    Ns = np.array([65, 129], np.int32)
    eps = np.array([0.6, 0.4])
    c = coeffs(12, 2, 6)
    T = 0.15
    print("adjoint checkpoint intervals", flush=True)
    _, L1, g1, _ = run_gpu(Ns, eps, c, 3, T, 1)
    for K in (5, 32, 10 ** 6):
        _, L2, g2, _ = run_gpu(Ns, eps, c, 3, T, K)
        assert np.array_equal(L1, L2) and np.array_equal(g1, g2), K


def test_adjoint_batched_equals_single():
    Ns = np.array([129, 65, 129, 257], np.int32)
    eps = np.array([0.3, 0.7, 0.5, 0.2])
    c = coeffs(13, 4, 5)
    print("adjoint batched vs single", flush=True)
    _, L, g, _ = run_gpu(Ns, eps, c, 4, 0.1, 9)
    for b in (1, 2):
        _, Ls, gs, _ = run_gpu(Ns[b:b + 1], eps[b:b + 1], np.ascontiguousarray(c[b:b + 1]), 4, 0.1, 9)
        assert Ls[0] == L[b] and np.array_equal(gs[0], g[b])


def test_adjoint_collapsed_instance_is_invalid():
    """A strong pulse that drives min A below the threshold on the way: valid 0,
    zero gradient, L evaluated where the evolution stopped (same as the oracle);
    its neighbour in the batch is unaffected."""
    Ns = np.array([129, 129], np.int32)
    eps = np.array([0.1, 0.8])
    c = np.ascontiguousarray(np.vstack([coeffs(14, 1, 6)[0], np.array([1.0, 0.8, 0.6, 0.4, 0.2, 0.1])]))
    thr, T = 0.15, 1.0  # the second starts at min A 0.21 and falls below 0.1 before t = 1
    print("adjoint collapse", flush=True)
    b, L, g, v = run_gpu(Ns, eps, c, 3, T, 16, thr=thr)
    r0 = O.objective(129, 0.1, c[0], T=T, J=3, K=16, a_collapse=thr)
    r1 = O.objective(129, 0.8, c[1], T=T, J=3, K=16, a_collapse=thr)
    assert r0["valid"] and not r1["valid"]
    assert v[0] == 1 and v[1] == 0
    assert np.all(g[1] == 0.0)
    assert abs(L[1] - r1["L"]) <= 1e-9 * abs(r1["L"])
    assert relmax(g[0], r0["grad"]) <= GTOL
    st = b.status()
    assert st["state"][1] == adscl.COLLAPSED and st["state"][0] == adscl.DONE


def test_adjoint_gradient_against_gpu_central_differences():
    """Independent of the oracle: dL/dc against central differences of the
    library's own L (step 1e-6), N=129, 6 modes, eps=0.8, 0.3 time units."""
    N, Jc, J, T = 129, 6, 4, 0.3
    c = coeffs(15, 1, Jc)
    eps = np.array([0.8])
    print("adjoint vs GPU finite differences", flush=True)
    b = adscl.Batch([N], a_collapse=0.0, n_modes=Jc)
    L, g, v = b.adjoint(eps, c, J, T, 64)
    h = 1e-6
    cs = []
    for k in range(Jc):
        for s in (+1, -1):
            cc = c.copy()
            cc[0, k] += s * h
            cs.append(cc[0])
    # all perturbations as one batch
    bb = adscl.Batch([N] * len(cs), a_collapse=0.0, n_modes=Jc)
    Lp, _, _ = bb.adjoint(np.full(len(cs), 0.8), np.ascontiguousarray(np.array(cs)), J, T, 64)
    fd = (Lp[0::2] - Lp[1::2]) / (2 * h)
    assert v[0] == 1
    assert relmax(g[0], fd) <= 1e-6, (g[0], fd)


def test_adjoint_full_grid_sizes_short_window():
    """The grid sizes of the 4097-point single-instance and the 2049/4097
    batched gradient workloads (their seeded coefficients, amplitude raised to
    1 so that 64 steps of the N=4097 instance, 32 of N=2049, already drift
    nonlinearly), 16 modes in, drift of 16 modes."""
    c3 = I.config3()
    c4 = I.config4(4)
    Ns = np.concatenate([c3["N"], c4["N"]]).astype(np.int32)
    eps = np.ones(len(Ns))
    c = np.ascontiguousarray(np.vstack([c3["c"], c4["c"]])[:, :16])
    T = 64 * O.dt_of(4097)
    print("adjoint full sizes", list(Ns), flush=True)
    _, L, g, v = run_gpu(Ns, eps, c, 16, T, 16, n_modes=32)
    for b, N in enumerate(Ns):
        ref = O.objective(int(N), float(eps[b]), c[b], T=T, J=16, K=16)
        assert v[b] == 1 and ref["valid"]
        assert abs(L[b] - ref["L"]) <= LTOL * ref["L"], (b, L[b], ref["L"])
        e = relmax(g[b], ref["grad"])
        assert e <= GTOL, "instance %d (N=%d): gradient error %.3e" % (b, N, e)


def test_adjoint_zero_time():
    c = coeffs(16, 2, 4)
    _, L, g, v = run_gpu(np.array([65, 33], np.int32), np.array([0.5, 0.5]), c, 4, 0.0, 8)
    assert np.all(L == 0.0) and np.all(g == 0.0) and np.all(v == 1)


def test_autograd_function_hands_out_the_adjoint_gradient():
    import torch
    from paper_1706_07413_amd.autograd import drift_loss
    Ns = np.array([65, 129], np.int32)
    c_np = coeffs(17, 2, 5)
    print("autograd wrapper", flush=True)
    b = adscl.Batch(Ns, a_collapse=0.0, n_modes=8)
    c = torch.tensor(c_np, device="cuda", requires_grad=True)
    eps = torch.tensor([0.5, 0.4], dtype=torch.float64, device="cuda")
    L, valid = drift_loss(b, c, eps, 4, 0.1, ckpt_every=8)
    w = torch.tensor([1.0, 2.0], dtype=torch.float64, device="cuda")
    (w * L).sum().backward()
    _, L2, g2, _ = run_gpu(Ns, np.array([0.5, 0.4]), c_np, 4, 0.1, 8, n_modes=8)
    assert np.array_equal(L.detach().cpu().numpy(), L2)
    assert np.array_equal(c.grad.cpu().numpy(), w.cpu().numpy()[:, None] * g2)
    assert valid.cpu().numpy().tolist() == [1, 1]


def test_descend_matches_oracle_and_masks_collapse():
    """Three descent iterations on a ragged batch; one instance collapses on
    the way and is masked.  Coefficients and objective history agree with the
    oracle's descent to 1e-8 (each iteration moves c by a step computed from a
    gradient that agrees to 1e-9)."""
    Ns = np.array([33, 65, 129, 65], np.int32)
    eps = np.array([0.5, 0.3, 0.8, 0.4])
    c0 = coeffs(22, len(Ns), 6)
    c0[2] = np.array([1.0, 0.8, 0.6, 0.4, 0.2, 0.1])
    J, T, K, iters, step0, thr = 3, 1.0, 64, 3, 0.05, 0.15
    print("descend vs oracle", flush=True)
    b = adscl.Batch(Ns, a_collapse=thr, n_modes=8)
    c, hist, act = b.descend(eps, c0, J, T, iters, step0=step0, ckpt_every=K)
    rc, rhist, ract = O.descend(Ns, eps, c0, J, T, K, iters, step0, a_collapse=thr)
    assert act.tolist() == ract.tolist() and act[2] == 0
    assert np.array_equal(np.isnan(hist), np.isnan(rhist))
    m = ~np.isnan(rhist)
    assert np.max(np.abs(hist[m] - rhist[m]) / np.abs(rhist[m])) <= 1e-8
    assert relmax(c, rc) <= 1e-8
    assert np.array_equal(c[2], c0[2])


def test_descend_graph_replays_equal_eager_iterations():
    """The captured iteration replayed 4 times gives, iteration by iteration,
    the same objective history and final coefficients as 4 directly enqueued
    iterations, bit for bit."""
    Ns = np.array([65, 129, 257], np.int32)
    eps = np.array([0.4, 0.6, 0.3])
    c0 = coeffs(23, 3, 8)
    print("descend graph vs eager", flush=True)
    b = adscl.Batch(Ns, a_collapse=0.0, n_modes=8)
    cg, hg, ag = b.descend(eps, c0, 4, 0.2, 4, step0=0.05, ckpt_every=16)
    ce, he, ae = b.descend(eps, c0, 4, 0.2, 4, step0=0.05, ckpt_every=16, eager=True)
    assert np.array_equal(hg, he) and np.array_equal(cg, ce) and np.array_equal(ag, ae)
    assert np.all(np.isfinite(hg))


# every launch configuration of the reverse kernel, full lanes (DPP exchange,
# adjoint state in LDS) and ragged grids (rows, state in the scratch), forced
# with ADSCL_TUNE at context creation
TUNED_ADJ = [(257, 4, 1), (513, 4, 2), (1025, 4, 4), (2049, 4, 8), (4097, 4, 16), (513, 8, 1), (1025, 8, 2),
             (2049, 8, 4), (1025, 16, 1), (2049, 16, 2), (4097, 16, 4), (449, 8, 1), (1901, 16, 2), (3333, 4, 16)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("N,P,W", TUNED_ADJ)
def test_adjoint_every_kernel_configuration_matches_oracle(monkeypatch, N, P, W, mode):
    monkeypatch.setenv("ADSCL_TUNE", "%d:%dx%d" % (N, P, W))
    set_mode(monkeypatch, mode)
    print("adjoint configuration", N, P, W, mode, flush=True)
    # 120 steps of eps = 2 data: the drift E_j(t_n) - E_j(0) is at least 1e-3 of
    # E_j, so L keeps about 11 digits
    Jc, J, K = 6, 3, 9
    T = 120 * 0.25 * (math.pi / 2) / (N - 1)
    eps = np.array([2.0])
    c = coeffs(5 + N, 1, Jc)
    b, L, g, v = run_gpu([N], eps, c, J, T, K)
    classes, cls = b.kernel_stats()
    assert (classes[cls[0]]["P"], classes[cls[0]]["W"]) == (P, W)
    ref = O.objective(N, 2.0, c[0], T=T, J=J, K=K)
    assert v[0] == int(ref["valid"]) == 1
    assert abs(L[0] - ref["L"]) <= LTOL * ref["L"], (L[0], ref["L"])
    e = relmax(g[0], ref["grad"])
    assert e <= GTOL, "N=%d %dx%d: gradient error %.3e" % (N, P, W, e)


@pytest.mark.parametrize("N,ns", [(65, 1), (257, 1), (513, 30), (769, 30), (1025, 30), (1537, 30), (2049, 30)])
def test_adjoint_strong_field_suffix_sums(N, ns):
    """Mode data at eps = 2 with e^-delta(0) of order 1e-9 (delta(0) = 21): the
    end-point cotangents of S near the origin are of order 1/e^-delta, so a
    suffix formed as a total minus a prefix loses about nine digits away from
    the origin; the reverse scans must sum from the outer end (summed as a total
    minus a prefix, these cases missed by 2e-7 to 1e-4).  Short windows make the
    gradient a small difference of the two end points' VJPs; below about 30
    steps on the larger grids that difference falls under the 1e-9 bar's
    rounding floor, so those use 30."""
    Jc, J, K = 6, 3, 9
    T = ns * 0.25 * (math.pi / 2) / (N - 1)
    c = coeffs(1030, 1, Jc)
    print("strong field N", N, "steps", ns, flush=True)
    _, L, g, v = run_gpu([N], np.array([2.0]), c, J, T, K)
    ref = O.objective(N, 2.0, c[0], T=T, J=J, K=K)
    assert v[0] == int(ref["valid"]) == 1
    e = relmax(g[0], ref["grad"])
    assert e <= GTOL, "N=%d, %d steps: gradient error %.3e" % (N, ns, e)
