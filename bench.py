#!/usr/bin/env python
"""Throughput benchmark of the batched AdS4 scalar-collapse evolution on one MI355X.

Workload (seeded, synthetic): 1024 independent instances of Gaussian initial
data, sigma ~ U[1/16, 1/4], eps log-uniform in [1, 40], grid sizes drawn from
{1025, 2049, 4097}, classical RK4 with dt = h/4, evolved to t = 50 or until
min A < 0.02, boundary-time gauge.  One benchmark step is one complete pass over
that batch: initial data and t = 0 constraint solve, then the evolution of every
instance to its end (or collapse), all on the GPU.

Metric: FP64 grid-point RK4 updates per second (one grid point advanced one
full RK4 step), counting only steps actually taken by instances that have not
collapsed.  Printed as one JSON line, with the roofline of the dominant kernel
launch and the CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "FP64 grid-point RK4 updates/s, batched vs single-instance; adjoint grads/s"
UNIT = "grid-point RK4 updates/s"
# Algorithmic work per grid point per RK4 stage of the scheme, counted from its
# definition (exp and the reciprocal are not counted as flops): q 3; p and sigma
# pre-multiplies 2; two 4-point cell rules 12; two scan adds 2; sigma E 1;
# m, A, e^-delta 4; w, f1, f2, g 4; two D stencils and cot^2 x 11; two KO
# stencils 18; right-hand-side adds 2; RK4 combination 8.
FLOP_PER_PT_STAGE = 67.0
BYTES_PER_PT_STEP = 32.0          # read (Phi, Pi)^n, write (Phi, Pi)^{n+1}
PEAK_FP64_TFLOPS = 78.6           # MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz
VALU_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9   # FP64 vector issue ceiling, lane-instructions/s
PEAK_HBM_GBS = 8000.0
# Counter figures of the dominant kernel (HBM bytes per launch from FETCH_SIZE /
# WRITE_SIZE scaled by the copy calibration; VALU and FP64 instructions per
# pt-stage from the SQ counters) are read from the profile summary, and only
# when the digest of the forward kernel's sources it records is the digest of
# the sources in this tree: after any change to the kernel they are null until
# measured again.
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "evolve_batched1024_counters.md")


def kernel_digest():
    """Digest of what the forward kernel is compiled from: stage.h and
    evolve.hip whole, the declarations of internal.h it uses (the per-instance
    status and constants and the kernel's argument block) and its compiler
    flags in build.py."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1706_07413_amd", "csrc")
    h = hashlib.sha256()
    for f in ("stage.h", "evolve.hip"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "internal.h")) as fh:
        t = fh.read()
    i = t.index("struct InstStatus")
    j = t.index("};", t.index("struct EvolveArgs")) + 2
    h.update(t[i:j].encode())
    with open(os.path.join(ROOT, "paper_1706_07413_amd", "build.py")) as fh:
        t = fh.read()
    h.update(t[t.index("def common_flags"):t.index("def _compile")].encode())
    h.update([l for l in t.splitlines() if l.startswith('EXTRA = {"evolve.hip"')][0].encode())
    return h.hexdigest()[:16]


def counter_figures():
    """{"P": .., "W": .., "traffic_bytes": .., "valu_per_pt_stage": .., "fp64_flop_per_pt_stage": ..}
    of the profile summary if it was measured on this tree's kernel, else None."""
    try:
        with open(COUNTER_PROFILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    dig = [l.split(":", 1)[1].strip() for l in lines if l.startswith("kernel-source-digest:")]
    fig = [l.split(":", 1)[1].strip() for l in lines if l.startswith("bench-figures:")]
    if not dig or not fig or dig[0] != kernel_digest():
        return None
    return json.loads(fig[0])


def pt_steps(N, steps):
    return float(np.sum(np.asarray(N, np.float64) * np.asarray(steps, np.float64)))


def adjoint_config3(adscl):
    """One gradient of the single-instance adjoint workload at its stated size
    (N = 4097, 32 mode coefficients, eps = 0.1, T = 100: 1 043 038 steps,
    drift of 16 mode energies, checkpoints every 512 steps)."""
    import torch
    from paper_1706_07413_amd import inputs as I
    cfg = I.config3()
    b = adscl.Batch(cfg["N"], gauge=cfg["gauge"], a_collapse=cfg["a_collapse"], n_modes=32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, g, v = b.adjoint(cfg["eps"], cfg["c"], cfg["J_obj"], cfg["T"], cfg["ckpt_every"])
    dt = time.perf_counter() - t0
    st = b.status()
    b.close()
    return {"workload": "adjoint_N4097: one instance, 32 modes, eps 0.1, T=100 (%d steps), J_obj 16, K 512"
                        % int(st["steps"][0]),
            "grads_per_s": 1.0 / dt, "s_per_gradient": dt, "valid": int(v[0]), "L": float(L[0]),
            "forward_pt_steps": float(cfg["N"][0]) * float(st["steps"][0])}


def adjoint_rate(adscl, T, iters=2, warmup=1):
    """Gradients per second of the batched descent loop: the 256-instance
    mode-data draw (N in {2049, 4097}, 32 modes, drift of 16 modes,
    checkpoints every 512 steps) over a window of T time units; each iteration
    is one forward evolution and one reverse sweep of every instance, replayed
    from a captured graph."""
    import torch
    from paper_1706_07413_amd import inputs as I
    cfg = I.config4()
    b = adscl.Batch(cfg["N"], gauge=cfg["gauge"], a_collapse=cfg["a_collapse"], n_modes=32)
    eps = torch.tensor(cfg["eps"], dtype=torch.float64, device="cuda")
    c = torch.tensor(cfg["c"], dtype=torch.float64, device="cuda")
    if warmup:
        b.descend(eps, c, cfg["J_obj"], T, warmup, ckpt_every=cfg["ckpt_every"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, hist, active = b.descend(eps, c, cfg["J_obj"], T, iters, ckpt_every=cfg["ckpt_every"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    n = len(cfg["N"])
    steps = np.ceil(T / (0.25 * (math.pi / 2) / (np.asarray(cfg["N"], np.float64) - 1)) - 1e-9)
    return {"workload": "batched_adjoint_gd_256: 256 instances, N in {2049,4097}, eps log-U[0.02,0.2], 32 modes, "
                        "J_obj 16, K 512, T=%g%s, %d descent iterations" % (
                            T, "" if T >= 100 else " (a window of the T=100 run)", iters),
            "L_first_last_mean_active": [float(np.nanmean(hist[0].cpu().numpy())),
                                         float(np.nanmean(hist[-1].cpu().numpy()))],
            "grads_per_s": n * iters / dt, "s_per_iteration": dt / iters,
            "forward_pt_steps_per_iteration": float(np.sum(steps * np.asarray(cfg["N"]))),
            "active": int(active.sum().item())}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, n_inst=64, steps=4096):
    """The oracle on the host's cores: the first `n_inst` instances of the
    workload, `steps` RK4 steps each (or to collapse), one instance per OpenMP
    thread, in the parity build (gcc -O2 -ffp-contract=off) and in a timing build
    of the same sources (-O3 -march=native, compiled here for this host)."""
    import tempfile

    import oracle as O
    from oracle import build as OB
    Ns, eps, sig = cfg["N"][:n_inst], cfg["eps"][:n_inst], cfg["sigma"][:n_inst]
    out = {}
    timing_so = os.path.join(tempfile.mkdtemp(prefix="adscl_oracle_"), "liboracle_timing.so")
    OB.build_timing(timing_so)
    for name, lib in (("O2", None), ("O3_native", O.timing_lib(timing_so))):
        t0 = time.perf_counter()
        st, _ = O.evolve_gaussian_batch(Ns, eps, sig, steps, gauge=cfg["gauge"], a_collapse=cfg["a_collapse"],
                                        lib=lib)
        dt = time.perf_counter() - t0
        out[name] = (pt_steps(Ns, st) / dt, O.threads(lib))
    v, cores = out["O3_native"]
    return dict(value=v, unit=UNIT, cores=cores, kind="oracle",
                sample="first %d instances of the 1024-instance workload (N in {1025,2049,4097}), %d RK4 steps "
                       "each or to collapse, one instance per OpenMP thread; oracle sources built -O3 "
                       "-march=native -ffp-contract=off (timing build)" % (n_inst, steps),
                parity_build_value=out["O2"][0], parity_build="gcc -O2 -ffp-contract=off",
                nproc=os.cpu_count(), cpu_model=cpu_model())


# kernel configurations at the tightest lane capacity of each benchmark grid
SINGLE_CANDIDATES = {1025: [(4, 4), (8, 2), (16, 1)], 2049: [(4, 8), (8, 4), (16, 2)],
                     4097: [(4, 16), (8, 8), (16, 4)]}


def single_instance_rates(adscl, steps):
    """Rate of one instance alone on the GPU, per grid size: the best of the
    configurations that hold the grid (the single-instance path is latency
    bound, so its best shape need not be the batch's)."""
    import torch
    rates, shapes = {}, {}
    for N, cands in SINGLE_CANDIDATES.items():
        for P, W in cands:
            os.environ["ADSCL_TUNE"] = "%d:%dx%d" % (N, P, W)
            try:
                b = adscl.Batch([N], a_collapse=0.02)
            finally:
                del os.environ["ADSCL_TUNE"]
            eps = torch.tensor([2.0], dtype=torch.float64, device="cuda")
            sig = torch.tensor([0.2], dtype=torch.float64, device="cuda")
            b.init_gaussian(eps, sig)
            b.step(64, 1e9)
            b.sync()
            t0 = time.perf_counter()
            b.step(steps, 1e9)
            b.sync()
            dt = time.perf_counter() - t0
            b.close()
            if N * steps / dt > rates.get(N, 0.0):
                rates[N] = N * steps / dt
                shapes[N] = "%dx%d" % (P, W)
    return rates, shapes


def large_instance_rate(adscl, steps=4096):
    """The 16385-point two-mode instance (0.05 (e_0 + 0.6 e_1), boundary time)
    alone on the GPU: 8 cooperating workgroups of 2048 points each."""
    from paper_1706_07413_amd import inputs as I
    cfg = I.config1()
    b = adscl.Batch(cfg["N"], gauge=cfg["gauge"], a_collapse=cfg["a_collapse"], n_modes=2)
    b.init_modes(cfg["eps"], np.ascontiguousarray(cfg["c"]))
    b.step(64, 1e9)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps, 1e9)
    b.sync()
    dt = time.perf_counter() - t0
    b.close()
    N = int(cfg["N"][0])
    out = {"workload": "single_twomode_N16385 (t=200 run), a window of %d RK4 steps" % steps,
           "pt_steps_per_s": N * steps / dt, "us_per_step": dt / steps * 1e6,
           "steps_per_s": steps / dt}
    # eight such instances (amplitudes 0.05 .. 0.085) side by side in one launch
    B = 8
    b = adscl.Batch(np.repeat(cfg["N"], B), gauge=cfg["gauge"], a_collapse=cfg["a_collapse"], n_modes=2)
    b.init_modes(0.05 + 0.005 * np.arange(B), np.ascontiguousarray(np.repeat(cfg["c"], B, axis=0)))
    b.step(64, 1e9)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps, 1e9)
    b.sync()
    dt8 = time.perf_counter() - t0
    b.close()
    out["batch_of_8"] = {"pt_steps_per_s": B * N * steps / dt8, "us_per_step": dt8 / steps * 1e6,
                         "over_single": (B * N * steps / dt8) / (N * steps / dt)}
    return out


def paper_table_rates(adscl, steps=2048):
    """The single-instance workloads of the paper's speed tables, on this GPU:
    the dynamic metric at N = 32769 and the frozen metric (A = 1, delta = 0,
    the linear wave) at N = 65537, two-mode data 0.05 (e_0 + 0.6 e_1), a window
    of `steps` steps after 64 warm-up steps: classical RK4, and at N = 32769
    also the paper's RK3, with A solved at every stage and with A evolved by
    Eq. (4) and re-integrated every 16 steps."""
    out = {}
    legs = (("dynamic_N32769", 32769, 0, 4, 0), ("frozen_N65537", 65537, adscl.FROZEN_METRIC, 4, 0),
            # the paper's own integrator (RK3), A solved at every stage and A
            # evolved by Eq. (4) with re-integration every 16 steps
            ("dynamic_N32769_rk3", 32769, 0, 3, 0), ("dynamic_N32769_rk3_evolvedA_K16", 32769, 0, 3, 16))
    for name, N, flags, rk, K in legs:
        b = adscl.Batch([N], a_collapse=0.01, n_modes=2, flags=flags, rk_order=rk, a_reint=K)
        b.init_modes(np.array([0.05]), np.array([[1.0, 0.6]]))
        b.step(64, 1e9)
        b.sync()
        t0 = time.perf_counter()
        b.step(steps, 1e9)
        b.sync()
        dt = time.perf_counter() - t0
        b.close()
        out[name] = {"pt_steps_per_s": N * steps / dt, "us_per_step": dt / steps * 1e6, "steps": steps,
                     "rk_order": rk, "a_reint": K}
    return out


def config1_full(adscl, chunk=65536, spectra_out=None):
    """The whole 16385-point two-mode run of the paper's production resolution:
    0.05 (e_0 + 0.6 e_1), boundary time, to t = 200 (8 344 303 RK4 steps), with
    (Phi, Pi, A, delta, m) stored every 1024 steps and the 64-mode energy
    spectrum of every stored state by the FP64 MFMA projection (8150 spectra,
    in batches of 512 states).  Progress goes to stderr, one line per chunk;
    with `spectra_out` the spectra are saved there (numpy, [states, 64])."""
    import torch
    from paper_1706_07413_amd import inputs as I
    cfg = I.config1()
    N = int(cfg["N"][0])
    J, every = int(cfg["n_modes"]), int(cfg["spec_every"])
    b = adscl.Batch(cfg["N"], gauge=cfg["gauge"], a_collapse=cfg["a_collapse"], n_modes=J)
    b.init_modes(cfg["eps"], np.ascontiguousarray(cfg["c"]))
    dt = 0.25 * (math.pi / 2) / (N - 1)
    n_final = int(math.ceil(cfg["T"] / dt - 1e-9))
    slots = n_final // every + 1
    snaps = torch.zeros((slots, 5, N), dtype=torch.float64, device="cuda")
    con0 = b.constraints()[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while steps < n_final:
        b.step(chunk, cfg["T"], snap_every=every, snaps=snaps)
        st = b.status()
        steps = int(st["steps"][0])
        print("config1: step %d of %d, t = %.3f, %.1f s, state %d" % (steps, n_final, st["t"][0],
              time.perf_counter() - t0, int(st["state"][0])), file=sys.stderr, flush=True)
        if st["state"][0] not in (adscl.RUNNING, adscl.DONE):
            break
    torch.cuda.synchronize()
    t_evolve = time.perf_counter() - t0
    t1 = time.perf_counter()
    E = torch.empty((slots, J), dtype=torch.float64, device="cuda")
    for s0 in range(0, slots, 512):
        e, _, _ = b.spectrum_snaps(J, snaps[s0:s0 + 512])
        E[s0:s0 + e.shape[0]] = e[:, 0, :]
    torch.cuda.synchronize()
    t_spec = time.perf_counter() - t1
    E = E.cpu().numpy()
    con1 = b.constraints()[0]
    st = b.status()
    b.close()
    if spectra_out:
        np.save(spectra_out, E)
    tot = E.sum(axis=1)
    return {"workload": "single_twomode_N16385 to t=200, spectra of 64 modes every %d steps" % every,
            "steps": int(st["steps"][0]), "state": int(st["state"][0]), "t": float(st["t"][0]),
            "evolve_s": t_evolve, "pt_steps_per_s": N * int(st["steps"][0]) / t_evolve,
            "us_per_step": t_evolve / max(int(st["steps"][0]), 1) * 1e6,
            "spectra": slots, "spectra_s": t_spec,
            "E0_E1_first": [float(E[0, 0]), float(E[0, 1])], "E0_E1_last": [float(E[-1, 0]), float(E[-1, 1])],
            "sum_E_first_last": [float(tot[0]), float(tot[-1])],
            "max_mode_with_1e-12_of_energy_last": int(np.max(np.nonzero(E[-1] > 1e-12 * tot[-1])[0])),
            "constraints_t0": [float(x) for x in con0], "constraints_end": [float(x) for x in con1]}


def qp_sweep(adscl, N, eps_values, t_max, rk, a_reint, chunk=262144):
    """The paper's collapse-time study (Sec. III): each approximate quasi-periodic
    family (k_d, mu) of Eq. (13) at every amplitude in `eps_values`, all as one
    batch on grid N, evolved to t_max or collapse (min A < 0.01, the paper's
    threshold); per instance the collapse time and the mass loss
    (M(0) - M(end)) / M(0) of the mass integral of Sec. II, and per family the
    least-squares line t_c = a + b / eps^2 over the instances that collapsed.
    Progress goes to stderr, one line per chunk of steps."""
    import torch
    from paper_1706_07413_amd import inputs as I
    fams = I.QP_FAMILIES
    J = 40
    rows = [(kd, mu, e) for kd, mu in fams for e in eps_values]
    n = len(rows)
    c = np.stack([I.qp_family(kd, mu, J) for kd, mu, _ in rows])
    eps = np.array([e for _, _, e in rows])
    b = adscl.Batch([N] * n, a_collapse=0.01, n_modes=J, rk_order=rk, a_reint=a_reint)
    b.init_modes(eps, np.ascontiguousarray(c))
    M0 = b.constraints()[:, 4].copy()
    n_final = int(math.ceil(t_max / (0.25 * (math.pi / 2) / (N - 1)) - 1e-9))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_done = 0
    while True:
        b.step(chunk, t_max)
        st = b.status()
        running = int(np.sum(st["state"] == adscl.RUNNING))
        steps_done = int(np.max(st["steps"]))
        print("qp sweep: step %d of %d, %d running, %d collapsed, %.1f s" % (
            steps_done, n_final, running, int(np.sum(st["state"] == adscl.COLLAPSED)), time.perf_counter() - t0),
            file=sys.stderr, flush=True)
        if running == 0:
            break
    elapsed = time.perf_counter() - t0
    con = b.constraints()
    b.close()
    M1 = con[:, 4]
    work = float(N) * float(np.sum(st["steps"]))
    fam_out = []
    for kd, mu in fams:
        sel = [i for i, r in enumerate(rows) if r[0] == kd and r[1] == mu]
        tc = [float(st["t_c"][i]) if st["state"][i] == adscl.COLLAPSED else None for i in sel]
        x = np.array([1.0 / eps[i] ** 2 for i, t in zip(sel, tc) if t is not None])
        y = np.array([t for t in tc if t is not None])
        fit = None
        if len(x) >= 3:
            B, A0 = np.polyfit(x, y, 1)
            pred = A0 + B * x
            r2 = 1.0 - np.sum((y - pred) ** 2) / max(np.sum((y - y.mean()) ** 2), 1e-300)
            fit = {"intercept": float(A0), "slope": float(B), "r2": float(r2), "points": int(len(x))}
        fam_out.append({"k_d": kd, "mu": mu, "eps": [float(eps[i]) for i in sel],
                        "inv_eps2": [float(1.0 / eps[i] ** 2) for i in sel], "t_c": tc,
                        "state": [int(st["state"][i]) for i in sel],
                        "mass_loss": [float((M0[i] - M1[i]) / M0[i]) for i in sel],
                        "max_residual_R_A'": [float(con[i, 0]) for i in sel], "fit_t_c_vs_inv_eps2": fit})
    return {"workload": "qp_sweep: the four approximate QP families (k_d in {3,5}, mu in {1,1.75}), 40 modes, "
                        "N=%d, RK%d%s, t_max=%g, collapse at min A < 0.01" % (
                            N, rk, "" if a_reint == 0 else " with A evolved (re-integrated every %d)" % a_reint,
                            t_max),
            "instances": n, "seconds": elapsed, "pt_steps_per_s": work / elapsed, "families": fam_out}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed passes over the batch")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--t-end", type=float, default=50.0,
                    help="end time of every pass (default: the workload's full run, 50)")
    ap.add_argument("--cpu-instances", type=int, default=64,
                    help="instances of the CPU baseline's sample (the workload's first ones)")
    ap.add_argument("--cpu-steps", type=int, default=4096, help="RK4 steps per instance of that sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--large-only", action="store_true",
                    help="only the large-grid legs (the 16385-point instance, eight side by side, the speed-table grids)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint gradient-rate leg")
    ap.add_argument("--adjoint-t", type=float, default=1.0, help="time window of the adjoint leg")
    ap.add_argument("--config1-full", action="store_true",
                    help="run only the whole 16385-point t=200 run with its spectra (about 7 minutes)")
    ap.add_argument("--spectra-out", default=None,
                    help="with --config1-full: save the spectra to this .npy file")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint leg and print its result (for profiling it)")
    ap.add_argument("--adjoint-iters", type=int, default=2, help="timed descent iterations of the adjoint leg")
    ap.add_argument("--adjoint-warmup", type=int, default=1, help="untimed descent iterations before them")
    ap.add_argument("--adjoint-full", action="store_true",
                    help="run only the adjoint workloads at their stated length (T = 100): one gradient of the "
                         "single instance, then --adjoint-iters descent iterations of the 256 instances")
    ap.add_argument("--qp-sweep", action="store_true",
                    help="run only the collapse-time sweep of the approximate quasi-periodic families")
    ap.add_argument("--qp-n", type=int, default=4097, help="grid of the sweep")
    ap.add_argument("--qp-eps", default="0.04,0.03525,0.03106,0.02737,0.02412,0.02125,0.01873,0.0165,0.01454,"
                                        "0.01281,0.01129,0.009951,0.008769,0.007727,0.006809,0.006",
                    help="comma-separated amplitudes of the sweep")
    ap.add_argument("--qp-tmax", type=float, default=500.0)
    ap.add_argument("--qp-rk", type=int, default=3, help="Runge-Kutta order of the sweep (the paper's: 3)")
    ap.add_argument("--qp-reint", type=int, default=0,
                    help="0: A solved at every stage; K: A evolved, re-integrated every K steps")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the workload, run a plain device copy of this many bytes "
                         "(calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_bytes:
        import torch
        n = args.copy_bytes // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "dispatches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the instances are independent, and a run on several "
              "GPUs would shard the batch by instance, which this benchmark does not do.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1706_07413_amd import adscl
    from paper_1706_07413_amd import inputs as I

    torch.cuda.set_device(0)
    cfg = I.config2()
    # kernel configuration per grid size (the batch's and the adjoint workload's),
    # measured on this GPU before any timed work
    tuned = adscl.autotune(sorted(set(int(n) for n in cfg["N"]) | {2049, 4097}), steps=256, apply=True)
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_rate(adscl, args.adjoint_t, args.adjoint_iters, args.adjoint_warmup)}))
        return
    if args.adjoint_full:
        r3 = adjoint_config3(adscl)
        print("adjoint_N4097 T=100: %.1f s per gradient" % r3["s_per_gradient"], file=sys.stderr, flush=True)
        r4 = adjoint_rate(adscl, 100.0, args.adjoint_iters, 0)
        print(json.dumps({"adjoint_config3_T100": r3, "adjoint_gd256_T100": r4}))
        return
    if args.qp_sweep:
        eps_values = [float(e) for e in args.qp_eps.split(",")]
        print(json.dumps({"qp_sweep": qp_sweep(adscl, args.qp_n, eps_values, args.qp_tmax, args.qp_rk,
                                               args.qp_reint)}))
        return
    if args.large_only:
        print(json.dumps({"large_instance": large_instance_rate(adscl), "paper_tables": paper_table_rates(adscl)}))
        return
    if args.config1_full:
        print(json.dumps({"config1_full": config1_full(adscl, spectra_out=args.spectra_out)}))
        return
    T = args.t_end
    eps = torch.tensor(cfg["eps"], dtype=torch.float64, device="cuda")
    sig = torch.tensor(cfg["sigma"], dtype=torch.float64, device="cuda")
    batch = adscl.Batch(cfg["N"], gauge=cfg["gauge"], a_collapse=cfg["a_collapse"], flags=adscl.TIME_KERNELS)

    def one_pass():
        batch.init_gaussian(eps, sig)
        batch.step(1 << 40, T)
        batch.sync()
        return batch.status()

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    work = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = one_pass()
        work += pt_steps(cfg["N"], st["steps"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = work / elapsed

    # roofline of the dominant launch (the class launch of the last pass that
    # did the most grid-point updates)
    classes, cls = batch.kernel_stats()
    work_k = [pt_steps(np.asarray(cfg["N"])[cls == j], st["steps"][cls == j]) for j in range(len(classes))]
    k = int(np.argmax(work_k))
    unit_steps = work_k[k]
    ms = classes[k]["last_ms"]
    pt_stage_rate = unit_steps * 4 / (ms * 1e-3)
    achieved = pt_stage_rate * FLOP_PER_PT_STAGE / 1e12
    cf = counter_figures()
    if cf is not None and (cf.get("P"), cf.get("W")) != (classes[k]["P"], classes[k]["W"]):
        cf = None
    states = np.bincount(st["state"], minlength=4)
    per_n = {}
    for n in (1025, 2049, 4097):
        sel = np.asarray(cfg["N"]) == n
        per_n[str(n)] = {"instances": int(sel.sum()), "collapsed": int((st["state"][sel] == 1).sum()),
                         "pt_steps": pt_steps(np.asarray(cfg["N"])[sel], st["steps"][sel])}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched_gaussian_1024: 1024 instances, N in {1025,2049,4097}, "
                               "eps log-U[1,40], sigma U[1/16,1/4], RK4 dt=h/4, t_end=%g, collapse min A<0.02" % T,
                   "instances": int(len(cfg["N"])), "t_end": T,
                   "pt_steps_per_pass": work / args.steps,
                   "collapsed": int(states[1]), "done": int(states[3]), "by_N": per_n},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": cf["traffic_bytes"] if cf else None,
                     "kernel": "evolve_kernel<P=%d,W=%d> (%d instances)" % (classes[k]["P"], classes[k]["W"],
                                                                          classes[k]["members"]),
                     "launch_ms": ms, "pt_stages_per_launch": unit_steps * 4,
                     "flop_per_pt_stage": FLOP_PER_PT_STAGE, "flop_count": "algorithmic, from the scheme",
                     "kernel_source_digest": kernel_digest(),
                     # from the SQ counters of this kernel (null when the kernel changed since)
                     "executed_fp64_flop_per_pt_stage": cf["fp64_flop_per_pt_stage"] if cf else None,
                     "executed_frac": (pt_stage_rate * cf["fp64_flop_per_pt_stage"] / 1e12 / PEAK_FP64_TFLOPS
                                       if cf else None),
                     "valu_instr_per_pt_stage": cf["valu_per_pt_stage"] if cf else None,
                     "valu_issue_frac": (pt_stage_rate * cf["valu_per_pt_stage"] / VALU_LANE_INSTR_PER_S
                                         if cf else None)},
        "effective_hbm_GBs": value * BYTES_PER_PT_STEP / 1e9,
        "launches": classes,
        "autotune": {str(N): {"P": P, "W": W, "pt_steps_per_s": r} for N, (P, W, r) in tuned.items()},
    }
    if not args.no_single:
        rates, shapes = single_instance_rates(adscl, 4096)
        N = np.asarray(cfg["N"])
        per = np.asarray(cfg["N"], np.float64) * st["steps"]
        t_single = sum(float(per[N == n].sum()) / rates[n] for n in rates)
        out["single_instance"] = {"rates": {str(n): r for n, r in rates.items()},
                                  "shapes": {str(n): v for n, v in shapes.items()},
                                  "batched_over_single": value / (work / args.steps / t_single)}
    if not args.no_single:
        out["large_instance"] = large_instance_rate(adscl)
        out["paper_tables"] = paper_table_rates(adscl)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_rate(adscl, args.adjoint_t, args.adjoint_iters, args.adjoint_warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_instances, args.cpu_steps)
    batch.close()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
