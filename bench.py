"""Throughput of the fused reduced ES-BGK + rotational-energy LB step on one GPU.

Workload (default): 3D Taylor-Green vortex on 256^3 bcc cells
(33,554,432 sites), Ma = 0.1, Re = 1600, delta = 2 (gamma = 7/5), Pr = 0.71,
mu_b/mu = 0.6; populations stored in FP32 as deviations from the rest
weights, per-site solve and reductions in FP64; CN reading, F3 equilibrium.
Synthetic analytic initial field, resident in HBM before the timed region.

Prints one JSON line.  MLUPS = 1e-6 x site updates per second (a cell holds
two sites).  The roofline object is for the dominant kernel (the fused
pull-collide kernel), timed live with HIP events on its own stream.

The "sweep" object is the batched-sweep experiment on the 512-case mix of
1D Couette layers (L ~ U{256..4096}, Kn ~ logU[1e-3, 1e-1]) and normal-shock
lines (Mach ~ U[1.1, 4]), run to residual 1e-8 (with a stated per-case step
cap) cold in one persistent batched launch per kind, warm-started from the
coordinate MLP (trained on the steady states that the solver reaches for a
second seeded set of 4096 cases), and one case at a time through the
single-grid path (a seeded subset, scaled to the whole set).  `--sweep` runs
it alone, `--no-sweep` skips it.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

THETA0 = 0.2948964908710633
HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS + % of HBM roofline (fused step); sweep time-to-residual 1e-8 plain vs batched+MLP"
KERNEL_SOURCES = ("pgk.hip", "device.hpp", "lattice.hpp", "e2.hpp")


def algorithmic_bytes(precision):
    """Bytes the method must move per site update.

    Whole step: every population read and written once (2 x 41 x elt) and
    theta_R read and written once (2 x 8).  Fused pull-collide kernel alone:
    the populations plus the theta_R read.
    """
    elt = 4 if precision == 1 else 8
    return dict(step=2 * 41 * elt + 16, k_lb=2 * 41 * elt + 8)


def tgv_params(n, Ma=0.1, Re=1600.0, gamma=1.4):
    U = Ma * math.sqrt(gamma * THETA0)
    nu = U * (n / (2 * math.pi)) / Re
    return U, nu


def cpu_baseline(n_cpu, steps_cpu):
    import numpy as np  # noqa: F401

    import oracle
    from oracle.params import resolve
    from paper_2201_05280_amd import inputs
    U, nu = tgv_params(n_cpu)
    p = resolve(nu, 0.71, 0.6, 2.0)
    o = oracle.Oracle(n_cpu, n_cpu, n_cpu)
    o.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    f = inputs.taylor_green(n_cpu, U)
    o.init(f["rho"], f["u"], f["thT"], f["thR"])
    o.step(1)  # first touch
    t0 = time.perf_counter()
    o.step(steps_cpu)
    dt = time.perf_counter() - t0
    ns = 2 * n_cpu ** 3
    out = dict(value=ns * steps_cpu / dt / 1e6, unit="MLUPS", cores=oracle.threads(), kind="oracle",
               sample="Taylor-Green %d^3 cells (%d sites, same Ma and Re), FP64 oracle, %d steps, %.1f s"
                      % (n_cpu, ns, steps_cpu, dt))
    out["thread_sweep"] = cpu_thread_sweep(oracle.threads())
    return out


def cpu_thread_sweep(max_threads, n=32, steps=20):
    """Oracle MLUPS on a small Taylor-Green sample (n^3 cells, `steps` steps)
    with 1, 2, 4, ... threads up to max_threads, each in a child process with
    OMP_NUM_THREADS set (the OpenMP team size is fixed at start-up)."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); import bench, oracle; "
            "from oracle.params import resolve; from paper_2201_05280_amd import inputs; "
            "U, nu = bench.tgv_params(%d); p = resolve(nu, 0.71, 0.6, 2.0); o = oracle.Oracle(%d, %d, %d); "
            "o.set_params(p['tau'], p['tau1'], p['b'], p['kr'], p['delta']); f = inputs.taylor_green(%d, U); "
            "o.init(f['rho'], f['u'], f['thT'], f['thR']); o.step(1); t0 = time.perf_counter(); o.step(%d); "
            "print(2 * %d ** 3 * %d / (time.perf_counter() - t0) / 1e6)") % (ROOT, n, n, n, n, n, steps, n, steps)
    res, t = {}, 1
    while t <= max_threads:
        env = dict(os.environ, OMP_NUM_THREADS=str(t))
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        if r.returncode == 0:
            res[str(t)] = round(float(r.stdout.strip().splitlines()[-1]), 2)
        t *= 2
    return {"sample": "Taylor-Green %d^3 cells, %d steps" % (n, steps), "MLUPS_by_threads": res}


def kernel_source_sha():
    """First 16 hex digits of the SHA-256 over the single-grid kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2201_05280_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(n, precision):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy kernel),
    or None when the kernel sources changed since the counters were taken or
    the workload differs."""
    path = os.path.join(ROOT, "profiles", "k_lb_tgv256_fp32dev.md")
    if n != 256 or precision != 1 or not os.path.exists(path):
        return None
    sha = kernel_source_sha()
    vals = {}
    for line in open(path):
        line = line.strip()
        for key in ("k_lb traffic_bytes_per_launch:", "source_sha256_16:"):
            if line.startswith(key):
                vals[key] = line[len(key):].split()[0]
    if vals.get("source_sha256_16:") != sha:
        return None
    return float(vals["k_lb traffic_bytes_per_launch:"])


def soa41_bytes(nbytes):
    """Largest size <= nbytes of 41 float arrays whose length is a multiple of
    64 (every array starts on a 256-byte boundary, as the populations do)."""
    return nbytes // (41 * 4 * 64) * (41 * 4 * 64)


def copy_probe(torch, nbytes=4 << 30, reps=10, quick=False):
    """Plain device copies of nbytes (n read + n written) timed with events:
    the runtime's own copy and the project's float4 copy kernels (quick: the
    runtime copy and the fastest kernel only)."""
    import ctypes
    L = ctypes.CDLL(os.path.join(ROOT, "paper_2201_05280_amd", "libpgk_probe.so"))
    L.pgk_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_void_p]
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream().cuda_stream
    out = {"bytes_moved": 2 * nbytes}
    variants = [("runtime", None)] + [("float4_b%d" % nb, (0, nb)) for nb in (512, 1024, 2048)] + \
               [("float4_nt_b%d" % nb, (1, nb)) for nb in (1024,)] + [("float1", (2, 0))] + \
               [("float4_x%d" % u, (v, 0)) for u, v in ((1, 7), (4, 3), (8, 4), (16, 5))]
    # the population layout of the fused step: 41 streams of one float per site
    variants.append(("soa41_streams", (6, 0)))
    if quick:
        variants = [("runtime", None), ("float4_x1", (7, 0)), ("float4_x4", (3, 0)), ("soa41_streams", (6, 0))]
    for name, v in variants:
        def run():
            if v is None:
                b.copy_(a)
            else:
                nb = nbytes if v[0] != 6 else soa41_bytes(nbytes)
                rc = L.pgk_probe_copy(b.data_ptr(), a.data_ptr(), nb, v[0], v[1], stream)
                assert rc == 0
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nb = nbytes if v is None or v[0] != 6 else soa41_bytes(nbytes)
        out[name + "_GBs"] = round(2 * nb / ms / 1e6, 1)
    del a, b
    return out


def single_grid_run(case, fields, tol, max_steps, time_cap=1e30, K=128, stream=None, stall=0):
    """One 1D case through the single-grid path: chunks of K steps, the
    one-step residual taken from two moment reads at the end of each chunk
    (the batched kernel's rule).  Stops at residual `tol` (status 1), a
    non-finite residual (2), `max_steps` or `time_cap` seconds (3), or when the
    residual has not halved within `stall` steps (4, 0 = off).  Returns
    (steps, residual, status, moments, seconds)."""
    import numpy as np

    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd import cases as C
    p = case["params"]
    shock = case["kind"] == C.SHOCK
    kind = pgk.DIRICHLET if shock else pgk.WALL
    s = pgk.Solver(case["L"], 1, 1, precision=pgk.FP64, bc_x=(kind, kind),
                   equilibrium=pgk.E2 if shock else pgk.F3, stream=stream)
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    if shock:
        up, dn = case["up"], case["down"]
        s.set_bc_x(0, up[0], (up[1], 0, 0), up[2])
        s.set_bc_x(1, dn[0], (dn[1], 0, 0), dn[2])
        axis = 0
    else:
        s.set_bc_x(0, 1.0, (0, 0, 0), THETA0)
        s.set_bc_x(1, 1.0, (0, case["U"], 0), THETA0)
        axis = 1
    s.init(fields["rho"], fields["u"], fields["thT"], fields["thR"])
    t0 = time.perf_counter()
    steps, resid, status, best, since, b = 0, 1.0, 3, 1e300, 0, None
    while steps < max_steps and time.perf_counter() - t0 < time_cap:
        s.step(K - 1)
        a = s.moments()
        s.step(1)
        b = s.moments()
        steps += K
        rs = []
        for k, v in (("rho", None), ("u", axis), ("thT", None), ("thR", None)):
            x0 = a[k] if v is None else a[k][v]
            x1 = b[k] if v is None else b[k][v]
            rs.append(float(np.linalg.norm(x1 - x0) / max(np.linalg.norm(x1), 1e-300)))
        # max() would pass over a NaN that is not its first argument
        resid = max(rs) if np.isfinite(rs).all() else float("nan")
        if not np.isfinite(resid):
            status = 2
            break
        if resid <= tol:
            status = 1
            break
        if resid < 0.5 * best:
            best, since = resid, 0
        elif stall and (since := since + K) >= stall:
            status = 4
            break
    dt = time.perf_counter() - t0
    s.close()
    return steps, resid, status, b, dt


def plain_case(case, tol, max_steps, time_cap, K=128):
    """One case from its cold start through the single-grid path (the plain,
    unbatched solver); returns (steps, residual, seconds)."""
    from paper_2201_05280_amd import cases as C
    steps, resid, _, _, dt = single_grid_run(case, C.cold_fields([case]), tol, max_steps, time_cap, K)
    return steps, resid, dt


def shear_wave_summary(steps=2000):
    """The 2D periodic shear wave, 64 x 64 x 1 cells, FP64 (nu 0.01, Pr 0.71,
    mu_b/mu 0.6, delta 2, u_x = 0.01 sin(2 pi y / 64)): amplitude decay over
    `steps` steps against exp(-nu k^2 t), and the drift of mass, momentum and
    total energy."""
    import numpy as np
    import torch

    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd import inputs
    n = 64
    p = pgk.resolve(0.01, 0.71, 0.6, 2.0)
    s = pgk.Solver(n, n, 1, precision=pgk.FP64)
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    f = inputs.shear_wave(n, n, 1, amp=0.01)
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    y = inputs.positions(n, n, 1)[1]
    mode = np.sin(2 * np.pi * y / n)
    a0 = float(f["u"][0] @ mode / (mode @ mode))
    c0 = s.conserved()
    s.step(steps)
    m = s.moments()
    c1 = s.conserved()
    # rate: a further run of the same length, the step graph already recorded
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    a1 = float(m["u"][0] @ mode / (mode @ mode))
    k = 2 * np.pi / n
    ratio, expect = a1 / a0, math.exp(-p["nu"] * k * k * steps)
    drift = [(c1[i] - c0[i]) / c0[0] for i in range(4)] + [(c1[4] - c0[4]) / c0[4]]
    return {"cells": "64x64x1", "sites": 2 * n * n, "steps": steps, "amplitude_ratio": round(ratio, 6),
            "exp_minus_nu_k2_t": round(expect, 6), "decay_rate_rel_err": round(math.log(ratio) / math.log(expect) - 1, 5),
            "conservation_drift": drift, "MLUPS": round(2 * n * n * steps / dt / 1e6, 1)}


def shock_summary(max_steps=60000):
    """Normal-shock lines of 4096 cells between Dirichlet faces holding the
    model's own jump states, E2 equilibrium, run until the one-step residual
    stops falling (or reaches 1e-11): Mach 1.5 (upstream at the lattice
    temperature) and Mach 3 (upstream theta 0.08), FP64 and FP32 storage."""
    import numpy as np
    import torch

    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd import inputs
    from paper_2201_05280_amd.shock import discrete_rankine_hugoniot, profile_metrics, tanh_profile

    L = 4096
    x = inputs.positions(L, 1, 1)[0]

    def resid(a, b):
        r = 0.0
        for k, v in (("rho", None), ("u", 0), ("thT", None), ("thR", None)):
            x0 = a[k] if v is None else a[k][v]
            x1 = b[k] if v is None else b[k][v]
            d = float(np.linalg.norm(x1 - x0) / np.linalg.norm(x1))
            r = max(r, d) if d == d else d   # a NaN stays NaN
        return r

    out = {"cells": L, "sites": 2 * L, "equilibrium": "E2", "delta": 2.0, "Pr": 0.71, "mu_b/mu": 0.8,
           "nu_upstream": "2 c_s (upstream mean free path nu sqrt(pi/(2 theta1)) = 2.97 cells)"}
    for Ma, th1 in ((1.5, THETA0), (3.0, 0.08)):
        up, down = discrete_rankine_hugoniot(Ma, 2.0, th1)
        _, ideal = inputs.rankine_hugoniot(Ma, 1.4, th1)
        nu = 2.0 * math.sqrt(1.4 * th1)
        p = pgk.resolve(nu, 0.71, 0.8, 2.0)
        lam1 = nu * math.sqrt(math.pi / (2 * th1))
        case = {"theta1": th1, "upstream": [round(v, 6) for v in up], "downstream": [round(v, 6) for v in down],
                "downstream_vs_ideal_gas_jump": [round(a / b - 1, 5) for a, b in zip(down, ideal)]}
        final = {}
        for prec, name in ((pgk.FP64, "fp64"), (pgk.FP32DEV, "fp32dev")):
            s = pgk.Solver(L, 1, 1, precision=prec, bc_x=(pgk.DIRICHLET, pgk.DIRICHLET), equilibrium=pgk.E2)
            s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
            s.set_bc_x(0, up[0], (up[1], 0, 0), up[2])
            s.set_bc_x(1, down[0], (down[1], 0, 0), down[2])
            f = tanh_profile(L, up, down)
            s.init(f["rho"], f["u"], f["thT"], f["thR"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            steps, hist = 0, []
            while steps < max_steps:
                s.step(4999)
                a = s.moments()
                s.step(1)
                b = s.moments()
                steps += 5000
                hist.append(resid(a, b))
                if hist[-1] < 1e-11 or (len(hist) > 3 and hist[-1] > 0.7 * hist[-4]):
                    break
            dt = time.perf_counter() - t0
            s.close()
            pos, thick = profile_metrics(x, b["rho"], up, down)
            final[name] = (pos, b)
            case[name] = {"steps": steps, "residual": float("%.3e" % hist[-1]), "seconds": round(dt, 2),
                          "MLUPS": round(2 * L * steps / dt / 1e6, 1), "shock_position": round(pos, 4),
                          "thickness_cells": round(thick, 3), "thickness_mean_free_paths": round(thick / lam1, 3)}
        # FP32 storage against FP64 at steady state: the shock may settle at a
        # slightly different place, so the profiles are compared with the two
        # positions aligned, each field normalised by its jump
        (p64, m64), (p32, m32) = final["fp64"], final["fp32dev"]
        o = np.argsort(x)
        xs = x[o]
        d = p32 - p64
        inside = (xs + d >= xs[0]) & (xs + d <= xs[-1])
        err = {}
        for k, v, j in (("rho", None, 0), ("u", 0, 1), ("thT", None, 2), ("thR", None, 2)):
            a32 = (m32[k] if v is None else m32[k][v])[o]
            a64 = (m64[k] if v is None else m64[k][v])[o]
            diff = (np.interp(xs[inside] + d, xs, a32) - a64[inside]) / abs(down[j] - up[j])
            err[k] = {"Linf": float("%.3e" % np.abs(diff).max()), "L2": float("%.3e" % np.sqrt((diff ** 2).mean()))}
        case["fp32dev_vs_fp64_profile_error_aligned"] = err
        case["fp32dev_vs_fp64_shift_cells"] = round(d, 4)
        out["Ma%.1f" % Ma] = case
    return out


def mlp_minibatch_summary(sizes=(4096, 8192)):
    """The same training at larger minibatches: more points per Adam step run
    the two kernels over more of the chip (higher points/s), and fewer Adam
    steps per epoch leave a higher loss after the same epochs."""
    out = []
    for mb in sizes:
        r = mlp_train_summary(batch=mb)
        out.append({k: r[k] for k in ("minibatch", "seconds", "us_per_minibatch", "points_per_s", "TFLOPs",
                                      "loss_first_last")})
    return out


def mlp_train_summary(n=291240, epochs=100, batch=2048):
    """Training rate of the warm-start network: n seeded synthetic points with
    the sweep's input shape (six features uniform in [-1, 1], four smooth
    targets), He-uniform start, epochs of minibatch Adam at 2e-3 / 5e-4 /
    1.25e-4 (40 / 30 / 30 epochs, the sweep's schedule).  The flop count per
    point is the forward product's 100,864 plus twice that for the backward
    pass (data and weight gradients)."""
    import numpy as np
    import torch

    from paper_2201_05280_amd.inputs import mlp_init
    from paper_2201_05280_amd.mlp import MLP

    rng = np.random.default_rng(220105282)
    X = rng.uniform(-1, 1, (n, 6)).astype(np.float32)
    Y = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], X[:, 2] ** 2 - 0.3, np.cos(X[:, 3] + X[:, 4]),
                  0.5 * X[:, 5] * X[:, 0]], 1).astype(np.float32)
    m = MLP(nmax=max(8192, batch))
    m.set_params(mlp_init(220105280))
    m.train(X[:8192], Y[:8192], epochs=1, batch=batch, lr=1e-3, seed=1)   # untimed warm-up
    m.set_params(mlp_init(220105280))
    stages = [(2e-3, 40), (5e-4, 30), (1.25e-4, 30)]
    total = sum(e for _, e in stages)
    stages = [(lr, e * epochs // total) for lr, e in stages]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for k, (lr, ep) in enumerate(stages):
        losses += list(m.train(X, Y, epochs=ep, batch=batch, lr=lr, seed=7 + k))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    m.close()
    ep = sum(e for _, e in stages)
    nmb = ep * ((n + batch - 1) // batch)
    flop = 3 * 100864 * n * ep
    return {"points": n, "epochs": ep, "minibatch": batch, "seconds": round(dt, 3),
            "us_per_minibatch": round(dt / nmb * 1e6, 1), "points_per_s": round(n * ep / dt),
            "TFLOPs": round(flop / dt / 1e12, 2), "bf16_peak_TFLOPs": 2500.0,
            "loss_first_last": [float("%.4g" % losses[0]), float("%.4g" % losses[-1])],
            "data": "synthetic, seeded"}


def sweep(args, extra=None):
    """Time to residual 1e-8 of a seeded mix of 1D cases (Couette layers and
    normal-shock lines): plain (one case at a time), batched cold, batched
    warm-started by the MLP.

    The network trains on every steady state the solver reached for the
    training cases, together with `extra` (features, targets, training-case
    descriptions) from an earlier sweep, and starts a held-out case only when
    its Mach and Knudsen numbers lie within the range of the converged
    training cases of its kind; any other case starts cold (the plain LB is
    the fallback).  Returns (report, (features, targets, converged cases))."""
    import numpy as np
    import torch

    from paper_2201_05280_amd import cases as C
    from paper_2201_05280_amd.batch import Batch
    from paper_2201_05280_amd.inputs import mlp_init
    from paper_2201_05280_amd.mlp import MLP
    from paper_2201_05280_amd.shock import profile_metrics

    S = 220105280
    tol = 1e-8
    kw = dict(L_range=(args.sweep_lmin, args.sweep_lmax), Kn_range=(args.sweep_knmin, args.sweep_knmax),
              shock_fraction=args.sweep_shock_frac, shock_Ma_range=(args.sweep_mamin, args.sweep_mamax),
              shock_Kn_range=(2e-3, 6e-3))
    cnt_t, cnt_r = {}, {}
    test, red_t = C.sweep_cases(args.sweep_n, S, counts=cnt_t, **kw)
    train, red_r = C.sweep_cases(args.sweep_train, S + 1, counts=cnt_r, **kw)
    is_shock = np.array([c["kind"] == C.SHOCK for c in test])
    out = {"metric": "sweep time-to-residual 1e-8 plain vs batched+MLP", "unit": "s", "tol": tol,
           "cases": len(test), "shock_cases": int(is_shock.sum()), "train_cases": len(train),
           "infeasible_at_draw": {
               "pr_mub_pairs_redrawn": {"held_out": red_t, "training": red_r},
               "shock_mach_without_jump_states_redrawn": {"held_out": cnt_t["shock_no_states"],
                                                          "training": cnt_r["shock_no_states"]},
               "shocks_with_upstream_below_theta0": {"held_out": cnt_t["shock_cold_upstream"],
                                                     "training": cnt_r["shock_cold_upstream"]}},
           "distribution": "L~U{%d..%d}, delta in {2,3}, Pr~U[0.67,1], mu_b/mu~U[0,2] (infeasible pairs redrawn); "
                           "%.0f%% Couette (F3): Ma_w~U[0.1,0.5], Kn=nu/(c_s L)~logU[%g,%g]; "
                           "%.0f%% normal shocks (E2): Ma~U[%g,%g] (upstream at theta0, or at the warmest "
                           "theta1 <= 0.12 with E2 jump states above about Mach 2.65), Kn=lambda1/L~logU[0.002,0.006]"
                           % (args.sweep_lmin, args.sweep_lmax, 100 * (1 - args.sweep_shock_frac), args.sweep_knmin,
                              args.sweep_knmax, 100 * args.sweep_shock_frac, args.sweep_mamin, args.sweep_mamax),
           "step_cap_per_case": {"held_out": args.sweep_max_steps, "training": args.sweep_train_max_steps},
           "wall_time_budget_per_batch_s": {"held_out": args.sweep_time_budget or None,
                                            "training": args.sweep_train_time_budget or None},
           "stall_window_steps": {"couette": args.sweep_stall, "shock": args.sweep_stall_shock}}

    def run_batch(cs, fields, label, tune_only=False, max_steps=None, train_budget=None):
        """Run the cases to the tolerance: the Couette layers (F3, any
        work-group size) and the shock lines (E2, work-groups of 256) as two
        batches, each one persistent launch per chunk on its own stream, run
        concurrently from two host threads; results in the order of cs."""
        import threading
        offs = np.concatenate([[0], np.cumsum([2 * c["L"] for c in cs])])
        groups = [[i for i, c in enumerate(cs) if c["kind"] == k] for k in (C.COUETTE, C.SHOCK)]
        groups = [g for g in groups if g]
        res = [None] * len(groups)

        wall = [0.0] * len(groups)

        def worker(j, idx):
            tw = time.perf_counter()
            stream = torch.cuda.Stream()
            sub = [cs[i] for i in idx]
            sel = np.concatenate([np.arange(offs[i], offs[i + 1]) for i in idx])
            b = Batch(C.to_batch_cases(sub), stream=stream)
            b.init(fields["rho"][sel], fields["u"][:, sel], fields["thT"][sel], fields["thR"][sel])
            b.config(0, 0)
            b.stall(args.sweep_stall_shock if cs[idx[0]]["kind"] == C.SHOCK else args.sweep_stall)
            stream.synchronize()
            # tune_only: let the autotuner time its candidates and cache the choice;
            # otherwise advance in stages of 256 to 2048 steps, each about 10 s
            # of work (a capped case runs on when the cap rises), report each
            # stage and stop when the wall-time budget is spent
            cap = 512 if tune_only else (max_steps or args.sweep_max_steps)
            done, stage = 0, 256
            while True:
                ts = time.perf_counter()
                done = min(cap, done + stage)
                steps, resid, status = b.run(done, tol)
                # next stage: about 10 s of work, 256 to 2048 steps
                per = (time.perf_counter() - ts) / stage
                stage = int(min(2048, max(256, 10.0 / max(per, 1e-9) // 256 * 256)))
                print("# %s %s: %d steps, running %d of %d, %.1f s" % (label, cs[idx[0]]["kind"], done,
                      int((status == 3).sum()) if done < cap else 0, len(idx), time.perf_counter() - tw),
                      file=sys.stderr, flush=True)
                if done >= cap or not (status == 3).any():
                    break
                budget = train_budget if train_budget is not None else args.sweep_time_budget
                if not tune_only and budget and time.perf_counter() - tw > budget:
                    break   # out of wall time: the cases still running stay capped
            res[j] = (idx, sel, steps, resid, status, b.moments(), b.tuned())
            b.close()
            wall[j] = time.perf_counter() - tw

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = [threading.Thread(target=worker, args=(j, g)) for j, g in enumerate(groups)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        dt = time.perf_counter() - t0
        if any(r is None for r in res):
            raise RuntimeError("a batch failed")
        n, ns = len(cs), int(offs[-1])
        steps, resid, status = np.zeros(n, dtype=np.int64), np.zeros(n), np.zeros(n, dtype=np.int64)
        m = dict(rho=np.zeros(ns), u=np.zeros((3, ns)), thT=np.zeros(ns), thR=np.zeros(ns))
        cfg = []
        for (idx, sel, st, rs, stt, mm, tuned), w in zip(res, wall):
            steps[idx], resid[idx], status[idx] = st, rs, stt
            for k in ("rho", "thT", "thR"):
                m[k][sel] = mm[k]
            m["u"][:, sel] = mm["u"]
            cfg.append({"kind": cs[idx[0]]["kind"], "cases": len(idx), "wg": tuned[0], "K": tuned[1],
                        "ns_per_site_update": round(tuned[2], 4), "wall_s": round(w, 2)})

        print("# %s: %.2f s, steps median %d max %d, status counts %s, configs %s"
              % (label, dt, np.median(steps), steps.max(), np.bincount(status, minlength=5).tolist(), cfg),
              file=sys.stderr, flush=True)
        return dict(time=dt, steps=steps, status=status, resid=resid, m=m, cfg=cfg)

    # training data: steady states of the training cases (cold batched runs);
    # the first run also settles the autotuner's choice for this case mix
    t_gen0 = time.perf_counter()
    tr = run_batch(train, C.cold_fields(train), "train cold", max_steps=args.sweep_train_max_steps,
                   train_budget=args.sweep_train_time_budget)
    t_gen = time.perf_counter() - t_gen0
    tr_shock = np.array([c["kind"] == C.SHOCK for c in train])
    ok = np.repeat(tr["status"] == 1, [2 * c["L"] for c in train])
    X = C.features(train)[ok]
    Y = C.targets(train, tr["m"])[ok]
    conv = [c for c, st in zip(train, tr["status"]) if st == 1]
    own_points = int(len(X))
    if extra is not None:
        X, Y, conv = np.concatenate([X, extra[0]]), np.concatenate([Y, extra[1]]), conv + extra[2]
    mlp = MLP(nmax=max(8192, args.sweep_mlp_batch))
    mlp.set_params(mlp_init(S))
    t0 = time.perf_counter()
    losses = []
    for k, stage in enumerate(args.sweep_lr_schedule.split(",")):
        lr, ep = stage.split(":")
        losses += list(mlp.train(X, Y, epochs=int(ep), batch=args.sweep_mlp_batch, lr=float(lr), seed=S + k))
    t_train = time.perf_counter() - t0
    print("# mlp trained on %d points in %.1f s, loss %.3e -> %.3e" % (len(X), t_train, losses[0], losses[-1]),
          file=sys.stderr, flush=True)

    # settle the autotuner's choice for the held-out mix outside the timed runs,
    # so that the cold and the warm run use the same configuration
    run_batch(test, C.cold_fields(test), "held-out tuning (untimed)", tune_only=True)
    cold = run_batch(test, C.cold_fields(test), "held-out cold")
    t0 = time.perf_counter()
    y = mlp.forward(C.features(test)).cpu().numpy()
    t_infer = time.perf_counter() - t0
    # warm start inside the range of the converged training cases of the same
    # kind (Mach and log Kn); cold start elsewhere
    rng_kind = {}
    for kind in (C.COUETTE, C.SHOCK):
        cc = [c for c in conv if c["kind"] == kind]
        if cc:
            rng_kind[kind] = (min(c["Ma"] for c in cc), max(c["Ma"] for c in cc),
                              min(c["Kn"] for c in cc), max(c["Kn"] for c in cc))
    inside = np.array([c["kind"] in rng_kind and rng_kind[c["kind"]][0] <= c["Ma"] <= rng_kind[c["kind"]][1]
                       and rng_kind[c["kind"]][2] <= c["Kn"] <= rng_kind[c["kind"]][3] for c in test])
    wf, cf = C.fields_from_prediction(test, y, recentre_shocks=args.sweep_recentre), C.cold_fields(test)
    site_in = np.repeat(inside, [2 * c["L"] for c in test])
    for key in ("rho", "thT", "thR"):
        wf[key] = np.where(site_in, wf[key], cf[key])
    wf["u"] = np.where(site_in[None, :], wf["u"], cf["u"])
    warm = run_batch(test, wf, "held-out warm")
    mlp.close()
    # the plain start is the fallback: a warm-started case whose run diverged
    # (a predicted state out of the lattice's reach) runs again from the cold
    # start; its steps and the rerun's time count for the warm pipeline
    warm_first_status = warm["status"].copy()
    redo = [i for i in range(len(test)) if inside[i] and warm["status"][i] == 2]
    t_redo = 0.0
    if redo:
        sub = [test[i] for i in redo]
        rr = run_batch(sub, C.cold_fields(sub), "held-out warm fallback (cold start)")
        t_redo = rr["time"]
        o_t = np.concatenate([[0], np.cumsum([2 * c["L"] for c in test])])
        o_s = np.concatenate([[0], np.cumsum([2 * c["L"] for c in sub])])
        for j, i in enumerate(redo):
            warm["status"][i], warm["resid"][i] = rr["status"][j], rr["resid"][j]
            warm["steps"][i] += rr["steps"][j]
            for key in ("rho", "thT", "thR"):
                warm["m"][key][o_t[i]:o_t[i + 1]] = rr["m"][key][o_s[j]:o_s[j + 1]]
            warm["m"]["u"][:, o_t[i]:o_t[i + 1]] = rr["m"]["u"][:, o_s[j]:o_s[j + 1]]
        warm["time"] += t_redo

    # final match of warm and cold converged states.  Couette: max |du|/U
    # against the bound (R_cold + R_warm) / r_slow of two runs stopped at
    # residuals R (r_slow = pi^2 nu / L_eff^2, the slowest shear mode of a
    # layer whose walls slip by a mean free path lambda each, L_eff = L + 2
    # lambda).  Shock: a shock between Dirichlet faces may
    # settle anywhere, so the shift of its position is reported and the
    # density profiles are compared with the positions aligned (max |drho| over
    # the jump rho2 - rho1).
    both = (cold["status"] == 1) & (warm["status"] == 1)
    worst_c, worst_s, shift, o = 0.0, 0.0, 0.0, 0
    from paper_2201_05280_amd.inputs import positions
    for k_c, (c, ok_c) in enumerate(zip(test, both)):
        n = 2 * c["L"]
        if ok_c:
            sl = slice(o, o + n)
            if c["kind"] == C.SHOCK:
                # compare the profiles with the two shock positions aligned
                dr = c["down"][0] - c["up"][0]
                x = positions(c["L"], 1, 1)[0]
                order = np.argsort(x)
                xs, rw, rc_ = x[order], warm["m"]["rho"][sl][order], cold["m"]["rho"][sl][order]
                pw = profile_metrics(x, warm["m"]["rho"][sl], c["up"], c["down"])[0]
                pc = profile_metrics(x, cold["m"]["rho"][sl], c["up"], c["down"])[0]
                d = pw - pc
                keep = (xs + d >= xs[0]) & (xs + d <= xs[-1])
                aligned = np.interp(xs[keep] + d, xs, rw)
                worst_s = max(worst_s, float(np.abs(aligned - rc_[keep]).max() / dr))
                shift = max(shift, abs(d))
            else:
                du = np.abs(warm["m"]["u"][1][sl] - cold["m"]["u"][1][sl]).max() / c["U"]
                lam = c["nu"] * math.sqrt(math.pi / (2 * THETA0))
                r_slow = math.pi ** 2 * c["nu"] / (c["L"] + 2 * lam) ** 2
                worst_c = max(worst_c, du / ((cold["resid"][k_c] + warm["resid"][k_c]) / r_slow))
        o += n
    # plain: a seeded subset of the held-out cases, one at a time through the
    # single-grid path; a case stopped by the time cap is charged its measured
    # time per step times the steps the batched run took (same arithmetic,
    # so the same step count: checked on the cases that finish)
    idx = np.random.default_rng(S).choice(len(test), size=min(args.sweep_plain, len(test)), replace=False)
    tp, n_full, step_match = 0.0, 0, True
    for i in idx:
        st, rs, dt = plain_case(test[i], tol, min(args.sweep_max_steps, int(cold["steps"][i])), args.sweep_plain_cap)
        if rs <= tol or st >= int(cold["steps"][i]):
            n_full += 1
            tp += dt
            step_match &= abs(st - int(cold["steps"][i])) <= 128
        else:
            tp += dt / st * int(cold["steps"][i])
        print("# plain case %d (%s): L=%d steps %d (batched %d) %.2f s"
              % (i, test[i]["kind"], test[i]["L"], st, cold["steps"][i], dt), file=sys.stderr, flush=True)
    plain_est = tp * len(test) / len(idx)   # unbiased for a uniform random subset

    def counts(r, mask):
        return {k: int(((r["status"] == v) & mask).sum()) for k, v in
                (("converged", 1), ("diverged", 2), ("capped", 3), ("stalled", 4))}

    conv_both = (cold["status"] == 1) & (warm["status"] == 1)
    mach = np.array([c["Ma"] for c in test])
    bands = (("Ma<1.6", 0.0, 1.6), ("1.6<=Ma<2.65", 1.6, 2.65), ("Ma>=2.65", 2.65, 99.0))

    def by_mach(r):
        return {nm: counts(r, is_shock & (mach >= lo) & (mach < hi)) for nm, lo, hi in bands}

    def med(a, mask):
        return int(np.median(a[mask])) if mask.any() else None

    out.update({
        "plain_subset_cases": len(idx), "plain_subset_time": round(tp, 2), "plain_subset_run_to_end": n_full,
        "plain_steps_match_batched": bool(step_match),
        "plain_estimated_time": round(plain_est, 1),
        "batched_cold_time": round(cold["time"], 2), "batched_warm_time": round(warm["time"] + t_infer, 2),
        "batched_warm_plus_training_time": round(warm["time"] + t_infer + t_train, 2),
        "warm_pipeline_time_with_data_generation": round(t_gen + t_train + t_infer + warm["time"], 2),
        "training_data_generation_time": round(t_gen, 2),
        "training_cases_by_status": {"couette": counts(tr, ~tr_shock), "shock": counts(tr, tr_shock)},
        "mlp_inference_time": round(t_infer, 3), "mlp_train_time": round(t_train, 1),
        "mlp_train_points": int(len(X)), "mlp_train_points_from_this_training_set": own_points,
        "held_out_warm_started": {"couette": int((inside & ~is_shock).sum()), "shock": int((inside & is_shock).sum()),
                                  "rule": "Mach and Kn within the range of the converged training cases of the "
                                          "same kind; every other case starts cold",
                                  "shock_profiles_recentred_at_L/2": bool(args.sweep_recentre)},
        "warm_fallback_to_cold_start": {
            "cases": len(redo), "rerun_time": round(t_redo, 2),
            "rule": "a warm-started case whose run diverged runs again from the cold start (included in the "
                    "warm time, steps and outcomes)",
            "warm_first_attempt": {"couette": counts({"status": warm_first_status}, ~is_shock),
                                   "shock": counts({"status": warm_first_status}, is_shock)}},
        "mlp_loss_first_last": [float(losses[0]), float(losses[-1])], "mlp_schedule": args.sweep_lr_schedule,
        "mlp_minibatch": args.sweep_mlp_batch,
        "mlp_loss_curve_every_5_epochs": [float("%.4g" % v) for v in losses[::5]],
        "couette": {"cold": counts(cold, ~is_shock), "warm": counts(warm, ~is_shock),
                    "residual_at_stop_median": {"cold": float("%.3g" % np.median(cold["resid"][~is_shock]))
                                                if (~is_shock).any() else None,
                                                "warm": float("%.3g" % np.median(warm["resid"][~is_shock]))
                                                if (~is_shock).any() else None},
                    "steps_cold_median": med(cold["steps"], ~is_shock),
                    "steps_warm_median": med(warm["steps"], ~is_shock),
                    "steps_cold_median_converged_both": med(cold["steps"], ~is_shock & conv_both),
                    "steps_warm_median_converged_both": med(warm["steps"], ~is_shock & conv_both),
                    "warm_vs_cold_max_du_over_bound": round(worst_c, 3)},
        "shock": {"cold": counts(cold, is_shock), "warm": counts(warm, is_shock),
                  "residual_at_stop_median": {"cold": float("%.3g" % np.median(cold["resid"][is_shock]))
                                              if is_shock.any() else None,
                                              "warm": float("%.3g" % np.median(warm["resid"][is_shock]))
                                              if is_shock.any() else None},
                  "steps_cold_median": med(cold["steps"], is_shock),
                  "steps_warm_median": med(warm["steps"], is_shock),
                  "steps_cold_median_converged_both": med(cold["steps"], is_shock & conv_both),
                  "steps_warm_median_converged_both": med(warm["steps"], is_shock & conv_both),
                  "cold_by_mach": by_mach(cold), "warm_by_mach": by_mach(warm),
                  "warm_vs_cold_max_drho_over_jump_aligned": round(worst_s, 6),
                  "warm_vs_cold_max_shift_cells": round(shift, 4)},
        "steps_cold_total": int(cold["steps"].sum()), "steps_warm_total": int(warm["steps"].sum()),
        "batch_configs": cold["cfg"],
        "speedup_warm_vs_cold": round(cold["time"] / (warm["time"] + t_infer), 3),
        "speedup_batched_cold_vs_plain": round(plain_est / cold["time"], 2),
        "speedup_batched_warm_vs_plain": round(plain_est / (warm["time"] + t_infer), 2),
    })
    return out, (X, Y, conv)


def sweeps(args):
    """The reduced mix first (every case converges; its steady states also
    train the network of the second run), then the stated 512/4096-case mix
    under its caps.  A failure is reported in place of the object."""
    out, extra = {}, None
    if not args.no_sweep_reduced:
        try:
            out["sweep_reduced"], extra = sweep(reduced_args(args))
        except Exception as e:  # noqa: BLE001
            print("# sweep_reduced failed: %r" % (e,), file=sys.stderr, flush=True)
            out["sweep_reduced"] = {"error": repr(e)}
    try:
        out["sweep"], _ = sweep(args, extra)
    except Exception as e:  # noqa: BLE001
        print("# sweep failed: %r" % (e,), file=sys.stderr, flush=True)
        out["sweep"] = {"error": repr(e)}
    return out


def reduced_args(args):
    """The reduced mix whose every case can reach the residual: 256 held-out
    and 512 training cases, L ~ U{128..512}, Couette Kn ~ logU[1e-2, 1e-1],
    shocks to Mach 1.6, no caps that bind."""
    import copy
    r = copy.copy(args)
    r.sweep_n, r.sweep_train, r.sweep_lmin, r.sweep_lmax = 256, 512, 128, 512
    r.sweep_knmin, r.sweep_knmax, r.sweep_mamin, r.sweep_mamax = 1e-2, 1e-1, 1.1, 1.6
    r.sweep_max_steps = r.sweep_train_max_steps = 400000
    r.sweep_time_budget = r.sweep_train_time_budget = 0.0
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--precision", choices=["fp32dev", "fp64"], default="fp32dev")
    ap.add_argument("--equilibrium", choices=["f3", "f4", "e2"], default="f3",
                    help="equilibrium of the Taylor-Green run (the benchmark configuration is F3)")
    ap.add_argument("--cpu-n", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sweep", action="store_true", help="run only the batched sweep / warm-start experiment")
    ap.add_argument("--no-sweep", action="store_true", help="skip the sweep experiment")
    ap.add_argument("--no-shock", action="store_true", help="skip the normal-shock lines")
    ap.add_argument("--shock", action="store_true", help="run only the normal-shock lines")
    ap.add_argument("--mlp-train", action="store_true", help="run only the warm-start network's training rate")
    ap.add_argument("--sweep-n", type=int, default=512, help="held-out cases (seed 220105280)")
    ap.add_argument("--sweep-train", type=int, default=4096, help="training cases (seed 220105281)")
    ap.add_argument("--sweep-lmin", type=int, default=256)
    ap.add_argument("--sweep-lmax", type=int, default=4096)
    ap.add_argument("--sweep-knmin", type=float, default=1e-3)
    ap.add_argument("--sweep-knmax", type=float, default=1e-1)
    ap.add_argument("--sweep-mamin", type=float, default=1.1, help="shock Mach range")
    ap.add_argument("--sweep-mamax", type=float, default=4.0)
    ap.add_argument("--sweep-max-steps", type=int, default=16384,
                    help="step cap per held-out case (a case still running there counts as capped)")
    ap.add_argument("--sweep-train-max-steps", type=int, default=8192,
                    help="step cap per training case (only converged training states train the network)")
    ap.add_argument("--sweep-time-budget", type=float, default=60.0,
                    help="wall seconds per batched held-out run after which the cases still running count as "
                         "capped (0 = none)")
    ap.add_argument("--sweep-train-time-budget", type=float, default=30.0,
                    help="the same for the run that generates the training states")
    ap.add_argument("--no-sweep-reduced", action="store_true",
                    help="skip the second sweep on the reduced mix that converges in full")
    ap.add_argument("--sweep-mlp-batch", type=int, default=2048, help="MLP training minibatch")
    ap.add_argument("--sweep-lr-schedule", default="2e-3:40,5e-4:30,1.25e-4:30",
                    help="MLP training stages lr:epochs[,lr:epochs...] (Adam state carried across stages)")
    ap.add_argument("--sweep-recentre", type=int, default=1,
                    help="1: move each predicted shock to the cold start's position (L/2); 0: as predicted")
    ap.add_argument("--sweep-plain", type=int, default=8)
    ap.add_argument("--sweep-plain-cap", type=float, default=10.0)
    ap.add_argument("--sweep-shock-frac", type=float, default=0.5)
    ap.add_argument("--sweep-stall", type=int, default=25600,
                    help="Couette: steps without halving the residual before a case counts as stalled")
    ap.add_argument("--sweep-stall-shock", type=int, default=6400,
                    help="shock lines: the same window (a converging shock halves its residual every ~100 steps)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also time a plain device copy (torch) as the achievable-bandwidth reference")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the z-slab decomposition is a design note); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        print(json.dumps(sweeps(args)), flush=True)
        return
    if args.shock:
        print(json.dumps(shock_summary()), flush=True)
        return
    if args.mlp_train:
        print(json.dumps({"mlp_train": mlp_train_summary()}), flush=True)
        return

    import torch

    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd import inputs

    precision = pgk.FP32DEV if args.precision == "fp32dev" else pgk.FP64
    n = args.n
    U, nu = tgv_params(n)
    p = pgk.resolve(nu, 0.71, 0.6, 2.0)
    print("# resolved", {k: round(v, 6) for k, v in p.items()}, file=sys.stderr, flush=True)
    eq = {"f3": pgk.F3, "f4": pgk.F4, "e2": pgk.E2}[args.equilibrium]
    s = pgk.Solver(n, n, n, precision=precision, equilibrium=eq)
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    f = inputs.taylor_green(n, U)
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    del f
    ns = s.ns
    print("# init done, %d sites" % ns, file=sys.stderr, flush=True)

    s.step(args.warmup)
    torch.cuda.synchronize()
    c0 = s.conserved()
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = s.kernel_times()
    s.set_timing(False)
    c1 = s.conserved()
    print("# timed %d steps in %.3f s; kernels %s" % (args.steps, dt, kt), file=sys.stderr, flush=True)

    ms_step = 1e3 * dt / args.steps
    mlups = ns * args.steps / dt / 1e6
    ab = algorithmic_bytes(precision)
    lb_ms, lb_n = kt["k_lb"]
    lb_avg_s = lb_ms / lb_n / 1e3
    achieved = ab["k_lb"] * ns / lb_avg_s / 1e9
    step_gbs = ab["step"] * ns / (dt / args.steps) / 1e9
    drift = [(c1[i] - c0[i]) / c0[0] for i in range(4)] + [(c1[4] - c0[4]) / c0[4]]

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if precision == pgk.FP32DEV else "f64",
        "data": "synthetic",
        "config": {
            "workload": "3D Taylor-Green vortex, %d^3 bcc cells (%d sites), Ma 0.1, Re 1600, "
                        "delta 2, Pr 0.71, mu_b/mu 0.6, %s populations, CN, %s"
                        % (n, ns, args.precision, args.equilibrium.upper()),
            "cells": n ** 3, "sites": ns, "tau": p["tau"], "tau1": p["tau1"], "b": p["b"], "k_r": p["kr"],
        },
        "roofline": {
            "bound": "hbm", "kernel": "k_lb (fused pull-moments-solve-%s-collide)" % args.equilibrium.upper(),
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(n, precision) if args.equilibrium == "f3" else None,
            "bytes_per_site": ab["k_lb"], "avg_launch_ms": round(lb_avg_s * 1e3, 4),
        },
        "step_roofline": {"algorithmic_bytes_per_site": ab["step"], "achieved_GBs": round(step_gbs, 1),
                          "frac": round(step_gbs / HBM_PEAK_GBS, 4)},
        # slot k_mc holds the fused transport kernel k_tr when no separate diffusion ran
        "kernels_ms_avg": {("k_tr" if k == "k_mc" and kt["k_dif"][1] == 0 else k): round(v[0] / max(v[1], 1), 4)
                           for k, v in kt.items() if v[1] > 0},
        "conservation_drift": drift,
    }
    s.close()
    # the bandwidth a plain copy reaches on this device, beside the kernel's
    cp = copy_probe(torch, reps=5, quick=not args.copy_probe)
    best = max(v for k, v in cp.items() if k.endswith("_GBs") and k != "soa41_streams_GBs")
    rf = out["roofline"]
    rf["copy_reference_GBs"] = best
    rf["copy_soa41_streams_GBs"] = cp["soa41_streams_GBs"]
    if rf["traffic"]:
        actual = rf["traffic"] / (rf["avg_launch_ms"] * 1e-3) / 1e9
        rf["actual_GBs_from_traffic"] = round(actual, 1)
        rf["actual_over_copy_reference"] = round(actual / best, 4)
        rf["actual_over_soa41_copy"] = round(actual / cp["soa41_streams_GBs"], 4)
    if args.copy_probe:
        out["copy_probe"] = cp
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.cpu_steps)
    # the side experiments report into the line; a failure in one of them is
    # recorded there and never costs the headline measurement
    for key, skip, fn in (("shear_wave", False, shear_wave_summary), ("shock", args.no_shock, shock_summary),
                          ("mlp_train", args.no_sweep, mlp_train_summary),
                          ("mlp_train_larger_minibatches", args.no_sweep, mlp_minibatch_summary)):
        if skip:
            continue
        try:
            out[key] = fn()
        except Exception as e:  # noqa: BLE001
            print("# %s failed: %r" % (key, e), file=sys.stderr, flush=True)
            out[key] = {"error": repr(e)}
    if not args.no_sweep:
        out.update(sweeps(args))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
