"""Batched sweep (persistent kernel + graph replay + autotuner) on the GPU.

Each batched case must equal the same case run alone through the single-grid
path (the same device code in double precision: identical up to the few-ulp
differences of the compiler's FMA contraction in the two kernels) and the FP64
oracle (1e-12).  The case mix covers the three diffusion paths of the kernel
(registers for lines up to 512 cells, LDS up to 2048 sites, global memory
beyond) and sub-cycled diffusion;
convergence, divergence and the tuner are exercised on small
cases.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.params import resolve
from paper_2201_05280_amd import inputs

pytestmark = pytest.mark.gpu

TH0 = oracle.THETA0


def _cases():
    import paper_2201_05280_amd as pgk
    out = []
    specs = [
        # (L, bc, targets, faces)
        (24, pgk.WALL, (0.05, 0.71, 0.8, 2.0), dict(u=((0, 0, 0), (0, 0.05, 0)), theta=(TH0, TH0 * 1.02))),
        (37, pgk.WALL, (0.2, 0.9, 1.2, 3.0), dict(u=((0, -0.02, 0), (0, 0.03, 0.01)), theta=(TH0, TH0))),
        (4, pgk.WALL, (0.02, 0.7, 0.6, 2.0), dict(u=((0, 0, 0), (0, 0.02, 0)), theta=(TH0, TH0))),
        (64, pgk.DIRICHLET, (0.05, 0.71, 0.8, 2.0),
         dict(rho=(1.02, 0.99), u=((0.03, 0, 0), (0.03, 0, 0)), theta=(TH0 * 1.01, TH0))),
        (19, pgk.DIRICHLET, (0.1, 1.0, 1.0, 3.0),
         dict(rho=(1.0, 1.05), u=((0.02, 0, 0), (0.019, 0, 0)), theta=(TH0, TH0 * 1.03))),
        # several diffusion sub-steps per step, in LDS
        (40, pgk.WALL, (0.6, 0.71, 0.8, 2.0), dict(u=((0, 0, 0), (0, 0.04, 0)), theta=(TH0, TH0 * 1.05))),
        # 700 cells: beyond the two-wavefront chain (512 cells): the chain over
        # every wavefront with 256 threads, the LDS path with 512
        (700, pgk.WALL, (0.4, 0.8, 1.0, 3.0), dict(u=((0, 0.0, 0), (0, 0.02, 0)), theta=(TH0, TH0 * 1.02))),
        # 2060 sites: beyond the LDS path (2048 sites): the chain with its
        # conductances in LDS with 256 threads, the register chain with 512
        (1030, pgk.WALL, (0.3, 0.8, 1.0, 2.0), dict(u=((0, 0.01, 0), (0, 0.03, 0)), theta=(TH0 * 1.01, TH0))),
        # 8192 sites: the chain with its conductances in LDS at its limit
        # (128 KiB) with 256 threads, global memory with 512
        (4096, pgk.WALL, (0.5, 0.75, 1.2, 2.0), dict(u=((0, 0.01, 0), (0, 0.0, 0)), theta=(TH0 * 1.02, TH0))),
        # 8400 sites: beyond every chain (8192 sites of conductances in LDS):
        # diffused in global memory
        (4200, pgk.WALL, (0.3, 0.8, 1.0, 2.0), dict(u=((0, 0.0, 0), (0, 0.02, 0)), theta=(TH0, TH0 * 1.01))),
    ]
    for L, bc, tg, faces in specs:
        p = resolve(*tg)
        out.append(dict(L=L, bc=bc, p=p, faces=faces, vel_axis=1 if bc == pgk.WALL else 0))
    return out


def _fields(L, seed, bc):
    f = inputs.random_smooth(L, 1, 1, seed=seed, amp_rho=0.01, amp_u=0.01, amp_th=0.01)
    return f


def _build(specs, variant=0):
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd.batch import Batch, make_case
    cases = []
    for sp in specs:
        p = sp["p"]
        fc = sp["faces"]
        cases.append(make_case(sp["L"], sp["bc"], (p["tau"], p["tau1"], p["b"], p["kr"], p["delta"]),
                               rho=fc.get("rho", (1.0, 1.0)), u=fc["u"], theta=fc["theta"],
                               vel_axis=sp["vel_axis"], variant=variant))
    b = Batch(cases)
    fields = [_fields(sp["L"], 10 + i, sp["bc"]) for i, sp in enumerate(specs)]
    cat = {k: np.concatenate([f[k] for f in fields], axis=-1) for k in ("rho", "thT", "thR")}
    cat["u"] = np.concatenate([f["u"] for f in fields], axis=1)
    b.init(cat["rho"], cat["u"], cat["thT"], cat["thR"])
    return b, fields


def _single(sp, f, steps, variant=0):
    import paper_2201_05280_amd as pgk
    s = pgk.Solver(sp["L"], 1, 1, precision=pgk.FP64, variant=variant, bc_x=(sp["bc"], sp["bc"]))
    p = sp["p"]
    s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
    fc = sp["faces"]
    for side in (0, 1):
        s.set_bc_x(side, fc.get("rho", (1.0, 1.0))[side], fc["u"][side], fc["theta"][side])
    s.init(f["rho"], f["u"], f["thT"], f["thR"])
    s.step(steps)
    m = s.moments()
    s.close()
    return m


@pytest.mark.parametrize("variant", [0, 1])
def test_batched_cases_equal_single_grid_runs(variant):
    specs = _cases()
    b, fields = _build(specs, variant)
    b.config(256, 20)
    steps, resid, status = b.run(60, 0.0)
    assert (steps == 60).all(), steps
    assert (status == 3).all(), status                 # stopped at max_steps
    bm = b.moments()
    for c, sp in enumerate(specs):
        sl = b.case_slice(c)
        sm = _single(sp, fields[c], 60, variant)
        for k in ("rho", "thT", "thR"):
            err = np.abs(bm[k][sl] - sm[k]).max() / np.abs(sm[k]).max()
            assert err <= 1e-13, (c, k, err)
        err = np.abs(bm["u"][:, sl] - sm["u"]).max() / max(np.abs(sm["u"]).max(), 1e-2)
        assert err <= 1e-13, (c, "u", err)
    b.close()


def test_batched_state_is_the_same_bits_under_every_launch_shape():
    # work-groups of 256 and 512 threads, chunks of 20 and 12 steps (a run
    # advances by whole chunks), and a
    # second identical run: the per-site arithmetic does not depend on the
    # launch shape (only the residual's reduction does, and it never feeds
    # back), so after 60 steps every case's state is the same bits; the cases
    # cover the register, LDS and global-memory diffusion paths
    specs = _cases()
    ref = None
    for wg, K in ((256, 20), (512, 20), (256, 12), (256, 20)):
        b, _ = _build(specs)
        b.config(wg, K)
        steps, _, _ = b.run(60, 0.0)
        assert (steps == 60).all(), (wg, K, steps)
        m = b.moments()
        b.close()
        if ref is None:
            ref = m
            continue
        for k in ("rho", "u", "thT", "thR"):
            assert np.array_equal(m[k], ref[k]), (wg, K, k, float(np.abs(m[k] - ref[k]).max()))


def test_batched_cases_match_oracle():
    specs = _cases()
    b, fields = _build(specs)
    b.config(512, 25)
    b.run(50, 0.0)
    bm = b.moments()
    for c, sp in enumerate(specs):
        sl = b.case_slice(c)
        o = oracle.Oracle(sp["L"], 1, 1)
        p = sp["p"]
        o.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        fc = sp["faces"]
        for side in (0, 1):
            o.set_bc_x(side, sp["bc"], fc.get("rho", (1.0, 1.0))[side], fc["u"][side], fc["theta"][side])
        f = fields[c]
        o.init(f["rho"], f["u"], f["thT"], f["thR"])
        o.step(50)
        om = o.moments()
        for k in ("rho", "thT", "thR"):
            err = np.abs(bm[k][sl] - om[k]).max() / np.abs(om[k]).max()
            assert err < 1e-12, (c, k, err)
        err = np.abs(bm["u"][:, sl] - om["u"]).max() / max(np.abs(om["u"]).max(), 1e-2)
        assert err < 1e-12, (c, "u", err)
    b.close()


def test_couette_case_converges_to_linear_profile():
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd.batch import Batch, make_case
    L, U = 16, 0.03
    p = resolve(0.5, 0.71, 0.8, 2.0)                 # large viscosity: fast diffusion
    c = make_case(L, pgk.WALL, (p["tau"], p["tau1"], p["b"], p["kr"], p["delta"]),
                  u=((0, 0, 0), (0, U, 0)), theta=(TH0, TH0), vel_axis=1)
    b = Batch([c])
    f = inputs.uniform(L, 1, 1)
    b.init(f["rho"], f["u"], f["thT"], f["thR"])
    b.config(256, 50)
    steps, resid, status = b.run(200000, 1e-10)
    assert status[0] == 1, (status, resid, steps)
    assert resid[0] <= 1e-10
    m = b.moments()
    x = inputs.positions(L, 1, 1)[0]
    uy = m["u"][1]
    order = np.argsort(x)
    assert np.all(np.diff(uy[order]) > 0)            # monotonic shear profile
    # walls at x = -1/4 and L - 1/4: the profile is linear between slip values
    fit = np.polyfit(x, uy, 1)
    assert np.abs(np.polyval(fit, x) - uy).max() < 0.02 * U
    mid = np.polyval(fit, (L - 0.5) / 2)
    assert abs(mid - U / 2) < 0.02 * U
    b.close()


def test_divergence_is_flagged_per_case():
    specs = _cases()[:3]
    b, fields = _build(specs)
    # plant a non-finite density in case 1 from the host (a single negative
    # density is smoothed away by the streaming; a NaN cannot be)
    sl = b.case_slice(1)
    rho = np.concatenate([f["rho"] for f in fields])
    rho[sl.start + 3] = np.nan
    u = np.concatenate([f["u"] for f in fields], axis=1)
    thT = np.concatenate([f["thT"] for f in fields])
    thR = np.concatenate([f["thR"] for f in fields])
    b.init(rho, u, thT, thR)
    b.config(256, 10)
    steps, resid, status = b.run(40, 0.0)
    assert status[1] == 2, status
    assert status[0] == 3 and status[2] == 3, status
    assert steps[1] == 10 and steps[0] == 40
    b.close()


def test_autotuner_picks_and_caches(tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PGK_TUNE_CACHE", str(cache))
    specs = _cases()
    b, _ = _build(specs)
    b.config(0, 0)
    steps, resid, status = b.run(300, 0.0)
    wg, K, ns = b.tuned()
    assert wg in (256, 512) and K >= 2 and ns > 0
    d = json.loads(cache.read_text())
    assert len(d) == 1 and list(d.values())[0] == [wg, K]
    assert (steps >= 300).all()
    b.close()
    # a second batch of the same shape reuses the cached choice
    b2, _ = _build(specs)
    b2.config(0, 0)
    b2.run(40, 0.0)
    assert b2.tuned()[:2] == (wg, K)
    b2.close()


def _shock_spec(Ma, L, delta, nu_cs=2.0):
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd.shock import discrete_rankine_hugoniot
    up, down = discrete_rankine_hugoniot(Ma, delta)
    cs = np.sqrt((5 + delta) / (3 + delta) * TH0)
    p = resolve(nu_cs * cs, 0.71, 0.8, delta)
    return dict(L=L, bc=pgk.DIRICHLET, p=p, eq=pgk.E2, vel_axis=0,
                faces=dict(rho=(up[0], down[0]), u=((up[1], 0, 0), (down[1], 0, 0)), theta=(up[2], down[2])),
                up=up, down=down)


def test_batched_e2_shocks_beside_f3_couette():
    # one launch holding E2 shock lines and an F3 Couette layer: every case
    # equals its single-grid run and the oracle
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd.batch import Batch, make_case
    from paper_2201_05280_amd.shock import tanh_profile
    specs = [_shock_spec(1.5, 64, 2.0), _shock_spec(1.2, 40, 3.0, nu_cs=1.0), dict(_cases()[0], eq=pgk.F3)]
    cases, fields = [], []
    for i, sp in enumerate(specs):
        p, fc = sp["p"], sp["faces"]
        cases.append(make_case(sp["L"], sp["bc"], (p["tau"], p["tau1"], p["b"], p["kr"], p["delta"]),
                               rho=fc.get("rho", (1.0, 1.0)), u=fc["u"], theta=fc["theta"], vel_axis=sp["vel_axis"],
                               equilibrium=sp["eq"]))
        fields.append(tanh_profile(sp["L"], sp["up"], sp["down"], width=3.0) if "up" in sp
                      else _fields(sp["L"], 10 + i, sp["bc"]))
    b = Batch(cases)
    cat = {k: np.concatenate([f[k] for f in fields], axis=-1) for k in ("rho", "thT", "thR")}
    cat["u"] = np.concatenate([f["u"] for f in fields], axis=1)
    b.init(cat["rho"], cat["u"], cat["thT"], cat["thR"])
    with pytest.raises(RuntimeError):
        b.config(512, 25)                 # E2 batches run with work-groups of 256
    b.config(256, 25)
    steps, resid, status = b.run(50, 0.0)
    assert (steps == 50).all() and (status == 3).all(), (steps, status)
    bm = b.moments()
    for c, sp in enumerate(specs):
        sl = b.case_slice(c)
        fc, p, f = sp["faces"], sp["p"], fields[c]
        s = pgk.Solver(sp["L"], 1, 1, precision=pgk.FP64, bc_x=(sp["bc"], sp["bc"]), equilibrium=sp["eq"])
        s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        o = oracle.Oracle(sp["L"], 1, 1, equilibrium=oracle.E2 if sp["eq"] == pgk.E2 else oracle.F3)
        o.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        for side in (0, 1):
            s.set_bc_x(side, fc.get("rho", (1.0, 1.0))[side], fc["u"][side], fc["theta"][side])
            o.set_bc_x(side, sp["bc"], fc.get("rho", (1.0, 1.0))[side], fc["u"][side], fc["theta"][side])
        s.init(f["rho"], f["u"], f["thT"], f["thR"])
        o.init(f["rho"], f["u"], f["thT"], f["thR"])
        s.step(50)
        o.step(50)
        sm, om = s.moments(), o.moments()
        s.close()
        for ref, bar in ((sm, 1e-13), (om, 1e-12)):
            for k in ("rho", "thT", "thR"):
                err = np.abs(bm[k][sl] - ref[k]).max() / np.abs(ref[k]).max()
                assert err <= bar, (c, k, err, bar)
            err = np.abs(bm["u"][:, sl] - ref["u"]).max() / max(np.abs(ref["u"]).max(), 1e-2)
            assert err <= bar, (c, "u", err, bar)
    b.close()


def test_batch_refuses_a_face_state_without_e2_equilibrium():
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd.batch import Batch, make_case
    p = resolve(0.05, 0.71, 0.8, 2.0)
    c = make_case(16, pgk.DIRICHLET, (p["tau"], p["tau1"], p["b"], p["kr"], p["delta"]), rho=(1.0, 1.0),
                  u=((0.4, 0, 0), (0.4, 0, 0)), theta=(0.05, 0.05), vel_axis=0, equilibrium=pgk.E2)
    with pytest.raises(RuntimeError, match="EINFEASIBLE"):
        Batch([c])


def test_stall_detection_stops_a_slow_case():
    # a window shorter than the slow mode's halving time (~0.07 L^2/nu steps)
    # stops the case as STALLED; with detection off the same case converges
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd.batch import Batch, make_case
    L, U = 48, 0.03
    p = resolve(0.05, 0.71, 0.8, 2.0)
    out = []
    for window in (512, 0):
        c = make_case(L, pgk.WALL, (p["tau"], p["tau1"], p["b"], p["kr"], p["delta"]),
                      u=((0, 0, 0), (0, U, 0)), theta=(TH0, TH0), vel_axis=1)
        b = Batch([c])
        f = inputs.uniform(L, 1, 1)
        b.init(f["rho"], f["u"], f["thT"], f["thR"])
        b.config(256, 64)
        b.stall(window)
        out.append(b.run(400000, 1e-10))
        b.close()
    (s1, r1, st1), (s0, r0, st0) = out
    assert st1[0] == 4 and r1[0] > 1e-10 and s1[0] < s0[0], (st1, r1, s1, s0)
    assert st0[0] == 1 and r0[0] <= 1e-10, (st0, r0)


def test_largest_case_equals_single_grid():
    # L = 8192 cells (the largest line a batch takes) next to the smallest (4)
    import paper_2201_05280_amd as pgk
    specs = [dict(L=8192, bc=pgk.WALL, p=resolve(0.4, 0.8, 1.0, 2.0), vel_axis=1,
                  faces=dict(u=((0, 0.0, 0), (0, 0.02, 0)), theta=(TH0, TH0 * 1.01))),
             dict(_cases()[2])]
    b, fields = _build(specs)
    b.config(512, 10)
    steps, resid, status = b.run(30, 0.0)
    assert (steps == 30).all()
    bm = b.moments()
    for c, sp in enumerate(specs):
        sl = b.case_slice(c)
        sm = _single(sp, fields[c], 30)
        for k in ("rho", "thT", "thR"):
            err = np.abs(bm[k][sl] - sm[k]).max() / np.abs(sm[k]).max()
            assert err <= 1e-13, (c, k, err)
    b.close()


def _host_residual(a, b, sl, axis):
    """max over rho, u_axis, theta_T, theta_R of ||phi^n - phi^(n-1)||_2 / ||phi^n||_2"""
    r = 0.0
    for k in ("rho", "u", "thT", "thR"):
        x0 = a[k][axis][sl] if k == "u" else a[k][sl]
        x1 = b[k][axis][sl] if k == "u" else b[k][sl]
        d = float(np.linalg.norm(x1 - x0) / np.linalg.norm(x1))
        r = max(r, d) if d == d else d   # a NaN stays NaN
    return r


def test_in_kernel_residual_equals_host_two_read_residual():
    """The residual each case reports (computed inside the persistent kernel
    from its last two steps) equals the same definition evaluated on the host
    from moment reads of the state at steps n-1 and n.  The two states come
    from two batches run from the same start with chunks of 3 and of 2 steps
    (the state does not depend on the chunking), so the host sees exactly the
    values the kernel summed; only the order of the sums differs."""
    specs = _cases()
    b1, _ = _build(specs)
    b1.config(256, 3)
    steps1, _, _ = b1.run(57, 0.0)
    assert (steps1 == 57).all()
    m1 = b1.moments()
    b1.close()
    b2, _ = _build(specs)
    b2.config(256, 2)
    steps2, resid, status = b2.run(58, 0.0)
    assert (steps2 == 58).all() and (status == 3).all()
    m2 = b2.moments()
    for c, sp in enumerate(specs):
        h = _host_residual(m1, m2, b2.case_slice(c), sp["vel_axis"])
        print("case", c, "kernel residual %.15e host %.15e" % (resid[c], h))
        assert h > 1e-12
        assert abs(resid[c] - h) <= 1e-12 * h, (c, resid[c], h)
    b2.close()


def test_single_grid_runs_stop_at_the_batched_step():
    """The plain path (one case at a time through the single-grid solver, the
    residual taken from two moment reads at the end of every chunk of K steps)
    stops each case at the step where the batched kernel stopped it with the
    same K: the two evaluate one residual definition on the same states."""
    import paper_2201_05280_amd as pgk
    from paper_2201_05280_amd import _lib
    from paper_2201_05280_amd import cases as C
    from paper_2201_05280_amd.batch import Batch
    cs, _ = C.sweep_cases(4, 11, L_range=(24, 64), Kn_range=(0.05, 0.1), shock_fraction=0.0)
    K, tol = 32, 1e-6
    f = C.cold_fields(cs)
    b = Batch(C.to_batch_cases(cs))
    b.init(f["rho"], f["u"], f["thT"], f["thR"])
    b.config(256, K)
    steps, resid, status = b.run(200000, tol)
    b.close()
    assert (status == _lib.CASE_CONVERGED).all(), status
    for c, case in enumerate(cs):
        p = case["params"]
        s = pgk.Solver(case["L"], 1, 1, precision=pgk.FP64, bc_x=(pgk.WALL, pgk.WALL))
        s.set_params(p["tau"], p["tau1"], p["b"], p["kr"], p["delta"])
        s.set_bc_x(0, 1.0, (0, 0, 0), TH0)
        s.set_bc_x(1, 1.0, (0, case["U"], 0), TH0)
        g = C.cold_fields([case])
        s.init(g["rho"], g["u"], g["thT"], g["thR"])
        n, r = 0, 1.0
        while r > tol and n < 200000:
            s.step(K - 1)
            a = s.moments()
            s.step(1)
            bm = s.moments()
            n += K
            r = 0.0
            for k, v in (("rho", None), ("u", 1), ("thT", None), ("thR", None)):
                x0 = a[k] if v is None else a[k][v]
                x1 = bm[k] if v is None else bm[k][v]
                d = float(np.linalg.norm(x1 - x0) / np.linalg.norm(x1))
                r = max(r, d) if d == d else d   # a NaN stays NaN
        s.close()
        print("case", c, "L", case["L"], "batched", int(steps[c]), resid[c], "single grid", n, r)
        assert n == int(steps[c]), (c, n, steps[c])
        assert abs(r - resid[c]) <= 1e-9 * resid[c]
