"""Throughput benchmark of the Zakharov/HOS wave step on one MI355X.

Workload (default): 512 x 512 periodic grid, 200 m x 200 m, depth 20 m,
g = 9.81, HOS order M = 4, FP64, RK4 with dt = 0.05 s and the state filter,
seeded JONSWAP random-phase sea state (k_p = 2 pi / 12.5 m, gamma 3.3,
steepness 0.1, seed 1).  One step = one RK4 step (four right-hand sides:
the DtN series, the Bernoulli term, the RK4 combination and the filter).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line: the whole-job throughput in grid-point-steps/s with
the state resident in HBM when the timed region starts, the roofline of the
dominant kernel (algorithmic bytes / its average launch time, timed with HIP
events on the launch stream in a separate instrumented pass), and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "grid-point-steps/sec (RK4, HOS order M) + %HBM roofline; learned/FP32 vs FP64 at 1e-4"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(w, eta, psi, nsteps, workers=None):
    """The CPU oracle (numpy/pocketfft, FP64, as it stands) on nsteps RK4 steps
    of the same workload; `workers` FFT threads (default os.cpu_count())."""
    from oracle.hos import Grid, HOSModel, PocketDFT

    workers = workers or os.cpu_count() or 1
    g = Grid(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], dft=PocketDFT(workers=workers))
    m = HOSModel(g, w["M"])
    t0 = time.perf_counter()
    m.step(eta, psi, w["dt"], nsteps)
    t = time.perf_counter() - t0
    return {"value": round(w["nx"] * w["ny"] * nsteps / t, 1), "unit": "grid-point-steps/s", "cores": workers,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{nsteps} RK4 steps of the benchmark workload ({t:.1f} s, pocketfft workers={workers})"}


def copy_ceiling(mib=2048, reps=5):
    """Measured HBM ceiling: a plain device-to-device copy of `mib` MiB
    (bytes read + bytes written per second, best of `reps`, HIP events on
    the current stream)."""
    import torch

    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * n * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return {"GB_per_s": round(best, 1), "bytes_per_copy": 2 * n * 8, "kind": "device-to-device copy"}


def kernel_source_hash():
    """Hash of the HIP kernel sources, the planner that schedules them and the
    build script that holds the compiler flags: a counter record applies to
    the build it was taken on."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_2608_25203_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")) or f == "zk_plan.cpp":
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    with open(os.path.join(HERE, "paper_2608_25203_amd", "build.py"), "rb") as fh:
        h.update(b"build.py" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    record (FETCH_SIZE and WRITE_SIZE runs scaled by a copy calibration), or
    None when the record is missing or was taken on other kernel sources."""
    path = os.path.join(HERE, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    key = f"{workload}/fp{precision}/{kernel}"
    r = rec.get(key)
    if not r or r.get("kernel_source_hash") != kernel_source_hash():
        return None
    return r["bytes_per_launch"]


def rel_max(a, b):
    """max |a - b| / max |b| over one field (the error measure of the parity tests)."""
    return float((a - b).abs().max().item() / max(b.abs().max().item(), 1e-300))


def precision_form(segments=(1, 9, 90, 400)):
    """FP32-transform form against the FP64 run on the 2048 x 2048, M = 5
    workload: both advance the same JONSWAP state for sum(segments) RK4 steps
    (in calls of the given lengths); reported are each run's grid-point-steps/s
    and the max relative eta and psi error of the FP32 form after each call."""
    import torch

    from paper_2608_25203_amd.inputs import WORKLOADS, jonswap_state
    from paper_2608_25203_amd.zk import Solver

    w = WORKLOADS["c3_2048_m5"]
    eta, psi = jonswap_state(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["kp"], w["steepness"],
                             w["seed"])
    dev = torch.device("cuda:0")
    runs, shapes = {}, {}
    for prec in (64, 32):
        s = Solver(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["M"], precision=prec, check=False,
                   device=dev)
        shapes[prec] = {k: {"T": v[0], "E": v[1]} for k, v in s.autotune(w["dt"], reps=2).items()}
        e = torch.tensor(eta, dtype=torch.float64, device=dev)
        p = torch.tensor(psi, dtype=torch.float64, device=dev)
        ew, pw = e.clone(), p.clone()
        s.step(ew, pw, w["dt"], 2)  # warmup on a copy (uploads the schedule)
        del ew, pw
        torch.cuda.synchronize()
        snaps, t = [], 0.0
        for k in segments:
            t0 = time.perf_counter()
            s.step(e, p, w["dt"], k)
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            snaps.append((e.clone(), p.clone()) if prec == 64 else (e, p))
            if prec == 32:
                e64, p64 = runs[64]["snaps"][len(snaps) - 1]
                snaps[-1] = (rel_max(e, e64), rel_max(p, p64))
                e, p = e.clone(), p.clone()
        runs[prec] = {"snaps": snaps, "time": t}
        print(f"# precision form: fp{prec} {sum(segments)} steps in {t:.2f} s", file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()
    nsteps = sum(segments)
    npts = w["nx"] * w["ny"]
    cum = [sum(segments[:i + 1]) for i in range(len(segments))]
    errs = [{"step": c, "eta_rel_err": round(a, 9), "psi_rel_err": round(b, 9)}
            for c, (a, b) in zip(cum, runs[32]["snaps"])]
    v64 = npts * nsteps / runs[64]["time"]
    v32 = npts * nsteps / runs[32]["time"]
    worst = max(max(d["eta_rel_err"], d["psi_rel_err"]) for d in errs)
    return {"workload": f"c3_2048_m5: {w['nx']}x{w['ny']}, 2pi x 2pi, deep, M={w['M']}, RK4 dt={w['dt']}, "
                        f"JONSWAP steepness {w['steepness']}, {nsteps} steps",
            "fp64_value": round(v64, 1), "fp32_value": round(v32, 1), "unit": "grid-point-steps/s",
            "speedup": round(v32 / v64, 3), "errors_vs_fp64": errs, "max_rel_err": worst,
            "within_1e-4": bool(worst <= 1e-4), "team_shapes": shapes}


def closure_form(nsteps=1000, audit_every=10, tol=1e-4, floor_tol=2e-3):
    """Learned closure on its training geometry (1024 x 1024, 2 pi, deep,
    k_p = 32, dt = 0.007, JONSWAP steepness 0.1, seed 42) against plain
    order 6 in FP64 over nsteps RK4 steps: grid-point-steps/s and the max
    relative eta error of order 2 alone, of order 2 + network (low order in
    FP64 and in FP32), and of the audited closure (audit every `audit_every`
    steps, fallback to order 6 while the DtN error exceeds `tol`; again at
    `floor_tol`, above the network's error floor)."""
    import json as _json

    import numpy as np
    import torch

    from paper_2608_25203_amd.inputs import WORKLOADS, jonswap_state
    from paper_2608_25203_amd.zk import Closure, Net, Solver

    wdir = os.path.join(HERE, "paper_2608_25203_amd", "weights")
    meta = _json.load(open(os.path.join(wdir, "closure_c5.json")))
    params = np.load(os.path.join(wdir, "closure_c5.npy"), allow_pickle=False)
    w = WORKLOADS["c5_1024_m6"]
    n, L, dt = w["nx"], w["Lx"], w["dt"]
    eta, psi = jonswap_state(n, n, L, L, w["depth"], w["g"], w["kp"], w["steepness"], w["seed"])
    dev = torch.device("cuda:0")
    full = Solver(n, n, L, L, w["depth"], w["g"], 6, check=False, device=dev)
    low64 = Solver(n, n, L, L, w["depth"], w["g"], 2, check=False, device=dev)
    low32 = Solver(n, n, L, L, w["depth"], w["g"], 2, precision=32, check=False, device=dev)
    for sv in (full, low64, low32):
        sv.autotune(dt, reps=2)
    net = Net(n * n, device=dev)
    net.set_params(params)
    clo64 = Closure(low64, full, net, meta["k0"], meta["eta_scale"], meta["out_scale"])
    clo32 = Closure(low32, full, net, meta["k0"], meta["eta_scale"], meta["out_scale"])

    def run(advance, warm=True):
        if warm:
            e, p = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (eta, psi))
            advance(e, p, 2)
        e, p = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (eta, psi))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        advance(e, p, nsteps)
        torch.cuda.synchronize()
        return e, time.perf_counter() - t0

    e6, t6 = run(lambda e, p, k: full.step(e, p, dt, k))
    out = {"workload": f"c5_1024_m6: {n}x{n}, 2pi x 2pi, deep, k_p={w['kp']:g}, RK4 dt={dt}, JONSWAP steepness "
                       f"{w['steepness']}, seed {w['seed']}, {nsteps} steps; reference: order 6, FP64",
           "unit": "grid-point-steps/s", "order6_fp64_value": round(n * n * nsteps / t6, 1)}
    cases = {"order2_fp64": lambda e, p, k: low64.step(e, p, dt, k),
             "closure_fp64": lambda e, p, k: clo64.step(e, p, dt, k),
             "closure_fp32": lambda e, p, k: clo32.step(e, p, dt, k)}
    for name, adv in cases.items():
        e, t = run(adv)
        out[name] = {"value": round(n * n * nsteps / t, 1), "speedup_vs_order6": round(t6 / t, 3),
                     "eta_rel_err_vs_order6": rel_max(e, e6)}
        print(f"# closure form: {name} {t:.2f} s, eta err {out[name]['eta_rel_err_vs_order6']:.3e}",
              file=sys.stderr, flush=True)
    # audited runs: at the 1e-4 fallback tolerance, and at one just above the
    # network's DtN error floor on this workload (which it can pass)
    for name, tl in (("closure_audited_fp32", tol), ("closure_audited_fp32_above_floor", floor_tol)):
        clo32.close()
        clo32 = Closure(low32, full, net, meta["k0"], meta["eta_scale"], meta["out_scale"])
        e, t = run(lambda e, p, k: clo32.step(e, p, dt, k, audit_every, tl), warm=False)  # noqa: B023
        st = clo32.stats()
        out[name] = {"value": round(n * n * nsteps / t, 1), "speedup_vs_order6": round(t6 / t, 3),
                     "eta_rel_err_vs_order6": rel_max(e, e6), "audit_every": audit_every, "tol": tl,
                     "closure_steps": st["closure_steps"], "fallback_steps": st["fallback_steps"],
                     "audits": st["audits"], "acceptance_rate": st["closure_steps"] / max(1, nsteps),
                     "max_audited_dtn_err": st["max_err"]}
        print(f"# closure form: {name} {t:.2f} s, accepted {st['closure_steps']} of {nsteps}", file=sys.stderr,
              flush=True)
    st = out["closure_audited_fp32"]
    if st["closure_steps"] < nsteps / 2:
        out["note"] = (f"the audited closure accepted {st['closure_steps']} of {nsteps} steps at tol {tol:g} (largest "
                       f"audited DtN error {st['max_audited_dtn_err']:.2e}): the network's DtN error sits above the "
                       "tolerance, so of the reduced forms only the FP32 precision form meets the 1e-4 bound with a "
                       "speed-up (precision_form); the unaudited closure rows are speed and eta error without that "
                       f"bound, and closure_audited_fp32_above_floor is the audited form at tol {floor_tol:g}")
    for o in (clo64, clo32, net, low64, low32, full):
        o.close()
    torch.cuda.empty_cache()
    return out


def closure_steps_only(nsteps):
    """A short run for kernel profiles: nsteps closure RK4 steps (order 2 in
    FP32 plus the network) and nsteps plain order-2 FP32 steps on the closure
    workload (1024 x 1024, steepness 0.1), after two warmup steps each."""
    import json as _json

    import numpy as np
    import torch

    from paper_2608_25203_amd.inputs import WORKLOADS, jonswap_state
    from paper_2608_25203_amd.zk import Closure, Net, Solver

    wdir = os.path.join(HERE, "paper_2608_25203_amd", "weights")
    meta = _json.load(open(os.path.join(wdir, "closure_c5.json")))
    params = np.load(os.path.join(wdir, "closure_c5.npy"), allow_pickle=False)
    w = WORKLOADS["c5_1024_m6"]
    n, L, dt = w["nx"], w["Lx"], w["dt"]
    eta, psi = jonswap_state(n, n, L, L, w["depth"], w["g"], w["kp"], w["steepness"], w["seed"])
    full = Solver(n, n, L, L, w["depth"], w["g"], 6, check=False)
    low = Solver(n, n, L, L, w["depth"], w["g"], 2, precision=32, check=False)
    net = Net(n * n)
    net.set_params(params)
    clo = Closure(low, full, net, meta["k0"], meta["eta_scale"], meta["out_scale"])
    out = {}
    for name, adv in (("closure_fp32", lambda e, p, k: clo.step(e, p, dt, k)),
                      ("order2_fp32", lambda e, p, k: low.step(e, p, dt, k))):
        e, p = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (eta, psi))
        adv(e, p, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        adv(e, p, nsteps)
        torch.cuda.synchronize()
        out[name + "_ms_per_step"] = round(1e3 * (time.perf_counter() - t0) / nsteps, 4)
    for o in (clo, net, low, full):
        o.close()
    return out


def batch_form(nsteps=100, seq_steps=20, ntiles=256):
    """Many independent tiles in one batch: 256 tiles drawn from
    default_rng(4) -- size uniform in {128, 256, 512, 1024}^2 with 1 m
    spacing, M uniform in 3..6, depth uniform in [10, 200] m, JONSWAP
    steepness uniform in [0.02, 0.12] (k_p = 2 pi / 16 m, seed 1000 + i) --
    FP32 transforms with FP64 series and state, RK4 dt = 0.05 s, team shapes
    autotuned, each step replayed as a HIP graph.  Whole-batch grid-point-
    steps/s, beside the same tiles stepped one context after another."""
    import numpy as np
    import torch

    from paper_2608_25203_amd.inputs import jonswap_state
    from paper_2608_25203_amd.zk import Batch, Solver

    rng = np.random.default_rng(4)
    kp, dt, g = 2 * math.pi / 16.0, 0.05, 9.81
    tiles, states = [], []
    for i in range(ntiles):
        n = int(rng.choice([128, 256, 512, 1024]))
        M = int(rng.integers(3, 7))
        h = float(rng.uniform(10.0, 200.0))
        st = float(rng.uniform(0.02, 0.12))
        tiles.append(dict(nx=n, ny=n, Lx=float(n), Ly=float(n), depth=h, M=M))
        states.append(jonswap_state(n, n, float(n), float(n), h, g, kp, st, 1000 + i))
    print(f"# batch form: {ntiles} tiles generated", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    pts = sum(t["nx"] * t["ny"] for t in tiles)
    b = Batch(tiles, g=g, precision=32, device=dev)
    es = [torch.tensor(e, dtype=torch.float64, device=dev) for e, _ in states]
    ps = [torch.tensor(p, dtype=torch.float64, device=dev) for _, p in states]
    b.set_fields(es, ps)
    tuning = b.autotune(dt, reps=2)
    b.step(dt, 2)  # warm-up: graphs replayed once
    for k, (e, p) in enumerate(states):  # restore the initial state in the same buffers
        es[k].copy_(torch.from_numpy(e))
        ps[k].copy_(torch.from_numpy(p))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(dt, nsteps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    print(f"# batch form: {nsteps} batched steps in {tb:.2f} s", file=sys.stderr, flush=True)
    st_b = b.stats()
    # the persistent form: one launch per step, the same tiles and steps
    bp = Batch(tiles, g=g, precision=32, device=dev, persistent=True)
    ep = [torch.tensor(e, dtype=torch.float64, device=dev) for e, _ in states]
    pp = [torch.tensor(p, dtype=torch.float64, device=dev) for _, p in states]
    bp.set_fields(ep, pp)
    tuning_p = bp.autotune(dt, reps=2)
    bp.step(dt, 2)
    for k, (e, p) in enumerate(states):
        ep[k].copy_(torch.from_numpy(e))
        pp[k].copy_(torch.from_numpy(p))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bp.step(dt, nsteps)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    print(f"# batch form: {nsteps} persistent steps in {tp:.2f} s", file=sys.stderr, flush=True)
    pdiff = max(rel_max(ep[k], es[k]) for k in range(ntiles))
    st_p = bp.stats()
    bp.close()
    del b, es, ps, bp, ep, pp
    torch.cuda.empty_cache()
    # the same tiles one context after another (seq_steps steps, same start)
    solvers, es2, ps2 = [], [], []
    for t, (e, p) in zip(tiles, states):
        solvers.append(Solver(t["nx"], t["ny"], t["Lx"], t["Ly"], t["depth"], g, t["M"], precision=32, check=False,
                              device=dev))
        es2.append(torch.tensor(e, dtype=torch.float64, device=dev))
        ps2.append(torch.tensor(p, dtype=torch.float64, device=dev))
    for s, e, p in zip(solvers, es2, ps2):  # warm-up on copies
        s.step(e.clone(), p.clone(), dt, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e, p in zip(solvers, es2, ps2):
        s.step(e, p, dt, seq_steps)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    # the batch's result after seq_steps for the largest-M tile equals its context's
    bchk = Batch(tiles, g=g, precision=32, device=dev)
    es3 = [torch.tensor(e, dtype=torch.float64, device=dev) for e, _ in states]
    ps3 = [torch.tensor(p, dtype=torch.float64, device=dev) for _, p in states]
    bchk.set_fields(es3, ps3)
    bchk.step(dt, seq_steps)
    torch.cuda.synchronize()
    diff = max(rel_max(es3[k], es2[k]) for k in range(ntiles))
    bchk.close()
    for s in solvers:
        s.close()
    torch.cuda.empty_cache()
    sizes = {n: sum(1 for t in tiles if t["nx"] == n) for n in (128, 256, 512, 1024)}
    return {"workload": f"{ntiles} tiles, sizes {sizes} (1 m spacing), M 3..6, depth 10..200 m, JONSWAP "
                        f"steepness 0.02..0.12, k_p = 2 pi / 16 m, RK4 dt {dt} s, FP32 transforms",
            "grid_points": pts, "value": round(pts * nsteps / tb, 1), "unit": "grid-point-steps/s",
            "steps": nsteps, "ms_per_step": round(1e3 * tb / nsteps, 3),
            "sequential_value": round(pts * seq_steps / ts, 1), "sequential_steps": seq_steps,
            "speedup_vs_sequential": round((pts * nsteps / tb) / (pts * seq_steps / ts), 3),
            "phases_per_step": st_b["phases_per_step"], "launches_per_step": st_b["launches_per_step"],
            "graph": True, "tuning": tuning, "max_rel_diff_vs_sequential_eta": diff,
            "persistent": {"value": round(pts * nsteps / tp, 1), "ms_per_step": round(1e3 * tp / nsteps, 3),
                           "launches_per_step": st_p["launches_per_step"], "speedup_vs_graph": round(tb / tp, 3),
                           "max_rel_diff_vs_graph_eta": pdiff, "tuning": tuning_p}}


def ifab2_form(w, warmup, nsteps, rk4_value, rk4_eta):
    """The paper's own integrator (exact-linear Adams-Bashforth 2, Sec. 3.4)
    on the benchmark workload: the same warmup and timed calls as the RK4
    run, grid-point-steps/s of the timed call, and the max relative eta
    difference from the RK4 state after the same steps."""
    import numpy as np
    import torch

    from paper_2608_25203_amd.inputs import jonswap_state
    from paper_2608_25203_amd.zk import Solver

    eta, psi = jonswap_state(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["kp"], w["steepness"],
                             w["seed"])
    dev = torch.device("cuda:0")
    s = Solver(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["M"], check=False, device=dev,
               integrator="ifab2")
    e, p = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (eta, psi))
    if warmup > 0:
        s.step(e, p, w["dt"], warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(e, p, w["dt"], nsteps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    H = s.hamiltonian(e, p)
    v = w["nx"] * w["ny"] * nsteps / t
    s.close()
    return {"value": round(v, 1), "unit": "grid-point-steps/s", "ms_per_step": round(1e3 * t / nsteps, 4),
            "speedup_vs_rk4": round(v / rk4_value, 3), "eta_rel_diff_vs_rk4": rel_max(e, rk4_eta),
            "H_after": H, "steps": nsteps}


def _kernel_table(s, ncalls):
    st = s.kernel_stats()
    return {k: {"launches_per_call": v[3] / ncalls, "avg_us": round(1e3 * v[0] / v[3], 3),
                "GB_per_s": round(v[1] / (v[0] * 1e-3) / 1e9, 1)}
            for k, v in st.items() if v[3]}


def inverse_dno_form(w, ncalls=20, iters=8):
    """The inverse DNO map (eq:psi_inverse, eight fixed-point iterations) on
    the benchmark grid: v = G(eta) psi of the benchmark state, then psi back
    from (eta, v); ms per map, maps/s, and the recovery error of the
    zero-mean potential."""
    import torch

    from paper_2608_25203_amd.inputs import jonswap_state
    from paper_2608_25203_amd.zk import ZK_OPT_PROFILE, Solver

    eta, psi = jonswap_state(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["kp"], w["steepness"],
                             w["seed"])
    dev = torch.device("cuda:0")
    s = Solver(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["M"], check=False, device=dev)
    e, p = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (eta, psi))
    p = p - p.mean()
    v = s.dtn(e, p)
    out = s.inverse_dtn(e, v, iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(ncalls):
        out = s.inverse_dtn(e, v, iters)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / ncalls
    s.set_option(ZK_OPT_PROFILE, 1)
    s.reset_stats()
    s.inverse_dtn(e, v, iters)
    torch.cuda.synchronize()
    kern = _kernel_table(s, 1)
    s.close()
    return {"workload": f"{w['nx']}x{w['ny']}, M={w['M']}, {iters} iterations, FP64", "ms_per_map": round(1e3 * t, 4),
            "maps_per_s": round(1 / t, 1), "grid_points_per_s": round(w["nx"] * w["ny"] / t, 1),
            "psi_recovery_rel_err": rel_max(out, p), "kernels": kern}


def depth_velocity_form(w, nlayers=32, ncalls=10):
    """Bulk velocity at depth layers (Alg. ComputeVolumeVelFrom2D) of the
    benchmark state: nlayers depths evenly spaced from the surface plane to
    the bottom; ms per call, layer-points/s (one layer-point = the three
    velocity components at one grid point of one layer) and the per-kernel
    rates of the layer lifts."""
    import numpy as np
    import torch

    from paper_2608_25203_amd.inputs import jonswap_state
    from paper_2608_25203_amd.zk import ZK_OPT_PROFILE, Solver

    eta, psi = jonswap_state(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["kp"], w["steepness"],
                             w["seed"])
    dev = torch.device("cuda:0")
    s = Solver(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["M"], check=False, device=dev)
    e, p = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (eta, psi))
    ys = list(np.linspace(0.0, w["depth"], nlayers))
    out = s.depth_velocity(e, p, ys)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(ncalls):
        out = s.depth_velocity(e, p, ys)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / ncalls
    s.set_option(ZK_OPT_PROFILE, 1)
    s.reset_stats()
    s.depth_velocity(e, p, ys)
    torch.cuda.synchronize()
    kern = _kernel_table(s, 1)
    finite = bool(torch.isfinite(out).all().item())
    s.close()
    return {"workload": f"{w['nx']}x{w['ny']}, depth {w['depth']:g} m, {nlayers} layers in [0, depth], FP64",
            "ms_per_call": round(1e3 * t, 4), "us_per_layer": round(1e6 * t / nlayers, 2),
            "layer_points_per_s": round(w["nx"] * w["ny"] * nlayers / t, 1),
            "output_GB_per_s": round(3 * 8 * w["nx"] * w["ny"] * nlayers / t / 1e9, 1), "finite": finite,
            "kernels": kern}


# ms per step of Orders 2 and 3 on an RTX 4090 (tab:wave_prop_time_comp): deep and shallow water
PAPER_TANK_MS = {"deep": {2: 6.352, 3: 13.52}, "shallow": {2: 6.167, 3: 13.43}}
TANK_CASES = {"deep": (20.0, 2.0), "shallow": (1.0, 1.0)}  # depth (m), bump amplitude A (m)
# The paper states no eps for the deep tank; at eps = 1 its Order-2 run overflows (the collapsing
# bump forms a central jet), so that case is also timed at the largest eps of 0.05 steps that
# stays finite for all 2000 frames in the oracle.
DEEP_ORDER2_EPS_READING = 0.85


def paper_tank(nsteps=2000):
    """The paper's wave-propagation timing workload (Sec. 8, tab:wave_prop_time_comp):
    20 m x 20 m tank, 128 x 128 cells, reflecting walls on all sides (even
    extension to 256 x 256), Gaussian bump sigma = 1 m, R = 6 m, at rest,
    IF-AB2 with dt = 0.01 s, 2000 steps, at Orders 2 and 3 (M = 2, 3), deep
    (20 m, A = 2 m) and shallow (1 m, A = 1 m), eps = 1, and the deep Order-2
    case again at eps = 0.85; ms per step beside the paper's RTX 4090 figures
    (none for a run that overflowed)."""
    import torch

    from paper_2608_25203_amd.inputs import tank_bump
    from paper_2608_25203_amd.zk import Solver

    n, L, dt = 128, 20.0, 0.01
    dev = torch.device("cuda:0")
    out = {"workload": "20 m tank, 128^2 cells, reflecting walls (256^2 extended), Gaussian bump sigma = 1 m, "
                       "R = 6 m, at rest, IF-AB2 dt = 0.01 s, FP64",
           "steps": nsteps}
    runs = [(case, M, 1.0) for case in TANK_CASES for M in (2, 3)] + [("deep", 2, DEEP_ORDER2_EPS_READING)]
    for case, M, eps in runs:
        depth, A = TANK_CASES[case]
        eta, psi = tank_bump(n, n, L, L, A)
        s = Solver(n, n, L, L, depth, 9.81, M, eps=eps, check=False, device=dev, integrator="ifab2",
                   boundary="reflect")
        e, p = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (eta, psi))
        s.step(e.clone(), p.clone(), dt, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(e, p, dt, nsteps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / nsteps
        ref = PAPER_TANK_MS[case][M]
        fin = bool(torch.isfinite(e).all().item())
        rec = {"depth": depth, "A": A, "eps": eps, "ms_per_step": round(ms, 4), "paper_ms_per_step_rtx4090": ref,
               "speedup_vs_paper": round(ref / ms, 1) if fin else None, "finite": fin,
               "max_eta": float(e.abs().max().item()) if fin else None}
        if not fin:
            rec["note"] = "the state overflowed before the last step: no timing comparison"
        if eps != 1.0:
            rec["note"] = "eps reading: the paper states no eps for the deep tank; eps = 1 overflows"
        out[f"{case}_order{M}" + ("" if eps == 1.0 else f"_eps{eps:g}")] = rec
        s.close()
    return out


def c2_diagnostics(w, H_before, H_after, timed_steps):
    """Hamiltonian drift of the timed run and the linear-limit dispersion error
    (eps = 0, filter off) of single modes on the benchmark grid: measured
    frequency against omega = sqrt(g k tanh(k h)), beside the closed form
    arg R(i omega dt) / (omega dt) - 1 of classical RK4."""
    import numpy as np
    import torch

    from paper_2608_25203_amd.zk import Solver

    # H_drift_rel spans the timed run (timed_steps steps, filter on)
    out = {"H_drift_rel": (H_after - H_before) / H_before, "H_drift_steps": timed_steps}
    dev = torch.device("cuda:0")
    # the same run with the state filter off separates its damping from the drift
    from paper_2608_25203_amd.inputs import jonswap_state

    eta0, psi0 = jonswap_state(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["kp"], w["steepness"],
                               w["seed"])
    s = Solver(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["M"], filt=False, check=False, device=dev)
    e = torch.tensor(eta0, dtype=torch.float64, device=dev)
    p = torch.tensor(psi0, dtype=torch.float64, device=dev)
    H0 = s.hamiltonian(e, p)
    s.step(e, p, w["dt"], w["steps"])
    out["H_drift_rel_filter_off"] = (s.hamiltonian(e, p) - H0) / H0
    out["H_drift_filter_off_steps"] = w["steps"]
    s.close()
    nx, ny, Lx, h, g, dt = w["nx"], w["ny"], w["Lx"], w["depth"], w["g"], w["dt"]
    s = Solver(nx, ny, Lx, w["Ly"], h, g, w["M"], eps=0.0, filt=False, check=False, device=dev)
    x = np.arange(nx) * Lx / nx
    disp = []
    for m in (int(round(w["kp"] * Lx / (2 * np.pi))), nx // 2 - 1):
        k = 2 * np.pi * m / Lx
        om = math.sqrt(g * k * math.tanh(k * h))
        th = om * dt
        K = max(1, int(2.5 / th))
        eta = np.tile(1e-3 * np.cos(k * x), (ny, 1))
        psi = np.tile(1e-3 * g / om * np.sin(k * x), (ny, 1))
        e = torch.tensor(eta, dtype=torch.float64, device=dev)
        p = torch.tensor(psi, dtype=torch.float64, device=dev)
        s.step(e, p, dt, K)
        c0 = np.fft.rfft(eta[0])[m]
        c1 = np.fft.rfft(e[0].cpu().numpy())[m]
        om_num = -np.angle(c1 / c0) / (K * dt)
        z = 1j * th
        R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
        disp.append({"mode": m, "k": k, "omega": om, "steps": K, "measured_rel_err": om_num / om - 1,
                     "rk4_closed_form": float(np.angle(R) / th - 1)})
    s.close()
    out["dispersion"] = disp
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2_512_m4")
    ap.add_argument("--precision", type=int, default=64, choices=(32, 64))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default team shapes")
    ap.add_argument("--row-fft", choices=("auto", "stockham", "lanes"), default="auto",
                    help="form of the padded row transforms (auto: the autotuner's choice)")
    ap.add_argument("--row-programs", choices=("compiled", "interpreted"), default="compiled",
                    help="padded row programs as compiled straight-line shapes where built, or all interpreted")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision-form (2048^2 M=5), closure-form (1024^2) and batch-form (256 tiles) runs")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed benchmark run and its instrumented pass (no diagnostics or forms; for profiling)")
    ap.add_argument("--closure-steps", type=int, default=0,
                    help="only run this many closure and order-2 steps on the closure workload and exit (profiling)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration_mib:
        import torch

        n = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}), flush=True)
        return
    if args.closure_steps:
        print(json.dumps(closure_steps_only(args.closure_steps)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2608_25203_amd.inputs import WORKLOADS, jonswap_state
    from paper_2608_25203_amd.zk import ZK_OPT_PROFILE, ZK_OPT_ROW_FFT, ZK_OPT_ROW_PROGRAMS, ZK_ROW_FFT_LANES, Solver

    w = dict(WORKLOADS[args.workload])
    eta, psi = jonswap_state(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["kp"], w["steepness"],
                             w["seed"])
    dev = torch.device("cuda:0")
    s = Solver(w["nx"], w["ny"], w["Lx"], w["Ly"], w["depth"], w["g"], w["M"], precision=args.precision,
               check=False, device=dev)
    e = torch.tensor(eta, dtype=torch.float64, device=dev)
    p = torch.tensor(psi, dtype=torch.float64, device=dev)

    if args.row_programs != "compiled":
        s.set_option(ZK_OPT_ROW_PROGRAMS, 0)
    shapes = s.autotune(w["dt"], reps=3) if not args.no_autotune else s.team_shapes()
    if args.row_fft != "auto":
        s.set_option(ZK_OPT_ROW_FFT, ZK_ROW_FFT_LANES if args.row_fft == "lanes" else 0)
    # warmup (also uploads the dt-dependent schedule)
    if args.warmup > 0:
        s.step(e, p, w["dt"], args.warmup)
    torch.cuda.synchronize()

    H_before = s.hamiltonian(e, p)
    # timed region: exactly `steps` RK4 steps in one call, inputs resident in HBM
    t0 = time.perf_counter()
    s.step(e, p, w["dt"], args.steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    finite = bool(torch.isfinite(e).all().item() and torch.isfinite(p).all().item())
    H_after = s.hamiltonian(e, p)
    e_timed = e.clone()
    npts = w["nx"] * w["ny"]
    value = npts * args.steps / t

    # instrumented pass (separate): per-kernel event times, algorithmic bytes and FFT flops
    s.set_option(ZK_OPT_PROFILE, 1)
    s.reset_stats()
    nprof = min(args.steps, 100)
    s.step(e, p, w["dt"], nprof)
    torch.cuda.synchronize()
    st = s.kernel_stats()
    s.set_option(ZK_OPT_PROFILE, 0)
    # Each launch is bracketed by its own pair of HIP events on the launch
    # stream, so a bracket also holds that launch's dispatch gap.  The
    # brackets are scaled down so that they sum to the timed step, which
    # bounds the kernels' true durations from above (the kernels run
    # back-to-back in the timed call).
    ms_step = 1e3 * t / args.steps
    ev_ms_step = sum(v[0] for v in st.values()) / nprof
    tscale = min(1.0, ms_step / ev_ms_step) if ev_ms_step > 0 else 1.0
    kern = {k: {"ms_total": v[0] * tscale, "launches": v[3], "avg_us": (1e3 * v[0] * tscale / v[3]) if v[3] else 0.0,
                "avg_us_event_bracket": (1e3 * v[0] / v[3]) if v[3] else 0.0,
                "GB_per_s": (v[1] / (v[0] * tscale * 1e-3) / 1e9) if v[0] else 0.0,
                "fft_GFLOP_per_s": (v[2] / (v[0] * tscale * 1e-3) / 1e9) if v[0] else 0.0,
                "alg_bytes_per_launch": (v[1] / v[3]) if v[3] else 0.0}
            for k, v in st.items()}
    dom = max(kern, key=lambda k: kern[k]["ms_total"])
    d = kern[dom]
    achieved = d["GB_per_s"]
    ceiling = copy_ceiling()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.workload, args.precision, dom), "kernel": dom,
                "kernel_avg_us": round(d["avg_us"], 2),
                "alg_bytes_per_launch": d["alg_bytes_per_launch"],
                "copy_ceiling_GBs": ceiling["GB_per_s"],
                "frac_of_copy_ceiling": round(achieved / ceiling["GB_per_s"], 4),
                "kernel_time": f"HIP-event brackets per launch on the launch stream, scaled by {tscale:.4f} so that "
                               "they sum to the timed ms_per_step",
                "fft_GFLOP_per_s": round(d["fft_GFLOP_per_s"], 1),
                "fft_flop_peak_TFLOPs": FP64_PEAK_TFLOPS if args.precision == 64 else FP32_PEAK_TFLOPS}
    step_kernel_ms = sum(v["ms_total"] for v in kern.values()) / nprof

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32-transforms/f64-series",
        "data": "synthetic (seeded JONSWAP random-phase sea state)",
        "config": {"workload": f"{args.workload}: {w['nx']}x{w['ny']} grid, {w['Lx']:g} m x {w['Ly']:g} m, "
                               f"depth {w['depth']:g} m, HOS order M={w['M']}, RK4 dt={w['dt']}, "
                               f"JONSWAP steepness {w['steepness']}",
                   "nx": w["nx"], "ny": w["ny"], "M": w["M"], "dt": w["dt"], "precision": args.precision},
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "kernel_ms_per_step": round(step_kernel_ms, 4),
        "team_shapes": {k: {"T": v[0], "E": v[1]} for k, v in shapes.items()},
        "row_fft": "lanes" if s.get_option(ZK_OPT_ROW_FFT) == ZK_ROW_FFT_LANES else "stockham",
        "row_programs": "compiled" if s.get_option(ZK_OPT_ROW_PROGRAMS) else "interpreted",
        "finite": finite,
    }
    if args.headline_only:
        args.no_forms = args.no_cpu_baseline = True
    elif args.workload == "c2_512_m4":
        out["c2_diagnostics"] = c2_diagnostics(w, H_before, H_after, args.steps)
        out["c2_diagnostics"]["H_before"] = H_before
        out["ifab2_form"] = ifab2_form(w, args.warmup, args.steps, value, e_timed)
        out["paper_tank"] = paper_tank()
        out["inverse_dno_form"] = inverse_dno_form(w)
        out["depth_velocity_form"] = depth_velocity_form(w)
    if not args.no_forms:
        out["precision_form"] = precision_form()
        out["closure_form"] = closure_form()
        out["batch_form"] = batch_form()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, eta, psi, args.cpu_steps)
        out["cpu_baseline"]["single_core"] = cpu_baseline(w, eta, psi, 1, workers=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
