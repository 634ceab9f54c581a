#!/usr/bin/env python3
"""Benchmark of the KSE-Parareal hot path on one MI355X.

A step is one whole KSE-Parareal solve (coarse initialisation, then K times
fine sweep over all slices, subspace update and serial correction) of the
single-solve workload: 512 x 256 grid, c_s = 1, U = 0.1, P = 32 slices over
T = 1, K = 4 iterations, 4 seeded Gaussian pressure bumps plus N(0, 1e-3)
noise on u, w, FP64.  The initial state is resident in HBM before the timed
region.  `value` is solves per second through the batched form (one fused
fine-step launch over all slices per RK-3 step, replayed from a HIP graph).

Also reported on the same workload: the plain form (one launch per slice),
the serial GPU fine run F^P(u0) with the epsilon of eq. errorDef beside
each time, the fused fine-step kernel against the HBM roofline (48 bytes
per grid-point step, timed with HIP events on the library stream), a short
served stream (p50/p99 latency, solves/s), and the CPU oracle on a bounded
sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_POINT_STEP = 48.0   # read and write u, w, p once per RK-3 step
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fine_step_traffic_c2_512x256.md")
TRAFFIC_WORKLOAD = "c2_512x256"  # the workload the counters were taken on
FINE_SRC = os.path.join(ROOT, "paper_1510_02237_amd", "csrc", "fine.hip")


def fine_src_hash():
    import hashlib
    return hashlib.sha256(open(FINE_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per grid-point step of k_fine_step from the committed
    FETCH_SIZE / WRITE_SIZE counter summary, if it was taken on the current
    kernel source; else None."""
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if line.startswith("traffic_bytes_per_point_step:"):
            vals["b"] = float(line.split(":", 1)[1])
        if line.startswith("fine_hip_sha256_16:"):
            vals["h"] = line.split(":", 1)[1].strip()
    if vals.get("h") != fine_src_hash() or "b" not in vals:
        return None
    return vals["b"]


def _rel_l2(a, b):
    import numpy as np
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def timed_solves(ctx, u0, K, out, n):
    import torch
    torch.cuda.synchronize()
    ms_fine = 0.0
    pts = 0
    t0 = time.perf_counter()
    for _ in range(n):
        ctx.solve(u0, K, out=out)
        st = ctx.stats()
        ms_fine += st["ms_fine"]
        pts += st["fine_point_steps"]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / n, ms_fine, pts, st


def serve_leg(n_req, rate, seed=4, timeout=300.0, closed_loop=False):
    """Poisson stream of KSE-Parareal requests (grids 128x64..1024x512,
    U in [0, 0.3], P in {8,...,64}, K = 4) through the server.  With
    closed_loop every request is submitted at once (the same seeded mix:
    the draws do not depend on the rate) and solves/s is the server's
    throughput."""
    import ctypes
    import numpy as np
    from paper_1510_02237_amd import binding, workloads as W
    lib = binding.load()
    h = ctypes.c_void_p()
    rc = lib.pr_server_create(0, 0, 8, ctypes.byref(h))
    if rc:
        raise RuntimeError(f"pr_server_create: {rc}")
    reqs = W.serving_stream(n_req, rate, seed=seed)
    states = [W.request_state(r) for r in reqs]
    tickets = []
    lat = []
    t_start = time.perf_counter()
    try:
        for r, u0 in zip(reqs, states):
            while (not closed_loop
                   and time.perf_counter() - t_start < r["t_arrival"]):
                time.sleep(0.0005)
            p = r["prob"]
            o = binding.default_opts(nu_f=p["nu_f"], nu_c=p["nu_c"],
                                     n_sound=p["n_sound"],
                                     rank_tol=p["rank_tol"])
            t = ctypes.c_uint64()
            rc = lib.pr_submit_ex(h, ctypes.byref(binding.grid(p["nx"], p["nz"], p["T"])),
                                  p["c_s"], p["U"], p["dt_f"], p["dt_g"], p["P"],
                                  r["K"], ctypes.byref(o), u0.ctypes.data,
                                  ctypes.byref(t))
            if rc:
                raise RuntimeError(f"pr_submit: {rc}")
            tickets.append((t.value, u0.shape))
            if len(tickets) % 100 == 0:
                print(f"served stream: {len(tickets)}/{n_req} submitted at "
                      f"{time.perf_counter() - t_start:.0f} s",
                      file=sys.stderr, flush=True)
        for t, shape in tickets:
            out = np.empty(shape)
            l = ctypes.c_double()
            while True:
                rc = lib.pr_poll(h, t, out.ctypes.data, ctypes.byref(l))
                if rc != binding.PR_EAGAIN:
                    break
                if time.perf_counter() - t_start > timeout:
                    raise RuntimeError("served stream timed out")
                time.sleep(0.001)
            if rc:
                raise RuntimeError(f"request failed: {rc}")
            lat.append(l.value)
            if len(lat) % 100 == 0:
                print(f"served stream: {len(lat)}/{n_req} done at "
                      f"{time.perf_counter() - t_start:.0f} s",
                      file=sys.stderr, flush=True)
        wall = time.perf_counter() - t_start
    finally:
        lib.pr_server_destroy(h)
    lat = np.array(lat) * 1e3
    return dict(requests=n_req,
                arrival_rate_per_s=None if closed_loop else rate,
                closed_loop=closed_loop,
                p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)),
                solves_per_s=n_req / wall, wall_s=wall)


def cpu_baseline(prob, u0, K):
    """The oracle as it stands, on a bounded sample of the same workload,
    single-threaded (BLAS limited to one thread, like the paper's ATLAS QR):
    8 fine propagations F over a slice, 3 coarse propagations G, one of its
    subspace updates (pivoted QR) at m = 2P raw columns and one application
    of K at the rank that update gives.  The solve time uses the oracle's own
    call counts: P G for the prediction, P K F, 2 P K applications of K (it
    applies K to the new and the old iterate of every slice), and K pivoted
    QRs of P, 2P, ..., KP columns (cost scaled by m^2 at fixed d)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle
    from oracle import kse
    from oracle.operators import Params
    prm = Params(**prob)
    P = prob["P"]
    nF, nG, m = 8, 3, 2 * P
    rng = np.random.default_rng(0)
    A = rng.normal(size=(u0.size, m))
    FA = rng.normal(size=(u0.size, m))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for _ in range(nF):
            oracle.fine_F(u0, prm)
        tF = (time.perf_counter() - t0) / nF
        t0 = time.perf_counter()
        for _ in range(nG):
            oracle.coarse_G(u0, prm)
        tG = (time.perf_counter() - t0) / nG
        t0 = time.perf_counter()
        S, FS, _ = kse.subspace_update(A, FA, prm.rank_tol)
        tQR = time.perf_counter() - t0
        t0 = time.perf_counter()
        kse.kse_apply(u0, S, FS, prm)
        tK = time.perf_counter() - t0
    qr = tQR * sum((k * P) ** 2 for k in range(1, K + 1)) / m ** 2
    t_solve = P * tG + P * K * tF + 2 * P * K * tK + qr
    sampled = nF * tF + nG * tG + tQR + tK
    return dict(value=1.0 / t_solve, unit="solves/s", cores=1, kind="oracle",
                sample=(f"{sampled:.1f} s of oracle work on the "
                        f"{prob['nx']}x{prob['nz']} workload, one thread: "
                        f"F over a slice ({prm.n_f} RK-3 steps) {tF:.2f} s, "
                        f"G ({prm.n_g} steps) {tG:.3f} s, pivoted QR of "
                        f"{m} columns {tQR:.2f} s, K at rank {S.shape[1]} "
                        f"{tK:.3f} s; solve extrapolated as {P} G + {P * K} F"
                        f" + {2 * P * K} K + {K} QRs = {t_solve:.0f} s"))


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2_512x256")
    ap.add_argument("--serve", type=int, default=48,
                    help="requests in the served-latency leg (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="arrival rate of the served stream (default: the "
                         "frozen rate of workloads.SERVE_RATE)")
    ap.add_argument("--serve-calibrate", action="store_true",
                    help="run only the served stream closed-loop (every "
                         "request at once) and print its throughput")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed batched solves (for profiling)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the served stream (--serve requests at "
                         "--serve-rate) and print its summary")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="end with one device-to-device copy of this many "
                         "MiB (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the method is parallel in time within one device here",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1510_02237_amd import binding, workloads as W

    if args.serve_rate is None:
        args.serve_rate = W.SERVE_RATE
    if args.serve_calibrate:
        out = serve_leg(args.serve, args.serve_rate, timeout=1e9,
                        closed_loop=True)
        print(json.dumps(out))
        return
    if args.serve_only:
        out = serve_leg(args.serve, args.serve_rate, timeout=1e9)
        out["config"] = dict(workload="served stream", grids=list(W.SERVE_GRIDS),
                             slices=list(W.SERVE_SLICES), K=4, U="U[0, 0.3]",
                             max_inflight=8)
        print(json.dumps(out))
        return

    prob, K, u0 = W.config(args.workload)
    dev = torch.device("cuda:0")
    u0_d = torch.from_numpy(u0).to(dev)
    out = torch.empty_like(u0_d)
    ctx = binding.Context.from_problem(prob, form="batched")
    for _ in range(args.warmup):
        ctx.solve(u0_d, K, out=out)
    ms, ms_fine, pts, st = timed_solves(ctx, u0_d, K, out, args.steps)
    stage = stage_form(prob)
    # one launch per RK-3 step of every iteration of every window: the fused
    # step, or for per-row and per-column weights the fused three-stage tile
    # kernel; either reads and writes u, w, p once per step
    n_fine_launches = (args.steps * prob.get("windows", 1) * min(K, prob["P"])
                       * ctx_nf(prob))
    kernel_ms = ms_fine / n_fine_launches
    bpp = BYTES_PER_POINT_STEP
    achieved = bpp * pts / (ms_fine * 1e-3) / 1e9
    # the counters hold for the tile and chunk shape of the workload they
    # were taken on; other grids use other tiles
    tb = (measured_traffic()
          if not stage and args.workload == TRAFFIC_WORKLOAD else None)
    traffic = None if tb is None else tb * pts / n_fine_launches
    res = dict(
        metric="Parareal wall-time vs serial fine on GPU; stencil GB/s; "
               "p50/p99 served latency",
        value=1000.0 / ms, unit="solves/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=args.workload, grid=[prob["nx"], prob["nz"]],
                    P=prob["P"], K=K, U=prob["U"], c_s=prob["c_s"],
                    T=prob["T"], n_f=ctx_nf(prob), n_g=ctx_ng(prob),
                    windows=prob.get("windows", 1),
                    form="stagewise" if stage else "batched",
                    parallelism="time slices x tiles, 1 GPU"),
        phases_ms=dict(coarse_init=st["ms_coarse_init"], fine=st["ms_fine"],
                       update=st["ms_update"], chain=st["ms_chain"],
                       total=st["ms_total"]),
        ranks=st["rank"],
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBPS,
                      unit="GB/s", frac=achieved / HBM_PEAK_GBPS,
                      traffic=traffic,
                      kernel="k_stage3" if stage else "k_fine_step",
                      kernel_avg_ms=kernel_ms,
                      bytes_per_point_step=bpp,
                      algorithmic_bytes_per_launch=bpp * pts / n_fine_launches,
                      tile=None if stage else [st["tile_nt"], st["tile_zc"]],
                      fine_hip_sha256_16=fine_src_hash()),
        fine_point_updates_per_s=pts / (ms_fine * 1e-3),
    )
    if not args.no_extras:
        ref = ctx.serial_fine(u0_d).cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ser = ctx.serial_fine(u0_d)
        torch.cuda.synchronize()
        ser_ms = (time.perf_counter() - t0) * 1e3
        eps_b = _rel_l2(out.cpu().numpy(), ref)
        plain = binding.Context.from_problem(prob, form="plain")
        plain.solve(u0_d, K, out=out)
        pms, _, _, _ = timed_solves(plain, u0_d, K, out, max(1, args.steps // 2))
        eps_p = _rel_l2(out.cpu().numpy(), ref)
        coarse_only = ctx.solve(u0_d, 0).cpu().numpy()
        res["time_to_solution_ms"] = dict(
            batched=ms, plain=pms, serial_fine=ser_ms,
            eps_batched=eps_b, eps_plain=eps_p,
            eps_coarse_only=_rel_l2(coarse_only, ref),
            speedup_batched_vs_plain=pms / ms,
            speedup_batched_vs_serial_fine=ser_ms / ms)
        del ser
        res["windows"] = windows_leg(dev, max(1, args.steps // 2))
        res["instability"] = instability_leg()
        res["paper_tables"] = paper_tables_leg(dev)
        if args.serve > 0:
            res["served"] = serve_leg(args.serve, args.serve_rate)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(prob, u0, K)
        res["cpu_baseline"]["cpu_model"] = cpu_model()
        res["cpu_baseline"]["nproc"] = os.cpu_count()
    if args.calibrate_copy_mb > 0:
        n = args.calibrate_copy_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["calibration_copy_bytes"] = n * 8
    print(json.dumps(res))


def stage_form(prob):
    """True when the fine sweep of this workload runs in the stage form
    (per-row and per-column advective weights: the Section 3.1 pair, a
    z-velocity, a rotation or second-order acoustics), whose RK-3 step is
    one launch of the three-stage tile kernel."""
    return (prob.get("scheme", "split") == "rk3" or prob.get("V", 0.0) != 0.0
            or prob.get("gamma", 0.0) != 0.0
            or prob.get("fine_acoustic_order", 4) == 2)


def ctx_nf(prob):
    return int(round(prob["T"] / (prob.get("windows", 1) * prob["P"]) /
                     prob["dt_f"]))


def ctx_ng(prob):
    return int(round(prob["T"] / (prob.get("windows", 1) * prob["P"]) /
                     prob["dt_g"]))


def speedup_model(N_c, N_f, N_it, N_p, tau_c, tau_f, tau_qr):
    """Eq. speedup of one parallel step: N_t tau_f over the coarse
    prediction, N_it corrections and sweeps, and N_it subspace updates, with
    N_t = N_c N_f fine steps per parallel step."""
    N_t = N_c * N_f
    return N_t * tau_f / (N_c * tau_c + N_it * (N_c * tau_c + N_t / N_p * tau_f)
                          + N_it * tau_qr)


def instability_leg():
    """The instability example of Section 3.1 (workload demo_40x40): max|q|
    after every window for the serial fine run, the original Parareal and
    KSE-Parareal (the data of the paper's figure), computed by chaining
    one-window solves, plus the time of each whole solve."""
    import numpy as np
    from paper_1510_02237_amd import binding, workloads as W
    prob, K, u0 = W.config("demo_40x40")
    M = prob["windows"]
    one = dict(prob, windows=1, T=prob["T"] / M)
    c1 = binding.Context.from_problem(one)
    traj = {"fine": [], "parareal": [], "kse": []}
    qf = qp = qk = u0
    for _ in range(M):
        qf = c1.serial_fine(qf)
        qp = c1.solve(qp, K, parareal=True)
        qk = c1.solve(qk, K)
        traj["fine"].append(float(np.abs(qf).max()))
        traj["parareal"].append(float(np.abs(qp).max()))
        traj["kse"].append(float(np.abs(qk).max()))
    ctx = binding.Context.from_problem(prob)
    times = {}
    for name, kw in (("kse", {}), ("parareal", {"parareal": True})):
        ctx.solve(u0, K, **kw)
        t0 = time.perf_counter()
        ctx.solve(u0, K, **kw)
        times[name] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    ref = ctx.serial_fine(u0)
    times["serial_fine"] = (time.perf_counter() - t0) * 1e3
    return dict(workload="demo_40x40", windows=M, P=prob["P"], K=K,
                U=prob["U"], V=prob["V"], c_s=prob["c_s"],
                max_abs_q_per_window=traj, ms=times,
                eps_kse=_rel_l2(qk, ref), eps_parareal=_rel_l2(qp, ref))


PAPER_TABLES = os.path.join(ROOT, "tests", "golden", "paper_tables_1_2.json")


def paper_tables_leg(dev):
    """The solid-body-rotation runs of Section 3.2 on 40 x 40 cells: every
    cell (coarse CFL, P, K) of Tables 1 and 2 run to T = 2 (one coarse step
    per slice, T / (P dt_g) windows), with its time to solution on the GPU,
    the serial fine run's time, the error (eq. errorDef) and the paper's
    printed error and speedup beside it.  Plus the error after every tenth
    window for P = 6 (the data of the paper's error-versus-time figure),
    from chained one-window solves."""
    import torch
    from paper_1510_02237_amd import binding, workloads as W
    paper = {(c["cfl_c"], c["P"], c["K"]): c
             for c in json.load(open(PAPER_TABLES))["cells"]}
    u0 = torch.from_numpy(W.ic_cosine_bell(40, 40, centre=(0.5, 0.65))).to(dev)
    cells, ref, ser_ms = [], None, None
    for cc, P, K in W.PAPER_TABLE_CELLS:
        ctx = binding.Context.from_problem(W.rotation_problem(40, P, cc))
        if ref is None:
            ref = ctx.serial_fine(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.serial_fine(u0, out=ref)
            torch.cuda.synchronize()
            ser_ms = (time.perf_counter() - t0) * 1e3
            refh = ref.cpu().numpy()
        out = ctx.solve(u0, K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.solve(u0, K, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        pp = paper[(cc, P, K)]
        cells.append(dict(cfl_c=cc, P=P, K=K, windows=ctx.opts.windows, ms=ms,
                          speedup_vs_serial_fine=ser_ms / ms,
                          eps=_rel_l2(out.cpu().numpy(), refh),
                          paper_eps=pp["eps"], paper_speedup=pp["speedup"]))
    def energy(q):
        # total energy of Section 3.2.3: integral of u^2 + w^2 + p^2
        return float((q * q).sum()) / (40 * 40)

    traj, etraj = {}, {}
    for cc in (2.0, 4.0):
        prob = W.rotation_problem(40, 6, cc)
        M = prob["windows"]
        one = binding.Context.from_problem(
            dict(prob, windows=1, T=prob["T"] / M))
        for K in (1, 2, 3):
            qf, qk, e, en, enf = u0, u0, [], [], []
            for w in range(M):
                qf = one.serial_fine(qf)
                qk = one.solve(qk, K)
                if (w + 1) % 10 == 0:
                    e.append(_rel_l2(qk.cpu().numpy(), qf.cpu().numpy()))
                    en.append(energy(qk))
                    enf.append(energy(qf))
            traj[f"cfl_c={cc:g} K={K}"] = e
            etraj[f"cfl_c={cc:g} K={K}"] = en
        etraj[f"cfl_c={cc:g} serial fine"] = enf
    return dict(workload="rotation 40x40, T = 2 (Section 3.2)",
                serial_fine_ms=ser_ms, cells=cells,
                eps_every_10_windows_P6=traj,
                energy_every_10_windows_P6=dict(initial=energy(u0), **etraj))


def windows_leg(dev, steps):
    """The paper's decomposition of the 512x256 run (Section 2.1): every
    slice one coarse step, T / (P dt_g) windows of P slices in sequence."""
    import torch
    from paper_1510_02237_amd import binding, workloads as W
    prob, K, u0 = W.config("c2w_512x256")
    M, P = prob["windows"], prob["P"]
    n_f, n_g = ctx_nf(prob), ctx_ng(prob)
    u0_d = torch.from_numpy(u0).to(dev)
    out = torch.empty_like(u0_d)
    ctx = binding.Context.from_problem(prob, form="batched")
    ctx.solve(u0_d, K, out=out)
    ms, ms_fine, pts, st = timed_solves(ctx, u0_d, K, out, steps)
    ref = ctx.serial_fine(u0_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.serial_fine(u0_d, out=ref)
    torch.cuda.synchronize()
    ser_ms = (time.perf_counter() - t0) * 1e3
    refh = ref.cpu().numpy()
    eps = _rel_l2(out.cpu().numpy(), refh)
    eps0 = _rel_l2(ctx.solve(u0_d, 0).cpu().numpy(), refh)
    # tau_c: one coarse step of one state (the coarse predictions, M P n_g
    # dependent steps, device time); tau_f: one fine step of one state (the
    # serial run); tau_QR: one subspace update.
    tau_c = st["ms_coarse_init"] * 1e-3 / (M * P * n_g)
    tau_f = ser_ms * 1e-3 / (M * P * n_f)
    tau_qr = st["ms_update"] * 1e-3 / max(1, M * K)
    # Concurrency the batched sweep reaches: slice-steps at the serial rate
    # over the sweep time.
    slice_steps = pts / (prob["nx"] * prob["nz"])
    np_eff = slice_steps * tau_f / (ms_fine * 1e-3)
    return dict(
        workload="c2w_512x256", windows=M, P=P, K=K, n_f=n_f, n_g=n_g,
        ms=ms, serial_fine_ms=ser_ms, speedup_vs_serial_fine=ser_ms / ms,
        eps=eps, eps_coarse_only=eps0, phases_ms=dict(
            coarse_init=st["ms_coarse_init"], fine=st["ms_fine"],
            update=st["ms_update"], chain=st["ms_chain"]),
        tau_c_us=tau_c * 1e6, tau_f_us=tau_f * 1e6,
        tau_c_over_tau_f=tau_c / tau_f, tau_qr_ms=tau_qr * 1e3,
        model_speedup_np_eq_p=speedup_model(P, n_f, K, P, tau_c, tau_f, tau_qr),
        effective_np=np_eff,
        model_speedup_effective_np=speedup_model(P, n_f, K, np_eff, tau_c,
                                                 tau_f, tau_qr))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
