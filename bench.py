#!/usr/bin/env python3
"""Throughput of the NUFFT nonlocal-potential evaluation on one MI355X.

Workload: 2D potentials on [-16,16]^2 with a 512^2 grid; density exp(-(x^2+4y^2)) plus 8
seeded Gaussian bumps; kernels 1/(2 pi |x|) (polar-cancelled) and -ln|x|/(2 pi) (Gaussian
subtraction); 512 radial x 1024 azimuthal Fourier nodes; FP64 path (w = 24) and FP32 path
(w = 14).  One step = one FP64 potential evaluation with each kernel (the whole hot path:
moments, precorrect+FFT, interpolation+symbol, spreading, inverse FFT+postcorrect).
`value` = FP64 potential evaluations per second with inputs resident in HBM.

Prints ONE JSON line.  Options: --gpus N (only 1 is supported: one GPU), --steps K, --warmup W,
--mode full|prof (prof: a few evaluations plus a reference copy kernel, for rocprofv3 runs).
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_ALU = 78.6e12      # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP32_ALU = 157.3e12     # published FP32 vector peak (packed); non-packed issue is half
PEAK_HBM = 8.0e12


def kernel_sources_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1410_3584_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            return int(max(i.get("num_threads", 1) for i in info))
    except Exception:
        pass
    return os.cpu_count()


def cpu_baseline(n, L, rho, frac=2):
    """Time the FP64 oracle (direct sums) on 1/frac of the node set of the K2 evaluation and
    extrapolate linearly in the node count (both direct sums are linear in M)."""
    from oracle import potential as op
    dp = op.DirectPotential(n, L, op.COULOMB2D)
    M = dp.k.shape[0]
    sel = slice(0, M // frac)
    t0 = time.perf_counter()
    rh = op.type2_direct(rho, n, L, dp.k[sel])
    c = op.symbol_coeffs(op.COULOMB2D, dp.k[sel], dp.weight[sel], dp.kmag[sel], rh)
    op.type1_direct(c, n, L, dp.k[sel])
    dt = time.perf_counter() - t0
    per_eval = dt * frac
    return {"value": 1.0 / per_eval, "unit": "potential evals/s", "cores": blas_threads(),
            "kind": "oracle",
            "sample": f"FP64 direct type-2 + symbol + type-1 sums over {M // frac} of {M} nodes "
                      f"(1/{frac}) of one 512^2 Coulomb-2D evaluation, {dt:.1f} s, extrapolated x{frac}; "
                      f"host: {cpu_model()}"}


def sampled_parity(plan, rho_dev, rho_host, kernel, prec, rng):
    """Relative error of the GPU potential vs the oracle at sampled grid points, using the GPU's
    node values checked themselves at sampled nodes (same scheme as the parity tests)."""
    from oracle import potential as op
    n, L = plan.n, plan.L
    k, w = plan.nodes()
    rh = plan.type2(rho_dev).cpu().numpy().astype(np.complex128)
    sel = rng.choice(len(k), 64, replace=False)
    e2 = np.max(np.abs(rh[sel] - op.type2_direct(rho_host, n, L, k[sel]))) / np.max(np.abs(rh))
    kmag = np.linalg.norm(k, axis=1)
    m0 = m1 = None
    if kernel == op.LAPLACE2D:
        m0, m1 = op.moments(rho_host, n, L)
    c = op.symbol_coeffs(kernel, k, w, kmag, rh, m0, m1, plan.info.sigma)
    u = plan.potential(rho_dev).cpu().numpy().astype(np.float64)
    xs, _ = op.grid_axes(n, L)
    pts = [tuple(rng.integers(0, n[i]) for i in range(2)) for _ in range(24)]
    err = 0.0
    for p in pts:
        x = np.array([xs[0][p[0]], xs[1][p[1]]])
        v = float(np.real(np.sum(c * np.exp(1j * (k @ x)))))
        if kernel == op.LAPLACE2D:
            X, Y = np.array([[x[0]]]), np.array([[x[1]]])
            ax, ay = op.u12(X, Y, plan.info.sigma)
            v += m0 * op.u11(X, Y, plan.info.sigma)[0, 0] - (m1[0] * ax[0, 0] + m1[1] * ay[0, 0])
        err = max(err, abs(u[p] - v))
    return float(max(e2, err / np.max(np.abs(u))))


def stage_algorithmic(plan, stage):
    """Algorithmic work of one launch of a stage: (amount, unit, bound).
    interp / spread: 4 flops per stencil touch (two real FMAs on a complex value), w^d touches
    per node, M/2 nodes; FFT stages: bytes that must cross HBM once per pass."""
    info = plan.info
    d = info.dim
    w = 2 * info.msp
    es_c = 16 if info.prec == 0 else 8
    es_r = es_c // 2
    n = [info.n[i] for i in range(d)]
    N = int(np.prod(n))
    G = int(np.prod([2 * v for v in n]))
    if stage in ("interp", "spread"):
        return 4.0 * (w ** d) * info.n_half * info.batch, "flop", "alu"
    if stage == "fft_fwd":   # rows: read rho, write n0 oversampled rows; cols: read them, write grid
        rows = n[0] * 2 * n[1] * es_c
        return float(N * es_r + rows + rows + G * es_c) * info.batch, "byte", "hbm"
    if stage == "fft_inv":   # cols: read grid, write n0 rows; rows: read them, write u
        rows = n[0] * 2 * n[1] * es_c
        return float(G * es_c + rows + rows + N * es_r) * info.batch, "byte", "hbm"
    if stage == "zero":
        return float(G * es_c) * info.batch, "byte", "hbm"
    return float(N * es_r) * info.batch, "byte", "hbm"


def load_traffic(kernel_stage):
    """HBM bytes per launch of a stage from the committed rocprofv3 --pmc summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by the reading for a plain copy of known size), if that summary was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_potential_2d512.txt")
    vals = {}
    try:
        with open(path) as f:
            for line in f:
                line = line.split("#")[0].strip()
                if "=" in line:
                    k, v = line.split("=", 1)
                    vals[k.strip()] = v.strip()
    except OSError:
        return None
    if vals.get("sources") != kernel_sources_hash():
        return None
    v = vals.get(f"traffic_{kernel_stage}")
    return None if v is None else float(v)


def batched_evals(torch, nlf, n, L, rho, steps, warmup, batch=8):
    """The same 2D evaluations with `batch` fields per call (plans with opts.batch): potential
    evals/s (fields/s) of the K2/K3 alternation in FP64 and FP32, beside the single-field headline."""
    out = {"batch": batch, "unit": "potential evals/s"}
    for prec, dt, key in ((nlf.F64, torch.float64, "f64"), (nlf.F32, torch.float32, "f32")):
        r = torch.tensor(np.stack([rho] * batch), dtype=dt, device="cuda").contiguous()
        u = torch.empty_like(r)
        pk = [nlf.Plan(n, L, k, prec=prec, batch=batch) for k in (nlf.COULOMB2D, nlf.LAPLACE2D)]
        for _ in range(warmup):
            for p in pk:
                p.potential(r, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for p in pk:
                p.potential(r, u)
        torch.cuda.synchronize()
        out[key] = 2 * steps * batch / (time.perf_counter() - t0)
        del pk
    return out


def ground_states_per_s(torch, nlf, inputs):
    """Second half of the metric: 64 batched 2D ground states (grids drawn from 64^2/128^2/256^2 on
    [-16,16]^2, beta ~ U[10,1000], gamma ~ U[0.5,2], Coulomb 2D), gradient flow to
    max|phi^{n+1}-phi^n|/tau <= 1e-10, FP32 bulk then FP64 polish, one plan and stream per size
    class solved concurrently; timed once after an untimed warm-up solve of the same instances."""
    inst = inputs.ground_state_batch_2d(seed=3, count=64)
    groups = {}
    for d in inst:
        groups.setdefault(d["n"][0], []).append(d)
    keys = sorted(groups)
    streams = [torch.cuda.Stream() for _ in keys]
    plans = [nlf.Plan((k, k), (16.0, 16.0), nlf.COULOMB2D, prec=nlf.F32, batch=len(groups[k]), stream=s.cuda_stream)
             for k, s in zip(keys, streams)]
    betas = [[d["beta"] for d in groups[k]] for k in keys]
    gams = [[d["gamma"] for d in groups[k]] for k in keys]
    tuned = {str(k): p.autotune(reps=5)[0] for k, p in zip(keys, plans)}   # spreading decomposition per size
    kw = dict(tau=0.25, eps0=1e-10, max_iter=5000, mixed=True)
    nlf.ground_state_batch(plans, betas, gams, **kw)          # warm-up (twin plans, workspaces)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats, status = nlf.ground_state_batch(plans, betas, gams, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flat = [s for a in stats for s in a]
    return {"value": len(inst) / dt, "unit": "ground states/s", "instances": len(inst),
            "seconds": dt, "status": status, "tau": 0.25, "eps0": 1e-10, "schedule": "FP32 then FP64",
            "max_residual": max(s["residual"] for s in flat),
            "mean_outer_iters": float(np.mean([s["iters"] for s in flat])),
            "mean_fp32_iters": float(np.mean([s["iters_fp32"] for s in flat])),
            "sizes": {str(k): len(groups[k]) for k in keys},
            "spread_autotuned": {k: {"mode": ("gather", "scatter", "bins")[v[0]], "block": v[1], "item": v[2]}
                                 for k, v in tuned.items()}}


def dynamics_3d(torch, nlf, inputs, steps=20):
    """Third workload: 3D Coulomb-cubic time splitting on 256^3 of [-12,12]^3, harmonic trap,
    normalised Gaussian with seeded phase modulation, beta = 50, dt = 1e-3, Strang steps, FP64,
    with the split evaluation of the potential (Eq. '3.9'); one potential of the plain ball
    evaluation is timed beside it.  Reports steps/s over `steps` timed steps after 2 untimed
    ones, and the mass/energy drift over them."""
    n, L = (256,) * 3, (12.0,) * 3
    psi0 = inputs.psi0_phase_modulated(n, L, seed=0)
    psi = torch.tensor(psi0, dtype=torch.complex128, device="cuda")
    rho = (psi.abs() ** 2).contiguous()
    out = {"workload": "3D dynamics, 256^3 on [-12,12]^3, Coulomb, beta 50, dt 1e-3, Strang, FP64"}
    ball = nlf.Plan(n, L, nlf.COULOMB3D)
    ball.potential(rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ball.potential(rho)
    torch.cuda.synchronize()
    out["ball_potential_ms"] = 1e3 * (time.perf_counter() - t0)
    del ball
    torch.cuda.empty_cache()
    plan = nlf.Plan(n, L, nlf.COULOMB3D, split=True)
    u = plan.potential(rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        plan.potential(rho, u)
    torch.cuda.synchronize()
    out["split_potential_ms"] = 1e3 * (time.perf_counter() - t0) / 5
    plan.evolve(psi, 50.0, (1.0, 1.0, 1.0), 1e-3, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    diag = plan.evolve(psi, 50.0, (1.0, 1.0, 1.0), 1e-3, steps, diag_every=steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out.update({"steps": steps, "steps_per_s": steps / dt,
                "mass_drift": float(abs(diag[-1, 0, 0] - diag[0, 0, 0])),
                "energy_rel_drift": float(abs(diag[-1, 0, 1] - diag[0, 0, 1]) / abs(diag[0, 0, 1]))})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", choices=["full", "prof", "prof3d", "profgs"], default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ground-states", action="store_true")
    ap.add_argument("--no-dynamics-3d", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1410_3584_amd import inputs, nlf

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.mode == "prof3d":
        # the 3D dynamics workload's split potential evaluations and steps, for a kernel trace
        n3, L3 = (256,) * 3, (12.0,) * 3
        psi = torch.tensor(inputs.psi0_phase_modulated(n3, L3, seed=0), dtype=torch.complex128, device="cuda")
        rho3 = (psi.abs() ** 2).contiguous()
        plan = nlf.Plan(n3, L3, nlf.COULOMB3D, split=True)
        u = plan.potential(rho3)
        for _ in range(max(1, args.steps)):
            plan.potential(rho3, u)
        plan.evolve(psi, 50.0, (1.0, 1.0, 1.0), 1e-3, max(1, args.steps))
        torch.cuda.synchronize()
        print(json.dumps({"mode": "prof3d", "steps": args.steps}))
        return
    if args.mode == "profgs":
        # the batched ground-state workload alone, for a kernel trace
        gs = ground_states_per_s(torch, nlf, inputs)
        print(json.dumps({"mode": "profgs", "ground_states_per_s": gs["value"]}))
        return
    n, L, rho, _ = inputs.potential_2d_512(seed=1)
    dev = "cuda"
    r64 = torch.tensor(rho, dtype=torch.float64, device=dev)
    r32 = torch.tensor(rho, dtype=torch.float32, device=dev)
    plans = {
        ("K2", 0): nlf.Plan(n, L, nlf.COULOMB2D, prec=nlf.F64),
        ("K3", 0): nlf.Plan(n, L, nlf.LAPLACE2D, prec=nlf.F64),
        ("K2", 1): nlf.Plan(n, L, nlf.COULOMB2D, prec=nlf.F32),
        ("K3", 1): nlf.Plan(n, L, nlf.LAPLACE2D, prec=nlf.F32),
    }
    outs = {0: torch.empty(n, dtype=torch.float64, device=dev), 1: torch.empty(n, dtype=torch.float32, device=dev)}
    rin = {0: r64, 1: r32}

    def step(prec):
        plans[("K2", prec)].potential(rin[prec], outs[prec])
        plans[("K3", prec)].potential(rin[prec], outs[prec])

    if args.mode == "prof":
        # a few evaluations of every variant, then a plain copy of known size for calibrating
        # the HBM byte counters
        for _ in range(max(1, args.steps)):
            step(0)
            step(1)
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)   # 512 MiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "prof", "copy_bytes": a.numel() * 8}))
        return

    # ---- FP64 (headline) ----
    for _ in range(args.warmup):
        step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(0)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    # ---- FP32 ----
    for _ in range(args.warmup):
        step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(1)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    batched = None if args.no_batched else batched_evals(torch, nlf, n, L, rho, args.steps, args.warmup)

    # ---- live per-stage timing (HIP events on the plan's stream) for the roofline ----
    stage_avg = {}
    for key in (("K2", 0), ("K3", 0)):
        p = plans[key]
        p.set_profiling(True)
        p.stage_times(reset=True)
        for _ in range(args.steps):
            p.potential(rin[0], outs[0])
        st = p.stage_times(reset=True)
        p.set_profiling(False)
        stage_avg[key[0]] = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in st.items()}
    # dominant kernel: largest average launch time in the FP64 Laplace evaluation
    dom_stage = max(("interp", "spread", "fft_fwd", "fft_inv"), key=lambda s: stage_avg["K3"][s])
    amount, unit, bound = stage_algorithmic(plans[("K3", 0)], dom_stage)
    avg_s = stage_avg["K3"][dom_stage] * 1e-3
    if bound == "alu":
        achieved = amount / avg_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_ALU / 1e12, "unit": "TFLOP/s",
                "frac": achieved * 1e12 / PEAK_FP64_ALU}
    else:
        achieved = amount / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": achieved * 1e9 / PEAK_HBM}
    roof["traffic"] = load_traffic(dom_stage)
    roof["kernel"] = dom_stage
    roof["avg_launch_ms"] = stage_avg["K3"][dom_stage]

    # ---- parity of what was timed (sampled, vs the FP64 oracle) ----
    rng = np.random.default_rng(0)
    rho32_host = np.asarray(rho, dtype=np.float32).astype(np.float64)
    parity = {
        "K2_f64": sampled_parity(plans[("K2", 0)], r64, rho, 2, 0, rng),
        "K3_f64": sampled_parity(plans[("K3", 0)], r64, rho, 3, 0, rng),
        "K2_f32": sampled_parity(plans[("K2", 1)], r32, rho32_host, 2, 1, rng),
        "K3_f32": sampled_parity(plans[("K3", 1)], r32, rho32_host, 3, 1, rng),
    }

    cpu = None if args.no_cpu_baseline else cpu_baseline(n, L, rho)
    gs = None if args.no_ground_states else ground_states_per_s(torch, nlf, inputs)
    dyn = None if args.no_dynamics_3d else dynamics_3d(torch, nlf, inputs)

    value = 2 * args.steps / t64
    out = {
        "metric": "potential evals/sec at rel err 1e-10 (FP64) / 1e-6 (FP32); ground states/sec",
        "value": value,
        "unit": "potential evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t64 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D potential, 512^2 grid on [-16,16]^2, exp(-(x^2+4y^2)) + 8 seeded bumps, "
                               "kernels 1/(2 pi|x|) and -ln|x|/(2 pi) alternating, 512x1024 polar nodes, w=24",
                   "grid": [512, 512], "nodes": 524288, "msp_f64": 12, "msp_f32": 7},
        "fp32": {"value": 2 * args.steps / t32, "unit": "potential evals/s", "msp": 7},
        "batched": batched,
        "parity_rel_err": parity,
        "stage_ms": {k: {s: round(v, 5) for s, v in d.items()} for k, d in stage_avg.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "ground_states": gs,
        "dynamics_3d": dyn,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
