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

PEAK_FP64_ALU = 78.6e12      # FP64 vector and dense FP64 matrix peak: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
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


def oracle_reference(n, L, rho):
    """The FP64 oracle on the bench's 2D workload: its type-2 direct sum at every node, the
    Coulomb and Laplace node coefficients from it, and, timed as the CPU baseline, one
    evaluation's two direct sums: the type-2 sum over all nodes and the type-1 sum over half of
    them (the type-1 sum is linear in the node count, so its time is doubled)."""
    from oracle import potential as op
    d2 = op.DirectPotential(n, L, op.COULOMB2D)
    d3 = op.DirectPotential(n, L, op.LAPLACE2D)
    k, M = d2.k, d2.k.shape[0]
    t0 = time.perf_counter()
    rh = op.type2_direct(rho, n, L, k)
    t_t2 = time.perf_counter() - t0
    c2 = op.symbol_coeffs(op.COULOMB2D, k, d2.weight, d2.kmag, rh)
    half = slice(0, M // 2)
    t0 = time.perf_counter()
    op.type1_direct(c2[half], n, L, k[half])
    t_t1 = time.perf_counter() - t0
    m0, m1 = op.moments(rho, n, L)
    c3 = op.symbol_coeffs(op.LAPLACE2D, k, d3.weight, d3.kmag, rh, m0, m1, d3.sigma)
    per_eval = t_t2 + 2.0 * t_t1
    cpu = {"value": 1.0 / per_eval, "unit": "potential evals/s", "cores": blas_threads(), "kind": "oracle",
           "sample": f"FP64 direct sums of one 512^2 Coulomb-2D evaluation: type-2 over all {M} nodes "
                     f"({t_t2:.1f} s) and type-1 over {M // 2} of them ({t_t1:.1f} s, doubled); "
                     f"host: {cpu_model()}"}
    return {"k": k, "rhohat": rh, "c": {op.COULOMB2D: c2, op.LAPLACE2D: c3}, "m0": m0, "m1": m1,
            "sigma": d3.sigma, "cpu": cpu}


def parity_vs_oracle(plan, rho_dev, kernel, ref, pts):
    """Relative errors of what was timed against the oracle's own sums (no GPU value enters the
    oracle's side): the type-2 stage at every node, and the potential at the sampled grid points
    `pts`, where the oracle sums its node coefficients over the whole node set."""
    from oracle import potential as op
    n, L = plan.n, plan.L
    rh = plan.type2(rho_dev).cpu().numpy().astype(np.complex128)
    e2 = float(np.max(np.abs(rh - ref["rhohat"])) / np.max(np.abs(ref["rhohat"])))
    u = plan.potential(rho_dev).cpu().numpy().astype(np.float64)
    xs, _ = op.grid_axes(n, L)
    k, c = ref["k"], ref["c"][kernel]
    want = []
    for p in pts:
        x = np.array([xs[0][p[0]], xs[1][p[1]]])
        v = float(np.real(np.sum(c * np.exp(1j * (k @ x)))))
        if kernel == op.LAPLACE2D:
            X, Y = np.array([[x[0]]]), np.array([[x[1]]])
            ax, ay = op.u12(X, Y, ref["sigma"])
            m1 = ref["m1"]
            v += ref["m0"] * op.u11(X, Y, ref["sigma"])[0, 0] - (m1[0] * ax[0, 0] + m1[1] * ay[0, 0])
        want.append(v)
    want = np.array(want)
    got = np.array([u[p] for p in pts])
    eu = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    return {"type2_all_nodes": e2, "potential_sampled": eu}


def stage_algorithmic(plan, stage):
    """Algorithmic work of one launch of a stage: (amount, unit, bound).
    interp / spread: 5 flops per stencil touch (one weight product and two real FMAs on the
    complex value), w^d touches per node, M/2 nodes; FFT stages: bytes that must cross HBM once
    per pass."""
    info = plan.info
    d = info.dim
    w = 2 * info.msp
    es_c = 16 if info.prec == 0 else 8
    es_r = es_c // 2
    n = [info.n[i] for i in range(d)]
    N = int(np.prod(n))
    G = int(np.prod([2 * v for v in n]))
    if stage in ("interp", "spread"):
        return 5.0 * (w ** d) * info.n_half * info.batch, "flop", "alu"
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
    # the same batch in one persistent launch (timed the same way, after its own warm-up)
    nlf.ground_state_batch(plans, betas, gams, persistent=True, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, pstats, pstatus = nlf.ground_state_batch(plans, betas, gams, persistent=True, **kw)
    torch.cuda.synchronize()
    pdt = time.perf_counter() - t0
    pflat = [s for a in pstats for s in a]
    persistent = {"value": len(inst) / pdt, "seconds": pdt, "status": pstatus,
                  "one_launch": all(s["persistent"] == 1 for s in pflat),
                  "max_residual": max(s["residual"] for s in pflat)}
    return {"value": len(inst) / dt, "unit": "ground states/s", "instances": len(inst),
            "seconds": dt, "status": status, "tau": 0.25, "eps0": 1e-10, "schedule": "FP32 then FP64",
            "max_residual": max(s["residual"] for s in flat),
            "mean_outer_iters": float(np.mean([s["iters"] for s in flat])),
            "mean_fp32_iters": float(np.mean([s["iters_fp32"] for s in flat])),
            "sizes": {str(k): len(groups[k]) for k in keys},
            "spread_autotuned": {k: {"mode": ("gather", "scatter", "bins")[v[0]], "block": v[1], "item": v[2]}
                                 for k, v in tuned.items()},
            "persistent_launch": persistent}


def dynamics_3d(torch, nlf, inputs, steps=1000, diag_every=100):
    """Third workload: 3D Coulomb-cubic time splitting on 256^3 of [-12,12]^3, harmonic trap
    V = |x|^2/2, normalised Gaussian with seeded phase modulation, dt = 1e-3, Strang steps, FP64,
    the potential by the split evaluation (Eq. '3.9'); one potential of the plain ball evaluation
    is timed beside it.  For beta = +50 and beta = -10: `steps` timed steps from psi0 (after 2
    untimed steps on a copy), with mass and energy every `diag_every` steps (their evaluations
    are inside the timed region)."""
    n, L = (256,) * 3, (12.0,) * 3
    psi0 = torch.tensor(inputs.psi0_phase_modulated(n, L, seed=0), dtype=torch.complex128, device="cuda")
    rho = (psi0.abs() ** 2).contiguous()
    out = {"workload": f"3D dynamics, 256^3 on [-12,12]^3, Coulomb, dt 1e-3, {steps} Strang steps, FP64, "
                       "split evaluation"}
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
    for _ in range(3):
        plan.potential(rho, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        plan.potential(rho, u)
    torch.cuda.synchronize()
    out["split_potential_ms"] = 1e3 * (time.perf_counter() - t0) / 20
    for beta in (50.0, -10.0):
        warm = psi0.clone()
        plan.evolve(warm, beta, (1.0, 1.0, 1.0), 1e-3, 2)
        del warm
        psi = psi0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        diag = plan.evolve(psi, beta, (1.0, 1.0, 1.0), 1e-3, steps, diag_every=diag_every)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mass, en = diag[:, 0, 0], diag[:, 0, 1]
        out[f"beta_{beta:+g}"] = {
            "steps": steps, "steps_per_s": steps / dt, "seconds": dt,
            "t_final": steps * 1e-3,
            "mass_drift_max": float(np.max(np.abs(mass - mass[0]))),
            "energy_rel_drift_max": float(np.max(np.abs(en - en[0])) / abs(en[0])),
            "energy_every_100": [float(v) for v in en]}
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
    ap.add_argument("--dyn-steps", type=int, default=1000, help="Strang steps per beta of the 3D dynamics leg")
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
        print(json.dumps({"mode": "profgs", "ground_states_per_s": gs["value"],
                          "persistent_launch": gs["persistent_launch"]}))
        return
    n, L, rho, _ = inputs.potential_2d_512(seed=1)
    # rounded to FP32 values once: the FP64 and FP32 legs then evaluate the same density, and one
    # oracle result checks both
    rho = np.asarray(rho, dtype=np.float32).astype(np.float64)
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
    for key in (("K2", 0), ("K3", 0), ("K2", 1), ("K3", 1)):
        p = plans[key]
        p.set_profiling(True)
        p.stage_times(reset=True)
        for _ in range(args.steps):
            p.potential(rin[key[1]], outs[key[1]])
        st = p.stage_times(reset=True)
        p.set_profiling(False)
        stage_avg[key[0] + ("_f32" if key[1] else "")] = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in st.items()}
    # dominant kernel: largest average launch time in the FP64 Laplace evaluation
    dom_stage = max(("interp", "spread", "fft_fwd", "fft_inv"), key=lambda s: stage_avg["K3"][s])
    amount, unit, bound = stage_algorithmic(plans[("K3", 0)], dom_stage)
    avg_s = stage_avg["K3"][dom_stage] * 1e-3
    if bound == "alu":
        # the FP64 stencil kernels are dense contractions on the FP64 matrix cores (whose dense peak,
        # 78.6 TFLOP/s, equals the FP64 vector peak)
        achieved = amount / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_ALU / 1e12, "unit": "TFLOP/s",
                "frac": achieved * 1e12 / PEAK_FP64_ALU}
    else:
        achieved = amount / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": achieved * 1e9 / PEAK_HBM}
    roof["traffic"] = load_traffic(dom_stage)
    roof["kernel"] = dom_stage
    roof["avg_launch_ms"] = stage_avg["K3"][dom_stage]

    # ---- parity of what was timed, against the oracle's own full sums ----
    ref = oracle_reference(n, L, rho)
    rng = np.random.default_rng(0)
    pts = [tuple(int(v) for v in rng.integers(0, n[0], size=2)) for _ in range(48)] + [(256, 256), (0, 0)]
    parity = {
        "K2_f64": parity_vs_oracle(plans[("K2", 0)], r64, nlf.COULOMB2D, ref, pts),
        "K3_f64": parity_vs_oracle(plans[("K3", 0)], r64, nlf.LAPLACE2D, ref, pts),
        "K2_f32": parity_vs_oracle(plans[("K2", 1)], r32, nlf.COULOMB2D, ref, pts),
        "K3_f32": parity_vs_oracle(plans[("K3", 1)], r32, nlf.LAPLACE2D, ref, pts),
    }

    cpu = None if args.no_cpu_baseline else ref["cpu"]
    gs = None if args.no_ground_states else ground_states_per_s(torch, nlf, inputs)
    dyn = None if args.no_dynamics_3d else dynamics_3d(torch, nlf, inputs, steps=args.dyn_steps)

    value = 2 * args.steps / t64
    msp64, msp32 = plans[("K2", 0)].info.msp, plans[("K2", 1)].info.msp
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
        "config": {"workload": "2D potential, 512^2 grid on [-16,16]^2, exp(-(x^2+4y^2)) + 8 seeded bumps "
                               "(values rounded to FP32), kernels 1/(2 pi|x|) and -ln|x|/(2 pi) alternating, "
                               f"512x1024 polar nodes, w={2 * msp64} (FP64) / {2 * msp32} (FP32)",
                   "grid": [512, 512], "nodes": 524288, "msp_f64": msp64, "msp_f32": msp32},
        "fp32": {"value": 2 * args.steps / t32, "unit": "potential evals/s", "msp": msp32,
                 "ratio_to_f64": t64 / t32},
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
