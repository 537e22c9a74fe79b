"""Learned warm start for the gradient flow: data generation with the library's own batched
solver, training with the library's own network kernels, and the warm-vs-Gaussian comparison.
All numerical work runs in libnlf.so (nlf_ground_state*, nlf_ws_*); this module only arranges
the calls and the bookkeeping.

    python -m paper_1410_3584_amd.warmstart --dim 3 --n 64 --coarse 32 --train 2000 --test 200 --split
prints one JSON line with the held-out comparison (training targets solved on the --n grid and
restricted to the --coarse grid the network predicts).
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs, nlf


def features(betas, gammas):
    return np.array([[math.log(b)] + list(g) for b, g in zip(betas, gammas)], dtype=np.float32)


def solve_targets(instances, n_solve, n_coarse, L, kernel, dim, batch=100, tau=0.5, eps0=1e-9, split=False,
                  progress=False):
    """Ground states of the instances solved on the n_solve grid (FP64 flow, batched; split: the 3D
    potential by Eq. '3.9'), restricted to the coarse grid the network predicts: every
    (n_solve / n_coarse)-th point, both grids holding x_j = -L + j h on the same box."""
    import torch
    if n_solve % n_coarse:
        raise ValueError("the solve grid must refine the coarse grid")
    step = n_solve // n_coarse
    out = []
    for s in range(0, len(instances), batch):
        if progress:
            print(f"targets {s}/{len(instances)}", file=sys.stderr, flush=True)
        part = instances[s:s + batch]
        plan = nlf.Plan((n_solve,) * dim, (L,) * dim, kernel, batch=len(part), split=split)
        psi, st, status = plan.ground_state([d["beta"] for d in part], [d["gamma"] for d in part],
                                            tau=tau, eps0=eps0, max_iter=20000)
        if status != nlf.OK:
            raise RuntimeError(f"target solves returned status {status}")
        psi = psi.reshape((len(part),) + (n_solve,) * dim)[(slice(None),) + (slice(None, None, step),) * dim]
        out.append(psi.reshape(len(part), -1).float())
        del plan
    return torch.cat(out)


def train_model(X, T, hidden=128, epochs=3000, lr=2e-3, minibatch=0, seed=0):
    m = nlf.Model(X.shape[1], hidden, T.shape[1], seed=seed)
    Xh = X.cpu().numpy()
    m.set_standardisation(Xh.mean(0), Xh.std(0) + 1e-6)
    hist = m.train(X, T, epochs, minibatch=minibatch, lr=lr)
    return m, hist


def compare(model, instances, n, L, kernel, dim, coarse_n, tau=0.5, eps0=1e-10, prec=nlf.F64, mixed=False,
            split=False):
    """Held-out solves from the Gaussian start (nlf_ground_state) and from the learned start
    (nlf_ws_ground_state, Gaussian fallback judged by the one-step residual); split: the plan
    evaluates the 3D potential by the split of Eq. '3.9'."""
    import torch
    betas = [d["beta"] for d in instances]
    gams = [d["gamma"] for d in instances]
    B = len(instances)
    plan = nlf.Plan((n,) * dim, (L,) * dim, kernel, prec=prec, batch=B, split=split)
    kw = dict(tau=tau, eps0=eps0, max_iter=20000, mixed=mixed)
    model.ground_state(plan, betas[:1] * B, gams[:1] * B, coarse_n, **dict(kw, max_iter=1))   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st_g, stat_g = plan.ground_state(betas, gams, **kw)
    torch.cuda.synchronize()
    t_g = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st_w, stat_w, used = model.ground_state(plan, betas, gams, coarse_n, **kw)
    torch.cuda.synchronize()
    t_w = time.perf_counter() - t0
    dE = max(abs(a["E"] - b["E"]) for a, b in zip(st_g, st_w))
    return {"fields": B, "used_learned": int(sum(used)), "status_gauss": stat_g, "status_learned": stat_w,
            "iters_gauss_batch": max(s["iters"] for s in st_g), "iters_learned_batch": max(s["iters"] for s in st_w),
            "iters_gauss_mean": float(np.mean([s["iters"] for s in st_g])),
            "iters_learned_mean": float(np.mean([s["iters"] for s in st_w])),
            "seconds_gauss": t_g, "seconds_learned": t_w,
            "solves_per_s_gauss": B / t_g, "solves_per_s_learned": B / t_w,
            "max_energy_difference": dE,
            "max_residual_learned": max(s["residual"] for s in st_w)}


def per_field_iterations(plan, betas, gams, psi0, tau, eps0):
    """Outer steps each field needs, by solving the fields one at a time (diagnostic)."""
    out = []
    for i in range(len(betas)):
        single = nlf.Plan(plan.n, plan.L, plan.kernel, prec=plan.prec)
        p0 = None if psi0 is None else psi0[i].contiguous()
        _, st, _ = single.ground_state(betas[i], gams[i], tau=tau, eps0=eps0, psi0=p0, max_iter=20000, check_every=1)
        out.append(st[0]["iters"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--coarse", type=int, default=32)
    ap.add_argument("--target-n", type=int, default=0,
                    help="grid the training targets are solved on (default: --n), restricted to --coarse")
    ap.add_argument("--L", type=float, default=8.0)
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--tau", type=float, default=0.5)
    ap.add_argument("--split", action="store_true",
                    help="held-out solves with the split evaluation of the 3D potential (Eq. '3.9')")
    args = ap.parse_args()
    import torch
    kernel = nlf.COULOMB3D if args.dim == 3 else nlf.COULOMB2D
    mk = inputs.warmstart_instances_3d if args.dim == 3 else None
    tr = mk(0, args.train)
    te = mk(1, args.test)
    t0 = time.perf_counter()
    tn = args.target_n or args.n
    split = bool(args.split and args.dim == 3)
    T = solve_targets(tr, tn, args.coarse, args.L, kernel, args.dim, split=split, progress=True)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    print(f"targets: {len(tr)} solves in {t_data:.1f} s", file=sys.stderr, flush=True)
    X = torch.tensor(features([d["beta"] for d in tr], [d["gamma"] for d in tr]), device="cuda")
    t0 = time.perf_counter()
    model, hist = train_model(X, T, hidden=args.hidden, epochs=args.epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"trained: loss {hist[0]:.3e} -> {hist[-1]:.3e} in {t_train:.1f} s", file=sys.stderr, flush=True)
    # held-out prediction error on the coarse grid
    Tt = solve_targets(te, tn, args.coarse, args.L, kernel, args.dim, split=split)
    Xt = torch.tensor(features([d["beta"] for d in te], [d["gamma"] for d in te]), device="cuda")
    Yt = model.forward(Xt)
    rel = ((Yt - Tt).abs().amax(1) / Tt.abs().amax(1)).cpu().numpy()
    res = {"dim": args.dim, "n": args.n, "coarse": args.coarse, "target_n": tn, "train": args.train, "test": args.test,
           "split": split,
           "hidden": args.hidden, "epochs": args.epochs, "seconds_data": t_data, "seconds_train": t_train,
           "final_train_loss": float(hist[-1]), "heldout_coarse_rel_err_median": float(np.median(rel)),
           "heldout_coarse_rel_err_max": float(rel.max())}
    chunk = 50
    agg = {}
    for s in range(0, len(te), chunk):
        print(f"compare {s}/{len(te)}", file=sys.stderr, flush=True)
        r = compare(model, te[s:s + chunk], args.n, args.L, kernel, args.dim, args.coarse, tau=args.tau,
                    split=args.split and args.dim == 3)
        for k, v in r.items():
            agg.setdefault(k, []).append(v)
    res.update({"compare_chunks": agg})
    tg = sum(agg["seconds_gauss"])
    tw = sum(agg["seconds_learned"])
    res.update({"solves_per_s_gauss": len(te) / tg, "solves_per_s_learned": len(te) / tw,
                "mean_batch_iters_gauss": float(np.mean(agg["iters_gauss_batch"])),
                "mean_batch_iters_learned": float(np.mean(agg["iters_learned_batch"])),
                "mean_field_iters_gauss": float(np.mean(agg["iters_gauss_mean"])),
                "mean_field_iters_learned": float(np.mean(agg["iters_learned_mean"]))})
    print(json.dumps(res))


if __name__ == "__main__":
    main()
