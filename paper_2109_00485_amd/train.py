"""Training of the learned preconditioner on the GPU.

Pipeline (every numerical step runs in the library's kernels; this module
only orders the calls and moves device buffers between them):
  1. for each training matrix: a tight FP64 LOBPCG pass gives converged
     eigenvectors x*; a plain diagonal-preconditioned pass of the same matrix
     harvests (feature, diagonal step, exact correction, weight, X row)
     samples every `every` iterations (lobpcg_info.harvest);
  2. the standardiser (feature mean / std) is fitted on the harvested set;
  3. full-batch Adam on the group loss, step size decayed geometrically;
  4. evaluation: the same solve with the diagonal and with the learned
     preconditioner, compared by iterations, wall-clock and final residual.

The network scales the diagonal step 1/s(d_i - sigma_j); sigma_j = theta_j -
offset * (Ritz-value spread) (offset 0: the Ritz value itself).  A network is
trained for one offset, recorded with its weights, and must be used with the
same offset (Context.set_precond_offset).

Command line (synthetic matrices of a named workload, weights written as
JSON):  python -m paper_2109_00485_amd.train --workload random_sym_2m \
            --train-seeds 0:16 --eval-seeds 1000:1020 --out weights.json

A harvest too large for one process can be split: ``--shard-out FILE``
harvests the given training seeds and writes their samples to a compressed
file (features in FP32; the diagonal step, correction, weight and X row
rounded to BF16, which keeps FP32's range), and ``--shards A,B,...`` trains
on such files instead of harvesting.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import (F32, F64, MLP_HID, PRECOND_DIAG, PRECOND_MLP, Context, HarvestBuffer, Mlp, pack_params,
               unpack_params)


def init_params(seed: int, mu=None, sigma=None) -> np.ndarray:
    """He-normal hidden layers and a zero output layer: the untrained network is
    exactly the diagonal preconditioner."""
    rng = np.random.default_rng(seed)
    p = dict(W1=rng.standard_normal((MLP_HID, 4)) * np.sqrt(2.0 / 4), b1=np.zeros(MLP_HID),
             W2=rng.standard_normal((MLP_HID, MLP_HID)) * np.sqrt(2.0 / MLP_HID), b2=np.zeros(MLP_HID),
             w3=np.zeros(MLP_HID), b3=0.0,
             mu=np.zeros(4) if mu is None else np.asarray(mu), sigma=np.ones(4) if sigma is None else np.asarray(sigma))
    return pack_params(p)


def save_params(path: str, blob: np.ndarray, meta: dict):
    p = unpack_params(blob)
    out = {k: (np.asarray(v).tolist() if not isinstance(v, float) else v) for k, v in p.items()}
    out["meta"] = meta
    with open(path, "w") as fh:
        json.dump(out, fh)


def load_params(path: str) -> tuple[np.ndarray, dict]:
    with open(path) as fh:
        d = json.load(fh)
    meta = d.pop("meta", {})
    return pack_params({k: np.asarray(v, dtype=np.float64) if isinstance(v, list) else v for k, v in d.items()}), meta


def _log(msg):
    print(f"[train] {msg}", file=sys.stderr, flush=True)


def harvest_matrix(A, hb: HarvestBuffer, *, k=8, nev=5, every=10, rows=256, seed=0, tol_star=1e-9, tol=1e-6,
                   maxiter=5000, x0_seed=1, offset=0.0, star_offset=4.0):
    """Append one matrix's samples to hb (FP64 context for both passes).  The
    converged eigenvectors x* do not depend on the preconditioner that found
    them, so the tight pass uses the faster shift (``star_offset``); the
    harvesting pass uses the diagonal step the network is trained on
    (``offset``)."""
    import torch
    from synth import workloads as W
    ctx = Context.from_csr(A, dtype=F64)
    ctx.set_precond_offset(star_offset)
    X0 = torch.from_numpy(W.initial_block(A.n, k, seed=x0_seed)).cuda()
    Xs = X0.clone()
    r_star = ctx.solve(Xs, nev, tol=tol_star, maxiter=maxiter)
    ctx.set_precond_offset(offset)
    xstar = Xs[:, :nev].contiguous()
    hb.set_xstar(xstar, nev=nev, seed=seed)
    hb.h.every, hb.h.rows = every, rows
    g0 = hb.ngroups
    r = ctx.solve(X0.clone(), nev, tol=tol, maxiter=maxiter, harvest=hb)
    torch.cuda.synchronize()
    ctx.close()
    return dict(star_iters=r_star.iters, star_status=r_star.status, iters=r.iters, status=r.status,
                groups=hb.ngroups - g0)


def fit(net: Mlp, batch, steps=1500, lr=3e-3, lr_end=3e-4, log_every=100):
    losses = []
    for s in range(steps):
        lr_s = lr * (lr_end / lr) ** (s / max(steps - 1, 1))
        losses.append(net.train_step(batch, lr_s))
        if log_every and s % log_every == 0:
            _log(f"step {s:5d} loss {losses[-1]:.6f} lr {lr_s:.2e}")
    return losses


def compare(A, net: Mlp, *, k=8, nev=5, tol=1e-6, maxiter=5000, x0_seed=1, f32=True, offset=0.0,
            also_offset=None):
    """Diagonal vs learned preconditioner on one matrix: iterations, seconds, final
    residuals.  "diag" is the diagonal step the network was trained on (shift
    offset ``offset``); with offset > 0, "diag_theta" is the shift at theta_j;
    ``also_offset`` adds "diag_offset", the diagonal step with that offset."""
    import torch
    from synth import workloads as W
    ctx = Context.from_csr(A, dtype=F32 if f32 else F64)
    ctx.set_mlp(net)
    dt = np.float32 if f32 else np.float64
    X0 = torch.from_numpy(W.initial_block(A.n, k, seed=x0_seed, dtype=dt)).cuda()
    out = {}
    runs = [("diag", PRECOND_DIAG, offset), ("mlp", PRECOND_MLP, offset)]
    if offset > 0:
        runs.append(("diag_theta", PRECOND_DIAG, 0.0))
    if also_offset is not None:
        runs.append(("diag_offset", PRECOND_DIAG, float(also_offset)))
    for name, pc, c in runs:
        ctx.set_precond_offset(c)
        X = X0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.solve(X, nev, tol=tol, maxiter=maxiter, precond=pc)
        torch.cuda.synchronize()
        out[name] = dict(iters=r.iters, seconds=time.perf_counter() - t0, status=r.status,
                         evals=[float(v) for v in r.evals[:nev]], rel=[float(v) for v in r.rel[:nev]],
                         n_spmm=r.n_spmm)
    ctx.set_mlp(None)
    ctx.close()
    return out


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns, round to nearest even (finite inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def _bf16_value(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32)


def save_shard(path: str, batch, meta: dict):
    feat, U, T, w, Xrow, goff = (t.cpu().numpy() for t in batch.t)
    np.savez_compressed(path, feat=feat.astype(np.float32), U=_bf16_bits(U), T=_bf16_bits(T), w=_bf16_bits(w),
                        Xrow=_bf16_bits(Xrow), group_off=goff.astype(np.int64),
                        meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_shards(paths):
    """Concatenate shard files into one device batch (group offsets rebased)."""
    import torch
    from . import Batch
    parts, metas, base = [], [], 0
    for p in paths:
        with np.load(p, allow_pickle=False) as z:
            goff = z["group_off"]
            parts.append((z["feat"], _bf16_value(z["U"]), _bf16_value(z["T"]), _bf16_value(z["w"]),
                          _bf16_value(z["Xrow"]).reshape(z["Xrow"].shape), goff[:-1] + base))
            base += int(goff[-1])
            metas.append(json.loads(bytes(z["meta"]).decode()))
    cat = [np.concatenate([q[i] for q in parts]) for i in range(6)]
    cat[5] = np.concatenate([cat[5], [base]]).astype(np.int64)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in cat]
    return Batch(*dev), metas


def _seeds(spec: str):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="random_sym_2m")
    ap.add_argument("--n", type=int, default=None, help="override the workload's n")
    ap.add_argument("--train-seeds", default="0:16")
    ap.add_argument("--eval-seeds", default="1000:1020")
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--nev", type=int, default=5)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--rows", type=int, default=256)
    ap.add_argument("--capacity", type=int, default=20_000_000)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lr-end", type=float, default=3e-4)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--offset", type=float, default=0.0,
                    help="diagonal preconditioner shift offset, in Ritz-value spreads below theta_j")
    ap.add_argument("--shard-out", default=None, help="harvest only: write the samples to this file")
    ap.add_argument("--shards", default=None, help="train on these sample files (comma-separated)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None, help="JSON report of the evaluation")
    args = ap.parse_args(argv)
    import torch
    from synth import workloads as W
    torch.cuda.set_device(0)
    t_start = time.time()
    runs = []
    if args.shards:
        batch, shard_meta = load_shards(args.shards.split(","))
        runs = [r for m in shard_meta for r in m.get("runs", [])]
        train_seeds = ",".join(m.get("train_seeds", "?") for m in shard_meta)
        # the harvest settings come from the shards
        args.every, args.rows = shard_meta[0].get("every", args.every), shard_meta[0].get("rows", args.rows)
        nsamples, ngroups = batch.t[0].shape[0], batch.t[5].shape[0] - 1
        _log(f"{len(shard_meta)} shards: {nsamples} samples, {ngroups} groups, {len(runs)} runs")
    else:
        dummy = torch.zeros((1, args.nev), dtype=torch.float64, device="cuda")
        hb = HarvestBuffer(args.capacity, args.capacity // 16, args.k, dummy, args.nev, every=args.every,
                           rows=args.rows)
        for seed in _seeds(args.train_seeds):
            t0 = time.time()
            A = W.make_matrix(args.workload, seed=seed, n=args.n, f32=False)
            info = harvest_matrix(A, hb, k=args.k, nev=args.nev, every=args.every, rows=args.rows, seed=seed,
                                  offset=args.offset)
            runs.append(dict(seed=seed, **info))
            _log(f"seed {seed}: {info} samples {hb.nsamples} ({time.time() - t0:.1f}s)")
            if hb.full:
                raise RuntimeError("harvest buffer full: raise --capacity or lower --rows")
        batch = hb.batch()
        train_seeds, nsamples, ngroups = args.train_seeds, hb.nsamples, hb.ngroups
        if args.shard_out:
            save_shard(args.shard_out, batch, dict(workload=args.workload, n=args.n, train_seeds=args.train_seeds,
                                                   offset=args.offset, every=args.every, rows=args.rows,
                                                   runs=runs))
            _log(f"wrote {nsamples} samples / {ngroups} groups to {args.shard_out} "
                 f"({time.time() - t_start:.0f}s)")
            return
    if not args.out:
        raise SystemExit("--out is required unless --shard-out is given")
    net = Mlp(init_params(args.init_seed))
    net.fit_standardizer(batch.t[0])
    torch.cuda.synchronize()
    t0 = time.time()
    losses = fit(net, batch, steps=args.steps, lr=args.lr, lr_end=args.lr_end)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    _log(f"trained {args.steps} steps on {nsamples} samples / {ngroups} groups in {t_train:.1f}s: "
         f"loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    meta = dict(workload=args.workload, n=args.n, train_seeds=train_seeds, offset=args.offset,
                every=args.every, rows=args.rows,
                steps=args.steps, lr=args.lr, lr_end=args.lr_end, samples=nsamples, groups=ngroups,
                loss_first=losses[0], loss_last=losses[-1], train_seconds=t_train)
    blob = net.params()
    save_params(args.out, blob, meta)
    evals = []
    for seed in _seeds(args.eval_seeds):
        A = W.make_matrix(args.workload, seed=seed, n=args.n, f32=True)
        res = compare(A, net, k=args.k, nev=args.nev, offset=args.offset)
        evals.append(dict(seed=seed, **res))
        extra = f" | diag at theta {res['diag_theta']['iters']} it" if "diag_theta" in res else ""
        _log(f"eval {seed}: diag {res['diag']['iters']} it {res['diag']['seconds']:.3f}s | "
             f"mlp {res['mlp']['iters']} it {res['mlp']['seconds']:.3f}s{extra}")
    report = dict(meta=meta, runs=runs, eval=evals, losses=losses[:: max(1, len(losses) // 100)],
                  total_seconds=time.time() - t_start)
    if evals:
        di = np.array([e["diag"]["iters"] for e in evals]); mi = np.array([e["mlp"]["iters"] for e in evals])
        ds = np.array([e["diag"]["seconds"] for e in evals]); ms = np.array([e["mlp"]["seconds"] for e in evals])
        report["summary"] = dict(offset=args.offset, diag_iters_mean=float(di.mean()), mlp_iters_mean=float(mi.mean()),
                                 diag_seconds_mean=float(ds.mean()), mlp_seconds_mean=float(ms.mean()),
                                 iters_ratio=float(mi.mean() / di.mean()), seconds_ratio=float(ms.mean() / ds.mean()))
        if all("diag_theta" in e for e in evals):
            report["summary"]["diag_theta_iters_mean"] = float(np.mean([e["diag_theta"]["iters"] for e in evals]))
            report["summary"]["diag_theta_seconds_mean"] = float(np.mean([e["diag_theta"]["seconds"] for e in evals]))
        _log(f"summary: {report['summary']}")
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    print(json.dumps(report.get("summary", {})), flush=True)


if __name__ == "__main__":
    main()
