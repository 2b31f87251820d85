"""Learned warm start for PCPM PageRank: training and evaluation driver.

The network (include/pcpm.h, "learned warm start") maps the per-node graph
features of pcpm_ws_features to a prediction of log(n * PR*(v)); the start
vector is its softmax over the nodes.  Training targets are PageRank vectors
the library itself computes (pcpm_pagerank to a tight tolerance), and all
arithmetic -- features, forward, backward, Adam -- runs in the library's
kernels.  Python only draws the graphs and the random minibatch indices.

Plain uniform initialisation stays both the fallback (non-finite
prediction) and the reference the warm start is measured against; every
warm solve is still certified by the FP64 residual of pcpm_pagerank.

Command line:
  python -m paper_1709_07122_amd.warmstart train --graphs 200 --out weights.npy
  python -m paper_1709_07122_amd.warmstart eval --weights weights.npy --scale 24
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import dataclass

import numpy as np

from . import _pcpm as P

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "ws_mlp_rmat.npy")


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation; the columns of W1 that see the four padding
    features stay 0."""
    rng = np.random.default_rng(seed)
    F, H = P.WS_FEATURES, P.WS_HIDDEN
    W1 = rng.normal(0, np.sqrt(2.0 / 4), (H, F))
    W1[:, 4:] = 0.0
    W2 = rng.normal(0, np.sqrt(2.0 / H), (H, H))
    w3 = rng.normal(0, np.sqrt(1.0 / H), H)
    p = np.concatenate([W1.reshape(-1), np.zeros(H), W2.reshape(-1), np.zeros(H), w3, np.zeros(1)])
    assert p.size == P.WS_PARAMS
    return p.astype(np.float32)


def save(params, path):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    arr = params.detach().cpu().numpy() if hasattr(params, "detach") else np.asarray(params)
    np.save(path, arr.astype(np.float32), allow_pickle=False)


def load(path, device="cuda"):
    import torch

    arr = np.load(path, allow_pickle=False).astype(np.float32)
    if arr.size != P.WS_PARAMS:
        raise ValueError(f"{path}: expected {P.WS_PARAMS} parameters, got {arr.size}")
    return torch.from_numpy(arr).to(device)


@dataclass
class GraphSpec:
    scale: int
    edge_factor: float
    a: float
    seed: int

    def generate(self):
        import graphgen

        rest = 1.0 - self.a
        b = c = rest * 0.19 / 0.43  # keep b:c:d = .19:.19:.05 (reading of the training recipe)
        return graphgen.rmat(self.scale, self.edge_factor, self.a, b, c, seed=self.seed, relabel="random")


def training_specs(count: int = 200, scales=(18, 22), seed0: int = 1000):
    """Training graphs: RMAT scale uniform in [18, 22], a uniform in
    [0.45, 0.65], edge factor 16, seeds seed0 .. seed0+count-1."""
    rng = np.random.default_rng(seed0)
    return [GraphSpec(int(rng.integers(scales[0], scales[1] + 1)), 16, float(rng.uniform(0.45, 0.65)), seed0 + i)
            for i in range(count)]


def prepare(spec: GraphSpec, d=0.85, tol=1e-7, part_log2=14, keep=0, rng=None):
    """Features and targets of one graph (device tensors), subsampled to at
    most `keep` nodes when keep > 0."""
    import torch

    r, c = spec.generate()
    png = P.build_png(torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda(), part_log2=part_log2)
    feat, _ = P.ws_features(png, d)
    res = P.pagerank(png, d=d, tol=tol, max_iters=500, want_hist=False)
    y = P.ws_targets(res.pr)
    n = png.n
    png.close()
    if keep and n > keep:
        sel = torch.from_numpy(np.sort((rng or np.random.default_rng(spec.seed)).choice(n, keep, replace=False))).cuda()
        feat, y = feat.index_select(0, sel), y.index_select(0, sel)
    return feat.contiguous(), y.contiguous()


def train(specs, epochs: int = 30, batch: int = 16384, lr: float = 3e-3, seed: int = 0, d: float = 0.85,
          keep: int = 0, log=print):
    """Adam on the MSE between prediction and log(n * PR*) over all graphs'
    sampled nodes.  Returns (params tensor, history)."""
    import torch

    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    feats, ys = [], []
    for i, s in enumerate(specs):
        f, y = prepare(s, d=d, keep=keep, rng=rng)
        feats.append(f)
        ys.append(y)
        if log and (i + 1) % max(1, len(specs) // 10) == 0:
            log(f"  prepared {i + 1}/{len(specs)} graphs ({time.perf_counter() - t0:.1f} s)")
    feat = torch.cat(feats).contiguous()
    target = torch.cat(ys).contiguous()
    del feats, ys
    N = feat.shape[0]
    params = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    work = torch.empty(int(P.lib().pcpm_ws_work_floats(batch)), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    step = 0
    hist = []
    t1 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(N, device="cuda", generator=gen)
        tot = 0.0
        nb = 0
        for b0 in range(0, N, batch):
            idx = perm[b0:b0 + batch].contiguous()
            _, loss = P.ws_backward(params, feat, target, idx, grad=grad, work=work)
            step += 1
            lr_t = lr * (0.1 ** (ep / max(1, epochs - 1)))  # decays to lr/10
            P.ws_adam(params, grad, m, v, step, lr_t)
            tot += loss
            nb += 1
        hist.append(tot / nb)
        if log:
            log(f"  epoch {ep + 1}/{epochs}: mse {tot / nb:.5f} ({time.perf_counter() - t1:.1f} s)")
    info = {"samples": N, "graphs": len(specs), "prepare_s": t1 - t0, "train_s": time.perf_counter() - t1,
            "final_mse": hist[-1] if hist else None}
    return params, hist, info


def warm_start(png, params, d: float = 0.85):
    """Start vector predicted for this handle: (pr0, used_uniform)."""
    yhat, _ = P.ws_predict(png, params, d)
    return P.ws_init(yhat)


def compare(png, params, d: float = 0.85, tol: float = 1e-6, reps: int = 3):
    """Iterations and time to tol from the uniform start and from the learned
    start.  The warm time covers the prediction (one PCPM iteration for the
    first iterate, then the MLP with the features formed in its kernel), the
    normalisation and the solve; the in-degree count, done once per handle,
    is reported apart and added in warm_ms_first."""
    import torch

    out = torch.empty(png.n, dtype=torch.float32, device="cuda")
    yhat, count_ms = P.ws_predict(png, params, d)

    def cold():
        return P.pagerank(png, d=d, tol=tol, max_iters=500, out=out, want_hist=False)

    def warm():
        P.ws_predict(png, params, d, out=yhat)
        pr0, fb = P.ws_init(yhat)
        return P.pagerank(png, d=d, tol=tol, max_iters=500, init=pr0, out=out, want_hist=False), fb

    cold()
    warm()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        rc = cold()
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t) / reps * 1e3
    t = time.perf_counter()
    for _ in range(reps):
        rw, fb = warm()
    torch.cuda.synchronize()
    warm_ms = (time.perf_counter() - t) / reps * 1e3
    # per-kernel times of one more warm solve (events around every launch):
    # pcpm_ws_predict is the network's forward, pcpm_ws_init the softmax
    P.timing_enable(True)
    warm()
    torch.cuda.synchronize()
    P.timing_enable(False)
    kernels = {name: {"launches": v[0], "total_ms": v[1]} for name, v in P.timing_collect().items()}
    # the network's forward alone, on the feature matrix (pcpm_ws_forward)
    feat, _ = P.ws_features(png, d)
    P.ws_forward(params, feat)
    torch.cuda.synchronize()
    P.timing_enable(True)
    P.ws_forward(params, feat)
    torch.cuda.synchronize()
    P.timing_enable(False)
    fwd = P.timing_collect().get("pcpm_ws_forward")
    kernels["pcpm_ws_forward_on_features"] = {"launches": fwd[0], "total_ms": fwd[1]} if fwd else None
    del feat
    return {"cold_iters": rc.iters, "warm_iters": rw.iters, "cold_ms": cold_ms, "warm_ms": warm_ms,
            "warm_ms_first": warm_ms + count_ms, "indeg_count_ms": count_ms, "cold_resid": rc.resid,
            "warm_resid": rw.resid, "fallback": fb, "warm_kernels": kernels}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--graphs", type=int, default=200)
    t.add_argument("--scale-min", type=int, default=18)
    t.add_argument("--scale-max", type=int, default=22)
    t.add_argument("--epochs", type=int, default=30)
    t.add_argument("--batch", type=int, default=16384)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--keep", type=int, default=0, help="nodes sampled per graph (0: all)")
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--scale", type=int, default=24)
    e.add_argument("--seeds", type=int, nargs="+", default=[2000, 2001, 2002, 2003])
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch

    if args.cmd == "train":
        specs = training_specs(args.graphs, (args.scale_min, args.scale_max))
        params, hist, info = train(specs, epochs=args.epochs, batch=args.batch, lr=args.lr, keep=args.keep,
                                   log=lambda s: print(s, file=sys.stderr, flush=True))
        save(params, args.out)
        print(json.dumps({"weights": args.out, **info}))
    else:
        params = load(args.weights)
        import graphgen

        rows = []
        for sd in args.seeds:
            r, c = graphgen.rmat(args.scale, 16, seed=sd, relabel="random")
            png = P.build_png(torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda())
            rows.append({"seed": sd, **compare(png, params)})
            png.close()
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        print(json.dumps(rows))


if __name__ == "__main__":
    main()
