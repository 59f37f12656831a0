"""Learned warm start for RQI-PCGTLS (a project addition, not in the paper).

A small network (32 -> 3 x 256 GELU -> 1) predicts the relative gap
y = ln(1 - sigma_{n+1}^2 / sigma_0^2) from 32 cheap features of (A, b) that the solver computes next to
the initial step of Algorithm 2 (see tls_rqi_solve in include/tls.h). The
solver turns the prediction into a shift estimate and a warm candidate for
x_1, and keeps whichever of the warm and the plain x_1 has the smaller psi.

Everything here runs through the library: labels come from plain solves
(the method without the network), the network is trained by the library's
forward/backward/Adam kernels, and the evaluation compares plain and warm
solves of held-out problems, each judged against the plain solve's answer.

    python -m paper_2305_19028_amd.warmstart --train 2000 --test 256

At the configured scale (20000 training problems, 512 held out, m up to
50000 and n up to 5000) the problems are drawn on the device and the
training set is made in parts:

    python -m paper_2305_19028_amd.warmstart --device-gen --train 10000 --save-data part0.npz
    python -m paper_2305_19028_amd.warmstart --device-gen --train 10000 --seed0 10000 --save-data part1.npz
    python -m paper_2305_19028_amd.warmstart --device-gen --load-data part0.npz part1.npz --test 512
"""
from __future__ import annotations

import argparse
import json
import math
import statistics
import sys
import time

import numpy as np

from . import tls

PATHS = {"fp64": dict(u_q="fp64", u_p="fp64"), "mixed": dict(u_q="fp16", u_p="fp32")}


def _torch():
    import torch
    return torch


def _problem(seed, m_range, n_range, device_gen=False):
    """A problem from the host generator, or (device_gen) drawn on the
    device from the same recipe (tlsgen.device): the only practical way to
    make tens of thousands of problems up to 50000 x 5000."""
    if device_gen:
        from tlsgen import device
        return device.warmstart_problem(seed, m_range=m_range, n_range=n_range)
    import tlsgen
    return tlsgen.warmstart_problem(seed, m_range=m_range, n_range=n_range)


def _device_problem(p):
    if "At" in p:
        return tls.dense_t(p["At"]), p["b"]
    if "row_ptr" in p:
        return tls.csr(p["row_ptr"], p["col_idx"], p["val"], p["m"], p["n"]), p["b"]
    if p["kind"] == "dense":
        A = tls.dense(np.asfortranarray(p["A"]))
    else:
        A = tls.from_tlsgen(p["A"])
    return A, tls.device_vector(p["b"])


def solve(A, b, path="fp64", mlp=None, features=False, snapshots=None, kmax=40, patience=2):
    """One factor + solve; returns (x numpy, sigma, stats, factor ms, solve ms)."""
    torch = _torch()
    cfg = PATHS[path]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, _ = tls.tls_factor_precond(A, cfg["u_q"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kw = dict(u_p=cfg["u_p"], stop_patience=patience, kmax=kmax, x_snapshots=snapshots,
              features=1 if features else 0)
    if mlp is not None:
        kw["mlp"] = mlp
    x, sigma, st = tls.tls_rqi_solve(A, b, P, tls.default_opts(**kw))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return x.cpu().numpy(), sigma, st, (t1 - t0) * 1e3, (t2 - t1) * 1e3


GAP_FLOOR = 1e-13   # relative gaps below this are indistinguishable from rounding
CLIP = 1.0          # bound of the learned correction of the log gap


def label(sigma, sigma0):
    """y = ln(1 - sigma^2 / sigma_0^2), floored at ln(GAP_FLOOR)."""
    return math.log(max(1.0 - (sigma / sigma0) ** 2, GAP_FLOOR))


def base(F):
    """The quadrature estimate of the log gap (feature 31, floored at
    ln GAP_FLOOR by the solver); the network learns the correction to it."""
    return np.asarray(F, dtype=np.float64)[:, 31]


def make_dataset(seeds, m_range=(5000, 50000), n_range=(500, 5000), path="fp64", log=None,
                 device_gen=False):
    """Features and labels y = ln(1 - sigma_final^2 / sigma_0^2) from plain solves."""
    F, y = [], []
    for i, s in enumerate(seeds):
        p = _problem(s, m_range, n_range, device_gen)
        A, b = _device_problem(p)
        _, sigma, st, _, _ = solve(A, b, path, features=True)
        F.append(np.array(st["features"], dtype=np.float32))
        y.append(label(sigma, st["sigma_ls"]))
        if log and (i + 1) % 64 == 0:
            print(f"# dataset {i + 1}/{len(seeds)}", file=log, flush=True)
    return np.stack(F), np.array(y, dtype=np.float32)


def fit_norm(F):
    """Standardisation [mean, 1/std] (std floored so that constant features stay finite)."""
    mu = F.mean(axis=0)
    sd = F.std(axis=0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    return np.concatenate([mu, 1.0 / sd]).astype(np.float32)


def train(F, y, norm, epochs=200, batch=256, lr=1e-3, seed=7, log=None):
    """Adam on the mean squared error of the correction y - base(F), with
    the library's kernels; returns (theta device tensor, per-epoch mean loss)."""
    import tlsgen
    torch = _torch()
    theta = torch.as_tensor(tlsgen.mlp_init(seed)).cuda()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    Fd = torch.as_tensor(F).cuda()
    # the correction target, clipped to a factor e^{+-1}: beyond that the
    # label is rounding noise of a gap near the floor, not signal
    r = np.clip(np.asarray(y, dtype=np.float64) - base(F), -CLIP, CLIP)
    yd = torch.as_tensor(r.astype(np.float32)).cuda()
    nd = torch.as_tensor(norm).cuda()
    g = np.random.default_rng(seed)
    N = F.shape[0]
    step = 0
    hist = []
    ws = None
    for ep in range(epochs):
        perm = torch.as_tensor(g.permutation(N)).cuda()
        losses = []
        for s in range(0, N, batch):
            idx = perm[s:s + batch]
            if idx.numel() < 2:
                continue
            Xb = Fd[idx].contiguous()
            tb = yd[idx].contiguous()
            if ws is None or ws.nbytes < tls.lib().tls_mlp_workspace_size(Xb.shape[0]):
                ws = tls.Workspace(tls.lib().tls_mlp_workspace_size(max(batch, Xb.shape[0])))
            loss, _ = tls.tls_mlp_loss_grad(theta, nd, Xb, tb, grad_out=grad, ws=ws)
            step += 1
            tls.tls_mlp_adam(theta, m, v, grad, step, lr)
            losses.append(loss)
        hist.append(float(torch.stack(losses).mean()))
        if log and (ep + 1) % 50 == 0:
            print(f"# epoch {ep + 1}: loss {hist[-1]:.4g}", file=log, flush=True)
    return theta, hist


def shrink_to_validation(theta, norm, F, y):
    """Scale the network's output layer by the alpha in [0, 1] that minimises
    the squared error of base + alpha * net on a validation set (targets
    clipped as in training). alpha = 0 leaves the quadrature estimate alone:
    the correction is only kept to the extent that it helps on problems the
    network was not trained on. Returns alpha; theta is scaled in place."""
    torch = _torch()
    r = tls.tls_mlp_forward(theta, torch.as_tensor(norm).cuda(), F).cpu().numpy().astype(np.float64)
    t = np.clip(np.asarray(y, dtype=np.float64) - base(F), -CLIP, CLIP)
    rr = float(r @ r)
    alpha = 0.0 if rr == 0.0 else float(np.clip((r @ t) / rr, 0.0, 1.0))
    # the output layer: the last TLS_MLP_WIDTH weights and the bias
    theta[-(tls.MLP_WIDTH + 1):] *= alpha
    return alpha


def predict(theta, norm, F):
    """y_hat = base(F) + net(F), as the solver forms it."""
    torch = _torch()
    r = tls.tls_mlp_forward(theta, torch.as_tensor(norm).cuda(), F).cpu().numpy()
    return base(F) + r.astype(np.float64)


def _first_crossing(snaps, iters, xref, tol):
    for k in range(iters):
        if np.linalg.norm(snaps[k] - xref) <= tol * np.linalg.norm(xref):
            return k + 1
    return None


def evaluate(theta, norm, seeds, m_range=(5000, 50000), n_range=(500, 5000), path="mixed",
             tol=1e-10, log=None, device_gen=False):
    """Plain vs warm solves of held-out problems. The plain FP64 solve's answer
    judges both; returns a list of per-problem records."""
    torch = _torch()
    nd = torch.as_tensor(norm).cuda()
    out = []
    for i, s in enumerate(seeds):
        p = _problem(s, m_range, n_range, device_gen)
        A, b = _device_problem(p)
        xref, sref, _, _, _ = solve(A, b, "fp64")
        rec = {"seed": s, "kind": p["kind"], "m": p["m"], "n": p["n"]}
        for name, mlp in (("plain", None), ("warm", (theta, nd))):
            snaps = torch.zeros((40, A.n), dtype=torch.float64, device="cuda")
            x, sigma, st, tf, ts = solve(A, b, path, mlp=mlp, snapshots=snaps)
            kx = _first_crossing(snaps.cpu().numpy(), st["iters"], xref, tol)
            rec[name] = {
                "iters": st["iters"], "k_best": st["k_best"], "k_tol": kx,
                "ms": tf + ts, "ms_to_tol": (tf + st["t_ms"][kx - 1]) if kx else None,
                "err_sigma": abs(sigma - sref) / sref,
                "err_x": float(np.linalg.norm(x - xref) / np.linalg.norm(xref)),
                "warm_used": st["warm_used"], "sigma_hat": st["sigma_hat"],
                "sigma_ls": st["sigma_ls"], "psi_warm": st["psi_warm"], "psi_plain": st["psi_plain"],
            }
        rec["y_true"] = label(sref, rec["plain"]["sigma_ls"])
        out.append(rec)
        if log and (i + 1) % 32 == 0:
            print(f"# evaluated {i + 1}/{len(seeds)}", file=log, flush=True)
    return out


def summarize(recs):
    def mean(key, name):
        v = [r[name][key] for r in recs if r[name][key] is not None]
        return statistics.mean(v) if v else None
    s = {"problems": len(recs)}
    for name in ("plain", "warm"):
        s[name] = {"mean_k_tol": mean("k_tol", name), "mean_iters": mean("iters", name),
                   "mean_ms": mean("ms", name), "mean_ms_to_tol": mean("ms_to_tol", name),
                   "reached_tol": sum(r[name]["k_tol"] is not None for r in recs),
                   "max_err_sigma": max(r[name]["err_sigma"] for r in recs)}
    s["warm_used"] = sum(r["warm"]["warm_used"] for r in recs)
    return s


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--m", type=int, nargs=2, default=(5000, 50000))
    ap.add_argument("--n", type=int, nargs=2, default=(500, 5000))
    ap.add_argument("--path", default="mixed", choices=sorted(PATHS))
    ap.add_argument("--out", default=None)
    ap.add_argument("--device-gen", action="store_true",
                    help="draw the problems on the device (tlsgen.device)")
    ap.add_argument("--seed0", type=int, default=0, help="first training seed")
    ap.add_argument("--save-data", default=None, help="write the training set (npz) and stop")
    ap.add_argument("--load-data", nargs="*", default=None, help="training sets (npz) instead of solving")
    a = ap.parse_args(argv)
    log = sys.stderr
    train_seeds = list(range(a.seed0, a.seed0 + a.train))
    test_seeds = list(range(10 ** 6, 10 ** 6 + a.test))
    t0 = time.perf_counter()
    if a.load_data:
        parts = [np.load(f) for f in a.load_data]
        F = np.concatenate([q["F"] for q in parts])
        y = np.concatenate([q["y"] for q in parts])
        a.train = int(F.shape[0])
    else:
        F, y = make_dataset(train_seeds, tuple(a.m), tuple(a.n), a.path, log=log, device_gen=a.device_gen)
    if a.save_data:
        np.savez(a.save_data, F=F, y=y, seeds=np.array(train_seeds))
        print(json.dumps({"saved": a.save_data, "problems": int(F.shape[0]),
                          "seconds": time.perf_counter() - t0}))
        return
    t1 = time.perf_counter()
    norm = fit_norm(F)
    nv = max(1, int(F.shape[0]) // 5)       # a fifth held back for the shrinkage
    theta, hist = train(F[nv:], y[nv:], norm, epochs=a.epochs, log=log)
    alpha = shrink_to_validation(theta, norm, F[:nv], y[:nv])
    _torch().cuda.synchronize()
    t2 = time.perf_counter()
    recs = evaluate(theta, norm, test_seeds, tuple(a.m), tuple(a.n), a.path, log=log,
                    device_gen=a.device_gen)
    yt = np.array([r["y_true"] for r in recs])
    s = summarize(recs)
    s.update({"train": a.train, "epochs": a.epochs, "path": a.path, "m_range": a.m, "n_range": a.n,
              "device_gen": a.device_gen,
              "final_train_loss": hist[-1], "alpha": alpha, "dataset_s": t1 - t0, "train_s": t2 - t1,
              "y_test_mean": float(yt.mean()), "y_test_var": float(yt.var())})
    print(json.dumps(s))
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"summary": s, "records": recs}, f)


if __name__ == "__main__":
    main()
