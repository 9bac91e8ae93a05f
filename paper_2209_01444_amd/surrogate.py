"""Surrogate workflow: training data from batched lattice Boltzmann runs,
training of the U-Net with the library's own kernels, and the hybrid loop
that alternates network jumps of K main steps with lattice Boltzmann
segments, using the lattice Boltzmann solver as judge and fallback.

    python -m paper_2209_01444_amd.surrogate --size 512 --train-seeds 32

Hybrid loop (per cycle): checkpoint the solver on the device; read the
fields (phi, C, theta, ux, uy); jump: fields + network residual (or, for the
baseline without a network, the fields unchanged); restart the lattices at
the jumped fields, by default carrying over what the fields do not hold (the
flow lattice, the non-equilibrium parts, the time derivatives:
dlb_set_fields_ex with both continuation flags), or at equilibrium (p = 0,
phi first moment from the central-difference gradient); run L lattice
Boltzmann steps.  Judge:
the tip velocity implied by the jump, (s_after_jump - s_before)/K, must
agree within `tol` (2%) on every arm with the velocity expected from lattice
Boltzmann measurements: those of the plain window before the jump and of the
L-step window after it, interpolated linearly to the jump's mid-time (see
`judge`); otherwise the checkpoint is restored and K + L plain steps run
instead (fallback).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from paper_2209_01444_amd import dlb, workloads
from paper_2209_01444_amd import sur as sur_mod

FIELDS5 = ("phi", "C", "theta", "ux", "uy")

# A network trained by this module's command line at 512^2 (K = 100, 48
# training seeds, 100000 Adam steps; see save_bundle for the format)
BUNDLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet32_512_k100.npz")


def sweep_cases(count: int, size: int, seed: int):
    """Seeds drawn like the batched sweep, all at size x size."""
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        cfg, noise = workloads.thermosolutal_flow(
            size, size, seed=int(rng.integers(0, 2**31 - 1)), precision="f32",
            orient=float(rng.uniform(0.0, math.pi / 4)), u0=float(rng.uniform(0.0, 0.02)),
            delta=float(rng.uniform(0.3, 0.65)), eps4=float(rng.uniform(0.02, 0.05)))
        cfg["name"] = f"train_{i}"
        cases.append((cfg, noise))
    return cases


def make_dataset(cases, t0: int, K: int, pairs_per_seed: int):
    """Snapshots x(t0 + jK), j = 0..pairs_per_seed, of every member of one
    batch; returns device tensors X (inputs) and Y (K steps later)."""
    import torch

    b = dlb.Batch([c for c, _ in cases])
    for m, (_, noise) in zip(b.members, cases):
        m.init_seed(noise)
    b.step(t0)
    snaps = [[m.fields_device(FIELDS5) for m in b.members]]
    for _ in range(pairs_per_seed):
        b.step(K)
        snaps.append([m.fields_device(FIELDS5) for m in b.members])
    torch.cuda.synchronize()
    X = torch.stack([s for row in snaps[:-1] for s in row])
    Y = torch.stack([s for row in snaps[1:] for s in row])
    b.close()
    return X, Y


def normalization(X, Y):
    d = Y - X
    mean = X.mean(dim=(0, 2, 3)).cpu().numpy()
    std = X.std(dim=(0, 2, 3)).clamp_min(1e-6).cpu().numpy()
    rstd = d.std(dim=(0, 2, 3)).clamp_min(1e-9).cpu().numpy()
    return mean, std, rstd


def train(net, X, Y, iters: int, batch: int, lr: float, seed: int = 0, log_every: int = 100):
    import torch

    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    losses = []
    t0 = time.perf_counter()
    for it in range(iters):
        idx = torch.randint(0, n, (batch,), generator=g)
        xb = X[idx].contiguous()
        yb = Y[idx].contiguous()
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / iters))  # cosine decay
        loss = net.train_step(xb, yb, lr_t)
        losses.append(loss)
        if log_every and (it % log_every == 0 or it == iters - 1):
            print(json.dumps({"iter": it, "loss": loss, "lr": lr_t}), flush=True)
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def tips(solver) -> np.ndarray:
    return solver.reduce(allow_nonfinite=True)["tip_s"]


def run_plain(cfg, noise, T: int, every: int = 100):
    """Plain lattice Boltzmann to main step T; tip positions every `every`
    steps (reductions outside the timed span)."""
    import torch

    s = dlb.Solver(cfg).init_seed(noise)
    torch.cuda.synchronize()
    el, t, series = 0.0, 0, []
    while t < T:
        n = min(every, T - t)
        t0 = time.perf_counter()
        s.step(n)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        t += n
        series.append((t, tips(s)))
    a, b = series[-2][1], series[-1][1]
    return {"seconds": el, "tip_s": b, "tip_v": (b - a) / (series[-1][0] - series[-2][0]),
            "series": series, "solver": s}


def run_hybrid(cfg, noise, T: int, t_start: int, K: int, L: int, net=None, tol: float = 0.02,
               jump: str | None = None, restart: str = "continue"):
    """Hybrid time stepping to main step T (see module docstring).

    jump: "net" (the surrogate; default when `net` is given), "identity"
    (fields unchanged: the baseline without a network) or "lb" (the exact
    fields K lattice Boltzmann steps later, a diagnostic of the judge's floor:
    what re-initialisation and measurement cost).
    restart: "continue" (the flow lattice, the non-equilibrium parts and the
    time derivatives carry over the jump; the network's velocity output is
    not used) or "equilibrium" (every lattice restarts at equilibrium at the
    jumped fields, p = 0)."""
    import torch

    jump = jump or ("net" if net is not None else "identity")
    keep = restart == "continue"
    s = dlb.Solver(cfg).init_seed(noise)
    backup = dlb.Solver(cfg)
    H, W = cfg["ny"], cfg["nx"]
    out = torch.empty((1, 5, H, W), dtype=torch.float64, device=s.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(t_start - L)
    prev = (t_start - L, tips(s))  # start of the last plain LB window
    s.step(L)
    t = t_start
    accepted, fallbacks, errs, vj, vexp = 0, 0, [], [], []
    s_now = None  # tips of the current state when already measured
    while t + K + L + 100 <= T:
        backup.copy_from(s)
        s0 = tips(s) if s_now is None else s_now
        if jump == "lb":
            s.step(K)
        x = s.fields_device(FIELDS5)
        if jump == "net":
            net.forward(x[None].contiguous(), out)
        else:
            out.copy_(x[None].double())
        s.set_fields(out[0, 0], out[0, 1], out[0, 2], out[0, 3], out[0, 4], keep_flow=keep,
                     keep_noneq=keep)
        s1 = tips(s)
        s.step(L)
        s2 = tips(s)
        err, v_jump, v_exp = judge(prev, (t, s0), (t + K, s1), (t + K + L, s2))
        vj.append(v_jump.tolist())
        vexp.append(v_exp.tolist())
        errs.append(err)
        if err > tol:
            s.copy_from(backup)
            s.step(K)
            prev = (t + K, tips(s))
            s.step(L)
            s_now = None
            fallbacks += 1
        else:
            prev = (t + K, s1)
            s_now = s2  # the state after the L steps is the next cycle's start
            accepted += 1
        t += K + L
    s.step(T - 100 - t)
    a = tips(s)
    s.step(100)
    b = tips(s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"seconds": el, "tip_s": b, "tip_v": (b - a) / 100.0, "accepted": accepted,
            "fallbacks": fallbacks, "jump_errors": errs, "v_jump": vj, "v_expected": vexp, "solver": s}


def judge(before, start, after_jump, end):
    """Relative error of the tip velocity a jump implies.

    Each argument is (main step, tip positions of the 4 arms): `before` ..
    `start` is the last plain lattice Boltzmann window, `start` ..
    `after_jump` the jump, `after_jump` .. `end` the lattice Boltzmann window
    that follows it.  The expected jump velocity interpolates the two
    measured window velocities linearly to the jump's mid-time, so a tip that
    accelerates or decelerates steadily does not count as an error.
    Returns (worst relative error over the arms, jump velocity, expected)."""
    (tb, sb), (t0, s0), (t1, s1), (t2, s2) = before, start, after_jump, end
    v_b, v_j, v_a = (s0 - sb) / (t0 - tb), (s1 - s0) / (t1 - t0), (s2 - s1) / (t2 - t1)
    w = (0.5 * (t0 + t1) - 0.5 * (tb + t0)) / (0.5 * (t1 + t2) - 0.5 * (tb + t0))
    v_e = v_b + w * (v_a - v_b)
    with np.errstate(invalid="ignore", divide="ignore"):
        err = np.abs(v_j / v_e - 1)
    ok = np.all(np.isfinite(err)) and np.all(np.isfinite(v_j))
    return (float(err.max()) if ok else math.inf), v_j, v_e


def validation(net, X, Y):
    """Per-channel mean squared error of the normalised residual on (X, Y),
    evaluated with the library's forward pass one sample at a time."""
    import torch

    H, W = X.shape[2], X.shape[3]
    out = torch.empty((1, 5, H, W), dtype=torch.float64, device=X.device)
    rstd = torch.tensor(net.rstd, dtype=torch.float64, device=X.device)[:, None, None]
    acc = torch.zeros(5, dtype=torch.float64, device=X.device)
    base = torch.zeros(5, dtype=torch.float64, device=X.device)
    for i in range(X.shape[0]):
        net.forward(X[i:i + 1].contiguous(), out)
        d = (out[0] - Y[i].double()) / rstd
        r = (Y[i].double() - X[i].double()) / rstd
        acc += (d * d).mean(dim=(1, 2))
        base += (r * r).mean(dim=(1, 2))
    torch.cuda.synchronize()
    return (acc / X.shape[0]).tolist(), (base / X.shape[0]).tolist()


def compare(h, p):
    with np.errstate(invalid="ignore", divide="ignore"):
        return {"speedup": p["seconds"] / h["seconds"],
                "tip_v_rel_err": float(np.nanmax(np.abs(h["tip_v"] / p["tip_v"] - 1))),
                "tip_s_abs_err": float(np.nanmax(np.abs(h["tip_s"] - p["tip_s"]))),
                "accepted": h["accepted"], "fallbacks": h["fallbacks"]}


def conv_weight_mask() -> np.ndarray:
    """True at the entries of the flat parameter vector that hold 3x3
    convolution weights (which the forward pass uses in bfloat16)."""
    from paper_2209_01444_amd import sur as sm

    parts = []
    for _, _, cip, co in sm.layers():
        parts += [np.ones(9 * co * cip, dtype=bool), np.zeros(co, dtype=bool)]
    parts.append(np.zeros(165, dtype=bool))  # 1x1 head, FP32
    return np.concatenate(parts)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """FP32 -> bfloat16 bit patterns, rounded to nearest even (finite input)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def save_bundle(path: str, net, meta: dict) -> None:
    """Trained network as one .npz: the 3x3 weights as bfloat16 bit patterns
    (what the forward pass computes with, so nothing is lost for inference),
    biases and the 1x1 head in FP32, the input and residual normalisation,
    the loss weights and the training options (JSON text)."""
    flat = net.get_params()
    mask = conv_weight_mask()
    np.savez(path, w_bf16=to_bf16_bits(flat[mask]), rest=flat[~mask].astype(np.float32),
             mean=net.mean, std=net.std, rstd=net.rstd, loss_weights=np.asarray(net.loss_weights, np.float64),
             meta=np.array(json.dumps(meta)))


def load_bundle(path: str = BUNDLE, batch: int = 1):
    """The network of a save_bundle file on the GPU: (Surrogate, options)."""
    z = np.load(path)  # plain arrays only (no pickle)
    meta = json.loads(str(z["meta"]))
    mask = conv_weight_mask()
    flat = np.empty(mask.size, dtype=np.float32)
    flat[mask] = from_bf16_bits(z["w_bf16"])
    flat[~mask] = z["rest"]
    n = int(meta["size"])
    net = sur_mod.Surrogate(batch, n, n)
    net.set_params(flat)
    net.set_normalization(z["mean"], z["std"], z["rstd"])
    net.set_loss_weights(z["loss_weights"])
    return net, meta


def speedup_check(path: str = BUNDLE, T: int = 10000, L: int = 100, tol: float = 0.02) -> dict:
    """Time to main step T of the hybrid loop with a stored network against
    plain lattice Boltzmann, on the seed held out of its training, with the
    final tip-velocity error of every arm."""
    net, meta = load_bundle(path)
    cfg, noise = sweep_cases(int(meta["train_seeds"]) + 1, int(meta["size"]), int(meta["seed"]))[-1]
    run_plain(cfg, noise, 200)  # kernels loaded and launch paths warm before either timed run
    plain = run_plain(cfg, noise, T)
    hyb = run_hybrid(cfg, noise, T, int(meta["t0"]), int(meta["K"]), L, net, tol, restart=meta["restart"])
    r = compare(hyb, plain)
    r.update({"plain_seconds": plain["seconds"], "hybrid_seconds": hyb["seconds"],
              "jumps": hyb["accepted"] + hyb["fallbacks"], "size": int(meta["size"]), "K": int(meta["K"]),
              "L": L, "T": T, "tol": tol})
    net.close()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--train-seeds", type=int, default=32)
    ap.add_argument("--t0", type=int, default=500)
    ap.add_argument("--pairs", type=int, default=95)
    ap.add_argument("--K", type=int, default=100)
    ap.add_argument("--L", default="100", help="lattice Boltzmann steps after each jump; a comma list runs each")
    ap.add_argument("--iters", type=int, default=32000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=4e-4, help="peak of the cosine schedule (1e-3 diverged)")
    ap.add_argument("--T", type=int, default=10000)
    ap.add_argument("--tol", type=float, default=0.02)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--save", default="", help="write the trained network (.npz, see save_bundle) here")
    ap.add_argument("--load", default="", help="skip training: a network written by --save (its size, K, "
                    "seeds and restart replace the options given here)")
    ap.add_argument("--restart", default="continue", choices=("continue", "equilibrium"))
    ap.add_argument("--loss-weights", default="1,1,1,0,0",
                    help="per-channel loss weights (phi, C, theta, ux, uy); the continuation restart "
                         "keeps the flow lattice, so the velocity outputs are not used by default")
    args = ap.parse_args()
    import torch

    if args.load:
        net, meta = load_bundle(args.load, batch=args.batch)
        args.size, args.K, args.seed, args.train_seeds = meta["size"], meta["K"], meta["seed"], meta["train_seeds"]
        args.t0, args.restart, args.iters = meta["t0"], meta["restart"], meta["iters"]
        lw = np.asarray(net.loss_weights)
    n = args.size
    cases = sweep_cases(args.train_seeds + 1, n, args.seed)
    train_cases, test_case = cases[:-1], cases[-1]
    if args.load:
        X = make_dataset([test_case], args.t0, args.K, 1)[0]
        losses, t_train = [math.nan], 0.0
    else:
        t_gen = time.perf_counter()
        X, Y = make_dataset(train_cases, args.t0, args.K, args.pairs)
        t_gen = time.perf_counter() - t_gen
        mean, std, rstd = normalization(X, Y)
        print(json.dumps({"pairs": int(X.shape[0]), "gen_seconds": t_gen, "mean": mean.tolist(),
                          "std": std.tolist(), "rstd": rstd.tolist()}), flush=True)
        net = sur_mod.Surrogate(args.batch, n, n)
        net.set_params(sur_mod.flatten(init_params(args.seed)))
        net.set_normalization(mean, std, rstd)
        lw = np.array([float(v) for v in args.loss_weights.split(",")])
        net.set_loss_weights(lw)
        losses, t_train = train(net, X, Y, args.iters, args.batch, args.lr, seed=args.seed)
        del Y
    # forward timing at batch 1
    x1 = X[:1].contiguous()
    o1 = torch.empty((1, 5, n, n), dtype=torch.float64, device="cuda")
    net.forward(x1, o1)
    torch.cuda.synchronize()
    tf = time.perf_counter()
    for _ in range(20):
        net.forward(x1, o1)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - tf) / 20 * 1e3
    if args.save:
        save_bundle(args.save, net, {"size": n, "K": args.K, "t0": args.t0, "seed": args.seed,
                                     "train_seeds": args.train_seeds, "pairs": args.pairs, "iters": args.iters,
                                     "batch": args.batch, "lr": args.lr, "restart": args.restart})

    cfg, noise = test_case
    Xv, Yv = make_dataset([test_case], args.t0, args.K, (args.T - args.t0) // args.K - 1)
    val, val_identity = validation(net, Xv, Yv)
    del Xv, Yv
    print(json.dumps({"val_mse": val, "val_mse_identity": val_identity}), flush=True)
    plain = run_plain(cfg, noise, args.T)
    v_series = [(t1, ((b - a) / (t1 - t0)).round(6).tolist())
                for (t0, a), (t1, b) in zip(plain["series"][:-1], plain["series"][1:])]
    print(json.dumps({"plain_tip_v": v_series}), flush=True)
    Ls = [int(v) for v in str(args.L).split(",")]
    res = {
        "size": n, "train_pairs": int(X.shape[0]), "iters": args.iters, "train_seconds": t_train,
        "loss_weights": lw.tolist(),
        "loss_first": losses[0], "loss_last": float(np.mean(losses[-50:])), "forward_ms": fwd_ms,
        "forward_TFLOPs": 85.0e9 * (n / 512) ** 2 / (fwd_ms * 1e-3) / 1e12,
        "plain_seconds": plain["seconds"], "T": args.T, "K": args.K, "tol": args.tol, "restart": args.restart,
        "val_mse": val, "val_mse_identity": val_identity, "by_L": {},
    }
    for L in Ls:
        hyb = run_hybrid(cfg, noise, args.T, args.t0, args.K, L, net, args.tol, restart=args.restart)
        r = {"with_network": compare(hyb, plain),
             "jump_errors_with_network": [round(e, 4) if np.isfinite(e) else None for e in hyb["jump_errors"]]}
        if L == Ls[0]:
            base = run_hybrid(cfg, noise, args.T, args.t0, args.K, L, None, args.tol, restart=args.restart)
            exact = run_hybrid(cfg, noise, args.T, args.t0, args.K, L, None, args.tol, jump="lb",
                               restart=args.restart)
            r["without_network"] = compare(base, plain)
            r["with_exact_lb_jump"] = compare(exact, plain)
            r["jump_errors_exact_lb"] = [round(e, 4) if np.isfinite(e) else None for e in exact["jump_errors"]]
        res["by_L"][L] = r
        print(json.dumps({"L": L, **r}), flush=True)
    print(json.dumps(res), flush=True)


def init_params(seed: int) -> dict:
    """He-normal 3x3 weights, zero biases, small head (the residual starts near 0)."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, ci, cip, co in sur_mod.layers():
        P[name + ".W"] = rng.normal(size=(3, 3, co, ci)) * np.sqrt(2.0 / (9 * ci))
        P[name + ".b"] = np.zeros(co)
    P["head.W"] = rng.normal(size=(5, 32)) * 0.01
    P["head.b"] = np.zeros(5)
    return P


if __name__ == "__main__":
    main()
