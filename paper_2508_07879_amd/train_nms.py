"""Train neural min-sum weights and compare logical error rates with plain
min-sum at equal and larger iteration budgets.

Training data are (error, syndrome) pairs drawn from the same iid X-flip
noise the decoder is evaluated on, from a seed range disjoint from the
evaluation shots.  Loss: BCE between the true error bits and sigma(-Q),
averaged over all T iterations (see nms.bce_loss).  Optimiser: Adam.

    python -m paper_2508_07879_amd.train_nms --L 64 --p 0.05 --T 16 \
        --train-shots 1048576 --batch 4096 --epochs 4 --eval-shots 262144 \
        --out weights.pt --json results.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _batches(side, seed, shots, p, chunk):
    from workload import noise
    for lo in range(0, shots, chunk):
        yield noise.Batch(side, seed, np.arange(lo, min(shots, lo + chunk)), p)


def logical_fail_counts(lam_t, e_true_bits, err_words, conv, n):
    """Failures on the device: residual (e xor e_hat) against the logical
    basis as a 0/1 matrix product, parity = count mod 2."""
    import torch
    w = err_words.to(torch.int64) & 0xFFFFFFFF
    shifts = torch.arange(32, device=w.device, dtype=torch.int64)
    e_hat = ((w.unsqueeze(-1) >> shifts) & 1).reshape(w.shape[0], -1)[:, :n]
    rho = (e_hat ^ e_true_bits.to(torch.int64)).to(torch.float32)
    par = torch.remainder(rho @ lam_t, 2.0)
    flips = par.sum(dim=1) > 0
    return int((flips | (conv == 0)).sum().item())


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--p", type=float, default=0.05)
    ap.add_argument("--T", type=int, default=16)
    ap.add_argument("--train-shots", type=int, default=1 << 20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-shots", type=int, default=1 << 18)
    ap.add_argument("--train-seed", type=int, default=1_000_003)
    ap.add_argument("--eval-seed", type=int, default=2_000_003)
    ap.add_argument("--out", default="")
    ap.add_argument("--json", default="")
    ap.add_argument("--load", default="", help="evaluate these saved weights instead of training")
    args = ap.parse_args(argv)

    import torch

    from paper_2508_07879_amd import Decoder, nms
    from workload import lp

    dev = torch.device("cuda", 0)
    code = lp.lp_code(args.L)
    side = code.hz
    dec = Decoder(side)
    T = args.T
    report = dict(L=args.L, n=side.n, p=args.p, T=T, batch=args.batch, lr=args.lr, epochs=args.epochs,
                  train_shots=args.train_shots, eval_shots=args.eval_shots)

    if args.load:
        w, meta, _ = nms.load_weights(args.load, side)
        w = w.to(dev)
        T = int(w.shape[0])
        report.update(T=T, loaded=args.load, trained=meta)
        print(f"loaded weights [{T}][{side.nnz}] from {args.load}", flush=True)
    else:
        w = _train(args, dec, side, dev, report)
    return _evaluate(args, code, side, dec, dev, w, T, report)


def training_data(side, dev, seed, shots, p):
    """(syndromes, priors, error bits) of `shots` seeded training pairs,
    resident on the device."""
    import torch

    from workload import bits
    syn_all, pr_all, e_all = [], [], []
    for b in _batches(side, seed, shots, p, 65536):
        syn_all.append(torch.from_numpy(bits.pack_bits(b.s).view(np.int32)).to(dev))
        pr_all.append(torch.from_numpy(b.gamma).to(dev))
        e_all.append(torch.from_numpy(b.e).to(dev))
    return torch.cat(syn_all), torch.cat(pr_all), torch.cat(e_all)


def train(dec, side, dev, T, data, epochs, batch, lr, seed, log=print):
    """Adam on the BCE loss from all-alpha weights [T][nnz]; returns
    (weights, optimiser, mean loss per epoch)."""
    import torch

    from paper_2508_07879_amd import nms

    syn_all, pr_all, e_all = data
    shots = int(syn_all.shape[0])
    w = nms.init_weights(T, side.nnz, 0.75, device=dev).requires_grad_(True)
    opt = torch.optim.Adam([w], lr=lr)
    steps = shots // batch
    losses = []
    gen = torch.Generator(device="cpu").manual_seed(seed)
    for ep in range(epochs):
        perm = torch.randperm(shots, generator=gen).to(dev)
        ep_loss = torch.zeros((), device=dev)
        for s in range(steps):
            idx = perm[s * batch:(s + 1) * batch]
            post = nms.NeuralMinSum.apply(dec, w, syn_all[idx].contiguous(), pr_all[idx].contiguous())
            loss = nms.bce_loss(post, e_all[idx].to(torch.float32))
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            ep_loss += loss.detach()
        losses.append(float(ep_loss) / steps)
        if log:
            log(f"T={T} epoch {ep}: mean loss {losses[-1]:.6f}")
    torch.cuda.synchronize()
    return w, opt, losses


def _train(args, dec, side, dev, report):
    from paper_2508_07879_amd import nms

    T = args.T
    # ---- training data, resident on the device -----------------------------
    t0 = time.time()
    data = training_data(side, dev, args.train_seed, args.train_shots, args.p)
    report["train_data_s"] = time.time() - t0
    print(f"training data: {args.train_shots} shots in {report['train_data_s']:.1f} s", flush=True)
    t0 = time.time()
    w, opt, losses = train(dec, side, dev, T, data, args.epochs, args.batch, args.lr, args.train_seed,
                           log=lambda m: print(m, flush=True))
    report["train_s"] = time.time() - t0
    report["loss_per_epoch"] = losses
    if args.out:
        nms.save_weights(args.out, w, side, meta=report, optimizer=opt)
    del data
    return w


def evaluate(code, side, dec, dev, configs, eval_seed, eval_shots, p, log=print):
    """LER (Wilson 95 % CI), mean iterations, fallback rate and syndromes/s of
    each decoder configuration on the same held-out shots.  A configuration
    is (name, kind, T, fallback, weights): kind "nms" = neural min-sum for T
    iterations, then (fallback) plain min-sum from scratch for the shots that
    did not converge; "nmsc" = T neural iterations continued by plain
    min-sum up to 32 iterations in all; "ms" = plain min-sum for T
    iterations."""
    import torch

    from paper_2508_07879_amd import abi
    from workload import bits, gf2

    lam = gf2.logical_basis(code.hx.dense(), side.dense())
    lam_t = torch.from_numpy(lam.T.astype(np.float32)).to(dev)
    stats = {name: dict(fails=0, shots=0, iters=0, fallback=0, ms=0.0) for name, *_ in configs}
    for b in _batches(side, eval_seed, eval_shots, p, 65536):
        B = b.B
        syn = torch.from_numpy(bits.pack_bits(b.s).view(np.int32)).to(dev)
        pr = torch.from_numpy(b.gamma).to(dev)
        et = torch.from_numpy(b.e).to(dev)
        err, conv, it, _ = dec.outputs(B)
        used = torch.zeros(B, dtype=torch.uint8, device=dev)
        for name, kind, t, fb, wt in configs:
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            if kind == "nms":
                fbp = dec.params(max_iters=32) if fb else None
                abi.qldpc_nbp_decode(dec.handle, B, t, wt, fbp, syn, pr, err, conv, it, used)
            elif kind == "nmsc":
                abi.qldpc_nbp_decode_continue(dec.handle, B, t, wt, 32, 0.75, syn, pr, err, conv, it, used)
            else:
                abi.qldpc_decode_batch(dec.handle, dec.params(max_iters=t), B, syn, pr, err, conv, it, None)
            ev1.record()
            torch.cuda.synchronize()
            st = stats[name]
            st["ms"] += ev0.elapsed_time(ev1)
            st["fails"] += logical_fail_counts(lam_t, et, err, conv, side.n)
            st["shots"] += B
            st["iters"] += int(it.to(torch.int64).sum().item())
            if kind in ("nms", "nmsc"):
                st["fallback"] += int(used.to(torch.int64).sum().item())
    res = {}
    for name, st in stats.items():
        lo, hi = gf2.wilson(st["fails"], st["shots"])
        res[name] = dict(ler=st["fails"] / st["shots"], ci95=[lo, hi], mean_iters=st["iters"] / st["shots"],
                         fallback_rate=st["fallback"] / st["shots"],
                         syndromes_per_s=st["shots"] / (st["ms"] * 1e-3))
        if log:
            log(f"{name:22s} LER {res[name]['ler']:.5f} [{lo:.5f}, {hi:.5f}]  mean iters "
                f"{res[name]['mean_iters']:.2f}  fallback {res[name]['fallback_rate']:.4f}  "
                f"{res[name]['syndromes_per_s']:.3g} syn/s")
    return res


def study(dec, code, side, dev, Ts=(8, 16), p=0.05, train_shots=1 << 20, epochs=4, batch=4096, lr=1e-3,
          eval_shots=1 << 18, train_seed=1_000_003, eval_seed=2_000_003, log=None):
    """Trains weights at each T in Ts from the same training pairs (each T
    trained at its own T), then evaluates every neural mode at its T beside
    plain min-sum at 16 and 32 iterations on the same held-out shots."""
    t0 = time.time()
    data = training_data(side, dev, train_seed, train_shots, p)
    out = dict(p=p, train_shots=train_shots, epochs=epochs, batch=batch, lr=lr, eval_shots=eval_shots,
               train_seeds=f"shots 0..{train_shots - 1} of seed {train_seed}",
               eval_seeds=f"shots 0..{eval_shots - 1} of seed {eval_seed}", train_data_s=time.time() - t0,
               trained={})
    configs = [("ms_16", "ms", 16, False, None), ("ms_32", "ms", 32, False, None)]
    for T in Ts:
        t1 = time.time()
        w, _, losses = train(dec, side, dev, T, data, epochs, batch, lr, train_seed + T, log=log)
        out["trained"][f"T{T}"] = dict(train_s=time.time() - t1, loss_per_epoch=losses)
        wd = w.detach().contiguous()
        configs += [(f"nms_T{T}_fallback", "nms", T, True, wd), (f"nms_T{T}_nofallback", "nms", T, False, wd),
                    (f"nms_T{T}_continue", "nmsc", T, True, wd)]
    del data
    out["eval"] = evaluate(code, side, dec, dev, configs, eval_seed, eval_shots, p, log=log)
    return out


def _evaluate(args, code, side, dec, dev, w, T, report):
    wd = w.detach().contiguous()
    configs = []
    for t in sorted({max(1, T // 4), T // 2, (3 * T) // 4, T}):
        wt = wd[:t].contiguous()
        configs.append((f"nms_T{t}", "nms", t, True, wt))
        configs.append((f"nms_T{t}_nofallback", "nms", t, False, wt))
        configs.append((f"nms_T{t}_continue", "nmsc", t, True, wt))
    configs += [("ms_16", "ms", 16, False, None), ("ms_32", "ms", 32, False, None)]
    for t in sorted({max(1, T // 4), T // 2, (3 * T) // 4}):
        configs.append((f"ms_{t}", "ms", t, False, None))
    res = evaluate(code, side, dec, dev, configs, args.eval_seed, args.eval_shots, args.p,
                   log=lambda m: print(m, flush=True))
    report["eval"] = res
    report["note"] = ("neural rows with t < T evaluate the first t rows of weights trained at T "
                      "(truncations), not weights trained at t")
    if args.json:
        with open(args.json, "w") as f:
            json.dump(report, f, indent=1)
    return report


if __name__ == "__main__":
    main()
