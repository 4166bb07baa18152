"""Serving sweep: open-loop Poisson load against the continuous-batching
server at increasing offered rates, reporting p50 / p99 / p99.9 latency
(from scheduled arrival to completion) and delivered throughput.

Requests: 1 or 64 syndromes (half each) of a code drawn uniformly from the
served lifted codes, plain or neural min-sum (half each where weights are
loaded; weights not trained for a code default to all-alpha weights, which
decode exactly as plain min-sum and are flagged "untrained"), per-shot
noise rates uniform in [0.01, 0.08).

    python -m paper_2508_07879_amd.serve --L 32 64 128 --rates 1e3 1e4 1e5 3e5 1e6 2e6 \
        --duration 10 --weights 64=weights.pt --json sweep.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="+", default=[32, 64, 128])
    ap.add_argument("--rates", type=float, nargs="+", default=[1e3, 1e4, 1e5, 3e5, 1e6, 2e6])
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--T", type=int, default=16)
    ap.add_argument("--weights", nargs="*", default=[], help="L=path of trained neural weights")
    ap.add_argument("--pool", type=int, default=4096)
    ap.add_argument("--max-inflight", type=int, default=4)
    ap.add_argument("--max-batch-shots", type=int, default=8192)
    ap.add_argument("--queue", type=int, default=1 << 20)
    ap.add_argument("--hbm-budget", type=float, default=0, help="bytes (0 = no cap)")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--json", default="")
    args = ap.parse_args(argv)

    import torch

    from paper_2508_07879_amd import Decoder, abi, nms
    from workload import bits, lp, noise

    torch.cuda.set_device(0)
    codes = [lp.lp_code(L) for L in args.L]
    decs = [Decoder(c.hz) for c in codes]
    trained = {int(k): v for k, v in (w.split("=", 1) for w in args.weights)}
    weights, wstate = [], {}
    for L, c in zip(args.L, codes):
        if L in trained:
            w, meta, _ = nms.load_weights(trained[L], c.hz)
            T = int(w.shape[0])
            if T != args.T:
                raise ValueError(f"weights for L={L} have T={T}, expected {args.T}")
            weights.append(w.contiguous())
            wstate[L] = "trained"
        else:
            weights.append(nms.init_weights(args.T, c.hz.nnz, 0.75))
            wstate[L] = "untrained (all alpha)"
    pools_s, pools_p = [], []
    for i, c in enumerate(codes):
        p = noise.shot_rates(args.seed + i, np.arange(args.pool))
        b = noise.Batch(c.hz, args.seed + 100 + i, np.arange(args.pool), p)
        pools_s.append(np.ascontiguousarray(bits.pack_bits(b.s)))
        pools_p.append(np.ascontiguousarray(b.gamma))
    prm = decs[0].params(max_iters=32)
    srv = abi.qldpc_server_create([d.handle for d in decs], prm, nms_weights=weights, nms_T=args.T,
                                  hbm_budget=int(args.hbm_budget), max_inflight=args.max_inflight,
                                  max_batch_shots=args.max_batch_shots, queue_capacity=args.queue)
    out = dict(L=args.L, T=args.T, weights=wstate, duration_s=args.duration, points=[])
    try:
        slots, slot_bytes, _, _ = abi.qldpc_server_info(srv)
        out.update(slots=slots, slot_bytes=slot_bytes, max_batch_shots=args.max_batch_shots)
        abi.qldpc_server_loadgen(srv, 1e4, 0.2, pools_s, pools_p, seed=1)    # warm-up
        for r in args.rates:
            res, _ = abi.qldpc_server_loadgen(srv, r, args.duration, pools_s, pools_p, seed=int(r) % 1000003)
            res["offered_shots_per_s"] = r
            out["points"].append(res)
            print(json.dumps(res), file=sys.stderr, flush=True)
    finally:
        abi.qldpc_server_destroy(srv)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    main()
