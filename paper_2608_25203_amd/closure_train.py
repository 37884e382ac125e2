"""Train the learned DtN closure on snapshots the solver generates itself.

    python -m paper_2608_25203_amd.closure_train --out DIR [options]

1. Snapshots: seeded JONSWAP sea states on the 1024 x 1024, 2 pi x 2 pi,
   deep-water grid (k_p = 32, 32 grid points per peak wavelength), steepness drawn uniformly from [0.05, 0.2],
   advanced by the full-order (M = 6, FP64) RK4 solver; every `--every`
   steps the state is turned into one training sample by zk_closure_features
   (network inputs and the target (G^[6] - G^[2]) psi, normalised) and
   `--crops` random periodic crops of it are kept (zk_closure_crops).
2. Training: Adam on the masked MSE of the crops (halo 4) with the
   library's MFMA kernels (zk_cnn_train_step), cosine learning-rate decay;
   a held-out set of runs gives the validation loss.
3. Evaluation on held-out states: the relative L2 DtN error of order 2
   alone and of order 2 plus the network, both against order 6.

Writes DIR/closure_c5.npy (float32 parameters) and DIR/closure_c5.json
(normalisation constants, data and training record, evaluation).  Every
computation runs in libzk.so; torch only holds device memory.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2608_25203_amd.inputs import cnn_init_params, jonswap_state  # noqa: E402

GEOM = dict(nx=1024, ny=1024, L=2 * math.pi, g=9.81, kp=32.0, dt=0.007)
K0, ETA_SCALE, OUT_SCALE = 32.0, 0.1, 0.02
HALO = 4


def log(msg):
    print(f"[closure_train {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def make_objects(torch, max_pixels, low_precision=64):
    from paper_2608_25203_amd.zk import Closure, Net, Solver

    n, L, g = GEOM["nx"], GEOM["L"], GEOM["g"]
    low = Solver(n, n, L, L, math.inf, g, 2, precision=low_precision, check=False)
    full = Solver(n, n, L, L, math.inf, g, 6, check=True)
    net = Net(max(max_pixels, n * n))
    return low, full, net, Closure(low, full, net, K0, ETA_SCALE, OUT_SCALE)


def state(seed, steep, kmax_factor):
    n, L = GEOM["nx"], GEOM["L"]
    return jonswap_state(n, n, L, L, None, GEOM["g"], GEOM["kp"], steep, seed,
                         kmax=kmax_factor * GEOM["kp"] if kmax_factor else None)


def generate(torch, clo, full, seeds, steeps, snaps, every, crops, crop, kmax_factor, rng, tag):
    """Crops [N, 4, crop, crop] float32 on the device from M = 6 trajectories.

    A run the order-6 solver cannot carry through its whole window (a wave
    that steepens until the series diverges) is dropped with all of its
    snapshots: the states just before the blow-up have no trustworthy
    reference, and their targets can reach non-finite float32 values.  Returns the
    crops and the number of snapshots kept."""
    from paper_2608_25203_amd.zk import ZKError

    n = GEOM["nx"]
    out = torch.empty((len(seeds) * snaps * crops, 4, crop, crop), dtype=torch.float32, device="cuda")
    k = 0
    kept = dropped = 0
    t0 = time.time()
    for i, (seed, st) in enumerate(zip(seeds, steeps)):
        eta, psi = state(seed, st, kmax_factor)
        e = torch.tensor(eta, dtype=torch.float64, device="cuda")
        p = torch.tensor(psi, dtype=torch.float64, device="cuda")
        k0 = k
        for j in range(snaps):
            if j:
                try:
                    full.step(e, p, GEOM["dt"], every)
                except ZKError:
                    log(f"{tag}: run {seed} (steepness {st:.3f}) diverged at step {j * every}; run dropped")
                    k = k0
                    break
            smp = clo.features(e, p)
            offs = np.stack([rng.integers(0, n, crops), rng.integers(0, n, crops)], axis=1)
            out[k:k + crops] = clo.crops(smp, offs, crop, crop)
            k += crops
        if k > k0 and not bool(torch.isfinite(out[k0:k]).all().item()):
            log(f"{tag}: run {seed} (steepness {st:.3f}) gave non-finite samples; run dropped")
            k = k0
        if k > k0:
            kept += (k - k0) // crops
        else:
            dropped += 1
        if (i + 1) % 10 == 0 or i + 1 == len(seeds):
            log(f"{tag}: {i + 1}/{len(seeds)} runs ({dropped} dropped), {kept} snapshots, {k} crops, "
                f"{time.time() - t0:.1f} s")
    return out[:k], kept


def dtn_errors(torch, clo, low, full, e, p):
    """(||G2 - G6|| / ||G6||, ||G_closure - G6|| / ||G6||) in L2."""
    g6 = full.dtn(e, p)
    g2 = low.dtn(e, p)
    gc = clo.dtn(e, p)
    n6 = torch.linalg.vector_norm(g6).item()
    return (torch.linalg.vector_norm(g2 - g6).item() / n6, torch.linalg.vector_norm(gc - g6).item() / n6)


def evaluate(torch, clo, low, full, seeds, steeps, warm, kmax_factor):
    rows = []
    for seed in seeds:
        for st in steeps:
            eta, psi = state(seed, st, kmax_factor)
            e = torch.tensor(eta, dtype=torch.float64, device="cuda")
            p = torch.tensor(psi, dtype=torch.float64, device="cuda")
            if warm:
                from paper_2608_25203_amd.zk import ZKError

                try:
                    full.step(e, p, GEOM["dt"], warm)
                except ZKError:
                    log(f"eval seed {seed} steepness {st}: the order-6 run diverged within {warm} steps; skipped")
                    rows.append({"seed": seed, "steepness": st, "diverged": True})
                    continue
            e2, ec = dtn_errors(torch, clo, low, full, e, p)
            rows.append({"seed": seed, "steepness": st, "err_order2": e2, "err_closure": ec, "gain": e2 / ec})
            log(f"eval seed {seed} steepness {st}: order 2 {e2:.3e}, closure {ec:.3e}, gain {e2 / ec:.2f}")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--runs", type=int, default=100)
    ap.add_argument("--val-runs", type=int, default=6)
    ap.add_argument("--snaps", type=int, default=10)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--crops", type=int, default=10)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--kmax-factor", type=float, default=0.0,
                    help="spectral support k <= factor * k_p (0: the generator's default, min(4 k_p, kNyq / 2))")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=4)
    args = ap.parse_args()

    import torch

    assert torch.cuda.is_available(), "training runs on the GPU"
    os.makedirs(args.out, exist_ok=True)
    rng = np.random.default_rng(args.seed)
    low, full, net, clo = make_objects(torch, args.batch * args.crop * args.crop)
    net.set_params(np.concatenate([q.ravel() for q in cnn_init_params(args.seed)]).astype(np.float32))

    steeps = rng.uniform(0.05, 0.2, args.runs)
    train, nsnap = generate(torch, clo, full, [1000 + i for i in range(args.runs)], steeps, args.snaps, args.every,
                            args.crops, args.crop, args.kmax_factor, rng, "train")
    vsteeps = rng.uniform(0.05, 0.2, args.val_runs)
    val, _ = generate(torch, clo, full, [9000 + i for i in range(args.val_runs)], vsteeps, args.snaps, args.every,
                      2, args.crop, args.kmax_factor, rng, "val")
    tstd = float(train[:, 3].std().item())
    log(f"data: {nsnap} snapshots, {train.shape[0]} train crops, {val.shape[0]} val crops, target std {tstd:.3f}")

    def val_loss():
        tot, nb = 0.0, 0
        for i in range(0, val.shape[0] - args.batch + 1, args.batch):
            l, _ = net.gradient(val[i:i + args.batch].contiguous(), HALO)
            tot += l
            nb += 1
        return tot / max(nb, 1)

    hist = []
    v0 = val_loss()
    log(f"initial val loss {v0:.4e}")
    t0 = time.time()
    perm = torch.randperm(train.shape[0], device="cuda")
    pos = 0
    for it in range(args.steps):
        if pos + args.batch > train.shape[0]:
            perm = torch.randperm(train.shape[0], device="cuda")
            pos = 0
        batch = train.index_select(0, perm[pos:pos + args.batch]).contiguous()
        pos += args.batch
        lr = args.lr * 0.5 * (1 + math.cos(math.pi * it / args.steps))
        want = (it + 1) % 250 == 0
        l = net.train_step(batch, HALO, lr, want_loss=want)
        if want:
            v = val_loss()
            hist.append({"step": it + 1, "train_loss": l, "val_loss": v, "lr": lr})
            log(f"step {it + 1}: train {l:.4e} val {v:.4e} ({time.time() - t0:.1f} s)")
    train_time = time.time() - t0
    params = net.get_params()
    np.save(os.path.join(args.out, "closure_c5.npy"), params)

    ev = evaluate(torch, clo, low, full, [42, 43], [0.05, 0.1, 0.15, 0.2], 50, args.kmax_factor)
    rec = {"k0": K0, "eta_scale": ETA_SCALE, "out_scale": OUT_SCALE, "halo": HALO,
           "geometry": GEOM, "kmax_factor": args.kmax_factor,
           "data": {"runs": args.runs, "snapshots": nsnap, "snaps": args.snaps, "every": args.every,
                    "crops": args.crops,
                    "crop": args.crop, "train_crops": int(train.shape[0]), "val_crops": int(val.shape[0]),
                    "target_std": tstd},
           "training": {"steps": args.steps, "batch": args.batch, "lr": args.lr, "seconds": train_time,
                        "initial_val_loss": v0, "history": hist},
           "evaluation": ev}
    with open(os.path.join(args.out, "closure_c5.json"), "w") as f:
        json.dump(rec, f, indent=1)
    log(f"wrote {args.out}/closure_c5.npy and closure_c5.json")


if __name__ == "__main__":
    main()
