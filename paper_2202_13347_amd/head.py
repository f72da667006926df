"""Learned CP-validity and sub-pixel head: samples from seeded pairs, training
and evaluation.

Every computation (descriptors, matching, features, network, losses, Adam,
the decision) runs in libsfoc's kernels through the binding; this module
draws the inputs, labels them from the known shifts, shuffles batches
(torch indexing) and reports metrics.

Labels (not in the paper; defined from its Section 4.1 correctness
threshold): a CP with an interior peak is positive when its integer
displacement D = prior + (dy, dx) lies within 1.5 px of the true shift and
its template is not more than half covered by an occlusion patch; its
offset target is (true shift - D).

    python -m paper_2202_13347_amd.head train --pairs 2000 --epochs 8 --out head_params.f32
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "head_params.f32")
TRAIN_SEED0, TEST_SEED0 = 1_000_000, 2_000_000
CORRECT_PX = 1.5


def load_params(path: str = DEFAULT_PARAMS) -> np.ndarray:
    th = np.fromfile(path, dtype="<f4")
    if th.size != S.HEAD_PARAMS:
        raise ValueError(f"{path}: {th.size} values, expected {S.HEAD_PARAMS}")
    return th


def save_params(th, path: str):
    np.asarray(th, dtype="<f4").tofile(path)


def _occluded(ips, m, mask):
    """Templates more than half covered by the occlusion mask."""
    out = np.zeros(len(ips), dtype=bool)
    if mask is None:
        return out
    for i, (y, x) in enumerate(ips):
        ty, tx = y - m // 2, x - m // 2
        win = mask[max(ty, 0):ty + m, max(tx, 0):tx + m]
        out[i] = win.sum() > 0.5 * m * m
    return out


def pair_samples(pr, ips, mask, m: int, r: int, p, device="cuda"):
    """Library pipeline on one pair: descriptors, Fast-NCC with surfaces,
    head features; plus labels from the known shift.  Returns a dict of
    device tensors (crops, stats, cps) and host arrays."""
    import torch
    ref = torch.from_numpy(pr.ref).to(device)
    sen = torch.from_numpy(pr.sen).to(device)
    dips = torch.from_numpy(np.ascontiguousarray(ips, np.int32)).to(device)
    dref, i1, i2 = S.describe(ref, p, integrals=True)
    dsen, _, _ = S.describe(sen, p, integrals=False)
    cps, ncc = S.fastncc_match(dsen, dref, i1, i2, dips, m, r, want_ncc=True)
    crops, stats = S.head_features(dsen, dref, i1, i2, dips, m, r, ncc, cps)
    g = S.cps_to_numpy(cps)
    elig = (g["flags"] & (S.VALID | S.INCONSISTENT)) != 0
    D = np.stack([g["dy"], g["dx"]], 1).astype(np.float64)
    dist = np.hypot(D[:, 0] - pr.shift[0], D[:, 1] - pr.shift[1])
    occ = _occluded(ips, m, mask)
    label = ((dist <= CORRECT_PX) & ~occ).astype(np.float32)
    target = (pr.shift[None, :] - D).astype(np.float32)
    return dict(crops=crops, stats=stats, cps=cps, elig=elig, label=label, target=target, occ=occ,
                plain=g, shift=pr.shift)


def build(seeds, p=None, device="cuda", workers=8, log=None):
    """Training tensors (eligible CPs of the given seeds) on the device."""
    import torch
    p = p or S.preset("baseline")
    rec = synth.HEAD
    crops, stats, label, target = [], [], [], []
    t0 = time.perf_counter()
    pairs = synth.head_pairs(seeds, rec, workers=workers)
    for k, (pr, ips, mask) in enumerate(pairs):
        s = pair_samples(pr, ips, mask, rec["m"], rec["r"], p, device)
        idx = torch.from_numpy(np.nonzero(s["elig"])[0]).to(device)
        crops.append(s["crops"].index_select(0, idx))
        stats.append(s["stats"].index_select(0, idx))
        label.append(torch.from_numpy(s["label"][s["elig"]]).to(device))
        target.append(torch.from_numpy(s["target"][s["elig"]]).to(device))
        if log and (k + 1) % 200 == 0:
            log(f"samples: {k + 1} pairs, {sum(len(c) for c in label)} samples, {time.perf_counter() - t0:.1f} s")
    return dict(crops=torch.cat(crops), stats=torch.cat(stats), label=torch.cat(label),
                target=torch.cat(target).contiguous())


def train(head: S.Head, data: dict, epochs: int, batch: int = 256, lr: float = 1e-3, seed: int = 0, log=None):
    """Adam over shuffled batches; the learning rate falls by 10x over the
    last quarter of the steps.  Returns the mean loss per epoch."""
    import torch
    n = data["label"].shape[0]
    gen = torch.Generator().manual_seed(seed)
    steps_per = n // batch
    total = steps_per * epochs
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(data["label"].device)
        losses = []
        for s in range(steps_per):
            idx = perm[s * batch:(s + 1) * batch]
            rate = lr if k < 0.75 * total else lr * 0.1
            loss, _ = head.train_step(data["crops"].index_select(0, idx), data["stats"].index_select(0, idx),
                                      data["label"].index_select(0, idx),
                                      data["target"].index_select(0, idx).contiguous(), rate)
            losses.append(loss)
            k += 1
        ep_loss = float(torch.stack(losses).mean())
        hist.append(ep_loss)
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {ep_loss:.4f}")
    return hist


def evaluate(head: S.Head, seeds, p=None, device="cuda", threshold: float = 0.5, workers=8):
    """Plain (parabola + consistency) vs learned on held-out seeds: sub-pixel
    RMSE against the true shift over positive CPs, and the precision /
    recall of the VALID decision against the labels, over eligible CPs."""
    p = p or S.preset("baseline")
    rec = synth.HEAD
    rows = []
    for pr, ips, mask in synth.head_pairs(seeds, rec, workers=workers):
        s = pair_samples(pr, ips, mask, rec["m"], rec["r"], p, device)
        cps = s["cps"].clone()
        head.infer(s["crops"], s["stats"], cps, threshold)
        learned = S.cps_to_numpy(cps)
        for i in np.nonzero(s["elig"])[0]:
            rows.append((s["label"][i], s["target"][i, 0], s["target"][i, 1],
                         s["plain"]["sub_dy"][i], s["plain"]["sub_dx"][i], bool(s["plain"]["flags"][i] & S.VALID),
                         learned["sub_dy"][i], learned["sub_dx"][i], bool(learned["flags"][i] & S.VALID),
                         bool(s["occ"][i])))
    a = np.array(rows, dtype=np.float64)
    lab = a[:, 0] > 0.5
    pos = lab

    def rmse(sy, sx):
        return float(np.sqrt(np.mean((a[pos, sy] - a[pos, 1]) ** 2 + (a[pos, sx] - a[pos, 2]) ** 2)))

    def pr_rc(col):
        v = a[:, col] > 0.5
        tp = float((v & lab).sum())
        return tp / max(1.0, float(v.sum())), tp / max(1.0, float(lab.sum()))

    pp, rp = pr_rc(5)
    pl, rl = pr_rc(8)
    return dict(samples=int(len(a)), positives=int(pos.sum()), occluded=int(a[:, 9].sum()),
                rmse_plain=rmse(3, 4), rmse_learned=rmse(6, 7),
                precision_plain=pp, recall_plain=rp, precision_learned=pl, recall_learned=rl)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--pairs", type=int, default=2000)
    t.add_argument("--epochs", type=int, default=8)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--test-pairs", type=int, default=200)
    t.add_argument("--out", default=DEFAULT_PARAMS)
    t.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    import torch
    S.lib()
    dev = torch.device("cuda:0")
    data = build(range(TRAIN_SEED0, TRAIN_SEED0 + args.pairs), device=dev, workers=args.workers, log=log)
    n = int(data["label"].shape[0])
    log(f"training samples: {n} ({float(data['label'].mean()):.3f} positive)")
    head = S.Head(synth.head_init_params(args.seed), device=dev)
    t0 = time.perf_counter()
    train(head, data, args.epochs, args.batch, args.lr, args.seed, log=log)
    torch.cuda.synchronize()
    log(f"training: {time.perf_counter() - t0:.1f} s")
    save_params(head.params.cpu().numpy(), args.out)
    res = evaluate(head, range(TEST_SEED0, TEST_SEED0 + args.test_pairs), device=dev, workers=args.workers)
    log("held-out: " + " ".join(f"{k}={v:.4f}" if isinstance(v, float) else f"{k}={v}" for k, v in res.items()))
    return 0


if __name__ == "__main__":
    sys.exit(main())
