"""Plain FP64 CPU reference ("the oracle") for the learned CP-validity and
sub-pixel head that sits after Fast-NCC_SFOC matching.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import or call this module.  The GPU
library shares no code with it.

The head is not part of the paper.  The paper fixes what it consumes: the NCC
surface of Eq. 9 over the search offsets, its argmax CP and the parabola
refinement (Section 3.2.2), and the 1.5 px correctness threshold of
Section 4.1 that defines its training labels.  Its own definition is written
out here in full and every GPU kernel is checked against it:

Features of a CP whose integer peak (u*, v*) is interior to its (2r+1)^2
surface S:
  crop   33 x 33, crop[a][b] = S[u* - 16 + a][v* - 16 + b], -1 outside S;
  stats  s0 peak S[u*, v*];
         s1 largest S at offsets with max(|u - u*|, |v - v*|) > 1 (-1 if none);
         s2 mean of S;  s3 standard deviation of S (population);
         s4 sqrt(max(varT, 0) / mnz), the template's standard deviation
            (varT = R_TT - R_T^2 / mnz, Eq. 11-12, mnz = m*m*z);
         s5 sqrt(max(varS, 0) / mnz) of the search window at the peak (Eq. 16);
         s6 R_T / mnz, the template mean;
         s7 mean of the two second differences of S at the peak (the
            parabola curvatures of the peak fit).
Network (parameters in one float32 vector, in this order):
  conv1 3x3, 1 -> 32, stride 1, pad 1, ReLU          33x33 -> 33x33
  conv2 3x3, 32 -> 32, stride 2, pad 1, ReLU         33x33 -> 17x17
  conv3 3x3, 32 -> 32, stride 2, pad 1, ReLU         17x17 -> 9x9
  conv4 3x3, 32 -> 32, stride 2, pad 1, ReLU         9x9   -> 5x5
  fc1   (800 flattened channel-major + 8 stats) -> 32, ReLU
  fc2   32 -> 3: validity logit, sub-pixel offsets (oy, ox)
  each conv: weight [out, in, 3, 3] then bias [out]; each fc: weight
  [out, in] then bias [out].  Weights (not biases) enter every product
  rounded to bfloat16 (nearest even); sums are formed in float32 on the GPU
  and in float64 here.
Loss over a batch of B samples (mean over the batch):
  BCE(logit, y) + LAMBDA * y * (SmoothL1(oy - ty) + SmoothL1(ox - tx)),
  SmoothL1(d) = 0.5 d^2 / BETA if |d| < BETA else |d| - BETA / 2.
  Gradients flow to the bfloat16-rounded weights as if they were the
  parameters (the float32 master copy takes them unchanged).
Adam: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, no weight decay.
Inference on an eligible CP (interior peak: VALID or INCONSISTENT after the
consistency check): sigmoid(logit) >= threshold sets VALID else
INCONSISTENT, LEARNED is set, and the sub-pixel part becomes (oy, ox)
clipped to [-1.5, 1.5].  Other CPs keep the plain result (the fallback).

Parity status: every function here is pinned by the CPU tests (library
correlation, finite differences, closed forms and brute force).
"""
from __future__ import annotations

import numpy as np

from oracle import sfoc_oracle as O

CROP = 33
HALF = CROP // 2
NSTAT = 8
CH = 32
LAMBDA = 4.0
BETA = 0.1
CLIP = 1.5
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8

# (name, shape) of every parameter block, in storage order.
CONVS = [(1, CH, 1), (CH, CH, 2), (CH, CH, 2), (CH, CH, 2)]   # (in, out, stride)
SIDES = [33, 33, 17, 9, 5]                                     # input side of conv k, then output of conv4
FC1_IN = CH * SIDES[4] * SIDES[4] + NSTAT


def layout():
    out = []
    for k, (ci, co, _) in enumerate(CONVS):
        out.append((f"conv{k + 1}.w", (co, ci, 3, 3)))
        out.append((f"conv{k + 1}.b", (co,)))
    out.append(("fc1.w", (CH, FC1_IN)))
    out.append(("fc1.b", (CH,)))
    out.append(("fc2.w", (3, CH)))
    out.append(("fc2.b", (3,)))
    return out


N_PARAMS = sum(int(np.prod(s)) for _, s in layout())


def unpack(theta: np.ndarray) -> dict:
    """Flat parameter vector -> named float64 arrays (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in layout():
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in layout()])


# ------------------------------------------------------------ features -----
def crop_and_stats(S: np.ndarray, u: int, v: int, varT: float, varS: float, RT: float, mnz: float):
    """33 x 33 crop and the 8 statistics of one surface (see the module text)."""
    V = S.shape[0]
    crop = np.full((CROP, CROP), -1.0)
    for a in range(CROP):
        for b in range(CROP):
            y, x = u - HALF + a, v - HALF + b
            if 0 <= y < V and 0 <= x < V:
                crop[a, b] = S[y, x]
    second = -1.0
    for y in range(V):
        for x in range(V):
            if max(abs(y - u), abs(x - v)) > 1 and S[y, x] > second:
                second = S[y, x]
    c0 = S[u, v]
    curv = 0.5 * ((S[u - 1, v] - 2 * c0 + S[u + 1, v]) + (S[u, v - 1] - 2 * c0 + S[u, v + 1]))
    stats = np.array([c0, second, S.mean(), S.std(), np.sqrt(max(varT, 0.0) / mnz),
                      np.sqrt(max(varS, 0.0) / mnz), RT / mnz, curv])
    return crop, stats


def eligible(flags) -> np.ndarray:
    """CPs with an interior peak (VALID or INCONSISTENT after the check)."""
    f = np.asarray(flags, dtype=np.int64)
    return (f & (O.VALID | O.INCONSISTENT)) != 0


def features(Fs: np.ndarray, Fr: np.ndarray, ips, prior, m: int, r: int, cps, surfaces):
    """Crops (n, 33, 33) and stats (n, 8) of every CP (zeros where the CP is
    not eligible).  Fs, Fr: (H, W, z) descriptors; surfaces (n, V, V)."""
    n = len(cps)
    z = Fs.shape[2]
    mnz = float(m * m * z)
    G1, G2 = O.integral_feature_images(Fr)
    crops = np.zeros((n, CROP, CROP))
    stats = np.zeros((n, NSTAT))
    ok = eligible(cps["flags"])
    for i in range(n):
        if not ok[i]:
            continue
        pr = None if prior is None else prior[i]
        (ty, tx), (sy, sx) = O.window_origins(ips[i], pr, m, r)
        T = np.asarray(Fs[ty:ty + m, tx:tx + m, :], dtype=np.float64)
        RT, RTT = T.sum(), (T * T).sum()
        varT = RTT - RT * RT / mnz
        u, v = int(cps["dy"][i]) + r, int(cps["dx"][i]) + r
        RS = O.box_sum(G1, sy + u, sx + v, m, m)
        RSS = O.box_sum(G2, sy + u, sx + v, m, m)
        varS = RSS - RS * RS / mnz
        crops[i], stats[i] = crop_and_stats(np.asarray(surfaces[i], np.float64), u, v, varT, varS, RT, mnz)
    return crops, stats


# ------------------------------------------------------------- network -----
def bf16(w):
    return O.round_to_bf16(np.asarray(w, dtype=np.float64)).astype(np.float64)


def conv_forward(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int):
    """out[n, o, y, x] = b[o] + sum_{c, i, j} w[o, c, i, j] * xpad[n, c, s y + i, s x + j]
    with one zero of padding on each side."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    N, C, H, W = x.shape
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    out = np.zeros((N, w.shape[0], Ho, Wo)) + b[None, :, None, None]
    for i in range(3):
        for j in range(3):
            patch = xp[:, :, i:i + stride * (Ho - 1) + 1:stride, j:j + stride * (Wo - 1) + 1:stride]
            out += np.einsum("oc,ncyx->noyx", w[:, :, i, j], patch)
    return out


def conv_backward(x: np.ndarray, w: np.ndarray, dout: np.ndarray, stride: int):
    """Gradients (dx, dw, db) of conv_forward for an upstream gradient dout."""
    N, C, H, W = x.shape
    _, O_, Ho, Wo = dout.shape
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros(w.shape)
    for i in range(3):
        for j in range(3):
            sl = (slice(None), slice(None), slice(i, i + stride * (Ho - 1) + 1, stride),
                  slice(j, j + stride * (Wo - 1) + 1, stride))
            dw[:, :, i, j] = np.einsum("noyx,ncyx->oc", dout, xp[sl])
            dxp[sl] += np.einsum("oc,noyx->ncyx", w[:, :, i, j], dout)
    return dxp[:, :, 1:H + 1, 1:W + 1], dw, dout.sum(axis=(0, 2, 3))


def forward(theta, crops, stats, quantise: bool = True):
    """Network outputs (B, 3) and the activations the backward pass needs."""
    P = unpack(theta)
    q = bf16 if quantise else (lambda a: np.asarray(a, np.float64))
    x = np.asarray(crops, np.float64)[:, None, :, :]
    acts = [x]
    for k, (_, _, s) in enumerate(CONVS):
        x = np.maximum(conv_forward(x, q(P[f"conv{k + 1}.w"]), P[f"conv{k + 1}.b"], s), 0.0)
        acts.append(x)
    h = np.concatenate([x.reshape(len(x), -1), np.asarray(stats, np.float64)], axis=1)
    h1 = np.maximum(h @ q(P["fc1.w"]).T + P["fc1.b"], 0.0)
    out = h1 @ q(P["fc2.w"]).T + P["fc2.b"]
    return out, dict(acts=acts, h=h, h1=h1)


def bce_with_logits(l, y):
    l = np.asarray(l, np.float64)
    return np.maximum(l, 0.0) - l * y + np.log1p(np.exp(-np.abs(l)))


def smooth_l1(d):
    a = np.abs(d)
    return np.where(a < BETA, 0.5 * d * d / BETA, a - 0.5 * BETA)


def smooth_l1_grad(d):
    return np.where(np.abs(d) < BETA, d / BETA, np.sign(d))


def sigmoid(l):
    l = np.asarray(l, np.float64)
    return np.where(l >= 0, 1.0 / (1.0 + np.exp(-np.abs(l))), np.exp(-np.abs(l)) / (1.0 + np.exp(-np.abs(l))))


def loss(out, y, ty, tx):
    """Mean over the batch of the validity and offset losses."""
    B = len(out)
    y = np.asarray(y, np.float64)
    l = bce_with_logits(out[:, 0], y) + LAMBDA * y * (smooth_l1(out[:, 1] - ty) + smooth_l1(out[:, 2] - tx))
    return float(l.sum() / B)


def loss_grad(out, y, ty, tx):
    B = len(out)
    y = np.asarray(y, np.float64)
    g = np.zeros_like(out)
    g[:, 0] = (sigmoid(out[:, 0]) - y) / B
    g[:, 1] = LAMBDA * y * smooth_l1_grad(out[:, 1] - ty) / B
    g[:, 2] = LAMBDA * y * smooth_l1_grad(out[:, 2] - tx) / B
    return g


def backward(theta, crops, stats, y, ty, tx, quantise: bool = True):
    """(loss, gradient of the loss w.r.t. the parameter vector)."""
    P = unpack(theta)
    q = bf16 if quantise else (lambda a: np.asarray(a, np.float64))
    out, c = forward(theta, crops, stats, quantise)
    L = loss(out, y, ty, tx)
    g = {}
    d = loss_grad(out, y, ty, tx)
    g["fc2.w"] = d.T @ c["h1"]
    g["fc2.b"] = d.sum(axis=0)
    dh1 = (d @ q(P["fc2.w"])) * (c["h1"] > 0)
    g["fc1.w"] = dh1.T @ c["h"]
    g["fc1.b"] = dh1.sum(axis=0)
    dh = dh1 @ q(P["fc1.w"])
    acts = c["acts"]
    dx = dh[:, :CH * SIDES[4] * SIDES[4]].reshape(acts[4].shape)
    for k in range(len(CONVS) - 1, -1, -1):
        dx = dx * (acts[k + 1] > 0)
        dxin, dw, db = conv_backward(acts[k], q(P[f"conv{k + 1}.w"]), dx, CONVS[k][2])
        g[f"conv{k + 1}.w"] = dw
        g[f"conv{k + 1}.b"] = db
        dx = dxin
    return L, pack(g)


def adam_step(theta, grad, m, v, t: int, lr: float):
    """One Adam step (t counts from 1).  Returns (theta, m, v)."""
    theta = np.asarray(theta, np.float64)
    m = ADAM_B1 * np.asarray(m, np.float64) + (1 - ADAM_B1) * grad
    v = ADAM_B2 * np.asarray(v, np.float64) + (1 - ADAM_B2) * grad * grad
    mh = m / (1 - ADAM_B1 ** t)
    vh = v / (1 - ADAM_B2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


def apply(cps, out, threshold: float = 0.5):
    """Inference decision on CP records (a copy is returned)."""
    c = cps.copy()
    ok = eligible(c["flags"])
    p = sigmoid(out[:, 0])
    for i in np.nonzero(ok)[0]:
        f = int(c["flags"][i]) & ~(O.VALID | O.INCONSISTENT)
        f |= O.LEARNED | (O.VALID if p[i] >= threshold else O.INCONSISTENT)
        c["flags"][i] = f
        c["sub_dy"][i] = float(np.clip(out[i, 1], -CLIP, CLIP))
        c["sub_dx"][i] = float(np.clip(out[i, 2], -CLIP, CLIP))
    return c
