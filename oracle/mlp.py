"""CPU reference of the per-bead network of the learned initial guess.
TEST INFRASTRUCTURE ONLY.

Network (not part of the paper; the build's learned part): features
f = [r'(3), E'(3), one-hot type(2)], qn = Q_i/N_i;
h1 = tanh(W1 f + b1) (64), h2 = tanh(W2 h1 + b2) (64), o = W3 h2 + b3 (4),
q_hat = o[0:3] . E' + qn (1 + o[3]);  loss = mean (q_hat - q)^2.
Parameters are one flat vector: W1[64][8], b1[64], W2[64][64], b2[64],
W3[4][64], b3[4].  With ``bf16=True`` the operands of the two products that
the device runs on matrix cores (h1 W2^T forward; dz2^T h1 and dz2 W2 backward)
are rounded to bfloat16 (nearest, ties to even) first, as the device does.
"""
from __future__ import annotations

import numpy as np

F, H, O = 8, 64, 4
oW1, ob1 = 0, H * F
oW2 = ob1 + H
ob2 = oW2 + H * H
oW3 = ob2 + H
ob3 = oW3 + O * H
NPAR = ob3 + O


def bf16(x):
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    return (P[oW1:ob1].reshape(H, F), P[ob1:oW2], P[oW2:ob2].reshape(H, H), P[ob2:oW3],
            P[oW3:ob3].reshape(O, H), P[ob3:NPAR])


def forward(P, rows, bf=False):
    W1, b1, W2, b2, W3, b3 = unpack(P)
    r = np.asarray(rows, dtype=np.float64)
    f, qn = r[:, :F], r[:, F]
    h1 = np.tanh(f @ W1.T + b1)
    a, w = (bf16(h1), bf16(W2)) if bf else (h1, W2)
    h2 = np.tanh(a @ w.T + b2)
    o = h2 @ W3.T + b3
    q = np.sum(o[:, :3] * f[:, 3:6], axis=1) + qn * (1.0 + o[:, 3])
    return q, (f, qn, h1, h2, o)


def loss_grad(P, rows, bf=False):
    r = np.asarray(rows, dtype=np.float64)
    t = r[:, F + 1]
    q, (f, qn, h1, h2, o) = forward(P, rows, bf)
    W1, b1, W2, b2, W3, b3 = unpack(P)
    n = len(r)
    e = q - t
    loss = float(np.mean(e * e))
    dq = 2.0 * e / n
    dout = dq[:, None] * np.concatenate([f[:, 3:6], qn[:, None]], axis=1)
    gW3 = dout.T @ h2
    gb3 = dout.sum(0)
    dz2 = (dout @ W3) * (1.0 - h2 * h2)
    gb2 = dz2.sum(0)
    d2, a1, w2 = (bf16(dz2), bf16(h1), bf16(W2)) if bf else (dz2, h1, W2)
    gW2 = d2.T @ a1
    dh1 = d2 @ w2
    dz1 = dh1 * (1.0 - h1 * h1)
    gW1 = dz1.T @ f
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g
