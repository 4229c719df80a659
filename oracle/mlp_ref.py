"""FP64 CPU reference of the learned-start network (test infrastructure).

Only the tests use it.  Forward and backward of the 96 -> 256 -> 256 -> 256
-> 15 GELU network and its masked mean-squared error, written with numpy
matrix products; a `bf16` mode rounds at the same places the GPU kernels
store BF16 values (features, weights, activations and back-propagated
gradients), so that the kernels can be compared at FP32-accumulation
precision.  The feature encoding is re-derived here from the scene and the
batch, independently of the kernels.
"""
from __future__ import annotations

import numpy as np
from math import erf

F_IN, HID, F_OUT, F_OUTP = 96, 256, 15, 16
SIZES = [("W1", (HID, F_IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, HID)),
         ("b3", (HID,)), ("W4", (F_OUTP, HID)), ("b4", (F_OUTP,))]
NPAR = sum(int(np.prod(s)) for _, s in SIZES)

_erf = np.vectorize(erf)


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(flat):
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], np.float64).reshape(shp)
        o += k
    return out


def parse_blob(blob: bytes):
    """Weights, Adam moments and header of a saved network."""
    import json
    assert blob[:8] == b"MPTMLP01"
    hl = int(np.frombuffer(blob[8:12], np.uint32)[0])
    hdr = json.loads(blob[12:12 + hl].decode())
    arr = np.frombuffer(blob[12 + hl:], np.float32)
    n = hdr["params"]
    return hdr, arr[:n].copy(), arr[n:2 * n].copy(), arr[2 * n:3 * n].copy()


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / np.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + _erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def features(scene, batch):
    """The 96 inputs per solve: RX and TX in the frame centred on TX and
    scaled by 1/|RX-TX|, then per interaction slot a one-hot type, the object
    in that frame and a present bit."""
    n = batch.n
    F = np.zeros((n, F_IN))
    tx = scene.tx
    npl, nln, nq, nc = scene.counts
    for i in range(n):
        rx = batch.rx[batch.rx_index[i]]
        L = np.linalg.norm(rx - tx)
        L = L if L > 0 else 1.0
        F[i, 0:3] = (rx - tx) / L
        for k in range(batch.order[i]):
            g = batch.prim[k, i]
            base = 6 + 17 * k
            p = np.zeros(12)
            if g < npl:
                t, q = 0, scene.planes[g]
                p[0:3] = q[0:3]
                p[3] = (q[3] - q[0:3] @ tx) / L
            elif g < npl + nln:
                t, q = 1, scene.lines[g - npl]
                e = q[3:6]
                p[0:3] = e
                p[3:6] = (q[0:3] + ((tx - q[0:3]) @ e) * e - tx) / L
            elif g < npl + nln + nq:
                t, q = 2, scene.quadrics[g - npl - nln]
                p[0:3] = (q[0:3] - tx) / L
                p[3:9] = q[3:9] * L
                p[9:12] = q[9:12]
            else:
                t, q = 3, scene.circles[g - npl - nln - nq]
                p[0:3] = (q[0:3] - tx) / L
                p[3:6] = q[3:6]
                p[6] = q[6] / L
            F[i, base + t] = 1.0
            F[i, base + 4:base + 16] = p
            F[i, base + 16] = 1.0
    return F


def targets(scene, batch, x):
    """Target points in the frame: (x - TX)/|RX-TX|, [n][16] (last column 0)."""
    n = batch.n
    T = np.zeros((n, F_OUTP))
    for i in range(n):
        rx = batch.rx[batch.rx_index[i]]
        L = np.linalg.norm(rx - scene.tx)
        L = L if L > 0 else 1.0
        for j in range(3 * batch.order[i]):
            T[i, j] = (x[j, i] - scene.tx[j % 3]) / L
    return T


def loss_and_grad(P, X, T, mask, rounding=False):
    """Masked MSE and its gradient for parameters P (dict), inputs X [n][96],
    targets T and mask [n][16].  With rounding, values are rounded to BF16
    where the GPU stores BF16."""
    r = bf16 if rounding else (lambda a: a)
    W = {k: (r(v) if k.startswith("W") else v) for k, v in P.items()}
    X = r(X)
    Z1 = X @ W["W1"].T + W["b1"]
    H1 = r(gelu(Z1))
    Z2 = H1 @ W["W2"].T + W["b2"]
    H2 = r(gelu(Z2))
    Z3 = H2 @ W["W3"].T + W["b3"]
    H3 = r(gelu(Z3))
    Y = H3 @ W["W4"].T + W["b4"]
    D = (Y - T) * mask
    cnt = mask.sum()
    loss = (D ** 2).sum() / cnt
    dY = r(2.0 * D / cnt)
    G = {}
    G["W4"] = dY.T @ H3
    G["b4"] = dY.sum(0)
    dZ3 = r((dY @ W["W4"]) * gelu_d(Z3))
    G["W3"] = dZ3.T @ H2
    G["b3"] = dZ3.sum(0)
    dZ2 = r((dZ3 @ W["W3"]) * gelu_d(Z2))
    G["W2"] = dZ2.T @ H1
    G["b2"] = dZ2.sum(0)
    dZ1 = r((dZ2 @ W["W2"]) * gelu_d(Z1))
    G["W1"] = dZ1.T @ X
    G["b1"] = dZ1.sum(0)
    return loss, G, Y
