"""Learned pre-screen network (oracle, FP64) -- test infrastructure only.

Not part of the paper's method: a small 1D convolutional network that looks
at the zero-drift power |X|^2 of a block of 4096 Fourier bins and predicts
whether full FDAS would find a significant candidate in that block.  This
module writes the network out in plain NumPy float64 so that the GPU
training and inference kernels can be checked against it; it imports nothing
from the library.

Network (all convolutions are cross-correlations with zero padding 4,
kernel 9, 'same' length):
  a0[0][t]   = log(1 + P[t]),                  t < 4096   (input, P = |X|^2)
  z1 = conv(a0; W1, b1)  (1 -> 32)   a1 = maxpool4(relu(z1))   -> 32 x 1024
  z2 = conv(a1; W2, b2)  (32 -> 32)  a2 = maxpool4(relu(z2))   -> 32 x 256
  z3 = conv(a2; W3, b3)  (32 -> 32)  a3 = maxpool4(relu(z3))   -> 32 x 64
  z4 = conv(a3; W4, b4)  (32 -> 32)  h  = max_t relu(z4)       -> 32
  logit = wf . h + bf
  conv(x; W, b)[o][t] = b[o] + sum_i sum_{k<9} W[o][i][k] x[i][t + k - 4]
  maxpool4(y)[c][p] = max_{q<4} y[c][4p + q]   (ties: the first q)
Loss (mean over the batch, positive weight w):
  L = mean( -w y log s(logit) - (1 - y) log(1 - s(logit)) ),  s = logistic.

Parameters are one flat vector in the order W1, b1, W2, b2, W3, b3, W4, b4,
wf, bf (row-major W[o][i][k]).
"""

import numpy as np

C, K, PAD, POOL, BLOCK = 32, 9, 4, 4, 4096
LAYERS = [(1, C), (C, C), (C, C), (C, C)]


def param_shapes():
    shapes = []
    for cin, cout in LAYERS:
        shapes += [(cout, cin, K), (cout,)]
    shapes += [(C,), (1,)]
    return shapes


def n_params():
    return int(sum(np.prod(s) for s in param_shapes()))


def unpack(theta):
    out, o = [], 0
    for s in param_shapes():
        m = int(np.prod(s))
        out.append(np.asarray(theta[o:o + m], dtype=np.float64).reshape(s))
        o += m
    return out


def features(power):
    """Network input of one block: log(1 + P) (float64)."""
    return np.log1p(np.asarray(power, dtype=np.float64))


def conv(x, W, b):
    """Cross-correlation, zero padding 4: x [cin][L] -> [cout][L]."""
    cin, L = x.shape
    xp = np.zeros((cin, L + 2 * PAD))
    xp[:, PAD:PAD + L] = x
    cols = np.stack([xp[:, k:k + L] for k in range(K)], axis=1)  # [cin][K][L]
    return b[:, None] + np.einsum("oik,ikt->ot", W, cols)


def maxpool(y):
    c, L = y.shape
    r = y.reshape(c, L // POOL, POOL)
    arg = np.argmax(r, axis=2)  # first maximum
    return np.take_along_axis(r, arg[..., None], axis=2)[..., 0], arg


def forward(theta, x0):
    """logit and the cache needed by backward, for one block x0 [4096]."""
    W1, b1, W2, b2, W3, b3, W4, b4, wf, bf = unpack(theta)
    cache = {"x": [np.asarray(x0, dtype=np.float64)[None, :]]}
    a = cache["x"][0]
    for l, (W, b) in enumerate([(W1, b1), (W2, b2), (W3, b3)]):
        z = conv(a, W, b)
        r = np.maximum(z, 0.0)
        a, arg = maxpool(r)
        cache.setdefault("z", []).append(z)
        cache.setdefault("arg", []).append(arg)
        cache["x"].append(a)
    z4 = conv(a, W4, b4)
    r4 = np.maximum(z4, 0.0)
    t4 = np.argmax(r4, axis=1)
    h = r4[np.arange(C), t4]
    cache["z"].append(z4)
    cache["t4"] = t4
    cache["h"] = h
    logit = float(wf @ h + bf[0])
    return logit, cache


def softplus(x):
    """log(1 + e^x) without overflow."""
    return np.log1p(np.exp(-abs(x))) + max(x, 0.0)


def loss_and_dlogit(logit, label, w_pos):
    # -log s(l) = softplus(-l), -log(1 - s(l)) = softplus(l)
    s = 1.0 / (1.0 + np.exp(-logit))
    loss = w_pos * label * softplus(-logit) + (1.0 - label) * softplus(logit)
    dlogit = w_pos * label * (s - 1.0) + (1.0 - label) * s
    return loss, dlogit


def conv_backward(x, W, dz):
    """Gradients of conv(x; W, b) given dz [cout][L]: (dx, dW, db)."""
    cin, L = x.shape
    xp = np.zeros((cin, L + 2 * PAD))
    xp[:, PAD:PAD + L] = x
    dW = np.stack([dz @ xp[:, k:k + L].T for k in range(K)], axis=2)  # [cout][cin][K]
    db = dz.sum(axis=1)
    dxp = np.zeros_like(xp)
    for k in range(K):
        dxp[:, k:k + L] += W[:, :, k].T @ dz
    return dxp[:, PAD:PAD + L], dW, db


def backward(theta, cache, dlogit):
    """Gradient of the loss with respect to theta (flat), for one block."""
    W1, b1, W2, b2, W3, b3, W4, b4, wf, bf = unpack(theta)
    dwf = dlogit * cache["h"]
    dbf = np.array([dlogit])
    dh = dlogit * wf
    z4 = cache["z"][3]
    dz = np.zeros_like(z4)
    t4 = cache["t4"]
    for c in range(C):
        if z4[c, t4[c]] > 0.0:
            dz[c, t4[c]] = dh[c]
    grads = [None] * 8
    Ws = [W1, W2, W3, W4]
    for l in range(3, -1, -1):
        dx, dW, db = conv_backward(cache["x"][l], Ws[l], dz)
        grads[2 * l], grads[2 * l + 1] = dW, db
        if l == 0:
            break
        # through maxpool4(relu(z_l)) of the layer below
        z = cache["z"][l - 1]
        arg = cache["arg"][l - 1]
        dz = np.zeros_like(z)
        cc, pp = np.meshgrid(np.arange(z.shape[0]), np.arange(z.shape[1] // POOL), indexing="ij")
        tt = POOL * pp + arg
        keep = z[cc, tt] > 0.0
        dz[cc[keep], tt[keep]] = dx[keep]
    return np.concatenate([g.ravel() for g in grads] + [dwf, dbf])


def batch_loss_grad(theta, X, y, w_pos):
    """Mean loss and gradient over blocks X [B][4096] with labels y [B]."""
    tot, g = 0.0, np.zeros_like(np.asarray(theta, dtype=np.float64))
    for x0, lab in zip(X, y):
        logit, cache = forward(theta, x0)
        loss, dl = loss_and_dlogit(logit, float(lab), w_pos)
        tot += loss
        g += backward(theta, cache, dl)
    return tot / len(X), g / len(X)
