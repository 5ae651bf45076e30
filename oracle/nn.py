"""CPU oracle of the learned whole-lattice proposal (test infrastructure only).

Plain numpy in float64.  The model is an autoregressive network over the
spins of an L x L lattice in raster order (site i = y L + x): masked 3x3
convolutions with zero padding, so that the logit z_i of
q(s_i = +1 | s_<i) = sigmoid(z_i) depends only on earlier sites.

  layer 1: mask A (taps above-left, above, above-right, left), 1 -> C, ReLU
  layer 2: mask B (mask A plus the centre tap), C -> C, ReLU
  layer 3: mask B, C -> C, ReLU
  layer 4: mask B, C -> 1, the logits z

log q(s) = sum_i log sigmoid(s_i z_i).  Parameters are one flat vector:
for each layer, W[out][in][tap] then b[out].  Only tests, smoke() and the
benchmark's CPU baseline may import this module.
"""
from __future__ import annotations

import numpy as np

# taps (dy, dx) of the two masks, in this order
TAPS_A = ((-1, -1), (-1, 0), (-1, 1), (0, -1))
TAPS_B = TAPS_A + ((0, 0),)


def layers(C: int):
    """(in, out, taps) of the four layers."""
    return ((1, C, TAPS_A), (C, C, TAPS_B), (C, C, TAPS_B), (C, 1, TAPS_B))


def param_count(C: int) -> int:
    return sum(co * ci * len(t) + co for ci, co, t in layers(C))


def unpack(params: np.ndarray, C: int):
    """[(W [out, in, taps], b [out]), ...] views of the flat vector."""
    out, o = [], 0
    for ci, co, taps in layers(C):
        nW = co * ci * len(taps)
        out.append((params[o:o + nW].reshape(co, ci, len(taps)), params[o + nW:o + nW + co]))
        o += nW + co
    return out


def shifted(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """y[..., r, c] = x[..., r + dy, c + dx], zero outside the lattice."""
    y = np.zeros_like(x)
    H, W = x.shape[-2:]
    r0, r1 = max(0, -dy), min(H, H - dy)
    c0, c1 = max(0, -dx), min(W, W - dx)
    y[..., r0:r1, c0:c1] = x[..., r0 + dy:r1 + dy, c0 + dx:c1 + dx]
    return y


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray, taps) -> np.ndarray:
    """Masked convolution: x [B, in, L, L] -> [B, out, L, L]."""
    out = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for t, (dy, dx) in enumerate(taps):
        out += np.einsum("oi,bihw->bohw", W[:, :, t], shifted(x, dy, dx))
    return out + b[None, :, None, None]


def forward(params: np.ndarray, s: np.ndarray, C: int):
    """Logits z [B, L, L] and the post-ReLU hidden maps [h1, h2, h3]."""
    x = s.astype(np.float64)[:, None]
    hs = []
    for li, ((W, b), (_, _, taps)) in enumerate(zip(unpack(params, C), layers(C))):
        x = conv(x, W, b, taps)
        if li < 3:
            x = np.maximum(x, 0.0)
            hs.append(x)
    return x[:, 0], hs


def log_sigmoid(v: np.ndarray) -> np.ndarray:
    return -np.logaddexp(0.0, -v)


def logq(params: np.ndarray, s: np.ndarray, C: int) -> np.ndarray:
    """log q(s) of each configuration of s [B, L, L] (+1/-1)."""
    z, _ = forward(params, s, C)
    return log_sigmoid(s * z).sum(axis=(1, 2))


def loss_and_grad(params: np.ndarray, s: np.ndarray, C: int):
    """Mean negative log-likelihood over the batch and its gradient with
    respect to the flat parameter vector (backpropagation by hand)."""
    B = s.shape[0]
    sf = s.astype(np.float64)
    z, hs = forward(params, s, C)
    loss = -log_sigmoid(sf * z).sum() / B
    # d(-log sigmoid(s z))/dz = -s sigmoid(-s z)
    g = (-sf / (1.0 + np.exp(sf * z)))[:, None] / B
    ins = [sf[:, None]] + hs
    grads = []
    for li in (3, 2, 1, 0):
        W, _ = unpack(params, C)[li]
        taps = layers(C)[li][2]
        x = ins[li]
        gW = np.zeros_like(W)
        for t, (dy, dx) in enumerate(taps):
            gW[:, :, t] = np.einsum("bohw,bihw->oi", g, shifted(x, dy, dx))
        gb = g.sum(axis=(0, 2, 3))
        grads.append((gW, gb))
        if li == 0:
            break
        gx = np.zeros_like(x)
        for t, (dy, dx) in enumerate(taps):
            # out[p] uses x[p + d]: the gradient flows back to x[q] from out[q - d]
            gx += shifted(np.einsum("oi,bohw->bihw", W[:, :, t], g), -dy, -dx)
        g = gx * (x > 0)
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb]
    return loss, np.concatenate(flat)


def sample(params: np.ndarray, r: np.ndarray, L: int, C: int):
    """Draw configurations site by site in raster order: s_i = +1 iff
    r_i < q(s_i = +1 | s_<i) 2^32, with r [B, L*L] uint32 given.  Returns
    (s [B, L, L] int8, log q(s)).  Slow and plain: the whole network is
    re-evaluated for every site."""
    B = r.shape[0]
    s = np.zeros((B, L, L), dtype=np.int8)
    for i in range(L * L):
        y, x = divmod(i, L)
        z, _ = forward(params, s, C)
        p = 1.0 / (1.0 + np.exp(-z[:, y, x]))
        s[:, y, x] = np.where(r[:, i].astype(np.float64) < p * 4294967296.0, 1, -1)
    return s, logq(params, s, C)


def adam_step(params, m, v, grad, step: int, lr: float, b1: float, b2: float, eps: float):
    """One Adam update (Kingma and Ba) with bias correction; returns new
    (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def mh_log_ratio(beta: float, E_cur, E_prop, logq_cur, logq_prop):
    """log of the acceptance ratio of an independent proposal s' ~ q for the
    Boltzmann weight exp(-beta E): -beta (E' - E) + log q(s) - log q(s')."""
    return -beta * (np.asarray(E_prop, np.float64) - np.asarray(E_cur, np.float64)) + \
        np.asarray(logq_cur, np.float64) - np.asarray(logq_prop, np.float64)


def logq_sym(params: np.ndarray, s: np.ndarray, C: int) -> np.ndarray:
    """log of the Z2-symmetrised proposal q_sym(s) = (q(s) + q(-s)) / 2:
    sample from q, then negate the whole configuration with probability 1/2."""
    return np.logaddexp(logq(params, s, C), logq(params, -s, C)) - np.log(2.0)
