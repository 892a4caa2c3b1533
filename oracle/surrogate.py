"""Plain FP64 oracle of the learned Voigt surrogate.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by
``tests/`` alone; it shares no code with the GPU library.

The surrogate is not part of the paper's method.  It is a small network that
stands in for the series evaluation of K(x, y) = H_V(a = y, u = x) (§2.4)
where a certification against that series shows it accurate enough; the
series remains the fallback and the measure of its error.  Definitions:

* Features: f1 = x/25 - 1, f2 = (log10 y + 1)/3 (the training domain
  x in [0, 50], y in [1e-4, 1e2] maps onto [-1, 1]^2).
* Network: four hidden layers of 64 SiLU units (SiLU(z) = z / (1 + e^-z),
  Elfwing, Uchibe & Doya 2018), one linear output.  Parameters, one flat
  binary32 vector, row-major W[out][in]:
  W1[64][2] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64][64] b4[64]
  w5[64] b5[1]  (12737 values).
* Arithmetic of the GPU network: every weight matrix is used rounded to
  bfloat16 (round to nearest even of binary32's upper 16 bits); so is every
  hidden activation that enters a 64-wide product (the inputs of layers 2-5)
  and, in the backward pass, every layer gradient dZ that enters a product;
  sums are accumulated in binary32; biases and the first layer's features
  stay binary32.  ``emulate_bf16=True`` applies the same roundings and
  computes everything else in binary64.
* Target: the plain method's K (series for x^2+y^2 < 100, the 3-node rule
  beyond, §2.4) relative to the 3-node rule G3:
      z = asinh(ln(K / G3) / tau),  tau = 1e-5,
  so that K = G3 exp(tau sinh(z)).  z = 0 wherever the plain method itself
  uses the 3-node rule; the asinh compresses the series region's large
  corrections and keeps small ones resolvable.
* Loss: mean of w(z) (z_hat - z)^2 over the batch, w(z) = 1/(1 + (z/s)^2)
  (s = 0: w = 1), which spends less of the network on the core where
  |z| is large and no certification is possible anyway.  Update: Adam (Kingma & Ba
  2015, Algorithm 1) with bias-corrected moments.
"""
from __future__ import annotations

import numpy as np

import oracle

H = 64
TAU = 1e-5
X_MAX = 50.0
LOG10_Y_MIN, LOG10_Y_MAX = -4.0, 2.0

SHAPES = [("W1", (H, 2)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
          ("b3", (H,)), ("W4", (H, H)), ("b4", (H,)), ("w5", (H,)), ("b5", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 12737


def unpack(theta) -> dict:
    """Views of the flat parameter vector, in the documented order."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(a) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via binary32; returns the
    rounded values as float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(x, y) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.stack([x / 25.0 - 1.0, (np.log10(y) + 1.0) / 3.0], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x, y, emulate_bf16: bool = True):
    """Network output z_hat for each (x, y), and the cache of the backward
    pass."""
    p = unpack(theta)
    rnd = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a = features(x, y)
    zs, ins = [], []
    z = a @ rnd(p["W1"]).T + p["b1"]
    ins.append(a)
    zs.append(z)
    h = silu(z)
    for k in (2, 3, 4):
        hin = rnd(h)
        z = hin @ rnd(p["W%d" % k]).T + p["b%d" % k]
        ins.append(hin)
        zs.append(z)
        h = silu(z)
    hin = rnd(h)
    out = hin @ rnd(p["w5"]) + p["b5"][0]
    ins.append(hin)
    return out, {"zs": zs, "ins": ins, "p": p, "rnd": rnd}


def loss_and_grad(theta, x, y, target, emulate_bf16: bool = True, wscale: float = 0.0):
    """Weighted mean squared error of the output against ``target`` --
    mean of w (z_hat - z)^2 with w = 1/(1 + (z/wscale)^2), or w = 1 for
    wscale = 0 -- and its gradient with respect to the flat parameter vector
    (the roundings of the forward pass are treated as identities, as the
    GPU's backward pass does)."""
    out, c = forward(theta, x, y, emulate_bf16)
    p, rnd, zs, ins = c["p"], c["rnd"], c["zs"], c["ins"]
    n = len(out)
    t = np.asarray(target, dtype=np.float64)
    w = 1.0 / (1.0 + (t / wscale) ** 2) if wscale > 0 else np.ones_like(t)
    r = out - t
    loss = float(np.mean(w * r * r))
    d_out = 2.0 * w * r / n
    g = {"w5": ins[4].T @ d_out, "b5": np.array([d_out.sum()])}
    dh = np.outer(d_out, rnd(p["w5"]))
    for k in (4, 3, 2):
        dz = dh * dsilu(zs[k - 1])
        dzr = rnd(dz)
        g["W%d" % k] = dzr.T @ ins[k - 1]
        g["b%d" % k] = dz.sum(axis=0)
        dh = dzr @ rnd(p["W%d" % k])
    dz = dh * dsilu(zs[0])
    g["W1"] = dz.T @ ins[0]
    g["b1"] = dz.sum(axis=0)
    return loss, pack(g)


def adam_step(theta, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step counts from 1)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def plain_K(x, y) -> np.ndarray:
    """K(x, y) by the plain method's regions (§2.4)."""
    return oracle.voigt_H(np.asarray(y, dtype=np.float64), np.asarray(x, dtype=np.float64))


def target(x, y) -> np.ndarray:
    K = plain_K(x, y)
    G3 = oracle.voigt_gh3(np.asarray(y, dtype=np.float64), np.asarray(x, dtype=np.float64))
    return np.arcsinh(np.log(K / G3) / TAU)


def reconstruct(zhat, x, y) -> np.ndarray:
    """K_hat = G3 exp(tau sinh(z_hat))."""
    G3 = oracle.voigt_gh3(np.asarray(y, dtype=np.float64), np.asarray(x, dtype=np.float64))
    return G3 * np.exp(TAU * np.sinh(np.asarray(zhat, dtype=np.float64)))
