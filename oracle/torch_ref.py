"""Torch FP64 reference of the local model and its continuous NLL (CPU only).

TEST INFRASTRUCTURE ONLY: a second, independent formulation used to pin the
C oracle's network (via torch's own conv2d) and to provide reference
gradients (via autograd). It writes the joint mixture likelihood directly,

    p(r, g, b) = sum_m w_m P_m(r) P_m(g | r) P_m(b | r, g),

whereas the C oracle telescopes it into per-channel posteriors; agreement of
the two pins that factorisation.

Layer structure (Sec. 2.1: masked first convolution, then 1x1 layers):
a = conv_masked(x) + b; per block a += W2 elu(W1 elu(a) + b1) + b2;
theta = Wh elu(a) + bh. Inputs are normalised as v/127.5 - 1 and zero
padded (Eq. 3).
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as F

NMIX = 10


def causal_mask(h: int, dtype=torch.float64) -> torch.Tensor:
    """(2h+1)x(2h+1) mask of the taps pixel (i, j) may read (Eq. 3)."""
    K = 2 * h + 1
    m = torch.zeros(K, K, dtype=dtype)
    m[:h, :] = 1.0          # the h rows above, columns j-h..j+h
    m[h, :h] = 1.0          # own row, the h columns to the left
    return m


def split_params(params: torch.Tensor, h: int, C: int, n_blocks: int):
    K = 2 * h + 1
    out, o = {}, 0

    def take(name, shape):
        nonlocal o
        n = 1
        for s in shape:
            n *= s
        out[name] = params[o:o + n].reshape(shape)
        o += n

    take("conv_w", (C, 3, K, K))
    take("conv_b", (C,))
    for b in range(n_blocks):
        take(f"w1_{b}", (C, C))
        take(f"b1_{b}", (C,))
        take(f"w2_{b}", (C, C))
        take(f"b2_{b}", (C,))
    take("head_w", (10 * NMIX, C))
    take("head_b", (10 * NMIX,))
    assert o == params.numel()
    return out


def theta(params: torch.Tensor, h: int, C: int, n_blocks: int, imgs: torch.Tensor) -> torch.Tensor:
    """imgs: (N, H, W, 3) uint8 -> theta (N, H, W, 100) in the params' dtype."""
    P = split_params(params, h, C, n_blocks)
    x = imgs.to(params.dtype).permute(0, 3, 1, 2) / 127.5 - 1.0
    w = P["conv_w"] * causal_mask(h, params.dtype)
    a = F.conv2d(x, w, P["conv_b"], padding=h)
    for b in range(n_blocks):
        z = F.conv2d(F.elu(a), P[f"w1_{b}"][:, :, None, None], P[f"b1_{b}"])
        a = a + F.conv2d(F.elu(z), P[f"w2_{b}"][:, :, None, None], P[f"b2_{b}"])
    t = F.conv2d(F.elu(a), P["head_w"][:, :, None, None], P["head_b"])
    return t.permute(0, 2, 3, 1)


def _log_bin(v: torch.Tensor, mu: torch.Tensor, invs: torch.Tensor) -> torch.Tensor:
    """log P(symbol v) under logistic(mu, 1/invs) discretised to bins
    [(2v-256)/255, (2v-254)/255), open-ended at v = 0 and v = 255."""
    lo = (2.0 * v - 256.0) / 255.0
    hi = (2.0 * v - 254.0) / 255.0
    zlo = (lo - mu) * invs
    zhi = (hi - mu) * invs
    mid = F.logsigmoid(zhi) + F.logsigmoid(-zlo) + torch.log(-torch.expm1(zlo - zhi))
    first = F.logsigmoid(zhi)
    last = F.logsigmoid(-zlo)
    return torch.where(v <= 0, first, torch.where(v >= 255, last, mid))


def joint_log_prob(th: torch.Tensor, imgs: torch.Tensor) -> torch.Tensor:
    """Natural-log joint probability of each pixel, shape (N, H, W)."""
    x = imgs.to(th.dtype)
    xn = x / 127.5 - 1.0
    logit = th[..., 0:10]
    mu = [th[..., 10 + 10 * c:20 + 10 * c] for c in range(3)]
    ls = [torch.clamp(th[..., 40 + 10 * c:50 + 10 * c], min=-7.0) for c in range(3)]
    al, be, ga = torch.tanh(th[..., 70:80]), torch.tanh(th[..., 80:90]), torch.tanh(th[..., 90:100])
    r, g, b = x[..., 0:1], x[..., 1:2], x[..., 2:3]
    rn, gn = xn[..., 0:1], xn[..., 1:2]
    mr = mu[0]
    mg = mu[1] + al * rn
    mb = mu[2] + be * rn + ga * gn
    lw = torch.log_softmax(logit, dim=-1)
    lp = (lw + _log_bin(r, mr, torch.exp(-ls[0])) + _log_bin(g, mg, torch.exp(-ls[1]))
          + _log_bin(b, mb, torch.exp(-ls[2])))
    return torch.logsumexp(lp, dim=-1)


def nll_bits(params: torch.Tensor, h: int, C: int, n_blocks: int, imgs: torch.Tensor) -> torch.Tensor:
    """Continuous code length of each image in bits, shape (N,)."""
    th = theta(params, h, C, n_blocks, imgs)
    return -joint_log_prob(th, imgs).sum(dim=(1, 2)) / math.log(2.0)


def nll_grad(params, h, C, n_blocks, imgs, weights=None):
    """(bits per image, d(sum_n weights_n * bits_n)/d params), FP64 on CPU."""
    p = torch.as_tensor(params, dtype=torch.float64).clone().requires_grad_(True)
    im = torch.as_tensor(imgs)
    bits = nll_bits(p, h, C, n_blocks, im)
    wts = torch.ones_like(bits) if weights is None else torch.as_tensor(weights, dtype=torch.float64)
    (bits * wts).sum().backward()
    return bits.detach(), p.grad.detach()
