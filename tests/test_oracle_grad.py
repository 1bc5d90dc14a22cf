"""Pins of the reference gradient: central finite differences of the C oracle's
continuous NLL (FP64) against torch-FP64 autograd of the independent torch
formulation, on the tiny model (8x8x3 images, h=3, C=8, one block)."""
import numpy as np
import torch

import oracle
import synth
from oracle import torch_ref


def test_nll_agrees_between_formulations():
    d = synth.MODEL_DIMS["tiny"]
    p = synth.init_params(d["h"], d["C"], d["n_blocks"], d["seed"]).astype(np.float64)
    imgs = np.stack([synth.smooth_field_image(2.0, 3, 0, 8, 8, 500 + k) for k in range(3)])
    bits, _ = torch_ref.nll_grad(p, d["h"], d["C"], d["n_blocks"], imgs)
    m = oracle.Model.from_params(d["h"], d["C"], d["n_blocks"], p)
    for k in range(3):
        assert abs(m.stats(imgs[k])["cbits"] - float(bits[k])) <= 1e-10 * float(bits[k])


def test_finite_differences_match_autograd():
    d = synth.MODEL_DIMS["tiny"]
    h, C, nb = d["h"], d["C"], d["n_blocks"]
    p = synth.init_params(h, C, nb, d["seed"]).astype(np.float64)
    img = synth.smooth_field_image(2.0, 3, 0, 8, 8, 600)
    _, g = torch_ref.nll_grad(p, h, C, nb, img[None])
    g = g.numpy()

    def f(q):
        return oracle.Model.from_params(h, C, nb, q).stats(img)["cbits"]

    # fourth-order central differences (five-point stencil): truncation error
    # O(e^4), rounding error ~ 1e-16 |f| / e
    fd = np.zeros_like(p)
    for k in range(p.size):
        e = 1e-4 * max(1.0, abs(p[k]))
        vals = []
        for s in (2, 1, -1, -2):
            q = p.copy()
            q[k] += s * e
            vals.append(f(q))
        f2, f1, m1, m2 = vals
        fd[k] = (-f2 + 8 * f1 - 8 * m1 + m2) / (12 * e)
    # masked taps of the first kernel have exactly zero gradient in both
    K = 2 * h + 1
    conv = g[:C * 3 * K * K].reshape(C, 3, K, K)
    for dy in range(K):
        for dx in range(K):
            if not oracle.tap_live(h, dy, dx):
                assert np.all(conv[:, :, dy, dx] == 0.0)
    err = np.linalg.norm(fd - g) / np.linalg.norm(g)
    assert err < 1e-8, err
    assert np.abs(fd - g).max() <= 1e-8 * np.abs(g).max()
