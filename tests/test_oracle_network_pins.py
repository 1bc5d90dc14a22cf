"""Closed-form pins of the oracle's network body (Eq. 3 and the model of
Sec. 2.1: masked convolution, residual blocks of two 1x1 layers with ELU, 1x1
head), which the paper describes in words only.

Special weights reduce the network to values computed here by hand from the
ELU's definition (elu(v) = v for v > 0, e^v - 1 otherwise) and the input
scaling v / 127.5 - 1, so a dropped residual, a missing or misplaced ELU, a
bias added in the wrong place or a conv tap read from the wrong neighbour
fails one of them.
"""
import math

import numpy as np
import pytest

import oracle
import synth

H_, C_ = 3, 8


def params(nb, **named):
    """Flat parameter vector of an h = 3, C = 8 model with nb blocks: every
    tensor zero except the named ones (arrays, or scalars broadcast)."""
    out = []
    for name, shape in synth.param_shapes(H_, C_, nb):
        t = np.zeros(shape, dtype=np.float64)
        if name in named:
            t[...] = named[name]
        out.append(t.ravel())
    return np.concatenate(out)


def theta(p, nb, img):
    return oracle.Model.from_params(H_, C_, nb, p).theta_image(img)


def image(seed, H=6, W=7):
    return np.random.default_rng(seed).integers(0, 256, size=(H, W, 3), dtype=np.uint8)


def head(seed, col=None):
    """A head weight matrix (100 x C) and bias; col keeps one input channel."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(-1.0, 1.0, size=(100, C_))
    if col is not None:
        w[:, [c for c in range(C_) if c != col]] = 0.0
    return w, rng.uniform(-1.0, 1.0, size=100)


def test_zero_weights_give_the_head_bias():
    """With every weight zero the logits at every pixel are the head bias,
    whatever the biases of the layers below."""
    hw, hb = head(1)
    rng = np.random.default_rng(2)
    p = params(2, conv_b=rng.uniform(-1, 1, C_), b1_0=rng.uniform(-1, 1, C_), b2_0=rng.uniform(-1, 1, C_),
               b1_1=rng.uniform(-1, 1, C_), b2_1=rng.uniform(-1, 1, C_), head_b=hb)
    th = theta(p, 2, image(3))
    assert np.array_equal(th, np.broadcast_to(hb, th.shape))


def test_negative_branch_of_the_elu_before_the_head():
    """No blocks, conv bias -1: the head sees elu(-1) = e^-1 - 1 on every
    channel."""
    hw, hb = head(4)
    th = theta(params(0, conv_b=-1.0, head_w=hw, head_b=hb), 0, image(5))
    want = hw.sum(axis=1) * (math.exp(-1.0) - 1.0) + hb
    assert np.allclose(th, np.broadcast_to(want, th.shape), rtol=0, atol=1e-14)


def test_residual_adds_the_second_bias_of_every_block():
    """Both layers of two blocks with zero weights: a = conv bias + b2_0 + b2_1
    (the first biases only reach the head through the zero second layers),
    here -1 + 2 + 0.5 = 1.5 > 0, where the ELU is the identity."""
    hw, hb = head(6)
    p = params(2, conv_b=-1.0, b1_0=3.0, b2_0=2.0, b1_1=-4.0, b2_1=0.5, head_w=hw, head_b=hb)
    th = theta(p, 2, image(7))
    want = hw.sum(axis=1) * 1.5 + hb
    assert np.allclose(th, np.broadcast_to(want, th.shape), rtol=0, atol=1e-14)


def test_first_layer_of_a_block_acts_only_through_the_second():
    """With the second layer zero, the first layer's weights and bias do not
    change the logits at all (bitwise)."""
    hw, hb = head(8)
    rng = np.random.default_rng(9)
    base = dict(conv_w=rng.uniform(-0.3, 0.3, (C_, 3, 7, 7)), conv_b=rng.uniform(-1, 1, C_), head_w=hw, head_b=hb)
    a = theta(params(1, **base), 1, image(10))
    b = theta(params(1, w1_0=rng.uniform(-1, 1, (C_, C_)), b1_0=rng.uniform(-1, 1, C_), **base), 1, image(10))
    assert np.array_equal(a, b)


def test_elu_on_each_side_of_the_first_block_layer():
    """Identity 1x1 weights and conv bias -1: the block computes
    a1 = -1 + elu(elu(-1)), and the head sees elu(a1). Dropping any one ELU
    (block input, between the layers, head input) or the residual changes
    the value; scaling the second layer by 2 scales its term of a1."""
    hw, hb = head(11)
    eye = np.eye(C_)

    def elu(v):
        return v if v > 0 else math.exp(v) - 1.0

    for scale in (1.0, 2.0):
        p = params(1, conv_b=-1.0, w1_0=eye, w2_0=scale * eye, head_w=hw, head_b=hb)
        th = theta(p, 1, image(12))
        a1 = -1.0 + scale * elu(elu(-1.0))
        want = hw.sum(axis=1) * elu(a1) + hb
        assert np.allclose(th, np.broadcast_to(want, th.shape), rtol=0, atol=1e-14), scale


def test_block_weights_route_channel_to_channel():
    """Conv biases 0.5 + 0.1 c (all positive, so the ELUs pass them), a first
    layer with the single weight W1[1][0] = 1 and a second with W2[2][1] = 1:
    channel 0 feeds channel 1, which adds to channel 2, so a1[2] = 0.7 + 0.5
    while every other channel keeps its bias. A transposed weight index
    routes nothing to channel 2."""
    hw, hb = head(15, col=2)
    w1 = np.zeros((C_, C_))
    w1[1, 0] = 1.0
    w2 = np.zeros((C_, C_))
    w2[2, 1] = 1.0
    cb = 0.5 + 0.1 * np.arange(C_)
    th = theta(params(1, conv_b=cb, w1_0=w1, w2_0=w2, head_w=hw, head_b=hb), 1, image(16))
    want = hw[:, 2] * (0.7 + 0.5) + hb
    assert np.allclose(th, np.broadcast_to(want, th.shape), rtol=0, atol=1e-14)


@pytest.mark.parametrize("dy,dx,ch", [(2, 3, 0), (3, 2, 1), (0, 6, 2), (3, 0, 0)])
def test_single_conv_tap_reads_its_neighbour(dy, dx, ch):
    """One live conv tap (kernel row dy, column dx, colour ch) with weight 1
    on channel 0: pixel (i, j) sees the scaled value of pixel
    (i - 3 + dy, j - 3 + dx), colour ch, or 0 outside the image, through the
    ELU; the head keeps channel 0 only."""
    assert dy < 3 or dx < 3  # a live (causal) tap of the h = 3 kernel
    hw, hb = head(13, col=0)
    cw = np.zeros((C_, 3, 7, 7))
    cw[0, ch, dy, dx] = 1.0
    img = image(14, 7, 9)
    th = theta(params(0, conv_w=cw, head_w=hw, head_b=hb), 0, img)
    H, W, _ = img.shape
    for i in range(H):
        for j in range(W):
            y, x = i - 3 + dy, j - 3 + dx
            v = img[y, x, ch] / 127.5 - 1.0 if 0 <= y < H and 0 <= x < W else 0.0
            u = v if v > 0 else math.exp(v) - 1.0
            assert np.allclose(th[i, j], hw[:, 0] * u + hb, rtol=0, atol=1e-14), (i, j)
