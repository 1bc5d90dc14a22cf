"""GPU parity of the training objective and its hand-written gradient.

The HIP path (nellox_nll_fwd_train / nellox_nll_bwd through the C ABI)
against the FP64 torch reference (oracle/torch_ref.py, itself pinned to
finite differences and to the C oracle on the CPU). Bars: code length
within 1e-5 relative per image and per pixel (with a floor of 1e-5 bits);
gradient within 1e-4 relative: the norm of the difference over the norm of
the reference, over the whole vector and per tensor, and every element
within 1e-4 |g| + 1e-6 max |g|.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import torch_ref

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4
BITS_TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tr():
    from paper_2201_05213_amd import blob, train

    torch.cuda.set_device(0)
    return train, blob


def model(name, blob):
    b, _ = synth.model_blob(name)
    return blob.params_from_blob(b)


def crops(n, side, seed):
    pool = synth.training_pool(n=32)
    return synth.training_crops(pool, n, side, np.random.Generator(np.random.PCG64(seed)))


def gpu_bits_grad(train, dims, params, imgs, weights):
    p = torch.from_numpy(params).cuda().requires_grad_(True)
    x = torch.from_numpy(np.ascontiguousarray(imgs)).cuda()
    bits = train.nll_bits(p, dims, x)
    (bits * torch.as_tensor(weights, dtype=torch.float64, device="cuda")).sum().backward()
    torch.cuda.synchronize()
    return bits.detach().cpu().numpy(), p.grad.detach().cpu().numpy().astype(np.float64)


def ref_bits_grad(dims, params, imgs, weights):
    h, C, nb, _ = dims
    bits, g = torch_ref.nll_grad(torch.from_numpy(params.astype(np.float64)), h, C, nb,
                                 torch.from_numpy(np.ascontiguousarray(imgs)), weights)
    return bits.numpy(), g.numpy()


def tensor_slices(dims):
    h, C, nb, _ = dims
    K = 2 * h + 1
    out, o = [], 0
    for name, n in [("conv_w", C * 3 * K * K), ("conv_b", C)] + \
            sum([[(f"w1_{b}", C * C), (f"b1_{b}", C), (f"w2_{b}", C * C), (f"b2_{b}", C)] for b in range(nb)], []) + \
            [("head_w", 100 * C), ("head_b", 100)]:
        out.append((name, slice(o, o + n)))
        o += n
    return out


def compare(dims, params, imgs, weights, tr, label):
    train, _ = tr
    gb, gg = gpu_bits_grad(train, dims, params, imgs, weights)
    rb, rg = ref_bits_grad(dims, params, imgs, weights)
    bits_err = float(np.max(np.abs(gb - rb) / np.abs(rb)))
    err = float(np.linalg.norm(gg - rg) / np.linalg.norm(rg))
    per = {n: float(np.linalg.norm(gg[s] - rg[s]) / max(np.linalg.norm(rg[s]), 1e-300)) for n, s in tensor_slices(dims)}
    worst = max(per.items(), key=lambda kv: kv[1])
    say(f"[gpu] {label}: bits rel {bits_err:.2e}, grad rel {err:.2e}, worst tensor {worst[0]} {worst[1]:.2e}")
    assert bits_err <= BITS_TOL
    assert err <= GRAD_TOL
    for n, e in per.items():
        assert e <= GRAD_TOL, (n, e)
    # element by element: an error confined to small weights cannot hide in a norm
    bound = GRAD_TOL * np.abs(rg) + 1e-6 * np.abs(rg).max()
    bad = np.abs(gg - rg) > bound
    say(f"  per element: worst |diff| / bound {float((np.abs(gg - rg) / bound).max()):.3f}")
    assert not bad.any(), (int(bad.sum()), np.flatnonzero(bad)[:8])
    # per-pixel code length of the training forward against the FP64 joint likelihood
    h, C, nb, _ = dims
    pxg = train.nll_bits_per_px(torch.from_numpy(params).cuda(), dims,
                                torch.from_numpy(np.ascontiguousarray(imgs)).cuda()).cpu().numpy().astype(np.float64)
    with torch.no_grad():
        x = torch.from_numpy(np.ascontiguousarray(imgs))
        th = torch_ref.theta(torch.from_numpy(params.astype(np.float64)), h, C, nb, x)
        pxr = (-torch_ref.joint_log_prob(th, x) / np.log(2.0)).numpy()
    perr = np.abs(pxg - pxr)
    assert np.all(perr <= BITS_TOL * np.abs(pxr) + 1e-5), float(perr.max())
    # masked taps of the first kernel get no gradient
    h, C, _, _ = dims
    K = 2 * h + 1
    m = torch_ref.causal_mask(h).numpy().astype(bool)
    cw = gg[:C * 3 * K * K].reshape(C, 3, K, K)
    assert np.all(cw[:, :, ~m] == 0.0)
    return gg


def test_grad_tiny_8x8(tr):
    """Gradient check on the tiny model (8x8x3 images, h=3, C=8, one block)."""
    say("[gpu] train: tiny model, 2 images 8x8")
    _, blob = tr
    dims, params = model("tiny", blob)
    imgs = crops(2, 8, 7)
    compare(dims, params, imgs, [1.0, 1.0], tr, "tiny 2x8x8")
    # per-image weights of the loss
    compare(dims, params, imgs, [0.25, -1.5], tr, "tiny weighted")


def test_grad_tiny_edge_values(tr):
    """Pixels at 0 and 255 (edge bins) and a ragged tile (W = 5)."""
    say("[gpu] train: tiny model, edge values, 3 images 6x5")
    _, blob = tr
    dims, params = model("tiny", blob)
    rng = np.random.default_rng(3)
    imgs = rng.choice(np.array([0, 1, 2, 127, 128, 253, 254, 255], dtype=np.uint8), size=(3, 6, 5, 3))
    compare(dims, params, imgs, [1.0, 2.0, 0.5], tr, "tiny edge values")


@pytest.mark.parametrize("name", ["A", "C"])
def test_grad_models_A_C(tr, name):
    say(f"[gpu] train: model {name}, 8 crops 32x32")
    _, blob = tr
    dims, params = model(name, blob)
    compare(dims, params, crops(8, 32, 11), np.ones(8), tr, f"model {name} 8x32x32")


def test_grad_model_B_training_batch(tr):
    """The training configuration: model B, 64 random 32x32 crops."""
    say("[gpu] train: model B, 64 crops 32x32")
    _, blob = tr
    dims, params = model("B", blob)
    compare(dims, params, crops(64, 32, 5_999_999), np.ones(64), tr, "model B 64x32x32")


def test_grad_large_batch_is_sum_of_its_halves(tr):
    """Linearity past the training batch, where the oracle would be slow: 96
    synthetic 64x64 images (393,216 px, so the weight-gradient launch runs
    long chunks) and the same images in two halves of 48. Each image's code
    length is a sum over its own pixels, so the per-image bits must agree
    bitwise; the weighted gradient of the whole batch must equal the sum of
    the halves' gradients up to FP32 summation order, within
    1e-4 |g| + 1e-5 max |g| per element."""
    train, blob = tr
    dims, params = model("B", blob)
    imgs = synth.training_pool(n=96)
    w = np.random.default_rng(17).uniform(0.5, 1.5, size=96)
    say("[gpu] train: model B, 96 images 64x64 against its two halves")
    b_all, g_all = gpu_bits_grad(train, dims, params, imgs, w)
    b_lo, g_lo = gpu_bits_grad(train, dims, params, imgs[:48], w[:48])
    b_hi, g_hi = gpu_bits_grad(train, dims, params, imgs[48:], w[48:])
    assert np.array_equal(b_all, np.concatenate([b_lo, b_hi]))
    g_sum = g_lo + g_hi
    bound = GRAD_TOL * np.abs(g_sum) + 1e-5 * np.abs(g_sum).max()
    worst = float((np.abs(g_all - g_sum) / bound).max())
    say(f"  worst |diff| / bound {worst:.3f}")
    assert worst <= 1.0


def test_graph_replays_match_eager(tr):
    """Forward and backward captured once in a HIP graph (torch.cuda.graph)
    and replayed on new crops copied into its input buffer give bitwise the
    bits and the gradient of eager calls on the same crops. Eager work and a
    synchronisation run between the replays."""
    train, blob = tr
    dims, params = model("A", blob)
    p = torch.from_numpy(params).cuda().requires_grad_(True)
    batches = [torch.from_numpy(crops(8, 32, 100 + k)).cuda() for k in range(4)]
    w = torch.linspace(0.5, 1.5, 8, dtype=torch.float64, device="cuda")

    def eager(x):
        q = p.detach().clone().requires_grad_(True)
        bits = train.nll_bits(q, dims, x)
        (bits * w).sum().backward()
        return bits.detach().clone(), q.grad.detach().clone()

    ref = [eager(x) for x in batches]
    static_x = batches[0].clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            p.grad = None
            (train.nll_bits(p, dims, static_x) * w).sum().backward()
    torch.cuda.current_stream().wait_stream(side)
    p.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        static_bits = train.nll_bits(p, dims, static_x)
        (static_bits * w).sum().backward()
    say("[gpu] train: graph captured, replaying")
    for k in (1, 3, 0, 2):
        static_x.copy_(batches[k])
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(static_bits, ref[k][0]), k
        assert torch.equal(p.grad, ref[k][1]), k
        eager(batches[(k + 1) % 4])
        torch.cuda.synchronize()


def test_graph_training_steps_match_eager(tr):
    """Whole Adam steps (forward, backward, torch's fused Adam with
    capturable state) captured once as a graph: after three eager warm-up
    steps on a side stream and five replays on new crops, the parameters
    equal bitwise those of eight eager steps on the same crops."""
    train, blob = tr
    dims, params = model("A", blob)
    batches = [torch.from_numpy(crops(8, 32, 200 + k)).cuda() for k in range(8)]
    p = torch.nn.Parameter(torch.from_numpy(params).cuda())
    opt = torch.optim.Adam([p], lr=1e-3, fused=True)
    for x in batches:
        opt.zero_grad(set_to_none=True)
        (train.nll_bits(p, dims, x).sum() / x.numel()).backward()
        opt.step()
    pg = torch.nn.Parameter(torch.from_numpy(params).cuda())
    optg = torch.optim.Adam([pg], lr=1e-3, fused=True, capturable=True)
    sx = batches[0].clone()

    def body():
        (train.nll_bits(pg, dims, sx).sum() / sx.numel()).backward()
        optg.step()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for x in batches[:3]:
            sx.copy_(x)
            optg.zero_grad(set_to_none=True)
            body()
    torch.cuda.current_stream().wait_stream(side)
    optg.zero_grad(set_to_none=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        body()
    for x in batches[3:]:
        sx.copy_(x)
        graph.replay()
        torch.cuda.synchronize()
    assert torch.equal(pg.detach(), p.detach())


def test_backward_is_deterministic(tr):
    say("[gpu] train: determinism")
    train, blob = tr
    dims, params = model("A", blob)
    imgs = crops(16, 32, 1)
    g1 = gpu_bits_grad(train, dims, params, imgs, np.ones(16))[1]
    g2 = gpu_bits_grad(train, dims, params, imgs, np.ones(16))[1]
    assert np.array_equal(g1, g2)


def test_train_2000_adam_steps(tr):
    """The training configuration end to end: model B, 2000 Adam steps at
    lr 1e-3 on 64 random 32x32 crops per step from a pool of 512 synthetic
    64x64 images; bits/dim of 64 held-out images must drop."""
    say("[gpu] train: model B, 2000 Adam steps")
    train, blob = tr
    dims, params = model("B", blob)
    pool = torch.from_numpy(synth.training_pool(n=512)).cuda()
    held = torch.from_numpy(synth.training_pool(n=64, seed_base=5_500_000)).cuda()
    p0 = torch.from_numpy(params).cuda()
    before = train.bits_per_dim(p0, dims, held)
    p = train.fit(p0, dims, pool, 2000, np.random.Generator(np.random.PCG64(5_999_999)))
    after = train.bits_per_dim(p, dims, held)
    say(f"[gpu] model B held-out bits/dim {before:.4f} -> {after:.4f} after 2000 steps")
    assert np.isfinite(after) and after < before - 2.0


def test_adam_lowers_bits(tr):
    """A short run of Adam on the code length lowers bits/dim of held-out crops."""
    say("[gpu] train: 60 Adam steps, model A")
    train, blob = tr
    dims, params = model("A", blob)
    pool = synth.training_pool(n=64)
    rng = np.random.Generator(np.random.PCG64(5_999_999))
    held = torch.from_numpy(synth.training_crops(pool, 16, 32, np.random.default_rng(9))).cuda()
    p = torch.nn.Parameter(torch.from_numpy(params).cuda())
    opt = torch.optim.Adam([p], lr=1e-3)

    def bpd():
        with torch.no_grad():
            return float(train.nll_bits(p, dims, held).sum()) / (held.numel())

    before = bpd()
    for _ in range(60):
        x = torch.from_numpy(synth.training_crops(pool, 32, 32, rng)).cuda()
        opt.zero_grad()
        loss = train.nll_bits(p, dims, x).sum() / x.numel()
        loss.backward()
        opt.step()
    after = bpd()
    say(f"[gpu] bits/dim {before:.4f} -> {after:.4f}")
    assert after < before - 0.5
