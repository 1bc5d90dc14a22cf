"""Training the local model on its own code length (Eq. 2, Sec. 2.1).

`nll_bits(params, dims, imgs)` is the continuous code length -log2 p(x) of
each image, differentiable in `params` through a hand-written backward (the
mixture-logistic NLL and every layer down to the masked first convolution,
in the HIP library). `params` is the flat FP32 vector in the weight blob's
tensor order; `blob.params_from_blob` / `blob.blob_from_params` convert.

    dims = (h, C, n_blocks, 10)
    p = torch.nn.Parameter(torch.from_numpy(params).cuda())
    opt = torch.optim.Adam([p], lr=1e-3, fused=True)
    bits = nll_bits(p, dims, crops)          # crops: (N, H, W, 3) uint8 on the GPU
    (bits.sum() / crops[..., 0].numel() / 3).backward(); opt.step()

A whole step (forward, backward and a capturable Adam) can be captured once
with torch.cuda.graph and replayed on new crops copied into its input
tensor: the library's calls make no host synchronisation and allocate
through torch, and replays give bitwise the eager step's parameters.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import NelloxError, check, load

__all__ = ["param_count", "nll_bits", "nll_bits_per_px", "NLLFunction", "random_crops", "bits_per_dim", "fit"]


def _dims(dims) -> ctypes.Array:
    d = (ctypes.c_int32 * 4)(*[int(v) for v in dims])
    return d


def param_count(dims) -> int:
    n = load().nellox_param_count(_dims(dims))
    if n < 0:
        raise ValueError(f"invalid model dims {tuple(dims)}")
    return int(n)


def _check_inputs(params: torch.Tensor, dims, imgs: torch.Tensor):
    if params.dtype != torch.float32 or not params.is_cuda or params.dim() != 1 or not params.is_contiguous():
        raise ValueError("params must be a contiguous 1-D float32 CUDA tensor")
    if params.numel() != param_count(dims):
        raise ValueError(f"params has {params.numel()} entries, the model needs {param_count(dims)}")
    if imgs.dtype != torch.uint8 or imgs.dim() != 4 or imgs.shape[3] != 3 or not imgs.is_cuda \
            or not imgs.is_contiguous():
        raise ValueError("imgs must be a contiguous (N, H, W, 3) uint8 CUDA tensor")


class NLLFunction(torch.autograd.Function):
    """bits (N,) float64 = -log2 p(imgs[k]); backward: d/d params (FP32)."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, dims, imgs: torch.Tensor):
        _check_inputs(params, dims, imgs)
        L = load()
        n, H, W = (int(v) for v in imgs.shape[:3])
        d = _dims(dims)
        nb = L.nellox_train_workspace_bytes(d, n, H, W)
        if nb == 0:
            raise NelloxError(1, "nellox_train_workspace_bytes")
        ws = torch.empty(nb, dtype=torch.uint8, device=params.device)
        bits = torch.empty(n, dtype=torch.float64, device=params.device)
        stream = ctypes.c_void_p(torch.cuda.current_stream(params.device).cuda_stream)
        check(L.nellox_nll_fwd_train(params.data_ptr(), d, imgs.data_ptr(), n, H, W, bits.data_ptr(), None,
                                     ws.data_ptr(), ws.numel(), stream), "nellox_nll_fwd_train")
        ctx.save_for_backward(params, imgs)
        ctx.dims = tuple(int(v) for v in dims)
        ctx.ws = ws
        return bits

    @staticmethod
    def backward(ctx, grad_bits: torch.Tensor):
        if ctx.ws is None:
            # the workspace holding the forward's activations is released
            # after the first backward
            raise RuntimeError("nll_bits: a second backward through the same graph is not supported")
        params, imgs = ctx.saved_tensors
        L = load()
        n, H, W = (int(v) for v in imgs.shape[:3])
        gb = grad_bits.to(torch.float32).contiguous()
        grad = torch.empty_like(params)
        stream = ctypes.c_void_p(torch.cuda.current_stream(params.device).cuda_stream)
        check(L.nellox_nll_bwd(params.data_ptr(), _dims(ctx.dims), imgs.data_ptr(), n, H, W, gb.data_ptr(),
                               grad.data_ptr(), ctx.ws.data_ptr(), ctx.ws.numel(), stream), "nellox_nll_bwd")
        ctx.ws = None
        return grad, None, None


def nll_bits(params: torch.Tensor, dims, imgs: torch.Tensor) -> torch.Tensor:
    """Code length in bits of each image (float64, shape (N,)); differentiable in params."""
    return NLLFunction.apply(params, dims, imgs)


def nll_bits_per_px(params: torch.Tensor, dims, imgs: torch.Tensor) -> torch.Tensor:
    """Each pixel's code length -log2 p in bits as the training forward
    computes it (float32, shape (N, H, W)); not differentiable."""
    _check_inputs(params, dims, imgs)
    L = load()
    n, H, W = (int(v) for v in imgs.shape[:3])
    d = _dims(dims)
    nb = L.nellox_train_workspace_bytes(d, n, H, W)
    if nb == 0:
        raise NelloxError(1, "nellox_train_workspace_bytes")
    ws = torch.empty(nb, dtype=torch.uint8, device=params.device)
    bits = torch.empty(n, dtype=torch.float64, device=params.device)
    px = torch.empty((n, H, W), dtype=torch.float32, device=params.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream(params.device).cuda_stream)
    check(L.nellox_nll_fwd_train(params.data_ptr(), d, imgs.data_ptr(), n, H, W, bits.data_ptr(), px.data_ptr(),
                                 ws.data_ptr(), ws.numel(), stream), "nellox_nll_fwd_train")
    return px


def random_crops(pool: torch.Tensor, batch: int, crop: int, rng) -> torch.Tensor:
    """`batch` crop x crop windows of a (N, H, W, 3) uint8 GPU pool, at
    positions drawn from the numpy Generator `rng` (image, row, column)."""
    N, H, W, _ = pool.shape
    ii = torch.from_numpy(rng.integers(0, N, size=batch)).to(pool.device)
    yy = torch.from_numpy(rng.integers(0, H - crop + 1, size=batch)).to(pool.device)
    xx = torch.from_numpy(rng.integers(0, W - crop + 1, size=batch)).to(pool.device)
    ar = torch.arange(crop, device=pool.device)
    return pool[ii[:, None, None], (yy[:, None] + ar)[:, :, None], (xx[:, None] + ar)[:, None, :]].contiguous()


def bits_per_dim(params: torch.Tensor, dims, imgs: torch.Tensor) -> float:
    with torch.no_grad():
        return float(nll_bits(params, dims, imgs).sum()) / imgs.numel()


def fit(params: torch.Tensor, dims, pool: torch.Tensor, steps: int, rng, batch: int = 64, crop: int = 32,
        lr: float = 1e-3, on_step=None) -> torch.Tensor:
    """Adam on bits/dim of random crops of `pool`; returns the trained
    parameter vector (a new tensor). on_step(step, loss_tensor) is called
    after every step if given."""
    p = torch.nn.Parameter(params.detach().clone())
    # one parameter tensor: the fused update is one kernel per step
    opt = torch.optim.Adam([p], lr=lr, fused=True)
    for step in range(steps):
        x = random_crops(pool, batch, crop, rng)
        opt.zero_grad(set_to_none=True)
        loss = nll_bits(p, dims, x).sum() / x.numel()
        loss.backward()
        opt.step()
        if on_step is not None:
            on_step(step, loss)
    return p.detach()
