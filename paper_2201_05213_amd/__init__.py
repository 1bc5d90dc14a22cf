"""nellox: parallel neural local lossless compression on MI355X.

Python binding of the C ABI in include/nellox.h. Torch supplies device
memory and the stream; every step of coding runs in the HIP library.

    m = Model(blob)                          # weight blob (bytes)
    data, offs = m.encode(images, order=1, patch=(64, 64))
    out, status = m.decode(data, offs, shapes, order=1, patch=(64, 64))
    bits = m.nll(images)                     # -log2 p(x) per image
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from ._lib import NelloxDecodePlan, NelloxError, NelloxImage, NelloxOpts, check, load

__all__ = ["Model", "NelloxError", "load", "RASTER", "WAVEFRONT", "SHEARED", "ROWS"]

RASTER = 0
WAVEFRONT = 1
SHEARED = 2  # the wavefront order, decoded in the sheared layout (ShearLoC)


def _opts(order: int, patch, interleave: int = 1) -> NelloxOpts:
    ph, pw = (0, 0) if patch is None else (int(patch[0]), int(patch[1]))
    return NelloxOpts(int(order), ph, pw, int(interleave))


def _images(imgs: Sequence[torch.Tensor]):
    arr = (NelloxImage * max(len(imgs), 1))()
    for k, t in enumerate(imgs):
        if t.dtype != torch.uint8 or t.dim() != 3 or t.shape[2] != 3 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("images must be contiguous uint8 HxWx3 CUDA tensors")
        arr[k] = NelloxImage(t.data_ptr(), int(t.shape[0]), int(t.shape[1]))
    return arr


def _shape_images(shapes, device):
    return [torch.empty((int(h), int(w), 3), dtype=torch.uint8, device=device) for h, w in shapes]


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Model:
    """A model loaded onto the current GPU from a weight blob."""

    def __init__(self, blob: bytes, device=None):
        L = load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        with torch.cuda.device(self.device):
            check(L.nellox_model_create(buf, len(blob), ctypes.byref(h)), "nellox_model_create")
        self._h = h
        dims = (ctypes.c_int32 * 4)()
        hsh = ctypes.c_uint64()
        check(L.nellox_model_info(self._h, dims, ctypes.byref(hsh)), "nellox_model_info")
        self.h, self.C, self.n_blocks, self.n_mix = (int(d) for d in dims)
        self.hash = int(hsh.value)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                load().nellox_model_destroy(self._h)
                self._h = None
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def workspace(self, imgs_arr, n, opts, encode: bool = True) -> torch.Tensor:
        """Workspace for this batch: of every call (encode=True), or of every
        call but encode (decoding, sampling, NLL, debug)."""
        fn = load().nellox_workspace_bytes if encode else load().nellox_decode_workspace_bytes
        nb = fn(self._h, n, imgs_arr, ctypes.byref(opts))
        if nb == 0:
            raise NelloxError(1, "nellox_workspace_bytes")
        return torch.empty(nb, dtype=torch.uint8, device=self.device)

    @staticmethod
    def encode_bound(H: int, W: int, order: int = WAVEFRONT, patch=None, interleave: int = 1) -> int:
        o = _opts(order, patch, interleave)
        return int(load().nellox_encode_bound(H, W, ctypes.byref(o)))

    # ------------------------------------------------------------------ coding
    def encode(self, imgs: Sequence[torch.Tensor], order: int = WAVEFRONT, patch=None, sync: bool = True,
               ws: torch.Tensor | None = None, interleave: int = 1):
        """Returns (containers: uint8 CUDA tensor, offsets: int64 CUDA tensor
        of n+1). With sync=True the container tensor is trimmed to its size.
        interleave = rANS streams per lane (1, 2 or 4)."""
        L = load()
        n = len(imgs)
        o = _opts(order, patch, interleave)
        arr = _images(imgs)
        cap = sum(self.encode_bound(int(t.shape[0]), int(t.shape[1]), order, patch, interleave) for t in imgs)
        out = torch.empty(max(cap, 1), dtype=torch.uint8, device=self.device)
        offs = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        if ws is None:
            ws = self.workspace(arr, n, o)
        check(L.nellox_encode(self._h, n, arr, ctypes.byref(o), out.data_ptr(), out.numel(), offs.data_ptr(),
                              ws.data_ptr(), ws.numel(), _stream(self.device)), "nellox_encode")
        if sync:
            total = int(offs[-1].item())
            out = out[:total]
        return out, offs

    def decode(self, data: torch.Tensor, offsets: torch.Tensor, shapes, order: int = WAVEFRONT, patch=None,
               out: Sequence[torch.Tensor] | None = None, sync: bool = True, trace: bool = False,
               ws: torch.Tensor | None = None, interleave: int = 1):
        """Returns (images, status[, sym_dump]). With sync=True a non-OK
        status raises NelloxError. interleave must match the containers."""
        L = load()
        n = len(shapes)
        o = _opts(order, patch, interleave)
        imgs = _shape_images(shapes, self.device) if out is None else list(out)
        arr = _images(imgs)
        status = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        if ws is None:
            ws = self.workspace(arr, n, o, encode=False)
        data = data.contiguous()
        offsets = offsets.to(device=self.device, dtype=torch.int64).contiguous()
        if trace:
            npx = sum(int(h) * int(w) for h, w in shapes)
            dump = torch.zeros(max(npx * 3, 1), dtype=torch.int32, device=self.device)
            check(L.nellox_decode_trace(self._h, n, data.data_ptr(), offsets.data_ptr(), ctypes.byref(o), arr,
                                        status.data_ptr(), dump.data_ptr(), ws.data_ptr(), ws.numel(),
                                        _stream(self.device)), "nellox_decode_trace")
        else:
            check(L.nellox_decode(self._h, n, data.data_ptr(), offsets.data_ptr(), ctypes.byref(o), arr,
                                  status.data_ptr(), ws.data_ptr(), ws.numel(), _stream(self.device)),
                  "nellox_decode")
        status = status[:n]
        if sync:
            st = status.cpu()
            bad = [(k, int(v)) for k, v in enumerate(st.tolist()) if v != 0]
            if bad:
                raise NelloxError(bad[0][1], f"nellox_decode (image {bad[0][0]})")
        return (imgs, status, dump[:sum(int(h) * int(w) for h, w in shapes) * 3]) if trace else (imgs, status)

    def decode_prepare(self, out: Sequence[torch.Tensor], order: int = WAVEFRONT, patch=None, interleave: int = 1,
                       ws: torch.Tensor | None = None):
        """Plan a batch decode into the images `out` (preallocated, H x W x 3
        uint8): returns (plan, ws). decode_run(plan, ...) then only launches
        kernels and may be captured in a CUDA/HIP graph; keep `out` and `ws`
        alive as long as the plan is used."""
        L = load()
        n = len(out)
        o = _opts(order, patch, interleave)
        arr = _images(out)
        if ws is None:
            ws = self.workspace(arr, n, o, encode=False)
        plan = NelloxDecodePlan()
        check(L.nellox_decode_prepare(self._h, n, arr, ctypes.byref(o), ws.data_ptr(), ws.numel(), ctypes.byref(plan),
                                      _stream(self.device)), "nellox_decode_prepare")
        return plan, ws

    def decode_run(self, plan, data: torch.Tensor, offsets: torch.Tensor, status: torch.Tensor, ws: torch.Tensor):
        """Launch a prepared decode on the current stream (asynchronous;
        status: int32 CUDA tensor of n entries, 0 = OK)."""
        check(load().nellox_decode_run(self._h, ctypes.byref(plan), data.data_ptr(), offsets.data_ptr(),
                                       status.data_ptr(), ws.data_ptr(), _stream(self.device)), "nellox_decode_run")

    def sample(self, shapes, seeds, order: int = WAVEFRONT, patch=None, out: Sequence[torch.Tensor] | None = None,
               ws: torch.Tensor | None = None):
        """Draw one image per (H, W) in `shapes` (uint8 H x W x 3 on the
        model's device) by ancestral sampling; image k is a function of
        seeds[k] (a 64-bit integer), its size and the patch shape only."""
        L = load()
        n = len(shapes)
        if len(seeds) != n:
            raise ValueError("one seed per image")
        o = _opts(order, patch)
        imgs = _shape_images(shapes, self.device) if out is None else list(out)
        arr = _images(imgs)
        sd = (ctypes.c_uint64 * max(n, 1))(*[int(v) & 0xFFFFFFFFFFFFFFFF for v in seeds])
        if ws is None:
            ws = self.workspace(arr, n, o, encode=False)
        check(L.nellox_sample(self._h, n, sd, ctypes.byref(o), arr, ws.data_ptr(), ws.numel(), _stream(self.device)),
              "nellox_sample")
        return imgs

    def nll(self, imgs: Sequence[torch.Tensor], patch=None, per_pixel: bool = False):
        """Continuous code length -log2 p(x) per image (float64 CUDA tensor)."""
        L = load()
        n = len(imgs)
        o = _opts(WAVEFRONT, patch)
        arr = _images(imgs)
        ws = self.workspace(arr, n, o, encode=False)
        tot = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        npx = sum(int(t.shape[0]) * int(t.shape[1]) for t in imgs)
        px = torch.empty(max(npx, 1), dtype=torch.float32, device=self.device) if per_pixel else None
        check(L.nellox_nll(self._h, n, arr, ctypes.byref(o), px.data_ptr() if px is not None else None,
                           tot.data_ptr(), ws.data_ptr(), ws.numel(), _stream(self.device)), "nellox_nll")
        return (tot[:n], px[:npx]) if per_pixel else tot[:n]

    def debug_symbols(self, imgs: Sequence[torch.Tensor], patch=None):
        """Encoder symbols (start | freq << 16) per pixel/channel and the
        quantised ideal bits per image."""
        L = load()
        n = len(imgs)
        o = _opts(WAVEFRONT, patch)
        arr = _images(imgs)
        ws = self.workspace(arr, n, o, encode=False)
        npx = sum(int(t.shape[0]) * int(t.shape[1]) for t in imgs)
        sym = torch.zeros(max(npx * 3, 1), dtype=torch.int32, device=self.device)
        ideal = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        check(L.nellox_debug_symbols(self._h, n, arr, ctypes.byref(o), sym.data_ptr(), ideal.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream(self.device)), "nellox_debug_symbols")
        return sym[:npx * 3], ideal[:n]

    def debug_cdf(self, img: torch.Tensor, patch=None) -> torch.Tensor:
        """Full quantised CDF rows [H, W, 3, 257] (int32, CUDA)."""
        L = load()
        o = _opts(WAVEFRONT, patch)
        arr = _images([img])
        ws = self.workspace(arr, 1, o, encode=False)
        H, W = int(img.shape[0]), int(img.shape[1])
        cdf = torch.empty((H, W, 3, 257), dtype=torch.int32, device=self.device)
        check(L.nellox_debug_cdf(self._h, arr, ctypes.byref(o), cdf.data_ptr(), ws.data_ptr(), ws.numel(),
                                 _stream(self.device)), "nellox_debug_cdf")
        return cdf


def debug_check_monotone(device=None) -> dict:
    """Scan every finite FP32 value on the GPU and count order violations of
    the hardware exp2, reciprocal and rcp(1 + exp2(z)) (see nellox.h)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    check(load().nellox_debug_check_monotone(counts.data_ptr(), _stream(dev)), "nellox_debug_check_monotone")
    c = counts.cpu().tolist()
    return {"exp2_decreasing": c[0], "rcp_increasing": c[1], "sigmoid_increasing": c[2], "pairs": c[3]}


ROWS = -1  # interleave: one rANS stream per lane row


def container_streams(c: bytes) -> int:
    """rANS streams (stream table entries) of a container, from its header:
    lanes x K, or with row streams (stream byte 0) the lane rows, H per
    column of patches."""
    H, W = int.from_bytes(c[8:12], "little"), int.from_bytes(c[12:16], "little")
    pw = int.from_bytes(c[18:20], "little") or W
    nl = int.from_bytes(c[28:32], "little")
    return nl * c[7] if c[7] else -(-W // pw) * H


def payload_bits(data, offsets) -> list:
    """Coded bits per image: the stream payloads (final states and
    renormalisation bytes), without the header and the stream table."""
    d = bytes(data.cpu().numpy().tobytes()) if isinstance(data, torch.Tensor) else bytes(data)
    o = offsets.cpu().tolist() if isinstance(offsets, torch.Tensor) else list(offsets)
    out = []
    for k in range(len(o) - 1):
        c = d[o[k]:o[k + 1]]
        out.append(8 * (len(c) - 32 - 4 * container_streams(c)))
    return out


def peek(container: bytes):
    """(H, W, order, (patch_h, patch_w), interleave) of a container held on the host."""
    L = load()
    buf = ctypes.create_string_buffer(bytes(container[:64]), min(len(container), 64))
    H, W = ctypes.c_int32(), ctypes.c_int32()
    o = NelloxOpts()
    check(L.nellox_peek(buf, min(len(container), 64), ctypes.byref(H), ctypes.byref(W), ctypes.byref(o)),
          "nellox_peek")
    return H.value, W.value, o.order, (o.patch_h, o.patch_w), o.interleave
