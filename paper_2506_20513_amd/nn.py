"""Binding of the CNN kernels (include/fwi_nn.h) and the encoder-decoder
network of the learned gradient preconditioner built from them.

Every arithmetic step of the network (convolutions, their input and weight
gradients, pooling, upsampling, skips, ReLU, the loss and Adam) runs in the
HIP kernels; torch only provides device memory and the stream, and Python
only sequences the calls.

Network (4 levels, 32 / 64 / 128 / 256 channels, 3x3 convolutions, BF16
activations and weights, FP32 accumulation, FP32 master weights):

    level 0 (H x W):        in(4 -> padded 32) -> 32 -> 32 = s0
    level 1 (H/2 x W/2):    pool(s0) -> 64 -> 64 = s1
    level 2 (H/4 x W/4):    pool(s1) -> 128 -> 128 = s2
    level 3 (H/8 x W/8):    pool(s2) -> 256 -> 256 -> 128 = r3
    decoder:                up(r3) + s2 -> 128 -> 64 = r2
                            up(r2) + s1 -> 64 -> 32 = r1
                            up(r1) + s0 -> 32 -> out (linear, channels 0..1)

ReLU after every convolution except the last; skips are added, not
concatenated.  H and W must be multiples of 8.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import fwi

FWI_NN_OK = 0
FWI_NN_MSE_BLOCKS = 512
CPAD = 32                      # channels of the packed network input

EXPORTED = ("fwi_nn_conv3x3", "fwi_nn_flip", "fwi_nn_flip_layers", "fwi_nn_wgrad_workspace",
            "fwi_nn_wgrad",
            "fwi_nn_relu_bwd", "fwi_nn_pool2", "fwi_nn_pool2_bwd", "fwi_nn_pool2_bwd_add",
            "fwi_nn_up2_add",
            "fwi_nn_up2_bwd", "fwi_nn_add", "fwi_nn_mse", "fwi_nn_adam", "fwi_nn_to_bf16",
            "fwi_nn_pack4", "fwi_nn_unpack2")

_ready = False


def lib() -> ctypes.CDLL:
    global _ready
    L = fwi.lib()
    if not _ready:
        vp, sz, i32, f32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_float
        L.fwi_nn_conv3x3.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, vp]
        L.fwi_nn_flip.argtypes = [vp, vp, i32, i32, vp]
        L.fwi_nn_flip_layers.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.fwi_nn_wgrad_workspace.argtypes = [i32, i32, i32]
        L.fwi_nn_wgrad_workspace.restype = sz
        L.fwi_nn_wgrad.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, vp, sz, vp]
        L.fwi_nn_relu_bwd.argtypes = [vp, vp, vp, sz, vp]
        L.fwi_nn_pool2.argtypes = [vp, vp, i32, i32, i32, i32, vp]
        L.fwi_nn_pool2_bwd.argtypes = [vp, vp, i32, i32, i32, i32, vp]
        L.fwi_nn_pool2_bwd_add.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp]
        L.fwi_nn_up2_add.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp]
        L.fwi_nn_up2_bwd.argtypes = [vp, vp, i32, i32, i32, i32, vp]
        L.fwi_nn_add.argtypes = [vp, vp, vp, sz, vp]
        L.fwi_nn_mse.argtypes = [vp, vp, vp, vp, vp, sz, i32, i32, vp]
        L.fwi_nn_adam.argtypes = [vp, vp, vp, vp, vp, sz, f32, f32, f32, f32, i32, vp]
        L.fwi_nn_to_bf16.argtypes = [vp, vp, sz, vp]
        L.fwi_nn_pack4.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp]
        L.fwi_nn_unpack2.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp]
        for n in EXPORTED:
            if n != "fwi_nn_wgrad_workspace":
                getattr(L, n).restype = ctypes.c_int
        _ready = True
    return L


class NNError(RuntimeError):
    pass


def _ok(status, where):
    if status != FWI_NN_OK:
        raise NNError(f"{where}: status {status}")


def _p(t):
    return None if t is None else t.data_ptr()


def _s(stream):
    return fwi._stream(stream)


def _need(t, dtype, numel, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, need {numel}")


BF = torch.bfloat16
F32 = torch.float32


# ---------------------------------------------------------------------------
# Thin wrappers, one per entry point (shapes checked against the tensors)
# ---------------------------------------------------------------------------
def conv3x3(x, w, bias, y, N, H, W, Ci, Co, relu, stream=None):
    _need(x, BF, N * H * W * Ci, "x")
    _need(w, BF, Co * 9 * Ci, "w")
    _need(y, BF, N * H * W * Co, "y")
    if bias is not None:
        _need(bias, F32, Co, "bias")
    _ok(lib().fwi_nn_conv3x3(_p(x), _p(w), _p(bias), _p(y), N, H, W, Ci, Co, int(relu),
                             _s(stream)), "fwi_nn_conv3x3")


def flip(w, wf, Ci, Co, stream=None):
    _need(w, BF, Co * 9 * Ci, "w")
    _need(wf, BF, Co * 9 * Ci, "wf")
    _ok(lib().fwi_nn_flip(_p(w), _p(wf), Ci, Co, _s(stream)), "fwi_nn_flip")


def flip_layers(w, wf, offs, cis, cos, stream=None):
    """fwi_nn_flip for every (offset, Ci, Co) layer of the flat buffers w
    and wf (bf16, same length) in one launch."""
    n = len(offs)
    _need(w, BF, w.numel(), "w")
    _need(wf, BF, w.numel(), "wf")
    if n and offs[-1] + 9 * cis[-1] * cos[-1] > w.numel():
        raise ValueError("flip_layers: a layer runs past the end of w")
    o = (ctypes.c_int64 * n)(*offs)
    a = (ctypes.c_int32 * n)(*cis)
    b = (ctypes.c_int32 * n)(*cos)
    _ok(lib().fwi_nn_flip_layers(_p(w), _p(wf), n, o, a, b, _s(stream)), "fwi_nn_flip_layers")


def wgrad_workspace(Ci, Co, nsplit):
    return int(lib().fwi_nn_wgrad_workspace(Ci, Co, nsplit))


def wgrad(x, dz, dw, db, N, H, W, Ci, Co, nsplit, ws, stream=None):
    _need(x, BF, N * H * W * Ci, "x")
    _need(dz, BF, N * H * W * Co, "dz")
    _need(dw, F32, Co * 9 * Ci, "dw")
    _need(db, F32, Co, "db")
    _ok(lib().fwi_nn_wgrad(_p(x), _p(dz), _p(dw), _p(db), N, H, W, Ci, Co, nsplit, _p(ws),
                           ws.numel() * ws.element_size(), _s(stream)), "fwi_nn_wgrad")


def relu_bwd(y, dy, dz, n, stream=None):
    for t, nm in ((y, "y"), (dy, "dy"), (dz, "dz")):
        _need(t, BF, n, nm)
    _ok(lib().fwi_nn_relu_bwd(_p(y), _p(dy), _p(dz), n, _s(stream)), "fwi_nn_relu_bwd")


def pool2(x, y, N, H, W, C, stream=None):
    _need(x, BF, N * H * W * C, "x")
    _need(y, BF, N * (H // 2) * (W // 2) * C, "y")
    _ok(lib().fwi_nn_pool2(_p(x), _p(y), N, H, W, C, _s(stream)), "fwi_nn_pool2")


def pool2_bwd(dy, dx, N, H, W, C, stream=None):
    _need(dy, BF, N * (H // 2) * (W // 2) * C, "dy")
    _need(dx, BF, N * H * W * C, "dx")
    _ok(lib().fwi_nn_pool2_bwd(_p(dy), _p(dx), N, H, W, C, _s(stream)), "fwi_nn_pool2_bwd")


def pool2_bwd_add(dy, skip, dx, N, H, W, C, stream=None):
    """dx = pool2_bwd(dy) + skip (skip may be None)."""
    _need(dy, BF, N * (H // 2) * (W // 2) * C, "dy")
    if skip is not None:
        _need(skip, BF, N * H * W * C, "skip")
    _need(dx, BF, N * H * W * C, "dx")
    _ok(lib().fwi_nn_pool2_bwd_add(_p(dy), _p(skip), _p(dx), N, H, W, C, _s(stream)),
        "fwi_nn_pool2_bwd_add")


def up2_add(x, skip, y, N, Ho, Wo, C, stream=None):
    _need(x, BF, N * (Ho // 2) * (Wo // 2) * C, "x")
    _need(y, BF, N * Ho * Wo * C, "y")
    if skip is not None:
        _need(skip, BF, N * Ho * Wo * C, "skip")
    _ok(lib().fwi_nn_up2_add(_p(x), _p(skip), _p(y), N, Ho, Wo, C, _s(stream)), "fwi_nn_up2_add")


def up2_bwd(dy, dx, N, Hi, Wi, C, stream=None):
    _need(dy, BF, N * 4 * Hi * Wi * C, "dy")
    _need(dx, BF, N * Hi * Wi * C, "dx")
    _ok(lib().fwi_nn_up2_bwd(_p(dy), _p(dx), N, Hi, Wi, C, _s(stream)), "fwi_nn_up2_bwd")


def add(a, b, y, n, stream=None):
    for t, nm in ((a, "a"), (b, "b"), (y, "y")):
        _need(t, BF, n, nm)
    _ok(lib().fwi_nn_add(_p(a), _p(b), _p(y), n, _s(stream)), "fwi_nn_add")


def mse(y, target, dy, loss, partials, P, C, cout, stream=None):
    _need(y, BF, P * C, "y")
    _need(target, F32, P * cout, "target")
    if dy is not None:
        _need(dy, BF, P * C, "dy")
    _need(loss, torch.float64, 1, "loss")
    _need(partials, torch.float64, FWI_NN_MSE_BLOCKS, "partials")
    _ok(lib().fwi_nn_mse(_p(y), _p(target), _p(dy), _p(loss), _p(partials), P, C, cout,
                         _s(stream)), "fwi_nn_mse")


def adam(w, g, m, v, wb, n, lr, beta1, beta2, eps, step, stream=None):
    for t, nm in ((w, "w"), (g, "g"), (m, "m"), (v, "v")):
        _need(t, F32, n, nm)
    if wb is not None:
        _need(wb, BF, n, "wb")
    _ok(lib().fwi_nn_adam(_p(w), _p(g), _p(m), _p(v), _p(wb), n, lr, beta1, beta2, eps, step,
                          _s(stream)), "fwi_nn_adam")


def to_bf16(a, b, n, stream=None):
    _need(a, F32, n, "a")
    _need(b, BF, n, "b")
    _ok(lib().fwi_nn_to_bf16(_p(a), _p(b), n, _s(stream)), "fwi_nn_to_bf16")


def pack4(planes, scale, x, N, H, W, C=CPAD, stream=None):
    _need(planes, F32, N * 4 * H * W, "planes")
    _need(scale, F32, N * 4, "scale")
    _need(x, BF, N * H * W * C, "x")
    _ok(lib().fwi_nn_pack4(_p(planes), _p(scale), _p(x), N, H, W, C, _s(stream)), "fwi_nn_pack4")


def unpack2(y, scale, out, N, H, W, C, stream=None):
    _need(y, BF, N * H * W * C, "y")
    _need(scale, F32, N * 2, "scale")
    _need(out, F32, N * 2 * H * W, "out")
    _ok(lib().fwi_nn_unpack2(_p(y), _p(scale), _p(out), N, H, W, C, _s(stream)),
        "fwi_nn_unpack2")


# ---------------------------------------------------------------------------
# The network
# ---------------------------------------------------------------------------
# (name, Ci, Co, level, relu) in forward order
LAYERS = (("e0a", CPAD, 32, 0, True), ("e0b", 32, 32, 0, True),
          ("e1a", 32, 64, 1, True), ("e1b", 64, 64, 1, True),
          ("e2a", 64, 128, 2, True), ("e2b", 128, 128, 2, True),
          ("e3a", 128, 256, 3, True), ("e3b", 256, 256, 3, True), ("d3", 256, 128, 3, True),
          ("d2a", 128, 128, 2, True), ("d2b", 128, 64, 2, True),
          ("d1a", 64, 64, 1, True), ("d1b", 64, 32, 1, True),
          ("d0a", 32, 32, 0, True), ("out", 32, 32, 0, False))
NOUT = 2
ALIGN = 64                     # parameter offsets in elements (128-byte aligned bf16 views)


def _align(n):
    return (n + ALIGN - 1) // ALIGN * ALIGN


def init_params(seed: int = 0, in_channels: int = 4, out_scale: float = 0.0) -> np.ndarray:
    """FP32 master parameters, flat, in the layout of Net: per layer the
    weights [Co][3][3][Ci] then the bias [Co], each block starting at a
    multiple of 64 elements.  He-normal weights (fan-in 9 x used input
    channels), zero biases.  The output layer's NOUT used channels start at
    out_scale times a He-normal draw (0: the network starts as the zero
    predictor), its other channels at zero."""
    rng = np.random.default_rng(seed)
    out = np.zeros(param_count(), np.float32)
    for (name, ci, co, _, relu), (wo, bo) in zip(LAYERS, param_offsets()):
        fan = 9 * (in_channels if name == "e0a" else ci)
        w = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / fan)
        if name == "e0a":
            w[:, :, :, in_channels:] = 0.0
        if not relu:
            w *= out_scale
            w[NOUT:] = 0.0
        out[wo:wo + w.size] = w.ravel()
    return out


def param_offsets():
    offs, o = [], 0
    for _, ci, co, _, _ in LAYERS:
        wo = o
        o = _align(o + co * 9 * ci)
        bo = o
        o = _align(o + co)
        offs.append((wo, bo))
    return offs


def param_count():
    _, ci, co, _, _ = LAYERS[-1]
    wo, bo = param_offsets()[-1]
    return _align(bo + co)


class Net:
    """Parameters, optimiser state and activation buffers of the network on
    one device.  forward() / backward() / adam_step() enqueue kernels on the
    current stream; buffers are (re)allocated when the batch shape changes.

    The weight gradient of a layer splits its pixel sum over nsplit blocks
    per channel tile: about WGRAD_BLOCKS blocks in all, at most
    WGRAD_MAX_SPLIT partial sums (each is a full weight tensor for the
    reduction to read)."""

    WGRAD_BLOCKS = 1024
    WGRAD_MAX_SPLIT = 1024
    WGRAD_CHUNK = 32

    def __init__(self, params: np.ndarray | torch.Tensor | None = None, seed: int = 0,
                 device="cuda", out_scale: float = 0.0):
        self.device = torch.device(device)
        n = param_count()
        p = init_params(seed, out_scale=out_scale) if params is None else params
        self.w32 = torch.as_tensor(p, dtype=F32).to(self.device).contiguous().clone()
        if self.w32.numel() != n:
            raise ValueError(f"expected {n} parameters, got {self.w32.numel()}")
        self.wbf = torch.empty(n, dtype=BF, device=self.device)
        to_bf16(self.w32, self.wbf, n)
        self.grad = torch.zeros(n, dtype=F32, device=self.device)
        self.m = torch.zeros(n, dtype=F32, device=self.device)
        self.v = torch.zeros(n, dtype=F32, device=self.device)
        self.step = 0
        self.offs = param_offsets()
        self._shape = None
        # flipped weights of every layer but the first, at the offsets of
        # the weights in wbf, made by one launch per backward pass
        self._wflip = torch.empty(n, dtype=BF, device=self.device)
        self._flip_table = ([self.offs[k][0] for k in range(1, len(LAYERS))],
                            [LAYERS[k][1] for k in range(1, len(LAYERS))],
                            [LAYERS[k][2] for k in range(1, len(LAYERS))])
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.partials = torch.zeros(FWI_NN_MSE_BLOCKS, dtype=torch.float64, device=self.device)

    # -- parameter views --------------------------------------------------
    def w(self, k):
        _, ci, co, _, _ = LAYERS[k]
        wo, _ = self.offs[k]
        return self.wbf[wo:wo + co * 9 * ci]

    def b(self, k):
        _, ci, co, _, _ = LAYERS[k]
        _, bo = self.offs[k]
        return self.w32[bo:bo + co]

    def gw(self, k):
        _, ci, co, _, _ = LAYERS[k]
        wo, _ = self.offs[k]
        return self.grad[wo:wo + co * 9 * ci]

    def gb(self, k):
        _, ci, co, _, _ = LAYERS[k]
        _, bo = self.offs[k]
        return self.grad[bo:bo + co]

    def state_dict(self):
        return {"params": self.w32.detach().cpu().numpy().copy(), "step": self.step}

    # -- buffers ------------------------------------------------------------
    def _buffers(self, N, H, W):
        if H % 8 or W % 8:
            raise ValueError(f"image {H}x{W}: both sides must be multiples of 8")
        if self._shape == (N, H, W):
            return
        dev = self.device
        hw = [(H >> l, W >> l) for l in range(4)]

        def act(level, c):
            h, w = hw[level]
            return torch.empty(N * h * w * c, dtype=BF, device=dev)

        # per layer: input view and output buffer
        self.out = [act(lv, co) for _, ci, co, lv, _ in LAYERS]
        self.pooled = [None, act(1, 32), act(2, 64), act(3, 128)]   # pool(s0), pool(s1), pool(s2)
        self.upped = {2: act(2, 128), 1: act(1, 64), 0: act(0, 32)}  # up(r) + skip
        maxn = max(t.numel() for t in self.out)
        self.g1 = torch.empty(maxn, dtype=BF, device=dev)
        self.g2 = torch.empty(maxn, dtype=BF, device=dev)
        self.g3 = torch.empty(maxn, dtype=BF, device=dev)
        self.gskip = {0: act(0, 32), 1: act(1, 64), 2: act(2, 128)}
        # weight-gradient split: enough blocks to fill the chip, at most one
        # chunk (WGRAD_CHUNK pixels, the kernel's staging step) each
        self.nsplit = []
        wsb = 0
        for _, ci, co, lv, _ in LAYERS:
            h, w = hw[lv]
            chunks = (N * h * w + self.WGRAD_CHUNK - 1) // self.WGRAD_CHUNK
            tiles = (co // 32) * (ci // 32)
            ns = int(max(1, min(chunks, (self.WGRAD_BLOCKS + tiles - 1) // tiles,
                                self.WGRAD_MAX_SPLIT)))
            self.nsplit.append(ns)
            wsb = max(wsb, wgrad_workspace(ci, co, ns))
        self.wsg = torch.empty((wsb + 3) // 4, dtype=F32, device=dev)
        self._shape = (N, H, W)

    def _input_of(self, k, x):
        """Input buffer of layer k in the forward order of LAYERS."""
        name = LAYERS[k][0]
        prev = {"e0a": None, "e0b": 0, "e1a": "p1", "e1b": 2, "e2a": "p2", "e2b": 4,
                "e3a": "p3", "e3b": 6, "d3": 7, "d2a": "u2", "d2b": 9, "d1a": "u1",
                "d1b": 11, "d0a": "u0", "out": 13}[name]
        if prev is None:
            return x
        if isinstance(prev, int):
            return self.out[prev]
        if prev[0] == "p":
            return self.pooled[int(prev[1])]
        return self.upped[int(prev[1])]

    # -- forward ------------------------------------------------------------
    def forward(self, x, N, H, W):
        """x: packed input [N][H][W][32] bf16.  Returns the output buffer
        [N][H][W][32] (channels 0..1 meaningful)."""
        self._buffers(N, H, W)
        _need(x, BF, N * H * W * CPAD, "x")
        self._x = x
        hw = [(H >> l, W >> l) for l in range(4)]
        for k, (name, ci, co, lv, relu) in enumerate(LAYERS):
            if name in ("e1a", "e2a", "e3a"):
                src = self.out[k - 1]
                h, w = hw[lv - 1]
                pool2(src, self.pooled[lv], N, h, w, ci)
            if name in ("d2a", "d1a", "d0a"):
                h, w = hw[lv]
                up2_add(self.out[k - 1], self.out[2 * lv + 1], self.upped[lv], N, h, w, ci)
            h, w = hw[lv]
            conv3x3(self._input_of(k, x), self.w(k), self.b(k), self.out[k], N, h, w, ci, co, relu)
        return self.out[-1]

    # -- backward -----------------------------------------------------------
    def backward(self, dy):
        """dy: gradient of the loss w.r.t. the output [N][H][W][32] bf16.
        Fills self.grad (weights and biases of every layer).

        Going backwards, G_k (the gradient w.r.t. the output of layer k)
        becomes dz_k = relu'(out_k) * G_k, which gives the weight gradient
        and, through the flipped weights, D_k = the gradient w.r.t. the
        layer input.  D_k goes to the producer of that input: straight to
        layer k-1; through the adjoint of pooling (plus the skip gradient
        kept from the decoder) to the encoder output of the level above; or,
        at a decoder merge up(r) + s, to the skip buffer of s and through
        the adjoint of upsampling to r."""
        N, H, W = self._shape
        _need(dy, BF, N * H * W * CPAD, "dy")
        hw = [(H >> l, W >> l) for l in range(4)]
        bufs = (self.g1, self.g2, self.g3)

        def other(*used):
            return next(b for b in bufs if all(b is not u for u in used))

        flip_layers(self.wbf, self._wflip, *self._flip_table)
        cur = dy
        for k in range(len(LAYERS) - 1, -1, -1):
            name, ci, co, lv, relu = LAYERS[k]
            h, w = hw[lv]
            if relu:
                dz = other(cur)
                relu_bwd(self.out[k], cur, dz, N * h * w * co)
            else:
                dz = cur
            wgrad(self._input_of(k, self._x), dz, self.gw(k), self.gb(k), N, h, w, ci, co,
                  self.nsplit[k], self.wsg)
            if k == 0:
                break
            wo = self.offs[k][0]
            wf = self._wflip[wo:wo + ci * 9 * co]
            merge = name in ("d2a", "d1a", "d0a")
            dx = self.gskip[lv] if merge else other(dz, cur)
            conv3x3(dz, wf, None, dx, N, h, w, co, ci, False)
            if name in ("e1a", "e2a", "e3a"):
                hp, wp = hw[lv - 1]
                g = other(dx)
                pool2_bwd_add(dx, self.gskip[lv - 1], g, N, hp, wp, ci)
                cur = g
            elif merge:
                hi, wi = hw[lv + 1]
                g = other(dz)
                up2_bwd(dx, g, N, hi, wi, ci)
                cur = g
            else:
                cur = dx

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        adam(self.w32, self.grad, self.m, self.v, self.wbf, self.w32.numel(), lr, beta1, beta2,
             eps, self.step)

    def loss_and_grad(self, y, target, dy, N, H, W):
        """MSE of channels 0..1 of y against target [N][H][W][2] (FP32);
        fills dy [N][H][W][32] and self.loss (device double)."""
        mse(y, target, dy, self.loss, self.partials, N * H * W, 32, NOUT)
        return self.loss


# ---------------------------------------------------------------------------
# Throughput measurement
# ---------------------------------------------------------------------------
def conv_flops(N: int, H: int, W: int, training: bool) -> float:
    """Algorithmic FLOPs (2 per multiply-add) of the convolutions of one
    forward pass, or of a training step: forward, weight gradient and input
    gradient (none for the first layer)."""
    tot = 0.0
    for k, (_, ci, co, lv, _) in enumerate(LAYERS):
        f = 2.0 * N * (H >> lv) * (W >> lv) * 9 * ci * co
        tot += f * ((3 if k else 2) if training else 1)
    return tot


HBM_PEAK_BPS = 8.0e12          # MI355X HBM3E, AMD public specification
BF16_PEAK_FLOPS = 2.5e15       # MI355X dense BF16 MFMA, AMD public specification


def layer_report(net: "Net", N: int, H: int, W: int, reps: int = 20) -> list:
    """Per layer of a training step: the average time of its forward
    convolution, its input-gradient convolution (flipped weights) and its
    weight gradient, each against its own roofline bound max(flops / BF16
    peak, bytes / HBM peak).  Bytes count the activations read and written
    once (bf16) and the weights; flops are 2 * 9 * Ci * Co per pixel."""
    hw = [(H >> lv, W >> lv) for lv in range(4)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    rows = []
    for k, (name, ci, co, lv, relu) in enumerate(LAYERS):
        h, w = hw[lv]
        npx = N * h * w
        x = torch.zeros(npx * ci, dtype=BF, device=net.device)
        y = torch.zeros(npx * co, dtype=BF, device=net.device)
        wf = torch.empty(co * 9 * ci, dtype=BF, device=net.device)
        flip(net.w(k), wf, ci, co)
        flops = 2.0 * 9 * ci * co * npx
        act_bytes = 2.0 * npx * (ci + co)
        kinds = {
            "fwd": (lambda: conv3x3(x, net.w(k), net.b(k), y, N, h, w, ci, co, relu),
                    act_bytes + 2.0 * 9 * ci * co),
            "dgrad": (lambda: conv3x3(y, wf, None, x, N, h, w, co, ci, False),
                      act_bytes + 2.0 * 9 * ci * co),
            "wgrad": (lambda: wgrad(x, y, net.gw(k), net.gb(k), N, h, w, ci, co, net.nsplit[k],
                                    net.wsg),
                      act_bytes + 4.0 * 9 * ci * co),
        }
        rec = {"layer": name, "Ci": ci, "Co": co, "image": [h, w], "GFLOP": round(flops / 1e9, 3)}
        for kind, (fn, nbytes) in kinds.items():
            t = timed(fn)
            bound = max(flops / BF16_PEAK_FLOPS, nbytes / HBM_PEAK_BPS)
            rec[kind] = {"us": round(t * 1e6, 2), "TFLOPs": round(flops / t / 1e12, 1),
                         "bound": "mfma" if flops / BF16_PEAK_FLOPS >= nbytes / HBM_PEAK_BPS
                         else "hbm", "frac_of_bound": round(bound / t, 4)}
        rows.append(rec)
    return rows


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="throughput of the preconditioner network kernels")
    ap.add_argument("--layers", action="store_true",
                    help="also time every layer's three convolution kernels against their bounds")
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--size", default="128x128", help="training image HxW")
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--infer", default="1024x2048", help="inference image HxW (batch 1)")
    ap.add_argument("--infer-reps", type=int, default=10)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("nn: no GPU visible", file=sys.stderr)
        return 1
    H, W = (int(v) for v in args.size.split("x"))
    N = args.batch
    g = torch.Generator(device="cuda").manual_seed(0)
    planes = torch.randn(N, 4, H, W, generator=g, device="cuda")
    tgt = torch.randn(N, H, W, NOUT, generator=g, device="cuda") * 0.1
    sc = torch.ones(N, 4, device="cuda")
    net = Net(seed=0, out_scale=0.1)
    x = torch.empty(N * H * W * CPAD, dtype=BF, device="cuda")
    dy = torch.empty(N * H * W * CPAD, dtype=BF, device="cuda")

    def step():
        pack4(planes, sc, x, N, H, W)
        y = net.forward(x, N, H, W)
        net.loss_and_grad(y, tgt, dy, N, H, W)
        net.backward(dy)
        net.adam_step(1e-4)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    out = {"train": {"batch": N, "image": [H, W], "ms_per_step": round(ms, 4),
                     "TFLOPs": round(conv_flops(N, H, W, True) / ms * 1e-9, 2)}}
    Hi, Wi = (int(v) for v in args.infer.split("x"))
    pl = torch.randn(1, 4, Hi, Wi, generator=g, device="cuda")
    xi = torch.empty(Hi * Wi * CPAD, dtype=BF, device="cuda")
    pack4(pl, torch.ones(1, 4, device="cuda"), xi, 1, Hi, Wi)
    net.forward(xi, 1, Hi, Wi)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.infer_reps):
        net.forward(xi, 1, Hi, Wi)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.infer_reps
    out["infer"] = {"image": [Hi, Wi], "ms": round(ms, 4),
                    "TFLOPs": round(conv_flops(1, Hi, Wi, False) / ms * 1e-9, 2)}
    out["peak_bf16_TFLOPs"] = 2500.0
    if args.layers:
        net._buffers(N, H, W)
        out["layers"] = layer_report(net, N, H, W)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
