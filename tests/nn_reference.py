"""Plain PyTorch (CPU, float64) reference of the preconditioner network in
paper_2506_20513_amd/nn.py, for the parity tests of its HIP kernels.

It follows the network's definition layer by layer with torch's own conv2d,
avg_pool2d, nearest upsampling and their autograd-free adjoints, rounding to
bfloat16 wherever the kernels store a bfloat16 tensor, so that the only
remaining differences are the order of the float32 sums inside the kernels
(and the rare bfloat16 rounding flips those cause)."""
from __future__ import annotations

import torch
import torch.nn.functional as F


def rb(t: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 and back (the kernels' storage format)."""
    return t.to(torch.bfloat16).to(t.dtype)


def nhwc(t):
    return t.permute(0, 2, 3, 1).contiguous()


def nchw(t):
    return t.permute(0, 3, 1, 2).contiguous()


def layer_params(flat, layers, offsets):
    """[(weight [Co][Ci][3][3] bf16-rounded float64, bias [Co] float64)]"""
    out = []
    for (_, ci, co, _, _), (wo, bo) in zip(layers, offsets):
        w = torch.as_tensor(flat[wo:wo + co * 9 * ci], dtype=torch.float64).reshape(co, 3, 3, ci)
        out.append((rb(w).permute(0, 3, 1, 2).contiguous(),
                    torch.as_tensor(flat[bo:bo + co], dtype=torch.float64)))
    return out


def forward(x_nhwc, params, layers):
    """x_nhwc: packed input (bf16 values as float64).  Returns (output NCHW,
    saved) where saved holds every layer input / output for backward."""
    x = nchw(x_nhwc.to(torch.float64))
    outs, ins = [], []
    for k, (name, ci, co, lv, relu) in enumerate(layers):
        if name == "e0a":
            inp = x
        elif name in ("e1a", "e2a", "e3a"):
            inp = rb(F.avg_pool2d(outs[k - 1], 2))
        elif name in ("d2a", "d1a", "d0a"):
            inp = rb(F.interpolate(outs[k - 1], scale_factor=2, mode="nearest") + outs[2 * lv + 1])
        else:
            inp = outs[k - 1]
        w, b = params[k]
        z = F.conv2d(inp, w, b, padding=1)
        y = rb(torch.relu(z) if relu else z)
        ins.append(inp)
        outs.append(y)
    return outs[-1], (ins, outs)


def mse_grad(y, target_nhwc, nout):
    """loss = mean over pixels and the first nout channels of (y - t)^2 and
    dL/dy (zero in the other channels, bf16-rounded as the kernel stores it)."""
    t = nchw(target_nhwc.to(torch.float64))
    d = y[:, :nout] - t
    P = y.shape[0] * y.shape[2] * y.shape[3]
    loss = float((d * d).sum()) / (P * nout)
    g = torch.zeros_like(y)
    g[:, :nout] = rb((2.0 * d / (P * nout)).to(torch.float32)).to(torch.float64)
    return loss, g


def backward(dy, saved, params, layers):
    """Gradients [(dW [Co][3][3][Ci], db [Co])] in the kernels' weight
    layout, with bf16 rounding of every stored gradient tensor."""
    ins, outs = saved
    grads = [None] * len(layers)
    gskip = {}
    cur = dy
    for k in range(len(layers) - 1, -1, -1):
        name, ci, co, lv, relu = layers[k]
        w, _ = params[k]
        dz = rb(cur * (outs[k] > 0)) if relu else cur
        dw = torch.nn.grad.conv2d_weight(ins[k], w.shape, dz, padding=1)
        grads[k] = (dw.permute(0, 2, 3, 1).contiguous(), dz.sum(dim=(0, 2, 3)))
        if k == 0:
            break
        dx = rb(torch.nn.grad.conv2d_input(ins[k].shape, w, dz, padding=1))
        if name in ("e1a", "e2a", "e3a"):
            g = rb(F.interpolate(dx, scale_factor=2, mode="nearest") * 0.25)
            cur = rb(g + gskip[lv - 1])
        elif name in ("d2a", "d1a", "d0a"):
            gskip[lv] = dx
            cur = rb(F.avg_pool2d(dx, 2) * 4.0)
        else:
            cur = dx
    return grads
