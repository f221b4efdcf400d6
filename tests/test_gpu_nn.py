"""Parity of the CNN kernels of the learned preconditioner (include/fwi_nn.h)
with a plain PyTorch float64 reference on the CPU.

Tolerances: every kernel stores bfloat16 (unit roundoff 2^-9) from float32
arithmetic on exact bfloat16 products, so one output differs from the
float64 value rounded once to bfloat16 by at most one bfloat16 step plus
the float32 summation error.  Per element we allow 2^-8 |ref| plus 1e-5
times the sum of the absolute terms (float32 sums of up to ~10^4 terms);
weight gradients, stored in float32, get the summation term only.  The
whole network is compared with a reference that rounds at the same points
(tests/nn_reference.py); its tolerances are stated at the test."""
import numpy as np
import pytest

from paper_2506_20513_amd import nn
from tests import nn_reference as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    nn.lib()


def _bf(shape, seed, scale=1.0):
    import torch
    g = torch.Generator().manual_seed(seed)
    return (torch.randn(*shape, generator=g, dtype=torch.float64) * scale).to(torch.bfloat16)


def _dev(t):
    return t.contiguous().cuda()


def _conv_ref(x, w, b, relu):
    import torch
    import torch.nn.functional as F
    y = F.conv2d(R.nchw(x.double()), w.double().permute(0, 3, 1, 2), b, padding=1)
    ya = F.conv2d(R.nchw(x.double().abs()), w.double().abs().permute(0, 3, 1, 2), None, padding=1)
    if relu:
        y = torch.relu(y)
    return R.nhwc(y), R.nhwc(ya)


def _close_bf16(got, ref, absref, what):
    got = got.double().cpu()
    err = (got - ref).abs()
    bound = 2.0 ** -8 * ref.abs() + 1e-5 * absref + 1e-30
    worst = float((err / bound).max())
    print(f"{what}: max err / bound = {worst:.3g}, max |err| = {float(err.max()):.3g}", flush=True)
    assert worst <= 1.0


@pytest.mark.parametrize("N,H,W,Ci,Co,relu", [(2, 13, 70, 32, 64, 1), (1, 9, 130, 64, 96, 0),
                                              (3, 5, 17, 96, 32, 1), (1, 1, 1, 32, 32, 0),
                                              # LDS-tiled kernel, 128-pixel blocks: 64- and
                                              # 32-channel tiles
                                              (8, 61, 67, 32, 256, 1), (16, 61, 67, 32, 96, 0),
                                              # 64-pixel blocks (fewer than 512 of 128):
                                              # 64- and 32-channel tiles, ragged tail,
                                              # several input-channel chunks
                                              (4, 64, 64, 32, 128, 1), (4, 61, 67, 32, 96, 1),
                                              (4, 64, 96, 96, 64, 0), (1, 64, 128, 64, 256, 1)])
def test_conv3x3_matches_reference(N, H, W, Ci, Co, relu):
    import torch
    x = _bf((N, H, W, Ci), 1)
    w = _bf((Co, 3, 3, Ci), 2, 0.1)
    b = torch.randn(Co, generator=torch.Generator().manual_seed(3), dtype=torch.float64).float()
    y = torch.empty(N * H * W * Co, dtype=torch.bfloat16, device="cuda")
    nn.conv3x3(_dev(x), _dev(w), _dev(b), y, N, H, W, Ci, Co, relu)
    torch.cuda.synchronize()
    ref, aref = _conv_ref(x, w, b.double(), relu)
    _close_bf16(y.view(N, H, W, Co), ref, aref + b.double().abs(), f"conv {N}x{H}x{W} {Ci}->{Co}")


def test_flipped_conv_is_the_input_gradient():
    import torch
    N, H, W, Ci, Co = 2, 11, 67, 64, 32
    x = _bf((N, H, W, Ci), 4).double().requires_grad_(True)
    w = _bf((Co, 3, 3, Ci), 5, 0.1)
    g = _bf((N, H, W, Co), 6)
    y, _ = _conv_ref(x, w, None, False)
    (y * g.double()).sum().backward()
    wf = torch.empty(Co * 9 * Ci, dtype=torch.bfloat16, device="cuda")
    nn.flip(_dev(w), wf, Ci, Co)
    dx = torch.empty(N * H * W * Ci, dtype=torch.bfloat16, device="cuda")
    nn.conv3x3(_dev(g), wf, None, dx, N, H, W, Co, Ci, 0)
    torch.cuda.synchronize()
    aref, _ = _conv_ref(g.abs(), w.permute(3, 1, 2, 0).flip(1, 2).contiguous().abs(), None, False)
    _close_bf16(dx.view(N, H, W, Ci), x.grad, aref, "input gradient")


def test_flip_layers_matches_per_layer_flips():
    """One launch for every layer but the first, against fwi_nn_flip per
    layer; elements between the layers (bias and alignment slots) keep what
    they held."""
    import torch
    net = nn.Net(seed=3)
    wf = torch.full_like(net.wbf, 7.0)
    offs, cis, cos = net._flip_table
    nn.flip_layers(net.wbf, wf, offs, cis, cos)
    ref = torch.full_like(net.wbf, 7.0)
    for k in range(1, len(nn.LAYERS)):
        _, ci, co, _, _ = nn.LAYERS[k]
        wo = net.offs[k][0]
        nn.flip(net.w(k), ref[wo:wo + co * 9 * ci], ci, co)
    torch.cuda.synchronize()
    assert torch.equal(wf.cpu(), ref.cpu())


@pytest.mark.parametrize("N,H,W,Ci,Co,nsplit", [(2, 10, 37, 32, 64, 1), (2, 10, 37, 32, 64, 3),
                                                 (2, 10, 37, 32, 64, 700),
                                                 # chunks crossing rows and images, odd width
                                                 (3, 7, 13, 32, 64, 5),
                                                 # several channel tiles both ways
                                                 (2, 9, 21, 64, 96, 2), (1, 1, 1, 32, 32, 1),
                                                 # rows wider than a chunk; one-pixel-wide images
                                                 (2, 5, 100, 32, 32, 7), (4, 3, 1, 32, 32, 2)])
def test_weight_gradient_matches_reference(N, H, W, Ci, Co, nsplit):
    import torch
    x = _bf((N, H, W, Ci), 7)
    w = _bf((Co, 3, 3, Ci), 8, 0.1).double().requires_grad_(True)
    g = _bf((N, H, W, Co), 9)
    y, _ = _conv_ref(x, w, None, False)
    (y * g.double()).sum().backward()
    wa = w.detach().abs().requires_grad_(True)
    ya, _ = _conv_ref(x.abs(), wa, None, False)
    (ya * g.double().abs()).sum().backward()
    ws = torch.empty(nn.wgrad_workspace(Ci, Co, nsplit) // 4, dtype=torch.float32, device="cuda")
    dw = torch.full((Co * 9 * Ci,), float("nan"), device="cuda")
    db = torch.full((Co,), float("nan"), device="cuda")
    nn.wgrad(_dev(x), _dev(g), dw, db, N, H, W, Ci, Co, nsplit, ws)
    torch.cuda.synchronize()
    err = (dw.double().cpu().view(Co, 3, 3, Ci) - w.grad).abs()
    worst = float((err / (1e-5 * wa.grad + 1e-30)).max())
    print("weight gradient: max err / bound", worst, flush=True)
    assert worst <= 1.0
    dbr = g.double().sum(dim=(0, 1, 2))
    assert float((db.double().cpu() - dbr).abs().max()) <= 1e-5 * float(g.double().abs().sum(dim=(0, 1, 2)).max())


@pytest.mark.parametrize("C", [32, 4])   # 8-channel vector kernels, and the scalar ones
def test_elementwise_kernels_match_reference(C):
    import torch
    import torch.nn.functional as F
    N, H, W = 2, 6, 10
    x = _bf((N, H, W, C), 10)
    s = _bf((N, H, W, C), 11)
    dev = lambda t: _dev(t)
    # pooling and its adjoint
    y = torch.empty(N * (H // 2) * (W // 2) * C, dtype=torch.bfloat16, device="cuda")
    nn.pool2(dev(x), y, N, H, W, C)
    ref = R.nhwc(F.avg_pool2d(R.nchw(x.double()), 2))
    q = _bf((N, H // 2, W // 2, C), 12)
    dx = torch.empty(N * H * W * C, dtype=torch.bfloat16, device="cuda")
    nn.pool2_bwd(dev(q), dx, N, H, W, C)
    ref_b = R.nhwc(F.interpolate(R.nchw(q.double()), scale_factor=2, mode="nearest") * 0.25)
    dxs = torch.empty_like(dx)
    nn.pool2_bwd_add(dev(q), dev(s), dxs, N, H, W, C)
    dx2 = torch.empty_like(dx)
    nn.add(dx, dev(s), dx2, x.numel())
    # upsampling + skip and its adjoint
    u = torch.empty(N * H * W * C, dtype=torch.bfloat16, device="cuda")
    nn.up2_add(dev(q), dev(s), u, N, H, W, C)
    ref_u = R.nhwc(F.interpolate(R.nchw(q.double()), scale_factor=2, mode="nearest")) + s.double()
    u0 = torch.empty_like(u)
    nn.up2_add(dev(q), None, u0, N, H, W, C)
    du = torch.empty(N * (H // 2) * (W // 2) * C, dtype=torch.bfloat16, device="cuda")
    nn.up2_bwd(dev(x), du, N, H // 2, W // 2, C)
    ref_du = R.nhwc(F.avg_pool2d(R.nchw(x.double()), 2) * 4.0)
    # relu backward and add
    dz = torch.empty_like(dx)
    nn.relu_bwd(dev(x), dev(s), dz, x.numel())
    ref_dz = torch.where(x.double() > 0, s.double(), torch.zeros_like(s.double()))
    a = torch.empty_like(dx)
    nn.add(dev(x), dev(s), a, x.numel())
    torch.cuda.synchronize()
    # fused adjoint + skip: the same bf16 values as the two calls
    assert torch.equal(dxs.cpu(), dx2.cpu())
    cases = [(y, ref, "pool"), (dx, ref_b, "pool adjoint"), (dxs, ref_b + s.double(), "pool adjoint + skip"),
             (u, ref_u, "up + skip"),
             (u0, R.nhwc(F.interpolate(R.nchw(q.double()), scale_factor=2, mode="nearest")), "up"),
             (du, ref_du, "up adjoint"), (dz, ref_dz, "relu backward"),
             (a, x.double() + s.double(), "add")]
    # misaligned operands (2-byte offset) take the scalar kernels
    n = x.numel() - 1
    xs, ss = dev(x).view(-1)[1:], dev(s).view(-1)[1:]
    dz2 = torch.empty(n + 1, dtype=torch.bfloat16, device="cuda")[1:]
    a2 = torch.empty(n + 1, dtype=torch.bfloat16, device="cuda")[1:]
    nn.relu_bwd(xs, ss, dz2, n)
    nn.add(xs, ss, a2, n)
    torch.cuda.synchronize()
    cases += [(dz2, ref_dz.reshape(-1)[1:], "relu backward, misaligned"),
              (a2, (x.double() + s.double()).reshape(-1)[1:], "add, misaligned")]
    for got, r, what in cases:
        got = got.double().cpu().reshape(r.shape)
        # one rounding to bf16 of a value computed exactly (or within float32)
        assert torch.equal(got, R.rb(r)) or float(((got - r).abs() / (2 ** -8 * r.abs() + 1e-30)).max()) <= 1.0, what


def test_mse_adam_pack_unpack():
    import torch
    P, C, cout = 4099, 32, 2
    y = _bf((P, C), 13)
    t = torch.randn(P, cout, generator=torch.Generator().manual_seed(14), dtype=torch.float64).float()
    dy = torch.empty(P * C, dtype=torch.bfloat16, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    part = torch.empty(nn.FWI_NN_MSE_BLOCKS, dtype=torch.float64, device="cuda")
    nn.mse(_dev(y), _dev(t), dy, loss, part, P, C, cout)
    torch.cuda.synchronize()
    d = y.double()[:, :cout] - t.double()
    assert abs(float(loss) - float((d * d).mean())) <= 1e-12 * float((d * d).mean())
    g = torch.zeros(P, C, dtype=torch.float64)
    g[:, :cout] = R.rb((2 * d / (P * cout)).float()).double()
    got = dy.double().cpu().view(P, C)
    assert float(((got - g).abs() / (2 ** -8 * g.abs() + 1e-30)).max()) <= 1.0
    # the element-wise form (channel count not a multiple of 8)
    P2, C2, c2 = 37, 5, 3
    y2 = _bf((P2, C2), 18)
    t2 = torch.randn(P2, c2, generator=torch.Generator().manual_seed(19), dtype=torch.float64).float()
    dy2 = torch.empty(P2 * C2, dtype=torch.bfloat16, device="cuda")
    nn.mse(_dev(y2), _dev(t2), dy2, loss, part, P2, C2, c2)
    torch.cuda.synchronize()
    d2 = y2.double()[:, :c2] - t2.double()
    assert abs(float(loss) - float((d2 * d2).mean())) <= 1e-12 * float((d2 * d2).mean())
    g2 = torch.zeros(P2, C2, dtype=torch.float64)
    g2[:, :c2] = R.rb((2 * d2 / (P2 * c2)).float()).double()
    got2 = dy2.double().cpu().view(P2, C2)
    assert float(((got2 - g2).abs() / (2 ** -8 * g2.abs() + 1e-30)).max()) <= 1.0
    # Adam, two steps, against the textbook update in float64
    n = 1000
    gen = torch.Generator().manual_seed(15)
    w0 = torch.randn(n, generator=gen, dtype=torch.float64)
    gs = [torch.randn(n, generator=gen, dtype=torch.float64) for _ in range(2)]
    w, m, v = _dev(w0.float()), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    wb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    wr, mr, vr = w0.float().double(), torch.zeros(n, dtype=torch.float64), torch.zeros(n, dtype=torch.float64)
    for k, gk in enumerate(gs, 1):
        nn.adam(w, _dev(gk.float()), m, v, wb, n, 1e-2, 0.9, 0.999, 1e-8, k)
        gk = gk.float().double()
        mr = 0.9 * mr + 0.1 * gk
        vr = 0.999 * vr + 0.001 * gk * gk
        wr = wr - 1e-2 * (mr / (1 - 0.9 ** k)) / ((vr / (1 - 0.999 ** k)).sqrt() + 1e-8)
    torch.cuda.synchronize()
    assert float((w.double().cpu() - wr).abs().max()) <= 1e-6 * float(wr.abs().max())
    assert torch.equal(wb.cpu(), w.cpu().to(torch.bfloat16))
    # pack / unpack
    N, H, W = 2, 8, 24
    planes = torch.randn(N, 4, H, W, generator=gen, dtype=torch.float64).float()
    sc = torch.tensor([[0.5, 2.0, 1.0, 3.0], [1.5, 0.25, 1.0, 1.0]], dtype=torch.float32)
    x = torch.empty(N * H * W * nn.CPAD, dtype=torch.bfloat16, device="cuda")
    nn.pack4(_dev(planes), _dev(sc), x, N, H, W)
    out = torch.empty(N * 2 * H * W, dtype=torch.float32, device="cuda")
    sc2 = torch.tensor([[2.0, 0.5], [1.0, 4.0]], dtype=torch.float32)
    nn.unpack2(x, _dev(sc2), out, N, H, W, nn.CPAD)
    torch.cuda.synchronize()
    ref = torch.zeros(N, H, W, nn.CPAD)
    ref[..., :4] = (planes * sc[:, :, None, None]).permute(0, 2, 3, 1)
    assert torch.equal(x.cpu().view(N, H, W, nn.CPAD), ref.to(torch.bfloat16))
    ref_out = ref.to(torch.bfloat16).float()[..., :2].permute(0, 3, 1, 2) * sc2[:, :, None, None]
    assert torch.equal(out.cpu().view(N, 2, H, W), ref_out)


@pytest.mark.parametrize("N,H,W", [(2, 24, 72), (2, 128, 128)])
def test_network_forward_backward_matches_reference(N, H, W):
    """The whole network (2 x 24 x 72: every layer on the small-layer
    kernel, ragged tiles; 2 x 128 x 128: the full-resolution layers on the
    LDS-tiled kernel) against the rounding-matched reference.
    A float32 sum that lands on the other side of a bfloat16 rounding
    boundary than the float64 one changes the next layer's sums, which
    flips further roundings, so the two sides drift apart until every
    stored tensor differs by about one rounding (u = 2^-9 ~ 2e-3) per stage
    it went through, adding like a random walk: sqrt(15) u ~ 8e-3 over the
    15 forward stages, sqrt(30) u ~ 1.1e-2 over forward and backward.  The
    bounds, in relative L2 per tensor, are 1e-2 for the output and 2e-2 for
    each layer's weight and bias gradient; a wrong index or a dropped term
    gives errors of order one."""
    import torch
    # a non-zero output layer, so that every layer receives a gradient
    params = nn.init_params(seed=3, out_scale=0.1)
    net = nn.Net(params)
    planes = torch.randn(N, 4, H, W, generator=torch.Generator().manual_seed(16)).float()
    sc = torch.ones(N, 4)
    x = torch.empty(N * H * W * nn.CPAD, dtype=torch.bfloat16, device="cuda")
    nn.pack4(_dev(planes), _dev(sc), x, N, H, W)
    tgt = torch.randn(N, H, W, 2, generator=torch.Generator().manual_seed(17)).float()
    y = net.forward(x, N, H, W)
    dy = torch.empty_like(y)
    loss = net.loss_and_grad(y, _dev(tgt), dy, N, H, W)
    net.backward(dy)
    torch.cuda.synchronize()
    P = R.layer_params(params, nn.LAYERS, nn.param_offsets())
    yr, saved = R.forward(x.cpu().view(N, H, W, nn.CPAD).double(), P, nn.LAYERS)
    lr, dyr = R.mse_grad(yr, tgt, nn.NOUT)
    grads = R.backward(dyr, saved, P, nn.LAYERS)
    yg = y.double().cpu().view(N, H, W, nn.CPAD)
    e = float(torch.linalg.norm(yg - R.nhwc(yr)) / torch.linalg.norm(yr))
    print("network output rel L2", e, "loss", float(loss), lr, flush=True)
    assert e <= 1e-2
    assert abs(float(loss) - lr) <= 5e-3 * lr
    worst = 0.0
    for k, (name, ci, co, _, _) in enumerate(nn.LAYERS):
        gw = net.gw(k).double().cpu().view(co, 3, 3, ci)
        gb = net.gb(k).double().cpu()
        rw, rbias = grads[k]
        if name == "out":   # only the used output channels carry gradient
            rw, rbias, gw, gb = rw[:nn.NOUT], rbias[:nn.NOUT], gw[:nn.NOUT], gb[:nn.NOUT]
        ew = float(torch.linalg.norm(gw - rw) / torch.linalg.norm(rw))
        eb = float(torch.linalg.norm(gb - rbias) / max(float(torch.linalg.norm(rbias)), 1e-30))
        print(f"layer {name}: weight-gradient rel L2 {ew:.2e}, bias {eb:.2e}", flush=True)
        worst = max(worst, ew, eb)
    assert worst <= 2e-2


def test_training_steps_reduce_the_loss():
    """A few Adam steps on one fixed batch lower the loss (the kernels'
    gradient is a descent direction of their own forward map)."""
    import torch
    N, H, W = 4, 32, 32
    net = nn.Net(seed=5, out_scale=0.1)
    gen = torch.Generator().manual_seed(18)
    planes = torch.randn(N, 4, H, W, generator=gen).float()
    tgt = (0.5 * planes[:, :2] + 0.1).permute(0, 2, 3, 1).contiguous()
    x = torch.empty(N * H * W * nn.CPAD, dtype=torch.bfloat16, device="cuda")
    nn.pack4(_dev(planes), _dev(torch.ones(N, 4)), x, N, H, W)
    t = _dev(tgt)
    losses = []
    for _ in range(30):
        y = net.forward(x, N, H, W)
        dy = torch.empty_like(y)
        losses.append(float(net.loss_and_grad(y, t, dy, N, H, W)))
        net.backward(dy)
        net.adam_step(1e-3)
    torch.cuda.synchronize()
    print("losses", losses[0], losses[10], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]
