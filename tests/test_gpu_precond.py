"""The learned-preconditioner pipeline on the GPU at a small scale: pairs
from plain L-BFGS runs on seeded 128x128 models, training through the CNN
kernels, and an inversion that tries the network's step first and falls
back to L-BFGS.  Checks the structure of the data, that training lowers the
loss, and that the learned run keeps the plain run's guarantees (monotone
objective, every accepted step passes the decrease test)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def test_pairs_training_and_learned_inversion():
    import torch
    from paper_2506_20513_amd import fwi_loop as FL
    from paper_2506_20513_amd import precond as PC
    st = FL.Settings(tv_weight=1e-3)
    ds, stats = PC.generate(2, 4, 10000, st, log=lambda m: print(m, flush=True))
    print("generate", stats, flush=True)
    assert ds.planes.shape == (8, 4, 128, 128) and ds.targets.shape == (8, 128, 128, 2)
    # two runs at a time, each on its own stream: the same pairs bit for bit
    ds2, stats2 = PC.generate(2, 4, 10000, st, log=None, workers=2)
    assert stats2["workers"] == 2
    for a, b in ((ds.planes, ds2.planes), (ds.scales, ds2.scales), (ds.targets, ds2.targets)):
        assert torch.equal(a, b)
    assert torch.isfinite(ds.planes).all() and torch.isfinite(ds.targets).all()
    # the last pair of a run is one step: its target is that step, nonzero
    assert float(ds.targets[3].abs().max()) > 0
    # the first gradient of each run is normalised to unit rms
    for i in (0, 4):
        for c in (0, 1):
            r = float(torch.sqrt(torch.mean((ds.planes[i, c] * ds.scales[i, c]).double() ** 2)))
            assert abs(r - 1.0) < 1e-4
    net, hist = PC.train(ds, epochs=20, batch=2, lr=1e-3, val_frac=0.0, warmup=10,
                         log=lambda m: print(m, flush=True))
    ids = hist["train_ids"]
    zero = float((ds.targets[ids].double() ** 2).mean())
    fit = PC.mean_loss(net, ds, ids, batch=4)
    print("training pairs: zero predictor", zero, "trained", fit, flush=True)
    assert fit < 0.5 * zero
    cfg, prob, obs, _, _, e0, s0 = PC.tiny_problem(50000, 6.0)
    res = PC.compare(net, [("held-out", prob, obs, e0, s0)], 4, st,
                     log=lambda m: print(m, flush=True))
    r = res[0]
    assert r["learned_evaluations"] >= 1 and r["plain_evaluations"] >= 1
    # objective monotone in the learned run as well
    obj = PC.Objective(prob, obs, e0, s0, st)
    pc = PC.Preconditioner(net)
    run = PC.minimise(obj, 4, proposer=lambda x, g: pc(obj, x, g))
    fs = [it.f for it in run.log]
    assert all(b <= a for a, b in zip(fs, fs[1:]))
    assert pc.calls >= 1
    # applied at half resolution (pool, network, upsample): a finite proposal
    # of the model's shape, zero on the fixed surface rows, constant on 2x2 blocks
    pc2 = PC.Preconditioner(net, 2)
    f0, g0 = obj(obj.x0)
    d = pc2(obj, obj.x0, g0)
    assert d.shape == obj.x0.shape and torch.isfinite(d).all()
    assert float(d[~obj.free].abs().max()) == 0.0
    u = d[: obj.ny * obj.nx].view(obj.ny, obj.nx)[8:, :]
    assert torch.equal(u[0::2, 0::2], u[1::2, 1::2])


def test_survey_pairs_and_training_over_two_image_sizes():
    import math

    import torch
    from paper_2506_20513_amd import fwi_loop as FL
    from paper_2506_20513_amd import precond as PC
    st = FL.Settings(tv_weight=1e-3)
    tiny, _ = PC.generate(2, 4, 10000, st, log=None)
    big, stats = PC.generate(1, 2, 20000, st, log=lambda m: print(m, flush=True), kind="survey")
    print("generate survey", stats, flush=True)
    assert big.planes.shape == (2, 4, 256, 512) and big.targets.shape == (2, 256, 512, 2)
    assert torch.isfinite(big.planes).all() and torch.isfinite(big.targets).all()
    for c in (0, 1):
        r = float(torch.sqrt(torch.mean((big.planes[0, c] * big.scales[0, c]).double() ** 2)))
        assert abs(r - 1.0) < 1e-4
    # batch 2 of 128x128 images is 1 of 256x512 (at least one image per batch)
    net, hist = PC.train([tiny, big], epochs=2, batch=2, lr=1e-3, val_frac=0.0, warmup=2,
                         log=lambda m: print(m, flush=True))
    assert hist["steps"] == 2 * (8 // 2 + 2 // 1)
    assert all(math.isfinite(e["train_loss"]) for e in hist["epochs"])
    # the trained network applies to either size
    for ds in (tiny, big):
        assert math.isfinite(PC.mean_loss(net, ds, torch.arange(2, device=ds.planes.device), 1))
