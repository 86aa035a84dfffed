"""The learned warm start end to end on a small scale: a dataset of
G-ICP-labelled pairs from seeded trajectories, training through the library's
kernels, and the comparison with the constant-velocity initial pose on
held-out trajectories (with the fallback)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_warmstart_train_and_evaluate():
    import torch

    import paper_2403_12550_amd as g
    from paper_2403_12550_amd import warmstart as ws
    from paper_2403_12550_amd import warmstart_train as wt
    torch.cuda.set_device(0)
    print("[case] warmstart small", flush=True)
    ctx = g.Context(0)
    net = ws.WarmStartNet(ctx, 0)
    X, Y = wt.build_dataset(g, ctx, net, list(range(wt.TRAIN_SEED0, wt.TRAIN_SEED0 + 6)), workers=4)
    assert X.shape == (600, 4096, 6) and Y.shape == (600, 6)
    # labels are relative poses of at most 8 cm / 4 degrees per frame
    assert float(Y[:, :3].norm(dim=1).max()) < np.radians(4.5)
    y0, cache, _ = net.forward(X[:64], want_cache=True)
    first = float(net.backward(X[:64], cache, y0, Y[:64])[1].item())
    hist = wt.train(net, X, Y, epochs=6, batch=32, lr=1e-3)
    assert hist[-1] < 0.5 * first, (first, hist)
    ev = wt.evaluate(g, ctx, net, [wt.TEST_SEED0], workers=1)
    assert ev["pairs"] == 100
    # the fallback converges at least wherever the constant-velocity start does
    assert ev["net_fallback"]["converged_frac"] >= ev["cv"]["converged_frac"] - 1e-9
    for name in ("cv", "net", "net_fallback"):
        assert np.isfinite(ev[name]["mean_iterations"])
    ctx.close()
