"""Warm-start network on the GPU against the oracle, and its use in the solver."""
import numpy as np
import pytest

from oracle import cnn

pytestmark = pytest.mark.gpu


def _params(seed, last=0.3):
    rng = np.random.default_rng(seed)
    p = cnn.init_params(seed, scale_last=last)
    p = [(W, 0.05 * rng.standard_normal(b.shape)) for W, b in p]
    return cnn.flatten(p).astype(np.float32)


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_forward_matches_oracle():
    import torch
    from paper_1705_06603_amd import _lib as dl
    flat = _params(1)
    net = dl.Net(4, 64, 64, params=flat)
    rng = np.random.default_rng(2)
    B, H, W = 2, 32, 64
    img = rng.random((B, H, W)).astype(np.float32)
    valid = [[32, 64], [30, 50]]
    out = net.forward(torch.tensor(img, device="cuda"), valid=valid).cpu().numpy()
    P = cnn.unflatten(flat.astype(np.float64))
    for b, (vh, vw) in enumerate(valid):
        x = img[b:b + 1, :vh, :vw].astype(np.float64)
        ref16, _ = cnn.forward(P, x, bf16=True)
        ref64, _ = cnn.forward(P, x, bf16=False)
        assert _rel(out[b, :vh, :vw], ref16[0]) <= 5e-3
        assert _rel(out[b, :vh, :vw] - x[0], ref16[0] - x[0]) <= 5e-3
        assert _rel(out[b, :vh, :vw], ref64[0]) <= 3e-2
        assert np.all(out[b, vh:, :] == 0) and np.all(out[b, :, vw:] == 0)
    net.close()


def test_loss_and_gradients_match_oracle():
    import torch
    from paper_1705_06603_amd import _lib as dl
    flat = _params(3)
    net = dl.Net(2, 16, 32, params=flat)
    rng = np.random.default_rng(4)
    img = rng.random((2, 16, 32)).astype(np.float32)
    tgt = rng.random((2, 16, 32)).astype(np.float32)
    loss, g = net.loss_grad(torch.tensor(img, device="cuda"), torch.tensor(tgt, device="cuda"))
    ref_loss, ref_grads, _ = cnn.loss_and_grads(cnn.unflatten(flat.astype(np.float64)), img.astype(np.float64),
                                                tgt.astype(np.float64), bf16=True)
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    G = cnn.unflatten(g.astype(np.float64))
    for li in range(4):
        assert _rel(G[li][0], ref_grads[li][0]) <= 5e-3, (li, "W", _rel(G[li][0], ref_grads[li][0]))
        assert _rel(G[li][1], ref_grads[li][1]) <= 5e-3, (li, "b", _rel(G[li][1], ref_grads[li][1]))
    net.close()


def test_adam_steps_match_oracle():
    """Three Adam steps on the GPU against the oracle's Adam recurrence fed
    the GPU's own gradient of each step (the gradients themselves are
    compared with the oracle above), so that every parameter's update is
    compared to fp32 rounding, none excepted."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    flat = _params(5)
    net = dl.Net(2, 16, 32, params=flat)
    rng = np.random.default_rng(6)
    img = torch.tensor(rng.random((2, 16, 32)).astype(np.float32), device="cuda")
    tgt = torch.tensor(rng.random((2, 16, 32)).astype(np.float32), device="cuda")
    lr = 1e-3
    w_prev = flat.astype(np.float64)
    m = np.zeros_like(w_prev)
    v = np.zeros_like(w_prev)
    for k in (1, 2, 3):
        _, g = net.loss_grad(img, tgt)            # the gradient this step uses
        net.train_step(img, tgt, lr)
        w_gpu = net.get_params().astype(np.float64)
        w_ref, m, v = cnn.adam_step(w_prev, g.astype(np.float64), m, v, k, lr)
        err = np.abs(w_gpu - w_ref)
        tol = 2e-7 * np.abs(w_ref) + 1e-5 * lr
        assert np.all(err <= tol), (k, float(np.max(err - tol)))
        assert np.max(np.abs(w_gpu - w_prev)) > 0.5 * lr   # the step moved the weights
        w_prev = w_gpu
    net.close()


def test_training_reduces_loss():
    import torch
    from paper_1705_06603_amd import _lib as dl
    net = dl.Net(8, 32, 32, seed=7)
    rng = np.random.default_rng(8)
    img = rng.random((8, 32, 32)).astype(np.float32)
    # target: a 3x3 box blur of the input (a map the network can represent)
    pad = np.pad(img, ((0, 0), (1, 1), (1, 1)))
    tgt = sum(pad[:, dy:dy + 32, dx:dx + 32] for dy in range(3) for dx in range(3)) / 9.0
    ti, tt = torch.tensor(img, device="cuda"), torch.tensor(tgt.astype(np.float32), device="cuda")
    losses = [net.train_step(ti, tt, 2e-3) for _ in range(80)]
    assert losses[-1] < 0.3 * losses[0], (losses[0], losses[-1])
    net.close()


def _small_ctx():
    from tests._gpu import context_of
    from tests.test_gpu_solver import _mid_problem
    prob = _mid_problem(seed=9)
    return context_of(prob), prob


def test_warm_start_falls_back_when_network_does_not_help():
    from paper_1705_06603_amd import _lib as dl
    ctx, prob = _small_ctx()
    N = ctx.tiles[0].frame
    # zero last layer: the network returns its input, i.e. the plain start
    flat = _params(10)
    P = cnn.unflatten(flat.astype(np.float64))
    P[3] = (np.zeros_like(P[3][0]), np.zeros_like(P[3][1]))
    net = dl.Net(ctx.n_tiles, N, N, params=cnn.flatten(P))
    use, nf = ctx.init_cnn(net)
    assert nf == ctx.n_tiles and not use.any()
    x_w, _ = ctx.get_state()
    ctx.init()
    x_p, _ = ctx.get_state()
    assert np.array_equal(x_w.cpu().numpy(), x_p.cpu().numpy())
    # a network with exploding output: every tile falls back
    P[3] = (np.ones_like(P[3][0]) * 50.0, np.ones_like(P[3][1]) * 50.0)
    net.set_params(cnn.flatten(P))
    use, nf = ctx.init_cnn(net)
    assert nf == ctx.n_tiles
    net.close()
    ctx.close()


def test_trained_warm_start_gains_over_plain_start():
    """Trained on converged plain-solver pairs (residual 1e-4) of fresh scenes
    of the 256 x 256 workload's generator, the network starts a held-out
    scene closer to that scene's converged solution than the plain start,
    and the warm-started solve reaches residual 1e-4 in fewer rounds."""
    from paper_1705_06603_amd import _lib as dl
    from paper_1705_06603_amd import train as tr
    from paper_1705_06603_amd import workloads
    w = workloads.WORKLOADS["small"]
    ctx, _ = tr.workload_context(w)
    N = ctx.tiles[0].frame
    ins, outs = tr.make_pairs(ctx, w, seeds=range(100, 108), crop=128, crops_per_tile=4, tol=1e-4,
                              max_rounds=3000)
    net = dl.Net(16, N, N, seed=11)
    losses = tr.train(net, ins, outs, steps=250, batch=16, lr=2e-3)
    print(f"training loss: first 25 steps {np.mean(losses[:25]):.4e}, last 25 {np.mean(losses[-25:]):.4e}")
    assert np.mean(losses[-25:]) < np.mean(losses[:25])
    # held-out scene
    tr.observe_scene(ctx, w, 999)
    res_plain = tr.solve_plain(ctx, w, tol=1e-4, max_rounds=3000)
    assert res_plain[-1] <= 1e-4
    x_star = ctx.get_state()[0].cpu().numpy()
    ctx.init()
    x_plain = ctx.get_state()[0].cpu().numpy()
    use, nf = ctx.init_cnn(net)
    x_warm = ctx.get_state()[0].cpu().numpy()
    d_plain = np.linalg.norm(x_plain - x_star)
    d_warm = np.linalg.norm(x_warm - x_star)
    res_warm = []
    while len(res_warm) < 3000:
        res_warm += ctx.run(50, w.n_inner, tol=1e-4)
        if res_warm[-1] <= 1e-4:
            break
    print(f"distance to the converged solution: plain {d_plain:.4e} warm {d_warm:.4e}, tiles kept "
          f"{int(use.sum())}/{len(use)}; rounds to 1e-4: plain {len(res_plain)} warm {len(res_warm)}")
    assert d_warm < d_plain
    assert res_warm[-1] <= 1e-4 and len(res_warm) < len(res_plain)
    net.close()
    ctx.close()


def test_inference_only_network():
    """Forward buffers only: the same output as a trainable network with the
    same weights, and training calls are refused."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    flat = _params(4)
    a = dl.Net(2, 64, 64, params=flat)
    b = dl.Net(2, 64, 64, params=flat, inference_only=True)
    rng = np.random.default_rng(6)
    img = torch.tensor(rng.random((2, 64, 64)).astype(np.float32), device="cuda")
    oa = a.forward(img, valid=[[64, 64], [40, 50]]).cpu().numpy()
    ob = b.forward(img, valid=[[64, 64], [40, 50]]).cpu().numpy()
    assert np.array_equal(oa, ob)
    with pytest.raises(dl.DeblurError) as e:
        b.train_step(img, img, 1e-3)
    assert e.value.code == -5
    a.close()
    b.close()


@pytest.mark.parametrize("seed", [4, 5])
def test_fused_forward_equals_layer_by_layer_and_matches_oracle(seed):
    """The fused forward kernel (inference-only network: all four layers of a
    28 x 28 block in one workgroup, activations in LDS) against the
    layer-by-layer kernels (trainable network) on images whose size and valid
    regions cut the 28-pixel blocks unevenly, and against the bf16 oracle."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    flat = _params(seed)
    B, H, W = 3, 96, 160
    valid = [[96, 160], [70, 150], [29, 31]]
    rng = np.random.default_rng(seed)
    img = (3.0 * rng.random((B, H, W))).astype(np.float32)
    a = dl.Net(B, H, W, params=flat)
    b = dl.Net(B, H, W, params=flat, inference_only=True)
    t = torch.tensor(img, device="cuda")
    oa = a.forward(t, valid=valid).cpu().numpy()
    ob = b.forward(t, valid=valid).cpu().numpy()
    diff = float(np.max(np.abs(oa - ob)))
    print(f"fused vs layer by layer: max |difference| {diff:.3e}, identical {np.array_equal(oa, ob)}")
    assert diff <= 1e-6 * float(np.max(np.abs(oa)))
    P = cnn.unflatten(flat.astype(np.float64))
    for k, (vh, vw) in enumerate(valid):
        x = img[k:k + 1, :vh, :vw].astype(np.float64)
        ref16, _ = cnn.forward(P, x, bf16=True)
        assert _rel(ob[k, :vh, :vw], ref16[0]) <= 5e-3
        assert np.all(ob[k, vh:, :] == 0) and np.all(ob[k, :, vw:] == 0)
    a.close()
    b.close()

