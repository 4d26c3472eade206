"""The surrogate network's GPU kernels against the FP64 oracle.

The GPU computes in BF16 with FP32 accumulation: inputs, weights, hidden
activations and back-propagated gradients are rounded to BF16 (8-bit
significand, relative rounding 2^-9).  To isolate the kernels' own error the
oracle receives BF16-representable weights and inputs; the remaining
differences come from rounding the activations and gradients between layers.
Bounds (relative L2): forward output and gradients 1e-2 (measured ~2e-3).
"""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

DIMS = [5, 512, 512, 512, 512, 258]


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14119_amd import flashkin
    return torch, flashkin


def bf16(a):
    """Round float32 values to the nearest BF16 (ties to even), as float32."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def layer_slices(dims):
    out, off = [], 0
    for l in range(len(dims) - 1):
        nw = dims[l] * dims[l + 1]
        out.append((slice(off, off + nw), slice(off + nw, off + nw + dims[l + 1])))
        off += nw + dims[l + 1]
    return out


def make_case(dims, m, seed):
    rng = np.random.default_rng(seed)
    p = bf16(omlp.init_params(dims, seed).astype(np.float32))
    # nonzero biases so the bias paths are exercised
    for _, sb in layer_slices(dims):
        p[sb] = bf16(0.1 * rng.standard_normal(sb.stop - sb.start).astype(np.float32))
    x = bf16(rng.uniform(-1, 1, (m, dims[0])).astype(np.float32))
    t = rng.standard_normal((m, dims[-1])).astype(np.float32)
    return p, x, t


@pytest.mark.parametrize("dims,m", [(DIMS, 256), ([3, 40, 33, 7], 32), ([5, 64, 70], 48)])
def test_forward_and_gradients_match_oracle(env, dims, m):
    torch, fk = env
    p, x, t = make_case(dims, m, seed=len(dims) + m)
    net = fk.MLP(dims, max_batch=max(m, 64))
    net.set_params(p)
    assert np.array_equal(net.params(), p)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    yd = torch.empty((m, dims[-1]), dtype=torch.float32, device="cuda")
    net.forward(xd.data_ptr(), m, yd.data_ptr())
    loss = net.backward(td.data_ptr(), m)
    g = net.grads()
    y_ref, _ = omlp.forward(p, dims, x)
    loss_ref, g_ref = omlp.loss_and_grads(p, dims, x, t)
    e_y = rel_l2(yd.cpu().numpy(), y_ref)
    print(dims, "forward", e_y, "loss", loss, loss_ref)
    assert e_y < 1e-2
    assert abs(loss - loss_ref) < 1e-2 * loss_ref
    for l, (sw, sb) in enumerate(layer_slices(dims)):
        ew, eb = rel_l2(g[sw], g_ref[sw]), rel_l2(g[sb], g_ref[sb])
        print("  layer", l, "dW", ew, "db", eb)
        assert ew < 1e-2 and eb < 1e-2, (l, ew, eb)
    net.close()


def test_adamw_step_matches_oracle(env):
    torch, fk = env
    dims = [5, 64, 70]
    m = 48
    p, x, t = make_case(dims, m, seed=4)
    net = fk.MLP(dims, max_batch=64)
    net.set_params(p)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    mom = np.zeros(p.size)
    vel = np.zeros(p.size)
    cur = p.astype(np.float64)
    for step in (1, 2, 3):
        net.forward(xd.data_ptr(), m)
        net.backward(td.data_ptr(), m)
        g = net.grads().astype(np.float64)
        net.adamw(step, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.05)
        cur, mom, vel = omlp.adamw(cur, g, mom, vel, step, dims, 1e-2, 0.9, 0.999, 1e-8, 0.05)
        got = net.params().astype(np.float64)
        assert np.allclose(got, cur, rtol=2e-6, atol=1e-7), step
        cur = got
    net.close()


def test_training_reduces_loss(env):
    """A smooth synthetic regression on the full-size network: the training
    loop (forward, backward, AdamW on the GPU) cuts the loss tenfold."""
    torch, fk = env
    rng = np.random.default_rng(0)
    m = 256
    x = rng.uniform(-1, 1, (1024, 5)).astype(np.float32)
    basis = rng.standard_normal((5, 258)).astype(np.float32)
    t = np.sin(x @ basis).astype(np.float32)
    net = fk.MLP(DIMS, max_batch=m)
    net.set_params(omlp.init_params(DIMS, 1).astype(np.float32))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    losses = []
    for step in range(1, 301):
        lo = (step - 1) % 4 * m
        net.forward(xd[lo:lo + m].data_ptr(), m)
        losses.append(net.backward(td[lo:lo + m].data_ptr(), m))
        net.adamw(step, lr=1e-3, weight_decay=1e-4)
    print("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.1 * losses[0]
    # the device-side running sum saw the same 300 losses
    mean, count = net.take_loss()
    assert count == 300 and mean == pytest.approx(float(np.mean(losses)), rel=1e-6)
    # without reading the loss back, steps only queue work; the sum keeps them
    for step in range(301, 305):
        lo = (step - 1) % 4 * m
        net.forward(xd[lo:lo + m].data_ptr(), m)
        assert net.backward(td[lo:lo + m].data_ptr(), m, read_loss=False) is None
        net.adamw(step, lr=1e-3, weight_decay=1e-4)
    mean, count = net.take_loss()
    assert count == 4 and 0.0 < mean < losses[0]
    assert net.take_loss() == (0.0, 0)
    net.close()


# ---------------------------------------------------------------- fused step

@pytest.mark.parametrize("dims,m", [(DIMS, 256), ([3, 40, 33, 7], 32), ([5, 64, 70], 48), (DIMS, 16)])
def test_train_step_matches_oracle_and_the_separate_calls(env, dims, m):
    """fk_mlp_train_step (loss in the output GEMM, AdamW in the weight-gradient
    tiles) against the FP64
    oracle's loss and gradients (1e-2, as the separate calls), against the
    separate calls' loss (1e-5) and gradients, and its AdamW step against the
    oracle's step applied to its own gradients (as the separate AdamW).  The
    48- and 16-row batches end in half tiles."""
    torch, fk = env
    p, x, t = make_case(dims, m, seed=3 * len(dims) + m)
    mb = max(m, 64)
    sep, fused = fk.MLP(dims, max_batch=mb), fk.MLP(dims, max_batch=mb)
    sep.set_params(p)
    fused.set_params(p)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    sep.forward(xd.data_ptr(), m)
    loss_sep = sep.backward(td.data_ptr(), m)
    g_sep = sep.grads()
    fused.take_loss()
    fused.train_step(xd.data_ptr(), td.data_ptr(), m, 1, lr=1e-3, weight_decay=0.01)
    loss, count = fused.take_loss()
    g = fused.grads()
    loss_ref, g_ref = omlp.loss_and_grads(p, dims, x, t)
    print(dims, m, "loss", loss, loss_sep, loss_ref)
    assert count == 1 and loss == pytest.approx(loss_sep, rel=1e-5)
    assert abs(loss - loss_ref) < 1e-2 * loss_ref
    for l, (sw, sb) in enumerate(layer_slices(dims)):
        ew, eb = rel_l2(g[sw], g_ref[sw]), rel_l2(g[sb], g_ref[sb])
        sw_, sb_ = rel_l2(g[sw], g_sep[sw]), rel_l2(g[sb], g_sep[sb])
        print("  layer", l, "vs oracle", ew, eb, "vs separate", sw_, sb_)
        assert ew < 1e-2 and eb < 1e-2, (l, ew, eb)
        assert sw_ < 5e-3 and sb_ < 5e-3, (l, sw_, sb_)
    z = np.zeros(p.size)
    want, _, _ = omlp.adamw(p.astype(np.float64), g.astype(np.float64), z, z, 1, dims, 1e-3, 0.9, 0.999, 1e-8, 0.01)
    assert np.allclose(fused.params().astype(np.float64), want, rtol=2e-6, atol=1e-7)
    sep.close()
    fused.close()


def test_train_step_trains_like_the_separate_calls(env):
    """300 steps of the smooth regression of test_training_reduces_loss with
    the fused step: the loss falls tenfold and ends within 10% of the
    separate calls' run from the same start."""
    torch, fk = env
    rng = np.random.default_rng(0)
    m = 256
    x = rng.uniform(-1, 1, (1024, 5)).astype(np.float32)
    basis = rng.standard_normal((5, 258)).astype(np.float32)
    t = np.sin(x @ basis).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    p0 = omlp.init_params(DIMS, 1).astype(np.float32)
    runs = {}
    for mode in ("separate", "fused"):
        net = fk.MLP(DIMS, max_batch=m)
        net.set_params(p0)
        net.take_loss()
        first = last = None
        for step in range(1, 301):
            lo = (step - 1) % 4 * m
            if mode == "fused":
                net.train_step(xd[lo:lo + m].data_ptr(), td[lo:lo + m].data_ptr(), m, step, lr=1e-3,
                               weight_decay=1e-4)
            else:
                net.forward(xd[lo:lo + m].data_ptr(), m)
                net.backward(td[lo:lo + m].data_ptr(), m, read_loss=False)
                net.adamw(step, lr=1e-3, weight_decay=1e-4)
            if step == 1:
                first = net.take_loss()[0]
            if step == 300:
                last = net.take_loss()[0]
        runs[mode] = (first, last)
        net.close()
    print(runs)
    f0, f1 = runs["fused"]
    s0, s1 = runs["separate"]
    assert f0 == pytest.approx(s0, rel=1e-5)
    assert f1 < 0.1 * f0
    assert abs(f1 - s1) < 0.1 * s1


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_random_networks_train_step(env, seed):
    """Seeded random network shapes (one to five layers, widths 1 to 300,
    batches of 16 to 128 rows): the training step's loss and every gradient
    against the oracle (1e-2) and its AdamW step against the oracle's step
    applied to its own gradients."""
    torch, fk = env
    rng = np.random.default_rng(seed)
    depth = int(rng.integers(1, 6))
    dims = [int(rng.integers(1, 12))] + [int(rng.integers(1, 301)) for _ in range(depth - 1)] + [int(rng.integers(1, 200))]
    m = 16 * int(rng.integers(1, 9))
    p, x, t = make_case(dims, m, seed=100 + seed)
    net = fk.MLP(dims, max_batch=max(m, 64))
    net.set_params(p)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    net.take_loss()
    net.train_step(xd.data_ptr(), td.data_ptr(), m, 1, lr=1e-3, weight_decay=0.01)
    loss, count = net.take_loss()
    g = net.grads()
    loss_ref, g_ref = omlp.loss_and_grads(p, dims, x, t)
    print(dims, m, "loss", loss, loss_ref)
    assert count == 1 and abs(loss - loss_ref) < 1e-2 * loss_ref
    for l, (sw, sb) in enumerate(layer_slices(dims)):
        ew, eb = rel_l2(g[sw], g_ref[sw]), rel_l2(g[sb], g_ref[sb])
        print("  layer", l, ew, eb)
        assert ew < 1e-2 and eb < 1e-2, (l, ew, eb)
    z = np.zeros(p.size)
    want, _, _ = omlp.adamw(p.astype(np.float64), g.astype(np.float64), z, z, 1, dims, 1e-3, 0.9, 0.999, 1e-8, 0.01)
    assert np.allclose(net.params().astype(np.float64), want, rtol=2e-6, atol=1e-7)
    net.close()
