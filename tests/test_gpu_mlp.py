"""GPU checks of the learned warm start: the network's kernels against the FP64 NumPy
MLP oracle, the feature pass against its plain definition, training behaviour, and
a small end-to-end warm-versus-cold comparison.

Bars.  The network takes BF16 operands with FP32 accumulation, so it is compared with
the oracle run with the same BF16 operand rounding (bf16=True): forward outputs to
1e-4 relative (2-norm), gradient blocks to 2e-3 relative.  Features (FP64 sums,
FP32 output) to 1e-6 relative per element.  The warm start changes only where the
iteration begins, so warm solutions must match the oracle's converged solution as
the cold ones do.
"""
import numpy as np
import pytest

from paper_1902_08653_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPE = (8, 96, 80, 2)     # widths that are not multiples of the 64-wide GEMM tile


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_08653_amd import cdm
    cdm.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def mo():
    from oracle import mlp_oracle
    return mlp_oracle


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make_net(shape=SHAPE, max_rows=512, seed=0):
    from paper_1902_08653_amd import cdm
    net = cdm.Mlp(*shape, max_rows=max_rows)
    rng = np.random.default_rng(seed)
    w = (rng.standard_normal(net.nparam) * 0.3).astype(np.float32)
    net.set_weights(w)
    return net, w


def data(rows, nin, nout, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, nin)).astype(np.float32)
    T = rng.standard_normal((rows, nout)).astype(np.float32)
    return X, T


@pytest.mark.parametrize("rows", [1, 63, 300, 512])
def test_forward_vs_oracle(dev, mo, rows):
    net, w = make_net()
    X, _ = data(rows, SHAPE[0], SHAPE[3], rows)
    Y = net.forward(torch.from_numpy(X).to(dev))
    torch.cuda.synchronize()
    want = mo.forward(w.astype(np.float64), SHAPE, X, bf16=True)["Y"]
    assert relerr(Y.cpu().numpy().astype(np.float64), want) <= 1e-4
    net.close()


@pytest.mark.parametrize("rows", [5, 300, 512])
def test_gradients_vs_oracle(dev, mo, rows):
    net, w = make_net(seed=1)
    X, T = data(rows, SHAPE[0], SHAPE[3], 100 + rows)
    g, parts = net.gradients(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    want = mo.gradients(w.astype(np.float64), SHAPE, X, T, bf16=True)
    for got_b, want_b in zip(mo.split(g, SHAPE), mo.split(want, SHAPE)):
        assert relerr(got_b, want_b) <= 2e-3
    loss = float(parts.double().sum().cpu()) / (rows * SHAPE[3])
    assert abs(loss - mo.loss(w.astype(np.float64), SHAPE, X, T, bf16=True)) <= 1e-4 * loss
    # against the exact FP64 gradient the kernel may be off by no more than the BF16
    # operand rounding itself (the oracle's distance, computed on the CPU: 3.8e-2 at 5
    # rows, 5.4e-3 at 300, 4.2e-3 at 512) plus the parity bar above
    exact = mo.gradients(w.astype(np.float64), SHAPE, X, T)
    assert relerr(g, exact) <= relerr(want, exact) + 2e-3
    net.close()


@pytest.mark.parametrize("rows", [300, 512, 130, 8192])
def test_gradients_vs_oracle_wide(dev, mo, rows):
    """Widths 256 take the 128 x 128 tiled GEMM for the products with M, N >= 128 (the
    layer-2 forward, dW2 when the row count is a multiple of 4, dA1): same bars as the
    narrow network; 300 and 130 rows leave ragged tiles (130 also sends dW2 back to the
    generic kernel); 8192 rows split the weight gradients along K (8 chunks summed in
    order)."""
    shape = (8, 256, 256, 2)
    from paper_1902_08653_amd import cdm
    net = cdm.Mlp(*shape, max_rows=max(rows, 512))
    w = (np.random.default_rng(3).standard_normal(net.nparam) * 0.3).astype(np.float32)
    net.set_weights(w)
    X, T = data(rows, shape[0], shape[3], 300 + rows)
    g, parts = net.gradients(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev))
    Y = net.forward(torch.from_numpy(X).to(dev))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    want = mo.gradients(w.astype(np.float64), shape, X, T, bf16=True)
    for got_b, want_b in zip(mo.split(g, shape), mo.split(want, shape)):
        assert relerr(got_b, want_b) <= 2e-3
    assert relerr(Y.cpu().numpy().astype(np.float64), mo.forward(w.astype(np.float64), shape, X, bf16=True)["Y"]) <= 1e-4
    net.close()


def test_train_steps_match_adam(dev, mo):
    net, w = make_net(seed=2)
    lr = 1e-3
    wo = w.astype(np.float64)
    m1 = np.zeros_like(wo)
    m2 = np.zeros_like(wo)
    for step, rows in ((1, 300), (2, 200)):
        X, T = data(rows, SHAPE[0], SHAPE[3], 7 * step)
        net.train_step(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev), lr)
        g = mo.gradients(wo, SHAPE, X, T, bf16=True)
        w_prev = wo
        wo, m1, m2 = mo.adam_step(wo, g, m1, m2, step, lr)
        got = net.get_weights().astype(np.float64)
        big = np.abs(g) > 1e-2 * np.abs(g).max()
        assert np.max(np.abs((got - w_prev)[big] - (wo - w_prev)[big])) <= 2e-2 * lr
        assert np.max(np.abs(got - wo)) <= 2.5 * lr * step
        wo = got   # continue from the device weights, so small differences do not compound
    net.close()


def test_training_reduces_loss(dev):
    """A smooth synthetic regression target: Adam on the device must fit it."""
    from paper_1902_08653_amd import cdm
    rng = np.random.default_rng(5)
    X = rng.standard_normal((8192, 8)).astype(np.float32)
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 1], np.tanh(X[:, 2] * X[:, 3])], axis=1).astype(np.float32)
    net = cdm.Mlp(8, 128, 128, 2, max_rows=2048)
    net.init(0)
    Xd, Td = torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev)

    def loss():
        tot = 0.0
        for s in range(0, 8192, 2048):
            _, parts = net.gradients(Xd[s:s + 2048], Td[s:s + 2048])
            tot += float(parts.double().sum().cpu())
        return tot / (8192 * 2)

    l0 = loss()
    for ep in range(40):
        for s in range(0, 8192, 1024):
            net.train_step(Xd[s:s + 1024], Td[s:s + 1024], 3e-3)
    l1 = loss()
    print(f"training loss {l0:.4f} -> {l1:.4f}")
    assert l1 < 0.1 * l0
    net.close()


def test_predict_is_chunked_forward(dev, mo):
    """cdm_mlp_predict evaluates in chunks of max_rows; rows are independent, so the
    result equals one forward pass bit for bit, written as complex."""
    from paper_1902_08653_amd import cdm
    X, _ = data(300, 8, 2, 11)
    Xd = torch.from_numpy(X).to(dev)
    a = cdm.Mlp(*SHAPE, max_rows=128)
    b = cdm.Mlp(*SHAPE, max_rows=512)
    w = (np.random.default_rng(4).standard_normal(a.nparam) * 0.3).astype(np.float32)
    a.set_weights(w)
    b.set_weights(w)
    for dt in (torch.complex128, torch.complex64):
        x0 = a.predict(Xd, dt)
        Y = b.forward(Xd)
        torch.cuda.synchronize()
        xr = torch.view_as_real(x0).cpu().numpy()
        assert np.array_equal(xr, Y.cpu().numpy().astype(xr.dtype))
    want = mo.forward(w.astype(np.float64), SHAPE, X, bf16=True)["Y"]
    assert relerr(torch.view_as_real(a.predict(Xd, torch.complex128)).cpu().numpy(), want) <= 1e-4
    a.close()
    b.close()


@pytest.mark.parametrize("shape", [(8, 512, 512, 2), (8, 256, 256, 2), (5, 256, 256, 2)])
@pytest.mark.parametrize("rows", [1, 127, 300, 1000])
def test_fused_predict_vs_oracle(dev, mo, shape, rows):
    """Widths 256 / 512 with two outputs take the fused one-launch inference kernel
    (activations only in LDS).  Same operand rounding as the layered pass, different
    summation order.  A pre-activation summed in another order (FP32 here, FP64 in the
    oracle) can round to the neighbouring BF16 value, which moves that row's output by
    about one BF16 ulp of one term; so the bars are 5e-4 relative over the whole
    output and at most 2% of rows off by more than 1e-4 of their norm, against the
    BF16-operand oracle and against the layered forward pass of the same weights.  Row
    counts cover one partial tile, several tiles and a ragged tail."""
    from paper_1902_08653_amd import cdm
    nin = shape[0]
    X, _ = data(rows, nin, 2, 17 + rows)
    Xd = torch.from_numpy(X).to(dev)
    net = cdm.Mlp(*shape, max_rows=1024)
    rng = np.random.default_rng(6)
    w = (rng.standard_normal(net.nparam) * np.sqrt(2.0 / shape[1])).astype(np.float32)
    net.set_weights(w)
    want = mo.forward(w.astype(np.float64), shape, X, bf16=True)["Y"]
    Y = net.forward(Xd).cpu().numpy().astype(np.float64)
    for dt in (torch.complex128, torch.complex64):
        x0 = net.predict(Xd, dt)
        torch.cuda.synchronize()
        got = torch.view_as_real(x0).cpu().numpy().astype(np.float64)
        for ref in (want, Y):
            assert relerr(got, ref) <= 5e-4
            row = np.linalg.norm(got - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-6)
            assert np.mean(row > 1e-4) <= 0.02
    net.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_features_vs_oracle(dev, mo, prec):
    from paper_1902_08653_amd import cdm
    dt = np.complex128 if prec == "c128" else np.complex64
    insts = [inputs.batch_instance(i, seed0=300, m_lo=64, m_hi=300, dtype=dt) for i in range(23)]
    Hf, yf, m, n, *_ = inputs.pack_batch(insts, dt)
    plan = cdm.BatchedPlan(m, n, precision=prec, T_max=1)
    F = plan.features(torch.from_numpy(Hf).to(dev), torch.from_numpy(yf).to(dev), N0=0.1, Ex=1.0)
    torch.cuda.synchronize()
    got = F.cpu().numpy().astype(np.float64)
    want = mo.features([(ins.H.astype(np.complex128), ins.y.astype(np.complex128)) for ins in insts], 0.1)
    assert got.shape == want.shape
    assert np.all(np.abs(got - want) <= 1e-6 * np.maximum(1.0, np.abs(want)))
    plan.close()


def test_warm_start_end_to_end(dev, orc):
    """Miniature of the learned warm start: train on solved instances of the uneven
    distribution (m in 64..256), then solve held-out instances cold and warm to a
    relative step of 1e-8.  Both must reach the oracle's converged solution; the
    sweep counts are reported, and the warm start must not cost sweeps on average."""
    from paper_1902_08653_amd import cdm
    from paper_1902_08653_amd.warmstart import WarmStart
    lam = 0.1
    # training set: seeds disjoint from the held-out ones
    Htr, ytr, mtr, ntr = inputs.batch_uneven_device(384, seed0=1_000_000, m_lo=64, m_hi=256,
                                                    dtype=torch.complex128, device=dev)
    ptr = cdm.BatchedPlan(mtr, ntr, precision="c128", T_max=500, tol=1e-11)
    xs, _ = ptr.solve(Htr, ytr, N0=lam)
    ws = WarmStart(hidden=512, max_rows=16384, seed=0)
    F, T = ws.training_rows(ptr, Htr, ytr, xs, N0=lam)
    hist = ws.fit(F, T, epochs=30, batch=2048, lr=1e-3, seed=0)
    print("warm-start training loss per epoch:", ["%.4f" % h for h in hist[::5]], "%.4f" % hist[-1])
    assert hist[-1] < hist[0]
    # held-out set on the host, so the oracle sees the same values
    insts = [inputs.batch_instance(i, seed0=0, m_lo=64, m_hi=256) for i in range(64)]
    Hf, yf, m, n, _, _, x_off = inputs.pack_batch(insts)
    Hd, yd = torch.from_numpy(Hf).to(dev), torch.from_numpy(yf).to(dev)
    plan = cdm.BatchedPlan(m, n, precision="c128", T_max=500, tol=1e-8)
    xc, ic = plan.solve(Hd, yd, N0=lam)
    xw, iw = ws.solve(plan, Hd, yd, N0=lam)
    torch.cuda.synchronize()
    ic, iw = cdm.parse_info(ic), cdm.parse_info(iw)
    assert not np.any(ic["flags"] & 4) and not np.any(iw["flags"] & 4)
    sc, sw = ic["sweeps"].astype(float), iw["sweeps"].astype(float)
    print(f"held-out sweeps to 1e-8: cold mean {sc.mean():.2f} median {np.median(sc):.1f}, "
          f"warm mean {sw.mean():.2f} median {np.median(sw):.1f}")
    xc, xw = xc.cpu().numpy(), xw.cpu().numpy()
    for k in range(0, 64, 8):
        ref = orc.local_cd(insts[k].H, insts[k].y, lam, 2000, tol=1e-14)["x"]
        sl = slice(int(x_off[k]), int(x_off[k]) + int(n[k]))
        assert relerr(xc[sl], ref) <= 1e-6
        assert relerr(xw[sl], ref) <= 1e-6
    assert sw.mean() <= sc.mean()
    ws.close()
    plan.close()
    ptr.close()
