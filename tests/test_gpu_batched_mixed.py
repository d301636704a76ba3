"""GPU parity of the mixed-precision batched engine (cdm_create_batched with
CDM_MIXED_C64 / CDM_MIXED_BF16).

Each instance runs FP64 outer steps (r = y - H x, g = H^H r - lambda x) around FP32
inner CD sweeps from a complex64 or BF16 copy of H.  Its fixed point is the FP64
stationarity of eq. (1), so the bar is the FP64 solution itself: the oracle's CD run
to a relative step of 1e-14 (a closed form up to rounding), compared per instance at
1e-9 relative for an outer tolerance of 1e-11.  Ragged sizes put rows past the last
full tile in every instance; the largest instance uses the 8-rows-per-thread tile.
"""
import numpy as np
import pytest

from paper_1902_08653_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ["mixed-c64", "mixed-bf16"]
_NAME = {"mixed-c64": "mixed-c64", "mixed-bf16": "bf16"}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_08653_amd import cdm
    cdm.lib()
    return torch.device("cuda:0")


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def exact(orc, inst):
    return orc.local_cd(inst.H, inst.y, 0.1, T_max=5000, tol=1e-14)["x"]


def solve(dev, ins, prec, tol=1e-11, x0=None, residual=False, autotune=False, T_max=30):
    from paper_1902_08653_amd import cdm
    Hf, yf, m, n, ho, yo, xo = inputs.pack_batch(ins, dtype=np.complex128)
    plan = cdm.BatchedPlan(m, n, precision=_NAME[prec], T_max=T_max, tol=tol, residual=residual,
                           autotune=autotune)
    desc = plan.describe()
    H = torch.from_numpy(Hf).to(dev)
    y = torch.from_numpy(yf).to(dev)
    x0d = None if x0 is None else torch.from_numpy(np.concatenate(x0).astype(np.complex128)).to(dev)
    x, info = plan.solve(H, y, N0=0.1, x0=x0d)
    torch.cuda.synchronize()
    out = x.cpu().numpy(), cdm.parse_info(info), xo, n, desc
    plan.close()
    return out


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_batched_reaches_fp64_solution(dev, orc, prec):
    ins = [inputs.batch_instance(i, m_lo=64, m_hi=900) for i in range(30)]
    x, rec, xo, n, desc = solve(dev, ins, prec)
    assert '"engine": "wg-batched-mixed"' in desc, desc
    for k, inst in enumerate(ins):
        assert rec["flags"][k] == 0, (k, rec[k])
        assert 1 <= rec["sweeps"][k] <= rec["reserved"][k]
        # the last outer correction is below tol, or its geometric successor is
        # (c_s^2 / c_{s-1} <= tol with c_{s-1} <= 1)
        assert rec["rel_step"][k] <= np.sqrt(1e-11)
        assert relerr(x[xo[k]:xo[k] + n[k]], exact(orc, inst)) <= 1e-9, k


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_batched_largest_tile(dev, orc, prec):
    """m = 2048 (4 rows per thread on 512 threads), n = 1 and n = 3, next to other instances."""
    rng = np.random.default_rng(5)
    shapes = [(2048, 1100), (65, 32), (1500, 700), (64, 1), (1025, 3)]
    ins = []
    for mi, ni in shapes:
        H = (rng.standard_normal((mi, ni)) + 1j * rng.standard_normal((mi, ni))) / np.sqrt(2 * mi)
        y = (rng.standard_normal(mi) + 1j * rng.standard_normal(mi)) / np.sqrt(2)
        ins.append(inputs.DenseInstance(H=H, y=y, seed=-1))
    x, rec, xo, n, _ = solve(dev, ins, prec)
    for k, inst in enumerate(ins):
        assert rec["flags"][k] == 0
        assert relerr(x[xo[k]:xo[k] + n[k]], exact(orc, inst)) <= 1e-9, k


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_batched_warm_start(dev, orc, prec):
    """From a start near the solution the refinement needs fewer outer steps and
    reaches the same point."""
    ins = [inputs.batch_instance(i, m_lo=64, m_hi=600) for i in range(12)]
    ex = [exact(orc, inst) for inst in ins]
    rng = np.random.default_rng(2)
    x0 = [e + 1e-4 * (rng.standard_normal(e.shape) + 1j * rng.standard_normal(e.shape)) for e in ex]
    xc, rc, xo, n, _ = solve(dev, ins, prec)
    xw, rw, _, _, _ = solve(dev, ins, prec, x0=x0)
    for k in range(len(ins)):
        assert relerr(xw[xo[k]:xo[k] + n[k]], ex[k]) <= 1e-9
    assert rw["reserved"].sum() < rc["reserved"].sum()


def test_mixed_batched_fp64_residual(dev, orc):
    ins = [inputs.batch_instance(i, m_lo=64, m_hi=500) for i in range(8)]
    x, rec, xo, n, _ = solve(dev, ins, "mixed-c64", residual=True)
    for k, inst in enumerate(ins):
        want = orc.normal_residual(inst.H, inst.y, 0.1, x[xo[k]:xo[k] + n[k]])
        assert abs(rec["resid"][k] - want) <= 1e-6 * want + 1e-15
        assert rec["resid"][k] <= 1e-10


def test_mixed_batched_outer_cap_flags(dev, orc):
    """T_max caps the outer steps; an instance that does not reach tol is flagged."""
    ins = [inputs.batch_instance(i, m_lo=200, m_hi=400) for i in range(4)]
    x, rec, xo, n, _ = solve(dev, ins, "mixed-bf16", tol=1e-13, T_max=1)
    assert np.all(rec["sweeps"] == 1)
    assert np.all(rec["flags"] & 4)


def test_mixed_batched_autotune_and_graph_replay(dev, orc):
    from paper_1902_08653_amd import cdm
    ins = [inputs.batch_instance(i, m_lo=64, m_hi=900) for i in range(40)]
    Hf, yf, m, n, ho, yo, xo = inputs.pack_batch(ins, dtype=np.complex128)
    plan = cdm.BatchedPlan(m, n, precision="mixed-c64", T_max=12, tol=1e-10, autotune=True)
    assert '"autotune_ms": {' in plan.describe()
    H = torch.from_numpy(Hf).to(dev)
    y = torch.from_numpy(yf).to(dev)
    x_e, info_e = plan.solve(H, y, N0=0.1)
    torch.cuda.synchronize()
    ref_x = x_e.cpu().numpy()
    x = torch.zeros_like(x_e)
    info = torch.zeros_like(info_e)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.solve(H, y, N0=0.1, x=x, info=info)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.solve(H, y, N0=0.1, x=x, info=info)
    for rep in range(3):
        x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), ref_x), rep
        _ = (H[:10] * 2).sum().item()
    for k in [0, 21, 39]:
        assert relerr(ref_x[xo[k]:xo[k] + n[k]], exact(orc, ins[k])) <= 1e-8
    plan.close()
