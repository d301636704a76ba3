"""GPU parity of the decentralized form of Algorithm 1 at the C ABI: uneven clusters
(cdm_desc.Bc), caller fusion weights (cdm_solve lambda_c), a dropped cluster, the
N0 = 0 limit of the Sec. III weights, and the data-dependent info flags (NaN/Inf
input, no convergence within T_max) on the plain product path.

Bars: 1e-10 relative (complex128) and 1e-5 (complex64, oracle on the FP32-rounded
inputs) at the same sweep count; sweep counts and flags exact.
"""
import numpy as np
import pytest

from paper_1902_08653_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DT = {"c128": np.complex128, "c64": np.complex64}
TOL = {"c128": 1e-10, "c64": 1e-5}
INFO_ZERO_COLUMN, INFO_NONFINITE, INFO_NOT_CONVERGED = 1, 2, 4


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_08653_amd import cdm
    cdm.lib()
    return torch.device("cuda:0")


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def rounded(a, prec):
    return np.asarray(a).astype(DT[prec]).astype(np.complex128)


def solve(dev, H, y, prec="c128", T=3, tol=0.0, lam=0.1, C=1, Bc=None, lambda_c=None, x0=None,
          engine="auto", problem="uplink", rho=0.0):
    from paper_1902_08653_amd import cdm
    B, U = H.shape
    plan = cdm.Plan(B, U, C_clusters=C, precision=prec, T_max=T, tol=tol, engine=engine, Bc=Bc,
                    problem=problem)
    Hd = torch.from_numpy(np.ascontiguousarray(H.T).astype(DT[prec])).to(dev)
    yd = torch.from_numpy(np.asarray(y).astype(DT[prec])).to(dev)
    wd = None if lambda_c is None else torch.tensor(np.asarray(lambda_c, np.float64), device=dev)
    x0d = None if x0 is None else torch.from_numpy(np.asarray(x0).astype(DT[prec])).to(dev)
    x, info = plan.solve(Hd, yd, N0=lam, Ex=1.0, rho=rho, lambda_c=wd, x0=x0d)
    torch.cuda.synchronize()
    out = x.cpu().numpy().astype(np.complex128), cdm.parse_info(info), plan.describe()
    plan.close()
    return out


# uneven cluster sizes (Sec. II-A allows any partition of the antennas into C blocks)
SIZES = [[40, 56, 32], [1, 63, 64, 17], [128], [300, 212], [13, 13, 13, 13, 13, 13, 13, 13]]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("sizes", SIZES)
@pytest.mark.parametrize("T", [1, 3])
def test_uneven_clusters_match_oracle(dev, orc, prec, sizes, T):
    B, U = sum(sizes), 12
    inst = inputs.dense_uplink(B, U, seed=len(sizes) * 10 + T)
    x, info, desc = solve(dev, inst.H, inst.y, prec, T=T, C=len(sizes), Bc=sizes)
    assert '"engine": "wg"' in desc
    ref = orc.uplink_cd(rounded(inst.H, prec), rounded(inst.y, prec), N0=0.1, Ex=1.0, T_max=T,
                        C_clusters=len(sizes), Bc=sizes)
    assert np.all(info["sweeps"] == T)
    assert np.all(info["flags"] == 0)
    assert relerr(x, ref["x"]) <= TOL[prec]


def test_uneven_clusters_tolerance_mode(dev, orc):
    sizes = [200, 330, 70]
    inst = inputs.dense_uplink(sum(sizes), 48, seed=3)
    x, info, _ = solve(dev, inst.H, inst.y, "c128", T=200, tol=1e-9, C=3, Bc=sizes)
    ref = orc.uplink_cd(inst.H, inst.y, N0=0.1, Ex=1.0, T_max=200, tol=1e-9, C_clusters=3, Bc=sizes)
    # each cluster stops on its own; rounding may move a stop by one sweep
    assert np.all(np.abs(info["sweeps"].astype(int) - ref["sweeps"].astype(int)) <= 1)
    assert np.all(info["flags"] == 0)
    if np.array_equal(info["sweeps"], ref["sweeps"]):
        assert relerr(x, ref["x"]) <= 1e-10
    else:
        assert relerr(x, ref["x"]) <= 1e-8


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_caller_fusion_weights(dev, orc, prec):
    sizes = [32, 48, 24, 40]
    inst = inputs.dense_uplink(sum(sizes), 8, seed=12)
    w = np.array([0.1, 0.4, 0.2, 0.3])
    x, info, _ = solve(dev, inst.H, inst.y, prec, T=3, C=4, Bc=sizes, lambda_c=w)
    ref = orc.uplink_cd(rounded(inst.H, prec), rounded(inst.y, prec), N0=0.1, Ex=1.0, T_max=3,
                        C_clusters=4, Bc=sizes, lam_c=w)
    assert relerr(x, ref["x"]) <= TOL[prec]
    # the weights are used as given: the fused x is the weighted sum of the local x
    xl = ref["x_local"]
    assert relerr(x, (w[:, None] * xl).sum(0)) <= TOL[prec]


def test_dropped_cluster(dev, orc):
    """A cluster whose data is lost gets weight 0 and the Sec. III weights of the
    others are renormalised to sum to 1 (the remaining clusters' estimates fused)."""
    sizes = [32, 32, 32, 32]
    inst = inputs.dense_uplink(128, 8, seed=21)
    full = orc.uplink_cd(inst.H, inst.y, N0=0.1, Ex=1.0, T_max=3, C_clusters=4)
    w = full["weights"].copy()
    w[2] = 0.0
    w /= w.sum()
    x, info, _ = solve(dev, inst.H, inst.y, "c128", T=3, C=4, lambda_c=w)
    ref = orc.uplink_cd(inst.H, inst.y, N0=0.1, Ex=1.0, T_max=3, C_clusters=4, lam_c=w)
    assert relerr(x, ref["x"]) <= 1e-10
    # the dropped cluster's local estimate (even a non-finite one) does not enter
    keep = [0, 1, 3]
    want = sum(w[c] * full["x_local"][c] for c in keep)
    assert relerr(x, want) <= 1e-10


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_default_weights_at_zero_noise(dev, orc, prec):
    """N0 = 0 (lambda = 0, every B_c >= U): the Sec. III weights stay finite, since the
    common factor N0/U cancels."""
    sizes = [40, 24, 64]
    inst = inputs.dense_uplink(sum(sizes), 16, seed=5)
    x, info, _ = solve(dev, inst.H, inst.y, prec, T=4, lam=0.0, C=3, Bc=sizes)
    ref = orc.uplink_cd(rounded(inst.H, prec), rounded(inst.y, prec), N0=0.0, Ex=1.0, T_max=4,
                        C_clusters=3, Bc=sizes)
    assert np.all(np.isfinite(x))
    assert np.all(info["flags"] == 0)
    assert relerr(x, ref["x"]) <= TOL[prec]


def test_zero_noise_infeasible_cluster_is_rejected(dev):
    from paper_1902_08653_amd import cdm
    inst = inputs.dense_uplink(64, 16, seed=1)
    with pytest.raises(cdm.CdmError) as e:
        solve(dev, inst.H, inst.y, "c128", T=2, lam=0.0, C=2, Bc=[50, 14])
    assert e.value.status == -6


def test_downlink_uneven_clusters(dev, orc):
    sizes = [24, 40, 16]
    inst = inputs.dense_uplink(sum(sizes), 8, seed=9)
    s = inputs.dense_uplink(8, 1, seed=10).y[:8]
    x, info, _ = solve(dev, inst.H, s, "c128", T=4, C=3, Bc=sizes, problem="downlink", rho=2.0)
    ref = orc.downlink_cd(inst.H, s, rho=2.0, T_max=4, C_clusters=3, Bc=sizes)
    assert relerr(x, ref["x"]) <= 1e-10
    row0 = 0
    for b in sizes:
        assert abs(np.linalg.norm(x[row0:row0 + b]) - 2.0 / np.sqrt(3)) <= 1e-12
        row0 += b


# ---------------------------------------------------------------- info flags
@pytest.mark.parametrize("engine,B,U", [("wg", 600, 200), ("panel", 4096, 300)])
@pytest.mark.parametrize("where", ["H", "y"])
def test_nonfinite_input_is_flagged(dev, engine, B, U, where):
    inst = inputs.dense_uplink(B, U, seed=2)
    H, y = np.array(inst.H), np.array(inst.y)
    if where == "H":
        H[B // 3, U // 2] = np.nan
    else:
        y[B // 2] = np.inf
    x, info, desc = solve(dev, H, y, "c128", T=2, engine=engine)
    assert ('"engine": "%s"' % engine) in desc
    assert info["flags"][0] & INFO_NONFINITE
    assert info["sweeps"][0] == 2
    assert not np.all(np.isfinite(x))


def test_nonfinite_input_in_a_batch_is_flagged_per_instance(dev):
    from paper_1902_08653_amd import cdm
    ins = [inputs.batch_instance(i, m_lo=64, m_hi=300) for i in range(6)]
    Hf, yf, m, n, ho, yo, xo = inputs.pack_batch(ins, dtype=np.complex64)
    Hf = np.array(Hf)
    Hf[ho[3] + 5] = np.nan        # instance 3 only
    plan = cdm.BatchedPlan(m, n, precision="c64", T_max=3)
    x, info = plan.solve(torch.from_numpy(Hf).to(dev), torch.from_numpy(yf).to(dev), N0=0.1)
    torch.cuda.synchronize()
    rec = cdm.parse_info(info)
    assert [bool(f & INFO_NONFINITE) for f in rec["flags"]] == [k == 3 for k in range(6)]
    plan.close()


@pytest.mark.parametrize("engine,B,U,prec", [("wg", 600, 200, "c128"), ("wg", 600, 200, "c64"),
                                             ("panel", 4096, 300, "c128"), ("panel", 8192, 300, "c64")])
def test_cap_without_convergence_is_flagged(dev, orc, engine, B, U, prec):
    """A plain tolerance-mode solve that reaches T_max without meeting tol reports
    CDM_INFO_NOT_CONVERGED, and x is the oracle's after T_max sweeps."""
    inst = inputs.dense_uplink(B, U, seed=4)
    x, info, desc = solve(dev, inst.H, inst.y, prec, T=3, tol=1e-14, engine=engine)
    assert ('"engine": "%s"' % engine) in desc
    assert info["sweeps"][0] == 3
    assert info["flags"][0] == INFO_NOT_CONVERGED
    assert info["rel_step"][0] > 1e-14
    ref = orc.local_cd(rounded(inst.H, prec), rounded(inst.y, prec), 0.1, T_max=3)
    assert relerr(x, ref["x"]) <= TOL[prec]
