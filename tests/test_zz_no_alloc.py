"""cdm_solve_noalloc (the entry point that allocates nothing) against the plan-based
cdm_create + cdm_solve, through the C ABI.

Both run the same per-cluster kernels with the same launch shape, so the outputs must
agree to the parity bar (1e-10 complex128, 1e-5 complex64; they are in fact expected
to be identical) and the sweep counts and flags exactly.  Two calls in a row, the
second with a smaller input, show that the static scratch carries nothing from one
call into the next.  Sizes beyond the static array are rejected before any launch.
"""
import numpy as np
import pytest

from paper_1902_08653_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DT = {"c128": np.complex128, "c64": np.complex64}
TOL = {"c128": 1e-10, "c64": 1e-5}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_08653_amd import cdm
    cdm.lib()
    return torch.device("cuda:0")


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _case(B, U, seed, prec, dev):
    inst = inputs.dense_uplink(B, U, seed=seed)
    Hd = torch.from_numpy(np.ascontiguousarray(inst.H.T).astype(DT[prec])).to(dev)
    yd = torch.from_numpy(inst.y.astype(DT[prec])).to(dev)
    return inst, Hd, yd


def _with_plan(Hd, yd, B, U, C, Bc, prec, T, tol, lambda_c=None, problem="uplink", rho=0.0, N0=0.1):
    from paper_1902_08653_amd import cdm
    plan = cdm.Plan(B, U, C_clusters=C, precision=prec, T_max=T, tol=tol, Bc=Bc, problem=problem,
                    engine="wg")
    x, info = plan.solve(Hd, yd, N0=N0, rho=rho, lambda_c=lambda_c)
    torch.cuda.synchronize()
    out = x.cpu().numpy(), cdm.parse_info(info)
    plan.close()
    return out


def _no_alloc(Hd, yd, B, U, C, Bc, prec, T, tol, lambda_c=None, problem="uplink", rho=0.0, N0=0.1):
    from paper_1902_08653_amd import cdm
    x, info = cdm.solve_noalloc(Hd, yd, B, U, C_clusters=C, Bc=Bc, precision=prec, T_max=T, tol=tol,
                                problem=problem, N0=N0, rho=rho, lambda_c=lambda_c)
    torch.cuda.synchronize()
    return x.cpu().numpy(), cdm.parse_info(info)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_no_alloc_matches_plan_twice_then_smaller(dev, prec):
    # first call: 5 uneven clusters, 48 users, tolerance mode
    big = dict(B=5 * 96 + 17, U=48, C=5, Bc=[96, 96, 113, 96, 96], T=200, tol=1e-9 if prec == "c128" else 1e-5)
    # second call, right after: a smaller input (fewer clusters, rows and users), fixed sweeps
    small = dict(B=2 * 40, U=16, C=2, Bc=None, T=3, tol=0.0)
    for k, cfg in enumerate([big, small]):
        inst, Hd, yd = _case(cfg["B"], cfg["U"], 30 + k, prec, dev)
        xa, ia = _no_alloc(Hd, yd, cfg["B"], cfg["U"], cfg["C"], cfg["Bc"], prec, cfg["T"], cfg["tol"])
        xb, ib = _with_plan(Hd, yd, cfg["B"], cfg["U"], cfg["C"], cfg["Bc"], prec, cfg["T"], cfg["tol"])
        assert np.array_equal(ia["sweeps"], ib["sweeps"]) and np.array_equal(ia["flags"], ib["flags"])
        assert relerr(xa, xb) <= TOL[prec]
        assert np.all(np.isfinite(xa))


def test_no_alloc_single_cluster_caller_weights_and_downlink(dev):
    # C = 1 (no fusion), then C = 4 with caller weights, then the downlink precoder
    inst, Hd, yd = _case(300, 40, 7, "c128", dev)
    xa, ia = _no_alloc(Hd, yd, 300, 40, 1, None, "c128", 4, 0.0)
    xb, ib = _with_plan(Hd, yd, 300, 40, 1, None, "c128", 4, 0.0)
    assert relerr(xa, xb) <= 1e-10 and np.array_equal(ia["sweeps"], ib["sweeps"])
    w = torch.tensor([0.4, 0.0, 0.35, 0.25], dtype=torch.float64, device=dev)
    inst, Hd, yd = _case(4 * 32, 8, 8, "c128", dev)
    xa, _ = _no_alloc(Hd, yd, 128, 8, 4, None, "c128", 3, 0.0, lambda_c=w)
    xb, _ = _with_plan(Hd, yd, 128, 8, 4, None, "c128", 3, 0.0, lambda_c=w)
    assert relerr(xa, xb) <= 1e-10
    s = torch.from_numpy(inputs.dense_uplink(8, 1, seed=9).y[:8]).to(dev)
    xa, _ = _no_alloc(Hd, s, 128, 8, 4, [24, 40, 32, 32], "c128", 3, 0.0, problem="downlink", rho=1.5)
    xb, _ = _with_plan(Hd, s, 128, 8, 4, [24, 40, 32, 32], "c128", 3, 0.0, problem="downlink", rho=1.5)
    assert relerr(xa, xb) <= 1e-10


def test_no_alloc_rejects_sizes_beyond_the_scratch(dev):
    from paper_1902_08653_amd import cdm
    inst, Hd, yd = _case(65 * 2, 4, 1, "c64", dev)
    with pytest.raises(cdm.CdmError) as e:           # more clusters than the records hold
        _no_alloc(Hd, yd, 130, 4, 65, None, "c64", 2, 0.0)
    assert e.value.status == -2
    # 64 clusters x 8192 users x 16 B = 8 MiB of local estimates > 4 MiB
    B, U = 64 * 8192, 8192
    H = torch.zeros(1, dtype=torch.complex128, device=dev)   # never read: rejected first
    y = torch.zeros(1, dtype=torch.complex128, device=dev)
    with pytest.raises(cdm.CdmError) as e:
        cdm.solve_noalloc(H, y, B, U, C_clusters=64, precision="c128", T_max=1)
    assert e.value.status == -2
    assert b"static scratch" in cdm.lib().cdm_last_error()
