"""Parity at the full single-instance size (B = 16384, U = 8192, seed 1), in the
launch configuration the benchmark times (auto engine = cooperative panel engine).

The oracle runs the same number of sweeps on the same inputs; the converged
tolerance-mode result is checked against the FP64 stationarity condition of
eq. (1) on the GPU and against the oracle's own converged solution elsewhere
(bench.py), which takes ~40 s of CPU.
"""
import numpy as np
import pytest

from paper_1902_08653_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B, U, SEED, LAM = 16384, 8192, 1, 0.1


@pytest.fixture(scope="module")
def inst():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return inputs.dense_uplink(B, U, SEED)


@pytest.mark.parametrize("prec,bar", [("c128", 1e-10), ("c64", 1e-5)])
def test_fullsize_two_sweeps_match_oracle(inst, orc, prec, bar):
    from paper_1902_08653_amd import cdm
    dt = np.complex128 if prec == "c128" else np.complex64
    dev = torch.device("cuda:0")
    plan = cdm.Plan(B, U, precision=prec, T_max=2, tol=0.0)
    assert '"engine": "panel"' in plan.describe()
    Hc = torch.from_numpy(np.ascontiguousarray(inst.H.T).astype(dt, copy=False)).to(dev)
    y = torch.from_numpy(inst.y.astype(dt)).to(dev)
    x, info = plan.solve(Hc, y, N0=LAM, Ex=1.0)
    torch.cuda.synchronize()
    rec = cdm.parse_info(info)[0]
    xg = x.cpu().numpy().astype(np.complex128)
    del Hc
    H64 = inst.H if prec == "c128" else inst.H.astype(dt).astype(np.complex128)
    y64 = inst.y if prec == "c128" else inst.y.astype(dt).astype(np.complex128)
    ref = orc.local_cd(H64, y64, LAM, T_max=2)
    err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
    print(prec, plan.describe(), "err", err)
    assert rec["sweeps"] == 2 and rec["flags"] == 0
    assert err <= bar
    plan.close()


def test_fullsize_tolerance_mode_stationarity(inst):
    """Converged solve (rel. step <= 1e-11): the FP64 normal-equation residual of
    eq. (1) is at the level the step implies, and the GPU stopped by its own rule."""
    from paper_1902_08653_amd import cdm
    dev = torch.device("cuda:0")
    plan = cdm.Plan(B, U, precision="c128", T_max=200, tol=1e-11, residual=True)
    Hc = torch.from_numpy(np.ascontiguousarray(inst.H.T)).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    x, info = plan.solve(Hc, y, N0=LAM, Ex=1.0)
    torch.cuda.synchronize()
    rec = cdm.parse_info(info)[0]
    print("sweeps", rec["sweeps"], "rel_step", rec["rel_step"], "resid", rec["resid"])
    assert rec["flags"] == 0 and rec["rel_step"] <= 1e-11
    assert 20 <= rec["sweeps"] <= 120
    assert rec["resid"] <= 1e-10
    plan.close()
