"""GPU parity of the panel engine's look-ahead schedule.

The look-ahead schedule forms panel K+1's partial products before panel K's update
and corrects them with the cross block H_{K+1}^H H_K; in exact arithmetic every
delta equals the sequential sweep's.  Cases: ragged last panels, both precisions,
warm start, tolerance mode, the mixed-precision inner solves, and agreement with the
two-hop schedule (CDM_F_NO_LOOKAHEAD).  The two-panel form (CDM_F_DEEP_LOOKAHEAD:
partials of panel K+3 after panel K, with the distance-two correction applied by the
reducers) is held to the same bars.  Bars as in test_gpu_parity: 1e-10 (c128),
1e-5 (c64, oracle on the FP32-rounded inputs), sweep counts exact at fixed T.
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


def solve(dev, H, y, prec, T, tol=0.0, lookahead=True, x0=None, lam=0.1, panel=0):
    """lookahead: True (one panel ahead), "deep" (two panels ahead where complex128 with
    64-column panels has at least three panels, else one) or False (the two-hop
    schedule)."""
    from paper_1902_08653_amd import cdm
    B, U = H.shape
    plan = cdm.Plan(B, U, precision=prec, T_max=T, tol=tol, engine="panel", lookahead=lookahead, panel=panel)
    desc = plan.describe()
    dt = DT.get(prec, np.complex128)
    Hd = torch.from_numpy(np.ascontiguousarray(H.T).astype(dt)).to(dev)
    yd = torch.from_numpy(np.asarray(y).astype(dt)).to(dev)
    x0d = None if x0 is None else torch.from_numpy(np.asarray(x0).astype(dt)).to(dev)
    x, info = plan.solve(Hd, yd, N0=lam, Ex=1.0, x0=x0d)
    torch.cuda.synchronize()
    out = x.cpu().numpy().astype(np.complex128), cdm.parse_info(info)[0], desc
    plan.close()
    return out


def deep(desc):
    return '"lookahead_panels": 2' in desc


def oracle_in(H, y, prec):
    dt = DT.get(prec, np.complex128)
    return H.astype(dt).astype(np.complex128), np.asarray(y).astype(dt).astype(np.complex128)


# (B, U): the look-ahead needs B >= 64 * panel width: 64 * 64 for complex128 and complex64
# (64-column panels), 64 * 128 for the mixed forms' FP32 inner solve (128-column panels)
# (complex64 and the mixed forms' inner solve gather b of the next step during the step, with
# their own paths for one panel, whose next b needs this step's x, and for two panels)
CASES = [("c128", 4096, 1000), ("c128", 4160, 64), ("c128", 4096, 37), ("c64", 8192, 1000), ("c64", 8192, 200),
         ("c64", 4096, 700), ("c64", 4096, 64), ("c64", 4160, 37), ("c64", 4096, 100)]


@pytest.mark.parametrize("prec,B,U", CASES)
@pytest.mark.parametrize("T", [1, 3])
def test_lookahead_fixed_sweeps_match_oracle(dev, orc, prec, B, U, T):
    inst = inputs.dense_uplink(B, U, 11 + U)
    x, rec, desc = solve(dev, inst.H, inst.y, prec, T)
    assert '"schedule": "lookahead"' in desc, desc
    Ho, yo = oracle_in(inst.H, inst.y, prec)
    ref = orc.local_cd(Ho, yo, 0.1, T)
    assert rec["sweeps"] == T and rec["flags"] == 0
    assert relerr(x, ref["x"]) <= TOL[prec]


@pytest.mark.parametrize("prec,B,U", [("c128", 4096, 1000), ("c64", 8192, 1000)])
def test_lookahead_equals_two_hop(dev, prec, B, U):
    inst = inputs.dense_uplink(B, U, 5)
    xa, ra, da = solve(dev, inst.H, inst.y, prec, 4, lookahead=True)
    xb, rb, db = solve(dev, inst.H, inst.y, prec, 4, lookahead=False)
    assert '"schedule": "lookahead"' in da and '"schedule": "two-hop"' in db
    assert ra["sweeps"] == rb["sweeps"] == 4
    assert relerr(xa, xb) <= TOL[prec]


@pytest.mark.parametrize("B,U", [(4096, 1000), (16448, 700)])
def test_two_hop_64_column_panels(dev, orc, B, U):
    """The two-hop schedule on 64-column complex128 panels (two rows per lane, the planner's
    only 64-column two-hop form; its M_K staging goes through registers), with a ragged last
    row block at B = 16448."""
    rpl = 2
    inst = inputs.dense_uplink(B, U, 17 + U)
    x, rec, desc = solve(dev, inst.H, inst.y, "c128", 3, lookahead=False, panel=64)
    assert '"schedule": "two-hop"' in desc and '"panel": 64' in desc and '"rpl": %d' % rpl in desc, desc
    ref = orc.local_cd(inst.H, inst.y, 0.1, 3)
    assert rec["sweeps"] == 3 and rec["flags"] == 0
    assert relerr(x, ref["x"]) <= 1e-10


def test_lookahead_warm_start(dev, orc):
    inst = inputs.dense_uplink(4096, 1000, 3)
    x0 = np.random.default_rng(1).standard_normal(1000) * 0.3 + 0j
    x, rec, _ = solve(dev, inst.H, inst.y, "c128", 2, x0=x0)
    ref = orc.local_cd(inst.H, inst.y, 0.1, 2, x0=x0)
    assert relerr(x, ref["x"]) <= 1e-10


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_lookahead_tolerance_mode(dev, orc, prec):
    B, U = (4096, 1000) if prec == "c128" else (8192, 1000)
    inst = inputs.dense_uplink(B, U, 8)
    tol = 1e-9 if prec == "c128" else 1e-5
    x, rec, _ = solve(dev, inst.H, inst.y, prec, 300, tol=tol)
    Ho, yo = oracle_in(inst.H, inst.y, prec)
    ref = orc.local_cd(Ho, yo, 0.1, 300, tol=tol)
    assert rec["flags"] == 0 and rec["rel_step"] <= tol
    assert abs(int(rec["sweeps"]) - int(ref["sweeps"])) <= 1
    at = orc.local_cd(Ho, yo, 0.1, int(rec["sweeps"]))
    assert relerr(x, at["x"]) <= TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lookahead_mixed_refinement(dev, orc, prec):
    """Mixed precision on the look-ahead inner solves reaches the FP64 solution, to the
    1e-10 bar of the full-size mixed forms."""
    inst = inputs.dense_uplink(8192, 1000, 21)
    x, rec, desc = solve(dev, inst.H, inst.y, prec, 60, tol=1e-12)
    assert '"schedule": "lookahead"' in desc, desc
    ref = orc.local_cd(inst.H, inst.y, 0.1, 2000, tol=1e-14)
    assert rec["flags"] == 0 and rec["rel_step"] <= 1e-12
    assert relerr(x, ref["x"]) <= 1e-10


@pytest.mark.parametrize("prec,U", [("bf16", 100), ("fp8", 128), ("bf16", 200), ("fp8", 250)])
def test_lookahead_mixed_one_or_two_panels(dev, orc, prec, U):
    """The mixed forms' inner solve (128-column FP32 panels) with one panel (ragged and
    full) and two panels (the second ragged), to the FP64 solution at the 1e-10 bar."""
    inst = inputs.dense_uplink(8192, U, 31 + U)
    x, rec, desc = solve(dev, inst.H, inst.y, prec, 60, tol=1e-12)
    assert '"schedule": "lookahead"' in desc, desc
    ref = orc.local_cd(inst.H, inst.y, 0.1, 2000, tol=1e-14)
    assert rec["flags"] == 0 and rec["rel_step"] <= 1e-12
    assert relerr(x, ref["x"]) <= 1e-10


# complex128, two panels ahead: three panels, a ragged fourth, many panels
DEEP_CASES = [(4096, 192), (4096, 200), (4160, 1000), (8192, 515)]


@pytest.mark.parametrize("B,U", DEEP_CASES)
@pytest.mark.parametrize("T", [1, 2, 5])
def test_two_panel_lookahead_matches_oracle(dev, orc, B, U, T):
    inst = inputs.dense_uplink(B, U, 31 + U)
    x, rec, desc = solve(dev, inst.H, inst.y, "c128", T, lookahead="deep")
    assert deep(desc), desc
    ref = orc.local_cd(inst.H, inst.y, 0.1, T)
    assert rec["sweeps"] == T and rec["flags"] == 0
    assert relerr(x, ref["x"]) <= 1e-10


@pytest.mark.parametrize("B,U", [(4096, 200), (4096, 1000)])
def test_two_panel_lookahead_equals_one_panel_and_two_hop(dev, B, U):
    inst = inputs.dense_uplink(B, U, 6)
    xd, rd, dd = solve(dev, inst.H, inst.y, "c128", 4, lookahead="deep")
    xs, rs, ds = solve(dev, inst.H, inst.y, "c128", 4)
    xt, rt, dt = solve(dev, inst.H, inst.y, "c128", 4, lookahead=False)
    assert deep(dd) and '"lookahead_panels": 1' in ds and '"schedule": "two-hop"' in dt
    assert rd["sweeps"] == rs["sweeps"] == rt["sweeps"] == 4
    assert relerr(xd, xs) <= 1e-10 and relerr(xd, xt) <= 1e-10


def test_two_panel_lookahead_warm_start_and_tolerance(dev, orc):
    inst = inputs.dense_uplink(4096, 600, 4)
    x0 = np.random.default_rng(2).standard_normal(600) * 0.3 + 0j
    x, rec, desc = solve(dev, inst.H, inst.y, "c128", 3, x0=x0, lookahead="deep")
    assert deep(desc)
    ref = orc.local_cd(inst.H, inst.y, 0.1, 3, x0=x0)
    assert relerr(x, ref["x"]) <= 1e-10
    x, rec, _ = solve(dev, inst.H, inst.y, "c128", 300, tol=1e-10, lookahead="deep")
    ref = orc.local_cd(inst.H, inst.y, 0.1, 300, tol=1e-10)
    assert rec["flags"] == 0 and abs(int(rec["sweeps"]) - int(ref["sweeps"])) <= 1
    at = orc.local_cd(inst.H, inst.y, 0.1, int(rec["sweeps"]))
    assert relerr(x, at["x"]) <= 1e-10


def test_one_or_two_panels_keep_the_one_panel_schedule(dev, orc):
    for U in (64, 128):
        inst = inputs.dense_uplink(4096, U, U)
        x, rec, desc = solve(dev, inst.H, inst.y, "c128", 3, lookahead="deep")
        assert '"lookahead_panels": 1' in desc, desc
        assert relerr(x, orc.local_cd(inst.H, inst.y, 0.1, 3)["x"]) <= 1e-10
