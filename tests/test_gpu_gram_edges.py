"""GPU parity at shapes that reach the edges of the panel Gram kernels (the pre-pass that
forms the panel blocks H_K^H H_K and H_K^H H_{K-1} on the matrix cores):

* complex128 (FP64 MFMA) and complex64 (FP32 MFMA): a row count that is not a multiple of
  the kernel's 32-row step, a ragged last panel, and a padded leading dimension (ldh > B,
  the padding filled with values that must not be read), for the one-panel and (complex128)
  the two-panel look-ahead schedules (the latter also forms the distance-two blocks);
* BF16 and FP8 copies (mixed-precision refinement): B = 8196, not a multiple of 8 or 16,
  so the copy's columns are not 16-byte aligned and every tile is staged element by
  element, with a ragged last panel and the look-ahead's cross blocks.

Reference: the FP64 oracle's Alg. 1 (local CD) at the same sweep count (complex128, bar
1e-10; complex64 on the FP32-rounded inputs, bar 1e-5), or its converged solution (mixed
precision, bar 1e-10 as for the full-size mixed forms).
"""
import numpy as np
import pytest

from paper_1902_08653_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_08653_amd import cdm
    cdm.lib()
    return torch.device("cuda:0")


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def padded(H, pad, seed):
    """H^T (U x B) stored with leading dimension B + pad; the padding holds large values."""
    U, B = H.shape[1], H.shape[0]
    rng = np.random.default_rng(seed)
    buf = (rng.standard_normal((U, B + pad)) * 1e6).astype(np.complex128)
    buf[:, :B] = H.T
    return buf


@pytest.mark.parametrize("lookahead", [True, "deep"])
def test_c128_unaligned_rows_ragged_panel_padded_ld(dev, orc, lookahead):
    from paper_1902_08653_amd import cdm
    B, U, T = 4133, 700, 3
    inst = inputs.dense_uplink(B, U, 41)
    plan = cdm.Plan(B, U, precision="c128", T_max=T, tol=0.0, lookahead=lookahead)
    desc = plan.describe()
    assert '"schedule": "lookahead"' in desc, desc
    if lookahead == "deep":
        assert '"lookahead_panels": 2' in desc, desc
    Hd = torch.from_numpy(padded(inst.H, 3, 7)).to(dev)
    assert Hd.shape[1] == B + 3
    yd = torch.from_numpy(inst.y).to(dev)
    x, info = plan.solve(Hd, yd, N0=0.1)
    torch.cuda.synchronize()
    rec = cdm.parse_info(info)[0]
    plan.close()
    ref = orc.local_cd(inst.H, inst.y, 0.1, T)
    assert rec["sweeps"] == T and rec["flags"] == 0
    assert relerr(x.cpu().numpy(), ref["x"]) <= 1e-10


def test_c64_unaligned_rows_ragged_panel_padded_ld(dev, orc):
    from paper_1902_08653_amd import cdm
    B, U, T = 4133, 700, 3
    inst = inputs.dense_uplink(B, U, 45)
    plan = cdm.Plan(B, U, precision="c64", T_max=T, tol=0.0, engine="panel")
    desc = plan.describe()
    assert '"schedule": "lookahead"' in desc, desc
    Hd = torch.from_numpy(padded(inst.H, 5, 9).astype(np.complex64)).to(dev)
    assert Hd.shape[1] == B + 5
    yd = torch.from_numpy(inst.y.astype(np.complex64)).to(dev)
    x, info = plan.solve(Hd, yd, N0=0.1)
    torch.cuda.synchronize()
    rec = cdm.parse_info(info)[0]
    plan.close()
    Ho = inst.H.astype(np.complex64).astype(np.complex128)
    yo = inst.y.astype(np.complex64).astype(np.complex128)
    ref = orc.local_cd(Ho, yo, 0.1, T)
    assert rec["sweeps"] == T and rec["flags"] == 0
    assert relerr(x.cpu().numpy().astype(np.complex128), ref["x"]) <= 1e-5


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_mixed_unaligned_copy_ragged_panel(dev, orc, kind):
    from paper_1902_08653_amd import cdm
    B, U = 8196, 700
    inst = inputs.dense_uplink(B, U, 43)
    plan = cdm.Plan(B, U, precision=kind, T_max=60, tol=1e-12)
    desc = plan.describe()
    assert '"schedule": "lookahead"' in desc, desc
    Hd = torch.from_numpy(np.ascontiguousarray(inst.H.T)).to(dev)
    yd = torch.from_numpy(inst.y).to(dev)
    x, info = plan.solve(Hd, yd, N0=0.1)
    torch.cuda.synchronize()
    rec = cdm.parse_info(info)[0]
    plan.close()
    ref = orc.local_cd(inst.H, inst.y, 0.1, T_max=2000, tol=1e-14)
    assert rec["flags"] == 0 and rec["rel_step"] <= 1e-12
    assert relerr(x.cpu().numpy(), ref["x"]) <= 1e-10
