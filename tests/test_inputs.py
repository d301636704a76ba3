"""Seeded generators: reproducibility, layout and the stated distributions."""
import numpy as np

from paper_1902_08653_amd import inputs


def test_dense_layout_and_seed():
    a = inputs.dense_uplink(64, 32, 0)
    b = inputs.dense_uplink(64, 32, 0)
    assert a.H.shape == (64, 32) and a.H.flags.f_contiguous
    assert np.array_equal(a.H, b.H) and np.array_equal(a.y, b.y)
    c = inputs.dense_uplink(64, 32, 1)
    assert not np.array_equal(a.H, c.H)


def test_dense_variance():
    a = inputs.dense_uplink(2048, 256, 3)
    col = np.mean(np.abs(a.H) ** 2, axis=0) * 2048
    assert abs(col.mean() - 1.0) < 0.01
    assert abs(np.mean(a.H.real ** 2) * 2 * 2048 - 1.0) < 0.02
    assert abs(np.mean(np.abs(a.y) ** 2) - 1.0) < 0.1


def test_sparse_pattern_and_scaling():
    s = inputs.sparse_uplink(2000, 500, 0.01, seed=2)
    nnz = s.rowptr[-1]
    assert abs(nnz / (2000 * 500) - 0.01) < 0.001
    for i in range(0, 2000, 97):
        cols = s.colidx[s.rowptr[i]:s.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
    e = np.zeros(500)
    np.add.at(e, s.colidx, np.abs(s.val) ** 2)
    assert abs(e.mean() - 1.0) < 0.05


def test_batch_sizes_and_instances():
    m, n = inputs.batch_sizes(64, 0)
    assert np.all((m >= 64) & (m <= 2048)) and np.array_equal(n, m // 2)
    ins = inputs.batch_instance(5, 0)
    assert ins.B == m[5] and ins.U == n[5]
    Hf, yf, mm, nn, ho, yo, xo = inputs.pack_batch([inputs.batch_instance(i) for i in range(4)])
    i = 2
    Hi = Hf[ho[i]:ho[i] + mm[i] * nn[i]].reshape(nn[i], mm[i]).T
    assert np.array_equal(Hi, inputs.batch_instance(i).H)


def test_qam16_unit_energy():
    bits = np.array(np.meshgrid(*[[0, 1]] * 4)).reshape(4, -1).T
    sym = inputs.qam16_symbols(bits)
    assert len(set(np.round(sym, 12))) == 16
    assert abs(np.mean(np.abs(sym) ** 2) - 1.0) < 1e-12
