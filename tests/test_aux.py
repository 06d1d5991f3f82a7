"""Host-side helpers: CSR validation, problem cache and SPAI parameter files with checksums."""
import numpy as np
import pytest

import paper_2404_13216_amd as pk
import synthgen as g


def test_csr_validate():
    p = g.problem("rand_1m", scale=2000)
    pk.csr_validate(p.A)
    bad = g.CSR(p.A.n, p.A.row_ptr, p.A.col_idx.copy(), p.A.val)
    bad.col_idx[5] = p.A.n
    with pytest.raises(ValueError):
        pk.csr_validate(bad)
    uns = g.CSR(3, np.array([0, 2, 3, 3], np.int32), np.array([1, 0, 2], np.int32), np.ones(3))
    with pytest.raises(ValueError):
        pk.csr_validate(uns)
    with pytest.raises(ValueError):
        pk.csr_validate(g.CSR(2, np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32), np.ones(2)))


def test_problem_cache_roundtrip(tmp_path):
    p = g.problem("cd3d_256_var", scale=6)
    path = str(tmp_path / "prob.npz")
    d = g.save_problem(path, p)
    q = g.load_problem(path)
    assert q.name == p.name and q.A.n == p.A.n
    for a, b in ((q.A.row_ptr, p.A.row_ptr), (q.A.col_idx, p.A.col_idx), (q.A.val, p.A.val), (q.b, p.b)):
        assert np.array_equal(a, b)
    with np.load(path) as z:
        data = {k: z[k] for k in z.files}
    data["val"] = data["val"].copy()
    data["val"][0] += 1.0
    np.savez(path, **data)
    with pytest.raises(ValueError):
        g.load_problem(path)
    assert len(d) == 64


def test_spai_param_file(tmp_path):
    from paper_2404_13216_amd import spai
    th = np.random.default_rng(0).standard_normal(spai.NPARAM).astype(np.float32)
    path = str(tmp_path / "w.npz")
    spai.save_params(path, th)
    back = spai.load_params(path, device="cpu")
    assert np.array_equal(back.numpy(), th)
    with np.load(path) as z:
        data = {k: z[k] for k in z.files}
    data["params"] = data["params"].copy()
    data["params"][3] = 0.0
    np.savez(path, **data)
    with pytest.raises(ValueError):
        spai.load_params(path, device="cpu")
