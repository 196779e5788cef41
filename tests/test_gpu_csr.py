"""GPU parity of the sparse (CSR) path against the oracle.

The sketch of a CSR row is evaluated directly from its nonzeros and the
contraction goes through a CSC copy of A; the oracle uses a library sparse
product and an FFT, so agreement is to rounding (same bars as the dense
tests; pivots bit-exact on screened inputs).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_1601_04280_amd as rlu
import synth
from oracle import rlu as R

from parity import compare_factors, rel_fro, screened

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def csr_dev(row_ptr, col, val):
    return (torch.from_numpy(np.asarray(row_ptr, dtype=np.int32)).to(DEV),
            torch.from_numpy(np.asarray(col, dtype=np.int32)).to(DEV),
            torch.from_numpy(np.asarray(val, dtype=np.float64)).to(DEV))


def make_csr(m, n, density, seed, long_rows=(), empty_rows=(), plant=False):
    if plant:
        row_ptr, col, val = synth.random_csr(m, n, density, seed, plant_rank=8, plant_rows=max(1, m // 20),
                                             plant_scale=50.0)
    else:
        row_ptr, col, val = synth.random_csr(m, n, density, seed)
    a = sp.csr_matrix((val, col, row_ptr), shape=(m, n)).tolil()
    rng = np.random.default_rng(seed + 1)
    for i in long_rows:
        cols = rng.choice(n, size=min(n, 300), replace=False)
        a[i, cols] = rng.standard_normal(len(cols))
    for i in empty_rows:
        a[i, :] = 0
    a = a.tocsr()
    a.eliminate_zeros()
    a.sort_indices()
    return a


@pytest.mark.parametrize("m,n,l,s,seed", [(500, 400, 20, 64, 1), (300, 5000, 100, 4096, 2),
                                          (1000, 3000, 130, 256, 3), (64, 100, 2, 2, 4)])
def test_csr_sketch_matches_oracle(m, n, l, s, seed):
    a = make_csr(m, n, 0.02, seed, long_rows=(3, 7), empty_rows=(0, 5))
    Y = rlu.sketch(k=1, l=l, s=s, seed=seed, csr=(*csr_dev(a.indptr, a.indices, a.data), m, n)).cpu().numpy()
    ref = R.sketch_y(None, R.Params(1, l, s, seed), csr=(a.indptr, a.indices, a.data, m, n))
    assert rel_fro(Y, ref) <= 1e-10
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.all(Y[0] == 0) and np.all(Y[5] == 0)


@pytest.mark.parametrize("m,n,l,s,seed", [(500, 400, 20, 64, 11), (300, 5000, 100, 4096, 12), (64, 100, 2, 2, 14)])
def test_csr_hadamard_sketch_matches_oracle(m, n, l, s, seed):
    a = make_csr(m, n, 0.02, seed, long_rows=(3, 7), empty_rows=(0, 5))
    Y = rlu.sketch(k=1, l=l, s=s, seed=seed, csr=(*csr_dev(a.indptr, a.indices, a.data), m, n),
                   flags=rlu.RLU_FLAG_HADAMARD).cpu().numpy()
    ref = R.sketch_y(None, R.Params(1, l, s, seed, "hadamard"), csr=(a.indptr, a.indices, a.data, m, n))
    assert rel_fro(Y, ref) <= 1e-10
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.all(Y[0] == 0) and np.all(Y[5] == 0)


@pytest.mark.parametrize("m,n,k,l,s,density", [(3000, 2000, 20, 30, 256, 0.01), (5000, 4000, 60, 70, 512, 0.005),
                                               (800, 1200, 40, 100, 1024, 0.05)])
def test_csr_factor_matches_oracle(m, n, k, l, s, density):
    a = make_csr(m, n, density, m + n, plant=True)
    csr_np = (a.indptr, a.indices, a.data, m, n)
    for sd in range(1, 20):
        o = R.rlu(None, R.Params(k, l, s, sd), csr=csr_np)
        if screened(o):
            break
    else:
        pytest.skip("no screened seed")
    g = rlu.factor(k=k, l=l, s=s, seed=sd, csr=(*csr_dev(a.indptr, a.indices, a.data), m, n),
                   keep_intermediates=True)
    compare_factors(a.toarray(), g, o)
    assert g.info_dict()["bad_index"] == 0


def test_csr_and_dense_paths_agree():
    a = make_csr(2000, 1500, 0.02, 9, plant=True)
    d = torch.from_numpy(a.toarray()).to(DEV)
    gs = rlu.factor(k=20, l=30, s=256, seed=3, csr=(*csr_dev(a.indptr, a.indices, a.data), 2000, 1500),
                    keep_intermediates=True)
    gd = rlu.factor(d, k=20, l=30, s=256, seed=3, keep_intermediates=True)
    assert rel_fro(gs.Y.cpu().numpy(), gd.Y.cpu().numpy()) <= 1e-12
    assert torch.equal(gs.perm_r, gd.perm_r) and torch.equal(gs.perm_c, gd.perm_c)
    assert rel_fro(gs.U.cpu().numpy(), gd.U.cpu().numpy()) <= 1e-9


def test_csr_bad_column_index_is_reported():
    a = make_csr(200, 150, 0.05, 11)
    col = a.indices.copy()
    col[10] = 150                         # out of range
    with pytest.raises(rlu.RluError) as e:
        rlu.factor(k=4, l=8, s=16, seed=1, csr=(*csr_dev(a.indptr, col, a.data), 200, 150))
    assert e.value.status == rlu.RLU_ERR_INVALID_ARG


def test_csr_empty_matrix():
    m, n = 100, 80
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    g = rlu.factor(k=4, l=8, s=16, seed=1,
                   csr=(torch.from_numpy(row_ptr).to(DEV), torch.zeros(0, dtype=torch.int32, device=DEV),
                        torch.zeros(0, dtype=torch.float64, device=DEV), m, n))
    assert g.info_dict()["zero_pivots_y"] == 8 and g.info_dict()["zero_pivots_b"] == 8
    assert torch.count_nonzero(g.U) == 0


def test_csr_column_count_limit():
    """The CSC copy groups columns into at most 16384 buckets of up to 32768
    columns, so a CSR matrix may have at most 2^29 columns; more is rejected
    before anything runs (the column-pivoted LU's own limit, n <= 2^19,
    applies to rlu_factor below that)."""
    m = 50
    row_ptr = torch.zeros(m + 1, dtype=torch.int32, device=DEV)
    empty_i = torch.zeros(0, dtype=torch.int32, device=DEV)
    empty_v = torch.zeros(0, dtype=torch.float64, device=DEV)
    for n, ok in [((1 << 29) + 1, False), (1 << 19, True)]:   # workspace query: no output allocation
        if ok:
            assert rlu.workspace_size(k=4, l=8, s=16, csr=(row_ptr, empty_i, empty_v, m, n)) > 0
            continue
        with pytest.raises(rlu.RluError) as e:
            rlu.workspace_size(k=4, l=8, s=16, csr=(row_ptr, empty_i, empty_v, m, n))
        assert e.value.status == rlu.RLU_ERR_INVALID_ARG
        assert "2^29" in str(e.value)
