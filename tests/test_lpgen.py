"""The seeded input generators: shapes, sparsity structure and value
distributions of the workload recipes, and the planted feasible point."""
import numpy as np
import pytest

import lpgen


def _rows(inst):
    return np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))


def _planted_ok(inst):
    A = inst.scipy_csr()
    r = A @ inst.x_planted - inst.h
    scale = 1.0 + np.abs(inst.h).max()
    eq = np.abs(r[: inst.m_zero]).max(initial=0.0) <= 1e-10 * scale
    ge = (r[inst.m_zero:] >= -1e-10 * scale).all()
    box = (inst.x_planted >= inst.l).all() and (inst.x_planted <= inst.u).all()
    return eq and ge and box


def test_c0_recipe():
    inst = lpgen.c0_instance(0)
    assert (inst.m, inst.n, inst.nnz, inst.m_zero) == (200, 500, 2500, 200)
    rows = _rows(inst)
    # 5 distinct rows per column
    per_col = np.bincount(inst.col_idx, minlength=inst.n)
    assert (per_col == 5).all()
    pairs = set(zip(rows.tolist(), inst.col_idx.tolist()))
    assert len(pairs) == inst.nnz
    assert (inst.l == 0).all() and (inst.u == 10).all()
    assert (inst.c >= 0).all() and (inst.c <= 1).all()
    assert _planted_ok(inst)
    # values N(0,1)
    assert abs(inst.val.mean()) < 0.1 and abs(inst.val.std() - 1) < 0.1


def test_generators_are_seeded():
    a, b = lpgen.c0_instance(3), lpgen.c0_instance(3)
    assert np.array_equal(a.val, b.val) and np.array_equal(a.col_idx, b.col_idx)
    c = lpgen.c0_instance(4)
    assert not np.array_equal(a.val, c.val)


def test_c1_recipe_small():
    inst = lpgen.c1_instance(0, m=20000, n=40000)
    lens = np.diff(inst.row_ptr)
    assert lens.min() >= 1 and lens.max() <= 5000
    # truncated Zipf(1.5): P(len = 1) = 1 / sum_{k<=5000} k^-1.5 ~ 0.384
    z = sum(k ** -1.5 for k in range(1, 5001))
    assert abs((lens == 1).mean() - 1 / z) < 0.02
    # distinct columns within each row
    for r in range(0, inst.m, 997):
        cols = inst.col_idx[inst.row_ptr[r]:inst.row_ptr[r + 1]]
        assert len(np.unique(cols)) == len(cols)
    assert _planted_ok(inst)


def test_c2_batch_sizes():
    insts = lpgen.c2_batch(count=40, m_lo=1000, m_hi=50000)
    ms = np.array([i.m for i in insts])
    assert ms.min() >= 1000 and ms.max() <= 50000
    assert all(i.n == 2 * i.m and i.nnz == 8 * i.n for i in insts)
    # log-uniform: about half below the geometric mean of the range
    assert 0.25 < (ms < np.sqrt(1000 * 50000)).mean() < 0.75


def test_c3_family_shares_the_pattern():
    base = lpgen.c3_family_base(m=200, n=400, seed=2)
    assert base.nnz == 3000                     # 7.5 n: half the columns 8 rows, half 7
    per_col = np.bincount(base.col_idx, minlength=base.n)
    assert sorted(set(per_col.tolist())) == [7, 8] and (per_col == 8).sum() == 200
    a, b = lpgen.c3_perturb(base, 0), lpgen.c3_perturb(base, 1)
    assert a.val is base.val and np.array_equal(a.col_idx, b.col_idx)
    ra = a.h / base.h - 1
    assert 0.07 < ra.std() < 0.13               # 10% relative noise
    assert not np.array_equal(a.c, b.c)


def test_c4_scales():
    inst = lpgen.c4_instance(0, m=300, n=700, per_col=6)
    A = abs(inst.scipy_csr())
    rmax = A.max(axis=1).toarray().ravel()
    # row scales spread over about 6 decades
    assert np.log10(rmax.max() / rmax.min()) > 4
    assert _planted_ok(inst)


def test_dense_runs_edge_case():
    inst = lpgen.dense_runs_instance(0)
    assert inst.n == 64 * inst.m
    # row i holds the 64 consecutive columns [64 i, 64 i + 64)
    for i in (0, 17, inst.m - 1):
        cols = set(inst.col_idx[inst.row_ptr[i]:inst.row_ptr[i + 1]].tolist())
        assert set(range(64 * i, 64 * i + 64)) <= cols
    assert _planted_ok(inst)


@pytest.mark.parametrize("mz", [0, 30, 60])
def test_planted_geq_rows(mz):
    inst = lpgen.planted_lp(lpgen.rng_for(55, mz), 60, 150, per_col=3, m_zero=mz)
    assert inst.m_zero == mz and _planted_ok(inst)
