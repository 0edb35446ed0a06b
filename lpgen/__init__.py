"""Seeded synthetic LP instances shaped like the workloads of the PDCS LP path.

This module only draws random data and assembles it into CSR arrays; it holds
none of the solver's arithmetic.  Both the FP64 CPU oracle (under ``oracle/``)
and the HIP solver consume what it returns, so the two sides see identical
inputs without sharing any code.

Every instance is the LP of the paper's conic form (Section 1.1, eq. prob_cp)
restricted to box-bounded variables and zero / nonnegative row cones:

    min c^T x   s.t.  (G x - h)[:m_zero] = 0,  (G x - h)[m_zero:] >= 0,  l <= x <= u.

Random streams use ``numpy.random.default_rng([15504, config_id, instance_id])``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "LPInstance",
    "csr_from_columns",
    "planted_lp",
    "c0_instance",
    "c1_instance",
    "c2_batch",
    "c3_family_base",
    "c3_perturb",
    "c4_instance",
    "zipf_row_lengths",
    "rng_for",
    "dense_runs_instance",
    "infeasible_sum_row",
    "infeasible_free_columns",
    "infeasible_geq_pair",
    "unbounded_positive_columns",
    "unbounded_free_pair",
]


@dataclass
class LPInstance:
    """LP data in CSR form (row_ptr int64[m+1], col_idx int32[nnz], val f64[nnz])."""

    m: int
    n: int
    m_zero: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    h: np.ndarray
    c: np.ndarray
    l: np.ndarray
    u: np.ndarray
    name: str = "lp"
    x_planted: np.ndarray | None = None
    meta: dict = field(default_factory=dict)
    soc: tuple = ()  # dimensions of second-order-cone row blocks (after the nonnegative rows)
    n_exp: int = 0   # exponential-cone blocks of 3 rows (after the second-order-cone blocks)
    n_dexp: int = 0  # dual-exponential-cone blocks of 3 rows (the last rows)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m_nonneg(self) -> int:
        return self.m - self.m_zero

    def scipy_csr(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.m, self.n))


def rng_for(config_id: int, instance_id: int = 0) -> np.random.Generator:
    return np.random.default_rng([15504, int(config_id), int(instance_id)])


def _distinct_rows_per_column(rng, m: int, n: int, k) -> tuple[np.ndarray, np.ndarray]:
    """For column j draw k[j] distinct row indices, uniform over [0, m).

    Duplicates inside a column are redrawn until none remain, so the result is a
    uniform draw of a k[j]-subset per column.  Returns (row, col) entry lists.
    """
    k = np.broadcast_to(np.asarray(k, dtype=np.int64), (n,))
    if np.any(k > m):
        raise ValueError("more nonzeros per column than rows")
    col = np.repeat(np.arange(n, dtype=np.int64), k)
    row = rng.integers(0, m, size=col.size, dtype=np.int64)
    while True:
        key = col * m + row
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.nonzero(ks[1:] == ks[:-1])[0] + 1
        if dup.size == 0:
            break
        idx = order[dup]
        row[idx] = rng.integers(0, m, size=idx.size, dtype=np.int64)
    return row, col


def _distinct_cols_per_row(rng, m: int, n: int, lengths: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """For row i draw lengths[i] distinct columns, uniform over [0, n)."""
    row = np.repeat(np.arange(m, dtype=np.int64), lengths)
    col = rng.integers(0, n, size=row.size, dtype=np.int64)
    while True:
        key = row * n + col
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.nonzero(ks[1:] == ks[:-1])[0] + 1
        if dup.size == 0:
            break
        idx = order[dup]
        col[idx] = rng.integers(0, n, size=idx.size, dtype=np.int64)
    return row, col


def csr_from_columns(m: int, n: int, row: np.ndarray, col: np.ndarray, val: np.ndarray):
    """Sort (row, col, val) triplets into CSR order (rows, then columns ascending)."""
    key = row.astype(np.int64) * n + col.astype(np.int64)
    order = np.argsort(key, kind="stable")
    r = row[order]
    counts = np.bincount(r, minlength=m).astype(np.int64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, col[order].astype(np.int32), np.ascontiguousarray(val[order], dtype=np.float64)


def _csr_matvec(row_ptr, col_idx, val, x):
    """Plain CSR product used only to plant a feasible right-hand side b = A x0."""
    import scipy.sparse as sp

    m = row_ptr.size - 1
    n = x.size
    return sp.csr_matrix((val, col_idx, row_ptr), shape=(m, n)) @ x


def planted_lp(
    rng,
    m: int,
    n: int,
    per_col=None,
    row_lengths=None,
    m_zero: int | None = None,
    row_scale=None,
    col_scale=None,
    upper: float = 10.0,
    name: str = "lp",
) -> LPInstance:
    """Random LP with a planted interior point (the shared recipe of all configs).

    A has either ``per_col`` distinct uniform rows per column or ``row_lengths``
    distinct uniform columns per row, values N(0,1), optionally scaled as
    diag(row_scale) A diag(col_scale).  x0 ~ U[0,5]^n, h = A x0, c ~ U[0,1]^n,
    0 <= x <= upper.  Rows are equalities unless ``m_zero`` < m, in which case
    the remaining rows are ">=" rows (still satisfied with equality by x0).
    """
    if row_lengths is not None:
        row, col = _distinct_cols_per_row(rng, m, n, np.asarray(row_lengths, dtype=np.int64))
    else:
        row, col = _distinct_rows_per_column(rng, m, n, per_col)
    val = rng.standard_normal(row.size)
    if row_scale is not None:
        val = val * np.asarray(row_scale)[row]
    if col_scale is not None:
        val = val * np.asarray(col_scale)[col]
    row_ptr, col_idx, val = csr_from_columns(m, n, row, col, val)
    x0 = rng.uniform(0.0, 5.0, size=n)
    h = _csr_matvec(row_ptr, col_idx, val, x0)
    c = rng.uniform(0.0, 1.0, size=n)
    l = np.zeros(n)
    u = np.full(n, float(upper))
    mz = m if m_zero is None else int(m_zero)
    return LPInstance(m, n, mz, row_ptr, col_idx, val, h, c, l, u, name=name, x_planted=x0)


def c0_instance(seed: int = 0, m: int = 200, n: int = 500, per_col: int = 5) -> LPInstance:
    """Plain single LP: m=200, n=500, 5 nonzeros per column (nnz = 2500)."""
    return planted_lp(rng_for(0, seed), m, n, per_col=per_col, name=f"c0_m{m}_n{n}_s{seed}")


def zipf_row_lengths(rng, m: int, s: float = 1.5, max_len: int = 5000) -> np.ndarray:
    """Row lengths from a Zipf(s) law truncated to [1, max_len], by inverse CDF."""
    k = np.arange(1, max_len + 1, dtype=np.float64)
    p = k ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(m)
    return (np.searchsorted(cdf, u, side="left") + 1).astype(np.int64)


def c1_instance(seed: int = 0, m: int = 1_000_000, n: int = 2_000_000, s: float = 1.5,
                max_len: int = 5000) -> LPInstance:
    """Single large LP: power-law (truncated Zipf) row lengths, m=1e6, n=2e6."""
    rng = rng_for(1, seed)
    lengths = np.minimum(zipf_row_lengths(rng, m, s, max_len), n)
    inst = planted_lp(rng, m, n, row_lengths=lengths, name=f"c1_m{m}_n{n}_zipf{s}_s{seed}")
    inst.meta["zipf_s"] = s
    return inst


def c2_batch(count: int = 512, m_lo: int = 1000, m_hi: int = 50_000, per_col: int = 8,
             seed: int = 0) -> list[LPInstance]:
    """Batch of independent LPs, m log-uniform in [m_lo, m_hi], n = 2m, 8 nnz/col."""
    out = []
    for b in range(count):
        rng = rng_for(2, seed * 100_000 + b)
        m = int(round(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi)))))
        out.append(planted_lp(rng, m, 2 * m, per_col=per_col, name=f"c2_{b}"))
    return out


def c3_family_base(m: int = 20_000, n: int = 40_000, seed: int = 0) -> LPInstance:
    """Shared-pattern base LP for the warm-start family (nnz = 7.5 * n exactly).

    After a random permutation the first n/2 columns get 8 rows, the rest 7.
    """
    rng = rng_for(3, seed)
    perm = rng.permutation(n)
    k = np.empty(n, dtype=np.int64)
    k[perm[: n // 2]] = 8
    k[perm[n // 2:]] = 7
    return planted_lp(rng, m, n, per_col=k, name=f"c3base_m{m}_n{n}")


def c3_perturb(base: LPInstance, k: int, rel: float = 0.1) -> LPInstance:
    """Family member k: h and c multiplied elementwise by (1 + rel * N(0,1))."""
    rng = rng_for(30, k)
    xi = rng.standard_normal(base.m)
    zeta = rng.standard_normal(base.n)
    return LPInstance(base.m, base.n, base.m_zero, base.row_ptr, base.col_idx, base.val,
                      base.h * (1.0 + rel * xi), base.c * (1.0 + rel * zeta), base.l, base.u,
                      name=f"{base.name}_k{k}")


def c4_instance(seed: int = 0, m: int = 200_000, n: int = 500_000, per_col: int = 10) -> LPInstance:
    """Ill-conditioned LP: A = R A0 C, R_ii = 10^U[-3,3], C_jj = 10^U[-2,2]."""
    rng = rng_for(4, seed)
    rs = 10.0 ** rng.uniform(-3.0, 3.0, size=m)
    cs = 10.0 ** rng.uniform(-2.0, 2.0, size=n)
    return planted_lp(rng, m, n, per_col=per_col, row_scale=rs, col_scale=cs,
                      name=f"c4_m{m}_n{n}_s{seed}")


def dense_runs_instance(seed: int = 0, m: int = 256, run: int = 64, coupling: int = 1) -> LPInstance:
    """Edge-case LP for sorted-column layouts: row i holds the ``run`` consecutive
    columns [run*i, run*(i+1)) (a long run of one row between neighbouring
    gathered indices), plus ``coupling`` uniform random rows per column so the
    rows interact.  Values N(0,1), planted as in ``planted_lp``."""
    rng = rng_for(90, seed)
    n = m * run
    row_a = np.repeat(np.arange(m, dtype=np.int64), run)
    col_a = np.arange(n, dtype=np.int64)
    row_b, col_b = _distinct_rows_per_column(rng, m, n, coupling)
    keep = row_b != col_b // run
    row = np.concatenate([row_a, row_b[keep]])
    col = np.concatenate([col_a, col_b[keep]])
    val = rng.standard_normal(row.size)
    row_ptr, col_idx, val = csr_from_columns(m, n, row, col, val)
    x0 = rng.uniform(0.0, 5.0, size=n)
    h = _csr_matvec(row_ptr, col_idx, val, x0)
    c = rng.uniform(0.0, 1.0, size=n)
    return LPInstance(m, n, m, row_ptr, col_idx, val, h, c, np.zeros(n), np.full(n, 10.0),
                      name=f"dense_runs_{seed}", x_planted=x0)



def dense_columns_instance(seed: int = 0, m: int = 5000, n: int = 600_000, per_col: int = 2,
                           dense: int = 3) -> LPInstance:
    """Edge-case LP for chunked layouts: ``per_col`` uniform random rows per
    column over more than 2^18 columns (several gathered-index windows), plus
    ``dense`` columns spread over the index range that hold an entry in every
    row (thousands of entries of one gathered index within one band).  Values
    N(0,1), planted as in ``planted_lp``."""
    rng = rng_for(91, seed)
    row_a, col_a = _distinct_rows_per_column(rng, m, n, per_col)
    dcols = np.linspace(n // (2 * dense), n - 1 - n // (2 * dense), dense).astype(np.int64)
    row_b = np.tile(np.arange(m, dtype=np.int64), dense)
    col_b = np.repeat(dcols, m)
    keep = ~np.isin(col_a, dcols)
    row = np.concatenate([row_a[keep], row_b])
    col = np.concatenate([col_a[keep], col_b])
    val = rng.standard_normal(row.size)
    row_ptr, col_idx, val = csr_from_columns(m, n, row, col, val)
    x0 = rng.uniform(0.0, 5.0, size=n)
    h = _csr_matvec(row_ptr, col_idx, val, x0)
    c = rng.uniform(0.0, 1.0, size=n)
    return LPInstance(m, n, m, row_ptr, col_idx, val, h, c, np.zeros(n), np.full(n, 10.0),
                      name=f"dense_columns_{seed}", x_planted=x0)


def soc_instance(seed: int = 0, m_zero: int = 60, n: int = 300, blocks=(3, 5, 8, 16, 40), per_col: int = 3,
                 upper: float = 10.0) -> LPInstance:
    """Conic variant of the C0 recipe with second-order-cone rows (the socG
    option): ``m_zero`` equality rows followed by one block per entry of
    ``blocks``, (G x - h)_block = (t, w) with ||w|| <= t.  Each column gets
    ``per_col`` distinct uniform rows over all rows, values N(0,1); x0 ~ U[0,5]
    is planted strictly feasible: h = G x0 on the equality rows and
    h = G x0 - s0 on a block, with s0 = (||w|| + 1 + |N(0,1)|, w), w ~ N(0, I);
    c ~ U[0,1]; 0 <= x <= upper."""
    rng = rng_for(92, seed)
    blocks = tuple(int(d) for d in blocks)
    m = m_zero + sum(blocks)
    row, col = _distinct_rows_per_column(rng, m, n, per_col)
    val = rng.standard_normal(row.size)
    row_ptr, col_idx, val = csr_from_columns(m, n, row, col, val)
    x0 = rng.uniform(0.0, 5.0, size=n)
    h = _csr_matvec(row_ptr, col_idx, val, x0)
    r = m_zero
    for d in blocks:
        w = rng.standard_normal(d - 1)
        s0 = np.concatenate([[np.linalg.norm(w) + 1.0 + abs(rng.standard_normal())], w])
        h[r:r + d] -= s0
        r += d
    c = rng.uniform(0.0, 1.0, size=n)
    return LPInstance(m, n, m_zero, row_ptr, col_idx, val, h, c, np.zeros(n), np.full(n, upper),
                      name=f"soc_{seed}", x_planted=x0, soc=blocks)

def exp_instance(seed: int = 0, m_zero: int = 40, n: int = 200, m_nonneg: int = 20, n_exp: int = 12,
                 n_dexp: int = 8, per_col: int = 3, upper: float = 10.0) -> LPInstance:
    """Conic variant of the C0 recipe with exponential-cone rows (the expG and
    dual_expG options): ``m_zero`` equality rows, ``m_nonneg`` >= rows, then
    ``n_exp`` blocks (G x - h)_block = (x, y, z) in K_exp (y exp(x / y) <= z) and
    ``n_dexp`` blocks in K_exp* (-u exp(v / u) <= e w).  Each column gets
    ``per_col`` distinct uniform rows, values N(0,1); x0 ~ U[0,5] is planted
    strictly feasible: h = G x0 on the equality rows, h = G x0 - s on the others
    with s interior to the row's cone (>= rows: s ~ U[0.5, 1.5]; K_exp:
    s = (a, b, (1.5 + U) b e^(a / b)), a ~ U[-2, 1], b ~ U[0.5, 2]; K_exp*:
    s = (-a, b, (1.5 + U) a e^(-b / a) / e), a ~ U[0.5, 2], b ~ U[-1, 2]);
    c ~ U[0,1]; 0 <= x <= upper."""
    rng = rng_for(93, seed)
    m = m_zero + m_nonneg + 3 * (n_exp + n_dexp)
    row, col = _distinct_rows_per_column(rng, m, n, per_col)
    val = rng.standard_normal(row.size)
    row_ptr, col_idx, val = csr_from_columns(m, n, row, col, val)
    x0 = rng.uniform(0.0, 5.0, size=n)
    h = _csr_matvec(row_ptr, col_idx, val, x0)
    r = m_zero
    h[r:r + m_nonneg] -= rng.uniform(0.5, 1.5, size=m_nonneg)
    r += m_nonneg
    for _ in range(n_exp):
        a, b = rng.uniform(-2.0, 1.0), rng.uniform(0.5, 2.0)
        h[r:r + 3] -= np.array([a, b, (1.5 + rng.uniform()) * b * np.exp(a / b)])
        r += 3
    for _ in range(n_dexp):
        a, b = rng.uniform(0.5, 2.0), rng.uniform(-1.0, 2.0)
        h[r:r + 3] -= np.array([-a, b, (1.5 + rng.uniform()) * a * np.exp(-b / a) / np.e])
        r += 3
    c = rng.uniform(0.0, 1.0, size=n)
    return LPInstance(m, n, m_zero, row_ptr, col_idx, val, h, c, np.zeros(n), np.full(n, upper),
                      name=f"exp_{seed}", x_planted=x0, n_exp=n_exp, n_dexp=n_dexp)


# ---------------------------------------------------------------------------
# Infeasible and unbounded variants of the C0 recipe (tests of exit codes 2-5).
# Each takes a planted feasible LP and adds or changes data so that no
# feasible point (or no finite optimum) remains; HiGHS confirms the status in
# the tests.
# ---------------------------------------------------------------------------
def _with_rows(inst: LPInstance, rows: np.ndarray, rhs: np.ndarray, equality: bool, name: str) -> LPInstance:
    """Append dense rows (as zero-cone rows placed after the existing zero rows,
    or as ">=" rows at the end)."""
    import scipy.sparse as sp

    G = inst.scipy_csr()
    R = sp.csr_matrix(np.atleast_2d(rows))
    if equality:
        mz = inst.m_zero
        G2 = sp.vstack([G[:mz], R, G[mz:]]).tocsr()
        h2 = np.concatenate([inst.h[:mz], rhs, inst.h[mz:]])
        mz2 = mz + R.shape[0]
    else:
        G2 = sp.vstack([G, R]).tocsr()
        h2 = np.concatenate([inst.h, rhs])
        mz2 = inst.m_zero
    G2.sort_indices()
    return LPInstance(G2.shape[0], inst.n, mz2, G2.indptr.astype(np.int64), G2.indices.astype(np.int32),
                      G2.data.astype(np.float64), h2, inst.c.copy(), inst.l.copy(), inst.u.copy(), name=name)


def infeasible_sum_row(seed: int = 0, m: int = 200, n: int = 500) -> LPInstance:
    """C0 plus the equality row sum_j x_j = 100 n: beyond reach of 0 <= x <= 10."""
    base = c0_instance(seed, m, n)
    return _with_rows(base, np.ones((1, n)), np.array([100.0 * n]), True, f"infeas_sum_m{m}_n{n}_s{seed}")


def infeasible_free_columns(seed: int = 0, m: int = 200, n: int = 500, free: int = 50, lower_only: int = 50) -> LPInstance:
    """C0 with the first ``free`` columns free and the next ``lower_only``
    without an upper bound, plus the equality row sum_{j >= free+lower_only} x_j
    = 100 n over the boxed columns only: infeasible, and its Farkas certificate
    must also respect the infinite bounds (Lambda_j = {0} or R+ there)."""
    base = c0_instance(seed, m, n)
    row = np.zeros(n)
    row[free + lower_only:] = 1.0
    inst = _with_rows(base, row[None, :], np.array([100.0 * n]), True, f"infeas_free_m{m}_n{n}_s{seed}")
    inst.l[:free] = -np.inf
    inst.u[:free] = np.inf
    inst.u[free:free + lower_only] = np.inf
    return inst


def infeasible_exp_sum_row(seed: int = 0, **kw) -> LPInstance:
    """exp_instance(seed, **kw) plus the equality row sum_j x_j = 100 n: beyond
    reach of the box 0 <= x <= upper (the cone blocks stay the last rows)."""
    base = exp_instance(seed, **kw)
    inst = _with_rows(base, np.ones((1, base.n)), np.array([100.0 * base.n]), True, f"infeas_exp_s{seed}")
    inst.soc, inst.n_exp, inst.n_dexp = base.soc, base.n_exp, base.n_dexp
    return inst


def infeasible_geq_pair(seed: int = 0, m: int = 200, n: int = 500) -> LPInstance:
    """C0 plus two ">=" rows a^T x >= 1 and -a^T x >= 1 (a ~ N(0,1)): contradictory."""
    base = c0_instance(seed, m, n)
    a = rng_for(92, seed).standard_normal(n)
    return _with_rows(base, np.vstack([a, -a]), np.array([1.0, 1.0]), False, f"infeas_geq_m{m}_n{n}_s{seed}")


def unbounded_positive_columns(seed: int = 0, m: int = 200, n: int = 500, k: int = 5) -> LPInstance:
    """All rows ">=" (planted as C0); the first k columns get |values|, cost -1
    and no upper bound: raising them keeps Gx >= h and lowers the cost forever."""
    inst = planted_lp(rng_for(93, seed), m, n, per_col=5, m_zero=0, name=f"unbdd_pos_m{m}_n{n}_s{seed}")
    cols = inst.col_idx < k
    inst.val = np.where(cols, np.abs(inst.val), inst.val)
    inst.c[:k] = -1.0
    inst.u[:k] = np.inf
    return inst


def unbounded_free_pair(seed: int = 0, m: int = 200, n: int = 500, free: int = 20) -> LPInstance:
    """C0 with the first ``free`` columns free, column 1 a copy of column 0,
    c_0 = -1 and c_1 = 0: the direction e_0 - e_1 keeps Gx = h and lowers the
    cost without bound."""
    import scipy.sparse as sp

    base = c0_instance(seed, m, n)
    G = base.scipy_csr().tolil()
    G[:, 1] = G[:, 0]
    G = G.tocsr()
    G.sort_indices()
    c = base.c.copy()
    c[0], c[1] = -1.0, 0.0
    l = base.l.copy()
    u = base.u.copy()
    l[:free] = -np.inf
    u[:free] = np.inf
    return LPInstance(m, n, base.m_zero, G.indptr.astype(np.int64), G.indices.astype(np.int32),
                      G.data.astype(np.float64), base.h.copy(), c, l, u, name=f"unbdd_free_m{m}_n{n}_s{seed}")
