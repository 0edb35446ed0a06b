"""Plain FP64 CPU oracle for the PDCS method on linear programs.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: it is used by ``tests/``, by ``__graft_entry__.smoke()`` (to check
one small GPU solve) and by the CPU-baseline leg of ``bench.py``.  It shares no
code with the HIP solver; the two sides only share the seeded input generators
in ``lpgen``.

What it computes (paper: "A Technical Note on the Implementation and Use of
PDCS", arXiv 2603.15504):

* the conic problem of Section 1.1 (eq. prob_cp) with every variable
  box-bounded (n2 = 0) and row cones in the paper's order: zero-cone
  (equality) rows, nonnegative-cone (>=) rows, then second-order-cone blocks
  (the socG option of Section 3), exponential-cone and dual-exponential-cone
  blocks (expG, dual_expG), so K_d* = {0}^m_zero x R+^m_nonneg x K_soc x ... x
  K_exp x ... x K_exp* x ... and K_d = R^m_zero x R+^m_nonneg x K_soc x ... x
  K_exp* x ... x K_exp x ... (the second-order cone is self-dual); after
  diagonal rescaling the blocks become rescaled cones (Section 2.6),
  projected onto by one-dimensional root finds (``proj_scaled_soc``,
  ``proj_scaled_exp``);
* Algorithm "PDCS with preconditioning" (Section 2.6): diagonal rescaling, the
  PDCS loop of Algorithm 1 (Section 2) on the rescaled data, then unscaling;
* inside it: OnePDHG (eq. PDHG, Section 1.2), AdaptiveStepPDHG (Function 2,
  eq. adaptive_step_size, Section 2.1), the reflection parameter (eq.
  adaptive_reflection / tolerance / tolerance-2, Section 2.2), the reflected
  Halpern and averaging updates (Algorithm 1), GetRestartCandidate and the
  three restart conditions with the KKT_omega fallback (Section 2.3), the
  bisection for the normalized duality gap (Algorithm 3, eq. compute_rho,
  compute_zt, compute_zt_2, Section 2.4), the primal weight (Section 2.5) and
  the termination errors of Section 3 (eq. PDCS_terminate_tolerance_abs/rel)
  and the infeasibility tests of the option list of Section 3 (exit codes 2-5
  of the exit-code table), read as tests on rays (see ``infeasibility_ratios``).

Everything is float64; products with G use scipy.sparse CSR.  Steps follow the
paper's order and notation; nothing is fused or reordered.  Where the paper is
silent or ambiguous the reading taken is stated at the point of use.

Every function here is pinned by the CPU tests (HiGHS optimum, vertex brute
force, closed forms, invariants).  The full trajectory (iteration counts after
the first restart check) is parity unpinned: restart decisions are
discontinuous in rounding.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

# Restart thresholds (Section 2.3) and primal-weight constants (Section 2.5).
BETA_SUFFICIENT = 0.4
BETA_NECESSARY = 0.8
BETA_ARTIFICIAL = 0.223
THETA = 0.5
OMEGA_MIN, OMEGA_MAX = 1e-5, 1e5
TINY = 1e-10

EXIT_OPTIMAL = 0
EXIT_MAX_ITER = 1
EXIT_PRIMAL_INFEASIBLE_LOW_ACC = 2
EXIT_PRIMAL_INFEASIBLE_HIGH_ACC = 3
EXIT_DUAL_INFEASIBLE_LOW_ACC = 4
EXIT_DUAL_INFEASIBLE_HIGH_ACC = 5
EXIT_TIME_LIMIT = 6
EXIT_CONTINUE = 7
EXIT_NUMERICAL_ERROR = 8


# --------------------------------------------------------------------------
# Problem data
# --------------------------------------------------------------------------
@dataclass
class LPData:
    """min c^T x  s.t.  Gx - h in K_d*,  l <= x <= u   (eq. prob_cp, boxed variables).

    Rows: m_zero zero-cone rows, then nonnegative-cone rows, then the
    second-order-cone blocks of dimensions ``soc`` (each block (t, w) with
    ||w|| <= t).  ``cone_scale`` (None = all ones) holds positive row factors e
    of rescaled data: its K_d* blocks are diag(e) K_soc and its K_d blocks
    diag(1/e) K_soc (the cones of Gx - h and y after rows are multiplied by e,
    Section 2.6)."""

    G: sp.csr_matrix
    h: np.ndarray
    c: np.ndarray
    l: np.ndarray
    u: np.ndarray
    m_zero: int
    soc: tuple = ()
    cone_scale: np.ndarray | None = None
    n_exp: int = 0    # exponential-cone blocks (3 rows each) after the second-order-cone blocks
    n_dexp: int = 0   # dual-exponential-cone blocks (3 rows each), the last rows

    @property
    def m(self) -> int:
        return self.G.shape[0]

    @property
    def n(self) -> int:
        return self.G.shape[1]

    def proj_Kd(self, y):
        return proj_Kd(y, self.m_zero, self.soc, self.cone_scale, self.n_exp, self.n_dexp)

    def proj_Kd_star(self, v):
        return proj_Kd_star(v, self.m_zero, self.soc, self.cone_scale, self.n_exp, self.n_dexp)

    @property
    def has_cones(self) -> bool:
        return bool(self.soc) or self.n_exp > 0 or self.n_dexp > 0


def lpdata_from_arrays(m, n, m_zero, row_ptr, col_idx, val, h, c, l, u, soc=(), n_exp=0, n_dexp=0) -> LPData:
    G = sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col_idx), np.asarray(row_ptr)),
                      shape=(int(m), int(n)))
    soc = tuple(int(d) for d in soc)
    n_exp, n_dexp = int(n_exp), int(n_dexp)
    if (any(d < 1 for d in soc) or n_exp < 0 or n_dexp < 0 or
            int(m_zero) + sum(soc) + 3 * (n_exp + n_dexp) > int(m)):
        raise ValueError("cone blocks (second-order: dimension >= 1; exponential: 3 rows) must fit after the zero rows")
    return LPData(G, np.asarray(h, np.float64), np.asarray(c, np.float64),
                  np.asarray(l, np.float64), np.asarray(u, np.float64), int(m_zero), soc, None, n_exp, n_dexp)


def lpdata_from_instance(inst) -> LPData:
    return lpdata_from_arrays(inst.m, inst.n, inst.m_zero, inst.row_ptr, inst.col_idx,
                              inst.val, inst.h, inst.c, inst.l, inst.u, getattr(inst, "soc", ()),
                              getattr(inst, "n_exp", 0), getattr(inst, "n_dexp", 0))


# --------------------------------------------------------------------------
# Projections (Section 1.1, eq. defn_Lambda1; Section 1.2)
# --------------------------------------------------------------------------
def proj_box(x, l, u):
    """Projection onto [l, u] (componentwise clip; +-inf bounds allowed)."""
    return np.minimum(np.maximum(x, l), u)


def proj_soc(v):
    """Projection onto the second-order cone {(t, w): ||w|| <= t} (closed form)."""
    v = np.asarray(v, dtype=np.float64)
    t, w = v[0], v[1:]
    nw = float(np.linalg.norm(w))
    if nw <= t:
        return v.copy()
    if nw <= -t:
        return np.zeros_like(v)
    a = 0.5 * (t + nw)
    return np.concatenate([[a], (a / nw) * w])


def proj_scaled_soc(v, e):
    """Projection onto the rescaled cone E K_soc = {E z : z in K_soc}, E = diag(e) > 0
    (Section 2.6: after diagonal rescaling the projection is a root find).

    Derivation (KKT conditions of min ||p - v||^2 s.t. ||p_bar / e_bar|| <= p0 / e0):
    v itself if it lies in the cone; 0 if v lies in the polar cone -E^{-1} K_soc
    (||v_bar * e_bar|| <= -v0 e0); otherwise the constraint is active with
    multiplier mu > 0, s = p0 / e0 = v0 / e0 + mu / e0^2 and
    p_i = v_i e_i^2 s / (e_i^2 s + mu), where mu is the root of
        f(mu) = sum_i v_i^2 e_i^2 / (e_i^2 s(mu) + mu)^2 - 1,
    strictly decreasing on mu > max(0, -v0 e0), positive at that left end and
    non-positive at mu = ||v_bar * e_bar||.  The root is found by bisection
    until the bracket is narrower than 2^-52 of its right end (the resolution
    of a float64 mu).
    """
    v = np.asarray(v, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    v0, vb = float(v[0]), v[1:]
    e0, eb = float(e[0]), e[1:]
    if float(np.linalg.norm(vb / eb)) <= v0 / e0:
        return v.copy()
    if float(np.linalg.norm(vb * eb)) <= -v0 * e0:
        return np.zeros_like(v)
    q = vb * vb * eb * eb
    e2 = eb * eb

    def f(mu):
        s = v0 / e0 + mu / (e0 * e0)
        return float(np.sum(q / (e2 * s + mu) ** 2)) - 1.0

    lo = max(0.0, -v0 * e0)
    hi = max(lo, float(np.linalg.norm(vb * eb)))
    while f(hi) > 0.0:  # only by rounding at the right end
        hi = 2.0 * hi + 1e-300
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi or hi - lo <= 2.0 ** -52 * hi:
            break
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    s = v0 / e0 + mu / (e0 * e0)
    return np.concatenate([[e0 * s], vb * e2 * s / (e2 * s + mu)])


# Exponential cones (the expG and dual_expG options of Section 3), in the
# convention (x, y, z): K_exp = closure of {y > 0, y exp(x / y) <= z}, and its
# dual K_exp* = closure of {(u, v, w): u < 0, -u exp(v / u) <= e w}.
def in_exp_cone(q) -> bool:
    """Membership in K_exp (exact comparisons; the boundary y = 0 is the face
    {x <= 0, z >= 0})."""
    x, y, z = (float(t) for t in q)
    if y > 0.0:
        return z > 0.0 and x <= y * np.log(z / y)
    return y == 0.0 and x <= 0.0 and z >= 0.0


def in_exp_dual(q) -> bool:
    """Membership in K_exp* (the boundary u = 0 is the face {v >= 0, w >= 0})."""
    u, v, w = (float(t) for t in q)
    if u < 0.0:
        return w > 0.0 and np.log(-u) + v / u <= 1.0 + np.log(w)
    return u == 0.0 and v >= 0.0 and w >= 0.0


def proj_scaled_exp(v, f):
    """Projection onto the rescaled cone F K_exp = {F q : q in K_exp}, F = diag(f) > 0
    (Section 2.6: after rescaling, a one-dimensional root find).

    v itself if v / f lies in K_exp; 0 if v lies in the polar cone -F^{-1} K_exp*
    (-f v in K_exp*).  Otherwise the projection lies on the boundary of F K_exp,
    which is the face {(a, 0, b): a <= 0, b >= 0} (nearest point: clip) together
    with the rays s F a(r), a(r) = (r, 1, e^r), s >= 0.  On the ray of r the best
    s is <F a, v> / ||F a||^2, leaving the angle function
    theta(r) = <F a(r), v> / ||F a(r)||, whose derivative has the sign of
        h(r) = A be - B al r + C e^r (al r^2 - al r + be) + ga e^2r (A (1 - r) - B)
    (A, B, C = f * v; al, be, ga = f^2).  Every local maximum of theta on
    [-300, 300] is bracketed by a + to - sign change of h on a 0.05 grid and
    bisected to the resolution of a float64.  Above the grid the rays lie within
    e^-300 of the face's edge (0, 0, 1).  Below it they approach the edge
    (-1, 0, 0) only like 1 / |r|, but their third coordinate is below e^-300
    of the others: there h(r) is A be - B al r up to that relative size, whose
    root r = (v_1 / f_1) / (v_2 / f_2) (x / y of v / f, when v_1 < 0 < v_2) is
    one more candidate if it lies below the grid.  A candidate meets the
    optimality conditions of the projection (Moreau: p in the cone, v - p in its
    polar cone -F^{-1} K_exp*, <p, v - p> = 0) when its residual v - p is a
    nonpositive multiple of F^{-1} n(r), n(r) = (-1, r - 1, e^-r) the normal of
    K_exp along the ray (the face clip: when -F (v - p) lies in K_exp*); such a
    candidate is the projection, so the nearest of these wins, and the nearest
    of all candidates only when none qualifies.  (Near the apex a ray candidate
    and the face clip can lie within rounding of the same distance from v while
    the points themselves differ by the square root of that rounding.)
    """
    v = np.asarray(v, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    if in_exp_cone(v / f):
        return v.copy()
    if in_exp_dual(-f * v):
        return np.zeros(3)
    best = np.array([min(v[0], 0.0), 0.0, max(v[2], 0.0)])
    bestd = float(np.linalg.norm(v - best))
    best_ok = in_exp_dual(-f * (v - best))
    A, B, C = f * v
    al, be, ga = f * f

    def h(r):
        E = np.exp(r)
        return A * be - B * al * r + C * E * (al * r * r - al * r + be) + ga * E * E * (A * (1.0 - r) - B)

    grid = np.linspace(-300.0, 300.0, 12001)
    hs = h(grid)
    roots = []
    for i in np.nonzero((hs[:-1] > 0.0) & (hs[1:] <= 0.0))[0]:
        lo, hi = float(grid[i]), float(grid[i + 1])
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:
                break
            if h(mid) > 0.0:
                lo = mid
            else:
                hi = mid
        roots.append(0.5 * (lo + hi))
    if v[0] < 0.0 < v[1] and (v[0] / f[0]) / (v[1] / f[1]) < grid[0]:
        roots.append((v[0] / f[0]) / (v[1] / f[1]))
    for r in roots:
        a = f * np.array([r, 1.0, np.exp(r)])
        s = float(a @ v) / float(a @ a)
        if s > 0.0:
            p = s * a
            d = float(np.linalg.norm(v - p))
            # n(r) times min(1, e^r), which stays finite at both ends
            n = np.array([-np.exp(r), (r - 1.0) * np.exp(r), 1.0]) if r <= 0.0 else np.array([-1.0, r - 1.0, np.exp(-r)])
            ok = float((v - p) @ (n / f)) <= 0.0
            if (ok and not best_ok) or (ok == best_ok and d < bestd):
                best, bestd, best_ok = p, d, ok
    return best


def proj_scaled_exp_dual(v, f):
    """Projection onto F K_exp* (F = diag(f) > 0) by Moreau's decomposition:
    F K_exp* is the dual cone of C = F^{-1} K_exp, so P(v) = v + P_C(-v)."""
    v = np.asarray(v, dtype=np.float64)
    return v + proj_scaled_exp(-v, 1.0 / np.asarray(f, dtype=np.float64))


def _cone_blocks(m, soc, n_exp=0, n_dexp=0):
    """(kind, start, end) row ranges of the cone blocks, the last rows in the
    order second-order ("soc"), exponential ("exp"), dual exponential ("dexp")."""
    r = m - sum(soc) - 3 * (n_exp + n_dexp)
    out = []
    for d in soc:
        out.append(("soc", r, r + d))
        r += d
    for kind, cnt in (("exp", n_exp), ("dexp", n_dexp)):
        for _ in range(cnt):
            out.append((kind, r, r + 3))
            r += 3
    return out


def _soc_blocks(m, soc):
    """(start, end) row ranges of the second-order-cone blocks when they are the last rows."""
    return [(a, b) for _, a, b in _cone_blocks(m, soc)]


def proj_Kd(y, m_zero, soc=(), scale=None, n_exp=0, n_dexp=0):
    """Projection onto K_d = R^m_zero x R+^m_nonneg x K_soc x ... x K_exp* x ... x
    K_exp x ... (dual variables of the rows: the dual of each row block's cone);
    with row factors ``scale`` the blocks are diag(1/scale) of those cones."""
    out = np.array(y, dtype=np.float64, copy=True)
    m = out.size
    m_cone = m - sum(soc) - 3 * (n_exp + n_dexp)
    out[m_zero:m_cone] = np.maximum(out[m_zero:m_cone], 0.0)
    for kind, a, b in _cone_blocks(m, soc, n_exp, n_dexp):
        e = np.ones(b - a) if scale is None else 1.0 / scale[a:b]
        if kind == "soc":
            out[a:b] = proj_soc(out[a:b]) if scale is None else proj_scaled_soc(out[a:b], e)
        elif kind == "exp":
            out[a:b] = proj_scaled_exp_dual(out[a:b], e)
        else:
            out[a:b] = proj_scaled_exp(out[a:b], e)
    return out


def proj_Kd_star(v, m_zero, soc=(), scale=None, n_exp=0, n_dexp=0):
    """Projection onto K_d* = {0}^m_zero x R+^m_nonneg x K_soc x ... x K_exp x ... x
    K_exp* x ... (the cones of G x - h); with row factors ``scale`` the blocks are
    diag(scale) of those cones."""
    out = np.array(v, dtype=np.float64, copy=True)
    m = out.size
    m_cone = m - sum(soc) - 3 * (n_exp + n_dexp)
    out[:m_zero] = 0.0
    out[m_zero:m_cone] = np.maximum(out[m_zero:m_cone], 0.0)
    for kind, a, b in _cone_blocks(m, soc, n_exp, n_dexp):
        e = np.ones(b - a) if scale is None else scale[a:b]
        if kind == "soc":
            out[a:b] = proj_soc(out[a:b]) if scale is None else proj_scaled_soc(out[a:b], e)
        elif kind == "exp":
            out[a:b] = proj_scaled_exp(out[a:b], e)
        else:
            out[a:b] = proj_scaled_exp_dual(out[a:b], e)
    return out


def proj_Lambda(lam, l, u):
    """Projection onto Lambda of eq. defn_Lambda1.

    Lambda_i = {0} if both bounds are infinite, R- if only u is finite, R+ if
    only l is finite, R if both are finite.
    """
    lf = np.isfinite(l)
    uf = np.isfinite(u)
    out = np.array(lam, dtype=np.float64, copy=True)
    both_inf = ~lf & ~uf
    only_u = ~lf & uf
    only_l = lf & ~uf
    out[both_inf] = 0.0
    out[only_u] = np.minimum(out[only_u], 0.0)
    out[only_l] = np.maximum(out[only_l], 0.0)
    return out


# --------------------------------------------------------------------------
# Diagonal rescaling (Section 2.6, eq. rescaled_prob, Algorithm 4)
# --------------------------------------------------------------------------
def ruiz_l2_scaling(G: sp.csr_matrix, ruiz_iters: int = 10, l2_pass: bool = True):
    """Return positive diagonals (D1, D2) with G_hat = D1 G D2.

    The paper does not say how D1, D2 are chosen.  Reading taken: Ruiz
    equilibration (each pass divides row i by sqrt(max_j |G_hat_ij|) and column
    j by sqrt(max_i |G_hat_ij|), both taken from the same current matrix) for
    ``ruiz_iters`` passes, then one pass dividing rows and columns by the square
    roots of their Euclidean norms.  Empty rows or columns keep factor 1.
    """
    m, n = G.shape
    A = abs(G).tocsr()
    D1 = np.ones(m)
    D2 = np.ones(n)

    def current():
        return sp.diags(D1) @ A @ sp.diags(D2)

    for _ in range(ruiz_iters):
        M = current()
        rmax = np.asarray(M.max(axis=1).todense()).ravel()
        cmax = np.asarray(M.max(axis=0).todense()).ravel()
        r = np.where(rmax > 0, np.sqrt(rmax), 1.0)
        s = np.where(cmax > 0, np.sqrt(cmax), 1.0)
        D1 = D1 / r
        D2 = D2 / s
    if l2_pass:
        M = current()
        M2 = M.multiply(M)
        rn = np.sqrt(np.asarray(M2.sum(axis=1)).ravel())
        cn = np.sqrt(np.asarray(M2.sum(axis=0)).ravel())
        r = np.where(rn > 0, np.sqrt(rn), 1.0)
        s = np.where(cn > 0, np.sqrt(cn), 1.0)
        D1 = D1 / r
        D2 = D2 / s
    return D1, D2


def rescale(lp: LPData, D1, D2) -> LPData:
    """Rescaled data of eq. rescaled_prob: G^=D1 G D2, c^=D2 c, h^=D1 h, l^=l/D2, u^=u/D2;
    the row cones become diag(D1) K_d* (and diag(1/D1) K_d for y)."""
    Gs = (sp.diags(D1) @ lp.G @ sp.diags(D2)).tocsr()
    scale = D1 if lp.cone_scale is None else lp.cone_scale * D1
    return LPData(Gs, D1 * lp.h, D2 * lp.c, lp.l / D2, lp.u / D2, lp.m_zero, lp.soc,
                  np.asarray(scale, np.float64) if lp.has_cones else None, lp.n_exp, lp.n_dexp)


# --------------------------------------------------------------------------
# One PDHG step (Section 1.2, eq. PDHG)
# --------------------------------------------------------------------------
def one_pdhg(lp: LPData, x, y, tau, sigma):
    xh = proj_box(x - tau * (lp.c - lp.G.T @ y), lp.l, lp.u)
    yh = lp.proj_Kd(y + sigma * (lp.h - lp.G @ (2.0 * xh - x)))
    return xh, yh


# --------------------------------------------------------------------------
# Error metrics
# --------------------------------------------------------------------------
def dual_objective(lp: LPData, y, lam):
    """<y, h> + l^T lam+ - u^T lam-  (eq. dual_conic).

    Reading: 0 * inf is taken as 0, i.e. the bound terms sum over finite bounds
    only; lam+ = max(lam, 0), lam- = max(-lam, 0).
    """
    lf = np.isfinite(lp.l)
    uf = np.isfinite(lp.u)
    lp_term = np.dot(lp.l[lf], np.maximum(lam[lf], 0.0))
    um_term = np.dot(lp.u[uf], np.maximum(-lam[uf], 0.0))
    return float(np.dot(y, lp.h) + lp_term - um_term)


def abs_errors_l2(lp: LPData, x, y):
    """Absolute errors of eq. tolerance-3 (Euclidean norms) with lam = c - G^T y.

    Returns (err_p, err_d, err_gap, pobj, dobj).
    """
    r = lp.G @ x - lp.h
    err_p = float(np.linalg.norm(r - lp.proj_Kd_star(r)))
    lam = lp.c - lp.G.T @ y
    err_d = float(np.linalg.norm(lam - proj_Lambda(lam, lp.l, lp.u)))
    pobj = float(np.dot(lp.c, x))
    dobj = dual_objective(lp, y, lam)
    return err_p, err_d, abs(pobj - dobj), pobj, dobj


def rel_errors_l2(lp: LPData, x, y):
    """Relative errors of eq. tolerance-2: L2 numerators, 1+||h||_1, 1+||c||_1, 1+|pobj|+|dobj|."""
    ep, ed, eg, pobj, dobj = abs_errors_l2(lp, x, y)
    rp = ep / (1.0 + np.sum(np.abs(lp.h)))
    rd = ed / (1.0 + np.sum(np.abs(lp.c)))
    rg = eg / (1.0 + abs(pobj) + abs(dobj))
    return rp, rd, rg


def max_err(lp: LPData, x, y) -> float:
    """maxErr of eq. tolerance."""
    return float(max(rel_errors_l2(lp, x, y)))


def reflection_parameter(maxerr: float) -> float:
    """AdaptiveReflectionParameter (eq. adaptive_reflection): Proj_[0,1](-0.1 log10(maxErr) + 0.2).

    Reading: maxErr = 0 gives beta = 1 (the limit of the formula).
    """
    if maxerr <= 0.0:
        return 1.0
    return float(min(1.0, max(0.0, -0.1 * math.log10(maxerr) + 0.2)))


def kkt_omega(err_p, err_d, err_gap, omega):
    """Weighted KKT error of Section 2.3 (used when the bisection fails)."""
    return math.sqrt(omega ** 2 * err_p ** 2 + err_d ** 2 / omega ** 2 + err_gap ** 2)


def termination_errors(lp: LPData, x, y):
    """Unscaled errors of eq. PDCS_terminate_tolerance_abs and _rel (infinity norms).

    Returns a dict with abs_p, abs_d, abs_gap, rel_p, rel_d, rel_gap, pobj, dobj.
    """
    Gx = lp.G @ x
    r = Gx - lp.h
    pr = lp.proj_Kd_star(r)
    abs_p = float(np.max(np.abs(r - pr), initial=0.0))
    GTy = lp.G.T @ y
    lam = lp.c - GTy
    abs_d = float(np.max(np.abs(lam - proj_Lambda(lam, lp.l, lp.u)), initial=0.0))
    pobj = float(np.dot(lp.c, x))
    dobj = dual_objective(lp, y, lam)
    abs_gap = abs(pobj - dobj)
    inf = lambda v: float(np.max(np.abs(v), initial=0.0))
    rel_p = abs_p / (1.0 + max(inf(lp.h), inf(Gx), inf(pr)))
    rel_d = abs_d / (1.0 + max(inf(lp.c), inf(GTy)))
    rel_gap = abs_gap / (1.0 + max(abs(pobj), abs(dobj)))
    return dict(abs_p=abs_p, abs_d=abs_d, abs_gap=abs_gap, rel_p=rel_p, rel_d=rel_d,
                rel_gap=rel_gap, pobj=pobj, dobj=dobj)


def is_optimal(err: dict, rel_tol: float, abs_tol: float) -> bool:
    """Reading: optimal when all three absolute errors are within abs_tol, or all three
    relative errors are within rel_tol (Section 3 lists both tolerances)."""
    a = max(err["abs_p"], err["abs_d"], err["abs_gap"]) <= abs_tol
    r = max(err["rel_p"], err["rel_d"], err["rel_gap"]) <= rel_tol
    return bool(a or r)


# --------------------------------------------------------------------------
# Infeasibility tests (Section 3, options eps_{primal,dual}_infeasible_{low,high}_acc;
# exit codes 2-5 of the exit-code table)
# --------------------------------------------------------------------------
def proj_box_recession(d, l, u):
    """Projection onto the recession cone of [l, u]: 0 where both bounds are finite,
    R+ where only l is finite, R- where only u is finite, R where neither is."""
    lf = np.isfinite(l)
    uf = np.isfinite(u)
    out = np.array(d, dtype=np.float64, copy=True)
    out[lf & uf] = 0.0
    only_l = lf & ~uf
    only_u = ~lf & uf
    out[only_l] = np.maximum(out[only_l], 0.0)
    out[only_u] = np.minimum(out[only_u], 0.0)
    return out


def rounding_bound(count: int) -> float:
    """gamma_N = N u / (1 - N u) with u = 2^-53: a bound on the relative error of a
    sum of N floating-point terms (Higham, Accuracy and Stability of Numerical
    Algorithms, eq. 3.4)."""
    nu = max(int(count), 1) * 2.0 ** -53
    return nu / (1.0 - nu)


def infeasibility_ratios(lp: LPData, ray_x, ray_y):
    """The two ratios of the infeasibility options, evaluated on a ray.

    Reading.  Applied literally to an iterate, the primal ratio
    err_abs,d(lam) / (<y, h> + l^T lam+ - u^T lam-) is 0 for every LP whose
    variables are all boxed (Lambda = R there, eq. defn_Lambda1), feasible or
    not.  The tests are therefore read as certificate tests on rays, i.e. on the
    homogeneous problem (c and h replaced by 0 in the residuals):

    * primal infeasibility: ray_y in K_d, lam = -G^T ray_y;
      ratio_p = err_abs,d(lam) / f with f = h^T ray_y + l^T lam+ - u^T lam-
      (finite bounds only).  A ray with f > 0 and err_abs,d(lam) = 0 is a Farkas
      certificate: every x with Gx - h in K_d*, l <= x <= u would give
      f <= 0.
    * dual infeasibility: ray_x in the recession cone of the box; the residual
      err_rel,p of the homogeneous problem is the Euclidean norm of
      G ray_x - Proj_{K_d*}(G ray_x) (its denominator 1 + ||h||_1 is 1 there);
      ratio_d = err_rel,p / (-c^T ray_x).  A ray with -c^T ray_x > 0 and zero
      residual proves the primal unbounded.
    * a denominator that is not positive, or not larger than the rounding
      bound gamma_N of its own sum (N terms, ``rounding_bound``) times the sum
      of its terms' magnitudes, makes the ratio +inf: the test cannot pass on
      a denominator that is rounding noise.

    Returns (ratio_p, ratio_d).
    """
    lam = -(lp.G.T @ ray_y)
    num_p = float(np.linalg.norm(lam - proj_Lambda(lam, lp.l, lp.u)))
    lf = np.isfinite(lp.l)
    uf = np.isfinite(lp.u)
    terms = [lp.h * ray_y, lp.l[lf] * np.maximum(lam[lf], 0.0), -lp.u[uf] * np.maximum(-lam[uf], 0.0)]
    f = float(sum(np.sum(t) for t in terms))
    mag = float(sum(np.sum(np.abs(t)) for t in terms))
    nterm = sum(t.size for t in terms)
    ratio_p = num_p / f if f > rounding_bound(nterm) * mag else math.inf
    r = lp.G @ ray_x
    num_d = float(np.linalg.norm(r - lp.proj_Kd_star(r)))
    cx = lp.c * ray_x
    g = -float(np.sum(cx))
    ratio_d = num_d / g if g > rounding_bound(cx.size) * float(np.sum(np.abs(cx))) else math.inf
    return ratio_p, ratio_d


TREND_CHECKS = 3


class InfeasibilityMonitor:
    """Low- and high-accuracy infeasibility tests of the option list (Section 3).

    Reading of the trend clause: the low-accuracy primal test passes at a check
    when ratio_p < eps_primal_infeasible_low_acc and the dual objective of the
    PDHG output z_hat is strictly larger than at the previous check; it fires
    once it has passed at TREND_CHECKS consecutive checks.  The dual test is
    the same with ratio_d and the negated primal objective -c^T x_hat (the
    primal objective decreases without bound on an unbounded LP).  The
    high-accuracy tests fire on the ratio alone.  A tolerance of 0 switches its
    test off.  Priority at one check: high-accuracy primal, high-accuracy dual,
    low-accuracy primal, low-accuracy dual.
    """

    def __init__(self, opts):
        self.eps = (opts.eps_primal_infeasible_low_acc, opts.eps_dual_infeasible_low_acc,
                    opts.eps_primal_infeasible_high_acc, opts.eps_dual_infeasible_high_acc)
        self.trend_p = 0
        self.trend_d = 0
        self.prev_dobj = None
        self.prev_negp = None

    @property
    def enabled(self) -> bool:
        return any(e > 0.0 for e in self.eps)

    def update(self, ratio_p, ratio_d, pobj, dobj):
        """Feed one check; returns an exit code (2-5) or None."""
        lo_p, lo_d, hi_p, hi_d = self.eps
        up_p = self.prev_dobj is not None and dobj > self.prev_dobj
        up_d = self.prev_negp is not None and -pobj > self.prev_negp
        self.prev_dobj, self.prev_negp = dobj, -pobj
        self.trend_p = self.trend_p + 1 if (ratio_p < lo_p and up_p) else 0
        self.trend_d = self.trend_d + 1 if (ratio_d < lo_d and up_d) else 0
        if ratio_p < hi_p:
            return EXIT_PRIMAL_INFEASIBLE_HIGH_ACC
        if ratio_d < hi_d:
            return EXIT_DUAL_INFEASIBLE_HIGH_ACC
        if self.trend_p >= TREND_CHECKS:
            return EXIT_PRIMAL_INFEASIBLE_LOW_ACC
        if self.trend_d >= TREND_CHECKS:
            return EXIT_DUAL_INFEASIBLE_LOW_ACC
        return None


# --------------------------------------------------------------------------
# Adaptive step size (Section 2.1, Function 2)
# --------------------------------------------------------------------------
def eta_bar(lp: LPData, dx, dy, omega):
    """Step-size limit: (1/2) ||(dx, dy)||_omega^2 / |dy^T G dx|, +inf when the
    denominator vanishes (reading: such a step is always accepted)."""
    num = 0.5 * (omega * np.dot(dx, dx) + np.dot(dy, dy) / omega)
    den = abs(float(np.dot(dy, lp.G @ dx)))
    if den == 0.0:
        return math.inf
    return float(num / den)


def eta_next(etabar, eta, kbar):
    """eta' = min((1-(kbar+1)^-0.3) eta_bar, (1+(kbar+1)^-0.6) eta)."""
    return min((1.0 - (kbar + 1) ** -0.3) * etabar, (1.0 + (kbar + 1) ** -0.6) * eta)


def adaptive_step_pdhg(lp: LPData, x, y, omega, eta, kbar, trace=None, max_kbar=1 << 62):
    """AdaptiveStepPDHG (Function 2).

    Reading of the trial counter: kbar counts every trial, accepted or not, and
    is incremented at the top of each trial, so the first trial of a solve uses
    kbar = 1 (with kbar = 0 the first factor of eta' would be zero).
    Returns (x_hat, y_hat, eta, eta', kbar, n_trials); x_hat is None when the
    trial budget ``max_kbar`` ran out on a rejected trial.
    """
    trials = 0
    while True:
        kbar += 1
        trials += 1
        tau = eta / omega
        sigma = eta * omega
        xh, yh = one_pdhg(lp, x, y, tau, sigma)
        eb = eta_bar(lp, xh - x, yh - y, omega)
        ep = eta_next(eb, eta, kbar)
        acc = eta < eb
        if trace is not None:
            trace.append(dict(kbar=kbar, eta=eta, eta_bar=eb, eta_next=ep, accepted=bool(acc)))
        if acc:
            return xh, yh, eta, ep, kbar, trials
        if not math.isfinite(ep) or ep <= 0.0:
            raise FloatingPointError("step size collapsed")
        eta = ep
        if kbar >= max_kbar:
            return None, None, eta, ep, kbar, trials


# --------------------------------------------------------------------------
# Normalized duality gap (Sections 2.3-2.4, Algorithm 3)
# --------------------------------------------------------------------------
def z_of_t(lp: LPData, x, y, b1, b2, tau, sigma, t):
    """z(t) of eq. compute_zt_2: (Proj_X(x + t tau b1), Proj_Y(y + t sigma b2))."""
    return proj_box(x + t * tau * b1, lp.l, lp.u), lp.proj_Kd(y + t * sigma * b2)


def n_norm(dx, dy, tau, sigma):
    """||(dx, dy)||_N with N = diag(I/tau, I/sigma)."""
    return math.sqrt(float(np.dot(dx, dx)) / tau + float(np.dot(dy, dy)) / sigma)


def gap_direction(lp: LPData, x, y):
    """b = (G^T y - c, h - G x) of eq. compute_rho."""
    return lp.G.T @ y - lp.c, lp.h - lp.G @ x


def normalized_gap(lp: LPData, x, y, tau, sigma, r, rel_eps=1e-6, max_doublings=64,
                   b=None):
    """rho^N(r; z) by Algorithm 3 (exponential search, then bisection on t).

    Readings (the algorithm leaves t0, eps and the returned point open):
    * t0 = r / sqrt(tau ||b1||^2 + sigma ||b2||^2): without projection this t
      gives ||z - z(t)||_N = r, and projection is nonexpansive, so z(t0) lies in
      the ball;
    * the search doubles t at most ``max_doublings`` times; if a doubling does
      not move the distance (every coordinate sits on a bound) the value at the
      current t is returned;
    * bisection stops when t_right - t_left <= rel_eps * t_right, and the value
      is taken at t_left (a point inside the ball);
    * r <= 0 or non-finite r returns NaN (treated by the caller as a numerical
      issue); b = 0 returns 0.
    """
    if not (r > 0.0) or not math.isfinite(r):
        return math.nan
    b1, b2 = gap_direction(lp, x, y) if b is None else b

    def dist(t):
        xt, yt = z_of_t(lp, x, y, b1, b2, tau, sigma, t)
        return n_norm(xt - x, yt - y, tau, sigma), xt, yt

    def value(xt, yt):
        return (float(np.dot(b1, xt - x)) + float(np.dot(b2, yt - y))) / r

    scale = math.sqrt(tau * float(np.dot(b1, b1)) + sigma * float(np.dot(b2, b2)))
    if scale == 0.0:
        return 0.0
    t0 = r / scale
    d0, x0, y0 = dist(t0)
    if d0 > r:
        t_left, t_right = 0.0, t0
    else:
        t_prev, d_prev, xp, yp = t0, d0, x0, y0
        bracket = False
        for _ in range(max_doublings):
            t = 2.0 * t_prev
            d, xt, yt = dist(t)
            if d > r:
                t_left, t_right = t_prev, t
                bracket = True
                break
            if d <= d_prev:  # saturated: z(2t) = z(t)
                return value(xp, yp)
            t_prev, d_prev, xp, yp = t, d, xt, yt
        if not bracket:
            return value(xp, yp)
    while t_right - t_left > rel_eps * t_right:
        t_mid = 0.5 * (t_left + t_right)
        d, _, _ = dist(t_mid)
        if d < r:
            t_left = t_mid
        else:
            t_right = t_mid
    _, xt, yt = dist(t_left)
    return value(xt, yt)


# --------------------------------------------------------------------------
# Primal weight (Section 2.5)
# --------------------------------------------------------------------------
def primal_weight_init(c, h):
    nc = float(np.linalg.norm(c))
    nh = float(np.linalg.norm(h))
    if nc > TINY and nh > TINY:
        return nc / nh
    return 1.0


def primal_weight_update(dx, dy, omega_prev, omega0):
    """PrimalWeightUpdate with theta = 0.5, then the reset to the initial weight when
    omega leaves [1e-5, 1e5]."""
    if dx > TINY and dy > TINY:
        omega = math.exp(THETA * math.log(dy / dx) + (1.0 - THETA) * math.log(omega_prev))
    else:
        omega = omega_prev
    if omega > OMEGA_MAX or omega < OMEGA_MIN:
        omega = omega0
    return omega


# --------------------------------------------------------------------------
# Restart logic (Section 2.3)
# --------------------------------------------------------------------------
def restart_decision(t, k, kbar, metric_c, metric_anchor, metric_prev):
    """Restart conditions 1-3 with beta_sufficient/necessary/artificial = 0.4/0.8/0.223.

    Readings: in the first interval (t = 0) the anchor has no predecessor, so
    conditions 1 and 2 are off; condition 2 compares with the candidate of the
    previous check in the same interval and is off at the interval's first check.
    """
    if k >= BETA_ARTIFICIAL * kbar:
        return True, 3
    if t == 0 or metric_anchor is None:
        return False, 0
    if metric_c <= BETA_SUFFICIENT * metric_anchor:
        return True, 1
    if metric_prev is not None and metric_c > metric_prev and metric_c <= BETA_NECESSARY * metric_anchor:
        return True, 2
    return False, 0


def _valid_rho(v):
    return v is not None and math.isfinite(v) and v >= 0.0


# --------------------------------------------------------------------------
# The solver (Algorithm 4 around Algorithm 1)
# --------------------------------------------------------------------------
@dataclass
class Options:
    rel_tol: float = 1e-6
    abs_tol: float = 1e-6
    max_iter: int = 1 << 62          # trial budget (exit code 1)
    time_limit: float = 1000.0       # seconds (exit code 6)
    use_preconditioner: bool = True
    ruiz_iters: int = 10
    l2_pass: bool = True
    method: str = "auto"             # auto | average | halpern (candidate rule)
    use_kkt_restart: bool = False    # compare candidates and restart on KKT_omega (Section 2.3)
    use_duality_gap_restart: bool = True  # the normalized duality gap as restart metric (Section 3)
    check_every: int = 64            # restart / termination check period, in trials
    kkt_restart_freq: int = 0        # check period when KKT_omega is the metric (0: check_every)
    duality_gap_restart_freq: int = 0  # check period when the gap is the metric (0: check_every)
    bisect_rel_eps: float = 1e-6
    max_doublings: int = 64
    eps_primal_infeasible_low_acc: float = 1e-12
    eps_dual_infeasible_low_acc: float = 1e-12
    eps_primal_infeasible_high_acc: float = 1e-16
    eps_dual_infeasible_high_acc: float = 1e-16

    def gap_metric(self) -> bool:
        """Reading of the restart options: the normalized duality gap is the metric
        unless use_kkt_restart is set or use_duality_gap_restart is cleared, in
        which case KKT_omega is (and the gap is not computed)."""
        return bool(self.use_duality_gap_restart) and not self.use_kkt_restart

    def period(self) -> int:
        """Trials between restart checks: the frequency option of the metric in
        use, or check_every when that option is 0."""
        f = self.duality_gap_restart_freq if self.gap_metric() else self.kkt_restart_freq
        return int(f) if f > 0 else int(self.check_every)


@dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    lam: np.ndarray
    exit_code: int
    pobj: float
    dobj: float
    errors: dict
    iters: int                     # kbar: all trials
    accepted: int
    restarts: int
    checks: int
    time_sec: float
    D1: np.ndarray
    D2: np.ndarray
    setup_sec: float = 0.0         # scaling and start point, before the first trial
    state: dict = field(default_factory=dict)
    trace: list = field(default_factory=list)
    checks_log: list = field(default_factory=list)


def solve(lp: LPData, opts: Options | None = None, x0=None, y0=None, trace: bool = False) -> Result:
    """PDCS with preconditioning (Algorithm 4) on an LP.

    Readings fixed here (all stated in the design notes):
    * the restart/termination check runs after an accepted trial whose trial
      count kbar is a multiple of ``check_every`` (the paper's options check every
      duality_gap_restart_freq iterations);
    * the restart candidates are the PDHG output z_hat^{t,k+1} and the eta-weighted
      average of the PDHG outputs of the interval; both lie in X x Y, which the
      normalized duality gap requires;
    * tau, sigma inside N are eta_hat/omega and eta_hat*omega at the check;
    * the anchor's metric is the candidate's value at the check that restarted;
    * termination is evaluated on the unscaled candidate at each check (and on
      the start point); the returned point is that candidate;
    * the infeasibility tests (``InfeasibilityMonitor``) run at each check that
      does not terminate, on the rays Proj(D2 (x_hat - x_start)) and
      Proj(D1 (y_hat - y_start)) (projections onto the recession cone of the box
      and onto K_d; z_start is the projected start point z^{0,0}).  On an
      infeasible or unbounded LP the iterates drift along a certificate, and
      the displacement since the start grows with the trial count while its
      error stays bounded, so the ratios fall like 1/kbar; the displacement
      since the anchor of the current interval would not.  Such an exit
      returns z_hat.
    """
    opts = opts or Options()
    t_start = time.perf_counter()
    m, n = lp.m, lp.n
    if opts.use_preconditioner:
        D1, D2 = ruiz_l2_scaling(lp.G, opts.ruiz_iters, opts.l2_pass)
    else:
        D1, D2 = np.ones(m), np.ones(n)
    sl = rescale(lp, D1, D2)

    def unscale(xs, ys):
        return D2 * xs, D1 * ys

    # Start point (reading: 0 when none is given), mapped to the scaled space and projected.
    xs = np.zeros(n) if x0 is None else np.asarray(x0, np.float64) / D2
    ys = np.zeros(m) if y0 is None else np.asarray(y0, np.float64) / D1
    x = proj_box(xs, sl.l, sl.u)
    y = sl.proj_Kd(ys)
    x_start, y_start = x.copy(), y.copy()

    gmax = float(np.max(np.abs(sl.G.data), initial=0.0))
    eta_hat = 1.0 / gmax if gmax > 0 else 1.0
    omega0 = primal_weight_init(sl.c, sl.h)
    omega = omega0
    kbar = 0
    accepted = 0
    restarts = 0
    checks = 0
    t = 0
    k = 0
    xa, ya = x.copy(), y.copy()
    Sx, Sy, SH = np.zeros(n), np.zeros(m), 0.0
    xh, yh = x.copy(), y.copy()
    metric_anchor = None
    metric_prev = None
    trial_log = [] if trace else None
    checks_log = []
    use_gap = opts.gap_metric()
    period = opts.period()
    monitor = InfeasibilityMonitor(opts)

    def finish(code, xs_, ys_):
        xu, yu = unscale(xs_, ys_)
        err = termination_errors(lp, xu, yu)
        lam = lp.c - lp.G.T @ yu
        return Result(xu, yu, lam, code, err["pobj"], err["dobj"], err, kbar, accepted,
                      restarts, checks, time.perf_counter() - t_start, D1, D2, setup_sec,
                      state=dict(x=x.copy(), y=y.copy(), x_hat=xh.copy(), y_hat=yh.copy(),
                                 x_anchor=xa.copy(), y_anchor=ya.copy(), Sx=Sx.copy(),
                                 Sy=Sy.copy(), SH=SH, omega=omega, omega0=omega0,
                                 eta_hat=eta_hat, kbar=kbar, k=k, t=t),
                      trace=trial_log or [], checks_log=checks_log)

    setup_sec = time.perf_counter() - t_start
    # Termination test of the start point.
    xu, yu = unscale(x, y)
    if is_optimal(termination_errors(lp, xu, yu), opts.rel_tol, opts.abs_tol):
        return finish(EXIT_OPTIMAL, x, y)

    while True:
        # ---- AdaptiveStepPDHG (Algorithm 1: the PDHG step with line search) ----
        out = adaptive_step_pdhg(sl, x, y, omega, eta_hat, kbar, trial_log, opts.max_iter)
        xh_new, yh_new, eta_k, eta_p, kbar, _ = out
        if xh_new is None:  # trial budget ran out during rejections
            return finish(EXIT_MAX_ITER, xh, yh)
        if not (np.all(np.isfinite(xh_new)) and np.all(np.isfinite(yh_new))):
            return finish(EXIT_NUMERICAL_ERROR, xh, yh)
        xh, yh = xh_new, yh_new
        eta_hat = eta_p
        accepted += 1
        # ---- reflection parameter beta at z_hat (Algorithm 1) ----
        beta = reflection_parameter(max_err(sl, xh, yh))
        if trial_log is not None:
            trial_log[-1]["beta"] = beta
        # ---- reflected Halpern update (Algorithm 1) ----
        a = (k + 1.0) / (k + 2.0)
        bcoef = 1.0 / (k + 2.0)
        x = a * ((1.0 + beta) * xh - beta * x) + bcoef * xa
        y = a * ((1.0 + beta) * yh - beta * y) + bcoef * ya
        # ---- eta-weighted average of the PDHG outputs (Algorithm 1) ----
        Sx = Sx + eta_k * xh
        Sy = Sy + eta_k * yh
        SH += eta_k
        k += 1

        if kbar % period == 0:
            checks += 1
            tau_c = eta_hat / omega
            sig_c = eta_hat * omega
            cands = {}
            if opts.method in ("auto", "halpern"):
                cands["cur"] = (xh, yh)
            if opts.method in ("auto", "average"):
                cands["avg"] = (Sx / SH, Sy / SH)
            info = {}
            for name, (cx, cy) in cands.items():
                r = n_norm(cx - xa, cy - ya, tau_c, sig_c)
                rho = (normalized_gap(sl, cx, cy, tau_c, sig_c, r, opts.bisect_rel_eps,
                                      opts.max_doublings) if use_gap else math.nan)
                ep, ed, eg, _, _ = abs_errors_l2(sl, cx, cy)
                info[name] = dict(rho=rho, kkt=kkt_omega(ep, ed, eg, omega), err=(ep, ed, eg), r=r)
            # Numerical issue (Section 2.3): any gap value of this check, of the
            # anchor or of the previous candidate that is negative, NaN or has
            # r = 0 switches every comparison of this check to KKT_omega.
            stored = [d["rho"] for d in (metric_anchor, metric_prev) if d is not None]
            use_kkt = not use_gap or not all(
                _valid_rho(v) for v in [i["rho"] for i in info.values()] + stored)
            key = "kkt" if use_kkt else "rho"
            if "cur" in info and "avg" in info:
                chosen = "cur" if info["cur"][key] <= info["avg"][key] else "avg"
            else:
                chosen = next(iter(info))
            cx, cy = cands[chosen]
            mc = info[chosen][key]
            m_anchor = None if metric_anchor is None else metric_anchor[key]
            m_prev = None if metric_prev is None else metric_prev[key]
            restart, rule = restart_decision(t, k, kbar, mc, m_anchor, m_prev)
            xu, yu = unscale(cx, cy)
            err = termination_errors(lp, xu, yu)
            done = is_optimal(err, opts.rel_tol, opts.abs_tol)
            checks_log.append(dict(kbar=kbar, k=k, t=t, chosen=chosen, use_kkt=use_kkt,
                                   rho={nm: v["rho"] for nm, v in info.items()},
                                   r={nm: v["r"] for nm, v in info.items()},
                                   restart=bool(restart or done), rule=rule, omega=omega,
                                   rel=max(err["rel_p"], err["rel_d"], err["rel_gap"])))
            if done:
                x, y = cx.copy(), cy.copy()
                xh, yh = cx.copy(), cy.copy()
                return finish(EXIT_OPTIMAL, cx, cy)
            if monitor.enabled:
                ray_x = proj_box_recession(D2 * (xh - x_start), lp.l, lp.u)
                ray_y = lp.proj_Kd(D1 * (yh - y_start))
                ratio_p, ratio_d = infeasibility_ratios(lp, ray_x, ray_y)
                e_h = termination_errors(lp, D2 * xh, D1 * yh)
                code = monitor.update(ratio_p, ratio_d, e_h["pobj"], e_h["dobj"])
                checks_log[-1].update(ratio_p=ratio_p, ratio_d=ratio_d)
                if code is not None:
                    res = finish(code, xh, yh)
                    res.state.update(ray_x=ray_x, ray_y=ray_y)
                    return res
            if restart:
                # PrimalWeightUpdate(z^{t+1,0}, z^{t,0}, omega^t) and the new anchor.
                dxn = float(np.linalg.norm(cx - xa))
                dyn = float(np.linalg.norm(cy - ya))
                omega = primal_weight_update(dxn, dyn, omega, omega0)
                ep, ed, eg = info[chosen]["err"]
                metric_anchor = dict(rho=info[chosen]["rho"], kkt=kkt_omega(ep, ed, eg, omega))
                metric_prev = None
                xa, ya = cx.copy(), cy.copy()
                x, y = cx.copy(), cy.copy()
                Sx, Sy, SH = np.zeros(n), np.zeros(m), 0.0
                k = 0
                t += 1
                restarts += 1
            else:
                metric_prev = dict(rho=info[chosen]["rho"], kkt=info[chosen]["kkt"])
        if kbar >= opts.max_iter:
            return finish(EXIT_MAX_ITER, xh, yh)
        if time.perf_counter() - t_start > opts.time_limit:
            return finish(EXIT_TIME_LIMIT, xh, yh)
