// HIP kernels of the PDCS LP solver for gfx950.
//
// One trial of AdaptiveStepPDHG (Function 2) is five launches:
//   k_primal   : deferred reflected-Halpern commit of x and of G^T y (Algorithm 1:
//                reflection and averaging), then x_hat = Proj_[l,u](x - tau (c - G^T y))   (eq. PDHG)
//   k_dual     : CSR SpMV G x_hat with the dual step fused into the row epilogue:
//                Halpern commit of y and of G x, then
//                y_hat = Proj_Kd(y + sigma (h - 2 G x_hat + G x))          (eq. PDHG)
//   k_fin_ls   : step-size test of Function 2 (eta_bar, eta')
//   k_lam      : transposed SpMV G^T y_hat with the dual-slack epilogue
//                lam = c - G^T y_hat and its error terms (eq. tolerance-3)
//   k_fin_beta : reflection parameter (eq. adaptive_reflection)
// G x and G^T y of the Halpern iterate are maintained by the same linear
// combination as the iterate, so a trial reads the matrix once (G x_hat) and
// an accepted trial twice (plus G^T y_hat).
//
// Every K trials a restart check runs (Section 2.3): candidate products with
// FP64 values, N-norm radii, the bisection of Algorithm 3 as a multisection
// (kProbes values of t per pass over the vectors), the restart conditions,
// the primal-weight update (Section 2.5) and the termination test (Section 3).
#include "pdcs_dev.h"
#include "pdcs_launch.h"

#include <math.h>

#include <algorithm>

namespace pdcs {

// ===========================================================================
// Second-order-cone row blocks (socG option of Section 3, rescaled cones of
// Section 2.6)
// ===========================================================================
// Projection of one block v (element i read by ld(i)) onto diag(e) K_soc,
// K_soc = {(t, w): ||w|| <= t}, e_i = ef(i) > 0, by one wave; element i of the
// result goes to st(i, p_i), each by the lane that read v_i.  From the KKT
// conditions: v itself inside the cone; 0 inside the polar cone -diag(1/e)
// K_soc (||w e_w|| <= -t e_t); otherwise the multiplier mu > 0 is the root of
//   F(mu) = sum_i v_i^2 e_i^2 / (e_i^2 s + mu)^2 = 1,  s = v_0 / e_0 + mu / e_0^2
// (sum over i >= 1), F decreasing, F > 1 at max(0, -v_0 e_0) and F <= 1 at
// ||w e_w||: Newton steps on 1 - F^-1/2 (linear in mu when one term
// dominates), kept inside the bracket, then p_0 = e_0 s and
// p_i = v_i e_i^2 s / (e_i^2 s + mu).  FP64 throughout; the
// first kSocCache elements of each lane stay in registers.
constexpr int kSocCache = 4;

template <class LD, class EF, class ST>
__device__ __forceinline__ void wave_proj_soc(int d, const LD& ld, const EF& ef, const ST& st) {
  const int lane = threadIdx.x & (kWave - 1);
  const double v0 = ld(0), e0 = ef(0);
  double vr[kSocCache], er[kSocCache];
#pragma unroll
  for (int k = 0; k < kSocCache; ++k) {
    const int i = lane + k * kWave;
    vr[k] = i < d ? ld(i) : 0.0;
    er[k] = i < d ? ef(i) : 1.0;
  }
  // fn(i, v_i, e_i) over this lane's elements i >= 1
  const auto each = [&](auto&& fn) {
#pragma unroll
    for (int k = 0; k < kSocCache; ++k) {
      const int i = lane + k * kWave;
      if (i >= 1 && i < d) fn(i, vr[k], er[k]);
    }
    for (int i = lane + kSocCache * kWave; i < d; i += kWave) fn(i, ld(i), ef(i));
  };
  double in_w = 0.0, po_w = 0.0;
  each([&](int, double v, double e) {
    in_w += (v / e) * (v / e);
    po_w += (v * e) * (v * e);
  });
  in_w = wave_sum(in_w);
  po_w = wave_sum(po_w);
  if (sqrt(in_w) <= v0 / e0) {
    if (lane == 0) st(0, v0);
    each([&](int i, double v, double) { st(i, v); });
    return;
  }
  if (sqrt(po_w) <= -v0 * e0) {
    if (lane == 0) st(0, 0.0);
    each([&](int i, double, double) { st(i, 0.0); });
    return;
  }
  const double ie02 = 1.0 / (e0 * e0);
  double lo = fmax(0.0, -v0 * e0), hi = fmax(lo, sqrt(po_w));
  // phi = 1 - F^-1/2 is < 0 at lo and >= 0 at hi; a Newton step that leaves
  // the bracket is replaced by the secant step of phi over it (bisection while
  // phi is unknown at an end), and one that lands within rounding of an end
  // (the root sits at that end) ends the search there
  double mu = lo, flo = NAN, fhi = NAN;
#pragma unroll 1
  for (int it = 0; it < 200; ++it) {
    const double sv = v0 / e0 + mu * ie02;
    double F = 0.0, dF = 0.0;
    each([&](int, double v, double e) {
      const double e2 = e * e;
      const double den = e2 * sv + mu, q = v * v * e2;
      if (q > 0.0) {  // (a zero term stays zero at den = 0, which mu = 0 with v_0 = 0 gives)
        F += q / (den * den);
        dF -= 2.0 * q * (e2 * ie02 + 1.0) / (den * den * den);
      }
    });
    F = wave_sum(F);
    dF = wave_sum(dF);
    const double rs = 1.0 / sqrt(F);
    const double phi = 1.0 - rs;
    if (F > 1.0) lo = mu, flo = phi;
    else hi = mu, fhi = phi;
    if (F == 1.0 || !(hi > lo) || hi - lo <= 4e-16 * hi) break;
    double next = mu - 2.0 * phi / (rs * rs * rs * dF);
    if (!(next > lo && next < hi)) {
      if (fabs(next - lo) <= 4e-16 * lo) {
        mu = lo;
        break;
      }
      if (fabs(next - hi) <= 4e-16 * hi) {
        mu = hi;
        break;
      }
      next = (flo == flo && fhi == fhi) ? lo - flo * (hi - lo) / (fhi - flo) : 0.5 * (lo + hi);
      if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
    }
    if (fabs(next - mu) <= 4e-16 * next) {
      mu = next;
      break;
    }
    mu = next;
  }
  const double sv = v0 / e0 + mu * ie02;
  if (lane == 0) st(0, e0 * sv);
  each([&](int i, double v, double e) {
    const double e2 = e * e;
    st(i, v * e2 * sv / (e2 * sv + mu));
  });
}

// ===========================================================================
// Exponential-cone row blocks (expG and dual_expG options of Section 3)
// ===========================================================================
// K_exp = closure {(x, y, z): y > 0, y e^(x / y) <= z}; its dual cone
// K_exp* = closure {(u, v, w): u < 0, -u e^(v / u) <= e w}.
__device__ __forceinline__ bool exp_cone_has(double x, double y, double z) {
  if (y > 0.0) return z > 0.0 && x <= y * log(z / y);
  return y == 0.0 && x <= 0.0 && z >= 0.0;
}

__device__ __forceinline__ bool exp_dual_has(double u, double v, double w) {
  if (u < 0.0) return w > 0.0 && log(-u) + v / u <= 1.0 + log(w);
  return u == 0.0 && v >= 0.0 && w >= 0.0;
}

// (u, v, w) in K_exp* up to 1e-15 of its size (rounding).
__device__ __forceinline__ bool exp_dual_near(double u, double v, double w) {
  const double sc = 1e-15 * (fabs(u) + fabs(v) + fabs(w));
  if (u < -sc) return -u * exp(v / u) <= M_E * w + sc;
  return v >= -sc && w >= -sc;
}

// A point to project onto F K_exp: v, f and 1 / f.
struct ExpPoint {
  double v[3], f[3], fi[3];
};

// Sign of the slope of the angle between v and the boundary ray of F K_exp
// through F a(r), a(r) = (r, 1, e^r): the triple product
// det[v, F a(r), F^-1 n(r)], n(r) = (-1, r - 1, e^-r) the element of K_exp*
// normal to the cone along the ray (F a(r) x F^-1 n(r) points along the
// derivative of the unit ray), times e^r, divided by e^2r for r > 0 so that
// it stays finite.  E = e^r and iE = e^-r are passed in.
__device__ __forceinline__ double exp_ray_turn(double r, double E, double iE, const ExpPoint& P) {
  double a0, a1, a2, m0, m1, m2;  // a = F a(r), m = e^r F^-1 n(r), both times e^-r when r > 0
  if (r <= 0.0) {
    a0 = P.f[0] * r, a1 = P.f[1], a2 = P.f[2] * E;
    m0 = -E * P.fi[0], m1 = E * (r - 1.0) * P.fi[1], m2 = P.fi[2];
  } else {
    a0 = P.f[0] * r * iE, a1 = P.f[1] * iE, a2 = P.f[2];
    m0 = -P.fi[0], m1 = (r - 1.0) * P.fi[1], m2 = iE * P.fi[2];
  }
  return P.v[0] * (a1 * m2 - a2 * m1) + P.v[1] * (a2 * m0 - a0 * m2) + P.v[2] * (a0 * m1 - a1 * m0);
}

// The slope t at r (one exp), its derivative dt and the size sc of the terms
// summed into t (|t| <= 1e-15 sc is rounding noise: r is a root).
__device__ __forceinline__ void exp_ray_turn_d(double r, const ExpPoint& P, double& t, double& dt, double& sc) {
  double a0, a1, a2, m0, m1, m2, da0, da1, da2, dm0, dm1, dm2;
  const double q = exp(-fabs(r));  // e^r for r <= 0, e^-r above
  if (r <= 0.0) {
    const double E = q;
    a0 = P.f[0] * r, a1 = P.f[1], a2 = P.f[2] * E;
    m0 = -E * P.fi[0], m1 = E * (r - 1.0) * P.fi[1], m2 = P.fi[2];
    da0 = P.f[0], da1 = 0.0, da2 = a2;
    dm0 = m0, dm1 = E * r * P.fi[1], dm2 = 0.0;
  } else {  // both vectors times e^-r: the derivative of t e^-2r, whose sign change is the same
    const double iE = q;
    a0 = P.f[0] * r * iE, a1 = P.f[1] * iE, a2 = P.f[2];
    m0 = -P.fi[0], m1 = (r - 1.0) * P.fi[1], m2 = iE * P.fi[2];
    da0 = P.f[0] * (1.0 - r) * iE, da1 = -a1, da2 = 0.0;
    dm0 = 0.0, dm1 = P.fi[1], dm2 = -m2;
  }
  const double c0 = a1 * m2 - a2 * m1, c1 = a2 * m0 - a0 * m2, c2 = a0 * m1 - a1 * m0;
  t = P.v[0] * c0 + P.v[1] * c1 + P.v[2] * c2;
  sc = fabs(P.v[0]) * (fabs(a1 * m2) + fabs(a2 * m1)) + fabs(P.v[1]) * (fabs(a2 * m0) + fabs(a0 * m2)) +
       fabs(P.v[2]) * (fabs(a0 * m1) + fabs(a1 * m0));
  dt = P.v[0] * (da1 * m2 - da2 * m1 + a1 * dm2 - a2 * dm1) + P.v[1] * (da2 * m0 - da0 * m2 + a2 * dm0 - a0 * dm2) +
       P.v[2] * (da0 * m1 - da1 * m0 + a0 * dm1 - a1 * dm0);
}

// Candidate on the ray of r: the nearest point s F a(r), s = <F a, v> / |F a|^2,
// kept in (bd, b) when s > 0 and it is nearer than bd; cert is set when it is
// nearer and v - p is a nonpositive multiple of F^-1 n(r) (at a root of the
// slope v - p is parallel to it): then -F (v - p) lies in K_exp*, p in F K_exp
// and <p, v - p> = 0, which makes p the projection.
__device__ __forceinline__ void exp_ray_candidate(double r, const ExpPoint& P, double& bd, double& b0, double& b1,
                                                  double& b2, bool& cert) {
  const double q = exp(-fabs(r));  // e^r for r <= 0, e^-r above
  const double E = r <= 0.0 ? q : 1.0 / q;
  const double q0 = P.f[0] * r, q1 = P.f[1], q2 = P.f[2] * E;
  const double s = (q0 * P.v[0] + q1 * P.v[1] + q2 * P.v[2]) / (q0 * q0 + q1 * q1 + q2 * q2);
  if (!(s > 0.0)) return;
  const double c0 = s * q0, c1 = s * q1, c2 = s * q2;
  const double d0 = P.v[0] - c0, d1 = P.v[1] - c1, d2 = P.v[2] - c2;
  const double d = d0 * d0 + d1 * d1 + d2 * d2;
  // m = F^-1 n(r) min(1, e^r); at a root v - p is parallel to m, so the cosine
  // of their angle is -1 (the projection) or +1 (not): the test takes the
  // sign with room for rounding, and a residual at the rounding level of v
  // (v on the boundary: p is then within that level of the projection)
  const double m0 = r <= 0.0 ? -E * P.fi[0] : -P.fi[0];
  const double m1 = r <= 0.0 ? (r - 1.0) * E * P.fi[1] : (r - 1.0) * P.fi[1];
  const double m2 = r <= 0.0 ? P.fi[2] : q * P.fi[2];
  const double w = d0 * m0 + d1 * m1 + d2 * m2;
  const double vv = P.v[0] * P.v[0] + P.v[1] * P.v[1] + P.v[2] * P.v[2];
  const bool ok = w <= 0.5 * sqrt(d * (m0 * m0 + m1 * m1 + m2 * m2)) || d <= 1e-24 * vv;
  // a certified candidate is the projection: it replaces an uncertified one
  // even when rounding makes it look no nearer (near the apex the face clip
  // and the projection can be within rounding of the same distance from v
  // while the points differ by the square root of that rounding)
  if (!((ok && !cert) || (ok == cert && d < bd))) return;
  bd = d, b0 = c0, b1 = c1, b2 = c2, cert = ok;
}

// One scan of the rays by the wave: lane l takes cells [l C, l C + C) of
// width h from r = -32 C h, every + to - sign change of the slope is refined
// to full precision and its candidate kept (exp_ray_candidate).  e^r runs by
// multiplication with g = e^h (ig = e^-h) along a lane's cells (the
// refinement uses exp itself).
// (Loops are kept rolled throughout, so that each kernel holds one compact
// copy of the projection.)
__device__ __forceinline__ void exp_scan(int C, double h, double g, double ig, const ExpPoint& P, double& bd,
                                         double& b0, double& b1, double& b2, bool& cert) {
  const int lane = threadIdx.x & (kWave - 1);
  const double r_first = -0.5 * kWave * C * h;
  int k = lane * C;
  double lo = r_first + k * h;
  const double q = exp(-fabs(lo));
  double E = lo <= 0.0 ? q : 1.0 / q, iE = lo <= 0.0 ? 1.0 / q : q;
  double t_lo = exp_ray_turn(lo, E, iE, P);
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    ++k;
    const double hi = r_first + k * h;
    E *= g, iE *= ig;
    const double t_hi = exp_ray_turn(hi, E, iE, P);
    if (t_lo > 0.0 && t_hi <= 0.0) {
      // Newton steps from the secant point of the cell, kept inside the
      // bracket [x, z] (slope > 0 at x, <= 0 at z; bisection when a step
      // leaves it), until the slope is rounding noise
      double x = lo, z = hi;
      double r = (lo * t_hi - hi * t_lo) / (t_hi - t_lo);
      if (!(r > x && r < z)) r = 0.5 * (x + z);
#pragma unroll 1
      for (int it = 0; it < 100; ++it) {
        double t, dt, sc;
        exp_ray_turn_d(r, P, t, dt, sc);
        if (fabs(t) <= 1e-15 * sc) break;
        if (t > 0.0) x = r;
        else z = r;
        double nr = r - t / dt;
        if (!(nr > x && nr < z)) nr = 0.5 * (x + z);
        if (!(nr > x && nr < z)) break;
        r = nr;
      }
      exp_ray_candidate(r, P, bd, b0, b1, b2, cert);
    }
    lo = hi;
    t_lo = t_hi;
  }
}

// Best candidate over the wave: certified before uncertified, then the nearest
// (ties: the lowest lane), among the lanes that hold a certified candidate or,
// when need_cert is false, among all.  Returns whether any lane took part.
__device__ __forceinline__ bool exp_wave_pick(double bd, double b0, double b1, double b2, bool cert, bool need_cert,
                                              double (&p)[3]) {
  const int lane = threadIdx.x & (kWave - 1);
  const bool eligible = cert || !need_cert;
  double d = eligible ? bd : INFINITY;
  int who = eligible ? lane : kWave;
  int rank = cert ? 0 : 1;
  for (int off = 1; off < kWave; off <<= 1) {
    const double od = __shfl_xor(d, off);
    const int ow = __shfl_xor(who, off), orank = __shfl_xor(rank, off);
    const double o0 = __shfl_xor(b0, off), o1 = __shfl_xor(b1, off), o2 = __shfl_xor(b2, off);
    if (ow < kWave &&
        (who == kWave || orank < rank || (orank == rank && (od < d || (od == d && ow < who)))))
      d = od, who = ow, rank = orank, b0 = o0, b1 = o1, b2 = o2;
  }
  if (who == kWave) return false;
  p[0] = b0, p[1] = b1, p[2] = b2;
  return true;
}

// Projection of v onto F K_exp, F = diag(f) > 0, by one wave (every lane gets
// the result).  v itself if v / f is in K_exp; 0 if -F v is in K_exp* (the
// polar cone); the clip onto the face {(x, 0, z): x <= 0, z >= 0} if -F times
// its residual is in K_exp* up to rounding (then the clip is within rounding
// of the projection: this takes the points whose projection lies on a ray
// so far out that it meets the face's edge to working precision); otherwise,
// among the face's clip and the
// best points of the rays s F a(r): the local maxima of the angle along the
// rays (+ to - sign changes of exp_ray_turn) and, for rays below the scanned
// range, whose third coordinate is then below e^-300 of the others, the ray
// through v's own x / y, r = (v_1 / f_1) / (v_2 / f_2).  A first scan on a
// coarse grid (step 0.4 over |r| <= 307.2) ends the search when a candidate
// carries the projection's certificate; else a scan on a fine grid (step
// 0.05 over |r| <= 300.8) takes a certified candidate if one turns up, else
// the nearest of all candidates.  Above the
// scanned range the rays lie within e^-300 of the face's edge (0, 0, 1).
constexpr double kExpTail = -300.0;

__device__ __forceinline__ void exp_proj_wave(const double (&v)[3], const double (&f)[3], double (&p)[3]) {
  ExpPoint P;
  for (int i = 0; i < 3; ++i) P.v[i] = v[i], P.f[i] = f[i], P.fi[i] = 1.0 / f[i];
  if (exp_cone_has(v[0] / f[0], v[1] / f[1], v[2] / f[2])) {
    p[0] = v[0], p[1] = v[1], p[2] = v[2];
    return;
  }
  if (exp_dual_has(-f[0] * v[0], -f[1] * v[1], -f[2] * v[2])) {
    p[0] = p[1] = p[2] = 0.0;
    return;
  }
  const double face[3] = {fmin(v[0], 0.0), 0.0, fmax(v[2], 0.0)};
  if (exp_dual_near(-f[0] * (v[0] - face[0]), -f[1] * v[1], -f[2] * (v[2] - face[2]))) {
    p[0] = face[0], p[1] = face[1], p[2] = face[2];
    return;
  }
  const double face_d = (v[0] - face[0]) * (v[0] - face[0]) + v[1] * v[1] + (v[2] - face[2]) * (v[2] - face[2]);
  const bool tail = v[0] < 0.0 && v[1] > 0.0 && (v[0] * P.fi[0]) / (v[1] * P.fi[1]) < kExpTail;
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {  // coarse, then fine
    double bd = face_d, b0 = face[0], b1 = face[1], b2 = face[2];
    bool cert = false;
    if (tail && lane == 0) exp_ray_candidate((v[0] * P.fi[0]) / (v[1] * P.fi[1]), P, bd, b0, b1, b2, cert);
    // e^0.4, e^-0.4, e^0.05, e^-0.05 to double precision
    exp_scan(pass == 0 ? 24 : 188, pass == 0 ? 0.4 : 0.05, pass == 0 ? 1.4918246976412703 : 1.0512710963760241,
             pass == 0 ? 0.6703200460356393 : 0.951229424500714, P, bd, b0, b1, b2, cert);
    if (exp_wave_pick(bd, b0, b1, b2, cert, pass == 0, p)) return;
  }
}

// Projection of a 3-row block onto F K_exp (dual = false) or onto F K_exp*
// (dual = true: F K_exp* is the dual cone of F^-1 K_exp, so by Moreau's
// decomposition P(v) = v + P_{F^-1 K_exp}(-v)), by one wave; ld, ef and st as
// in wave_proj_soc (element i stored by lane i).
template <class LD, class EF, class ST>
__device__ __forceinline__ void wave_proj_exp(bool dual, const LD& ld, const EF& ef, const ST& st) {
  const int lane = threadIdx.x & (kWave - 1);
  const double v[3] = {ld(0), ld(1), ld(2)};
  const double f[3] = {ef(0), ef(1), ef(2)};
  const double w[3] = {dual ? -v[0] : v[0], dual ? -v[1] : v[1], dual ? -v[2] : v[2]};
  const double g[3] = {dual ? 1.0 / f[0] : f[0], dual ? 1.0 / f[1] : f[1], dual ? 1.0 / f[2] : f[2]};
  double q[3];
  exp_proj_wave(w, g, q);
  const double p[3] = {dual ? v[0] + q[0] : q[0], dual ? v[1] + q[1] : q[1], dual ? v[2] + q[2] : q[2]};
  if (lane < 3) st(lane, lane == 0 ? p[0] : (lane == 1 ? p[1] : p[2]));
}

// Cone block kinds of the block table.
constexpr int kConeSoc = 0, kConeExp = 1, kConeDualExp = 2;

// Projection of one cone block of kind `kind` at a primal site (the cone of
// G x - h: K_soc, K_exp or K_exp*) or a dual site (the cone of y, its dual:
// K_soc, K_exp* or K_exp), rescaled by diag(ef).
template <class LD, class EF, class ST>
__device__ __forceinline__ void wave_proj_cone(int kind, bool dual_site, int d, const LD& ld, const EF& ef,
                                               const ST& st) {
  if (kind == kConeSoc) wave_proj_soc(d, ld, ef, st);
  else wave_proj_exp((kind == kConeExp) == dual_site, ld, ef, st);
}

// The cone blocks of row range b, each with S independent tasks (sub = 0 ..
// S - 1), are handled by the waves of its workgroup: task j of the range
// (block j / S, sub j mod S) by wave j mod kWavesPerBlock;
// fn(first row, dimension, kind, sub).
template <int S, class FN>
__device__ __forceinline__ void for_cone_tasks(const Ranges& R, int b, const FN& fn) {
  if (!R.blk_soc0) return;
  const int wave = threadIdx.x / kWave;
  const int q0 = R.blk_soc0[b], n = (R.blk_soc1[b] - q0) * S;
#pragma unroll 1
  for (int j = wave; j < n; j += kWavesPerBlock) {
    const int q = q0 + j / S;
    fn(R.soc_r0[q], R.soc_dim[q], (int)R.soc_kind[q], j % S);
  }
}

template <class FN>
__device__ __forceinline__ void for_cone_blocks(const Ranges& R, int b, const FN& fn) {
  for_cone_tasks<1>(R, b, [&](int r0, int dim, int kind, int) { fn(r0, dim, kind); });
}

// Projection of count vectors of dimension dim (v, f and out: dim doubles
// each, contiguous) onto diag(f) K, K = K_soc (cone 0), K_exp (cone 1) or
// K_exp* (cone 2, dim 3), one wave each.
__global__ __launch_bounds__(kBlock) void k_proj_cone(int cone, int dim, const double* __restrict__ v,
                                                      const double* __restrict__ f, double* __restrict__ out,
                                                      int64_t count) {
  const int64_t q = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (q >= count) return;
  const size_t o = (size_t)q * dim;
  const auto ld = [&](int i) { return v[o + i]; };
  const auto ef = [&](int i) { return f[o + i]; };
  const auto st = [&](int i, double p) { out[o + i] = p; };
  if (cone == 0) wave_proj_soc(dim, ld, ef, st);
  else wave_proj_exp(cone == 2, ld, ef, st);
}

// ===========================================================================
// Iteration kernels
// ===========================================================================

// K3: primal step over the columns of the instance.
// The five passes of a trial are device functions of the workgroup's range or
// instance, so that k_trials_wg can run them back to back inside one workgroup.
template <typename T>
__device__ __forceinline__ void primal_body(int b, const Ranges& R, const IterPtrs<T>& it, const DataPtrs<T>& d,
                                            Inst* inst, int prec, double* rec) {
  __shared__ double lds[kWavesPerBlock * 2];
  const Inst& I = inst[R.blk_inst[b]];
  if (I.status != kActive || I.precision != prec) return;
  const bool commit = I.pending != 0;
  const bool avg = I.use_avg != 0;
  const double ca = I.ca, cb = I.cb, beta = I.beta, etak = I.eta_k;
  const double tau = I.eta / I.omega;
  double acc[2] = {0.0, 0.0};
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    double x = (double)it.x[j];
    double gty = (double)it.gty[j];
    if (commit) {
      const double xh = (double)it.xh[j];
      const double gh = (double)it.gtyh[j];
      x = (double)(T)(ca * ((1.0 + beta) * xh - beta * x) + cb * (double)it.xa[j]);
      gty = (double)(T)(ca * ((1.0 + beta) * gh - beta * gty) + cb * (double)it.gtya[j]);
      it.x[j] = (T)x;
      it.gty[j] = (T)gty;
      if (avg) it.sx[j] = (T)((double)it.sx[j] + etak * xh);
    }
    const double c = (double)d.c[j];
    const double xn = (double)(T)clampd(x - tau * (c - gty), (double)d.l[j], (double)d.u[j]);
    it.xh[j] = (T)xn;
    const double dx = xn - x;
    acc[0] += dx * dx;
    acc[1] += c * xn;
  }
  block_sum_store<2>(acc, lds, rec + (size_t)b * 2);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_primal(Ranges R, IterPtrs<T> it, DataPtrs<T> d,
                                                   Inst* __restrict__ inst, int prec,
                                                   double* __restrict__ rec) {
  primal_body<T>(blockIdx.x, R, it, d, inst, prec, rec);
}

// K1: CSR SpMV G x_hat with the fused dual step.  Record: ||dy||^2,
// dy^T G dx, ||(G x_hat - h) - Proj_Kd*(.)||^2, h^T y_hat.
template <typename T>
struct DualEpilogue {
  IterPtrs<T> it;
  DataPtrs<T> d;
  bool commit, avg;
  double ca, cb, beta, etak, sigma;
  int mz_end, soc_start;
  __device__ __forceinline__ void operator()(int r, double s, double (&acc)[4]) const {
    double y = (double)it.y[r];
    double gx = (double)it.gx[r];
    if (commit) {
      const double yh = (double)it.yh[r];
      const double gh = (double)it.gxh[r];
      y = (double)(T)(ca * ((1.0 + beta) * yh - beta * y) + cb * (double)it.ya[r]);
      gx = (double)(T)(ca * ((1.0 + beta) * gh - beta * gx) + cb * (double)it.gxa[r]);
      it.y[r] = (T)y;
      it.gx[r] = (T)gx;
      if (avg) it.sy[r] = (T)((double)it.sy[r] + etak * yh);
    }
    const double hv = (double)d.h[r];
    const double gxn = (double)(T)s;
    const double v = y + sigma * (hv - 2.0 * gxn + gx);
    if (r >= soc_start) {  // cone block row: projected with its block afterwards
      it.yh[r] = (T)v;
      it.gxh[r] = (T)gxn;
      return;
    }
    const bool zero_row = r < mz_end;
    const double yn = (double)(T)(zero_row ? v : fmax(v, 0.0));
    it.yh[r] = (T)yn;
    it.gxh[r] = (T)gxn;
    const double dy = yn - y;
    acc[0] += dy * dy;
    acc[1] += dy * (gxn - gx);
    const double res = gxn - hv;
    const double pr = zero_row ? res : fmin(res, 0.0);
    acc[2] += pr * pr;
    acc[3] += hv * yn;
  }
};

template <typename T>
__device__ __forceinline__ DualEpilogue<T> make_dual_epilogue(const Inst& I, const IterPtrs<T>& it,
                                                              const DataPtrs<T>& d) {
  DualEpilogue<T> e;
  e.it = it;
  e.d = d;
  e.commit = I.pending != 0;
  e.avg = I.use_avg != 0;
  e.ca = I.ca;
  e.cb = I.cb;
  e.beta = I.beta;
  e.etak = I.eta_k;
  e.sigma = I.eta * I.omega;
  e.mz_end = I.row0 + I.m_zero;
  e.soc_start = I.soc_start;
  return e;
}

template <typename T>
__device__ __forceinline__ void lam_epilogue(int j, double s, const IterPtrs<T>& it, const DataPtrs<T>& d,
                                             double (&acc)[3]) {
  const double g = (double)(T)s;
  it.gtyh[j] = (T)g;
  const double lam = (double)d.c[j] - g;
  const double lo = (double)d.l[j], hi = (double)d.u[j];
  const bool lf = isfinite(lo), uf = isfinite(hi);
  double res;
  if (!lf && !uf) res = lam;
  else if (!lf) res = fmax(lam, 0.0);
  else if (!uf) res = fmin(lam, 0.0);
  else res = 0.0;
  acc[0] += res * res;
  if (lf) acc[1] += lo * fmax(lam, 0.0);
  if (uf) acc[2] += hi * fmax(-lam, 0.0);
}

template <typename T, typename TM>
__device__ __forceinline__ void dual_body(int b, const RowBlocks& rb, const MatPtrs<TM>& A, const IterPtrs<T>& it,
                                          const DataPtrs<T>& d, Inst* inst, int prec, double* rec) {
  __shared__ double lds[kRowBlockCap + kWavesPerBlock * 4];
  const Inst& I = inst[rb.blk_inst[b]];
  if (I.status != kActive || I.precision != prec) return;
  const DualEpilogue<T> epi = make_dual_epilogue(I, it, d);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const T* const xs[1] = {it.xh};
  block_rows<1>(rb.blk_row0[b], rb.blk_row1[b], A.ptr, A.idx, A.val, xs, lds,
                [&](int r, const double* s) { epi(r, s[0], acc); });
  __syncthreads();
  block_sum_store<4>(acc, lds, rec + (size_t)b * 4);
}

template <typename T, typename TM>
__global__ __launch_bounds__(kBlock) void k_dual(RowBlocks rb, MatPtrs<TM> A, IterPtrs<T> it,
                                                 DataPtrs<T> d, Inst* __restrict__ inst, int prec,
                                                 double* __restrict__ rec) {
  dual_body<T, TM>(blockIdx.x, rb, A, it, d, inst, prec, rec);
}

// ---------------------------------------------------------------------------
// Band-tile SpMV for single large instances (layout: BandTiles).  The gathers
// of a band-tile stay inside one window of the gathered vector, held in the L2
// of the XCDs that serve the window, and since the entries are sorted by
// gathered index the 64 lanes of a wave instruction read few cache lines.  Each
// wave sums its band in a private LDS array with plain read-modify-writes: the
// host never lets two entries of one 64-entry group share a slot, and LDS
// operations of one wave complete in issue order, so no atomics are needed and
// the result does not depend on scheduling.  The entry stream is software
// pipelined: packed entries and values are loaded two iterations ahead and the
// gathers one iteration ahead of the accumulation.  Output: part[panel * R + r].
// ---------------------------------------------------------------------------
// Instances a check or evaluation pass works on.
// kModeRay: the infeasibility rays of a check, FP64 vectors whatever the
// instance's iterate precision.
enum Mode : int { kModeCheck = 0, kModeEvalStart = 1, kModeEvalFinal = 2, kModeRay = 3 };

__device__ __forceinline__ bool mode_selects(const Inst& I, int mode) {
  if (mode == kModeCheck) return I.status == kActive && I.check_due != 0;
  if (mode == kModeEvalStart) return I.status == kActive;
  if (mode == kModeRay) return I.status == kActive && I.check_due != 0 && I.ray_due != 0;
  return I.status == kDone && I.exit_code != 0;
}

// Precision filter of the check products: the ray pass serves every instance.
__device__ __forceinline__ bool prec_selects(const Inst& I, int mode, int prec) {
  return mode == kModeRay || I.precision == prec;
}

// One wave's band-tile t: part[panel * R + r] = sum over the tile's entries of
// row r of val * x[col], values TV, gathered vector TX, accumulation and output TA.
template <typename TV, typename TX, typename TA>
__device__ __forceinline__ void band_tile_product(const BandTiles& bt, int t, TA* a, const TV* __restrict__ val,
                                                  const TX* __restrict__ x, TA* __restrict__ part, int64_t R) {
  constexpr int U = kBandUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  // the sink slot of the padding is never read and stays uninitialized
  const int used = bt.used[t];
  for (int i = lane; i < used; i += kWave) a[i] = TA(0);
  const TX* xs = x + bt.col0[t];
  const int e0 = bt.start[t];
  const int nit = (bt.start[t + 1] - e0) / (U * kWave);
  const uint32_t* pp = bt.pk + e0 + lane;
  const TV* vp = val + e0 + lane;
  constexpr uint32_t kSlotMask = (1u << kBandSlotBits) - 1u;
  uint32_t pA[U], pB[U], pC[U];
  TV vA[U], vB[U], vC[U];
  TX xA[U], xB[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    pA[u] = pB[u] = pC[u] = 0u;
    vA[u] = vB[u] = vC[u] = TV(0);
    xA[u] = xB[u] = TX(0);
  }
  if (nit > 0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      pA[u] = __builtin_nontemporal_load(pp + u * kWave);
      vA[u] = __builtin_nontemporal_load(vp + u * kWave);
    }
  }
  if (nit > 1) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      pB[u] = __builtin_nontemporal_load(pp + (U + u) * kWave);
      vB[u] = __builtin_nontemporal_load(vp + (U + u) * kWave);
    }
  }
  if (nit > 0) {
#pragma unroll
    for (int u = 0; u < U; ++u) xA[u] = xs[pA[u] >> kBandSlotBits];
  }
  for (int it = 0; it < nit; ++it) {
    if (it + 2 < nit) {
      const int off = (it + 2) * U * kWave;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        pC[u] = __builtin_nontemporal_load(pp + off + u * kWave);
        vC[u] = __builtin_nontemporal_load(vp + off + u * kWave);
      }
    }
    if (it + 1 < nit) {
#pragma unroll
      for (int u = 0; u < U; ++u) xB[u] = xs[pB[u] >> kBandSlotBits];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t sl = pA[u] & kSlotMask;
      a[sl] = a[sl] + (TA)vA[u] * (TA)xA[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      pA[u] = pB[u];
      vA[u] = vB[u];
      xA[u] = xB[u];
      pB[u] = pC[u];
      vB[u] = vC[u];
    }
  }
  // fold the extra slots into their rows (one lane per run, runs own distinct rows)
  for (int r = bt.run_start[t] + lane; r < bt.run_start[t + 1]; r += kWave) {
    const int row = bt.run_row[r];
    TA s = a[row];
    for (int q = bt.run_ext[r]; q < bt.run_ext[r + 1]; ++q) s += a[bt.ext[q]];
    a[row] = s;
  }
  const int nr = bt.nrows[t];
  TA* out = part + (size_t)bt.panel[t] * R + bt.row0[t];
  for (int i = lane; i < nr; i += kWave) out[i] = a[i];
}

// Trial products (K1: G x_hat, K2: G^T y_hat) in the iterate precision T.
template <typename T>
__global__ __launch_bounds__(kBandWaves * kWave) void k_band_spmv(BandTiles bt, const T* __restrict__ val,
                                                                  const T* __restrict__ x, T* __restrict__ part,
                                                                  int64_t R, const Inst* __restrict__ inst,
                                                                  int prec, int need_acc) {
  __shared__ T acc[kBandWaves * kBandSlots];
  const int g = bt.slot[blockIdx.x];
  if (g < 0) return;
  const int w = threadIdx.x / kWave;
  const int t = bt.group[g * kBandWaves + w];
  if (t < 0) return;
  if (inst) {  // solver passes: only instances iterating in this precision (and accepted, for G^T y)
    const Inst& I = inst[bt.tinst[t]];
    if (I.status != kActive || I.precision != prec || (need_acc && I.last_acc == 0)) return;
  }
  band_tile_product<T, T, T>(bt, t, acc + w * kBandSlots, val, x, part, R);
}

// Check / evaluation products with FP64 values of vectors in the iterate
// precision TX (which = 1: the average candidate, skipped where unused).
template <typename TX>
__global__ __launch_bounds__(kBandWaves * kWave) void k_band_cand(BandTiles bt, const double* __restrict__ val,
                                                                  const TX* __restrict__ x,
                                                                  double* __restrict__ part, int64_t R,
                                                                  const Inst* __restrict__ inst, int prec, int mode,
                                                                  int which) {
  __shared__ double acc[kBandWaves * kBandSlots];
  const int g = bt.slot[blockIdx.x];
  if (g < 0) return;
  const int w = threadIdx.x / kWave;
  const int t = bt.group[g * kBandWaves + w];
  if (t < 0) return;
  const Inst& I = inst[bt.tinst[t]];
  if (!mode_selects(I, mode) || !prec_selects(I, mode, prec)) return;
  if (which == 1 && mode == kModeCheck && I.use_avg == 0) return;
  band_tile_product<double, TX, double>(bt, t, acc + w * kBandSlots, val, x, part, R);
}

// Window sums of the check / evaluation products, per instance.
__global__ __launch_bounds__(kBlock) void k_band_combine2(Ranges Rg, int P, int64_t R,
                                                          const double* __restrict__ part0,
                                                          const double* __restrict__ part1,
                                                          double* __restrict__ out0, double* __restrict__ out1,
                                                          const Inst* __restrict__ inst, int mode) {
  const int b = blockIdx.x;
  const Inst& I = inst[Rg.blk_inst[b]];
  if (!mode_selects(I, mode)) return;
  const bool two = part1 != nullptr && (mode != kModeCheck || I.use_avg != 0);
  const int r1 = Rg.blk_end[b];
  for (int r = Rg.blk_start[b] + (int)threadIdx.x; r < r1; r += kBlock) {
    double s0 = 0.0, s1 = 0.0;
    for (int p = 0; p < P; ++p) {
      s0 += part0[(size_t)p * R + r];
      if (two) s1 += part1[(size_t)p * R + r];
    }
    out0[r] = s0;
    if (two) out1[r] = s1;
  }
}

// Sum of the P window partial sums per row (plain product of the band layout).
template <typename T>
__global__ void k_band_sum(const T* __restrict__ part, int P, int64_t R, T* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) s += (double)part[(size_t)p * R + r];
  out[r] = (T)s;
}

// Set-up: band-tile values from the scaled CSR (CSC) values.
__global__ void k_band_vals(const int32_t* __restrict__ src, int64_t n, const double* __restrict__ v64,
                            double* __restrict__ o64, float* __restrict__ o32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int32_t q = src[e];
  const double v = q >= 0 ? v64[q] : 0.0;
  o64[e] = v;
  o32[e] = (float)v;
}

// K1b: combine the P partial sums of G x_hat per row, then the dual step
// (same epilogue and record as k_dual).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dual_epi(Ranges R, const T* __restrict__ part, int P,
                                                     int64_t M, IterPtrs<T> it, DataPtrs<T> d,
                                                     const double* __restrict__ D1, Inst* __restrict__ inst,
                                                     int prec, double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock * 4];
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (I.status != kActive || I.precision != prec) return;
  const DualEpilogue<T> epi = make_dual_epilogue(I, it, d);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int r1 = R.blk_end[b];
  for (int r = R.blk_start[b] + (int)threadIdx.x; r < r1; r += kBlock) {
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += (double)part[(size_t)p * M + r];
    epi(r, s, acc);
  }
  if (R.blk_soc0 && R.blk_soc1[b] > R.blk_soc0[b]) {
    __syncthreads();  // the blocks' unprojected values and committed iterates are in memory
    // task 0: y_hat = Proj onto diag(1/D1) of the block's dual cone of the
    // stored value, with the line-search terms; task 1: the primal residual
    // of the reflection parameter, (G x_hat - h) against diag(D1) of the
    // block's cone (independent: task 1 reads neither y nor y_hat)
    // (the terms go through scalars: acc itself, written from the lambdas,
    // would be kept in scratch memory)
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
    for_cone_tasks<2>(R, b, [&](int r0, int dim, int kind, int pass) {
      const bool dual = pass == 0;
      wave_proj_cone(
          kind, dual, dim,
          [&](int i) { return dual ? (double)it.yh[r0 + i] : (double)it.gxh[r0 + i] - (double)d.h[r0 + i]; },
          [&](int i) { return dual ? 1.0 / D1[r0 + i] : D1[r0 + i]; },
          [&](int i, double p) {
            const int r = r0 + i;
            if (dual) {
              const double yn = (double)(T)p;
              it.yh[r] = (T)yn;
              const double dy = yn - (double)it.y[r];
              t0 += dy * dy;
              t1 += dy * ((double)it.gxh[r] - (double)it.gx[r]);
              t3 += (double)d.h[r] * yn;
            } else {
              const double pr = ((double)it.gxh[r] - (double)d.h[r]) - p;
              t2 += pr * pr;
            }
          });
    });
    acc[0] += t0;
    acc[1] += t1;
    acc[2] += t2;
    acc[3] += t3;
  }
  block_sum_store<4>(acc, lds, rec + (size_t)b * 4);
}

// K2b: combine the P partial sums of G^T y_hat per column, then the dual-slack
// epilogue (same record as k_lam).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lam_epi(Ranges R, const T* __restrict__ part, int P,
                                                    int64_t N, IterPtrs<T> it, DataPtrs<T> d,
                                                    Inst* __restrict__ inst, int prec,
                                                    double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock * 3];
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (I.status != kActive || I.precision != prec || I.last_acc == 0) return;
  double acc[3] = {0.0, 0.0, 0.0};
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += (double)part[(size_t)p * N + j];
    lam_epilogue<T>(j, s, it, d, acc);
  }
  block_sum_store<3>(acc, lds, rec + (size_t)b * 3);
}

// F1: line-search decision of Function 2, one workgroup per instance.
// pf: when non-null, pf[0] = (kbar + 1)^-0.3 and pf[1] = (kbar + 1)^-0.6 for the
// kbar this trial reaches, computed beforehand by an otherwise idle thread
__device__ __forceinline__ void fin_ls_body(int iid, const int32_t* iblk_p, const double* rec_p,
                                            const int32_t* iblk_d, const double* rec_d, Inst* inst,
                                            const double* pf = nullptr) {
  __shared__ double lds[kWavesPerBlock * 4];
  Inst& I = inst[iid];
  if (I.status != kActive) return;
  double p[2], q[4];
  reduce_records<2, 2>(rec_p, iblk_p[iid], iblk_p[iid + 1], lds, p);
  reduce_records<4, 4>(rec_d, iblk_d[iid], iblk_d[iid + 1], lds, q);
  if (threadIdx.x != 0) return;
  I.pending = 0;
  I.check_due = 0;
  I.kbar += 1;
  if (I.precision == kFP64) I.fp64_iters += 1;
  const double dx2 = p[0], dy2 = q[0], dydg = q[1];
  const double omega = I.omega, eta = I.eta;
  const double num = 0.5 * (omega * dx2 + dy2 / omega);
  const double den = fabs(dydg);
  const double etabar = den > 0.0 ? num / den : (double)INFINITY;
  const double kb1 = (double)I.kbar + 1.0;
  const double p3 = pf ? pf[0] : pow(kb1, -0.3), p6 = pf ? pf[1] : pow(kb1, -0.6);
  const double eta_next = fmin((1.0 - p3) * etabar, (1.0 + p6) * eta);
  const bool bad = !isfinite(num) || isnan(etabar) || isnan(q[2]) || isnan(q[3]) || isnan(p[1]) ||
                   !(eta_next > 0.0) || !isfinite(eta_next);
  if (I.trace && I.kbar <= I.trace_cap) {
    double* tr = I.trace + (I.kbar - 1) * kTraceStride;
    tr[0] = (double)I.kbar;
    tr[1] = eta;
    tr[2] = etabar;
    tr[3] = dx2;
    tr[4] = dy2;
    tr[5] = dydg;
    tr[6] = eta < etabar ? 1.0 : 0.0;
    tr[7] = eta_next;
    for (int f = 8; f < kTraceStride; ++f) tr[f] = NAN;
    tr[9] = (double)I.k;
    if (bad) {  // the failing trial's reductions, for diagnosis
      tr[10] = p[1];
      tr[11] = q[3];
      tr[14] = q[2];
    }
  }
  if (bad) {
    I.status = kDone;
    I.exit_code = 8;
    I.last_acc = 0;
    return;
  }
  if (eta < etabar) {
    I.last_acc = 1;
    I.eta_k = eta;
    I.eta_hat = eta_next;
    I.accepted += 1;
    I.dx2 = dx2;
    I.dy2 = dy2;
    I.dydgdx = dydg;
    I.errp2 = q[2];
    I.hy = q[3];
    I.cx = p[1];
  } else {
    I.last_acc = 0;
    if (I.kbar >= I.max_iter) {
      I.status = kDone;
      I.exit_code = 1;
    }
  }
  I.eta = eta_next;
}

__global__ __launch_bounds__(kBlock) void k_fin_ls(const int32_t* __restrict__ iblk_p,
                                                   const double* __restrict__ rec_p,
                                                   const int32_t* __restrict__ iblk_d,
                                                   const double* __restrict__ rec_d,
                                                   Inst* __restrict__ inst) {
  fin_ls_body(blockIdx.x, iblk_p, rec_p, iblk_d, rec_d, inst);
}

// K2: transposed SpMV G^T y_hat over the columns with the dual-slack epilogue.
// Record: ||lam - Proj_Lambda lam||^2, sum l lam+, sum u lam- (finite bounds).
template <typename T, typename TM>
__device__ __forceinline__ void lam_body(int b, const RowBlocks& rb, const MatPtrs<TM>& AT, const IterPtrs<T>& it,
                                         const DataPtrs<T>& d, Inst* inst, int prec, double* rec) {
  __shared__ double lds[kRowBlockCap + kWavesPerBlock * 3];
  const Inst& I = inst[rb.blk_inst[b]];
  if (I.status != kActive || I.precision != prec || I.last_acc == 0) return;
  double acc[3] = {0.0, 0.0, 0.0};
  const T* const ys[1] = {it.yh};
  block_rows<1>(rb.blk_row0[b], rb.blk_row1[b], AT.ptr, AT.idx, AT.val, ys, lds,
                [&](int j, const double* s) { lam_epilogue<T>(j, s[0], it, d, acc); });
  __syncthreads();
  block_sum_store<3>(acc, lds, rec + (size_t)b * 3);
}

template <typename T, typename TM>
__global__ __launch_bounds__(kBlock) void k_lam(RowBlocks rb, MatPtrs<TM> AT, IterPtrs<T> it,
                                                DataPtrs<T> d, Inst* __restrict__ inst, int prec,
                                                double* __restrict__ rec) {
  lam_body<T, TM>(blockIdx.x, rb, AT, it, d, inst, prec, rec);
}

// F2: reflection parameter at z_hat (eq. adaptive_reflection with the relative
// errors of eq. tolerance-2), then schedule the Halpern commit.
__device__ __forceinline__ void fin_beta_body(int iid, const int32_t* iblk_l, const double* rec_l, Inst* inst) {
  __shared__ double lds[kWavesPerBlock * 3];
  Inst& I = inst[iid];
  if (I.status != kActive || I.last_acc == 0) return;
  double q[3];
  reduce_records<3, 3>(rec_l, iblk_l[iid], iblk_l[iid + 1], lds, q);
  if (threadIdx.x != 0) return;
  const double errp = sqrt(I.errp2), errd = sqrt(q[0]);
  const double pobj = I.cx;
  const double dobj = I.hy + q[1] - q[2];
  const double gap = fabs(pobj - dobj);
  const double rp = errp / (1.0 + I.h1);
  const double rd = errd / (1.0 + I.c1);
  const double rg = gap / (1.0 + fabs(pobj) + fabs(dobj));
  const double me = fmax(rp, fmax(rd, rg));
  if (isnan(me) || isnan(rp) || isnan(rd) || isnan(rg)) {
    I.status = kDone;
    I.exit_code = 8;
    return;
  }
  const double beta = me > 0.0 ? clampd(-0.1 * log10(me) + 0.2, 0.0, 1.0) : 1.0;
  if (I.trace && I.kbar <= I.trace_cap) {
    double* tr = I.trace + (I.kbar - 1) * kTraceStride;
    tr[8] = beta;
    tr[10] = I.cx;
    tr[11] = I.hy;
    tr[12] = q[1];
    tr[13] = q[2];
    tr[14] = I.errp2;
    tr[15] = q[0];
  }
  const double k = (double)I.k;
  I.beta = beta;
  I.ca = (k + 1.0) / (k + 2.0);
  I.cb = 1.0 / (k + 2.0);
  I.pending = 1;
  I.sum_eta += I.eta_k;
  I.k += 1;
  I.check_due = (I.kbar % I.check_every) == 0 ? 1 : 0;
  if (!I.check_due && I.kbar >= I.max_iter) {
    I.status = kDone;
    I.exit_code = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_fin_beta(const int32_t* __restrict__ iblk_l,
                                                     const double* __restrict__ rec_l,
                                                     Inst* __restrict__ inst) {
  fin_beta_body(blockIdx.x, iblk_l, rec_l, inst);
}

// A chunk of K trials of one instance per workgroup (small instances, row
// blocks): the passes of k_primal, k_dual, k_fin_ls, k_lam and k_fin_beta in
// order over the instance's blocks, separated by workgroup barriers instead
// of kernel boundaries.  All waves of the workgroup share one CU and its L1,
// so a barrier makes every global write of the previous pass visible.  The
// decisions are read from the instance record after each barrier, the same
// for every thread, so every barrier is reached by the whole workgroup.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_trials_wg(Ranges vcol, RowBlocks brow, RowBlocks bcol, MatPtrs<T> A,
                                                      MatPtrs<T> AT, IterPtrs<T> it, DataPtrs<T> d,
                                                      Inst* __restrict__ inst, int prec, double* rec_p,
                                                      double* rec_d, double* rec_l, int K) {
  const int iid = blockIdx.x;
  const int p0 = vcol.inst_blk0[iid], p1 = vcol.inst_blk0[iid + 1];
  const int d0 = brow.inst_blk0[iid], d1 = brow.inst_blk0[iid + 1];
  const int l0 = bcol.inst_blk0[iid], l1 = bcol.inst_blk0[iid + 1];
  for (int s = 0; s < K; ++s) {
    {
      const Inst& I = inst[iid];
      if (I.status != kActive || I.precision != prec) break;
    }
    for (int b = p0; b < p1; ++b) primal_body<T>(b, vcol, it, d, inst, prec, rec_p);
    __syncthreads();
    for (int b = d0; b < d1; ++b) dual_body<T, T>(b, brow, A, it, d, inst, prec, rec_d);
    __syncthreads();
    fin_ls_body(iid, vcol.inst_blk0, rec_p, brow.inst_blk0, rec_d, inst);
    __syncthreads();
    for (int b = l0; b < l1; ++b) lam_body<T, T>(b, bcol, AT, it, d, inst, prec, rec_l);
    __syncthreads();
    fin_beta_body(iid, bcol.inst_blk0, rec_l, inst);
    __syncthreads();
  }
}

// Row-wise passes of the LDS-resident chunk kernel (instances whose rows and
// columns hold at most kLdsRowMax entries): one thread per row of G (dual
// step) or of G^T (dual slack), the dot product in FP64 in entry order, and one
// record for the whole instance.
// One thread's dot product of entries [q0, q1) with x, in entry order (FP64);
// four entries' indices, values and gathers are requested before they are added.
template <typename T>
__device__ __forceinline__ double row_dot_seq(int q0, int q1, const int32_t* idx, const T* val, const T* x) {
  double s = 0.0;
  int q = q0;
  for (; q + 4 <= q1; q += 4) {
    int c[4];
    double v[4], g[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c[u] = idx[q + u];
      v[u] = (double)val[q + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) g[u] = (double)x[c[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) s += v[u] * g[u];
  }
  for (; q < q1; ++q) s += (double)val[q] * (double)x[idx[q]];
  return s;
}

template <typename T>
__device__ __forceinline__ void dual_rows_lds(int r0, int r1, const MatPtrs<T>& A, const IterPtrs<T>& it,
                                              const DataPtrs<T>& d, const Inst& I, double* rec) {
  __shared__ double lds[kWavesPerBlock * 4];
  if (I.status != kActive) return;
  const DualEpilogue<T> epi = make_dual_epilogue(I, it, d);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
    const double s = row_dot_seq(A.ptr[r], A.ptr[r + 1], A.idx, A.val, it.xh);
    epi(r, s, acc);
  }
  block_sum_store<4>(acc, lds, rec);
}

template <typename T>
__device__ __forceinline__ void lam_rows_lds(int c0, int c1, const MatPtrs<T>& AT, const IterPtrs<T>& it,
                                             const DataPtrs<T>& d, const Inst& I, double* rec) {
  __shared__ double lds[kWavesPerBlock * 3];
  if (I.status != kActive || I.last_acc == 0) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int j = c0 + (int)threadIdx.x; j < c1; j += kBlock) {
    const double s = row_dot_seq(AT.ptr[j], AT.ptr[j + 1], AT.idx, AT.val, it.yh);
    lam_epilogue<T>(j, s, it, d, acc);
  }
  block_sum_store<3>(acc, lds, rec);
}

template <typename T>
__device__ __forceinline__ void lds_copy(T* __restrict__ dst, const T* __restrict__ src, int64_t n) {
  for (int64_t i = threadIdx.x; i < n; i += kBlock) dst[i] = src[i];
}

// k_trials_wg with the instance resident in LDS: the kernel copies its
// iterates, data, matrix rows and columns, schedule tables and Inst record
// into LDS, runs the chunk's K trials there (pointers into LDS, offset so that
// the device functions keep using global indices), then writes back what the
// trials change.  Every dependent step of a trial is then an LDS access
// instead of an HBM round trip.  The host launches it only when the largest
// instance fits (dynamic LDS of lds_layout(...).total bytes).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_trials_lds(Ranges vcol, RowBlocks brow, RowBlocks bcol, MatPtrs<T> A,
                                                       MatPtrs<T> AT, IterPtrs<T> it, DataPtrs<T> d,
                                                       Inst* __restrict__ inst, int prec, int K, int rowwise) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  __shared__ Inst Ish;
  __shared__ int32_t iblk[6];
  const int iid = blockIdx.x;
  {
    const uint64_t* s = reinterpret_cast<const uint64_t*>(&inst[iid]);
    uint64_t* t = reinterpret_cast<uint64_t*>(&Ish);
    for (int i = threadIdx.x; i < (int)(sizeof(Inst) / 8); i += kBlock) t[i] = s[i];
    if (threadIdx.x == 0) {
      iblk[0] = vcol.inst_blk0[iid];
      iblk[1] = vcol.inst_blk0[iid + 1];
      iblk[2] = brow.inst_blk0[iid];
      iblk[3] = brow.inst_blk0[iid + 1];
      iblk[4] = bcol.inst_blk0[iid];
      iblk[5] = bcol.inst_blk0[iid + 1];
    }
  }
  __syncthreads();
  if (Ish.status != kActive || Ish.precision != prec || K < 1) return;
  const int r0 = Ish.row0, m = Ish.rows, c0 = Ish.col0, n = Ish.cols;
  const int p0 = iblk[0], np = iblk[1] - p0, d0 = iblk[2], nd = iblk[3] - d0, l0 = iblk[4], nl = iblk[5] - l0;
  const int q0 = A.ptr[r0], nnz = A.ptr[r0 + m] - q0;
  const int t0 = AT.ptr[c0];
  const LdsLayout L = lds_layout(m, n, nnz, np, nd, nl, sizeof(T));
  T* vec = reinterpret_cast<T*>(dyn + L.vec);
  T* dat = reinterpret_cast<T*>(dyn + L.dat);
  // iterates (x-like: n values each, then y-like: m values each)
  T* const xs[7] = {it.x, it.xa, it.xh, it.gty, it.gtya, it.gtyh, it.sx};
  T* const ys[7] = {it.y, it.ya, it.yh, it.gx, it.gxa, it.gxh, it.sy};
  for (int v = 0; v < 7; ++v) lds_copy(vec + (size_t)v * n, xs[v] + c0, n);
  for (int v = 0; v < 7; ++v) lds_copy(vec + (size_t)7 * n + (size_t)v * m, ys[v] + r0, m);
  lds_copy(dat, d.c + c0, n);
  lds_copy(dat + n, d.l + c0, n);
  lds_copy(dat + 2 * n, d.u + c0, n);
  lds_copy(dat + 3 * n, d.h + r0, m);
  int32_t* rp = reinterpret_cast<int32_t*>(dyn + L.rp);
  int32_t* ci = reinterpret_cast<int32_t*>(dyn + L.ci);
  T* va = reinterpret_cast<T*>(dyn + L.va);
  int32_t* cp = reinterpret_cast<int32_t*>(dyn + L.cp);
  int32_t* ri = reinterpret_cast<int32_t*>(dyn + L.ri);
  T* vt = reinterpret_cast<T*>(dyn + L.vt);
  lds_copy(rp, A.ptr + r0, m + 1);
  lds_copy(ci, A.idx + q0, nnz);
  lds_copy(va, A.val + q0, nnz);
  lds_copy(cp, AT.ptr + c0, n + 1);
  lds_copy(ri, AT.idx + t0, nnz);
  lds_copy(vt, AT.val + t0, nnz);
  double* recp = reinterpret_cast<double*>(dyn + L.rec);
  double* recd = recp + 2 * max(np, 1);
  double* recl = recd + 4 * max(nd, 1);
  int32_t* bt = reinterpret_cast<int32_t*>(dyn + L.blk);
  lds_copy(bt, vcol.blk_start + p0, np);
  lds_copy(bt + np, vcol.blk_end + p0, np);
  lds_copy(bt + 2 * np, vcol.blk_inst + p0, np);
  int32_t* bd = bt + 3 * np;
  lds_copy(bd, brow.blk_row0 + d0, nd);
  lds_copy(bd + nd, brow.blk_row1 + d0, nd);
  lds_copy(bd + 2 * nd, brow.blk_inst + d0, nd);
  int32_t* bl = bd + 3 * nd;
  lds_copy(bl, bcol.blk_row0 + l0, nl);
  lds_copy(bl + nl, bcol.blk_row1 + l0, nl);
  lds_copy(bl + 2 * nl, bcol.blk_inst + l0, nl);
  __syncthreads();
  // the same structures over LDS, indexed with global row, column, entry,
  // block and instance numbers
  IterPtrs<T> li = it;
  T* const lx[7] = {vec, vec + n, vec + 2 * n, vec + 3 * n, vec + 4 * n, vec + 5 * n, vec + 6 * n};
  T* const ly0 = vec + (size_t)7 * n;
  li.x = lx[0] - c0;
  li.xa = lx[1] - c0;
  li.xh = lx[2] - c0;
  li.gty = lx[3] - c0;
  li.gtya = lx[4] - c0;
  li.gtyh = lx[5] - c0;
  li.sx = lx[6] - c0;
  li.y = ly0 - r0;
  li.ya = ly0 + m - r0;
  li.yh = ly0 + 2 * m - r0;
  li.gx = ly0 + 3 * m - r0;
  li.gxa = ly0 + 4 * m - r0;
  li.gxh = ly0 + 5 * m - r0;
  li.sy = ly0 + 6 * m - r0;
  const DataPtrs<T> ld{dat - c0, dat + n - c0, dat + 2 * n - c0, dat + 3 * n - r0};
  const MatPtrs<T> LA{rp - r0, ci - q0, va - q0};
  const MatPtrs<T> LAT{cp - c0, ri - t0, vt - t0};
  Ranges lv = vcol;
  lv.blk_start = bt - p0;
  lv.blk_end = bt + np - p0;
  lv.blk_inst = bt + 2 * np - p0;
  lv.inst_blk0 = iblk - iid;
  RowBlocks lr = brow;
  lr.blk_row0 = bd - d0;
  lr.blk_row1 = bd + nd - d0;
  lr.blk_inst = bd + 2 * nd - d0;
  lr.inst_blk0 = iblk + 2 - iid;
  RowBlocks lc = bcol;
  lc.blk_row0 = bl - l0;
  lc.blk_row1 = bl + nl - l0;
  lc.blk_inst = bl + 2 * nl - l0;
  lc.inst_blk0 = iblk + 4 - iid;
  Inst* li_inst = &Ish - iid;
  double* rp_ = recp - 2 * (size_t)p0;
  double* rd_ = recd - 4 * (size_t)d0;
  double* rl_ = recl - 3 * (size_t)l0;
  // Row-wise instances take one range for the primal pass and the row-wise
  // passes, each leaving one record (one[] is the per-instance block table of
  // a single record); the others keep their blocks.
  __shared__ int32_t one[2], rng[3];
  __shared__ double pf[2];
  if (threadIdx.x == 0) {
    one[0] = 0;
    one[1] = 1;
    rng[0] = c0;
    rng[1] = c0 + n;
    rng[2] = iid;
  }
  if (threadIdx.x == kWave) {  // line-search factors of the first trial
    const double kb = (double)Ish.kbar + 2.0;
    pf[0] = pow(kb, -0.3);
    pf[1] = pow(kb, -0.6);
  }
  __syncthreads();
  Ranges l1 = vcol;
  l1.blk_start = rng;
  l1.blk_end = rng + 1;
  l1.blk_inst = rng + 2;
  for (int s = 0; s < K; ++s) {
    if (Ish.status != kActive || Ish.precision != prec) break;
    if (rowwise) {
      primal_body<T>(0, l1, li, ld, li_inst, prec, recp);
      __syncthreads();
      dual_rows_lds<T>(r0, r0 + m, LA, li, ld, Ish, recd);
      __syncthreads();
      fin_ls_body(iid, one - iid, recp, one - iid, recd, li_inst, pf);
      __syncthreads();
      lam_rows_lds<T>(c0, c0 + n, LAT, li, ld, Ish, recl);
      __syncthreads();
      fin_beta_body(iid, one - iid, recl, li_inst);
    } else {
      for (int b = p0; b < p0 + np; ++b) primal_body<T>(b, lv, li, ld, li_inst, prec, rp_);
      __syncthreads();
      for (int b = d0; b < d0 + nd; ++b) dual_body<T, T>(b, lr, LA, li, ld, li_inst, prec, rd_);
      __syncthreads();
      fin_ls_body(iid, lv.inst_blk0, rp_, lr.inst_blk0, rd_, li_inst, pf);
      __syncthreads();
      for (int b = l0; b < l0 + nl; ++b) lam_body<T, T>(b, lc, LAT, li, ld, li_inst, prec, rl_);
      __syncthreads();
      fin_beta_body(iid, lc.inst_blk0, rl_, li_inst);
    }
    // every thread has passed the finalizer's reductions; thread 0 may still be
    // in its scalar part (which does not touch kbar), while wave 1 forms the
    // next trial's line-search factors
    if (threadIdx.x == kWave) {
      const double kb = (double)Ish.kbar + 2.0;
      pf[0] = pow(kb, -0.3);
      pf[1] = pow(kb, -0.6);
    }
    __syncthreads();
  }
  // write back what trials change: x, x_hat, G^T y, G^T y_hat, S_x and the row
  // counterparts (anchors and data are read-only here), then the record
  const int wx[5] = {0, 2, 3, 5, 6};
  for (int v = 0; v < 5; ++v) {
    const T* src = vec + (size_t)wx[v] * n;
    T* dst = xs[wx[v]] + c0;
    for (int i = threadIdx.x; i < n; i += kBlock) dst[i] = src[i];
    const T* sy_ = ly0 + (size_t)wx[v] * m;
    T* dy_ = ys[wx[v]] + r0;
    for (int i = threadIdx.x; i < m; i += kBlock) dy_[i] = sy_[i];
  }
  {
    const uint64_t* s = reinterpret_cast<const uint64_t*>(&Ish);
    uint64_t* t = reinterpret_cast<uint64_t*>(&inst[iid]);
    for (int i = threadIdx.x; i < (int)(sizeof(Inst) / 8); i += kBlock) t[i] = s[i];
  }
}

// ===========================================================================
// Restart / termination check
// ===========================================================================

// Apply the pending Halpern commit, then form the average candidate S / sum(eta).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_commit_avg(Ranges R, T* __restrict__ z,
                                                       T* __restrict__ zh, const T* __restrict__ za,
                                                       T* __restrict__ g, const T* __restrict__ gh,
                                                       const T* __restrict__ ga, T* __restrict__ s,
                                                       T* __restrict__ zbar, Inst* __restrict__ inst,
                                                       int prec) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (I.status != kActive || I.check_due == 0 || I.precision != prec) return;
  const bool commit = I.pending != 0;
  const bool avg = I.use_avg != 0;
  const double ca = I.ca, cb = I.cb, beta = I.beta, etak = I.eta_k;
  const double inv_sum = 1.0 / I.sum_eta;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double zhv = (double)zh[j];
    double sv = avg ? (double)s[j] : 0.0;
    if (commit) {
      z[j] = (T)(ca * ((1.0 + beta) * zhv - beta * (double)z[j]) + cb * (double)za[j]);
      g[j] = (T)(ca * ((1.0 + beta) * (double)gh[j] - beta * (double)g[j]) + cb * (double)ga[j]);
      if (avg) {
        sv = (double)(T)(sv + etak * zhv);
        s[j] = (T)sv;
      }
    }
    if (avg) zbar[j] = (T)(sv * inv_sum);
  }
}

// Two products with one matrix pass: out0 = A in0, out1 = A in1 (FP64 values,
// FP64 output).  in1 may be null.  Selected instances only.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_spmv2(RowBlocks rb, MatPtrs<double> A, const T* __restrict__ in0,
                                                  const T* __restrict__ in1, double* __restrict__ out0,
                                                  double* __restrict__ out1, const Inst* __restrict__ inst,
                                                  int prec, int mode) {
  __shared__ double lds[2 * kRowBlockCap + kWavesPerBlock * 2];
  const int b = blockIdx.x;
  const Inst& I = inst[rb.blk_inst[b]];
  if (!mode_selects(I, mode) || !prec_selects(I, mode, prec)) return;
  const bool two = (in1 != nullptr) && (mode != kModeCheck || I.use_avg != 0);
  if (two) {
    const T* const xs[2] = {in0, in1};
    block_rows<2>(rb.blk_row0[b], rb.blk_row1[b], A.ptr, A.idx, A.val, xs, lds, [&](int r, const double* s) {
      out0[r] = s[0];
      out1[r] = s[1];
    });
  } else {
    const T* const xs[1] = {in0};
    block_rows<1>(rb.blk_row0[b], rb.blk_row1[b], A.ptr, A.idx, A.val, xs, lds,
                  [&](int r, const double* s) { out0[r] = s[0]; });
  }
}

// Candidate reductions over the columns.  Per candidate c (0: PDHG output or
// evaluated point, 1: average): sums ||x_c - x_a||^2, ||b1||^2, ||lam - Proj lam||^2,
// sum l lam+, sum u lam-, c^T x_c; maxima of the unscaled dual residual and |G^T y|.
// Record layout: [c0 sums(6), c1 sums(6), c0 max(2), c1 max(2)].
constexpr int kCandColsNV = 16, kCandColsNS = 12;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cand_cols(Ranges R, const T* __restrict__ x0,
                                                      const T* __restrict__ x1, const T* __restrict__ xa,
                                                      const double* __restrict__ g0,
                                                      const double* __restrict__ g1,
                                                      DataPtrs<double> d, const double* __restrict__ D2,
                                                      const Inst* __restrict__ inst, int prec, int mode,
                                                      double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock * kCandColsNV];
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (!mode_selects(I, mode) || I.precision != prec) return;
  const int nc = (mode == kModeCheck && I.use_avg) ? 2 : 1;
  double acc[kCandColsNV];
#pragma unroll
  for (int i = 0; i < kCandColsNV; ++i) acc[i] = 0.0;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double c = d.c[j], lo = d.l[j], hi = d.u[j], dj = D2[j];
    const bool lf = isfinite(lo), uf = isfinite(hi);
    const double xav = (double)xa[j];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= nc) break;
      const double xc = (double)(q == 0 ? x0[j] : x1[j]);
      const double gty = q == 0 ? g0[j] : g1[j];
      const double dxa = xc - xav;
      const double lam = c - gty;
      double res;
      if (!lf && !uf) res = lam;
      else if (!lf) res = fmax(lam, 0.0);
      else if (!uf) res = fmin(lam, 0.0);
      else res = 0.0;
      acc[q * 6 + 0] += dxa * dxa;
      acc[q * 6 + 1] += lam * lam;
      acc[q * 6 + 2] += res * res;
      if (lf) acc[q * 6 + 3] += lo * fmax(lam, 0.0);
      if (uf) acc[q * 6 + 4] += hi * fmax(-lam, 0.0);
      acc[q * 6 + 5] += c * xc;
      acc[12 + q * 2 + 0] = fmax(acc[12 + q * 2 + 0], fabs(res) / dj);
      acc[12 + q * 2 + 1] = fmax(acc[12 + q * 2 + 1], fabs(gty) / dj);
    }
  }
  block_summax_store<kCandColsNV, kCandColsNS>(acc, lds, rec + (size_t)b * kCandColsNV);
}

// Candidate reductions over the rows: sums ||y_c - y_a||^2, ||b2||^2,
// ||(Gx-h) - Proj_Kd*||^2, h^T y_c; maxima of the unscaled primal residual,
// |G x| and |Proj_Kd*(G x - h)|.  Layout: [c0 sums(4), c1 sums(4), c0 max(3), c1 max(3)].
constexpr int kCandRowsNV = 14, kCandRowsNS = 8;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cand_rows(Ranges R, const T* __restrict__ y0,
                                                      const T* __restrict__ y1, const T* __restrict__ ya,
                                                      const double* __restrict__ g0,
                                                      const double* __restrict__ g1,
                                                      DataPtrs<double> d, const double* __restrict__ D1,
                                                      const Inst* __restrict__ inst, int prec, int mode,
                                                      double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock * kCandRowsNV];
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (!mode_selects(I, mode) || I.precision != prec) return;
  const int nc = (mode == kModeCheck && I.use_avg) ? 2 : 1;
  const int mz_end = I.row0 + I.m_zero;
  double acc[kCandRowsNV];
#pragma unroll
  for (int i = 0; i < kCandRowsNV; ++i) acc[i] = 0.0;
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) {
    if (i >= I.soc_start) continue;  // cone block rows: below
    const double h = d.h[i], di = D1[i];
    const double yav = (double)ya[i];
    const bool zero_row = i < mz_end;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= nc) break;
      const double yc = (double)(q == 0 ? y0[i] : y1[i]);
      const double gx = q == 0 ? g0[i] : g1[i];
      const double dya = yc - yav;
      const double res = gx - h;
      const double pr = zero_row ? res : fmin(res, 0.0);
      const double proj = zero_row ? 0.0 : fmax(res, 0.0);
      acc[q * 4 + 0] += dya * dya;
      acc[q * 4 + 1] += res * res;
      acc[q * 4 + 2] += pr * pr;
      acc[q * 4 + 3] += h * yc;
      acc[8 + q * 3 + 0] = fmax(acc[8 + q * 3 + 0], fabs(pr) / di);
      acc[8 + q * 3 + 1] = fmax(acc[8 + q * 3 + 1], fabs(gx) / di);
      acc[8 + q * 3 + 2] = fmax(acc[8 + q * 3 + 2], proj / di);
    }
  }
  // cone blocks: the same terms, with the residual r = G x - h projected onto
  // diag(D1) of the block's cone for the scaled L2 term and, unscaled (r / D1),
  // onto the cone itself for the infinity-norm termination terms
  // (one task per block, candidate q and scaled / unscaled projection, spread
  // over the waves, with one inlined projection; the terms go through scalars
  // to acc)
  // per candidate: sums c[q][0..3] for acc[q*4 + i], maxima c[q][4..6] for acc[8 + q*3 + i - 4]
  double c00 = 0.0, c01 = 0.0, c02 = 0.0, c03 = 0.0, c04 = 0.0, c05 = 0.0, c06 = 0.0;
  double c10 = 0.0, c11 = 0.0, c12 = 0.0, c13 = 0.0, c14 = 0.0, c15 = 0.0, c16 = 0.0;
  for_cone_tasks<2 * kMaxCand>(R, b, [&](int r0, int dim, int kind, int task) {
    const int q = task >> 1, pass = task & 1;
    if (q < nc) {
      const T* yq = q == 0 ? y0 : y1;
      const double* gq = q == 0 ? g0 : g1;
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0, t5 = 0.0, t6 = 0.0;
      if (pass == 0) {
        for (int i = (int)(threadIdx.x & (kWave - 1)); i < dim; i += kWave) {
          const int r = r0 + i;
          const double yc = (double)yq[r], gx = gq[r], h = d.h[r];
          const double dya = yc - (double)ya[r], res = gx - h;
          t0 += dya * dya;
          t1 += res * res;
          t3 += h * yc;
          t5 = fmax(t5, fabs(gx) / D1[r]);
        }
      }
      const bool scaled = pass == 0;
      wave_proj_cone(
          kind, false, dim,
          [&](int i) { return scaled ? gq[r0 + i] - d.h[r0 + i] : (gq[r0 + i] - d.h[r0 + i]) / D1[r0 + i]; },
          [&](int i) { return scaled ? D1[r0 + i] : 1.0; },
          [&](int i, double p) {
            if (scaled) {
              const double pr = (gq[r0 + i] - d.h[r0 + i]) - p;
              t2 += pr * pr;
            } else {
              const double ru = (gq[r0 + i] - d.h[r0 + i]) / D1[r0 + i];
              t4 = fmax(t4, fabs(ru - p));
              t6 = fmax(t6, fabs(p));
            }
          });
      if (q == 0) {
        c00 += t0, c01 += t1, c02 += t2, c03 += t3;
        c04 = fmax(c04, t4), c05 = fmax(c05, t5), c06 = fmax(c06, t6);
      } else {
        c10 += t0, c11 += t1, c12 += t2, c13 += t3;
        c14 = fmax(c14, t4), c15 = fmax(c15, t5), c16 = fmax(c16, t6);
      }
    }
  });
  acc[0] += c00, acc[1] += c01, acc[2] += c02, acc[3] += c03;
  acc[4] += c10, acc[5] += c11, acc[6] += c12, acc[7] += c13;
  acc[8] = fmax(acc[8], c04), acc[9] = fmax(acc[9], c05), acc[10] = fmax(acc[10], c06);
  acc[11] = fmax(acc[11], c14), acc[12] = fmax(acc[12], c15), acc[13] = fmax(acc[13], c16);
  block_summax_store<kCandRowsNV, kCandRowsNS>(acc, lds, rec + (size_t)b * kCandRowsNV);
}

// Combine the candidate reductions: radii, KKT errors, termination errors,
// and the start of the bisection (t0 = r / sqrt(tau|b1|^2 + sigma|b2|^2)).
__global__ __launch_bounds__(kBlock) void k_cand_fin(Ranges rc, const double* __restrict__ rec_c,
                                                     Ranges rr, const double* __restrict__ rec_r,
                                                     Inst* __restrict__ inst, int mode) {
  __shared__ double lds[kWavesPerBlock * kCandColsNV];
  const int iid = blockIdx.x;
  Inst& I = inst[iid];
  if (!mode_selects(I, mode)) return;
  double cs[kCandColsNV], rs[kCandRowsNV];
  reduce_records<kCandColsNV, kCandColsNS>(rec_c, rc.inst_blk0[iid], rc.inst_blk0[iid + 1], lds, cs);
  reduce_records<kCandRowsNV, kCandRowsNS>(rec_r, rr.inst_blk0[iid], rr.inst_blk0[iid + 1], lds, rs);
  if (threadIdx.x != 0) return;
  const int nc = (mode == kModeCheck && I.use_avg) ? 2 : 1;
  const double omega = I.omega;
  const double tau = I.eta_hat / omega, sigma = I.eta_hat * omega;
  for (int q = 0; q < nc; ++q) {
    CandState& C = I.cand[q];
    C.dxa2 = cs[q * 6 + 0];
    C.dya2 = rs[q * 4 + 0];
    const double b1sq = cs[q * 6 + 1], b2sq = rs[q * 4 + 1];
    C.errd = sqrt(cs[q * 6 + 2]);
    C.errp = sqrt(rs[q * 4 + 2]);
    C.pobj = cs[q * 6 + 5];
    C.dobj = rs[q * 4 + 3] + cs[q * 6 + 3] - cs[q * 6 + 4];
    C.gap = fabs(C.pobj - C.dobj);
    C.kkt = sqrt(omega * omega * C.errp * C.errp + C.errd * C.errd / (omega * omega) + C.gap * C.gap);
    C.abs_p = rs[8 + q * 3 + 0];
    C.abs_d = cs[12 + q * 2 + 0];
    C.abs_gap = C.gap;
    C.rel_p = C.abs_p / (1.0 + fmax(I.h_inf, fmax(rs[8 + q * 3 + 1], rs[8 + q * 3 + 2])));
    C.rel_d = C.abs_d / (1.0 + fmax(I.c_inf, cs[12 + q * 2 + 1]));
    C.rel_gap = C.gap / (1.0 + fmax(fabs(C.pobj), fabs(C.dobj)));
    C.r = sqrt(C.dxa2 / tau + C.dya2 / sigma);
    C.scale = sqrt(tau * b1sq + sigma * b2sq);
    C.rho = NAN;
    C.val_lo = 0.0;
    C.t_lo = 0.0;
    C.t_hi = 0.0;
    C.doublings = 0;
    C.bracketed = 0;
    C.last_dist = -1.0;
    if (mode != kModeCheck || I.force_kkt) {
      C.phase = kPhaseOff;  // KKT_omega is the restart metric: no bisection
    } else if (!(C.r > 0.0) || !isfinite(C.r)) {
      C.phase = kPhaseDone;  // invalid radius: numerical issue
    } else if (C.scale == 0.0) {
      C.phase = kPhaseDone;
      C.rho = 0.0;
    } else {
      C.phase = kPhaseExp;
      C.t_base = C.r / C.scale;
    }
  }
  if (nc < 2) I.cand[1].phase = kPhaseOff;
  if (mode == kModeCheck) I.pending = 0;
}

__device__ __forceinline__ double probe_t(const CandState& C, int p) {
  if (C.phase == kPhaseExp) return C.t_base * (double)(1u << p);
  return C.t_lo + (C.t_hi - C.t_lo) * (double)(p + 1) / (double)(kProbes + 1);
}

// One multisection pass: for the candidate blockIdx.y (if still searching) and
// every probe t, sum ||x(t) - x||^2 / tau and b1^T (x(t) - x) over the columns
// (eq. compute_zt_2).  Records: [candidate][workgroup][probe][2].
constexpr int kProbeNV = kProbes * 2;
template <typename T>
__device__ __forceinline__ void probe_cols_body(int b, int q, const Ranges& R, const T* x0, const T* x1,
                                                const double* g0, const double* g1, const DataPtrs<double>& d,
                                                const Inst* inst, int prec, double* rec) {
  __shared__ double lds[kWavesPerBlock * kProbeNV];
  const Inst& I = inst[R.blk_inst[b]];
  if (I.status != kActive || I.check_due == 0 || I.precision != prec) return;
  const CandState& C = I.cand[q];
  if (C.phase != kPhaseExp && C.phase != kPhaseBisect) return;
  const double tau = I.eta_hat / I.omega;
  double tq[kProbes];
#pragma unroll
  for (int p = 0; p < kProbes; ++p) tq[p] = probe_t(C, p) * tau;
  double acc[kProbeNV];
#pragma unroll
  for (int i = 0; i < kProbeNV; ++i) acc[i] = 0.0;
  const double inv_tau = 1.0 / tau;
  const T* xs = q == 0 ? x0 : x1;
  const double* gs = q == 0 ? g0 : g1;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double lo = d.l[j], hi = d.u[j];
    const double xc = (double)xs[j];
    const double b1 = gs[j] - d.c[j];
#pragma unroll
    for (int p = 0; p < kProbes; ++p) {
      const double dx = clampd(xc + tq[p] * b1, lo, hi) - xc;
      acc[p * 2 + 0] += dx * dx * inv_tau;
      acc[p * 2 + 1] += b1 * dx;
    }
  }
  block_sum_store<kProbeNV>(acc, lds, rec + ((size_t)q * R.nblk + b) * kProbeNV);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_probe_cols(Ranges R, const T* __restrict__ x0,
                                                       const T* __restrict__ x1,
                                                       const double* __restrict__ g0,
                                                       const double* __restrict__ g1,
                                                       DataPtrs<double> d, const Inst* __restrict__ inst,
                                                       int prec, double* __restrict__ rec) {
  probe_cols_body<T>(blockIdx.x, blockIdx.y, R, x0, x1, g0, g1, d, inst, prec, rec);
}

template <typename T>
__device__ __forceinline__ void probe_rows_body(int b, int q, const Ranges& R, const T* y0, const T* y1,
                                                const double* g0, const double* g1, const DataPtrs<double>& d,
                                                const double* D1, const Inst* inst, int prec, double* rec) {
  __shared__ double lds[kWavesPerBlock * kProbeNV];
  const Inst& I = inst[R.blk_inst[b]];
  if (I.status != kActive || I.check_due == 0 || I.precision != prec) return;
  const CandState& C = I.cand[q];
  if (C.phase != kPhaseExp && C.phase != kPhaseBisect) return;
  const double sigma = I.eta_hat * I.omega;
  const int mz_end = I.row0 + I.m_zero;
  const double inv_sigma = 1.0 / sigma;
  const T* ys = q == 0 ? y0 : y1;
  const double* gs = q == 0 ? g0 : g1;
  // cone blocks first: y(t) = Proj onto diag(1/D1) (dual cone) of
  // y + t sigma b2, one task per block and probe spread over the waves (one
  // inlined projection); each wave's sums go to its own LDS slots.  (Done
  // before the element loop below, whose 48 per-probe values are then not
  // live across the projection: the kernel keeps more waves per SIMD.)
  __shared__ double cone_acc[kWavesPerBlock][kProbeNV];
  const bool cones = R.blk_soc0 && R.blk_soc1[b] > R.blk_soc0[b];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  if (cones) {
    for (int i = lane; i < kProbeNV; i += kWave) cone_acc[wave][i] = 0.0;
    for_cone_tasks<kProbes>(R, b, [&](int r0, int dim, int kind, int p) {
      const double tp = probe_t(C, p) * sigma;
      double dd = 0.0, bd = 0.0;
      wave_proj_cone(
          kind, true, dim, [&](int i) { return (double)ys[r0 + i] + tp * (d.h[r0 + i] - gs[r0 + i]); },
          [&](int i) { return 1.0 / D1[r0 + i]; },
          [&](int i, double pv) {
            const double yc = (double)ys[r0 + i];
            const double dy = pv - yc;
            dd += dy * dy;
            bd += (d.h[r0 + i] - gs[r0 + i]) * dy;
          });
      dd = wave_sum(dd);
      bd = wave_sum(bd);
      if (lane == 0) {
        cone_acc[wave][p * 2 + 0] += dd * inv_sigma;
        cone_acc[wave][p * 2 + 1] += bd;
      }
    });
  }
  double tq[kProbes];
#pragma unroll
  for (int p = 0; p < kProbes; ++p) tq[p] = probe_t(C, p) * sigma;
  double acc[kProbeNV];
#pragma unroll
  for (int i = 0; i < kProbeNV; ++i) acc[i] = 0.0;
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) {
    if (i >= I.soc_start) continue;  // cone block rows: above
    const bool zero_row = i < mz_end;
    const double yc = (double)ys[i];
    const double b2 = d.h[i] - gs[i];
#pragma unroll
    for (int p = 0; p < kProbes; ++p) {
      const double v = yc + tq[p] * b2;
      const double dy = (zero_row ? v : fmax(v, 0.0)) - yc;
      acc[p * 2 + 0] += dy * dy * inv_sigma;
      acc[p * 2 + 1] += b2 * dy;
    }
  }
  if (cones && lane == 0) {  // the wave's cone sums join acc in its lane 0
#pragma unroll
    for (int i = 0; i < kProbeNV; ++i) acc[i] += cone_acc[wave][i];
  }
  block_sum_store<kProbeNV>(acc, lds, rec + ((size_t)q * R.nblk + b) * kProbeNV);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_probe_rows(Ranges R, const T* __restrict__ y0,
                                                       const T* __restrict__ y1,
                                                       const double* __restrict__ g0,
                                                       const double* __restrict__ g1,
                                                       DataPtrs<double> d, const double* __restrict__ D1,
                                                       const Inst* __restrict__ inst, int prec,
                                                       double* __restrict__ rec) {
  probe_rows_body<T>(blockIdx.x, blockIdx.y, R, y0, y1, g0, g1, d, D1, inst, prec, rec);
}

// Update every candidate's bracket from one multisection pass (Algorithm 3:
// exponential search from t0, then bisection; here kProbes points per pass).
__device__ __forceinline__ void probe_fin_body(int iid, const Ranges& rc, const double* rec_c, const Ranges& rr,
                                               const double* rec_r, Inst* inst) {
  __shared__ double red[kBlock];
  // the bracket update below indexes probes at run time: its inputs live in
  // LDS (registers indexed at run time would go to scratch memory)
  __shared__ double s_dist[kMaxCand][kProbes], s_val[kMaxCand][kProbes], s_t[kMaxCand][kProbes];
  __shared__ double s_cols[kProbeNV], s_rows[kProbeNV];
  Inst& I = inst[iid];
  if (I.status != kActive || I.check_due == 0) return;
  const bool s0 = I.cand[0].phase == kPhaseExp || I.cand[0].phase == kPhaseBisect;
  const bool s1 = I.cand[1].phase == kPhaseExp || I.cand[1].phase == kPhaseBisect;
  if (!s0 && !s1) return;
#pragma unroll
  for (int q = 0; q < kMaxCand; ++q) {
    const bool sq = q == 0 ? s0 : s1;
    if (!sq) continue;  // uniform across the workgroup
    reduce_records_wide<kProbeNV>(rec_c + (size_t)q * rc.nblk * kProbeNV, rc.inst_blk0[iid], rc.inst_blk0[iid + 1],
                                  red, s_cols);
    reduce_records_wide<kProbeNV>(rec_r + (size_t)q * rr.nblk * kProbeNV, rr.inst_blk0[iid], rr.inst_blk0[iid + 1],
                                  red, s_rows);
    if (threadIdx.x == 0) {
      const CandState& C = I.cand[q];
      for (int p = 0; p < kProbes; ++p) {
        s_dist[q][p] = sqrt(s_cols[p * 2] + s_rows[p * 2]);
        s_val[q][p] = s_cols[p * 2 + 1] + s_rows[p * 2 + 1];
        s_t[q][p] = probe_t(C, p);
      }
    }
  }
  if (threadIdx.x != 0) return;
  const double eps = I.bisect_eps;
  for (int q = 0; q < kMaxCand; ++q) {
    CandState& C = I.cand[q];
    if (C.phase != kPhaseExp && C.phase != kPhaseBisect) continue;
    const double* dist = s_dist[q];
    const double* val = s_val[q];
    const double* tp = s_t[q];
    if (C.phase == kPhaseExp) {
      bool decided = false;
      for (int p = 0; p < kProbes; ++p) {
        const bool first = (C.doublings == 0 && p == 0);
        if (dist[p] > C.r) {
          if (first) {
            C.t_lo = 0.0;
            C.val_lo = 0.0;
          } else {
            C.t_lo = p > 0 ? tp[p - 1] : C.t_base * 0.5;
            // val_lo was recorded with the previous probe
          }
          C.t_hi = tp[p];
          C.phase = kPhaseBisect;
          decided = true;
          break;
        }
        if (!first && dist[p] <= C.last_dist) {  // saturated: z(2t) = z(t)
          C.phase = kPhaseDone;
          decided = true;
          break;
        }
        C.last_dist = dist[p];
        C.val_lo = val[p];
        C.t_lo = tp[p];
        C.doublings += 1;
      }
      if (!decided) {
        C.t_base = tp[kProbes - 1] * 2.0;
        if (C.doublings >= 64) C.phase = kPhaseDone;
      }
    } else {
      int last_in = -1;
      for (int p = 0; p < kProbes; ++p)
        if (dist[p] < C.r) last_in = p;
      const double new_hi = (last_in + 1 < kProbes) ? tp[last_in + 1] : C.t_hi;
      if (last_in >= 0) {
        C.t_lo = tp[last_in];
        C.val_lo = val[last_in];
      }
      C.t_hi = new_hi;
    }
    if (C.phase == kPhaseBisect && C.t_hi - C.t_lo <= eps * C.t_hi) C.phase = kPhaseDone;
  }
}

__global__ __launch_bounds__(kBlock) void k_probe_fin(Ranges rc, const double* __restrict__ rec_c,
                                                      Ranges rr, const double* __restrict__ rec_r,
                                                      Inst* __restrict__ inst) {
  probe_fin_body(blockIdx.x, rc, rec_c, rr, rec_r, inst);
}

// All multisection passes of a restart check in one launch, one workgroup per
// instance of precision prec (the layouts that run trials in one workgroup per
// instance; no cone blocks there).  Wave w evaluates candidate w % 2 on the
// columns (w < 2) or the rows (w >= 2) of the whole instance, with the
// arithmetic of k_probe_cols / k_probe_rows, and leaves its sums in the record
// of the instance's first block; k_probe_fin's update then reads that one
// record per side.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_probes_wg(Ranges ccol, Ranges crow, const T* x0, const T* x1,
                                                      const T* y0, const T* y1, const double* gc0,
                                                      const double* gc1, const double* gr0, const double* gr1,
                                                      DataPtrs<double> d, Inst* inst, int prec, double* rec_c,
                                                      double* rec_r, int passes) {
  __shared__ int32_t first[4];
  const int iid = blockIdx.x;
  {
    const Inst& I = inst[iid];
    if (I.status != kActive || I.check_due == 0 || I.precision != prec) return;  // uniform
  }
  if (threadIdx.x == 0) {
    first[0] = ccol.inst_blk0[iid];
    first[1] = first[0] + 1;
    first[2] = crow.inst_blk0[iid];
    first[3] = first[2] + 1;
  }
  __syncthreads();
  Ranges rc1 = ccol, rr1 = crow;
  rc1.inst_blk0 = first - iid;
  rr1.inst_blk0 = first + 2 - iid;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int q = wave & 1;
  const bool cols = wave < 2;
  for (int pass = 0; pass < passes; ++pass) {
    const Inst& I = inst[iid];
    const CandState& C = I.cand[q];
    if (C.phase == kPhaseExp || C.phase == kPhaseBisect) {  // uniform within the wave
      double acc[kProbeNV];
#pragma unroll
      for (int i = 0; i < kProbeNV; ++i) acc[i] = 0.0;
      if (cols) {
        const double tau = I.eta_hat / I.omega, inv_tau = 1.0 / tau;
        double tq[kProbes];
#pragma unroll
        for (int p = 0; p < kProbes; ++p) tq[p] = probe_t(C, p) * tau;
        const T* xs = q == 0 ? x0 : x1;
        const double* gs = q == 0 ? gc0 : gc1;
        for (int j = I.col0 + lane; j < I.col0 + I.cols; j += kWave) {
          const double lo = d.l[j], hi = d.u[j];
          const double xc = (double)xs[j];
          const double b1 = gs[j] - d.c[j];
#pragma unroll
          for (int p = 0; p < kProbes; ++p) {
            const double dx = clampd(xc + tq[p] * b1, lo, hi) - xc;
            acc[p * 2 + 0] += dx * dx * inv_tau;
            acc[p * 2 + 1] += b1 * dx;
          }
        }
      } else {
        const double sigma = I.eta_hat * I.omega, inv_sigma = 1.0 / sigma;
        const int mz_end = I.row0 + I.m_zero;
        double tq[kProbes];
#pragma unroll
        for (int p = 0; p < kProbes; ++p) tq[p] = probe_t(C, p) * sigma;
        const T* ys = q == 0 ? y0 : y1;
        const double* gs = q == 0 ? gr0 : gr1;
        for (int i = I.row0 + lane; i < I.row0 + I.rows; i += kWave) {
          const bool zero_row = i < mz_end;
          const double yc = (double)ys[i];
          const double b2 = d.h[i] - gs[i];
#pragma unroll
          for (int p = 0; p < kProbes; ++p) {
            const double v = yc + tq[p] * b2;
            const double dy = (zero_row ? v : fmax(v, 0.0)) - yc;
            acc[p * 2 + 0] += dy * dy * inv_sigma;
            acc[p * 2 + 1] += b2 * dy;
          }
        }
      }
      double* rec = cols ? rec_c + ((size_t)q * ccol.nblk + first[0]) * kProbeNV
                         : rec_r + ((size_t)q * crow.nblk + first[2]) * kProbeNV;
#pragma unroll
      for (int i = 0; i < kProbeNV; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0) rec[i] = s;
      }
    }
    __syncthreads();
    probe_fin_body(iid, rc1, rec_c, rr1, rec_r, inst);
    __syncthreads();
  }
}

// Restart decision (Section 2.3), primal weight (Section 2.5), termination
// (Section 3) and the mixed-precision polish switch.  Thread 0 only.
__global__ void k_decide(Inst* __restrict__ inst, int nb) {
  const int iid = blockIdx.x * blockDim.x + threadIdx.x;
  if (iid >= nb) return;
  Inst& I = inst[iid];
  if (I.status != kActive || I.check_due == 0) return;
  I.checks += 1;
  I.ray_due = 0;
  const int nc = I.use_avg ? 2 : 1;
  bool all_valid = true;
  for (int q = 0; q < nc; ++q) {
    CandState& C = I.cand[q];
    if (C.phase == kPhaseBisect) C.phase = kPhaseDone;  // pass budget spent: take t_lo
    if (C.phase == kPhaseExp) C.phase = kPhaseDone;
    if (I.force_kkt) C.rho = NAN;  // the gap is not computed
    else if (!(C.r > 0.0) || !isfinite(C.r)) C.rho = NAN;
    else if (C.scale == 0.0) C.rho = 0.0;
    else C.rho = C.val_lo / C.r;
    if (!(C.rho >= 0.0) || !isfinite(C.rho)) all_valid = false;
  }
  for (int q = 0; q < kMaxCand; ++q) {
    I.chk_rho[q] = q < nc ? I.cand[q].rho : NAN;
    I.chk_r[q] = q < nc ? I.cand[q].r : NAN;
  }
  if (I.has_anchor && !(I.rho_anchor >= 0.0 && isfinite(I.rho_anchor))) all_valid = false;
  if (I.has_prev && !(I.rho_prev >= 0.0 && isfinite(I.rho_prev))) all_valid = false;
  const bool use_kkt = I.force_kkt != 0 || !all_valid;
  int ch;
  if (I.method == 1) ch = 1;
  else if (I.method == 2 || nc == 1) ch = 0;
  else {
    const double m0 = use_kkt ? I.cand[0].kkt : I.cand[0].rho;
    const double m1 = use_kkt ? I.cand[1].kkt : I.cand[1].rho;
    ch = (m0 <= m1) ? 0 : 1;
  }
  CandState& C = I.cand[ch];
  const double mc = use_kkt ? C.kkt : C.rho;
  const double ma = use_kkt ? I.kkt_anchor : I.rho_anchor;
  const double mp = use_kkt ? I.kkt_prev : I.rho_prev;
  I.use_kkt = use_kkt;
  I.chosen = ch;
  I.pobj = C.pobj;
  I.dobj = C.dobj;
  I.abs_p = C.abs_p;
  I.abs_d = C.abs_d;
  I.abs_gap = C.abs_gap;
  I.rel_p = C.rel_p;
  I.rel_d = C.rel_d;
  I.rel_gap = C.rel_gap;
  const double amax = fmax(C.abs_p, fmax(C.abs_d, C.abs_gap));
  const double rmax = fmax(C.rel_p, fmax(C.rel_d, C.rel_gap));
  const bool optimal = (amax <= I.abs_tol) || (rmax <= I.rel_tol);
  bool restart = false;
  if ((double)I.k >= 0.223 * (double)I.kbar) restart = true;
  else if (I.has_anchor) {
    if (mc <= 0.4 * ma) restart = true;
    else if (I.has_prev && mc > mp && mc <= 0.8 * ma) restart = true;
  }
  I.optimal = optimal ? 1 : 0;
  I.switch_fp64 = 0;
  if (!optimal && I.precision == kFP32) {
    // Two signs that FP32 storage limits the attainable error.  Near the
    // tolerance (within 100x of rel_tol): stall_checks checks without a 10%
    // improvement of the best error (a slow linear descent still improves by
    // that much within the window; an error at a rounding floor does not).  At
    // any level: 8 x stall_checks checks without any new record low -- a
    // steady (even slow) descent keeps setting records, while an error that
    // fluctuates at a rounding floor sets them ever more rarely.
    if (!(rmax >= 0.9 * I.best_rel) || rmax > 100.0 * I.rel_tol) {
      I.best_rel = rmax;
      I.stall = 0;
    } else {
      I.stall += 1;
    }
    if (rmax < I.best_any) {
      I.best_any = rmax;
      I.stall_any = 0;
    } else {
      I.stall_any += 1;
    }
    if ((I.polish_tol > 0.0 && rmax <= I.polish_tol) ||
        (I.stall_checks > 0 && (I.stall >= I.stall_checks || I.stall_any >= 8 * I.stall_checks))) {
      I.switch_fp64 = 1;
      restart = true;
    }
  }
  if (optimal) {
    I.restart = 1;
    return;
  }
  if (isnan(rmax)) {
    I.restart = 0;
    I.status = kDone;
    I.exit_code = 8;
    return;
  }
  I.restart = restart ? 1 : 0;
  I.ray_due = I.infeas_on;
  if (restart) {
    const double dx = sqrt(C.dxa2), dy = sqrt(C.dya2);
    double w = I.omega;
    if (dx > 1e-10 && dy > 1e-10) w = exp(0.5 * log(dy / dx) + 0.5 * log(w));
    if (w > 1e5 || w < 1e-5) w = I.omega0;
    I.omega = w;
    I.rho_anchor = C.rho;
    I.kkt_anchor = sqrt(w * w * C.errp * C.errp + C.errd * C.errd / (w * w) + C.gap * C.gap);
    I.has_anchor = 1;
    I.has_prev = 0;
    I.k = 0;
    I.sum_eta = 0.0;
    I.t += 1;
    I.restarts += 1;
  } else {
    I.rho_prev = C.rho;
    I.kkt_prev = C.kkt;
    I.has_prev = 1;
  }
  // trial budget spent: stop after this check (k_check_end), once the
  // infeasibility tests of the check have run
  if (I.kbar >= I.max_iter) I.stop_max_iter = 1;
}

// Apply a restart (anchor <- candidate, products refreshed from the FP64-value
// candidate products) or, for an optimal candidate, write the unscaled answer.
// Columns: x, G^T y, average sums, x_out = D2 x, lam_out = (c_hat - G^T y_hat)/D2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restart_cols(Ranges R, IterPtrs<T> it, IterPtrs<double> it64,
                                                         const double* __restrict__ g0,
                                                         const double* __restrict__ g1,
                                                         DataPtrs<double> d, const double* __restrict__ D2,
                                                         double* __restrict__ xout, double* __restrict__ lamout,
                                                         const Inst* __restrict__ inst, int prec) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (I.check_due == 0 || I.restart == 0 || I.precision != prec) return;
  const int ch = I.chosen;
  const T* xc = ch == 0 ? it.xh : it.xbar;
  const double* gc = ch == 0 ? g0 : g1;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double xv = (double)xc[j];
    const double gv = gc[j];
    if (I.optimal) {
      xout[j] = D2[j] * xv;
      lamout[j] = (d.c[j] - gv) / D2[j];
    } else if (I.switch_fp64) {
      it64.x[j] = xv;
      it64.xa[j] = xv;
      it64.xh[j] = xv;
      it64.gty[j] = gv;
      it64.gtya[j] = gv;
      it64.gtyh[j] = gv;
      it64.sx[j] = 0.0;
    } else {
      const T xt = (T)xv, gt = (T)gv;
      it.x[j] = xt;
      it.xa[j] = xt;
      it.gty[j] = gt;
      it.gtya[j] = gt;
      it.sx[j] = (T)0;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restart_rows(Ranges R, IterPtrs<T> it, IterPtrs<double> it64,
                                                         const double* __restrict__ g0,
                                                         const double* __restrict__ g1,
                                                         const double* __restrict__ D1,
                                                         double* __restrict__ yout,
                                                         const Inst* __restrict__ inst, int prec) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (I.check_due == 0 || I.restart == 0 || I.precision != prec) return;
  const int ch = I.chosen;
  const T* yc = ch == 0 ? it.yh : it.ybar;
  const double* gc = ch == 0 ? g0 : g1;
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) {
    const double yv = (double)yc[i];
    const double gv = gc[i];
    if (I.optimal) {
      yout[i] = D1[i] * yv;
    } else if (I.switch_fp64) {
      it64.y[i] = yv;
      it64.ya[i] = yv;
      it64.yh[i] = yv;
      it64.gx[i] = gv;
      it64.gxa[i] = gv;
      it64.gxh[i] = gv;
      it64.sy[i] = 0.0;
    } else {
      const T yt = (T)yv, gt = (T)gv;
      it.y[i] = yt;
      it.ya[i] = yt;
      it.gx[i] = gt;
      it.gxa[i] = gt;
      it.sy[i] = (T)0;
    }
  }
}

__global__ void k_check_end(Inst* __restrict__ inst, int nb) {
  const int iid = blockIdx.x * blockDim.x + threadIdx.x;
  if (iid >= nb) return;
  Inst& I = inst[iid];
  if (I.check_due == 0) return;
  if (I.optimal && I.status == kActive) {
    I.status = kDone;
    I.exit_code = 0;
  }
  if (I.stop_max_iter && I.status == kActive) {
    I.status = kDone;
    I.exit_code = 1;
  }
  if (I.switch_fp64 && I.status == kActive) {
    I.precision = kFP64;
    I.switch_fp64 = 0;
    I.best_rel = INFINITY;
    I.stall = 0;
    I.best_any = INFINITY;
    I.stall_any = 0;
  }
  I.check_due = 0;
  I.restart = 0;
  I.ray_due = 0;
}

// ===========================================================================
// Infeasibility tests (option list of Section 3; exit codes 2-5)
// ===========================================================================
// The tests run on rays: the displacement of the PDHG output z_hat from the
// projected start point, r_x = Proj_rec(x_hat - x_start) onto the recession
// cone of the box and r_y = Proj_Kd(y_hat - y_start), in the rescaled space
// (both projections commute with the positive diagonal scaling).  Unscaled,
// G^T (D1 r_y) = D2^{-1} G_hat^T r_y and G (D2 r_x) = D1^{-1} G_hat r_x.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ray_vec_cols(Ranges R, const T* __restrict__ xh,
                                                         const double* __restrict__ xs0, DataPtrs<double> d,
                                                         double* __restrict__ rx, const Inst* __restrict__ inst,
                                                         int prec) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (!mode_selects(I, kModeRay) || I.precision != prec) return;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    double v = (double)xh[j] - xs0[j];
    const bool lf = isfinite(d.l[j]), uf = isfinite(d.u[j]);
    if (lf && uf) v = 0.0;
    else if (lf) v = fmax(v, 0.0);
    else if (uf) v = fmin(v, 0.0);
    rx[j] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ray_vec_rows(Ranges R, const T* __restrict__ yh,
                                                         const double* __restrict__ ys0, const double* __restrict__ D1,
                                                         double* __restrict__ ry, const Inst* __restrict__ inst,
                                                         int prec) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (!mode_selects(I, kModeRay) || I.precision != prec) return;
  const int mz_end = I.row0 + I.m_zero;
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) {
    if (i >= I.soc_start) continue;  // cone block rows: below
    const double v = (double)yh[i] - ys0[i];
    ry[i] = i < mz_end ? v : fmax(v, 0.0);
  }
  // cone blocks: the unscaled ray D1 (y_hat - y_start) projected onto the dual cone,
  // stored scaled back by 1 / D1 like the other rows
  for_cone_blocks(R, b, [&](int r0, int dim, int kind) {
    wave_proj_cone(
        kind, true, dim, [&](int i) { return D1[r0 + i] * ((double)yh[r0 + i] - ys0[r0 + i]); }, [](int) { return 1.0; },
        [&](int i, double p) { ry[r0 + i] = p / D1[r0 + i]; });
  });
}

// Column terms, with lam = -(G_hat^T r_y)_j / D2_j (the unscaled -G^T r_y) and
// the unscaled bounds l_j = l_hat_j D2_j, u_j = u_hat_j D2_j:
//   [0] ||lam - Proj_Lambda lam||^2   [1] sum l lam+ - u lam- (finite bounds)
//   [2] its terms' magnitudes          [3] number of those terms
//   [4] c^T r_x (= c_hat^T r_x)         [5] its terms' magnitudes
constexpr int kRayColsNV = 6;
__global__ __launch_bounds__(kBlock) void k_ray_cols(Ranges R, const double* __restrict__ rx,
                                                     const double* __restrict__ rgty, DataPtrs<double> d,
                                                     const double* __restrict__ D2, const Inst* __restrict__ inst,
                                                     double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock * kRayColsNV];
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (!mode_selects(I, kModeRay)) return;
  double acc[kRayColsNV] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double dj = D2[j];
    const double lam = -rgty[j] / dj;
    const double lo = d.l[j], hi = d.u[j];
    const bool lf = isfinite(lo), uf = isfinite(hi);
    double viol;
    if (!lf && !uf) viol = lam;               // Lambda_j = {0}
    else if (!lf) viol = fmax(lam, 0.0);      // R-
    else if (!uf) viol = fmin(lam, 0.0);      // R+
    else viol = 0.0;                          // R
    acc[0] += viol * viol;
    if (lf) {
      const double t = (lo * dj) * fmax(lam, 0.0);
      acc[1] += t;
      acc[2] += fabs(t);
      acc[3] += 1.0;
    }
    if (uf) {
      const double t = -(hi * dj) * fmax(-lam, 0.0);
      acc[1] += t;
      acc[2] += fabs(t);
      acc[3] += 1.0;
    }
    const double cx = rx ? d.c[j] * rx[j] : 0.0;
    acc[4] += cx;
    acc[5] += fabs(cx);
  }
  block_sum_store<kRayColsNV>(acc, lds, rec + (size_t)b * kRayColsNV);
}

// Row terms: [0] h^T r_y (= h_hat^T r_y), [1] its terms' magnitudes,
// [2] ||G r_x - Proj_Kd*(G r_x)||^2 with (G r_x)_i = (G_hat r_x)_i / D1_i
// (zero when no instance has a nonzero primal ray: rgx null).
constexpr int kRayRowsNV = 3;
__global__ __launch_bounds__(kBlock) void k_ray_rows(Ranges R, const double* __restrict__ ry,
                                                     const double* __restrict__ rgx, DataPtrs<double> d,
                                                     const double* __restrict__ D1, const Inst* __restrict__ inst,
                                                     double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock * kRayRowsNV];
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (!mode_selects(I, kModeRay)) return;
  const int mz_end = I.row0 + I.m_zero;
  double acc[kRayRowsNV] = {0.0, 0.0, 0.0};
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) {
    const double t = d.h[i] * ry[i];
    acc[0] += t;
    acc[1] += fabs(t);
    if (rgx && i < I.soc_start) {
      const double r = rgx[i] / D1[i];
      const double res = i < mz_end ? r : fmin(r, 0.0);
      acc[2] += res * res;
    }
  }
  // cone blocks: the unscaled G r_x against the block's cone
  if (rgx)
    for_cone_blocks(R, b, [&](int r0, int dim, int kind) {
      wave_proj_cone(
          kind, false, dim, [&](int i) { return rgx[r0 + i] / D1[r0 + i]; }, [](int) { return 1.0; },
          [&](int i, double p) {
            const double res = rgx[r0 + i] / D1[r0 + i] - p;
            acc[2] += res * res;
          });
    });
  block_sum_store<kRayRowsNV>(acc, lds, rec + (size_t)b * kRayRowsNV);
}

// gamma_N = N u / (1 - N u), u = 2^-53: relative error bound of a sum of N terms.
__device__ __forceinline__ double rounding_bound(double count) {
  const double nu = fmax(count, 1.0) * 0x1p-53;
  return nu / (1.0 - nu);
}

// Ratios, trend counters and the exit decision of the infeasibility tests.
// Priority: high-accuracy primal (3), high-accuracy dual (5), low-accuracy
// primal (2), low-accuracy dual (4); a tolerance of 0 never passes.
__global__ __launch_bounds__(kBlock) void k_ray_fin(Ranges rc, const double* __restrict__ rec_c, Ranges rr,
                                                    const double* __restrict__ rec_r, Inst* __restrict__ inst) {
  __shared__ double lds[kWavesPerBlock * kRayColsNV];
  const int iid = blockIdx.x;
  Inst& I = inst[iid];
  if (!mode_selects(I, kModeRay)) return;
  double cs[kRayColsNV], rs[kRayRowsNV];
  reduce_records<kRayColsNV, kRayColsNV>(rec_c, rc.inst_blk0[iid], rc.inst_blk0[iid + 1], lds, cs);
  reduce_records<kRayRowsNV, kRayRowsNV>(rec_r, rr.inst_blk0[iid], rr.inst_blk0[iid + 1], lds, rs);
  if (threadIdx.x != 0) return;
  const double f = rs[0] + cs[1];
  const double fmag = rs[1] + cs[2];
  const double ratio_p = f > rounding_bound((double)I.rows + cs[3]) * fmag ? sqrt(cs[0]) / f : (double)INFINITY;
  const double g = -cs[4];
  const double ratio_d = g > rounding_bound((double)I.cols) * cs[5] ? sqrt(rs[2]) / g : (double)INFINITY;
  const double pobj = I.cand[0].pobj, dobj = I.cand[0].dobj;
  const bool up_p = I.has_prev_obj && dobj > I.prev_dobj;
  const bool up_d = I.has_prev_obj && -pobj > I.prev_negp;
  I.prev_dobj = dobj;
  I.prev_negp = -pobj;
  I.has_prev_obj = 1;
  I.trend_p = (ratio_p < I.eps_inf[0] && up_p) ? I.trend_p + 1 : 0;
  I.trend_d = (ratio_d < I.eps_inf[1] && up_d) ? I.trend_d + 1 : 0;
  I.ratio_p = ratio_p;
  I.ratio_d = ratio_d;
  int code = 0;
  if (ratio_p < I.eps_inf[2]) code = 3;
  else if (ratio_d < I.eps_inf[3]) code = 5;
  else if (I.trend_p >= kTrendChecks) code = 2;
  else if (I.trend_d >= kTrendChecks) code = 4;
  if (code) {
    I.status = kDone;
    I.exit_code = code;
    I.restart = 0;
    I.switch_fp64 = 0;
  }
}

// Device warm starts into the packed FP64 start vector.
template <typename TW>
__global__ void k_pack_warm(const void* const* __restrict__ src, const int32_t* __restrict__ off, int B,
                            double* __restrict__ out, int32_t* __restrict__ nan_flag) {
  for (int b = blockIdx.y; b < B; b += gridDim.y) {
    const int o0 = off[b], len = off[b + 1] - off[b];
    const TW* sp = static_cast<const TW*>(src[b]);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x) {
      const double v = sp ? (double)sp[e] : 0.0;
      if (isnan(v)) *nan_flag = 1;
      out[o0 + e] = v;
    }
  }
}

// Evaluated point (start point or final point): termination test and output.
__global__ void k_eval_fin(Inst* __restrict__ inst, int nb, int mode) {
  const int iid = blockIdx.x * blockDim.x + threadIdx.x;
  if (iid >= nb) return;
  Inst& I = inst[iid];
  if (!mode_selects(I, mode)) return;
  const CandState& C = I.cand[0];
  I.pobj = C.pobj;
  I.dobj = C.dobj;
  I.abs_p = C.abs_p;
  I.abs_d = C.abs_d;
  I.abs_gap = C.abs_gap;
  I.rel_p = C.rel_p;
  I.rel_d = C.rel_d;
  I.rel_gap = C.rel_gap;
  if (mode == kModeEvalStart) {
    const double amax = fmax(C.abs_p, fmax(C.abs_d, C.abs_gap));
    const double rmax = fmax(C.rel_p, fmax(C.rel_d, C.rel_gap));
    I.optimal = ((amax <= I.abs_tol) || (rmax <= I.rel_tol)) ? 1 : 0;
  } else {
    I.optimal = 0;
  }
}

// Write the evaluated point (x_hat, y_hat) unscaled.  Start mode: only for
// instances found optimal (which then stop); final mode: every selected instance.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_eval_out_cols(Ranges R, const T* __restrict__ xh,
                                                          const double* __restrict__ g0,
                                                          DataPtrs<double> d, const double* __restrict__ D2,
                                                          double* __restrict__ xout, double* __restrict__ lamout,
                                                          const Inst* __restrict__ inst, int prec, int mode) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (!mode_selects(I, mode) || I.precision != prec) return;
  if (mode == kModeEvalStart && !I.optimal) return;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    xout[j] = D2[j] * (double)xh[j];
    lamout[j] = (d.c[j] - g0[j]) / D2[j];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_eval_out_rows(Ranges R, const T* __restrict__ yh,
                                                          const double* __restrict__ D1,
                                                          double* __restrict__ yout,
                                                          const Inst* __restrict__ inst, int prec, int mode) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (!mode_selects(I, mode) || I.precision != prec) return;
  if (mode == kModeEvalStart && !I.optimal) return;
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) yout[i] = D1[i] * (double)yh[i];
}

__global__ void k_eval_start_end(Inst* __restrict__ inst, int nb) {
  const int iid = blockIdx.x * blockDim.x + threadIdx.x;
  if (iid >= nb) return;
  Inst& I = inst[iid];
  if (I.status == kActive && I.optimal) {
    I.status = kDone;
    I.exit_code = 0;
  }
}

// Counts of active instances per precision, for the host loop.
__global__ void k_summary(const Inst* __restrict__ inst, int nb, int32_t* __restrict__ out) {
  __shared__ int32_t cnt[2];
  if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
  __syncthreads();
  int a32 = 0, a64 = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    if (inst[i].status == kActive) {
      if (inst[i].precision == kFP32) ++a32;
      else ++a64;
    }
  }
  atomicAdd(&cnt[0], a32);
  atomicAdd(&cnt[1], a64);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = cnt[0];
    out[1] = cnt[1];
  }
}

__global__ void k_timeout(Inst* __restrict__ inst, int nb) {
  const int iid = blockIdx.x * blockDim.x + threadIdx.x;
  if (iid >= nb) return;
  if (inst[iid].status == kActive) {
    inst[iid].status = kDone;
    inst[iid].exit_code = 6;
  }
}

// Apply a pending Halpern commit (used to export the internal state at exit).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flush_commit(Ranges R, T* __restrict__ z,
                                                         const T* __restrict__ zh, const T* __restrict__ za,
                                                         T* __restrict__ g, const T* __restrict__ gh,
                                                         const T* __restrict__ ga, T* __restrict__ s,
                                                         const Inst* __restrict__ inst, int prec) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (I.pending == 0 || I.precision != prec) return;
  const double ca = I.ca, cb = I.cb, beta = I.beta, etak = I.eta_k;
  const bool avg = I.use_avg != 0;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double zhv = (double)zh[j];
    z[j] = (T)(ca * ((1.0 + beta) * zhv - beta * (double)z[j]) + cb * (double)za[j]);
    g[j] = (T)(ca * ((1.0 + beta) * (double)gh[j] - beta * (double)g[j]) + cb * (double)ga[j]);
    if (avg) s[j] = (T)((double)s[j] + etak * zhv);
  }
}

__global__ void k_clear_pending(Inst* __restrict__ inst, int nb) {
  const int iid = blockIdx.x * blockDim.x + threadIdx.x;
  if (iid < nb) inst[iid].pending = 0;
}

// ===========================================================================
// Set-up: diagonal rescaling (Section 2.6), norms, start point
// ===========================================================================

// Per row of a CSR-like structure: max_j (D1_i |a_ij|) D2_j   (mode 0)
// or sum_j ((D1_i a_ij) D2_j)^2 (mode 1).  For the transposed structure pass
// swap=1, so that the row scale is indexed by the stored index.
__global__ __launch_bounds__(kBlock) void k_scale_stat(Tiles tl, MatPtrs<double> A,
                                                       const double* __restrict__ Drow,
                                                       const double* __restrict__ Dcol, int swap,
                                                       int mode, double* __restrict__ out) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int t1 = tl.blk_tile1[b];
  for (int t = tl.blk_tile0[b] + wave; t < t1; t += kWavesPerBlock) {
    const int r0 = tl.tile_row0[t], r1 = tl.tile_row1[t], lg = tl.tile_lg[t];
    const int L = 1 << lg;
    const int r = r0 + (lane >> lg);
    const int li = lane & (L - 1);
    double s = 0.0;
    if (r < r1) {
      const int p1 = A.ptr[r + 1];
      for (int p = A.ptr[r] + li; p < p1; p += L) {
        const int c = A.idx[p];
        const double di = swap ? Drow[c] : Drow[r];
        const double dj = swap ? Dcol[r] : Dcol[c];
        if (mode == 0) {
          s = fmax(s, (di * fabs(A.val[p])) * dj);
        } else {
          const double e = (di * A.val[p]) * dj;
          s += e * e;
        }
      }
    }
    if (mode == 0) {
      for (int off = L >> 1; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off, kWave));
    } else {
      s = group_sum(s, L);
    }
    if (li == 0 && r < r1) out[r] = s;
  }
}

// D <- D / sqrt(stat) (Ruiz, mode 0) or D <- D / sqrt(sqrt(stat)) (L2, mode 1); 0 keeps D.
__global__ void k_scale_update(double* __restrict__ D, const double* __restrict__ stat, int n, int mode) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = stat[i];
  if (s > 0.0) {
    const double r = mode == 0 ? sqrt(s) : sqrt(sqrt(s));
    D[i] = D[i] / r;
  }
}

__global__ void k_fill(double* __restrict__ p, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Scaled values: a_hat = (D1_i a_ij) D2_j, FP64 and FP32 copies.
__global__ __launch_bounds__(kBlock) void k_scale_vals(Tiles tl, MatPtrs<double> A,
                                                       const double* __restrict__ Drow,
                                                       const double* __restrict__ Dcol, int swap,
                                                       int vmod, double* __restrict__ v64,
                                                       float* __restrict__ v32) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int t1 = tl.blk_tile1[b];
  for (int t = tl.blk_tile0[b] + wave; t < t1; t += kWavesPerBlock) {
    const int r0 = tl.tile_row0[t], r1 = tl.tile_row1[t], lg = tl.tile_lg[t];
    const int L = 1 << lg;
    const int r = r0 + (lane >> lg);
    const int li = lane & (L - 1);
    if (r < r1) {
      const int rr = vmod > 0 ? r % vmod : r;  // panel-major structures: real row of virtual row r
      const int p1 = A.ptr[r + 1];
      for (int p = A.ptr[r] + li; p < p1; p += L) {
        const int c = A.idx[p];
        const double di = swap ? Drow[c] : Drow[rr];
        const double dj = swap ? Dcol[rr] : Dcol[c];
        const double e = (di * A.val[p]) * dj;
        v64[p] = e;
        v32[p] = (float)e;
      }
    }
  }
}

// Rescaled vectors: c_hat = D2 c, l_hat = l / D2, u_hat = u / D2 (columns).
__global__ __launch_bounds__(kBlock) void k_scale_cols(Ranges R, const double* __restrict__ c,
                                                       const double* __restrict__ l,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ D2,
                                                       DataMut d64, DataMut32 d32) {
  const int b = blockIdx.x;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double dj = D2[j];
    const double cv = dj * c[j], lv = l[j] / dj, uv = u[j] / dj;
    d64.c[j] = cv;
    d64.l[j] = lv;
    d64.u[j] = uv;
    d32.c[j] = (float)cv;
    d32.l[j] = (float)lv;
    d32.u[j] = (float)uv;
  }
}

__global__ __launch_bounds__(kBlock) void k_scale_rows(Ranges R, const double* __restrict__ h,
                                                       const double* __restrict__ D1, DataMut d64,
                                                       DataMut32 d32) {
  const int b = blockIdx.x;
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) {
    const double hv = D1[i] * h[i];
    d64.h[i] = hv;
    d32.h[i] = (float)hv;
  }
}

// Norm records over columns: |c_hat|_1, |c_hat|_2^2 (sums); |c|_inf (max).
__global__ __launch_bounds__(kBlock) void k_norm_cols(Ranges R, const double* __restrict__ chat,
                                                      const double* __restrict__ c,
                                                      double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock * 3];
  const int b = blockIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double v = chat[j];
    acc[0] += fabs(v);
    acc[1] += v * v;
    acc[2] = fmax(acc[2], fabs(c[j]));
  }
  block_summax_store<3, 2>(acc, lds, rec + (size_t)b * 3);
}

// Norm records over rows: |h_hat|_1, |h_hat|_2^2 (sums); |h|_inf (max).
__global__ __launch_bounds__(kBlock) void k_norm_rows(Ranges R, const double* __restrict__ hhat,
                                                      const double* __restrict__ h,
                                                      double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock * 3];
  const int b = blockIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) {
    const double v = hhat[i];
    acc[0] += fabs(v);
    acc[1] += v * v;
    acc[2] = fmax(acc[2], fabs(h[i]));
  }
  block_summax_store<3, 2>(acc, lds, rec + (size_t)b * 3);
}

// max |G_hat_ij| per workgroup of the CSR schedule.
__global__ __launch_bounds__(kBlock) void k_norm_mat(Tiles tl, const int32_t* __restrict__ ptr,
                                                     const double* __restrict__ v64,
                                                     double* __restrict__ rec) {
  __shared__ double lds[kWavesPerBlock];
  const int b = blockIdx.x;
  double acc[1] = {0.0};
  const int t0 = tl.blk_tile0[b], t1 = tl.blk_tile1[b];
  if (t1 > t0) {
    const int p0 = ptr[tl.tile_row0[t0]], p1 = ptr[tl.tile_row1[t1 - 1]];
    for (int p = p0 + (int)threadIdx.x; p < p1; p += kBlock) acc[0] = fmax(acc[0], fabs(v64[p]));
  }
  block_summax_store<1, 0>(acc, lds, rec + b);
}

// Per-instance set-up of the scalars from the norm records (Algorithm 1
// inputs: eta_hat = 1/||G_hat||_inf read as max |G_hat_ij|, primal weight
// initialization of Section 2.5).
__global__ __launch_bounds__(kBlock) void k_init_inst(Ranges rc, const double* __restrict__ rec_c,
                                                      Ranges rr, const double* __restrict__ rec_r,
                                                      Tiles tr, const double* __restrict__ rec_m,
                                                      Inst* __restrict__ inst) {
  __shared__ double lds[kWavesPerBlock * 3];
  const int iid = blockIdx.x;
  Inst& I = inst[iid];
  double cs[3], rs[3], ms[1];
  reduce_records<3, 2>(rec_c, rc.inst_blk0[iid], rc.inst_blk0[iid + 1], lds, cs);
  reduce_records<3, 2>(rec_r, rr.inst_blk0[iid], rr.inst_blk0[iid + 1], lds, rs);
  reduce_records<1, 0>(rec_m, tr.inst_blk0[iid], tr.inst_blk0[iid + 1], lds, ms);
  if (threadIdx.x != 0) return;
  I.c1 = cs[0];
  I.c2 = sqrt(cs[1]);
  I.c_inf = cs[2];
  I.h1 = rs[0];
  I.h2 = sqrt(rs[1]);
  I.h_inf = rs[2];
  I.gmax = ms[0];
  I.eta_hat = ms[0] > 0.0 ? 1.0 / ms[0] : 1.0;
  I.eta = I.eta_hat;
  I.omega0 = (I.c2 > 1e-10 && I.h2 > 1e-10) ? I.c2 / I.h2 : 1.0;
  I.omega = I.omega0;
}

// Start point: x = Proj_[l,u](x0 / D2), y = Proj_Kd(y0 / D1); anchor = x_hat = x.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_start_cols(Ranges R, const double* __restrict__ x0,
                                                       const double* __restrict__ D2, DataPtrs<double> d,
                                                       IterPtrs<T> it, double* __restrict__ xs0,
                                                       const Inst* __restrict__ inst, int prec) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (I.precision != prec) return;
  const int j1 = R.blk_end[b];
  for (int j = R.blk_start[b] + (int)threadIdx.x; j < j1; j += kBlock) {
    const double v = x0 ? x0[j] / D2[j] : 0.0;
    const T x = (T)clampd(v, d.l[j], d.u[j]);
    if (xs0) xs0[j] = (double)x;
    it.x[j] = x;
    it.xa[j] = x;
    it.xh[j] = x;
    it.sx[j] = (T)0;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_start_rows(Ranges R, const double* __restrict__ y0,
                                                       const double* __restrict__ D1, IterPtrs<T> it,
                                                       double* __restrict__ ys0, const Inst* __restrict__ inst,
                                                       int prec) {
  const int b = blockIdx.x;
  const Inst& I = inst[R.blk_inst[b]];
  if (I.precision != prec) return;
  const int mz_end = I.row0 + I.m_zero;
  const int i1 = R.blk_end[b];
  for (int i = R.blk_start[b] + (int)threadIdx.x; i < i1; i += kBlock) {
    if (i >= I.soc_start) continue;  // cone block rows: below
    const double v = y0 ? y0[i] / D1[i] : 0.0;
    const T y = (T)(i < mz_end ? v : fmax(v, 0.0));
    if (ys0) ys0[i] = (double)y;
    it.y[i] = y;
    it.ya[i] = y;
    it.yh[i] = y;
    it.sy[i] = (T)0;
  }
  // cone blocks: y0 / D1 projected onto diag(1/D1) (dual cone)
  for_cone_blocks(R, b, [&](int r0, int dim, int kind) {
    wave_proj_cone(
        kind, true, dim, [&](int i) { return y0 ? y0[r0 + i] / D1[r0 + i] : 0.0; }, [&](int i) { return 1.0 / D1[r0 + i]; },
        [&](int i, double p) {
          const int r = r0 + i;
          const T y = (T)p;
          if (ys0) ys0[r] = (double)y;
          it.y[r] = y;
          it.ya[r] = y;
          it.yh[r] = y;
          it.sy[r] = (T)0;
        });
  });
}

// Copy FP64 products into the maintained products of the start point.
template <typename T>
__global__ void k_set_products(T* __restrict__ g, T* __restrict__ ga, T* __restrict__ gh,
                               const double* __restrict__ src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T v = (T)src[i];
  g[i] = v;
  ga[i] = v;
  gh[i] = v;
}

// Plain product out = A in (unscaled or scaled values) for the public SpMV call.
template <typename T, typename TM>
__global__ __launch_bounds__(kBlock) void k_spmv_plain(RowBlocks rb, MatPtrs<TM> A, const T* __restrict__ in,
                                                       T* __restrict__ out) {
  __shared__ double lds[kRowBlockCap + kWavesPerBlock];
  const int b = blockIdx.x;
  const T* const xs[1] = {in};
  block_rows<1>(rb.blk_row0[b], rb.blk_row1[b], A.ptr, A.idx, A.val, xs, lds,
                [&](int r, const double* s) { out[r] = (T)s[0]; });
}

// ===========================================================================
// Launchers
// ===========================================================================
static inline dim3 grid1(int n) { return dim3((unsigned)(n > 0 ? n : 0)); }

template <typename T>
static void launch_primal_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it,
                            const DataPtrs<T>& d) {
  if (k.vcol.nblk > 0)
    k_primal<T><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, it, d, k.inst, prec, k.rec_primal);
}

template <typename T>
static const T* band_val(const KernelCtx& k, int which);
template <>
const float* band_val<float>(const KernelCtx& k, int which) {
  return which ? k.bvalT32 : k.bval32;
}
template <>
const double* band_val<double>(const KernelCtx& k, int which) {
  return which ? k.bvalT64 : k.bval64;
}

template <typename T>
static void launch_dual_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it,
                          const DataPtrs<T>& d, const MatPtrs<T>& A, T* part) {
  if (k.use_band) {
    if (k.band1.nslot > 0)
      k_band_spmv<T><<<grid1(k.band1.nslot), kBandWaves * kWave, 0, s>>>(k.band1, band_val<T>(k, 0), it.xh, part,
                                                                         k.M, k.inst, prec, 0);
  } else if (k.brow.nblk > 0) {
    k_dual<T, T><<<grid1(k.brow.nblk), kBlock, 0, s>>>(k.brow, A, it, d, k.inst, prec, k.rec_dual);
  }
}

template <typename T>
static void launch_dual_epi_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it,
                              const DataPtrs<T>& d, const T* part) {
  if (k.use_band && k.vrow.nblk > 0)
    k_dual_epi<T><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, part, k.band1.P, k.M, it, d,
                                                         k.D1, k.inst, prec, k.rec_dual_epi);
}

template <typename T>
static void launch_lam_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it,
                         const DataPtrs<T>& d, const MatPtrs<T>& AT, T* part) {
  if (k.use_band) {
    if (k.band2.nslot > 0)
      k_band_spmv<T><<<grid1(k.band2.nslot), kBandWaves * kWave, 0, s>>>(k.band2, band_val<T>(k, 1), it.yh, part,
                                                                         k.N, k.inst, prec, 1);
    if (k.vcol.nblk > 0)
      k_lam_epi<T><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, part, k.band2.P, k.N, it, d, k.inst, prec,
                                                          k.rec_lam_epi);
  } else if (k.bcol.nblk > 0) {
    k_lam<T, T><<<grid1(k.bcol.nblk), kBlock, 0, s>>>(k.bcol, AT, it, d, k.inst, prec, k.rec_lam);
  }
}

// part 0: primal pass; part 1: the SpMV G x_hat (fused with the dual step on
// row blocks; band tiles write partial sums); part 2: the rest of the trial.
void launch_trial_part(const KernelCtx& k, hipStream_t s, int mask, int part) {
  if (part == 0) {
    if (mask & 1) launch_primal_t<float>(k, s, kFP32, k.it32, k.d32);
    if (mask & 2) launch_primal_t<double>(k, s, kFP64, k.it64, k.d64);
    return;
  }
  if (part == 1) {
    if (mask & 1) launch_dual_t<float>(k, s, kFP32, k.it32, k.d32, k.A32, k.bpart32);
    if (mask & 2) launch_dual_t<double>(k, s, kFP64, k.it64, k.d64, k.A64, k.bpart64);
    return;
  }
  if (mask & 1) launch_dual_epi_t<float>(k, s, kFP32, k.it32, k.d32, k.bpart32);
  if (mask & 2) launch_dual_epi_t<double>(k, s, kFP64, k.it64, k.d64, k.bpart64);
  const bool split = k.use_band != 0;
  k_fin_ls<<<grid1(k.nb), kBlock, 0, s>>>(k.vcol.inst_blk0, k.rec_primal,
                                           split ? k.vrow.inst_blk0 : k.brow.inst_blk0,
                                           split ? k.rec_dual_epi : k.rec_dual, k.inst);
  if (mask & 1) launch_lam_t<float>(k, s, kFP32, k.it32, k.d32, k.AT32, k.bpartT32);
  if (mask & 2) launch_lam_t<double>(k, s, kFP64, k.it64, k.d64, k.AT64, k.bpartT64);
  k_fin_beta<<<grid1(k.nb), kBlock, 0, s>>>(split ? k.vcol.inst_blk0 : k.bcol.inst_blk0,
                                             split ? k.rec_lam_epi : k.rec_lam, k.inst);
}

// Dynamic LDS the LDS-resident chunk kernel can take: the device's LDS per
// workgroup less the kernel's static LDS; the first call per precision also
// raises the kernel's dynamic-LDS limit to that size.
template <typename T>
static size_t lds_capacity_t() {
  static size_t cap = 0;
  static bool done = false;
  if (!done) {
    done = true;
    int dev = 0, max_lds = 0, optin = 0;
    hipFuncAttributes fa{};
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) {
      if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess)
        max_lds = std::max(max_lds, optin);
    }
    if (max_lds > 0 && hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_trials_lds<T>)) == hipSuccess &&
        (size_t)max_lds > fa.sharedSizeBytes + 1024) {
      const size_t c = (size_t)max_lds - fa.sharedSizeBytes - 1024;
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_trials_lds<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)c) == hipSuccess)
        cap = c;
    }
    (void)hipGetLastError();
  }
  return cap;
}

size_t trials_lds_capacity(int prec) { return prec == kFP32 ? lds_capacity_t<float>() : lds_capacity_t<double>(); }

void launch_trials_wg(const KernelCtx& k, hipStream_t s, int mask, int K) {
  if (k.nb < 1 || K < 1) return;
  if (mask & 1) {
    if (k.lds_trials32 > 0)
      k_trials_lds<float><<<k.nb, kBlock, k.lds_trials32, s>>>(k.vcol, k.brow, k.bcol, k.A32, k.AT32, k.it32, k.d32,
                                                              k.inst, kFP32, K, k.lds_rowwise);
    else
      k_trials_wg<float><<<k.nb, kBlock, 0, s>>>(k.vcol, k.brow, k.bcol, k.A32, k.AT32, k.it32, k.d32, k.inst, kFP32,
                                                 k.rec_primal, k.rec_dual, k.rec_lam, K);
  }
  if (mask & 2) {
    if (k.lds_trials64 > 0)
      k_trials_lds<double><<<k.nb, kBlock, k.lds_trials64, s>>>(k.vcol, k.brow, k.bcol, k.A64, k.AT64, k.it64,
                                                               k.d64, k.inst, kFP64, K, k.lds_rowwise);
    else
      k_trials_wg<double><<<k.nb, kBlock, 0, s>>>(k.vcol, k.brow, k.bcol, k.A64, k.AT64, k.it64, k.d64, k.inst, kFP64,
                                                  k.rec_primal, k.rec_dual, k.rec_lam, K);
  }
}

void launch_trial(const KernelCtx& k, hipStream_t s, int mask) {
  launch_trial_part(k, s, mask, 0);
  launch_trial_part(k, s, mask, 1);
  launch_trial_part(k, s, mask, 2);
}

template <typename T>
static void launch_cand_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it,
                          const T* x0, const T* x1, const T* y0, const T* y1, int mode) {
  if (k.use_band) {
    // band tiles with FP64 values: one pass per vector, then the window sums
    if (k.band1.nslot > 0) {
      k_band_cand<T><<<grid1(k.band1.nslot), kBandWaves * kWave, 0, s>>>(k.band1, k.bval64, x0, k.bpart64, k.M,
                                                                         k.inst, prec, mode, 0);
      if (x1)
        k_band_cand<T><<<grid1(k.band1.nslot), kBandWaves * kWave, 0, s>>>(k.band1, k.bval64, x1, k.bpart64b, k.M,
                                                                           k.inst, prec, mode, 1);
    }
    if (k.vrow.nblk > 0)
      k_band_combine2<<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, k.band1.P, k.M, k.bpart64,
                                                             x1 ? k.bpart64b : nullptr, k.cgx0, k.cgx1, k.inst, mode);
    if (k.band2.nslot > 0) {
      k_band_cand<T><<<grid1(k.band2.nslot), kBandWaves * kWave, 0, s>>>(k.band2, k.bvalT64, y0, k.bpartT64, k.N,
                                                                         k.inst, prec, mode, 0);
      if (y1)
        k_band_cand<T><<<grid1(k.band2.nslot), kBandWaves * kWave, 0, s>>>(k.band2, k.bvalT64, y1, k.bpartT64b,
                                                                           k.N, k.inst, prec, mode, 1);
    }
    if (k.vcol.nblk > 0)
      k_band_combine2<<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, k.band2.P, k.N, k.bpartT64,
                                                             y1 ? k.bpartT64b : nullptr, k.cgty0, k.cgty1, k.inst,
                                                             mode);
  } else if (k.brow.nblk > 0) {
    k_spmv2<T><<<grid1(k.brow.nblk), kBlock, 0, s>>>(k.brow, k.A64, x0, x1, k.cgx0, k.cgx1, k.inst, prec, mode);
  }
  if (!k.use_band && k.bcol.nblk > 0) {
    k_spmv2<T><<<grid1(k.bcol.nblk), kBlock, 0, s>>>(k.bcol, k.AT64, y0, y1, k.cgty0, k.cgty1, k.inst, prec,
                                                      mode);
  }
  if (k.vcol.nblk > 0)
    k_cand_cols<T><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, x0, x1, it.xa, k.cgty0, k.cgty1, k.d64, k.D2,
                                                          k.inst, prec, mode, k.rec_cand_c);
  if (k.vrow.nblk > 0)
    k_cand_rows<T><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, y0, y1, it.ya, k.cgx0, k.cgx1, k.d64, k.D1,
                                                          k.inst, prec, mode, k.rec_cand_r);
}

template <typename T>
static void launch_check_pre_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it) {
  if (k.vcol.nblk > 0)
    k_commit_avg<T><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, it.x, it.xh, it.xa, it.gty, it.gtyh, it.gtya,
                                                           it.sx, it.xbar, k.inst, prec);
  if (k.vrow.nblk > 0)
    k_commit_avg<T><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, it.y, it.yh, it.ya, it.gx, it.gxh, it.gxa,
                                                           it.sy, it.ybar, k.inst, prec);
  launch_cand_t<T>(k, s, prec, it, it.xh, it.xbar, it.yh, it.ybar, kModeCheck);
}

template <typename T>
static void launch_probe_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it) {
  if (k.ccol.nblk > 0)
    k_probe_cols<T><<<dim3(k.ccol.nblk, kMaxCand), kBlock, 0, s>>>(k.ccol, it.xh, it.xbar, k.cgty0, k.cgty1, k.d64,
                                                           k.inst, prec, k.rec_probe_c);
  if (k.crow.nblk > 0)
    k_probe_rows<T><<<dim3(k.crow.nblk, kMaxCand), kBlock, 0, s>>>(k.crow, it.yh, it.ybar, k.cgx0, k.cgx1, k.d64,
                                                                    k.D1, k.inst, prec, k.rec_probe_r);
}

template <typename T>
static void launch_restart_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it) {
  if (k.vcol.nblk > 0)
    k_restart_cols<T><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, it, k.it64, k.cgty0, k.cgty1, k.d64, k.D2,
                                                             k.xout, k.lamout, k.inst, prec);
  if (k.vrow.nblk > 0)
    k_restart_rows<T><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, it, k.it64, k.cgx0, k.cgx1, k.D1, k.yout,
                                                             k.inst, prec);
}

// Products of the rays with FP64 values (every selected instance, whatever
// its precision): rgty = G_hat^T r_y, and rgx = G_hat r_x when some instance
// has an unbounded column.
static void launch_ray_products(const KernelCtx& k, hipStream_t s) {
  if (k.use_band) {
    if (k.band2.nslot > 0)
      k_band_cand<double><<<grid1(k.band2.nslot), kBandWaves * kWave, 0, s>>>(k.band2, k.bvalT64, k.ry, k.bpartT64,
                                                                              k.N, k.inst, kFP64, kModeRay, 0);
    if (k.vcol.nblk > 0)
      k_band_combine2<<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, k.band2.P, k.N, k.bpartT64, nullptr, k.rgty,
                                                             nullptr, k.inst, kModeRay);
    if (k.ray_x) {
      if (k.band1.nslot > 0)
        k_band_cand<double><<<grid1(k.band1.nslot), kBandWaves * kWave, 0, s>>>(k.band1, k.bval64, k.rx, k.bpart64,
                                                                                k.M, k.inst, kFP64, kModeRay, 0);
      if (k.vrow.nblk > 0)
        k_band_combine2<<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, k.band1.P, k.M, k.bpart64, nullptr, k.rgx,
                                                               nullptr, k.inst, kModeRay);
    }
    return;
  }
  if (k.bcol.nblk > 0) {
    k_spmv2<double><<<grid1(k.bcol.nblk), kBlock, 0, s>>>(k.bcol, k.AT64, k.ry, nullptr, k.rgty, nullptr, k.inst,
                                                           kFP64, kModeRay);
  }
  if (!k.ray_x) return;
  if (k.brow.nblk > 0) {
    k_spmv2<double><<<grid1(k.brow.nblk), kBlock, 0, s>>>(k.brow, k.A64, k.rx, nullptr, k.rgx, nullptr, k.inst,
                                                           kFP64, kModeRay);
  }
}

template <typename T>
static void launch_ray_vec_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it) {
  if (k.vcol.nblk > 0 && k.ray_x)
    k_ray_vec_cols<T><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, it.xh, k.xs0, k.d64, k.rx, k.inst, prec);
  if (k.vrow.nblk > 0)
    k_ray_vec_rows<T><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, it.yh, k.ys0, k.D1, k.ry, k.inst, prec);
}

// The infeasibility tests of one check (instances selected by k_decide).
static void launch_ray(const KernelCtx& k, hipStream_t s, int mask) {
  if (mask & 1) launch_ray_vec_t<float>(k, s, kFP32, k.it32);
  if (mask & 2) launch_ray_vec_t<double>(k, s, kFP64, k.it64);
  launch_ray_products(k, s);
  // the candidate records are free once k_cand_fin has run
  if (k.vcol.nblk > 0)
    k_ray_cols<<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, k.ray_x ? k.rx : nullptr, k.rgty, k.d64, k.D2, k.inst,
                                                      k.rec_cand_c);
  if (k.vrow.nblk > 0)
    k_ray_rows<<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, k.ry, k.ray_x ? k.rgx : nullptr, k.d64, k.D1, k.inst,
                                                      k.rec_cand_r);
  k_ray_fin<<<grid1(k.nb), kBlock, 0, s>>>(k.vcol, k.rec_cand_c, k.vrow, k.rec_cand_r, k.inst);
}

void launch_check(const KernelCtx& k, hipStream_t s, int mask) {
  const int nbt = (k.nb + 63) / 64;
  if (mask & 1) launch_check_pre_t<float>(k, s, kFP32, k.it32);
  if (mask & 2) launch_check_pre_t<double>(k, s, kFP64, k.it64);
  k_cand_fin<<<grid1(k.nb), kBlock, 0, s>>>(k.vcol, k.rec_cand_c, k.vrow, k.rec_cand_r, k.inst, kModeCheck);
  if (k.wg_trials && !k.use_band) {
    if (mask & 1)
      k_probes_wg<float><<<k.nb, kBlock, 0, s>>>(k.ccol, k.crow, k.it32.xh, k.it32.xbar, k.it32.yh, k.it32.ybar,
                                                 k.cgty0, k.cgty1, k.cgx0, k.cgx1, k.d64, k.inst, kFP32,
                                                 k.rec_probe_c, k.rec_probe_r, k.probe_passes);
    if (mask & 2)
      k_probes_wg<double><<<k.nb, kBlock, 0, s>>>(k.ccol, k.crow, k.it64.xh, k.it64.xbar, k.it64.yh, k.it64.ybar,
                                                  k.cgty0, k.cgty1, k.cgx0, k.cgx1, k.d64, k.inst, kFP64,
                                                  k.rec_probe_c, k.rec_probe_r, k.probe_passes);
  } else {
    for (int pass = 0; pass < k.probe_passes; ++pass) {
      if (mask & 1) launch_probe_t<float>(k, s, kFP32, k.it32);
      if (mask & 2) launch_probe_t<double>(k, s, kFP64, k.it64);
      k_probe_fin<<<grid1(k.nb), kBlock, 0, s>>>(k.ccol, k.rec_probe_c, k.crow, k.rec_probe_r, k.inst);
    }
  }
  k_decide<<<nbt, 64, 0, s>>>(k.inst, k.nb);
  if (k.infeas) launch_ray(k, s, mask);
  if (mask & 1) launch_restart_t<float>(k, s, kFP32, k.it32);
  if (mask & 2) launch_restart_t<double>(k, s, kFP64, k.it64);
  k_check_end<<<nbt, 64, 0, s>>>(k.inst, k.nb);
}

void launch_summary(const KernelCtx& k, hipStream_t s, int32_t* out) {
  k_summary<<<1, kBlock, 0, s>>>(k.inst, k.nb, out);
}

void launch_timeout(const KernelCtx& k, hipStream_t s) {
  k_timeout<<<(k.nb + 63) / 64, 64, 0, s>>>(k.inst, k.nb);
}

template <typename T>
static void launch_eval_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it, int mode) {
  launch_cand_t<T>(k, s, prec, it, it.xh, nullptr, it.yh, nullptr, mode);
}

template <typename T>
static void launch_eval_out_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it, int mode) {
  if (k.vcol.nblk > 0)
    k_eval_out_cols<T><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, it.xh, k.cgty0, k.d64, k.D2, k.xout,
                                                              k.lamout, k.inst, prec, mode);
  if (k.vrow.nblk > 0)
    k_eval_out_rows<T><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, it.yh, k.D1, k.yout, k.inst, prec, mode);
}

void launch_eval(const KernelCtx& k, hipStream_t s, int mask, int final_mode) {
  const int mode = final_mode ? kModeEvalFinal : kModeEvalStart;
  const int nbt = (k.nb + 63) / 64;
  if (mask & 1) launch_eval_t<float>(k, s, kFP32, k.it32, mode);
  if (mask & 2) launch_eval_t<double>(k, s, kFP64, k.it64, mode);
  k_cand_fin<<<grid1(k.nb), kBlock, 0, s>>>(k.vcol, k.rec_cand_c, k.vrow, k.rec_cand_r, k.inst, mode);
  k_eval_fin<<<nbt, 64, 0, s>>>(k.inst, k.nb, mode);
  if (mask & 1) launch_eval_out_t<float>(k, s, kFP32, k.it32, mode);
  if (mask & 2) launch_eval_out_t<double>(k, s, kFP64, k.it64, mode);
  if (!final_mode) k_eval_start_end<<<nbt, 64, 0, s>>>(k.inst, k.nb);
}

template <typename T>
static void launch_flush_t(const KernelCtx& k, hipStream_t s, int prec, const IterPtrs<T>& it) {
  if (k.vcol.nblk > 0)
    k_flush_commit<T><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, it.x, it.xh, it.xa, it.gty, it.gtyh,
                                                             it.gtya, it.sx, k.inst, prec);
  if (k.vrow.nblk > 0)
    k_flush_commit<T><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, it.y, it.yh, it.ya, it.gx, it.gxh, it.gxa,
                                                             it.sy, k.inst, prec);
}

void launch_flush_commit(const KernelCtx& k, hipStream_t s, int mask) {
  if (mask & 1) launch_flush_t<float>(k, s, kFP32, k.it32);
  if (mask & 2) launch_flush_t<double>(k, s, kFP64, k.it64);
  k_clear_pending<<<(k.nb + 63) / 64, 64, 0, s>>>(k.inst, k.nb);
}

// ---- set-up ----
void launch_setup(const KernelCtx& k, const SetupCtx& su, hipStream_t s, int mask) {
  const int tpb = 256;
  auto blocks = [&](int64_t n) { return dim3((unsigned)((n + tpb - 1) / tpb)); };
  if (k.M > 0) k_fill<<<blocks(k.M), tpb, 0, s>>>(k.D1, 1.0, k.M);
  if (k.N > 0) k_fill<<<blocks(k.N), tpb, 0, s>>>(k.D2, 1.0, k.N);
  if (su.precondition) {
    for (int it = 0; it < su.ruiz_iters; ++it) {
      if (k.trow.nblk > 0)
        k_scale_stat<<<grid1(k.trow.nblk), kBlock, 0, s>>>(k.trow, su.A, k.D1, k.D2, 0, 0, su.stat_r);
      if (k.tcol.nblk > 0)
        k_scale_stat<<<grid1(k.tcol.nblk), kBlock, 0, s>>>(k.tcol, su.AT, k.D1, k.D2, 1, 0, su.stat_c);
      if (k.M > 0) k_scale_update<<<blocks(k.M), tpb, 0, s>>>(k.D1, su.stat_r, (int)k.M, 0);
      if (k.N > 0) k_scale_update<<<blocks(k.N), tpb, 0, s>>>(k.D2, su.stat_c, (int)k.N, 0);
    }
    if (su.l2_pass) {
      if (k.trow.nblk > 0)
        k_scale_stat<<<grid1(k.trow.nblk), kBlock, 0, s>>>(k.trow, su.A, k.D1, k.D2, 0, 1, su.stat_r);
      if (k.tcol.nblk > 0)
        k_scale_stat<<<grid1(k.tcol.nblk), kBlock, 0, s>>>(k.tcol, su.AT, k.D1, k.D2, 1, 1, su.stat_c);
      if (k.M > 0) k_scale_update<<<blocks(k.M), tpb, 0, s>>>(k.D1, su.stat_r, (int)k.M, 1);
      if (k.N > 0) k_scale_update<<<blocks(k.N), tpb, 0, s>>>(k.D2, su.stat_c, (int)k.N, 1);
    }
  }
  if (k.trow.nblk > 0)
    k_scale_vals<<<grid1(k.trow.nblk), kBlock, 0, s>>>(k.trow, su.A, k.D1, k.D2, 0, 0, su.val64, su.val32);
  if (k.tcol.nblk > 0)
    k_scale_vals<<<grid1(k.tcol.nblk), kBlock, 0, s>>>(k.tcol, su.AT, k.D1, k.D2, 1, 0, su.valT64, su.valT32);
  if (k.use_band) {
    if (su.bn > 0)
      k_band_vals<<<blocks(su.bn), tpb, 0, s>>>(su.bsrc, su.bn, su.val64, su.bval64, su.bval32);
    if (su.bnT > 0)
      k_band_vals<<<blocks(su.bnT), tpb, 0, s>>>(su.bsrcT, su.bnT, su.valT64, su.bvalT64, su.bvalT32);
  }
  if (k.vcol.nblk > 0)
    k_scale_cols<<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, su.c, su.l, su.u, k.D2, su.d64m, su.d32m);
  if (k.vrow.nblk > 0)
    k_scale_rows<<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, su.h, k.D1, su.d64m, su.d32m);
  if (k.vcol.nblk > 0) k_norm_cols<<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, su.d64m.c, su.c, su.rec_nc);
  if (k.vrow.nblk > 0) k_norm_rows<<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, su.d64m.h, su.h, su.rec_nr);
  if (k.trow.nblk > 0) k_norm_mat<<<grid1(k.trow.nblk), kBlock, 0, s>>>(k.trow, su.A.ptr, su.val64, su.rec_nm);
  k_init_inst<<<grid1(k.nb), kBlock, 0, s>>>(k.vcol, su.rec_nc, k.vrow, su.rec_nr, k.trow, su.rec_nm, k.inst);
  // start point and its products
  if (mask & 1) {
    if (k.vcol.nblk > 0)
      k_start_cols<float><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, su.x0, k.D2, k.d64, k.it32, k.xs0, k.inst,
                                                                 kFP32);
    if (k.vrow.nblk > 0)
      k_start_rows<float><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, su.y0, k.D1, k.it32, k.ys0, k.inst, kFP32);
  }
  if (mask & 2) {
    if (k.vcol.nblk > 0)
      k_start_cols<double><<<grid1(k.vcol.nblk), kBlock, 0, s>>>(k.vcol, su.x0, k.D2, k.d64, k.it64, k.xs0, k.inst,
                                                                  kFP64);
    if (k.vrow.nblk > 0)
      k_start_rows<double><<<grid1(k.vrow.nblk), kBlock, 0, s>>>(k.vrow, su.y0, k.D1, k.it64, k.ys0, k.inst, kFP64);
  }
  // FP64-value products of the start point: eval mode computes cgx0 = G x_hat, cgty0 = G^T y_hat
  launch_eval(k, s, mask, 0);
  if (mask & 1) {
    if (k.M > 0) k_set_products<float><<<blocks(k.M), tpb, 0, s>>>(k.it32.gx, k.it32.gxa, k.it32.gxh, k.cgx0, k.M);
    if (k.N > 0)
      k_set_products<float><<<blocks(k.N), tpb, 0, s>>>(k.it32.gty, k.it32.gtya, k.it32.gtyh, k.cgty0, k.N);
  }
  if (mask & 2) {
    if (k.M > 0) k_set_products<double><<<blocks(k.M), tpb, 0, s>>>(k.it64.gx, k.it64.gxa, k.it64.gxh, k.cgx0, k.M);
    if (k.N > 0)
      k_set_products<double><<<blocks(k.N), tpb, 0, s>>>(k.it64.gty, k.it64.gtya, k.it64.gtyh, k.cgty0, k.N);
  }
}

void launch_spmv_plain(const RowBlocks& rb, int prec, const int32_t* ptr, const int32_t* idx, const void* val,
                       const void* in, void* out, hipStream_t s) {
  if (rb.nblk <= 0) return;
  if (prec == kFP64) {
    MatPtrs<double> A{ptr, idx, (const double*)val};
    k_spmv_plain<double, double><<<grid1(rb.nblk), kBlock, 0, s>>>(rb, A, (const double*)in, (double*)out);
  } else {
    MatPtrs<float> A{ptr, idx, (const float*)val};
    k_spmv_plain<float, float><<<grid1(rb.nblk), kBlock, 0, s>>>(rb, A, (const float*)in, (float*)out);
  }
}

// One K1 pass on its own (for schedule timing).
void launch_band_plain(const BandTiles& bt, int prec, const void* val, const void* in, void* part, int64_t R,
                       void* out, hipStream_t s) {
  if (bt.nslot <= 0 || R <= 0) return;
  const dim3 g((unsigned)((R + 255) / 256));
  if (prec == kFP64) {
    k_band_spmv<double><<<grid1(bt.nslot), kBandWaves * kWave, 0, s>>>(bt, (const double*)val, (const double*)in,
                                                                       (double*)part, R, nullptr, kFP64, 0);
    k_band_sum<double><<<g, 256, 0, s>>>((const double*)part, bt.P, R, (double*)out);
  } else {
    k_band_spmv<float><<<grid1(bt.nslot), kBandWaves * kWave, 0, s>>>(bt, (const float*)val, (const float*)in,
                                                                      (float*)part, R, nullptr, kFP32, 0);
    k_band_sum<float><<<g, 256, 0, s>>>((const float*)part, bt.P, R, (float*)out);
  }
}

void launch_band_vals(const int32_t* src, int64_t n, const double* v64, double* o64, float* o32, hipStream_t s) {
  if (n > 0) k_band_vals<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, n, v64, o64, o32);
}

__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

void launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n > 0) k_to_f32<<<(unsigned)std::min<int64_t>((n + 255) / 256, 65536), 256, 0, s>>>(in, out, n);
}

void launch_proj_cone(int cone, int dim, const double* v, const double* f, double* out, int64_t count,
                      hipStream_t s) {
  if (count > 0)
    k_proj_cone<<<(unsigned)((count + kWavesPerBlock - 1) / kWavesPerBlock), kBlock, 0, s>>>(cone, dim, v, f, out,
                                                                                           count);
}

void launch_pack_warm(const void* const* src, const int32_t* off, int B, int64_t maxlen, int dtype, double* out,
                      int32_t* nan_flag, hipStream_t s) {
  if (B <= 0 || maxlen <= 0) return;
  const dim3 g((unsigned)std::min<int64_t>((maxlen + 255) / 256, 1024), (unsigned)std::min(B, 4096));
  if (dtype == 0) k_pack_warm<double><<<g, 256, 0, s>>>(src, off, B, out, nan_flag);
  else k_pack_warm<float><<<g, 256, 0, s>>>(src, off, B, out, nan_flag);
}

void launch_dual_only(const KernelCtx& k, hipStream_t s, int prec) {
  if (prec == kFP32) launch_dual_t<float>(k, s, kFP32, k.it32, k.d32, k.A32, k.bpart32);
  else launch_dual_t<double>(k, s, kFP64, k.it64, k.d64, k.A64, k.bpart64);
}

}  // namespace pdcs
