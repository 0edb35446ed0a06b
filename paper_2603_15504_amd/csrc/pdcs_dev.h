// Device-side definitions shared by the PDCS kernels (gfx950, wave64).
//
// Data layout.  A launch covers a batch of B >= 1 LPs packed block-diagonally:
// instance b owns rows [row0, row0 + rows) and columns [col0, col0 + cols) of
// the concatenated matrix and of every m- and n-vector.  Work is handed out to
// workgroups through per-workgroup ranges that never straddle two instances,
// so every workgroup reads its instance's scalars once and writes one
// deterministic partial-sum record; a per-instance finalize kernel reduces the
// records of its instance in a fixed order (no floating-point atomics).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdcs {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kProbes = 16;        // t values per bisection pass
constexpr int kMaxCand = 2;        // restart candidates: current PDHG output, average

enum Status : int32_t { kActive = 0, kDone = 1 };
enum Prec : int32_t { kFP64 = 0, kFP32 = 1 };

// Bisection phases for the normalized duality gap.
enum Phase : int32_t { kPhaseOff = 0, kPhaseExp = 1, kPhaseBisect = 2, kPhaseDone = 3 };

struct CandState {
  // reductions of the candidate pass
  double dxa2, dya2;        // ||x_c - x_a||^2, ||y_c - y_a||^2
  double r, scale;          // N-norm radius and sqrt(tau|b1|^2 + sigma|b2|^2)
  double errp, errd, gap, pobj, dobj, kkt;   // scaled L2 errors and KKT_omega
  double abs_p, abs_d, abs_gap, rel_p, rel_d, rel_gap;   // unscaled inf-norm errors
  // bisection state
  double t_lo, t_hi, t_base, val_lo, last_dist;
  int32_t phase, doublings, bracketed, pad;
  double rho;
};

// Per-instance scalar state.  Written only by the single-block finalize
// kernels (thread 0) and by the host at set-up.
struct Inst {
  // geometry
  int32_t row0, rows, col0, cols;
  int32_t m_zero, precision, status, exit_code;
  // step size, weight, reflection
  double omega, omega0, eta, eta_hat, eta_k, beta;
  double ca, cb;            // Halpern coefficients (k+1)/(k+2), 1/(k+2) of the pending commit
  double sum_eta;           // sum of accepted eta in the current restart interval
  // norms of the rescaled data (and inf-norms of the unscaled data)
  double h1, c1, h2, c2, gmax, h_inf, c_inf;
  // counters
  int64_t kbar, k, t, accepted, restarts, checks, fp64_iters, max_iter;
  int64_t check_every;
  int32_t pending, last_acc, check_due, method;
  int32_t use_avg, has_anchor, has_prev, switch_fp64;
  // line-search reductions kept for the reflection parameter
  double dx2, dy2, dydgdx, errp2, hy, cx;
  // restart bookkeeping
  double rho_anchor, kkt_anchor, rho_prev, kkt_prev;
  int32_t restart, chosen, optimal, use_kkt;
  double best_rel, rel_tol, abs_tol, polish_tol, bisect_eps;
  int64_t stall, stall_checks;
  // termination errors of the last evaluated point
  double pobj, dobj, abs_p, abs_d, abs_gap, rel_p, rel_d, rel_gap;
  CandState cand[kMaxCand];
};

// Schedule of a CSR-like pass: wavefront tiles grouped into workgroup ranges.
struct Tiles {
  const int32_t* tile_row0;    // first row of the tile
  const int32_t* tile_row1;    // one past the last row
  const int32_t* tile_lg;      // log2(lanes per row)
  const int32_t* blk_tile0;    // per workgroup: first tile
  const int32_t* blk_tile1;    // per workgroup: one past the last tile
  const int32_t* blk_inst;     // per workgroup: instance
  const int32_t* inst_blk0;    // per instance: first workgroup (B+1 entries)
  int32_t nblk;
};

// Schedule of an elementwise pass: contiguous element ranges per workgroup.
struct Ranges {
  const int32_t* blk_start;
  const int32_t* blk_end;
  const int32_t* blk_inst;
  const int32_t* inst_blk0;    // per instance: first workgroup (B+1 entries)
  int32_t nblk;
};

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Sum NV values over the workgroup; thread 0..NV-1 of the block write out[i].
// lds must hold kWavesPerBlock * NV doubles.  Order is fixed: deterministic.
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* lds, double* out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = wave_sum(v[i]);
    if (lane == 0) lds[wave * NV + i] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) s += lds[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// As block_sum_store, but the first NS entries are sums and the rest maxima.
template <int NV, int NS>
__device__ __forceinline__ void block_summax_store(double (&v)[NV], double* lds, double* out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = (i < NS) ? wave_sum(v[i]) : wave_max(v[i]);
    if (lane == 0) lds[wave * NV + i] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    double s = lds[i];
    for (int w = 1; w < kWavesPerBlock; ++w) s = (i < NS) ? s + lds[w * NV + i] : fmax(s, lds[w * NV + i]);
    out[i] = s;
  }
}

// Reduce the NV-wide records [b0, b1) of one instance inside one workgroup;
// the first NS fields are summed, the rest take the maximum.  Result is
// returned to every thread.  Fixed order: deterministic.
template <int NV, int NS>
__device__ __forceinline__ void reduce_records(const double* rec, int b0, int b1, double* lds,
                                               double (&res)[NV]) {
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = (i < NS) ? 0.0 : 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += kBlock) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double v = rec[(size_t)b * NV + i];
      acc[i] = (i < NS) ? acc[i] + v : fmax(acc[i], v);
    }
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = (i < NS) ? wave_sum(acc[i]) : wave_max(acc[i]);
    if (lane == 0) lds[wave * NV + i] = s;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = lds[i];
    for (int w = 1; w < kWavesPerBlock; ++w) s = (i < NS) ? s + lds[w * NV + i] : fmax(s, lds[w * NV + i]);
    res[i] = s;
  }
  __syncthreads();
}

// Row-dot over a CSR row segment by a group of L lanes (lane li of the group),
// FP64 accumulation, loads unrolled by 4 to keep several gathers in flight.
template <typename TM, typename TV>
__device__ __forceinline__ double row_dot(const int32_t* __restrict__ col, const TM* __restrict__ val,
                                          const TV* __restrict__ x, int p0, int p1, int li, int L) {
  double s = 0.0;
  int p = p0 + li;
  for (; p + 3 * L < p1; p += 4 * L) {
    const int c0 = col[p], c1 = col[p + L], c2 = col[p + 2 * L], c3 = col[p + 3 * L];
    const double v0 = (double)val[p], v1 = (double)val[p + L], v2 = (double)val[p + 2 * L],
                 v3 = (double)val[p + 3 * L];
    const double x0 = (double)x[c0], x1 = (double)x[c1], x2 = (double)x[c2], x3 = (double)x[c3];
    s += v0 * x0;
    s += v1 * x1;
    s += v2 * x2;
    s += v3 * x3;
  }
  for (; p < p1; p += L) s += (double)val[p] * (double)x[col[p]];
  return s;
}

// Sum over the L-lane groups of a wavefront (L a power of two <= 64).
__device__ __forceinline__ double group_sum(double s, int L) {
  for (int off = L >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
  return s;
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
  return fmin(fmax(v, lo), hi);
}

}  // namespace pdcs
