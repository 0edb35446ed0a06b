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
constexpr int kCheckCoarsen = 8;   // multisection passes: blocks this many times larger than the trial passes
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
  int32_t force_kkt;  // option: restart decisions on KKT_omega instead of the normalized gap
  double best_rel, rel_tol, abs_tol, polish_tol, bisect_eps;
  int64_t stall, stall_checks;
  double best_any;    // lowest relative KKT error of the FP32 phase
  int64_t stall_any;  // checks since that record
  // termination errors of the last evaluated point
  double pobj, dobj, abs_p, abs_d, abs_gap, rel_p, rel_d, rel_gap;
  CandState cand[kMaxCand];
  double chk_rho[kMaxCand], chk_r[kMaxCand];  // values of the last restart check
  // infeasibility tests of the option list of Section 3 (exit codes 2-5)
  double eps_inf[4];        // tolerances: primal low, dual low, primal high, dual high
  double ratio_p, ratio_d;  // ratios of the last check (NaN: not evaluated)
  double prev_dobj, prev_negp;  // dual objective and -(primal objective) of z_hat at the previous check
  int32_t infeas_on, ray_due, trend_p, trend_d;
  int32_t has_prev_obj, stop_max_iter;
  int32_t soc_start;        // first second-order-cone row (row0 + rows when none)
  int32_t pad_inf1;
  double* trace;            // per-trial scalars of the first trace_cap trials (or null)
  int64_t trace_cap;
};
constexpr int kTrendChecks = 3;  // consecutive checks the low-accuracy infeasibility tests must pass
constexpr int kTraceStride = 16;  // kbar, eta, eta_bar, dx2, dy2, dy^T G dx, accepted, eta', beta, k,
                                  // then for accepted trials: c^T x_hat, h^T y_hat, sum l lam+, sum u lam-, err_p^2, err_d^2

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

// Row-block schedule of a CSR-like pass (one workgroup per block): either a
// single row of any length, or several consecutive rows holding at most
// kRowBlockCap nonzeros, which are staged as products in LDS.
constexpr int kRowBlockCap = 2048;
struct RowBlocks {
  const int32_t* blk_row0;     // first row of the block
  const int32_t* blk_row1;     // one past the last row
  const int32_t* blk_inst;     // instance (or panel) of the block
  const int32_t* inst_blk0;    // per instance: first block (B+1 entries)
  int32_t nblk;
};

// Band-tile layout of a sparse matrix for single large instances.  A band-tile
// holds the entries of one band of at most kBandRows consecutive rows whose
// gathered index falls in one window of at most 2^kBandColBits indices.  Its
// entries are sorted by gathered index and padded to whole iterations of
// kBandUnroll * kWave entries; entry e packs (index - window start) <<
// kBandSlotBits | slot, where slot < kBandSlots names the LDS accumulator it
// adds into: slots below the band's row count are the rows themselves, higher
// slots are extra accumulators of rows that repeat within one group of kWave
// consecutive entries (no two entries of such a group share a slot), and the
// last slot is the sink of the padding.  A workgroup runs kBandWaves waves, each
// on one band-tile of the same window index.  In a batch every instance has its
// own bands and windows; an instance with fewer windows than the batch's
// largest count has empty tiles (zero partial sums) for the missing ones.
constexpr int kBandRows = 8192;
constexpr int kBandSlots = 9216;
constexpr int kBandSlotBits = 14;
constexpr int kBandColBits = 32 - kBandSlotBits;
constexpr int kBandWaves = 2;
constexpr int kBandUnroll = 16;
struct BandTiles {
  const int32_t* group;      // per workgroup slot group, per wave: band-tile or -1
  const int32_t* slot;       // launch slot -> group (-1: idle); slot s runs on XCD s % 8
  const int32_t* start;      // per band-tile: first entry (ntile + 1 entries)
  const int32_t* row0;       // per band-tile: first row
  const int32_t* nrows;      // per band-tile: rows
  const int32_t* used;       // per band-tile: slots in use (rows + extra slots; the sink excluded)
  const int32_t* tinst;      // per band-tile: instance (bands never cross instances)
  const int32_t* col0;       // per band-tile: window start
  const int32_t* panel;      // per band-tile: window index (partial-sum array)
  const int32_t* run_start;  // per band-tile: first run (ntile + 1 entries)
  const int32_t* run_row;    // per run: row (band-local) owning extra slots
  const int32_t* run_ext;    // per run: first extra slot in ext (nrun + 1 entries)
  const int32_t* ext;        // extra slots, grouped by run
  const uint32_t* pk;        // packed entries
  int32_t nslot;             // launch slots (workgroups)
  int32_t P;                 // windows
};

// Schedule of an elementwise pass: contiguous element ranges per workgroup.
// Row ranges never split a cone block: the blocks inside range b are
// [blk_soc0[b], blk_soc1[b]) of the table (soc_r0: first row, soc_dim:
// dimension, soc_kind: 0 second-order cone, 1 exponential cone, 2 dual
// exponential cone); all five are null when no instance has cone blocks.
struct Ranges {
  const int32_t* blk_start;
  const int32_t* blk_end;
  const int32_t* blk_inst;
  const int32_t* inst_blk0;    // per instance: first workgroup (B+1 entries)
  const int32_t* blk_soc0;
  const int32_t* blk_soc1;
  const int32_t* soc_r0;
  const int32_t* soc_dim;
  const int8_t* soc_kind;
  int32_t nblk;
};

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
// One DPP lane move of a double (both 32-bit halves with the same control):
// lanes whose source is outside the pattern, or whose row is masked off,
// receive +0.0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes, returned to every lane: data-parallel-primitive lane
// moves inside the VALU instead of LDS-crossbar shuffles.  Pairs and quads
// (quad permutes), then rows of 16 (row shifts by 4 and 8: lane 15 of a row
// holds its row's sum), then rows 1 and 3 take lane 15 of the row before and
// rows 2 and 3 take lane 31, so lane 63 holds the total, which is read back
// as a uniform value.  Fixed order: deterministic.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_move<0x114>(v);       // row_shr:4
  v += dpp_move<0x118>(v);       // row_shr:8
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
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
// Sums of NV-value records b0..b1-1 (NV dividing kBlock) into out[0..NV) in
// LDS: thread t adds value t % NV of every (kBlock / NV)-th record, reading
// consecutive doubles across threads, then the kBlock / NV partial sums of
// each value are added in a fixed order.  red: kBlock doubles of LDS.
template <int NV>
__device__ __forceinline__ void reduce_records_wide(const double* rec, int b0, int b1, double* red, double* out) {
  static_assert(kBlock % NV == 0, "record width divides the block");
  if (b1 - b0 == 1) {  // a single record (uniform across the workgroup)
    if (threadIdx.x < NV) out[threadIdx.x] = rec[(size_t)b0 * NV + threadIdx.x];
    __syncthreads();
    return;
  }
  constexpr int R = kBlock / NV;
  const int i = threadIdx.x % NV;
  int b = b0 + (int)threadIdx.x / NV;
  double acc = 0.0;
  for (; b + 3 * R < b1; b += 4 * R) {
    const double v0 = rec[(size_t)b * NV + i], v1 = rec[(size_t)(b + R) * NV + i];
    const double v2 = rec[(size_t)(b + 2 * R) * NV + i], v3 = rec[(size_t)(b + 3 * R) * NV + i];
    acc += v0;
    acc += v1;
    acc += v2;
    acc += v3;
  }
  for (; b < b1; b += R) acc += rec[(size_t)b * NV + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = red[threadIdx.x];
    for (int k = 1; k < R; ++k) t += red[k * NV + threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

template <int NV, int NS>
__device__ __forceinline__ void reduce_records(const double* rec, int b0, int b1, double* lds,
                                               double (&res)[NV]) {
  if (b1 - b0 == 1) {  // a single record (uniform across the workgroup): every thread reads it
#pragma unroll
    for (int i = 0; i < NV; ++i) res[i] = rec[(size_t)b0 * NV + i];
    return;
  }
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  // four records per step: independent loads in flight before they are combined
  constexpr int U = NV <= 8 ? 4 : 1;
  int b = b0 + (int)threadIdx.x;
  for (; b + (U - 1) * kBlock < b1; b += U * kBlock) {
    double v[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < NV; ++i) v[u][i] = rec[(size_t)(b + u * kBlock) * NV + i];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] = (i < NS) ? acc[i] + v[u][i] : fmax(acc[i], v[u][i]);
  }
  for (; b < b1; b += kBlock) {
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

// As row_dot, but the matrix stream (indices and values, read once per pass)
// uses non-temporal loads so that it does not evict the gathered vector from L2.
template <typename TM, typename TV>
__device__ __forceinline__ double row_dot_stream(const int32_t* __restrict__ col, const TM* __restrict__ val,
                                                 const TV* __restrict__ x, int p0, int p1, int li, int L) {
  double s = 0.0;
  int p = p0 + li;
  for (; p + 3 * L < p1; p += 4 * L) {
    const int c0 = __builtin_nontemporal_load(col + p);
    const int c1 = __builtin_nontemporal_load(col + p + L);
    const int c2 = __builtin_nontemporal_load(col + p + 2 * L);
    const int c3 = __builtin_nontemporal_load(col + p + 3 * L);
    const double v0 = (double)__builtin_nontemporal_load(val + p);
    const double v1 = (double)__builtin_nontemporal_load(val + p + L);
    const double v2 = (double)__builtin_nontemporal_load(val + p + 2 * L);
    const double v3 = (double)__builtin_nontemporal_load(val + p + 3 * L);
    const double x0 = (double)x[c0], x1 = (double)x[c1], x2 = (double)x[c2], x3 = (double)x[c3];
    s += v0 * x0;
    s += v1 * x1;
    s += v2 * x2;
    s += v3 * x3;
  }
  for (; p < p1; p += L)
    s += (double)__builtin_nontemporal_load(val + p) * (double)x[__builtin_nontemporal_load(col + p)];
  return s;
}

// Products of one row block with NV gathered vectors, reduced per row; fn(r, s)
// is called exactly once per row r of the block, by one thread, with s[k] the
// row's dot product with xs[k] (FP64 accumulation).  lds: NV * kRowBlockCap
// doubles plus kWavesPerBlock * NV doubles.  Every thread of the workgroup must
// call this (it synchronizes).
template <int NV, typename TM, typename TV, class Fn>
__device__ __forceinline__ void block_rows(int r0, int r1, const int32_t* __restrict__ ptr,
                                           const int32_t* __restrict__ idx, const TM* __restrict__ val,
                                           const TV* const (&xs)[NV], double* lds, Fn&& fn) {
  const int tid = threadIdx.x;
  const int R = r1 - r0;
  const int q0 = ptr[r0], q1 = ptr[r1];
  if (R == 1) {
    // one row of any length: register accumulation, unrolled streaming loads
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    int q = q0 + tid;
    for (; q + 3 * kBlock < q1; q += 4 * kBlock) {
      int c[4];
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        c[u] = __builtin_nontemporal_load(idx + q + u * kBlock);
        v[u] = (double)__builtin_nontemporal_load(val + q + u * kBlock);
      }
#pragma unroll
      for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[k] += v[u] * (double)xs[k][c[u]];
    }
    for (; q < q1; q += kBlock) {
      const int c = __builtin_nontemporal_load(idx + q);
      const double v = (double)__builtin_nontemporal_load(val + q);
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += v * (double)xs[k][c];
    }
    double* red = lds + NV * kRowBlockCap;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double w = wave_sum(s[k]);
      if (lane == 0) red[wave * NV + k] = w;
    }
    __syncthreads();
    if (tid == 0) {
      double t[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        t[k] = 0.0;
        for (int w = 0; w < kWavesPerBlock; ++w) t[k] += red[w * NV + k];
      }
      fn(r0, t);
    }
    return;
  }
  // several rows, at most kRowBlockCap nonzeros: stage the products in LDS
  const int n = q1 - q0;
  for (int i0 = 0; i0 < n; i0 += 4 * kBlock) {
    int c[4];
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * kBlock + tid;
      c[u] = i < n ? __builtin_nontemporal_load(idx + q0 + i) : 0;
      v[u] = i < n ? (double)__builtin_nontemporal_load(val + q0 + i) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * kBlock + tid;
      if (i < n) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * kRowBlockCap + i] = v[u] * (double)xs[k][c[u]];
      }
    }
  }
  __syncthreads();
  if (R <= kBlock) {
    int T = 64;
    while (T > 1 && T * R > kBlock) T >>= 1;
    const int g = tid / T, li = tid & (T - 1);
    const int r = r0 + g;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    if (g < R) {
      const int a = ptr[r] - q0, e = ptr[r + 1] - q0;
      for (int i = a + li; i < e; i += T)
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += lds[k * kRowBlockCap + i];
    }
#pragma unroll
    for (int k = 0; k < NV; ++k)
      for (int off = T >> 1; off > 0; off >>= 1) s[k] += __shfl_xor(s[k], off, kWave);
    if (li == 0 && g < R) fn(r, s);
  } else {
    for (int r = r0 + tid; r < r1; r += kBlock) {
      const int a = ptr[r] - q0, e = ptr[r + 1] - q0;
      double s[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] = 0.0;
      for (int i = a; i < e; ++i)
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += lds[k * kRowBlockCap + i];
      fn(r, s);
    }
  }
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
