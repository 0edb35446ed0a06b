// Host-visible launch interface of the PDCS kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdcs_dev.h"

namespace pdcs {

// Iterates of one precision, all in the rescaled space (Section 2.6):
// Halpern iterate (x, y), anchor (xa, ya), last PDHG output (xh, yh), the
// maintained products G x, G x_a, G x_hat, G^T y, G^T y_a, G^T y_hat, the
// eta-weighted sums of the interval (sx, sy) and the average candidate.
template <typename T>
struct IterPtrs {
  T *x, *y, *xa, *ya, *xh, *yh;
  T *gx, *gxa, *gxh, *gty, *gtya, *gtyh;
  T *sx, *sy, *xbar, *ybar;
};

// Rescaled problem vectors: c_hat, l_hat, u_hat (columns) and h_hat (rows).
template <typename T>
struct DataPtrs {
  const T *c, *l, *u, *h;
};
struct DataMut {
  double *c, *l, *u, *h;
};
struct DataMut32 {
  float *c, *l, *u, *h;
};

template <typename TM>
struct MatPtrs {
  const int32_t* ptr;
  const int32_t* idx;
  const TM* val;
};

// Longest row or column for the row-wise passes of k_trials_lds.
constexpr int kLdsRowMax = 64;

// Cone blocks per row range: in the elementwise passes (two projections per
// block in the dual epilogue: one per wave), and in the restart checks (one
// block, its multisection probes or candidate terms spread over the waves).
constexpr int kConeBlocksPerRange = kWavesPerBlock / 2;
constexpr int kConeBlocksPerCheckRange = 1;

// LDS footprint of one instance in k_trials_lds: the 14 iterate vectors the
// trials touch, c, l, u, h, both CSR copies of the instance's part of G and
// the three per-block record arrays.  Shared by the host (choice of kernel,
// dynamic LDS size) and the kernel (carving), so both agree.
struct LdsLayout {
  size_t vec, dat, rp, ci, va, cp, ri, vt, rec, blk, total;
};
__host__ __device__ inline size_t lds_align16(size_t b) { return (b + 15) & ~(size_t)15; }
__host__ __device__ inline LdsLayout lds_layout(int64_t m, int64_t n, int64_t nnz, int64_t nb_p, int64_t nb_d,
                                                int64_t nb_l, size_t s) {
  LdsLayout L;
  L.vec = 0;                                            // x xa xh gty gtya gtyh sx | y ya yh gx gxa gxh sy
  L.dat = L.vec + lds_align16((size_t)(7 * n + 7 * m) * s);  // c l u | h
  L.rp = L.dat + lds_align16((size_t)(3 * n + m) * s);
  L.ci = L.rp + lds_align16((size_t)(m + 1) * 4);
  L.va = L.ci + lds_align16((size_t)nnz * 4);
  L.cp = L.va + lds_align16((size_t)nnz * s);
  L.ri = L.cp + lds_align16((size_t)(n + 1) * 4);
  L.vt = L.ri + lds_align16((size_t)nnz * 4);
  L.rec = L.vt + lds_align16((size_t)nnz * s);
  // one record per block, at least one per pass (the row-wise passes)
  L.blk = L.rec + lds_align16((size_t)(2 * (nb_p > 1 ? nb_p : 1) + 4 * (nb_d > 1 ? nb_d : 1) +
                                       3 * (nb_l > 1 ? nb_l : 1)) * 8);
  L.total = L.blk + lds_align16((size_t)(3 * nb_p + 3 * nb_d + 3 * nb_l) * 4);
  return L;
}

struct KernelCtx {
  int nb;
  int64_t M, N;
  Tiles trow, tcol;   // CSR of G (rows) and of G^T (columns): wavefront tiles (set-up passes)
  RowBlocks brow, bcol;  // the same structures in row blocks (iteration passes)
  Ranges vrow, vcol;  // elementwise passes over rows and columns
  Ranges crow, ccol;  // the multisection passes: kCheckCoarsen times larger blocks
  Inst* inst;
  IterPtrs<float> it32;
  IterPtrs<double> it64;
  DataPtrs<float> d32;
  DataPtrs<double> d64;
  MatPtrs<float> A32, AT32;
  MatPtrs<double> A64, AT64;
  double *cgx0, *cgx1, *cgty0, *cgty1;  // FP64-value products of the candidates
  double *D1, *D2;
  double *xout, *yout, *lamout;
  double *rec_primal, *rec_dual, *rec_lam, *rec_cand_c, *rec_cand_r, *rec_probe_c, *rec_probe_r;
  int probe_passes;
  double *rec_dual_epi, *rec_lam_epi;
  // Infeasibility tests: projected start point (FP64, rescaled space), the
  // two rays and their products G_hat r_x (rows) and G_hat^T r_y (columns).
  int infeas;   // some instance runs the tests
  int ray_x;    // some instance has a column with an infinite bound (else r_x = 0)
  double *xs0, *ys0, *rx, *ry, *rgx, *rgty;
  // Band-tile layout (single instances): when use_band is set, the two SpMVs of
  // a trial run on band1 (G, windows over x) and band2 (G^T, windows over y),
  // writing band1.P (band2.P) partial sums per row that the epilogues combine.
  int use_band;
  BandTiles band1, band2;
  const float *bval32, *bvalT32;
  const double *bval64, *bvalT64;
  float *bpart32, *bpartT32;
  double *bpart64, *bpartT64, *bpart64b, *bpartT64b;  // b: second vector of the check products

  // chunks of trials run by k_trials_wg (row blocks, no split, no bands), by
  // k_trials_lds with this many bytes of dynamic LDS when nonzero
  int wg_trials;
  int lds_trials32, lds_trials64;
  int lds_rowwise;  // every row of G and of G^T has at most kLdsRowMax entries: row-wise passes

  // the K1 (K2) product is split into partial sums plus an epilogue pass
  bool split1() const { return use_band != 0; }
  bool split2() const { return use_band != 0; }
};

struct SetupCtx {
  int precondition, ruiz_iters, l2_pass;
  MatPtrs<double> A, AT;          // unscaled values
  const double *c, *l, *u, *h;    // unscaled vectors
  double *val64, *valT64;
  float *val32, *valT32;
  DataMut d64m;
  DataMut32 d32m;
  double *stat_r, *stat_c, *rec_nc, *rec_nr, *rec_nm;
  const double *x0, *y0;          // device start point (unscaled) or null
  // band-tile values: entry e takes the scaled CSR (CSC) value at src[e] (-1: padding)
  const int32_t *bsrc, *bsrcT;
  int64_t bn, bnT;
  double *bval64, *bvalT64;
  float *bval32, *bvalT32;
};

void launch_setup(const KernelCtx& k, const SetupCtx& su, hipStream_t s, int mask);
void launch_trial(const KernelCtx& k, hipStream_t s, int mask);
// K trials of every instance, one workgroup per instance (k.wg_trials layouts)
void launch_trials_wg(const KernelCtx& k, hipStream_t s, int mask, int K);
// LDS left for the instance data of the LDS-resident chunk kernel (bytes)
size_t trials_lds_capacity(int prec);
void launch_check(const KernelCtx& k, hipStream_t s, int mask);
void launch_summary(const KernelCtx& k, hipStream_t s, int32_t* out);
void launch_timeout(const KernelCtx& k, hipStream_t s);
void launch_eval(const KernelCtx& k, hipStream_t s, int mask, int final_mode);
void launch_flush_commit(const KernelCtx& k, hipStream_t s, int mask);
void launch_spmv_plain(const RowBlocks& rb, int prec, const int32_t* ptr, const int32_t* idx, const void* val,
                       const void* in, void* out, hipStream_t s);
void launch_dual_only(const KernelCtx& k, hipStream_t s, int prec);
// Plain product with band tiles: partial sums into part (P x R), then out = their sum.
void launch_band_plain(const BandTiles& bt, int prec, const void* val, const void* in, void* part, int64_t R,
                       void* out, hipStream_t s);
void launch_band_vals(const int32_t* src, int64_t n, const double* v64, double* o64, float* o32, hipStream_t s);
// out[i] = (float)in[i], i < n
void launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
// count vectors of dimension dim (contiguous in v, f, out) projected onto
// diag(f) K, K = K_soc (cone 0), K_exp (1) or K_exp* (2, dim 3).
void launch_proj_cone(int cone, int dim, const double* v, const double* f, double* out, int64_t count,
                      hipStream_t s);
// Warm starts from device pointers: out[off[b] + e] = src[b][e] (FP64 or FP32
// source, dtype 0 / 1; a null src[b] gives zeros), e < off[b + 1] - off[b];
// *nan_flag is set to 1 when a value is NaN.
void launch_pack_warm(const void* const* src, const int32_t* off, int B, int64_t maxlen, int dtype, double* out,
                      int32_t* nan_flag, hipStream_t s);

// Trial split for kernel timing: K3, K1, and the rest of the trial.
void launch_trial_part(const KernelCtx& k, hipStream_t s, int mask, int part);

}  // namespace pdcs
