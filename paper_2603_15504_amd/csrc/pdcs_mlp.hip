// Warm-start MLP for families of LPs: v = W3 relu(W2 relu(W1 u + b1) + b2) + b3.
//
// BF16 weights and activations feed the matrix cores (v_mfma_f32_32x32x16_bf16
// on gfx950) with FP32 accumulation; an FP32 master copy of the weights takes
// the Adam updates.  Every GEMM is C = op(A) op(B) with row-major operands,
// tiled 128 x 128 x 32 per workgroup (four wavefronts of 64 x 64), split along
// K when M x N alone cannot fill the chip; split partials are summed in a fixed
// order, so results are deterministic.  The products' epilogues do the rest of
// a training step where the data already sits in registers: bias and ReLU in
// the forward pass, the loss and its gradient in the output layer, the ReLU
// mask in the backward pass, and Adam in the weight-gradient products, so FP32
// weight gradients never travel through HBM during training.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/pdcs.h"
#include "pdcs_engine.h"

using namespace pdcs;

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TM = 128, TN = 128;

__device__ __forceinline__ bf16 to_bf16(float v) { return (bf16)v; }

// One operand tile (128 rows of op(X) x KT) staged through registers.  op(X)
// row r, column k lives at X[k * ld + r] when trans, else X[r * ld + k].  Each
// thread loads KT / 16 8-element vectors, each along the source's contiguous
// direction:
//   not trans: vector e = tid + 256 q holds row e / (KT/8), k-block e % (KT/8);
//   trans    : thread t holds rows 8 (t % 16) .. +7 for the KT/16 consecutive
//              k = (t / 16) KT/16 + q, one vector per k; lanes 0-15 of a k read
//              256 contiguous bytes.  The store transposes these in registers so
//              that each row goes to LDS as one run of KT/16 k-values.
// vec: the launch guarantees 16-byte alignment of the source and ld % 8 == 0,
// so whole vectors inside the bounds load with one 16-byte access; anything
// else loads element by element.
//
// LDS holds 128 rows of KT + 8 elements.  The 16-byte blocks of a row are
// swizzled by the row's group of eight (block b of row r sits at block
// b ^ ((r / 8) mod KT/8)): the transposed stores of 16 lanes (rows eight apart)
// and the MFMA reads of 32 lanes (32 consecutive rows) then fall on different
// banks.
template <int KT>
struct TileRegs {
  bf16x8 v[KT / 16];
};

template <int KT>
__device__ __forceinline__ int swz(int row, int blk) {
  return blk ^ ((row >> 3) & (KT / 8 - 1));
}

template <int KT>
__device__ __forceinline__ void tile_load(const bf16* __restrict__ X, int ld, int trans, int vec, int r0, int R,
                                          int k0, int kend, TileRegs<KT>& t) {
  const int tid = threadIdx.x;
  constexpr int KQ = KT / 16;
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    bf16x8 v;
    if (!trans) {
      const int e = tid + q * 256;
      const int gr = r0 + e / (KT / 8), gk = k0 + (e % (KT / 8)) * 8;
      if (vec && gr < R && gk + 8 <= kend) {
        v = *reinterpret_cast<const bf16x8*>(X + (size_t)gr * ld + gk);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (gr < R && gk + i < kend) ? X[(size_t)gr * ld + gk + i] : to_bf16(0.0f);
      }
    } else {
      const int gr = r0 + (tid & 15) * 8, gk = k0 + (tid >> 4) * KQ + q;
      if (vec && gk < kend && gr + 8 <= R) {
        v = *reinterpret_cast<const bf16x8*>(X + (size_t)gk * ld + gr);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (gk < kend && gr + i < R) ? X[(size_t)gk * ld + gr + i] : to_bf16(0.0f);
      }
    }
    t.v[q] = v;
  }
}

template <int KT>
__device__ __forceinline__ void tile_store(bf16 (*S)[KT + 8], int trans, const TileRegs<KT>& t) {
  const int tid = threadIdx.x;
  constexpr int KQ = KT / 16;
  if (!trans) {
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int e = tid + q * 256;
      const int rr = e / (KT / 8), blk = e % (KT / 8);
      *reinterpret_cast<bf16x8*>(&S[rr][swz<KT>(rr, blk) * 8]) = t.v[q];
    }
  } else {
    typedef __bf16 bf16xq __attribute__((ext_vector_type(KQ)));
    const int rb = (tid & 15) * 8, kq = (tid >> 4) * KQ;  // k-run kq .. kq + KQ - 1: within one 8-block
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      bf16xq w;
#pragma unroll
      for (int q = 0; q < KQ; ++q) w[q] = t.v[q][i];
      const int row = rb + i;
      *reinterpret_cast<bf16xq*>(&S[row][swz<KT>(row, kq >> 3) * 8 + (kq & 7)]) = w;
    }
  }
}

// How a GEMM output element is used once its FP32 sum s is known.
//   EPI_STORE: C[z][row][col] = s (split partials, or a plain FP32 product)
//   EPI_ACT  : s (+ bias[col]), ReLU, times (mask[idx] > 0) -- the derivative of
//              ReLU read from the BF16 activation it produced -- stored as FP32
//              and/or BF16
//   EPI_ADAM : s is the gradient of weight idx: Adam on the FP32 master weight
//              and its moments, and the BF16 copy the next products read, so the
//              gradient itself never reaches memory
//   EPI_MSE  : s + bias[col] is the network output; with the target t
//              (standardized per column when tmu is set) the loss gradient
//              g = 2 (v - t) * gscale goes out as BF16, and each workgroup leaves
//              one loss partial (FP64) and per-column sums of g for its row tile
enum { EPI_STORE = 0, EPI_ACT = 1, EPI_ADAM = 2, EPI_MSE = 3 };

struct Epi {
  const float* bias = nullptr;
  int relu = 0;
  const bf16* mask = nullptr;
  float* out32 = nullptr;
  bf16* out16 = nullptr;
  float *p = nullptr, *m = nullptr, *v = nullptr;
  bf16* w16 = nullptr;
  float lr = 0, b1 = 0, b2 = 0, eps = 0, c1 = 1, c2 = 1;
  const float* t = nullptr;
  const float* tmu = nullptr;
  const float* tinv = nullptr;
  float gscale = 0;
  int vec4 = 0;  // EPI_ADAM: N % 4 == 0, p / m / v 16-byte and w16 8-byte aligned
  float* colpart = nullptr;
  double* lossp = nullptr;
};

__device__ __forceinline__ void epi_act(const Epi& e, size_t idx, int col, float s) {
  if (e.bias) s += e.bias[col];
  if (e.relu) s = fmaxf(s, 0.0f);
  if (e.mask) s = (float)e.mask[idx] > 0.0f ? s : 0.0f;
  if (e.out32) e.out32[idx] = s;
  if (e.out16) e.out16[idx] = to_bf16(s);
}

// Raw buffer access (vector memory instructions with a uniform resource):
// 32-bit byte offsets, per lane plus uniform.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ float4 bload4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  typedef int i32x4 __attribute__((ext_vector_type(4)));
  const i32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
  return make_float4(__int_as_float(v[0]), __int_as_float(v[1]), __int_as_float(v[2]), __int_as_float(v[3]));
}
__device__ __forceinline__ void bstore4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float4 x) {
  typedef int i32x4 __attribute__((ext_vector_type(4)));
  const i32x4 v = {__float_as_int(x.x), __float_as_int(x.y), __float_as_int(x.z), __float_as_int(x.w)};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore_2x32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t lo,
                                            uint32_t hi) {
  typedef int i32x2 __attribute__((ext_vector_type(2)));
  const i32x2 v = {(int)lo, (int)hi};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, bf16 x) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, (int)voff, (int)soff, 0);
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// C = op(A)[M x K] op(B)[K x N] by 128 x 128 output tiles, split S =
// gridDim.x / (gx * gy) ways along K (split z takes every S-th K-tile):
//   op(A)[m][k] = ta ? A[k * lda + m] : A[m * lda + k]
//   op(B)[k][n] = tb ? B[n * ldb + k] : B[k * ldb + n]
// (op(B) is staged as its transpose, rows n, so both tiles are row x k.)
// Workgroups are dispatched to the 8 XCDs round-robin by linear index; the
// index is remapped so that consecutive logical tiles share an XCD, and the
// tile order runs fastest along the shorter grid side, so the tiles that read
// the same operand panel (the same K-chunk of a split product, the same row or
// column panel otherwise) meet in one L2.
template <int KIND, int KT>
__global__ __launch_bounds__(256) void k_gemm(const bf16* __restrict__ A, int lda, int ta, int veca,
                                              const bf16* __restrict__ B, int ldb, int tb, int vecb,
                                              float* __restrict__ C, int M, int N, int K, int gx,
                                              int gy, Epi e) {
  // operand tiles for the K-loop; the Adam epilogue reuses the same LDS to
  // stage the FP32 output tile (rows padded by 4 floats)
  constexpr int kTileBytes = (TM + TN) * (KT + 8) * 2;
  constexpr int kStageBytes = KIND == EPI_ADAM ? TM * (TN + 4) * 4 : 0;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kTileBytes > kStageBytes ? kTileBytes : kStageBytes];
  bf16(*As)[KT + 8] = reinterpret_cast<bf16(*)[KT + 8]>(smem);
  bf16(*Bs)[KT + 8] = reinterpret_cast<bf16(*)[KT + 8]>(smem + TM * (KT + 8) * 2);
  const int L = blockIdx.x, total = gridDim.x;
  const int full = total & ~7;
  const int Q = L < full ? (L & 7) * (full >> 3) + (L >> 3) : L;
  const int tiles = gx * gy;
  const int z = Q / tiles, tq = Q - z * tiles;
  int bx, by;
  if (gx <= gy) {
    bx = tq % gx;
    by = tq / gx;
  } else {
    by = tq % gy;
    bx = tq / gy;
  }
  const int m0 = by * TM, n0 = bx * TN;
  // K-tiles z, z + S, z + 2S, ... of the S-way split: the workgroups of one
  // output tile read adjacent K-tiles at about the same time, so each row of an
  // operand is fetched in long runs rather than one K-tile at a time
  const int S = total / tiles, kstep = S * KT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  TileRegs<KT> ra, rb;
  if (z * KT < K) {
    tile_load<KT>(A, lda, ta, veca, m0, M, z * KT, min(K, z * KT + KT), ra);
    tile_load<KT>(B, ldb, !tb, vecb, n0, N, z * KT, min(K, z * KT + KT), rb);
  }
  for (int k0 = z * KT; k0 < K; k0 += kstep) {
    tile_store<KT>(As, ta, ra);
    tile_store<KT>(Bs, !tb, rb);
    __syncthreads();
    const int kn = k0 + kstep;
    if (kn < K) {  // prefetch the next tile while the matrix cores work
      tile_load<KT>(A, lda, ta, veca, m0, M, kn, min(K, kn + KT), ra);
      tile_load<KT>(B, ldb, !tb, vecb, n0, N, kn, min(K, kn + KT), rb);
    }
#pragma unroll
    for (int kk = 0; kk < KT; kk += 16) {
      bf16x8 a[2], b[2];
      const int kb = (kk >> 3) + (lane >> 5);  // 16-byte block of k-values kk + 8 (lane / 32) ..
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm + i * 32 + (lane & 31);
        a[i] = *reinterpret_cast<const bf16x8*>(&As[row][swz<KT>(row, kb) * 8]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row = wn + j * 32 + (lane & 31);
        b[j] = *reinterpret_cast<const bf16x8*>(&Bs[row][swz<KT>(row, kb) * 8]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator element r of acc[i][j] holds output (row0 + i*32 + (r/4)*8 + r%4, col0 + j*32)
  const int row0 = m0 + wm + (lane >> 5) * 4, col0 = n0 + wn + (lane & 31);
  if constexpr (KIND == EPI_STORE) {
    float* Cz = C + (size_t)z * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + i * 32 + (r / 4) * 8 + (r % 4), col = col0 + j * 32;
          if (row < M && col < N) Cz[(size_t)row * N + col] = acc[i][j][r];
        }
  } else if constexpr (KIND == EPI_ACT) {
    // per 16-element group: the bias (one column) and the masks are loaded
    // before the first store, so the loads are all in flight together
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = col0 + j * 32;
        const float bv = (e.bias && col < N) ? e.bias[col] : 0.0f;
        float mk[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + i * 32 + (r / 4) * 8 + (r % 4);
          mk[r] = (e.mask && row < M && col < N) ? (float)e.mask[(size_t)row * N + col] : 1.0f;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + i * 32 + (r / 4) * 8 + (r % 4);
          if (row < M && col < N) {
            float s = acc[i][j][r] + bv;
            if (e.relu) s = fmaxf(s, 0.0f);
            if (!(mk[r] > 0.0f)) s = 0.0f;
            const size_t idx = (size_t)row * N + col;
            if (e.out32) e.out32[idx] = s;
            if (e.out16) e.out16[idx] = to_bf16(s);
          }
        }
      }
  } else if constexpr (KIND == EPI_ADAM) {
    // Element offsets are 32-bit (each weight matrix holds < 2^30 entries).
    // Interior tiles address the moments and weights through buffer resources:
    // one per-lane byte offset per column half plus a uniform row offset, so an
    // element costs no address registers.  The 64 accumulators go in 8 groups
    // of 8; the loads of group q+1 are issued before group q is updated and
    // stored, so they are in flight meanwhile.  Tiles that stick out of the
    // matrix take the guarded loop.
    if (e.vec4 && m0 + TM <= M && n0 + TN <= N) {
      // The tile goes through LDS so that each thread updates whole 16-byte
      // runs of a row: thread t takes columns 4 (t % 32) .. +3 of rows
      // t / 32 + 8 q (q < 16), in 4 groups of 4 rows; the first group's
      // weights and moments are requested before the tile is staged, and each
      // next group's before the current one is updated.
      float(*S)[TN + 4] = reinterpret_cast<float(*)[TN + 4]>(smem);
      const int lr = threadIdx.x >> 5, lc = (threadIdx.x & 31) * 4;
      // buffer resources: one per-lane offset, the row step as a uniform offset
      const uint32_t bytes = (uint32_t)M * (uint32_t)N * 4u;
      const __amdgpu_buffer_rsrc_t rp = make_rsrc(e.p, bytes), rm = make_rsrc(e.m, bytes),
                                   rv = make_rsrc(e.v, bytes), rw = make_rsrc(e.w16, bytes / 2);
      const uint32_t vo = (uint32_t)(m0 + lr) * (uint32_t)N + (uint32_t)(n0 + lc);  // element offset
      const uint32_t s8 = 8u * (uint32_t)N;                                          // elements per 8 rows
      float4 cp[4], cm[4], cv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cp[u] = bload4(rp, vo * 4u, (uint32_t)u * s8 * 4u);
        cm[u] = bload4(rm, vo * 4u, (uint32_t)u * s8 * 4u);
        cv[u] = bload4(rv, vo * 4u, (uint32_t)u * s8 * 4u);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r)
            S[wm + i * 32 + (r / 4) * 8 + (lane >> 5) * 4 + (r % 4)][wn + j * 32 + (lane & 31)] = acc[i][j][r];
      __syncthreads();
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float4 np_[4], nm[4], nv[4];
        if (g + 1 < 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t so = (uint32_t)(4 * (g + 1) + u) * s8 * 4u;
            np_[u] = bload4(rp, vo * 4u, so);
            nm[u] = bload4(rm, vo * 4u, so);
            nv[u] = bload4(rv, vo * 4u, so);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = 4 * g + u;
          const uint32_t so = (uint32_t)q * s8;
          const float4 g4 = *reinterpret_cast<const float4*>(&S[lr + 8 * q][lc]);
          const float gg[4] = {g4.x, g4.y, g4.z, g4.w};
          const float pp[4] = {cp[u].x, cp[u].y, cp[u].z, cp[u].w};
          const float mm[4] = {cm[u].x, cm[u].y, cm[u].z, cm[u].w};
          const float vv[4] = {cv[u].x, cv[u].y, cv[u].z, cv[u].w};
          float po[4], mo[4], vq[4];
          unsigned short wo[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            mo[k] = e.b1 * mm[k] + (1.0f - e.b1) * gg[k];
            vq[k] = e.b2 * vv[k] + (1.0f - e.b2) * gg[k] * gg[k];
            po[k] = pp[k] - e.lr * (mo[k] / e.c1) / (sqrtf(vq[k] / e.c2) + e.eps);
            wo[k] = __builtin_bit_cast(unsigned short, to_bf16(po[k]));
          }
          bstore4(rm, vo * 4u, so * 4u, make_float4(mo[0], mo[1], mo[2], mo[3]));
          bstore4(rv, vo * 4u, so * 4u, make_float4(vq[0], vq[1], vq[2], vq[3]));
          bstore4(rp, vo * 4u, so * 4u, make_float4(po[0], po[1], po[2], po[3]));
          bstore_2x32(rw, vo * 2u, so * 2u, (uint32_t)wo[0] | ((uint32_t)wo[1] << 16),
                      (uint32_t)wo[2] | ((uint32_t)wo[3] << 16));
        }
        if (g + 1 < 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            cp[u] = np_[u];
            cm[u] = nm[u];
            cv[u] = nv[u];
          }
        }
      }
    } else if (m0 + TM <= M && n0 + TN <= N) {
      const uint32_t bytes = (uint32_t)M * (uint32_t)N * 4u;
      const __amdgpu_buffer_rsrc_t rp = make_rsrc(e.p, bytes), rm = make_rsrc(e.m, bytes),
                                   rv = make_rsrc(e.v, bytes), rw = make_rsrc(e.w16, bytes / 2);
      const uint32_t un = (uint32_t)N;
      const uint32_t vbase = (uint32_t)row0 * un + (uint32_t)col0;  // element offset of (row0, col0)
      auto soff = [&](int q, int rr) {  // uniform element offset of group q, element rr
        const int i = q >> 2, h = q & 1;
        return (uint32_t)(i * 32 + h * 16 + (rr / 4) * 8 + (rr % 4)) * un;
      };
      float cp[8], cm[8], cv[8];
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const uint32_t s = soff(0, rr) * 4u, v = vbase * 4u;
        cp[rr] = bload(rp, v, s);
        cm[rr] = bload(rm, v, s);
        cv[rr] = bload(rv, v, s);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float np_[8], nm[8], nv[8];
        if (q + 1 < 8) {
          const uint32_t v = (vbase + (uint32_t)((((q + 1) >> 1) & 1) * 32)) * 4u;
#pragma unroll
          for (int rr = 0; rr < 8; ++rr) {
            const uint32_t s = soff(q + 1, rr) * 4u;
            np_[rr] = bload(rp, v, s);
            nm[rr] = bload(rm, v, s);
            nv[rr] = bload(rv, v, s);
          }
        }
        const int i = q >> 2, j = (q >> 1) & 1, h = q & 1;
        const uint32_t ve = vbase + (uint32_t)(j * 32);
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
          const uint32_t s = soff(q, rr);
          const float g = acc[i][j][h * 8 + rr];
          const float mi = e.b1 * cm[rr] + (1.0f - e.b1) * g;
          const float vi = e.b2 * cv[rr] + (1.0f - e.b2) * g * g;
          const float pi = cp[rr] - e.lr * (mi / e.c1) / (sqrtf(vi / e.c2) + e.eps);
          bstore(rm, ve * 4u, s * 4u, mi);
          bstore(rv, ve * 4u, s * 4u, vi);
          bstore(rp, ve * 4u, s * 4u, pi);
          bstore16(rw, ve * 2u, s * 2u, to_bf16(pi));
        }
        if (q + 1 < 8) {
#pragma unroll
          for (int rr = 0; rr < 8; ++rr) {
            cp[rr] = np_[rr];
            cm[rr] = nm[rr];
            cv[rr] = nv[rr];
          }
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = row0 + i * 32 + (r / 4) * 8 + (r % 4), col = col0 + j * 32;
            if (row < M && col < N) {
              const uint32_t o = (uint32_t)row * (uint32_t)N + (uint32_t)col;
              const float g = acc[i][j][r];
              const float mi = e.b1 * e.m[o] + (1.0f - e.b1) * g;
              const float vi = e.b2 * e.v[o] + (1.0f - e.b2) * g * g;
              const float pi = e.p[o] - e.lr * (mi / e.c1) / (sqrtf(vi / e.c2) + e.eps);
              e.m[o] = mi;
              e.v[o] = vi;
              e.p[o] = pi;
              e.w16[o] = to_bf16(pi);
            }
          }
    }
  } else {
    static_assert(KIND == EPI_MSE, "unknown epilogue");
    __shared__ float csum[2][TN];
    __shared__ double lsum[4];
    float cs[2] = {0.0f, 0.0f};
    double e2 = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = col0 + j * 32;
        const bool cok = col < N;
        const float bv = cok ? e.bias[col] : 0.0f;
        const float mu = (cok && e.tmu) ? e.tmu[col] : 0.0f;
        const float inv = (cok && e.tmu) ? e.tinv[col] : 1.0f;
        float tv[16];  // targets of the group, loaded before the first store
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + i * 32 + (r / 4) * 8 + (r % 4);
          tv[r] = (row < M && cok) ? e.t[(size_t)row * N + col] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + i * 32 + (r / 4) * 8 + (r % 4);
          if (row < M && cok) {
            const float vo = acc[i][j][r] + bv;
            const float tt = e.tmu ? (tv[r] - mu) * inv : tv[r];
            const float d = vo - tt;
            e2 += (double)d * (double)d;
            const float g = 2.0f * d * e.gscale;
            e.out16[(size_t)row * N + col] = to_bf16(g);
            cs[j] += g;
          }
        }
      }
    // column sums: the two row halves of the wave, then the two waves of a column half
#pragma unroll
    for (int j = 0; j < 2; ++j) cs[j] += __shfl_xor(cs[j], 32, 64);
    if (lane < 32) {
      csum[wave >> 1][wn + lane] = cs[0];
      csum[wave >> 1][wn + 32 + lane] = cs[1];
    }
    e2 = wave_sum64(e2);
    if (lane == 0) lsum[wave] = e2;
    __syncthreads();
    const int c = threadIdx.x;
    if (c < TN && n0 + c < N) e.colpart[(size_t)by * N + n0 + c] = csum[0][c] + csum[1][c];
    if (threadIdx.x == 0) e.lossp[(size_t)by * gx + bx] = ((lsum[0] + lsum[1]) + lsum[2]) + lsum[3];
  }
}

// Split products: out = sum_z part[z] in a fixed order, then the EPI_ACT use.
// The split partials of 4 consecutive elements per thread (16-byte loads, 8
// splits' loads in flight), summed in split order.
__global__ void k_epilogue(const float* __restrict__ part, int splits, int64_t MN, int N, Epi e) {
  const int64_t i = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= MN) return;
  if (MN % 4 == 0) {
    float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll 8
    for (int z = 0; z < splits; ++z) {
      const float4 p = *reinterpret_cast<const float4*>(part + (size_t)z * MN + i);
      s.x += p.x, s.y += p.y, s.z += p.z, s.w += p.w;
    }
    const float sv[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) epi_act(e, (size_t)(i + k), (int)((i + k) % N), sv[k]);
    return;
  }
  for (int64_t j = i; j < i + 4 && j < MN; ++j) {
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[(size_t)z * MN + j];
    epi_act(e, (size_t)j, (int)(j % N), s);
  }
}

__global__ void k_to_bf16(const float* __restrict__ in, bf16* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = to_bf16(in[i]);
}

// Standardized BF16 input: (u - mean) / scale per feature (identity when mean
// is null).  Four consecutive elements per thread (one 16-byte load, one
// 8-byte store) when vec4 (n % 4 == 0 and both arrays 16 / 8-byte aligned).
__global__ void k_in_norm(const float* __restrict__ in, const float* __restrict__ mu,
                          const float* __restrict__ inv_scale, int64_t n, int d, int vec4, bf16* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec4) {
    if (4 * t >= n) return;
    const float4 v4 = reinterpret_cast<const float4*>(in)[t];
    float v[4] = {v4.x, v4.y, v4.z, v4.w};
    if (mu) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int j = (int)((4 * t + k) % d);
        v[k] = (v[k] - mu[j]) * inv_scale[j];
      }
    }
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    bf16x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = to_bf16(v[k]);
    reinterpret_cast<bf16x4*>(out)[t] = o;
    return;
  }
  if (t >= n) return;
  float v = in[t];
  if (mu) {
    const int j = (int)(t % d);
    v = (v - mu[j]) * inv_scale[j];
  }
  out[t] = to_bf16(v);
}

// Network output in the caller's units: z * scale + mean per feature.
__global__ void k_out_denorm(const float* __restrict__ z, const float* __restrict__ mu,
                             const float* __restrict__ scale, int64_t n, int d, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = z[i];
  if (mu) {
    const int j = (int)(i % d);
    v = v * scale[j] + mu[j];
  }
  out[i] = v;
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double scale, float* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(red[0] * scale);
}

// Column sums of a [rows x cols] FP32 matrix (bias gradients), fixed order.
__global__ void k_colsum(const float* __restrict__ g, int rows, int cols, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; ++r) s += g[(size_t)r * cols + c];
  out[c] = s;
}

// First level of a column sum over many rows: workgroup (x, y) adds rows
// [y * chunk, (y + 1) * chunk) of 64 columns, wave w taking every fourth row
// from w with four independent partial sums; part[y][col] = the waves' sums in
// order.  Fixed order: deterministic.
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ g, int rows, int cols, int chunk,
                                                     float* __restrict__ part) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  if (c < cols) {
    int r = r0 + wave;
    for (; r + 12 < r1; r += 16) {
      s0 += g[(size_t)r * cols + c];
      s1 += g[(size_t)(r + 4) * cols + c];
      s2 += g[(size_t)(r + 8) * cols + c];
      s3 += g[(size_t)(r + 12) * cols + c];
    }
    for (; r < r1; r += 4) s0 += g[(size_t)r * cols + c];
  }
  red[wave][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (wave == 0 && c < cols) part[(size_t)blockIdx.y * cols + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Adam step on FP32 parameters outside the weight matrices (whose updates run
// inside their gradient products): three segments [o, o + n) in one launch,
// the three bias vectors.
__global__ void k_adam3(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, int64_t o0, int64_t n0, int64_t o1, int64_t n1, int64_t o2,
                        int64_t n2, float lr, float b1, float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t j;
  if (i < n0) {
    j = o0 + i;
  } else if ((i -= n0) < n1) {
    j = o1 + i;
  } else if ((i -= n1) < n2) {
    j = o2 + i;
  } else {
    return;
  }
  const float gi = g[j];
  const float mi = b1 * m[j] + (1.0f - b1) * gi;
  const float vi = b2 * v[j] + (1.0f - b2) * gi * gi;
  m[j] = mi;
  v[j] = vi;
  p[j] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline dim3 lin(int64_t n, int t = 256) { return dim3((unsigned)((n + t - 1) / t)); }

}  // namespace

struct pdcs_mlp_s {
  int64_t din = 0, w = 0, dout = 0, np = 0;
  int64_t off_w1 = 0, off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0;
  DBuf params, grads, adam_m, adam_v, wbf;  // wbf: BF16 W1 | W2 | W3
  // feature standardization (in: mean, 1/scale; out: mean, scale, 1/scale)
  DBuf in_mu, in_inv, out_mu, out_sc, out_inv;
  bool norm_in = false, norm_out = false;
  const float* imu() const { return norm_in ? in_mu.as<float>() : nullptr; }
  const float* omu() const { return norm_out ? out_mu.as<float>() : nullptr; }
  int64_t step = 0;
  int64_t cap = 0;    // batch capacity of the activation buffers
  int64_t last = 0;   // batch of the last forward / gradient / training call
  bool have_grad_acts = false;  // the last call computed the backward activations
  // activations: BF16 operands of the products (input, h1, h2, dL/dv, dL/dz2,
  // dL/dz1), the FP32 output, FP32 masked hidden gradients (bias sums), the
  // loss gradient's per-row-tile column sums and the loss partials
  DBuf u16, h1_16, h2_16, vout, dv16, dz16a, dz16b, dh, colpart, part, cspart, lossp, lossv;
  size_t part_bytes = 0, cs_bytes = 0;
  hipStream_t stream = nullptr;

  bf16* W1() const { return wbf.as<bf16>(); }
  bf16* W2() const { return wbf.as<bf16>() + w * din; }
  bf16* W3() const { return wbf.as<bf16>() + w * din + w * w; }
  float* P(int64_t off) const { return params.as<float>() + off; }
  float* G(int64_t off) const { return grads.as<float>() + off; }
  float* Mo(int64_t off) const { return adam_m.as<float>() + off; }
  float* Vo(int64_t off) const { return adam_v.as<float>() + off; }

  void refresh_bf16(hipStream_t s) {
    k_to_bf16<<<lin(w * din), 256, 0, s>>>(P(off_w1), W1(), w * din);
    k_to_bf16<<<lin(w * w), 256, 0, s>>>(P(off_w2), W2(), w * w);
    k_to_bf16<<<lin(dout * w), 256, 0, s>>>(P(off_w3), W3(), dout * w);
  }

  void ensure(int64_t B) {
    if (B <= cap) return;
    cap = B;
    const int64_t rt = (B + TM - 1) / TM;  // row tiles of the output layer
    u16.alloc(B * din * 2);
    h1_16.alloc(B * w * 2);
    h2_16.alloc(B * w * 2);
    vout.alloc(B * dout * 4);
    dv16.alloc(B * dout * 2);
    dz16a.alloc(B * w * 2);
    dz16b.alloc(B * w * 2);
    dh.alloc(B * w * 4);
    colpart.alloc(rt * dout * 4);
    lossp.alloc(rt * ((dout + TN - 1) / TN) * 8);
    lossv.alloc(8);
  }

  // op(A)[M x K] op(B)[K x N] with epilogue `kind`.  Products whose output tiles
  // alone cannot fill the chip are split along K (EPI_STORE / EPI_ACT only);
  // the partials are then summed in a fixed order.  EPI_STORE writes e.out32.
  // The tile depth is 64 for K-ranges of 128 or more (128-deep tiles halve the
  // steps of long ranges but double the LDS, and measured 2% slower per step
  // at batch 256), 32 below.
  void gemm(int kind, const bf16* A, int lda, int ta, const bf16* Bm, int ldb, int tb, int M, int N, int K,
            Epi e, hipStream_t s) {
    const int gx = (N + TN - 1) / TN, gy = (M + TM - 1) / TM;
    const int tiles = gx * gy;
    if (kind == EPI_ADAM) e.vec4 = adam_vec4(e, N);
    // (products of a few tiles split down to K-ranges of 128: a handful of
    // workgroups walking the whole K serially would leave the chip idle)
    int splits = 1;
    const int min_range = tiles < 64 ? 128 : 512;
    if (kind == EPI_STORE || kind == EPI_ACT)
      while (tiles * splits < 512 && K / (splits * 2) >= min_range) splits *= 2;
    int kchunk = (K + splits - 1) / splits;
    const int kt = kchunk >= 128 ? 64 : 32;
    kchunk = (kchunk + kt - 1) / kt * kt;
    splits = (K + kchunk - 1) / kchunk;
    if (splits < 1) splits = 1;
    if (splits > 1) {
      const size_t need = (size_t)splits * M * N * 4;
      if (need > part_bytes) {
        part.alloc(need);
        part_bytes = need;
      }
      launch(EPI_STORE, kt, A, lda, ta, Bm, ldb, tb, part.as<float>(), M, N, K, gx, gy, splits, e, s);
      k_epilogue<<<lin(((int64_t)M * N + 3) / 4), 256, 0, s>>>(part.as<float>(), splits, (int64_t)M * N, N, e);
      return;
    }
    launch(kind, kt, A, lda, ta, Bm, ldb, tb, kind == EPI_STORE ? e.out32 : nullptr, M, N, K, gx, gy, 1, e, s);
  }

  template <int KIND>
  static void launch_kt(int kt, dim3 grid, const bf16* A, int lda, int ta, int veca, const bf16* Bm, int ldb, int tb,
                        int vecb, float* C, int M, int N, int K, int gx, int gy, const Epi& e,
                        hipStream_t s) {
    if (kt == 64)
      k_gemm<KIND, 64><<<grid, 256, 0, s>>>(A, lda, ta, veca, Bm, ldb, tb, vecb, C, M, N, K, gx, gy, e);
    else
      k_gemm<KIND, 32><<<grid, 256, 0, s>>>(A, lda, ta, veca, Bm, ldb, tb, vecb, C, M, N, K, gx, gy, e);
  }

  static void launch(int kind, int kt, const bf16* A, int lda, int ta, const bf16* Bm, int ldb, int tb, float* C, int M,
                     int N, int K, int gx, int gy, int splits, const Epi& e, hipStream_t s) {
    // 16-byte vector loads need 16-byte aligned operands with row strides in whole vectors
    const int veca = ((uintptr_t)A % 16 == 0 && lda % 8 == 0) ? 1 : 0;
    const int vecb = ((uintptr_t)Bm % 16 == 0 && ldb % 8 == 0) ? 1 : 0;
    const dim3 grid((unsigned)(gx * gy * splits));
    switch (kind) {
      case EPI_STORE:
        launch_kt<EPI_STORE>(kt, grid, A, lda, ta, veca, Bm, ldb, tb, vecb, C, M, N, K, gx, gy, e, s);
        break;
      case EPI_ACT:
        launch_kt<EPI_ACT>(kt, grid, A, lda, ta, veca, Bm, ldb, tb, vecb, C, M, N, K, gx, gy, e, s);
        break;
      case EPI_ADAM:
        launch_kt<EPI_ADAM>(kt, grid, A, lda, ta, veca, Bm, ldb, tb, vecb, C, M, N, K, gx, gy, e, s);
        break;
      default:
        launch_kt<EPI_MSE>(kt, grid, A, lda, ta, veca, Bm, ldb, tb, vecb, C, M, N, K, gx, gy, e, s);
    }
  }

  // Column sums of g [rows x cols] into out (fixed order): one pass for a few
  // rows, else 32-row partial sums by many workgroups, then their sum.
  void colsum(const float* g, int64_t rows, int64_t cols, float* out, hipStream_t s) {
    if (rows <= 32) {
      k_colsum<<<lin(cols), 256, 0, s>>>(g, (int)rows, (int)cols, out);
      return;
    }
    const int chunk = 32;
    const int64_t ny = (rows + chunk - 1) / chunk;
    const size_t need = (size_t)ny * cols * 4;
    if (need > cs_bytes) {
      cspart.alloc(need);
      cs_bytes = need;
    }
    k_colsum_part<<<dim3((unsigned)((cols + 63) / 64), (unsigned)ny), 256, 0, s>>>(g, (int)rows, (int)cols, chunk,
                                                                                  cspart.as<float>());
    k_colsum<<<lin(cols), 256, 0, s>>>(cspart.as<float>(), (int)ny, (int)cols, out);
  }

  static Epi act(const float* bias, int relu, const bf16* mask, float* out32, bf16* out16) {
    Epi e;
    e.bias = bias;
    e.relu = relu;
    e.mask = mask;
    e.out32 = out32;
    e.out16 = out16;
    return e;
  }

  // Adam (step `step`, learning rate lr) on the weights at offset off: the
  // weight-gradient product's epilogue when `adam`, else the gradient is stored.
  Epi wgrad(bool adam, int64_t off, bf16* w16, float lr) const {
    Epi e;
    if (!adam) {
      e.out32 = G(off);
      return e;
    }
    e.p = P(off);
    e.m = Mo(off);
    e.v = Vo(off);
    e.w16 = w16;
    e.lr = lr;
    e.b1 = 0.9f;
    e.b2 = 0.999f;
    e.eps = 1e-8f;
    e.c1 = 1.0f - std::pow(e.b1, (float)step);
    e.c2 = 1.0f - std::pow(e.b2, (float)step);
    return e;
  }

  // 16-byte runs of weight rows: the Adam epilogue's staged path
  static int adam_vec4(const Epi& e, int64_t N) {
    return (N % 4 == 0 && (uintptr_t)e.p % 16 == 0 && (uintptr_t)e.m % 16 == 0 && (uintptr_t)e.v % 16 == 0 &&
            (uintptr_t)e.w16 % 8 == 0)
               ? 1
               : 0;
  }

  // Standardized BF16 input and the two hidden layers (BF16, after ReLU).
  void hidden(const float* in, int64_t B, hipStream_t s) {
    ensure(B);
    last = B;
    const int64_t n = B * din;
    const int vec4 = (n % 4 == 0 && (uintptr_t)in % 16 == 0 && (uintptr_t)u16.p % 8 == 0) ? 1 : 0;
    k_in_norm<<<lin(vec4 ? n / 4 : n), 256, 0, s>>>(in, imu(), in_inv.as<float>(), n, (int)din, vec4, u16.as<bf16>());
    gemm(EPI_ACT, u16.as<bf16>(), din, 0, W1(), din, 1, B, w, din, act(P(off_b1), 1, nullptr, nullptr, h1_16.as<bf16>()),
         s);
    gemm(EPI_ACT, h1_16.as<bf16>(), w, 0, W2(), w, 1, B, w, w, act(P(off_b2), 1, nullptr, nullptr, h2_16.as<bf16>()),
         s);
  }

  void forward(const float* in, int64_t B, hipStream_t s) {
    hidden(in, B, s);
    have_grad_acts = false;
    gemm(EPI_ACT, h2_16.as<bf16>(), w, 0, W3(), w, 1, B, dout, w, act(P(off_b3), 0, nullptr, vout.as<float>(), nullptr),
         s);
  }

  // Forward and backward of the mean squared error; the weight gradients are
  // stored in `grads`, or, when `adam`, applied as an Adam step inside the
  // weight-gradient products (each layer's BF16 weights are read by the
  // backward product before its own update rewrites them).  Bias gradients go
  // to `grads` either way; the loss stays on the device (lossv), summed from
  // its partials only when `need_loss`.
  void train(const float* in, const float* target, int64_t B, bool adam, float lr, bool need_loss, hipStream_t s) {
    hidden(in, B, s);
    have_grad_acts = true;
    const int64_t n = B * dout;
    const int rt = (int)((B + TM - 1) / TM), ct = (int)((dout + TN - 1) / TN);
    // output layer fused with the loss: dv16 = BF16 dL/dv, column sums, loss partials
    Epi mse;
    mse.bias = P(off_b3);
    mse.t = target;
    mse.tmu = omu();
    mse.tinv = out_inv.as<float>();
    mse.gscale = 1.0f / (float)n;
    mse.out16 = dv16.as<bf16>();
    mse.colpart = colpart.as<float>();
    mse.lossp = lossp.as<double>();
    gemm(EPI_MSE, h2_16.as<bf16>(), w, 0, W3(), w, 1, B, dout, w, mse, s);
    if (need_loss) k_sum_parts<<<1, 256, 0, s>>>(lossp.as<double>(), rt * ct, 1.0 / (double)n, lossv.as<float>());
    colsum(colpart.as<float>(), rt, dout, G(off_b3), s);
    // layer 3: dZ2 = (dV W3) * (h2 > 0) before W3 changes, then dW3 = dV^T H2
    gemm(EPI_ACT, dv16.as<bf16>(), dout, 0, W3(), w, 0, B, w, dout,
         act(nullptr, 0, h2_16.as<bf16>(), dh.as<float>(), dz16a.as<bf16>()), s);
    gemm(adam ? EPI_ADAM : EPI_STORE, dv16.as<bf16>(), dout, 1, h2_16.as<bf16>(), w, 0, dout, w, B,
         wgrad(adam, off_w3, W3(), lr), s);
    colsum(dh.as<float>(), B, w, G(off_b2), s);
    // layer 2: dZ1 = (dZ2 W2) * (h1 > 0), then dW2 = dZ2^T H1
    gemm(EPI_ACT, dz16a.as<bf16>(), w, 0, W2(), w, 0, B, w, w,
         act(nullptr, 0, h1_16.as<bf16>(), dh.as<float>(), dz16b.as<bf16>()), s);
    gemm(adam ? EPI_ADAM : EPI_STORE, dz16a.as<bf16>(), w, 1, h1_16.as<bf16>(), w, 0, w, w, B,
         wgrad(adam, off_w2, W2(), lr), s);
    colsum(dh.as<float>(), B, w, G(off_b1), s);
    // layer 1: dW1 = dZ1^T U
    gemm(adam ? EPI_ADAM : EPI_STORE, dz16b.as<bf16>(), w, 1, u16.as<bf16>(), din, 0, w, din, B,
         wgrad(adam, off_w1, W1(), lr), s);
    if (adam) {  // the biases: FP32 only, one small pass
      const Epi e = wgrad(true, off_b1, nullptr, lr);
      k_adam3<<<lin(2 * w + dout), 256, 0, s>>>(params.as<float>(), grads.as<float>(), adam_m.as<float>(),
                                                 adam_v.as<float>(), off_b1, w, off_b2, w, off_b3, dout, lr, e.b1,
                                                 e.b2, e.eps, e.c1, e.c2);
    }
  }
};

extern "C" {

int pdcs_mlp_create(int64_t d_in, int64_t width, int64_t d_out, uint64_t seed, pdcs_mlp* out) {
  try {
    if (!out || d_in < 1 || width < 1 || d_out < 1 || d_in > (1 << 26) || d_out > (1 << 26) || width > 8192 ||
        width * d_in >= ((int64_t)1 << 30) || width * d_out >= ((int64_t)1 << 30))
      throw Error(PDCS_ERR_INVALID_ARG, "bad MLP sizes (each weight matrix must hold fewer than 2^30 entries)");
    *out = nullptr;
    auto net = new pdcs_mlp_s();
    std::unique_ptr<pdcs_mlp_s> guard(net);
    net->din = d_in;
    net->w = width;
    net->dout = d_out;
    net->off_w1 = 0;
    net->off_b1 = width * d_in;
    net->off_w2 = net->off_b1 + width;
    net->off_b2 = net->off_w2 + width * width;
    net->off_w3 = net->off_b2 + width;
    net->off_b3 = net->off_w3 + d_out * width;
    net->np = net->off_b3 + d_out;
    HIP_OK(hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking));
    // Glorot-uniform weights, zero biases, from a seeded host generator
    std::vector<float> p(net->np, 0.0f);
    std::mt19937_64 gen(seed);
    auto fill = [&](int64_t off, int64_t fan_out, int64_t fan_in) {
      const float a = std::sqrt(6.0f / (float)(fan_in + fan_out));
      std::uniform_real_distribution<float> U(-a, a);
      for (int64_t i = 0; i < fan_out * fan_in; ++i) p[off + i] = U(gen);
    };
    fill(net->off_w1, width, d_in);
    fill(net->off_w2, width, width);
    fill(net->off_w3, d_out, width);
    net->params.alloc(net->np * 4);
    net->grads.alloc(net->np * 4);
    net->adam_m.alloc(net->np * 4);
    net->adam_v.alloc(net->np * 4);
    net->wbf.alloc((width * d_in + width * width + d_out * width) * 2);
    HIP_OK(hipMemcpy(net->params.p, p.data(), net->np * 4, hipMemcpyHostToDevice));
    std::vector<float> z(net->np, 0.0f);
    HIP_OK(hipMemcpy(net->adam_m.p, z.data(), net->np * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(net->adam_v.p, z.data(), net->np * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(net->grads.p, z.data(), net->np * 4, hipMemcpyHostToDevice));
    net->refresh_bf16(net->stream);
    HIP_OK(hipStreamSynchronize(net->stream));
    *out = guard.release();
    return PDCS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return PDCS_ERR_OOM;
  }
}

// the caller's stream; NULL is the HIP null stream (ordered with the caller's
// default-stream work), never the library's own non-blocking stream
static hipStream_t pick(pdcs_mlp, void* stream) { return (hipStream_t)stream; }

int pdcs_mlp_forward(pdcs_mlp net, const float* in_dev, float* out_dev, int64_t batch, void* stream) {
  try {
    if (!net || !in_dev || !out_dev || batch < 1) throw Error(PDCS_ERR_INVALID_ARG, "bad forward arguments");
    hipStream_t s = pick(net, stream);
    net->forward(in_dev, batch, s);
    k_out_denorm<<<lin(batch * net->dout), 256, 0, s>>>(net->vout.as<float>(), net->omu(), net->out_sc.as<float>(),
                                                       batch * net->dout, (int)net->dout, out_dev);
    HIP_OK(hipGetLastError());
    return PDCS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

int pdcs_mlp_gradients(pdcs_mlp net, const float* in_dev, const float* target_dev, int64_t batch, float* grad_dev,
                       float* loss_out, void* stream) {
  try {
    if (!net || !in_dev || !target_dev || batch < 1) throw Error(PDCS_ERR_INVALID_ARG, "bad gradient arguments");
    hipStream_t s = pick(net, stream);
    net->train(in_dev, target_dev, batch, false, 0.0f, loss_out != nullptr, s);
    if (grad_dev) HIP_OK(hipMemcpyAsync(grad_dev, net->grads.p, net->np * 4, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipGetLastError());
    float loss = 0.0f;
    if (loss_out) HIP_OK(hipMemcpyAsync(&loss, net->lossv.p, 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (loss_out) *loss_out = loss;
    return PDCS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

int pdcs_mlp_train_step(pdcs_mlp net, const float* in_dev, const float* target_dev, int64_t batch, float lr,
                        float* loss_out, void* stream) {
  try {
    if (!net || !in_dev || !target_dev || batch < 1 || !(lr > 0.0f))
      throw Error(PDCS_ERR_INVALID_ARG, "bad train arguments");
    hipStream_t s = pick(net, stream);
    net->step += 1;
    net->train(in_dev, target_dev, batch, true, lr, loss_out != nullptr, s);
    HIP_OK(hipGetLastError());
    if (loss_out) {  // without a loss pointer the step stays asynchronous on `stream`
      float loss = 0.0f;
      HIP_OK(hipMemcpyAsync(&loss, net->lossv.p, 4, hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      *loss_out = loss;
    }
    return PDCS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

int pdcs_mlp_activation(pdcs_mlp net, int64_t which, float* host_out, int64_t count) {
  try {
    if (!net || !host_out || which < 0 || which > 5) throw Error(PDCS_ERR_INVALID_ARG, "bad activation arguments");
    if (net->last < 1 || (which >= 3 && !net->have_grad_acts))
      throw Error(PDCS_ERR_INVALID_ARG, "no activation of that kind from the last call");
    const int64_t B = net->last;
    const bf16* src[6] = {net->u16.as<bf16>(), net->h1_16.as<bf16>(), net->h2_16.as<bf16>(),
                          net->dv16.as<bf16>(), net->dz16a.as<bf16>(), net->dz16b.as<bf16>()};
    const int64_t dim[6] = {net->din, net->w, net->w, net->dout, net->w, net->w};
    if (count != B * dim[which]) throw Error(PDCS_ERR_INVALID_ARG, "count must be batch x features");
    HIP_OK(hipDeviceSynchronize());
    std::vector<uint16_t> raw(count);
    HIP_OK(hipMemcpy(raw.data(), src[which], count * 2, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < count; ++i) {
      const uint32_t bits = (uint32_t)raw[i] << 16;
      std::memcpy(&host_out[i], &bits, 4);
    }
    return PDCS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

int pdcs_mlp_num_params(pdcs_mlp net, int64_t* count) {
  if (!net || !count) {
    set_last_error("null argument");
    return PDCS_ERR_INVALID_ARG;
  }
  *count = net->np;
  return PDCS_OK;
}

int pdcs_mlp_get_params(pdcs_mlp net, float* params_host) {
  try {
    if (!net || !params_host) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(params_host, net->params.p, net->np * 4, hipMemcpyDeviceToHost));
    return PDCS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

int pdcs_mlp_set_normalization(pdcs_mlp net, const float* in_mean, const float* in_scale, const float* out_mean,
                               const float* out_scale) {
  try {
    if (!net) throw Error(PDCS_ERR_INVALID_ARG, "null network");
    if ((in_mean == nullptr) != (in_scale == nullptr) || (out_mean == nullptr) != (out_scale == nullptr))
      throw Error(PDCS_ERR_INVALID_ARG, "mean and scale must be given together");
    auto check = [](const float* mu, const float* sc, int64_t d) {
      for (int64_t j = 0; j < d; ++j)
        if (!std::isfinite(mu[j]) || !std::isfinite(sc[j]) || !(sc[j] > 0.0f))
          throw Error(PDCS_ERR_INVALID_ARG, "means must be finite and scales finite and positive");
    };
    HIP_OK(hipDeviceSynchronize());
    if (in_mean) {
      check(in_mean, in_scale, net->din);
      std::vector<float> inv(net->din);
      for (int64_t j = 0; j < net->din; ++j) inv[j] = 1.0f / in_scale[j];
      net->in_mu.alloc(net->din * 4);
      net->in_inv.alloc(net->din * 4);
      HIP_OK(hipMemcpy(net->in_mu.p, in_mean, net->din * 4, hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(net->in_inv.p, inv.data(), net->din * 4, hipMemcpyHostToDevice));
    }
    net->norm_in = in_mean != nullptr;
    if (out_mean) {
      check(out_mean, out_scale, net->dout);
      std::vector<float> inv(net->dout);
      for (int64_t j = 0; j < net->dout; ++j) inv[j] = 1.0f / out_scale[j];
      net->out_mu.alloc(net->dout * 4);
      net->out_sc.alloc(net->dout * 4);
      net->out_inv.alloc(net->dout * 4);
      HIP_OK(hipMemcpy(net->out_mu.p, out_mean, net->dout * 4, hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(net->out_sc.p, out_scale, net->dout * 4, hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(net->out_inv.p, inv.data(), net->dout * 4, hipMemcpyHostToDevice));
    }
    net->norm_out = out_mean != nullptr;
    return PDCS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

int pdcs_mlp_set_params(pdcs_mlp net, const float* params_host) {
  try {
    if (!net || !params_host) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    HIP_OK(hipMemcpy(net->params.p, params_host, net->np * 4, hipMemcpyHostToDevice));
    net->refresh_bf16(net->stream);
    HIP_OK(hipStreamSynchronize(net->stream));
    return PDCS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

void pdcs_mlp_destroy(pdcs_mlp net) {
  if (!net) return;
  if (net->stream) (void)hipStreamDestroy(net->stream);
  delete net;
}

}  // extern "C"
