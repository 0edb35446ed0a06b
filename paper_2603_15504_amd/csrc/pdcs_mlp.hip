// Warm-start MLP for families of LPs: v = W3 relu(W2 relu(W1 u + b1) + b2) + b3.
//
// BF16 weights and activations feed the matrix cores (v_mfma_f32_32x32x16_bf16
// on gfx950) with FP32 accumulation; an FP32 master copy of the weights takes
// the Adam updates.  Every GEMM is C = op(A) op(B) with row-major operands,
// tiled 128 x 128 x 32 per workgroup (four wavefronts of 64 x 64), split along
// K when M x N alone cannot fill the chip; split partials are summed in a fixed
// order by the epilogue kernels (bias, ReLU, BF16 copies), so results are
// deterministic.
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

constexpr int TM = 128, TN = 128, TK = 32, LDK = TK + 8;  // LDS row stride: 80 B (16 B aligned)

__device__ __forceinline__ bf16 to_bf16(float v) { return (bf16)v; }

// One operand tile (128 rows of op(X) x TK) staged through registers.  op(X)
// row r, column k lives at X[k * ld + r] when trans, else X[r * ld + k].  Each
// thread owns two 8-element vectors of the tile: along k when the source is
// k-contiguous (not trans), along r otherwise.  vec: the launch guarantees
// 16-byte alignment of the source and ld % 8 == 0, so whole vectors inside the
// bounds load with one 16-byte access; anything else loads element by element.
struct TileRegs {
  bf16x8 v[2];
};

__device__ __forceinline__ void tile_load(const bf16* __restrict__ X, int ld, int trans, int vec, int r0, int R,
                                          int k0, int kend, TileRegs& t) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + q * 256;  // vector index in the tile: 512 vectors of 8
    int rr, kk;
    if (!trans) {
      rr = e / (TK / 8);
      kk = (e % (TK / 8)) * 8;
    } else {
      kk = e / (TM / 8);
      rr = (e % (TM / 8)) * 8;
    }
    const int gr = r0 + rr, gk = k0 + kk;
    bf16x8 v;
    if (!trans) {
      if (vec && gr < R && gk + 8 <= kend) {
        v = *reinterpret_cast<const bf16x8*>(X + (size_t)gr * ld + gk);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (gr < R && gk + i < kend) ? X[(size_t)gr * ld + gk + i] : to_bf16(0.0f);
      }
    } else {
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

__device__ __forceinline__ void tile_store(bf16 (*S)[LDK], int trans, const TileRegs& t) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + q * 256;
    if (!trans) {
      const int rr = e / (TK / 8), kk = (e % (TK / 8)) * 8;
      *reinterpret_cast<bf16x8*>(&S[rr][kk]) = t.v[q];
    } else {
      const int kk = e / (TM / 8), rr = (e % (TM / 8)) * 8;
#pragma unroll
      for (int i = 0; i < 8; ++i) S[rr + i][kk] = t.v[q][i];
    }
  }
}

// C_part[z] = op(A)[m0:m0+128, kz] * op(B)[kz, n0:n0+128]
//   op(A)[m][k] = ta ? A[k * lda + m] : A[m * lda + k]
//   op(B)[k][n] = tb ? B[n * ldb + k] : B[k * ldb + n]
// (op(B) is staged as its transpose, rows n, so both tiles are row x k.)
__global__ __launch_bounds__(256) void k_gemm(const bf16* __restrict__ A, int lda, int ta, int veca,
                                              const bf16* __restrict__ B, int ldb, int tb, int vecb,
                                              float* __restrict__ C, int M, int N, int K, int kchunk) {
  __shared__ __attribute__((aligned(16))) bf16 As[TM][LDK];
  __shared__ __attribute__((aligned(16))) bf16 Bs[TN][LDK];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  TileRegs ra, rb;
  if (kbeg < kend) {
    tile_load(A, lda, ta, veca, m0, M, kbeg, kend, ra);
    tile_load(B, ldb, !tb, vecb, n0, N, kbeg, kend, rb);
  }
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    tile_store(As, ta, ra);
    tile_store(Bs, !tb, rb);
    __syncthreads();
    if (k0 + TK < kend) {  // prefetch the next tile while the matrix cores work
      tile_load(A, lda, ta, veca, m0, M, k0 + TK, kend, ra);
      tile_load(B, ldb, !tb, vecb, n0, N, k0 + TK, kend, rb);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 16) {
      bf16x8 a[2], b[2];
      const int ko = kk + (lane >> 5) * 8;
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + i * 32 + (lane & 31)][ko]);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + j * 32 + (lane & 31)][ko]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float* Cz = C + (size_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + i * 32 + (r / 4) * 8 + (lane >> 5) * 4 + (r % 4);
        const int col = n0 + wn + j * 32 + (lane & 31);
        if (row < M && col < N) Cz[(size_t)row * N + col] = acc[i][j][r];
      }
}

// out = sum_z part[z] (+ bias[col]) then optional ReLU; FP32 and/or BF16 copies.
// grad_mask: when non-null, out = sum * (mask > 0) (derivative of ReLU at mask).
__global__ void k_epilogue(const float* __restrict__ part, int splits, int64_t MN, int N,
                           const float* __restrict__ bias, int relu, const float* __restrict__ grad_mask,
                           float* __restrict__ out32, bf16* __restrict__ out16) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MN) return;
  float s = 0.0f;
  for (int z = 0; z < splits; ++z) s += part[(size_t)z * MN + i];
  if (bias) s += bias[i % N];
  if (relu) s = fmaxf(s, 0.0f);
  if (grad_mask) s = grad_mask[i] > 0.0f ? s : 0.0f;
  if (out32) out32[i] = s;
  if (out16) out16[i] = to_bf16(s);
}

__global__ void k_to_bf16(const float* __restrict__ in, bf16* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = to_bf16(in[i]);
}

// Standardized BF16 input: (u - mean) / scale per feature (identity when mean is null).
__global__ void k_in_norm(const float* __restrict__ in, const float* __restrict__ mu,
                          const float* __restrict__ inv_scale, int64_t n, int d, bf16* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = in[i];
  if (mu) {
    const int j = (int)(i % d);
    v = (v - mu[j]) * inv_scale[j];
  }
  out[i] = to_bf16(v);
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

// Per-block partial sums of (v - t)^2 with t standardized like the outputs
// ((t - mean) / scale per feature when mean is non-null); dv = 2 (v - t) / count;
// BF16 copy of dv.
__global__ void k_mse(const float* __restrict__ v, const float* __restrict__ t, int64_t n, float scale,
                      const float* __restrict__ tmu, const float* __restrict__ tinv, int d,
                      float* __restrict__ dv, bf16* __restrict__ dv16, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (i < n) {
    float ti = t[i];
    if (tmu) {
      const int j = (int)(i % d);
      ti = (ti - tmu[j]) * tinv[j];
    }
    const float d = v[i] - ti;
    e2 = (double)d * (double)d;
    const float g = 2.0f * d * scale;
    dv[i] = g;
    dv16[i] = to_bf16(g);
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
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

// Adam step on the FP32 master weights; BF16 copies of the weight matrices.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
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
  int64_t cap = 0;  // batch capacity of the activation buffers
  DBuf u16, z1, h1_16, z2, h2_16, vout, dv, dv16, dh, dz16a, dz16b, part, lossp, lossv;
  size_t part_bytes = 0;
  hipStream_t stream = nullptr;

  bf16* W1() const { return wbf.as<bf16>(); }
  bf16* W2() const { return wbf.as<bf16>() + w * din; }
  bf16* W3() const { return wbf.as<bf16>() + w * din + w * w; }
  float* P(int64_t off) const { return params.as<float>() + off; }
  float* G(int64_t off) const { return grads.as<float>() + off; }

  void refresh_bf16(hipStream_t s) {
    k_to_bf16<<<lin(w * din), 256, 0, s>>>(P(off_w1), W1(), w * din);
    k_to_bf16<<<lin(w * w), 256, 0, s>>>(P(off_w2), W2(), w * w);
    k_to_bf16<<<lin(dout * w), 256, 0, s>>>(P(off_w3), W3(), dout * w);
  }

  void ensure(int64_t B) {
    if (B <= cap) return;
    cap = B;
    u16.alloc(B * din * 2);
    z1.alloc(B * w * 4);
    h1_16.alloc(B * w * 2);
    z2.alloc(B * w * 4);
    h2_16.alloc(B * w * 2);
    vout.alloc(B * dout * 4);
    dv.alloc(B * dout * 4);
    dv16.alloc(B * dout * 2);
    dh.alloc(B * w * 4);
    dz16a.alloc(B * w * 2);
    dz16b.alloc(B * w * 2);
    lossp.alloc(((B * dout + 255) / 256) * 8);
    lossv.alloc(8);
  }

  // C[M x N] (+bias, relu | grad mask) <- op(A) op(B); split along K as needed.
  void gemm(const bf16* A, int lda, int ta, const bf16* Bm, int ldb, int tb, int M, int N, int K,
            const float* bias, int relu, const float* mask, float* out32, bf16* out16, hipStream_t s) {
    const int gx = (N + TN - 1) / TN, gy = (M + TM - 1) / TM;
    int splits = 1;
    const int tiles = gx * gy;
    while (tiles * splits < 512 && K / (splits * 2) >= 256) splits *= 2;
    int kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + TK - 1) / TK * TK;
    splits = (K + kchunk - 1) / kchunk;
    // unsplit products with a plain FP32 result are written in place
    const bool direct = splits == 1 && !bias && !relu && !mask && out32 && !out16;
    const size_t need = (size_t)splits * M * N * 4;
    if (!direct && need > part_bytes) {
      part.alloc(need);
      part_bytes = need;
    }
    // 16-byte vector loads need 16-byte aligned operands with row strides in whole vectors
    const int veca = ((uintptr_t)A % 16 == 0 && lda % 8 == 0) ? 1 : 0;
    const int vecb = ((uintptr_t)Bm % 16 == 0 && ldb % 8 == 0) ? 1 : 0;
    k_gemm<<<dim3(gx, gy, splits), 256, 0, s>>>(A, lda, ta, veca, Bm, ldb, tb, vecb,
                                               direct ? out32 : part.as<float>(), M, N, K, kchunk);
    if (!direct)
      k_epilogue<<<lin((int64_t)M * N), 256, 0, s>>>(part.as<float>(), splits, (int64_t)M * N, N, bias, relu,
                                                     mask, out32, out16);
  }

  void forward(const float* in, int64_t B, hipStream_t s) {
    ensure(B);
    k_in_norm<<<lin(B * din), 256, 0, s>>>(in, imu(), in_inv.as<float>(), B * din, (int)din, u16.as<bf16>());
    gemm(u16.as<bf16>(), din, 0, W1(), din, 1, B, w, din, P(off_b1), 1, nullptr, z1.as<float>(), h1_16.as<bf16>(), s);
    gemm(h1_16.as<bf16>(), w, 0, W2(), w, 1, B, w, w, P(off_b2), 1, nullptr, z2.as<float>(), h2_16.as<bf16>(), s);
    gemm(h2_16.as<bf16>(), w, 0, W3(), w, 1, B, dout, w, P(off_b3), 0, nullptr, vout.as<float>(), nullptr, s);
  }

  // Gradients of the mean squared error into `grads`; loss (host) returned.
  float backward(const float* target, int64_t B, hipStream_t s) {
    const int64_t n = B * dout;
    const int nb = (int)((n + 255) / 256);
    k_mse<<<nb, 256, 0, s>>>(vout.as<float>(), target, n, 1.0f / (float)n, omu(), out_inv.as<float>(), (int)dout,
                             dv.as<float>(), dv16.as<bf16>(), lossp.as<double>());
    k_sum_parts<<<1, 256, 0, s>>>(lossp.as<double>(), nb, 1.0 / (double)n, lossv.as<float>());
    // layer 3: dW3 = dV^T H2, db3 = colsum dV, dH2 = dV W3, dZ2 = dH2 * (z2 > 0)
    gemm(dv16.as<bf16>(), dout, 1, h2_16.as<bf16>(), w, 0, dout, w, B, nullptr, 0, nullptr, G(off_w3), nullptr, s);
    k_colsum<<<lin(dout), 256, 0, s>>>(dv.as<float>(), B, dout, G(off_b3));
    gemm(dv16.as<bf16>(), dout, 0, W3(), w, 0, B, w, dout, nullptr, 0, z2.as<float>(), dh.as<float>(),
         dz16a.as<bf16>(), s);
    // layer 2
    gemm(dz16a.as<bf16>(), w, 1, h1_16.as<bf16>(), w, 0, w, w, B, nullptr, 0, nullptr, G(off_w2), nullptr, s);
    k_colsum<<<lin(w), 256, 0, s>>>(dh.as<float>(), B, w, G(off_b2));
    gemm(dz16a.as<bf16>(), w, 0, W2(), w, 0, B, w, w, nullptr, 0, z1.as<float>(), dh.as<float>(), dz16b.as<bf16>(),
         s);
    // layer 1
    gemm(dz16b.as<bf16>(), w, 1, u16.as<bf16>(), din, 0, w, din, B, nullptr, 0, nullptr, G(off_w1), nullptr, s);
    k_colsum<<<lin(w), 256, 0, s>>>(dh.as<float>(), B, w, G(off_b1));
    float loss = 0.0f;
    HIP_OK(hipMemcpyAsync(&loss, lossv.p, 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return loss;
  }
};

extern "C" {

int pdcs_mlp_create(int64_t d_in, int64_t width, int64_t d_out, uint64_t seed, pdcs_mlp* out) {
  try {
    if (!out || d_in < 1 || width < 1 || d_out < 1 || d_in > (1 << 26) || d_out > (1 << 26) || width > 8192)
      throw Error(PDCS_ERR_INVALID_ARG, "bad MLP sizes");
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
    net->forward(in_dev, batch, s);
    const float loss = net->backward(target_dev, batch, s);
    if (grad_dev) HIP_OK(hipMemcpyAsync(grad_dev, net->grads.p, net->np * 4, hipMemcpyDeviceToDevice, s));
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
    net->forward(in_dev, batch, s);
    const float loss = net->backward(target_dev, batch, s);
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - std::pow(b1, (float)net->step), c2 = 1.0f - std::pow(b2, (float)net->step);
    k_adam<<<lin(net->np), 256, 0, s>>>(net->params.as<float>(), net->grads.as<float>(), net->adam_m.as<float>(),
                                        net->adam_v.as<float>(), net->np, lr, b1, b2, eps, c1, c2);
    net->refresh_bf16(s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    if (loss_out) *loss_out = loss;
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
