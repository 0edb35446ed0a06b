// Host side of the PDCS LP solver: problem validation and CSR transposition,
// block-diagonal batch packing, wavefront-tile schedules, the chunked solve
// loop (hipGraph replay of check_every trials plus one restart check), and
// the C ABI declared in include/pdcs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pdcs.h"
#include "pdcs_engine.h"
#include "pdcs_launch.h"

using namespace pdcs;

namespace pdcs {

thread_local std::string g_err;

void set_last_error(const std::string& msg) { g_err = msg; }

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------
void DBuf::alloc(size_t b) {
  release();
  if (b == 0) b = 256;
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error(e == hipErrorOutOfMemory ? PDCS_ERR_OOM : PDCS_ERR_HIP,
                std::string("hipMalloc(") + std::to_string(b) + "): " + hipGetErrorString(e));
  }
  bytes = b;
}

void DBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

template <typename T>
static void upload(DBuf& d, const std::vector<T>& h) {
  d.alloc(h.size() * sizeof(T));
  if (!h.empty()) HIP_OK(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------------------
// Problem validation and transposition
// ---------------------------------------------------------------------------
int64_t HostProblem::cone_rows() const {
  int64_t rows = 3 * (n_exp + n_dexp);
  for (int32_t d : soc) rows += d;
  return rows;
}

void HostProblem::build(int64_t m_, int64_t n_, int64_t mz, const int64_t* row_ptr, const int32_t* col_idx,
                        const double* val, const double* h_, const double* c_, const double* l_,
                        const double* u_, int64_t n_soc, const int64_t* soc_dims, int64_t n_exp_,
                        int64_t n_dexp_) {
  if (m_ < 0 || n_ < 1) throw Error(PDCS_ERR_INVALID_ARG, "need m >= 0 and n >= 1");
  if (mz < 0 || mz > m_) throw Error(PDCS_ERR_INVALID_ARG, "m_zero must lie in [0, m]");
  if (n_soc < 0 || (n_soc > 0 && !soc_dims)) throw Error(PDCS_ERR_INVALID_ARG, "bad second-order-cone list");
  if (n_exp_ < 0 || n_dexp_ < 0) throw Error(PDCS_ERR_INVALID_ARG, "negative number of exponential-cone blocks");
  soc.clear();
  int64_t soc_rows = 0;
  for (int64_t q = 0; q < n_soc; ++q) {
    if (soc_dims[q] < 1) throw Error(PDCS_ERR_INVALID_ARG, "second-order-cone dimensions must be >= 1");
    soc_rows += soc_dims[q];
    if (soc_rows > m_ - mz) throw Error(PDCS_ERR_INVALID_ARG, "second-order-cone rows exceed the rows after m_zero");
    soc.push_back((int32_t)soc_dims[q]);
  }
  if (n_exp_ > (m_ - mz - soc_rows) / 3 || n_dexp_ > (m_ - mz - soc_rows) / 3 - n_exp_)
    throw Error(PDCS_ERR_INVALID_ARG, "cone rows exceed the rows after m_zero");
  n_exp = n_exp_;
  n_dexp = n_dexp_;
  if (m_ >= INT32_MAX || n_ >= INT32_MAX) throw Error(PDCS_ERR_SIZE, "m and n must be < 2^31 - 1");
  if (!row_ptr) throw Error(PDCS_ERR_INVALID_ARG, "row_ptr is null");
  if (!c_) throw Error(PDCS_ERR_INVALID_ARG, "c is null");
  if (m_ > 0 && !h_) throw Error(PDCS_ERR_INVALID_ARG, "h is null");
  if (row_ptr[0] != 0) throw Error(PDCS_ERR_INVALID_ARG, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < m_; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) throw Error(PDCS_ERR_INVALID_ARG, "row_ptr is not nondecreasing");
  const int64_t nz = row_ptr[m_];
  if (nz >= INT32_MAX) throw Error(PDCS_ERR_SIZE, "nnz must be < 2^31 - 1");
  if (nz > 0 && (!col_idx || !val)) throw Error(PDCS_ERR_INVALID_ARG, "col_idx or val is null");
  m = m_;
  n = n_;
  m_zero = mz;
  nnz = nz;
  rp.resize(m + 1);
  for (int64_t i = 0; i <= m; ++i) rp[i] = (int32_t)row_ptr[i];
  ci.assign(col_idx, col_idx + nz);
  v.assign(val, val + nz);
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      const int32_t c = col_idx[p];
      if (c < 0 || c >= n) throw Error(PDCS_ERR_INVALID_ARG, "column index out of range");
      if (p > row_ptr[i] && c <= col_idx[p - 1])
        throw Error(PDCS_ERR_INVALID_ARG, "column indices must increase strictly within a row");
      if (!std::isfinite(val[p])) throw Error(PDCS_ERR_INVALID_ARG, "non-finite matrix value");
    }
  }
  h.assign(m, 0.0);
  for (int64_t i = 0; i < m; ++i) {
    if (!std::isfinite(h_[i])) throw Error(PDCS_ERR_INVALID_ARG, "non-finite h");
    h[i] = h_[i];
  }
  c.assign(c_, c_ + n);
  l.assign(n, 0.0);
  u.assign(n, std::numeric_limits<double>::infinity());
  for (int64_t j = 0; j < n; ++j) {
    if (!std::isfinite(c[j])) throw Error(PDCS_ERR_INVALID_ARG, "non-finite c");
    if (l_) l[j] = l_[j];
    if (u_) u[j] = u_[j];
    if (std::isnan(l[j]) || std::isnan(u[j])) throw Error(PDCS_ERR_INVALID_ARG, "NaN bound");
    if (l[j] > u[j]) throw Error(PDCS_ERR_INVALID_ARG, "l > u");
    if (l[j] == std::numeric_limits<double>::infinity() || u[j] == -std::numeric_limits<double>::infinity())
      throw Error(PDCS_ERR_INVALID_ARG, "l = +inf or u = -inf");
  }
  // Transpose by a stable counting sort: rows stay ascending inside each column.
  cp.assign(n + 1, 0);
  for (int64_t p = 0; p < nz; ++p) cp[ci[p] + 1]++;
  for (int64_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
  ri.resize(nz);
  vt.resize(nz);
  std::vector<int32_t> fill(cp.begin(), cp.end() - 1);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      const int32_t q = fill[ci[p]]++;
      ri[q] = (int32_t)i;
      vt[q] = v[p];
    }
}

// ---------------------------------------------------------------------------
// Schedules
// ---------------------------------------------------------------------------
static int lanes_for(int rows) {
  int L = 64;
  while (L > 1 && L * rows > 64) L >>= 1;
  return L;
}

static int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

// Wavefront tiles over the rows of a CSR structure (instance-aligned):
// a row longer than 64 * iter_max is a tile of its own (the wavefront strides
// over it); otherwise consecutive rows share a tile as long as each row's
// group of lanes needs at most iter_max passes.  Tiles are then grouped into
// workgroups of about block_work units (nonzeros plus 4 per row).
void TileSet::build(const std::vector<int32_t>& ptr, const std::vector<int64_t>& inst_r0, const Schedule& s,
                    const std::vector<char>* active) {
  std::vector<int32_t> t0, t1, tlg, bt0, bt1, binst, iblk0;
  const int64_t cap = 64LL * s.iter_max;
  const int B = (int)inst_r0.size() - 1;
  iblk0.push_back(0);
  for (int b = 0; b < B; ++b) {
    int64_t r = inst_r0[b];
    const int64_t end = (active && !(*active)[b]) ? r : inst_r0[b + 1];
    const size_t first = t0.size();
    while (r < end) {
      const int64_t len0 = ptr[r + 1] - ptr[r];
      if (len0 > cap) {
        t0.push_back((int32_t)r);
        t1.push_back((int32_t)(r + 1));
        tlg.push_back(6);
        ++r;
        continue;
      }
      const int64_t start = r;
      int R = 0;
      int64_t maxlen = 0;
      while (r < end && R < 64) {
        const int64_t len = ptr[r + 1] - ptr[r];
        if (len > cap) break;
        const int nR = R + 1;
        const int64_t nmax = std::max(maxlen, len);
        const int L = lanes_for(nR);
        if ((nmax + L - 1) / L > s.iter_max) break;
        R = nR;
        maxlen = nmax;
        ++r;
      }
      t0.push_back((int32_t)start);
      t1.push_back((int32_t)r);
      tlg.push_back(ilog2(lanes_for(R)));
    }
    size_t i = first;
    const size_t tend = t0.size();
    while (i < tend) {
      size_t j = i;
      int64_t acc = 0;
      while (j < tend) {
        const int64_t w = (int64_t)(ptr[t1[j]] - ptr[t0[j]]) + 4LL * (t1[j] - t0[j]);
        if (j > i && acc + w > s.block_nnz) break;
        acc += w;
        ++j;
      }
      bt0.push_back((int32_t)i);
      bt1.push_back((int32_t)j);
      binst.push_back(b);
      i = j;
    }
    iblk0.push_back((int32_t)bt0.size());
  }
  ntiles = (int)t0.size();
  nblk = (int)bt0.size();
  h_bt0 = bt0;
  h_bt1 = bt1;
  h_t0 = t0;
  h_t1 = t1;
  h_binst = binst;
  upload(row0, t0);
  upload(row1, t1);
  upload(lg, tlg);
  upload(btile0, bt0);
  upload(btile1, bt1);
  upload(binst_d, binst);
  upload(iblk0_d, iblk0);
}

Tiles TileSet::view() const {
  Tiles t;
  t.tile_row0 = row0.as<int32_t>();
  t.tile_row1 = row1.as<int32_t>();
  t.tile_lg = lg.as<int32_t>();
  t.blk_tile0 = btile0.as<int32_t>();
  t.blk_tile1 = btile1.as<int32_t>();
  t.blk_inst = binst_d.as<int32_t>();
  t.inst_blk0 = iblk0_d.as<int32_t>();
  t.nblk = nblk;
  return t;
}

static int threads_per_row(int R) {
  int T = 64;
  while (T > 1 && T * R > 256) T >>= 1;
  return T;
}

void RowBlockSet::build(const std::vector<int32_t>& ptr, const std::vector<int64_t>& inst_r0, int red_max,
                        const std::vector<char>* active) {
  std::vector<int32_t> a, e, bi, iblk0;
  const int B = (int)inst_r0.size() - 1;
  const int64_t cap = kRowBlockCap;
  iblk0.push_back(0);
  for (int b = 0; b < B; ++b) {
    int64_t r = inst_r0[b];
    const int64_t end = (active && !(*active)[b]) ? r : inst_r0[b + 1];
    while (r < end) {
      const int64_t len0 = ptr[r + 1] - ptr[r];
      if (len0 > cap) {
        a.push_back((int32_t)r);
        e.push_back((int32_t)(r + 1));
        bi.push_back(b);
        ++r;
        continue;
      }
      const int64_t start = r;
      int64_t nnz = 0, maxlen = 0;
      int R = 0;
      while (r < end && R < 4096) {
        const int64_t len = ptr[r + 1] - ptr[r];
        if (len > cap || nnz + len > cap) break;
        const int nR = R + 1;
        const int64_t nmax = std::max(maxlen, len);
        int64_t cost;
        if (nR <= 256) {
          const int T = threads_per_row(nR);
          cost = (nmax + T - 1) / T;
        } else {
          cost = ((nR + 255) / 256) * nmax;
        }
        if (nR > 1 && cost > red_max) break;
        R = nR;
        nnz += len;
        maxlen = nmax;
        ++r;
      }
      a.push_back((int32_t)start);
      e.push_back((int32_t)r);
      bi.push_back(b);
    }
    iblk0.push_back((int32_t)a.size());
  }
  nblk = (int)a.size();
  h_binst = bi;
  h_iblk0 = iblk0;
  upload(r0, a);
  upload(r1, e);
  upload(binst_d, bi);
  upload(iblk0_d, iblk0);
}

RowBlocks RowBlockSet::view() const {
  RowBlocks r;
  r.blk_row0 = r0.as<int32_t>();
  r.blk_row1 = r1.as<int32_t>();
  r.blk_inst = binst_d.as<int32_t>();
  r.inst_blk0 = iblk0_d.as<int32_t>();
  r.nblk = nblk;
  return r;
}

void RangeSet::build(const std::vector<int64_t>& inst_off, int per_block, const std::vector<char>* active) {
  std::vector<int32_t> st, en, bi, iblk0, s0, s1;
  const int B = (int)inst_off.size() - 1;
  const bool cones = soc && !soc->empty();
  size_t q = 0;  // next cone block (cone blocks are in row order)
  iblk0.push_back(0);
  for (int b = 0; b < B; ++b) {
    const int64_t stop = (active && !(*active)[b]) ? inst_off[b] : inst_off[b + 1];
    if (cones)
      while (q < soc->r0.size() && soc->r0[q] < inst_off[b]) ++q;
    int64_t s = inst_off[b];
    while (s < stop) {
      int64_t e = std::min<int64_t>(s + per_block, stop);
      const size_t q0 = q;
      if (cones) {
        // a range ends at a cone block boundary: blocks starting inside it are
        // taken whole, and a range that reaches a block's rows takes the block;
        // a range holds at most cone_cap blocks, so that the blocks' tasks
        // spread over the waves of many workgroups
        while (q < soc->r0.size() && soc->r0[q] < e && soc->r0[q] < stop) {
          if (q - q0 == (size_t)cone_cap) {
            e = soc->r0[q];
            break;
          }
          e = std::max<int64_t>(e, (int64_t)soc->r0[q] + soc->dim[q]);
          ++q;
        }
      }
      st.push_back((int32_t)s);
      en.push_back((int32_t)e);
      bi.push_back(b);
      s0.push_back((int32_t)q0);
      s1.push_back((int32_t)q);
      s = e;
    }
    if (cones)  // cone blocks of an inactive instance
      while (q < soc->r0.size() && soc->r0[q] < inst_off[b + 1]) ++q;
    iblk0.push_back((int32_t)st.size());
  }
  nblk = (int)st.size();
  h_iblk0 = iblk0;
  upload(start, st);
  upload(end, en);
  upload(binst_d, bi);
  upload(iblk0_d, iblk0);
  if (cones) {
    upload(soc0_d, s0);
    upload(soc1_d, s1);
  } else {
    soc0_d.release();
    soc1_d.release();
  }
}

Ranges RangeSet::view() const {
  Ranges r;
  r.blk_start = start.as<int32_t>();
  r.blk_end = end.as<int32_t>();
  r.blk_inst = binst_d.as<int32_t>();
  r.inst_blk0 = iblk0_d.as<int32_t>();
  const bool cones = soc && !soc->empty() && soc0_d.p;
  r.blk_soc0 = cones ? soc0_d.as<int32_t>() : nullptr;
  r.blk_soc1 = cones ? soc1_d.as<int32_t>() : nullptr;
  r.soc_r0 = cones ? soc->r0_d.as<int32_t>() : nullptr;
  r.soc_dim = cones ? soc->dim_d.as<int32_t>() : nullptr;
  r.soc_kind = cones ? soc->kind_d.as<int8_t>() : nullptr;
  r.nblk = nblk;
  return r;
}

// ---------------------------------------------------------------------------
// Band tiles
// ---------------------------------------------------------------------------
namespace {
struct BandBuild {
  std::vector<int32_t> start, row0, nrows, used, col0, panel, tinst, run_start, run_row, run_ext, ext, src;
  std::vector<uint32_t> pk;
  std::vector<int64_t> work;  // entries per band-tile
  std::vector<size_t> sizes() const {
    return {start.size(), row0.size(), nrows.size(), col0.size(), panel.size(), run_start.size(), run_row.size(),
            run_ext.size(), ext.size(), src.size(), pk.size(), work.size(), used.size(), tinst.size()};
  }
  void truncate(const std::vector<size_t>& z) {
    start.resize(z[0]);
    row0.resize(z[1]);
    nrows.resize(z[2]);
    col0.resize(z[3]);
    panel.resize(z[4]);
    run_start.resize(z[5]);
    run_row.resize(z[6]);
    run_ext.resize(z[7]);
    ext.resize(z[8]);
    src.resize(z[9]);
    pk.resize(z[10]);
    work.resize(z[11]);
    used.resize(z[12]);
    tinst.resize(z[13]);
  }
};

// Entries of rows [r0, r1) with gathered index in window p, sorted by gathered
// index (rotated to start at window offset `shift`), with accumulator slots
// assigned per 64-entry group; false if the band needs more than
// kBandSlots - 1 slots.
bool build_band_tile(int64_t r0, int64_t r1, int p, int64_t c0, int64_t c1, int64_t shift, int inst,
                     const std::vector<int32_t>& ptr, const std::vector<int32_t>& idx, std::vector<int32_t>& stamp,
                     std::vector<int32_t>& next, int32_t& gid, BandBuild& out) {
  // sort key: the index relative to the window start, rotated by `shift`, so
  // that tiles of one window sweep it from different starting points
  const int64_t W = std::max<int64_t>(1, c1 - c0);
  std::vector<std::pair<uint64_t, int32_t>> E;
  for (int64_t r = r0; r < r1; ++r)
    for (int64_t q = ptr[r]; q < ptr[r + 1]; ++q) {
      const int64_t c = idx[q];
      if (c >= c0 && c < c1) {
        const int64_t key = (c - c0 + W - shift) % W;
        E.push_back({((uint64_t)key << 20) | (uint64_t)(r - r0), (int32_t)q});
      }
    }
  std::sort(E.begin(), E.end());
  const int nr = (int)(r1 - r0);
  std::fill(next.begin(), next.end(), -1);
  int nxt = nr;
  const size_t base = out.pk.size();
  out.start.push_back((int32_t)base);
  out.row0.push_back((int32_t)r0);
  out.nrows.push_back(nr);
  out.col0.push_back((int32_t)c0);
  out.panel.push_back(p);
  out.tinst.push_back(inst);
  for (size_t k = 0; k < E.size(); ++k) {
    if (k % kWave == 0) ++gid;
    const uint32_t col = (uint32_t)(((int64_t)(E[k].first >> 20) + shift) % W);
    int s = (int)(E[k].first & 0xFFFFFu);
    while (stamp[s] == gid) {
      if (next[s] < 0) {
        if (nxt >= kBandSlots - 1) return false;
        next[s] = nxt++;
      }
      s = next[s];
    }
    stamp[s] = gid;
    out.pk.push_back((col << kBandSlotBits) | (uint32_t)s);
    out.src.push_back(E[k].second);
  }
  const size_t q = (size_t)kBandUnroll * kWave;
  while ((out.pk.size() - base) % q) {
    out.pk.push_back((uint32_t)(kBandSlots - 1));
    out.src.push_back(-1);
  }
  for (int r = 0; r < nr; ++r) {
    if (next[r] < 0) continue;
    out.run_row.push_back(r);
    for (int e = next[r]; e >= 0; e = next[e]) out.ext.push_back(e);
    out.run_ext.push_back((int32_t)out.ext.size());
  }
  out.run_start.push_back((int32_t)out.run_row.size());
  out.work.push_back((int64_t)E.size());
  out.used.push_back(nxt);
  return true;
}
}  // namespace

void BandSet::build(const std::vector<int64_t>& r0s, const std::vector<int64_t>& g0s, const std::vector<int32_t>& ptr,
                    const std::vector<int32_t>& idx, const BandSchedule& bs) {
  const int NB = (int)r0s.size() - 1;
  R = r0s[NB];
  const int64_t G = g0s[NB];
  const int64_t wmax = (int64_t)1 << kBandColBits;
  // windows per instance; P is the batch's largest count
  std::vector<int> Pb(NB);
  P = 1;
  for (int b = 0; b < NB; ++b) {
    Pb[b] = (int)std::max<int64_t>(1, (g0s[b + 1] - g0s[b] + wmax - 1) / wmax);
    P = std::max(P, Pb[b]);
  }
  // band height: as tall as possible (better gather locality, fewer
  // iterations' worth of fixed cost per tile) while keeping at least about
  // bs.min_tiles (384 by default) band-tiles to spread over the 256 CUs.  On
  // the m = 2e5, n = 5e5 LP (nnz 5e6) a trial took 0.131 / 0.105 / 0.112 /
  // 0.130 ms with at least 192 / 384 / 768 / 1536 tiles; larger problems reach
  // 8192-row bands anyway.
  auto tiles_for = [&](int64_t rb) {
    int64_t t = 0;
    for (int b = 0; b < NB; ++b) t += ((r0s[b + 1] - r0s[b] + rb - 1) / rb) * P;
    return t;
  };
  int64_t rb = std::min<int64_t>(bs.rows, kBandRows);
  while (rb > 256 && tiles_for(rb) < bs.min_tiles) rb /= 2;
  band_rows = (int)rb;
  BandBuild bb;
  bb.run_start.push_back(0);
  bb.run_ext.push_back(0);
  std::vector<int32_t> stamp(kBandSlots, -1), next(kBandSlots, -1);
  int32_t gid = 0;
  std::vector<std::pair<int64_t, int64_t>> bands;  // row ranges, split on slot overflow
  // Per instance of a batch, bands no taller than needed for about
  // bs.entry_cap (32 Ki) entries per window, so that tiles of very different instances stay
  // comparable in work and the tiles still running at the end of a launch
  // are short (a single instance keeps the height chosen above).  On the 512-LP batch the batched
  // G x_hat took 0.284 ms with 64 Ki, 0.251 with 32 Ki, 0.275 with 16 Ki.
  for (int b = 0; b < NB; ++b) {
    const int64_t gb = g0s[b], wb = g0s[b + 1] - g0s[b];
    const int64_t W = std::max<int64_t>(1, (wb + Pb[b] - 1) / Pb[b]);
    int64_t rbb = rb;
    if (NB > 1) {
      const int64_t rows_b = r0s[b + 1] - r0s[b];
      const int64_t nnz_b = rows_b > 0 ? (int64_t)ptr[r0s[b + 1]] - ptr[r0s[b]] : 0;
      const double per_row = rows_b > 0 ? (double)nnz_b / (double)rows_b / (double)Pb[b] : 1.0;
      while (rbb > 256 && (double)rbb * per_row > (double)bs.entry_cap) rbb /= 2;
    }
    // Band boundaries with about equal entries (the count of rbb-row bands,
    // each at most rbb rows): with heavy-tailed row lengths, fixed heights
    // leave some bands far heavier than others, and the heaviest sets the time.
    std::vector<std::pair<int64_t, int64_t>> cuts;
    {
      const int64_t ra = r0s[b], re = r0s[b + 1];
      const int64_t nbands = (re - ra + rbb - 1) / rbb;
      const double target = nbands > 0 ? (double)((int64_t)ptr[re] - ptr[ra]) / (double)nbands : 0.0;
      int64_t r = ra;
      while (r < re) {
        int64_t e = r + 1;
        while (e < re && e - r < rbb && (double)((int64_t)ptr[e + 1] - ptr[r]) <= target) ++e;
        cuts.push_back({r, e});
        r = e;
      }
    }
    std::vector<std::pair<int64_t, int64_t>> todo(cuts.rbegin(), cuts.rend());
    while (!todo.empty()) {
      const auto br = todo.back();
      todo.pop_back();
      const std::vector<size_t> save = bb.sizes();
      bool ok = true;
      for (int p = 0; p < P && ok; ++p) {
        // window p of instance b (empty beyond its own window count)
        const int64_t c0 = p < Pb[b] ? gb + std::min<int64_t>(wb, p * W) : gb;
        const int64_t c1 = p < Pb[b] ? gb + std::min<int64_t>(wb, (p + 1) * W) : gb;
        // Tiles of one window run at the same time and at about the same pace:
        // started at the same index they would all gather from the same few
        // KiB of the window, a handful of L2 channels, at any moment.  Each
        // band starts its sweep at its own offset, spread over the window.
        const int64_t rows_b = std::max<int64_t>(1, r0s[b + 1] - r0s[b]);
        const int64_t shift = c1 > c0 ? (int64_t)((double)(br.first - r0s[b]) / (double)rows_b * (double)(c1 - c0)) % (c1 - c0) : 0;
        ok = build_band_tile(br.first, br.second, p, c0, c1, shift, b, ptr, idx, stamp, next, gid, bb);
      }
      if (ok) {
        bands.push_back(br);
        continue;
      }
      if (br.second - br.first <= 1) throw Error(PDCS_ERR_SIZE, "band tile slot overflow");
      bb.truncate(save);
      const int64_t mid = br.first + (br.second - br.first) / 2;
      todo.push_back({mid, br.second});
      todo.push_back({br.first, mid});
    }
  }
  bb.start.push_back((int32_t)bb.pk.size());
  if (bb.pk.size() >= (size_t)INT32_MAX) throw Error(PDCS_ERR_SIZE, "band tiles exceed 2^31 entries");
  ntile = (int)bands.size() * P;
  nent = (int64_t)bb.pk.size();
  // workgroups: kBandWaves consecutive bands of one window; windows routed to
  // XCDs (slot s runs on XCD s % 8), window p to the XCDs x with x % P == p
  const int nb = (int)bands.size();
  const int ng = (nb + kBandWaves - 1) / kBandWaves;
  std::vector<int32_t> grp;
  std::vector<std::vector<int32_t>> per_xcd(8);
  std::vector<int64_t> load(8, 0);
  // In a batch, every tile of an instance goes to one XCD (largest instances
  // first, each to the least loaded XCD), so that the instance's gathered
  // vector is fetched into one L2 only; instances holding more than 1/16 of
  // the work are spread over the XCDs like a single problem.
  std::vector<int> inst_xcd(NB, -1);
  if (NB > 1) {
    std::vector<int64_t> iw(NB, 0);
    int64_t total = 0;
    for (int t = 0; t < ntile; ++t) {
      iw[bb.tinst[t]] += bb.work[t] + 1;
      total += bb.work[t] + 1;
    }
    std::vector<int> order(NB);
    for (int b = 0; b < NB; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return iw[a] > iw[c]; });
    for (int b : order) {
      if (iw[b] * 16 > total) continue;
      int x = 0;
      for (int q = 1; q < 8; ++q)
        if (load[q] < load[x]) x = q;
      inst_xcd[b] = x;
      load[x] += iw[b];
    }
  }
  for (int p = 0; p < P; ++p)
    for (int g = 0; g < ng; ++g) {
      const int gi = (int)(grp.size() / kBandWaves);
      int64_t work = 0;
      int first = -1;
      for (int w = 0; w < kBandWaves; ++w) {
        const int b = g * kBandWaves + w;
        const int t = b < nb ? b * P + p : -1;
        grp.push_back(t);
        if (t >= 0) {
          work += bb.work[t];
          if (first < 0) first = t;
        }
      }
      int best = first >= 0 && NB > 1 ? inst_xcd[bb.tinst[first]] : -1;
      if (best < 0) {
        for (int x = 0; x < 8; ++x) {
          const bool serves = NB > 1 || (P >= 8 ? (p % 8 == x) : (x % P == p));
          if (serves && (best < 0 || load[x] < load[best])) best = x;
        }
        load[best] += work + 1;
      }
      per_xcd[best].push_back(gi);
    }
  size_t depth = 0;
  for (auto& l : per_xcd) depth = std::max(depth, l.size());
  std::vector<int32_t> sl(depth * 8, -1);
  for (int x = 0; x < 8; ++x)
    for (size_t k = 0; k < per_xcd[x].size(); ++k) sl[k * 8 + x] = per_xcd[x][k];
  nslot = (int)sl.size();
  // every index the kernel reads, checked before anything reaches the device
  auto fail = [](const char* what) { throw Error(PDCS_ERR_STATE, std::string("band layout check: ") + what); };
  if ((int)bb.start.size() != ntile + 1 || (int)bb.run_start.size() != ntile + 1 || (int)bb.used.size() != ntile)
    fail("tile tables");
  if (bb.run_ext.size() != bb.run_row.size() + 1 || bb.src.size() != bb.pk.size()) fail("run tables");
  for (int32_t g : sl)
    if (g >= (int32_t)(grp.size() / kBandWaves)) fail("slot table");
  for (int32_t t : grp)
    if (t >= ntile) fail("group table");
  for (int t = 0; t < ntile; ++t) {
    const int64_t e0 = bb.start[t], e1 = bb.start[t + 1];
    if (e1 < e0 || (e1 - e0) % ((int64_t)kBandUnroll * kWave)) fail("tile padding");
    if (bb.nrows[t] < 0 || bb.nrows[t] > kBandRows || (int64_t)bb.row0[t] + bb.nrows[t] > R) fail("tile rows");
    if (bb.panel[t] < 0 || bb.panel[t] >= P || bb.col0[t] < 0) fail("tile window");
    if (bb.used[t] < bb.nrows[t] || bb.used[t] > kBandSlots - 1) fail("tile slots");
    const int ti = bb.tinst[t];
    if (ti < 0 || ti >= NB || bb.row0[t] < r0s[ti] || (int64_t)bb.row0[t] + bb.nrows[t] > r0s[ti + 1]) fail("tile instance");
    if (bb.start[t + 1] > bb.start[t] && (bb.col0[t] < g0s[ti] || bb.col0[t] >= g0s[ti + 1])) fail("tile window instance");
    if (e1 > e0 && bb.col0[t] >= G) fail("tile window start");
    for (int64_t e = e0; e < e1; ++e) {
      const uint32_t slot_e = bb.pk[e] & ((1u << kBandSlotBits) - 1u);
      const int64_t col = (int64_t)bb.col0[t] + (bb.pk[e] >> kBandSlotBits);
      if ((slot_e >= (uint32_t)bb.used[t] && slot_e != (uint32_t)(kBandSlots - 1)) || col >= g0s[ti + 1]) fail("entry");
      if (bb.src[e] >= 0 && (bb.src[e] >= ptr[R] || idx[bb.src[e]] != col)) fail("entry source");
    }
    for (int32_t r = bb.run_start[t]; r < bb.run_start[t + 1]; ++r) {
      if (bb.run_row[r] < 0 || bb.run_row[r] >= bb.nrows[t]) fail("run row");
      for (int32_t q = bb.run_ext[r]; q < bb.run_ext[r + 1]; ++q)
        if (bb.ext[q] < bb.nrows[t] || bb.ext[q] >= bb.used[t]) fail("extra slot");
    }
  }
  upload(group, grp);
  upload(slot, sl);
  upload(start, bb.start);
  upload(row0, bb.row0);
  upload(nrows, bb.nrows);
  upload(used, bb.used);
  upload(tinst, bb.tinst);
  upload(col0, bb.col0);
  upload(panel, bb.panel);
  upload(run_start, bb.run_start);
  upload(run_row, bb.run_row);
  upload(run_ext, bb.run_ext);
  upload(ext, bb.ext);
  upload(pk, bb.pk);
  upload(src, bb.src);
  val32.alloc((size_t)nent * 4);
  val64.alloc((size_t)nent * 8);
  part32.alloc((size_t)P * R * 4);
  part64.alloc((size_t)P * R * 8);
  part64b.alloc((size_t)P * R * 8);
}

void BandSet::reset() {
  P = 1;
  ntile = nslot = 0;
  R = nent = 0;
  band_rows = 0;
  for (DBuf* d : {&group, &slot, &start, &row0, &nrows, &used, &tinst, &col0, &panel, &run_start, &run_row, &run_ext,
                  &ext, &pk, &src, &val32, &val64, &part32, &part64, &part64b, &orig32, &orig64})
    d->release();
}

BandTiles BandSet::view() const {
  BandTiles b{};
  b.group = group.as<int32_t>();
  b.slot = slot.as<int32_t>();
  b.start = start.as<int32_t>();
  b.row0 = row0.as<int32_t>();
  b.nrows = nrows.as<int32_t>();
  b.used = used.as<int32_t>();
  b.tinst = tinst.as<int32_t>();
  b.col0 = col0.as<int32_t>();
  b.panel = panel.as<int32_t>();
  b.run_start = run_start.as<int32_t>();
  b.run_row = run_row.as<int32_t>();
  b.run_ext = run_ext.as<int32_t>();
  b.ext = ext.as<int32_t>();
  b.pk = pk.as<uint32_t>();
  b.nslot = nslot;
  b.P = P;
  return b;
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
template <typename T>
void IterBufs<T>::alloc(int64_t N, int64_t M) {
  const int64_t sz[16] = {N, M, N, M, N, M, M, M, M, N, N, N, N, M, N, M};
  for (int i = 0; i < 16; ++i) b[i].alloc((size_t)sz[i] * sizeof(T));
  T** f = reinterpret_cast<T**>(&p);
  for (int i = 0; i < 16; ++i) f[i] = b[i].as<T>();
  ready = true;
}
template struct IterBufs<float>;
template struct IterBufs<double>;

Engine::Engine(const std::vector<const HostProblem*>& probs) {
  HIP_OK(hipGetDevice(&device));
  HIP_OK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  B = (int)probs.size();
  row0.assign(B + 1, 0);
  col0.assign(B + 1, 0);
  std::vector<int64_t> nz0(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    row0[b + 1] = row0[b] + probs[b]->m;
    col0[b + 1] = col0[b] + probs[b]->n;
    nz0[b + 1] = nz0[b] + probs[b]->nnz;
    mzero.push_back(probs[b]->m_zero);
  }
  M = row0[B];
  N = col0[B];
  NNZ = nz0[B];
  if (M >= INT32_MAX || N >= INT32_MAX || NNZ >= INT32_MAX)
    throw Error(PDCS_ERR_SIZE, "batch too large for 32-bit indexing");
  h_rp.resize(M + 1);
  h_cp.resize(N + 1);
  std::vector<int32_t> ci(NNZ), ri(NNZ);
  std::vector<double> v(NNZ), vt(NNZ), h(M), c(N), l(N), u(N);
  for (int b = 0; b < B; ++b) {
    const HostProblem& P = *probs[b];
    for (int64_t i = 0; i < P.m; ++i) h_rp[row0[b] + i] = (int32_t)(nz0[b] + P.rp[i]);
    for (int64_t j = 0; j < P.n; ++j) h_cp[col0[b] + j] = (int32_t)(nz0[b] + P.cp[j]);
    for (int64_t p = 0; p < P.nnz; ++p) {
      ci[nz0[b] + p] = (int32_t)(col0[b] + P.ci[p]);
      ri[nz0[b] + p] = (int32_t)(row0[b] + P.ri[p]);
    }
    std::copy(P.v.begin(), P.v.end(), v.begin() + nz0[b]);
    std::copy(P.vt.begin(), P.vt.end(), vt.begin() + nz0[b]);
    std::copy(P.h.begin(), P.h.end(), h.begin() + row0[b]);
    std::copy(P.c.begin(), P.c.end(), c.begin() + col0[b]);
    std::copy(P.l.begin(), P.l.end(), l.begin() + col0[b]);
    std::copy(P.u.begin(), P.u.end(), u.begin() + col0[b]);
  }
  h_rp[M] = (int32_t)NNZ;
  h_cp[N] = (int32_t)NNZ;
  h_ci = ci;  // kept for the band tiles
  h_ri = ri;
  upload(d_rp, h_rp);
  upload(d_ci, ci);
  upload(d_v, v);
  upload(d_cp, h_cp);
  upload(d_ri, ri);
  upload(d_vt, vt);
  upload(d_h, h);
  upload(d_c, c);
  upload(d_l, l);
  upload(d_u, u);
  for (DBuf* bf : {&val64, &valT64}) bf->alloc((size_t)NNZ * 8);
  for (DBuf* bf : {&val32, &valT32}) bf->alloc((size_t)NNZ * 4);
  for (DBuf* bf : {&h64, &D1, &cgx0, &cgx1, &yout, &stat_r}) bf->alloc((size_t)M * 8);
  for (DBuf* bf : {&c64, &l64, &u64, &D2, &cgty0, &cgty1, &xout, &lamout, &stat_c}) bf->alloc((size_t)N * 8);
  h32.alloc((size_t)M * 4);
  for (DBuf* bf : {&c32, &l32, &u32}) bf->alloc((size_t)N * 4);
  d_inst.alloc(sizeof(Inst) * (size_t)std::max(B, 1));
  d_summary.alloc(16);
  {
    std::vector<int32_t> r0i(row0.begin(), row0.end()), c0i(col0.begin(), col0.end());
    upload(d_row0i, r0i);
    upload(d_col0i, c0i);
  }
  for (int64_t j = 0; j < N && !any_unbounded; ++j) any_unbounded = !std::isfinite(l[j]) || !std::isfinite(u[j]);
  // cone blocks: the last rows of each instance, in row order (second-order,
  // then exponential, then dual exponential)
  for (int b = 0; b < B; ++b) {
    const HostProblem& P = *probs[b];
    int64_t r = row0[b + 1] - P.cone_rows();
    socstart.push_back(r);
    auto add = [&](int32_t d, int8_t kind) {
      soc.r0.push_back((int32_t)r);
      soc.dim.push_back(d);
      soc.kind.push_back(kind);
      r += d;
    };
    for (int32_t d : P.soc) add(d, 0);
    for (int64_t q = 0; q < P.n_exp; ++q) add(3, 1);
    for (int64_t q = 0; q < P.n_dexp; ++q) add(3, 2);
  }
  if (!soc.empty()) {
    upload(soc.r0_d, soc.r0);
    upload(soc.dim_d, soc.dim);
    upload(soc.kind_d, soc.kind);
  }
  vrow.soc = &soc;
  crow.soc = &soc;
  HIP_OK(hipHostMalloc((void**)&h_summary, 16, hipHostMallocDefault));
  build_schedule();
}

Engine::~Engine() {
  clear_graphs();
  if (h_summary) (void)hipHostFree(h_summary);
  for (auto& e : events) (void)hipEventDestroy(e);
  if (stream) (void)hipStreamDestroy(stream);
}

void Engine::clear_graphs() {
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  graphs.clear();
}

void Engine::build_iteration_schedules(const std::vector<char>* active) {
  clear_graphs();
  trow.build(h_rp, row0, sched, active);
  tcol.build(h_cp, col0, sched, active);
  brow.build(h_rp, row0, sched.iter_max * 4, active);
  bcol.build(h_cp, col0, sched.iter_max * 4, active);
  vrow.cone_cap = kConeBlocksPerRange;
  vrow.build(row0, sched.vec_per_block, active);
  vcol.build(col0, sched.vec_per_block, active);
  // The multisection passes reduce 32 values per element into per-workgroup
  // records that one workgroup per instance sums: larger blocks mean fewer
  // records and fewer block reductions, with the same arithmetic.  Blocks
  // grow up to kCheckCoarsen times, keeping about one block per CU.
  auto check_block = [&](const std::vector<int64_t>& off) {
    int64_t total = 0;
    for (size_t b = 0; b + 1 < off.size(); ++b)
      if (!active || (*active)[b]) total += off[b + 1] - off[b];
    const int64_t f = std::max<int64_t>(1, std::min<int64_t>(kCheckCoarsen, total / (256 * (int64_t)sched.vec_per_block)));
    return (int)(sched.vec_per_block * f);
  };
  crow.cone_cap = kConeBlocksPerCheckRange;
  crow.build(row0, check_block(row0), active);
  ccol.build(col0, check_block(col0), active);
}

void Engine::build_schedule() {
  build_iteration_schedules(nullptr);
  // cone blocks are projected in the row epilogues of the split dual pass,
  // which the band layout always takes
  const bool want_band = layout == PDCS_LAYOUT_BANDS || !soc.empty() ||
                         (layout == PDCS_LAYOUT_AUTO && NNZ >= ((int64_t)1 << 22));
  if (want_band && !band1.nslot && !band2.nslot) {
    band1.build(row0, col0, h_rp, h_ci, bsched);
    band2.build(col0, row0, h_cp, h_ri, bsched);
  }
  use_band = want_band;
  // one workgroup per instance for whole chunks of trials: forced, or
  // automatically when every instance fits in LDS in FP64 (the workgroup then
  // runs its trials out of LDS; on global memory it would be slower than the
  // row-block kernels), on row blocks
  plan_lds_trials();
  wg_trials = !want_band &&
              (layout == PDCS_LAYOUT_WORKGROUP || (layout == PDCS_LAYOUT_AUTO && lds_bytes[1] > 0));
  if (!wg_trials) lds_bytes[0] = lds_bytes[1] = 0;
  rec_dual_epi.alloc((size_t)std::max(vrow.nblk, 1) * 4 * 8);
  rec_lam_epi.alloc((size_t)std::max(vcol.nblk, 1) * 3 * 8);
  const int nr = std::max(brow.nblk, 1), nc = std::max(bcol.nblk, 1);
  const int vr = std::max(vrow.nblk, 1), vc = std::max(vcol.nblk, 1);
  rec_primal.alloc((size_t)vc * 2 * 8);
  rec_dual.alloc((size_t)nr * 4 * 8);
  rec_lam.alloc((size_t)nc * 3 * 8);
  rec_cand_c.alloc((size_t)vc * 16 * 8);
  rec_cand_r.alloc((size_t)vr * 14 * 8);
  rec_probe_c.alloc((size_t)vc * 2 * 32 * 8);
  rec_probe_r.alloc((size_t)vr * 2 * 32 * 8);
  rec_nc.alloc((size_t)vc * 3 * 8);
  rec_nr.alloc((size_t)vr * 3 * 8);
  rec_nm.alloc((size_t)std::max(trow.nblk, 1) * 8);
}

// Dynamic LDS of k_trials_lds for the largest instance, per precision (0 when
// some instance does not fit next to the kernel's static LDS: the chunk kernel
// then works on global memory).  The block tables are those of the full
// schedule; compaction only removes blocks, and inactive instances exit before
// touching LDS.
void Engine::plan_lds_trials() {
  lds_bytes[0] = lds_bytes[1] = 0;
  if (!soc.empty()) return;
  size_t need[2] = {0, 0};
  for (int b = 0; b < B; ++b) {
    const int64_t m = row0[b + 1] - row0[b], n = col0[b + 1] - col0[b];
    const int64_t nnz = h_rp[row0[b + 1]] - h_rp[row0[b]];
    const int64_t np = vcol.h_iblk0[b + 1] - vcol.h_iblk0[b];
    const int64_t nd = brow.h_iblk0[b + 1] - brow.h_iblk0[b];
    const int64_t nl = bcol.h_iblk0[b + 1] - bcol.h_iblk0[b];
    need[0] = std::max(need[0], lds_layout(m, n, nnz, np, nd, nl, 4).total);
    need[1] = std::max(need[1], lds_layout(m, n, nnz, np, nd, nl, 8).total);
  }
  for (int pi = 0; pi < 2; ++pi) {
    const size_t avail = trials_lds_capacity(pi == 0 ? kFP32 : kFP64);
    lds_bytes[pi] = need[pi] <= avail ? need[pi] : 0;
  }
  // short rows and columns everywhere: one thread per row in the dual and
  // dual-slack passes (long ones keep the block schedule's lanes per row)
  int64_t longest = 0;
  for (int64_t r = 0; r < M; ++r) longest = std::max<int64_t>(longest, h_rp[r + 1] - h_rp[r]);
  for (int64_t c = 0; c < N; ++c) longest = std::max<int64_t>(longest, h_cp[c + 1] - h_cp[c]);
  lds_rowwise = longest <= kLdsRowMax;
}

void Engine::ensure_iter(int prec) {
  if (prec == kFP32 && !it32.ready) it32.alloc(N, M);
  if (prec == kFP64 && !it64.ready) it64.alloc(N, M);
}

KernelCtx Engine::ctx(int probe_passes) const {
  KernelCtx k{};
  k.nb = B;
  k.M = M;
  k.N = N;
  k.trow = trow.view();
  k.tcol = tcol.view();
  k.brow = brow.view();
  k.bcol = bcol.view();
  k.vrow = vrow.view();
  k.vcol = vcol.view();
  k.crow = crow.view();
  k.ccol = ccol.view();
  k.inst = d_inst.as<Inst>();
  k.it32 = it32.p;
  k.it64 = it64.p;
  k.d32 = DataPtrs<float>{c32.as<float>(), l32.as<float>(), u32.as<float>(), h32.as<float>()};
  k.d64 = DataPtrs<double>{c64.as<double>(), l64.as<double>(), u64.as<double>(), h64.as<double>()};
  k.A32 = MatPtrs<float>{d_rp.as<int32_t>(), d_ci.as<int32_t>(), val32.as<float>()};
  k.AT32 = MatPtrs<float>{d_cp.as<int32_t>(), d_ri.as<int32_t>(), valT32.as<float>()};
  k.A64 = MatPtrs<double>{d_rp.as<int32_t>(), d_ci.as<int32_t>(), val64.as<double>()};
  k.AT64 = MatPtrs<double>{d_cp.as<int32_t>(), d_ri.as<int32_t>(), valT64.as<double>()};
  k.cgx0 = cgx0.as<double>();
  k.cgx1 = cgx1.as<double>();
  k.cgty0 = cgty0.as<double>();
  k.cgty1 = cgty1.as<double>();
  k.D1 = D1.as<double>();
  k.D2 = D2.as<double>();
  k.xout = xout.as<double>();
  k.yout = yout.as<double>();
  k.lamout = lamout.as<double>();
  k.rec_primal = rec_primal.as<double>();
  k.rec_dual = rec_dual.as<double>();
  k.rec_lam = rec_lam.as<double>();
  k.rec_cand_c = rec_cand_c.as<double>();
  k.rec_cand_r = rec_cand_r.as<double>();
  k.rec_probe_c = rec_probe_c.as<double>();
  k.rec_probe_r = rec_probe_r.as<double>();
  k.probe_passes = probe_passes;
  k.wg_trials = wg_trials ? 1 : 0;
  k.lds_trials32 = (int)lds_bytes[0];
  k.lds_trials64 = (int)lds_bytes[1];
  k.lds_rowwise = lds_rowwise ? 1 : 0;
  k.rec_dual_epi = rec_dual_epi.as<double>();
  k.rec_lam_epi = rec_lam_epi.as<double>();
  k.infeas = infeas_on;
  k.ray_x = any_unbounded ? 1 : 0;
  k.xs0 = xs0.as<double>();
  k.ys0 = ys0.as<double>();
  k.rx = rx.as<double>();
  k.ry = ry.as<double>();
  k.rgx = rgx.as<double>();
  k.rgty = rgty.as<double>();
  k.use_band = use_band && !band_suspended ? 1 : 0;
  if (k.use_band) {
    k.band1 = band1.view();
    k.band2 = band2.view();
    k.bval32 = band1.val32.as<float>();
    k.bval64 = band1.val64.as<double>();
    k.bvalT32 = band2.val32.as<float>();
    k.bvalT64 = band2.val64.as<double>();
    k.bpart32 = band1.part32.as<float>();
    k.bpart64 = band1.part64.as<double>();
    k.bpartT32 = band2.part32.as<float>();
    k.bpartT64 = band2.part64.as<double>();
    k.bpart64b = band1.part64b.as<double>();
    k.bpartT64b = band2.part64b.as<double>();
  }
  return k;
}

static void validate_options(const pdcs_options& o) {
  if (!(o.rel_tol >= 0) || !(o.abs_tol >= 0)) throw Error(PDCS_ERR_INVALID_ARG, "tolerances must be >= 0");
  if (o.check_every < 1 || o.check_every > 100000) throw Error(PDCS_ERR_INVALID_ARG, "check_every in [1, 1e5]");
  if (o.max_iter < 0) throw Error(PDCS_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (o.method < 0 || o.method > 2) throw Error(PDCS_ERR_INVALID_ARG, "unknown method");
  if (o.precision < 0 || o.precision > 1) throw Error(PDCS_ERR_INVALID_ARG, "unknown precision");
  if (o.ruiz_iters < 0 || o.ruiz_iters > 1000) throw Error(PDCS_ERR_INVALID_ARG, "ruiz_iters in [0, 1000]");
  if (o.probe_passes < 1 || o.probe_passes > 64) throw Error(PDCS_ERR_INVALID_ARG, "probe_passes in [1, 64]");
  if (o.use_kkt_restart < 0 || o.use_kkt_restart > 1) throw Error(PDCS_ERR_INVALID_ARG, "use_kkt_restart is 0 or 1");
  if (!(o.bisect_rel_eps > 0)) throw Error(PDCS_ERR_INVALID_ARG, "bisect_rel_eps must be > 0");
  if (std::isnan(o.time_limit)) throw Error(PDCS_ERR_INVALID_ARG, "time_limit is NaN");
  if (o.use_duality_gap_restart < 0 || o.use_duality_gap_restart > 1)
    throw Error(PDCS_ERR_INVALID_ARG, "use_duality_gap_restart is 0 or 1");
  if (o.kkt_restart_freq < 0 || o.kkt_restart_freq > 100000 || o.duality_gap_restart_freq < 0 ||
      o.duality_gap_restart_freq > 100000)
    throw Error(PDCS_ERR_INVALID_ARG, "restart frequencies in [0, 1e5]");
  if (o.print_freq < 1) throw Error(PDCS_ERR_INVALID_ARG, "print_freq must be >= 1");
  for (double e : {o.eps_primal_infeasible_low_acc, o.eps_dual_infeasible_low_acc, o.eps_primal_infeasible_high_acc,
                   o.eps_dual_infeasible_high_acc})
    if (!(e >= 0.0) || !std::isfinite(e)) throw Error(PDCS_ERR_INVALID_ARG, "infeasibility tolerances must be finite and >= 0");
}

// Restart metric and check period (option list of Section 3): the normalized
// duality gap unless use_kkt_restart is set or use_duality_gap_restart is
// cleared; the period is the metric's frequency option, or check_every when 0.
static bool gap_metric(const pdcs_options& o) { return o.use_duality_gap_restart != 0 && o.use_kkt_restart == 0; }
static int64_t check_period(const pdcs_options& o) {
  const int64_t f = gap_metric(o) ? o.duality_gap_restart_freq : o.kkt_restart_freq;
  return f > 0 ? f : o.check_every;
}

void Engine::enqueue_chunk(const KernelCtx& k, int mask, int64_t K, bool timed) {
  if (k.wg_trials && !k.use_band && !timed) {  // timed runs keep the per-pass launches
    launch_trials_wg(k, stream, mask, (int)K);
    launch_check(k, stream, mask);
    launch_summary(k, stream, d_summary.as<int32_t>());
    return;
  }
  for (int64_t s = 0; s < K; ++s) {
    launch_trial_part(k, stream, mask, 0);
    if (timed) {
      if (ev_used + 2 > events.size()) {
        for (int i = 0; i < 256; ++i) {
          hipEvent_t e;
          HIP_OK(hipEventCreate(&e));
          events.push_back(e);
        }
      }
      HIP_OK(hipEventRecord(events[ev_used], stream));
      launch_trial_part(k, stream, mask, 1);
      HIP_OK(hipEventRecord(events[ev_used + 1], stream));
      ev_used += 2;
    } else {
      launch_trial_part(k, stream, mask, 1);
    }
    launch_trial_part(k, stream, mask, 2);
  }
  launch_check(k, stream, mask);
  launch_summary(k, stream, d_summary.as<int32_t>());
}

void Engine::harvest_events() {
  for (size_t i = 0; i + 1 < ev_used; i += 2) {
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, events[i], events[i + 1]));
    timed_ms += ms;
    timed_count += 1;
  }
  ev_used = 0;
}

std::vector<pdcs_result> Engine::solve(const pdcs_options& o, const WarmStart& ws) {
  validate_options(o);
  const double* const* x0s = ws.hx;
  const double* const* y0s = ws.hy;
  const bool gap = gap_metric(o);
  const int64_t period = check_period(o);
  const int probe_passes = gap ? (int)o.probe_passes : 0;
  infeas_on = (o.eps_primal_infeasible_low_acc > 0 || o.eps_dual_infeasible_low_acc > 0 ||
               o.eps_primal_infeasible_high_acc > 0 || o.eps_dual_infeasible_high_acc > 0)
                  ? 1
                  : 0;
  if (infeas_on && !rx.p) {
    for (DBuf* bf : {&xs0, &rx, &rgty}) bf->alloc((size_t)N * 8);
    for (DBuf* bf : {&ys0, &ry, &rgx}) bf->alloc((size_t)M * 8);
  }
  HIP_OK(hipGetLastError());
  const auto t_start = std::chrono::steady_clock::now();
  if (band_suspended) {  // left over from a solve that ended early
    band_suspended = false;
    build_iteration_schedules(nullptr);
  }
  const bool mixed = o.precision == PDCS_PRECISION_MIXED;
  ensure_iter(kFP64);
  if (mixed) ensure_iter(kFP32);
  const int start_mask = mixed ? 1 : 2;
  const int alloc_mask = (it32.ready ? 1 : 0) | (it64.ready ? 2 : 0);
  // per-instance scalars
  std::vector<Inst> hi(B);
  for (int b = 0; b < B; ++b) {
    Inst& I = hi[b];
    std::memset(&I, 0, sizeof(Inst));
    I.row0 = (int32_t)row0[b];
    I.rows = (int32_t)(row0[b + 1] - row0[b]);
    I.col0 = (int32_t)col0[b];
    I.cols = (int32_t)(col0[b + 1] - col0[b]);
    I.m_zero = (int32_t)mzero[b];
    I.soc_start = (int32_t)socstart[b];
    I.precision = mixed ? kFP32 : kFP64;
    I.status = kActive;
    I.exit_code = PDCS_EXIT_CONTINUE;
    I.max_iter = o.max_iter;
    I.check_every = period;
    I.method = (int32_t)o.method;
    I.use_avg = o.method != PDCS_METHOD_HALPERN ? 1 : 0;
    I.force_kkt = gap ? 0 : 1;
    I.infeas_on = infeas_on;
    I.eps_inf[0] = o.eps_primal_infeasible_low_acc;
    I.eps_inf[1] = o.eps_dual_infeasible_low_acc;
    I.eps_inf[2] = o.eps_primal_infeasible_high_acc;
    I.eps_inf[3] = o.eps_dual_infeasible_high_acc;
    I.ratio_p = I.ratio_d = std::numeric_limits<double>::quiet_NaN();
    I.rel_tol = o.rel_tol;
    I.abs_tol = o.abs_tol;
    I.polish_tol = o.polish_switch_tol;
    I.stall_checks = o.stall_checks;
    I.bisect_eps = o.bisect_rel_eps;
    I.best_rel = std::numeric_limits<double>::infinity();
    I.best_any = std::numeric_limits<double>::infinity();
    I.stall_any = 0;
    I.omega = I.omega0 = 1.0;
    I.eta = I.eta_hat = 1.0;
  }
  if (o.trace_trials > 0) {
    d_trace.alloc((size_t)o.trace_trials * kTraceStride * 8);
    hi[0].trace = d_trace.as<double>();
    hi[0].trace_cap = o.trace_trials;
  }
  HIP_OK(hipMemcpyAsync(d_inst.p, hi.data(), sizeof(Inst) * B, hipMemcpyHostToDevice, stream));
  // optional warm start (unscaled, host)
  const double* dx0 = nullptr;
  const double* dy0 = nullptr;
  if (x0s || y0s) {
    std::vector<double> hx(N, 0.0), hy(M, 0.0);
    bool anyx = false, anyy = false;
    for (int b = 0; b < B; ++b) {
      if (x0s && x0s[b]) {
        anyx = true;
        for (int64_t j = 0; j < col0[b + 1] - col0[b]; ++j) {
          if (std::isnan(x0s[b][j])) throw Error(PDCS_ERR_INVALID_ARG, "NaN in x0");
          hx[col0[b] + j] = x0s[b][j];
        }
      }
      if (y0s && y0s[b]) {
        anyy = true;
        for (int64_t i = 0; i < row0[b + 1] - row0[b]; ++i) {
          if (std::isnan(y0s[b][i])) throw Error(PDCS_ERR_INVALID_ARG, "NaN in y0");
          hy[row0[b] + i] = y0s[b][i];
        }
      }
    }
    if (anyx) {
      warm_x.alloc((size_t)N * 8);
      HIP_OK(hipMemcpyAsync(warm_x.p, hx.data(), (size_t)N * 8, hipMemcpyHostToDevice, stream));
      dx0 = warm_x.as<double>();
    }
    if (anyy) {
      warm_y.alloc((size_t)M * 8);
      HIP_OK(hipMemcpyAsync(warm_y.p, hy.data(), (size_t)M * 8, hipMemcpyHostToDevice, stream));
      dy0 = warm_y.as<double>();
    }
    HIP_OK(hipStreamSynchronize(stream));
  }
  if (ws.dx || ws.dy) {
    // device warm starts: wait for the caller's work on its stream, then pack
    // the per-instance arrays into the FP64 start vectors (NaN is rejected)
    hipEvent_t ready;
    HIP_OK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    hipError_t e1 = hipEventRecord(ready, ws.caller);
    hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(stream, ready, 0) : e1;
    (void)hipEventDestroy(ready);
    HIP_OK(e2);
    if (!d_flag.p) d_flag.alloc(256);
    HIP_OK(hipMemsetAsync(d_flag.p, 0, 4, stream));
    if (!warm_ptr.p) warm_ptr.alloc(sizeof(void*) * (size_t)B);
    int64_t maxc = 0, maxr = 0;
    for (int b = 0; b < B; ++b) {
      maxc = std::max<int64_t>(maxc, col0[b + 1] - col0[b]);
      maxr = std::max<int64_t>(maxr, row0[b + 1] - row0[b]);
    }
    for (int side = 0; side < 2; ++side) {
      const void* const* src = side == 0 ? ws.dx : ws.dy;
      if (!src) continue;
      std::vector<const void*> tbl(src, src + B);
      HIP_OK(hipMemcpyAsync(warm_ptr.p, tbl.data(), sizeof(void*) * (size_t)B, hipMemcpyHostToDevice, stream));
      DBuf& dst = side == 0 ? warm_x : warm_y;
      dst.alloc((size_t)(side == 0 ? N : M) * 8);
      launch_pack_warm(warm_ptr.as<const void*>(), (side == 0 ? d_col0i : d_row0i).as<int32_t>(), B,
                       side == 0 ? maxc : maxr, ws.dtype, dst.as<double>(), d_flag.as<int32_t>(), stream);
      HIP_OK(hipGetLastError());
      HIP_OK(hipStreamSynchronize(stream));  // the pointer table is reused by the other side
      if (side == 0) dx0 = warm_x.as<double>();
      else dy0 = warm_y.as<double>();
    }
    int32_t nan_seen = 0;
    HIP_OK(hipMemcpy(&nan_seen, d_flag.p, 4, hipMemcpyDeviceToHost));
    if (nan_seen) throw Error(PDCS_ERR_INVALID_ARG, "NaN in the device warm start");
  }
  KernelCtx k = ctx(probe_passes);
  SetupCtx su{};
  su.precondition = o.use_preconditioner ? 1 : 0;
  su.ruiz_iters = (int)o.ruiz_iters;
  su.l2_pass = o.l2_pass ? 1 : 0;
  su.A = MatPtrs<double>{d_rp.as<int32_t>(), d_ci.as<int32_t>(), d_v.as<double>()};
  su.AT = MatPtrs<double>{d_cp.as<int32_t>(), d_ri.as<int32_t>(), d_vt.as<double>()};
  su.c = d_c.as<double>();
  su.l = d_l.as<double>();
  su.u = d_u.as<double>();
  su.h = d_h.as<double>();
  su.val64 = val64.as<double>();
  su.valT64 = valT64.as<double>();
  su.val32 = val32.as<float>();
  su.valT32 = valT32.as<float>();
  su.d64m = DataMut{c64.as<double>(), l64.as<double>(), u64.as<double>(), h64.as<double>()};
  su.d32m = DataMut32{c32.as<float>(), l32.as<float>(), u32.as<float>(), h32.as<float>()};
  su.stat_r = stat_r.as<double>();
  su.stat_c = stat_c.as<double>();
  su.rec_nc = rec_nc.as<double>();
  su.rec_nr = rec_nr.as<double>();
  su.rec_nm = rec_nm.as<double>();
  su.x0 = dx0;
  su.y0 = dy0;
  if (use_band) {
    su.bsrc = band1.src.as<int32_t>();
    su.bsrcT = band2.src.as<int32_t>();
    su.bn = band1.nent;
    su.bnT = band2.nent;
    su.bval64 = band1.val64.as<double>();
    su.bval32 = band1.val32.as<float>();
    su.bvalT64 = band2.val64.as<double>();
    su.bvalT32 = band2.val32.as<float>();
  }
  launch_setup(k, su, stream, start_mask);
  HIP_OK(hipGetLastError());

  const bool timed = o.time_kernels != 0;
  const bool use_graph = o.use_graph != 0 && !timed;
  timed_ms = 0.0;
  timed_count = 0;
  ev_used = 0;
  launch_summary(k, stream, d_summary.as<int32_t>());
  int64_t chunks = 0;
  int64_t printed = 0;  // progress lines written (verbose = 1: one per print_freq trials)
  // Retire-and-compact: when the active instances of a batch have halved
  // since the schedules were built, rebuild the iteration schedules over the
  // active ones only, so finished instances stop costing workgroups.
  int active_built = B;
  bool compacted = false;
  while (true) {
    HIP_OK(hipMemcpyAsync(h_summary, d_summary.p, 8, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (timed) harvest_events();
    const int a32 = h_summary[0], a64 = h_summary[1];
    const bool print_now = o.verbose > 1 || (o.verbose == 1 && chunks * period / o.print_freq > printed);
    if (o.verbose && chunks > 0 && print_now) {
      printed = chunks * period / o.print_freq;
      Inst I0;
      HIP_OK(hipMemcpy(&I0, d_inst.p, sizeof(Inst), hipMemcpyDeviceToHost));
      std::fprintf(stderr,
                   "[pdcs] %.1fs kbar %lld k %lld t %lld restarts %lld omega %.3e eta %.3e rel(p,d,g) %.2e %.2e %.2e "
                   "rho(cur,avg,anchor) %.3e %.3e %.3e chosen %d kkt %d prec %s active %d\n",
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(),
                   (long long)I0.kbar, (long long)I0.k, (long long)I0.t, (long long)I0.restarts, I0.omega,
                   I0.eta_hat, I0.rel_p, I0.rel_d, I0.rel_gap, I0.cand[0].rho, I0.cand[1].rho, I0.rho_anchor,
                   I0.chosen, I0.use_kkt, I0.precision == kFP32 ? "fp32" : "fp64", a32 + a64);
    }
    if (a32 + a64 == 0) break;
    if (o.compact && B >= 8 && a32 + a64 <= active_built / 2) {
      std::vector<Inst> cur(B);
      HIP_OK(hipMemcpy(cur.data(), d_inst.p, sizeof(Inst) * B, hipMemcpyDeviceToHost));
      std::vector<char> act(B, 0);
      int64_t act_nnz = 0;
      for (int b = 0; b < B; ++b) {
        act[b] = cur[b].status == kActive ? 1 : 0;
        if (act[b]) act_nnz += h_rp[row0[b + 1]] - h_rp[row0[b]];
      }
      build_iteration_schedules(&act);
      // the automatic layout choice, made again for the instances still running:
      // few large tiles would leave most of the chip idle, compacted row blocks do not
      if (layout == PDCS_LAYOUT_AUTO && soc.empty() && act_nnz < ((int64_t)1 << 22)) band_suspended = true;
      k = ctx(probe_passes);
      active_built = a32 + a64;
      compacted = true;
    }
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (el >= o.time_limit) {
      launch_timeout(k, stream);
      break;
    }
    const int mask = (a32 ? 1 : 0) | (a64 ? 2 : 0);
    if (use_graph) {
      // everything that changes the captured launch sequence is in the key
      const int64_t key = ((int64_t)mask << 48) | ((int64_t)infeas_on << 47) | (period << 8) | probe_passes;
      auto it = graphs.find(key);
      if (it == graphs.end()) {
        hipGraph_t g;
        HIP_OK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        enqueue_chunk(k, mask, period, false);
        HIP_OK(hipStreamEndCapture(stream, &g));
        hipGraphExec_t ge;
        HIP_OK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        it = graphs.emplace(key, ge).first;
      }
      HIP_OK(hipGraphLaunch(it->second, stream));
    } else {
      enqueue_chunk(k, mask, period, timed);
    }
    HIP_OK(hipGetLastError());
    ++chunks;
  }
  if (compacted) {  // the final evaluation covers every instance
    build_iteration_schedules(nullptr);
    band_suspended = false;
    k = ctx(probe_passes);
  }
  // final point of instances that stopped without an optimal candidate
  launch_eval(k, stream, alloc_mask, 1);
  if (o.keep_state) launch_flush_commit(k, stream, alloc_mask);
  HIP_OK(hipGetLastError());
  std::vector<Inst> fin(B);
  HIP_OK(hipMemcpyAsync(fin.data(), d_inst.p, sizeof(Inst) * B, hipMemcpyDeviceToHost, stream));
  // results own a device copy of the outputs
  auto out = std::make_shared<OutBlock>();
  out->M = M;
  out->N = N;
  out->x.alloc((size_t)N * 8);
  out->lam.alloc((size_t)N * 8);
  out->y.alloc((size_t)M * 8);
  out->D1.alloc((size_t)M * 8);
  out->D2.alloc((size_t)N * 8);
  HIP_OK(hipMemcpyAsync(out->x.p, xout.p, (size_t)N * 8, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(out->lam.p, lamout.p, (size_t)N * 8, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(out->y.p, yout.p, (size_t)M * 8, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(out->D1.p, D1.p, (size_t)M * 8, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(out->D2.p, D2.p, (size_t)N * 8, hipMemcpyDeviceToDevice, stream));
  if (o.keep_state) {
    for (int pi = 0; pi < 2; ++pi) {
      const bool ok = pi == 0 ? it64.ready : it32.ready;
      if (!ok) continue;
      const size_t es = pi == 0 ? 8 : 4;
      void* src[8];
      if (pi == 0) {
        const IterPtrs<double>& q = it64.p;
        void* s8[8] = {q.x, q.y, q.xh, q.yh, q.xa, q.ya, q.gtyh, q.gxh};
        std::memcpy(src, s8, sizeof(src));
      } else {
        const IterPtrs<float>& q = it32.p;
        void* s8[8] = {q.x, q.y, q.xh, q.yh, q.xa, q.ya, q.gtyh, q.gxh};
        std::memcpy(src, s8, sizeof(src));
      }
      for (int v = 0; v < 8; ++v) {
        const size_t len = (v % 2 == 0) ? (size_t)N : (size_t)M;
        out->st[pi][v].alloc(len * es);
        HIP_OK(hipMemcpyAsync(out->st[pi][v].p, src[v], len * es, hipMemcpyDeviceToDevice, stream));
      }
    }
  }
  HIP_OK(hipStreamSynchronize(stream));
  const double elapsed = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  std::vector<pdcs_result> res(B);
  for (int b = 0; b < B; ++b) {
    const Inst& I = fin[b];
    auto* r = new pdcs_result_s();
    r->out = out;
    r->row0 = row0[b];
    r->col0 = col0[b];
    r->m = row0[b + 1] - row0[b];
    r->n = col0[b + 1] - col0[b];
    std::memset(&r->info, 0, sizeof(r->info));
    r->info.exit_code = I.exit_code;
    r->info.iters = I.kbar;
    r->info.accepted_iters = I.accepted;
    r->info.restarts = I.restarts;
    r->info.checks = I.checks;
    r->info.fp64_iters = I.fp64_iters;
    r->info.pobj = I.pobj;
    r->info.dobj = I.dobj;
    r->info.abs_p = I.abs_p;
    r->info.abs_d = I.abs_d;
    r->info.abs_gap = I.abs_gap;
    r->info.rel_p = I.rel_p;
    r->info.rel_d = I.rel_d;
    r->info.rel_gap = I.rel_gap;
    r->info.time_sec = elapsed;
    r->info.omega = I.omega;
    r->info.eta_hat = I.eta_hat;
    r->info.spmv_avg_ms = timed_count ? timed_ms / (double)timed_count : 0.0;
    r->info.spmv_launches = timed_count;
    std::memset(&r->st, 0, sizeof(r->st));
    r->st.omega = I.omega;
    r->st.omega0 = I.omega0;
    r->st.eta_hat = I.eta_hat;
    r->st.eta = I.eta;
    r->st.beta = I.beta;
    r->st.sum_eta = I.sum_eta;
    r->st.kbar = I.kbar;
    r->st.k = I.k;
    r->st.t = I.t;
    r->st.accepted = I.accepted;
    r->st.precision = I.precision == kFP32 ? PDCS_PRECISION_MIXED : PDCS_PRECISION_FP64;
    r->st.rho_cur = I.chk_rho[0];
    r->st.rho_avg = I.chk_rho[1];
    r->st.r_cur = I.chk_r[0];
    r->st.r_avg = I.chk_r[1];
    r->st.chosen = I.chosen;
    r->st.ratio_p = I.ratio_p;
    r->st.ratio_d = I.ratio_d;
    r->st.trend_p = I.trend_p;
    r->st.trend_d = I.trend_d;
    r->has_state = o.keep_state != 0;
    if (b == 0 && o.trace_trials > 0) {
      const int64_t rows = std::min<int64_t>(o.trace_trials, I.kbar);
      r->trace.resize((size_t)rows * kTraceStride);
      if (rows > 0)
        HIP_OK(hipMemcpy(r->trace.data(), d_trace.p, (size_t)rows * kTraceStride * 8, hipMemcpyDeviceToHost));
    }
    res[b] = r;
  }
  return res;
}

// Rebuild both band layouts with the current band schedule (the scaled band
// values are filled in by the next solve's set-up).
void Engine::rebuild_bands() {
  clear_graphs();
  band1.reset();
  band2.reset();
  build_schedule();
}

// Time `reps` launches of the SpMV-with-dual-step kernel on the current state.
double Engine::time_dual(int prec, int reps) {
  const KernelCtx k = ctx(7);
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  launch_dual_only(k, stream, prec);
  HIP_OK(hipEventRecord(e0, stream));
  for (int i = 0; i < reps; ++i) launch_dual_only(k, stream, prec);
  HIP_OK(hipEventRecord(e1, stream));
  HIP_OK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

}  // namespace pdcs

// ===========================================================================
// C ABI
// ===========================================================================
namespace {
template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return PDCS_ERR_OOM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return PDCS_ERR_INVALID_ARG;
  }
}
}  // namespace

extern "C" {

void pdcs_options_default(pdcs_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rel_tol = 1e-6;
  o->abs_tol = 1e-6;
  o->time_limit = 1000.0;
  o->max_iter = INT64_MAX / 4;
  o->use_preconditioner = 1;
  o->ruiz_iters = 10;
  o->l2_pass = 1;
  o->method = PDCS_METHOD_AUTO;
  o->check_every = 64;
  o->precision = PDCS_PRECISION_FP64;
  o->stall_checks = 512;
  o->polish_switch_tol = 0.0;
  o->bisect_rel_eps = 1e-6;
  o->use_graph = 1;
  o->verbose = 0;
  o->keep_state = 0;
  o->time_kernels = 0;
  o->probe_passes = 7;
  o->compact = 1;
  o->use_duality_gap_restart = 1;
  o->kkt_restart_freq = 0;
  o->duality_gap_restart_freq = 0;
  o->print_freq = 2000;
  o->eps_primal_infeasible_low_acc = 1e-12;
  o->eps_dual_infeasible_low_acc = 1e-12;
  o->eps_primal_infeasible_high_acc = 1e-16;
  o->eps_dual_infeasible_high_acc = 1e-16;
}

const char* pdcs_status_string(int code) {
  switch (code) {
    case 0: return "optimal";
    case 1: return "max_iter";
    case 2: return "primal_infeasible_low_acc";
    case 3: return "primal_infeasible_high_acc";
    case 4: return "dual_infeasible_low_acc";
    case 5: return "dual_infeasible_high_acc";
    case 6: return "time_limit";
    case 7: return "continue";
    case 8: return "numerical_error";
    default: return "unknown";
  }
}

const char* pdcs_last_error(void) { return g_err.c_str(); }

int pdcs_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

int pdcs_problem_create(int64_t m, int64_t n, int64_t m_zero, const int64_t* row_ptr, const int32_t* col_idx,
                        const double* val, const double* h, const double* c, const double* l, const double* u,
                        pdcs_problem* out) {
  return guarded([&]() {
    if (!out) throw Error(PDCS_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    auto p = std::make_unique<pdcs_problem_s>();
    p->hp.build(m, n, m_zero, row_ptr, col_idx, val, h, c, l, u);
    std::vector<const HostProblem*> v{&p->hp};
    p->eng = std::make_unique<Engine>(v);
    p->eng->prepare_plain();
    *out = p.release();
    return PDCS_OK;
  });
}

int pdcs_problem_create_conic(int64_t m, int64_t n, int64_t m_zero, int64_t n_soc, const int64_t* soc_dims,
                              const int64_t* row_ptr, const int32_t* col_idx, const double* val, const double* h,
                              const double* c, const double* l, const double* u, pdcs_problem* out) {
  return guarded([&]() {
    if (!out) throw Error(PDCS_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    auto p = std::make_unique<pdcs_problem_s>();
    p->hp.build(m, n, m_zero, row_ptr, col_idx, val, h, c, l, u, n_soc, soc_dims);
    std::vector<const HostProblem*> v{&p->hp};
    p->eng = std::make_unique<Engine>(v);
    p->eng->prepare_plain();
    *out = p.release();
    return PDCS_OK;
  });
}

int pdcs_problem_create_cones(int64_t m, int64_t n, int64_t m_zero, int64_t n_soc, const int64_t* soc_dims,
                              int64_t n_exp, int64_t n_dexp, const int64_t* row_ptr, const int32_t* col_idx,
                              const double* val, const double* h, const double* c, const double* l, const double* u,
                              pdcs_problem* out) {
  return guarded([&]() {
    if (!out) throw Error(PDCS_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    auto p = std::make_unique<pdcs_problem_s>();
    p->hp.build(m, n, m_zero, row_ptr, col_idx, val, h, c, l, u, n_soc, soc_dims, n_exp, n_dexp);
    std::vector<const HostProblem*> v{&p->hp};
    p->eng = std::make_unique<Engine>(v);
    p->eng->prepare_plain();
    *out = p.release();
    return PDCS_OK;
  });
}

int pdcs_project_cone(int64_t cone, int64_t dim, int64_t count, const double* v, const double* f, double* out,
                      double* kernel_ms) {
  return guarded([&]() {
    if (cone < 0 || cone > 2) throw Error(PDCS_ERR_INVALID_ARG, "cone must be 0, 1 or 2");
    if (dim < 1 || (cone != 0 && dim != 3)) throw Error(PDCS_ERR_INVALID_ARG, "bad cone dimension");
    if (count < 0) throw Error(PDCS_ERR_INVALID_ARG, "count must be >= 0");
    if (count == 0) return PDCS_OK;
    if (!v || !f || !out) throw Error(PDCS_ERR_INVALID_ARG, "null array");
    if (dim > ((int64_t)1 << 24) || count > ((int64_t)1 << 28) / dim)
      throw Error(PDCS_ERR_SIZE, "count * dim must be <= 2^28");
    for (int64_t i = 0; i < dim * count; ++i) {
      if (!(f[i] > 0.0) || !std::isfinite(f[i])) throw Error(PDCS_ERR_INVALID_ARG, "factors must be finite and > 0");
      if (!std::isfinite(v[i])) throw Error(PDCS_ERR_INVALID_ARG, "points must be finite");
    }
    const size_t bytes = (size_t)count * dim * sizeof(double);
    DBuf dv, df, dout;
    dv.alloc(bytes);
    df.alloc(bytes);
    dout.alloc(bytes);
    HIP_OK(hipMemcpy(dv.p, v, bytes, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(df.p, f, bytes, hipMemcpyHostToDevice));
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (kernel_ms) {
      HIP_OK(hipEventCreate(&ev[0]));
      HIP_OK(hipEventCreate(&ev[1]));
      HIP_OK(hipEventRecord(ev[0], nullptr));
    }
    launch_proj_cone((int)cone, (int)dim, dv.as<double>(), df.as<double>(), dout.as<double>(), count, nullptr);
    hipError_t le = hipGetLastError();
    if (kernel_ms) {
      float ms = 0.0f;
      hipError_t e1 = hipEventRecord(ev[1], nullptr);
      hipError_t e2 = e1 == hipSuccess ? hipEventSynchronize(ev[1]) : e1;
      hipError_t e3 = e2 == hipSuccess ? hipEventElapsedTime(&ms, ev[0], ev[1]) : e2;
      (void)hipEventDestroy(ev[0]);
      (void)hipEventDestroy(ev[1]);
      HIP_OK(e3);
      *kernel_ms = ms;
    }
    HIP_OK(le);
    HIP_OK(hipMemcpy(out, dout.p, bytes, hipMemcpyDeviceToHost));
    return PDCS_OK;
  });
}

void pdcs_problem_destroy(pdcs_problem p) { delete p; }

int pdcs_problem_dims(pdcs_problem p, int64_t* m, int64_t* n, int64_t* nnz) {
  return guarded([&]() {
    if (!p) throw Error(PDCS_ERR_INVALID_ARG, "problem is null");
    if (m) *m = p->hp.m;
    if (n) *n = p->hp.n;
    if (nnz) *nnz = p->hp.nnz;
    return PDCS_OK;
  });
}

// Unscaled values in the storage order of the current layout, for the plain
// products: FP32 copies of the CSR / CSC values, and with band tiles the FP64
// and FP32 values in band-entry order.  Made once per layout, so that the plain
// products themselves allocate nothing.
void Engine::prepare_plain() {
  if (NNZ > 0 && !orig32.p) {
    orig32.alloc((size_t)NNZ * 4);
    origT32.alloc((size_t)NNZ * 4);
    launch_to_f32(d_v.as<double>(), orig32.as<float>(), NNZ, stream);
    launch_to_f32(d_vt.as<double>(), origT32.as<float>(), NNZ, stream);
  }
  if (use_band) {
    for (int tr = 0; tr < 2; ++tr) {
      BandSet& bs = tr ? band2 : band1;
      if (bs.nent > 0 && !bs.orig64.p) {
        bs.orig64.alloc((size_t)bs.nent * 8);
        bs.orig32.alloc((size_t)bs.nent * 4);
        launch_band_vals(bs.src.as<int32_t>(), bs.nent, tr ? d_vt.as<double>() : d_v.as<double>(),
                         bs.orig64.as<double>(), bs.orig32.as<float>(), stream);
      }
    }
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(stream));
}

// One plain product with the unscaled values; `part` receives the band
// layout's window partial sums (P x R values of the product's precision).
static void plain_spmv(Engine& e, bool transpose, bool f32, const void* in_dev, void* out_dev, void* part,
                       hipStream_t s) {
  if (e.use_band) {
    BandSet& bs = transpose ? e.band2 : e.band1;
    if (bs.nent > 0 && !bs.orig64.p) throw Error(PDCS_ERR_STATE, "band values not prepared");
    launch_band_plain(bs.view(), f32 ? kFP32 : kFP64, f32 ? bs.orig32.p : bs.orig64.p, in_dev, part, bs.R, out_dev, s);
  } else if (!transpose) {
    launch_spmv_plain(e.brow.view(), f32 ? kFP32 : kFP64, e.d_rp.as<int32_t>(), e.d_ci.as<int32_t>(),
                      f32 ? e.orig32.p : e.d_v.p, in_dev, out_dev, s);
  } else {
    launch_spmv_plain(e.bcol.view(), f32 ? kFP32 : kFP64, e.d_cp.as<int32_t>(), e.d_ri.as<int32_t>(),
                      f32 ? e.origT32.p : e.d_vt.p, in_dev, out_dev, s);
  }
  HIP_OK(hipGetLastError());
}

int pdcs_problem_spmv(pdcs_problem p, int64_t transpose, int64_t precision, const void* in_dev, void* out_dev,
                      void* stream) {
  return guarded([&]() {
    if (!p || !in_dev || !out_dev) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    if (precision != PDCS_PRECISION_FP64 && precision != PDCS_PRECISION_MIXED)
      throw Error(PDCS_ERR_INVALID_ARG, "unknown precision");
    Engine& e = *p->eng;
    const bool f32 = precision == PDCS_PRECISION_MIXED;
    BandSet& bs = transpose ? e.band2 : e.band1;
    plain_spmv(e, transpose != 0, f32, in_dev, out_dev, f32 ? bs.part32.p : bs.part64.p, (hipStream_t)stream);
    return PDCS_OK;
  });
}

// Scratch memory of pdcs_problem_spmv_noalloc: the band layout's window
// partial sums.  A file-scope device array, one copy per GPU, held until the
// process ends; every call on one GPU shares it.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device

// The device address of `scratch` on device `dev` (current), resolved once per
// device: the array's name in host code is a host-side stand-in, not a device
// address.
static void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error(PDCS_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !ptr)
      throw Error(PDCS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(err));
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

int pdcs_problem_spmv_noalloc(pdcs_problem p, int64_t transpose, int64_t precision, const void* in_dev,
                              void* out_dev, void* stream) {
  return guarded([&]() {
    if (!p || !in_dev || !out_dev) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    if (precision != PDCS_PRECISION_FP64 && precision != PDCS_PRECISION_MIXED)
      throw Error(PDCS_ERR_INVALID_ARG, "unknown precision");
    Engine& e = *p->eng;
    int cur = -1;
    HIP_OK(hipGetDevice(&cur));
    if (cur != e.device) throw Error(PDCS_ERR_INVALID_ARG, "the problem's device is not the current device");
    const bool f32 = precision == PDCS_PRECISION_MIXED;
    void* part = nullptr;
    if (e.use_band) {
      const BandSet& bs = transpose ? e.band2 : e.band1;
      const size_t need = (size_t)bs.P * (size_t)bs.R * (f32 ? 4 : 8);
      if (need > kNoAllocScratchBytes)
        throw Error(PDCS_ERR_SIZE, "window partial sums (" + std::to_string(need) + " B) exceed the " +
                                       std::to_string(kNoAllocScratchBytes) + " B scratch array");
      part = noalloc_scratch(cur);
    }
    plain_spmv(e, transpose != 0, f32, in_dev, out_dev, part, (hipStream_t)stream);
    return PDCS_OK;
  });
}

int pdcs_problem_set_layout(pdcs_problem p, int64_t layout) {
  return guarded([&]() {
    if (!p) throw Error(PDCS_ERR_INVALID_ARG, "problem is null");
    if (layout < PDCS_LAYOUT_AUTO || layout > PDCS_LAYOUT_WORKGROUP) throw Error(PDCS_ERR_INVALID_ARG, "unknown layout");
    p->eng->layout = (int)layout;
    p->eng->build_schedule();
    p->eng->prepare_plain();
    return PDCS_OK;
  });
}

int pdcs_solve(pdcs_problem p, const pdcs_options* opts, const double* x0, const double* y0, void* stream,
               pdcs_result* out) {
  return guarded([&]() {
    if (!p || !out) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    pdcs_options o;
    if (opts) o = *opts;
    else pdcs_options_default(&o);
    const double* xs[1] = {x0};
    const double* ys[1] = {y0};
    (void)stream;
    WarmStart ws;
    ws.hx = x0 ? xs : nullptr;
    ws.hy = y0 ? ys : nullptr;
    auto r = p->eng->solve(o, ws);
    *out = r[0];
    return PDCS_OK;
  });
}

int pdcs_solve_device(pdcs_problem p, const pdcs_options* opts, const void* x0_dev, const void* y0_dev,
                      int64_t warm_dtype, void* stream, pdcs_result* out) {
  return guarded([&]() {
    if (!p || !out) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    if (warm_dtype != PDCS_PRECISION_FP64 && warm_dtype != PDCS_PRECISION_MIXED)
      throw Error(PDCS_ERR_INVALID_ARG, "warm_dtype must be PDCS_PRECISION_FP64 or PDCS_PRECISION_MIXED");
    *out = nullptr;
    pdcs_options o;
    if (opts) o = *opts;
    else pdcs_options_default(&o);
    const void* xs[1] = {x0_dev};
    const void* ys[1] = {y0_dev};
    WarmStart ws;
    ws.dx = x0_dev ? xs : nullptr;
    ws.dy = y0_dev ? ys : nullptr;
    ws.dtype = warm_dtype == PDCS_PRECISION_MIXED ? 1 : 0;
    ws.caller = (hipStream_t)stream;
    auto r = p->eng->solve(o, ws);
    *out = r[0];
    return PDCS_OK;
  });
}

int pdcs_result_info(pdcs_result r, pdcs_info* out) {
  return guarded([&]() {
    if (!r || !out) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    *out = r->info;
    return PDCS_OK;
  });
}

static void copy_out(const DBuf& src, int64_t off, int64_t len, double* dst, int64_t want) {
  if (!dst) throw Error(PDCS_ERR_INVALID_ARG, "destination is null");
  if (want != len) throw Error(PDCS_ERR_INVALID_ARG, "length mismatch");
  if (len > 0) HIP_OK(hipMemcpy(dst, src.as<double>() + off, (size_t)len * 8, hipMemcpyDeviceToHost));
}

static void copy_out_device(const DBuf& src, int64_t off, int64_t len, double* dst, int64_t want, void* stream) {
  if (!dst) throw Error(PDCS_ERR_INVALID_ARG, "destination is null");
  if (want != len) throw Error(PDCS_ERR_INVALID_ARG, "length mismatch");
  if (len > 0)
    HIP_OK(hipMemcpyAsync(dst, src.as<double>() + off, (size_t)len * 8, hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

int pdcs_result_primal_device(pdcs_result r, double* x_dev, int64_t n, void* stream) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    copy_out_device(r->out->x, r->col0, r->n, x_dev, n, stream);
    return PDCS_OK;
  });
}

int pdcs_result_dual_device(pdcs_result r, double* y_dev, int64_t m, void* stream) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    if (r->m == 0 && m == 0) return PDCS_OK;
    copy_out_device(r->out->y, r->row0, r->m, y_dev, m, stream);
    return PDCS_OK;
  });
}

int pdcs_result_slack_device(pdcs_result r, double* lam_dev, int64_t n, void* stream) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    copy_out_device(r->out->lam, r->col0, r->n, lam_dev, n, stream);
    return PDCS_OK;
  });
}

int pdcs_result_primal(pdcs_result r, double* x, int64_t n) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    copy_out(r->out->x, r->col0, r->n, x, n);
    return PDCS_OK;
  });
}

int pdcs_result_dual(pdcs_result r, double* y, int64_t m) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    if (r->m == 0 && m == 0) return PDCS_OK;
    copy_out(r->out->y, r->row0, r->m, y, m);
    return PDCS_OK;
  });
}

int pdcs_result_slack(pdcs_result r, double* lam, int64_t n) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    copy_out(r->out->lam, r->col0, r->n, lam, n);
    return PDCS_OK;
  });
}

int pdcs_result_scaling(pdcs_result r, double* D1, int64_t m, double* D2, int64_t n) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    if (r->m > 0 || m > 0) copy_out(r->out->D1, r->row0, r->m, D1, m);
    copy_out(r->out->D2, r->col0, r->n, D2, n);
    return PDCS_OK;
  });
}

int pdcs_result_state(pdcs_result r, pdcs_state_scalars* s, double* x, double* y, double* x_hat, double* y_hat,
                      double* x_a, double* y_a) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    if (s) *s = r->st;
    double* dst[6] = {x, y, x_hat, y_hat, x_a, y_a};
    bool want = false;
    for (double* d : dst) want = want || d;
    if (!want) return PDCS_OK;
    if (!r->has_state) throw Error(PDCS_ERR_STATE, "solve ran without keep_state");
    const int pi = r->st.precision == PDCS_PRECISION_MIXED ? 1 : 0;
    for (int v = 0; v < 6; ++v) {
      if (!dst[v]) continue;
      const bool xlike = (v % 2 == 0);
      const int64_t off = xlike ? r->col0 : r->row0;
      const int64_t len = xlike ? r->n : r->m;
      if (len == 0) continue;
      const DBuf& src = r->out->st[pi][v];
      if (!src.p) throw Error(PDCS_ERR_STATE, "state not kept");
      if (pi == 0) {
        HIP_OK(hipMemcpy(dst[v], src.as<double>() + off, (size_t)len * 8, hipMemcpyDeviceToHost));
      } else {
        std::vector<float> tmp(len);
        HIP_OK(hipMemcpy(tmp.data(), src.as<float>() + off, (size_t)len * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < len; ++i) dst[v][i] = (double)tmp[i];
      }
    }
    return PDCS_OK;
  });
}

int pdcs_result_products(pdcs_result r, double* gty_hat, double* gx_hat) {
  return guarded([&]() {
    if (!r) throw Error(PDCS_ERR_INVALID_ARG, "result is null");
    if (!r->has_state) throw Error(PDCS_ERR_STATE, "solve ran without keep_state");
    const int pi = r->st.precision == PDCS_PRECISION_MIXED ? 1 : 0;
    double* dst[2] = {gty_hat, gx_hat};
    for (int v = 0; v < 2; ++v) {
      if (!dst[v]) continue;
      const int64_t off = v == 0 ? r->col0 : r->row0;
      const int64_t len = v == 0 ? r->n : r->m;
      const DBuf& src = r->out->st[pi][6 + v];
      if (len == 0) continue;
      if (pi == 0) {
        HIP_OK(hipMemcpy(dst[v], src.as<double>() + off, (size_t)len * 8, hipMemcpyDeviceToHost));
      } else {
        std::vector<float> tmp(len);
        HIP_OK(hipMemcpy(tmp.data(), src.as<float>() + off, (size_t)len * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < len; ++i) dst[v][i] = (double)tmp[i];
      }
    }
    return PDCS_OK;
  });
}

int pdcs_result_trace(pdcs_result r, double* out, int64_t max_trials, int64_t* count) {
  return guarded([&]() {
    if (!r || !out || !count || max_trials < 0) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    const int64_t rows = std::min<int64_t>(max_trials, (int64_t)(r->trace.size() / kTraceStride));
    std::memcpy(out, r->trace.data(), (size_t)rows * kTraceStride * 8);
    *count = rows;
    return PDCS_OK;
  });
}

void pdcs_result_destroy(pdcs_result r) { delete r; }

int pdcs_batch_create(int64_t count, const pdcs_problem* probs, pdcs_batch* out) {
  return guarded([&]() {
    if (!out || !probs || count < 1) throw Error(PDCS_ERR_INVALID_ARG, "bad batch arguments");
    *out = nullptr;
    std::vector<const HostProblem*> v;
    for (int64_t i = 0; i < count; ++i) {
      if (!probs[i]) throw Error(PDCS_ERR_INVALID_ARG, "null problem in batch");
      v.push_back(&probs[i]->hp);
    }
    auto b = std::make_unique<pdcs_batch_s>();
    b->eng = std::make_unique<Engine>(v);
    *out = b.release();
    return PDCS_OK;
  });
}

int pdcs_batch_solve(pdcs_batch b, const pdcs_options* opts, const double* const* x0s, const double* const* y0s,
                     void* stream, pdcs_result* results) {
  return guarded([&]() {
    if (!b || !results) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    pdcs_options o;
    if (opts) o = *opts;
    else pdcs_options_default(&o);
    (void)stream;
    WarmStart ws;
    ws.hx = x0s;
    ws.hy = y0s;
    auto r = b->eng->solve(o, ws);
    for (size_t i = 0; i < r.size(); ++i) results[i] = r[i];
    return PDCS_OK;
  });
}

int pdcs_batch_solve_device(pdcs_batch b, const pdcs_options* opts, const void* const* x0s_dev,
                            const void* const* y0s_dev, int64_t warm_dtype, void* stream, pdcs_result* results) {
  return guarded([&]() {
    if (!b || !results) throw Error(PDCS_ERR_INVALID_ARG, "null argument");
    if (warm_dtype != PDCS_PRECISION_FP64 && warm_dtype != PDCS_PRECISION_MIXED)
      throw Error(PDCS_ERR_INVALID_ARG, "warm_dtype must be PDCS_PRECISION_FP64 or PDCS_PRECISION_MIXED");
    pdcs_options o;
    if (opts) o = *opts;
    else pdcs_options_default(&o);
    WarmStart ws;
    ws.dx = x0s_dev;
    ws.dy = y0s_dev;
    ws.dtype = warm_dtype == PDCS_PRECISION_MIXED ? 1 : 0;
    ws.caller = (hipStream_t)stream;
    auto r = b->eng->solve(o, ws);
    for (size_t i = 0; i < r.size(); ++i) results[i] = r[i];
    return PDCS_OK;
  });
}

int pdcs_batch_schedule(pdcs_batch b, int64_t* iter_max, int64_t* block_nnz, int64_t* vec_per_block) {
  return guarded([&]() {
    if (!b) throw Error(PDCS_ERR_INVALID_ARG, "batch is null");
    if (iter_max) *iter_max = b->eng->sched.iter_max;
    if (block_nnz) *block_nnz = b->eng->sched.block_nnz;
    if (vec_per_block) *vec_per_block = b->eng->sched.vec_per_block;
    return PDCS_OK;
  });
}

int pdcs_batch_set_schedule(pdcs_batch b, int64_t iter_max, int64_t block_nnz, int64_t vec_per_block) {
  return guarded([&]() {
    if (!b) throw Error(PDCS_ERR_INVALID_ARG, "batch is null");
    if (iter_max < 1 || iter_max > 64 || block_nnz < 64 || block_nnz > (1 << 24) || vec_per_block < 256 ||
        vec_per_block > (1 << 22))
      throw Error(PDCS_ERR_INVALID_ARG, "schedule out of range");
    b->eng->sched = Schedule{(int)iter_max, (int)block_nnz, (int)vec_per_block};
    b->eng->build_schedule();
    return PDCS_OK;
  });
}

int pdcs_batch_set_layout(pdcs_batch b, int64_t layout) {
  return guarded([&]() {
    if (!b) throw Error(PDCS_ERR_INVALID_ARG, "batch is null");
    if (layout < PDCS_LAYOUT_AUTO || layout > PDCS_LAYOUT_WORKGROUP) throw Error(PDCS_ERR_INVALID_ARG, "unknown layout");
    b->eng->layout = (int)layout;
    b->eng->build_schedule();
    return PDCS_OK;
  });
}

static void set_band_schedule(Engine& e, int64_t rows, int64_t min_tiles, int64_t entry_cap) {
  if (rows < 256 || rows > kBandRows || (rows & (rows - 1)) != 0)
    throw Error(PDCS_ERR_INVALID_ARG, "band rows must be a power of two in [256, 8192]");
  if (min_tiles < 1 || min_tiles > (1 << 20)) throw Error(PDCS_ERR_INVALID_ARG, "min_tiles in [1, 2^20]");
  if (entry_cap < 1024 || entry_cap > (1 << 24)) throw Error(PDCS_ERR_INVALID_ARG, "entry_cap in [1024, 2^24]");
  e.bsched = BandSchedule{(int)rows, (int)min_tiles, (int)entry_cap};
  e.rebuild_bands();
}

static void get_band_schedule(const Engine& e, int64_t* rows, int64_t* min_tiles, int64_t* entry_cap,
                              int64_t* built_rows, int64_t* windows) {
  if (rows) *rows = e.bsched.rows;
  if (min_tiles) *min_tiles = e.bsched.min_tiles;
  if (entry_cap) *entry_cap = e.bsched.entry_cap;
  if (built_rows) *built_rows = e.use_band ? e.band1.band_rows : 0;
  if (windows) *windows = e.use_band ? e.band1.P : 0;
}

int pdcs_problem_set_band_schedule(pdcs_problem p, int64_t rows, int64_t min_tiles, int64_t entry_cap) {
  return guarded([&]() {
    if (!p) throw Error(PDCS_ERR_INVALID_ARG, "problem is null");
    set_band_schedule(*p->eng, rows, min_tiles, entry_cap);
    p->eng->prepare_plain();
    return PDCS_OK;
  });
}

int pdcs_batch_set_band_schedule(pdcs_batch b, int64_t rows, int64_t min_tiles, int64_t entry_cap) {
  return guarded([&]() {
    if (!b) throw Error(PDCS_ERR_INVALID_ARG, "batch is null");
    set_band_schedule(*b->eng, rows, min_tiles, entry_cap);
    return PDCS_OK;
  });
}

int pdcs_problem_band_schedule(pdcs_problem p, int64_t* rows, int64_t* min_tiles, int64_t* entry_cap,
                               int64_t* built_rows, int64_t* windows) {
  return guarded([&]() {
    if (!p) throw Error(PDCS_ERR_INVALID_ARG, "problem is null");
    get_band_schedule(*p->eng, rows, min_tiles, entry_cap, built_rows, windows);
    return PDCS_OK;
  });
}

int pdcs_batch_band_schedule(pdcs_batch b, int64_t* rows, int64_t* min_tiles, int64_t* entry_cap,
                             int64_t* built_rows, int64_t* windows) {
  return guarded([&]() {
    if (!b) throw Error(PDCS_ERR_INVALID_ARG, "batch is null");
    get_band_schedule(*b->eng, rows, min_tiles, entry_cap, built_rows, windows);
    return PDCS_OK;
  });
}

int pdcs_batch_autotune(pdcs_batch b, double time_budget_ms) {
  return guarded([&]() {
    if (!b) throw Error(PDCS_ERR_INVALID_ARG, "batch is null");
    b->eng->autotune(time_budget_ms);
    return PDCS_OK;
  });
}

void pdcs_batch_destroy(pdcs_batch b) { delete b; }

}  // extern "C"

namespace pdcs {

// Autotuner: time the SpMV-with-dual-step kernel (FP32 and FP64) and the
// primal pass over a grid of schedules on this batch, keep the fastest.
void Engine::autotune(double budget_ms) {
  if (budget_ms <= 0) budget_ms = 2000.0;
  pdcs_options o;
  pdcs_options_default(&o);
  o.precision = PDCS_PRECISION_MIXED;
  o.max_iter = 1;
  o.use_graph = 0;
  {
    auto rs = solve(o, WarmStart{});
    for (auto* r : rs) delete r;
  }
  // re-activate every instance so that the timed kernels do their full work
  std::vector<Inst> hi(B);
  HIP_OK(hipMemcpy(hi.data(), d_inst.p, sizeof(Inst) * B, hipMemcpyDeviceToHost));
  for (auto& I : hi) {
    I.status = kActive;
    I.pending = 0;
  }
  HIP_OK(hipMemcpy(d_inst.p, hi.data(), sizeof(Inst) * B, hipMemcpyHostToDevice));
  struct Cand {
    int iter_max, block_nnz;
  };
  const Cand cands[] = {{4, 4096}, {8, 4096}, {8, 8192}, {8, 16384}, {16, 8192}, {16, 16384}, {32, 16384},
                        {32, 32768}};
  const auto t0 = std::chrono::steady_clock::now();
  auto spent = [&]() { return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(); };
  // Row blocks: the layout of small batches, and of a band batch's tail once
  // compaction leaves fewer than 2^22 nonzeros running (timed with the bands
  // set aside).
  const bool band = use_band;
  band_suspended = band;
  Schedule best = sched;
  double best_t = 1e300;
  for (const Cand& c : cands) {
    sched.iter_max = c.iter_max;
    sched.block_nnz = c.block_nnz;
    build_schedule();
    const double t = time_dual(kFP32, 5) + time_dual(kFP64, 3);
    if (t < best_t) {
      best_t = t;
      best = sched;
    }
    if (spent() > (band ? 0.25 : 1.0) * budget_ms) break;
  }
  sched = best;
  build_schedule();
  band_suspended = false;
  if (!band) return;
  // Band tiles: band height, tile minimum and, in a batch, the per-window entry
  // cap of an instance's bands, timed on the trial product G x_hat (each
  // candidate rebuilds both band layouts on the host).  The candidates bracket
  // the defaults by a factor of 2.
  const BandSchedule base = bsched;
  const BandSchedule bc[] = {base,
                             {base.rows, base.min_tiles, std::max(1024, base.entry_cap / 2)},
                             {base.rows, base.min_tiles, base.entry_cap * 2},
                             {base.rows, base.min_tiles * 2, base.entry_cap},
                             {std::max(256, base.rows / 2), base.min_tiles, base.entry_cap}};
  BandSchedule bbest = base;
  double bbest_t = 1e300;
  for (const BandSchedule& c : bc) {
    if (&c != &bc[0] && spent() > budget_ms) break;
    bsched = c;
    rebuild_bands();
    const double t = time_dual(kFP32, 5);
    if (t < bbest_t) {
      bbest_t = t;
      bbest = c;
    }
  }
  bsched = bbest;
  rebuild_bands();
}

}  // namespace pdcs
