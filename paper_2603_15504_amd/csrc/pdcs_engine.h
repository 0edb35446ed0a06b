// Host-side objects of the PDCS LP solver (device buffers, schedules, engine).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pdcs.h"
#include "pdcs_launch.h"

namespace pdcs {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define HIP_OK(expr)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) {                                                                        \
      (void)hipGetLastError();                                                                     \
      throw ::pdcs::Error(PDCS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    }                                                                                              \
  } while (0)

// Owning device allocation (never zero-sized, so pointers are always valid).
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void alloc(size_t b);
  void release();
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// One validated LP in host memory, with its transpose (CSC) built.
struct HostProblem {
  int64_t m = 0, n = 0, m_zero = 0, nnz = 0;
  std::vector<int32_t> rp, ci, cp, ri;
  std::vector<double> v, vt, h, c, l, u;
  std::vector<int32_t> soc;  // second-order-cone block dimensions (after the nonnegative rows)
  int64_t n_exp = 0, n_dexp = 0;  // exponential / dual-exponential blocks of 3 rows (the last rows)
  int64_t cone_rows() const;
  void build(int64_t m, int64_t n, int64_t mz, const int64_t* row_ptr, const int32_t* col_idx,
             const double* val, const double* h, const double* c, const double* l, const double* u,
             int64_t n_soc = 0, const int64_t* soc_dims = nullptr, int64_t n_exp = 0, int64_t n_dexp = 0);
};

// Tile schedule parameters (chosen by pdcs_batch_autotune or set explicitly).
struct Schedule {
  int iter_max = 8;        // passes per lane group in a multi-row wavefront tile
  int block_nnz = 8192;    // work units (nonzeros + 4 per row) per workgroup
  int vec_per_block = 1024;  // elements per workgroup in elementwise passes
};

struct TileSet {
  DBuf row0, row1, lg, btile0, btile1, binst_d, iblk0_d;
  int nblk = 0, ntiles = 0;
  std::vector<int32_t> h_bt0, h_bt1, h_t0, h_t1, h_binst;
  // active: optional per-instance mask; instances outside it get no workgroups
  void build(const std::vector<int32_t>& ptr, const std::vector<int64_t>& inst_r0, const Schedule& s,
             const std::vector<char>* active = nullptr);
  Tiles view() const;
};

// Row blocks: a single row of any length, or consecutive rows with at most
// kRowBlockCap nonzeros whose per-row reduction needs at most red_max passes.
struct RowBlockSet {
  DBuf r0, r1, binst_d, iblk0_d;
  int nblk = 0;
  std::vector<int32_t> h_binst, h_iblk0;  // host copies: block -> instance, instance -> first block
  void build(const std::vector<int32_t>& ptr, const std::vector<int64_t>& inst_r0, int red_max,
             const std::vector<char>* active = nullptr);
  RowBlocks view() const;
};

// Cone row blocks of all instances: first (absolute) row, dimension and kind
// (0 second-order, 1 exponential, 2 dual exponential) of each block, in row order.
struct SocTable {
  std::vector<int32_t> r0, dim;
  std::vector<int8_t> kind;
  DBuf r0_d, dim_d, kind_d;
  bool empty() const { return r0.empty(); }
};

struct RangeSet {
  DBuf start, end, binst_d, iblk0_d, soc0_d, soc1_d;
  int nblk = 0;
  std::vector<int32_t> h_iblk0;  // host copy: instance -> first block
  const SocTable* soc = nullptr;  // set for row ranges that must not split cone blocks
  int cone_cap = 1;               // at most this many cone blocks per range
  void build(const std::vector<int64_t>& inst_off, int per_block, const std::vector<char>* active = nullptr);
  Ranges view() const;
};

// Shape of the band tiles: the tallest band height (a power of two, at most
// kBandRows), halved while fewer than min_tiles band-tiles would result; in a
// batch, bands are further cut to at most about entry_cap entries per window.
struct BandSchedule {
  int rows = kBandRows;
  int min_tiles = 384;
  int entry_cap = 32768;
};

// Band-tile layout of a CSR-like structure (see BandTiles), per instance of a
// batch.  src maps every packed entry to its position in
// the CSR order (-1 for padding), so the scaled values can be filled in.
struct BandSet {
  int P = 1;
  int ntile = 0, nslot = 0;
  int64_t R = 0, nent = 0;
  DBuf group, slot, start, row0, nrows, used, tinst, col0, panel, run_start, run_row, run_ext, ext, pk, src;
  DBuf val32, val64, part32, part64, part64b;
  DBuf orig32, orig64;  // unscaled values (plain products), filled by Engine::prepare_plain
  // instance b: rows [r0s[b], r0s[b+1]) gathering from [g0s[b], g0s[b+1])
  int band_rows = 0;  // band height chosen by build
  void reset();       // back to the unbuilt state, device memory released
  void build(const std::vector<int64_t>& r0s, const std::vector<int64_t>& g0s, const std::vector<int32_t>& ptr,
             const std::vector<int32_t>& idx, const BandSchedule& bs);
  BandTiles view() const;
};

template <typename T>
struct IterBufs {
  DBuf b[16];
  IterPtrs<T> p{};
  bool ready = false;
  void alloc(int64_t N, int64_t M);
};

// Device copies of one solve's outputs, shared by the results of a batch.
struct OutBlock {
  int64_t M = 0, N = 0;
  DBuf x, y, lam, D1, D2;
  DBuf st[2][8];  // [fp64, fp32] x [x, y, x_hat, y_hat, x_a, y_a, G^T y_hat, G x_hat]
};

// Where a solve's warm start comes from: host arrays (hx / hy) or device
// pointers (dx / dy, FP64 when dtype is 0, FP32 when 1) that become readable
// once the work enqueued on `caller` has run.  All null: no warm start.
struct WarmStart {
  const double* const* hx = nullptr;
  const double* const* hy = nullptr;
  const void* const* dx = nullptr;
  const void* const* dy = nullptr;
  int dtype = 0;
  hipStream_t caller = nullptr;
};

struct Engine {
  int B = 0;
  int device = 0;                                // HIP device current at creation
  int64_t M = 0, N = 0, NNZ = 0;
  std::vector<int64_t> row0, col0, mzero, socstart;  // socstart: first cone row per instance
  std::vector<int32_t> h_rp, h_cp;
  DBuf d_rp, d_ci, d_v, d_cp, d_ri, d_vt, d_h, d_c, d_l, d_u;
  DBuf orig32, origT32;
  DBuf val64, valT64, val32, valT32;
  DBuf h64, c64, l64, u64, h32, c32, l32, u32;
  DBuf D1, D2, cgx0, cgx1, cgty0, cgty1, xout, yout, lamout, stat_r, stat_c;
  DBuf rec_primal, rec_dual, rec_lam, rec_cand_c, rec_cand_r, rec_probe_c, rec_probe_r;
  DBuf rec_nc, rec_nr, rec_nm;
  DBuf d_inst, d_summary, warm_x, warm_y, d_trace;
  DBuf d_row0i, d_col0i, warm_ptr, d_flag;       // instance offsets, device warm-start pointer table
  DBuf xs0, ys0, rx, ry, rgx, rgty;              // infeasibility rays (FP64)
  bool any_unbounded = false;                    // some column has an infinite bound
  int infeas_on = 0;                             // the running solve runs the infeasibility tests
  int32_t* h_summary = nullptr;
  IterBufs<float> it32;
  IterBufs<double> it64;
  Schedule sched;
  TileSet trow, tcol;
  RowBlockSet brow, bcol;
  SocTable soc;                // second-order-cone row blocks (absolute rows)
  RangeSet vrow, vcol;
  RangeSet crow, ccol;         // coarser blocks for the multisection passes
  std::vector<int32_t> h_ci, h_ri;
  DBuf rec_dual_epi, rec_lam_epi;
  int layout = PDCS_LAYOUT_AUTO;
  bool use_band = false;
  bool wg_trials = false;           // chunks of trials by one workgroup per instance
  size_t lds_bytes[2] = {0, 0};     // FP32 / FP64: dynamic LDS of the LDS-resident chunk kernel (0: not used)
  bool lds_rowwise = false;         // its dual and dual-slack passes take one thread per row
  void plan_lds_trials();
  bool band_suspended = false;      // auto layout: the active instances of a batch fell below the band threshold
  BandSet band1, band2;             // band tiles of G (gathers x) and G^T (gathers y)
  BandSchedule bsched;              // shape of both band layouts
  hipStream_t stream = nullptr;
  std::map<int64_t, hipGraphExec_t> graphs;
  std::vector<hipEvent_t> events;
  size_t ev_used = 0;
  double timed_ms = 0.0;
  int64_t timed_count = 0;

  explicit Engine(const std::vector<const HostProblem*>& probs);
  ~Engine();
  void build_schedule();
  // iteration schedules over the instances in `active` (all when null)
  void build_iteration_schedules(const std::vector<char>* active);
  void clear_graphs();
  void ensure_iter(int prec);
  KernelCtx ctx(int probe_passes) const;
  void enqueue_chunk(const KernelCtx& k, int mask, int64_t K, bool timed);
  void harvest_events();
  std::vector<struct pdcs_result_s*> solve(const pdcs_options& o, const WarmStart& ws);
  double time_dual(int prec, int reps);
  double time_band_trial(int reps);
  void rebuild_bands();
  // unscaled values in the storage order of the current layout (plain products)
  void prepare_plain();
  void autotune(double budget_ms);
};

}  // namespace pdcs

struct pdcs_problem_s {
  pdcs::HostProblem hp;
  std::unique_ptr<pdcs::Engine> eng;
};

struct pdcs_result_s {
  std::shared_ptr<pdcs::OutBlock> out;
  int64_t row0 = 0, col0 = 0, m = 0, n = 0;
  pdcs_info info{};
  pdcs_state_scalars st{};
  bool has_state = false;
  std::vector<double> trace;
};

struct pdcs_batch_s {
  std::unique_ptr<pdcs::Engine> eng;
};
