// Internal definitions of the tensor butterfly library: plan layout, error
// handling and complex helpers shared by the host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "tb.h"

namespace tb {

constexpr int kMaxD = 6;          // modes handled by the construction and the generic apply
constexpr int kMaxDTuned = 3;     // modes handled by the tuned apply kernels
constexpr int kMaxCols = 88;      // widest ID (columns) the GPU QR accepts

using cd = std::complex<double>;

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);
tb_status fail(tb_status s, const std::string& msg);

#define TB_HIP_TRY(expr)                                                      \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return ::tb::fail(TB_ERR_HIP, std::string(#expr) + ": " +              \
                                        hipGetErrorString(e_));              \
  } while (0)

#define TB_TRY(expr)                                                          \
  do {                                                                        \
    tb_status s_ = (expr);                                                    \
    if (s_ != TB_OK) return s_;                                               \
  } while (0)

// ------------------------------------------------------------------ plan --
// One interpolative decomposition, host side, true rank.
struct IdRec {
  int r = 0, c = 0;
  std::vector<int> skel;  // r global per-mode indices, pivot order
  std::vector<cd> X;      // r x c, row-major
};

// One level of one side of the butterfly.
//
// Items at level l of the source side are (s, tau): s a source middle
// multi-set (level Ls), tau a target multi-set at level l; flat item index
// s_flat * 2^(d l) + tau_flat.  Target side: (t, nu), t at level Lt, nu at
// level l, item t_flat * 2^(d l) + nu_flat.  Every item holds, per mode k,
// nb = 2^depth IDs (depth = Lt - l on the source side, Ls - l on the target
// side), one per tree node below the middle-level node of that mode.
//
// Device layout (padded to the level's largest rank per mode, zeros in the
// padding):
//   X:   [item][k][blk][R[k]][A[k]]  A[k] = leaf (l = 0) or 2 R_prev[k]; a
//        column j of an ID maps to padded column j (first child, j < r1)
//        or R_prev + j - r1 (second child)
//   item tensors in the workspace: dims (nb R[0], ..., nb R[d-1]) row-major,
//        right-hand side innermost.
struct Level {
  int l = 0, nitems = 0, nb = 1;
  int R[kMaxD] = {};
  int A[kMaxD] = {};
  std::vector<IdRec> ids;  // [item][k][blk]
  long long mat_item_stride = 0;        // complex elements per item
  long long mat_k_off[kMaxD] = {};
  long long E = 0;                      // entries per item tensor
  double2* X64 = nullptr;
  float2* X32 = nullptr;
  int* rank_d = nullptr;                // true ranks [item][k][blk]
  mutable int pair_max = -1;            // largest sum of two sibling blocks' ranks (-1: not yet known)
  const IdRec& id(int item, int k, int blk, int d) const {
    return ids[((size_t)item * d + k) * nb + blk];
  }
};

// Per-pair metadata for the cores, device side: RT, RS, RTp, rt[kMaxD] (at
// 3), rs[kMaxD] (at kMetaRs).
constexpr int kMetaRs = 3 + kMaxD;
constexpr int kPairMeta = 3 + 2 * kMaxD;

struct StageEvent {
  int stage;
  hipEvent_t start, stop;
};

struct Workspace {
  void* base = nullptr;
  size_t bytes = 0;
};

// Launch configuration of one apply kernel (0 = the built-in heuristic).
struct LaunchCfg {
  int G = 0;      // transfer: outputs per thread along the new mode (1 or 8)
  int QT = 0;     // transfer: right-hand sides per workgroup (1, 2, 4, 8)
  int split = 0;  // transfer: 1 = one workgroup per block (no slicing)
  int core = 0;   // core: 1 = vector, 1 RHS per pass; 2 = vector, 4; 3 = FP32 MFMA;
                  // 4 = BF16 MFMA (BF16 cores); 5-7 = BF16 MFMA, second form (three
                  // tiles); 8, 9 = adjoint vector kernel, 16-lane column groups, 1 / 4 RHS
  int alt = 0;    // fan-in: 1 = children in turn, mode 0 in registers; 2 = children in
                  // turn, mode 0 first; fan-out or fan-in, FP32: 3 = flat staging;
                  // fan-out or fan-in: 4 = register fibers; leaves: 5 = one wave per box
  int mfma = 0;   // transfer levels: 1 = mode products on the matrix cores
  int V = 0;      // transfer: right-hand sides per thread (1 or 4; 4 needs QT >= 4)
};

struct Plan {
  int kind = 0, d = 0, leaf = 8, L = 0, Lt = 0, Ls = 0;
  long long n = 0;
  double omega = 0, tol = 0, eps_id = 0;
  double ra = 2, rb = 1, rden = 3;
  std::vector<double> nux;           // TB_KERNEL_NUDFT: d * n target coordinates
  double* nux_d = nullptr;
  int proxy_pair = 2, proxy_other = 4;
  std::vector<Level> src, tgt;

  // cores: pair index t_flat * nS + s_flat, column-major R_T x R_S padded to
  // RTp rows (multiple of 4), pairs contiguous
  long long nT = 0, nS = 0, npairs = 0;
  std::vector<int> pair_meta;        // npairs * kPairMeta
  std::vector<long long> core_off;   // npairs (elements)
  long long core_total = 0;          // elements incl. padding
  unsigned store_mask = TB_STORE_C64;
  void* cores[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // indexed by tb_dtype
  // TB_CQ16 cores: one scale per core column at col_off[pair] + column
  float* core_scale = nullptr;
  std::vector<long long> col_off;    // npairs (columns before the pair)
  long long* col_off_d = nullptr;
  long long col_total = 0;
  int* pair_meta_d = nullptr;
  long long* core_off_d = nullptr;
  // core work lists: forward row panels of 64 VR rows (index log2 VR, for
  // VR = 1, 2, 4 rows per 16-byte load)
  std::vector<int2> fwd_units[3];
  int2* fwd_units_d[3] = {nullptr, nullptr, nullptr};
  // many right-hand sides (matrix cores): 256-row / 256-column panels
  std::vector<int2> mfma_fwd_units, mfma_adj_units;
  int2* mfma_fwd_units_d = nullptr;
  int2* mfma_adj_units_d = nullptr;
  // adjoint panels (pair, first column) of 64 columns: vector and on-the-fly
  std::vector<int2> adj_units;
  int2* adj_units_d = nullptr;
  // device skeleton tables of the two top levels (core evaluation)
  int* top_src_skel_d = nullptr;     // [item][k][Rs]
  int* top_tgt_skel_d = nullptr;     // [item][k][Rt]

  size_t device_bytes = 0;
  size_t max_device_bytes = 0;
  double construct_ms = 0;
  Workspace ws;
  std::vector<void*> allocations;
  bool timing = false;
  std::vector<StageEvent> events;
  // autotuned launch configurations per (tb_dtype, nrhs): one entry per
  // kernel launch of the forward sequence followed by the adjoint one
  std::map<std::pair<int, long long>, std::vector<LaunchCfg>> tuned;

  ~Plan();
};

// host helpers (plan.cpp)
tb_status dev_alloc(Plan& p, void** ptr, size_t bytes);
tb_status finalize_plan(Plan& p, hipStream_t stream);  // pads + uploads factors
tb_status build_core_tables(Plan& p);
tb_status set_nudft_points(Plan& p, const double* x);  // checks, copies, uploads
long long apply_cmacs(const Plan& p, long long* per_stage = nullptr);
void stage_io_entries(const Plan& p, long long* out5);

// kernels launched by host code
tb_status launch_core_eval(Plan& p, hipStream_t stream, const double2* host_cores);
tb_status run_apply(Plan& p, const void* in, void* out, long long nrhs,
                    tb_dtype io, bool adjoint, hipStream_t stream,
                    void* ws_ext = nullptr, size_t ws_cap = 0);
tb_status run_construct_ids(Plan& p, hipStream_t stream);
tb_status prepare_workspace(Plan& p, long long nrhs, tb_dtype io);
tb_status run_autotune(Plan& p, long long nrhs, tb_dtype io, const char* cache, hipStream_t stream,
                       int* trials);
void drop_graphs_for(const Plan* p);

inline int ipow2(int e) { return 1 << e; }

}  // namespace tb
