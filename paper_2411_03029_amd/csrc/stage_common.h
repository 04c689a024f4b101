// Shared by the transfer-stage kernels (apply.hip, stage_flat.hip): the
// arguments of one transfer step between a fine level and its coarse side,
// block and tree bookkeeping, and the workgroup-to-work mapping.
#pragma once

#include <hip/hip_runtime.h>

#include "cplx.h"
#include "tb_internal.h"

namespace tb {

constexpr int kThreads = 256;

struct StageArgs {
  int nb, nblk, lvl;              // blocks per mode, nb^d, fine level
  int nsplit, chunk;              // slices of the first output mode
  int R[kMaxD], A[kMaxD];         // fine padded ranks, coarse block sizes
  long long mat_item_stride;
  long long mat_k_off[kMaxD];
  long long fineE;                // entries per fine item
  long long fst[kMaxD];           // fine item strides (entries)
  int coarse_global;              // coarse is the caller's (nrhs, n^d) array
  long long coarseE;
  long long cst[kMaxD];           // coarse item strides (entries)
  long long n, ndim;              // n and n^d (global arrays)
  int outer_level, outer_block;   // outer multi-set level and block size
  int nrhs;
  int conj;
  const int* rank_f;              // true ranks of the fine level [item][k][blk]
  const int* rank_c;              // true ranks of the coarse level (null: leaves)
  int nb_c;                       // blocks per mode of a coarse item
  int Rc[kMaxD];                  // padded ranks of the coarse level
  int fib_out, fib_in;            // longest contracted extent of a fan-out / fan-in mode product
  int aff_blocks;                 // item blocks of one outer middle multi-set in the launch (0: none)
};

// True extent of mode k of the coarse block beta_k: the two children's
// skeletons of sizes h1, h2 sit at offsets 0 and Rc in the padded block.
// Leaves (caller's array) are dense: h1 = A, no second part.
struct Seg {
  int c, h1, off2;
  __device__ int pos(int j) const { return j < h1 ? j : off2 + (j - h1); }
};

template <int D>
__device__ __forceinline__ void unflatten_blk(int f, int nb, int* beta) {
#pragma unroll
  for (int k = D - 1; k >= 0; --k) {
    beta[k] = f % nb;
    f /= nb;
  }
}

template <int D>
__device__ __forceinline__ int parent_of(int item, int l) {
  int outer = item >> (D * l);
  int inner = item & ((1 << (D * l)) - 1);
  int pin = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int b = (inner >> (l * (D - 1 - k))) & ((1 << l) - 1);
    pin = (pin << (l - 1)) | (b >> 1);
  }
  return (outer << (D * (l - 1))) | pin;
}

template <int D>
__device__ __forceinline__ int child_of(int citem, int l, int c) {
  // citem at level l - 1; child c in [0, 2^D) at level l
  int outer = citem >> (D * (l - 1));
  int pin = citem & ((1 << (D * (l - 1))) - 1);
  int inner = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int pk = (l > 1) ? (pin >> ((l - 1) * (D - 1 - k))) & ((1 << (l - 1)) - 1) : 0;
    int ck = (c >> (D - 1 - k)) & 1;
    inner = (inner << l) | (2 * pk + ck);
  }
  return (outer << (D * l)) | inner;
}

// Address of element (j_0..j_{D-1}, q) of coarse block beta of coarse item
// `citem` (intermediate) or of outer block `citem` (global array).
template <int D>
struct CoarseAddr {
  long long base;
  long long stride[D];
  long long qstride;
  __device__ void init(const StageArgs& a, int citem, const int* beta, int q0) {
    if (a.coarse_global) {
      int o[D];
      unflatten_blk<D>(citem, 1 << a.outer_level, o);
      long long st = 1;
      base = 0;
#pragma unroll
      for (int k = D - 1; k >= 0; --k) {
        stride[k] = st;
        base += (long long)(o[k] * a.outer_block + beta[k] * a.A[k]) * st;
        st *= a.n;
      }
      qstride = a.ndim;
      base += (long long)q0 * a.ndim;
    } else {
      base = (long long)citem * a.coarseE;
#pragma unroll
      for (int k = 0; k < D; ++k) base += (long long)beta[k] * a.A[k] * a.cst[k];
      base = base * a.nrhs + q0;
#pragma unroll
      for (int k = 0; k < D; ++k) stride[k] = a.cst[k] * a.nrhs;
      qstride = 1;
    }
  }
};

template <int D>
__device__ __forceinline__ long long fine_base(const StageArgs& a, int fi, const int* beta, int q0,
                                               long long* stride) {
  long long base = (long long)fi * a.fineE;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    base += (long long)beta[k] * a.R[k] * a.fst[k];
    stride[k] = a.fst[k] * a.nrhs;
  }
  return base * a.nrhs + q0;
}

template <int D>
__device__ __forceinline__ void coarse_segs(const StageArgs& a, int citem, const int* beta, Seg* sg) {
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (a.rank_c == nullptr) {
      sg[k].c = a.A[k];
      sg[k].h1 = a.A[k];
      sg[k].off2 = 0;
    } else {
      const int* rc = a.rank_c + ((long long)citem * D + k) * a.nb_c + 2 * beta[k];
      sg[k].h1 = rc[0];
      sg[k].c = rc[0] + rc[1];
      sg[k].off2 = a.Rc[k];
    }
  }
}

// Register-blocked mode product shared by the stage kernels:
//   acc[g] += sum_{j < nj} m(g, j) x(j),  g < ng (wave-uniform, ng <= G).
// One thread owns a fiber x of the contracted mode and G outputs along the
// new mode, so each input element is loaded once per group of G outputs.
// G = 1 keeps every thread busy on small blocks (one right-hand side);
// G = 8 cuts loads when right-hand sides fill the workgroup.  The stage
// kernels take G (kG) as a template parameter; the autotuner picks it.
// Outputs g >= ng repeat row ng - 1 (an in-bounds read) and are never
// stored: the inner loop carries no per-output branch.
template <int G, class C, class MF, class XF>
__device__ __forceinline__ void gdot(C (&acc)[G], int ng, int nj, MF m, XF x) {
  int row[G];
#pragma unroll
  for (int g = 0; g < G; ++g) row[g] = min(g, ng - 1);
#pragma unroll 2
  for (int j = 0; j < nj; ++j) {
    const C xv = x(j);
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = cfma(acc[g], m(row[g], j), xv);
  }
}

template <int G, class C>
__device__ __forceinline__ void gzero(C (&acc)[G]) {
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = czero<C>();
}

// gdot with V right-hand sides per thread as well (x(j, v) is element j of
// right-hand side v): each matrix element loaded serves V products.  The
// order of the sum per output is the one of gdot.
template <int G, int V, class C, class MF, class XF>
__device__ __forceinline__ void gdotv(C (&acc)[G][V], int ng, int nj, MF m, XF x) {
  int row[G];
#pragma unroll
  for (int g = 0; g < G; ++g) row[g] = min(g, ng - 1);
#pragma unroll 2
  for (int j = 0; j < nj; ++j) {
    C xv[V];
#pragma unroll
    for (int v = 0; v < V; ++v) xv[v] = x(j, v);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const C mv = m(row[g], j);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[g][v] = cfma(acc[g][v], mv, xv[v]);
    }
  }
}

template <int G, int V, class C>
__device__ __forceinline__ void gzero2(C (&acc)[G][V]) {
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[g][v] = czero<C>();
}


// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// xcd_item maps workgroup b of n to work item u so that groups of g
// consecutive items (items that share data: the right-hand-side tiles of
// one block or core panel) run back to back on one XCD, while successive
// groups still go round-robin over the XCDs (irregular work stays balanced).
// The tail that does not fill 8 whole groups keeps the identity map; a
// bijection on [0, n) for any n and g.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int b, int n, int g) {
  const int span = kXcds * g;
  if (g <= 1 || b >= n / span * span) return b;
  const int x = b % kXcds, i = b / kXcds;  // i-th workgroup on XCD x
  return ((i / g) * kXcds + x) * g + i % g;
}

// Workgroup b of n -> work item, so that the items of one outer middle
// multi-set (s on the source side, t on the target side; `per` consecutive
// items each) all run on XCD (outer mod 8): successive launches of one side
// then read their inputs from the L2 that wrote them.  Needs n to be a
// multiple of 8 per; otherwise the XCD-grouped map of groups of g.
__device__ __forceinline__ int xcd_outer(int b, int n, long long per, int g) {
  const long long span = kXcds * per;
  if (per <= 0 || n % span != 0) return xcd_item(b, n, g);
  const int x = b % kXcds, r = b / kXcds;
  const long long outer = x + (long long)kXcds * (r / per);
  return (int)(outer * per + r % per);
}

// Workgroup -> (block, slice, right-hand-side tile); the tile index runs
// fastest, and the blocks of one outer middle multi-set share an XCD (or,
// when their count does not allow it, groups of one block's slices and
// tiles do), so that workgroups sharing cache lines run in the same L2.
struct StageBid {
  int item_blk, split, q0;
};
__device__ __forceinline__ StageBid stage_bid(const StageArgs& a, int QT) {
  const int nqt = (a.nrhs + QT - 1) / QT;
  const int g = nqt * a.nsplit;
  int bid = xcd_outer(blockIdx.x, gridDim.x, (long long)a.aff_blocks * g, g);
  StageBid s;
  s.q0 = (bid % nqt) * QT;
  bid /= nqt;
  s.split = bid % a.nsplit;
  s.item_blk = bid / a.nsplit;
  return s;
}

constexpr int kMaxChildren = 1 << kMaxDTuned;  // fan-in children of the tuned kernels

// Flat-staged transfer stages (stage_flat.hip), FP32, one right-hand side
// per workgroup; mode 1 = slices for about 1024 workgroups, 2 = whole blocks.
long long flat_lds_elems(const StageArgs& a, int d, bool fanout, int chunk);
tb_status launch_stage_flat_f32(StageArgs a, int d, bool fanout, int n_items, const void* in, void* out,
                                const void* mats, hipStream_t stream, int mode, int lds_limit);

// Register-fiber transfer stages (stage_fiber.hip), FP32 or FP64, one
// right-hand side per workgroup; xm bounds the contracted extents.
constexpr int kFibMaxLen = 32;
tb_status launch_stage_fib(bool fp64, const StageArgs& a, int d, bool fanout, int xm, long long nwg,
                           size_t lds, const void* in, void* out, const void* mats, hipStream_t stream);

// Leaf stages with one workgroup of 1 or 4 waves per leaf box
// (stage_leaf.hip), FP32 or FP64, one right-hand side per workgroup; leaf
// sizes 4, 8 and 16.
long long leaf_wave_lds_elems(const StageArgs& a, int d, bool fanout);
tb_status launch_leaf_wave(bool fp64, const StageArgs& a, int d, bool fanout, int waves, int n_items,
                           const void* in, void* out, const void* mats, hipStream_t stream, int lds_limit);

// Fan-in transfer stage on the matrix cores (stage_mfma4.hip), d = 3, FP32:
// four right-hand sides per workgroup on 4 x 4 matrix-core blocks, the
// children in turn, the coarse block accumulated in registers; fine ranks
// up to 8 and coarse blocks up to 16 per mode, transfer levels only.
tb_status launch_fanin_m4(const StageArgs& a, int d, int n_items, const void* in, void* out,
                          const void* mats, hipStream_t stream);
// The fan-out counterpart: one fine block and four right-hand sides per
// workgroup of four waves, in two halves of its first mode.
tb_status launch_fanout_m4(const StageArgs& a, int d, int n_items, const void* in, void* out,
                           const void* mats, hipStream_t stream);
// The leaf fan-in (target leaf, source leaf of the adjoint), leaf size 8:
// one leaf box and four right-hand sides per workgroup.
tb_status launch_leaf_fanin_m4(const StageArgs& a, int d, int n_items, const void* in, void* out,
                               const void* mats, hipStream_t stream);

// Generic apply for any number of modes (apply_generic.hip): per-workgroup
// scratch in global memory, FP64 (fp64) or FP32.
struct GenCoreArgs {
  int d, nrhs;
  long long nS, nT;              // middle multi-sets per side
  long long Es, Et;              // entries per top-level item (source / target)
  int Rs[kMaxD], Rt[kMaxD];      // padded ranks of the top levels
};
size_t gen_stage_scratch(const StageArgs& a, int d, bool fanout, int n_items, size_t esz);
tb_status launch_gen_stage(bool fp64, const StageArgs& a, int d, bool fanout, int n_items, const void* in,
                           void* out, const void* mats, void* scratch, hipStream_t stream);
tb_status launch_gen_core(bool fp64, const GenCoreArgs& g, bool adjoint, const void* cores,
                          const long long* core_off, const int* meta, long long npairs, int max_rt,
                          int max_rs, const void* in, void* out, hipStream_t stream);

}  // namespace tb
