// Contraction of a tensor butterfly with an input tensor (Algorithm 2) and
// its conjugate transpose, as HIP kernels for gfx950.
//
// Every transfer step of Algorithm 2 connects the items of one level l
// ("fine": they own the interpolation/transfer matrices) with their parents
// at level l - 1 ("coarse"), or with the caller's array for l = 0.  Along each
// mode the factor is block diagonal, so the multi-mode product splits into
// independent blocks: block beta of a fine item (R_0 x ... x R_{d-1}) pairs
// with block beta of its coarse item (A_0 x ... x A_{d-1}), A_k = 2 R_prev
// (the two children's skeletons) or the leaf size.
//
//   fan-out  coarse -> fine, op = M (source side forward, contract_transfer
//            of Algorithm 2) or conj(M) (target side adjoint)
//   fan-in   sum over the 2^d fine children -> coarse, op = M^T (target side
//            forward, the accumulation into the parent of Algorithm 2) or
//            M^H (source side adjoint)
//   core     G_{t,s} = K(tbar, sbar) F_{t,s} (forward) or C^H (adjoint)
//
// One workgroup handles one block; the first mode product reads the block
// straight from global memory, the middle ones run in LDS and the last one
// writes global memory (fan-out) or accumulates in registers over the
// children (fan-in), so a block never needs more than two LDS buffers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cplx.h"
#include "tb_internal.h"

namespace tb {

constexpr int kThreads = 256;
constexpr int kMaxPer = 32;     // fan-in outputs per thread (registers)
constexpr int kCoreRows = 64;   // forward core: rows per workgroup
constexpr int kCoreCols = 16;   // adjoint core: columns per workgroup

struct StageArgs {
  int nb, nblk, lvl;              // blocks per mode, nb^d, fine level
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
  int nrhs, Q;
  int conj;
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

// Loads the d matrices of (item, beta) into LDS, conjugated on request.
template <class C, int D>
__device__ void load_mats(const StageArgs& a, const C* mats, int item, const int* beta, C* sm,
                          C** mk) {
  int off = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    mk[k] = sm + off;
    int cnt = a.R[k] * a.A[k];
    const C* src = mats + (long long)item * a.mat_item_stride + a.mat_k_off[k] +
                   (long long)beta[k] * cnt;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
      C v = src[i];
      if (a.conj) v.y = -v.y;
      mk[k][i] = v;
    }
    off += cnt;
  }
}

template <int D>
__device__ __forceinline__ int mats_lds(const StageArgs& a) {
  int s = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) s += a.R[k] * a.A[k];
  return s;
}

// --------------------------------------------------------------- fan-out --
// fine(a_0..a_{D-1}, q) = sum_j prod_k M_k[a_k][j_k] coarse(j_0..j_{D-1}, q)
template <class T, int D>
__global__ void __launch_bounds__(kThreads)
    stage_fanout(StageArgs a, const typename CplxOf<T>::type* __restrict__ coarse,
                 typename CplxOf<T>::type* __restrict__ fine,
                 const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int fi = blockIdx.x / a.nblk;
  int beta[D];
  unflatten_blk<D>(blockIdx.x % a.nblk, a.nb, beta);
  const int q0 = blockIdx.y * a.Q;
  const int Q = min(a.Q, a.nrhs - q0);
  C* mk[D];
  load_mats<C, D>(a, mats, fi, beta, sm, mk);
  C* buf1 = sm + mats_lds<D>(a);
  const int citem = a.coarse_global ? (fi >> (D * a.lvl)) : parent_of<D>(fi, a.lvl);
  CoarseAddr<D> ca;
  ca.init(a, citem, beta, q0);
  long long fs[D];
  const long long fb = fine_base<D>(a, fi, beta, q0, fs);
  const int R0 = a.R[0], A0 = a.A[0];
  __syncthreads();
  if constexpr (D == 2) {
    const int A1 = a.A[1], R1 = a.R[1];
    // buf1[a0][j1][q] = sum_j0 M0[a0][j0] coarse(j0, j1, q)
    for (int idx = threadIdx.x; idx < R0 * A1 * Q; idx += blockDim.x) {
      int q = idx % Q, t = idx / Q, j1 = t % A1, a0 = t / A1;
      const C* src = coarse + ca.base + j1 * ca.stride[1] + q * ca.qstride;
      C acc = czero<C>();
      for (int j0 = 0; j0 < A0; ++j0) acc = cfma(acc, mk[0][a0 * A0 + j0], src[j0 * ca.stride[0]]);
      buf1[idx] = acc;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < R0 * R1 * Q; idx += blockDim.x) {
      int q = idx % Q, t = idx / Q, a1 = t % R1, a0 = t / R1;
      const C* src = buf1 + (a0 * A1) * Q + q;
      C acc = czero<C>();
      for (int j1 = 0; j1 < A1; ++j1) acc = cfma(acc, mk[1][a1 * A1 + j1], src[j1 * Q]);
      fine[fb + a0 * fs[0] + a1 * fs[1] + q] = acc;
    }
  } else {
    const int A1 = a.A[1], A2 = a.A[2], R1 = a.R[1], R2 = a.R[2];
    C* buf2 = buf1 + R0 * A1 * A2 * Q;
    for (int idx = threadIdx.x; idx < R0 * A1 * A2 * Q; idx += blockDim.x) {
      int q = idx % Q, t = idx / Q, j2 = t % A2;
      t /= A2;
      int j1 = t % A1, a0 = t / A1;
      const C* src = coarse + ca.base + j1 * ca.stride[1] + j2 * ca.stride[2] + q * ca.qstride;
      C acc = czero<C>();
      for (int j0 = 0; j0 < A0; ++j0) acc = cfma(acc, mk[0][a0 * A0 + j0], src[j0 * ca.stride[0]]);
      buf1[idx] = acc;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < R0 * R1 * A2 * Q; idx += blockDim.x) {
      int q = idx % Q, t = idx / Q, j2 = t % A2;
      t /= A2;
      int a1 = t % R1, a0 = t / R1;
      const C* src = buf1 + ((a0 * A1) * A2 + j2) * Q + q;
      C acc = czero<C>();
      for (int j1 = 0; j1 < A1; ++j1) acc = cfma(acc, mk[1][a1 * A1 + j1], src[j1 * A2 * Q]);
      buf2[idx] = acc;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < R0 * R1 * R2 * Q; idx += blockDim.x) {
      int q = idx % Q, t = idx / Q, a2 = t % R2;
      t /= R2;
      int a1 = t % R1, a0 = t / R1;
      const C* src = buf2 + ((a0 * R1 + a1) * A2) * Q + q;
      C acc = czero<C>();
      for (int j2 = 0; j2 < A2; ++j2) acc = cfma(acc, mk[2][a2 * A2 + j2], src[j2 * Q]);
      fine[fb + a0 * fs[0] + a1 * fs[1] + a2 * fs[2] + q] = acc;
    }
  }
}

// ---------------------------------------------------------------- fan-in --
// coarse(a_0..a_{D-1}, q) = sum_children sum_j prod_k M_k[j_k][a_k] fine_c(j, q)
template <class T, int D>
__global__ void __launch_bounds__(kThreads)
    stage_fanin(StageArgs a, const typename CplxOf<T>::type* __restrict__ fine,
                typename CplxOf<T>::type* __restrict__ coarse,
                const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int ci = blockIdx.x / a.nblk;
  int beta[D];
  unflatten_blk<D>(blockIdx.x % a.nblk, a.nb, beta);
  const int q0 = blockIdx.y * a.Q;
  const int Q = min(a.Q, a.nrhs - q0);
  const int nchild = a.coarse_global ? 1 : (1 << D);
  C acc[kMaxPer];
#pragma unroll
  for (int i = 0; i < kMaxPer; ++i) acc[i] = czero<C>();
  int nout = Q;
#pragma unroll
  for (int k = 0; k < D; ++k) nout *= a.A[k];
  C* buf1 = sm + mats_lds<D>(a);
  const int R0 = a.R[0], A0 = a.A[0];
  for (int c = 0; c < nchild; ++c) {
    const int fi = a.coarse_global ? ci : child_of<D>(ci, a.lvl, c);
    C* mk[D];
    __syncthreads();
    load_mats<C, D>(a, mats, fi, beta, sm, mk);
    long long fs[D];
    const long long fb = fine_base<D>(a, fi, beta, q0, fs);
    __syncthreads();
    if constexpr (D == 2) {
      const int R1 = a.R[1], A1 = a.A[1];
      // buf1[a0][j1][q] = sum_j0 M0[j0][a0] fine(j0, j1, q)
      for (int idx = threadIdx.x; idx < A0 * R1 * Q; idx += blockDim.x) {
        int q = idx % Q, t = idx / Q, j1 = t % R1, a0 = t / R1;
        const C* src = fine + fb + j1 * fs[1] + q;
        C s = czero<C>();
        for (int j0 = 0; j0 < R0; ++j0) s = cfma(s, mk[0][j0 * A0 + a0], src[j0 * fs[0]]);
        buf1[idx] = s;
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kMaxPer; ++i) {
        int idx = threadIdx.x + i * kThreads;
        if (idx < nout) {
          int q = idx % Q, t = idx / Q, a1 = t % A1, a0 = t / A1;
          const C* src = buf1 + (a0 * R1) * Q + q;
          C s = acc[i];
          for (int j1 = 0; j1 < R1; ++j1) s = cfma(s, mk[1][j1 * A1 + a1], src[j1 * Q]);
          acc[i] = s;
        }
      }
    } else {
      const int R1 = a.R[1], R2 = a.R[2], A1 = a.A[1], A2 = a.A[2];
      C* buf2 = buf1 + A0 * R1 * R2 * Q;
      for (int idx = threadIdx.x; idx < A0 * R1 * R2 * Q; idx += blockDim.x) {
        int q = idx % Q, t = idx / Q, j2 = t % R2;
        t /= R2;
        int j1 = t % R1, a0 = t / R1;
        const C* src = fine + fb + j1 * fs[1] + j2 * fs[2] + q;
        C s = czero<C>();
        for (int j0 = 0; j0 < R0; ++j0) s = cfma(s, mk[0][j0 * A0 + a0], src[j0 * fs[0]]);
        buf1[idx] = s;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < A0 * A1 * R2 * Q; idx += blockDim.x) {
        int q = idx % Q, t = idx / Q, j2 = t % R2;
        t /= R2;
        int a1 = t % A1, a0 = t / A1;
        const C* src = buf1 + ((a0 * R1) * R2 + j2) * Q + q;
        C s = czero<C>();
        for (int j1 = 0; j1 < R1; ++j1) s = cfma(s, mk[1][j1 * A1 + a1], src[j1 * R2 * Q]);
        buf2[idx] = s;
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kMaxPer; ++i) {
        int idx = threadIdx.x + i * kThreads;
        if (idx < nout) {
          int q = idx % Q, t = idx / Q, a2 = t % A2;
          t /= A2;
          int a1 = t % A1, a0 = t / A1;
          const C* src = buf2 + ((a0 * A1 + a1) * R2) * Q + q;
          C s = acc[i];
          for (int j2 = 0; j2 < R2; ++j2) s = cfma(s, mk[2][j2 * A2 + a2], src[j2 * Q]);
          acc[i] = s;
        }
      }
    }
  }
  CoarseAddr<D> ca;
  ca.init(a, ci, beta, q0);
#pragma unroll
  for (int i = 0; i < kMaxPer; ++i) {
    int idx = threadIdx.x + i * kThreads;
    if (idx < nout) {
      int q = idx % Q, t = idx / Q;
      long long off = ca.base + q * ca.qstride;
#pragma unroll
      for (int k = D - 1; k >= 0; --k) {
        off += (long long)(t % a.A[k]) * ca.stride[k];
        t /= a.A[k];
      }
      coarse[off] = acc[i];
    }
  }
}

// ------------------------------------------------------------------ core --
struct CoreArgs {
  long long nS, nT;              // middle multi-sets per side
  long long Es, Et;              // entries per top-level item (source / target)
  int Rs[kMaxD], Rt[kMaxD];      // padded ranks of the top levels
  int nrhs, Q;
};

template <int D>
__device__ __forceinline__ long long padded_pos(int flat, const int* r, const int* Rp) {
  // flat index over true ranks r (mode D-1 fastest) -> padded position
  long long pos = 0, st = 1;
#pragma unroll
  for (int k = D - 1; k >= 0; --k) {
    pos += (long long)(flat % r[k]) * st;
    flat /= r[k];
    st *= Rp[k];
  }
  return pos;
}

template <int D>
__device__ __forceinline__ bool is_padding(long long pos, const int* r, const int* Rp) {
  bool pad = false;
#pragma unroll
  for (int k = D - 1; k >= 0; --k) {
    pad |= (pos % Rp[k]) >= r[k];
    pos /= Rp[k];
  }
  return pad;
}

// G_{t,s}(rows) = C_{t,s}(rows, :) F_{t,s}; one workgroup = 64 rows of one
// pair, its four waves split the columns and reduce through LDS.
template <class T, class CS, int D>
__global__ void __launch_bounds__(kThreads)
    core_fwd(CoreArgs a, const CS* __restrict__ cores, const long long* __restrict__ core_off,
             const int* __restrict__ meta, const int2* __restrict__ units,
             const typename CplxOf<T>::type* __restrict__ F, typename CplxOf<T>::type* __restrict__ G) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* x = reinterpret_cast<C*>(smem_raw);
  const int2 u = units[blockIdx.x];
  const int pair = u.x, r0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[6 + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = blockIdx.y * a.Q;
  const int Q = min(a.Q, a.nrhs - q0);
  for (int idx = threadIdx.x; idx < RS * Q; idx += blockDim.x) {
    int q = idx % Q, b = idx / Q;
    x[idx] = F[(sitem * a.Es + padded_pos<D>(b, rs, a.Rs)) * a.nrhs + q0 + q];
  }
  C* red = x + RS * Q;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = r0 + lane;
  const int per = (RS + 3) / 4;
  const int j0 = w * per, j1 = min(RS, j0 + per);
  constexpr int QM = 8;
  C acc[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) acc[q] = czero<C>();
  if (row < RTp) {
    const CS* col = cores + core_off[pair] + row;
    for (int j = j0; j < j1; ++j) {
      C c;
      if constexpr (sizeof(CS) == 4) {   // packed bf16 pair
        unsigned v = reinterpret_cast<const unsigned*>(col)[(long long)j * RTp];
        c.x = bf16_to_f32((unsigned short)(v & 0xffff));
        c.y = bf16_to_f32((unsigned short)(v >> 16));
      } else {
        CS v = col[(long long)j * RTp];
        c.x = v.x;
        c.y = v.y;
      }
#pragma unroll
      for (int q = 0; q < QM; ++q)
        if (q < Q) acc[q] = cfma(acc[q], c, x[j * Q + q]);
    }
  }
#pragma unroll
  for (int q = 0; q < QM; ++q)
    if (q < Q) red[(w * 64 + lane) * Q + q] = acc[q];
  __syncthreads();
  if (w == 0 && row < RT) {
    long long pos = padded_pos<D>(row, rt, a.Rt);
    for (int q = 0; q < Q; ++q) {
      C v = red[lane * Q + q];
      v = cadd(v, red[(64 + lane) * Q + q]);
      v = cadd(v, red[(128 + lane) * Q + q]);
      v = cadd(v, red[(192 + lane) * Q + q]);
      G[(titem * a.Et + pos) * a.nrhs + q0 + q] = v;
    }
  }
  if (r0 == 0) {  // padding of the output item is written as zeros
    for (long long p = threadIdx.x; p < a.Et; p += blockDim.x)
      if (is_padding<D>(p, rt, a.Rt))
        for (int q = 0; q < Q; ++q) G[(titem * a.Et + p) * a.nrhs + q0 + q] = czero<C>();
  }
}

// F_{t,s}(cols) = C_{t,s}(:, cols)^H G_{t,s}; one workgroup = 16 columns of
// one pair, each wave reduces four columns across its lanes.
template <class T, class CS, int D>
__global__ void __launch_bounds__(kThreads)
    core_adj(CoreArgs a, const CS* __restrict__ cores, const long long* __restrict__ core_off,
             const int* __restrict__ meta, const int2* __restrict__ units,
             const typename CplxOf<T>::type* __restrict__ G, typename CplxOf<T>::type* __restrict__ F) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* y = reinterpret_cast<C*>(smem_raw);
  const int2 u = units[blockIdx.x];
  const int pair = u.x, c0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[6 + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = blockIdx.y * a.Q;
  const int Q = min(a.Q, a.nrhs - q0);
  for (int idx = threadIdx.x; idx < RTp * Q; idx += blockDim.x) {
    int q = idx % Q, r = idx / Q;
    y[idx] = r < RT ? G[(titem * a.Et + padded_pos<D>(r, rt, a.Rt)) * a.nrhs + q0 + q] : czero<C>();
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int QM = 8;
  for (int cc = 0; cc < 4; ++cc) {
    const int col = c0 + w * 4 + cc;
    if (col >= RS) break;
    const CS* cp = cores + core_off[pair] + (long long)col * RTp;
    C acc[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) acc[q] = czero<C>();
    for (int r = lane; r < RTp; r += 64) {
      C c;
      if constexpr (sizeof(CS) == 4) {
        unsigned v = reinterpret_cast<const unsigned*>(cp)[r];
        c.x = bf16_to_f32((unsigned short)(v & 0xffff));
        c.y = bf16_to_f32((unsigned short)(v >> 16));
      } else {
        CS v = cp[r];
        c.x = v.x;
        c.y = v.y;
      }
#pragma unroll
      for (int q = 0; q < QM; ++q)
        if (q < Q) acc[q] = cfma_conj(acc[q], c, y[r * Q + q]);
    }
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      if (q < Q) {
        T re = acc[q].x, im = acc[q].y;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          re += __shfl_xor(re, off, 64);
          im += __shfl_xor(im, off, 64);
        }
        acc[q].x = re;
        acc[q].y = im;
      }
    }
    if (lane == 0) {
      long long pos = padded_pos<D>(col, rs, a.Rs);
      for (int q = 0; q < Q; ++q) F[(sitem * a.Es + pos) * a.nrhs + q0 + q] = acc[q];
    }
  }
  if (c0 == 0) {
    for (long long p = threadIdx.x; p < a.Es; p += blockDim.x)
      if (is_padding<D>(p, rs, a.Rs))
        for (int q = 0; q < Q; ++q) F[(sitem * a.Es + p) * a.nrhs + q0 + q] = czero<C>();
  }
}

// ------------------------------------------------------------------ host --
static int g_lds_limit = 0;

static tb_status lds_limit(int* out) {
  if (!g_lds_limit) {
    int dev = 0, v = 0;
    TB_HIP_TRY(hipGetDevice(&dev));
    TB_HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    g_lds_limit = std::max(v, 32768);
  }
  *out = g_lds_limit;
  return TB_OK;
}

template <class K>
static tb_status set_lds(K kernel, size_t bytes) {
  if (bytes > 65536)
    TB_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return TB_OK;
}

struct Buffers {
  std::vector<size_t> src_off, tgt_off;  // byte offsets in the workspace
  size_t total = 0;
};

static Buffers layout(const Plan& p, long long nrhs, size_t esz) {
  Buffers b;
  size_t off = 0;
  auto add = [&](const Level& lv) {
    size_t bytes = (size_t)lv.nitems * lv.E * nrhs * esz;
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  for (const Level& lv : p.src) b.src_off.push_back(add(lv));
  for (const Level& lv : p.tgt) b.tgt_off.push_back(add(lv));
  b.total = off;
  return b;
}

// Fills the stage arguments connecting fine level `fine` (index l) with its
// coarse side: the level below, or the caller's array (l = 0).
static StageArgs stage_args(const Plan& p, const Level& fine, const Level* coarse, bool source,
                            int nrhs, bool conj) {
  StageArgs a{};
  const int d = p.d;
  a.nb = fine.nb;
  a.nblk = 1;
  for (int k = 0; k < d; ++k) a.nblk *= fine.nb;
  a.lvl = fine.l;
  for (int k = 0; k < d; ++k) {
    a.R[k] = fine.R[k];
    a.A[k] = fine.A[k];
    a.mat_k_off[k] = fine.mat_k_off[k];
  }
  a.mat_item_stride = fine.mat_item_stride;
  a.fineE = fine.E;
  long long st = 1;
  for (int k = d - 1; k >= 0; --k) {
    a.fst[k] = st;
    st *= (long long)fine.nb * fine.R[k];
  }
  a.n = p.n;
  a.ndim = 1;
  for (int k = 0; k < d; ++k) a.ndim *= p.n;
  a.coarse_global = coarse ? 0 : 1;
  if (coarse) {
    a.coarseE = coarse->E;
    st = 1;
    for (int k = d - 1; k >= 0; --k) {
      a.cst[k] = st;
      st *= (long long)coarse->nb * coarse->R[k];
    }
  }
  a.outer_level = source ? p.Ls : p.Lt;
  a.outer_block = (int)(p.n >> a.outer_level);
  a.nrhs = nrhs;
  a.conj = conj ? 1 : 0;
  return a;
}

static int fanout_lds_per_q(const StageArgs& a, int d) {
  if (d == 2) return a.R[0] * a.A[1];
  return a.R[0] * a.A[1] * a.A[2] + a.R[0] * a.R[1] * a.A[2];
}

static int fanin_lds_per_q(const StageArgs& a, int d) {
  if (d == 2) return a.A[0] * a.R[1];
  return a.A[0] * a.R[1] * a.R[2] + a.A[0] * a.A[1] * a.R[2];
}

template <class T>
static tb_status launch_stage(const Plan& p, StageArgs a, bool fanout, int n_items, const void* in,
                              void* out, const void* mats, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  const int d = p.d;
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  int mats_elems = 0;
  for (int k = 0; k < d; ++k) mats_elems += a.R[k] * a.A[k];
  int per_q = fanout ? fanout_lds_per_q(a, d) : fanin_lds_per_q(a, d);
  int qmax = (int)((limit / (int)sizeof(C) - mats_elems) / std::max(per_q, 1));
  if (!fanout) {
    int nout = 1;
    for (int k = 0; k < d; ++k) nout *= a.A[k];
    qmax = std::min(qmax, kMaxPer * kThreads / nout);
  }
  if (qmax < 1)
    return fail(TB_ERR_UNSUPPORTED, "transfer block exceeds the per-workgroup LDS/register budget");
  a.Q = std::min(a.nrhs, qmax);
  size_t lds = (size_t)(mats_elems + (size_t)per_q * a.Q) * sizeof(C);
  dim3 grid((unsigned)(n_items * a.nblk), (unsigned)((a.nrhs + a.Q - 1) / a.Q));
  if (fanout) {
    if (d == 2) {
      TB_TRY(set_lds(stage_fanout<T, 2>, lds));
      stage_fanout<T, 2><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
    } else {
      TB_TRY(set_lds(stage_fanout<T, 3>, lds));
      stage_fanout<T, 3><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
    }
  } else {
    if (d == 2) {
      TB_TRY(set_lds(stage_fanin<T, 2>, lds));
      stage_fanin<T, 2><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
    } else {
      TB_TRY(set_lds(stage_fanin<T, 3>, lds));
      stage_fanin<T, 3><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
    }
  }
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

template <class T, class CS>
static tb_status launch_core(const Plan& p, bool adjoint, int nrhs, const void* cores, const void* in,
                             void* out, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  const int d = p.d;
  const Level& st = p.src[p.Lt];
  const Level& tt = p.tgt[p.Ls];
  CoreArgs a{};
  a.nS = p.nS;
  a.nT = p.nT;
  a.Es = st.E;
  a.Et = tt.E;
  for (int k = 0; k < d; ++k) {
    a.Rs[k] = st.R[k];
    a.Rt[k] = tt.R[k];
  }
  a.nrhs = nrhs;
  a.Q = std::min(nrhs, 8);
  int maxRS = 0, maxRTp = 0;
  for (long long pr = 0; pr < p.npairs; ++pr) {
    maxRS = std::max(maxRS, p.pair_meta[(size_t)pr * kPairMeta + 1]);
    maxRTp = std::max(maxRTp, p.pair_meta[(size_t)pr * kPairMeta + 2]);
  }
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  size_t lds;
  for (;;) {
    lds = adjoint ? (size_t)maxRTp * a.Q * sizeof(C)
                  : ((size_t)maxRS * a.Q + (size_t)kThreads * a.Q) * sizeof(C);
    if (lds <= (size_t)limit || a.Q == 1) break;
    a.Q = std::max(1, a.Q / 2);
  }
  if (lds > (size_t)limit) return fail(TB_ERR_UNSUPPORTED, "core block exceeds the LDS budget");
  const bool is_bf16 = sizeof(CS) == 4;
  (void)is_bf16;
  if (!adjoint) {
    dim3 grid((unsigned)p.fwd_units.size(), (unsigned)((nrhs + a.Q - 1) / a.Q));
    if (d == 2) {
      TB_TRY(set_lds(core_fwd<T, CS, 2>, lds));
      core_fwd<T, CS, 2><<<grid, kThreads, lds, stream>>>(a, (const CS*)cores, p.core_off_d, p.pair_meta_d,
                                                         p.fwd_units_d, (const C*)in, (C*)out);
    } else {
      TB_TRY(set_lds(core_fwd<T, CS, 3>, lds));
      core_fwd<T, CS, 3><<<grid, kThreads, lds, stream>>>(a, (const CS*)cores, p.core_off_d, p.pair_meta_d,
                                                         p.fwd_units_d, (const C*)in, (C*)out);
    }
  } else {
    dim3 grid((unsigned)p.adj_units.size(), (unsigned)((nrhs + a.Q - 1) / a.Q));
    if (d == 2) {
      TB_TRY(set_lds(core_adj<T, CS, 2>, lds));
      core_adj<T, CS, 2><<<grid, kThreads, lds, stream>>>(a, (const CS*)cores, p.core_off_d, p.pair_meta_d,
                                                         p.adj_units_d, (const C*)in, (C*)out);
    } else {
      TB_TRY(set_lds(core_adj<T, CS, 3>, lds));
      core_adj<T, CS, 3><<<grid, kThreads, lds, stream>>>(a, (const CS*)cores, p.core_off_d, p.pair_meta_d,
                                                         p.adj_units_d, (const C*)in, (C*)out);
    }
  }
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

// Records an event pair around one stage launch when timing is enabled.
template <class F>
static tb_status timed(Plan& p, int stage, hipStream_t stream, F&& launch) {
  if (!p.timing) return launch();
  StageEvent e{stage, nullptr, nullptr};
  TB_HIP_TRY(hipEventCreate(&e.start));
  TB_HIP_TRY(hipEventCreate(&e.stop));
  TB_HIP_TRY(hipEventRecord(e.start, stream));
  tb_status st = launch();
  TB_HIP_TRY(hipEventRecord(e.stop, stream));
  p.events.push_back(e);
  return st;
}

template <class T, class CS>
static tb_status apply_typed(Plan& p, const void* in, void* out, long long nrhs, bool adjoint,
                             const void* cores, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  const size_t esz = sizeof(C);
  Buffers b = layout(p, nrhs, esz);
  if (p.ws.bytes < b.total) {
    if (p.ws.base) {
      TB_HIP_TRY(hipDeviceSynchronize());
      TB_HIP_TRY(hipFree(p.ws.base));
      p.device_bytes -= p.ws.bytes;
      p.ws.base = nullptr;
      p.ws.bytes = 0;
    }
    if (p.max_device_bytes && p.device_bytes + b.total > p.max_device_bytes)
      return fail(TB_ERR_OOM, "apply workspace exceeds the plan's device memory cap");
    hipError_t e = hipMalloc(&p.ws.base, b.total);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p.ws.base = nullptr;
      return fail(TB_ERR_OOM, std::string("apply workspace: ") + hipGetErrorString(e));
    }
    p.ws.bytes = b.total;
    p.device_bytes += b.total;
  }
  char* ws = static_cast<char*>(p.ws.base);
  auto S = [&](int l) { return (void*)(ws + b.src_off[l]); };
  auto Tb = [&](int l) { return (void*)(ws + b.tgt_off[l]); };
  auto mats = [&](const Level& lv) -> const void* {
    return sizeof(T) == 8 ? (const void*)lv.X64 : (const void*)lv.X32;
  };
  const int rhs = (int)nrhs;
  if (!adjoint) {
    // (1) V then W: coarse (f or level l-1) -> fine (level l)
    for (int l = 0; l <= p.Lt; ++l) {
      const Level& lv = p.src[l];
      StageArgs a = stage_args(p, lv, l ? &p.src[l - 1] : nullptr, true, rhs, false);
      TB_TRY(timed(p, l ? TB_STAGE_SRC_TRANSFER : TB_STAGE_SRC_LEAF, stream, [&] {
        return launch_stage<T>(p, a, true, lv.nitems, l ? S(l - 1) : in, S(l), mats(lv), stream);
      }));
    }
    // (2) cores
    TB_TRY(timed(p, TB_STAGE_CORE, stream, [&] {
      return launch_core<T, CS>(p, false, rhs, cores, S(p.Lt), Tb(p.Ls), stream);
    }));
    // (3) P^T accumulated into the parents, then U^T into u
    for (int l = p.Ls; l >= 0; --l) {
      const Level& lv = p.tgt[l];
      StageArgs a = stage_args(p, lv, l ? &p.tgt[l - 1] : nullptr, false, rhs, false);
      int ncoarse = l ? p.tgt[l - 1].nitems : lv.nitems;
      TB_TRY(timed(p, l ? TB_STAGE_TGT_TRANSFER : TB_STAGE_TGT_LEAF, stream, [&] {
        return launch_stage<T>(p, a, false, ncoarse, Tb(l), l ? Tb(l - 1) : out, mats(lv), stream);
      }));
    }
  } else {
    for (int l = 0; l <= p.Ls; ++l) {
      const Level& lv = p.tgt[l];
      StageArgs a = stage_args(p, lv, l ? &p.tgt[l - 1] : nullptr, false, rhs, true);
      TB_TRY(timed(p, l ? TB_STAGE_TGT_TRANSFER_ADJ : TB_STAGE_TGT_LEAF_ADJ, stream, [&] {
        return launch_stage<T>(p, a, true, lv.nitems, l ? Tb(l - 1) : in, Tb(l), mats(lv), stream);
      }));
    }
    TB_TRY(timed(p, TB_STAGE_CORE_ADJ, stream, [&] {
      return launch_core<T, CS>(p, true, rhs, cores, Tb(p.Ls), S(p.Lt), stream);
    }));
    for (int l = p.Lt; l >= 0; --l) {
      const Level& lv = p.src[l];
      StageArgs a = stage_args(p, lv, l ? &p.src[l - 1] : nullptr, true, rhs, true);
      int ncoarse = l ? p.src[l - 1].nitems : lv.nitems;
      TB_TRY(timed(p, l ? TB_STAGE_SRC_TRANSFER_ADJ : TB_STAGE_SRC_LEAF_ADJ, stream, [&] {
        return launch_stage<T>(p, a, false, ncoarse, S(l), l ? S(l - 1) : out, mats(lv), stream);
      }));
    }
  }
  return TB_OK;
}

tb_status run_apply(Plan& p, const void* in, void* out, long long nrhs, tb_dtype io, bool adjoint,
                    hipStream_t stream) {
  if (!in || !out) return fail(TB_ERR_INVALID_ARG, "null input or output pointer");
  if (nrhs < 1 || nrhs > (1 << 20)) return fail(TB_ERR_INVALID_ARG, "nrhs must be in [1, 2^20]");
  if (io < TB_C128 || io > TB_CBF16) return fail(TB_ERR_INVALID_ARG, "unknown tb_dtype");
  if (!p.cores[io])
    return fail(TB_ERR_INVALID_ARG,
                "the plan holds no cores of the requested precision (see store_mask)");
  if (in == out) return fail(TB_ERR_INVALID_ARG, "input and output must not alias");
  switch (io) {
    case TB_C128: return apply_typed<double, double2>(p, in, out, nrhs, adjoint, p.cores[io], stream);
    case TB_C64: return apply_typed<float, float2>(p, in, out, nrhs, adjoint, p.cores[io], stream);
    case TB_CBF16: return apply_typed<float, unsigned>(p, in, out, nrhs, adjoint, p.cores[io], stream);
  }
  return fail(TB_ERR_INVALID_ARG, "unknown tb_dtype");
}

}  // namespace tb

extern "C" tb_status tb_apply(tb_plan ph, const void* f, void* u, long long nrhs, tb_dtype io,
                              void* hip_stream) {
  if (!ph) return tb::fail(TB_ERR_INVALID_ARG, "tb_apply: null plan");
  return tb::run_apply(*reinterpret_cast<tb::Plan*>(ph), f, u, nrhs, io, false,
                       static_cast<hipStream_t>(hip_stream));
}

extern "C" tb_status tb_apply_adjoint(tb_plan ph, const void* g, void* v, long long nrhs, tb_dtype io,
                                      void* hip_stream) {
  if (!ph) return tb::fail(TB_ERR_INVALID_ARG, "tb_apply_adjoint: null plan");
  return tb::run_apply(*reinterpret_cast<tb::Plan*>(ph), g, v, nrhs, io, true,
                       static_cast<hipStream_t>(hip_stream));
}
