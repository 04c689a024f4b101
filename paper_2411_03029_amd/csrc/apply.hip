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
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <type_traits>

#include "cplx.h"
#include "stage_common.h"
#include "tb_internal.h"

namespace tb {

// --------------------------------------------------------------- fan-out --
// fine(a_0..a_{D-1}, q) = sum_j prod_k M_k[a_k][j_k] coarse(j_0..j_{D-1}, q)
// over true ranks (rows a_k < r_k) and the coarse block's true entries,
// for a_0 in this workgroup's slice [lo, lo + na).  Padding is never
// written or read: every consumer loops over true extents only.
template <class T, int D, int QT, int kG, int kV>
__global__ void __launch_bounds__(kThreads)
    stage_fanout(StageArgs a, const typename CplxOf<T>::type* __restrict__ coarse,
                 typename CplxOf<T>::type* __restrict__ fine,
                 const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  constexpr int NQV = QT / kV;  // threads along the right-hand sides
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const StageBid sb = stage_bid(a, QT);
  const int fi = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  int r[D];
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
  const int lo = sb.split * a.chunk;
  const int na = min(r[0], lo + a.chunk) - lo;
  // the coarse segments do not depend on the fine ranks: their loads are
  // issued before the slice test, in the same memory round trip
  const int citem = a.coarse_global ? (fi >> (D * a.lvl)) : parent_of<D>(fi, a.lvl);
  Seg sg[D];
  coarse_segs<D>(a, citem, beta, sg);
  if (na <= 0) return;
  const int q0 = sb.q0;
  const int Qa = min(QT, a.nrhs - q0);
  CoarseAddr<D> ca;
  ca.init(a, citem, beta, q0);
  long long fs[D];
  const long long fb = fine_base<D>(a, fi, beta, q0, fs);
  const C* mbase = mats + (long long)fi * a.mat_item_stride;
  // compact copies in LDS: rows [lo, lo + na) of M_0 (read in place from
  // global memory when G = 1: one use per load), all true rows of M_1..
  C* mk[D];
  int off = 0;
  const C* M0g = mbase + a.mat_k_off[0] + (long long)beta[0] * a.R[0] * a.A[0];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    mk[k] = sm + off;
    const C* src = mbase + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
    const int ck = sg[k].c;
    const int r0 = k == 0 ? lo : 0;
    const int nr = k == 0 ? (kG == 1 ? 0 : na) : r[k];
    for (int i = threadIdx.x; i < nr * ck; i += kThreads) {
      const int row = i / ck, j = i % ck;
      C v = src[(r0 + row) * a.A[k] + sg[k].pos(j)];
      if (a.conj) v.y = -v.y;
      mk[k][i] = v;
    }
    off += k == 0 ? a.chunk * a.A[0] : a.R[k] * a.A[k];
  }
  C* buf1 = sm + off;
  const int c0 = sg[0].c, c1 = sg[1].c;
  const int ng0 = (na + kG - 1) / kG;
  // M_0[lo + ai][compact j]
  auto m0 = [&](int ai, int j) -> C {
    if constexpr (kG == 1) {
      C v = M0g[(lo + ai) * a.A[0] + sg[0].pos(j)];
      if (a.conj) v.y = -v.y;
      return v;
    } else {
      return mk[0][ai * c0 + j];
    }
  };
  if constexpr (kG > 1) __syncthreads();
  if constexpr (D == 2) {
    // buf1[ai][j1][q] = sum_j0 M0[lo+ai][j0] coarse(j0, j1, q)
    for (int idx = threadIdx.x; idx < ng0 * c1 * NQV; idx += kThreads) {
      int qi, j1, t;
      if (a.coarse_global) {  // mode 1 is contiguous in the caller's array
        j1 = idx % c1;
        t = idx / c1;
        qi = t % NQV;
        t /= NQV;
      } else {
        qi = idx % NQV;
        t = idx / NQV;
        j1 = t % c1;
        t /= c1;
      }
      const int q = qi * kV;
      const int a0 = t * kG, ng = min(kG, na - a0);
      C acc[kG][kV];
      gzero2(acc);
      if (q < Qa) {
        const C* src = coarse + ca.base + sg[1].pos(j1) * ca.stride[1] + q * ca.qstride;
        const int vmax = min(kV, Qa - q) - 1;
        gdotv(acc, ng, c0, [&](int g, int j) { return m0(a0 + g, j); },
              [&](int j, int v) { return src[sg[0].pos(j) * ca.stride[0] + min(v, vmax) * ca.qstride]; });
      }
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v) buf1[((a0 + g) * c1 + j1) * QT + q + v] = acc[g][v];
    }
    __syncthreads();
    // fine[lo+ai][a1][q] = sum_j1 M1[a1][j1] buf1[ai][j1][q]
    const int ng1 = (r[1] + kG - 1) / kG;
    for (int idx = threadIdx.x; idx < ng1 * na * NQV; idx += kThreads) {
      const int q = (idx % NQV) * kV;
      int t = idx / NQV;
      const int ai = t % na, a1 = (t / na) * kG, ng = min(kG, r[1] - a1);
      if (q >= Qa) continue;
      C acc[kG][kV];
      gzero2(acc);
      const C* src = buf1 + (ai * c1) * QT + q;
      gdotv(acc, ng, c1, [&](int g, int j) { return mk[1][(a1 + g) * c1 + j]; },
            [&](int j, int v) { return src[j * QT + v]; });
      C* dst = fine + fb + (lo + ai) * fs[0] + q;
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v)
            if (v < Qa - q) dst[(a1 + g) * fs[1] + v] = acc[g][v];
    }
  } else {
    const int c2 = sg[2].c;
    C* buf2 = buf1 + a.chunk * a.A[1] * a.A[2] * QT;
    // buf1[ai][j1][j2][q] = sum_j0 M0[lo+ai][j0] coarse(j0, j1, j2, q)
    for (int idx = threadIdx.x; idx < ng0 * c1 * c2 * NQV; idx += kThreads) {
      int qi, j2, t;
      if (a.coarse_global) {
        j2 = idx % c2;
        t = idx / c2;
        qi = t % NQV;
        t /= NQV;
      } else {
        qi = idx % NQV;
        t = idx / NQV;
        j2 = t % c2;
        t /= c2;
      }
      const int q = qi * kV;
      const int j1 = t % c1, a0 = (t / c1) * kG, ng = min(kG, na - a0);
      C acc[kG][kV];
      gzero2(acc);
      if (q < Qa) {
        const C* src = coarse + ca.base + sg[1].pos(j1) * ca.stride[1] + sg[2].pos(j2) * ca.stride[2] +
                       q * ca.qstride;
        const int vmax = min(kV, Qa - q) - 1;
        gdotv(acc, ng, c0, [&](int g, int j) { return m0(a0 + g, j); },
              [&](int j, int v) { return src[sg[0].pos(j) * ca.stride[0] + min(v, vmax) * ca.qstride]; });
      }
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v) buf1[(((a0 + g) * c1 + j1) * c2 + j2) * QT + q + v] = acc[g][v];
    }
    __syncthreads();
    // buf2[ai][a1][j2][q] = sum_j1 M1[a1][j1] buf1[ai][j1][j2][q]
    const int ng1 = (r[1] + kG - 1) / kG;
    for (int idx = threadIdx.x; idx < ng1 * na * c2 * NQV; idx += kThreads) {
      const int q = (idx % NQV) * kV;
      int t = idx / NQV;
      const int j2 = t % c2;
      t /= c2;
      const int ai = t % na, a1 = (t / na) * kG, ng = min(kG, r[1] - a1);
      C acc[kG][kV];
      gzero2(acc);
      const C* src = buf1 + ((ai * c1) * c2 + j2) * QT + q;
      gdotv(acc, ng, c1, [&](int g, int j) { return mk[1][(a1 + g) * c1 + j]; },
            [&](int j, int v) { return src[j * c2 * QT + v]; });
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v) buf2[((ai * r[1] + a1 + g) * c2 + j2) * QT + q + v] = acc[g][v];
    }
    __syncthreads();
    // fine[lo+ai][a1][a2][q] = sum_j2 M2[a2][j2] buf2[ai][a1][j2][q]
    const int ng2 = (r[2] + kG - 1) / kG;
    for (int idx = threadIdx.x; idx < ng2 * na * r[1] * NQV; idx += kThreads) {
      const int q = (idx % NQV) * kV;
      int t = idx / NQV;
      const int a1 = t % r[1];
      t /= r[1];
      const int ai = t % na, a2 = (t / na) * kG, ng = min(kG, r[2] - a2);
      if (q >= Qa) continue;
      C acc[kG][kV];
      gzero2(acc);
      const C* src = buf2 + ((ai * r[1] + a1) * c2) * QT + q;
      gdotv(acc, ng, c2, [&](int g, int j) { return mk[2][(a2 + g) * c2 + j]; },
            [&](int j, int v) { return src[j * QT + v]; });
      C* dst = fine + fb + (lo + ai) * fs[0] + a1 * fs[1] + q;
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v)
            if (v < Qa - q) dst[(a2 + g) * fs[2] + v] = acc[g][v];
    }
  }
}

// ---------------------------------------------------------------- fan-in --
// coarse(a_0..a_{D-1}, q) = sum_children sum_j prod_k M_k[j_k][a_k] fine_c(j, q)
// over the children's true ranks, for the coarse block's true entries with
// a_0 in this workgroup's slice [lo, lo + na) (compact numbering).  All
// children are processed together: two barriers per workgroup.
constexpr int kStageU = 8;  // staging loads in flight per thread (fan-in)

// Stages the fan-in children's matrices of modes [K0, D) in LDS, compact:
// child c's block starts at mall[c * msz]; mode 0's slice rows [lo, lo + na)
// are transposed to [ai][j] (na x r_0(c)); mode k >= 1 is r_k(c) x c_k (row
// stride c_k) at offset chunk * R_0 + sum of R_k' * A_k' over 1 <= k' < k.
// Per mode, the slices of all the children go in one flat pass with
// kStageU loads in flight per thread before any LDS store: one memory round
// trip per kStageU * kThreads entries instead of one per child.
template <int D, int K0, class C>
__device__ __forceinline__ void stage_child_mats(C* mall, int msz, const StageArgs& a,
                                                 const C* __restrict__ mats, const int* cfi,
                                                 const int (*crk)[kMaxD], int nchild, const Seg* sg,
                                                 const int* beta, int lo, int na) {
  int moff = a.chunk * a.R[0];
#pragma unroll
  for (int k = K0; k < D; ++k) {
    const int ck = sg[k].c;
    const int mo = k == 0 ? 0 : moff;
    if (k > 0) moff += a.R[k] * a.A[k];
    int cend[kMaxChildren];
    int tot = 0;
#pragma unroll
    for (int c = 0; c < kMaxChildren; ++c) {
      tot += c < nchild ? (k == 0 ? na * crk[c][0] : crk[c][k] * ck) : 0;
      cend[c] = tot;
    }
    const long long kbase = a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
    for (int e0 = threadIdx.x; e0 < tot; e0 += kStageU * kThreads) {
      C v[kStageU];
      int dst[kStageU];
#pragma unroll
      for (int u = 0; u < kStageU; ++u) {
        const int e = e0 + u * kThreads;
        dst[u] = -1;
        if (e < tot) {
          int c = 0, start = 0;  // the child whose slice holds entry e
#pragma unroll
          for (int cc = 0; cc + 1 < kMaxChildren; ++cc)
            if (e >= cend[cc]) {
              c = cc + 1;
              start = cend[cc];
            }
          const int i = e - start;
          long long off;
          if (k == 0) {
            const int r0 = crk[c][0], ai = i / r0, j = i % r0;
            off = (long long)j * a.A[0] + sg[0].pos(lo + ai);
          } else {
            const int row = i / ck, j = i % ck;
            off = (long long)row * a.A[k] + sg[k].pos(j);
          }
          v[u] = mats[(long long)cfi[c] * a.mat_item_stride + kbase + off];
          dst[u] = c * msz + mo + i;
        }
      }
#pragma unroll
      for (int u = 0; u < kStageU; ++u)
        if (dst[u] >= 0) {
          C x = v[u];
          if (a.conj) x.y = -x.y;
          mall[dst[u]] = x;
        }
    }
  }
}

template <class T, int D, int QT, bool SM, int kG, int kV>
__global__ void __launch_bounds__(kThreads)
    stage_fanin(StageArgs a, const typename CplxOf<T>::type* __restrict__ fine,
                typename CplxOf<T>::type* __restrict__ coarse,
                const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  constexpr int NQV = QT / kV;  // threads along the right-hand sides
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const StageBid sb = stage_bid(a, QT);
  const int ci = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  Seg sg[D];
  coarse_segs<D>(a, ci, beta, sg);
  const int lo = sb.split * a.chunk;
  const int na = min(sg[0].c, lo + a.chunk) - lo;
  const int q0 = sb.q0;
  const int Qa = min(QT, a.nrhs - q0);
  const int nchild = a.coarse_global ? 1 : (1 << D);
  // children: item, ranks, fine base
  __shared__ int cfi[kMaxChildren], crk[kMaxChildren][kMaxD];
  __shared__ long long cfb[kMaxChildren];
  if (threadIdx.x < nchild) {
    const int c = threadIdx.x;
    const int fi = a.coarse_global ? ci : child_of<D>(ci, a.lvl, c);
    cfi[c] = fi;
#pragma unroll
    for (int k = 0; k < D; ++k) crk[c][k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
    long long fs_[D];
    cfb[c] = fine_base<D>(a, fi, beta, q0, fs_);
  }
  // tested after the children's rank loads are issued (one round trip for
  // both); uniform over the workgroup, before any barrier
  if (na <= 0) return;
  long long fs[D];
  (void)fine_base<D>(a, 0, beta, 0, fs);   // strides only
  __syncthreads();
  const int A0 = a.A[0];
  const int R1 = a.R[1];
  const int c1 = sg[1].c;
  // per child, compact in LDS (SM): M_0[j][lo + ai] transposed to
  // [ai][j] (na x r_0), then M_k (r_k x c_k, row stride c_k) for k >= 1;
  // without SM the padded matrices are read from global memory
  int msz = a.chunk * a.R[0];
#pragma unroll
  for (int k = 1; k < D; ++k) msz += a.R[k] * a.A[k];
  C* mall = sm;
  if constexpr (SM && kG == 1 && kV == 1) {
    // one output per thread: the block is small and latency-bound, so the
    // flat staging pays; mode 0 stays in global memory (read from LDS it
    // was slower)
    stage_child_mats<D, 1>(mall, msz, a, mats, cfi, crk, nchild, sg, beta, lo, na);
  } else {
    // register-blocked forms: the flat pass's registers would cost occupancy
    for (int c = 0; SM && c < nchild; ++c) {
      const C* mbase = mats + (long long)cfi[c] * a.mat_item_stride;
      int off = c * msz;
      if (kG > 1) {
        const C* src = mbase + a.mat_k_off[0] + (long long)beta[0] * a.R[0] * A0;
        const int r0 = crk[c][0];
        for (int i = threadIdx.x; i < na * r0; i += kThreads) {
          const int ai = i / r0, j = i % r0;
          C v = src[j * A0 + sg[0].pos(lo + ai)];
          if (a.conj) v.y = -v.y;
          mall[off + i] = v;
        }
      }
      off += a.chunk * a.R[0];
#pragma unroll
      for (int k = 1; k < D; ++k) {
        const C* src = mbase + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
        const int ck = sg[k].c, rk = crk[c][k];
        for (int i = threadIdx.x; i < rk * ck; i += kThreads) {
          const int row = i / ck, j = i % ck;
          C v = src[row * a.A[k] + sg[k].pos(j)];
          if (a.conj) v.y = -v.y;
          mall[off + i] = v;
        }
        off += a.R[k] * a.A[k];
      }
    }
  }
  C* buf1 = sm + (SM ? nchild * msz : 0);
  // M_0(c)[j][lo + ai]
  auto mat0 = [&](int c, int ai, int j) -> C {
    if constexpr (SM && kG > 1) {
      return mall[c * msz + ai * crk[c][0] + j];
    } else {
      C v = mats[(long long)cfi[c] * a.mat_item_stride + a.mat_k_off[0] +
                 (long long)beta[0] * a.R[0] * A0 + j * A0 + sg[0].pos(lo + ai)];
      if (a.conj) v.y = -v.y;
      return v;
    }
  };
  // M_k(c)[j][jo]: row j, compact column jo of child c's matrix for mode k
  auto mat = [&](int c, int k, int j, int jo) -> C {
    if constexpr (SM) {
      const int off = a.chunk * a.R[0] + (k == 1 ? 0 : a.R[1] * a.A[1]);
      return mall[c * msz + off + j * sg[k].c + jo];
    } else {
      C v = mats[(long long)cfi[c] * a.mat_item_stride + a.mat_k_off[k] +
                 (long long)beta[k] * a.R[k] * a.A[k] + j * a.A[k] + sg[k].pos(jo)];
      if (a.conj) v.y = -v.y;
      return v;
    }
  };
  const int ng0 = (na + kG - 1) / kG;
  if constexpr (kG > 1) __syncthreads();  // staged M_0 slices
  if constexpr (D == 2) {
    // buf1[c][ai][j1][q] = sum_j0 M0_c[j0][pos(lo+ai)] fine_c(j0, j1, q), j1 < r1(c)
    const int per_c = na * R1 * QT;
    for (int idx = threadIdx.x; idx < nchild * ng0 * R1 * NQV; idx += kThreads) {
      const int q = (idx % NQV) * kV;
      int t = idx / NQV;
      const int j1 = t % R1;
      t /= R1;
      const int a0 = (t % ng0) * kG, c = t / ng0, ng = min(kG, na - a0);
      if (j1 >= crk[c][1]) continue;
      C acc[kG][kV];
      gzero2(acc);
      if (q < Qa) {
        const C* src = fine + cfb[c] + j1 * fs[1] + q;
        const int vmax = min(kV, Qa - q) - 1;
        gdotv(acc, ng, crk[c][0], [&](int g, int j) { return mat0(c, a0 + g, j); },
              [&](int j, int v) { return src[j * fs[0] + min(v, vmax)]; });
      }
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v) buf1[c * per_c + ((a0 + g) * R1 + j1) * QT + q + v] = acc[g][v];
    }
    __syncthreads();
    CoarseAddr<D> ca;
    ca.init(a, ci, beta, q0);
    // coarse[lo+ai][j1o][q] = sum_c sum_j1 M1_c[j1][j1o] buf1[c][ai][j1][q]
    const int ng1 = (c1 + kG - 1) / kG;
    for (int idx = threadIdx.x; idx < ng1 * na * NQV; idx += kThreads) {
      int qi, ai, t;
      if (a.coarse_global) {
        ai = idx % na;
        t = idx / na;
        qi = t % NQV;
        t /= NQV;
      } else {
        qi = idx % NQV;
        t = idx / NQV;
        ai = t % na;
        t /= na;
      }
      const int q = qi * kV;
      const int j1o = t * kG, ng = min(kG, c1 - j1o);
      if (q >= Qa) continue;
      C acc[kG][kV];
      gzero2(acc);
      for (int c = 0; c < nchild; ++c) {
        const C* src = buf1 + c * per_c + (ai * R1) * QT + q;
        gdotv(acc, ng, crk[c][1], [&](int g, int j) { return mat(c, 1, j, j1o + g); },
              [&](int j, int v) { return src[j * QT + v]; });
      }
      C* dst = coarse + ca.base + sg[0].pos(lo + ai) * ca.stride[0] + q * ca.qstride;
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v)
            if (v < Qa - q) dst[sg[1].pos(j1o + g) * ca.stride[1] + v * ca.qstride] = acc[g][v];
    }
  } else {
    const int R2 = a.R[2];
    const int c2 = sg[2].c;
    const int per_c1 = na * R1 * R2 * QT;
    const int per_c2 = na * a.A[1] * R2 * QT;
    C* buf2 = buf1 + nchild * per_c1;
    // buf1[c][ai][j1][j2][q] = sum_j0 M0_c[j0][pos(lo+ai)] fine_c(j0, j1, j2, q)
    for (int idx = threadIdx.x; idx < nchild * ng0 * R1 * R2 * NQV; idx += kThreads) {
      const int q = (idx % NQV) * kV;
      int t = idx / NQV;
      const int j2 = t % R2;
      t /= R2;
      const int j1 = t % R1;
      t /= R1;
      const int a0 = (t % ng0) * kG, c = t / ng0, ng = min(kG, na - a0);
      if (j1 >= crk[c][1] || j2 >= crk[c][2]) continue;
      C acc[kG][kV];
      gzero2(acc);
      if (q < Qa) {
        const C* src = fine + cfb[c] + j1 * fs[1] + j2 * fs[2] + q;
        const int vmax = min(kV, Qa - q) - 1;
        gdotv(acc, ng, crk[c][0], [&](int g, int j) { return mat0(c, a0 + g, j); },
              [&](int j, int v) { return src[j * fs[0] + min(v, vmax)]; });
      }
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v)
            buf1[c * per_c1 + (((a0 + g) * R1 + j1) * R2 + j2) * QT + q + v] = acc[g][v];
    }
    __syncthreads();
    // buf2[c][ai][j1o][j2][q] = sum_j1 M1_c[j1][j1o] buf1[c][ai][j1][j2][q]
    const int ng1 = (c1 + kG - 1) / kG;
    for (int idx = threadIdx.x; idx < nchild * ng1 * na * R2 * NQV; idx += kThreads) {
      const int q = (idx % NQV) * kV;
      int t = idx / NQV;
      const int j2 = t % R2;
      t /= R2;
      const int ai = t % na;
      t /= na;
      const int j1o = (t % ng1) * kG, c = t / ng1, ng = min(kG, c1 - j1o);
      if (j2 >= crk[c][2]) continue;
      C acc[kG][kV];
      gzero2(acc);
      const C* src = buf1 + c * per_c1 + ((ai * R1) * R2 + j2) * QT + q;
      gdotv(acc, ng, crk[c][1], [&](int g, int j) { return mat(c, 1, j, j1o + g); },
            [&](int j, int v) { return src[j * R2 * QT + v]; });
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v)
            buf2[c * per_c2 + ((ai * a.A[1] + j1o + g) * R2 + j2) * QT + q + v] = acc[g][v];
    }
    __syncthreads();
    CoarseAddr<D> ca;
    ca.init(a, ci, beta, q0);
    // coarse[lo+ai][j1o][j2o][q] = sum_c sum_j2 M2_c[j2][j2o] buf2[c][ai][j1o][j2][q]
    const int ng2 = (c2 + kG - 1) / kG;
    for (int idx = threadIdx.x; idx < ng2 * na * c1 * NQV; idx += kThreads) {
      int qi, j1o, t;
      if (a.coarse_global) {
        j1o = idx % c1;
        t = idx / c1;
        qi = t % NQV;
        t /= NQV;
      } else {
        qi = idx % NQV;
        t = idx / NQV;
        j1o = t % c1;
        t /= c1;
      }
      const int q = qi * kV;
      const int ai = t % na, j2o = (t / na) * kG, ng = min(kG, c2 - j2o);
      if (q >= Qa) continue;
      C acc[kG][kV];
      gzero2(acc);
      for (int c = 0; c < nchild; ++c) {
        const C* src = buf2 + c * per_c2 + ((ai * a.A[1] + j1o) * R2) * QT + q;
        gdotv(acc, ng, crk[c][2], [&](int g, int j) { return mat(c, 2, j, j2o + g); },
              [&](int j, int v) { return src[j * QT + v]; });
      }
      C* dst = coarse + ca.base + sg[0].pos(lo + ai) * ca.stride[0] + sg[1].pos(j1o) * ca.stride[1] +
               q * ca.qstride;
#pragma unroll
      for (int g = 0; g < kG; ++g)
        if (g < ng)
#pragma unroll
          for (int v = 0; v < kV; ++v)
            if (v < Qa - q) dst[sg[2].pos(j2o + g) * ca.stride[2] + v * ca.qstride] = acc[g][v];
    }
  }
}

// ------------------------------------------ fan-in, children in turn (2) --
// The sum of stage_fanin with the 2^d children taken one after the other and
// the first mode contracted first, on the slice's rows: one child's
// intermediates live in LDS at a time, and the slice of the coarse block
// accumulates in LDS, each entry owned by one thread for all the children,
// so the order of the sum per output is that of stage_fanin.  It needs far
// less LDS per right-hand side than stage_fanin, so wider RHS tiles fit.
template <class T, int D, int QT, int kG, int kV>
__global__ void __launch_bounds__(kThreads)
    stage_fanin_turn(StageArgs a, const typename CplxOf<T>::type* __restrict__ fine,
                     typename CplxOf<T>::type* __restrict__ coarse,
                     const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  constexpr int NQV = QT / kV;  // threads along the right-hand sides
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const StageBid sb = stage_bid(a, QT);
  const int ci = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  Seg sg[D];
  coarse_segs<D>(a, ci, beta, sg);
  const int lo = sb.split * a.chunk;
  const int na = min(sg[0].c, lo + a.chunk) - lo;
  const int q0 = sb.q0;
  const int Qa = min(QT, a.nrhs - q0);
  const int nchild = a.coarse_global ? 1 : (1 << D);
  __shared__ int cfi[kMaxChildren], crk[kMaxChildren][kMaxD];
  __shared__ long long cfb[kMaxChildren];
  if (threadIdx.x < nchild) {
    const int c = threadIdx.x;
    const int fi = a.coarse_global ? ci : child_of<D>(ci, a.lvl, c);
    cfi[c] = fi;
#pragma unroll
    for (int k = 0; k < D; ++k) crk[c][k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
    long long fs_[D];
    cfb[c] = fine_base<D>(a, fi, beta, q0, fs_);
  }
  // tested after the children's rank loads are issued (one round trip for
  // both); uniform over the workgroup, before any barrier
  if (na <= 0) return;
  long long fs[D];
  (void)fine_base<D>(a, 0, beta, 0, fs);   // strides only
  __syncthreads();
  const int R1 = a.R[1];
  const int c1 = sg[1].c;
  // every child's matrices, compact in LDS: M_0[j][lo + ai] transposed to
  // [ai][j] (na x r_0), then M_k (r_k x c_k, row stride c_k) for k >= 1
  int msz = a.chunk * a.R[0];
#pragma unroll
  for (int k = 1; k < D; ++k) msz += a.R[k] * a.A[k];
  C* mall = sm;
  if constexpr (D == 3) {
    stage_child_mats<D, 0>(mall, msz, a, mats, cfi, crk, nchild, sg, beta, lo, na);
  } else {
    // d = 2: the flat pass's registers would cost occupancy
    const int A0 = a.A[0];
    for (int c = 0; c < nchild; ++c) {
      const C* mbase = mats + (long long)cfi[c] * a.mat_item_stride;
      int off = c * msz;
      {
        const C* src = mbase + a.mat_k_off[0] + (long long)beta[0] * a.R[0] * A0;
        const int r0 = crk[c][0];
        for (int i = threadIdx.x; i < na * r0; i += kThreads) {
          const int ai = i / r0, j = i % r0;
          C v = src[j * A0 + sg[0].pos(lo + ai)];
          if (a.conj) v.y = -v.y;
          mall[off + i] = v;
        }
      }
      off += a.chunk * a.R[0];
#pragma unroll
      for (int k = 1; k < D; ++k) {
        const C* src = mbase + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
        const int ck = sg[k].c, rk = crk[c][k];
        for (int i = threadIdx.x; i < rk * ck; i += kThreads) {
          const int row = i / ck, j = i % ck;
          C v = src[row * a.A[k] + sg[k].pos(j)];
          if (a.conj) v.y = -v.y;
          mall[off + i] = v;
        }
        off += a.R[k] * a.A[k];
      }
    }
  }
  C* buf1 = sm + nchild * msz;
  auto mat0 = [&](int c, int ai, int j) -> C { return mall[c * msz + ai * crk[c][0] + j]; };
  auto mat = [&](int c, int k, int j, int jo) -> C {
    const int off = a.chunk * a.R[0] + (k == 1 ? 0 : a.R[1] * a.A[1]);
    return mall[c * msz + off + j * sg[k].c + jo];
  };
  const int ng0 = (na + kG - 1) / kG;
  CoarseAddr<D> ca;
  ca.init(a, ci, beta, q0);
  __syncthreads();  // staged matrices
  if constexpr (D == 2) {
    C* accb = buf1 + a.chunk * R1 * QT;  // [ai][j1o][q]
    const int ng1 = (c1 + kG - 1) / kG;
    for (int c = 0; c < nchild; ++c) {
      // buf1[ai][j1][q] = sum_j0 M0_c[j0][pos(lo+ai)] fine_c(j0, j1, q), j1 < r1(c)
      for (int idx = threadIdx.x; idx < ng0 * R1 * NQV; idx += kThreads) {
        const int q = (idx % NQV) * kV;
        int t = idx / NQV;
        const int j1 = t % R1, a0 = (t / R1) * kG, ng = min(kG, na - a0);
        if (j1 >= crk[c][1]) continue;
        C acc[kG][kV];
        gzero2(acc);
        if (q < Qa) {
          const C* src = fine + cfb[c] + j1 * fs[1] + q;
          const int vmax = min(kV, Qa - q) - 1;
          gdotv(acc, ng, crk[c][0], [&](int g, int j) { return mat0(c, a0 + g, j); },
                [&](int j, int v) { return src[j * fs[0] + min(v, vmax)]; });
        }
#pragma unroll
        for (int g = 0; g < kG; ++g)
          if (g < ng)
#pragma unroll
            for (int v = 0; v < kV; ++v) buf1[((a0 + g) * R1 + j1) * QT + q + v] = acc[g][v];
      }
      __syncthreads();
      // coarse[lo+ai][j1o][q] (+)= sum_j1 M1_c[j1][j1o] buf1[ai][j1][q]
      const bool last = c == nchild - 1;
      for (int idx = threadIdx.x; idx < ng1 * na * NQV; idx += kThreads) {
        int qi, ai, t;
        if (a.coarse_global) {
          ai = idx % na;
          t = idx / na;
          qi = t % NQV;
          t /= NQV;
        } else {
          qi = idx % NQV;
          t = idx / NQV;
          ai = t % na;
          t /= na;
        }
        const int q = qi * kV;
        const int j1o = t * kG, ng = min(kG, c1 - j1o);
        if (q >= Qa) continue;
        C acc[kG][kV];
        C* ab = accb + (ai * a.A[1] + j1o) * QT + q;
        gzero2(acc);
        if (c > 0) {
#pragma unroll
          for (int g = 0; g < kG; ++g)
            if (g < ng)
#pragma unroll
              for (int v = 0; v < kV; ++v) acc[g][v] = ab[g * QT + v];
        }
        const C* src = buf1 + (ai * R1) * QT + q;
        gdotv(acc, ng, crk[c][1], [&](int g, int j) { return mat(c, 1, j, j1o + g); },
              [&](int j, int v) { return src[j * QT + v]; });
        if (!last) {
#pragma unroll
          for (int g = 0; g < kG; ++g)
            if (g < ng)
#pragma unroll
              for (int v = 0; v < kV; ++v) ab[g * QT + v] = acc[g][v];
        } else {
          C* dst = coarse + ca.base + sg[0].pos(lo + ai) * ca.stride[0] + q * ca.qstride;
#pragma unroll
          for (int g = 0; g < kG; ++g)
            if (g < ng)
#pragma unroll
              for (int v = 0; v < kV; ++v)
                if (v < Qa - q) dst[sg[1].pos(j1o + g) * ca.stride[1] + v * ca.qstride] = acc[g][v];
        }
      }
      __syncthreads();  // buf1 is rewritten by the next child
    }
  } else {
    const int R2 = a.R[2];
    const int c2 = sg[2].c;
    C* buf2 = buf1 + a.chunk * R1 * R2 * QT;        // [ai][j1o][j2][q]
    C* accb = buf2 + a.chunk * a.A[1] * R2 * QT;    // [ai][j1o][j2o][q]
    const int ng1 = (c1 + kG - 1) / kG;
    const int ng2 = (c2 + kG - 1) / kG;
    for (int c = 0; c < nchild; ++c) {
      // buf1[ai][j1][j2][q] = sum_j0 M0_c[j0][pos(lo+ai)] fine_c(j0, j1, j2, q)
      for (int idx = threadIdx.x; idx < ng0 * R1 * R2 * NQV; idx += kThreads) {
        const int q = (idx % NQV) * kV;
        int t = idx / NQV;
        const int j2 = t % R2;
        t /= R2;
        const int j1 = t % R1, a0 = (t / R1) * kG, ng = min(kG, na - a0);
        if (j1 >= crk[c][1] || j2 >= crk[c][2]) continue;
        C acc[kG][kV];
        gzero2(acc);
        if (q < Qa) {
          const C* src = fine + cfb[c] + j1 * fs[1] + j2 * fs[2] + q;
          const int vmax = min(kV, Qa - q) - 1;
          gdotv(acc, ng, crk[c][0], [&](int g, int j) { return mat0(c, a0 + g, j); },
                [&](int j, int v) { return src[j * fs[0] + min(v, vmax)]; });
        }
#pragma unroll
        for (int g = 0; g < kG; ++g)
          if (g < ng)
#pragma unroll
            for (int v = 0; v < kV; ++v) buf1[(((a0 + g) * R1 + j1) * R2 + j2) * QT + q + v] = acc[g][v];
      }
      __syncthreads();
      // buf2[ai][j1o][j2][q] = sum_j1 M1_c[j1][j1o] buf1[ai][j1][j2][q]
      for (int idx = threadIdx.x; idx < ng1 * na * R2 * NQV; idx += kThreads) {
        const int q = (idx % NQV) * kV;
        int t = idx / NQV;
        const int j2 = t % R2;
        t /= R2;
        const int ai = t % na, j1o = (t / na) * kG, ng = min(kG, c1 - j1o);
        if (j2 >= crk[c][2]) continue;
        C acc[kG][kV];
        gzero2(acc);
        const C* src = buf1 + ((ai * R1) * R2 + j2) * QT + q;
        gdotv(acc, ng, crk[c][1], [&](int g, int j) { return mat(c, 1, j, j1o + g); },
              [&](int j, int v) { return src[j * R2 * QT + v]; });
#pragma unroll
        for (int g = 0; g < kG; ++g)
          if (g < ng)
#pragma unroll
            for (int v = 0; v < kV; ++v) buf2[((ai * a.A[1] + j1o + g) * R2 + j2) * QT + q + v] = acc[g][v];
      }
      __syncthreads();
      // coarse[lo+ai][j1o][j2o][q] (+)= sum_j2 M2_c[j2][j2o] buf2[ai][j1o][j2][q]
      const bool last = c == nchild - 1;
      for (int idx = threadIdx.x; idx < ng2 * na * c1 * NQV; idx += kThreads) {
        int qi, j1o, t;
        if (a.coarse_global) {
          j1o = idx % c1;
          t = idx / c1;
          qi = t % NQV;
          t /= NQV;
        } else {
          qi = idx % NQV;
          t = idx / NQV;
          j1o = t % c1;
          t /= c1;
        }
        const int q = qi * kV;
        const int ai = t % na, j2o = (t / na) * kG, ng = min(kG, c2 - j2o);
        if (q >= Qa) continue;
        C acc[kG][kV];
        C* ab = accb + ((ai * a.A[1] + j1o) * a.A[2] + j2o) * QT + q;
        gzero2(acc);
        if (c > 0) {
#pragma unroll
          for (int g = 0; g < kG; ++g)
            if (g < ng)
#pragma unroll
              for (int v = 0; v < kV; ++v) acc[g][v] = ab[g * QT + v];
        }
        const C* src = buf2 + ((ai * a.A[1] + j1o) * R2) * QT + q;
        gdotv(acc, ng, crk[c][2], [&](int g, int j) { return mat(c, 2, j, j2o + g); },
              [&](int j, int v) { return src[j * QT + v]; });
        if (!last) {
#pragma unroll
          for (int g = 0; g < kG; ++g)
            if (g < ng)
#pragma unroll
              for (int v = 0; v < kV; ++v) ab[g * QT + v] = acc[g][v];
        } else {
          C* dst = coarse + ca.base + sg[0].pos(lo + ai) * ca.stride[0] + sg[1].pos(j1o) * ca.stride[1] +
                   q * ca.qstride;
#pragma unroll
          for (int g = 0; g < kG; ++g)
            if (g < ng)
#pragma unroll
              for (int v = 0; v < kV; ++v)
                if (v < Qa - q) dst[sg[2].pos(j2o + g) * ca.stride[2] + v * ca.qstride] = acc[g][v];
        }
      }
    }
  }
}

// ------------------------------------------------------ fan-in, in turn --
// The same sum as stage_fanin, with the 2^d children taken one after the
// other: per child the modes D-1 .. 1 are contracted through LDS (one
// child's intermediates at a time) and mode 0 is accumulated in registers.
// Each thread owns up to kSeqFib output fibers (a_1..a_{D-1}, q) and all
// rows a_0 of its slice (at most kSeqRows), so nothing is re-read across
// slices unless the coarse block has more than kSeqRows rows.
constexpr int kSeqRows = 16;

template <class T>
struct SeqFib {
  static constexpr int value = sizeof(T) == 8 ? 2 : 4;
};

template <class T, int D, int QT>
__global__ void __launch_bounds__(kThreads)
    stage_fanin_seq(StageArgs a, const typename CplxOf<T>::type* __restrict__ fine,
                    typename CplxOf<T>::type* __restrict__ coarse,
                    const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  constexpr int kF = SeqFib<T>::value;
  constexpr int kGs = 8;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const StageBid sb = stage_bid(a, QT);
  const int ci = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  Seg sg[D];
  coarse_segs<D>(a, ci, beta, sg);
  const int lo = sb.split * a.chunk;
  const int na = min(sg[0].c, lo + a.chunk) - lo;
  const int q0 = sb.q0;
  const int Qa = min(QT, a.nrhs - q0);
  const int nchild = a.coarse_global ? 1 : (1 << D);
  __shared__ int cfi[kMaxChildren], crk[kMaxChildren][kMaxD];
  __shared__ long long cfb[kMaxChildren];
  if (threadIdx.x < nchild) {
    const int c = threadIdx.x;
    const int fi = a.coarse_global ? ci : child_of<D>(ci, a.lvl, c);
    cfi[c] = fi;
#pragma unroll
    for (int k = 0; k < D; ++k) crk[c][k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
    long long fs_[D];
    cfb[c] = fine_base<D>(a, fi, beta, q0, fs_);
  }
  // tested after the children's rank loads are issued (one round trip for
  // both); uniform over the workgroup, before any barrier
  if (na <= 0) return;
  long long fs[D];
  (void)fine_base<D>(a, 0, beta, 0, fs);  // strides only
  __syncthreads();
  // every child's matrices, compact: M_0 [j][ai] (r_0 x na), M_k [j][a_k]
  // (r_k x c_k) for k >= 1
  int msz = a.R[0] * a.chunk;
#pragma unroll
  for (int k = 1; k < D; ++k) msz += a.R[k] * a.A[k];
  for (int c = 0; c < nchild; ++c) {
    const C* mbase = mats + (long long)cfi[c] * a.mat_item_stride;
    int off = c * msz;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const C* src = mbase + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
      const int ck = k == 0 ? na : sg[k].c, rk = crk[c][k], j0 = k == 0 ? lo : 0;
      for (int i = threadIdx.x; i < rk * ck; i += kThreads) {
        const int row = i / ck, j = i % ck;
        C v = src[row * a.A[k] + sg[k].pos(j0 + j)];
        if (a.conj) v.y = -v.y;
        sm[off + i] = v;
      }
      off += k == 0 ? a.R[0] * a.chunk : a.R[k] * a.A[k];
    }
  }
  C* t1 = sm + nchild * msz;
  const int c1 = sg[1].c;
  const int c2 = D == 3 ? sg[D - 1].c : 1;
  C* t2 = t1 + (D == 3 ? a.R[0] * a.R[1] * a.A[D - 1] * QT : 0);
  // output fibers: (a_1, q) for D = 2, (a_1, a_2, q) for D = 3; the
  // contiguous index of the destination runs fastest
  const int nfib = c1 * c2 * QT;
  auto fiber = [&](int f, int* a1, int* a2, int* q) {
    if (a.coarse_global) {
      const int inner = D == 3 ? c2 : c1;
      const int x = f % inner, t = f / inner;
      *q = t % QT;
      if (D == 3) {
        *a2 = x;
        *a1 = t / QT;
      } else {
        *a1 = x;
        *a2 = 0;
      }
    } else {
      *q = f % QT;
      const int t = f / QT;
      *a2 = D == 3 ? t % c2 : 0;
      *a1 = D == 3 ? t / c2 : t;
    }
  };
  C acc[kF][kSeqRows];
#pragma unroll
  for (int f = 0; f < kF; ++f)
#pragma unroll
    for (int r = 0; r < kSeqRows; ++r) acc[f][r] = czero<C>();
  __syncthreads();
  for (int c = 0; c < nchild; ++c) {
    const int r0 = crk[c][0], r1 = crk[c][1];
    const C* M0c = sm + c * msz;
    const C* M1c = M0c + a.R[0] * a.chunk;
    const C* fc = fine + cfb[c];
    const C* xin;  // [j0][a1][a2][q] input of the mode-0 step
    if constexpr (D == 2) {
      // t1[j0][a1][q] = sum_j1 M1c[j1][a1] fine_c(j0, j1, q)
      const int ng = (c1 + kGs - 1) / kGs;
      for (int idx = threadIdx.x; idx < ng * r0 * QT; idx += kThreads) {
        const int q = idx % QT;
        const int t = idx / QT;
        const int j0 = t % r0, a1 = (t / r0) * kGs, n1 = min(kGs, c1 - a1);
        C o[kGs];
        gzero(o);
        if (q < Qa)
          gdot(o, n1, r1, [&](int g, int j) { return M1c[j * c1 + a1 + g]; },
               [&](int j) { return fc[j0 * fs[0] + j * fs[1] + q]; });
#pragma unroll
        for (int g = 0; g < kGs; ++g)
          if (g < n1) t1[(j0 * c1 + a1 + g) * QT + q] = o[g];
      }
      xin = t1;
    } else {
      const int r2 = crk[c][2];
      const C* M2c = M1c + a.R[1] * a.A[1];
      // t1[j0][j1][a2][q] = sum_j2 M2c[j2][a2] fine_c(j0, j1, j2, q)
      const int ng2 = (c2 + kGs - 1) / kGs;
      for (int idx = threadIdx.x; idx < ng2 * r0 * r1 * QT; idx += kThreads) {
        const int q = idx % QT;
        int t = idx / QT;
        const int j1 = t % r1;
        t /= r1;
        const int j0 = t % r0, a2 = (t / r0) * kGs, n2 = min(kGs, c2 - a2);
        C o[kGs];
        gzero(o);
        if (q < Qa)
          gdot(o, n2, r2, [&](int g, int j) { return M2c[j * c2 + a2 + g]; },
               [&](int j) { return fc[j0 * fs[0] + j1 * fs[1] + j * fs[2] + q]; });
#pragma unroll
        for (int g = 0; g < kGs; ++g)
          if (g < n2) t1[((j0 * r1 + j1) * c2 + a2 + g) * QT + q] = o[g];
      }
      __syncthreads();
      // t2[j0][a1][a2][q] = sum_j1 M1c[j1][a1] t1[j0][j1][a2][q]
      const int ng1 = (c1 + kGs - 1) / kGs;
      for (int idx = threadIdx.x; idx < ng1 * r0 * c2 * QT; idx += kThreads) {
        const int q = idx % QT;
        int t = idx / QT;
        const int a2 = t % c2;
        t /= c2;
        const int j0 = t % r0, a1 = (t / r0) * kGs, n1 = min(kGs, c1 - a1);
        C o[kGs];
        gzero(o);
        const C* src = t1 + ((j0 * r1) * c2 + a2) * QT + q;
        gdot(o, n1, r1, [&](int g, int j) { return M1c[j * c1 + a1 + g]; },
             [&](int j) { return src[j * c2 * QT]; });
#pragma unroll
        for (int g = 0; g < kGs; ++g)
          if (g < n1) t2[((j0 * c1 + a1 + g) * c2 + a2) * QT + q] = o[g];
      }
      xin = t2;
    }
    __syncthreads();
    // acc[f][ai] += sum_j0 M0c[j0][ai] xin[j0][a1][a2][q]
#pragma unroll
    for (int f = 0; f < kF; ++f) {
      const int fid = threadIdx.x + f * kThreads;
      if (fid < nfib) {
        int a1, a2, q;
        fiber(fid, &a1, &a2, &q);
        const C* src = xin + (a1 * c2 + a2) * QT + q;
        for (int j0 = 0; j0 < r0; ++j0) {
          const C xv = src[j0 * c1 * c2 * QT];
#pragma unroll
          for (int r = 0; r < kSeqRows; ++r)
            if (r < na) acc[f][r] = cfma(acc[f][r], M0c[j0 * na + r], xv);
        }
      }
    }
    __syncthreads();
  }
  CoarseAddr<D> ca;
  ca.init(a, ci, beta, q0);
#pragma unroll
  for (int f = 0; f < kF; ++f) {
    const int fid = threadIdx.x + f * kThreads;
    if (fid < nfib) {
      int a1, a2, q;
      fiber(fid, &a1, &a2, &q);
      if (q < Qa) {
        C* dst = coarse + ca.base + sg[1].pos(a1) * ca.stride[1] + q * ca.qstride;
        if (D == 3) dst += sg[D - 1].pos(a2) * ca.stride[D - 1];
#pragma unroll
        for (int r = 0; r < kSeqRows; ++r)
          if (r < na) dst[sg[0].pos(lo + r) * ca.stride[0]] = acc[f][r];
      }
    }
  }
}

// ------------------------------------------------------------------ core --
struct CoreArgs {
  long long nS, nT;              // middle multi-sets per side
  long long Es, Et;              // entries per top-level item (source / target)
  int Rs[kMaxD], Rt[kMaxD];      // padded ranks of the top levels
  int nrhs;
  const float* colscale;         // TB_CQ16: scale per core column
  const long long* col_off;      // TB_CQ16: first column of each pair
};

// A TB_CQ16 core entry: int16 real part (low half) and imaginary part (high
// half) of the entry / its column's scale.
struct Q16 {
  unsigned w;
};

// 16-byte vector loads of the stored cores: VR consecutive rows per lane.
template <class CS>
struct CoreVec;
template <>
struct CoreVec<float2> {
  static constexpr int VR = 2;
  using V = float4;
  __device__ static void get(const V& v, float2* c) {
    c[0] = make_float2(v.x, v.y);
    c[1] = make_float2(v.z, v.w);
  }
};
template <>
struct CoreVec<double2> {
  static constexpr int VR = 1;
  using V = double2;
  __device__ static void get(const V& v, double2* c) { c[0] = v; }
};
template <>
struct CoreVec<unsigned> {  // packed (bf16 re, bf16 im)
  static constexpr int VR = 4;
  using V = uint4;
  __device__ static float2 one(unsigned u) {
    return make_float2(bf16_to_f32((unsigned short)(u & 0xffff)), bf16_to_f32((unsigned short)(u >> 16)));
  }
  __device__ static void get(const V& v, float2* c) {
    c[0] = one(v.x);
    c[1] = one(v.y);
    c[2] = one(v.z);
    c[3] = one(v.w);
  }
};
template <>
struct CoreVec<Q16> {
  static constexpr int VR = 4;
  using V = uint4;
  __device__ static float2 one(unsigned u) {
    return make_float2((float)(short)(u & 0xffffu), (float)(short)(u >> 16));
  }
  __device__ static void get(const V& v, float2* c) {
    c[0] = one(v.x);
    c[1] = one(v.y);
    c[2] = one(v.z);
    c[3] = one(v.w);
  }
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

constexpr int kUnroll = 8;

// G_{t,s}(rows) = C_{t,s}(rows, :) F_{t,s}.  A workgroup owns 64 VR rows of
// one pair (VR per lane, one 16-byte load per column); its four waves split
// the columns, keep kUnroll column loads in flight and reduce through LDS.
template <class T, class CS, int D, int QT>
__global__ void __launch_bounds__(kThreads)
    core_fwd(CoreArgs a, const CS* __restrict__ cores, const long long* __restrict__ core_off,
             const int* __restrict__ meta, const int2* __restrict__ units,
             const typename CplxOf<T>::type* __restrict__ F, typename CplxOf<T>::type* __restrict__ G) {
  using C = typename CplxOf<T>::type;
  using CV = CoreVec<CS>;
  constexpr int VR = CV::VR;
  extern __shared__ unsigned char smem_raw[];
  C* x = reinterpret_cast<C*>(smem_raw);
  const int2 u = units[blockIdx.x];
  if (u.x < 0) return;  // padding of the XCD-grouped unit list (whole workgroup)
  const int pair = u.x, r0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = blockIdx.y * QT;
  const int Qa = min(QT, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = r0 + lane * VR;
  const int per = (RS + 3) / 4;
  const int j0 = w * per, j1 = min(RS, j0 + per);
  // the first kUnroll columns are requested before F is staged, so that the
  // stream of cores is under way during the staging and its barrier
  const typename CV::V* col = reinterpret_cast<const typename CV::V*>(cores + core_off[pair] + min(row, RTp - VR));
  const long long cstride = RTp / VR;   // in vectors
  typename CV::V vv[kUnroll];
  const bool first = row < RTp && j0 + kUnroll <= j1;
  if (first) {
#pragma unroll
    for (int uu = 0; uu < kUnroll; ++uu) vv[uu] = col[(long long)(j0 + uu) * cstride];
  }
  for (int idx = threadIdx.x; idx < RS * QT; idx += kThreads) {
    const int q = idx % QT, b = idx / QT;
    C v = q < Qa ? F[(sitem * a.Es + padded_pos<D>(b, rs, a.Rs)) * a.nrhs + q0 + q] : czero<C>();
    if constexpr (std::is_same<CS, Q16>::value) {  // C = Q S: the column scales go with F
      const T sc = a.colscale[a.col_off[pair] + b];
      v.x *= sc;
      v.y *= sc;
    }
    x[idx] = v;
  }
  C* red = x + RS * QT;
  __syncthreads();
  C acc[VR][QT];
#pragma unroll
  for (int v = 0; v < VR; ++v)
#pragma unroll
    for (int q = 0; q < QT; ++q) acc[v][q] = czero<C>();
  if (row < RTp) {
    int j = j0;
    for (; j + kUnroll <= j1; j += kUnroll) {
      if (j != j0 || !first) {
#pragma unroll
        for (int uu = 0; uu < kUnroll; ++uu) vv[uu] = col[(long long)(j + uu) * cstride];
      }
#pragma unroll
      for (int uu = 0; uu < kUnroll; ++uu) {
        C c[VR];
        CV::get(vv[uu], c);
#pragma unroll
        for (int q = 0; q < QT; ++q) {
          const C xv = x[(j + uu) * QT + q];
#pragma unroll
          for (int v = 0; v < VR; ++v) acc[v][q] = cfma(acc[v][q], c[v], xv);
        }
      }
    }
    for (; j < j1; ++j) {
      C c[VR];
      CV::get(col[(long long)j * cstride], c);
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        const C xv = x[j * QT + q];
#pragma unroll
        for (int v = 0; v < VR; ++v) acc[v][q] = cfma(acc[v][q], c[v], xv);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < VR; ++v)
#pragma unroll
    for (int q = 0; q < QT; ++q) red[((w * 64 + lane) * VR + v) * QT + q] = acc[v][q];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int v = 0; v < VR; ++v) {
      const int r = row + v;
      if (r < RT) {
        const long long pos = padded_pos<D>(r, rt, a.Rt);
#pragma unroll
        for (int q = 0; q < QT; ++q) {
          if (q < Qa) {
            C sum = red[(lane * VR + v) * QT + q];
            sum = cadd(sum, red[((64 + lane) * VR + v) * QT + q]);
            sum = cadd(sum, red[((128 + lane) * VR + v) * QT + q]);
            sum = cadd(sum, red[((192 + lane) * VR + v) * QT + q]);
            G[(titem * a.Et + pos) * a.nrhs + q0 + q] = sum;
          }
        }
      }
    }
  }
  if (r0 == 0) {  // padding of the output item is written as zeros
    for (long long p = threadIdx.x; p < a.Et; p += kThreads)
      if (is_padding<D>(p, rt, a.Rt))
        for (int q = 0; q < Qa; ++q) G[(titem * a.Et + p) * a.nrhs + q0 + q] = czero<C>();
  }
}

constexpr int kAdjCols = 8;   // columns per wave and group in the adjoint core kernel

// F_{t,s}(cols) = C_{t,s}(:, cols)^H G_{t,s}.  A workgroup owns kGrp groups
// of 4 kAdjCols columns of one pair (one staging of G serves them all); in
// each group a wave takes kAdjCols columns, its lanes sweep the rows (VR per
// lane per 16-byte load, kAdjCols loads in flight) and the partial dot
// products are reduced across the wave.  The first group's first loads are
// issued before G is staged.
template <class T, class CS, int D, int QT, int kGrp>
__global__ void __launch_bounds__(kThreads)
    core_adj(CoreArgs a, const CS* __restrict__ cores, const long long* __restrict__ core_off,
             const int* __restrict__ meta, const int2* __restrict__ units,
             const typename CplxOf<T>::type* __restrict__ G, typename CplxOf<T>::type* __restrict__ F) {
  using C = typename CplxOf<T>::type;
  using CV = CoreVec<CS>;
  constexpr int VR = CV::VR;
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
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = blockIdx.y * QT;
  const int Qa = min(QT, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const typename CV::V* base = reinterpret_cast<const typename CV::V*>(cores + core_off[pair]);
  const long long cstride = RTp / VR;
  // columns of group g: cb(g) .. cb(g) + ncol(g) - 1; columns past the last
  // one re-read the last valid column (results unused)
  auto cb_of = [&](int g) { return c0 + (g * 4 + w) * kAdjCols; };
  auto ncol_of = [&](int g) { return max(0, min(kAdjCols, RS - cb_of(g))); };
  auto colp = [&](int g, int i) {
    const int nc = ncol_of(g);
    return base + (long long)(min(cb_of(g) + min(i, max(nc - 1, 0)), RS - 1)) * cstride;
  };
  typename CV::V vv[kAdjCols];
  const bool first = ncol_of(0) > 0 && lane * VR < RTp;
  if (first) {
#pragma unroll
    for (int i = 0; i < kAdjCols; ++i) vv[i] = colp(0, i)[lane];
  }
  for (int idx = threadIdx.x; idx < RTp * QT; idx += kThreads) {
    const int q = idx % QT, r = idx / QT;
    y[idx] = (r < RT && q < Qa) ? G[(titem * a.Et + padded_pos<D>(r, rt, a.Rt)) * a.nrhs + q0 + q]
                                : czero<C>();
  }
  __syncthreads();
#pragma unroll 1
  for (int g = 0; g < kGrp; ++g) {
    const int cb = cb_of(g), ncol = ncol_of(g);
    C acc[kAdjCols][QT];
#pragma unroll
    for (int i = 0; i < kAdjCols; ++i)
#pragma unroll
      for (int q = 0; q < QT; ++q) acc[i][q] = czero<C>();
    const typename CV::V* cp[kAdjCols];
#pragma unroll
    for (int i = 0; i < kAdjCols; ++i) cp[i] = colp(g, i);
    if (ncol > 0) {
      for (int rb = lane * VR; rb < RTp; rb += 64 * VR) {
        if (g != 0 || rb != lane * VR || !first) {
#pragma unroll
          for (int i = 0; i < kAdjCols; ++i) vv[i] = cp[i][rb / VR];
        }
        C yv[VR][QT];
#pragma unroll
        for (int v = 0; v < VR; ++v)
#pragma unroll
          for (int q = 0; q < QT; ++q) yv[v][q] = y[(rb + v) * QT + q];
#pragma unroll
        for (int i = 0; i < kAdjCols; ++i) {
          C c[VR];
          CV::get(vv[i], c);
#pragma unroll
          for (int v = 0; v < VR; ++v)
#pragma unroll
            for (int q = 0; q < QT; ++q) acc[i][q] = cfma_conj(acc[i][q], c[v], yv[v][q]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kAdjCols; ++i)
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        T re = acc[i][q].x, im = acc[i][q].y;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          re += __shfl_xor(re, o, 64);
          im += __shfl_xor(im, o, 64);
        }
        acc[i][q].x = re;
        acc[i][q].y = im;
      }
    if (lane < ncol) {
      // lane i writes column cb + i (values are identical across lanes)
#pragma unroll
      for (int i = 0; i < kAdjCols; ++i)
        if (i == lane) {
          const long long pos = padded_pos<D>(cb + i, rs, a.Rs);
          T sc = T(1);
          if constexpr (std::is_same<CS, Q16>::value) sc = a.colscale[a.col_off[pair] + cb + i];
#pragma unroll
          for (int q = 0; q < QT; ++q)
            if (q < Qa) {
              C v = acc[i][q];
              if constexpr (std::is_same<CS, Q16>::value) {
                v.x *= sc;
                v.y *= sc;
              }
              F[(sitem * a.Es + pos) * a.nrhs + q0 + q] = v;
            }
        }
    }
  }
  if (c0 == 0) {
    for (long long p = threadIdx.x; p < a.Es; p += kThreads)
      if (is_padding<D>(p, rs, a.Rs))
        for (int q = 0; q < Qa; ++q) F[(sitem * a.Es + p) * a.nrhs + q0 + q] = czero<C>();
  }
}

// The adjoint with 16-lane column groups: each wave is four groups of 16
// lanes, a group owns kAdjCols columns and its lanes sweep the rows (VR per
// lane per load), so a column's partial sums are reduced over 16 lanes (four
// steps) instead of 64.  A workgroup owns a 256-column panel (two passes of
// 4 waves x 4 groups x kAdjCols columns) and stages G once for it.
template <class T, class CS, int D, int QT>
__global__ void __launch_bounds__(kThreads)
    core_adj16(CoreArgs a, const CS* __restrict__ cores, const long long* __restrict__ core_off,
               const int* __restrict__ meta, const int2* __restrict__ units,
               const typename CplxOf<T>::type* __restrict__ G, typename CplxOf<T>::type* __restrict__ F) {
  using C = typename CplxOf<T>::type;
  using CV = CoreVec<CS>;
  constexpr int VR = CV::VR;
  constexpr int kPass = 4 * 4 * kAdjCols;  // columns per pass of the workgroup
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
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = blockIdx.y * QT;
  const int Qa = min(QT, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int grp = lane >> 4, gl = lane & 15;
  const typename CV::V* base = reinterpret_cast<const typename CV::V*>(cores + core_off[pair]);
  const long long cstride = RTp / VR;
  for (int idx = threadIdx.x; idx < RTp * QT; idx += kThreads) {
    const int q = idx % QT, r = idx / QT;
    y[idx] = (r < RT && q < Qa) ? G[(titem * a.Et + padded_pos<D>(r, rt, a.Rt)) * a.nrhs + q0 + q]
                                : czero<C>();
  }
  __syncthreads();
#pragma unroll 1
  for (int pass = 0; pass < 256 / kPass; ++pass) {
    const int cb = c0 + pass * kPass + (w * 4 + grp) * kAdjCols;
    const int ncol = max(0, min(kAdjCols, RS - cb));
    C acc[kAdjCols][QT];
#pragma unroll
    for (int i = 0; i < kAdjCols; ++i)
#pragma unroll
      for (int q = 0; q < QT; ++q) acc[i][q] = czero<C>();
    // columns past the last one re-read the last valid column (results unused)
    const typename CV::V* cp[kAdjCols];
#pragma unroll
    for (int i = 0; i < kAdjCols; ++i)
      cp[i] = base + (long long)min(cb + min(i, max(ncol - 1, 0)), RS - 1) * cstride;
    if (ncol > 0) {
      for (int rb = gl * VR; rb < RTp; rb += 16 * VR) {
        typename CV::V vv[kAdjCols];
#pragma unroll
        for (int i = 0; i < kAdjCols; ++i) vv[i] = cp[i][rb / VR];
        C yv[VR][QT];
#pragma unroll
        for (int v = 0; v < VR; ++v)
#pragma unroll
          for (int q = 0; q < QT; ++q) yv[v][q] = y[(rb + v) * QT + q];
#pragma unroll
        for (int i = 0; i < kAdjCols; ++i) {
          C c[VR];
          CV::get(vv[i], c);
#pragma unroll
          for (int v = 0; v < VR; ++v)
#pragma unroll
            for (int q = 0; q < QT; ++q) acc[i][q] = cfma_conj(acc[i][q], c[v], yv[v][q]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kAdjCols; ++i)
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        T re = acc[i][q].x, im = acc[i][q].y;
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {  // within the 16-lane group
          re += __shfl_xor(re, o, 64);
          im += __shfl_xor(im, o, 64);
        }
        acc[i][q].x = re;
        acc[i][q].y = im;
      }
    if (gl < ncol) {
      // lane gl of the group writes column cb + gl (values equal across the group)
#pragma unroll
      for (int i = 0; i < kAdjCols; ++i)
        if (i == gl) {
          const long long pos = padded_pos<D>(cb + i, rs, a.Rs);
          T sc = T(1);
          if constexpr (std::is_same<CS, Q16>::value) sc = a.colscale[a.col_off[pair] + cb + i];
#pragma unroll
          for (int q = 0; q < QT; ++q)
            if (q < Qa) {
              C v = acc[i][q];
              if constexpr (std::is_same<CS, Q16>::value) {
                v.x *= sc;
                v.y *= sc;
              }
              F[(sitem * a.Es + pos) * a.nrhs + q0 + q] = v;
            }
        }
    }
  }
  if (c0 == 0) {
    for (long long p = threadIdx.x; p < a.Es; p += kThreads)
      if (is_padding<D>(p, rs, a.Rs))
        for (int q = 0; q < Qa; ++q) F[(sitem * a.Es + p) * a.nrhs + q0 + q] = czero<C>();
  }
}

// -------------------------------------------------- on-the-fly cores --
// K(tbar, sbar) evaluated inside the core contraction instead of streamed
// from memory (no stored cores).  Every kernel is exp(2 pi i rev) * amp:
//   Fourier    rev = -(x . k) / n with x integer and k = j - n/2: an int32
//              sum reduced exactly modulo n (a power of two), amp = 1;
//   Helmholtz  rev = omega rho / (2 pi), amp = 1 / rho: the squared
//              distance n^2 rho^2 is a sum of squares of integer index
//              differences (plus n^2 for the plates' separation), exact in
//              FP64, then rho via rsqrt;
//   Radon      d = 2: rev = x . k + sqrt(c1(x)^2 k1^2 + c2(x)^2 k2^2), with
//              c1(x)^2, c2(x)^2 precomputed per target point; d = 3: rev =
//              x . k + c(x) |k| with c per target and |k| per source point;
//              amp = 1, in FP64;
//   NUDFT      rev = x . y with the target's coordinates x and y = j/n,
//              amp = 1, in FP64.
// The fraction of a turn goes to FP32 sine and cosine; the product with F
// runs in FP32.  A point is four ints (Fourier, Helmholtz: the per-mode
// grid indices, the source's first index shifted by 2n for the cube
// offset) or four doubles (Radon: x1, x2, c1^2, c2^2 on the target side,
// k1, k2 on the source side; NUDFT: the coordinates).
constexpr int kOtfChunk = 1024;  // points of the contracted index staged at a time

struct OtfSpec {
  const double* nux;  // non-uniform DFT: d * n target coordinates
  long long n;
  double omega_rev;  // omega / (2 pi)
  double ra, rb, rden;
  int Rs_sk, Rt_sk;  // row length of the skeleton tables
};

template <int KIND>
struct OtfPoint {
  using V = int4;
};
template <>
struct OtfPoint<TB_KERNEL_RADON> {
  using V = double4;
};
template <>
struct OtfPoint<TB_KERNEL_NUDFT> {
  using V = double4;
};

template <int KIND, int D>
__device__ __forceinline__ typename OtfPoint<KIND>::V otf_target(const OtfSpec& o, const int* ti) {
  if constexpr (KIND == TB_KERNEL_NUDFT) {  // the target's coordinates
    return make_double4(o.nux[ti[0]], o.nux[o.n + ti[1]], D == 3 ? o.nux[2 * o.n + ti[D - 1]] : 0.0, 0.0);
  } else if constexpr (KIND == TB_KERNEL_RADON && D == 3) {
    const double inv = 1.0 / (double)o.n;
    double x[3], sp = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      x[k] = ti[k] * inv;
      double sk, ck;
      sincospi(2.0 * x[k], &sk, &ck);
      sp *= sk;
    }
    return make_double4(x[0], x[1], x[2], (o.ra + o.rb * sp) / o.rden);
  } else if constexpr (KIND == TB_KERNEL_RADON) {
    const double inv = 1.0 / (double)o.n;
    const double x1 = ti[0] * inv, x2 = ti[1] * inv;
    double s1, c1, s2, c2;
    sincospi(2.0 * x1, &s1, &c1);
    sincospi(2.0 * x2, &s2, &c2);
    const double a1 = (o.ra + o.rb * s1 * s2) / o.rden, a2 = (o.ra + o.rb * c1 * c2) / o.rden;
    return make_double4(x1, x2, a1 * a1, a2 * a2);
  } else {
    return make_int4(ti[0], ti[1], D == 3 ? ti[D - 1] : 0, 0);
  }
}

template <int KIND, int D>
__device__ __forceinline__ typename OtfPoint<KIND>::V otf_source(const OtfSpec& o, const int* sj) {
  const int h = (int)(o.n / 2);
  if constexpr (KIND == TB_KERNEL_NUDFT) {  // y = j/n, exact (n is a power of two)
    const double inv = 1.0 / (double)o.n;
    return make_double4(sj[0] * inv, sj[1] * inv, D == 3 ? sj[D - 1] * inv : 0.0, 0.0);
  } else if constexpr (KIND == TB_KERNEL_RADON && D == 3) {
    const double k0 = sj[0] - h, k1 = sj[1] - h, k2 = sj[2] - h;
    return make_double4(k0, k1, k2, sqrt(k0 * k0 + k1 * k1 + k2 * k2));
  } else if constexpr (KIND == TB_KERNEL_RADON) {
    return make_double4((double)(sj[0] - h), (double)(sj[1] - h), 0.0, 0.0);
  } else if constexpr (KIND == TB_KERNEL_FOURIER) {
    return make_int4(sj[0] - h, sj[1] - h, D == 3 ? sj[D - 1] - h : 0, 0);
  } else if constexpr (D == 3) {  // cubes: y = j/n + (2, 0, 0), index j_0 + 2n
    return make_int4(sj[0] + 2 * (int)o.n, sj[1], sj[2], 0);
  } else {  // plates: in-plane indices (the plane distance enters as n^2)
    return make_int4(sj[0], sj[1], 0, 0);
  }
}

// 1/sqrt(q), q > 0: the hardware estimate (v_rsq_f64, about 2^-23 relative)
// and one Newton step, y (3 - q y^2) / 2, which brings it to about 1e-14
__device__ __forceinline__ double rsqrt64(double q) {
  double y = __builtin_amdgcn_rsq(q);
  return y * fma(-0.5 * q * y, y, 1.5);
}

// entry from target point x and source point y
template <int KIND, int D>
__device__ __forceinline__ float2 otf_entry(const OtfSpec& o, const typename OtfPoint<KIND>::V& x,
                                            const typename OtfPoint<KIND>::V& y) {
  float f, amp = 1.f;
  if constexpr (KIND == TB_KERNEL_FOURIER) {
    int p = x.x * y.x + x.y * y.y;  // |p| < 3 n^2 / 2 < 2^31 for n <= 2^15
    if (D == 3) p += x.z * y.z;
    const int nm = (int)o.n - 1;
    f = (float)((-p) & nm) * (1.f / (float)o.n);  // exact: n is a power of two
  } else if constexpr (KIND == TB_KERNEL_HELMHOLTZ) {
    const double d0 = (double)(x.x - y.x), d1 = (double)(x.y - y.y), d2 = (double)(x.z - y.z);
    const double inv = 1.0 / (double)o.n;
    const double gap = D == 2 ? (double)o.n * (double)o.n : 0.0;  // plates: distance 1 = n steps
    const double r2 = (fma(d0, d0, fma(d1, d1, d2 * d2)) + gap) * (inv * inv);  // exact scaling
    const double ir = rsqrt64(r2);  // the cubes are apart: r2 >= 1
    const double rev = o.omega_rev * (r2 * ir);
    f = (float)(rev - floor(rev));
    amp = (float)ir;
  } else if constexpr (KIND == TB_KERNEL_NUDFT) {  // x.y
    const double rev = fma(x.x, y.x, fma(x.y, y.y, x.z * y.z));
    f = (float)(rev - floor(rev));
  } else if constexpr (D == 3) {  // Radon 3-D: x.k + c |k|
    const double rev = fma(x.x, y.x, fma(x.y, y.y, fma(x.z, y.z, x.w * y.w)));
    f = (float)(rev - floor(rev));
  } else {
    const double q = x.z * y.x * y.x + x.w * y.y * y.y;
    const double rev = x.x * y.x + x.y * y.y + (q > 0.0 ? q * rsqrt64(q) : 0.0);
    f = (float)(rev - floor(rev));
  }
  // v_sin_f32 / v_cos_f32 take the angle in revolutions
  return make_float2(amp * __builtin_amdgcn_cosf(f), amp * __builtin_amdgcn_sinf(f));
}

// per-mode skeleton indices of flat row (or column) index r of a pair
template <int D>
__device__ __forceinline__ void otf_index(const int* skel, long long item, int Rsk, const int* rk, int r,
                                          int* idx) {
#pragma unroll
  for (int k = D - 1; k >= 0; --k) {
    idx[k] = skel[(item * D + k) * Rsk + r % rk[k]];
    r /= rk[k];
  }
}

// G_{t,s}(rows) = K(tbar, sbar)(rows, :) F_{t,s}: 64 rows per workgroup, one
// per lane, the four waves split the columns and reduce through LDS.
template <int KIND, int D, int QT>
__global__ void __launch_bounds__(kThreads)
    core_fwd_otf(CoreArgs a, OtfSpec o, const int* __restrict__ meta, const int2* __restrict__ units,
                 const int* __restrict__ sskel, const int* __restrict__ tskel, const float2* __restrict__ F,
                 float2* __restrict__ G) {
  using P = typename OtfPoint<KIND>::V;
  extern __shared__ unsigned char smem_raw[];
  const int2 u = units[blockIdx.x];
  if (u.x < 0) return;  // padding of the XCD-grouped unit list (whole workgroup)
  const int pair = u.x, r0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = blockIdx.y * QT;
  const int Qa = min(QT, a.nrhs - q0);
  // the source points and F of at most kOtfChunk columns at a time
  const int CH = min(RS, kOtfChunk);
  P* yv = reinterpret_cast<P*>(smem_raw);                 // [CH]
  float2* x = reinterpret_cast<float2*>(yv + CH);          // [CH][QT]
  float2* red = x + CH * QT;                               // [256][QT]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = r0 + lane;
  P xv;
  {
    int ti[D];
    otf_index<D>(tskel, titem, o.Rt_sk, rt, min(row, RT - 1), ti);
    xv = otf_target<KIND, D>(o, ti);
  }
  float2 acc[QT];
#pragma unroll
  for (int q = 0; q < QT; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int c0 = 0; c0 < RS; c0 += CH) {
    const int nc = min(CH, RS - c0);
    if (c0 > 0) __syncthreads();  // the previous chunk is read
    for (int b = threadIdx.x; b < nc; b += kThreads) {
      int sj[D];
      otf_index<D>(sskel, sitem, o.Rs_sk, rs, c0 + b, sj);
      yv[b] = otf_source<KIND, D>(o, sj);
    }
    for (int idx = threadIdx.x; idx < nc * QT; idx += kThreads) {
      const int q = idx % QT, b = idx / QT;
      x[idx] = q < Qa ? F[(sitem * a.Es + padded_pos<D>(c0 + b, rs, a.Rs)) * a.nrhs + q0 + q]
                      : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int per = (nc + 3) / 4;
    const int j0 = w * per, j1 = min(nc, j0 + per);
    for (int j = j0; j < j1; ++j) {
      const float2 c = otf_entry<KIND, D>(o, xv, yv[j]);
#pragma unroll
      for (int q = 0; q < QT; ++q) acc[q] = cfma(acc[q], c, x[j * QT + q]);
    }
  }
#pragma unroll
  for (int q = 0; q < QT; ++q) red[(w * 64 + lane) * QT + q] = acc[q];
  __syncthreads();
  if (w == 0 && row < RT) {
    const long long pos = padded_pos<D>(row, rt, a.Rt);
#pragma unroll
    for (int q = 0; q < QT; ++q)
      if (q < Qa) {
        float2 sum = red[lane * QT + q];
        sum = cadd(sum, red[(64 + lane) * QT + q]);
        sum = cadd(sum, red[(128 + lane) * QT + q]);
        sum = cadd(sum, red[(192 + lane) * QT + q]);
        G[(titem * a.Et + pos) * a.nrhs + q0 + q] = sum;
      }
  }
  if (r0 == 0) {  // padding of the output item is written as zeros
    for (long long p = threadIdx.x; p < a.Et; p += kThreads)
      if (is_padding<D>(p, rt, a.Rt))
        for (int q = 0; q < Qa; ++q) G[(titem * a.Et + p) * a.nrhs + q0 + q] = make_float2(0.f, 0.f);
  }
}

// F_{t,s}(cols) = K(tbar, sbar)(:, cols)^H G_{t,s}: 64 columns per
// workgroup, one per lane, the four waves split the rows.
template <int KIND, int D, int QT>
__global__ void __launch_bounds__(kThreads)
    core_adj_otf(CoreArgs a, OtfSpec o, const int* __restrict__ meta, const int2* __restrict__ units,
                 const int* __restrict__ sskel, const int* __restrict__ tskel, const float2* __restrict__ G,
                 float2* __restrict__ F) {
  using P = typename OtfPoint<KIND>::V;
  extern __shared__ unsigned char smem_raw[];
  const int2 u = units[blockIdx.x];
  const int pair = u.x, c0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = blockIdx.y * QT;
  const int Qa = min(QT, a.nrhs - q0);
  // the target points and G of at most kOtfChunk rows at a time
  const int CH = min(RT, kOtfChunk);
  P* xr = reinterpret_cast<P*>(smem_raw);                 // [CH]
  float2* g = reinterpret_cast<float2*>(xr + CH);          // [CH][QT]
  float2* red = g + CH * QT;                               // [256][QT]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = c0 + lane;
  P yv;
  {
    int sj[D];
    otf_index<D>(sskel, sitem, o.Rs_sk, rs, min(col, RS - 1), sj);
    yv = otf_source<KIND, D>(o, sj);
  }
  float2 acc[QT];
#pragma unroll
  for (int q = 0; q < QT; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int r0 = 0; r0 < RT; r0 += CH) {
    const int nr = min(CH, RT - r0);
    if (r0 > 0) __syncthreads();  // the previous chunk is read
    for (int b = threadIdx.x; b < nr; b += kThreads) {
      int ti[D];
      otf_index<D>(tskel, titem, o.Rt_sk, rt, r0 + b, ti);
      xr[b] = otf_target<KIND, D>(o, ti);
    }
    for (int idx = threadIdx.x; idx < nr * QT; idx += kThreads) {
      const int q = idx % QT, b = idx / QT;
      g[idx] = q < Qa ? G[(titem * a.Et + padded_pos<D>(r0 + b, rt, a.Rt)) * a.nrhs + q0 + q]
                      : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int per = (nr + 3) / 4;
    const int i0 = w * per, i1 = min(nr, i0 + per);
    for (int i = i0; i < i1; ++i) {
      const float2 c = otf_entry<KIND, D>(o, xr[i], yv);
#pragma unroll
      for (int q = 0; q < QT; ++q) acc[q] = cfma_conj(acc[q], c, g[i * QT + q]);
    }
  }
#pragma unroll
  for (int q = 0; q < QT; ++q) red[(w * 64 + lane) * QT + q] = acc[q];
  __syncthreads();
  if (w == 0 && col < RS) {
    const long long pos = padded_pos<D>(col, rs, a.Rs);
#pragma unroll
    for (int q = 0; q < QT; ++q)
      if (q < Qa) {
        float2 sum = red[lane * QT + q];
        sum = cadd(sum, red[(64 + lane) * QT + q]);
        sum = cadd(sum, red[(128 + lane) * QT + q]);
        sum = cadd(sum, red[(192 + lane) * QT + q]);
        F[(sitem * a.Es + pos) * a.nrhs + q0 + q] = sum;
      }
  }
  if (c0 == 0) {
    for (long long p = threadIdx.x; p < a.Es; p += kThreads)
      if (is_padding<D>(p, rs, a.Rs))
        for (int q = 0; q < Qa; ++q) F[(sitem * a.Es + p) * a.nrhs + q0 + q] = make_float2(0.f, 0.f);
  }
}

// --------------------------------------------------------- MFMA cores --
// Many right-hand sides: the core contraction is a dense complex GEMM per
// pair, G (R_T x Q) = C (R_T x R_S) F (R_S x Q), run on the matrix cores as
// four real v_mfma_f32_16x16x4f32 per complex 16 x 16 x 4 step:
//   Gr += Cr Fr - Ci Fi,   Gi += Cr Fi + Ci Fr.
// Lane layout of the 16x16x4 f32 MFMA: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register j holds D[4 (l / 16) + j][l % 16].
// BF16 cores are widened to FP32 in registers (FP32 accumulation).
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMQ = 32;    // right-hand sides per workgroup (two 16-wide tiles)
constexpr int kMT = 4;     // 16-row (or 16-column) tiles per wave
constexpr int kMKC = 64;   // forward: rows of F staged per chunk
constexpr int kMKA = 16;   // adjoint: rows of C and G staged per chunk

template <class CS>
__device__ __forceinline__ float2 load_core1(const CS* p) {
  if constexpr (sizeof(CS) == 4) {
    const unsigned u = *reinterpret_cast<const unsigned*>(p);
    return CoreVec<unsigned>::one(u);
  } else {
    return *reinterpret_cast<const float2*>(p);
  }
}

__device__ __forceinline__ void cmfma(v4f& ar, v4f& ai, float2 x, float2 y) {
  ar = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.x, ar, 0, 0, 0);
  ar = __builtin_amdgcn_mfma_f32_16x16x4f32(-x.y, y.y, ar, 0, 0, 0);
  ai = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.y, ai, 0, 0, 0);
  ai = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, y.x, ai, 0, 0, 0);
}

// Forward: a workgroup owns 4 waves x kMT x 16 = 256 rows of one pair and
// kMQ right-hand sides; F is staged through LDS in chunks of kMKC rows.
template <class CS, int D>
__global__ void __launch_bounds__(kThreads)
    core_fwd_mfma(CoreArgs a, const CS* __restrict__ cores, const long long* __restrict__ core_off,
                  const int* __restrict__ meta, const int2* __restrict__ units,
                  const float2* __restrict__ F, float2* __restrict__ G) {
  __shared__ float2 fs[kMKC * kMQ];
  // flattened (unit, RHS tile) with the tile fastest, XCD-contiguous
  const int nqt = (a.nrhs + kMQ - 1) / kMQ;
  const int item = xcd_item(blockIdx.x, gridDim.x, nqt);
  const int2 u = units[item / nqt];
  const int pair = u.x, r0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = (item % nqt) * kMQ;
  const int Qa = min(kMQ, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const CS* cb = cores + core_off[pair];
  v4f accr[kMT][2], acci[kMT][2];
#pragma unroll
  for (int i = 0; i < kMT; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accr[i][c] = v4f{0, 0, 0, 0};
      acci[i][c] = v4f{0, 0, 0, 0};
    }
  int rowc[kMT];
  bool live[kMT];
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    const int tile0 = r0 + (w + 4 * i) * 16;
    live[i] = tile0 < RT;
    rowc[i] = min(tile0 + (lane & 15), RTp - 1);
  }
  for (int kc = 0; kc < RS; kc += kMKC) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kMKC * kMQ; idx += kThreads) {
      const int kk = kc + idx / kMQ, q = idx % kMQ;
      fs[idx] = (kk < RS && q < Qa) ? F[(sitem * a.Es + padded_pos<D>(kk, rs, a.Rs)) * a.nrhs + q0 + q]
                                    : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int kend = min(kMKC, RS - kc);
    for (int ks = 0; ks < kend; ks += 4) {
      const int kcl = min(kc + ks + (lane >> 4), RS - 1);
      float2 av[kMT];
#pragma unroll
      for (int i = 0; i < kMT; ++i) av[i] = load_core1(cb + (long long)kcl * RTp + rowc[i]);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float2 bv = fs[(ks + (lane >> 4)) * kMQ + c * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < kMT; ++i)
          if (live[i]) cmfma(accr[i][c], acci[i][c], av[i], bv);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    if (!live[i]) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = r0 + (w + 4 * i) * 16 + 4 * (lane >> 4) + j;
        const int col = c * 16 + (lane & 15);
        if (row < RT && col < Qa)
          G[(titem * a.Et + padded_pos<D>(row, rt, a.Rt)) * a.nrhs + q0 + col] =
              make_float2(accr[i][c][j], acci[i][c][j]);
      }
  }
}

// Adjoint: F (R_S x Q) = C^H G.  A workgroup owns 256 columns of one pair
// and kMQ right-hand sides; 16-row slabs of C (all 256 columns) and of G are
// staged through LDS, so the global reads stay column-contiguous while each
// lane reads the transposed fragment from LDS.
template <class CS, int D>
__global__ void __launch_bounds__(kThreads)
    core_adj_mfma(CoreArgs a, const CS* __restrict__ cores, const long long* __restrict__ core_off,
                  const int* __restrict__ meta, const int2* __restrict__ units,
                  const float2* __restrict__ G, float2* __restrict__ F) {
  constexpr int kCols = 4 * kMT * 16;           // 256
  constexpr int kLd = kMKA + 1;                 // padded column length in LDS
  __shared__ float2 cs_[kCols * kLd];
  __shared__ float2 gs[kMKA * kMQ];
  // flattened (unit, RHS tile) with the tile fastest, XCD-contiguous
  const int nqt = (a.nrhs + kMQ - 1) / kMQ;
  const int item = xcd_item(blockIdx.x, gridDim.x, nqt);
  const int2 u = units[item / nqt];
  const int pair = u.x, c0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = (item % nqt) * kMQ;
  const int Qa = min(kMQ, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const CS* cb = cores + core_off[pair];
  v4f accr[kMT][2], acci[kMT][2];
#pragma unroll
  for (int i = 0; i < kMT; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accr[i][c] = v4f{0, 0, 0, 0};
      acci[i][c] = v4f{0, 0, 0, 0};
    }
  bool live[kMT];
#pragma unroll
  for (int i = 0; i < kMT; ++i) live[i] = c0 + (w + 4 * i) * 16 < RS;
  for (int k0 = 0; k0 < RTp; k0 += kMKA) {
    __syncthreads();
    // C slab: rows k0..k0+15 of columns c0..c0+255 (zero past the pair)
    for (int idx = threadIdx.x; idx < kCols * kMKA; idx += kThreads) {
      const int col = idx / kMKA, r = idx % kMKA;
      const int gc = c0 + col, gr = k0 + r;
      float2 v = make_float2(0.f, 0.f);
      if (gc < RS && gr < RTp) v = load_core1(cb + (long long)gc * RTp + gr);
      cs_[col * kLd + r] = v;
    }
    for (int idx = threadIdx.x; idx < kMKA * kMQ; idx += kThreads) {
      const int r = idx / kMQ, q = idx % kMQ;
      const int gr = k0 + r;
      gs[idx] = (gr < RT && q < Qa) ? G[(titem * a.Et + padded_pos<D>(gr, rt, a.Rt)) * a.nrhs + q0 + q]
                                    : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kMKA; ks += 4) {
      float2 bv[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = gs[(ks + (lane >> 4)) * kMQ + c * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < kMT; ++i) {
        if (!live[i]) continue;
        float2 av = cs_[((w + 4 * i) * 16 + (lane & 15)) * kLd + ks + (lane >> 4)];
        av.y = -av.y;  // conj(C)
#pragma unroll
        for (int c = 0; c < 2; ++c) cmfma(accr[i][c], acci[i][c], av, bv[c]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    if (!live[i]) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = c0 + (w + 4 * i) * 16 + 4 * (lane >> 4) + j;
        const int q = c * 16 + (lane & 15);
        if (col < RS && q < Qa)
          F[(sitem * a.Es + padded_pos<D>(col, rs, a.Rs)) * a.nrhs + q0 + q] =
              make_float2(accr[i][c][j], acci[i][c][j]);
      }
  }
}

// On-the-fly cores on the matrix cores (many right-hand sides): the
// kernels above with every A fragment evaluated as K(tbar, sbar) from the
// skeleton points instead of loaded, FP64 phase and FP32 sine and cosine as
// in the vector on-the-fly kernels.  At nrhs right-hand sides each entry
// serves nrhs complex products, so its evaluation amortises.
//
// Forward: each lane keeps the target points of its kMT rows in registers;
// the source points of a chunk of kMKC columns are staged in LDS beside F.
template <int KIND, int D>
__global__ void __launch_bounds__(kThreads)
    core_fwd_mfma_otf(CoreArgs a, OtfSpec o, const int* __restrict__ meta, const int2* __restrict__ units,
                      const int* __restrict__ sskel, const int* __restrict__ tskel,
                      const float2* __restrict__ F, float2* __restrict__ G) {
  using P = typename OtfPoint<KIND>::V;
  __shared__ float2 fs[kMKC * kMQ];
  __shared__ P sp[kMKC];
  const int nqt = (a.nrhs + kMQ - 1) / kMQ;
  const int item = xcd_item(blockIdx.x, gridDim.x, nqt);
  const int2 u = units[item / nqt];
  const int pair = u.x, r0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = (item % nqt) * kMQ;
  const int Qa = min(kMQ, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v4f accr[kMT][2], acci[kMT][2];
#pragma unroll
  for (int i = 0; i < kMT; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accr[i][c] = v4f{0, 0, 0, 0};
      acci[i][c] = v4f{0, 0, 0, 0};
    }
  bool live[kMT];
  P tp[kMT];
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    const int tile0 = r0 + (w + 4 * i) * 16;
    live[i] = tile0 < RT;
    int ti[D];
    otf_index<D>(tskel, titem, o.Rt_sk, rt, min(tile0 + (lane & 15), RT - 1), ti);
    tp[i] = otf_target<KIND, D>(o, ti);
  }
  for (int kc = 0; kc < RS; kc += kMKC) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kMKC * kMQ; idx += kThreads) {
      const int kk = kc + idx / kMQ, q = idx % kMQ;
      fs[idx] = (kk < RS && q < Qa) ? F[(sitem * a.Es + padded_pos<D>(kk, rs, a.Rs)) * a.nrhs + q0 + q]
                                    : make_float2(0.f, 0.f);
    }
    for (int idx = threadIdx.x; idx < kMKC; idx += kThreads) {
      int sj[D];  // columns past the pair take the last one's point (their F is zero)
      otf_index<D>(sskel, sitem, o.Rs_sk, rs, min(kc + idx, RS - 1), sj);
      sp[idx] = otf_source<KIND, D>(o, sj);
    }
    __syncthreads();
    const int kend = min(kMKC, RS - kc);
    for (int ks = 0; ks < kend; ks += 4) {
      const P y = sp[ks + (lane >> 4)];
      float2 av[kMT];
#pragma unroll
      for (int i = 0; i < kMT; ++i) av[i] = otf_entry<KIND, D>(o, tp[i], y);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float2 bv = fs[(ks + (lane >> 4)) * kMQ + c * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < kMT; ++i)
          if (live[i]) cmfma(accr[i][c], acci[i][c], av[i], bv);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    if (!live[i]) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = r0 + (w + 4 * i) * 16 + 4 * (lane >> 4) + j;
        const int col = c * 16 + (lane & 15);
        if (row < RT && col < Qa)
          G[(titem * a.Et + padded_pos<D>(row, rt, a.Rt)) * a.nrhs + q0 + col] =
              make_float2(accr[i][c][j], acci[i][c][j]);
      }
  }
}

// Adjoint: the source points of the workgroup's 256 columns are staged once,
// the target points of each 16-row slab beside G, and the slab of entries is
// evaluated into LDS where the stored-core kernel loads it.
template <int KIND, int D>
__global__ void __launch_bounds__(kThreads)
    core_adj_mfma_otf(CoreArgs a, OtfSpec o, const int* __restrict__ meta, const int2* __restrict__ units,
                      const int* __restrict__ sskel, const int* __restrict__ tskel,
                      const float2* __restrict__ G, float2* __restrict__ F) {
  using P = typename OtfPoint<KIND>::V;
  constexpr int kCols = 4 * kMT * 16;           // 256
  constexpr int kLd = kMKA + 1;                 // padded column length in LDS
  __shared__ float2 cs_[kCols * kLd];
  __shared__ float2 gs[kMKA * kMQ];
  __shared__ P sp[kCols];
  __shared__ P tpl[kMKA];
  const int nqt = (a.nrhs + kMQ - 1) / kMQ;
  const int item = xcd_item(blockIdx.x, gridDim.x, nqt);
  const int2 u = units[item / nqt];
  const int pair = u.x, c0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = (item % nqt) * kMQ;
  const int Qa = min(kMQ, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int idx = threadIdx.x; idx < kCols; idx += kThreads) {
    int sj[D];  // columns past the pair take the last one's point (never used)
    otf_index<D>(sskel, sitem, o.Rs_sk, rs, min(c0 + idx, RS - 1), sj);
    sp[idx] = otf_source<KIND, D>(o, sj);
  }
  v4f accr[kMT][2], acci[kMT][2];
#pragma unroll
  for (int i = 0; i < kMT; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accr[i][c] = v4f{0, 0, 0, 0};
      acci[i][c] = v4f{0, 0, 0, 0};
    }
  bool live[kMT];
#pragma unroll
  for (int i = 0; i < kMT; ++i) live[i] = c0 + (w + 4 * i) * 16 < RS;
  for (int k0 = 0; k0 < RT; k0 += kMKA) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kMKA; idx += kThreads) {
      int ti[D];
      otf_index<D>(tskel, titem, o.Rt_sk, rt, min(k0 + idx, RT - 1), ti);
      tpl[idx] = otf_target<KIND, D>(o, ti);
    }
    for (int idx = threadIdx.x; idx < kMKA * kMQ; idx += kThreads) {
      const int r = idx / kMQ, q = idx % kMQ;
      const int gr = k0 + r;
      gs[idx] = (gr < RT && q < Qa) ? G[(titem * a.Et + padded_pos<D>(gr, rt, a.Rt)) * a.nrhs + q0 + q]
                                    : make_float2(0.f, 0.f);
    }
    __syncthreads();
    // slab of entries: rows k0..k0+15 of columns c0..c0+255 (zero past the pair)
    for (int idx = threadIdx.x; idx < kCols * kMKA; idx += kThreads) {
      const int col = idx / kMKA, r = idx % kMKA;
      float2 v = make_float2(0.f, 0.f);
      if (c0 + col < RS && k0 + r < RT) v = otf_entry<KIND, D>(o, tpl[r], sp[col]);
      cs_[col * kLd + r] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kMKA; ks += 4) {
      float2 bv[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = gs[(ks + (lane >> 4)) * kMQ + c * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < kMT; ++i) {
        if (!live[i]) continue;
        float2 av = cs_[((w + 4 * i) * 16 + (lane & 15)) * kLd + ks + (lane >> 4)];
        av.y = -av.y;  // conj(C)
#pragma unroll
        for (int c = 0; c < 2; ++c) cmfma(accr[i][c], acci[i][c], av, bv[c]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    if (!live[i]) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = c0 + (w + 4 * i) * 16 + 4 * (lane >> 4) + j;
        const int q = c * 16 + (lane & 15);
        if (col < RS && q < Qa)
          F[(sitem * a.Es + padded_pos<D>(col, rs, a.Rs)) * a.nrhs + q0 + q] =
              make_float2(accr[i][c][j], acci[i][c][j]);
      }
  }
}

// BF16 cores on BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation).  A complex product is one real product per output part
// with real and imaginary parts interleaved along k: with k' = 2 k + p,
//   forward  Gr: A = (Cr, -Ci), Gi: A = (Ci, Cr), B = (Fr, Fi);
//   adjoint  Fr: A = (Cr, Ci),  Fi: A = (-Ci, Cr), B = (Gr, Gi)  (conj(C)).
// A stored core is one 32-bit word (bf16 re low, bf16 im high), so each A
// pair is the word itself, the word with a sign bit flipped, or the word
// with its halves swapped.  The FP32 right-hand sides are split into
// bf16 hi + lo (two products), so their rounding (about 2^-17) stays far
// below that of the BF16 cores.  Lane layout: lane l supplies A[l % 16][8 (l
// / 16) + i] and B[8 (l / 16) + i][l % 16], i = 0..7; accumulator register j
// holds D[4 (l / 16) + j][l % 16].
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
constexpr int kBK = 64;       // complex k staged per chunk
constexpr int kBLd = kBK + 4;  // LDS row stride in words: 16-byte aligned, 2-way banked

__device__ __forceinline__ unsigned pack_bf16(float re, float im) {
  return (unsigned)f32_to_bf16(re) | ((unsigned)f32_to_bf16(im) << 16);
}
__device__ __forceinline__ void split_bf16(float2 v, unsigned* hi, unsigned* lo) {
  const unsigned h = pack_bf16(v.x, v.y);
  *hi = h;
  *lo = pack_bf16(v.x - bf16_to_f32((unsigned short)(h & 0xffff)),
                  v.y - bf16_to_f32((unsigned short)(h >> 16)));
}
__device__ __forceinline__ v8bf as_v8bf(uint4 u) { return __builtin_bit_cast(v8bf, u); }
__device__ __forceinline__ unsigned swap16(unsigned u) { return (u >> 16) | (u << 16); }
__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Forward: 256 rows of one pair (4 waves x kMT 16-row tiles) and kMQ
// right-hand sides per workgroup; F staged through LDS as bf16 hi/lo,
// [q][k] so that a lane's 8 k-values are one 16-byte read.
template <int D>
__global__ void __launch_bounds__(kThreads)
    core_fwd_mfma_bf16(CoreArgs a, const unsigned* __restrict__ cores, const long long* __restrict__ core_off,
                       const int* __restrict__ meta, const int2* __restrict__ units,
                       const float2* __restrict__ F, float2* __restrict__ G) {
  __shared__ uint4 fhi[kMQ * kBLd / 4], flo[kMQ * kBLd / 4];
  // flattened (unit, RHS tile) with the tile fastest, XCD-contiguous
  const int nqt = (a.nrhs + kMQ - 1) / kMQ;
  const int item = xcd_item(blockIdx.x, gridDim.x, nqt);
  const int2 u = units[item / nqt];
  const int pair = u.x, r0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = (item % nqt) * kMQ;
  const int Qa = min(kMQ, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned* cb = cores + core_off[pair];
  unsigned* fh = reinterpret_cast<unsigned*>(fhi);
  unsigned* fl = reinterpret_cast<unsigned*>(flo);
  v4f accr[kMT][2], acci[kMT][2];
#pragma unroll
  for (int i = 0; i < kMT; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accr[i][c] = v4f{0, 0, 0, 0};
      acci[i][c] = v4f{0, 0, 0, 0};
    }
  int rowc[kMT];
  bool live[kMT];
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    const int tile0 = r0 + (w + 4 * i) * 16;
    live[i] = tile0 < RT;
    rowc[i] = min(tile0 + (lane & 15), RTp - 1);
  }
  for (int kc = 0; kc < RS; kc += kBK) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kBK * kMQ; idx += kThreads) {
      const int kk = idx / kMQ, q = idx % kMQ, k = kc + kk;  // q fastest: coalesced reads
      const float2 v = (k < RS && q < Qa) ? F[(sitem * a.Es + padded_pos<D>(k, rs, a.Rs)) * a.nrhs + q0 + q]
                                          : make_float2(0.f, 0.f);
      split_bf16(v, &fh[q * kBLd + kk], &fl[q * kBLd + kk]);
    }
    __syncthreads();
    const int kend = min(kBK, RS - kc);
    for (int ks = 0; ks < kend; ks += 16) {
      const int kl = ks + 4 * (lane >> 4);  // first of this lane's 4 complex k
      uint4 bh[2], bl[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int q = c * 16 + (lane & 15);
        bh[c] = fhi[(q * kBLd + kl) / 4];
        bl[c] = flo[(q * kBLd + kl) / 4];
      }
#pragma unroll
      for (int i = 0; i < kMT; ++i) {
        if (!live[i]) continue;
        unsigned cw[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) cw[e] = cb[(long long)min(kc + kl + e, RS - 1) * RTp + rowc[i]];
        const v8bf ar = as_v8bf(make_uint4(cw[0] ^ 0x80000000u, cw[1] ^ 0x80000000u, cw[2] ^ 0x80000000u,
                                           cw[3] ^ 0x80000000u));
        const v8bf ai = as_v8bf(make_uint4(swap16(cw[0]), swap16(cw[1]), swap16(cw[2]), swap16(cw[3])));
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          accr[i][c] = mfma_bf16(ar, as_v8bf(bh[c]), accr[i][c]);
          accr[i][c] = mfma_bf16(ar, as_v8bf(bl[c]), accr[i][c]);
          acci[i][c] = mfma_bf16(ai, as_v8bf(bh[c]), acci[i][c]);
          acci[i][c] = mfma_bf16(ai, as_v8bf(bl[c]), acci[i][c]);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    if (!live[i]) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = r0 + (w + 4 * i) * 16 + 4 * (lane >> 4) + j;
        const int col = c * 16 + (lane & 15);
        if (row < RT && col < Qa)
          G[(titem * a.Et + padded_pos<D>(row, rt, a.Rt)) * a.nrhs + q0 + col] =
              make_float2(accr[i][c][j], acci[i][c][j]);
      }
  }
}

// Adjoint: 256 columns of one pair and kMQ right-hand sides per workgroup;
// a lane's 4 consecutive rows of its column are one 16-byte load (the cores
// are column-major), G staged through LDS as bf16 hi/lo, [q][row].
template <int D>
__global__ void __launch_bounds__(kThreads)
    core_adj_mfma_bf16(CoreArgs a, const unsigned* __restrict__ cores, const long long* __restrict__ core_off,
                       const int* __restrict__ meta, const int2* __restrict__ units,
                       const float2* __restrict__ G, float2* __restrict__ F) {
  __shared__ uint4 ghi[kMQ * kBLd / 4], glo[kMQ * kBLd / 4];
  // flattened (unit, RHS tile) with the tile fastest, XCD-contiguous
  const int nqt = (a.nrhs + kMQ - 1) / kMQ;
  const int item = xcd_item(blockIdx.x, gridDim.x, nqt);
  const int2 u = units[item / nqt];
  const int pair = u.x, c0 = u.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  int rt[D], rs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const int q0 = (item % nqt) * kMQ;
  const int Qa = min(kMQ, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned* cb = cores + core_off[pair];
  unsigned* gh = reinterpret_cast<unsigned*>(ghi);
  unsigned* gl = reinterpret_cast<unsigned*>(glo);
  v4f accr[kMT][2], acci[kMT][2];
#pragma unroll
  for (int i = 0; i < kMT; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accr[i][c] = v4f{0, 0, 0, 0};
      acci[i][c] = v4f{0, 0, 0, 0};
    }
  int colc[kMT];
  bool live[kMT];
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    const int tile0 = c0 + (w + 4 * i) * 16;
    live[i] = tile0 < RS;
    colc[i] = min(tile0 + (lane & 15), RS - 1);
  }
  for (int kc = 0; kc < RT; kc += kBK) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kBK * kMQ; idx += kThreads) {
      const int kk = idx / kMQ, q = idx % kMQ, k = kc + kk;
      const float2 v = (k < RT && q < Qa) ? G[(titem * a.Et + padded_pos<D>(k, rt, a.Rt)) * a.nrhs + q0 + q]
                                          : make_float2(0.f, 0.f);
      split_bf16(v, &gh[q * kBLd + kk], &gl[q * kBLd + kk]);
    }
    __syncthreads();
    const int kend = min(kBK, RT - kc);
    for (int ks = 0; ks < kend; ks += 16) {
      const int kl = ks + 4 * (lane >> 4);
      // rows kc + kl .. + 3: inside the padded column (RTp is a multiple of
      // 4); past it the staged G is zero, so any finite row does
      const int kr = min(kc + kl, RTp - 4);
      uint4 bh[2], bl[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int q = c * 16 + (lane & 15);
        bh[c] = ghi[(q * kBLd + kl) / 4];
        bl[c] = glo[(q * kBLd + kl) / 4];
      }
#pragma unroll
      for (int i = 0; i < kMT; ++i) {
        if (!live[i]) continue;
        const uint4 cw = *reinterpret_cast<const uint4*>(cb + (long long)colc[i] * RTp + kr);
        const v8bf ar = as_v8bf(cw);
        const v8bf ai = as_v8bf(make_uint4(swap16(cw.x) ^ 0x8000u, swap16(cw.y) ^ 0x8000u,
                                           swap16(cw.z) ^ 0x8000u, swap16(cw.w) ^ 0x8000u));
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          accr[i][c] = mfma_bf16(ar, as_v8bf(bh[c]), accr[i][c]);
          accr[i][c] = mfma_bf16(ar, as_v8bf(bl[c]), accr[i][c]);
          acci[i][c] = mfma_bf16(ai, as_v8bf(bh[c]), acci[i][c]);
          acci[i][c] = mfma_bf16(ai, as_v8bf(bl[c]), acci[i][c]);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kMT; ++i) {
    if (!live[i]) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = c0 + (w + 4 * i) * 16 + 4 * (lane >> 4) + j;
        const int q = c * 16 + (lane & 15);
        if (col < RS && q < Qa)
          F[(sitem * a.Es + padded_pos<D>(col, rs, a.Rs)) * a.nrhs + q0 + q] =
              make_float2(accr[i][c][j], acci[i][c][j]);
      }
  }
}

// BF16 cores on the matrix cores, second form: one workgroup owns 64 MTW
// output rows (adjoint: columns) of one pair and NQ = 16 NQT right-hand sides
// (every wave keeps MTW x NQT complex 16 x 16 tiles).  Each wave
// owns 16 MTW consecutive rows, so a 16-row tile reads whole cache lines of
// a core column.  The padded positions of the contracted index and of the
// workgroup's output rows are tabulated in LDS once, the right-hand sides of
// the next staged chunk (64 deep, 32 for 128 right-hand sides) are loaded
// into registers while the current chunk is multiplied, and the core
// fragments of the next 32 contracted indices are loaded before the
// products of the current 32.  Same products, in the same order per
// accumulator, as above: hi and lo parts of the FP32 right-hand sides
// against the BF16 core words.
template <int MTW_, int NQT>
struct Bf16Tile {
  static constexpr int MTW = MTW_;           // 16-row tiles per wave
  static constexpr int kRows = 64 * MTW;     // output rows per workgroup
  static constexpr int NQ = 16 * NQT;        // right-hand sides per workgroup
  static constexpr int kSub = 256 / kRows;   // workgroups per 256-row unit
  static constexpr int KC = NQT == 8 ? 32 : 64;        // contracted depth per staged chunk
  static constexpr int kLd4 = (KC + 4) / 4;            // LDS row stride in uint4 (conflict-free)
  static constexpr int kTasks = NQ * (KC / 4) / kThreads;  // (q, 4 k) staging tasks per thread
};

template <int D, bool ADJ, int MTW_, int NQT>
__global__ void __launch_bounds__(kThreads)
    core_mfma_bf16_v2(CoreArgs a, const unsigned* __restrict__ cores, const long long* __restrict__ core_off,
                      const int* __restrict__ meta, const int2* __restrict__ units,
                      const float2* __restrict__ in, float2* __restrict__ out) {
  using TL = Bf16Tile<MTW_, NQT>;
  constexpr int MTW = TL::MTW, NQ = TL::NQ, kRows = TL::kRows, KC = TL::KC, kLd4 = TL::kLd4;
  __shared__ uint4 bhi[NQ * kLd4], blo[NQ * kLd4];
  __shared__ int mpos[kRows];
  extern __shared__ int kpos[];  // padded position of every contracted index
  // flattened (unit, sub-panel, RHS tile), the tile fastest; the tiles that
  // share a core panel run back to back on one XCD
  const int nqt = (a.nrhs + NQ - 1) / NQ;
  const int item = xcd_item(blockIdx.x, gridDim.x, nqt);
  const int qt = item % nqt, sub = (item / nqt) % TL::kSub;
  const int2 u = units[item / (nqt * TL::kSub)];
  const int pair = u.x;
  const int m0 = u.y + sub * kRows;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  const int M = ADJ ? RS : RT, K = ADJ ? RT : RS;
  if (m0 >= M) return;  // the whole workgroup lies past the pair
  int mr[D], kr[D], MR[D], KR[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    mr[k] = ADJ ? m[kMetaRs + k] : m[3 + k];
    kr[k] = ADJ ? m[3 + k] : m[kMetaRs + k];
    MR[k] = ADJ ? a.Rs[k] : a.Rt[k];
    KR[k] = ADJ ? a.Rt[k] : a.Rs[k];
  }
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const long long inb = ADJ ? titem * a.Et : sitem * a.Es;
  const long long outb = ADJ ? sitem * a.Es : titem * a.Et;
  const int q0 = qt * NQ;
  const int Qa = min(NQ, a.nrhs - q0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned* cb = cores + core_off[pair];
  for (int i = threadIdx.x; i < K; i += kThreads) kpos[i] = (int)padded_pos<D>(i, kr, KR);
  for (int i = threadIdx.x; i < kRows; i += kThreads)
    mpos[i] = m0 + i < M ? (int)padded_pos<D>(m0 + i, mr, MR) : 0;
  v4f accr[MTW][NQT], acci[MTW][NQT];
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int c = 0; c < NQT; ++c) {
      accr[i][c] = v4f{0, 0, 0, 0};
      acci[i][c] = v4f{0, 0, 0, 0};
    }
  const int wrow = m0 + w * 16 * MTW;  // first row of this wave
  int mcl[MTW];                        // this lane's (clamped) row or column
  bool live[MTW];
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    live[i] = wrow + 16 * i < M;
    mcl[i] = ADJ ? min(wrow + 16 * i + (lane & 15), RS - 1) : min(wrow + 16 * i + (lane & 15), RTp - 1);
  }
  // core words of this lane for the 4 contracted indices k .. k + 3 of tile i
  auto load_a = [&](uint4 (&aw)[MTW], int k) {
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
      if (!live[i]) continue;
      if constexpr (ADJ) {
        // rows k .. k + 3 lie inside the padded column (RTp is a multiple
        // of 4); past it the staged right-hand side is zero, so any
        // in-bounds row does
        aw[i] = *reinterpret_cast<const uint4*>(cb + (long long)mcl[i] * RTp + min(k, RTp - 4));
      } else {
        aw[i].x = cb[(long long)min(k, K - 1) * RTp + mcl[i]];
        aw[i].y = cb[(long long)min(k + 1, K - 1) * RTp + mcl[i]];
        aw[i].z = cb[(long long)min(k + 2, K - 1) * RTp + mcl[i]];
        aw[i].w = cb[(long long)min(k + 3, K - 1) * RTp + mcl[i]];
      }
    }
  };
  // staging: task j of this thread is right-hand side q = idx % NQ and the
  // contracted indices 4 (idx / NQ) .. + 3 of the chunk (q fastest: each
  // read of a k row is contiguous over q)
  float2 fv[TL::kTasks][4];
  __syncthreads();  // kpos, mpos
  auto fetch_b = [&](int kc) {
#pragma unroll
    for (int j = 0; j < TL::kTasks; ++j) {
      const int idx = threadIdx.x + j * kThreads;
      const int q = idx % NQ, k4 = idx / NQ;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = kc + 4 * k4 + e;
        fv[j][e] = (k < K && q < Qa) ? in[(inb + kpos[k]) * a.nrhs + q0 + q] : make_float2(0.f, 0.f);
      }
    }
  };
  auto store_b = [&]() {
#pragma unroll
    for (int j = 0; j < TL::kTasks; ++j) {
      const int idx = threadIdx.x + j * kThreads;
      const int q = idx % NQ, k4 = idx / NQ;
      uint4 h, l;
      split_bf16(fv[j][0], &h.x, &l.x);
      split_bf16(fv[j][1], &h.y, &l.y);
      split_bf16(fv[j][2], &h.z, &l.z);
      split_bf16(fv[j][3], &h.w, &l.w);
      bhi[q * kLd4 + k4] = h;
      blo[q * kLd4 + k4] = l;
    }
  };
  // the core fragments run two 16-deep steps (one 32-deep step) ahead of
  // the products, across chunk boundaries; the right-hand sides one chunk
  const int kq = 4 * (lane >> 4);  // this lane's first k of a 16-deep step
  uint4 acur[2][MTW], anxt[2][MTW];
  load_a(acur[0], kq);
  load_a(acur[1], 16 + kq);
  fetch_b(0);
  for (int kc = 0; kc < K; kc += KC) {
    __syncthreads();  // the previous chunk's fragments are read
    store_b();
    __syncthreads();
    if (kc + KC < K) fetch_b(kc + KC);
    const int kend = min(KC, K - kc);
    for (int ks = 0; ks < kend; ks += 32) {
      if (kc + ks + 32 < K) {
        load_a(anxt[0], kc + ks + 32 + kq);
        load_a(anxt[1], kc + ks + 48 + kq);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint4 bh[NQT], bl[NQT];
#pragma unroll
        for (int c = 0; c < NQT; ++c) {
          const int q = c * 16 + (lane & 15);
          bh[c] = bhi[q * kLd4 + (ks + 16 * h + kq) / 4];
          bl[c] = blo[q * kLd4 + (ks + 16 * h + kq) / 4];
        }
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
          if (!live[i]) continue;
          const uint4 cw = acur[h][i];
          v8bf ar, ai;
          if constexpr (ADJ) {
            ar = as_v8bf(cw);
            ai = as_v8bf(make_uint4(swap16(cw.x) ^ 0x8000u, swap16(cw.y) ^ 0x8000u, swap16(cw.z) ^ 0x8000u,
                                    swap16(cw.w) ^ 0x8000u));
          } else {
            ar = as_v8bf(make_uint4(cw.x ^ 0x80000000u, cw.y ^ 0x80000000u, cw.z ^ 0x80000000u,
                                    cw.w ^ 0x80000000u));
            ai = as_v8bf(make_uint4(swap16(cw.x), swap16(cw.y), swap16(cw.z), swap16(cw.w)));
          }
#pragma unroll
          for (int c = 0; c < NQT; ++c) {
            accr[i][c] = mfma_bf16(ar, as_v8bf(bh[c]), accr[i][c]);
            acci[i][c] = mfma_bf16(ai, as_v8bf(bh[c]), acci[i][c]);
          }
#pragma unroll
          for (int c = 0; c < NQT; ++c) {
            accr[i][c] = mfma_bf16(ar, as_v8bf(bl[c]), accr[i][c]);
            acci[i][c] = mfma_bf16(ai, as_v8bf(bl[c]), acci[i][c]);
          }
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < MTW; ++i) acur[h][i] = anxt[h][i];
    }
  }
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    if (!live[i]) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rl = w * 16 * MTW + 16 * i + 4 * (lane >> 4) + j;  // row within the workgroup
      if (m0 + rl >= M) continue;
      float2* dst = out + (outb + mpos[rl]) * a.nrhs + q0;
#pragma unroll
      for (int c = 0; c < NQT; ++c) {
        const int q = c * 16 + (lane & 15);
        if (q < Qa) dst[q] = make_float2(accr[i][c][j], acci[i][c][j]);
      }
    }
  }
}

// ----------------------------------------------- MFMA transfer stages --
// A mode product of a transfer block, out[a][col] = sum_j M[a][j] in[j][col]
// (complex; a < nA new-mode entries, j < K contracted entries, col over the
// other modes and the right-hand sides), as one real product on
// v_mfma_f32_16x16x4f32: with the real index k = 2 j + p (p = 0 real part,
// 1 imaginary part) the A fragment holds
//   rows 0..7  (real parts of outputs a):      Mr[a][j] (p = 0), -Mi[a][j] (p = 1)
//   rows 8..15 (imaginary parts of the same a): Mi[a][j] (p = 0),  Mr[a][j] (p = 1)
// and the B fragment the parts p of in[j][col] (b(j, col, p) returns it).  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register i of lane l
// is D[4 (l / 16) + i][l % 16].  A row tile covers 8 outputs, a column tile
// 16 columns; kXT column tiles share each A fragment.
constexpr int kXT = 4;       // column tiles per pass
constexpr int kXItems = 4;   // persistent (row tile, column group) items per wave

// B element (j, col, part p) = src[colofs(col) + jofs(j) + p] (float
// offsets; colofs < 0 marks a zero column, e.g. a right-hand side past the
// end): the column part is computed once per tile, the j part once per step.
template <class MF, class T, class CF, class JF>
__device__ __forceinline__ void xmfma(v4f (&acc)[kXT], int rt, int ct0, int K, int nA, int ncols, MF m,
                                      const T* __restrict__ src, CF colofs, JF jofs) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4, p = kk & 1;
  const int a = rt * 8 + (r & 7);
  const bool im_row = r >= 8;
  long long co[kXT];
#pragma unroll
  for (int t = 0; t < kXT; ++t) {
    const int col = (ct0 + t) * 16 + r;
    co[t] = col < ncols ? colofs(col) : -1;
  }
  const int nks = (K + 1) >> 1;
  for (int ks = 0; ks < nks; ++ks) {
    const int j = 2 * ks + (kk >> 1);
    const bool jv = j < K;
    float av = 0.f;
    long long jo = 0;
    if (jv) {
      jo = jofs(j) + p;
      if (a < nA) {
        const float2 mv = m(a, j);
        av = im_row ? (p ? mv.x : mv.y) : (p ? -mv.y : mv.x);
      }
    }
#pragma unroll
    for (int t = 0; t < kXT; ++t) {
      const float bv = (jv && co[t] >= 0) ? src[co[t] + jo] : 0.f;
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
    }
  }
}

// w(a, col, part, value) for every valid output of the tiles in acc
template <class WF>
__device__ __forceinline__ void xstore(const v4f (&acc)[kXT], int rt, int ct0, int nA, int ncols, WF w) {
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4, c = lane & 15;
#pragma unroll
  for (int t = 0; t < kXT; ++t) {
    const int col = (ct0 + t) * 16 + c;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * kk + i;
      const int a = rt * 8 + (row & 7);
      if (a < nA) w(a, col, row >> 3, acc[t][i]);
    }
  }
}

__device__ __forceinline__ void xzero(v4f (&acc)[kXT]) {
#pragma unroll
  for (int t = 0; t < kXT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
}

// all (row tile, column group) items of a product, spread over the waves
template <class MF, class T, class CF, class JF, class WF>
__device__ __forceinline__ void xproduct(int K, int nA, int ncols, MF m, const T* src, CF colofs, JF jofs,
                                         WF w) {
  const int wave = threadIdx.x >> 6;
  const int nrt = (nA + 7) >> 3;
  const int ngrp = ((ncols + 15) / 16 + kXT - 1) / kXT;
  for (int it = wave; it < nrt * ngrp; it += kThreads / 64) {
    const int rt = it % nrt, ct0 = (it / nrt) * kXT;
    v4f acc[kXT];
    xzero(acc);
    xmfma(acc, rt, ct0, K, nA, ncols, m, src, colofs, jofs);
    xstore(acc, rt, ct0, nA, ncols, w);
  }
}

// Fan-out (transfer levels: the coarse side is a workspace tensor with the
// right-hand side innermost) on the matrix cores, one block per workgroup.
// Columns of each product: the not-yet-contracted modes, then q fastest.
template <int D, int QT>
__global__ void __launch_bounds__(kThreads)
    stage_fanout_mfma(StageArgs a, const float2* __restrict__ coarse, float2* __restrict__ fine,
                      const float2* __restrict__ mats) {
  extern __shared__ unsigned char smem_raw[];
  float2* sm = reinterpret_cast<float2*>(smem_raw);
  const StageBid sb = stage_bid(a, QT);
  const int fi = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  int r[D];
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
  const int citem = parent_of<D>(fi, a.lvl);
  Seg sg[D];
  coarse_segs<D>(a, citem, beta, sg);
  const int q0 = sb.q0;
  const int Qa = min(QT, a.nrhs - q0);
  CoarseAddr<D> ca;
  ca.init(a, citem, beta, q0);
  long long fs[D];
  const long long fb = fine_base<D>(a, fi, beta, q0, fs);
  const float2* mbase = mats + (long long)fi * a.mat_item_stride;
  float2* mk[D];
  int off = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    mk[k] = sm + off;
    const float2* src = mbase + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
    const int ck = sg[k].c;
    for (int i = threadIdx.x; i < r[k] * ck; i += kThreads) {
      const int row = i / ck, j = i % ck;
      float2 v = src[row * a.A[k] + sg[k].pos(j)];
      if (a.conj) v.y = -v.y;
      mk[k][i] = v;
    }
    off += a.R[k] * a.A[k];
  }
  float* y1 = reinterpret_cast<float*>(sm + off);
  const int c0 = sg[0].c, c1 = sg[1].c;
  __syncthreads();
  const float* cf = reinterpret_cast<const float*>(coarse);
  if constexpr (D == 2) {
    // y1[a0][col], col = j1 QT + q
    xproduct(
        c0, r[0], c1 * QT, [&](int a0, int j) { return mk[0][a0 * c0 + j]; }, cf,
        [&](int col) -> long long {
          const int q = col % QT, j1 = col / QT;
          if (q >= Qa) return -1;
          return 2 * (ca.base + sg[1].pos(j1) * ca.stride[1] + q);
        },
        [&](int j) -> long long { return 2 * (sg[0].pos(j) * ca.stride[0]); },
        [&](int a0, int col, int part, float v) { y1[2 * (a0 * (c1 * QT) + col) + part] = v; });
    __syncthreads();
    // fine[a0][a1][q], col = a0 QT + q
    const int n1 = c1 * QT;
    xproduct(
        c1, r[1], r[0] * QT, [&](int a1, int j) { return mk[1][a1 * c1 + j]; }, (const float*)y1,
        [&](int col) -> long long {
          const int q = col % QT, a0 = col / QT;
          return 2 * (a0 * n1 + q);
        },
        [&](int j) -> long long { return 2 * (j * QT); },
        [&](int a1, int col, int part, float v) {
          const int q = col % QT, a0 = col / QT;
          if (q < Qa) reinterpret_cast<float*>(fine + fb + a0 * fs[0] + a1 * fs[1] + q)[part] = v;
        });
  } else {
    const int c2 = sg[2].c;
    const int n1 = c1 * c2 * QT;
    float* y2 = y1 + 2 * a.R[0] * a.A[1] * a.A[2] * QT;
    // y1[a0][col], col = (j1 c2 + j2) QT + q
    xproduct(
        c0, r[0], n1, [&](int a0, int j) { return mk[0][a0 * c0 + j]; }, cf,
        [&](int col) -> long long {
          const int q = col % QT, t = col / QT;
          if (q >= Qa) return -1;
          const int j2 = t % c2, j1 = t / c2;
          return 2 * (ca.base + sg[1].pos(j1) * ca.stride[1] + sg[2].pos(j2) * ca.stride[2] + q);
        },
        [&](int j) -> long long { return 2 * (sg[0].pos(j) * ca.stride[0]); },
        [&](int a0, int col, int part, float v) { y1[2 * (a0 * n1 + col) + part] = v; });
    __syncthreads();
    // y2[a0][a1][j2][q] from columns (a0 c2 + j2) QT + q
    xproduct(
        c1, r[1], r[0] * c2 * QT, [&](int a1, int j) { return mk[1][a1 * c1 + j]; }, (const float*)y1,
        [&](int col) -> long long {
          const int q = col % QT, t = col / QT;
          const int j2 = t % c2, a0 = t / c2;
          return 2 * (a0 * n1 + j2 * QT + q);
        },
        [&](int j) -> long long { return 2 * (j * c2 * QT); },
        [&](int a1, int col, int part, float v) {
          const int q = col % QT, t = col / QT;
          const int j2 = t % c2, a0 = t / c2;
          y2[2 * (((a0 * r[1] + a1) * c2 + j2) * QT + q) + part] = v;
        });
    __syncthreads();
    // fine[a0][a1][a2][q] from columns (a0 r1 + a1) QT + q
    xproduct(
        c2, r[2], r[0] * r[1] * QT, [&](int a2, int j) { return mk[2][a2 * c2 + j]; }, (const float*)y2,
        [&](int col) -> long long {
          const int q = col % QT, t = col / QT;
          return 2 * (t * c2 * QT + q);
        },
        [&](int j) -> long long { return 2 * (j * QT); },
        [&](int a2, int col, int part, float v) {
          const int q = col % QT, t = col / QT;
          const int a1 = t % r[1], a0 = t / r[1];
          if (q < Qa)
            reinterpret_cast<float*>(fine + fb + a0 * fs[0] + a1 * fs[1] + a2 * fs[2] + q)[part] = v;
        });
  }
}

// Fan-in (transfer levels) on the matrix cores with the children in turn:
// per child the modes D-1 .. 1 go through LDS, and the first mode's product
// accumulates in MFMA registers held across the children; one coarse block
// per workgroup.
template <int D, int QT>
__global__ void __launch_bounds__(kThreads)
    stage_fanin_mfma(StageArgs a, const float2* __restrict__ fine, float2* __restrict__ coarse,
                     const float2* __restrict__ mats) {
  extern __shared__ unsigned char smem_raw[];
  float2* sm = reinterpret_cast<float2*>(smem_raw);
  const StageBid sb = stage_bid(a, QT);
  const int ci = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  Seg sg[D];
  coarse_segs<D>(a, ci, beta, sg);
  const int q0 = sb.q0;
  const int Qa = min(QT, a.nrhs - q0);
  constexpr int nchild = 1 << D;
  __shared__ int cfi[kMaxChildren], crk[kMaxChildren][kMaxD];
  __shared__ long long cfb[kMaxChildren];
  if (threadIdx.x < nchild) {
    const int c = threadIdx.x;
    const int fi = child_of<D>(ci, a.lvl, c);
    cfi[c] = fi;
#pragma unroll
    for (int k = 0; k < D; ++k) crk[c][k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
    long long fs_[D];
    cfb[c] = fine_base<D>(a, fi, beta, q0, fs_);
  }
  long long fs[D];
  (void)fine_base<D>(a, 0, beta, 0, fs);
  __syncthreads();
  // every child's matrices, compact: M_k [j][a_k] (r_k x c_k)
  int msz = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) msz += a.R[k] * a.A[k];
  for (int c = 0; c < nchild; ++c) {
    const float2* mbase = mats + (long long)cfi[c] * a.mat_item_stride;
    int off = c * msz;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const float2* src = mbase + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
      const int ck = sg[k].c, rk = crk[c][k];
      for (int i = threadIdx.x; i < rk * ck; i += kThreads) {
        const int row = i / ck, j = i % ck;
        float2 v = src[row * a.A[k] + sg[k].pos(j)];
        if (a.conj) v.y = -v.y;
        sm[off + i] = v;
      }
      off += a.R[k] * a.A[k];
    }
  }
  float* t1 = reinterpret_cast<float*>(sm + nchild * msz);
  float* t2 = t1 + 2 * a.R[0] * a.R[1] * a.A[D - 1] * QT;
  const int c0 = sg[0].c, c1 = sg[1].c;
  const int c2 = D == 3 ? sg[D - 1].c : 1;
  // output columns: (a1 [, a2]) then q fastest
  const int ncols = c1 * c2 * QT;
  const int wave = threadIdx.x >> 6;
  const int nrt = (c0 + 7) >> 3;
  const int ngrp = ((ncols + 15) / 16 + kXT - 1) / kXT;
  const int nitems = nrt * ngrp;
  v4f acc[kXItems][kXT];
#pragma unroll
  for (int i = 0; i < kXItems; ++i) xzero(acc[i]);
  __syncthreads();
  for (int c = 0; c < nchild; ++c) {
    const int r0 = crk[c][0], r1 = crk[c][1];
    const float2* M0c = sm + c * msz;
    const float2* M1c = M0c + a.R[0] * a.A[0];
    const float2* fc = fine + cfb[c];
    const float* fcf = reinterpret_cast<const float*>(fc);
    const float* xin;
    if constexpr (D == 2) {
      // t1[j0][a1][q] from columns j0 QT + q
      xproduct(
          r1, c1, r0 * QT, [&](int a1, int j) { return M1c[j * c1 + a1]; }, fcf,
          [&](int col) -> long long {
            const int q = col % QT, j0 = col / QT;
            if (q >= Qa) return -1;
            return 2 * (j0 * fs[0] + q);
          },
          [&](int j) -> long long { return 2 * (j * fs[1]); },
          [&](int a1, int col, int part, float v) {
            const int q = col % QT, j0 = col / QT;
            t1[2 * ((j0 * c1 + a1) * QT + q) + part] = v;
          });
      xin = t1;
    } else {
      const int r2 = crk[c][2];
      const float2* M2c = M1c + a.R[1] * a.A[1];
      // t1[j0][j1][a2][q] from columns (j0 r1 + j1) QT + q
      xproduct(
          r2, c2, r0 * r1 * QT, [&](int a2, int j) { return M2c[j * c2 + a2]; }, fcf,
          [&](int col) -> long long {
            const int q = col % QT, t = col / QT;
            if (q >= Qa) return -1;
            const int j1 = t % r1, j0 = t / r1;
            return 2 * (j0 * fs[0] + j1 * fs[1] + q);
          },
          [&](int j) -> long long { return 2 * (j * fs[2]); },
          [&](int a2, int col, int part, float v) {
            const int q = col % QT, t = col / QT;
            t1[2 * ((t * c2 + a2) * QT + q) + part] = v;
          });
      __syncthreads();
      // t2[j0][a1][a2][q] from columns (j0 c2 + a2) QT + q
      xproduct(
          r1, c1, r0 * c2 * QT, [&](int a1, int j) { return M1c[j * c1 + a1]; }, (const float*)t1,
          [&](int col) -> long long {
            const int q = col % QT, t = col / QT;
            const int a2 = t % c2, j0 = t / c2;
            return 2 * ((j0 * r1 * c2 + a2) * QT + q);
          },
          [&](int j) -> long long { return 2 * (j * c2 * QT); },
          [&](int a1, int col, int part, float v) {
            const int q = col % QT, t = col / QT;
            const int a2 = t % c2, j0 = t / c2;
            t2[2 * (((j0 * c1 + a1) * c2 + a2) * QT + q) + part] = v;
          });
      xin = t2;
    }
    __syncthreads();
    // acc += M0c^T xin: out a0 over columns (a1 [, a2]) QT + q
#pragma unroll
    for (int i = 0; i < kXItems; ++i) {
      const int it = wave + i * (kThreads / 64);
      if (it < nitems)
        xmfma(acc[i], it % nrt, (it / nrt) * kXT, r0, c0, ncols,
              [&](int a0, int j) { return M0c[j * c0 + a0]; }, xin,
              [&](int col) -> long long { return 2 * col; },
              [&](int j) -> long long { return 2 * (j * ncols); });
    }
    __syncthreads();
  }
  CoarseAddr<D> ca;
  ca.init(a, ci, beta, q0);
#pragma unroll
  for (int i = 0; i < kXItems; ++i) {
    const int it = wave + i * (kThreads / 64);
    if (it < nitems)
      xstore(acc[i], it % nrt, (it / nrt) * kXT, c0, ncols, [&](int a0, int col, int part, float v) {
        const int q = col % QT, t = col / QT;
        if (q >= Qa) return;
        long long o = ca.base + sg[0].pos(a0) * ca.stride[0] + q;
        if (D == 3) o += sg[1].pos(t / c2) * ca.stride[1] + sg[D - 1].pos(t % c2) * ca.stride[D - 1];
        else o += sg[1].pos(t) * ca.stride[1];
        reinterpret_cast<float*>(coarse + o)[part] = v;
      });
  }
}

// ------------------------------------------------------------------ host --
constexpr int kTargetWorkgroups = 2048;  // enough to cover 256 CUs several times

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

static tb_status ensure_workspace(Plan& p, size_t bytes) {
  if (p.ws.bytes >= bytes) return TB_OK;
  if (p.ws.base) {
    drop_graphs_for(&p);  // cached graphs hold the old workspace address
    TB_HIP_TRY(hipDeviceSynchronize());
    TB_HIP_TRY(hipFree(p.ws.base));
    p.device_bytes -= p.ws.bytes;
    p.ws.base = nullptr;
    p.ws.bytes = 0;
  }
  if (p.max_device_bytes && p.device_bytes + bytes > p.max_device_bytes)
    return fail(TB_ERR_OOM, "apply workspace exceeds the plan's device memory cap");
  hipError_t e = hipMalloc(&p.ws.base, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p.ws.base = nullptr;
    return fail(TB_ERR_OOM, std::string("apply workspace: ") + hipGetErrorString(e));
  }
  p.ws.bytes = bytes;
  p.device_bytes += bytes;
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
  a.rank_f = fine.rank_d;
  a.rank_c = coarse ? coarse->rank_d : nullptr;
  a.nb_c = coarse ? coarse->nb : 1;
  for (int k = 0; k < d; ++k) a.Rc[k] = coarse ? coarse->R[k] : 0;
  a.outer_level = source ? p.Ls : p.Lt;
  a.outer_block = (int)(p.n >> a.outer_level);
  a.nrhs = nrhs;
  a.conj = conj ? 1 : 0;
  // longest contracted extents: a fan-out contracts the coarse block's true
  // extents (two sibling skeletons, or the dense leaf boxes), a fan-in the
  // fine ranks
  a.fib_in = 0;
  for (int k = 0; k < d; ++k) a.fib_in = std::max(a.fib_in, fine.R[k]);
  if (coarse) {
    if (coarse->pair_max < 0) {
      int m = 0;
      for (int it = 0; it < coarse->nitems; ++it)
        for (int k = 0; k < d; ++k)
          for (int b = 0; b + 1 < coarse->nb; b += 2)
            m = std::max(m, coarse->id(it, k, b, d).r + coarse->id(it, k, b + 1, d).r);
      coarse->pair_max = m;
    }
    a.fib_out = coarse->pair_max;
  } else {
    a.fib_out = 0;
    for (int k = 0; k < d; ++k) a.fib_out = std::max(a.fib_out, fine.A[k]);
  }
  return a;
}

template <class T, int D, int QT, int G, int V>
static tb_status launch_fanout(StageArgs a, dim3 grid, size_t lds, const void* in, void* out,
                               const void* mats, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  TB_TRY(set_lds(stage_fanout<T, D, QT, G, V>, lds));
  stage_fanout<T, D, QT, G, V><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
  return TB_OK;
}

template <class T, int D, int QT, int G, int V>
static tb_status launch_fanin(StageArgs a, bool sm, dim3 grid, size_t lds, const void* in, void* out,
                              const void* mats, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  if (sm) {
    TB_TRY(set_lds(stage_fanin<T, D, QT, true, G, V>, lds));
    stage_fanin<T, D, QT, true, G, V><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out,
                                                                      (const C*)mats);
  } else {
    TB_TRY(set_lds(stage_fanin<T, D, QT, false, G, V>, lds));
    stage_fanin<T, D, QT, false, G, V><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out,
                                                                       (const C*)mats);
  }
  return TB_OK;
}

// LDS elements of one workgroup for a slice of `chunk` entries of the first
// mode and QT right-hand sides (padded extents bound the true ones).
static long long stage_lds_elems(const StageArgs& a, int d, bool fanout, int chunk, int QT,
                                 bool sm = true) {
  long long msz = 0;
  for (int k = 1; k < d; ++k) msz += (long long)a.R[k] * a.A[k];
  if (fanout) {
    long long e = msz + (long long)chunk * a.A[0];
    if (d == 2) e += (long long)chunk * a.A[1] * QT;
    else e += (long long)chunk * a.A[1] * a.A[2] * QT + (long long)chunk * a.R[1] * a.A[2] * QT;
    return e;
  }
  const long long nchild = a.coarse_global ? 1 : (1LL << d);
  long long e = sm ? nchild * (msz + (long long)chunk * a.R[0]) : 0;
  if (d == 2) e += nchild * chunk * a.R[1] * QT;
  else e += nchild * chunk * a.R[1] * a.R[2] * QT + nchild * chunk * a.A[1] * a.R[2] * QT;
  return e;
}

// LDS elements and feasibility of stage_fanin_seq for a slice of `chunk`
// rows and QT right-hand sides (padded extents bound the true ones).
static long long seq_lds_elems(const StageArgs& a, int d, int chunk, int QT) {
  const long long nchild = a.coarse_global ? 1 : (1LL << d);
  long long msz = (long long)a.R[0] * chunk;
  for (int k = 1; k < d; ++k) msz += (long long)a.R[k] * a.A[k];
  long long e = nchild * msz;
  if (d == 2) e += (long long)a.R[0] * a.A[1] * QT;
  else e += (long long)a.R[0] * a.R[1] * a.A[2] * QT + (long long)a.R[0] * a.A[1] * a.A[2] * QT;
  return e;
}

template <class T, int D>
static tb_status launch_fanin_seq(StageArgs a, int QT, dim3 grid, size_t lds, const void* in, void* out,
                                  const void* mats, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  switch (QT) {
#define TB_SEQ_CASE(Q)                                                                            \
  case Q:                                                                                         \
    TB_TRY(set_lds(stage_fanin_seq<T, D, Q>, lds));                                               \
    stage_fanin_seq<T, D, Q><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats); \
    return TB_OK;
    TB_SEQ_CASE(1)
    TB_SEQ_CASE(2)
    TB_SEQ_CASE(4)
    TB_SEQ_CASE(8)
#undef TB_SEQ_CASE
  }
  return fail(TB_ERR_INVALID_ARG, "bad RHS tile");
}

template <class T>
static tb_status launch_stage_seq(const Plan& p, StageArgs a, int n_items, const void* in, void* out,
                                  const void* mats, hipStream_t stream, const LaunchCfg& cfg) {
  using C = typename CplxOf<T>::type;
  const int d = p.d;
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  const long long budget = std::min<long long>(limit, 80 * 1024);
  const long long fib1 = d == 2 ? a.A[1] : (long long)a.A[1] * a.A[2];
  const int chunk = std::min(a.A[0], kSeqRows);
  const int qcap = cfg.QT > 0 ? cfg.QT : 8;
  int QT = 1;
  while (QT * 2 <= qcap && QT * 2 <= a.nrhs) QT *= 2;
  while (QT > 1 && (seq_lds_elems(a, d, chunk, QT) * (long long)sizeof(C) > budget ||
                    fib1 * QT > (long long)SeqFib<T>::value * kThreads))
    QT /= 2;
  if (cfg.QT > 0 && QT != cfg.QT) return fail(TB_ERR_UNSUPPORTED, "RHS tile does not fit this stage");
  if (fib1 * QT > (long long)SeqFib<T>::value * kThreads)
    return fail(TB_ERR_UNSUPPORTED, "coarse block too wide for the in-turn fan-in");
  const size_t lds = (size_t)seq_lds_elems(a, d, chunk, QT) * sizeof(C);
  if (lds > (size_t)limit) return fail(TB_ERR_UNSUPPORTED, "in-turn fan-in exceeds the LDS limit");
  const long long blocks = (long long)n_items * a.nblk;
  a.chunk = chunk;
  a.nsplit = (a.A[0] + chunk - 1) / chunk;
  const long long nwg = blocks * a.nsplit * ((a.nrhs + QT - 1) / QT);
  if (nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many right-hand sides for one launch");
  dim3 grid((unsigned)nwg);
  const tb_status st = d == 2 ? launch_fanin_seq<T, 2>(a, QT, grid, lds, in, out, mats, stream)
                              : launch_fanin_seq<T, 3>(a, QT, grid, lds, in, out, mats, stream);
  TB_TRY(st);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

// LDS elements of the matrix-core transfer kernels (one block, QT
// right-hand sides; padded extents bound the true ones) and the number of
// persistent accumulator items of the fan-in.
static long long xmfma_lds_elems(const StageArgs& a, int d, bool fanout, int QT) {
  long long msz = 0;
  for (int k = 0; k < d; ++k) msz += (long long)a.R[k] * a.A[k];
  if (fanout) {
    if (d == 2) return msz + (long long)a.R[0] * a.A[1] * QT;
    return msz + (long long)a.R[0] * a.A[1] * a.A[2] * QT + (long long)a.R[0] * a.R[1] * a.A[2] * QT;
  }
  const long long nchild = 1LL << d;
  if (d == 2) return nchild * msz + (long long)a.R[0] * a.A[1] * QT;
  return nchild * msz + (long long)a.R[0] * a.R[1] * a.A[2] * QT + (long long)a.R[0] * a.A[1] * a.A[2] * QT;
}

static long long xmfma_items(const StageArgs& a, int d, int QT) {
  const long long ncols = (d == 2 ? a.A[1] : (long long)a.A[1] * a.A[2]) * QT;
  const long long nrt = (a.A[0] + 7) / 8;
  const long long ngrp = ((ncols + 15) / 16 + kXT - 1) / kXT;
  return nrt * ngrp;
}

template <int D, int QT>
static tb_status launch_xmfma_q(StageArgs a, bool fanout, dim3 grid, size_t lds, const void* in, void* out,
                                const void* mats, hipStream_t stream) {
  if (fanout) {
    TB_TRY(set_lds(stage_fanout_mfma<D, QT>, lds));
    stage_fanout_mfma<D, QT><<<grid, kThreads, lds, stream>>>(a, (const float2*)in, (float2*)out,
                                                              (const float2*)mats);
  } else {
    TB_TRY(set_lds(stage_fanin_mfma<D, QT>, lds));
    stage_fanin_mfma<D, QT><<<grid, kThreads, lds, stream>>>(a, (const float2*)in, (float2*)out,
                                                             (const float2*)mats);
  }
  return TB_OK;
}

template <int D>
static tb_status launch_xmfma_d(StageArgs a, bool fanout, int QT, dim3 grid, size_t lds, const void* in,
                                void* out, const void* mats, hipStream_t stream) {
  switch (QT) {
    case 1: return launch_xmfma_q<D, 1>(a, fanout, grid, lds, in, out, mats, stream);
    case 2: return launch_xmfma_q<D, 2>(a, fanout, grid, lds, in, out, mats, stream);
    case 4: return launch_xmfma_q<D, 4>(a, fanout, grid, lds, in, out, mats, stream);
    default: return launch_xmfma_q<D, 8>(a, fanout, grid, lds, in, out, mats, stream);
  }
}

template <class T>
static tb_status launch_stage_xmfma(const Plan& p, StageArgs a, bool fanout, int n_items, const void* in,
                                    void* out, const void* mats, hipStream_t stream, const LaunchCfg& cfg) {
  if (sizeof(T) != 4) return fail(TB_ERR_UNSUPPORTED, "matrix-core transfers are FP32 only");
  if (a.coarse_global) return fail(TB_ERR_UNSUPPORTED, "matrix-core transfers cover transfer levels only");
  const int d = p.d;
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  const long long budget = std::min<long long>(limit, 80 * 1024);
  const int qcap = cfg.QT > 0 ? cfg.QT : 8;
  int QT = 1;
  while (QT * 2 <= qcap && QT * 2 <= a.nrhs) QT *= 2;
  auto fits = [&](int q, long long cap) {
    return xmfma_lds_elems(a, d, fanout, q) * (long long)sizeof(float2) <= cap &&
           (fanout || xmfma_items(a, d, q) <= (long long)kXItems * (kThreads / 64));
  };
  while (QT > 1 && !fits(QT, budget)) QT /= 2;
  if (cfg.QT > 0 && QT != cfg.QT) return fail(TB_ERR_UNSUPPORTED, "RHS tile does not fit this stage");
  if (!fits(QT, limit)) return fail(TB_ERR_UNSUPPORTED, "block too large for the matrix-core transfer");
  const size_t lds = (size_t)xmfma_lds_elems(a, d, fanout, QT) * sizeof(float2);
  a.chunk = fanout ? a.R[0] : a.A[0];
  a.nsplit = 1;
  const long long nwg = (long long)n_items * a.nblk * ((a.nrhs + QT - 1) / QT);
  if (nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many right-hand sides for one launch");
  dim3 grid((unsigned)nwg);
  const tb_status st = d == 2 ? launch_xmfma_d<2>(a, fanout, QT, grid, lds, in, out, mats, stream)
                              : launch_xmfma_d<3>(a, fanout, QT, grid, lds, in, out, mats, stream);
  TB_TRY(st);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

template <class T, int D, int G>
static tb_status launch_stage_g(StageArgs a, bool fanout, bool sm, int QT, int V, dim3 grid, size_t lds,
                                const void* in, void* out, const void* mats, hipStream_t stream) {
  if (V == 4) {  // four right-hand sides per thread: tiles of 4 or 8
    if (fanout)
      return QT == 4 ? launch_fanout<T, D, 4, G, 4>(a, grid, lds, in, out, mats, stream)
                     : launch_fanout<T, D, 8, G, 4>(a, grid, lds, in, out, mats, stream);
    return QT == 4 ? launch_fanin<T, D, 4, G, 4>(a, sm, grid, lds, in, out, mats, stream)
                   : launch_fanin<T, D, 8, G, 4>(a, sm, grid, lds, in, out, mats, stream);
  }
  if (fanout) {
    switch (QT) {
      case 1: return launch_fanout<T, D, 1, G, 1>(a, grid, lds, in, out, mats, stream);
      case 2: return launch_fanout<T, D, 2, G, 1>(a, grid, lds, in, out, mats, stream);
      case 4: return launch_fanout<T, D, 4, G, 1>(a, grid, lds, in, out, mats, stream);
      default: return launch_fanout<T, D, 8, G, 1>(a, grid, lds, in, out, mats, stream);
    }
  }
  switch (QT) {
    case 1: return launch_fanin<T, D, 1, G, 1>(a, sm, grid, lds, in, out, mats, stream);
    case 2: return launch_fanin<T, D, 2, G, 1>(a, sm, grid, lds, in, out, mats, stream);
    case 4: return launch_fanin<T, D, 4, G, 1>(a, sm, grid, lds, in, out, mats, stream);
    default: return launch_fanin<T, D, 8, G, 1>(a, sm, grid, lds, in, out, mats, stream);
  }
}

// LDS elements of stage_fanin_turn for a slice of `chunk` rows and QT
// right-hand sides (padded extents bound the true ones).
static long long turn_lds_elems(const StageArgs& a, int d, int chunk, int QT) {
  const long long nchild = a.coarse_global ? 1 : (1LL << d);
  long long msz = (long long)chunk * a.R[0];
  for (int k = 1; k < d; ++k) msz += (long long)a.R[k] * a.A[k];
  long long e = nchild * msz;
  if (d == 2) return e + (long long)chunk * (a.R[1] + a.A[1]) * QT;
  return e + (long long)chunk *
                 ((long long)a.R[1] * a.R[2] + (long long)a.A[1] * a.R[2] + (long long)a.A[1] * a.A[2]) * QT;
}

template <class T, int D, int QT, int V>
static tb_status launch_fanin_turn(StageArgs a, dim3 grid, size_t lds, const void* in, void* out,
                                   const void* mats, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  TB_TRY(set_lds(stage_fanin_turn<T, D, QT, 8, V>, lds));
  stage_fanin_turn<T, D, QT, 8, V><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out,
                                                                   (const C*)mats);
  return TB_OK;
}

template <class T, int D>
static tb_status launch_turn_q(StageArgs a, int QT, int V, dim3 grid, size_t lds, const void* in, void* out,
                               const void* mats, hipStream_t stream) {
  if (V == 4)
    return QT == 4 ? launch_fanin_turn<T, D, 4, 4>(a, grid, lds, in, out, mats, stream)
                   : launch_fanin_turn<T, D, 8, 4>(a, grid, lds, in, out, mats, stream);
  switch (QT) {
    case 1: return launch_fanin_turn<T, D, 1, 1>(a, grid, lds, in, out, mats, stream);
    case 2: return launch_fanin_turn<T, D, 2, 1>(a, grid, lds, in, out, mats, stream);
    case 4: return launch_fanin_turn<T, D, 4, 1>(a, grid, lds, in, out, mats, stream);
    default: return launch_fanin_turn<T, D, 8, 1>(a, grid, lds, in, out, mats, stream);
  }
}

// Fan-in with the children in turn and the first mode first
// (stage_fanin_turn; 8 outputs per thread): the same tile and slice choices
// as launch_stage, with its own LDS size.
template <class T>
static tb_status launch_stage_turn(const Plan& p, StageArgs a, int n_items, const void* in, void* out,
                                   const void* mats, hipStream_t stream, const LaunchCfg& cfg) {
  using C = typename CplxOf<T>::type;
  const int d = p.d;
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  const long long budget = std::min<long long>(limit, 80 * 1024);
  const long long blocks = (long long)n_items * a.nblk;
  const int dim = a.A[0];
  const int qcap = cfg.QT > 0 ? cfg.QT : 8;
  int QT = 1;
  while (QT * 2 <= qcap && QT * 2 <= a.nrhs) QT *= 2;
  while (QT > 1 && turn_lds_elems(a, d, 1, QT) * (long long)sizeof(C) > budget) QT /= 2;
  if (cfg.QT > 0 && QT != cfg.QT) return fail(TB_ERR_UNSUPPORTED, "RHS tile does not fit this stage");
  if (cfg.G != 0 && cfg.G != 8) return fail(TB_ERR_UNSUPPORTED, "the in-turn fan-in takes 8 outputs per thread");
  const int V = cfg.V > 0 ? cfg.V : 1;
  if (V != 1 && (V != 4 || QT < 4)) return fail(TB_ERR_UNSUPPORTED, "RHS per thread needs a tile of 4 or 8");
  int chunk = cfg.split == 1
                  ? dim
                  : (int)std::max<long long>(1, (dim * blocks + kTargetWorkgroups - 1) / kTargetWorkgroups);
  chunk = std::min(chunk, dim);
  while (chunk > 1 && turn_lds_elems(a, d, chunk, QT) * (long long)sizeof(C) > budget) --chunk;
  const size_t lds = (size_t)turn_lds_elems(a, d, chunk, QT) * sizeof(C);
  if (lds > (size_t)limit) return fail(TB_ERR_UNSUPPORTED, "in-turn fan-in exceeds the LDS limit");
  a.chunk = chunk;
  a.nsplit = (dim + chunk - 1) / chunk;
  const long long nwg = blocks * a.nsplit * ((a.nrhs + QT - 1) / QT);
  if (nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many right-hand sides for one launch");
  dim3 grid((unsigned)nwg);
  const tb_status st = d == 2 ? launch_turn_q<T, 2>(a, QT, V, grid, lds, in, out, mats, stream)
                              : launch_turn_q<T, 3>(a, QT, V, grid, lds, in, out, mats, stream);
  TB_TRY(st);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

// One transfer launch.  cfg fields left at 0 take the heuristic: the
// largest RHS tile QT <= 8 that fits the LDS budget, G = 8 from QT = 4 on,
// and slices of the first mode until about kTargetWorkgroups workgroups
// exist (split = 1: one slice per block when it fits).
// Register-fiber stages (stage_fiber.hip): one right-hand side per
// workgroup, slices of the first output mode for about kTargetWorkgroups
// workgroups (or whole blocks), two workgroups' LDS per CU where possible.
template <class T>
static tb_status launch_stage_fiber(const Plan& p, StageArgs a, bool fanout, int n_items, const void* in,
                                    void* out, const void* mats, hipStream_t stream, const LaunchCfg& cfg) {
  using C = typename CplxOf<T>::type;
  const int d = p.d;
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  const long long budget = std::min<long long>(limit, 80 * 1024);
  const long long blocks = (long long)n_items * a.nblk * a.nrhs;
  const int dim = fanout ? a.R[0] : a.A[0];
  int chunk = cfg.split == 1
                  ? dim
                  : (int)std::max<long long>(1, (dim * blocks + kTargetWorkgroups - 1) / kTargetWorkgroups);
  chunk = std::max(1, std::min(chunk, dim));
  while (chunk > 1 && stage_lds_elems(a, d, fanout, chunk, 1, true) * (long long)sizeof(C) > budget) --chunk;
  const size_t lds = (size_t)stage_lds_elems(a, d, fanout, chunk, 1, true) * sizeof(C);
  if (lds + 256 > (size_t)limit)
    return fail(TB_ERR_UNSUPPORTED, "transfer block exceeds the per-workgroup LDS budget");
  a.chunk = chunk;
  a.nsplit = (dim + chunk - 1) / chunk;
  const long long nwg = blocks * a.nsplit;
  return launch_stage_fib(sizeof(T) == 8, a, d, fanout, fanout ? a.fib_out : a.fib_in, nwg, lds, in, out,
                          mats, stream);
}

template <class T>
static tb_status launch_stage(const Plan& p, StageArgs a, bool fanout, int n_items, const void* in,
                              void* out, const void* mats, hipStream_t stream, const LaunchCfg& cfg) {
  using C = typename CplxOf<T>::type;
  if (fanout) {  // item blocks per outer middle multi-set (fine items): the
                 // fan-outs of one side read what the previous fan-out wrote
                 // for the same outer multi-set; a fan-in reads the core's or
                 // its children's outputs, written from every XCD, and keeps
                 // the balanced round-robin map (measured slower with it)
    const long long per = (1LL << (p.d * a.lvl)) * a.nblk;
    a.aff_blocks = per < (1LL << 30) ? (int)per : 0;
  }
  if (cfg.alt == 4) return launch_stage_fiber<T>(p, a, fanout, n_items, in, out, mats, stream, cfg);
  if (cfg.alt == 5) {  // leaves: one wave per leaf box
    int limit = 0;
    TB_TRY(lds_limit(&limit));
    return launch_leaf_wave(sizeof(T) == 8, a, p.d, fanout, cfg.split == 1 ? 4 : 1, n_items, in, out, mats,
                            stream, limit);
  }
  if (cfg.alt == 3) {  // flat staging, one right-hand side per workgroup
    if constexpr (sizeof(T) != 4) {
      return fail(TB_ERR_UNSUPPORTED, "flat-staged transfer stages are FP32 only");
    } else {
      int limit = 0;
      TB_TRY(lds_limit(&limit));
      return launch_stage_flat_f32(a, p.d, fanout, n_items, in, out, mats, stream, cfg.split == 1 ? 2 : 1,
                                   limit);
    }
  }
  if (cfg.mfma == 2) {  // transfer levels on 4 x 4 matrix-core blocks, d = 3
    if constexpr (sizeof(T) != 4) {
      return fail(TB_ERR_UNSUPPORTED, "the 4 x 4 matrix-core transfers are FP32 only");
    } else {
      if (fanout) return launch_fanout_m4(a, p.d, n_items, in, out, mats, stream);
      return a.coarse_global ? launch_leaf_fanin_m4(a, p.d, n_items, in, out, mats, stream)
                             : launch_fanin_m4(a, p.d, n_items, in, out, mats, stream);
    }
  }
  if (cfg.mfma == 1) return launch_stage_xmfma<T>(p, a, fanout, n_items, in, out, mats, stream, cfg);
  if (cfg.alt == 1 || cfg.alt == 2) {
    if (fanout) return fail(TB_ERR_UNSUPPORTED, "no in-turn variant of the fan-out");
    return cfg.alt == 1 ? launch_stage_seq<T>(p, a, n_items, in, out, mats, stream, cfg)
                        : launch_stage_turn<T>(p, a, n_items, in, out, mats, stream, cfg);
  }
  const int d = p.d;
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  // keep two workgroups' LDS per CU where possible
  const long long budget = std::min<long long>(limit, 80 * 1024);
  const long long blocks = (long long)n_items * a.nblk;
  const int dim = fanout ? a.R[0] : a.A[0];
  // fan-in matrices are staged in LDS when they fit, else read from global
  const bool sm = fanout || stage_lds_elems(a, d, false, 1, 1, true) * (long long)sizeof(C) <= budget;
  const int qcap = cfg.QT > 0 ? cfg.QT : 8;
  int QT = 1;
  while (QT * 2 <= qcap && QT * 2 <= a.nrhs) QT *= 2;
  while (QT > 1 && stage_lds_elems(a, d, fanout, 1, QT, sm) * (long long)sizeof(C) > budget) QT /= 2;
  if (cfg.QT > 0 && QT != cfg.QT) return fail(TB_ERR_UNSUPPORTED, "RHS tile does not fit this stage");
  int chunk = cfg.split == 1
                  ? dim
                  : (int)std::max<long long>(1, (dim * blocks + kTargetWorkgroups - 1) / kTargetWorkgroups);
  chunk = std::min(chunk, dim);
  while (chunk > 1 && stage_lds_elems(a, d, fanout, chunk, QT, sm) * (long long)sizeof(C) > budget) --chunk;
  const size_t lds = (size_t)stage_lds_elems(a, d, fanout, chunk, QT, sm) * sizeof(C);
  if (lds > (size_t)limit)
    return fail(TB_ERR_UNSUPPORTED, "transfer block exceeds the per-workgroup LDS budget");
  a.chunk = chunk;
  a.nsplit = (dim + chunk - 1) / chunk;
  const long long nwg = blocks * a.nsplit * ((a.nrhs + QT - 1) / QT);
  if (nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many right-hand sides for one launch");
  dim3 grid((unsigned)nwg);
  const int G = cfg.G > 0 ? cfg.G : (QT >= 4 ? 8 : 1);
  const int V = cfg.V > 0 ? cfg.V : 1;
  if (V != 1 && (V != 4 || QT < 4)) return fail(TB_ERR_UNSUPPORTED, "RHS per thread needs a tile of 4 or 8");
  tb_status st;
  if (G == 8)
    st = d == 2 ? launch_stage_g<T, 2, 8>(a, fanout, sm, QT, V, grid, lds, in, out, mats, stream)
                : launch_stage_g<T, 3, 8>(a, fanout, sm, QT, V, grid, lds, in, out, mats, stream);
  else
    st = d == 2 ? launch_stage_g<T, 2, 1>(a, fanout, sm, QT, V, grid, lds, in, out, mats, stream)
                : launch_stage_g<T, 3, 1>(a, fanout, sm, QT, V, grid, lds, in, out, mats, stream);
  TB_TRY(st);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

template <class T, class CS, int D, int QT>
static tb_status launch_core_q(const Plan& p, CoreArgs a, bool adjoint, const void* cores,
                               const void* in, void* out, int maxRS, int maxRTp, int limit,
                               hipStream_t stream, bool grouped = false) {
  using C = typename CplxOf<T>::type;
  constexpr int VR = CoreVec<CS>::VR;
  const unsigned gy = (unsigned)((a.nrhs + QT - 1) / QT);
  if (!adjoint) {
    const size_t lds = ((size_t)maxRS * QT + (size_t)kThreads * VR * QT) * sizeof(C);
    if (lds > (size_t)limit) return fail(TB_ERR_UNSUPPORTED, "core block exceeds the LDS budget");
    const int lv = VR == 1 ? 0 : (VR == 2 ? 1 : 2);
    TB_TRY(set_lds(core_fwd<T, CS, D, QT>, lds));
    core_fwd<T, CS, D, QT><<<dim3((unsigned)p.fwd_units[lv].size(), gy), kThreads, lds, stream>>>(
        a, (const CS*)cores, p.core_off_d, p.pair_meta_d, p.fwd_units_d[lv], (const C*)in, (C*)out);
  } else {
    const size_t lds = (size_t)maxRTp * QT * sizeof(C);
    if (lds > (size_t)limit) return fail(TB_ERR_UNSUPPORTED, "core block exceeds the LDS budget");
    if (grouped) {  // 16-lane column groups, 256-column panels
      TB_TRY(set_lds(core_adj16<T, CS, D, QT>, lds));
      core_adj16<T, CS, D, QT><<<dim3((unsigned)p.mfma_adj_units.size(), gy), kThreads, lds, stream>>>(
          a, (const CS*)cores, p.core_off_d, p.pair_meta_d, p.mfma_adj_units_d, (const C*)in, (C*)out);
    } else {  // 64-column panels (two column groups per workgroup)
      TB_TRY(set_lds(core_adj<T, CS, D, QT, 2>, lds));
      core_adj<T, CS, D, QT, 2><<<dim3((unsigned)p.adj_units.size(), gy), kThreads, lds, stream>>>(
          a, (const CS*)cores, p.core_off_d, p.pair_meta_d, p.adj_units_d, (const C*)in, (C*)out);
    }
  }
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

constexpr int kMfmaMinRhs = 8;   // from this many right-hand sides the matrix cores run the core

template <class CS, int D>
static tb_status launch_core_mfma(const Plan& p, const CoreArgs& a, bool adjoint, const void* cores,
                                  const void* in, void* out, hipStream_t stream, bool bf16_mfma = false) {
  const unsigned gy = (unsigned)((a.nrhs + kMQ - 1) / kMQ);
  if constexpr (sizeof(CS) == 4) {
    if (bf16_mfma) {
      if (!adjoint)
        core_fwd_mfma_bf16<D><<<dim3((unsigned)p.mfma_fwd_units.size() * gy), kThreads, 0, stream>>>(
            a, (const unsigned*)cores, p.core_off_d, p.pair_meta_d, p.mfma_fwd_units_d, (const float2*)in,
            (float2*)out);
      else
        core_adj_mfma_bf16<D><<<dim3((unsigned)p.mfma_adj_units.size() * gy), kThreads, 0, stream>>>(
            a, (const unsigned*)cores, p.core_off_d, p.pair_meta_d, p.mfma_adj_units_d, (const float2*)in,
            (float2*)out);
      TB_HIP_TRY(hipGetLastError());
      return TB_OK;
    }
  }
  if (!adjoint)
    core_fwd_mfma<CS, D><<<dim3((unsigned)p.mfma_fwd_units.size() * gy), kThreads, 0, stream>>>(
        a, (const CS*)cores, p.core_off_d, p.pair_meta_d, p.mfma_fwd_units_d, (const float2*)in, (float2*)out);
  else
    core_adj_mfma<CS, D><<<dim3((unsigned)p.mfma_adj_units.size() * gy), kThreads, 0, stream>>>(
        a, (const CS*)cores, p.core_off_d, p.pair_meta_d, p.mfma_adj_units_d, (const float2*)in, (float2*)out);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

// BF16 cores, second form (MTW 16-row tiles per wave, NQ = 16 NQT
// right-hand sides per workgroup): every 256-row (adjoint: 256-column) unit
// is split into 256 / (64 MTW) workgroups; those past the pair's extent
// return at once.
template <int D, bool ADJ, int MTW, int NQT>
static tb_status launch_core_bf16_v2(const Plan& p, const CoreArgs& a, const void* cores, const void* in,
                                     void* out, int maxK, hipStream_t stream) {
  using TL = Bf16Tile<MTW, NQT>;
  const std::vector<int2>& units = ADJ ? p.mfma_adj_units : p.mfma_fwd_units;
  const int2* units_d = ADJ ? p.mfma_adj_units_d : p.mfma_fwd_units_d;
  const long long nqt = (a.nrhs + TL::NQ - 1) / TL::NQ;
  const long long nblocks = (long long)units.size() * TL::kSub * nqt;
  if (nblocks > (1LL << 31) - 1) return fail(TB_ERR_UNSUPPORTED, "core grid too large");
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  const size_t lds = (size_t)maxK * sizeof(int);
  const size_t fixed = 2 * sizeof(uint4) * TL::NQ * TL::kLd4 + sizeof(int) * TL::kRows;
  if (lds + fixed > (size_t)limit) return fail(TB_ERR_UNSUPPORTED, "core position table exceeds LDS");
  TB_TRY(set_lds(core_mfma_bf16_v2<D, ADJ, MTW, NQT>, lds + fixed));
  core_mfma_bf16_v2<D, ADJ, MTW, NQT><<<dim3((unsigned)nblocks), kThreads, lds, stream>>>(
      a, (const unsigned*)cores, p.core_off_d, p.pair_meta_d, units_d, (const float2*)in, (float2*)out);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

// form: 5 = 256 rows x 32 right-hand sides per workgroup, 6 = 128 x 64,
// 7 = 128 x 32
template <int D, bool ADJ>
static tb_status launch_core_bf16_form(const Plan& p, const CoreArgs& a, int form, const void* cores,
                                       const void* in, void* out, int maxK, hipStream_t stream) {
  switch (form) {
    case 5: return launch_core_bf16_v2<D, ADJ, 4, 2>(p, a, cores, in, out, maxK, stream);
    case 6: return launch_core_bf16_v2<D, ADJ, 2, 4>(p, a, cores, in, out, maxK, stream);
    default: return launch_core_bf16_v2<D, ADJ, 2, 2>(p, a, cores, in, out, maxK, stream);
  }
}

template <class T, class CS>
static tb_status launch_core(const Plan& p, bool adjoint, int nrhs, const void* cores, const void* in,
                             void* out, hipStream_t stream, const LaunchCfg& cfg) {
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
  a.colscale = p.core_scale;
  a.col_off = p.col_off_d;
  int maxRS = 0, maxRTp = 0;
  for (long long pr = 0; pr < p.npairs; ++pr) {
    maxRS = std::max(maxRS, p.pair_meta[(size_t)pr * kPairMeta + 1]);
    maxRTp = std::max(maxRTp, p.pair_meta[(size_t)pr * kPairMeta + 2]);
  }
  constexpr bool kQ16 = std::is_same<CS, Q16>::value;  // vector kernels only
  if (kQ16 && cfg.core >= 3 && cfg.core <= 7)
    return fail(TB_ERR_UNSUPPORTED, "16-bit cores run on the vector core kernels");
  const bool grouped = cfg.core == 8 || cfg.core == 9;  // adjoint with 16-lane column groups
  if (grouped && !adjoint) return fail(TB_ERR_UNSUPPORTED, "16-lane column groups are an adjoint kernel");
  if constexpr (std::is_same<CS, unsigned>::value) {  // BF16 cores
    if (cfg.core >= 5 && cfg.core <= 7) {
      int maxRT = 0;
      for (long long pr = 0; pr < p.npairs; ++pr) maxRT = std::max(maxRT, p.pair_meta[(size_t)pr * kPairMeta]);
      const int maxK = adjoint ? maxRT : maxRS;
      if (d == 2)
        return adjoint ? launch_core_bf16_form<2, true>(p, a, cfg.core, cores, in, out, maxK, stream)
                       : launch_core_bf16_form<2, false>(p, a, cfg.core, cores, in, out, maxK, stream);
      return adjoint ? launch_core_bf16_form<3, true>(p, a, cfg.core, cores, in, out, maxK, stream)
                     : launch_core_bf16_form<3, false>(p, a, cfg.core, cores, in, out, maxK, stream);
    }
    if (cfg.core == 4 || (cfg.core == 0 && nrhs >= kMfmaMinRhs))
      return d == 2 ? launch_core_mfma<CS, 2>(p, a, adjoint, cores, in, out, stream, true)
                    : launch_core_mfma<CS, 3>(p, a, adjoint, cores, in, out, stream, true);
  } else {
    if (cfg.core >= 4 && cfg.core <= 7) return fail(TB_ERR_UNSUPPORTED, "BF16 matrix cores need BF16 cores");
  }
  if constexpr (sizeof(T) == 4 && !kQ16) {
    if (cfg.core == 3 || (cfg.core == 0 && nrhs >= kMfmaMinRhs))
      return d == 2 ? launch_core_mfma<CS, 2>(p, a, adjoint, cores, in, out, stream)
                    : launch_core_mfma<CS, 3>(p, a, adjoint, cores, in, out, stream);
  } else {
    if (cfg.core == 3) return fail(TB_ERR_UNSUPPORTED, "no matrix-core path for FP64");
  }
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  using C = typename CplxOf<T>::type;
  const size_t need4 = adjoint ? (size_t)maxRTp * 4 * sizeof(C)
                               : ((size_t)maxRS * 4 + (size_t)kThreads * CoreVec<CS>::VR * 4) * sizeof(C);
  const int cq = grouped ? cfg.core - 7 : cfg.core;  // 1 or 4 right-hand sides per pass
  if (cq == 2 && need4 > (size_t)limit) return fail(TB_ERR_UNSUPPORTED, "core tile exceeds LDS");
  if (cq == 1 || nrhs == 1 || need4 > (size_t)limit)
    return d == 2 ? launch_core_q<T, CS, 2, 1>(p, a, adjoint, cores, in, out, maxRS, maxRTp, limit, stream, grouped)
                  : launch_core_q<T, CS, 3, 1>(p, a, adjoint, cores, in, out, maxRS, maxRTp, limit, stream, grouped);
  return d == 2 ? launch_core_q<T, CS, 2, 4>(p, a, adjoint, cores, in, out, maxRS, maxRTp, limit, stream, grouped)
                : launch_core_q<T, CS, 3, 4>(p, a, adjoint, cores, in, out, maxRS, maxRTp, limit, stream, grouped);
}

// Core contraction with the cores evaluated on the fly (TB_C64_OTF); cfg.core
// 1 or 2 picks the vector kernels with 1 or 4 right-hand sides per pass, 3
// (the default from kMfmaMinRhs right-hand sides) the FP32 matrix cores.
static tb_status launch_core_otf(const Plan& p, bool adjoint, int nrhs, const void* in, void* out,
                                 hipStream_t stream, const LaunchCfg& cfg) {
  if (p.kind == TB_KERNEL_DFT)
    return fail(TB_ERR_UNSUPPORTED, "no on-the-fly cores for the bit-reversed uniform DFT");
  const int d = p.d;
  const Level& st = p.src[p.Lt];
  const Level& tt = p.tgt[p.Ls];
  CoreArgs a{};
  a.nS = p.nS;
  a.nT = p.nT;
  a.Es = st.E;
  a.Et = tt.E;
  OtfSpec o{};
  o.nux = p.nux_d;
  o.n = p.n;
  o.omega_rev = p.omega / (2.0 * 3.14159265358979323846);
  o.ra = p.ra;
  o.rb = p.rb;
  o.rden = p.rden;
  for (int k = 0; k < d; ++k) {
    a.Rs[k] = st.R[k];
    a.Rt[k] = tt.R[k];
    o.Rs_sk = std::max(o.Rs_sk, st.R[k]);
    o.Rt_sk = std::max(o.Rt_sk, tt.R[k]);
  }
  a.nrhs = nrhs;
  int maxRS = 0, maxRT = 0;
  for (long long pr = 0; pr < p.npairs; ++pr) {
    maxRT = std::max(maxRT, p.pair_meta[(size_t)pr * kPairMeta]);
    maxRS = std::max(maxRS, p.pair_meta[(size_t)pr * kPairMeta + 1]);
  }
  if (cfg.core > 3) return fail(TB_ERR_UNSUPPORTED, "on-the-fly cores take core kernel 1, 2 or 3");
  if (cfg.core == 3 || (cfg.core == 0 && nrhs >= kMfmaMinRhs)) {  // matrix cores
    if (p.kind == TB_KERNEL_FOURIER && p.n > (1 << 15))
      return fail(TB_ERR_UNSUPPORTED, "on-the-fly Fourier cores need n <= 32768");
    const unsigned gy = (unsigned)((nrhs + kMQ - 1) / kMQ);
    const std::vector<int2>& mu = adjoint ? p.mfma_adj_units : p.mfma_fwd_units;
    const int2* mu_d = adjoint ? p.mfma_adj_units_d : p.mfma_fwd_units_d;
    const unsigned grid = (unsigned)(mu.size() * gy);
    auto go = [&](auto kern) -> tb_status {
      kern<<<grid, kThreads, 0, stream>>>(a, o, p.pair_meta_d, mu_d, p.top_src_skel_d, p.top_tgt_skel_d,
                                          (const float2*)in, (float2*)out);
      TB_HIP_TRY(hipGetLastError());
      return TB_OK;
    };
    auto by_kind = [&](auto kind_tag) -> tb_status {
      constexpr int K = decltype(kind_tag)::value;
      if (d == 2) return adjoint ? go(core_adj_mfma_otf<K, 2>) : go(core_fwd_mfma_otf<K, 2>);
      return adjoint ? go(core_adj_mfma_otf<K, 3>) : go(core_fwd_mfma_otf<K, 3>);
    };
    switch (p.kind) {
      case TB_KERNEL_FOURIER: return by_kind(std::integral_constant<int, TB_KERNEL_FOURIER>{});
      case TB_KERNEL_HELMHOLTZ: return by_kind(std::integral_constant<int, TB_KERNEL_HELMHOLTZ>{});
      case TB_KERNEL_NUDFT: return by_kind(std::integral_constant<int, TB_KERNEL_NUDFT>{});
      case TB_KERNEL_RADON: return by_kind(std::integral_constant<int, TB_KERNEL_RADON>{});
      default: return fail(TB_ERR_UNSUPPORTED, "no on-the-fly entries for this kernel");
    }
  }
  const int QT = (cfg.core == 2 || (cfg.core == 0 && nrhs >= 4)) ? 4 : 1;
  int limit = 0;
  TB_TRY(lds_limit(&limit));
  if (p.kind == TB_KERNEL_FOURIER && p.n > (1 << 15))
    return fail(TB_ERR_UNSUPPORTED, "on-the-fly Fourier cores need n <= 32768");
  const int along = std::min(adjoint ? maxRT : maxRS, kOtfChunk);
  const size_t point =
      (p.kind == TB_KERNEL_RADON || p.kind == TB_KERNEL_NUDFT) ? sizeof(double4) : sizeof(int4);
  const size_t lds = (size_t)along * point + ((size_t)along + kThreads) * QT * sizeof(float2);
  if (lds > (size_t)limit) return fail(TB_ERR_UNSUPPORTED, "on-the-fly core block exceeds the LDS limit");
  const std::vector<int2>& units = adjoint ? p.adj_units : p.fwd_units[0];
  const int2* units_d = adjoint ? p.adj_units_d : p.fwd_units_d[0];
  dim3 grid((unsigned)units.size(), (unsigned)((nrhs + QT - 1) / QT));
  auto go = [&](auto kern) -> tb_status {
    TB_TRY(set_lds(kern, lds));
    kern<<<grid, kThreads, lds, stream>>>(a, o, p.pair_meta_d, units_d, p.top_src_skel_d, p.top_tgt_skel_d,
                                          (const float2*)in, (float2*)out);
    TB_HIP_TRY(hipGetLastError());
    return TB_OK;
  };
  auto by_kind = [&](auto kind_tag) -> tb_status {
    constexpr int K = decltype(kind_tag)::value;
    if (d == 2) {
      if (adjoint) return QT == 4 ? go(core_adj_otf<K, 2, 4>) : go(core_adj_otf<K, 2, 1>);
      return QT == 4 ? go(core_fwd_otf<K, 2, 4>) : go(core_fwd_otf<K, 2, 1>);
    }
    if (adjoint) return QT == 4 ? go(core_adj_otf<K, 3, 4>) : go(core_adj_otf<K, 3, 1>);
    return QT == 4 ? go(core_fwd_otf<K, 3, 4>) : go(core_fwd_otf<K, 3, 1>);
  };
  switch (p.kind) {
    case TB_KERNEL_FOURIER: return by_kind(std::integral_constant<int, TB_KERNEL_FOURIER>{});
    case TB_KERNEL_HELMHOLTZ: return by_kind(std::integral_constant<int, TB_KERNEL_HELMHOLTZ>{});
    case TB_KERNEL_NUDFT: return by_kind(std::integral_constant<int, TB_KERNEL_NUDFT>{});
    default:
      return by_kind(std::integral_constant<int, TB_KERNEL_RADON>{});
  }
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

// The kernel launches of one apply, in order; run(cfg) enqueues one launch.
struct Step {
  int stage;
  bool core, fanout;
  std::function<tb_status(const LaunchCfg&)> run;
};

// ws_ext (nullable): a workspace of ws_cap bytes owned by the caller of the
// apply; otherwise the plan's own workspace, grown on demand.
template <class T, class CS>
static tb_status build_steps(Plan& p, const void* in, void* out, long long nrhs, bool adjoint,
                             const void* cores, hipStream_t stream, std::vector<Step>* steps,
                             bool otf = false, void* ws_ext = nullptr, size_t ws_cap = 0) {
  using C = typename CplxOf<T>::type;
  const size_t esz = sizeof(C);
  Buffers b = layout(p, nrhs, esz);
  if (ws_ext) {
    if (b.total > ws_cap)
      return fail(TB_ERR_OOM, "apply needs " + std::to_string(b.total) +
                                  " bytes of workspace; the allocation-free scratch holds " +
                                  std::to_string(ws_cap));
  } else {
    TB_TRY(ensure_workspace(p, b.total));
  }
  char* ws = static_cast<char*>(ws_ext ? ws_ext : p.ws.base);
  auto S = [ws, b](int l) { return (void*)(ws + b.src_off[l]); };
  auto Tb = [ws, b](int l) { return (void*)(ws + b.tgt_off[l]); };
  auto mats = [](const Level& lv) -> const void* {
    return sizeof(T) == 8 ? (const void*)lv.X64 : (const void*)lv.X32;
  };
  const int rhs = (int)nrhs;
  Plan* pp = &p;
  auto stage = [&](int id, const Level& lv, const Level* coarse, bool source, bool conj, bool fanout,
                   int n_items, const void* src, void* dst) {
    StageArgs a = stage_args(p, lv, coarse, source, rhs, conj);
    const void* m = mats(lv);
    steps->push_back({id, false, fanout, [=](const LaunchCfg& c) {
                        return launch_stage<T>(*pp, a, fanout, n_items, src, dst, m, stream, c);
                      }});
  };
  auto core = [&](bool adj, const void* src, void* dst) {
    steps->push_back({adj ? TB_STAGE_CORE_ADJ : TB_STAGE_CORE, true, false, [=](const LaunchCfg& c) {
                        if constexpr (sizeof(T) == 4) {
                          if (otf) return launch_core_otf(*pp, adj, rhs, src, dst, stream, c);
                        }
                        return launch_core<T, CS>(*pp, adj, rhs, cores, src, dst, stream, c);
                      }});
  };
  steps->clear();
  if (!adjoint) {
    // (1) V then W: coarse (f or level l-1) -> fine (level l)
    for (int l = 0; l <= p.Lt; ++l)
      stage(l ? TB_STAGE_SRC_TRANSFER : TB_STAGE_SRC_LEAF, p.src[l], l ? &p.src[l - 1] : nullptr, true,
            false, true, p.src[l].nitems, l ? S(l - 1) : in, S(l));
    // (2) cores
    core(false, S(p.Lt), Tb(p.Ls));
    // (3) P^T accumulated into the parents, then U^T into u
    for (int l = p.Ls; l >= 0; --l)
      stage(l ? TB_STAGE_TGT_TRANSFER : TB_STAGE_TGT_LEAF, p.tgt[l], l ? &p.tgt[l - 1] : nullptr, false,
            false, false, l ? p.tgt[l - 1].nitems : p.tgt[l].nitems, Tb(l), l ? Tb(l - 1) : out);
  } else {
    for (int l = 0; l <= p.Ls; ++l)
      stage(l ? TB_STAGE_TGT_TRANSFER_ADJ : TB_STAGE_TGT_LEAF_ADJ, p.tgt[l], l ? &p.tgt[l - 1] : nullptr,
            false, true, true, p.tgt[l].nitems, l ? Tb(l - 1) : in, Tb(l));
    core(true, Tb(p.Ls), S(p.Lt));
    for (int l = p.Lt; l >= 0; --l)
      stage(l ? TB_STAGE_SRC_TRANSFER_ADJ : TB_STAGE_SRC_LEAF_ADJ, p.src[l], l ? &p.src[l - 1] : nullptr,
            true, true, false, l ? p.src[l - 1].nitems : p.src[l].nitems, S(l), l ? S(l - 1) : out);
  }
  return TB_OK;
}

static int steps_per_direction(const Plan& p) { return p.Lt + p.Ls + 3; }

// The same sequence for d above the tuned kernels' 3 modes, on the generic
// kernels (apply_generic.hip): FP64 or FP32 with stored cores.  The stage
// scratch follows the level buffers in the workspace.
template <class T>
static tb_status build_steps_generic(Plan& p, const void* in, void* out, long long nrhs, bool adjoint,
                                     const void* cores, hipStream_t stream, std::vector<Step>* steps,
                                     void* ws_ext, size_t ws_cap) {
  using C = typename CplxOf<T>::type;
  const size_t esz = sizeof(C);
  const bool fp64 = sizeof(T) == 8;
  Buffers b = layout(p, nrhs, esz);
  const int rhs = (int)nrhs;
  const int d = p.d;
  size_t scr = 0;
  auto scratch_of = [&](const Level& lv, const Level* coarse, bool source, bool fanout, int n_items) {
    StageArgs a = stage_args(p, lv, coarse, source, rhs, false);
    scr = std::max(scr, gen_stage_scratch(a, d, fanout, n_items, esz));
  };
  for (int l = 0; l <= p.Lt; ++l) {
    scratch_of(p.src[l], l ? &p.src[l - 1] : nullptr, true, true, p.src[l].nitems);
    scratch_of(p.src[l], l ? &p.src[l - 1] : nullptr, true, false, l ? p.src[l - 1].nitems : p.src[l].nitems);
  }
  for (int l = 0; l <= p.Ls; ++l) {
    scratch_of(p.tgt[l], l ? &p.tgt[l - 1] : nullptr, false, true, p.tgt[l].nitems);
    scratch_of(p.tgt[l], l ? &p.tgt[l - 1] : nullptr, false, false, l ? p.tgt[l - 1].nitems : p.tgt[l].nitems);
  }
  const size_t scr_off = (b.total + 255) / 256 * 256;
  const size_t total = scr_off + scr;
  if (ws_ext) {
    if (total > ws_cap)
      return fail(TB_ERR_OOM, "apply needs " + std::to_string(total) +
                                  " bytes of workspace; the allocation-free scratch holds " +
                                  std::to_string(ws_cap));
  } else {
    TB_TRY(ensure_workspace(p, total));
  }
  char* ws = static_cast<char*>(ws_ext ? ws_ext : p.ws.base);
  void* scratch = ws + scr_off;
  auto S = [ws, b](int l) { return (void*)(ws + b.src_off[l]); };
  auto Tb = [ws, b](int l) { return (void*)(ws + b.tgt_off[l]); };
  auto mats = [](const Level& lv) -> const void* {
    return sizeof(T) == 8 ? (const void*)lv.X64 : (const void*)lv.X32;
  };
  Plan* pp = &p;
  auto stage = [&](int id, const Level& lv, const Level* coarse, bool source, bool conj, bool fanout,
                   int n_items, const void* src, void* dst) {
    StageArgs a = stage_args(p, lv, coarse, source, rhs, conj);
    const void* m = mats(lv);
    steps->push_back({id, false, fanout, [=](const LaunchCfg&) {
                        return launch_gen_stage(fp64, a, d, fanout, n_items, src, dst, m, scratch, stream);
                      }});
  };
  GenCoreArgs g{};
  g.d = d;
  g.nrhs = rhs;
  g.nS = p.nS;
  g.nT = p.nT;
  g.Es = p.src[p.Lt].E;
  g.Et = p.tgt[p.Ls].E;
  for (int k = 0; k < d; ++k) {
    g.Rs[k] = p.src[p.Lt].R[k];
    g.Rt[k] = p.tgt[p.Ls].R[k];
  }
  int max_rt = 0, max_rs = 0;
  for (long long pr = 0; pr < p.npairs; ++pr) {
    max_rt = std::max(max_rt, p.pair_meta[(size_t)pr * kPairMeta]);
    max_rs = std::max(max_rs, p.pair_meta[(size_t)pr * kPairMeta + 1]);
  }
  auto core = [&](bool adj, const void* src, void* dst) {
    steps->push_back({adj ? TB_STAGE_CORE_ADJ : TB_STAGE_CORE, true, false, [=](const LaunchCfg&) {
                        return launch_gen_core(fp64, g, adj, cores, pp->core_off_d, pp->pair_meta_d,
                                               pp->npairs, max_rt, max_rs, src, dst, stream);
                      }});
  };
  steps->clear();
  if (!adjoint) {
    for (int l = 0; l <= p.Lt; ++l)
      stage(l ? TB_STAGE_SRC_TRANSFER : TB_STAGE_SRC_LEAF, p.src[l], l ? &p.src[l - 1] : nullptr, true,
            false, true, p.src[l].nitems, l ? S(l - 1) : in, S(l));
    core(false, S(p.Lt), Tb(p.Ls));
    for (int l = p.Ls; l >= 0; --l)
      stage(l ? TB_STAGE_TGT_TRANSFER : TB_STAGE_TGT_LEAF, p.tgt[l], l ? &p.tgt[l - 1] : nullptr, false,
            false, false, l ? p.tgt[l - 1].nitems : p.tgt[l].nitems, Tb(l), l ? Tb(l - 1) : out);
  } else {
    for (int l = 0; l <= p.Ls; ++l)
      stage(l ? TB_STAGE_TGT_TRANSFER_ADJ : TB_STAGE_TGT_LEAF_ADJ, p.tgt[l], l ? &p.tgt[l - 1] : nullptr,
            false, true, true, p.tgt[l].nitems, l ? Tb(l - 1) : in, Tb(l));
    core(true, Tb(p.Ls), S(p.Lt));
    for (int l = p.Lt; l >= 0; --l)
      stage(l ? TB_STAGE_SRC_TRANSFER_ADJ : TB_STAGE_SRC_LEAF_ADJ, p.src[l], l ? &p.src[l - 1] : nullptr,
            true, true, false, l ? p.src[l - 1].nitems : p.src[l].nitems, S(l), l ? S(l - 1) : out);
  }
  return TB_OK;
}

// With a caller workspace (ws_ext) no event is recorded: per-stage timing
// creates events, and that path promises to allocate nothing.
template <class T, class CS>
static tb_status apply_typed(Plan& p, tb_dtype io, const void* in, void* out, long long nrhs, bool adjoint,
                             const void* cores, hipStream_t stream, void* ws_ext, size_t ws_cap) {
  std::vector<Step> steps;
  tb_status built;
  if (p.d > kMaxDTuned) {
    if (io != TB_C128 && io != TB_C64)
      return fail(TB_ERR_UNSUPPORTED, "d > 3 applies run in FP64 or FP32 with stored cores");
    built = build_steps_generic<T>(p, in, out, nrhs, adjoint, cores, stream, &steps, ws_ext, ws_cap);
  } else {
    built = build_steps<T, CS>(p, in, out, nrhs, adjoint, cores, stream, &steps, io == TB_C64_OTF, ws_ext,
                               ws_cap);
  }
  TB_TRY(built);
  const auto it = p.tuned.find({(int)io, nrhs});
  const LaunchCfg none{};
  const int base = adjoint ? steps_per_direction(p) : 0;
  for (size_t i = 0; i < steps.size(); ++i) {
    const LaunchCfg& cfg = it == p.tuned.end() ? none : it->second[base + i];
    if (ws_ext)
      TB_TRY(steps[i].run(cfg));
    else
      TB_TRY(timed(p, steps[i].stage, stream, [&] { return steps[i].run(cfg); }));
  }
  return TB_OK;
}

static bool valid_io(int io) { return io >= TB_C128 && io <= TB_CQ16; }

// on-the-fly applies need no stored cores
static bool has_cores(const Plan& p, int io) {
  return io == TB_C64_OTF || (io != TB_C64_OTF && p.cores[io]);
}

tb_status run_apply(Plan& p, const void* in, void* out, long long nrhs, tb_dtype io, bool adjoint,
                    hipStream_t stream, void* ws_ext, size_t ws_cap) {
  if (!in || !out) return fail(TB_ERR_INVALID_ARG, "null input or output pointer");
  if (nrhs < 1 || nrhs > (1 << 20)) return fail(TB_ERR_INVALID_ARG, "nrhs must be in [1, 2^20]");
  if (!valid_io(io)) return fail(TB_ERR_INVALID_ARG, "unknown tb_dtype");
  if (!has_cores(p, io))
    return fail(TB_ERR_INVALID_ARG,
                "the plan holds no cores of the requested precision (see store_mask)");
  if (in == out) return fail(TB_ERR_INVALID_ARG, "input and output must not alias");
  void* cs = io == TB_C64_OTF ? nullptr : p.cores[io];
  switch (io) {
    case TB_C128: return apply_typed<double, double2>(p, io, in, out, nrhs, adjoint, cs, stream, ws_ext, ws_cap);
    case TB_C64: return apply_typed<float, float2>(p, io, in, out, nrhs, adjoint, cs, stream, ws_ext, ws_cap);
    case TB_CBF16: return apply_typed<float, unsigned>(p, io, in, out, nrhs, adjoint, cs, stream, ws_ext, ws_cap);
    case TB_C64_OTF: return apply_typed<float, float2>(p, io, in, out, nrhs, adjoint, cs, stream, ws_ext, ws_cap);
    case TB_CQ16: return apply_typed<float, Q16>(p, io, in, out, nrhs, adjoint, cs, stream, ws_ext, ws_cap);
  }
  return fail(TB_ERR_INVALID_ARG, "unknown tb_dtype");
}

// --------------------------------------------------- allocation-free apply --
// The apply's intermediates (one buffer per level, the whole workspace of
// tb_apply) in a file-scope device array instead of plan-owned memory, for
// callers that cannot allocate.  Each device holds its own copy of the array
// for the life of the process.  In host code its name is a host-side stand-in,
// so its device address is looked up once per device (with that device
// current) and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[TB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

static tb_status scratch_address(void** out) {
  int dev = 0;
  TB_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(TB_ERR_UNSUPPORTED, "device index beyond the allocation-free apply's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(TB_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TB_OK;
}

tb_status run_apply_noalloc(Plan& p, const void* in, void* out, long long nrhs, tb_dtype io,
                            bool adjoint, hipStream_t stream) {
  void* ws = nullptr;
  TB_TRY(scratch_address(&ws));
  return run_apply(p, in, out, nrhs, io, adjoint, stream, ws, (size_t)TB_NOALLOC_SCRATCH_BYTES);
}

// ------------------------------------------------------------ autotuner --
// For every kernel launch of both directions, in sequence order, the
// candidate configurations are timed (one fitting run, then the best of
// kTuneReps launches under HIP events, each preceded by the launches before
// it with their chosen configurations) on zero-filled buffers of the
// requested shape, and the fastest is kept in p.tuned[(io, nrhs)].
constexpr int kTuneReps = 3;

static uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ULL;
  }
  return h;
}

// Identifies the shapes of every launch: construction inputs, levels and
// every true rank.
static uint64_t plan_signature(const Plan& p) {
  uint64_t h = 1469598103934665603ULL;
  const long long head[] = {(long long)p.kind, p.d, p.leaf, p.L, p.Lt, p.Ls, p.n, p.npairs};
  h = fnv1a(h, head, sizeof(head));
  h = fnv1a(h, &p.omega, sizeof(p.omega));
  h = fnv1a(h, &p.tol, sizeof(p.tol));
  for (const auto* side : {&p.src, &p.tgt})
    for (const Level& lv : *side) {
      const long long dims[] = {lv.nitems, lv.nb, lv.R[0], lv.R[1], lv.R[2], lv.A[0], lv.A[1], lv.A[2]};
      h = fnv1a(h, dims, sizeof(dims));
      for (int k = 3; k < p.d; ++k) {
        const long long more[] = {lv.R[k], lv.A[k]};
        h = fnv1a(h, more, sizeof(more));
      }
      for (const IdRec& id : lv.ids) {
        const int rc[] = {id.r, id.c};
        h = fnv1a(h, rc, sizeof(rc));
      }
    }
  return h;
}

static std::vector<LaunchCfg> stage_candidates(long long nrhs, bool fanout, bool fp32) {
  std::vector<LaunchCfg> out;
  for (int qt : {1, 2, 4, 8}) {
    if (qt > 1 && qt > nrhs) break;
    for (int g : {1, 8})
      for (int split : {0, 1})
        for (int v : {1, 4}) {
          if (v == 4 && qt < 4) continue;  // four right-hand sides per thread
          LaunchCfg c;
          c.G = g;
          c.QT = qt;
          c.split = split;
          c.V = v;
          out.push_back(c);
        }
    if (!fanout) {
      LaunchCfg c;
      c.QT = qt;
      c.alt = 1;
      out.push_back(c);
      for (int v : {1, 4}) {  // children in turn, first mode first
        if (v == 4 && qt < 4) continue;
        LaunchCfg t;
        t.QT = qt;
        t.G = 8;
        t.alt = 2;
        t.V = v;
        out.push_back(t);
      }
    }
    if (fp32) {
      LaunchCfg c;
      c.QT = qt;
      c.mfma = 1;
      out.push_back(c);
    }
  }
  if (fp32 && nrhs >= 2) {  // 4 x 4 matrix-core blocks (d = 3 transfer levels)
    LaunchCfg c;
    c.mfma = 2;
    out.push_back(c);
  }
  if (fp32)
    for (int split : {0, 1}) {  // flat staging, one right-hand side per workgroup
      LaunchCfg c;
      c.alt = 3;
      c.split = split;
      out.push_back(c);
    }
  if (nrhs <= 4) {
    for (int split : {0, 1}) {  // register fibers, one right-hand side per workgroup
      LaunchCfg c;
      c.alt = 4;
      c.split = split;
      out.push_back(c);
    }
    for (int split : {0, 1}) {  // leaves: one workgroup of 1 or 4 waves per box (transfers reject it)
      LaunchCfg w;
      w.alt = 5;
      w.split = split;
      out.push_back(w);
    }
  }
  return out;
}

static std::vector<LaunchCfg> core_candidates(long long nrhs, tb_dtype io) {
  std::vector<LaunchCfg> out;
  LaunchCfg c;
  c.core = 1;
  out.push_back(c);
  if (nrhs >= 2) {
    c.core = 2;
    out.push_back(c);
  }
  if (io != TB_C64_OTF) {  // adjoint with 16-lane column groups (forward slots reject it)
    c.core = 8;
    out.push_back(c);
    if (nrhs >= 2) {
      c.core = 9;
      out.push_back(c);
    }
  }
  if (io != TB_C128 && io != TB_CQ16 && nrhs >= 4) {  // FP32 matrix cores (stored or on the fly)
    c.core = 3;
    out.push_back(c);
  }
  if (io == TB_CBF16 && nrhs >= 4) {
    c.core = 4;
    out.push_back(c);
    for (int v = 5; v <= 7; ++v) {  // second form, three workgroup tiles
      if (v == 6 && nrhs <= 32) continue;  // 64 right-hand sides per workgroup
      c.core = v;
      out.push_back(c);
    }
  }
  return out;
}

static bool read_cache(const char* path, uint64_t sig, int io, long long nrhs, size_t nslots,
                       std::vector<LaunchCfg>* cfg) {
  FILE* fh = std::fopen(path, "r");
  if (!fh) return false;
  char line[8192];
  bool found = false;
  while (!found && std::fgets(line, sizeof(line), fh)) {
    unsigned long long s = 0;
    int fio = 0, n = 0, pos = 0;
    long long fr = 0;
    if (std::sscanf(line, "tbtune5 %llx %d %lld %d%n", &s, &fio, &fr, &n, &pos) != 4) continue;
    if (s != sig || fio != io || fr != nrhs || (size_t)n != nslots) continue;
    std::vector<LaunchCfg> v(n);
    const char* q = line + pos;
    bool ok = true;
    for (int i = 0; i < n && ok; ++i) {
      int used = 0;
      ok = std::sscanf(q, " %d,%d,%d,%d,%d,%d,%d%n", &v[i].G, &v[i].QT, &v[i].split, &v[i].core,
                       &v[i].alt, &v[i].mfma, &v[i].V, &used) == 7;
      q += used;
    }
    if (ok) {
      *cfg = v;
      found = true;
    }
  }
  std::fclose(fh);
  return found;
}

static void append_cache(const char* path, uint64_t sig, int io, long long nrhs,
                         const std::vector<LaunchCfg>& cfg) {
  FILE* fh = std::fopen(path, "a");
  if (!fh) return;
  std::fprintf(fh, "tbtune5 %016llx %d %lld %d", (unsigned long long)sig, io, nrhs, (int)cfg.size());
  for (const LaunchCfg& c : cfg)
    std::fprintf(fh, " %d,%d,%d,%d,%d,%d,%d", c.G, c.QT, c.split, c.core, c.alt, c.mfma, c.V);
  std::fprintf(fh, "\n");
  std::fclose(fh);
}

template <class T, class CS>
static tb_status tune_typed(Plan& p, tb_dtype io, long long nrhs, hipStream_t stream,
                            std::vector<LaunchCfg>* best, int* trials) {
  using C = typename CplxOf<T>::type;
  long long ndim = 1;
  for (int k = 0; k < p.d; ++k) ndim *= p.n;
  const size_t bytes = (size_t)(nrhs * ndim) * sizeof(C);
  if (p.max_device_bytes && p.device_bytes + 2 * bytes > p.max_device_bytes)
    return fail(TB_ERR_OOM, "autotune buffers exceed the plan's device memory cap");
  void* bin = nullptr;
  void* bout = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    if (bin) (void)hipFree(bin);
    if (bout) (void)hipFree(bout);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  tb_status st = TB_OK;
  auto check = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == TB_OK) {
      (void)hipGetLastError();
      st = fail(TB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
  };
  check(hipMalloc(&bin, bytes), "autotune input");
  check(hipMalloc(&bout, bytes), "autotune output");
  check(hipEventCreate(&e0), "hipEventCreate");
  check(hipEventCreate(&e1), "hipEventCreate");
  const bool was_timing = p.timing;
  p.timing = false;
  best->assign(2 * steps_per_direction(p), LaunchCfg{});
  for (int dir = 0; dir < 2 && st == TB_OK; ++dir) {
    std::vector<Step> steps;
    st = build_steps<T, CS>(p, bin, bout, nrhs, dir == 1, io == TB_C64_OTF ? nullptr : p.cores[io], stream,
                            &steps, io == TB_C64_OTF);
    if (st != TB_OK) break;
    check(hipMemsetAsync(bin, 0, bytes, stream), "hipMemsetAsync");
    check(hipMemsetAsync(p.ws.base, 0, p.ws.bytes, stream), "hipMemsetAsync");
    const int base = dir * steps_per_direction(p);
    for (size_t i = 0; i < steps.size() && st == TB_OK; ++i) {
      const auto cands = steps[i].core ? core_candidates(nrhs, io) : stage_candidates(nrhs, steps[i].fanout, io != TB_C128);
      float best_ms = 1e30f;
      LaunchCfg pick{};
      for (const LaunchCfg& c : cands) {
        if (steps[i].run(c) != TB_OK) {  // does not fit this launch
          (void)hipGetLastError();
          continue;
        }
        float ms = 1e30f;
        for (int r = 0; r < kTuneReps && st == TB_OK; ++r) {
          // the launches before this one, with their chosen configurations,
          // so that the candidate meets the input and cache state of a real
          // apply rather than its own previous run
          for (size_t k = 0; k < i && st == TB_OK; ++k) st = steps[k].run((*best)[base + k]);
          check(hipEventRecord(e0, stream), "hipEventRecord");
          st = st == TB_OK ? steps[i].run(c) : st;
          check(hipEventRecord(e1, stream), "hipEventRecord");
          check(hipEventSynchronize(e1), "hipEventSynchronize");
          float t = 0.f;
          check(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
          ms = std::min(ms, t);
        }
        ++*trials;
        if (ms < best_ms) {
          best_ms = ms;
          pick = c;
        }
      }
      if (st == TB_OK && best_ms >= 1e29f) st = fail(TB_ERR_UNSUPPORTED, "no launch configuration fits");
      (*best)[base + i] = pick;
    }
  }
  p.timing = was_timing;
  if (st == TB_OK) check(hipStreamSynchronize(stream), "hipStreamSynchronize");
  release();
  return st;
}

tb_status run_autotune(Plan& p, long long nrhs, tb_dtype io, const char* cache, hipStream_t stream,
                       int* trials) {
  if (nrhs < 1 || nrhs > (1 << 20)) return fail(TB_ERR_INVALID_ARG, "nrhs must be in [1, 2^20]");
  if (!valid_io(io)) return fail(TB_ERR_INVALID_ARG, "unknown tb_dtype");
  if (!has_cores(p, io)) return fail(TB_ERR_INVALID_ARG, "the plan holds no cores of the requested precision");
  if (p.d > kMaxDTuned)
    return fail(TB_ERR_UNSUPPORTED, "d > 3 applies have one launch shape (nothing to tune)");
  int count = 0;
  const uint64_t sig = plan_signature(p);
  const size_t nslots = 2 * (size_t)steps_per_direction(p);
  std::vector<LaunchCfg> best;
  if (!(cache && read_cache(cache, sig, io, nrhs, nslots, &best))) {
    tb_status st = TB_OK;
    switch (io) {
      case TB_C128: st = tune_typed<double, double2>(p, io, nrhs, stream, &best, &count); break;
      case TB_C64: st = tune_typed<float, float2>(p, io, nrhs, stream, &best, &count); break;
      case TB_CBF16: st = tune_typed<float, unsigned>(p, io, nrhs, stream, &best, &count); break;
      case TB_C64_OTF: st = tune_typed<float, float2>(p, io, nrhs, stream, &best, &count); break;
      case TB_CQ16: st = tune_typed<float, Q16>(p, io, nrhs, stream, &best, &count); break;
    }
    TB_TRY(st);
    if (cache) append_cache(cache, sig, io, nrhs, best);
  }
  drop_graphs_for(&p);  // captured graphs hold the previous configurations
  p.tuned[{(int)io, nrhs}] = best;
  if (trials) *trials = count;
  return TB_OK;
}

tb_status prepare_workspace(Plan& p, long long nrhs, tb_dtype io) {
  const size_t esz = io == TB_C128 ? sizeof(double2) : sizeof(float2);
  return ensure_workspace(p, layout(p, nrhs, esz).total);
}

// ------------------------------------------------------- batched graphs --
struct GraphKey {
  std::vector<const Plan*> plans;
  std::vector<const void*> in;
  std::vector<void*> out;
  std::vector<long long> nrhs;
  int adjoint = 0;
  int io = 0;
  bool operator==(const GraphKey& o) const {
    return plans == o.plans && in == o.in && out == o.out && nrhs == o.nrhs && adjoint == o.adjoint &&
           io == o.io;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

constexpr size_t kMaxCachedGraphs = 32;
static std::recursive_mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;
static std::vector<hipStream_t> g_branch_streams;

static void destroy_entry(GraphEntry& e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  e.exec = nullptr;
  e.graph = nullptr;
}

void drop_graphs_for(const Plan* p) {
  std::lock_guard<std::recursive_mutex> lk(g_graph_mu);
  for (size_t i = 0; i < g_graphs.size();) {
    bool uses = false;
    for (const Plan* q : g_graphs[i].key.plans) uses |= q == p;
    if (uses) {
      destroy_entry(g_graphs[i]);
      g_graphs.erase(g_graphs.begin() + (long)i);
    } else {
      ++i;
    }
  }
}

static tb_status capture_batched(const GraphKey& key, std::vector<Plan*>& plans, hipStream_t stream,
                                 GraphEntry* out_entry) {
  const int np = (int)plans.size();
  while ((int)g_branch_streams.size() < np) {
    hipStream_t st = nullptr;
    TB_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    g_branch_streams.push_back(st);
  }
  // workspaces must exist before capture (no allocation inside a graph)
  for (int i = 0; i < np; ++i) TB_TRY(prepare_workspace(*plans[i], key.nrhs[i], (tb_dtype)key.io));
  TB_HIP_TRY(hipDeviceSynchronize());
  std::vector<hipEvent_t> ev(np + 1, nullptr);
  for (auto& e : ev) TB_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  auto cleanup = [&]() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  hipStream_t cap = stream;
  hipStream_t own = nullptr;
  if (cap == nullptr) {  // the legacy default stream cannot be captured
    TB_HIP_TRY(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    cap = own;
  }
  std::vector<bool> timing(np);
  for (int i = 0; i < np; ++i) {
    timing[i] = plans[i]->timing;
    plans[i]->timing = false;
  }
  tb_status st = TB_OK;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) st = fail(TB_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  if (st == TB_OK) {
    e = hipEventRecord(ev[np], cap);
    for (int i = 0; i < np && e == hipSuccess; ++i) e = hipStreamWaitEvent(g_branch_streams[i], ev[np], 0);
    if (e != hipSuccess) st = fail(TB_ERR_HIP, std::string("graph fork: ") + hipGetErrorString(e));
    std::vector<bool> joined(np, false);
    for (int i = 0; i < np && st == TB_OK; ++i) {
      st = run_apply(*plans[i], key.in[i], key.out[i], key.nrhs[i], (tb_dtype)key.io, key.adjoint != 0,
                     g_branch_streams[i]);
      if (st == TB_OK) {
        e = hipEventRecord(ev[i], g_branch_streams[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cap, ev[i], 0);
        if (e != hipSuccess) st = fail(TB_ERR_HIP, std::string("graph join: ") + hipGetErrorString(e));
        joined[i] = e == hipSuccess;
      }
    }
    // after a failure, join every forked branch back so that the capture
    // ends cleanly and the branch streams leave capture mode; the graph is
    // then discarded
    for (int i = 0; i < np; ++i)
      if (!joined[i] && hipEventRecord(ev[i], g_branch_streams[i]) == hipSuccess)
        (void)hipStreamWaitEvent(cap, ev[i], 0);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    if (st == TB_OK && e != hipSuccess)
      st = fail(TB_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    if (st == TB_OK) {
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        st = fail(TB_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        (void)hipGraphDestroy(graph);
      } else {
        out_entry->key = key;
        out_entry->graph = graph;
        out_entry->exec = exec;
      }
    } else if (graph) {
      (void)hipGraphDestroy(graph);
    }
  }
  for (int i = 0; i < np; ++i) plans[i]->timing = timing[i];
  cleanup();
  if (own) (void)hipStreamDestroy(own);
  return st;
}

tb_status run_batched(int nplans, const tb_plan* handles, const void* const* in, void* const* out,
                      const long long* nrhs, int adjoint, tb_dtype io, hipStream_t stream) {
  if (nplans < 1 || nplans > 256 || !handles || !in || !out || !nrhs)
    return fail(TB_ERR_INVALID_ARG, "tb_apply_batched: need 1..256 plans and non-null arrays");
  if (!valid_io(io)) return fail(TB_ERR_INVALID_ARG, "unknown tb_dtype");
  GraphKey key;
  std::vector<Plan*> plans;
  for (int i = 0; i < nplans; ++i) {
    Plan* p = reinterpret_cast<Plan*>(handles[i]);
    if (!p || !in[i] || !out[i]) return fail(TB_ERR_INVALID_ARG, "tb_apply_batched: null plan or array");
    if (nrhs[i] < 1 || nrhs[i] > (1 << 20)) return fail(TB_ERR_INVALID_ARG, "nrhs must be in [1, 2^20]");
    if (!has_cores(*p, io)) return fail(TB_ERR_INVALID_ARG, "a plan holds no cores of the requested precision");
    if (in[i] == out[i]) return fail(TB_ERR_INVALID_ARG, "input and output must not alias");
    for (Plan* q : plans)
      if (q == p) return fail(TB_ERR_INVALID_ARG, "tb_apply_batched: plans must be distinct");
    plans.push_back(p);
    key.plans.push_back(p);
    key.in.push_back(in[i]);
    key.out.push_back(out[i]);
    key.nrhs.push_back(nrhs[i]);
  }
  key.adjoint = adjoint ? 1 : 0;
  key.io = io;
  std::lock_guard<std::recursive_mutex> lk(g_graph_mu);
  GraphEntry* hit = nullptr;
  for (GraphEntry& e : g_graphs)
    if (e.key == key) hit = &e;
  if (!hit) {
    if (g_graphs.size() >= kMaxCachedGraphs) {  // oldest first
      destroy_entry(g_graphs.front());
      g_graphs.erase(g_graphs.begin());
    }
    GraphEntry fresh;
    TB_TRY(capture_batched(key, plans, stream, &fresh));
    g_graphs.push_back(fresh);
    hit = &g_graphs.back();
  }
  TB_HIP_TRY(hipGraphLaunch(hit->exec, stream));
  return TB_OK;
}

tb_status batched_reset() {
  std::lock_guard<std::recursive_mutex> lk(g_graph_mu);
  for (GraphEntry& e : g_graphs) destroy_entry(e);
  g_graphs.clear();
  return TB_OK;
}

}  // namespace tb

extern "C" tb_status tb_apply_batched(int nplans, const tb_plan* plans, const void* const* in,
                                      void* const* out, const long long* nrhs, int adjoint, tb_dtype io,
                                      void* hip_stream) {
  return tb::run_batched(nplans, plans, in, out, nrhs, adjoint, io, static_cast<hipStream_t>(hip_stream));
}

extern "C" tb_status tb_batched_reset(void) { return tb::batched_reset(); }

extern "C" tb_status tb_plan_set_launch(tb_plan ph, long long nrhs, tb_dtype io, int slot,
                                        const tb_launch_cfg* cfg) {
  tb::Plan* p = reinterpret_cast<tb::Plan*>(ph);
  if (!p || !cfg) return tb::fail(TB_ERR_INVALID_ARG, "null plan or configuration");
  if (nrhs < 1 || nrhs > (1 << 20)) return tb::fail(TB_ERR_INVALID_ARG, "nrhs must be in [1, 2^20]");
  if (!tb::valid_io(io)) return tb::fail(TB_ERR_INVALID_ARG, "unknown tb_dtype");
  const int nslots = 2 * tb::steps_per_direction(*p);
  if (slot < 0 || slot >= nslots) return tb::fail(TB_ERR_INVALID_ARG, "launch slot out of range");
  const int g = cfg->outputs_per_thread, q = cfg->rhs_tile;
  if (!(g == 0 || g == 1 || g == 8) || !(q == 0 || q == 1 || q == 2 || q == 4 || q == 8) ||
      cfg->whole_blocks < 0 || cfg->whole_blocks > 1 || cfg->core_kernel < 0 || cfg->core_kernel > 9 ||
      cfg->fanin_in_turn < 0 || cfg->fanin_in_turn > 2 || cfg->transfer_mfma < 0 || cfg->transfer_mfma > 2 ||
      !(cfg->rhs_per_thread == 0 || cfg->rhs_per_thread == 1 || cfg->rhs_per_thread == 4) ||
      cfg->flat_stage < 0 || cfg->flat_stage > 3 || (cfg->flat_stage && cfg->fanin_in_turn))
    return tb::fail(TB_ERR_INVALID_ARG, "launch configuration field out of range");
  auto& v = p->tuned[{(int)io, nrhs}];
  if ((int)v.size() != nslots) v.assign(nslots, tb::LaunchCfg{});
  tb::LaunchCfg c;
  c.G = g;
  c.QT = q;
  c.split = cfg->whole_blocks;
  c.core = cfg->core_kernel;
  c.alt = cfg->flat_stage == 3 ? 5 : cfg->flat_stage == 2 ? 4 : cfg->flat_stage ? 3 : cfg->fanin_in_turn;
  c.mfma = cfg->transfer_mfma;
  c.V = cfg->rhs_per_thread;
  v[slot] = c;
  tb::drop_graphs_for(p);
  return TB_OK;
}

extern "C" tb_status tb_plan_autotune(tb_plan ph, long long nrhs, tb_dtype io, const char* cache_path,
                                      void* hip_stream, int* trials) {
  tb::Plan* p = reinterpret_cast<tb::Plan*>(ph);
  if (!p) return tb::fail(TB_ERR_INVALID_ARG, "null plan");
  return tb::run_autotune(*p, nrhs, io, cache_path, static_cast<hipStream_t>(hip_stream), trials);
}

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

extern "C" tb_status tb_apply_noalloc(tb_plan ph, const void* in, void* out, long long nrhs, tb_dtype io,
                                      int adjoint, void* hip_stream) {
  if (!ph) return tb::fail(TB_ERR_INVALID_ARG, "tb_apply_noalloc: null plan");
  return tb::run_apply_noalloc(*reinterpret_cast<tb::Plan*>(ph), in, out, nrhs, io, adjoint != 0,
                               static_cast<hipStream_t>(hip_stream));
}
