// Flat-staged transfer stages: one right-hand side per workgroup
// (Algorithm 2 steps 1 and 3, and the same stages of the adjoint).
//
// At one right-hand side a transfer block holds a few thousand entries and
// its mode products a few tens of thousands of multiply-adds, so a kernel
// that reads its block from global memory inside the first mode product
// waits on one memory round trip per contracted index.  Here a workgroup
// first loads everything it reads into LDS in one pass:
//
//   fan-out  the coarse block (the padded box A_0 x .. x A_{D-1}), the rows
//            of M_0 in its slice and the whole M_1 .. M_{D-1};
//   fan-in   the padded fine blocks (R_0 x .. x R_{D-1}) of all 2^D
//            children and, per child, the slice's columns of M_0 and the
//            whole M_1 .. M_{D-1};
//
// with kFlatU loads in flight per thread before any LDS store.  Every
// address of that pass depends only on launch-uniform values, so the true
// ranks and the coarse block's segments are read in the same memory round
// trip.  The D mode products then run from LDS over true extents only (the
// padding of the staged boxes is never read), and the last one writes
// global memory.
//
// Slices run over padded positions of the first output mode (fan-out: the
// fine rows, fan-in: the coarse rows), so that a slice's matrix rows or
// columns are known before the ranks are.
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace tb {

constexpr int kFlatThreads = 512;
constexpr int kFlatU = 16;  // staging loads in flight per thread

// q = e / m, r = e - q m for 0 <= e < 2^22 and 1 <= m <= 2^16, through an
// FP32 reciprocal: the rounding errors of e * (1/m) stay below 1/m, so the
// floor is exact.
struct FDiv {
  int m;
  float inv;
  __device__ void init(int mm) {
    m = mm;
    inv = 1.0f / (float)mm;
  }
  __device__ int quot(int e) const {
    int q = (int)((float)e * inv);
    const int r = e - q * m;  // fix the rare off-by-one at exact multiples
    return r < 0 ? q - 1 : (r >= m ? q + 1 : q);
  }
};

// Sum over the true positions of a coarse block's mode: the first child's
// [0, h1) and the second child's [off2, off2 + c - h1).
template <class C, class F>
__device__ __forceinline__ C seg_sum(C acc, const Seg& s, F term) {
#pragma unroll 4
  for (int p = 0; p < s.h1; ++p) acc = term(acc, p);
  const int e2 = s.off2 + (s.c - s.h1);
#pragma unroll 4
  for (int p = s.off2; p < e2; ++p) acc = term(acc, p);
  return acc;
}

// Compact index of padded position p of a coarse block's mode, or -1 for
// padding.
__device__ __forceinline__ int seg_compact(const Seg& s, int p) {
  if (p < s.h1) return p;
  const int j = s.h1 + (p - s.off2);
  return (p >= s.off2 && j < s.c) ? j : -1;
}

// ------------------------------------------------------------- fan-out --
// fine(a_0.., q) = sum_j prod_k M_k[a_k][j_k] coarse(j_0.., q) over the
// coarse block's true positions, for fine rows a_0 in this workgroup's
// slice [lo, lo + chunk) below the true rank r_0.
template <class T, int D>
__global__ void __launch_bounds__(kFlatThreads)
    stage_fanout_flat(StageArgs a, const typename CplxOf<T>::type* __restrict__ coarse,
                      typename CplxOf<T>::type* __restrict__ fine,
                      const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const StageBid sb = stage_bid(a, 1);
  const int fi = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  const int lo = sb.split * a.chunk;
  const int nrow = min(a.chunk, a.R[0] - lo);  // padded fine rows of the slice
  const int citem = a.coarse_global ? (fi >> (D * a.lvl)) : parent_of<D>(fi, a.lvl);
  const int q0 = sb.q0;
  CoarseAddr<D> ca;
  ca.init(a, citem, beta, q0);
  const C* mb = mats + (long long)fi * a.mat_item_stride;
  const C* mk[D];
#pragma unroll
  for (int k = 0; k < D; ++k) mk[k] = mb + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
  // LDS: X box (A_0 .. A_{D-1}) | M0 slice (nrow x A_0) | M_1 (R_1 x A_1)
  //      [| M_2 (R_2 x A_2)] | B1 (chunk x c_1 [x c_2])
  const int A0 = a.A[0], A1 = a.A[1], A2 = D == 3 ? a.A[2] : 1;
  const int nX = A0 * A1 * A2;
  const int nM0 = nrow * A0;
  const int nM1 = a.R[1] * A1;
  const int nM2 = D == 3 ? a.R[2] * A2 : 0;
  C* X = sm;
  C* M0 = X + nX;
  C* M1 = M0 + nM0;
  C* M2 = M1 + nM1;
  C* B1 = X + nX + a.chunk * A0 + nM1 + nM2;
  const int total = nX + nM0 + nM1 + nM2;
  const int conj = a.conj;
  FDiv dA2, dA1;
  dA2.init(A2);
  dA1.init(A1);
  // true ranks and segments, read in the same round trip as the staging
  int r[D];
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
  Seg sg[D];
  coarse_segs<D>(a, citem, beta, sg);
  const long long s0 = ca.stride[0], s1 = ca.stride[1], s2 = D == 3 ? ca.stride[D - 1] : 0;
  for (int e0 = threadIdx.x; e0 < total; e0 += kFlatU * kFlatThreads) {
    const C* p[kFlatU];
#pragma unroll
    for (int u = 0; u < kFlatU; ++u) {
      const int e = e0 + u * kFlatThreads;
      const C* q = mb;
      if (e < nX) {
        const int row = D == 3 ? dA2.quot(e) : e;
        const int p2 = e - row * A2;
        const int p0 = dA1.quot(row);
        const int p1 = row - p0 * A1;
        q = coarse + ca.base + p0 * s0 + p1 * s1 + (D == 3 ? p2 * s2 : 0);
      } else if (e < nX + nM0) {
        q = mk[0] + (long long)lo * A0 + (e - nX);
      } else if (e < nX + nM0 + nM1) {
        q = mk[1] + (e - nX - nM0);
      } else if (e < total) {
        q = mk[D - 1] + (e - nX - nM0 - nM1);
      }
      p[u] = q;
    }
    C v[kFlatU];
#pragma unroll
    for (int u = 0; u < kFlatU; ++u) v[u] = *p[u];
#pragma unroll
    for (int u = 0; u < kFlatU; ++u) {
      const int e = e0 + u * kFlatThreads;
      if (e < total) {
        C x = v[u];
        if (conj && e >= nX) x.y = -x.y;
        sm[e] = x;
      }
    }
  }
  __syncthreads();
  const int na = min(nrow, r[0] - lo);
  if (na <= 0) return;  // uniform over the workgroup: no barrier follows for it
  const int c1 = sg[1].c;
  long long fs[D];
  const long long fb = fine_base<D>(a, fi, beta, q0, fs);
  if constexpr (D == 2) {
    // B1[ai][j1] = sum_j0 M0[lo+ai][j0] X[j0][j1]
    for (int idx = threadIdx.x; idx < na * c1; idx += kFlatThreads) {
      const int ai = idx / c1, j1 = idx - ai * c1;
      const int p1 = sg[1].pos(j1);
      const C* m = M0 + ai * A0;
      B1[idx] = seg_sum(czero<C>(), sg[0], [&](C acc, int p0) { return cfma(acc, m[p0], X[p0 * A1 + p1]); });
    }
    __syncthreads();
    // fine[lo+ai][a1] = sum_j1 M1[a1][j1] B1[ai][j1]
    for (int idx = threadIdx.x; idx < na * r[1]; idx += kFlatThreads) {
      const int ai = idx / r[1], a1 = idx - ai * r[1];
      const C* m = M1 + a1 * A1;
      const C* b = B1 + ai * c1;
      C acc = czero<C>();
      int j1 = 0;
      acc = seg_sum(acc, sg[1], [&](C s, int p1) { return cfma(s, m[p1], b[j1++]); });
      fine[fb + (long long)(lo + ai) * fs[0] + (long long)a1 * fs[1]] = acc;
    }
  } else {
    const int c2 = sg[2].c;
    // B1[ai][j1][j2] = sum_j0 M0[lo+ai][j0] X[j0][j1][j2]
    for (int idx = threadIdx.x; idx < na * c1 * c2; idx += kFlatThreads) {
      const int t = idx / c2, j2 = idx - t * c2;
      const int ai = t / c1, j1 = t - ai * c1;
      const C* x = X + sg[1].pos(j1) * A2 + sg[2].pos(j2);
      const C* m = M0 + ai * A0;
      const int pl = A1 * A2;
      B1[idx] = seg_sum(czero<C>(), sg[0], [&](C acc, int p0) { return cfma(acc, m[p0], x[p0 * pl]); });
    }
    __syncthreads();
    // B2[ai][a1][j2] = sum_j1 M1[a1][j1] B1[ai][j1][j2]; X is free now
    C* B2 = X;
    for (int idx = threadIdx.x; idx < na * r[1] * c2; idx += kFlatThreads) {
      const int t = idx / c2, j2 = idx - t * c2;
      const int ai = t / r[1], a1 = t - ai * r[1];
      const C* m = M1 + a1 * A1;
      const C* b = B1 + (ai * c1) * c2 + j2;
      int j1 = 0;
      B2[idx] = seg_sum(czero<C>(), sg[1], [&](C s, int p1) {
        const C v = cfma(s, m[p1], b[j1 * c2]);
        ++j1;
        return v;
      });
    }
    __syncthreads();
    // fine[lo+ai][a1][a2] = sum_j2 M2[a2][j2] B2[ai][a1][j2]
    for (int idx = threadIdx.x; idx < na * r[1] * r[2]; idx += kFlatThreads) {
      const int t = idx / r[2], a2 = idx - t * r[2];
      const int ai = t / r[1], a1 = t - ai * r[1];
      const C* m = M2 + a2 * A2;
      const C* b = B2 + (ai * r[1] + a1) * c2;
      int j2 = 0;
      const C acc = seg_sum(czero<C>(), sg[2], [&](C s, int p2) { return cfma(s, m[p2], b[j2++]); });
      fine[fb + (long long)(lo + ai) * fs[0] + (long long)a1 * fs[1] + (long long)a2 * fs[2]] = acc;
    }
  }
}

// -------------------------------------------------------------- fan-in --
// coarse(p_0.., q) = sum_children sum_j prod_k M_k(c)[j_k][p_k] fine_c(j, q)
// for the coarse block's true positions, p_0 in this workgroup's slice of
// padded rows [plo, plo + chunk).
template <class T, int D>
__global__ void __launch_bounds__(kFlatThreads)
    stage_fanin_flat(StageArgs a, const typename CplxOf<T>::type* __restrict__ fine,
                     typename CplxOf<T>::type* __restrict__ coarse,
                     const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const StageBid sb = stage_bid(a, 1);
  const int ci = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  const int plo = sb.split * a.chunk;
  const int nrow = min(a.chunk, a.A[0] - plo);  // padded coarse rows of the slice
  const int q0 = sb.q0;
  const int nch = a.coarse_global ? 1 : (1 << D);
  const int R0 = a.R[0], R1 = a.R[1], R2 = D == 3 ? a.R[2] : 1;
  const int A0 = a.A[0], A1 = a.A[1], A2 = D == 3 ? a.A[2] : 1;
  // per child, in LDS at stride per_child: the fine box (R0 R1 [R2]), the
  // slice's columns of M0 as [pi][j0] (nrow x R0), M1 (R1 x A1), M2 (R2 x A2)
  const int box = R0 * R1 * R2;
  const int offM0 = box, offM1 = box + nrow * R0, offM2 = offM1 + R1 * A1;
  const int per_child = offM2 + (D == 3 ? R2 * A2 : 0);
  const int total = nch * per_child;
  __shared__ long long cfb[kMaxChildren], cmb[kMaxChildren];
  __shared__ int crk[kMaxChildren][kMaxD];
  long long fs[D];
  (void)fine_base<D>(a, 0, beta, 0, fs);  // strides only
  if (threadIdx.x < nch) {
    const int c = threadIdx.x;
    const int fi = a.coarse_global ? ci : child_of<D>(ci, a.lvl, c);
    long long fs_[D];
    cfb[c] = fine_base<D>(a, fi, beta, q0, fs_);
    cmb[c] = (long long)fi * a.mat_item_stride;
  }
  __syncthreads();
  if (threadIdx.x < nch) {  // ranks: loaded beside the staging loads
    const int c = threadIdx.x;
    const int fi = a.coarse_global ? ci : child_of<D>(ci, a.lvl, c);
#pragma unroll
    for (int k = 0; k < D; ++k) crk[c][k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
  }
  Seg sg[D];
  coarse_segs<D>(a, ci, beta, sg);
  FDiv dPC, dR2, dR1, dR0;
  dPC.init(per_child);
  dR2.init(R2);
  dR1.init(R1);
  dR0.init(R0);
  const long long k0 = a.mat_k_off[0] + (long long)beta[0] * R0 * A0;
  const long long k1 = a.mat_k_off[1] + (long long)beta[1] * R1 * A1;
  const long long k2 = a.mat_k_off[D - 1] + (long long)beta[D - 1] * a.R[D - 1] * a.A[D - 1];
  const int conj = a.conj;
  for (int e0 = threadIdx.x; e0 < total; e0 += kFlatU * kFlatThreads) {
    const C* p[kFlatU];
#pragma unroll
    for (int u = 0; u < kFlatU; ++u) {
      const int e = e0 + u * kFlatThreads;
      const C* q = mats;
      if (e < total) {
        const int c = dPC.quot(e);
        const int i = e - c * per_child;
        if (i < box) {
          const int row = D == 3 ? dR2.quot(i) : i;
          const int j2 = i - row * R2;
          const int j0 = dR1.quot(row);
          const int j1 = row - j0 * R1;
          q = fine + cfb[c] + j0 * fs[0] + j1 * fs[1] + (D == 3 ? j2 * fs[D - 1] : 0);
        } else if (i < offM1) {  // M0(c)[j0][plo + pi] into slot [pi][j0]
          const int ii = i - offM0;
          const int pi = dR0.quot(ii), j0 = ii - pi * R0;
          q = mats + cmb[c] + k0 + (long long)j0 * A0 + plo + pi;
        } else if (i < offM2) {
          q = mats + cmb[c] + k1 + (i - offM1);
        } else {
          q = mats + cmb[c] + k2 + (i - offM2);
        }
      }
      p[u] = q;
    }
    C v[kFlatU];
#pragma unroll
    for (int u = 0; u < kFlatU; ++u) v[u] = *p[u];
#pragma unroll
    for (int u = 0; u < kFlatU; ++u) {
      const int e = e0 + u * kFlatThreads;
      if (e < total) {
        C x = v[u];
        if (conj && e - dPC.quot(e) * per_child >= box) x.y = -x.y;
        sm[e] = x;
      }
    }
  }
  C* Bst = sm + total;  // B1 (nch x nrow x R1 [x R2]), then B2
  __syncthreads();
  const int c1 = sg[1].c;
  CoarseAddr<D> ca;
  ca.init(a, ci, beta, q0);
  if constexpr (D == 2) {
    // B1[c][pi][j1] = sum_j0 M0_c[j0][plo+pi] X_c[j0][j1]
    const int per_c = nrow * R1;
    for (int idx = threadIdx.x; idx < nch * per_c; idx += kFlatThreads) {
      const int t = idx / R1, j1 = idx - t * R1;
      const int c = t / nrow, pi = t - c * nrow;
      if (j1 >= crk[c][1] || seg_compact(sg[0], plo + pi) < 0) continue;
      const C* m = sm + c * per_child + offM0 + pi * R0;
      const C* x = sm + c * per_child + j1;
      const int r0 = crk[c][0];
      C acc = czero<C>();
#pragma unroll 4
      for (int j0 = 0; j0 < r0; ++j0) acc = cfma(acc, m[j0], x[j0 * R1]);
      Bst[idx] = acc;
    }
    __syncthreads();
    // coarse[plo+pi][a1] = sum_c sum_j1 M1_c[j1][a1] B1[c][pi][j1]
    for (int idx = threadIdx.x; idx < nrow * c1; idx += kFlatThreads) {
      const int pi = idx / c1, a1 = idx - pi * c1;
      if (seg_compact(sg[0], plo + pi) < 0) continue;
      const int p1 = sg[1].pos(a1);
      C acc = czero<C>();
      for (int c = 0; c < nch; ++c) {
        const C* m = sm + c * per_child + offM1 + p1;
        const C* b = Bst + (c * nrow + pi) * R1;
        const int r1 = crk[c][1];
#pragma unroll 4
        for (int j1 = 0; j1 < r1; ++j1) acc = cfma(acc, m[j1 * A1], b[j1]);
      }
      coarse[ca.base + (long long)(plo + pi) * ca.stride[0] + (long long)p1 * ca.stride[1]] = acc;
    }
  } else {
    const int c2 = sg[2].c;
    // B1[c][pi][j1][j2] = sum_j0 M0_c[j0][plo+pi] X_c[j0][j1][j2]
    const int per_c1 = nrow * R1 * R2;
    for (int idx = threadIdx.x; idx < nch * per_c1; idx += kFlatThreads) {
      const int t = idx / R2, j2 = idx - t * R2;
      const int t2 = t / R1, j1 = t - t2 * R1;
      const int c = t2 / nrow, pi = t2 - c * nrow;
      if (j1 >= crk[c][1] || j2 >= crk[c][2] || seg_compact(sg[0], plo + pi) < 0) continue;
      const C* m = sm + c * per_child + offM0 + pi * R0;
      const C* x = sm + c * per_child + j1 * R2 + j2;
      const int r0 = crk[c][0], pl = R1 * R2;
      C acc = czero<C>();
#pragma unroll 4
      for (int j0 = 0; j0 < r0; ++j0) acc = cfma(acc, m[j0], x[j0 * pl]);
      Bst[idx] = acc;
    }
    __syncthreads();
    // B2[c][pi][a1][j2] = sum_j1 M1_c[j1][a1] B1[c][pi][j1][j2]
    C* B2 = Bst + nch * per_c1;
    const int per_c2 = nrow * c1 * R2;
    for (int idx = threadIdx.x; idx < nch * per_c2; idx += kFlatThreads) {
      const int t = idx / R2, j2 = idx - t * R2;
      const int t2 = t / c1, a1 = t - t2 * c1;
      const int c = t2 / nrow, pi = t2 - c * nrow;
      if (j2 >= crk[c][2] || seg_compact(sg[0], plo + pi) < 0) continue;
      const C* m = sm + c * per_child + offM1 + sg[1].pos(a1);
      const C* b = Bst + ((c * nrow + pi) * R1) * R2 + j2;
      const int r1 = crk[c][1];
      C acc = czero<C>();
#pragma unroll 4
      for (int j1 = 0; j1 < r1; ++j1) acc = cfma(acc, m[j1 * A1], b[j1 * R2]);
      B2[idx] = acc;
    }
    __syncthreads();
    // coarse[plo+pi][a1][a2] = sum_c sum_j2 M2_c[j2][a2] B2[c][pi][a1][j2]
    for (int idx = threadIdx.x; idx < nrow * c1 * c2; idx += kFlatThreads) {
      const int t = idx / c2, a2 = idx - t * c2;
      const int pi = t / c1, a1 = t - pi * c1;
      if (seg_compact(sg[0], plo + pi) < 0) continue;
      const int p2 = sg[2].pos(a2);
      C acc = czero<C>();
      for (int c = 0; c < nch; ++c) {
        const C* m = sm + c * per_child + offM2 + p2;
        const C* b = B2 + ((c * nrow + pi) * c1 + a1) * R2;
        const int r2 = crk[c][2];
#pragma unroll 4
        for (int j2 = 0; j2 < r2; ++j2) acc = cfma(acc, m[j2 * A2], b[j2]);
      }
      coarse[ca.base + (long long)(plo + pi) * ca.stride[0] + (long long)sg[1].pos(a1) * ca.stride[1] +
             (long long)p2 * ca.stride[2]] = acc;
    }
  }
}

// ---------------------------------------------------------------- host --
// LDS elements of one flat workgroup for slices of `chunk` padded rows
// (padded extents bound the true ones).
long long flat_lds_elems(const StageArgs& a, int d, bool fanout, int chunk) {
  const long long R1 = a.R[1], R2 = d == 3 ? a.R[2] : 1;
  const long long A0 = a.A[0], A1 = a.A[1], A2 = d == 3 ? a.A[2] : 1;
  if (fanout)  // X box, M0 slice, M1, M2, B1 (B2 reuses X)
    return A0 * A1 * A2 + chunk * A0 + R1 * A1 + (d == 3 ? R2 * A2 : 0) + chunk * A1 * A2;
  const long long nch = a.coarse_global ? 1 : (1LL << d);
  const long long per_child = (long long)a.R[0] * R1 * R2 + (long long)a.R[0] * chunk + R1 * A1 +
                              (d == 3 ? R2 * A2 : 0);
  long long e = nch * per_child + nch * chunk * R1 * R2;
  if (d == 3) e += nch * chunk * A1 * R2;
  return e;
}

template <class T, int D>
static tb_status launch_flat_d(const StageArgs& a, bool fanout, dim3 grid, size_t lds, const void* in,
                               void* out, const void* mats, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  const void* k = fanout ? reinterpret_cast<const void*>(stage_fanout_flat<T, D>)
                         : reinterpret_cast<const void*>(stage_fanin_flat<T, D>);
  if (lds > 65536)
    TB_HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (fanout)
    stage_fanout_flat<T, D><<<grid, kFlatThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
  else
    stage_fanin_flat<T, D><<<grid, kFlatThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

constexpr long long kFlatTargetWg = 1024;

tb_status launch_stage_flat_f32(StageArgs a, int d, bool fanout, int n_items, const void* in, void* out,
                                const void* mats, hipStream_t stream, int mode, int lds_limit) {
  const long long blocks = (long long)n_items * a.nblk * a.nrhs;
  const int dim = fanout ? a.R[0] : a.A[0];
  const long long budget = std::min<long long>(lds_limit, 80 * 1024);
  // mode 1: slices sized for about kFlatTargetWg workgroups; mode 2: whole
  // blocks where the LDS allows
  int chunk = dim;
  if (mode == 1) chunk = (int)std::max<long long>(1, (dim * blocks + kFlatTargetWg - 1) / kFlatTargetWg);
  chunk = std::max(1, std::min(chunk, dim));
  while (chunk > 1 && flat_lds_elems(a, d, fanout, chunk) * (long long)sizeof(float2) > budget) --chunk;
  const size_t lds = (size_t)flat_lds_elems(a, d, fanout, chunk) * sizeof(float2);
  if (lds > (size_t)lds_limit) return fail(TB_ERR_UNSUPPORTED, "flat stage exceeds the LDS of a workgroup");
  // the staging's FP32-reciprocal divisions need indices below 2^22
  if (flat_lds_elems(a, d, fanout, chunk) >= (1LL << 22))
    return fail(TB_ERR_UNSUPPORTED, "flat stage block too large");
  a.chunk = chunk;
  a.nsplit = (dim + chunk - 1) / chunk;
  const long long nwg = blocks * a.nsplit;
  if (nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many right-hand sides for one launch");
  dim3 grid((unsigned)nwg);
  return d == 2 ? launch_flat_d<float, 2>(a, fanout, grid, lds, in, out, mats, stream)
                : launch_flat_d<float, 3>(a, fanout, grid, lds, in, out, mats, stream);
}

}  // namespace tb
