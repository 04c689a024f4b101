// Register-fiber transfer stages: one right-hand side per workgroup
// (Algorithm 2 steps 1 and 3, and the same stages of the adjoint).
//
// At one right-hand side a transfer block holds a few thousand entries and
// its mode products a few tens of thousands of multiply-adds, so a stage
// lasts about as long as one workgroup: the sum of its dependent memory
// round trips and of its dependent LDS reads.  Here every mode product is
// cut into fibers of its contracted mode.  A thread loads one fiber into
// registers, all of its loads issued together, then forms that fiber's
// outputs with the matrix read from LDS; the matrix reads of one output do
// not depend on each other, so they are in flight together as well.  A
// product with few fibers gives each fiber's outputs to several threads.
// The first mode's fibers come from global memory and are requested before
// the matrices are staged, so that one memory round trip serves both:
//
//   fan-out  first-mode fibers of the coarse block (its true positions);
//            M_0 (the rows of this workgroup's slice) and M_1 .. M_{D-1},
//            transposed and compact in LDS; the intermediates in LDS; the
//            last mode writes the fine block;
//   fan-in   first-mode fibers of every child's fine block; the children's
//            matrices in LDS; the last mode sums over the children, kFibG
//            outputs per thread, and writes the coarse block.
//
// A fiber is an array of XM registers (a template parameter, at least the
// longest contracted extent of the launch).  Its entries past the true
// length are zero and meet a valid matrix row (the last true one), so every
// read of the dot product is unconditional and the padding adds zeros.
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace tb {

constexpr int kFibU = 8;  // staging loads in flight per thread
constexpr int kFibG = 4;  // outputs per thread of the fan-in's last mode

// Work items of one mode product: nfib fibers times ngrp groups of their
// outputs (group g takes outputs g, g + ngrp, ...).  Fibers run fastest
// over the threads, so that the lanes of a wave mostly share an output
// index and read the same matrix entries.
struct FibItems {
  int nfib, ngrp, n;
  __device__ FibItems(int nf, int nout) : nfib(nf) {
    ngrp = nf > 0 ? max(1, min(nout, kThreads / nf)) : 1;
    n = nf * ngrp;
  }
};

// x[j] = at(j) for j < len, zero after.
template <int XM, class C, class AF>
__device__ __forceinline__ void fiber_load(C (&x)[XM], int len, AF at) {
#pragma unroll
  for (int j = 0; j < XM; ++j) x[j] = j < len ? at(j) : czero<C>();
}

// acc + sum_{j < len} m(j) x[j]; rows past len repeat row len - 1 (a finite
// value times a zero entry of x).
template <int XM, class C, class MF>
__device__ __forceinline__ C fiber_dot(C acc, const C (&x)[XM], int len, MF m) {
  if (len <= 0) return acc;
  const int jl = len - 1;
#pragma unroll
  for (int j = 0; j < XM; ++j) acc = cfma(acc, m(min(j, jl)), x[j]);
  return acc;
}

// ------------------------------------------------------------- fan-out --
// fine(a_0.., q) = sum_j prod_k M_k[a_k][j_k] coarse(j_0.., q) over the
// coarse block's true positions, fine rows a_0 in this workgroup's slice.
template <class T, int D, int XM>
__global__ void __launch_bounds__(kThreads)
    stage_fanout_fib(StageArgs a, const typename CplxOf<T>::type* __restrict__ coarse,
                     typename CplxOf<T>::type* __restrict__ fine,
                     const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const StageBid sb = stage_bid(a, 1);
  const int fi = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  int r[D];
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
  const int lo = sb.split * a.chunk;
  const int na = min(r[0], lo + a.chunk) - lo;
  const int citem = a.coarse_global ? (fi >> (D * a.lvl)) : parent_of<D>(fi, a.lvl);
  Seg sg[D];
  coarse_segs<D>(a, citem, beta, sg);  // loads issued with the fine ranks'
  if (na <= 0) return;                 // uniform over the workgroup
  CoarseAddr<D> ca;
  ca.init(a, citem, beta, sb.q0);
  long long fs[D];
  const long long fb = fine_base<D>(a, fi, beta, sb.q0, fs);
  const int chunk = a.chunk, A0 = a.A[0], A1 = a.A[1], A2 = D == 3 ? a.A[2] : 1;
  const int R1 = a.R[1], R2 = D == 3 ? a.R[2] : 1;
  const int c0 = sg[0].c, c1 = sg[1].c, c2 = D == 3 ? sg[2].c : 1;
  // LDS: Mt0 [A0][chunk] | Mt1 [A1][R1] | Mt2 [A2][R2] | B1 [chunk][A1][A2] | B2 [chunk][R1][A2]
  // with Mt_k[j][o] = M_k[row o][true column j], conjugated for the adjoint
  C* Mt0 = sm;
  C* Mt1 = Mt0 + A0 * chunk;
  C* Mt2 = Mt1 + A1 * R1;
  C* B1 = Mt2 + (D == 3 ? A2 * R2 : 0);
  C* B2 = B1 + chunk * A1 * A2;

  // first mode: fibers (j1, j2) of the coarse block
  const FibItems m0(c1 * c2, na);
  C x[XM];
  auto load0 = [&](int it) {
    const int f = it % m0.nfib;
    const int j1 = f / c2, j2 = f - j1 * c2;
    long long base = ca.base + (long long)sg[1].pos(j1) * ca.stride[1];
    if constexpr (D == 3) base += (long long)sg[2].pos(j2) * ca.stride[2];
    const C* src = coarse + base;
    const long long s0 = ca.stride[0];
    fiber_load<XM>(x, c0, [&](int j) { return src[sg[0].pos(j) * s0]; });
  };
  if (threadIdx.x < m0.n) load0(threadIdx.x);

  // the matrices, all modes in one pass, kFibU loads in flight per thread
  {
    const C* mb = mats + (long long)fi * a.mat_item_stride;
    const long long mo0 = a.mat_k_off[0] + (long long)beta[0] * a.R[0] * A0;
    const long long mo1 = a.mat_k_off[1] + (long long)beta[1] * R1 * A1;
    const long long mo2 = D == 3 ? a.mat_k_off[D - 1] + (long long)beta[D - 1] * R2 * A2 : 0;
    const int n0 = c0 * na, n1 = c1 * r[1], n2 = D == 3 ? c2 * r[D - 1] : 0;
    const int ntot = n0 + n1 + n2;
    for (int e0 = threadIdx.x; e0 < ntot; e0 += kFibU * kThreads) {
      C v[kFibU];
      int dst[kFibU];
#pragma unroll
      for (int u = 0; u < kFibU; ++u) {
        const int e = e0 + u * kThreads;
        dst[u] = -1;
        if (e < n0) {
          const int j = e / na, o = e - j * na;
          v[u] = mb[mo0 + (long long)(lo + o) * A0 + sg[0].pos(j)];
          dst[u] = j * chunk + o;
        } else if (e < n0 + n1) {
          const int i = e - n0, j = i / r[1], o = i - j * r[1];
          v[u] = mb[mo1 + (long long)o * A1 + sg[1].pos(j)];
          dst[u] = (int)(Mt1 - sm) + j * R1 + o;
        } else if (e < ntot) {
          const int i = e - n0 - n1, j = i / r[D - 1], o = i - j * r[D - 1];
          v[u] = mb[mo2 + (long long)o * A2 + sg[D - 1].pos(j)];
          dst[u] = (int)(Mt2 - sm) + j * R2 + o;
        }
      }
#pragma unroll
      for (int u = 0; u < kFibU; ++u)
        if (dst[u] >= 0) {
          C t = v[u];
          if (a.conj) t.y = -t.y;
          sm[dst[u]] = t;
        }
    }
  }
  __syncthreads();

  if constexpr (D == 2) {
    // B1[ai][j1] = sum_j0 M0[lo+ai][j0] coarse(j0, j1)
    for (int it = threadIdx.x; it < m0.n; it += kThreads) {
      if (it != (int)threadIdx.x) load0(it);
      const int j1 = it % m0.nfib, g = it / m0.nfib;
      for (int ai = g; ai < na; ai += m0.ngrp)
        B1[ai * A1 + j1] = fiber_dot<XM>(czero<C>(), x, c0, [&](int j) { return Mt0[j * chunk + ai]; });
    }
    __syncthreads();
    // fine[lo+ai][a1] = sum_j1 M1[a1][j1] B1[ai][j1]
    const FibItems m1(na, r[1]);
    for (int it = threadIdx.x; it < m1.n; it += kThreads) {
      const int ai = it % m1.nfib, g = it / m1.nfib;
      fiber_load<XM>(x, c1, [&](int j) { return B1[ai * A1 + j]; });
      C* dst = fine + fb + (long long)(lo + ai) * fs[0];
      for (int a1 = g; a1 < r[1]; a1 += m1.ngrp)
        dst[(long long)a1 * fs[1]] = fiber_dot<XM>(czero<C>(), x, c1, [&](int j) { return Mt1[j * R1 + a1]; });
    }
  } else {
    // B1[ai][j1][j2] = sum_j0 M0[lo+ai][j0] coarse(j0, j1, j2)
    for (int it = threadIdx.x; it < m0.n; it += kThreads) {
      if (it != (int)threadIdx.x) load0(it);
      const int f = it % m0.nfib, g = it / m0.nfib;
      const int j1 = f / c2, j2 = f - j1 * c2;
      for (int ai = g; ai < na; ai += m0.ngrp)
        B1[(ai * A1 + j1) * A2 + j2] =
            fiber_dot<XM>(czero<C>(), x, c0, [&](int j) { return Mt0[j * chunk + ai]; });
    }
    __syncthreads();
    // B2[ai][a1][j2] = sum_j1 M1[a1][j1] B1[ai][j1][j2]
    const FibItems m1(na * c2, r[1]);
    for (int it = threadIdx.x; it < m1.n; it += kThreads) {
      const int f = it % m1.nfib, g = it / m1.nfib;
      const int ai = f / c2, j2 = f - ai * c2;
      const C* src = B1 + ai * A1 * A2 + j2;
      fiber_load<XM>(x, c1, [&](int j) { return src[j * A2]; });
      for (int a1 = g; a1 < r[1]; a1 += m1.ngrp)
        B2[(ai * R1 + a1) * A2 + j2] = fiber_dot<XM>(czero<C>(), x, c1, [&](int j) { return Mt1[j * R1 + a1]; });
    }
    __syncthreads();
    // fine[lo+ai][a1][a2] = sum_j2 M2[a2][j2] B2[ai][a1][j2]
    const FibItems m2(na * r[1], r[2]);
    for (int it = threadIdx.x; it < m2.n; it += kThreads) {
      const int f = it % m2.nfib, g = it / m2.nfib;
      const int ai = f / r[1], a1 = f - ai * r[1];
      const C* src = B2 + (ai * R1 + a1) * A2;
      fiber_load<XM>(x, c2, [&](int j) { return src[j]; });
      C* dst = fine + fb + (long long)(lo + ai) * fs[0] + (long long)a1 * fs[1];
      for (int a2 = g; a2 < r[2]; a2 += m2.ngrp)
        dst[(long long)a2 * fs[2]] = fiber_dot<XM>(czero<C>(), x, c2, [&](int j) { return Mt2[j * R2 + a2]; });
    }
  }
}

// -------------------------------------------------------------- fan-in --
// coarse(a_0.., q) = sum_children sum_j prod_k M_k[j_k][a_k] fine_c(j, q)
// over the children's true ranks, for the coarse block's true entries with
// a_0 in this workgroup's slice (compact numbering).
template <class T, int D, int XM>
__global__ void __launch_bounds__(kThreads)
    stage_fanin_fib(StageArgs a, const typename CplxOf<T>::type* __restrict__ fine,
                    typename CplxOf<T>::type* __restrict__ coarse,
                    const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const StageBid sb = stage_bid(a, 1);
  const int ci = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  Seg sg[D];
  coarse_segs<D>(a, ci, beta, sg);
  const int lo = sb.split * a.chunk;
  const int na = min(sg[0].c, lo + a.chunk) - lo;
  const int q0 = sb.q0;
  const int nchild = a.coarse_global ? 1 : (1 << D);
  __shared__ int cfi[kMaxChildren], crk[kMaxChildren][kMaxDTuned];
  __shared__ long long cfb[kMaxChildren];
  if ((int)threadIdx.x < nchild) {
    const int c = threadIdx.x;
    const int fi = a.coarse_global ? ci : child_of<D>(ci, a.lvl, c);
    cfi[c] = fi;
#pragma unroll
    for (int k = 0; k < D; ++k) crk[c][k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
    long long fs_[D];
    cfb[c] = fine_base<D>(a, fi, beta, q0, fs_);
  }
  if (na <= 0) return;  // after the children's rank loads; uniform, before any barrier
  long long fs[D];
  (void)fine_base<D>(a, 0, beta, 0, fs);  // strides only
  CoarseAddr<D> ca;
  ca.init(a, ci, beta, q0);
  __syncthreads();
  const int chunk = a.chunk, R0 = a.R[0], R1 = a.R[1], R2 = D == 3 ? a.R[2] : 1;
  const int A0 = a.A[0], A1 = a.A[1], A2 = D == 3 ? a.A[2] : 1;
  const int c1 = sg[1].c, c2 = D == 3 ? sg[2].c : 1;
  // LDS per child c (at c * msz): Mt0 [R0][chunk] (Mt0[j][ai] = M0_c[j][pos(lo + ai)]),
  // Mt1 [R1][A1], Mt2 [R2][A2] (Mt_k[j][jo] = M_k[j][pos(jo)]); then B1 [c][chunk][R1][R2]
  // and B2 [c][chunk][A1][R2]
  const int msz = chunk * R0 + R1 * A1 + (D == 3 ? R2 * A2 : 0);
  const int off1 = chunk * R0, off2 = off1 + R1 * A1;
  const int per1 = chunk * R1 * R2, per2 = chunk * A1 * R2;
  C* B1 = sm + nchild * msz;
  C* B2 = B1 + nchild * per1;

  // first mode: fibers (c, j1, j2) of the children's blocks, j_k < r_k(c)
  int fend[kMaxChildren];
  {
    int tot = 0;
#pragma unroll
    for (int c = 0; c < kMaxChildren; ++c) {
      tot += c < nchild ? crk[c][1] * (D == 3 ? crk[c][D - 1] : 1) : 0;
      fend[c] = tot;
    }
  }
  const FibItems m0(fend[kMaxChildren - 1], na);
  auto fib0 = [&](int f, int& c, int& j1, int& j2) {
    c = 0;
    int start = 0;
#pragma unroll
    for (int cc = 0; cc + 1 < kMaxChildren; ++cc)
      if (f >= fend[cc]) {
        c = cc + 1;
        start = fend[cc];
      }
    const int i = f - start;
    if constexpr (D == 3) {
      const int r2c = crk[c][2];
      j1 = i / r2c;
      j2 = i - j1 * r2c;
    } else {
      j1 = i;
      j2 = 0;
    }
  };
  C x[XM];
  auto load0 = [&](int it) {
    int c, j1, j2;
    fib0(it % m0.nfib, c, j1, j2);
    const C* src = fine + cfb[c] + (long long)j1 * fs[1] + (D == 3 ? (long long)j2 * fs[D - 1] : 0);
    const long long s0 = fs[0];
    fiber_load<XM>(x, crk[c][0], [&](int j) { return src[j * s0]; });
  };
  if ((int)threadIdx.x < m0.n) load0(threadIdx.x);

  // every child's matrices, all modes in one pass
  {
    int e0end[kMaxChildren], e1end[kMaxChildren], e2end[kMaxChildren];
    int t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
    for (int c = 0; c < kMaxChildren; ++c) {
      const bool on = c < nchild;
      t0 += on ? crk[c][0] * na : 0;
      t1 += on ? crk[c][1] * c1 : 0;
      t2 += on && D == 3 ? crk[c][D - 1] * c2 : 0;
      e0end[c] = t0;
      e1end[c] = t1;
      e2end[c] = t2;
    }
    const long long mo0 = a.mat_k_off[0] + (long long)beta[0] * R0 * A0;
    const long long mo1 = a.mat_k_off[1] + (long long)beta[1] * R1 * A1;
    const long long mo2 = D == 3 ? a.mat_k_off[D - 1] + (long long)beta[D - 1] * R2 * A2 : 0;
    const int ntot = t0 + t1 + t2;
    auto which = [](const int* end, int e, int& start) {
      int c = 0;
      start = 0;
#pragma unroll
      for (int cc = 0; cc + 1 < kMaxChildren; ++cc)
        if (e >= end[cc]) {
          c = cc + 1;
          start = end[cc];
        }
      return c;
    };
    for (int eb = threadIdx.x; eb < ntot; eb += kFibU * kThreads) {
      C v[kFibU];
      int dst[kFibU];
#pragma unroll
      for (int u = 0; u < kFibU; ++u) {
        const int e = eb + u * kThreads;
        dst[u] = -1;
        int start;
        if (e < t0) {
          const int c = which(e0end, e, start), i = e - start;
          const int j = i / na, o = i - j * na;
          v[u] = mats[(long long)cfi[c] * a.mat_item_stride + mo0 + (long long)j * A0 + sg[0].pos(lo + o)];
          dst[u] = c * msz + j * chunk + o;
        } else if (e < t0 + t1) {
          const int c = which(e1end, e - t0, start), i = e - t0 - start;
          const int j = i / c1, o = i - j * c1;
          v[u] = mats[(long long)cfi[c] * a.mat_item_stride + mo1 + (long long)j * A1 + sg[1].pos(o)];
          dst[u] = c * msz + off1 + j * A1 + o;
        } else if (e < ntot) {
          const int c = which(e2end, e - t0 - t1, start), i = e - t0 - t1 - start;
          const int j = i / c2, o = i - j * c2;
          v[u] = mats[(long long)cfi[c] * a.mat_item_stride + mo2 + (long long)j * A2 + sg[D - 1].pos(o)];
          dst[u] = c * msz + off2 + j * A2 + o;
        }
      }
#pragma unroll
      for (int u = 0; u < kFibU; ++u)
        if (dst[u] >= 0) {
          C t = v[u];
          if (a.conj) t.y = -t.y;
          sm[dst[u]] = t;
        }
    }
  }
  __syncthreads();

  // B1[c][ai][j1][j2] = sum_j0 M0_c[j0][pos(lo+ai)] fine_c(j0, j1, j2)
  for (int it = threadIdx.x; it < m0.n; it += kThreads) {
    if (it != (int)threadIdx.x) load0(it);
    int c, j1, j2;
    fib0(it % m0.nfib, c, j1, j2);
    const int g = it / m0.nfib, r0c = crk[c][0];
    const C* mt = sm + c * msz;
    C* dst = B1 + c * per1 + j1 * R2 + j2;
    for (int ai = g; ai < na; ai += m0.ngrp)
      dst[ai * R1 * R2] = fiber_dot<XM>(czero<C>(), x, r0c, [&](int j) { return mt[j * chunk + ai]; });
  }
  __syncthreads();

  if constexpr (D == 2) {
    // coarse[lo+ai][j1o] = sum_c sum_j1 M1_c[j1][pos(j1o)] B1[c][ai][j1]
    const int ngo = (c1 + kFibG - 1) / kFibG;
    for (int it = threadIdx.x; it < na * ngo; it += kThreads) {
      const int ai = it % na, o0 = (it / na) * kFibG;
      C acc[kFibG];
#pragma unroll
      for (int g = 0; g < kFibG; ++g) acc[g] = czero<C>();
      for (int c = 0; c < nchild; ++c) {
        const int r1c = crk[c][1];
        const C* src = B1 + c * per1 + ai * R1;
        fiber_load<XM>(x, r1c, [&](int j) { return src[j]; });
        const C* mt = sm + c * msz + off1;
#pragma unroll
        for (int g = 0; g < kFibG; ++g) {
          const int o = min(o0 + g, c1 - 1);
          acc[g] = fiber_dot<XM>(acc[g], x, r1c, [&](int j) { return mt[j * A1 + o]; });
        }
      }
      C* dst = coarse + ca.base + (long long)sg[0].pos(lo + ai) * ca.stride[0];
#pragma unroll
      for (int g = 0; g < kFibG; ++g)
        if (o0 + g < c1) dst[(long long)sg[1].pos(o0 + g) * ca.stride[1]] = acc[g];
    }
  } else {
    // B2[c][ai][j1o][j2] = sum_j1 M1_c[j1][pos(j1o)] B1[c][ai][j1][j2], j2 < r2(c)
    int f1end[kMaxChildren];
    {
      int tot = 0;
#pragma unroll
      for (int c = 0; c < kMaxChildren; ++c) {
        tot += c < nchild ? na * crk[c][2] : 0;
        f1end[c] = tot;
      }
    }
    const FibItems m1(f1end[kMaxChildren - 1], c1);
    for (int it = threadIdx.x; it < m1.n; it += kThreads) {
      const int f = it % m1.nfib, g = it / m1.nfib;
      int c = 0, start = 0;
#pragma unroll
      for (int cc = 0; cc + 1 < kMaxChildren; ++cc)
        if (f >= f1end[cc]) {
          c = cc + 1;
          start = f1end[cc];
        }
      const int r2c = crk[c][2], r1c = crk[c][1];
      const int i = f - start, ai = i / r2c, j2 = i - ai * r2c;
      const C* src = B1 + c * per1 + ai * R1 * R2 + j2;
      fiber_load<XM>(x, r1c, [&](int j) { return src[j * R2]; });
      const C* mt = sm + c * msz + off1;
      C* dst = B2 + c * per2 + ai * A1 * R2 + j2;
      for (int j1o = g; j1o < c1; j1o += m1.ngrp)
        dst[j1o * R2] = fiber_dot<XM>(czero<C>(), x, r1c, [&](int j) { return mt[j * A1 + j1o]; });
    }
    __syncthreads();
    // coarse[lo+ai][j1o][j2o] = sum_c sum_j2 M2_c[j2][pos(j2o)] B2[c][ai][j1o][j2]
    const int ngo = (c2 + kFibG - 1) / kFibG;
    const int nf = na * c1;
    for (int it = threadIdx.x; it < nf * ngo; it += kThreads) {
      const int f = it % nf, o0 = (it / nf) * kFibG;
      const int ai = f / c1, j1o = f - ai * c1;
      C acc[kFibG];
#pragma unroll
      for (int g = 0; g < kFibG; ++g) acc[g] = czero<C>();
      for (int c = 0; c < nchild; ++c) {
        const int r2c = crk[c][2];
        const C* src = B2 + c * per2 + (ai * A1 + j1o) * R2;
        fiber_load<XM>(x, r2c, [&](int j) { return src[j]; });
        const C* mt = sm + c * msz + off2;
#pragma unroll
        for (int g = 0; g < kFibG; ++g) {
          const int o = min(o0 + g, c2 - 1);
          acc[g] = fiber_dot<XM>(acc[g], x, r2c, [&](int j) { return mt[j * A2 + o]; });
        }
      }
      C* dst = coarse + ca.base + (long long)sg[0].pos(lo + ai) * ca.stride[0] +
               (long long)sg[1].pos(j1o) * ca.stride[1];
#pragma unroll
      for (int g = 0; g < kFibG; ++g)
        if (o0 + g < c2) dst[(long long)sg[2].pos(o0 + g) * ca.stride[2]] = acc[g];
    }
  }
}

// ---------------------------------------------------------------- host --
template <class T, int D, int XM>
static tb_status fib_launch(const StageArgs& a, bool fanout, long long nwg, size_t lds, const void* in,
                            void* out, const void* mats, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  const void* k = fanout ? reinterpret_cast<const void*>(stage_fanout_fib<T, D, XM>)
                         : reinterpret_cast<const void*>(stage_fanin_fib<T, D, XM>);
  if (lds > 65536)
    TB_HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const dim3 grid((unsigned)nwg);
  if (fanout)
    stage_fanout_fib<T, D, XM><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
  else
    stage_fanin_fib<T, D, XM><<<grid, kThreads, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

template <class T, int D>
static tb_status fib_launch_xm(const StageArgs& a, bool fanout, int xm, long long nwg, size_t lds,
                               const void* in, void* out, const void* mats, hipStream_t stream) {
  if (xm <= 8) return fib_launch<T, D, 8>(a, fanout, nwg, lds, in, out, mats, stream);
  if (xm <= 16) return fib_launch<T, D, 16>(a, fanout, nwg, lds, in, out, mats, stream);
  if (xm <= 24) return fib_launch<T, D, 24>(a, fanout, nwg, lds, in, out, mats, stream);
  return fib_launch<T, D, 32>(a, fanout, nwg, lds, in, out, mats, stream);
}

tb_status launch_stage_fib(bool fp64, const StageArgs& a, int d, bool fanout, int xm, long long nwg,
                           size_t lds, const void* in, void* out, const void* mats, hipStream_t stream) {
  if (xm > kFibMaxLen)
    return fail(TB_ERR_UNSUPPORTED, "register-fiber stages take contracted extents up to " +
                                        std::to_string(kFibMaxLen));
  if (nwg < 1 || nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many workgroups for one launch");
  if (d == 2)
    return fp64 ? fib_launch_xm<double, 2>(a, fanout, xm, nwg, lds, in, out, mats, stream)
                : fib_launch_xm<float, 2>(a, fanout, xm, nwg, lds, in, out, mats, stream);
  return fp64 ? fib_launch_xm<double, 3>(a, fanout, xm, nwg, lds, in, out, mats, stream)
              : fib_launch_xm<float, 3>(a, fanout, xm, nwg, lds, in, out, mats, stream);
}

}  // namespace tb
