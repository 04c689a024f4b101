// Leaf stages with one workgroup per leaf box and right-hand side, of one
// wave or four (NT threads; the kernels keep the names of the one-wave form)
// (Algorithm 2 steps 1 and 3: the source leaf V and the target leaf U, and
// the same stages of the adjoint).
//
// A leaf box is dense (C_b^d points of the caller's array), and the leaf
// matrices are stored zero-padded to the level's largest rank, so every
// address a leaf stage reads is known before its ranks are: the box (or the
// padded fine block) and the three padded matrices are requested together
// with the ranks, in one memory round trip.  The mode products then run
// through LDS over the true ranks only (intermediates at padded positions
// are neither written nor read); with one wave the barriers between them
// cost next to nothing.
//
//   fan-out (source leaf; target leaf of the adjoint): fine(a) = sum_p
//     M_0[a_0][p_0] .. M_{D-1}[a_{D-1}][p_{D-1}] box(p), the last mode first;
//   fan-in (target leaf; source leaf of the adjoint): box(p) = sum_a
//     M_0[a_0][p_0] .. fine(a), the first mode first; the padded fine block
//     is requested whole, and its entries past the true ranks are dropped.
//
// AL is the leaf size (a template parameter, 4, 8 or 16; every mode's
// extent); ranks are at most AL.
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace tb {

constexpr int kWave = 64;

template <class C>
__device__ __forceinline__ C cmask(C v, bool keep) {
  return keep ? v : czero<C>();
}

// ------------------------------------------------------------- fan-out --
template <class T, int D, int AL, int NT>
__global__ void __launch_bounds__(NT)
    leaf_fanout_wave(StageArgs a, const typename CplxOf<T>::type* __restrict__ box,
                     typename CplxOf<T>::type* __restrict__ fine,
                     const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int lane = threadIdx.x;
  const StageBid sb = stage_bid(a, 1);
  const int fi = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  int r[D];
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
  CoarseAddr<D> ca;
  ca.init(a, fi, beta, sb.q0);  // leaves: the outer block of item fi
  long long fs[D];
  const long long fb = fine_base<D>(a, fi, beta, sb.q0, fs);
  const int R0 = a.R[0], R1 = a.R[1], R2 = D == 3 ? a.R[2] : 1;
  // LDS: M_k padded (R_k x AL, row-major) | T1 | T2
  C* M0 = sm;
  C* M1 = M0 + R0 * AL;
  C* M2 = M1 + R1 * AL;
  C* T1 = M2 + (D == 3 ? R2 * AL : 0);
  constexpr int kRows = D == 3 ? AL * AL : AL;   // box rows along the last mode
  constexpr int kRowsPerLane = (kRows + NT - 1) / NT;
  // the box rows, the matrices and the ranks: one round trip
  C x[kRowsPerLane][AL];
#pragma unroll
  for (int i = 0; i < kRowsPerLane; ++i) {
    const int row = lane + i * NT;
    if (row < kRows) {
      long long base = ca.base;
      if constexpr (D == 3)
        base += (long long)(row / AL) * ca.stride[0] + (long long)(row % AL) * ca.stride[1];
      else
        base += (long long)row * ca.stride[0];
#pragma unroll
      for (int p = 0; p < AL; ++p) x[i][p] = box[base + p];  // the last mode is contiguous
    }
  }
  {
    const C* mb = mats + (long long)fi * a.mat_item_stride;
    const int n0 = R0 * AL, n1 = R1 * AL, n2 = D == 3 ? R2 * AL : 0;
    for (int e = lane; e < n0 + n1 + n2; e += NT) {
      C v;
      if (e < n0)
        v = mb[a.mat_k_off[0] + (long long)beta[0] * R0 * AL + e];
      else if (e < n0 + n1)
        v = mb[a.mat_k_off[1] + (long long)beta[1] * R1 * AL + (e - n0)];
      else
        v = mb[a.mat_k_off[D - 1] + (long long)beta[D - 1] * R2 * AL + (e - n0 - n1)];
      if (a.conj) v.y = -v.y;
      sm[e] = v;
    }
  }
  __syncthreads();
  if constexpr (D == 3) {
    // T1[p0][p1][a2] = sum_p2 M2[a2][p2] box[p0][p1][p2]
#pragma unroll
    for (int i = 0; i < kRowsPerLane; ++i) {
      const int row = lane + i * NT;
      if (row < kRows)
        for (int a2 = 0; a2 < r[2]; ++a2) {
          C acc = czero<C>();
#pragma unroll
          for (int p = 0; p < AL; ++p) acc = cfma(acc, M2[a2 * AL + p], x[i][p]);
          T1[row * R2 + a2] = acc;
        }
    }
    __syncthreads();
    // T2[p0][a1][a2] = sum_p1 M1[a1][p1] T1[p0][p1][a2]
    C* T2 = T1 + AL * AL * R2;
    for (int it = lane; it < AL * r[2]; it += NT) {
      const int p0 = it / r[2], a2 = it % r[2];
      C t[AL];
#pragma unroll
      for (int p = 0; p < AL; ++p) t[p] = T1[(p0 * AL + p) * R2 + a2];
      for (int a1 = 0; a1 < r[1]; ++a1) {
        C acc = czero<C>();
#pragma unroll
        for (int p = 0; p < AL; ++p) acc = cfma(acc, M1[a1 * AL + p], t[p]);
        T2[(p0 * R1 + a1) * R2 + a2] = acc;
      }
    }
    __syncthreads();
    // fine[a0][a1][a2] = sum_p0 M0[a0][p0] T2[p0][a1][a2], true entries only
    for (int it = lane; it < r[1] * r[2]; it += NT) {
      const int a1 = it / r[2], a2 = it % r[2];
      C t[AL];
#pragma unroll
      for (int p = 0; p < AL; ++p) t[p] = T2[(p * R1 + a1) * R2 + a2];
      C* dst = fine + fb + (long long)a1 * fs[1] + (long long)a2 * fs[2];
      for (int a0 = 0; a0 < r[0]; ++a0) {
        C acc = czero<C>();
#pragma unroll
        for (int p = 0; p < AL; ++p) acc = cfma(acc, M0[a0 * AL + p], t[p]);
        dst[(long long)a0 * fs[0]] = acc;
      }
    }
  } else {
    // T1[p0][a1] = sum_p1 M1[a1][p1] box[p0][p1]
#pragma unroll
    for (int i = 0; i < kRowsPerLane; ++i) {
      const int row = lane + i * NT;
      if (row < kRows)
        for (int a1 = 0; a1 < r[1]; ++a1) {
          C acc = czero<C>();
#pragma unroll
          for (int p = 0; p < AL; ++p) acc = cfma(acc, M1[a1 * AL + p], x[i][p]);
          T1[row * R1 + a1] = acc;
        }
    }
    __syncthreads();
    // fine[a0][a1] = sum_p0 M0[a0][p0] T1[p0][a1]
    for (int a1 = lane; a1 < r[1]; a1 += NT) {
      C t[AL];
#pragma unroll
      for (int p = 0; p < AL; ++p) t[p] = T1[p * R1 + a1];
      C* dst = fine + fb + (long long)a1 * fs[1];
      for (int a0 = 0; a0 < r[0]; ++a0) {
        C acc = czero<C>();
#pragma unroll
        for (int p = 0; p < AL; ++p) acc = cfma(acc, M0[a0 * AL + p], t[p]);
        dst[(long long)a0 * fs[0]] = acc;
      }
    }
  }
}

// -------------------------------------------------------------- fan-in --
template <class T, int D, int AL, int NT>
__global__ void __launch_bounds__(NT)
    leaf_fanin_wave(StageArgs a, const typename CplxOf<T>::type* __restrict__ fine,
                    typename CplxOf<T>::type* __restrict__ box,
                    const typename CplxOf<T>::type* __restrict__ mats) {
  using C = typename CplxOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int lane = threadIdx.x;
  const StageBid sb = stage_bid(a, 1);
  const int fi = sb.item_blk / a.nblk;
  int beta[D];
  unflatten_blk<D>(sb.item_blk % a.nblk, a.nb, beta);
  int r[D];
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
  CoarseAddr<D> ca;
  ca.init(a, fi, beta, sb.q0);
  long long fs[D];
  const long long fb = fine_base<D>(a, fi, beta, sb.q0, fs);
  const int R0 = a.R[0], R1 = a.R[1], R2 = D == 3 ? a.R[2] : 1;
  C* M0 = sm;
  C* M1 = M0 + R0 * AL;
  C* M2 = M1 + R1 * AL;
  C* T1 = M2 + (D == 3 ? R2 * AL : 0);
  // fibres along the first mode of the padded fine block (entries past the
  // true ranks are read but masked), the matrices and the ranks: one round
  // trip; AL >= every padded rank
  constexpr int kFib = D == 3 ? AL * AL : AL;
  constexpr int kFibPerLane = (kFib + NT - 1) / NT;
  C x[kFibPerLane][AL];
  const int nfib = R1 * R2;
#pragma unroll
  for (int i = 0; i < kFibPerLane; ++i) {
    const int f = lane + i * NT;
    if (f < nfib) {
      const int a1 = f / R2, a2 = f % R2;
      const C* src = fine + fb + (long long)a1 * fs[1] + (D == 3 ? (long long)a2 * fs[D - 1] : 0);
#pragma unroll
      for (int j = 0; j < AL; ++j) x[i][j] = j < R0 ? src[(long long)j * fs[0]] : czero<C>();
    }
  }
  {
    const C* mb = mats + (long long)fi * a.mat_item_stride;
    const int n0 = R0 * AL, n1 = R1 * AL, n2 = D == 3 ? R2 * AL : 0;
    for (int e = lane; e < n0 + n1 + n2; e += NT) {
      C v;
      if (e < n0)
        v = mb[a.mat_k_off[0] + (long long)beta[0] * R0 * AL + e];
      else if (e < n0 + n1)
        v = mb[a.mat_k_off[1] + (long long)beta[1] * R1 * AL + (e - n0)];
      else
        v = mb[a.mat_k_off[D - 1] + (long long)beta[D - 1] * R2 * AL + (e - n0 - n1)];
      if (a.conj) v.y = -v.y;
      sm[e] = v;
    }
  }
  __syncthreads();
  if constexpr (D == 3) {
    // T1[p0][a1][a2] = sum_a0 M0[a0][p0] fine[a0][a1][a2]
#pragma unroll
    for (int i = 0; i < kFibPerLane; ++i) {
      const int f = lane + i * NT;
      const int a1 = f / R2, a2 = f % R2;
      if (f < nfib && a1 < r[1] && a2 < r[2]) {  // true entries only from here on
#pragma unroll
        for (int j = 0; j < AL; ++j) x[i][j] = cmask(x[i][j], j < r[0]);
        for (int p0 = 0; p0 < AL; ++p0) {
          C acc = czero<C>();
#pragma unroll
          for (int j = 0; j < AL; ++j)
            if (j < r[0]) acc = cfma(acc, M0[j * AL + p0], x[i][j]);
          T1[(p0 * R1 + a1) * R2 + a2] = acc;
        }
      }
    }
    __syncthreads();
    // T2[p0][p1][a2] = sum_a1 M1[a1][p1] T1[p0][a1][a2]
    C* T2 = T1 + AL * R1 * R2;
    for (int it = lane; it < AL * r[2]; it += NT) {
      const int p0 = it / r[2], a2 = it % r[2];
      C t[AL];
#pragma unroll
      for (int j = 0; j < AL; ++j) t[j] = j < r[1] ? T1[(p0 * R1 + j) * R2 + a2] : czero<C>();
      for (int p1 = 0; p1 < AL; ++p1) {
        C acc = czero<C>();
#pragma unroll
        for (int j = 0; j < AL; ++j)
          if (j < r[1]) acc = cfma(acc, M1[j * AL + p1], t[j]);
        T2[(p0 * AL + p1) * R2 + a2] = acc;
      }
    }
    __syncthreads();
    // box[p0][p1][p2] = sum_a2 M2[a2][p2] T2[p0][p1][a2]: one row per lane
    for (int row = lane; row < AL * AL; row += NT) {
      C t[AL];
#pragma unroll
      for (int j = 0; j < AL; ++j) t[j] = j < r[2] ? T2[row * R2 + j] : czero<C>();
      C* dst = box + ca.base + (long long)(row / AL) * ca.stride[0] + (long long)(row % AL) * ca.stride[1];
#pragma unroll
      for (int p2 = 0; p2 < AL; ++p2) {
        C acc = czero<C>();
#pragma unroll
        for (int j = 0; j < AL; ++j)
          if (j < r[2]) acc = cfma(acc, M2[j * AL + p2], t[j]);
        dst[p2] = acc;
      }
    }
  } else {
    // T1[p0][a1] = sum_a0 M0[a0][p0] fine[a0][a1]
#pragma unroll
    for (int i = 0; i < kFibPerLane; ++i) {
      const int a1 = lane + i * NT;
      if (a1 < nfib && a1 < r[1]) {  // true entries only from here on
#pragma unroll
        for (int j = 0; j < AL; ++j) x[i][j] = cmask(x[i][j], j < r[0]);
        for (int p0 = 0; p0 < AL; ++p0) {
          C acc = czero<C>();
#pragma unroll
          for (int j = 0; j < AL; ++j)
            if (j < r[0]) acc = cfma(acc, M0[j * AL + p0], x[i][j]);
          T1[p0 * R1 + a1] = acc;
        }
      }
    }
    __syncthreads();
    // box[p0][p1] = sum_a1 M1[a1][p1] T1[p0][a1]
    for (int p0 = lane; p0 < AL; p0 += NT) {
      C t[AL];
#pragma unroll
      for (int j = 0; j < AL; ++j) t[j] = j < r[1] ? T1[p0 * R1 + j] : czero<C>();
      C* dst = box + ca.base + (long long)p0 * ca.stride[0];
#pragma unroll
      for (int p1 = 0; p1 < AL; ++p1) {
        C acc = czero<C>();
#pragma unroll
        for (int j = 0; j < AL; ++j)
          if (j < r[1]) acc = cfma(acc, M1[j * AL + p1], t[j]);
        dst[p1] = acc;
      }
    }
  }
}

// ---------------------------------------------------------------- host --
long long leaf_wave_lds_elems(const StageArgs& a, int d, bool fanout) {
  const long long AL = a.A[0], R0 = a.R[0], R1 = a.R[1], R2 = d == 3 ? a.R[2] : 1;
  long long e = (R0 + R1 + (d == 3 ? R2 : 0)) * AL;
  if (d == 3)
    e += fanout ? AL * AL * R2 + AL * R1 * R2 : AL * R1 * R2 + AL * AL * R2;
  else
    e += AL * R1;
  return e;
}

template <class T, int D, int AL, int NT>
static tb_status leaf_go(const StageArgs& a, bool fanout, long long nwg, size_t lds, const void* in, void* out,
                         const void* mats, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  const void* k = fanout ? reinterpret_cast<const void*>(leaf_fanout_wave<T, D, AL, NT>)
                         : reinterpret_cast<const void*>(leaf_fanin_wave<T, D, AL, NT>);
  if (lds > 65536)
    TB_HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const dim3 grid((unsigned)nwg);
  if (fanout)
    leaf_fanout_wave<T, D, AL, NT><<<grid, NT, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
  else
    leaf_fanin_wave<T, D, AL, NT><<<grid, NT, lds, stream>>>(a, (const C*)in, (C*)out, (const C*)mats);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

template <class T, int D, int NT>
static tb_status leaf_go_al(const StageArgs& a, bool fanout, long long nwg, size_t lds, const void* in,
                            void* out, const void* mats, hipStream_t stream) {
  switch (a.A[0]) {
    case 4: return leaf_go<T, D, 4, NT>(a, fanout, nwg, lds, in, out, mats, stream);
    case 8: return leaf_go<T, D, 8, NT>(a, fanout, nwg, lds, in, out, mats, stream);
    case 16: return leaf_go<T, D, 16, NT>(a, fanout, nwg, lds, in, out, mats, stream);
  }
  return fail(TB_ERR_UNSUPPORTED, "wave-per-box leaves take leaf sizes 4, 8 and 16");
}

template <class T, int D>
static tb_status leaf_go_nt(const StageArgs& a, bool fanout, int waves, long long nwg, size_t lds,
                            const void* in, void* out, const void* mats, hipStream_t stream) {
  return waves == 4 ? leaf_go_al<T, D, 4 * kWave>(a, fanout, nwg, lds, in, out, mats, stream)
                    : leaf_go_al<T, D, kWave>(a, fanout, nwg, lds, in, out, mats, stream);
}

tb_status launch_leaf_wave(bool fp64, const StageArgs& a, int d, bool fanout, int waves, int n_items,
                           const void* in, void* out, const void* mats, hipStream_t stream, int lds_limit) {
  if (!a.coarse_global) return fail(TB_ERR_UNSUPPORTED, "wave-per-box kernels run the leaf stages only");
  for (int k = 0; k < d; ++k)
    if (a.A[k] != a.A[0] || a.R[k] > a.A[0])
      return fail(TB_ERR_UNSUPPORTED, "wave-per-box leaves need cubic leaf boxes");
  const size_t esz = fp64 ? sizeof(double2) : sizeof(float2);
  const size_t lds = (size_t)leaf_wave_lds_elems(a, d, fanout) * esz;
  if (lds > (size_t)lds_limit) return fail(TB_ERR_UNSUPPORTED, "leaf box exceeds the LDS of a workgroup");
  StageArgs b = a;
  b.nsplit = 1;
  b.chunk = fanout ? a.R[0] : a.A[0];
  const long long nwg = (long long)n_items * a.nblk * a.nrhs;
  if (nwg < 1 || nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many workgroups for one launch");
  if (d == 2)
    return fp64 ? leaf_go_nt<double, 2>(b, fanout, waves, nwg, lds, in, out, mats, stream)
                : leaf_go_nt<float, 2>(b, fanout, waves, nwg, lds, in, out, mats, stream);
  return fp64 ? leaf_go_nt<double, 3>(b, fanout, waves, nwg, lds, in, out, mats, stream)
              : leaf_go_nt<float, 3>(b, fanout, waves, nwg, lds, in, out, mats, stream);
}

}  // namespace tb
