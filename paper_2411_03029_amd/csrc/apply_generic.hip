// Contraction of a tensor butterfly with any number of modes D <= kMaxD
// (Algorithm 2 and its conjugate transpose), for the operators with d > 3:
// the high-dimensional uniform DFT of section 4.3 (d = 4 .. 6).
//
// The tuned kernels of apply.hip are written for d = 2 and 3.  Here every
// loop over modes runs to a runtime D, and the mode products of one block
// go through a per-workgroup scratch area in global memory (a block of the
// d = 5 DFT at n = 8 holds 8^5 entries, more than LDS):
//
//   fan-out  one workgroup per (fine block, right-hand side): the coarse
//            block is contracted mode by mode, M_0 first, over the coarse
//            block's true positions; the last product writes the fine block;
//   fan-in   one workgroup per (coarse block, right-hand side): each child's
//            fine block is contracted mode by mode with M_k^T and summed
//            into an accumulator, which is then written to the coarse
//            block's true positions;
//   core     one workgroup per (pair, right-hand side): rows (forward) or
//            columns (adjoint) per thread.
//
// Tensor layouts, true ranks, segments and the order of every sum are those
// of the tuned kernels; only the scheduling differs.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "stage_common.h"

namespace tb {

constexpr int kGenThreads = 256;

template <class C>
__device__ __forceinline__ C maybe_conj(C v, int conj) {
  if (conj) v.y = -v.y;
  return v;
}

// ------------------------------------------- bookkeeping for a runtime D --
__device__ __forceinline__ void unflatten_rt(int f, int nb, int D, int* beta) {
  for (int k = D - 1; k >= 0; --k) {
    beta[k] = f % nb;
    f /= nb;
  }
}

__device__ __forceinline__ int parent_rt(int item, int l, int D) {
  const int outer = item >> (D * l);
  const int inner = item & ((1 << (D * l)) - 1);
  int pin = 0;
  for (int k = 0; k < D; ++k) {
    const int b = (inner >> (l * (D - 1 - k))) & ((1 << l) - 1);
    pin = (pin << (l - 1)) | (b >> 1);
  }
  return (outer << (D * (l - 1))) | pin;
}

__device__ __forceinline__ int child_rt(int citem, int l, int c, int D) {
  const int outer = citem >> (D * (l - 1));
  const int pin = citem & ((1 << (D * (l - 1))) - 1);
  int inner = 0;
  for (int k = 0; k < D; ++k) {
    const int pk = (l > 1) ? (pin >> ((l - 1) * (D - 1 - k))) & ((1 << (l - 1)) - 1) : 0;
    const int ck = (c >> (D - 1 - k)) & 1;
    inner = (inner << l) | (2 * pk + ck);
  }
  return (outer << (D * l)) | inner;
}

// Base and per-mode strides of coarse block beta of coarse item `citem`
// (intermediate) or of outer block `citem` (the caller's array), for
// right-hand side q.
__device__ __forceinline__ void coarse_addr_rt(const StageArgs& a, int citem, const int* beta, int q, int D,
                                               long long* base, long long* stride) {
  if (a.coarse_global) {
    int o[kMaxD];
    unflatten_rt(citem, 1 << a.outer_level, D, o);
    long long st = 1, b = 0;
    for (int k = D - 1; k >= 0; --k) {
      stride[k] = st;
      b += (long long)(o[k] * a.outer_block + beta[k] * a.A[k]) * st;
      st *= a.n;
    }
    *base = b + (long long)q * a.ndim;
  } else {
    long long b = (long long)citem * a.coarseE;
    for (int k = 0; k < D; ++k) b += (long long)beta[k] * a.A[k] * a.cst[k];
    *base = b * a.nrhs + q;
    for (int k = 0; k < D; ++k) stride[k] = a.cst[k] * a.nrhs;
  }
}

__device__ __forceinline__ long long fine_base_rt(const StageArgs& a, int fi, const int* beta, int q, int D,
                                                  long long* stride) {
  long long b = (long long)fi * a.fineE;
  for (int k = 0; k < D; ++k) {
    b += (long long)beta[k] * a.R[k] * a.fst[k];
    stride[k] = a.fst[k] * a.nrhs;
  }
  return b * a.nrhs + q;
}

__device__ __forceinline__ void coarse_segs_rt(const StageArgs& a, int citem, const int* beta, int D, Seg* sg) {
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

// ------------------------------------------------------------- fan-out --
// fine(a, q) = sum_j prod_k M_k[a_k][j_k] coarse(j, q): the coarse box is
// contracted in mode order 0 .. D-1.  Intermediate k holds modes < k at the
// fine true ranks and modes >= k at the coarse padded positions, dense
// row-major; entries at padded positions are neither computed nor read.
template <class T>
__global__ void __launch_bounds__(kGenThreads)
    gen_fanout(StageArgs a, int D, const typename CplxOf<T>::type* __restrict__ coarse,
               typename CplxOf<T>::type* __restrict__ fine, const typename CplxOf<T>::type* __restrict__ mats,
               typename CplxOf<T>::type* __restrict__ scratch, long long half) {
  using C = typename CplxOf<T>::type;
  const int q = blockIdx.x % a.nrhs;
  const int item_blk = blockIdx.x / a.nrhs;
  const int fi = item_blk / a.nblk;
  int beta[kMaxD], r[kMaxD], cur[kMaxD];
  unflatten_rt(item_blk % a.nblk, a.nb, D, beta);
  for (int k = 0; k < D; ++k) r[k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
  const int citem = a.coarse_global ? (fi >> (D * a.lvl)) : parent_rt(fi, a.lvl, D);
  Seg sg[kMaxD];
  coarse_segs_rt(a, citem, beta, D, sg);
  long long cbase, cstr[kMaxD], fstr[kMaxD];
  coarse_addr_rt(a, citem, beta, q, D, &cbase, cstr);
  const long long fb = fine_base_rt(a, fi, beta, q, D, fstr);
  const C* mb = mats + (long long)fi * a.mat_item_stride;
  C* buf0 = scratch + (long long)blockIdx.x * 2 * half;
  C* buf1 = buf0 + half;
  for (int k = 0; k < D; ++k) cur[k] = a.A[k];
  for (int k = 0; k < D; ++k) {
    int ext[kMaxD];
    long long tot = 1;
    for (int i = 0; i < D; ++i) {
      ext[i] = i == k ? r[k] : cur[i];
      tot *= ext[i];
    }
    const C* Mk = mb + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
    const C* src = k == 0 ? coarse : ((k & 1) ? buf0 : buf1);
    C* dst = (k & 1) ? buf1 : buf0;
    // dense strides of the source (k > 0)
    long long sst[kMaxD];
    {
      long long st = 1;
      for (int i = D - 1; i >= 0; --i) {
        sst[i] = st;
        st *= cur[i];
      }
    }
    for (long long e = threadIdx.x; e < tot; e += kGenThreads) {
      int idx[kMaxD];
      long long t = e;
      for (int i = D - 1; i >= 0; --i) {
        idx[i] = (int)(t % ext[i]);
        t /= ext[i];
      }
      bool pad = false;
      for (int i = k + 1; i < D; ++i) pad |= idx[i] >= sg[i].h1 && (idx[i] < sg[i].off2 || idx[i] - sg[i].off2 + sg[i].h1 >= sg[i].c);
      if (pad) continue;
      long long off = k == 0 ? cbase : 0;
      long long sk;
      for (int i = 0; i < D; ++i)
        if (i != k) off += (long long)idx[i] * (k == 0 ? cstr[i] : sst[i]);
      sk = k == 0 ? cstr[k] : sst[k];
      const C* m = Mk + (long long)idx[k] * a.A[k];
      C acc = czero<C>();
      for (int j = 0; j < sg[k].c; ++j) {
        const int p = sg[k].pos(j);
        acc = cfma(acc, maybe_conj(m[p], a.conj), src[off + (long long)p * sk]);
      }
      if (k == D - 1) {
        long long fo = fb;
        for (int i = 0; i < D; ++i) fo += (long long)idx[i] * fstr[i];
        fine[fo] = acc;
      } else {
        dst[e] = acc;
      }
    }
    cur[k] = r[k];
    __syncthreads();
  }
}

// -------------------------------------------------------------- fan-in --
// coarse(p, q) = sum_children sum_j prod_k M_k(c)[j_k][p_k] fine_c(j, q):
// per child, mode order 0 .. D-1 over its true ranks, into compact coarse
// extents; summed over the children (in order) in the accumulator.
template <class T>
__global__ void __launch_bounds__(kGenThreads)
    gen_fanin(StageArgs a, int D, const typename CplxOf<T>::type* __restrict__ fine,
              typename CplxOf<T>::type* __restrict__ coarse, const typename CplxOf<T>::type* __restrict__ mats,
              typename CplxOf<T>::type* __restrict__ scratch, long long half) {
  using C = typename CplxOf<T>::type;
  const int q = blockIdx.x % a.nrhs;
  const int item_blk = blockIdx.x / a.nrhs;
  const int ci = item_blk / a.nblk;
  int beta[kMaxD];
  unflatten_rt(item_blk % a.nblk, a.nb, D, beta);
  Seg sg[kMaxD];
  coarse_segs_rt(a, ci, beta, D, sg);
  int cc[kMaxD];
  long long ctot = 1;
  for (int k = 0; k < D; ++k) {
    cc[k] = sg[k].c;
    ctot *= cc[k];
  }
  C* buf0 = scratch + (long long)blockIdx.x * 3 * half;
  C* buf1 = buf0 + half;
  C* acc = buf1 + half;
  for (long long e = threadIdx.x; e < ctot; e += kGenThreads) acc[e] = czero<C>();
  __syncthreads();
  const int nch = a.coarse_global ? 1 : (1 << D);
  for (int c = 0; c < nch; ++c) {
    const int fi = a.coarse_global ? ci : child_rt(ci, a.lvl, c, D);
    int r[kMaxD], cur[kMaxD];
    for (int k = 0; k < D; ++k) r[k] = a.rank_f[((long long)fi * D + k) * a.nb + beta[k]];
    long long fstr[kMaxD];
    const long long fb = fine_base_rt(a, fi, beta, q, D, fstr);
    const C* mb = mats + (long long)fi * a.mat_item_stride;
    for (int k = 0; k < D; ++k) cur[k] = r[k];
    for (int k = 0; k < D; ++k) {
      int ext[kMaxD];
      long long tot = 1;
      for (int i = 0; i < D; ++i) {
        ext[i] = i == k ? cc[k] : cur[i];
        tot *= ext[i];
      }
      const C* Mk = mb + a.mat_k_off[k] + (long long)beta[k] * a.R[k] * a.A[k];
      const C* src = k == 0 ? fine : ((k & 1) ? buf0 : buf1);
      C* dst = (k & 1) ? buf1 : buf0;
      long long sst[kMaxD];
      {
        long long st = 1;
        for (int i = D - 1; i >= 0; --i) {
          sst[i] = k == 0 ? fstr[i] : st;
          st *= cur[i];
        }
      }
      for (long long e = threadIdx.x; e < tot; e += kGenThreads) {
        int idx[kMaxD];
        long long t = e;
        for (int i = D - 1; i >= 0; --i) {
          idx[i] = (int)(t % ext[i]);
          t /= ext[i];
        }
        long long off = k == 0 ? fb : 0;
        for (int i = 0; i < D; ++i)
          if (i != k) off += (long long)idx[i] * sst[i];
        const int p = sg[k].pos(idx[k]);
        C s = czero<C>();
        for (int j = 0; j < r[k]; ++j)
          s = cfma(s, maybe_conj(Mk[(long long)j * a.A[k] + p], a.conj), src[off + (long long)j * sst[k]]);
        if (k == D - 1) acc[e] = cadd(acc[e], s);
        else dst[e] = s;
      }
      cur[k] = cc[k];
      __syncthreads();
    }
  }
  long long cbase, cstr[kMaxD];
  coarse_addr_rt(a, ci, beta, q, D, &cbase, cstr);
  for (long long e = threadIdx.x; e < ctot; e += kGenThreads) {
    long long t = e, off = cbase;
    for (int i = D - 1; i >= 0; --i) {
      off += (long long)sg[i].pos((int)(t % cc[i])) * cstr[i];
      t /= cc[i];
    }
    coarse[off] = acc[e];
  }
}

// ---------------------------------------------------------------- core --
__device__ __forceinline__ long long padded_pos_rt(int flat, const int* r, const int* Rp, int D) {
  long long pos = 0, st = 1;
  for (int k = D - 1; k >= 0; --k) {
    pos += (long long)(flat % r[k]) * st;
    flat /= r[k];
    st *= Rp[k];
  }
  return pos;
}

// forward: G_{t,s} = C F, one workgroup per (pair, panel of kGenThreads
// rows, right-hand side), a row per thread, the contracted F values (and
// their padded positions) staged in LDS kGenChunk at a time; adjoint:
// F_{t,s} = C^H G, one workgroup per (pair, panel of kGenCols columns,
// right-hand side), a column per wave at a time with the lanes over the
// rows (coalesced core reads) and a wave reduction, G staged likewise.
// Cores column-major, RTp rows per column.
constexpr int kGenChunk = 2048;
constexpr int kGenCols = 64;

template <class C>
__device__ __forceinline__ C wave_sum_c(C v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

template <class T>
__global__ void __launch_bounds__(kGenThreads)
    gen_core(GenCoreArgs g, int adjoint, int npanels, const typename CplxOf<T>::type* __restrict__ cores,
             const long long* __restrict__ core_off, const int* __restrict__ meta,
             const typename CplxOf<T>::type* __restrict__ in, typename CplxOf<T>::type* __restrict__ out) {
  using C = typename CplxOf<T>::type;
  __shared__ C xs[kGenChunk];
  const int q = blockIdx.x % g.nrhs;
  const int rest = blockIdx.x / g.nrhs;
  const int panel = rest % npanels;
  const int pair = rest / npanels;
  const int D = g.d;
  const int* m = meta + (long long)pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  int rt[kMaxD], rs[kMaxD];
  for (int k = 0; k < D; ++k) {
    rt[k] = m[3 + k];
    rs[k] = m[kMetaRs + k];
  }
  const long long t = pair / g.nS, s = pair % g.nS;
  const long long sitem = s * g.nT + t, titem = t * g.nS + s;
  const C* cp = cores + core_off[pair];
  if (!adjoint) {
    const int r = panel * kGenThreads + threadIdx.x;
    if (panel * kGenThreads >= RT) return;  // whole workgroup
    C acc = czero<C>();
    for (int b0 = 0; b0 < RS; b0 += kGenChunk) {
      const int nb = min(kGenChunk, RS - b0);
      __syncthreads();
      for (int i = threadIdx.x; i < nb; i += kGenThreads)
        xs[i] = in[(sitem * g.Es + padded_pos_rt(b0 + i, rs, g.Rs, D)) * g.nrhs + q];
      __syncthreads();
      if (r < RT)
        for (int i = 0; i < nb; ++i) acc = cfma(acc, cp[(long long)(b0 + i) * RTp + r], xs[i]);
    }
    if (r < RT) out[(titem * g.Et + padded_pos_rt(r, rt, g.Rt, D)) * g.nrhs + q] = acc;
  } else {
    const int c0 = panel * kGenCols;
    if (c0 >= RS) return;  // whole workgroup
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int kWaves = kGenThreads / 64;
    constexpr int kPer = kGenCols / kWaves;  // columns per wave
    C acc[kPer];
    for (int i = 0; i < kPer; ++i) acc[i] = czero<C>();
    for (int r0 = 0; r0 < RT; r0 += kGenChunk) {
      const int nr = min(kGenChunk, RT - r0);
      __syncthreads();
      for (int i = threadIdx.x; i < nr; i += kGenThreads)
        xs[i] = in[(titem * g.Et + padded_pos_rt(r0 + i, rt, g.Rt, D)) * g.nrhs + q];
      __syncthreads();
      for (int i = 0; i < kPer; ++i) {
        const int b = c0 + w * kPer + i;
        if (b >= RS) break;  // wave-uniform
        const C* col = cp + (long long)b * RTp + r0;
        for (int r = lane; r < nr; r += 64) acc[i] = cfma_conj(acc[i], col[r], xs[r]);
      }
    }
    for (int i = 0; i < kPer; ++i) {
      const int b = c0 + w * kPer + i;
      if (b >= RS) break;
      const C v = wave_sum_c(acc[i]);
      if (lane == 0) out[(sitem * g.Es + padded_pos_rt(b, rs, g.Rs, D)) * g.nrhs + q] = v;
    }
  }
}

// ---------------------------------------------------------------- host --
long long gen_box(const StageArgs& a, int d) {
  long long box = 1;
  for (int k = 0; k < d; ++k) box *= std::max(a.A[k], a.R[k]);
  return box;
}

template <class T>
static tb_status launch_gen_stage_t(const StageArgs& a, int d, bool fanout, int n_items, const void* in,
                                    void* out, const void* mats, void* scratch, hipStream_t stream) {
  using C = typename CplxOf<T>::type;
  const long long nwg = (long long)n_items * a.nblk * a.nrhs;
  if (nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many right-hand sides for one launch");
  const long long half = gen_box(a, d);
  if (fanout)
    gen_fanout<T><<<dim3((unsigned)nwg), kGenThreads, 0, stream>>>(a, d, (const C*)in, (C*)out, (const C*)mats,
                                                                  (C*)scratch, half);
  else
    gen_fanin<T><<<dim3((unsigned)nwg), kGenThreads, 0, stream>>>(a, d, (const C*)in, (C*)out, (const C*)mats,
                                                                 (C*)scratch, half);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

tb_status launch_gen_stage(bool fp64, const StageArgs& a, int d, bool fanout, int n_items, const void* in,
                           void* out, const void* mats, void* scratch, hipStream_t stream) {
  return fp64 ? launch_gen_stage_t<double>(a, d, fanout, n_items, in, out, mats, scratch, stream)
              : launch_gen_stage_t<float>(a, d, fanout, n_items, in, out, mats, scratch, stream);
}

size_t gen_stage_scratch(const StageArgs& a, int d, bool fanout, int n_items, size_t esz) {
  const long long nwg = (long long)n_items * a.nblk * a.nrhs;
  return (size_t)nwg * (fanout ? 2 : 3) * (size_t)gen_box(a, d) * esz;
}

tb_status launch_gen_core(bool fp64, const GenCoreArgs& g, bool adjoint, const void* cores,
                          const long long* core_off, const int* meta, long long npairs, int max_rt,
                          int max_rs, const void* in, void* out, hipStream_t stream) {
  const int npanels = adjoint ? (max_rs + kGenCols - 1) / kGenCols : (max_rt + kGenThreads - 1) / kGenThreads;
  const long long nwg = npairs * npanels * g.nrhs;
  if (nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many right-hand sides for one launch");
  if (fp64)
    gen_core<double><<<dim3((unsigned)nwg), kGenThreads, 0, stream>>>(
        g, adjoint ? 1 : 0, npanels, (const double2*)cores, core_off, meta, (const double2*)in, (double2*)out);
  else
    gen_core<float><<<dim3((unsigned)nwg), kGenThreads, 0, stream>>>(
        g, adjoint ? 1 : 0, npanels, (const float2*)cores, core_off, meta, (const float2*)in, (float2*)out);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

}  // namespace tb
