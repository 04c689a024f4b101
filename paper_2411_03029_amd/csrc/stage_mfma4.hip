// Transfer stages on the matrix cores, d = 3, FP32, four right-hand sides
// per workgroup (Algorithm 2 steps 1 and 3 at the transfer levels, and the
// same stages of the adjoint).
//
// Every mode product runs on v_mfma_f32_4x4x1f32: one instruction forms 16
// independent 4 x 4 outer products, each of four matrix entries (four rows
// of the output mode) with one input entry of the four right-hand sides.  A
// block of the instruction is one position of the two modes not being
// contracted, so the contracted mode needs no padding (K = 1) and the output
// mode is padded only to a multiple of four; where a mode has at most 8
// positions, the two halves of the blocks take two different tiles of rows
// (the matrix operand is per block).  A complex product is four real
// instructions.
//
// Fan-in (the 2^d children's tensors carried into their parent block: the
// target side of the forward apply; with M^H, the source side of the
// adjoint):
//
//   coarse(a_0, a_1, a_2, q) = sum_children sum_j M0_c[j_0][a_0] M1_c[j_1][a_1]
//                              M2_c[j_2][a_2] fine_c(j_0, j_1, j_2, q)
//
// One workgroup of four waves takes one coarse block, in groups of four a_0
// rows; wave w accumulates row a_0 = 4 s + w of group s over all children,
// in registers (16 x 16 entries of four right-hand sides: 8 complex values
// per lane).  Per group, the children are taken in turn: mode 0 (the
// group's tile of a_0) reads the child's input from global memory into
// registers (issued one child ahead, so the loads overlap the previous
// child's products) and writes LDS; then each wave takes its row through
// mode 1, into LDS of its own, and mode 2, into its accumulators.  Two
// workgroup barriers per child and group.  Holding one row per wave keeps
// the registers (145) and LDS (49 KB) within three workgroups per CU; each
// child's input is read once per group, mostly from L2.  The matrices of
// all eight children come into LDS at the start, in the same memory round
// trip as the ranks and the first child's input: they are staged at their
// padded columns, so their addresses do not depend on any rank.
//
// Fan-out (source side of the forward apply; target side of the adjoint
// with conj(M)) and the leaf fan-in: described above stage_fanout_m4 and
// leaf_fanin_m4.
//
// Limits (the host rejects other blocks): fine ranks up to 8 per mode,
// coarse blocks up to 16 per mode; the leaf form, leaf size 8.
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace tb {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kR = 8;    // largest padded fine rank per mode
constexpr int kC = 16;   // largest coarse block extent per mode
constexpr int kQ = 4;    // right-hand sides per workgroup
constexpr int kNch = 8;  // children of a coarse block (2^3)

__device__ __forceinline__ v4f mf(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

struct CAcc {
  v4f re, im;
};

__device__ __forceinline__ void czero4(CAcc& d) {
  d.re = v4f{0.f, 0.f, 0.f, 0.f};
  d.im = v4f{0.f, 0.f, 0.f, 0.f};
}

// column of the padded matrix that holds compact coarse entry e of mode k,
// for an output row past the true extent column 0 (its results are dropped)
__device__ __forceinline__ int pcol(const Seg& s, int e) { return e < s.c ? s.pos(e) : 0; }

// d[t] += M[k][col[t]] (x) x_k over k < nk for NT tiles of four output rows:
// x_k = src[k * xs] is this lane's input entry (its block's position, its
// right-hand side), M[k][col[t]] the matrix entry of its row in tile t.
// The tile count is a template parameter so that no branch separates the
// matrix-core instructions; the four real products of the tiles are
// interleaved so that consecutive instructions use different accumulators.
template <int NT, int MS = kC>
__device__ __forceinline__ void tiles_lds(CAcc (&d)[4], const float2* src, int xs, const float2* M,
                                          const int (&col)[4], int nk) {
  for (int k = 0; k < nk; ++k) {
    const float2 x = src[k * xs];
    float2 m[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) m[t] = M[k * MS + col[t]];
#pragma unroll
    for (int t = 0; t < NT; ++t) d[t].re = mf(m[t].x, x.x, d[t].re);
#pragma unroll
    for (int t = 0; t < NT; ++t) d[t].im = mf(m[t].x, x.y, d[t].im);
#pragma unroll
    for (int t = 0; t < NT; ++t) d[t].re = mf(-m[t].y, x.y, d[t].re);
#pragma unroll
    for (int t = 0; t < NT; ++t) d[t].im = mf(m[t].y, x.x, d[t].im);
  }
}

__device__ __forceinline__ void tiles_lds_n(int nt, CAcc (&d)[4], const float2* src, int xs, const float2* M,
                                            const int (&col)[4], int nk) {
  switch (nt) {
    case 1: tiles_lds<1>(d, src, xs, M, col, nk); break;
    case 2: tiles_lds<2>(d, src, xs, M, col, nk); break;
    case 3: tiles_lds<3>(d, src, xs, M, col, nk); break;
    default: tiles_lds<4>(d, src, xs, M, col, nk); break;
  }
}

// Fan-out form: the contracted index is the coarse block's compact entry
// j < s.c, at padded position s.pos(j) (two segments), and the matrix is
// staged transposed, Mt[padded position][output row] (row stride kR).
template <int NT>
__device__ __forceinline__ void seg_tiles(CAcc (&d)[4], const float2* src, int xs, const float2* Mt,
                                          const int (&row)[4], const Seg& sg) {
  tiles_lds<NT, kR>(d, src, xs, Mt, row, sg.h1);
  tiles_lds<NT, kR>(d, src + sg.h1 * xs, xs, Mt + sg.off2 * kR, row, sg.c - sg.h1);
}

// the same with the input entries in registers (b[k], k < nk <= kR)
template <int NT>
__device__ __forceinline__ void tiles_reg(CAcc (&d)[4], const float2 (&b)[kR], const float2* M,
                                          const int (&col)[4], int nk) {
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (k < nk) {
      float2 m[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) m[t] = M[k * kC + col[t]];
#pragma unroll
      for (int t = 0; t < NT; ++t) d[t].re = mf(m[t].x, b[k].x, d[t].re);
#pragma unroll
      for (int t = 0; t < NT; ++t) d[t].im = mf(m[t].x, b[k].y, d[t].im);
#pragma unroll
      for (int t = 0; t < NT; ++t) d[t].re = mf(-m[t].y, b[k].y, d[t].re);
#pragma unroll
      for (int t = 0; t < NT; ++t) d[t].im = mf(m[t].y, b[k].x, d[t].im);
    }
  }
}

}  // namespace

__global__ void __launch_bounds__(256, 3)
    stage_fanin_m4(StageArgs a, const float2* __restrict__ fine, float2* __restrict__ coarse,
                   const float2* __restrict__ mats) {
  __shared__ float2 smat[kNch * 3 * kR * kC];  // [child][mode][row j][padded column]
  __shared__ float2 sbuf1[4 * kR * kR * kQ];   // mode 0 output of a group of four a0 rows [a0 - 4s][j1][j2][q]
  __shared__ float2 sbuf2[4 * kR * kC * kQ];   // mode 1 output of one a_0 row per wave [w][j2][a1][q]
  __shared__ int srk[kNch][3];

  const StageBid sb = stage_bid(a, kQ);
  const int ci = sb.item_blk / a.nblk;
  int beta[3];
  unflatten_blk<3>(sb.item_blk % a.nblk, a.nb, beta);
  Seg sg[3];
  coarse_segs<3>(a, ci, beta, sg);
  const int q0 = sb.q0;
  const int Qa = min(kQ, a.nrhs - q0);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int blk = lane >> 2, qn = lane & 3;
  const int qc = min(qn, Qa - 1);
  const int R0 = a.R[0], R1 = a.R[1], R2 = a.R[2];
  long long fs[3];
  (void)fine_base<3>(a, 0, beta, 0, fs);  // strides only

  // this lane's mode-0 input of child c: rows j0 < kR at position
  // p = 16 w + blk of the padded (j1, j2) grid, right-hand side q0 + qc
  auto load_b = [&](int c, float2 (&b)[kR]) {
    const int fi = child_of<3>(ci, a.lvl, c);
    long long f_[3];
    const long long base = fine_base<3>(a, fi, beta, q0, f_);
    const int p = min(16 * w + blk, R1 * R2 - 1);
    const float2* src = fine + base + (p / R2) * fs[1] + (p % R2) * fs[2] + qc;
#pragma unroll
    for (int k = 0; k < kR; ++k) b[k] = src[min(k, R0 - 1) * fs[0]];
  };
  float2 b[kR];
  load_b(0, b);
  // ranks of the children
  int crank = 0;
  if (tid < kNch * 3) {
    const int c = tid / 3, k = tid % 3;
    const int fi = child_of<3>(ci, a.lvl, c);
    const int bk = k == 0 ? beta[0] : (k == 1 ? beta[1] : beta[2]);
    crank = a.rank_f[((long long)fi * 3 + k) * a.nb + bk];
  }
  // every child's padded matrices, all loads in flight before any store:
  // the first child's input, the ranks and the matrices take one memory
  // round trip together
  {
    constexpr int kPer = kNch * 3 * kR * kC / 256;
    float2 v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int c = e / (3 * kR * kC), k = (e / (kR * kC)) % 3, j = (e / kC) % kR, col = e % kC;
      // the mode varies across lanes: select its sizes from the uniform
      // arguments (indexing the argument arrays by it would read them from
      // memory, one dependent load each)
      const int Rk = k == 0 ? a.R[0] : (k == 1 ? a.R[1] : a.R[2]);
      const int Ak = k == 0 ? a.A[0] : (k == 1 ? a.A[1] : a.A[2]);
      const int bk = k == 0 ? beta[0] : (k == 1 ? beta[1] : beta[2]);
      const long long ok = k == 0 ? a.mat_k_off[0] : (k == 1 ? a.mat_k_off[1] : a.mat_k_off[2]);
      v[u] = make_float2(0.f, 0.f);
      if (j < Rk && col < Ak) {
        const int fi = child_of<3>(ci, a.lvl, c);
        v[u] = mats[(long long)fi * a.mat_item_stride + ok + ((long long)bk * Rk + j) * Ak + col];
      }
    }
    if (sg[0].c <= 0 || sg[1].c <= 0 || sg[2].c <= 0) return;  // no entries (uniform, before any barrier)
    if (tid < kNch * 3) srk[tid / 3][tid % 3] = crank;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      float2 x = v[u];
      if (a.conj) x.y = -x.y;
      smat[tid + 256 * u] = x;
    }
  }

  const int c0 = sg[0].c, c1 = sg[1].c, c2 = sg[2].c;
  const int nt1 = (c1 + 3) / 4, nt2 = (c2 + 3) / 4;
  // mode 1 pairs tiles of a1 across the two halves of an instruction's
  // blocks: block blk holds position j2h = blk % 8 of tile 2 tp + th
  const int th = blk >> 3, j2h = blk & 7;
  int col1p[4], col2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    col1p[t] = t < 2 ? pcol(sg[1], 4 * (2 * t + th) + qn) : 0;
    col2[t] = pcol(sg[2], 4 * t + qn);
  }
  CoarseAddr<3> ca;
  ca.init(a, ci, beta, q0);
  __syncthreads();  // ranks and matrices

  // row groups s of four a0 rows, outermost: wave w accumulates row
  // a0 = 4 s + w over all children, so the accumulators hold one row
  const int ngrp = (c0 + 3) / 4;
  for (int s = 0; s < ngrp; ++s) {
    CAcc acc[4];  // [tile t: a2 = 4 t + row]
#pragma unroll
    for (int t = 0; t < 4; ++t) czero4(acc[t]);
    int col0s[4] = {pcol(sg[0], 4 * s + qn), 0, 0, 0};
    const int a0 = 4 * s + w;
    for (int c = 0; c < kNch; ++c) {
      const int r0 = srk[c][0], r1 = srk[c][1], r2 = srk[c][2];
      // ---- mode 0, rows of group s: sbuf1[a0 - 4s][j1][j2][q] = sum_j0 M0[j0][a0] fine(j0, j1, j2, q)
      {
        const float2* M0 = smat + (c * 3 + 0) * kR * kC;
        const int p = 16 * w + blk;
        if (16 * w < R1 * R2 && (16 * w) / R2 < r1) {
          CAcc d[4];
          czero4(d[0]);
          tiles_reg<1>(d, b, M0, col0s, r0);
          const int j1 = p / R2, j2 = p % R2;
          if (p < R1 * R2 && j1 < r1 && j2 < r2) {  // rows past c0 land in unread padding
#pragma unroll
            for (int v = 0; v < 4; ++v)
              sbuf1[((v * kR + j1) * kR + j2) * kQ + qn] = make_float2(d[0].re[v], d[0].im[v]);
          }
        }
        // the next (group, child) input, in flight during modes 1 and 2
        if (c + 1 < kNch)
          load_b(c + 1, b);
        else if (s + 1 < ngrp)
          load_b(0, b);
      }
      __syncthreads();
      // ---- modes 1 and 2 for row a0 of this wave
      if (a0 < c0 && r1 > 0 && r2 > 0) {  // a child of rank 0 adds nothing
        const float2* M1 = smat + (c * 3 + 1) * kR * kC;
        const float2* M2 = smat + (c * 3 + 2) * kR * kC;
        float2* t1 = sbuf2 + w * kR * kC * kQ;  // [j2][a1][q] of this wave's row
        // t1[j2][a1][q] = sum_j1 M1[j1][a1] sbuf1[w][j1][j2][q]: a row has at
        // most 8 positions j2, so blocks 0-7 and 8-15 of an instruction take
        // two different tiles of a1 (the matrix operand is per block)
        CAcc d[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) czero4(d[t]);
        tiles_lds_n((nt1 + 1) / 2, d, sbuf1 + (w * kR * kR + min(j2h, r2 - 1)) * kQ + qn, kR * kQ, M1, col1p,
                    r1);
        if (j2h < r2) {  // rows past c1 land in unread padding
#pragma unroll
          for (int tp = 0; tp < 2; ++tp)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              t1[(j2h * kC + 4 * (2 * tp + th) + v) * kQ + qn] = make_float2(d[tp].re[v], d[tp].im[v]);
        }
        // acc += sum_j2 M2[j2][a2] t1[j2][a1][q], a1 = blk (the same wave
        // wrote t1: its LDS operations complete in order)
        tiles_lds_n(nt2, acc, t1 + min(blk, c1 - 1) * kQ + qn, kC * kQ, M2, col2, r2);
      }
      __syncthreads();  // sbuf1 is rewritten by the next child
    }
    // row a0 of the block's true entries
    if (a0 < c0 && blk < c1 && qn < Qa) {
      float2* dst = coarse + ca.base + sg[0].pos(a0) * ca.stride[0] + sg[1].pos(blk) * ca.stride[1] + qn;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a2 = 4 * t + v;
          if (a2 < c2) dst[sg[2].pos(a2) * ca.stride[2]] = make_float2(acc[t].re[v], acc[t].im[v]);
        }
    }
  }
}

tb_status launch_fanin_m4(const StageArgs& a, int d, int n_items, const void* in, void* out,
                          const void* mats, hipStream_t stream) {
  if (d != 3) return fail(TB_ERR_UNSUPPORTED, "the matrix-core fan-in is for d = 3");
  if (a.coarse_global || a.rank_c == nullptr)
    return fail(TB_ERR_UNSUPPORTED, "the matrix-core fan-in runs the transfer levels only");
  for (int k = 0; k < 3; ++k)
    if (a.R[k] > kR || a.A[k] > kC)
      return fail(TB_ERR_UNSUPPORTED, "matrix-core fan-in: ranks above 8 or coarse blocks above 16");
  StageArgs b = a;
  b.nsplit = 1;
  b.chunk = a.A[0];
  b.aff_blocks = 0;
  const long long nwg = (long long)n_items * a.nblk * ((a.nrhs + kQ - 1) / kQ);
  if (nwg < 1 || nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many workgroups for one launch");
  stage_fanin_m4<<<dim3((unsigned)nwg), 256, 0, stream>>>(b, (const float2*)in, (float2*)out,
                                                          (const float2*)mats);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

// ------------------------------------------------------------- fan-out --
// fine(a_0, a_1, a_2, q) = sum_j M0[a_0][j_0] M1[a_1][j_1] M2[a_2][j_2]
//                          coarse(j_0, j_1, j_2, q)
// (source side of the forward apply; conj(M) on the target side of the
// adjoint).  One workgroup of four waves takes one fine block and four
// right-hand sides, in two halves of four a_0 rows each.  Per half, mode 0
// reads the coarse block from global memory (16 positions (j_1, j_2) per
// instruction, the half's tile of a_0; each wave's next group of positions
// in flight while it multiplies the current one) into LDS; then wave w
// carries row a_0 = 4 h + w through mode 1 (positions j_2, two tiles of a_1)
// into LDS of its own and mode 2 (positions a_1, the two tiles of a_2 in the
// two halves of the blocks), which writes the fine block.  Holding one half
// of the mode-0 output (32 KB) lets three workgroups share a CU; the coarse
// block is read once per half, the second time mostly from L2.
__global__ void __launch_bounds__(256, 3)
    stage_fanout_m4(StageArgs a, const float2* __restrict__ coarse, float2* __restrict__ fine,
                    const float2* __restrict__ mats) {
  __shared__ float2 smt[3 * kC * kR];            // [mode][padded coarse position][row a]
  __shared__ float2 st0[4 * kC * kC * kQ];       // mode 0 output of a half [a0 - 4h][j1][j2][q], compact j
  __shared__ float2 st1[4 * kC * kR * kQ];       // mode 1 output of row a0 = 4h + w: [w][j2][a1][q]

  const StageBid sb = stage_bid(a, kQ);
  const int fi = sb.item_blk / a.nblk;
  int beta[3];
  unflatten_blk<3>(sb.item_blk % a.nblk, a.nb, beta);
  int r[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) r[k] = a.rank_f[((long long)fi * 3 + k) * a.nb + beta[k]];
  const int citem = parent_of<3>(fi, a.lvl);
  Seg sg[3];
  coarse_segs<3>(a, citem, beta, sg);
  const int q0 = sb.q0;
  const int Qa = min(kQ, a.nrhs - q0);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int blk = lane >> 2, qn = lane & 3;
  const int qc = min(qn, Qa - 1);
  // the matrices, transposed, at their padded coarse positions (384 entries)
  float2 mv[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + 256 * u;
    mv[u] = make_float2(0.f, 0.f);
    if (e < 3 * kC * kR) {
      const int k = e / (kC * kR), p = (e / kR) % kC, row = e % kR;
      const int Rk = k == 0 ? a.R[0] : (k == 1 ? a.R[1] : a.R[2]);
      const int Ak = k == 0 ? a.A[0] : (k == 1 ? a.A[1] : a.A[2]);
      const int bk = k == 0 ? beta[0] : (k == 1 ? beta[1] : beta[2]);
      const long long ok = k == 0 ? a.mat_k_off[0] : (k == 1 ? a.mat_k_off[1] : a.mat_k_off[2]);
      if (row < Rk && p < Ak) mv[u] = mats[(long long)fi * a.mat_item_stride + ok + ((long long)bk * Rk + row) * Ak + p];
      if (a.conj) mv[u].y = -mv[u].y;
    }
  }
  const int c0 = sg[0].c, c1 = sg[1].c, c2 = sg[2].c;
  if (c0 <= 0 || c1 <= 0 || c2 <= 0 || r[0] <= 0 || r[1] <= 0 || r[2] <= 0) return;  // uniform
#pragma unroll
  for (int u = 0; u < 2; ++u)
    if (tid + 256 * u < 3 * kC * kR) smt[tid + 256 * u] = mv[u];
  CoarseAddr<3> ca;
  ca.init(a, citem, beta, q0);
  long long fs[3];
  const long long fb = fine_base<3>(a, fi, beta, q0, fs);
  const int row[4] = {qn, 4 + qn, 0, 0};
  const int P = c1 * c2, ng = (P + 15) / 16;
  // this lane's mode-0 input for group g of positions (j1, j2)
  auto load_grp = [&](int g, float2 (&b)[kC]) {
    const int pc = min(16 * g + blk, P - 1);
    const int j1 = pc / c2, j2 = pc % c2;
    const float2* src = coarse + ca.base + sg[1].pos(j1) * ca.stride[1] + sg[2].pos(j2) * ca.stride[2] + qc;
#pragma unroll
    for (int k = 0; k < kC; ++k) b[k] = src[sg[0].pos(min(k, c0 - 1)) * ca.stride[0]];
  };
  float2 b[kC];
  if (w < ng) load_grp(w, b);
  __syncthreads();  // matrices

  const int nh = r[0] > 4 ? 2 : 1;
  for (int h = 0; h < nh; ++h) {
    // ---- mode 0, rows a0 = 4 h + v: st0[v][j1][j2][q] = sum_j0 M0[a0][j0] coarse(j0, j1, j2, q)
    for (int g = w; g < ng; g += 4) {
      float2 cur[kC];
#pragma unroll
      for (int k = 0; k < kC; ++k) cur[k] = b[k];
      // the next group of this wave (the first group again for the second half)
      const int gn = g + 4 < ng ? g + 4 : (h + 1 < nh ? w : -1);
      if (gn >= 0) load_grp(gn, b);
      CAcc d;
      czero4(d);
#pragma unroll
      for (int k = 0; k < kC; ++k) {
        if (k < c0) {
          const float2 m = smt[sg[0].pos(k) * kR + row[h]];
          d.re = mf(m.x, cur[k].x, d.re);
          d.im = mf(m.x, cur[k].y, d.im);
          d.re = mf(-m.y, cur[k].y, d.re);
          d.im = mf(m.y, cur[k].x, d.im);
        }
      }
      const int p = 16 * g + blk;
      if (p < P) {  // rows past r0 land in unread padding
        const int j1 = p / c2, j2 = p % c2;
#pragma unroll
        for (int v = 0; v < 4; ++v) st0[((v * kC + j1) * kC + j2) * kQ + qn] = make_float2(d.re[v], d.im[v]);
      }
    }
    __syncthreads();
    const int a0 = 4 * h + w;
    if (a0 < r[0]) {
      float2* t1 = st1 + w * kC * kR * kQ;  // [j2][a1][q]
      // ---- mode 1: t1[j2][a1][q] = sum_j1 M1[a1][j1] st0[w][j1][j2][q], j2 = blk
      {
        CAcc d[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) czero4(d[t]);
        seg_tiles<2>(d, st0 + (w * kC * kC + min(blk, c2 - 1)) * kQ + qn, kC * kQ, smt + kC * kR, row, sg[1]);
        if (blk < c2) {
#pragma unroll
          for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) t1[(blk * kR + 4 * t + v) * kQ + qn] = make_float2(d[t].re[v], d[t].im[v]);
        }
      }
      // ---- mode 2: fine[a0][a1][a2][q] = sum_j2 M2[a2][j2] t1[j2][a1][q]; the
      // block holds a1 = blk % 8 and rows a2 of tile blk / 8 (the same wave
      // wrote t1: its LDS operations complete in order)
      {
        const int a1 = blk & 7, th = blk >> 3;
        const int rowh[4] = {4 * th + qn, 0, 0, 0};
        CAcc d[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) czero4(d[t]);
        seg_tiles<1>(d, t1 + min(a1, r[1] - 1) * kQ + qn, kR * kQ, smt + 2 * kC * kR, rowh, sg[2]);
        if (a1 < r[1] && qn < Qa) {
          float2* dst = fine + fb + a0 * fs[0] + a1 * fs[1] + qn;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (4 * th + v < r[2]) dst[(4 * th + v) * fs[2]] = make_float2(d[0].re[v], d[0].im[v]);
        }
      }
    }
    if (h + 1 < nh) __syncthreads();  // st0 is rewritten by the second half
  }
}

tb_status launch_fanout_m4(const StageArgs& a, int d, int n_items, const void* in, void* out,
                           const void* mats, hipStream_t stream) {
  if (d != 3) return fail(TB_ERR_UNSUPPORTED, "the matrix-core fan-out is for d = 3");
  if (a.coarse_global || a.rank_c == nullptr)
    return fail(TB_ERR_UNSUPPORTED, "the matrix-core fan-out runs the transfer levels only");
  for (int k = 0; k < 3; ++k)
    if (a.R[k] > kR || a.A[k] > kC)
      return fail(TB_ERR_UNSUPPORTED, "matrix-core fan-out: ranks above 8 or coarse blocks above 16");
  StageArgs b = a;
  b.nsplit = 1;
  b.chunk = a.R[0];
  const long long nwg = (long long)n_items * a.nblk * ((a.nrhs + kQ - 1) / kQ);
  if (nwg < 1 || nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many workgroups for one launch");
  stage_fanout_m4<<<dim3((unsigned)nwg), 256, 0, stream>>>(b, (const float2*)in, (float2*)out,
                                                           (const float2*)mats);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

// --------------------------------------------------------- leaf fan-in --
// box(p_0, p_1, p_2, q) = sum_a M0[a_0][p_0] M1[a_1][p_1] M2[a_2][p_2] fine(a, q)
// (the target leaf of the forward apply; the source leaf of the adjoint
// with conj(M)), leaf size 8, the box in the caller's array.  One workgroup
// of four waves takes one leaf box and four right-hand sides.  The padded
// fine block, the padded matrices and the ranks come in one memory round
// trip.  Mode 0 (positions (a_1, a_2), both tiles of p_0) writes LDS; then
// wave w carries rows p_0 = w and w + 4 through mode 1 (positions a_2, the
// two tiles of p_1 in the two halves of the blocks) into LDS of its own and
// mode 2 (positions p_1, the two tiles of p_2 likewise), whose four outputs
// per lane are four consecutive points of one box row.
constexpr int kL = 8;  // leaf size

__global__ void __launch_bounds__(256)
    leaf_fanin_m4(StageArgs a, const float2* __restrict__ fine, float2* __restrict__ box,
                  const float2* __restrict__ mats) {
  __shared__ float2 smat[3 * kR * kL];            // [mode][row a][point p]
  __shared__ float2 st0[kL * kR * kR * kQ];       // mode 0 output [p0][a1][a2][q]
  __shared__ float2 st1[4 * kL * kR * kQ];        // mode 1 output of one row p0 per wave [w][p1][a2][q]

  const StageBid sb = stage_bid(a, kQ);
  const int fi = sb.item_blk / a.nblk;
  int beta[3];
  unflatten_blk<3>(sb.item_blk % a.nblk, a.nb, beta);
  int r[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) r[k] = a.rank_f[((long long)fi * 3 + k) * a.nb + beta[k]];
  const int q0 = sb.q0;
  const int Qa = min(kQ, a.nrhs - q0);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int blk = lane >> 2, qn = lane & 3;
  const int qc = min(qn, Qa - 1);
  const int R0 = a.R[0], R1 = a.R[1], R2 = a.R[2];
  long long fs[3];
  const long long fb = fine_base<3>(a, fi, beta, q0, fs);
  // this lane's mode-0 input: rows a0 < kR at position 16 w + blk of the
  // padded (a1, a2) grid
  float2 b[kR];
  {
    const int p = min(16 * w + blk, R1 * R2 - 1);
    const float2* src = fine + fb + (p / R2) * fs[1] + (p % R2) * fs[2] + qc;
#pragma unroll
    for (int k = 0; k < kR; ++k) b[k] = src[min(k, R0 - 1) * fs[0]];
  }
  float2 mv = make_float2(0.f, 0.f);
  if (tid < 3 * kR * kL) {
    const int k = tid / (kR * kL), row = (tid / kL) % kR, pt = tid % kL;
    const int Rk = k == 0 ? a.R[0] : (k == 1 ? a.R[1] : a.R[2]);
    const int bk = k == 0 ? beta[0] : (k == 1 ? beta[1] : beta[2]);
    const long long ok = k == 0 ? a.mat_k_off[0] : (k == 1 ? a.mat_k_off[1] : a.mat_k_off[2]);
    if (row < Rk) mv = mats[(long long)fi * a.mat_item_stride + ok + ((long long)bk * Rk + row) * kL + pt];
    if (a.conj) mv.y = -mv.y;
  }
  if (r[0] <= 0 || r[1] <= 0 || r[2] <= 0) return;  // uniform, before any barrier
  if (tid < 3 * kR * kL) smat[tid] = mv;
  CoarseAddr<3> ca;
  ca.init(a, fi, beta, q0);  // the box of item fi in the caller's array
  __syncthreads();  // matrices

  // ---- mode 0: st0[p0][a1][a2][q] = sum_a0 M0[a0][p0] fine(a0, a1, a2, q)
  if (16 * w < R1 * R2 && (16 * w) / R2 < r[1]) {
    CAcc d[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) czero4(d[t]);
#pragma unroll
    for (int k = 0; k < kR; ++k) {
      if (k < r[0]) {
        float2 m[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) m[t] = smat[k * kL + 4 * t + qn];
#pragma unroll
        for (int t = 0; t < 2; ++t) d[t].re = mf(m[t].x, b[k].x, d[t].re);
#pragma unroll
        for (int t = 0; t < 2; ++t) d[t].im = mf(m[t].x, b[k].y, d[t].im);
#pragma unroll
        for (int t = 0; t < 2; ++t) d[t].re = mf(-m[t].y, b[k].y, d[t].re);
#pragma unroll
        for (int t = 0; t < 2; ++t) d[t].im = mf(m[t].y, b[k].x, d[t].im);
      }
    }
    const int p = 16 * w + blk, a1 = p / R2, a2 = p % R2;
    if (p < R1 * R2 && a1 < r[1] && a2 < r[2]) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          st0[(((4 * t + v) * kR + a1) * kR + a2) * kQ + qn] = make_float2(d[t].re[v], d[t].im[v]);
    }
  }
  __syncthreads();
  const int th = blk >> 3, ph = blk & 7;  // tile half, position within the half
  const int rowh[4] = {4 * th + qn, 0, 0, 0};
  float2* t1 = st1 + w * kL * kR * kQ;  // [p1][a2][q]
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2) {
    const int p0 = w + 4 * s2;
    // ---- mode 1: t1[p1][a2][q] = sum_a1 M1[a1][p1] st0[p0][a1][a2][q], a2 = ph
    {
      CAcc d[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) czero4(d[t]);
      tiles_lds<1, kL>(d, st0 + (p0 * kR * kR + min(ph, r[2] - 1)) * kQ + qn, kR * kQ, smat + kR * kL, rowh,
                       r[1]);
      if (ph < r[2]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) t1[((4 * th + v) * kR + ph) * kQ + qn] = make_float2(d[0].re[v], d[0].im[v]);
      }
    }
    // ---- mode 2: box[p0][p1][p2][q] = sum_a2 M2[a2][p2] t1[p1][a2][q], p1 = ph
    // (the same wave wrote t1: its LDS operations complete in order)
    {
      CAcc d[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) czero4(d[t]);
      tiles_lds<1, kL>(d, t1 + ph * kR * kQ + qn, kQ, smat + 2 * kR * kL, rowh, r[2]);
      if (qn < Qa) {
        float2* dst = box + ca.base + p0 * ca.stride[0] + ph * ca.stride[1] + qn * ca.qstride;
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(4 * th + v) * ca.stride[2]] = make_float2(d[0].re[v], d[0].im[v]);
      }
    }
  }
}

tb_status launch_leaf_fanin_m4(const StageArgs& a, int d, int n_items, const void* in, void* out,
                               const void* mats, hipStream_t stream) {
  if (d != 3) return fail(TB_ERR_UNSUPPORTED, "the matrix-core leaf fan-in is for d = 3");
  if (!a.coarse_global) return fail(TB_ERR_UNSUPPORTED, "the matrix-core leaf fan-in runs the leaves only");
  for (int k = 0; k < 3; ++k)
    if (a.A[k] != kL || a.R[k] > kR)
      return fail(TB_ERR_UNSUPPORTED, "matrix-core leaf fan-in: leaf size 8 and ranks up to 8 only");
  StageArgs b = a;
  b.nsplit = 1;
  b.chunk = a.A[0];
  b.aff_blocks = 0;
  const long long nwg = (long long)n_items * a.nblk * ((a.nrhs + kQ - 1) / kQ);
  if (nwg < 1 || nwg >= (1LL << 31)) return fail(TB_ERR_UNSUPPORTED, "too many workgroups for one launch");
  leaf_fanin_m4<<<dim3((unsigned)nwg), 256, 0, stream>>>(b, (const float2*)in, (float2*)out,
                                                        (const float2*)mats);
  TB_HIP_TRY(hipGetLastError());
  return TB_OK;
}

}  // namespace tb
