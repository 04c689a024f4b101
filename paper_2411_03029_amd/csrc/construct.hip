// Construction of the tensor butterfly on the GPU (Algorithm 1).
//
//  * kernel entries K(x_i, y_j) in FP64 (section 2: any entry in O(1));
//  * one column interpolative decomposition per (side, level, item, mode,
//    node), section 2.1: the sampled unfolding (proxy rows x ID columns) is
//    generated chunk by chunk in LDS and reduced to its R factor by a
//    Householder QR of [R; chunk] (tall-skinny QR, FP64); the column-pivoted
//    QR then runs on the c x c factor, which gives the same pivots, ranks
//    and interpolation matrix as column-pivoted QR on the sampled unfolding
//    itself (A = QR, so every column norm and projection agrees);
//  * the middle-level cores K(tbar, sbar), evaluated in FP64 and stored in
//    the requested precisions.
//
// The host walks the levels of Algorithm 1 in order: the IDs of one level
// run in one launch, and their ranks and skeletons are read back to build
// the column lists of the next level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "cplx.h"
#include "tb_internal.h"

namespace tb {

constexpr int kIdThreads = 256;
constexpr double kTieRel = 1e-10;

struct KernelSpec {
  int kind, d;
  long long n;
  double omega, ra, rb, rden;
  const double* nux;  // non-uniform DFT: d * n target coordinates
};

// K(x^i, y^j) for multi-indices ti, sj, in FP64.
__device__ double2 entry(const KernelSpec& ks, const int* ti, const int* sj) {
  double s, c;
  if (ks.kind == TB_KERNEL_NUDFT) {
    // exp(2 pi i x.y), x_k = X[k][i_k], y = j/n: phase in FP64, and sincospi
    // reduces 2 phase modulo 2 exactly
    double ph = 0.0;
    for (int k = 0; k < ks.d; ++k) ph += ks.nux[(long long)k * ks.n + ti[k]] * (double)sj[k];
    sincospi(2.0 * (ph / (double)ks.n), &s, &c);
    return make_double2(c, s);
  }
  if (ks.kind == TB_KERNEL_FOURIER) {
    // exp(-2 pi i (i.k)/n), k = j - n/2, phase reduced exactly mod n
    long long p = 0;
    const long long h = ks.n / 2;
    for (int k = 0; k < ks.d; ++k) p += (long long)ti[k] * ((long long)sj[k] - h);
    p %= ks.n;
    if (p < 0) p += ks.n;
    sincospi(-2.0 * (double)p / (double)ks.n, &s, &c);
    return make_double2(c, s);
  }
  if (ks.kind == TB_KERNEL_DFT) {
    // exp(2 pi i br(i).br(j)/n): the bit-reversed indices' product is
    // reduced exactly modulo the power-of-two n
    const int bits = 63 - __clzll((unsigned long long)ks.n);
    unsigned long long p = 0;
    for (int k = 0; k < ks.d; ++k) {
      const unsigned long long x = __brev((unsigned)ti[k]) >> (32 - bits);
      const unsigned long long y = __brev((unsigned)sj[k]) >> (32 - bits);
      p += x * y;
    }
    p &= (unsigned long long)ks.n - 1;
    sincospi(2.0 * (double)p / (double)ks.n, &s, &c);
    return make_double2(c, s);
  }
  if (ks.kind == TB_KERNEL_HELMHOLTZ) {
    // exp(+i omega rho)/rho; d = 3: x = i/n, y = j/n + (2, 0, 0) (cubes);
    // d = 2: x = (i/n, 0), y = (j/n, 1) (parallel plates 1 apart)
    const double inv = 1.0 / (double)ks.n;
    double r2 = ks.d == 2 ? 1.0 : 0.0;
    for (int k = 0; k < ks.d; ++k) {
      double dx = (double)(ti[k] - sj[k]) * inv - ((k == 0 && ks.d == 3) ? 2.0 : 0.0);
      r2 += dx * dx;
    }
    const double rho = sqrt(r2);
    sincos(ks.omega * rho, &s, &c);
    return make_double2(c / rho, s / rho);
  }
  const double inv = 1.0 / (double)ks.n;
  if (ks.d == 3) {
    // 3-D Radon transform: phase x.k + c(x)|k|, c = (a + b s1 s2 s3)/den
    double ph = 0.0, k2 = 0.0, sp = 1.0;
    for (int k = 0; k < 3; ++k) {
      const double x = ti[k] * inv, kk = (double)(sj[k] - ks.n / 2);
      double sk, ck;
      sincospi(2.0 * x, &sk, &ck);
      sp *= sk;
      ph += x * kk;
      k2 += kk * kk;
    }
    ph += (ks.ra + ks.rb * sp) / ks.rden * sqrt(k2);
    sincospi(2.0 * ph, &s, &c);
    return make_double2(c, s);
  }
  // generalized Radon transform, d = 2
  const double x1 = ti[0] * inv, x2 = ti[1] * inv;
  const double k1 = (double)(sj[0] - ks.n / 2), k2 = (double)(sj[1] - ks.n / 2);
  double s1, c1, s2, c2;
  sincospi(2.0 * x1, &s1, &c1);
  sincospi(2.0 * x2, &s2, &c2);
  const double cc1 = (ks.ra + ks.rb * s1 * s2) / ks.rden;
  const double cc2 = (ks.ra + ks.rb * c1 * c2) / ks.rden;
  const double ph = x1 * k1 + x2 * k2 + sqrt(cc1 * cc1 * k1 * k1 + cc2 * cc2 * k2 * k2);
  // exp(2 pi i ph): sincospi reduces 2 ph modulo 2 exactly
  sincospi(2.0 * ph, &s, &c);
  return make_double2(c, s);
}

// ------------------------------------------------------------ ID kernel --
// Proxy list: node [lo, lo + len) sampled at cnt points
//   lo + floor((2q + 1) len / (2 cnt)), which is every index when cnt = len.
struct IdDesc {
  int lo[2 * kMaxD], len[2 * kMaxD], cnt[2 * kMaxD];  // target modes, then source
  int col_list;        // list (0..2d-1) replaced by the ID's columns
  int ncols, col_off;  // columns: global indices in cols[col_off ..]
  long long nrows;     // product of cnt
  long long x_off;     // output: X (ncols x ncols slot), skel (ncols slot)
};

struct IdArgs {
  KernelSpec ks;
  double eps;
  int mc;              // rows per chunk
  int nids;
};

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconjmul(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Householder reflection of the entries (x0, xs[...]) of one column:
// returns alpha (the new diagonal), sets v0 = x0 - alpha and scale
// 2 / ||v||^2 (0 when the column is already zero).
__device__ void reflector(double2 x0, double tail2, double2* alpha, double2* v0, double* scale) {
  double nrm2 = zabs2(x0) + tail2;
  if (nrm2 == 0.0) {
    *alpha = x0;
    *v0 = make_double2(0, 0);
    *scale = 0.0;
    return;
  }
  double nrm = sqrt(nrm2);
  double ax = sqrt(zabs2(x0));
  double2 ph = ax > 0 ? make_double2(x0.x / ax, x0.y / ax) : make_double2(1.0, 0.0);
  *alpha = make_double2(-ph.x * nrm, -ph.y * nrm);
  *v0 = make_double2(x0.x - alpha->x, x0.y - alpha->y);
  double vn2 = zabs2(*v0) + tail2;
  *scale = vn2 > 0 ? 2.0 / vn2 : 0.0;
}

// One workgroup per ID.  LDS: M = (c + mc) x c column-major (R on top,
// chunk below), plus small scratch.
__global__ void __launch_bounds__(kIdThreads)
    id_kernel(IdArgs a, const IdDesc* __restrict__ descs, const int* __restrict__ cols,
              double2* __restrict__ Xout, int* __restrict__ skel_out, int* __restrict__ rank_out) {
  extern __shared__ unsigned char smem_raw[];
  const IdDesc& D = descs[blockIdx.x];
  const int c = D.ncols;
  const int mc = a.mc;
  const int ld = c + mc;  // leading dimension (rows) of M
  double2* M = reinterpret_cast<double2*>(smem_raw);
  double2* shv = M + (size_t)ld * c;          // [0] v0, [1] alpha
  double* shd = reinterpret_cast<double*>(shv + 2);  // scratch doubles (>= 8 + c)
  int* perm = reinterpret_cast<int*>(shd + 8 + kMaxCols);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nw = kIdThreads / 64;
  const int d = a.ks.d;
  const int nl = 2 * d;

  for (int i = tid; i < ld * c; i += kIdThreads) M[i] = make_double2(0, 0);
  __syncthreads();

  // ---- tall-skinny QR over chunks of proxy rows
  for (long long r0 = 0; r0 < D.nrows; r0 += mc) {
    const int rows = (int)min((long long)mc, D.nrows - r0);
    for (int i = tid; i < mc; i += kIdThreads) {
      if (i < rows) {
        long long r = r0 + i;
        int ti[kMaxD], sj[kMaxD];
        for (int li = nl - 1; li >= 0; --li) {
          int q = (int)(r % D.cnt[li]);
          r /= D.cnt[li];
          int idx = D.lo[li] + (D.cnt[li] == D.len[li]
                                    ? q
                                    : (int)(((2LL * q + 1) * D.len[li]) / (2LL * D.cnt[li])));
          if (li < d) ti[li] = idx;
          else sj[li - d] = idx;
        }
        int* tgt = D.col_list < d ? ti : sj;
        const int km = D.col_list < d ? D.col_list : D.col_list - d;
        for (int j = 0; j < c; ++j) {
          tgt[km] = cols[D.col_off + j];
          M[(size_t)j * ld + c + i] = entry(a.ks, ti, sj);
        }
      } else {
        for (int j = 0; j < c; ++j) M[(size_t)j * ld + c + i] = make_double2(0, 0);
      }
    }
    __syncthreads();
    for (int j = 0; j < c; ++j) {
      // reflector of column j: entries M[j][j] and the chunk rows
      if (w == 0) {
        double t2 = 0.0;
        for (int i = lane; i < mc; i += 64) t2 += zabs2(M[(size_t)j * ld + c + i]);
        t2 = wave_sum(t2);
        if (lane == 0) {
          double2 al, v0;
          double sc;
          reflector(M[(size_t)j * ld + j], t2, &al, &v0, &sc);
          shv[0] = v0;
          shv[1] = al;
          shd[0] = sc;
        }
      }
      __syncthreads();
      const double2 v0 = shv[0];
      const double sc = shd[0];
      if (sc != 0.0) {
        for (int q = j + 1 + w; q < c; q += nw) {
          // the R-row term enters the wave sum once (lane 0)
          double2 s = lane == 0 ? zconjmul(v0, M[(size_t)q * ld + j]) : make_double2(0, 0);
          double sr = s.x, si = s.y;
          for (int i = lane; i < mc; i += 64) {
            double2 t = zconjmul(M[(size_t)j * ld + c + i], M[(size_t)q * ld + c + i]);
            sr += t.x;
            si += t.y;
          }
          sr = wave_sum(sr);
          si = wave_sum(si);
          const double2 f = make_double2(sc * sr, sc * si);
          if (lane == 0) {
            double2 u = zmul(v0, f);
            M[(size_t)q * ld + j].x -= u.x;
            M[(size_t)q * ld + j].y -= u.y;
          }
          for (int i = lane; i < mc; i += 64) {
            double2 u = zmul(M[(size_t)j * ld + c + i], f);
            M[(size_t)q * ld + c + i].x -= u.x;
            M[(size_t)q * ld + c + i].y -= u.y;
          }
        }
      }
      __syncthreads();
      if (tid == 0 && sc != 0.0) M[(size_t)j * ld + j] = shv[1];
      for (int i = tid; i < mc; i += kIdThreads) M[(size_t)j * ld + c + i] = make_double2(0, 0);
      __syncthreads();
    }
  }

  // ---- column-pivoted QR of the c x c factor (rows 0..c-1 of M)
  if (tid < c) perm[tid] = tid;
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < c; ++j)
      for (int i = 0; i <= j; ++i) s += zabs2(M[(size_t)j * ld + i]);
    shd[1] = sqrt(s);  // ||A||_F
  }
  __syncthreads();
  const double normA = shd[1];
  double* nrm = shd + 8;
  int rank = c;
  for (int k = 0; k < c; ++k) {
    for (int j = k + w; j < c; j += nw) {
      double s = 0.0;
      for (int i = k + lane; i < c; i += 64) s += zabs2(M[(size_t)j * ld + i]);
      s = wave_sum(s);
      if (lane == 0) nrm[j] = sqrt(s);
    }
    __syncthreads();
    if (tid == 0) {
      double tail2 = 0.0, mx = 0.0;
      for (int j = k; j < c; ++j) {
        tail2 += nrm[j] * nrm[j];
        mx = fmax(mx, nrm[j]);
      }
      int stop = (k >= 1 && sqrt(tail2) <= a.eps * normA) ? 1 : 0;
      int piv = k, best = 1 << 30;
      for (int j = k; j < c; ++j)
        if (nrm[j] >= (1.0 - kTieRel) * mx && perm[j] < best) {
          best = perm[j];
          piv = j;
        }
      shd[2] = stop;
      shd[3] = piv;
    }
    __syncthreads();
    if (shd[2] != 0.0) {
      rank = k;
      break;
    }
    const int piv = (int)shd[3];
    if (piv != k) {
      for (int i = tid; i < c; i += kIdThreads) {
        double2 t = M[(size_t)k * ld + i];
        M[(size_t)k * ld + i] = M[(size_t)piv * ld + i];
        M[(size_t)piv * ld + i] = t;
      }
      if (tid == 0) {
        int t = perm[k];
        perm[k] = perm[piv];
        perm[piv] = t;
      }
    }
    __syncthreads();
    if (w == 0) {
      double t2 = 0.0;
      for (int i = k + 1 + lane; i < c; i += 64) t2 += zabs2(M[(size_t)k * ld + i]);
      t2 = wave_sum(t2);
      if (lane == 0) {
        double2 al, v0;
        double sc;
        reflector(M[(size_t)k * ld + k], t2, &al, &v0, &sc);
        shv[0] = v0;
        shv[1] = al;
        shd[0] = sc;
      }
    }
    __syncthreads();
    const double2 v0 = shv[0];
    const double sc = shd[0];
    if (sc != 0.0) {
      for (int q = k + 1 + w; q < c; q += nw) {
        double2 s = lane == 0 ? zconjmul(v0, M[(size_t)q * ld + k]) : make_double2(0, 0);
        double sr = s.x, si = s.y;
        for (int i = k + 1 + lane; i < c; i += 64) {
          double2 t = zconjmul(M[(size_t)k * ld + i], M[(size_t)q * ld + i]);
          sr += t.x;
          si += t.y;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        const double2 f = make_double2(sc * sr, sc * si);
        if (lane == 0) {
          double2 u = zmul(v0, f);
          M[(size_t)q * ld + k].x -= u.x;
          M[(size_t)q * ld + k].y -= u.y;
        }
        for (int i = k + 1 + lane; i < c; i += 64) {
          double2 u = zmul(M[(size_t)k * ld + i], f);
          M[(size_t)q * ld + i].x -= u.x;
          M[(size_t)q * ld + i].y -= u.y;
        }
      }
    }
    __syncthreads();
    if (tid == 0 && sc != 0.0) M[(size_t)k * ld + k] = shv[1];
    for (int i = k + 1 + tid; i < c; i += kIdThreads) M[(size_t)k * ld + i] = make_double2(0, 0);
    __syncthreads();
  }
  if (normA == 0.0) rank = 1;

  // ---- X = [I, R11^{-1} R12] in original column order
  double2* X = Xout + D.x_off;  // r x c, row-major
  for (int i = tid; i < rank * c; i += kIdThreads) X[i] = make_double2(0, 0);
  __syncthreads();
  for (int i = tid; i < rank; i += kIdThreads) {
    X[(size_t)i * c + perm[i]] = make_double2(1, 0);
    skel_out[(size_t)blockIdx.x * kMaxCols + i] = cols[D.col_off + perm[i]];
  }
  for (int q = rank + tid; q < c; q += kIdThreads) {
    // back substitution R11 t = R12(:, q); rows rank-1 .. 0
    double2 tv[kMaxCols];
    for (int i = rank - 1; i >= 0; --i) {
      double2 s = M[(size_t)q * ld + i];
      for (int j = i + 1; j < rank; ++j) {
        double2 u = zmul(M[(size_t)j * ld + i], tv[j]);
        s.x -= u.x;
        s.y -= u.y;
      }
      double2 dd = M[(size_t)i * ld + i];
      double den = zabs2(dd);
      // s / dd
      tv[i] = den > 0 ? make_double2((s.x * dd.x + s.y * dd.y) / den, (s.y * dd.x - s.x * dd.y) / den)
                      : make_double2(0, 0);
    }
    for (int i = 0; i < rank; ++i) X[(size_t)i * c + perm[q]] = tv[i];
  }
  if (tid == 0) rank_out[blockIdx.x] = rank;
}

// ----------------------------------------------------------- core kernel --
struct CoreEvalArgs {
  KernelSpec ks;
  long long nS, nT;
  int Rs, Rt;          // row length of the skeleton tables (max padded rank)
  unsigned mask;
  int splits;
};

__global__ void __launch_bounds__(256)
    core_eval(CoreEvalArgs a, const int* __restrict__ meta, const long long* __restrict__ off,
              const int* __restrict__ sskel, const int* __restrict__ tskel, double2* __restrict__ c128,
              float2* __restrict__ c64, unsigned* __restrict__ cbf) {
  const int pair = blockIdx.y;
  const int* m = meta + pair * kPairMeta;
  const int RT = m[0], RS = m[1], RTp = m[2];
  const int d = a.ks.d;
  const long long t = pair / a.nS, s = pair % a.nS;
  const long long sitem = s * a.nT + t, titem = t * a.nS + s;
  const long long total = (long long)RTp * RS;
  const long long base = off[pair];
  for (long long e = blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)a.splits * 256) {
    const int row = (int)(e % RTp), col = (int)(e / RTp);
    double2 v = make_double2(0, 0);
    if (row < RT) {
      int ti[kMaxD], sj[kMaxD];
      int fr = row, fc = col;
      for (int k = d - 1; k >= 0; --k) {
        int rt = m[3 + k], rs = m[kMetaRs + k];
        ti[k] = tskel[(titem * d + k) * a.Rt + fr % rt];
        sj[k] = sskel[(sitem * d + k) * a.Rs + fc % rs];
        fr /= rt;
        fc /= rs;
      }
      v = entry(a.ks, ti, sj);
    }
    if (a.mask & TB_STORE_C128) c128[base + e] = v;
    if (a.mask & TB_STORE_C64) c64[base + e] = make_float2((float)v.x, (float)v.y);
    if (a.mask & TB_STORE_CBF16)
      cbf[base + e] = (unsigned)f32_to_bf16((float)v.x) | ((unsigned)f32_to_bf16((float)v.y) << 16);
  }
}

// TB_CQ16 encoding, one wave per core column: the scale is the column's
// largest real or imaginary magnitude / 32767 (FP32), and every part is
// rounded to the nearest multiple of it (an int16); real part in the low
// half of the word, imaginary part in the high half.  Padding rows hold 0.
__device__ __forceinline__ unsigned q16_pack(double re, double im, float s) {
  int qr = 0, qi = 0;
  if (s > 0.f) {
    qr = (int)rint(re / (double)s);
    qi = (int)rint(im / (double)s);
    qr = max(-32767, min(32767, qr));
    qi = max(-32767, min(32767, qi));
  }
  return (unsigned)(unsigned short)(short)qr | ((unsigned)(unsigned short)(short)qi << 16);
}

template <class S>
__global__ void __launch_bounds__(256)
    core_encode_q16(const int* __restrict__ meta, const long long* __restrict__ off,
                    const long long* __restrict__ col_off, const S* __restrict__ src,
                    unsigned* __restrict__ q, float* __restrict__ scale) {
  const int pair = blockIdx.x;
  const int col = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int* m = meta + pair * kPairMeta;
  const int RS = m[1], RTp = m[2];
  if (col >= RS) return;  // whole wave; the kernel has no barrier
  const long long b = off[pair] + (long long)col * RTp;
  double mx = 0.0;
  for (int r = lane; r < RTp; r += 64)
    mx = fmax(mx, fmax(fabs((double)src[b + r].x), fabs((double)src[b + r].y)));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  const float s = (float)(mx / 32767.0);
  for (int r = lane; r < RTp; r += 64) q[b + r] = q16_pack((double)src[b + r].x, (double)src[b + r].y, s);
  if (lane == 0) scale[col_off[pair] + col] = s;
}

static unsigned q16_pack_host(double re, double im, float s) {
  long qr = 0, qi = 0;
  if (s > 0.f) {
    qr = std::lrint(re / (double)s);
    qi = std::lrint(im / (double)s);
    qr = std::max(-32767L, std::min(32767L, qr));
    qi = std::max(-32767L, std::min(32767L, qi));
  }
  return (unsigned)(unsigned short)(short)qr | ((unsigned)(unsigned short)(short)qi << 16);
}

static KernelSpec spec_of(const Plan& p) {
  KernelSpec ks;
  ks.kind = p.kind;
  ks.d = p.d;
  ks.n = p.n;
  ks.omega = p.omega;
  ks.ra = p.ra;
  ks.rb = p.rb;
  ks.rden = p.rden;
  ks.nux = p.nux_d;
  return ks;
}

tb_status launch_core_eval(Plan& p, hipStream_t stream, const double2* host_cores) {
  unsigned mask = p.store_mask ? p.store_mask : TB_STORE_C64;
  const size_t esz[5] = {sizeof(double2), sizeof(float2), sizeof(unsigned), 0, sizeof(unsigned)};
  for (int t = 0; t < 5; ++t)
    if (esz[t] && (mask & (1u << t))) TB_TRY(dev_alloc(p, &p.cores[t], (size_t)p.core_total * esz[t]));
  if (mask & TB_STORE_CQ16)
    TB_TRY(dev_alloc(p, reinterpret_cast<void**>(&p.core_scale), (size_t)std::max(1LL, p.col_total) * sizeof(float)));
  if (host_cores && (mask & TB_STORE_CQ16)) {
    const size_t N = (size_t)p.core_total;
    std::vector<unsigned> h(N);
    std::vector<float> sc((size_t)p.col_total);
    for (long long pr = 0; pr < p.npairs; ++pr) {
      const int RS = p.pair_meta[(size_t)pr * kPairMeta + 1], RTp = p.pair_meta[(size_t)pr * kPairMeta + 2];
      for (int c = 0; c < RS; ++c) {
        const size_t b = (size_t)(p.core_off[(size_t)pr] + (long long)c * RTp);
        double mx = 0.0;
        for (int r = 0; r < RTp; ++r)
          mx = std::max(mx, std::max(std::fabs(host_cores[b + r].x), std::fabs(host_cores[b + r].y)));
        const float s = (float)(mx / 32767.0);
        for (int r = 0; r < RTp; ++r) h[b + r] = q16_pack_host(host_cores[b + r].x, host_cores[b + r].y, s);
        sc[(size_t)(p.col_off[(size_t)pr] + c)] = s;
      }
    }
    TB_HIP_TRY(hipMemcpy(p.cores[TB_CQ16], h.data(), N * sizeof(unsigned), hipMemcpyHostToDevice));
    TB_HIP_TRY(hipMemcpy(p.core_scale, sc.data(), sc.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  if (host_cores) {
    const size_t N = (size_t)p.core_total;
    if (mask & TB_STORE_C128)
      TB_HIP_TRY(hipMemcpy(p.cores[TB_C128], host_cores, N * sizeof(double2), hipMemcpyHostToDevice));
    if (mask & TB_STORE_C64) {
      std::vector<float2> h(N);
      for (size_t i = 0; i < N; ++i) h[i] = make_float2((float)host_cores[i].x, (float)host_cores[i].y);
      TB_HIP_TRY(hipMemcpy(p.cores[TB_C64], h.data(), N * sizeof(float2), hipMemcpyHostToDevice));
    }
    if (mask & TB_STORE_CBF16) {
      std::vector<unsigned> h(N);
      for (size_t i = 0; i < N; ++i)
        h[i] = (unsigned)f32_to_bf16((float)host_cores[i].x) |
               ((unsigned)f32_to_bf16((float)host_cores[i].y) << 16);
      TB_HIP_TRY(hipMemcpy(p.cores[TB_CBF16], h.data(), N * sizeof(unsigned), hipMemcpyHostToDevice));
    }
    return TB_OK;
  }
  if ((mask & 23u) == 0) return TB_OK;  // no stored cores (on-the-fly applies only)
  // TB_CQ16 alone: FP32 entries in a temporary buffer, encoded below
  float2* tmp64 = nullptr;
  if ((mask & TB_STORE_CQ16) && !(mask & (TB_STORE_C128 | TB_STORE_C64)))
    TB_HIP_TRY(hipMalloc(&tmp64, (size_t)p.core_total * sizeof(float2)));
  CoreEvalArgs a;
  a.ks = spec_of(p);
  a.nS = p.nS;
  a.nT = p.nT;
  a.Rs = 0;
  a.Rt = 0;
  for (int k = 0; k < p.d; ++k) {
    a.Rs = std::max(a.Rs, p.src[p.Lt].R[k]);
    a.Rt = std::max(a.Rt, p.tgt[p.Ls].R[k]);
  }
  a.mask = mask | (tmp64 ? TB_STORE_C64 : 0u);
  a.splits = 8;
  dim3 grid((unsigned)a.splits, (unsigned)p.npairs);
  float2* c64 = tmp64 ? tmp64 : (float2*)p.cores[TB_C64];
  core_eval<<<grid, 256, 0, stream>>>(a, p.pair_meta_d, p.core_off_d, p.top_src_skel_d, p.top_tgt_skel_d,
                                     (double2*)p.cores[TB_C128], c64, (unsigned*)p.cores[TB_CBF16]);
  tb_status st = hipGetLastError() == hipSuccess ? TB_OK : fail(TB_ERR_HIP, "core_eval launch failed");
  if (st == TB_OK && (mask & TB_STORE_CQ16)) {
    int maxRS = 1;
    for (long long pr = 0; pr < p.npairs; ++pr) maxRS = std::max(maxRS, p.pair_meta[(size_t)pr * kPairMeta + 1]);
    dim3 eg((unsigned)p.npairs, (unsigned)((maxRS + 3) / 4));
    if (p.cores[TB_C128])
      core_encode_q16<double2><<<eg, 256, 0, stream>>>(p.pair_meta_d, p.core_off_d, p.col_off_d,
                                                      (const double2*)p.cores[TB_C128],
                                                      (unsigned*)p.cores[TB_CQ16], p.core_scale);
    else
      core_encode_q16<float2><<<eg, 256, 0, stream>>>(p.pair_meta_d, p.core_off_d, p.col_off_d, c64,
                                                     (unsigned*)p.cores[TB_CQ16], p.core_scale);
    if (hipGetLastError() != hipSuccess) st = fail(TB_ERR_HIP, "core encoding launch failed");
  }
  if (tmp64) {
    if (hipStreamSynchronize(stream) != hipSuccess && st == TB_OK) st = fail(TB_ERR_HIP, "core encoding failed");
    (void)hipFree(tmp64);
  }
  return st;
}

// -------------------------------------------------------------- driver --
static int proxy_count(int p, int len) { return (p <= 0 || len <= p) ? len : p; }

static int flat_digit(int flat, int level, int d, int k) {
  return (flat >> (level * (d - 1 - k))) & ((1 << level) - 1);
}

// Runs the IDs of one level (source side if `source`), filling lv.ids.
static tb_status run_level(Plan& p, Level& lv, const Level* prev, bool source, hipStream_t stream,
                           int max_rank) {
  const int d = p.d;
  const int outer_lvl = source ? p.Ls : p.Lt;   // s (source) or t (target)
  const int depth = source ? p.Lt - lv.l : p.Ls - lv.l;
  const int nids = lv.nitems * d * lv.nb;
  std::vector<IdDesc> descs((size_t)nids);
  std::vector<int> cols;
  cols.reserve((size_t)nids * p.leaf * 2);
  long long xoff = 0;
  int cmax = 0;
  for (int it = 0; it < lv.nitems; ++it) {
    const int outer = it >> (d * lv.l);
    const int inner = it & ((1 << (d * lv.l)) - 1);
    for (int k = 0; k < d; ++k)
      for (int b = 0; b < lv.nb; ++b) {
        IdDesc& D = descs[((size_t)it * d + k) * lv.nb + b];
        D.col_off = (int)cols.size();
        if (!prev) {
          const int node = flat_digit(outer, outer_lvl, d, k) * (1 << depth) + b;
          for (int j = 0; j < p.leaf; ++j) cols.push_back(node * p.leaf + j);
        } else {
          int pin = 0;
          for (int m = 0; m < d; ++m) pin = (pin << (lv.l - 1)) | (flat_digit(inner, lv.l, d, m) >> 1);
          const int par = (outer << (d * (lv.l - 1))) | pin;
          for (int h = 0; h < 2; ++h) {
            const IdRec& ch = prev->id(par, k, 2 * b + h, d);
            cols.insert(cols.end(), ch.skel.begin(), ch.skel.end());
          }
        }
        D.ncols = (int)cols.size() - D.col_off;
        if (D.ncols > kMaxCols)
          return fail(TB_ERR_UNSUPPORTED, "an ID has " + std::to_string(D.ncols) +
                                              " columns, above the GPU limit of " +
                                              std::to_string(kMaxCols));
        cmax = std::max(cmax, D.ncols);
        const int pair_cnt = p.proxy_pair <= 0 ? -1 : p.proxy_pair * D.ncols;
        for (int m = 0; m < d; ++m) {
          // target list m, then source list m
          const int tl = m, sl = d + m;
          if (source) {
            const int tb = flat_digit(inner, lv.l, d, m);
            D.lo[tl] = tb * (int)(p.n >> lv.l);
            D.len[tl] = (int)(p.n >> lv.l);
            D.cnt[tl] = proxy_count(m == k ? pair_cnt : p.proxy_other, D.len[tl]);
            if (m == k) {
              D.lo[sl] = 0;
              D.len[sl] = 1;
              D.cnt[sl] = 1;
            } else {
              const int sb = flat_digit(outer, outer_lvl, d, m);
              D.lo[sl] = sb * (int)(p.n >> outer_lvl);
              D.len[sl] = (int)(p.n >> outer_lvl);
              D.cnt[sl] = proxy_count(p.proxy_other, D.len[sl]);
            }
          } else {
            const int nb_ = flat_digit(inner, lv.l, d, m);
            D.lo[sl] = nb_ * (int)(p.n >> lv.l);
            D.len[sl] = (int)(p.n >> lv.l);
            D.cnt[sl] = proxy_count(m == k ? pair_cnt : p.proxy_other, D.len[sl]);
            if (m == k) {
              D.lo[tl] = 0;
              D.len[tl] = 1;
              D.cnt[tl] = 1;
            } else {
              const int tb = flat_digit(outer, outer_lvl, d, m);
              D.lo[tl] = tb * (int)(p.n >> outer_lvl);
              D.len[tl] = (int)(p.n >> outer_lvl);
              D.cnt[tl] = proxy_count(p.proxy_other, D.len[tl]);
            }
          }
        }
        D.col_list = source ? d + k : k;
        D.nrows = 1;
        for (int li = 0; li < 2 * d; ++li) D.nrows *= D.cnt[li];
        D.x_off = xoff;
        xoff += (long long)D.ncols * D.ncols;
      }
  }
  // device buffers for this level
  IdDesc* descs_d = nullptr;
  int *cols_d = nullptr, *skel_d = nullptr, *rank_d = nullptr;
  double2* X_d = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(descs_d);
    (void)hipFree(cols_d);
    (void)hipFree(skel_d);
    (void)hipFree(rank_d);
    (void)hipFree(X_d);
  };
  auto hip_ok = [&](hipError_t e, const char* what) -> tb_status {
    if (e == hipSuccess) return TB_OK;
    cleanup();
    return fail(TB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  TB_TRY(hip_ok(hipMalloc(&descs_d, sizeof(IdDesc) * nids), "hipMalloc"));
  TB_TRY(hip_ok(hipMalloc(&cols_d, sizeof(int) * std::max<size_t>(1, cols.size())), "hipMalloc"));
  TB_TRY(hip_ok(hipMalloc(&skel_d, sizeof(int) * (size_t)nids * kMaxCols), "hipMalloc"));
  TB_TRY(hip_ok(hipMalloc(&rank_d, sizeof(int) * nids), "hipMalloc"));
  TB_TRY(hip_ok(hipMalloc(&X_d, sizeof(double2) * std::max<long long>(1, xoff)), "hipMalloc"));
  TB_TRY(hip_ok(hipMemcpyAsync(descs_d, descs.data(), sizeof(IdDesc) * nids, hipMemcpyHostToDevice, stream),
                "hipMemcpyAsync"));
  TB_TRY(hip_ok(hipMemcpyAsync(cols_d, cols.data(), sizeof(int) * cols.size(), hipMemcpyHostToDevice, stream),
                "hipMemcpyAsync"));
  IdArgs ia;
  ia.ks = spec_of(p);
  ia.eps = p.eps_id;
  ia.nids = nids;
  // chunk rows: keep the (c + mc) x c work matrix within the LDS budget
  int dev = 0, lds_max = 0;
  TB_TRY(hip_ok(hipGetDevice(&dev), "hipGetDevice"));
  TB_TRY(hip_ok(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                "hipDeviceGetAttribute"));
  const size_t extra = sizeof(double2) * 2 + sizeof(double) * (8 + kMaxCols) + sizeof(int) * kMaxCols;
  const size_t budget = std::min<size_t>((size_t)lds_max, 96 * 1024) - extra;
  int mc = (int)(budget / (sizeof(double2) * cmax)) - cmax;
  mc = std::min(256, mc / 16 * 16);
  if (mc < 16) {
    const size_t big = (size_t)lds_max - extra;
    mc = std::min(256, ((int)(big / (sizeof(double2) * cmax)) - cmax) / 16 * 16);
  }
  if (mc < 16) {
    cleanup();
    return fail(TB_ERR_UNSUPPORTED, "ID with " + std::to_string(cmax) + " columns exceeds the LDS budget");
  }
  ia.mc = mc;
  size_t lds = sizeof(double2) * ((size_t)(cmax + mc) * cmax) + extra;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(id_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    TB_TRY(hip_ok(e, "hipFuncSetAttribute"));
  }
  id_kernel<<<nids, kIdThreads, lds, stream>>>(ia, descs_d, cols_d, X_d, skel_d, rank_d);
  TB_TRY(hip_ok(hipGetLastError(), "id_kernel launch"));
  std::vector<int> ranks(nids), skel((size_t)nids * kMaxCols);
  std::vector<double2> X((size_t)std::max<long long>(1, xoff));
  TB_TRY(hip_ok(hipMemcpyAsync(ranks.data(), rank_d, sizeof(int) * nids, hipMemcpyDeviceToHost, stream),
                "hipMemcpyAsync"));
  TB_TRY(hip_ok(hipMemcpyAsync(skel.data(), skel_d, sizeof(int) * skel.size(), hipMemcpyDeviceToHost, stream),
                "hipMemcpyAsync"));
  TB_TRY(hip_ok(hipMemcpyAsync(X.data(), X_d, sizeof(double2) * X.size(), hipMemcpyDeviceToHost, stream),
                "hipMemcpyAsync"));
  TB_TRY(hip_ok(hipStreamSynchronize(stream), "hipStreamSynchronize"));
  cleanup();
  lv.ids.assign((size_t)nids, IdRec{});
  for (int i = 0; i < nids; ++i) {
    IdRec& id = lv.ids[(size_t)i];
    const IdDesc& D = descs[(size_t)i];
    id.r = ranks[(size_t)i];
    id.c = D.ncols;
    if (id.r < 1 || id.r > id.c) return fail(TB_ERR_NUMERIC, "ID returned an invalid rank");
    if (max_rank > 0 && id.r > max_rank)
      return fail(TB_ERR_NUMERIC, "ID rank " + std::to_string(id.r) + " exceeds max_rank " +
                                      std::to_string(max_rank));
    id.skel.assign(skel.begin() + (size_t)i * kMaxCols, skel.begin() + (size_t)i * kMaxCols + id.r);
    id.X.resize((size_t)id.r * id.c);
    for (size_t e = 0; e < id.X.size(); ++e) {
      double2 z = X[(size_t)D.x_off + e];
      id.X[e] = cd(z.x, z.y);
    }
  }
  return TB_OK;
}

}  // namespace tb

using namespace tb;

extern "C" tb_status tb_construct(tb_kernel kind, int d, long long n, double omega, double tol,
                                  const tb_options* opt, void* hip_stream, tb_plan* out) {
  if (!out) return fail(TB_ERR_INVALID_ARG, "tb_construct: null output");
  *out = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  tb_options o;
  std::memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (kind < TB_KERNEL_FOURIER || kind > TB_KERNEL_DFT)
    return fail(TB_ERR_INVALID_ARG, "unknown kernel kind");
  if (kind == TB_KERNEL_NUDFT && !o.nudft_x)
    return fail(TB_ERR_INVALID_ARG, "the non-uniform DFT needs tb_options.nudft_x");
  if (d < 1 || d > 8) return fail(TB_ERR_INVALID_ARG, "d must be in [1, 8]");
  if (d < 2 || d > (kind == TB_KERNEL_DFT ? kMaxD : 3))
    return fail(TB_ERR_UNSUPPORTED,
                "kernel/dimension pair not built (every kernel has d = 2 and 3, the uniform DFT 2 .. 6)");
  if (!(tol > 0.0 && tol < 1.0)) return fail(TB_ERR_INVALID_ARG, "tol must be in (0, 1)");
  if (kind == TB_KERNEL_HELMHOLTZ && !(omega > 0.0)) return fail(TB_ERR_INVALID_ARG, "omega must be > 0");
  const int leaf = o.leaf_size ? o.leaf_size : 8;
  if (leaf < 1 || leaf > 64) return fail(TB_ERR_INVALID_ARG, "leaf_size must be in [1, 64]");
  if (n < leaf || n > (1LL << 20)) return fail(TB_ERR_INVALID_ARG, "n out of range");
  if (kind == TB_KERNEL_DFT && (n < 2 || (n & (n - 1)) != 0))
    return fail(TB_ERR_INVALID_ARG, "the bit-reversal ordering needs n a power of two");
  int L = 0;
  while (((long long)leaf << L) < n) ++L;
  if (((long long)leaf << L) != n) return fail(TB_ERR_INVALID_ARG, "n must equal leaf_size * 2^L");
  auto plan = std::make_unique<Plan>();
  Plan& p = *plan;
  p.kind = kind;
  p.d = d;
  p.n = n;
  p.leaf = leaf;
  p.L = L;
  p.Lt = o.lt_override > 0 ? o.lt_override - 1 : L - L / 2;
  if (p.Lt > L) return fail(TB_ERR_INVALID_ARG, "lt_override beyond the tree depth");
  p.Ls = L - p.Lt;
  p.omega = kind == TB_KERNEL_HELMHOLTZ ? omega : 0.0;
  p.tol = tol;
  p.eps_id = tol * (o.id_tol_scale > 0 ? o.id_tol_scale : 0.3);
  p.proxy_pair = o.proxy_pair == 0 ? 2 : o.proxy_pair;
  p.proxy_other = o.proxy_other == 0 ? (d == 2 ? 4 * leaf : (d == 3 ? 4 : 2)) : o.proxy_other;
  if (o.radon_custom) {
    p.ra = o.radon_a;
    p.rb = o.radon_b;
    p.rden = o.radon_den;
    if (p.rden == 0.0) return fail(TB_ERR_INVALID_ARG, "radon_den must be nonzero");
  } else {  // section 4.2 constants for d = 3; the workloads' for d = 2
    p.ra = d == 3 ? 3.0 : 2.0;
    p.rb = 1.0;
    p.rden = d == 3 ? 100.0 : 3.0;
  }
  p.store_mask = o.store_mask ? o.store_mask : TB_STORE_C64;
  if (p.store_mask & ~31u) return fail(TB_ERR_INVALID_ARG, "unknown store_mask bits");
  p.max_device_bytes = o.max_device_bytes;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(TB_ERR_HIP, "no HIP device visible");
  }
  if (kind == TB_KERNEL_NUDFT) TB_TRY(set_nudft_points(p, o.nudft_x));
  p.src.resize(p.Lt + 1);
  for (int l = 0; l <= p.Lt; ++l) {
    Level& lv = p.src[l];
    lv.l = l;
    lv.nitems = 1 << (d * (p.Ls + l));
    lv.nb = 1 << (p.Lt - l);
    TB_TRY(run_level(p, lv, l ? &p.src[l - 1] : nullptr, true, stream, o.max_rank));
  }
  p.tgt.resize(p.Ls + 1);
  for (int l = 0; l <= p.Ls; ++l) {
    Level& lv = p.tgt[l];
    lv.l = l;
    lv.nitems = 1 << (d * (p.Lt + l));
    lv.nb = 1 << (p.Ls - l);
    TB_TRY(run_level(p, lv, l ? &p.tgt[l - 1] : nullptr, false, stream, o.max_rank));
  }
  TB_TRY(finalize_plan(p, stream));
  TB_TRY(launch_core_eval(p, stream, nullptr));
  TB_HIP_TRY(hipStreamSynchronize(stream));
  p.construct_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = reinterpret_cast<tb_plan>(plan.release());
  return TB_OK;
}
