// Host side of the tensor butterfly library: errors, plan layout (padding
// and upload of the factors, core tables), plan file I/O and the C entry
// points that do not launch kernels themselves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>

#include "tb_internal.h"

namespace tb {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

tb_status fail(tb_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

Plan::~Plan() {
  // Kernels of this plan may still be in flight on some stream.
  (void)hipDeviceSynchronize();
  drop_graphs_for(this);
  for (void* ptr : allocations) (void)hipFree(ptr);
  if (ws.base) (void)hipFree(ws.base);
  for (StageEvent& e : events) {
    (void)hipEventDestroy(e.start);
    (void)hipEventDestroy(e.stop);
  }
}

tb_status dev_alloc(Plan& p, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 256;
  if (p.max_device_bytes && p.device_bytes + bytes > p.max_device_bytes)
    return fail(TB_ERR_OOM, "plan would need " +
                                std::to_string(p.device_bytes + bytes) +
                                " device bytes, above the cap of " +
                                std::to_string(p.max_device_bytes));
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(e == hipErrorOutOfMemory ? TB_ERR_OOM : TB_ERR_HIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  p.allocations.push_back(*ptr);
  p.device_bytes += bytes;
  return TB_OK;
}

template <class T>
static tb_status upload(Plan& p, T** dst, const std::vector<T>& src) {
  void* ptr = nullptr;
  TB_TRY(dev_alloc(p, &ptr, src.size() * sizeof(T)));
  if (!src.empty())
    TB_HIP_TRY(hipMemcpy(ptr, src.data(), src.size() * sizeof(T),
                         hipMemcpyHostToDevice));
  *dst = static_cast<T*>(ptr);
  return TB_OK;
}

// Parent of a level-l item (same outer multi-set, inner multi-set halved).
static int parent_item(int item, int l, int d) {
  int outer = item >> (d * l);
  int inner = item & ((1 << (d * l)) - 1);
  int pin = 0;
  for (int k = 0; k < d; ++k) {
    int b = (inner >> (l * (d - 1 - k))) & ((1 << l) - 1);
    pin = (pin << (l - 1)) | (b >> 1);
  }
  return (outer << (d * (l - 1))) | pin;
}

static tb_status pad_level(Plan& p, Level& lv, const Level* prev) {
  const int d = p.d;
  for (int k = 0; k < d; ++k) {
    int rmax = 1;
    for (int it = 0; it < lv.nitems; ++it)
      for (int b = 0; b < lv.nb; ++b) rmax = std::max(rmax, lv.id(it, k, b, d).r);
    lv.R[k] = rmax;
    lv.A[k] = prev ? 2 * prev->R[k] : p.leaf;
  }
  long long off = 0;
  for (int k = 0; k < d; ++k) {
    lv.mat_k_off[k] = off;
    off += (long long)lv.nb * lv.R[k] * lv.A[k];
  }
  lv.mat_item_stride = off;
  lv.E = 1;
  for (int k = 0; k < d; ++k) lv.E *= (long long)lv.nb * lv.R[k];

  std::vector<double2> X64((size_t)lv.nitems * lv.mat_item_stride);
  for (auto& z : X64) z = make_double2(0.0, 0.0);
  for (int it = 0; it < lv.nitems; ++it) {
    int par = prev ? parent_item(it, lv.l, d) : -1;
    for (int k = 0; k < d; ++k) {
      for (int b = 0; b < lv.nb; ++b) {
        const IdRec& id = lv.id(it, k, b, d);
        int r1 = 0;
        if (prev) {
          r1 = prev->id(par, k, 2 * b, d).r;
          int r2 = prev->id(par, k, 2 * b + 1, d).r;
          if (id.c != r1 + r2)
            return fail(TB_ERR_IO, "ID column count does not match its children");
        } else if (id.c != p.leaf) {
          return fail(TB_ERR_IO, "leaf ID column count differs from the leaf size");
        }
        double2* M = X64.data() + (size_t)it * lv.mat_item_stride + lv.mat_k_off[k] +
                     (size_t)b * lv.R[k] * lv.A[k];
        for (int i = 0; i < id.r; ++i)
          for (int j = 0; j < id.c; ++j) {
            int pj = prev ? (j < r1 ? j : prev->R[k] + (j - r1)) : j;
            cd v = id.X[(size_t)i * id.c + j];
            M[(size_t)i * lv.A[k] + pj] = make_double2(v.real(), v.imag());
          }
      }
    }
  }
  std::vector<float2> X32(X64.size());
  for (size_t i = 0; i < X64.size(); ++i)
    X32[i] = make_float2((float)X64[i].x, (float)X64[i].y);
  TB_TRY(upload(p, &lv.X64, X64));
  TB_TRY(upload(p, &lv.X32, X32));
  std::vector<int> ranks(lv.ids.size());
  for (size_t i = 0; i < ranks.size(); ++i) ranks[i] = lv.ids[i].r;
  TB_TRY(upload(p, &lv.rank_d, ranks));
  return TB_OK;
}

tb_status set_nudft_points(Plan& p, const double* x) {
  if (!x) return fail(TB_ERR_INVALID_ARG, "the non-uniform DFT needs tb_options.nudft_x");
  const size_t N = (size_t)p.d * (size_t)p.n;
  for (int k = 0; k < p.d; ++k)
    for (long long i = 0; i < p.n; ++i) {
      const double v = x[(size_t)k * p.n + i];
      if (!(v >= 0.0 && v <= (double)(p.n - 1)))
        return fail(TB_ERR_INVALID_ARG, "NUDFT coordinates must lie in [0, n - 1]");
      if (i > 0 && v < x[(size_t)k * p.n + i - 1])
        return fail(TB_ERR_INVALID_ARG, "NUDFT coordinates must be non-decreasing within a mode");
    }
  p.nux.assign(x, x + N);
  TB_TRY(dev_alloc(p, reinterpret_cast<void**>(&p.nux_d), N * sizeof(double)));
  TB_HIP_TRY(hipMemcpy(p.nux_d, p.nux.data(), N * sizeof(double), hipMemcpyHostToDevice));
  return TB_OK;
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  The
// row panels of one pair share the cache lines where its columns meet and the
// pair's slice of F, so all panels of a pair go to one XCD.  Pairs are taken
// in decreasing order of their bytes (longest first) and each is dealt to the
// XCD with the fewest bytes so far; the list is interleaved so that entry u
// runs on XCD u % 8, each XCD's panels in that order.  Shorter queues are
// padded with empty units (pair -1), which the kernels skip.
static std::vector<int2> xcd_grouped(const std::vector<int2>& units, const std::vector<long long>& pair_bytes) {
  constexpr int kX = 8;
  struct Run {
    size_t i, j;
    long long w;
  };
  std::vector<Run> runs;
  size_t i = 0;
  while (i < units.size()) {
    size_t j = i;
    while (j < units.size() && units[j].x == units[i].x) ++j;
    runs.push_back({i, j, pair_bytes[(size_t)units[i].x]});
    i = j;
  }
  std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) { return a.w > b.w; });
  std::vector<std::vector<int2>> q(kX);
  std::vector<long long> load(kX, 0);
  for (const Run& r : runs) {
    int best = 0;
    for (int x = 1; x < kX; ++x)
      if (load[x] < load[best]) best = x;
    q[best].insert(q[best].end(), units.begin() + (long)r.i, units.begin() + (long)r.j);
    load[best] += r.w;
  }
  size_t len = 0;
  for (const auto& v : q) len = std::max(len, v.size());
  std::vector<int2> out(len * kX, make_int2(-1, 0));
  for (int x = 0; x < kX; ++x)
    for (size_t k = 0; k < q[x].size(); ++k) out[k * kX + x] = q[x][k];
  return out;
}

tb_status build_core_tables(Plan& p) {
  const int d = p.d;
  p.nT = 1LL << (d * p.Lt);
  p.nS = 1LL << (d * p.Ls);
  p.npairs = p.nT * p.nS;
  const Level& stop = p.src[p.Lt];
  const Level& ttop = p.tgt[p.Ls];
  p.pair_meta.assign((size_t)p.npairs * kPairMeta, 0);
  p.core_off.assign((size_t)p.npairs, 0);
  p.col_off.assign((size_t)p.npairs, 0);
  long long off = 0, cols = 0;
  for (auto& v : p.fwd_units) v.clear();
  p.mfma_fwd_units.clear();
  p.mfma_adj_units.clear();
  p.adj_units.clear();
  for (long long t = 0; t < p.nT; ++t)
    for (long long s = 0; s < p.nS; ++s) {
      long long pr = t * p.nS + s;
      int* m = &p.pair_meta[(size_t)pr * kPairMeta];
      int RT = 1, RS = 1;
      for (int k = 0; k < d; ++k) {
        int rt = ttop.id((int)(t * p.nS + s), k, 0, d).r;
        int rs = stop.id((int)(s * p.nT + t), k, 0, d).r;
        m[3 + k] = rt;
        m[kMetaRs + k] = rs;
        RT *= rt;
        RS *= rs;
      }
      int RTp = (RT + 3) / 4 * 4;
      m[0] = RT;
      m[1] = RS;
      m[2] = RTp;
      p.core_off[(size_t)pr] = off;
      off += (long long)RTp * RS;
      p.col_off[(size_t)pr] = cols;
      cols += RS;
      for (int lv = 0; lv < 3; ++lv)
        for (int r0 = 0; r0 < RT; r0 += 64 << lv) p.fwd_units[lv].push_back(make_int2((int)pr, r0));
      for (int r0 = 0; r0 < RT; r0 += 256) p.mfma_fwd_units.push_back(make_int2((int)pr, r0));
      for (int c0 = 0; c0 < RS; c0 += 256) p.mfma_adj_units.push_back(make_int2((int)pr, c0));
      for (int c0 = 0; c0 < RS; c0 += 64) p.adj_units.push_back(make_int2((int)pr, c0));
    }
  {
    std::vector<long long> bytes((size_t)p.npairs);
    for (long long pr = 0; pr < p.npairs; ++pr)
      bytes[(size_t)pr] = (long long)p.pair_meta[(size_t)pr * kPairMeta + 2] * p.pair_meta[(size_t)pr * kPairMeta + 1];
    for (auto& v : p.fwd_units) v = xcd_grouped(v, bytes);
  }
  p.core_total = off;
  p.col_total = cols;
  TB_TRY(upload(p, &p.pair_meta_d, p.pair_meta));
  TB_TRY(upload(p, &p.col_off_d, p.col_off));
  TB_TRY(upload(p, &p.core_off_d, p.core_off));
  for (int lv = 0; lv < 3; ++lv) TB_TRY(upload(p, &p.fwd_units_d[lv], p.fwd_units[lv]));
  TB_TRY(upload(p, &p.mfma_fwd_units_d, p.mfma_fwd_units));
  TB_TRY(upload(p, &p.mfma_adj_units_d, p.mfma_adj_units));
  TB_TRY(upload(p, &p.adj_units_d, p.adj_units));
  // skeleton tables of the two top levels, padded with a valid index
  int Rs = 0, Rt = 0;
  for (int k = 0; k < d; ++k) {
    Rs = std::max(Rs, stop.R[k]);
    Rt = std::max(Rt, ttop.R[k]);
  }
  std::vector<int> sk_s((size_t)stop.nitems * d * Rs, 0), sk_t((size_t)ttop.nitems * d * Rt, 0);
  for (int it = 0; it < stop.nitems; ++it)
    for (int k = 0; k < d; ++k) {
      const IdRec& id = stop.id(it, k, 0, d);
      for (int a = 0; a < Rs; ++a)
        sk_s[((size_t)it * d + k) * Rs + a] = id.skel[a < id.r ? a : 0];
    }
  for (int it = 0; it < ttop.nitems; ++it)
    for (int k = 0; k < d; ++k) {
      const IdRec& id = ttop.id(it, k, 0, d);
      for (int a = 0; a < Rt; ++a)
        sk_t[((size_t)it * d + k) * Rt + a] = id.skel[a < id.r ? a : 0];
    }
  TB_TRY(upload(p, &p.top_src_skel_d, sk_s));
  TB_TRY(upload(p, &p.top_tgt_skel_d, sk_t));
  return TB_OK;
}

tb_status finalize_plan(Plan& p, hipStream_t stream) {
  (void)stream;
  for (int l = 0; l <= p.Lt; ++l)
    TB_TRY(pad_level(p, p.src[l], l ? &p.src[l - 1] : nullptr));
  for (int l = 0; l <= p.Ls; ++l)
    TB_TRY(pad_level(p, p.tgt[l], l ? &p.tgt[l - 1] : nullptr));
  TB_TRY(build_core_tables(p));
  return TB_OK;
}

long long apply_cmacs(const Plan& p, long long* per_stage) {
  // exact complex multiply-adds of one apply per RHS, from true ranks and
  // the mode-by-mode order used by the oracle (modes 0..d-1); per_stage
  // (5 entries, nullable) receives the split by forward stage
  const int d = p.d;
  long long total = 0;
  long long split[5] = {0, 0, 0, 0, 0};
  auto side = [&](const std::vector<Level>& lv, bool source) {
    for (size_t l = 0; l < lv.size(); ++l) {
      const Level& L = lv[l];
      const long long before = total;
      for (int it = 0; it < L.nitems; ++it) {
        long long in_len[kMaxD], out_len[kMaxD];
        for (int k = 0; k < d; ++k) {
          in_len[k] = 0;
          out_len[k] = 0;
          for (int b = 0; b < L.nb; ++b) {
            in_len[k] += L.id(it, k, b, d).c;
            out_len[k] += L.id(it, k, b, d).r;
          }
        }
        // source: coarse (in = columns) -> fine (out = rank); target forward
        // maps rank -> columns; the multiply-add count of a block-diagonal
        // mode product is sum_blocks r*c times the other modes' lengths
        long long cur[kMaxD];
        for (int k = 0; k < d; ++k) cur[k] = source ? in_len[k] : out_len[k];
        for (int k = 0; k < d; ++k) {
          long long blocks = 0;
          for (int b = 0; b < L.nb; ++b)
            blocks += (long long)L.id(it, k, b, d).r * L.id(it, k, b, d).c;
          long long rest = 1;
          for (int m = 0; m < d; ++m)
            if (m != k) rest *= cur[m];
          total += blocks * rest;
          cur[k] = source ? out_len[k] : in_len[k];
        }
      }
      const int slot = source ? (l == 0 ? 0 : 1) : (l == 0 ? 4 : 3);
      split[slot] += total - before;
    }
  };
  side(p.src, true);
  side(p.tgt, false);
  const long long before_core = total;
  for (long long pr = 0; pr < p.npairs; ++pr)
    total += (long long)p.pair_meta[(size_t)pr * kPairMeta] *
             p.pair_meta[(size_t)pr * kPairMeta + 1];
  split[2] = total - before_core;
  if (per_stage)
    for (int i = 0; i < 5; ++i) per_stage[i] = split[i];
  return total;
}

// Entries of the tensors each forward stage family reads and writes, per
// right-hand side, at true ranks: an item tensor holds, per mode, the
// concatenated ranks of its blocks, and every tensor counts once (a parent
// read by its 2^d children is one read).  The leaves read or write the
// caller's n^d array; the core family counts F and G, not the cores.
void stage_io_entries(const Plan& p, long long* out5) {
  const int d = p.d;
  auto level_entries = [&](const Level& L) {
    long long e = 0;
    for (int it = 0; it < L.nitems; ++it) {
      long long prod = 1;
      for (int k = 0; k < d; ++k) {
        long long len = 0;
        for (int b = 0; b < L.nb; ++b) len += L.id(it, k, b, d).r;
        prod *= len;
      }
      e += prod;
    }
    return e;
  };
  long long nd = 1;
  for (int k = 0; k < d; ++k) nd *= p.n;
  for (int i = 0; i < 5; ++i) out5[i] = 0;
  if (p.src.empty() || p.tgt.empty()) return;
  out5[0] = nd + level_entries(p.src[0]);
  for (size_t l = 1; l < p.src.size(); ++l) out5[1] += level_entries(p.src[l - 1]) + level_entries(p.src[l]);
  out5[2] = level_entries(p.src.back()) + level_entries(p.tgt.back());
  for (size_t l = 1; l < p.tgt.size(); ++l) out5[3] += level_entries(p.tgt[l]) + level_entries(p.tgt[l - 1]);
  out5[4] = level_entries(p.tgt[0]) + nd;
}

// ------------------------------------------------------------- plan file --
static uint32_t crc32_table[256];
static bool crc32_ready = false;

static uint32_t crc32_update(uint32_t crc, const unsigned char* buf, size_t len) {
  if (!crc32_ready) {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      crc32_table[i] = c;
    }
    crc32_ready = true;
  }
  crc = ~crc;
  for (size_t i = 0; i < len; ++i) crc = crc32_table[(crc ^ buf[i]) & 0xFF] ^ (crc >> 8);
  return ~crc;
}

struct Reader {
  const std::vector<unsigned char>& b;
  size_t pos = 0;
  bool ok = true;
  template <class T>
  T get() {
    T v{};
    if (pos + sizeof(T) > b.size()) {
      ok = false;
      return v;
    }
    std::memcpy(&v, b.data() + pos, sizeof(T));
    pos += sizeof(T);
    return v;
  }
  bool raw(void* dst, size_t n) {
    if (pos + n > b.size()) return ok = false;
    std::memcpy(dst, b.data() + pos, n);
    pos += n;
    return true;
  }
};

static bool read_id(Reader& rd, IdRec& id, long long n) {
  id.r = rd.get<int32_t>();
  id.c = rd.get<int32_t>();
  if (!rd.ok || id.r < 1 || id.c < 1 || id.r > id.c || id.c > 4096) return false;
  id.skel.resize(id.r);
  if (!rd.raw(id.skel.data(), sizeof(int32_t) * id.r)) return false;
  for (int v : id.skel)
    if (v < 0 || v >= n) return false;
  id.X.resize((size_t)id.r * id.c);
  return rd.raw(id.X.data(), sizeof(cd) * id.X.size());
}

static void put_bytes(std::vector<unsigned char>& out, const void* src, size_t n) {
  const unsigned char* s = static_cast<const unsigned char*>(src);
  out.insert(out.end(), s, s + n);
}

}  // namespace tb

using namespace tb;

extern "C" const char* tb_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* tb_status_string(tb_status s) {
  switch (s) {
    case TB_OK: return "TB_OK";
    case TB_ERR_INVALID_ARG: return "TB_ERR_INVALID_ARG";
    case TB_ERR_UNSUPPORTED: return "TB_ERR_UNSUPPORTED";
    case TB_ERR_OOM: return "TB_ERR_OOM";
    case TB_ERR_HIP: return "TB_ERR_HIP";
    case TB_ERR_NUMERIC: return "TB_ERR_NUMERIC";
    case TB_ERR_IO: return "TB_ERR_IO";
  }
  return "unknown tb_status";
}

extern "C" void tb_destroy(tb_plan p) { delete reinterpret_cast<Plan*>(p); }

extern "C" tb_status tb_plan_info(tb_plan ph, tb_plan_info_t* info) {
  if (!ph || !info) return fail(TB_ERR_INVALID_ARG, "tb_plan_info: null argument");
  const Plan& p = *reinterpret_cast<Plan*>(ph);
  std::memset(info, 0, sizeof(*info));
  info->kind = p.kind;
  info->d = p.d;
  info->leaf = p.leaf;
  info->n = p.n;
  info->L = p.L;
  info->Lt = p.Lt;
  info->Ls = p.Ls;
  int rmin = 1 << 30, rmax = 0;
  long long nids = 0, fent = 0;
  for (const auto* side : {&p.src, &p.tgt})
    for (const Level& lv : *side)
      for (const IdRec& id : lv.ids) {
        rmin = std::min(rmin, id.r);
        rmax = std::max(rmax, id.r);
        ++nids;
        fent += (long long)id.r * id.c;
      }
  info->r_min = rmin;
  info->r_max = rmax;
  info->n_ids = nids;
  info->n_pairs = p.npairs;
  info->factor_entries = fent;
  long long ce = 0;
  for (long long pr = 0; pr < p.npairs; ++pr)
    ce += (long long)p.pair_meta[(size_t)pr * kPairMeta] * p.pair_meta[(size_t)pr * kPairMeta + 1];
  info->core_entries = ce;
  for (long long pr = 0; pr < p.npairs; ++pr) {
    info->core_rows += p.pair_meta[(size_t)pr * kPairMeta];
    info->core_cols += p.pair_meta[(size_t)pr * kPairMeta + 1];
  }
  info->apply_cmacs = apply_cmacs(p, info->stage_cmacs);
  stage_io_entries(p, info->stage_io_entries);
  info->omega = p.omega;
  info->tol = p.tol;
  info->eps_id = p.eps_id;
  info->store_mask = p.store_mask;
  info->device_bytes = p.device_bytes;
  info->construct_ms = p.construct_ms;
  return TB_OK;
}

extern "C" tb_status tb_plan_load(const char* path, const tb_options* opt,
                                  int recompute_cores, void* hip_stream, tb_plan* out) {
  if (!path || !out) return fail(TB_ERR_INVALID_ARG, "tb_plan_load: null argument");
  *out = nullptr;
  FILE* fh = std::fopen(path, "rb");
  if (!fh) return fail(TB_ERR_IO, std::string("cannot open plan file ") + path);
  std::vector<unsigned char> buf;
  {
    std::fseek(fh, 0, SEEK_END);
    long sz = std::ftell(fh);
    std::fseek(fh, 0, SEEK_SET);
    if (sz < 88) {
      std::fclose(fh);
      return fail(TB_ERR_IO, "plan file too short");
    }
    buf.resize((size_t)sz);
    size_t got = std::fread(buf.data(), 1, buf.size(), fh);
    std::fclose(fh);
    if (got != buf.size()) return fail(TB_ERR_IO, "short read of plan file");
  }
  uint32_t crc_file, zero;
  std::memcpy(&crc_file, buf.data() + buf.size() - 8, 4);
  std::memcpy(&zero, buf.data() + buf.size() - 4, 4);
  if (zero != 0 || crc32_update(0, buf.data(), buf.size() - 8) != crc_file)
    return fail(TB_ERR_IO, "plan file checksum mismatch");
  if (std::memcmp(buf.data(), "TBPLAN01", 8) != 0) return fail(TB_ERR_IO, "bad plan magic");

  auto plan = std::make_unique<Plan>();
  Plan& p = *plan;
  Reader rd{buf};
  rd.pos = 8;
  int hdr[8];
  for (int& h : hdr) h = rd.get<int32_t>();
  double dh[5];
  for (double& v : dh) v = rd.get<double>();
  p.kind = hdr[0];
  p.d = hdr[1];
  p.n = hdr[2];
  p.leaf = hdr[3];
  p.L = hdr[4];
  p.Lt = hdr[5];
  p.Ls = hdr[6];
  int has_cores = hdr[7];
  p.omega = dh[0];
  p.tol = dh[1];
  p.ra = dh[2];
  p.rb = dh[3];
  p.rden = dh[4];
  if (p.d < 2 || p.d > kMaxD || p.L < 0 || p.L > 12 || p.leaf < 1 || p.Lt < 0 ||
      p.Ls < 0 || p.Lt + p.Ls != p.L || ((long long)p.leaf << p.L) != p.n ||
      p.kind < 0 || p.kind > TB_KERNEL_DFT || (p.kind != TB_KERNEL_DFT && p.d > 3))
    return fail(TB_ERR_IO, "plan header is inconsistent");
  if (p.kind == TB_KERNEL_DFT && (p.n < 2 || (p.n & (p.n - 1)) != 0))
    return fail(TB_ERR_IO, "a uniform DFT plan needs n a power of two");
  if (p.kind == TB_KERNEL_NUDFT) {
    std::vector<double> x((size_t)p.d * p.n);
    for (double& v : x) v = rd.get<double>();
    if (!rd.ok) return fail(TB_ERR_IO, "truncated NUDFT coordinates");
    TB_TRY(set_nudft_points(p, x.data()));
  }
  if (opt) {
    p.store_mask = opt->store_mask ? opt->store_mask : TB_STORE_C64;
    p.max_device_bytes = opt->max_device_bytes;
    if (p.store_mask & ~31u) return fail(TB_ERR_INVALID_ARG, "unknown store_mask bits");
  }
  const int d = p.d;
  p.src.resize(p.Lt + 1);
  for (int l = 0; l <= p.Lt; ++l) {
    Level& lv = p.src[l];
    lv.l = l;
    lv.nitems = 1 << (d * (p.Ls + l));
    lv.nb = 1 << (p.Lt - l);
    lv.ids.resize((size_t)lv.nitems * d * lv.nb);
    for (IdRec& id : lv.ids)
      if (!read_id(rd, id, p.n)) return fail(TB_ERR_IO, "corrupt source ID record");
  }
  p.tgt.resize(p.Ls + 1);
  for (int l = 0; l <= p.Ls; ++l) {
    Level& lv = p.tgt[l];
    lv.l = l;
    lv.nitems = 1 << (d * (p.Lt + l));
    lv.nb = 1 << (p.Ls - l);
    lv.ids.resize((size_t)lv.nitems * d * lv.nb);
    for (IdRec& id : lv.ids)
      if (!read_id(rd, id, p.n)) return fail(TB_ERR_IO, "corrupt target ID record");
  }
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  TB_TRY(finalize_plan(p, stream));
  std::vector<double2> host_cores;
  if (has_cores) {
    host_cores.resize((size_t)p.core_total);
    for (auto& z : host_cores) z = make_double2(0, 0);
    for (long long pr = 0; pr < p.npairs; ++pr) {
      int RT = p.pair_meta[(size_t)pr * kPairMeta], RS = p.pair_meta[(size_t)pr * kPairMeta + 1];
      int RTp = p.pair_meta[(size_t)pr * kPairMeta + 2];
      std::vector<cd> blk((size_t)RT * RS);
      if (!rd.raw(blk.data(), sizeof(cd) * blk.size()))
        return fail(TB_ERR_IO, "plan file truncated in the cores");
      double2* dst = host_cores.data() + p.core_off[(size_t)pr];
      for (int a = 0; a < RT; ++a)
        for (int b = 0; b < RS; ++b) {
          cd v = blk[(size_t)a * RS + b];
          dst[(size_t)b * RTp + a] = make_double2(v.real(), v.imag());
        }
    }
  }
  if (rd.pos != buf.size() - 8) return fail(TB_ERR_IO, "trailing bytes in plan file");
  TB_TRY(launch_core_eval(p, stream, (has_cores && !recompute_cores) ? host_cores.data() : nullptr));
  TB_HIP_TRY(hipStreamSynchronize(stream));
  p.eps_id = 0;
  *out = reinterpret_cast<tb_plan>(plan.release());
  return TB_OK;
}

extern "C" tb_status tb_plan_save(tb_plan ph, const char* path) {
  if (!ph || !path) return fail(TB_ERR_INVALID_ARG, "tb_plan_save: null argument");
  Plan& p = *reinterpret_cast<Plan*>(ph);
  if (!p.cores[TB_C128] && !p.cores[TB_C64])
    return fail(TB_ERR_UNSUPPORTED, "tb_plan_save needs FP64 or FP32 cores in the plan");
  std::vector<unsigned char> out;
  out.reserve(1 << 20);
  put_bytes(out, "TBPLAN01", 8);
  int32_t hdr[8] = {p.kind, p.d, (int32_t)p.n, p.leaf, p.L, p.Lt, p.Ls, 1};
  put_bytes(out, hdr, sizeof(hdr));
  double dh[5] = {p.omega, p.tol, p.ra, p.rb, p.rden};
  put_bytes(out, dh, sizeof(dh));
  if (p.kind == TB_KERNEL_NUDFT) put_bytes(out, p.nux.data(), sizeof(double) * p.nux.size());
  for (const auto* side : {&p.src, &p.tgt})
    for (const Level& lv : *side)
      for (const IdRec& id : lv.ids) {
        int32_t rc[2] = {id.r, id.c};
        put_bytes(out, rc, sizeof(rc));
        put_bytes(out, id.skel.data(), sizeof(int32_t) * id.r);
        put_bytes(out, id.X.data(), sizeof(cd) * id.X.size());
      }
  TB_HIP_TRY(hipDeviceSynchronize());
  bool is64 = p.cores[TB_C128] != nullptr;
  size_t esz = is64 ? sizeof(double2) : sizeof(float2);
  std::vector<unsigned char> raw((size_t)p.core_total * esz);
  TB_HIP_TRY(hipMemcpy(raw.data(), is64 ? p.cores[TB_C128] : p.cores[TB_C64], raw.size(),
                       hipMemcpyDeviceToHost));
  for (long long pr = 0; pr < p.npairs; ++pr) {
    int RT = p.pair_meta[(size_t)pr * kPairMeta], RS = p.pair_meta[(size_t)pr * kPairMeta + 1];
    int RTp = p.pair_meta[(size_t)pr * kPairMeta + 2];
    for (int a = 0; a < RT; ++a)
      for (int b = 0; b < RS; ++b) {
        size_t idx = (size_t)p.core_off[(size_t)pr] + (size_t)b * RTp + a;
        cd v;
        if (is64) {
          double2 z;
          std::memcpy(&z, raw.data() + idx * esz, esz);
          v = cd(z.x, z.y);
        } else {
          float2 z;
          std::memcpy(&z, raw.data() + idx * esz, esz);
          v = cd(z.x, z.y);
        }
        put_bytes(out, &v, sizeof(v));
      }
  }
  uint32_t tail[2] = {crc32_update(0, out.data(), out.size()), 0};
  put_bytes(out, tail, sizeof(tail));
  FILE* fh = std::fopen(path, "wb");
  if (!fh) return fail(TB_ERR_IO, std::string("cannot write ") + path);
  size_t wrote = std::fwrite(out.data(), 1, out.size(), fh);
  std::fclose(fh);
  if (wrote != out.size()) return fail(TB_ERR_IO, "short write of plan file");
  return TB_OK;
}

extern "C" tb_status tb_plan_set_timing(tb_plan ph, int enable) {
  if (!ph) return fail(TB_ERR_INVALID_ARG, "tb_plan_set_timing: null plan");
  reinterpret_cast<Plan*>(ph)->timing = enable != 0;
  return TB_OK;
}

extern "C" tb_status tb_plan_stage_times(tb_plan ph, double* ms, long long* launches) {
  if (!ph) return fail(TB_ERR_INVALID_ARG, "tb_plan_stage_times: null plan");
  Plan& p = *reinterpret_cast<Plan*>(ph);
  if (ms)
    for (int i = 0; i < TB_NSTAGES; ++i) ms[i] = 0.0;
  if (launches)
    for (int i = 0; i < TB_NSTAGES; ++i) launches[i] = 0;
  tb_status st = TB_OK;
  for (StageEvent& e : p.events) {
    float t = 0.f;
    hipError_t err = hipEventSynchronize(e.stop);
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e.start, e.stop);
    if (err != hipSuccess && st == TB_OK)
      st = fail(TB_ERR_HIP, std::string("stage timing: ") + hipGetErrorString(err));
    if (e.stage >= 0 && e.stage < TB_NSTAGES) {
      if (ms) ms[e.stage] += t;
      if (launches) launches[e.stage] += 1;
    }
    (void)hipEventDestroy(e.start);
    (void)hipEventDestroy(e.stop);
  }
  p.events.clear();
  return st;
}
