// Batched groups: many independent statistics of uneven row counts in one
// persistent launch.
//
// The rows of group g are [row_offsets[g], row_offsets[g+1]).  Each group is
// cut into row tiles of a tuned height; the persistent wide kernel takes
// (row tile, super-tile) items from an atomic queue and writes one block
// record per row tile; a two-stage segmented merge then folds each group's
// records, in tile order, into that group's state (exact 128-bit totals for
// integer columns, Chan co-moments otherwise), so results do not depend on the
// order in which workgroups ran.  The four kernels (queue reset, persistent
// reduction, two merge stages) are captured once in a hipGraph and replayed
// for every call; all call-dependent inputs (plane addresses, tile table,
// tile count) live in device buffers the graph reads, so the graph stays valid
// from one wave of groups to the next.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "runtime.hpp"
#include "wide.hpp"

namespace st {
namespace {

constexpr int kMergeThreads = 256;
constexpr int kMergeBatch = 8;  // records (or partial states) whose loads are in flight together
constexpr int kChunk = 32;      // records per first-stage chunk

struct ChanE {
  double n, mi, mj, m2;
};

__device__ inline void chan_merge(ChanE& a, const ChanE& b) {
  if (b.n == 0.0) return;
  if (a.n == 0.0) {
    a = b;
    return;
  }
  const double n = a.n + b.n;
  const double di = b.mi - a.mi, dj = b.mj - a.mj;
  const double fb = b.n / n;
  const double w = a.n * b.n / n;
  a.m2 = a.m2 + b.m2 + di * dj * w;
  a.mi = a.mi + di * fb;
  a.mj = a.mj + dj * fb;
  a.n = n;
}

// The records of one group are folded in two stages, each in a fixed order:
//  1. k_seg_part: a chunk of at most kChunk consecutive records of one group
//     is folded, in record order, into a partial state (same layout as a
//     group state), so that a large group is spread over many workgroups;
//  2. k_seg_fold: each group's state absorbs its chunks' partial states in
//     chunk order.
// Chunk boundaries depend only on the tile table, so the result does not
// depend on the order in which workgroups ran.
struct SegChunk {
  int64_t k0, k1;  // records [k0, k1), all of one group
};

// Stage 1: grid-stride over the chunks (their count is read from device
// memory, so a captured graph serves every call).
__global__ __launch_bounds__(kMergeThreads) void k_seg_part(const uint64_t* __restrict__ rec,
                                                            const SegChunk* __restrict__ chunks,
                                                            const int64_t* __restrict__ nchunks, int p,
                                                            const uint8_t* __restrict__ intf,
                                                            uint64_t* __restrict__ parts,
                                                            DevStatus* status) {
  const Layout L = Layout::make(p);
  const int64_t W = rec_words(p);
  const int64_t E = p + L.T;
  const int64_t nch = *nchunks;
  uint32_t inexact = 0;
  for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const int64_t k0 = chunks[c].k0, k1 = chunks[c].k1;
    uint64_t* out = parts + c * L.words;
    for (int64_t e = threadIdx.x; e < E; e += kMergeThreads) {
      int i, j;
      const bool is_col = e < p;
      if (is_col) i = j = (int)e;
      else tri_inv(p, e - p, &i, &j);
      const int64_t t = is_col ? tri(p, i, i) : e - p;
      const bool ii = intf[i], ij = intf[j];
      ChanE acc{0.0, 0.0, 0.0, 0.0};
      i128 exact = 0;
      int64_t ntot = 0;
      // every word of a batch is loaded before the first of its merges,
      // which then run in record order
      for (int64_t kb = k0; kb < k1; kb += kMergeBatch) {
        uint64_t nbw[kMergeBatch], Kiw[kMergeBatch], Kjw[kMergeBatch], Siw[kMergeBatch],
            Sjw[kMergeBatch], Qw[kMergeBatch];
#pragma unroll
        for (int u = 0; u < kMergeBatch; ++u) {
          nbw[u] = Kiw[u] = Kjw[u] = Siw[u] = Sjw[u] = Qw[u] = 0;
          if (kb + u < k1) {
            const uint64_t* r = rec + (kb + u) * W;
            nbw[u] = r[0];
            Kiw[u] = r[2 + i];
            Kjw[u] = r[2 + j];
            Siw[u] = r[2 + p + i];
            Sjw[u] = r[2 + p + j];
            Qw[u] = r[2 + 2 * p + t];
          }
        }
#pragma unroll
        for (int u = 0; u < kMergeBatch; ++u) {
          const int64_t nb = (int64_t)nbw[u];
          if (nb == 0) continue;
          const double nbd = (double)nb;
          const double Si = __longlong_as_double((long long)Siw[u]);
          const double Sj = __longlong_as_double((long long)Sjw[u]);
          const double Qij = __longlong_as_double((long long)Qw[u]);
          ChanE b;
          b.n = nbd;
          b.mi = (ii ? (double)(int64_t)Kiw[u] : __longlong_as_double((long long)Kiw[u])) + Si / nbd;
          b.mj = (ij ? (double)(int64_t)Kjw[u] : __longlong_as_double((long long)Kjw[u])) + Sj / nbd;
          b.m2 = is_col ? 0.0 : Qij - Si * (Sj / nbd);
          chan_merge(acc, b);
          ntot += nb;
          if (is_col && ii) {
            const int64_t K = (int64_t)Kiw[u];
            if (!(Qij < kExactQ) || K >= kMaxShift || K <= -kMaxShift) inexact = 1;
            exact += (i128)(int64_t)Si + (i128)nb * (i128)K;
          } else if (!is_col && ii && ij) {
            const i128 Ki = (i128)(int64_t)Kiw[u], Kj = (i128)(int64_t)Kjw[u];
            exact += (i128)(int64_t)Qij + Ki * (i128)(int64_t)Sj + (i128)(int64_t)Si * Kj +
                     (i128)nb * Ki * Kj;
          }
        }
      }
      if (is_col) {
        store_i128(out + L.off_s + 2 * i, exact);
        out[L.off_mu + i] = (uint64_t)__double_as_longlong(acc.mi);
        if (e == 0) {
          out[0] = (uint64_t)ntot;
          out[1] = 0;
        }
      } else {
        store_i128(out + L.off_C + 2 * t, exact);
        out[L.off_M2 + t] = (uint64_t)__double_as_longlong(acc.m2);
      }
    }
  }
  if (inexact) atomicOr(&status->bits, ST_INEXACT);
}

// Stage 2: one workgroup per group; the group's state is updated in place.
// The old count and means are copied to LDS first (pair entries need the old
// means of their columns, which the column entries overwrite).
__global__ __launch_bounds__(kMergeThreads) void k_seg_fold(const uint64_t* __restrict__ parts,
                                                            const int64_t* __restrict__ gc, int p,
                                                            const uint8_t* __restrict__ intf,
                                                            uint64_t* __restrict__ states) {
  extern __shared__ double s_mu[];  // p old means, then old n
  const int g = blockIdx.x;
  const int64_t c0 = gc[g], c1 = gc[g + 1];
  if (c0 == c1) return;
  const Layout L = Layout::make(p);
  uint64_t* st = states + (int64_t)g * L.words;
  for (int i = threadIdx.x; i < p; i += kMergeThreads)
    s_mu[i] = __longlong_as_double((long long)st[L.off_mu + i]);
  if (threadIdx.x == 0) s_mu[p] = (double)(int64_t)st[0];
  __syncthreads();
  const int64_t n_old = (int64_t)s_mu[p];
  const int64_t E = p + L.T;
  for (int64_t e = threadIdx.x; e < E; e += kMergeThreads) {
    int i, j;
    const bool is_col = e < p;
    if (is_col) i = j = (int)e;
    else tri_inv(p, e - p, &i, &j);
    const int64_t t = is_col ? -1 : e - p;
    const bool both = intf[i] && intf[j];
    ChanE acc;
    acc.n = (double)n_old;
    acc.mi = s_mu[i];
    acc.mj = s_mu[j];
    acc.m2 = is_col ? 0.0 : __longlong_as_double((long long)st[L.off_M2 + t]);
    const int64_t xo = is_col ? L.off_s + 2 * i : L.off_C + 2 * t;
    i128 exact = load_i128(st + xo);
    int64_t ntot = n_old;
    for (int64_t cb = c0; cb < c1; cb += kMergeBatch) {
      uint64_t nw[kMergeBatch], mi[kMergeBatch], mj[kMergeBatch], m2[kMergeBatch], xl[kMergeBatch],
          xh[kMergeBatch];
#pragma unroll
      for (int u = 0; u < kMergeBatch; ++u) {
        nw[u] = mi[u] = mj[u] = m2[u] = xl[u] = xh[u] = 0;
        if (cb + u < c1) {
          const uint64_t* s = parts + (cb + u) * L.words;
          nw[u] = s[0];
          mi[u] = s[L.off_mu + i];
          mj[u] = s[L.off_mu + j];
          if (!is_col) m2[u] = s[L.off_M2 + t];
          xl[u] = s[xo];
          xh[u] = s[xo + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < kMergeBatch; ++u) {
        if (nw[u] == 0) continue;
        ChanE b;
        b.n = (double)(int64_t)nw[u];
        b.mi = __longlong_as_double((long long)mi[u]);
        b.mj = __longlong_as_double((long long)mj[u]);
        b.m2 = __longlong_as_double((long long)m2[u]);
        chan_merge(acc, b);
        ntot += (int64_t)nw[u];
        if (is_col || both) {
          const uint64_t w[2] = {xl[u], xh[u]};
          exact += load_i128(w);
        }
      }
    }
    store_i128(st + xo, exact);
    if (is_col) {
      st[L.off_mu + i] = (uint64_t)__double_as_longlong(acc.mi);
      if (e == 0) st[0] = (uint64_t)ntot;
    } else {
      st[L.off_M2 + t] = (uint64_t)__double_as_longlong(acc.m2);
    }
  }
}

// Per-group mean and covariance of the selected columns.
__global__ __launch_bounds__(256) void k_fin_groups(const uint64_t* __restrict__ states, int p,
                                                    const int32_t* __restrict__ sel, int q,
                                                    const uint8_t* __restrict__ intf, int ddof,
                                                    int64_t* n_out, double* mean_out,
                                                    double* cov_out) {
  const int g = blockIdx.x;
  const Layout L = Layout::make(p);
  const uint64_t* st = states + (int64_t)g * L.words;
  const int64_t n = (int64_t)st[0];
  if (threadIdx.x == 0) n_out[g] = n;
  double* mean = mean_out + (int64_t)g * q;
  double* cov = cov_out + (int64_t)g * q * q;
  for (int a = threadIdx.x; a < q; a += blockDim.x) {
    const int i = sel[a];
    mean[a] = n == 0 ? __builtin_nan("")
                     : (intf[i] ? exact_mean(st, L, i, n)
                                : __longlong_as_double((long long)st[L.off_mu + i]));
  }
  const double dn = (double)(n - ddof);
  for (int64_t idx = threadIdx.x; idx < (int64_t)q * q; idx += blockDim.x) {
    const int a = (int)(idx / q), b = (int)(idx % q);
    if (a > b) continue;
    double v;
    if (n <= ddof) {
      v = __builtin_nan("");
    } else {
      const int i = sel[a], j = sel[b];
      if (intf[i] && intf[j]) v = exact_cov(st, L, i, j, n, ddof);
      else v = __longlong_as_double((long long)st[L.off_M2 + tri(p, i, j)]) / dn;
    }
    cov[(int64_t)a * q + b] = v;
    cov[(int64_t)b * q + a] = v;
  }
}

// ---- autotuner ----------------------------------------------------------------

struct Tuned {
  int64_t tile_rows;
  int wg_per_cu;
};

std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tuned;

// What the tuned tile height and occupancy depend on: the device, the
// kernel (the 256-byte record kernel or the general one) and the layout of
// every column (type, plane, byte offset, plane row stride).
std::string tune_key(const stats_ctx* h, const char* arch, bool aos64) {
  std::string k = std::string(arch) + ":p" + std::to_string(h->p) + (aos64 ? ":rec" : ":gen");
  for (const auto& c : h->cols)
    k += ":" + std::to_string(c.dtype) + "." + std::to_string(c.plane) + "." +
         std::to_string(c.byte_offset) + "." + std::to_string(h->row_stride[c.plane]);
  return k;
}

bool tune_cache_lookup(const std::string& key, Tuned* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    *out = it->second;
    return true;
  }
  const char* path = std::getenv("STATS_TUNE_CACHE");
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char kbuf[512];
  long long tr;
  int wg;
  bool found = false;
  while (fscanf(f, "%511s %lld %d", kbuf, &tr, &wg) == 3) {
    if (key == kbuf) {
      out->tile_rows = tr;
      out->wg_per_cu = wg;
      found = true;
    }
  }
  fclose(f);
  if (found) g_tuned[key] = *out;
  return found;
}

void tune_cache_store(const std::string& key, const Tuned& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = t;
  const char* path = std::getenv("STATS_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %lld %d\n", key.c_str(), (long long)t.tile_rows, t.wg_per_cu);
  fclose(f);
}

}  // namespace

// Device buffers of a groups handle (inside aux2): slot table, super-tile
// list, row tiles, per-group tile offsets, tile count, queue head, merge
// chunks, per-group chunk offsets, chunk count.
struct SegBuffers {
  wide::SlotInfo* slots;
  int2* sts;
  wide::SegTile* rowtiles;
  int64_t* gt;
  int64_t* nrt;
  unsigned long long* counter;
  SegChunk* chunks;
  int64_t* gc;
  int64_t* nch;
};

// Upper bound on the merge chunks of cap_rt records in ngroups groups.
static int64_t chunk_cap(int64_t cap_rt, int ngroups) { return cap_rt / kChunk + ngroups; }

static SegBuffers seg_layout(stats_ctx* h, int ntiles_st, int64_t cap_rt, size_t* total) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t off = 0;
  SegBuffers b;
  char* base = (char*)h->aux2_dev;
  b.slots = (wide::SlotInfo*)(base + off);
  off += al(sizeof(wide::SlotInfo) * h->p);
  b.sts = (int2*)(base + off);
  off += al(sizeof(int2) * ntiles_st);
  b.rowtiles = (wide::SegTile*)(base + off);
  off += al(sizeof(wide::SegTile) * cap_rt);
  b.gt = (int64_t*)(base + off);
  off += al(sizeof(int64_t) * (h->ngroups + 1));
  b.nrt = (int64_t*)(base + off);
  off += 256;
  b.counter = (unsigned long long*)(base + off);
  off += 256;
  b.chunks = (SegChunk*)(base + off);
  off += al(sizeof(SegChunk) * chunk_cap(cap_rt, h->ngroups));
  b.gc = (int64_t*)(base + off);
  off += al(sizeof(int64_t) * (h->ngroups + 1));
  b.nch = (int64_t*)(base + off);
  off += 256;
  *total = off;
  return b;
}

static void build_rowtiles(const int64_t* off, int ngroups, int64_t T, int64_t max_rows,
                           std::vector<wide::SegTile>* tiles, std::vector<int64_t>* gt) {
  tiles->clear();
  gt->assign(ngroups + 1, 0);
  int64_t budget = max_rows;
  for (int g = 0; g < ngroups; ++g) {
    (*gt)[g] = (int64_t)tiles->size();
    for (int64_t r = off[g]; r < off[g + 1] && budget > 0; r += T) {
      wide::SegTile t;
      t.r0 = r;
      t.r1 = std::min(r + T, off[g + 1]);
      t.group = g;
      t.pad = 0;
      budget -= t.r1 - t.r0;
      tiles->push_back(t);
    }
  }
  (*gt)[ngroups] = (int64_t)tiles->size();
}

static int seg_prepare(stats_ctx* h, const void* const* planes, int ST, int64_t cap_rt,
                       SegBuffers* B, const std::vector<int2>& sts) {
  size_t need = 0;
  seg_layout(h, (int)sts.size(), cap_rt, &need);
  if (need > h->aux2_cap) {
    // buffers move: the captured graph must be rebuilt
    if (h->graph_exec) {
      (void)hipGraphExecDestroy(h->graph_exec);
      h->graph_exec = nullptr;
    }
    if (h->graph) {
      (void)hipGraphDestroy(h->graph);
      h->graph = nullptr;
    }
    int rc = ensure_dev(h, &h->aux2_dev, &h->aux2_cap, need);
    if (rc) return rc;
  }
  *B = seg_layout(h, (int)sts.size(), cap_rt, &need);
  std::vector<wide::SlotInfo> slots(h->p);
  for (int c = 0; c < h->p; ++c) {
    const stats_column& col = h->cols[c];
    wide::SlotInfo& s = slots[c];
    s.stride = h->row_stride[col.plane];
    s.base = (const char*)planes[col.plane] + col.byte_offset;
    s.kind = col.dtype;
    s.chk = (col.dtype == STATS_F32 || col.dtype == STATS_F64) && (col.flags & STATS_COL_INTEGER);
    s.isint = h->intf[c];
    s.pad[0] = s.pad[1] = 0;
  }
  hipError_t e = hipMemcpyAsync(B->slots, slots.data(), sizeof(wide::SlotInfo) * h->p,
                                hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B->sts, sts.data(), sizeof(int2) * sts.size(), hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "uploading segment tables");
  (void)ST;
  return STATS_OK;
}

// FP64 records of 256 bytes with column c at byte 8c (p <= 32), 16-byte
// aligned: the layout of k_seg_aos64.
static bool seg_aos64_layout(const stats_ctx* h, const void* const* planes) {
  if (h->p > 32) return false;
  const int pl = h->cols[0].plane;
  if (h->row_stride[pl] != 256 || ((uintptr_t)planes[pl] & 15u) != 0) return false;
  for (int c = 0; c < h->p; ++c) {
    const stats_column& col = h->cols[c];
    if (col.plane != pl || col.dtype != STATS_F64 || col.byte_offset != 8 * c) return false;
  }
  return true;
}

static void seg_launch(const stats_ctx* h, bool aos64, const wide::Args& a, const wide::SegArgs& g,
                       int ST, int nwg, hipStream_t s) {
  (void)h;
  if (aos64) launch_seg_aos64(a, g, nwg, s);
  else launch_seg(a, g, ST, nwg, s);
}

static int num_cus(int device) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0)
    n = 256;
  return n;
}

// Times the persistent reduction alone on (a sample of) this call's rows for
// each candidate tile height and occupancy; keeps the fastest per row.
static int autotune(stats_ctx* h, const void* const* planes, const int64_t* off, int ST,
                    const std::vector<int2>& sts, Tuned* best) {
  const bool aos64 = seg_aos64_layout(h, planes);
  const int64_t cands_T[] = {8192, 16384, 32768, 65536, 131072};
  const int cands_W[] = {2, 4, 8};
  const int64_t sample_rows = (int64_t)1 << 26;
  const int ncu = num_cus(h->device);
  double best_rate = -1.0;
  *best = Tuned{32768, 4};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(STATS_E_HIP, "hipEventCreate");
  int rc = STATS_OK;
  for (int64_t T : cands_T) {
    std::vector<wide::SegTile> tiles;
    std::vector<int64_t> gt;
    build_rowtiles(off, h->ngroups, T, sample_rows, &tiles, &gt);
    if (tiles.empty()) break;
    int64_t rows = 0;
    for (const auto& t : tiles) rows += t.r1 - t.r0;
    SegBuffers B;
    rc = seg_prepare(h, planes, ST, (int64_t)tiles.size(), &B, sts);
    if (rc) break;
    const int64_t nt = (int64_t)tiles.size();
    rc = ensure_dev(h, (void**)&h->rec, &h->rec_cap, (size_t)(nt * rec_words(h->p) * 8));
    if (rc) break;
    hipError_t e = hipMemcpyAsync(B.rowtiles, tiles.data(), sizeof(wide::SegTile) * nt,
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B.nrt, &nt, 8, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
      rc = hip_fail(h, e, "autotune upload");
      break;
    }
    wide::Args a;
    a.slots = B.slots;
    a.p = h->p;
    a.tiles = B.sts;
    a.ntiles = (int)sts.size();
    a.nblocks = nt;
    a.nrows = 0;
    a.R = T;
    a.rec = h->rec;
    a.status = h->status_dev;
    wide::SegArgs s{B.rowtiles, B.nrt, B.counter};
    for (int W : cands_W) {
      seg_launch(h, aos64, a, s, ST, ncu * W, h->stream);  // warm
      (void)hipEventRecord(e0, h->stream);
      seg_launch(h, aos64, a, s, ST, ncu * W, h->stream);
      (void)hipEventRecord(e1, h->stream);
      e = hipEventSynchronize(e1);
      if (e != hipSuccess) {
        rc = hip_fail(h, e, "autotune run");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double rate = rows / (ms > 0 ? ms : 1e-3);
      if (rate > best_rate) {
        best_rate = rate;
        *best = Tuned{T, W};
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the timing runs left garbage in the status word only through real
  // exactness violations, which the real run reports as well: clear it
  if (!rc) {
    hipError_t e = clear_status(h);
    if (e != hipSuccess) rc = hip_fail(h, e, "autotune reset");
  }
  return rc;
}

}  // namespace st

using namespace st;

extern "C" int stats_accumulate_segmented(stats_ctx* h, const void* const* planes,
                                          const int64_t* row_offsets, int32_t mem_kind) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups <= 0) return fail(STATS_E_STATE, "not a groups handle (use stats_open_groups)");
  if (!planes || !row_offsets) return fail(STATS_E_ARG, "NULL argument");
  if (mem_kind != STATS_MEM_DEVICE)
    return fail(STATS_E_ARG, "segmented input must be device-resident (STATS_MEM_DEVICE)");
  if (row_offsets[0] < 0) return fail(STATS_E_ARG, "row_offsets[0] < 0");
  for (int g = 0; g < h->ngroups; ++g)
    if (row_offsets[g + 1] < row_offsets[g]) return fail(STATS_E_ARG, "row_offsets must be non-decreasing");
  for (int k = 0; k < h->n_planes; ++k) {
    bool used = false;
    for (const auto& c : h->cols) used |= c.plane == k;
    if (used && !planes[k]) return fail(STATS_E_ARG, "plane " + std::to_string(k) + " is NULL");
  }
  DeviceGuard dg(h->device);
  if (!dg.ok) return fail(STATS_E_HIP, "hipSetDevice failed");
  const int p = h->p;
  const int ST = p <= 32 ? 32 : 64;
  const int ng = (p + ST - 1) / ST;
  std::vector<int2> sts;
  for (int A = 0; A < ng; ++A)
    for (int B = A; B < ng; ++B) sts.push_back(make_int2(A, B));

  // tile height and occupancy: configured, cached, or tuned now
  Tuned tu{h->block_rows, 4};
  if (!h->block_rows) {
    hipDeviceProp_t prop;
    const char* arch = "gfx";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    const std::string key = tune_key(h, arch, seg_aos64_layout(h, planes));
    if (!tune_cache_lookup(key, &tu)) {
      int rc = autotune(h, planes, row_offsets, ST, sts, &tu);
      if (rc) return rc;
      tune_cache_store(key, tu);
    }
  }
  h->seg_tile_rows = tu.tile_rows;
  h->seg_wg_per_cu = tu.wg_per_cu;

  std::vector<wide::SegTile> tiles;
  std::vector<int64_t> gt;
  build_rowtiles(row_offsets, h->ngroups, tu.tile_rows, INT64_MAX, &tiles, &gt);
  const int64_t nt = (int64_t)tiles.size();
  if (nt == 0) return STATS_OK;
  // merge chunks: runs of at most kChunk consecutive records of one group
  std::vector<SegChunk> chunks;
  std::vector<int64_t> gc(h->ngroups + 1, 0);
  for (int g = 0; g < h->ngroups; ++g) {
    gc[g] = (int64_t)chunks.size();
    for (int64_t k = gt[g]; k < gt[g + 1]; k += kChunk) chunks.push_back(SegChunk{k, std::min(k + kChunk, gt[g + 1])});
  }
  gc[h->ngroups] = (int64_t)chunks.size();
  const int64_t nch = (int64_t)chunks.size();
  // capacity grows in steps so that the graph is rarely rebuilt
  int64_t cap_rt = std::max<int64_t>(h->seg_cap_rt, 1024);
  while (cap_rt < nt) cap_rt *= 2;
  const size_t rec_need = (size_t)(cap_rt * rec_words(p) * 8);
  const size_t part_need = (size_t)chunk_cap(cap_rt, h->ngroups) * (size_t)Layout::make(p).words * 8;
  if (cap_rt != h->seg_cap_rt || rec_need > h->rec_cap || part_need > h->seg_part_cap) {
    if (h->graph_exec) {
      (void)hipGraphExecDestroy(h->graph_exec);
      h->graph_exec = nullptr;
    }
    if (h->graph) {
      (void)hipGraphDestroy(h->graph);
      h->graph = nullptr;
    }
  }
  SegBuffers B;
  int rc = seg_prepare(h, planes, ST, cap_rt, &B, sts);
  if (rc) return rc;
  if (rec_need > h->rec_cap) {
    rc = ensure_dev(h, (void**)&h->rec, &h->rec_cap, rec_need);
    if (rc) return rc;
  }
  if (part_need > h->seg_part_cap) {
    rc = ensure_dev(h, (void**)&h->seg_part, &h->seg_part_cap, part_need);
    if (rc) return rc;
  }
  h->seg_cap_rt = cap_rt;
  hipError_t e = hipMemcpyAsync(B.rowtiles, tiles.data(), sizeof(wide::SegTile) * nt,
                                hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B.gt, gt.data(), sizeof(int64_t) * gt.size(), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(B.nrt, &nt, 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B.chunks, chunks.data(), sizeof(SegChunk) * nch, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B.gc, gc.data(), sizeof(int64_t) * gc.size(), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(B.nch, &nch, 8, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // host vectors go out of scope
  if (e != hipSuccess) return hip_fail(h, e, "uploading segment tables");

  wide::Args a;
  a.slots = B.slots;
  a.p = p;
  a.tiles = B.sts;
  a.ntiles = (int)sts.size();
  a.nblocks = nt;
  a.nrows = 0;
  a.R = tu.tile_rows;
  a.rec = h->rec;
  a.status = h->status_dev;
  wide::SegArgs sa{B.rowtiles, B.nrt, B.counter};
  const int nwg = num_cus(h->device) * tu.wg_per_cu;
  const bool aos64 = seg_aos64_layout(h, planes);

  if (!h->graph_exec) {
    // capture on a private stream (the handle's stream may be a legacy default stream)
    if (!h->cap_stream) {
      e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(h, e, "hipStreamCreate(capture)");
    }
    e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamBeginCapture");
    seg_launch(h, aos64, a, sa, ST, nwg, h->cap_stream);
    hipLaunchKernelGGL(k_seg_part, dim3((unsigned)(num_cus(h->device) * 8)), dim3(kMergeThreads), 0,
                       h->cap_stream, h->rec, B.chunks, B.nch, p, h->intf_dev, h->seg_part, h->status_dev);
    const size_t shm = sizeof(double) * (size_t)(p + 1);
    hipLaunchKernelGGL(k_seg_fold, dim3((unsigned)h->ngroups), dim3(kMergeThreads), shm,
                       h->cap_stream, h->seg_part, B.gc, p, h->intf_dev, h->state[0]);
    e = hipStreamEndCapture(h->cap_stream, &h->graph);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
    h->graph_nwg = nwg;
    h->graph_aos64 = (int)aos64;
  }
  if (h->graph_nwg != nwg || h->graph_aos64 != (int)aos64) {
    (void)hipGraphExecDestroy(h->graph_exec);
    (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
    return stats_accumulate_segmented(h, planes, row_offsets, mem_kind);
  }
  Timer t;
  t.begin(h, STATS_K_SEGMENTED);
  e = hipGraphLaunch(h->graph_exec, h->stream);
  t.end();
  if (e != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
  return STATS_OK;
}

extern "C" int stats_finalize_groups(stats_ctx* h, const stats_finalize_opts* opts, int32_t* p_out,
                                     int64_t* n_out, double* mean_out, double* cov_out) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups <= 0) return fail(STATS_E_STATE, "not a groups handle");
  stats_finalize_opts def;
  memset(&def, 0, sizeof def);
  def.ddof = 1;
  const stats_finalize_opts* o = opts ? opts : &def;
  std::vector<int32_t> sel;
  int rc = selection(h, o, &sel);
  if (rc) return rc;
  DeviceGuard dg(h->device);
  rc = sync_handle(h);
  if (rc) return rc;
  const int q = (int)sel.size();
  const int64_t G = h->ngroups;
  const size_t words = (size_t)G * (1 + q + (size_t)q * q);
  rc = ensure_dev(h, (void**)&h->fin_out, &h->fin_out_cap, words * 8);
  if (!rc) rc = ensure_dev(h, (void**)&h->sel_dev, &h->sel_cap, (size_t)q * 4);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(h->sel_dev, sel.data(), (size_t)q * 4, hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "uploading selection");
  int64_t* dn = (int64_t*)h->fin_out;
  double* dmean = h->fin_out + G;
  double* dcov = dmean + G * q;
  {
    Timer t;
    t.begin(h, STATS_K_FINALIZE);
    hipLaunchKernelGGL(k_fin_groups, dim3((unsigned)G), dim3(256), 0, h->stream, h->state[0], h->p,
                       h->sel_dev, q, h->intf_dev, o->ddof, dn, dmean, dcov);
    t.end();
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "group finalize launch");
  std::vector<double> out(words);
  e = hipMemcpyAsync(out.data(), h->fin_out, words * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "group finalize");
  collect_timings(h);
  if (p_out) *p_out = q;
  if (n_out) memcpy(n_out, out.data(), (size_t)G * 8);
  if (mean_out) memcpy(mean_out, out.data() + G, (size_t)G * q * 8);
  if (cov_out) memcpy(cov_out, out.data() + G + G * q, (size_t)G * q * q * 8);
  return STATS_OK;
}

extern "C" int stats_group_raw(stats_ctx* h, int32_t g, int64_t* n, stats_i128* s_int, double* s_f64,
                               stats_i128* C_int, double* C_f64, uint8_t* exact_mask) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups <= 0) return fail(STATS_E_STATE, "not a groups handle");
  if (g < 0 || g >= h->ngroups) return fail(STATS_E_ARG, "group index out of range");
  DeviceGuard dg(h->device);
  int rc = sync_handle(h);
  if (rc) return rc;
  const Layout L = Layout::make(h->p);
  return raw_of_state(h, h->state[0] + (int64_t)g * L.words, n, s_int, s_f64, C_int, C_f64, exact_mask);
}
