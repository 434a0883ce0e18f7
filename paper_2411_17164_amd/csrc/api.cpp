// Host side of the xmgn C ABI: argument validation, the halo partitioner,
// batch plans, the activation tape and the forward / backward schedules.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <fstream>
#include <sstream>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <thread>
#include <stdexcept>
#include <vector>

#include "../../include/xmgn.h"
#include "kernels.hpp"

using namespace xmgn;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static xmgn_status fail(xmgn_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) return fail(XMGN_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define GUARD_BEGIN try {
#define GUARD_END                                                   \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    return fail(XMGN_ERR_OOM, "host allocation failed");            \
  }                                                                 \
  catch (const std::exception& ex) {                                \
    return fail(XMGN_ERR_INVALID, ex.what());                       \
  }                                                                 \
  catch (...) {                                                     \
    return fail(XMGN_ERR_INVALID, "unknown error");                 \
  }

extern "C" const char* xmgn_last_error(void) { return g_err.c_str(); }
extern "C" const char* xmgn_version(void) { return "xmgn 0.1 gfx950"; }

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
// Before memory that work already enqueued on `st` may still read is freed
// or rewritten from the host: wait for that work.  Refused while `st` is
// being captured into a graph (the replay would not see the new contents,
// and allocation is not allowed under capture).
static xmgn_status quiesce(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(XMGN_ERR_STATE, "a batch plan, weight plan or buffer would change during stream capture: "
                                "run one uncaptured step of the same batch first");
  HIPCHK(hipStreamSynchronize(st));
  return XMGN_OK;
}

struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // grow-only; contents are not preserved.  Growing waits for the work
  // enqueued on st (which may still read the old buffer) and is refused
  // under capture.
  xmgn_status ensure(size_t need, hipStream_t st) {
    if (need <= bytes && p) return XMGN_OK;
    if (xmgn_status s = quiesce(st)) return s;
    release();
    size_t b = need > 0 ? need : 16;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(XMGN_ERR_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
    }
    bytes = b;
    return XMGN_OK;
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

// Page-locked host memory (the offloaded activation tape): grow-only, contents
// not preserved.
struct HBuf {
  void* p = nullptr;
  size_t bytes = 0;
  HBuf() = default;
  HBuf(const HBuf&) = delete;
  HBuf& operator=(const HBuf&) = delete;
  ~HBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  xmgn_status ensure(size_t need, hipStream_t st) {
    if (need <= bytes && p) return XMGN_OK;
    if (xmgn_status s = quiesce(st)) return s;
    release();
    size_t b = need > 0 ? need : 16;
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(XMGN_ERR_OOM, "hipHostMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
    }
    bytes = b;
    return XMGN_OK;
  }
};

// ---------------------------------------------------------------------------
// model description and parameter layout
// ---------------------------------------------------------------------------
static xmgn_status check_desc(const xmgn_model_desc* d) {
  if (!d) return fail(XMGN_ERR_INVALID, "desc is NULL");
  if (d->hidden != 128 && d->hidden != 256 && d->hidden != 512)
    return fail(XMGN_ERR_UNSUPPORTED, "hidden must be 128, 256 or 512");
  if (d->hidden == 512 && d->precision != 1)
    return fail(XMGN_ERR_UNSUPPORTED, "hidden 512 runs in the BF16 form only (an FP32 edge tile exceeds LDS)");
  if (d->n_layers < 1 || d->n_layers > 64) return fail(XMGN_ERR_INVALID, "n_layers must be in [1, 64]");
  if (d->node_in < 1 || d->node_in > 32 || (d->node_in > 8 && d->node_in % 4 != 0))
    return fail(XMGN_ERR_INVALID, "node_in must be in [1, 8], or a multiple of 4 up to 32");
  if (d->edge_in != 4) return fail(XMGN_ERR_INVALID, "edge_in must be 4");
  if (d->out_dim < 1 || d->out_dim > 16) return fail(XMGN_ERR_INVALID, "out_dim must be in [1, 16]");
  if (d->activation != 0 && d->activation != 1) return fail(XMGN_ERR_INVALID, "activation must be 0 or 1");
  if (d->precision != 0 && d->precision != 1) return fail(XMGN_ERR_INVALID, "precision must be 0 or 1");
  if (d->aggregate != 0 && d->aggregate != 1) return fail(XMGN_ERR_INVALID, "aggregate must be 0 or 1");
  if (!(d->ln_eps > 0.f) || !std::isfinite(d->ln_eps)) return fail(XMGN_ERR_INVALID, "ln_eps must be positive");
  return XMGN_OK;
}

// Sizes of the tensors of each block, in blob order.
static std::vector<int64_t> block_sizes(const xmgn_model_desc* d, int block) {
  const int64_t H = d->hidden;
  switch (block) {
    case 0:
      return {H * d->node_in, H, H * H, H, H * H, H, H, H};
    case 1:
      return {H * d->edge_in, H, H * H, H, H * H, H, H, H};
    case 2:
      return {H * 3 * H, H, H * H, H, H, H};
    case 3:
      return {H * 2 * H, H, H * H, H, H, H};
    case 4:
      return {H * H, H, H * H, H, (int64_t)d->out_dim * H, d->out_dim};
  }
  return {};
}

static int64_t block_total(const xmgn_model_desc* d, int block) {
  auto s = block_sizes(d, block);
  return std::accumulate(s.begin(), s.end(), (int64_t)0);
}

static int64_t block_start(const xmgn_model_desc* d, int block, int layer) {
  const int64_t e0 = block_total(d, 0), e1 = block_total(d, 1);
  const int64_t le = block_total(d, 2), ln = block_total(d, 3);
  switch (block) {
    case 0:
      return 0;
    case 1:
      return e0;
    case 2:
      return e0 + e1 + (int64_t)layer * (le + ln);
    case 3:
      return e0 + e1 + (int64_t)layer * (le + ln) + le;
    case 4:
      return e0 + e1 + (int64_t)d->n_layers * (le + ln);
  }
  return -1;
}

static int64_t poff(const xmgn_model_desc* d, int block, int layer, int tensor) {
  auto s = block_sizes(d, block);
  int64_t o = block_start(d, block, layer);
  for (int i = 0; i < tensor; ++i) o += s[i];
  return o;
}

extern "C" xmgn_status xmgn_param_count(const xmgn_model_desc* desc, int64_t* count) {
  if (xmgn_status s = check_desc(desc)) return s;
  if (!count) return fail(XMGN_ERR_INVALID, "count is NULL");
  *count = block_start(desc, 4, 0) + block_total(desc, 4);
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_param_offset(const xmgn_model_desc* desc, int32_t block, int32_t layer, int32_t tensor,
                                         int64_t* offset) {
  if (xmgn_status s = check_desc(desc)) return s;
  if (!offset) return fail(XMGN_ERR_INVALID, "offset is NULL");
  if (block < 0 || block > 4) return fail(XMGN_ERR_INVALID, "block must be in [0, 4]");
  if ((block == 2 || block == 3) && (layer < 0 || layer >= desc->n_layers))
    return fail(XMGN_ERR_INVALID, "layer out of range");
  if (tensor < 0 || tensor >= (int)block_sizes(desc, block).size()) return fail(XMGN_ERR_INVALID, "tensor out of range");
  *offset = poff(desc, block, layer, tensor);
  return XMGN_OK;
}

// ---------------------------------------------------------------------------
// graphs and partitions (host)
// ---------------------------------------------------------------------------
struct xmgn_graph {
  int32_t n = 0;
  std::vector<int32_t> row_ptr, col;
};

struct PartHost {
  int32_t n_inner = 0;
  std::vector<int32_t> gid, hop, row_ptr, col;
};

// Every partition set gets a serial number of its own: a context caches the
// plan of its last batch by it, so a set freed and another allocated at the
// same address never match.
static uint64_t next_partset_serial() {
  static std::atomic<uint64_t> n{0};
  return ++n;
}

struct xmgn_partset {
  int32_t n_global = 0;
  int32_t halo = 0;
  std::vector<PartHost> parts;
  const uint64_t serial = next_partset_serial();
};

static xmgn_status check_csr(int32_t n, const int32_t* row_ptr, const int32_t* col) {
  if (n < 0) return fail(XMGN_ERR_INVALID, "n must be >= 0");
  if (!row_ptr || (row_ptr[n] > 0 && !col)) return fail(XMGN_ERR_INVALID, "row_ptr / col is NULL");
  if (row_ptr[0] != 0) return fail(XMGN_ERR_INVALID, "row_ptr[0] must be 0");
  for (int32_t r = 0; r < n; ++r) {
    if (row_ptr[r + 1] < row_ptr[r]) return fail(XMGN_ERR_INVALID, "row_ptr must be non-decreasing");
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      if (col[k] < 0 || col[k] >= n) return fail(XMGN_ERR_INVALID, "sender index out of range");
      if (col[k] == r) return fail(XMGN_ERR_INVALID, "self loops are not allowed");
      if (k > row_ptr[r] && col[k] <= col[k - 1]) return fail(XMGN_ERR_INVALID, "segments must be strictly ascending");
    }
  }
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_graph_from_csr(int32_t n, const int32_t* row_ptr, const int32_t* col, xmgn_graph** out) {
  GUARD_BEGIN
  if (!out) return fail(XMGN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (xmgn_status s = check_csr(n, row_ptr, col)) return s;
  auto g = std::make_unique<xmgn_graph>();
  g->n = n;
  g->row_ptr.assign(row_ptr, row_ptr + n + 1);
  g->col.assign(col, col + row_ptr[n]);
  *out = g.release();
  return XMGN_OK;
  GUARD_END
}

extern "C" xmgn_status xmgn_graph_info(const xmgn_graph* g, int32_t* n_nodes, int64_t* n_edges) {
  if (!g) return fail(XMGN_ERR_INVALID, "graph is NULL");
  if (n_nodes) *n_nodes = g->n;
  if (n_edges) *n_edges = (int64_t)g->col.size();
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_graph_export(const xmgn_graph* g, int32_t* row_ptr, int32_t* col) {
  if (!g) return fail(XMGN_ERR_INVALID, "graph is NULL");
  if (row_ptr) std::memcpy(row_ptr, g->row_ptr.data(), g->row_ptr.size() * sizeof(int32_t));
  if (col && !g->col.empty()) std::memcpy(col, g->col.data(), g->col.size() * sizeof(int32_t));
  return XMGN_OK;
}

extern "C" void xmgn_graph_destroy(xmgn_graph* g) { delete g; }

// Recursive coordinate bisection over ids with target sizes sizes[a:b).
static void rcb_split(const float* pos, std::vector<int32_t>& ids, size_t lo, size_t hi, const int32_t* sizes, int a,
                      int b, std::vector<int32_t>& part, int depth) {
  if (b - a == 1) {
    for (size_t i = lo; i < hi; ++i) part[ids[i]] = a;
    return;
  }
  const int m = a + (b - a) / 2;
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (size_t i = lo; i < hi; ++i)
    for (int c = 0; c < 3; ++c) {
      const double v = pos[(size_t)ids[i] * 3 + c];
      mn[c] = std::min(mn[c], v);
      mx[c] = std::max(mx[c], v);
    }
  int axis = 0;
  double best = mx[0] - mn[0];
  for (int c = 1; c < 3; ++c)
    if (mx[c] - mn[c] > best) {
      best = mx[c] - mn[c];
      axis = c;
    }
  std::sort(ids.begin() + lo, ids.begin() + hi, [&](int32_t x, int32_t y) {
    const float px = pos[(size_t)x * 3 + axis], py = pos[(size_t)y * 3 + axis];
    return px < py || (px == py && x < y);
  });
  size_t n_left = 0;
  for (int p = a; p < m; ++p) n_left += sizes[p];
  const size_t mid = lo + n_left;
  if (depth < 3) {
    std::thread t([&] { rcb_split(pos, ids, lo, mid, sizes, a, m, part, depth + 1); });
    rcb_split(pos, ids, mid, hi, sizes, m, b, part, depth + 1);
    t.join();
  } else {
    rcb_split(pos, ids, lo, mid, sizes, a, m, part, depth + 1);
    rcb_split(pos, ids, mid, hi, sizes, m, b, part, depth + 1);
  }
}

// One partition: inner nodes (ascending) plus a depth-hop in-edge halo.
static void build_part(const xmgn_graph* g, const std::vector<int32_t>& inner, int32_t depth, PartHost& P,
                       std::vector<int32_t>& loc) {
  P.n_inner = (int32_t)inner.size();
  P.gid = inner;
  P.hop.assign(inner.size(), 0);
  for (size_t i = 0; i < inner.size(); ++i) loc[inner[i]] = (int32_t)i;
  size_t f0 = 0, f1 = inner.size();
  for (int32_t h = 1; h <= depth && f1 > f0; ++h) {
    std::vector<int32_t> next;
    for (size_t i = f0; i < f1; ++i) {
      const int32_t r = P.gid[i];
      for (int32_t k = g->row_ptr[r]; k < g->row_ptr[r + 1]; ++k) {
        const int32_t s = g->col[k];
        if (loc[s] == -1) {
          loc[s] = -2;  // discovered at this hop
          next.push_back(s);
        }
      }
    }
    std::sort(next.begin(), next.end());
    for (int32_t s : next) {
      loc[s] = (int32_t)P.gid.size();
      P.gid.push_back(s);
      P.hop.push_back(h);
    }
    f0 = f1;
    f1 = P.gid.size();
  }
  const size_t nl = P.gid.size();
  P.row_ptr.assign(nl + 1, 0);
  for (size_t i = 0; i < nl; ++i) {
    const int32_t r = P.gid[i];
    const int32_t d = P.hop[i] < depth ? g->row_ptr[r + 1] - g->row_ptr[r] : 0;
    P.row_ptr[i + 1] = P.row_ptr[i] + d;
  }
  P.col.resize(P.row_ptr[nl]);
  for (size_t i = 0; i < nl; ++i) {
    if (P.hop[i] >= depth) continue;
    const int32_t r = P.gid[i];
    int32_t o = P.row_ptr[i];
    for (int32_t k = g->row_ptr[r]; k < g->row_ptr[r + 1]; ++k) P.col[o++] = loc[g->col[k]];
  }
  for (int32_t s : P.gid) loc[s] = -1;
}

static xmgn_status build_parts(const xmgn_graph* g, const std::vector<std::vector<int32_t>>& inner, int32_t depth,
                               xmgn_partset** out) {
  auto ps = std::make_unique<xmgn_partset>();
  ps->n_global = g->n;
  ps->halo = depth;
  const int np = (int)inner.size();
  ps->parts.resize(np);
  const int nt = std::max(1, std::min<int>(np, (int)std::min(8u, std::max(1u, std::thread::hardware_concurrency()))));
  std::vector<std::thread> pool;
  std::vector<std::string> errs(nt);
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t] {
      try {
        std::vector<int32_t> loc(g->n, -1);
        for (int p = t; p < np; p += nt) build_part(g, inner[p], depth, ps->parts[p], loc);
      } catch (const std::exception& ex) {
        errs[t] = ex.what();
      }
    });
  for (auto& th : pool) th.join();
  for (auto& e : errs)
    if (!e.empty()) return fail(XMGN_ERR_OOM, e);
  *out = ps.release();
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_partition_halo(const xmgn_graph* g, const float* pos, int32_t n_parts,
                                           const int32_t* part_sizes, int32_t halo_hops, xmgn_partset** out) {
  GUARD_BEGIN
  if (!out) return fail(XMGN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!g) return fail(XMGN_ERR_INVALID, "graph is NULL");
  if (!pos && g->n > 0) return fail(XMGN_ERR_INVALID, "pos is NULL");
  if (n_parts < 1) return fail(XMGN_ERR_INVALID, "n_parts must be >= 1");
  if (halo_hops < 1) return fail(XMGN_ERR_INVALID, "halo_hops must be >= 1");
  std::vector<int32_t> sizes(n_parts);
  if (part_sizes) {
    int64_t tot = 0;
    for (int p = 0; p < n_parts; ++p) {
      if (part_sizes[p] <= 0) return fail(XMGN_ERR_INVALID, "part sizes must be positive");
      sizes[p] = part_sizes[p];
      tot += part_sizes[p];
    }
    if (tot != g->n) return fail(XMGN_ERR_INVALID, "part sizes must sum to the node count");
  } else {
    if (n_parts > g->n) return fail(XMGN_ERR_INVALID, "more parts than nodes");
    for (int p = 0; p < n_parts; ++p) sizes[p] = (int32_t)((int64_t)g->n * (p + 1) / n_parts - (int64_t)g->n * p / n_parts);
  }
  for (int64_t i = 0; i < 3 * (int64_t)g->n; ++i)
    if (!std::isfinite(pos[i])) return fail(XMGN_ERR_INVALID, "pos holds NaN or Inf");
  std::vector<int32_t> ids(g->n), part(g->n);
  std::iota(ids.begin(), ids.end(), 0);
  rcb_split(pos, ids, 0, ids.size(), sizes.data(), 0, n_parts, part, 0);
  std::vector<std::vector<int32_t>> inner(n_parts);
  for (int p = 0; p < n_parts; ++p) inner[p].reserve(sizes[p]);
  for (int32_t i = 0; i < g->n; ++i) inner[part[i]].push_back(i);
  return build_parts(g, inner, halo_hops, out);
  GUARD_END
}

extern "C" xmgn_status xmgn_partition_explicit(const xmgn_graph* g, int32_t n_parts, const int32_t* n_inner,
                                               const int32_t* inner, int32_t halo_hops, xmgn_partset** out) {
  GUARD_BEGIN
  if (!out) return fail(XMGN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!g) return fail(XMGN_ERR_INVALID, "graph is NULL");
  if (n_parts < 1 || !n_inner || !inner) return fail(XMGN_ERR_INVALID, "bad part lists");
  if (halo_hops < 1) return fail(XMGN_ERR_INVALID, "halo_hops must be >= 1");
  std::vector<std::vector<int32_t>> lists(n_parts);
  int64_t o = 0;
  for (int p = 0; p < n_parts; ++p) {
    if (n_inner[p] <= 0) return fail(XMGN_ERR_INVALID, "each part needs at least one inner node");
    lists[p].assign(inner + o, inner + o + n_inner[p]);
    o += n_inner[p];
    std::sort(lists[p].begin(), lists[p].end());
    for (size_t i = 0; i < lists[p].size(); ++i) {
      if (lists[p][i] < 0 || lists[p][i] >= g->n) return fail(XMGN_ERR_INVALID, "inner node out of range");
      if (i > 0 && lists[p][i] == lists[p][i - 1]) return fail(XMGN_ERR_INVALID, "repeated inner node");
    }
  }
  return build_parts(g, lists, halo_hops, out);
  GUARD_END
}

extern "C" xmgn_status xmgn_partset_count(const xmgn_partset* ps, int32_t* n_parts, int32_t* n_global) {
  if (!ps) return fail(XMGN_ERR_INVALID, "partset is NULL");
  if (n_parts) *n_parts = (int32_t)ps->parts.size();
  if (n_global) *n_global = ps->n_global;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_partset_info(const xmgn_partset* ps, int32_t part, int32_t* n_inner, int32_t* n_halo,
                                         int64_t* n_edges) {
  if (!ps) return fail(XMGN_ERR_INVALID, "partset is NULL");
  if (part < 0 || part >= (int32_t)ps->parts.size()) return fail(XMGN_ERR_INVALID, "part out of range");
  const PartHost& P = ps->parts[part];
  if (n_inner) *n_inner = P.n_inner;
  if (n_halo) *n_halo = (int32_t)P.gid.size() - P.n_inner;
  if (n_edges) *n_edges = (int64_t)P.col.size();
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_partset_export(const xmgn_partset* ps, int32_t part, int32_t* global_ids, int32_t* hop,
                                           int32_t* row_ptr, int32_t* col) {
  if (!ps) return fail(XMGN_ERR_INVALID, "partset is NULL");
  if (part < 0 || part >= (int32_t)ps->parts.size()) return fail(XMGN_ERR_INVALID, "part out of range");
  const PartHost& P = ps->parts[part];
  if (global_ids) std::memcpy(global_ids, P.gid.data(), P.gid.size() * 4);
  if (hop) std::memcpy(hop, P.hop.data(), P.hop.size() * 4);
  if (row_ptr) std::memcpy(row_ptr, P.row_ptr.data(), P.row_ptr.size() * 4);
  if (col && !P.col.empty()) std::memcpy(col, P.col.data(), P.col.size() * 4);
  return XMGN_OK;
}

extern "C" void xmgn_partset_destroy(xmgn_partset* ps) { delete ps; }

// ---------------------------------------------------------------------------
// context, batch plans, weights, tape
// ---------------------------------------------------------------------------
struct Batch {
  const xmgn_partset* ps = nullptr;
  uint64_t ps_serial = 0;
  uint64_t last_use = 0;  // context clock of the last forward that used the plan
  std::vector<int32_t> part_ids;
  int mt_edge = 0, mt_edge_bwd = 0;
  int n = 0, n_inner = 0;
  int64_t E = 0;
  int n_etiles = 0;
  DBuf ints;  // gid | row_ptr | col | recv | csc_ptr | csc_edge | etiles | inner | etiles of the adjoint
  BatchView view{};
  BatchView view_b{};  // the same batch with the edge adjoint's tiles
};

struct BlockW {
  int64_t W1 = -1, W2 = -1, W3 = -1, W1T = -1, W2T = -1, W3T = -1, Brs = -1;
};

struct xmgn_ctx {
  int device = 0;
  int mt_edge = 0, mt_node = 0, grid = 0, nw_edge = 0;  // 0 = default
  int mt_edge_bwd = 0;                                  // 0 = the forward's edge tile
  int nw_edge_bwd = 0;                                  // 0 = the forward's waves per edge workgroup
  // Batch plans, one per (partition set, part list, edge-tile rows), kept
  // while the context lives (at most kMaxPlans, least recently used evicted),
  // so a step over several batches (waves of partitions) builds each plan
  // once and can then be captured and replayed; `cur` is the plan of the
  // last forward, the one its backward uses.
  static constexpr size_t kMaxPlans = 16;
  std::vector<std::unique_ptr<Batch>> plans;
  Batch* cur = nullptr;
  uint64_t plan_clock = 0;
  // weights
  xmgn_model_desc wdesc{};
  bool have_wplan = false;
  std::vector<PrepJob> jobs;
  int64_t blob_elems = 0;
  std::vector<BlockW> bw;  // per block: 0 enc_node, 1 enc_edge, 2+2l edge, 3+2l node, 2+2L dec
  DBuf jobs_dev, blob;
  // tape: mode 0 = two rolling slots (inference), 1 = every layer on the
  // device, 2 = every layer in page-locked host memory with two device slots
  DBuf h, e, m;
  int tape_mode = 0;
  bool offload = false;  // keep_tape forwards use mode 2
  HBuf ht;               // host tape: h [L+1][n][H] | e [L][E][H] | m [L][n][H] FP32
  hipStream_t cs = nullptr;          // copy stream of the offloaded tape
  std::vector<hipEvent_t> sev;       // ordering events between st and cs
  size_t sev_used = 0;
  // backward workspace
  DBuf dhA, dhMid, dm, Sr, Ss, deA, deB, fa, fb, fc, fd, dy, part, wpart, wfused, redtmp, lossp;
  DBuf part_e, wfused_e;  // the edge adjoint's partials, reduced with the node adjoint's at the end of a layer
  DBuf xe;    // edge features of the forward [E][4]
  DBuf optp;  // optimizer: per-workgroup squared-norm partials (FP64)
  DBuf zt;  // hidden activations of the edge MLPs [L][E][H] (BF16 forms, device-resident tape)
  DBuf at;  // their pre-activations [L][E][H] (BF16 SiLU forms, device-resident tape)
  bool tape_z = false, tape_a = false;
  bool tape_hidden = true;  // tape policy: BF16 forms keep z (and a) of every edge
  bool edge_split = false;  // edge forward form: node projections of W1 (see xmgn_ctx_set_edge_split)
  DBuf proj;                // [2][n][H] FP32 node projections of the current layer
  // per-kernel timing
  bool timing = false;
  std::vector<std::string> tnames;
  std::vector<std::vector<std::pair<hipEvent_t, hipEvent_t>>> tev;
  std::vector<hipEvent_t> tpool;
  size_t tpool_used = 0;
  // state of the last forward
  bool fwd_valid = false;
  bool fwd_tape = false;
  uint64_t fwd_serial = 0;  // counts the forwards that completed their enqueue
  xmgn_model_desc fdesc{};
  const float* f_params = nullptr;
  const float* f_node_in = nullptr;
};

static size_t tsize(const xmgn_model_desc* d) { return d->precision == 1 ? 2 : 4; }

static hipEvent_t pooled_event(xmgn_ctx* c) {
  if (c->tpool_used == c->tpool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->tpool.push_back(e);
  }
  return c->tpool[c->tpool_used++];
}

// Brackets the launches of one kernel class with events when timing is on.
struct KTimer {
  xmgn_ctx* c;
  hipStream_t st;
  int cls = -1;
  hipEvent_t a = nullptr;
  KTimer(xmgn_ctx* ctx, const char* name, hipStream_t s) : c(ctx), st(s) {
    if (!c->timing) return;
    for (size_t i = 0; i < c->tnames.size(); ++i)
      if (c->tnames[i] == name) cls = (int)i;
    if (cls < 0) {
      c->tnames.push_back(name);
      c->tev.emplace_back();
      cls = (int)c->tnames.size() - 1;
    }
    a = pooled_event(c);
    if (a) (void)hipEventRecord(a, st);
  }
  ~KTimer() {
    if (!c->timing || !a) return;
    hipEvent_t b = pooled_event(c);
    if (!b) return;
    (void)hipEventRecord(b, st);
    c->tev[cls].emplace_back(a, b);
  }
};
#define KT(name) KTimer kt_##__LINE__(c, name, st)

static Shape make_shape(const xmgn_ctx* c, const xmgn_model_desc* d) {
  Shape s{};
  s.H = d->hidden;
  s.prec = d->precision;
  s.act = d->activation;
  s.agg = d->aggregate;
  s.eps = d->ln_eps;
  int me = c->mt_edge > 0 ? std::min(c->mt_edge, 64) : 64, mn = c->mt_node > 0 ? c->mt_node : 64;
  // LDS budget: H = 256 runs 32-row node tiles and 32-row edge tiles, or in
  // the BF16 form 64-row edge tiles, or 128-row ones in the wide gathered
  // forward (not in the split form); H = 512 16-row node tiles and 32-row
  // edge tiles (a tile holds whole receiver segments), or 64-row ones in the
  // wide gathered forward.  The edge adjoint stays on 32 or 64 rows.
  const bool wide = d->precision == 1 && !c->edge_split;
  if (d->hidden == 256) {
    me = (d->precision == 1 && c->mt_edge == 64) || (wide && c->mt_edge == 128) ? c->mt_edge : 32;
    mn = 32;
  }
  if (d->hidden == 512) {  // the wide gathered forward by default (1.8x the 32-row kernel on C6)
    me = (wide && (c->mt_edge == 64 || c->mt_edge == 0)) ? 64 : 32;
    mn = 16;
  }
  s.mt_edge = me;
  s.mt_node = mn;
  // the edge adjoint may tile the same edges differently (BF16, H = 128 and
  // 256: 32 or 64 rows, independent of the forward)
  s.mt_edge_bwd = ((d->hidden == 128 || d->hidden == 256) && d->precision == 1 && c->mt_edge_bwd > 0)
                      ? c->mt_edge_bwd
                      : d->hidden == 512 ? 32 : std::min(me, 64);
  s.grid = c->grid > 0 ? c->grid : 1024;
  s.nw_edge = c->nw_edge > 0 ? c->nw_edge : d->hidden == 512 ? 8 : 4;  // H = 512: fewer spills at 8 waves
  s.nw_edge_bwd = c->nw_edge_bwd > 0 ? c->nw_edge_bwd : s.nw_edge;
  return s;
}

extern "C" xmgn_status xmgn_ctx_create(int32_t device, xmgn_ctx** out) {
  GUARD_BEGIN
  if (!out) return fail(XMGN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(XMGN_ERR_INVALID, "device out of range");
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(XMGN_ERR_UNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", not gfx950");
  auto c = std::make_unique<xmgn_ctx>();
  c->device = device;
  *out = c.release();
  return XMGN_OK;
  GUARD_END
}

extern "C" void xmgn_ctx_destroy(xmgn_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : ctx->tpool) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->sev) (void)hipEventDestroy(e);
  if (ctx->cs) (void)hipStreamDestroy(ctx->cs);
  delete ctx;
}

extern "C" xmgn_status xmgn_ctx_set_timing(xmgn_ctx* c, int32_t enable) {
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipDeviceSynchronize());
  c->timing = enable != 0;
  c->tnames.clear();
  c->tev.clear();
  c->tpool_used = 0;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_timing_count(const xmgn_ctx* c, int32_t* n) {
  if (!c || !n) return fail(XMGN_ERR_INVALID, "NULL argument");
  *n = (int32_t)c->tnames.size();
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_timing_read(xmgn_ctx* c, int32_t i, char* name, int32_t name_len, double* total_ms,
                                            int64_t* launches) {
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (i < 0 || i >= (int32_t)c->tnames.size()) return fail(XMGN_ERR_INVALID, "class out of range");
  double t = 0.0;
  for (auto& pr : c->tev[i]) {
    HIPCHK(hipEventSynchronize(pr.second));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
    t += ms;
  }
  if (name && name_len > 0) {
    std::strncpy(name, c->tnames[i].c_str(), (size_t)name_len - 1);
    name[name_len - 1] = 0;
  }
  if (total_ms) *total_ms = t;
  if (launches) *launches = (int64_t)c->tev[i].size();
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_set_tiles(xmgn_ctx* ctx, int32_t edge_rows, int32_t node_rows, int32_t grid,
                                          int32_t edge_waves) {
  if (!ctx) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (edge_waves != 0 && edge_waves != 4 && edge_waves != 8) return fail(XMGN_ERR_INVALID, "edge_waves must be 0, 4 or 8");
  if (edge_rows != 0 && edge_rows != 32 && edge_rows != 64 && edge_rows != 128)
    return fail(XMGN_ERR_INVALID, "edge_rows must be 0, 32, 64 or 128");
  if (node_rows != 0 && node_rows != 32 && node_rows != 64) return fail(XMGN_ERR_INVALID, "node_rows must be 0, 32 or 64");
  if (grid < 0 || (grid > 0 && (grid < 8 || grid % 8 != 0 || grid > 65536)))
    return fail(XMGN_ERR_INVALID, "grid must be 0 or a multiple of 8 in [8, 65536]");
  ctx->mt_edge = edge_rows;
  ctx->mt_node = node_rows;
  ctx->grid = grid;
  ctx->nw_edge = edge_waves;
  ctx->fwd_valid = false;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_set_bwd_tiles(xmgn_ctx* ctx, int32_t edge_rows, int32_t edge_waves) {
  if (!ctx) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (edge_rows != 0 && edge_rows != 32 && edge_rows != 64) return fail(XMGN_ERR_INVALID, "edge_rows must be 0, 32 or 64");
  if (edge_waves != 0 && edge_waves != 4 && edge_waves != 8) return fail(XMGN_ERR_INVALID, "edge_waves must be 0, 4 or 8");
  ctx->mt_edge_bwd = edge_rows;
  ctx->nw_edge_bwd = edge_waves;
  ctx->fwd_valid = false;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_get_bwd_tiles(const xmgn_ctx* ctx, int32_t* edge_rows, int32_t* edge_waves) {
  if (!ctx || !edge_rows || !edge_waves) return fail(XMGN_ERR_INVALID, "NULL argument");
  *edge_rows = ctx->mt_edge_bwd;
  *edge_waves = ctx->nw_edge_bwd;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_tape_serial(const xmgn_ctx* c, int64_t* serial) {
  if (!c || !serial) return fail(XMGN_ERR_INVALID, "NULL argument");
  *serial = c->fwd_valid && c->fwd_tape ? (int64_t)c->fwd_serial : 0;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_memory(const xmgn_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return fail(XMGN_ERR_INVALID, "NULL argument");
  int64_t t = 0;
  for (const auto& P : c->plans) t += (int64_t)P->ints.bytes;
  const DBuf* bufs[] = {&c->jobs_dev, &c->blob, &c->h, &c->e, &c->m, &c->dhA, &c->dhMid,
                        &c->dm, &c->Sr, &c->Ss, &c->deA, &c->deB, &c->fa, &c->fb, &c->fc, &c->fd,
                        &c->dy, &c->part, &c->wpart, &c->wfused, &c->redtmp, &c->lossp, &c->xe, &c->zt,
                        &c->part_e, &c->wfused_e, &c->proj,
                        &c->at, &c->optp};
  for (const DBuf* b : bufs) t += (int64_t)b->bytes;
  *bytes = t;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_host_memory(const xmgn_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return fail(XMGN_ERR_INVALID, "NULL argument");
  *bytes = (int64_t)c->ht.bytes;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_set_offload(xmgn_ctx* c, int32_t enable) {
  GUARD_BEGIN
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipDeviceSynchronize());
  if (enable && !c->cs) HIPCHK(hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking));
  c->offload = enable != 0;
  // the tape is re-allocated at its new size by the next forward
  c->h.release();
  c->e.release();
  c->m.release();
  c->zt.release();
  c->at.release();
  if (!c->offload) c->ht.release();
  c->fwd_valid = false;
  return XMGN_OK;
  GUARD_END
}

extern "C" xmgn_status xmgn_ctx_set_tape(xmgn_ctx* c, int32_t keep_hidden) {
  GUARD_BEGIN
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (keep_hidden != 0 && keep_hidden != 1) return fail(XMGN_ERR_INVALID, "keep_hidden must be 0 or 1");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipDeviceSynchronize());
  c->tape_hidden = keep_hidden != 0;
  c->zt.release();
  c->at.release();
  c->fwd_valid = false;
  return XMGN_OK;
  GUARD_END
}

extern "C" xmgn_status xmgn_ctx_get_tape(const xmgn_ctx* c, int32_t* keep_hidden) {
  if (!c || !keep_hidden) return fail(XMGN_ERR_INVALID, "NULL argument");
  *keep_hidden = c->tape_hidden ? 1 : 0;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_set_edge_split(xmgn_ctx* c, int32_t split) {
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (split != 0 && split != 1) return fail(XMGN_ERR_INVALID, "split must be 0 or 1");
  c->edge_split = split != 0;
  c->fwd_valid = false;
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_ctx_get_edge_split(const xmgn_ctx* c, int32_t* split) {
  if (!c || !split) return fail(XMGN_ERR_INVALID, "NULL argument");
  *split = c->edge_split ? 1 : 0;
  return XMGN_OK;
}

// Records an event (from the context's pool, one entry per use in a call) on
// `st` after the work enqueued on it so far.
static xmgn_status mark(xmgn_ctx* c, hipStream_t st, hipEvent_t* out) {
  if (c->sev_used == c->sev.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->sev.push_back(e);
  }
  *out = c->sev[c->sev_used++];
  HIPCHK(hipEventRecord(*out, st));
  return XMGN_OK;
}

// Orders everything enqueued so far on `from` before what is enqueued next on `to`.
static xmgn_status stream_order(xmgn_ctx* c, hipStream_t from, hipStream_t to) {
  hipEvent_t e;
  if (xmgn_status r = mark(c, from, &e)) return r;
  HIPCHK(hipStreamWaitEvent(to, e, 0));
  return XMGN_OK;
}

// Weight preparation plan: compute-type copies and transposes.
static void add_job(xmgn_ctx* c, int64_t src, int src_ld, int col0, int transpose, int rows, int cols, int64_t& dst,
                    int dst_ld = -1, int dst_col0 = 0, bool alloc = true) {
  PrepJob j{};
  j.src_off = src;
  j.src_ld = src_ld;
  j.src_col0 = col0;
  j.transpose = transpose;
  if (alloc) {
    dst = c->blob_elems;
    c->blob_elems += (int64_t)rows * (dst_ld > 0 ? dst_ld : cols);
    c->blob_elems = (c->blob_elems + 7) / 8 * 8;
  }
  j.dst_off = dst;
  j.dst_ld = dst_ld > 0 ? dst_ld : cols;
  j.dst_col0 = dst_col0;
  j.rows = rows;
  j.cols = cols;
  c->jobs.push_back(j);
}

static xmgn_status ensure_wplan(xmgn_ctx* c, const xmgn_model_desc* d, hipStream_t st) {
  if (c->have_wplan && std::memcmp(&c->wdesc, d, sizeof(*d)) == 0) return XMGN_OK;
  // the job table and the blob may still be read by enqueued kernels
  if (xmgn_status s = quiesce(st)) return s;
  c->have_wplan = false;
  c->jobs.clear();
  c->blob_elems = 0;
  const int H = d->hidden, L = d->n_layers;
  c->bw.assign(3 + 2 * L, BlockW{});
  for (int b = 0; b < 2; ++b) {
    BlockW& w = c->bw[b];
    add_job(c, poff(d, b, 0, 2), H, 0, 0, H, H, w.W2);
    add_job(c, poff(d, b, 0, 4), H, 0, 0, H, H, w.W3);
    add_job(c, poff(d, b, 0, 2), H, 0, 1, H, H, w.W2T);
    add_job(c, poff(d, b, 0, 4), H, 0, 1, H, H, w.W3T);
  }
  for (int l = 0; l < L; ++l) {
    BlockW& we = c->bw[2 + 2 * l];
    const int64_t W1e = poff(d, 2, l, 0), W2e = poff(d, 2, l, 2);
    add_job(c, W1e, 3 * H, 0, 0, H, 3 * H, we.W1);
    add_job(c, W2e, H, 0, 0, H, H, we.W2);
    add_job(c, W2e, H, 0, 1, H, H, we.W2T);
    add_job(c, W1e, 3 * H, 2 * H, 1, H, H, we.W1T);  // [c][j] = W1[j][2H + c]
    add_job(c, W1e, 3 * H, 0, 1, H, H, we.Brs, 2 * H, 0);
    add_job(c, W1e, 3 * H, H, 1, H, H, we.Brs, 2 * H, H, false);
    BlockW& wn = c->bw[3 + 2 * l];
    const int64_t W1n = poff(d, 3, l, 0), W2n = poff(d, 3, l, 2);
    add_job(c, W1n, 2 * H, 0, 0, H, 2 * H, wn.W1);
    add_job(c, W2n, H, 0, 0, H, H, wn.W2);
    add_job(c, W2n, H, 0, 1, H, H, wn.W2T);
    add_job(c, W1n, 2 * H, 0, 1, 2 * H, H, wn.W1T);
  }
  BlockW& wd = c->bw[2 + 2 * L];
  add_job(c, poff(d, 4, 0, 0), H, 0, 0, H, H, wd.W1);
  add_job(c, poff(d, 4, 0, 2), H, 0, 0, H, H, wd.W2);
  add_job(c, poff(d, 4, 0, 0), H, 0, 1, H, H, wd.W1T);
  add_job(c, poff(d, 4, 0, 2), H, 0, 1, H, H, wd.W2T);
  if (xmgn_status s = c->jobs_dev.ensure(c->jobs.size() * sizeof(PrepJob), st)) return s;
  HIPCHK(hipMemcpy(c->jobs_dev.p, c->jobs.data(), c->jobs.size() * sizeof(PrepJob), hipMemcpyHostToDevice));
  if (xmgn_status s = c->blob.ensure((size_t)c->blob_elems * tsize(d), st)) return s;
  c->wdesc = *d;
  c->have_wplan = true;
  return XMGN_OK;
}

static MlpW weights(const xmgn_ctx* c, const xmgn_model_desc* d, const float* params, int bi, int block, int layer) {
  const BlockW& b = c->bw[bi];
  const size_t ts = tsize(d);
  auto ptr = [&](int64_t o) -> const void* { return o < 0 ? nullptr : (const char*)c->blob.p + o * ts; };
  MlpW w{};
  w.W1 = ptr(b.W1);
  w.W2 = ptr(b.W2);
  w.W3 = ptr(b.W3);
  w.W1T = ptr(b.W1T);
  w.W2T = ptr(b.W2T);
  w.W3T = ptr(b.W3T);
  w.Brs = ptr(b.Brs);
  auto P = [&](int t) { return params + poff(d, block, layer, t); };
  if (block == 0 || block == 1) {
    w.W1f = P(0);
    w.b1 = P(1);
    w.b2 = P(3);
    w.b3 = P(5);
    w.gamma = P(6);
    w.beta = P(7);
  } else if (block == 2 || block == 3) {
    w.b1 = P(1);
    w.b2 = P(3);
    w.gamma = P(4);
    w.beta = P(5);
  } else {
    w.b1 = P(1);
    w.b2 = P(3);
    w.W1f = P(4);  // decoder last layer W3 [out][H], FP32
    w.b3 = P(5);
  }
  return w;
}

static xmgn_status ensure_batch(xmgn_ctx* c, const xmgn_partset* ps, const int32_t* part_ids, int32_t n_batch,
                                int mt_edge, int mt_edge_bwd, hipStream_t st) {
  const std::vector<int32_t> ids(part_ids, part_ids + n_batch);
  for (auto& P : c->plans)
    if (P->ps == ps && P->ps_serial == ps->serial && P->mt_edge == mt_edge && P->mt_edge_bwd == mt_edge_bwd &&
        P->part_ids == ids) {
      P->last_use = ++c->plan_clock;
      c->cur = P.get();
      return XMGN_OK;
    }
  c->cur = nullptr;
  if (c->plans.size() >= xmgn_ctx::kMaxPlans) {
    // the evicted plan's device arrays may still be read by enqueued kernels
    if (xmgn_status s = quiesce(st)) return s;
    auto lru = std::min_element(c->plans.begin(), c->plans.end(),
                                [](const auto& a, const auto& b) { return a->last_use < b->last_use; });
    c->plans.erase(lru);
  }
  auto owned = std::make_unique<Batch>();
  Batch& B = *owned;
  B.ps = ps;
  B.ps_serial = ps->serial;
  B.part_ids = ids;
  B.mt_edge = mt_edge;
  B.mt_edge_bwd = mt_edge_bwd;
  int64_t n = 0, E = 0, ni = 0;
  for (int32_t p : B.part_ids) {
    const PartHost& P = ps->parts[p];
    n += (int64_t)P.gid.size();
    E += (int64_t)P.col.size();
    ni += P.n_inner;
  }
  if (n >= (1ll << 31) - 1 || E >= (1ll << 31) - 1) return fail(XMGN_ERR_UNSUPPORTED, "batch exceeds int32 indexing");
  std::vector<int32_t> gid(n), row_ptr(n + 1), col(E), recv(E), csc_ptr(n + 1, 0), csc_edge(E), inner(ni), etiles;
  int64_t no = 0, eo = 0, io = 0;
  int maxdeg = 0;
  for (int32_t p : B.part_ids) {
    const PartHost& P = ps->parts[p];
    const int64_t nl = (int64_t)P.gid.size();
    for (int64_t i = 0; i < nl; ++i) {
      gid[no + i] = P.gid[i];
      row_ptr[no + i] = (int32_t)(eo + P.row_ptr[i]);
      const int d = P.row_ptr[i + 1] - P.row_ptr[i];
      maxdeg = std::max(maxdeg, d);
      for (int32_t k = P.row_ptr[i]; k < P.row_ptr[i + 1]; ++k) {
        col[eo + k] = (int32_t)(no + P.col[k]);
        recv[eo + k] = (int32_t)(no + i);
      }
    }
    for (int32_t i = 0; i < P.n_inner; ++i) inner[io + i] = (int32_t)(no + i);
    no += nl;
    eo += (int64_t)P.col.size();
    io += P.n_inner;
  }
  row_ptr[n] = (int32_t)E;
  if (maxdeg > std::min(mt_edge, mt_edge_bwd))
    return fail(XMGN_ERR_UNSUPPORTED, "in-degree " + std::to_string(maxdeg) + " exceeds the edge tile (" +
                                          std::to_string(std::min(mt_edge, mt_edge_bwd)) + " rows)");
  // sender CSR: stable counting sort by sender (edges already in receiver order)
  for (int64_t k = 0; k < E; ++k) ++csc_ptr[col[k] + 1];
  for (int64_t i = 0; i < n; ++i) csc_ptr[i + 1] += csc_ptr[i];
  {
    std::vector<int32_t> fill(csc_ptr.begin(), csc_ptr.end() - 1);
    for (int64_t k = 0; k < E; ++k) csc_edge[fill[col[k]]++] = (int32_t)k;
  }
  // edge tiles: whole receiver segments, at most mt edges and receivers;
  // each boundary as a (receiver, edge) pair
  auto make_tiles = [&](int mt) {
    std::vector<int32_t> t{0, 0};
    for (int64_t r = 0; r < n;) {
      int64_t cnt = 0, r1 = r;
      while (r1 < n && r1 - r < mt && cnt + (row_ptr[r1 + 1] - row_ptr[r1]) <= mt) {
        cnt += row_ptr[r1 + 1] - row_ptr[r1];
        ++r1;
      }
      t.push_back((int32_t)r1);
      t.push_back(row_ptr[r1]);
      r = r1;
    }
    return t;
  };
  etiles = make_tiles(mt_edge);
  const std::vector<int32_t> etiles_b = mt_edge_bwd == mt_edge ? std::vector<int32_t>{} : make_tiles(mt_edge_bwd);
  const int64_t nt = (int64_t)etiles.size() / 2 - 1;
  const int64_t total = n + (n + 1) + E + E + (n + 1) + E + 2 * (nt + 1) + ni + (int64_t)etiles_b.size() + 2;
  if (xmgn_status s = B.ints.ensure((size_t)total * 4, st)) return s;
  int32_t* d = B.ints.as<int32_t>();
  int64_t o = 0;
  auto up = [&](const std::vector<int32_t>& v) -> const int* {
    const int* ptr = d + o;
    if (!v.empty()) (void)hipMemcpy(d + o, v.data(), v.size() * 4, hipMemcpyHostToDevice);
    o += (int64_t)v.size();
    return ptr;
  };
  BatchView& V = B.view;
  V.n = (int)n;
  V.E = (int)E;
  V.gid = up(gid);
  V.row_ptr = up(row_ptr);
  V.col = up(col);
  V.recv = up(recv);
  V.csc_ptr = up(csc_ptr);
  V.csc_edge = up(csc_edge);
  o += o & 1;  // the (receiver, edge) pairs are read as 8-byte loads
  V.etiles = up(etiles);
  V.n_etiles = (int)nt;
  V.inner = up(inner);
  V.n_inner = (int)ni;
  B.view_b = V;
  if (!etiles_b.empty()) {
    o += o & 1;
    B.view_b.etiles = up(etiles_b);
    B.view_b.n_etiles = (int)etiles_b.size() / 2 - 1;
  }
  HIPCHK(hipGetLastError());
  B.n = (int)n;
  B.E = E;
  B.n_inner = (int)ni;
  B.n_etiles = (int)nt;
  B.last_use = ++c->plan_clock;
  c->plans.push_back(std::move(owned));
  c->cur = c->plans.back().get();
  return XMGN_OK;
}

static xmgn_status ensure_tape(xmgn_ctx* c, const xmgn_model_desc* d, bool full, bool z, bool a, hipStream_t st) {
  const size_t ts = tsize(d), H = d->hidden, L = d->n_layers;
  const size_t n = c->cur->n, E = c->cur->E;
  const int mode = !full ? 0 : c->offload ? 2 : 1;
  const size_t sh = mode == 1 ? L + 1 : 2, se = mode == 1 ? L : std::min<size_t>(L, 2),
               sm = mode == 1 ? L : mode == 2 ? std::min<size_t>(L, 2) : 1;
  if (xmgn_status s = c->h.ensure(sh * n * H * ts, st)) return s;
  if (xmgn_status s = c->e.ensure(se * E * H * ts, st)) return s;
  if (xmgn_status s = c->m.ensure(sm * n * H * 4, st)) return s;
  // the offloaded tape keeps no z: the edge adjoint recomputes it
  c->tape_z = mode == 1 && z;
  c->tape_a = c->tape_z && a;
  if (c->tape_z)
    if (xmgn_status s = c->zt.ensure(L * E * H * ts, st)) return s;
  if (c->tape_a)
    if (xmgn_status s = c->at.ensure(L * E * H * ts, st)) return s;
  if (mode == 2)
    if (xmgn_status s = c->ht.ensure(((L + 1) * n + L * E) * H * ts + L * n * H * 4, st)) return s;
  c->tape_mode = mode;
  return XMGN_OK;
}

// Device slot of layer l's checkpoint.
static void* hslot(xmgn_ctx* c, const xmgn_model_desc* d, int l) {
  const size_t s = c->tape_mode == 1 ? l : l % 2;
  return (char*)c->h.p + s * c->cur->n * d->hidden * tsize(d);
}
static void* eslot(xmgn_ctx* c, const xmgn_model_desc* d, int l) {
  const size_t s = c->tape_mode == 1 ? l : l % 2;
  return (char*)c->e.p + s * c->cur->E * d->hidden * tsize(d);
}
static void* zslot(xmgn_ctx* c, const xmgn_model_desc* d, int l) {
  if (!c->tape_z) return nullptr;
  return (char*)c->zt.p + (size_t)l * c->cur->E * d->hidden * tsize(d);
}
static void* aslot(xmgn_ctx* c, const xmgn_model_desc* d, int l) {
  if (!c->tape_a) return nullptr;
  return (char*)c->at.p + (size_t)l * c->cur->E * d->hidden * tsize(d);
}
static float* mslot(xmgn_ctx* c, const xmgn_model_desc* d, int l) {
  const size_t s = c->tape_mode == 1 ? l : c->tape_mode == 2 ? l % 2 : 0;
  return c->m.as<float>() + s * c->cur->n * d->hidden;
}

// Host copy of layer l's checkpoint in the offloaded tape.
static void* host_h(xmgn_ctx* c, const xmgn_model_desc* d, int l) {
  return (char*)c->ht.p + (size_t)l * c->cur->n * d->hidden * tsize(d);
}
static void* host_e(xmgn_ctx* c, const xmgn_model_desc* d, int l) {
  const size_t H = d->hidden, ts = tsize(d), L = d->n_layers;
  return (char*)c->ht.p + ((L + 1) * c->cur->n + (size_t)l * c->cur->E) * H * ts;
}
static void* host_m(xmgn_ctx* c, const xmgn_model_desc* d, int l) {
  const size_t H = d->hidden, ts = tsize(d), L = d->n_layers;
  return (char*)c->ht.p + ((L + 1) * c->cur->n + L * c->cur->E) * H * ts + (size_t)l * c->cur->n * H * 4;
}

// Offloaded tape, forward: copy, on the copy stream, the checkpoint rows the
// layer just made (h and e of level `lv`, m of level `lv - 1`; any may be
// skipped) once the work enqueued on st so far has finished.
// `done` receives an event that completes with these copies.
static xmgn_status tape_out(xmgn_ctx* c, const xmgn_model_desc* d, hipStream_t st, int lh, int le, int lm,
                            hipEvent_t* done) {
  const size_t H = d->hidden, ts = tsize(d), n = c->cur->n, E = c->cur->E;
  if (xmgn_status r = stream_order(c, st, c->cs)) return r;
  if (lh >= 0) HIPCHK(hipMemcpyAsync(host_h(c, d, lh), hslot(c, d, lh), n * H * ts, hipMemcpyDeviceToHost, c->cs));
  if (le >= 0) HIPCHK(hipMemcpyAsync(host_e(c, d, le), eslot(c, d, le), E * H * ts, hipMemcpyDeviceToHost, c->cs));
  if (lm >= 0) HIPCHK(hipMemcpyAsync(host_m(c, d, lm), mslot(c, d, lm), n * H * 4, hipMemcpyDeviceToHost, c->cs));
  return mark(c, c->cs, done);
}

// Offloaded tape, backward: bring layer l's checkpoint back into its device
// slot on the copy stream, after the work enqueued on st so far (the last
// reader of that slot) has finished.
static xmgn_status tape_in(xmgn_ctx* c, const xmgn_model_desc* d, hipStream_t st, int l, bool h, bool e, bool m,
                           hipEvent_t* done) {
  const size_t H = d->hidden, ts = tsize(d), n = c->cur->n, E = c->cur->E;
  if (xmgn_status r = stream_order(c, st, c->cs)) return r;
  if (h) HIPCHK(hipMemcpyAsync(hslot(c, d, l), host_h(c, d, l), n * H * ts, hipMemcpyHostToDevice, c->cs));
  if (e) HIPCHK(hipMemcpyAsync(eslot(c, d, l), host_e(c, d, l), E * H * ts, hipMemcpyHostToDevice, c->cs));
  if (m) HIPCHK(hipMemcpyAsync(mslot(c, d, l), host_m(c, d, l), n * H * 4, hipMemcpyHostToDevice, c->cs));
  return mark(c, c->cs, done);
}

// The offloaded tape leaves the last layers' checkpoints in their device
// slots, where the backward finds them: all of layer L-1 (slot (L-1) % 2),
// h^L, and e and m of layer L-2 (slot L % 2, whose h the forward overwrote
// with h^L).  Only the rest travels.
static bool tape_h_offloaded(int l, int L) { return l <= L - 2; }
static bool tape_em_offloaded(int l, int L) { return l <= L - 3; }

extern "C" xmgn_status xmgn_forward(xmgn_ctx* c, const xmgn_model_desc* d, const float* params, const xmgn_partset* ps,
                                    const int32_t* part_ids, int32_t n_batch, const float* node_in, const float* pos,
                                    const float* edge_norm, float* out, int32_t keep_tape, xmgn_stream stream) {
  GUARD_BEGIN
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (xmgn_status s = check_desc(d)) return s;
  if (!ps) return fail(XMGN_ERR_INVALID, "partset is NULL");
  if (!params || !node_in || !pos || !edge_norm || !out || !part_ids) return fail(XMGN_ERR_INVALID, "NULL argument");
  if (n_batch < 1 || n_batch > (int32_t)ps->parts.size()) return fail(XMGN_ERR_INVALID, "bad n_batch");
  {
    std::vector<int32_t> ids(part_ids, part_ids + n_batch);
    std::sort(ids.begin(), ids.end());
    for (size_t i = 0; i < ids.size(); ++i) {
      if (ids[i] < 0 || ids[i] >= (int32_t)ps->parts.size()) return fail(XMGN_ERR_INVALID, "part id out of range");
      if (i > 0 && ids[i] == ids[i - 1]) return fail(XMGN_ERR_INVALID, "repeated part id");
    }
  }
  EdgeNorm en{};
  for (int k = 0; k < 4; ++k) {
    en.mu[k] = edge_norm[k];
    en.sd[k] = edge_norm[4 + k];
    if (!std::isfinite(en.mu[k]) || !std::isfinite(en.sd[k]) || en.sd[k] == 0.f)
      return fail(XMGN_ERR_INVALID, "edge_norm must be finite with nonzero std");
  }
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const Shape s = make_shape(c, d);
  // from here on the batch plan and the tape change: a failure leaves no
  // forward for a backward to consume
  c->fwd_valid = false;
  if (xmgn_status r = ensure_batch(c, ps, part_ids, n_batch, s.mt_edge, s.mt_edge_bwd, st)) return r;
  if (xmgn_status r = ensure_wplan(c, d, st)) return r;
  const bool keep_z = c->tape_hidden && edge_z_tape(s);
  if (xmgn_status r = ensure_tape(c, d, keep_tape != 0, keep_z, keep_z && edge_a_tape(s), st)) return r;
  const BatchView& b = c->cur->view;
  const int L = d->n_layers;
  g_config_error = 0;
  { KT("prep"); launch_prep(params, c->blob.p, d->precision, c->jobs_dev.as<PrepJob>(), (int)c->jobs.size(), st); }
  { KT("enc_node_fwd"); launch_enc_node_fwd(s, b, weights(c, d, params, 0, 0, 0), node_in, d->node_in, hslot(c, d, 0), st); }
  if (xmgn_status r = c->xe.ensure((size_t)b.E * 4 * sizeof(float), st)) return r;
  { KT("edge_feat"); launch_edge_feat(b, pos, en, c->xe.as<float>(), st); }
  { KT("enc_edge_fwd"); launch_enc_edge_fwd(s, b, weights(c, d, params, 1, 1, 0), c->xe.as<float>(), eslot(c, d, 0), st); }
  // offloaded tape: copies[j] completes with the copies of the checkpoint rows
  // made before layer j (j = 0: the encoders).  Layer l overwrites the device
  // slot of layer l - 2, so it waits for copies[l - 1].
  const bool off = c->tape_mode == 2;
  c->sev_used = 0;
  std::vector<hipEvent_t> copies(L + 1, nullptr);
  if (off)
    if (xmgn_status r = tape_out(c, d, st, tape_h_offloaded(0, L) ? 0 : -1, tape_em_offloaded(0, L) ? 0 : -1, -1,
                                 &copies[0]))
      return r;
  // the split form (node projections of W1) runs where no adjoint will
  // recompute the first product in the gathered order: forwards without a
  // tape, and forwards whose tape keeps z (and a)
  const bool split = c->edge_split && (keep_tape == 0 || c->tape_z);
  float* pr = nullptr;
  float* pq = nullptr;
  if (split) {
    if (xmgn_status r = c->proj.ensure((size_t)2 * b.n * d->hidden * 4, st)) return r;
    pr = c->proj.as<float>();
    pq = pr + (size_t)b.n * d->hidden;
  }
  for (int l = 0; l < L; ++l) {
    if (off && l >= 1) HIPCHK(hipStreamWaitEvent(st, copies[l - 1], 0));
    const MlpW we = weights(c, d, params, 2 + 2 * l, 2, l);
    if (split) { KT("node_proj"); launch_node_proj(s, b, we, hslot(c, d, l), pr, pq, st); }
    { KT("edge_fwd"); launch_edge_fwd(s, b, we, hslot(c, d, l), eslot(c, d, l),
                    l + 1 < L ? eslot(c, d, l + 1) : nullptr, mslot(c, d, l), zslot(c, d, l), aslot(c, d, l),
                    pr, pq, st); }
    { KT("node_fwd"); launch_node_fwd(s, b, weights(c, d, params, 3 + 2 * l, 3, l), hslot(c, d, l), mslot(c, d, l), hslot(c, d, l + 1),
                    st); }
    if (off)
      if (xmgn_status r = tape_out(c, d, st, tape_h_offloaded(l + 1, L) ? l + 1 : -1,
                                   tape_em_offloaded(l + 1, L) ? l + 1 : -1, tape_em_offloaded(l, L) ? l : -1,
                                   &copies[l + 1]))
        return r;
  }
  { KT("dec_fwd"); launch_dec_fwd(s, b, weights(c, d, params, 2 + 2 * L, 4, 0), hslot(c, d, L), out, d->out_dim, st); }
  if (off) HIPCHK(hipStreamWaitEvent(st, copies[L], 0));  // the host tape is whole when the forward completes
  HIPCHK(hipGetLastError());
  if (g_config_error) return fail(XMGN_ERR_UNSUPPORTED, "tile configuration does not fit this kernel");
  c->fwd_valid = true;
  c->fwd_tape = keep_tape != 0;
  ++c->fwd_serial;
  c->fdesc = *d;
  c->f_params = params;
  c->f_node_in = node_in;
  return XMGN_OK;
  GUARD_END
}

extern "C" xmgn_status xmgn_mse_grad(xmgn_ctx* c, const float* out, const float* target, int64_t n_total, float* d_out,
                                     float* loss, xmgn_stream stream) {
  GUARD_BEGIN
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (!c->fwd_valid) return fail(XMGN_ERR_STATE, "no forward on this context");
  if (!out || !target || !d_out || !loss) return fail(XMGN_ERR_INVALID, "NULL argument");
  if (n_total < 1) return fail(XMGN_ERR_INVALID, "n_total must be >= 1");
  HIPCHK(hipSetDevice(c->device));
  const int G = 256;
  hipStream_t st = (hipStream_t)stream;
  if (xmgn_status s = c->lossp.ensure(G * sizeof(float), st)) return s;
  const double inv = 1.0 / ((double)n_total * c->fdesc.out_dim);
  KT("mse");
  launch_mse(out, target, c->cur->view.gid, c->cur->view.inner, c->cur->n_inner, c->fdesc.out_dim, inv, d_out,
             c->lossp.as<float>(), G, loss, st);
  HIPCHK(hipGetLastError());
  return XMGN_OK;
  GUARD_END
}

static void wgrad_run(xmgn_ctx* c, const Shape& s, WgradOp op, DBuf& wpart, hipStream_t st) {
  KT("wgrad");
  launch_wgrad(s, op, wpart.as<float>(), c->redtmp.as<float>(), st);
}
#define wgrad(s_, op_, wp_, st_) wgrad_run(c, s_, op_, wp_, st_)

static WgradOp wop(const void* A, int a_f32, int lda, int a0, const int* ia, const void* B, int b_f32, int ldb, int b0,
                   const int* ib, int R, int M, int N, float* dst, int ldd, int M_valid = -1) {
  WgradOp o{};
  o.A = A;
  o.a_f32 = a_f32;
  o.lda = lda;
  o.a0 = a0;
  o.ia = ia;
  o.B = B;
  o.b_f32 = b_f32;
  o.ldb = ldb;
  o.b0 = b0;
  o.ib = ib;
  o.R = R;
  o.M = M;
  o.N = N;
  o.M_valid = M_valid < 0 ? M : M_valid;
  o.dst = dst;
  o.ldd = ldd;
  return o;
}

extern "C" xmgn_status xmgn_backward(xmgn_ctx* c, const xmgn_model_desc* d, const float* params, const float* d_out,
                                     float* d_params, xmgn_stream stream) {
  GUARD_BEGIN
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (xmgn_status s = check_desc(d)) return s;
  if (!params || !d_out || !d_params) return fail(XMGN_ERR_INVALID, "NULL argument");
  if (!c->fwd_valid || !c->fwd_tape) return fail(XMGN_ERR_STATE, "backward needs a forward with keep_tape = 1");
  if (std::memcmp(&c->fdesc, d, sizeof(*d)) != 0 || params != c->f_params)
    return fail(XMGN_ERR_STATE, "backward must use the desc and params of the last forward");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const Shape s = make_shape(c, d);
  const BatchView& b = c->cur->view;
  const size_t H = d->hidden, n = c->cur->n, E = c->cur->E, ts = tsize(d);
  const int L = d->n_layers, G = s.grid;
  const size_t rows = std::max(n, E);
  constexpr int kLayerWgrads = 7;
  size_t wpart_stride = 0;
  for (DBuf* p : {&c->dhA, &c->dhMid, &c->dm, &c->Sr, &c->Ss})
    if (xmgn_status r = p->ensure(n * H * 4, st)) return r;
  for (DBuf* p : {&c->deA, &c->deB})
    if (xmgn_status r = p->ensure(E * H * 4, st)) return r;
  for (DBuf* p : {&c->fa, &c->fb, &c->fc, &c->fd})
    if (xmgn_status r = p->ensure(rows * H * ts, st)) return r;
  if (xmgn_status r = c->dy.ensure((size_t)c->cur->n_inner * 16 * 4, st)) return r;
  if (xmgn_status r = c->part.ensure((size_t)G * 13 * H * 4, st)) return r;
  {
    size_t need = 0;
    const int Rs[3] = {(int)n, (int)E, c->cur->n_inner};
    for (int R : Rs)
      need = std::max(need, wgrad_partial_floats(s, wop(nullptr, 0, 0, 0, nullptr, nullptr, 0, 0, 0, nullptr, R,
                                                        (int)H, (int)H, nullptr, 0)));
    // a layer's separate weight-gradient products (at most 3 node-side, 4
    // edge-side) each keep their partials until the layer's reductions run
    wpart_stride = need;
    if (xmgn_status r = c->wpart.ensure(kLayerWgrads * need * 4, st)) return r;
  }
  // the edge adjoint may accumulate its dense weight gradients itself
  // the edge adjoint runs on its own tiling of the batch's edges
  Shape se = s;
  se.mt_edge = s.mt_edge_bwd;
  se.nw_edge = s.nw_edge_bwd;
  const bool fw = edge_bwd_fuses_wgrad(se);
  const bool fw1e = edge_bwd_fuses_dw1e(se, c->tape_z);  // else the e-block of dW1 is a separate product
  if (fw) se.grid = std::min(s.grid, 512);
  const bool fnode = node_bwd_fuses_wgrad(s);
  if (enc_bwd_fuses_wgrad(s) || fnode) {
    // encoders: [<=256][2][H][H]; node adjoint: [<=512][H][H]
    const size_t mats = std::max((size_t)std::min(s.grid, 256) * 2, (size_t)std::min(s.grid, 512));
    if (xmgn_status r = c->wfused.ensure(mats * H * H * 4, st)) return r;
  }
  if (fw)  // edge adjoint: [se.grid][2][H][H]
    if (xmgn_status r = c->wfused_e.ensure((size_t)se.grid * 2 * H * H * 4, st)) return r;
  if (xmgn_status r = c->part_e.ensure((size_t)se.grid * 4 * H * 4, st)) return r;
  // one layer's batch of reductions: at most 9 H x H matrices and 8 H-vectors
  const size_t red_cols = std::max<size_t>(std::max<size_t>(H * H, 16 * H), 9 * H * H + 8 * H);
  if (xmgn_status r = c->redtmp.ensure(reduce_tmp_floats((int)red_cols) * 4, st)) return r;
  float* rt = c->redtmp.as<float>();
  float* part = c->part.as<float>();
  auto P = [&](int block, int layer, int t) { return d_params + poff(d, block, layer, t); };
  auto hl = [&](int l) { return hslot(c, d, l); };

  g_config_error = 0;
  // decoder
  { KT("fill"); launch_fill(c->dhA.as<float>(), n * H, 0.f, st); }
  {
    DecBwdOut o{c->dhA.as<float>(), c->fa.p, c->fb.p, c->fc.p, c->fd.p, c->dy.as<float>(), part};
    { KT("dec_bwd"); launch_dec_bwd(s, b, weights(c, d, params, 2 + 2 * L, 4, 0), hl(L), d_out, d->out_dim, o, st); }
    VecSeg segs[3] = {{0, (int)H, P(4, 0, 1)}, {(int)H, (int)H, P(4, 0, 3)}, {2 * (int)H, d->out_dim, P(4, 0, 5)}};
    launch_vec_reduce(part, G, 2 * (int)H + 16, segs, 3, rt, st);
    const int ni = c->cur->n_inner;
    wgrad(s, wop(c->dy.p, 1, 16, 0, nullptr, c->fb.p, 0, (int)H, 0, nullptr, ni, 16, (int)H, P(4, 0, 4), (int)H,
                 d->out_dim), c->wpart, st);
    wgrad(s, wop(c->fd.p, 0, (int)H, 0, nullptr, c->fa.p, 0, (int)H, 0, nullptr, ni, (int)H, (int)H, P(4, 0, 2), (int)H),
          c->wpart, st);
    wgrad(s, wop(c->fc.p, 0, (int)H, 0, nullptr, hl(L), 0, (int)H, 0, b.inner, ni, (int)H, (int)H, P(4, 0, 0), (int)H),
          c->wpart, st);
  }
  // processor layers, last to first
  Shape snode = s;  // node adjoint with W2 resident in LDS: two workgroups per CU
  if (fnode) snode.grid = std::min(s.grid, 512);
  const float* de_in = nullptr;
  DBuf* de_out = &c->deA;
  DBuf* de_other = &c->deB;
  // offloaded tape: layer l - 1's checkpoint comes back into its device slot
  // (last read by layer l + 1, or by the decoder) while layer l runs.
  const bool off = c->tape_mode == 2;
  c->sev_used = 0;
  std::vector<hipEvent_t> back(L, nullptr);
  for (int l = L - 1; l >= 0; --l) {
    if (off && back[l]) HIPCHK(hipStreamWaitEvent(st, back[l], 0));
    if (off && l >= 1 && tape_h_offloaded(l - 1, L)) {
      const bool em = tape_em_offloaded(l - 1, L);
      if (xmgn_status r = tape_in(c, d, st, l - 1, true, em, em, &back[l - 1])) return r;
    }
    const MlpW wn = weights(c, d, params, 3 + 2 * l, 3, l);
    NodeBwdOut no{c->dhMid.as<float>(), c->dm.as<float>(), c->fa.p, c->fb.p, c->fc.p, part,
                  fnode ? c->wfused.as<float>() : nullptr};
    { KT("node_bwd"); launch_node_bwd(snode, b, wn, hl(l), mslot(c, d, l), c->dhA.as<float>(), no, st); }
    // the layer's reductions of partial sums run as one batch at its end
    RedBatch rb;
    int n_wg = 0;
    auto wg = [&](const WgradOp& op) {
      if (n_wg >= kLayerWgrads) throw std::logic_error("more weight-gradient products in a layer than partials");
      KT("wgrad");
      launch_wgrad_partials(s, op, c->wpart.as<float>() + (size_t)(n_wg++) * wpart_stride, rb, st);
    };
    VecSeg ns[4] = {{0, (int)H, P(3, l, 1)}, {(int)H, (int)H, P(3, l, 3)}, {2 * (int)H, (int)H, P(3, l, 4)},
                    {3 * (int)H, (int)H, P(3, l, 5)}};
    rb.add_vec(part, snode.grid, 4 * (int)H, ns, 4);
    // dW1 = sum da [h ; m]^T (two products); dW2 = sum du z^T, fused or a product
    wg(wop(c->fa.p, 0, (int)H, 0, nullptr, hl(l), 0, (int)H, 0, nullptr, (int)n, (int)H, (int)H, P(3, l, 0),
           2 * (int)H));
    wg(wop(c->fa.p, 0, (int)H, 0, nullptr, mslot(c, d, l), 1, (int)H, 0, nullptr, (int)n, (int)H, (int)H,
           P(3, l, 0) + H, 2 * (int)H));
    if (fnode)
      rb.add(c->wfused.as<float>(), snode.grid, (int)(H * H), (int)H, (int)H, P(3, l, 2), (int)H);
    else
      wg(wop(c->fb.p, 0, (int)H, 0, nullptr, c->fc.p, 0, (int)H, 0, nullptr, (int)n, (int)H, (int)H, P(3, l, 2),
             (int)H));

    const MlpW we = weights(c, d, params, 2 + 2 * l, 2, l);
    EdgeBwdOut eo{de_out->as<float>(), c->Sr.as<float>(), c->fa.p, c->fb.p, c->fc.p, c->part_e.as<float>(),
                  fw ? c->wfused_e.as<float>() : nullptr};
    const void* zt = edge_z_tape(se) ? zslot(c, d, l) : nullptr;  // the forward's z, when it kept it
    const void* at = edge_a_tape(se) ? aslot(c, d, l) : nullptr;  // ... and a (SiLU)
    { KT("edge_bwd"); launch_edge_bwd(se, c->cur->view_b, we, hl(l), eslot(c, d, l), zt, at, de_in, c->dm.as<float>(), eo, st); }
    VecSeg es[4] = {{0, (int)H, P(2, l, 1)}, {(int)H, (int)H, P(2, l, 3)}, {2 * (int)H, (int)H, P(2, l, 4)},
                    {3 * (int)H, (int)H, P(2, l, 5)}};
    rb.add_vec(c->part_e.as<float>(), se.grid, 4 * (int)H, es, 4);
    if (fw) {
      rb.add(c->wfused_e.as<float>(), se.grid, 2 * (int)(H * H), (int)H, (int)H, P(2, l, 2), (int)H);
      if (fw1e)
        rb.add(c->wfused_e.as<float>() + H * H, se.grid, 2 * (int)(H * H), (int)H, (int)H, P(2, l, 0) + 2 * H,
               3 * (int)H);
    }
    { KT("sender_sum"); launch_sender_sum(s, b, c->fa.p, c->Ss.as<float>(), st); }
    { KT("node_dh"); launch_node_dh(s, b, we, c->dhMid.as<float>(), c->Sr.as<float>(), c->Ss.as<float>(), c->dhA.as<float>(), st); }
    wg(wop(c->Sr.p, 1, (int)H, 0, nullptr, hl(l), 0, (int)H, 0, nullptr, (int)n, (int)H, (int)H, P(2, l, 0),
           3 * (int)H));
    wg(wop(c->Ss.p, 1, (int)H, 0, nullptr, hl(l), 0, (int)H, 0, nullptr, (int)n, (int)H, (int)H, P(2, l, 0) + H,
           3 * (int)H));
    if (!fw1e)
      wg(wop(c->fa.p, 0, (int)H, 0, nullptr, eslot(c, d, l), 0, (int)H, 0, nullptr, (int)E, (int)H, (int)H,
             P(2, l, 0) + 2 * H, 3 * (int)H));
    if (!fw)
      wg(wop(c->fb.p, 0, (int)H, 0, nullptr, zt ? zt : c->fc.p, 0, (int)H, 0, nullptr, (int)E, (int)H, (int)H,
             P(2, l, 2), (int)H));
    if ((size_t)rb.tmp_floats > reduce_tmp_floats((int)red_cols))
      throw std::logic_error("a layer's reduction batch exceeds its scratch");
    { KT("wgrad"); launch_reduce_batch(rb, rt, st); }
    de_in = de_out->as<float>();
    std::swap(de_out, de_other);
  }
  // encoders
  const bool fe = enc_bwd_fuses_wgrad(s);
  Shape sn = s;  // encoders: with fused weight gradients, at most one workgroup per CU in flight
  if (fe) sn.grid = std::min(s.grid, 256);
  for (int blk = 1; blk >= 0; --blk) {
    const MlpW w = weights(c, d, params, blk, blk, 0);
    // more than 8 node inputs: the input layer's dW1 is a separate product
    // over its FP32 adjoint (S_r is free once the layers are done)
    const bool wide = blk == 0 && d->node_in > 8;
    EncBwdOut o{c->fa.p, c->fb.p, c->fc.p, c->fd.p, part, fe ? c->wfused.as<float>() : nullptr,
                wide ? c->Sr.as<float>() : nullptr};
    int R;
    int in_dim;
    if (blk == 1) {
      { KT("enc_edge_bwd"); launch_enc_edge_bwd(sn, b, w, c->xe.as<float>(), de_in, o, st); }
      R = (int)E;
      in_dim = 4;
    } else {
      { KT("enc_node_bwd"); launch_enc_node_bwd(sn, b, w, c->f_node_in, d->node_in, c->dhA.as<float>(), o, st); }
      R = (int)n;
      in_dim = d->node_in;
    }
    VecSeg vs[5] = {{0, (int)H, P(blk, 0, 1)}, {(int)H, (int)H, P(blk, 0, 3)}, {2 * (int)H, (int)H, P(blk, 0, 5)},
                    {3 * (int)H, (int)H, P(blk, 0, 6)}, {4 * (int)H, (int)H, P(blk, 0, 7)}};
    launch_vec_reduce(part, sn.grid, 13 * (int)H, vs, 5, rt, st);
    if (wide)
      wgrad(s, wop(c->Sr.p, 1, (int)H, 0, nullptr, c->f_node_in, 1, in_dim, 0, b.gid, (int)n, (int)H, in_dim,
                   P(blk, 0, 0), in_dim), c->wpart, st);
    else
      launch_vec_reduce_strided(part, sn.grid, 13 * (int)H, 5 * (int)H, (int)H, in_dim, 8, P(blk, 0, 0), in_dim, rt, st);
    if (fe) {
      KT("wgrad");
      launch_wgrad_reduce(c->wfused.as<float>(), sn.grid, (int)H, (int)H, P(blk, 0, 2), (int)H, 2 * (int)(H * H), rt, st);
      launch_wgrad_reduce(c->wfused.as<float>() + H * H, sn.grid, (int)H, (int)H, P(blk, 0, 4), (int)H,
                          2 * (int)(H * H), rt, st);
    } else {
      wgrad(s, wop(c->fd.p, 0, (int)H, 0, nullptr, c->fb.p, 0, (int)H, 0, nullptr, R, (int)H, (int)H, P(blk, 0, 4),
                   (int)H), c->wpart, st);
      wgrad(s, wop(c->fc.p, 0, (int)H, 0, nullptr, c->fa.p, 0, (int)H, 0, nullptr, R, (int)H, (int)H, P(blk, 0, 2),
                   (int)H), c->wpart, st);
    }
  }
  HIPCHK(hipGetLastError());
  if (g_config_error) return fail(XMGN_ERR_UNSUPPORTED, "tile configuration does not fit this kernel");
  return XMGN_OK;
  GUARD_END
}

extern "C" xmgn_status xmgn_grad_accumulate(float* acc, const float* g, int64_t n, xmgn_stream stream) {
  if (n < 0) return fail(XMGN_ERR_INVALID, "n must be >= 0");
  if (n > 0 && (!acc || !g)) return fail(XMGN_ERR_INVALID, "NULL argument");
  launch_accumulate(acc, g, n, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return XMGN_OK;
}

// Arguments of an optimizer step, checked on the host; the FP32 constants
// of the update, each rounded once from its FP64 value.
static xmgn_status adam_args(float* params, const float* grad, float* m, float* v, int64_t n, int64_t step,
                             double lr, double beta1, double beta2, double eps, double clip_norm, AdamArgs* a) {
  if (n < 0) return fail(XMGN_ERR_INVALID, "n must be >= 0");
  if (n > 0 && (!params || !grad || !m || !v)) return fail(XMGN_ERR_INVALID, "NULL argument");
  if (step < 1) return fail(XMGN_ERR_INVALID, "step is 1-based");
  if (!(std::isfinite(lr) && lr >= 0.0 && std::isfinite(eps) && eps > 0.0 && std::isfinite(clip_norm)))
    return fail(XMGN_ERR_INVALID, "lr must be finite and >= 0, eps finite and > 0, clip_norm finite");
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0))
    return fail(XMGN_ERR_INVALID, "betas must be in [0, 1)");
  *a = AdamArgs{(float)lr, (float)beta1, (float)beta2, (float)(1.0 - beta1), (float)(1.0 - beta2), (float)eps,
                (float)(1.0 - std::pow(beta1, (double)step)), (float)(1.0 - std::pow(beta2, (double)step)), clip_norm};
  return XMGN_OK;
}

extern "C" xmgn_status xmgn_adam_step(xmgn_ctx* c, float* params, const float* grad, float* m, float* v, int64_t n,
                                      int64_t step, double lr, double beta1, double beta2, double eps,
                                      double clip_norm, float* grad_norm, xmgn_stream stream) {
  GUARD_BEGIN
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  AdamArgs a{};
  if (xmgn_status r = adam_args(params, grad, m, v, n, step, lr, beta1, beta2, eps, clip_norm, &a)) return r;
  HIPCHK(hipSetDevice(c->device));
  const int G = kAdamScratchPartials;
  if (xmgn_status r = c->optp.ensure(G * sizeof(double), (hipStream_t)stream)) return r;
  launch_adam(params, grad, m, v, n, c->optp.as<double>(), G, a, grad_norm, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return XMGN_OK;
  GUARD_END
}

extern "C" xmgn_status xmgn_adam_step_noalloc(int32_t device, float* params, const float* grad, float* m, float* v,
                                              int64_t n, int64_t step, double lr, double beta1, double beta2,
                                              double eps, double clip_norm, float* grad_norm, xmgn_stream stream) {
  GUARD_BEGIN
  AdamArgs a{};
  if (xmgn_status r = adam_args(params, grad, m, v, n, step, lr, beta1, beta2, eps, clip_norm, &a)) return r;
  int n_dev = 0;
  HIPCHK(hipGetDeviceCount(&n_dev));
  if (device < 0 || device >= n_dev || device >= kMaxDevices) return fail(XMGN_ERR_INVALID, "device out of range");
  // the partial count is fixed (the array's size), so no n needs more
  const int G = kAdamScratchPartials;
  HIPCHK(hipSetDevice(device));
  double* partial = nullptr;
  const char* err = "";
  if (const int rc = adam_noalloc_scratch(device, &partial, &err))
    return fail(rc == -1 ? XMGN_ERR_INVALID : XMGN_ERR_HIP, std::string("optimizer scratch: ") + err);
  // k_sumsq writes all G partials before k_adam reads them (stream order),
  // so nothing of a previous call needs clearing
  launch_adam(params, grad, m, v, n, partial, G, a, grad_norm, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return XMGN_OK;
  GUARD_END
}

extern "C" double xmgn_cosine_lr(int64_t t, int64_t T, double lr_max, double lr_min) {
  if (T <= 0) return lr_min;
  const double x = (double)std::min<int64_t>(std::max<int64_t>(t, 0), T) / (double)T;
  return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + std::cos(M_PI * x));
}

extern "C" xmgn_status xmgn_build_knn(xmgn_ctx* c, const float* pos, int32_t n, const int32_t* level_end,
                                      int32_t n_levels, int32_t k_intra, int32_t k_cross, xmgn_graph** out,
                                      xmgn_stream stream) {
  GUARD_BEGIN
  if (!out) return fail(XMGN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (!pos || !level_end) return fail(XMGN_ERR_INVALID, "NULL argument");
  if (n < 2) return fail(XMGN_ERR_INVALID, "need at least 2 points");
  if (n_levels < 1 || n_levels > 8) return fail(XMGN_ERR_INVALID, "n_levels must be in [1, 8]");
  for (int l = 0; l < n_levels; ++l) {
    if (level_end[l] <= (l ? level_end[l - 1] : 0)) return fail(XMGN_ERR_INVALID, "level_end must increase");
  }
  if (level_end[n_levels - 1] != n) return fail(XMGN_ERR_INVALID, "last level_end must equal n");
  if (k_intra < 1 || k_intra > 16 || k_intra >= level_end[0]) return fail(XMGN_ERR_INVALID, "bad k_intra");
  if (k_cross < 0 || k_cross > 16 || (n_levels > 1 && k_cross >= level_end[0])) return fail(XMGN_ERR_INVALID, "bad k_cross");
  if (n_levels * k_intra + (n_levels - 1) * k_cross > 64) return fail(XMGN_ERR_UNSUPPORTED, "too many lists per node");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  int* rp = nullptr;
  int* col = nullptr;
  long long E = 0;
  const char* err = "";
  const int rc = knn_build(pos, n, level_end, n_levels, k_intra, n_levels > 1 ? k_cross : 0,
                           &rp, &col, &E, st, &err);
  if (rc != 0) return fail(rc == -2 ? XMGN_ERR_OOM : XMGN_ERR_HIP, std::string("kNN build failed: ") + err);
  auto g = std::make_unique<xmgn_graph>();
  g->n = n;
  g->row_ptr.resize(n + 1);
  g->col.resize(E);
  hipError_t e1 = hipMemcpy(g->row_ptr.data(), rp, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost);
  hipError_t e2 = E > 0 ? hipMemcpy(g->col.data(), col, (size_t)E * 4, hipMemcpyDeviceToHost) : hipSuccess;
  (void)hipFree(rp);
  (void)hipFree(col);
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(XMGN_ERR_HIP, "copy of the graph to the host failed");
  *out = g.release();
  return XMGN_OK;
  GUARD_END
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
static std::string tune_key(const xmgn_ctx* c, const xmgn_model_desc* d) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream k;
  k << arch.substr(0, arch.find(':')) << ":H" << d->hidden << ":L" << d->n_layers << ":p" << d->precision << ":a"
    << d->activation << ":g" << d->aggregate << ":t" << (c->tape_hidden ? 1 : 0) << ":s" << (c->edge_split ? 1 : 0)
    << ":n" << c->cur->n << ":E"
    << c->cur->E;
  return k.str();
}

extern "C" xmgn_status xmgn_autotune(xmgn_ctx* c, const xmgn_model_desc* d, const float* params,
                                     const xmgn_partset* ps, const int32_t* part_ids, int32_t n_batch,
                                     const float* node_in, const float* pos, const float* edge_norm, float* out,
                                     const float* d_out, float* d_params, const char* cache_path,
                                     int32_t* edge_rows, int32_t* node_rows, int32_t* grid, int32_t* edge_waves,
                                     float* step_ms, xmgn_stream stream) {
  GUARD_BEGIN
  if (!c) return fail(XMGN_ERR_INVALID, "ctx is NULL");
  if (xmgn_status s = check_desc(d)) return s;
  if (!d_out || !d_params) return fail(XMGN_ERR_INVALID, "NULL argument");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, c->device));
  const int cus = prop.multiProcessorCount;
  // the key needs the batch sizes: build the plan with the current tiles first
  if (xmgn_status r = xmgn_forward(c, d, params, ps, part_ids, n_batch, node_in, pos, edge_norm, out, 1, stream))
    return r;
  const std::string key = tune_key(c, d);
  int best[6] = {0, 0, 0, 0, 0, 0};  // edge rows, node rows, grid, edge waves, adjoint edge rows, adjoint waves
  float best_ms = -1.f;
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      std::istringstream is(line);
      std::string k;
      int e, n, g, wv, br, bw;
      float ms;
      if (is >> k >> e >> n >> g >> wv >> br >> bw >> ms && k == key) {
        best[0] = e;
        best[1] = n;
        best[2] = g;
        best[3] = wv;
        best[4] = br;
        best[5] = bw;
        best_ms = ms;
      }
    }
  }
  if (best_ms < 0.f) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    xmgn_status err = XMGN_OK;
    auto trial = [&](int er, int nr, int g, int wv, int br, int bw) -> xmgn_status {
      if (xmgn_status r = xmgn_ctx_set_tiles(c, er, nr, g, wv)) return r;
      if (xmgn_status r = xmgn_ctx_set_bwd_tiles(c, br, bw)) return r;
      auto step = [&]() -> xmgn_status {
        if (xmgn_status r = xmgn_forward(c, d, params, ps, part_ids, n_batch, node_in, pos, edge_norm, out, 1, stream))
          return r;
        return xmgn_backward(c, d, params, d_out, d_params, stream);
      };
      if (xmgn_status r = step()) return r;
      (void)hipEventRecord(a, st);
      for (int i = 0; i < 2; ++i)
        if (xmgn_status r = step()) return r;
      (void)hipEventRecord(b, st);
      (void)hipEventSynchronize(b);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      ms *= 0.5f;
      if (best_ms < 0.f || ms < best_ms) {
        best_ms = ms;
        best[0] = er;
        best[1] = nr;
        best[2] = g;
        best[3] = wv;
        best[4] = br;
        best[5] = bw;
      }
      return XMGN_OK;
    };
    std::vector<int> rows = d->hidden == 128 || (d->hidden == 256 && d->precision == 1) ? std::vector<int>{32, 64}
                                                                                         : std::vector<int>{32};
    if (d->hidden == 256 && d->precision == 1 && !c->edge_split) rows.push_back(128);  // the wide forward
    // stage 1: edge kernels (the bulk of the step), stage 2: node tiles
    for (int er : rows)
      for (int wv : {4, 8})
        for (int wpc : {4, 8})
          if (!err) err = trial(er, 32, ((cus * wpc + 7) / 8) * 8, wv, 0, 0);
    if (!err && d->hidden == 128) err = trial(best[0], 64, best[2], best[3], 0, 0);
    // stage 3: the edge adjoint on its own waves per workgroup and (BF16,
    // H = 128 and 256) its own tile rows, against each forward tiling and
    // wave count (stage 1 timed the adjoint on the forward's rows and waves
    // only)
    if (!err) {
      const bool own_rows = (d->hidden == 128 || d->hidden == 256) && d->precision == 1;
      const int nr = best[1], g = best[2];
      const std::vector<int> ers = own_rows ? rows : std::vector<int>{best[0]};
      const std::vector<int> brs = own_rows ? std::vector<int>{32, 64} : std::vector<int>{0};
      for (int er : ers)
        for (int wv : {4, 8})
          for (int br : brs)
            for (int bw : {4, 8})
              if (!err && !((br == 0 || br == er) && bw == wv)) err = trial(er, nr, g, wv, br, bw);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (err) return err;
    if (cache_path) {
      std::ofstream f(cache_path, std::ios::app);
      f << key << " " << best[0] << " " << best[1] << " " << best[2] << " " << best[3] << " " << best[4] << " "
        << best[5] << " " << best_ms << "\n";
    }
  }
  if (xmgn_status r = xmgn_ctx_set_tiles(c, best[0], best[1], best[2], best[3])) return r;
  if (xmgn_status r = xmgn_ctx_set_bwd_tiles(c, best[4], best[5])) return r;
  if (edge_rows) *edge_rows = best[0];
  if (node_rows) *node_rows = best[1];
  if (grid) *grid = best[2];
  if (edge_waves) *edge_waves = best[3];
  if (step_ms) *step_ms = best_ms;
  return XMGN_OK;
  GUARD_END
}
