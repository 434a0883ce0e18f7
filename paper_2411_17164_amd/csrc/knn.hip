// Multi-scale kNN graph construction on the GPU (Sec. III.B, III.C).
//
// Per level l (points [0, n_l)):
//   1. uniform grid over the level's bounding box: count -> scan -> scatter,
//      candidates stored in cell order as float4 {x, y, z, id};
//   2. one thread per query searches cells in growing Chebyshev shells
//      around its cell, keeping the K best candidates under the key (d2, id);
//      d2 is evaluated in FP64 as ((dx*dx + dy*dy) + dz*dz) without fused
//      multiply-add, so the ranking is exact and ties go to the lower index.
//      The search stops when the K-th best d2 is below the squared distance
//      from the query to every unvisited cell;
//   3. cross-level lists: queries of level l against the grid of level l-1.
// Then one thread per receiver merges its lists, sorts by sender id and
// drops repeated pairs (count pass, scan, write pass) into a CSR.
#include <hipcub/hipcub.hpp>

#include <cfloat>
#include <climits>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace xmgn {

struct GridInfo {
  double lo[3];
  double cs;
  double inv_cs;
  int dim[3];
};

__device__ __forceinline__ int cell_coord(double x, const GridInfo& g, int a) {
  const double t = floor((x - g.lo[a]) * g.inv_cs);
  int c = t < 0.0 ? 0 : (t > (double)(g.dim[a] - 1) ? g.dim[a] - 1 : (int)t);
  return c;
}

__global__ void k_bbox(const float* __restrict__ pos, int n, float* __restrict__ part) {
  __shared__ float s[6][256];
  float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    for (int a = 0; a < 3; ++a) {
      const float v = pos[(size_t)i * 3 + a];
      mn[a] = fminf(mn[a], v);
      mx[a] = fmaxf(mx[a], v);
    }
  for (int a = 0; a < 3; ++a) {
    s[a][threadIdx.x] = mn[a];
    s[3 + a][threadIdx.x] = mx[a];
  }
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + k]);
        s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + k]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_cell_count(const float* __restrict__ pos, int n, GridInfo g, int* __restrict__ cell,
                             int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int cx = cell_coord((double)pos[(size_t)i * 3 + 0], g, 0);
  const int cy = cell_coord((double)pos[(size_t)i * 3 + 1], g, 1);
  const int cz = cell_coord((double)pos[(size_t)i * 3 + 2], g, 2);
  const int c = (cz * g.dim[1] + cy) * g.dim[0] + cx;
  cell[i] = c;
  atomicAdd(count + c, 1);
}

__global__ void k_cell_scatter(const float* __restrict__ pos, int n, const int* __restrict__ cell,
                               const int* __restrict__ start, int* __restrict__ fill, float4* __restrict__ spos,
                               int* __restrict__ sorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cell[i];
  const int slot = start[c] + atomicAdd(fill + c, 1);
  spos[slot] = make_float4(pos[(size_t)i * 3], pos[(size_t)i * 3 + 1], pos[(size_t)i * 3 + 2], __int_as_float(i));
  sorted[slot] = i;
}

template <int K>
__global__ __launch_bounds__(256) void k_knn_query(const float4* __restrict__ spos, const int* __restrict__ start,
                                                   GridInfo g, const int* __restrict__ qorder, int nq,
                                                   const float* __restrict__ pos, int* __restrict__ out) {
#pragma clang fp contract(off)
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nq) return;
  const int q = qorder[t];
  const double qx = (double)pos[(size_t)q * 3], qy = (double)pos[(size_t)q * 3 + 1], qz = (double)pos[(size_t)q * 3 + 2];
  const int cx = cell_coord(qx, g, 0), cy = cell_coord(qy, g, 1), cz = cell_coord(qz, g, 2);
  double bd[K];
  int bj[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    bd[i] = DBL_MAX;
    bj[i] = INT_MAX;
  }
  for (int R = 0;; ++R) {
    const int z0 = max(cz - R, 0), z1 = min(cz + R, g.dim[2] - 1);
    const int y0 = max(cy - R, 0), y1 = min(cy + R, g.dim[1] - 1);
    const int x0 = max(cx - R, 0), x1 = min(cx + R, g.dim[0] - 1);
    auto visit = [&](int x, int y, int z) {
      const int c = (z * g.dim[1] + y) * g.dim[0] + x;
      const int s1 = start[c + 1];
      for (int s = start[c]; s < s1; ++s) {
        const float4 p = spos[s];
        const int j = __float_as_int(p.w);
        if (j == q) continue;
        const double dx = (double)p.x - qx, dy = (double)p.y - qy, dz = (double)p.z - qz;
        const double dxx = dx * dx, dyy = dy * dy, dzz = dz * dz;
        const double d2 = (dxx + dyy) + dzz;
        if (d2 < bd[K - 1] || (d2 == bd[K - 1] && j < bj[K - 1])) {
          double cd = d2;
          int cj = j;
#pragma unroll
          for (int i = 0; i < K; ++i) {
            const bool lt = (cd < bd[i]) || (cd == bd[i] && cj < bj[i]);
            const double td = lt ? bd[i] : cd;
            const int tj = lt ? bj[i] : cj;
            bd[i] = lt ? cd : bd[i];
            bj[i] = lt ? cj : bj[i];
            cd = td;
            cj = tj;
          }
        }
      }
    };
    // cells at Chebyshev distance exactly R from (cx, cy, cz)
    for (int z = z0; z <= z1; ++z) {
      const bool zf = (z == cz - R) || (z == cz + R);
      for (int y = y0; y <= y1; ++y) {
        if (zf || y == cy - R || y == cy + R) {
          for (int x = x0; x <= x1; ++x) visit(x, y, z);
        } else {
          if (cx - R >= 0) visit(cx - R, y, z);
          if (R > 0 && cx + R <= g.dim[0] - 1) visit(cx + R, y, z);
        }
      }
    }
    // lower bound on the distance to any cell outside the visited block
    const bool all = cx - R <= 0 && cy - R <= 0 && cz - R <= 0 && cx + R >= g.dim[0] - 1 &&
                     cy + R >= g.dim[1] - 1 && cz + R >= g.dim[2] - 1;
    if (all) break;
    double bound = DBL_MAX;
    const double qc[3] = {qx, qy, qz};
    const int cc[3] = {cx, cy, cz};
    for (int a = 0; a < 3; ++a) {
      if (cc[a] - R > 0) bound = fmin(bound, qc[a] - (g.lo[a] + (double)(cc[a] - R) * g.cs));
      if (cc[a] + R < g.dim[a] - 1) bound = fmin(bound, (g.lo[a] + (double)(cc[a] + R + 1) * g.cs) - qc[a]);
    }
    bound -= 1e-7 * g.cs;
    if (bound > 0.0 && bj[K - 1] != INT_MAX && bd[K - 1] < bound * bound) break;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) out[(size_t)q * K + i] = bj[i];
}

constexpr int KNN_MAXL = 8;
constexpr int KNN_MAXC = 64;
struct Lists {
  int n_levels;
  int level_end[KNN_MAXL];
  const int* intra[KNN_MAXL];
  const int* cross[KNN_MAXL];
  int k_intra, k_cross;
};

__device__ __forceinline__ int gather_sorted(const Lists& L, int r, int* buf) {
  int cnt = 0;
  for (int l = 0; l < L.n_levels; ++l) {
    if (r >= L.level_end[l]) continue;
    for (int i = 0; i < L.k_intra; ++i) buf[cnt++] = L.intra[l][(size_t)r * L.k_intra + i];
    if (l >= 1)
      for (int i = 0; i < L.k_cross; ++i) buf[cnt++] = L.cross[l][(size_t)r * L.k_cross + i];
  }
  for (int i = 1; i < cnt; ++i) {
    const int v = buf[i];
    int j = i - 1;
    while (j >= 0 && buf[j] > v) {
      buf[j + 1] = buf[j];
      --j;
    }
    buf[j + 1] = v;
  }
  int u = 0;
  for (int i = 0; i < cnt; ++i)
    if (i == 0 || buf[i] != buf[i - 1]) buf[u++] = buf[i];
  return u;
}

__global__ void k_union_count(Lists L, int n, int* __restrict__ deg) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int buf[KNN_MAXC];
  deg[r] = gather_sorted(L, r, buf);
}

__global__ void k_union_write(Lists L, int n, const int* __restrict__ row_ptr, int* __restrict__ col) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int buf[KNN_MAXC];
  const int u = gather_sorted(L, r, buf);
  int* dst = col + row_ptr[r];
  for (int i = 0; i < u; ++i) dst[i] = buf[i];
}

// ---------------------------------------------------------------------------
namespace {

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes > 0 ? bytes : 4); }
};

struct Grid {
  GridInfo info;
  int ncell = 0;
  DevBuf start, spos, sorted;
};

#define KNN_CHECK(x)                          \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) {                   \
      *err = hipGetErrorString(e_);           \
      return -3;                              \
    }                                         \
  } while (0)

int exclusive_scan(const int* in, int* out, int n, hipStream_t st, const char** err) {
  size_t tmp = 0;
  KNN_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in, out, n, st));
  DevBuf t;
  KNN_CHECK(t.alloc(tmp));
  KNN_CHECK(hipcub::DeviceScan::ExclusiveSum(t.p, tmp, in, out, n, st));
  KNN_CHECK(hipStreamSynchronize(st));
  return 0;
}

int build_grid(const float* pos, int n, Grid& g, hipStream_t st, const char** err) {
  const int nb = 256;
  DevBuf part;
  KNN_CHECK(part.alloc(nb * 6 * sizeof(float)));
  k_bbox<<<nb, 256, 0, st>>>(pos, n, (float*)part.p);
  std::vector<float> hp(nb * 6);
  KNN_CHECK(hipMemcpyAsync(hp.data(), part.p, hp.size() * sizeof(float), hipMemcpyDeviceToHost, st));
  KNN_CHECK(hipStreamSynchronize(st));
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int b = 0; b < nb; ++b)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::fmin(lo[a], (double)hp[b * 6 + a]);
      hi[a] = std::fmax(hi[a], (double)hp[b * 6 + 3 + a]);
    }
  double ext[3];
  for (int a = 0; a < 3; ++a) ext[a] = hi[a] - lo[a];
  // cell edge from the mean spacing of a surface sample: sqrt(8 A / n), A =
  // bounding-box surface area (a performance choice only; any edge is exact)
  const double area = 2.0 * (ext[0] * ext[1] + ext[1] * ext[2] + ext[0] * ext[2]);
  double cs = std::sqrt(8.0 * area / (double)n);
  const double emax = std::fmax(ext[0], std::fmax(ext[1], ext[2]));
  if (!(cs > 0.0)) cs = emax > 0.0 ? emax : 1.0;
  for (;;) {
    double cells = 1.0;
    for (int a = 0; a < 3; ++a) cells *= std::fmax(1.0, std::ceil(ext[a] / cs));
    if (cells <= (double)(1 << 24)) break;
    cs *= std::cbrt(cells / (double)(1 << 24)) * 1.01;
  }
  for (int a = 0; a < 3; ++a) {
    g.info.lo[a] = lo[a];
    g.info.dim[a] = (int)std::fmax(1.0, std::ceil(ext[a] / cs));
  }
  g.info.cs = cs;
  g.info.inv_cs = 1.0 / cs;
  g.ncell = g.info.dim[0] * g.info.dim[1] * g.info.dim[2];
  DevBuf cell, count, fill;
  KNN_CHECK(cell.alloc((size_t)n * sizeof(int)));
  KNN_CHECK(count.alloc((size_t)(g.ncell + 1) * sizeof(int)));
  KNN_CHECK(fill.alloc((size_t)(g.ncell + 1) * sizeof(int)));
  KNN_CHECK(g.start.alloc((size_t)(g.ncell + 1) * sizeof(int)));
  KNN_CHECK(g.spos.alloc((size_t)n * sizeof(float4)));
  KNN_CHECK(g.sorted.alloc((size_t)n * sizeof(int)));
  KNN_CHECK(hipMemsetAsync(count.p, 0, (size_t)(g.ncell + 1) * sizeof(int), st));
  KNN_CHECK(hipMemsetAsync(fill.p, 0, (size_t)(g.ncell + 1) * sizeof(int), st));
  k_cell_count<<<(n + 255) / 256, 256, 0, st>>>(pos, n, g.info, (int*)cell.p, (int*)count.p);
  if (int rc = exclusive_scan((const int*)count.p, (int*)g.start.p, g.ncell + 1, st, err)) return rc;
  k_cell_scatter<<<(n + 255) / 256, 256, 0, st>>>(pos, n, (const int*)cell.p, (const int*)g.start.p, (int*)fill.p,
                                                   (float4*)g.spos.p, (int*)g.sorted.p);
  KNN_CHECK(hipStreamSynchronize(st));
  return 0;
}

void launch_query(int k, const Grid& cand, const int* qorder, int nq, const float* pos, int* out, hipStream_t st) {
  const dim3 grid((nq + 255) / 256);
  const float4* sp = (const float4*)cand.spos.p;
  const int* s = (const int*)cand.start.p;
  switch (k) {
#define XMGN_KQ(KV) \
  case KV:          \
    k_knn_query<KV><<<grid, 256, 0, st>>>(sp, s, cand.info, qorder, nq, pos, out); \
    break;
    XMGN_KQ(1) XMGN_KQ(2) XMGN_KQ(3) XMGN_KQ(4) XMGN_KQ(5) XMGN_KQ(6) XMGN_KQ(7) XMGN_KQ(8)
    XMGN_KQ(9) XMGN_KQ(10) XMGN_KQ(11) XMGN_KQ(12) XMGN_KQ(13) XMGN_KQ(14) XMGN_KQ(15) XMGN_KQ(16)
#undef XMGN_KQ
    default:
      break;
  }
}

}  // namespace

int knn_build(const float* pos, int n, const int* level_end, int n_levels, int k_intra, int k_cross,
              int** row_ptr_out, int** col_out, long long* n_edges, hipStream_t st, const char** err) {
  *row_ptr_out = nullptr;
  *col_out = nullptr;
  std::vector<Grid> grids(n_levels);
  std::vector<DevBuf> intra(n_levels), cross(n_levels);
  for (int l = 0; l < n_levels; ++l) {
    const int nl = level_end[l];
    if (int rc = build_grid(pos, nl, grids[l], st, err)) return rc;
    KNN_CHECK(intra[l].alloc((size_t)nl * k_intra * sizeof(int)));
    launch_query(k_intra, grids[l], (const int*)grids[l].sorted.p, nl, pos, (int*)intra[l].p, st);
    if (l >= 1 && k_cross > 0) {
      KNN_CHECK(cross[l].alloc((size_t)nl * k_cross * sizeof(int)));
      launch_query(k_cross, grids[l - 1], (const int*)grids[l].sorted.p, nl, pos, (int*)cross[l].p, st);
    }
    KNN_CHECK(hipGetLastError());
  }
  Lists L{};
  L.n_levels = n_levels;
  L.k_intra = k_intra;
  L.k_cross = k_cross;
  for (int l = 0; l < n_levels; ++l) {
    L.level_end[l] = level_end[l];
    L.intra[l] = (const int*)intra[l].p;
    L.cross[l] = (l >= 1 && k_cross > 0) ? (const int*)cross[l].p : nullptr;
  }
  if (k_cross == 0) L.k_cross = 0;
  DevBuf deg;
  KNN_CHECK(deg.alloc((size_t)(n + 1) * sizeof(int)));
  KNN_CHECK(hipMemsetAsync(deg.p, 0, (size_t)(n + 1) * sizeof(int), st));
  k_union_count<<<(n + 255) / 256, 256, 0, st>>>(L, n, (int*)deg.p);
  int* row_ptr = nullptr;
  KNN_CHECK(hipMalloc(&row_ptr, (size_t)(n + 1) * sizeof(int)));
  if (int rc = exclusive_scan((const int*)deg.p, row_ptr, n + 1, st, err)) {
    (void)hipFree(row_ptr);
    return rc;
  }
  int E = 0;
  hipError_t e1 = hipMemcpyAsync(&E, row_ptr + n, sizeof(int), hipMemcpyDeviceToHost, st);
  hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(st) : e1;
  if (e2 != hipSuccess) {
    (void)hipFree(row_ptr);
    *err = hipGetErrorString(e2);
    return -3;
  }
  int* col = nullptr;
  hipError_t e3 = hipMalloc(&col, (size_t)(E > 0 ? E : 1) * sizeof(int));
  if (e3 != hipSuccess) {
    (void)hipFree(row_ptr);
    *err = hipGetErrorString(e3);
    return -2;
  }
  k_union_write<<<(n + 255) / 256, 256, 0, st>>>(L, n, row_ptr, col);
  hipError_t e4 = hipStreamSynchronize(st);
  if (e4 == hipSuccess) e4 = hipGetLastError();
  if (e4 != hipSuccess) {
    (void)hipFree(row_ptr);
    (void)hipFree(col);
    *err = hipGetErrorString(e4);
    return -3;
  }
  *row_ptr_out = row_ptr;
  *col_out = col;
  *n_edges = E;
  return 0;
}

}  // namespace xmgn
