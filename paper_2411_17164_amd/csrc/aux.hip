// Auxiliary kernels: weight gradients as row-sums of outer products
// (split over row chunks, reduced in a fixed order), fixed-order reductions
// of per-workgroup partial vectors, weight preparation (cast / transpose into
// the compute type), the masked MSE and gradient accumulation.
#include <mutex>
#include <stdexcept>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace xmgn {

int g_config_error = 0;

// ---------------------------------------------------------------------------
// wgrad: C[m][n] = sum_r A[r][a0 + m] * B[r][b0 + n].  A workgroup owns one
// chunk of rows and one 128x128 output block.  Rows go through LDS 128 at a
// time, transposed so that the row index is the MFMA k dimension; the loads
// of the next stage are issued before the products of the current one, so
// their round trip overlaps the MFMAs.
// ---------------------------------------------------------------------------
constexpr int WG_B = 128;  // output block edge
constexpr int WG_K = 128;  // rows per stage

template <typename T>
struct WgLds {
  static constexpr int PAD = 16 / sizeof(T);
  static constexpr int LD = WG_K + PAD;
};

// One thread's share of a stage: 4 columns (4 (t % 32)) of 16 rows
// (16 (t / 32)) of one operand, loaded as 8 (BF16) or 16 (FP32) bytes per row.
template <typename S>
struct Slab {
  using L = typename std::conditional<sizeof(S) == 4, float4, uint2>::type;
  L v[16];
  __device__ __forceinline__ void load(const S* base, int ld, int col0, const int* idx, int r0, int r_end, int c0,
                                       int C) {
    const int c = c0 + 4 * ((int)threadIdx.x & 31), rr = r0 + 16 * ((int)threadIdx.x >> 5);
    const S* p = base + col0 + c;
    // uniform branch: a gathered operand loads its 16 row indices first, so
    // that neither path waits between its data loads
    if (idx) {
      int ri[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) ri[j] = (c < C && rr + j < r_end) ? idx[rr + j] : -1;
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = ri[j] >= 0 ? *(const L*)(p + (size_t)ri[j] * ld) : L{};
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = (c < C && rr + j < r_end) ? *(const L*)(p + (size_t)(rr + j) * ld) : L{};
    }
  }
  // column q of the 4, as 16 consecutive k values
  template <typename T>
  __device__ __forceinline__ void store(T* dst) const {
    constexpr int LD = WgLds<T>::LD;
    T* d0 = dst + (4 * ((int)threadIdx.x & 31)) * LD + 16 * ((int)threadIdx.x >> 5);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T col[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if constexpr (sizeof(S) == 4) {
          col[j] = from_f<T>(((const float*)&v[j])[q]);
        } else {
          col[j] = from_f<T>(to_f(((const S*)&v[j])[q]));
        }
      }
#pragma unroll
      for (int j = 0; j < 16; j += 16 / (int)sizeof(T)) *(uint4*)(d0 + q * LD + j) = *(const uint4*)&col[j];
    }
  }
};

template <typename T, typename SA, typename SB>
__global__ __launch_bounds__(NTHR, 2) void k_wgrad(WgradOp op, int rows_per_chunk, int nbm, float* __restrict__ partial) {
  using V = typename TT<T>::V;
  constexpr int E = TT<T>::E, KC = 4 * E, LD = WgLds<T>::LD;
  __shared__ __align__(16) T At[WG_B * LD];
  __shared__ __align__(16) T Bt[WG_B * LD];
  const int chunk = blockIdx.x;
  const int bm = blockIdx.y % nbm, bn = blockIdx.y / nbm;
  const int m0 = bm * WG_B, nn0 = bn * WG_B;
  const int r_begin = chunk * rows_per_chunk;
  const int r_end = min(op.R, r_begin + rows_per_chunk);
  const int w = wave_id(), wm = w & 1, wn = w >> 1;
  const int l = lane_id(), li = l & 15, lg = l >> 4;
  f32x4 acc[4][4];
  zero_acc(acc);
  Slab<SA> sa;
  Slab<SB> sb;
  sa.load((const SA*)op.A, op.lda, op.a0, op.ia, r_begin, r_end, m0, op.M);
  sb.load((const SB*)op.B, op.ldb, op.b0, op.ib, r_begin, r_end, nn0, op.N);
  for (int r0 = r_begin; r0 < r_end; r0 += WG_K) {
    __syncthreads();  // the previous stage's products are done with At, Bt
    sa.template store<T>(At);
    sb.template store<T>(Bt);
    __syncthreads();
    if (r0 + WG_K < r_end) {  // next stage in flight during this stage's MFMAs
      sa.load((const SA*)op.A, op.lda, op.a0, op.ia, r0 + WG_K, r_end, m0, op.M);
      sb.load((const SB*)op.B, op.ldb, op.b0, op.ib, r0 + WG_K, r_end, nn0, op.N);
    }
#pragma unroll
    for (int k = 0; k < WG_K; k += KC) {
      V bfr[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) bfr[nb] = *(const V*)(Bt + (wn * 64 + nb * 16 + li) * LD + k + lg * E);
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const V a = *(const V*)(At + (wm * 64 + mb * 16 + li) * LD + k + lg * E);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = mma(a, bfr[nb], acc[mb][nb]);
      }
    }
  }
  float* out = partial + (size_t)chunk * op.M * op.N;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + mb * 16 + lg * 4 + r;
        const int n = nn0 + wn * 64 + nb * 16 + li;
        if (m < op.M && n < op.N) out[(size_t)m * op.N + n] = acc[mb][nb][r];
      }
}

// Fixed-order column sums of a [rows][stride] partial matrix, in two
// stages: stage 1 sums rows [s*per, (s+1)*per) of each column into
// tmp[s][col] (grid.y = split s); stage 2 adds the splits in order.  The
// result depends only on (rows, splits), never on scheduling.
constexpr int RED_SPLITS = 32;

__global__ void k_colsum_stage1(const float* __restrict__ src, int rows, int stride, int ncol, int per,
                                float* __restrict__ tmp) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  const int s = blockIdx.y;
  const int r0 = s * per, r1 = min(rows, r0 + per);
  float a0 = 0.f, a1 = 0.f;
  int r = r0;
  for (; r + 1 < r1; r += 2) {  // two independent loads in flight, fixed pairing
    a0 += src[(size_t)r * stride + j];
    a1 += src[(size_t)(r + 1) * stride + j];
  }
  if (r < r1) a0 += src[(size_t)r * stride + j];
  tmp[(size_t)s * ncol + j] = a0 + a1;
}

__global__ void k_wgrad_reduce(const float* __restrict__ tmp, int splits, int M_valid, int N,
                               float* __restrict__ dst, int ldd, int ncol) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M_valid * N) return;
  const int m = idx / N, n = idx - m * N;
  float s = 0.f;
  for (int k = 0; k < splits; ++k) s += tmp[(size_t)k * ncol + idx];
  dst[(size_t)m * ldd + n] = s;
}

size_t reduce_tmp_floats(int max_cols) { return (size_t)RED_SPLITS * (size_t)max_cols; }

// dst[m * ldd + n] = sum over r < rows of src[r * stride + m * N + n], m < M_valid.
// tmp: caller scratch of reduce_tmp_floats(M_valid * N) floats.
static void colsum_to(const float* src, int rows, int stride, int M_valid, int N, float* dst, int ldd, float* tmp,
                      hipStream_t st) {
  const int ncol = M_valid * N;
  const int splits = rows < RED_SPLITS ? (rows > 0 ? rows : 1) : RED_SPLITS;
  const int per = rows > 0 ? (rows + splits - 1) / splits : 0;
  k_colsum_stage1<<<dim3((ncol + 255) / 256, splits), 256, 0, st>>>(src, rows, stride, ncol, per, tmp);
  k_wgrad_reduce<<<(ncol + 255) / 256, 256, 0, st>>>(tmp, splits, M_valid, N, dst, ldd, ncol);
}

void launch_wgrad_reduce(const float* partial, int n_chunks, int M_valid, int N, float* dst, int ldd, int MN,
                         float* tmp, hipStream_t st) {
  colsum_to(partial, n_chunks, MN, M_valid, N, dst, ldd, tmp, st);
}

// Row chunks of a weight gradient: about 512 workgroups in all (two per CU),
// whole 128-row stages per chunk.
static int wgrad_chunks(const WgradOp& op, int* rows_per_chunk) {
  *rows_per_chunk = WG_K;
  if (op.R <= 0) return 0;
  const int blocks = ((op.M + WG_B - 1) / WG_B) * ((op.N + WG_B - 1) / WG_B);
  int target = 512 / blocks;
  const int max_chunks = (op.R + WG_K - 1) / WG_K;
  if (target > max_chunks) target = max_chunks;
  if (target < 1) target = 1;
  int rpc = (op.R + target - 1) / target;
  rpc = (rpc + WG_K - 1) / WG_K * WG_K;
  *rows_per_chunk = rpc;
  return (op.R + rpc - 1) / rpc;
}

size_t wgrad_partial_floats(const Shape&, const WgradOp& op) {
  int rpc;
  const int nc = wgrad_chunks(op, &rpc);
  return (size_t)(nc > 0 ? nc : 1) * op.M * op.N;
}

void launch_wgrad(const Shape& s, const WgradOp& op, float* partial, float* tmp, hipStream_t st) {
  int rpc;
  const int nc = wgrad_chunks(op, &rpc);
  const int nbm = (op.M + WG_B - 1) / WG_B, nbn = (op.N + WG_B - 1) / WG_B;
  if (nc > 0) {
    dim3 grid(nc, nbm * nbn);
    if (s.prec == 1) {
      if (op.a_f32 && op.b_f32) k_wgrad<bf16, float, float><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
      else if (op.a_f32) k_wgrad<bf16, float, bf16><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
      else if (op.b_f32) k_wgrad<bf16, bf16, float><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
      else k_wgrad<bf16, bf16, bf16><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
    } else {
      k_wgrad<float, float, float><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
    }
  }
  colsum_to(partial, nc, op.M * op.N, op.M_valid, op.N, op.dst, op.ldd, tmp, st);
}

void launch_wgrad_partials(const Shape& s, const WgradOp& op, float* partial, RedBatch& b, hipStream_t st) {
  int rpc;
  const int nc = wgrad_chunks(op, &rpc);
  const int nbm = (op.M + WG_B - 1) / WG_B, nbn = (op.N + WG_B - 1) / WG_B;
  if (nc > 0) {
    dim3 grid(nc, nbm * nbn);
    if (s.prec == 1) {
      if (op.a_f32 && op.b_f32) k_wgrad<bf16, float, float><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
      else if (op.a_f32) k_wgrad<bf16, float, bf16><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
      else if (op.b_f32) k_wgrad<bf16, bf16, float><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
      else k_wgrad<bf16, bf16, bf16><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
    } else {
      k_wgrad<float, float, float><<<grid, NTHR, 0, st>>>(op, rpc, nbm, partial);
    }
  }
  b.add(partial, nc, op.M * op.N, op.M_valid, op.N, op.dst, op.ldd);
}

// Batched form: blockIdx.z selects the job; the per-job work is exactly
// k_colsum_stage1's and k_wgrad_reduce's.
__global__ void k_colsum_batch1(RedBatch b, float* __restrict__ tmp) {
  const RedJob& jb = b.job[blockIdx.z];
  const int ncol = jb.M_valid * jb.N;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= ncol || s >= jb.splits) return;
  const int r0 = s * jb.per, r1 = min(jb.rows, r0 + jb.per);
  float a0 = 0.f, a1 = 0.f;
  int r = r0;
  for (; r + 1 < r1; r += 2) {
    a0 += jb.src[(size_t)r * jb.stride + j];
    a1 += jb.src[(size_t)(r + 1) * jb.stride + j];
  }
  if (r < r1) a0 += jb.src[(size_t)r * jb.stride + j];
  tmp[jb.tmp_off + (size_t)s * ncol + j] = a0 + a1;
}

__global__ void k_colsum_batch2(RedBatch b, const float* __restrict__ tmp) {
  const RedJob& jb = b.job[blockIdx.y];
  const int ncol = jb.M_valid * jb.N;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncol) return;
  const int m = idx / jb.N, n = idx - m * jb.N;
  float s = 0.f;
  for (int k = 0; k < jb.splits; ++k) s += tmp[jb.tmp_off + (size_t)k * ncol + idx];
  jb.dst[(size_t)m * jb.ldd + n] = s;
}

void RedBatch::add(const float* src, int rows, int stride, int M_valid, int N, float* dst, int ldd) {
  if (n >= kMaxRedJobs) throw std::runtime_error("reduction batch is full");
  RedJob& j = job[n++];
  j.src = src;
  j.dst = dst;
  j.rows = rows;
  j.stride = stride;
  j.M_valid = M_valid;
  j.N = N;
  j.ldd = ldd;
  j.splits = rows < RED_SPLITS ? (rows > 0 ? rows : 1) : RED_SPLITS;
  j.per = rows > 0 ? (rows + j.splits - 1) / j.splits : 0;
  j.tmp_off = tmp_floats;
  tmp_floats += (long long)j.splits * M_valid * N;
  if (M_valid * N > max_cols) max_cols = M_valid * N;
}

void RedBatch::add_vec(const float* partial, int G, int row, const VecSeg* segs, int n_seg) {
  for (int i = 0; i < n_seg; ++i) add(partial + segs[i].src, G, row, 1, segs[i].len, segs[i].dst, 0);
}

void launch_reduce_batch(const RedBatch& b, float* tmp, hipStream_t st) {
  if (b.n == 0) return;
  k_colsum_batch1<<<dim3((b.max_cols + 255) / 256, RED_SPLITS, b.n), 256, 0, st>>>(b, tmp);
  k_colsum_batch2<<<dim3((b.max_cols + 255) / 256, b.n), 256, 0, st>>>(b, tmp);
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of per-workgroup partial rows.
// ---------------------------------------------------------------------------
struct VecSegs {
  int n;
  int src[16];
  int len[16];
  int inner[16];       // elements per contiguous run
  int src_stride[16];  // partial-row stride between runs
  int dst_stride[16];
  float* dst[16];
};

__global__ void k_vec_reduce(const float* __restrict__ tmp, int splits, int row, VecSegs s) {
  const int seg = blockIdx.y;
  if (seg >= s.n) return;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < s.len[seg]; j += gridDim.x * blockDim.x) {
    const int run = j / s.inner[seg], k = j - run * s.inner[seg];
    const int src = s.src[seg] + run * s.src_stride[seg] + k;
    float acc = 0.f;
    for (int g = 0; g < splits; ++g) acc += tmp[(size_t)g * row + src];
    s.dst[seg][run * s.dst_stride[seg] + k] = acc;
  }
}

// stage 1 of the vector reductions: column sums of [G][row] in RED_SPLITS groups
static const float* vec_stage1(const float* partial, int G, int row, int* splits, float* tmp, hipStream_t st) {
  *splits = G < RED_SPLITS ? G : RED_SPLITS;
  const int per = (G + *splits - 1) / *splits;
  k_colsum_stage1<<<dim3((row + 255) / 256, *splits), 256, 0, st>>>(partial, G, row, row, per, tmp);
  return tmp;
}

void launch_vec_reduce(const float* partial, int G, int row, const VecSeg* segs, int n_seg, float* tmp,
                       hipStream_t st) {
  VecSegs s{};
  s.n = n_seg;
  int maxlen = 1;
  for (int i = 0; i < n_seg; ++i) {
    s.src[i] = segs[i].src;
    s.len[i] = segs[i].len;
    s.inner[i] = segs[i].len;
    s.src_stride[i] = 0;
    s.dst_stride[i] = 0;
    s.dst[i] = segs[i].dst;
    if (segs[i].len > maxlen) maxlen = segs[i].len;
  }
  int splits;
  const float* t1 = vec_stage1(partial, G, row, &splits, tmp, st);
  k_vec_reduce<<<dim3((maxlen + 255) / 256, n_seg), 256, 0, st>>>(t1, splits, row, s);
}

// Strided variant: dst[c * dst_stride + k] = sum_g partial[g][src + c * src_stride + k],
// c < runs, k < inner.
void launch_vec_reduce_strided(const float* partial, int G, int row, int src, int runs, int inner, int src_stride,
                               float* dst, int dst_stride, float* tmp, hipStream_t st) {
  VecSegs s{};
  s.n = 1;
  s.src[0] = src;
  s.len[0] = runs * inner;
  s.inner[0] = inner;
  s.src_stride[0] = src_stride;
  s.dst_stride[0] = dst_stride;
  s.dst[0] = dst;
  int splits;
  const float* t1 = vec_stage1(partial, G, row, &splits, tmp, st);
  k_vec_reduce<<<dim3((runs * inner + 255) / 256, 1), 256, 0, st>>>(t1, splits, row, s);
}

// ---------------------------------------------------------------------------
// Weight preparation: cast (and transpose) FP32 parameter matrices into the
// compute blob.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_prep(const float* __restrict__ params, T* __restrict__ blob, const PrepJob* __restrict__ jobs) {
  const PrepJob j = jobs[blockIdx.y];
  const int tot = j.rows * j.cols;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += gridDim.x * blockDim.x) {
    const int i = idx / j.cols, k = idx - i * j.cols;
    const float v = j.transpose ? params[j.src_off + (int64_t)k * j.src_ld + j.src_col0 + i]
                                : params[j.src_off + (int64_t)i * j.src_ld + j.src_col0 + k];
    blob[j.dst_off + (int64_t)i * j.dst_ld + j.dst_col0 + k] = from_f<T>(v);
  }
}

void launch_prep(const float* params, void* blob, int prec, const PrepJob* jobs_dev, int n_jobs, hipStream_t st) {
  if (n_jobs == 0) return;
  dim3 grid(64, n_jobs);
  if (prec == 1) k_prep<bf16><<<grid, 256, 0, st>>>(params, (bf16*)blob, jobs_dev);
  else k_prep<float><<<grid, 256, 0, st>>>(params, (float*)blob, jobs_dev);
}

// ---------------------------------------------------------------------------
__global__ void k_fill(float* p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
void launch_fill(float* p, size_t n, float v, hipStream_t st) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
}

__global__ void k_accumulate(float* __restrict__ acc, const float* __restrict__ g, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc[i] += g[i];
}
void launch_accumulate(float* acc, const float* g, int64_t n, hipStream_t st) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_accumulate<<<(unsigned)blocks, 256, 0, st>>>(acc, g, n);
}

// ---------------------------------------------------------------------------
// Optimizer: global-norm clipping and Adam.  The squared norm is summed in
// FP64, per workgroup over a fixed index set and then over the workgroups in
// order, so the step is deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ g, int64_t n,
                                               double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double x = g[i];
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n,
                                              const double* __restrict__ partial, int G, AdamArgs a,
                                              float* __restrict__ norm_out) {
  __shared__ float scale;
  if (threadIdx.x == 0) {
    double ss = 0.0;
    for (int k = 0; k < G; ++k) ss += partial[k];
    const double norm = sqrt(ss);
    scale = a.clip > 0.0 ? (float)fmin(1.0, a.clip / (norm + 1e-6)) : 1.f;
    if (blockIdx.x == 0 && norm_out) norm_out[0] = (float)norm;
  }
  __syncthreads();
  const float sc = scale;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i] * sc;
    const float mi = a.b1 * m[i] + a.c1 * gi;
    const float vi = a.b2 * v[i] + a.c2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= a.lr * (mi / a.bc1) / (sqrtf(vi / a.bc2) + a.eps);
  }
}

void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, double* partial, int G,
                 const AdamArgs& a, float* norm_out, hipStream_t st) {
  k_sumsq<<<G, 256, 0, st>>>(g, n, partial);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_adam<<<(unsigned)blocks, 256, 0, st>>>(p, g, m, v, n, partial, G, a, norm_out);
}

// ---------------------------------------------------------------------------
// Allocation-free optimizer step.  The clipping norm's per-workgroup
// partials live in `scratch`, a fixed array of the library on every device
// it runs on (held until the process ends), instead of a context buffer.
// In host code `scratch` names a host-side stand-in: its device address is
// looked up once per device and only that address is ever used.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kAdamScratchPartials];

static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices] = {};

int adam_noalloc_scratch(int device, double** out, const char** err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) {
    *err = "device index out of range";
    return -1;
  }
  if (!g_scratch_dev[device]) {
    // with `device` current (the caller made it so): this device's copy
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = hipGetErrorString(e);
      return -3;
    }
    g_scratch_dev[device] = (double*)ptr;
  }
  *out = g_scratch_dev[device];
  return 0;
}

// Masked MSE over the batch's inner rows: per-workgroup partial sums in a
// fixed order, then a single-workgroup fixed-order total.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out, const float* __restrict__ target,
                                             const int* __restrict__ gid, const int* __restrict__ inner, int n_inner,
                                             int C, double inv_norm, float* __restrict__ d_out,
                                             float* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  const int tot = n_inner * C;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < tot; idx += gridDim.x * 256) {
    const int i = idx / C, c = idx - i * C;
    const size_t o = (size_t)gid[inner[i]] * C + c;
    const double d = (double)out[o] - (double)target[o];
    s += d * d;
    d_out[o] = (float)(2.0 * d * inv_norm);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = (float)(red[0] * inv_norm);
}
__global__ void k_sum_partials(const float* __restrict__ partial, int G, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += partial[g];
    out[0] = (float)s;
  }
}

void launch_mse(const float* out, const float* target, const int* gid, const int* inner, int n_inner, int out_dim,
                double inv_norm, float* d_out, float* partial, int G, float* loss, hipStream_t st) {
  k_mse<<<G, 256, 0, st>>>(out, target, gid, inner, n_inner, out_dim, inv_norm, d_out, partial);
  k_sum_partials<<<1, 64, 0, st>>>(partial, G, loss);
}

}  // namespace xmgn
